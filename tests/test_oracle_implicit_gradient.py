"""Pin of the implicit reconstruction gradients that the autograd wrapper implements.

For c = M(gamma)^-1 b with M = W A^T C A W^T + alpha D(gamma), D_l ~ 1/gamma_l (the prior of
Eq. (fewha)), and L = w . c, the implicit-function rule gives, with lambda = M^-1 w,
    dL/dgamma_l = lambda_l^T (alpha D)_l c_l / gamma_l,     dL/ds = C A lambda (b = W A^T C s).
Checked on the tiny configuration against derivatives of exact dense solves (M assembled column
by column from the oracle's matrix-free M): a complex-step derivative in gamma, and the exact
directional derivative in s (L is linear in s).
"""
import numpy as np
import pytest

from paper_2009_00946_amd import synth
from oracle import Oracle


@pytest.fixture(scope="module")
def dense_c0():
    cfg = synth.load_config("c0_tiny")
    O = Oracle(cfg, precond=False)
    N = O.n_coef
    M = np.empty((N, N))
    e = np.zeros(N)
    for k in range(N):
        e[k] = 1.0
        M[:, k] = O.M(e)
        e[k] = 0.0
    return cfg, O, M


def test_implicit_gamma_gradient_matches_finite_differences(dense_c0):
    cfg, O, M = dense_c0
    N = O.n_coef
    s = O.Ahat(synth.layer_screens_flat(cfg, 0)) + O.slope_mask() * synth.slope_noise(cfg, 0)
    b = O.rhs(s)
    w = synth.normal_vector(N, 41)
    aD = cfg["alpha_reg"] * O.prior()
    c = np.linalg.solve(M, b)
    lam = np.linalg.solve(M, w)
    offs = np.cumsum([0] + [l["n"] ** 2 for l in cfg["layers"]])
    for l, lay in enumerate(cfg["layers"]):
        g = lay["cn2_weight"]
        sl = slice(offs[l], offs[l + 1])
        idx = np.arange(offs[l], offs[l + 1])
        formula = float(lam[sl] @ (aD[sl] * c[sl])) / g
        # complex-step derivative in gamma_l (D_l scales as 1/gamma_l): no subtractive
        # cancellation, so only the solve's own rounding (cond(M) ~ 8e7) limits it
        h = 1e-20
        Mc = M.astype(complex)
        Mc[idx, idx] += aD[sl] * (g / (g + 1j * h * g) - 1.0)
        cs = float(np.imag(w @ np.linalg.solve(Mc, b))) / (h * g)
        assert abs(formula - cs) <= 1e-8 * abs(cs), (l, formula, cs)


def test_implicit_slope_gradient_matches_finite_differences(dense_c0):
    cfg, O, M = dense_c0
    N = O.n_coef
    w = synth.normal_vector(N, 42)
    lam = np.linalg.solve(M, w)
    grad_s = O.slope_weights() * O.A(lam)
    # L is linear in s: its derivative along d is w . M^-1 b(d) exactly
    d = synth.normal_vector(O.n_slopes, 43)
    ref = float(w @ np.linalg.solve(M, O.rhs(d)))
    assert abs(float(d @ grad_s) - ref) <= 1e-7 * abs(ref)

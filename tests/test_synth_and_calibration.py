"""Pins of the seeded input generator and of the regularisation constant alpha_reg.

* The FFT phase screens must follow the von Karman structure function
  D(r) = 4 pi int f Phi(f) (1 - J0(2 pi f r)) df with Phi = 0.023 r0^-5/3 (f^2 + L0^-2)^-11/6,
  which tends to the Kolmogorov law 6.88 (r/r0)^(5/3) for L0 -> infinity (checked too).
* alpha_reg in each configuration must equal the calibration it is documented to be:
  1 / median over (layer, detail level) of D * empirical coefficient variance of 16 screens.
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.special

import kron_ref
from oracle import Oracle
from paper_2009_00946_amd import synth


def _vk_structure(r, r0, L0):
    f = lambda x: x * 0.023 * r0 ** (-5 / 3) * (x * x + (1 / L0) ** 2) ** (-11 / 6) * (1 - scipy.special.j0(2 * np.pi * x * r))
    val = 0.0
    edges = [0, 0.1 / r, 1 / r, 10 / r, 100 / r, 1000 / r, np.inf]
    for a, b in zip(edges[:-1], edges[1:]):
        val += scipy.integrate.quad(f, a, b, limit=400)[0]
    return 4 * np.pi * val


def test_structure_function_integral_kolmogorov_limit():
    r0 = 0.2
    for r in (0.1, 0.5):
        assert abs(_vk_structure(r, r0, 1e7) / (6.88 * (r / r0) ** (5 / 3)) - 1) < 0.01


def test_screens_follow_von_karman():
    cfg = synth.load_config("c1_elt_mcao")
    lay = cfg["layers"][0]
    n, dl = lay["n"], lay["spacing"]
    r0l = cfg["r0"] * lay["cn2_weight"] ** (-3 / 5)
    emp = {k: [] for k in (2, 4, 8)}
    for seed in range(8):
        rng = np.random.default_rng(seed)
        scr = synth.von_karman_screen(rng, 2 * n, dl, r0l, cfg["L0"])
        for k in emp:
            dx = scr[:, k:] - scr[:, :-k]
            dy = scr[k:, :] - scr[:-k, :]
            emp[k].append(0.5 * (np.mean(dx ** 2) + np.mean(dy ** 2)))
    for k, v in emp.items():
        theory = _vk_structure(k * dl, r0l, cfg["L0"])
        assert abs(np.mean(v) / theory - 1) < 0.1, (k, np.mean(v), theory)


def test_frozen_flow_shifts_by_one_cell():
    cfg = synth.load_config("c0_tiny")
    a = synth.layer_screens(cfg, 0)
    b = synth.layer_screens(cfg, 1)
    for lay, s0, s1 in zip(cfg["layers"], a, b):
        vx, vy = lay["flow"]
        assert np.array_equal(np.roll(s1, (vy, vx), axis=(0, 1))[1:-1, 1:-1], s0[1:-1, 1:-1])


def test_seeded_reproducibility():
    cfg = synth.load_config("t1_mixed")
    assert np.array_equal(synth.layer_screens_flat(cfg, 3), synth.layer_screens_flat(cfg, 3))
    assert np.array_equal(synth.slope_noise(cfg, 2), synth.slope_noise(cfg, 2))
    assert not np.array_equal(synth.slope_noise(cfg, 2), synth.slope_noise(cfg, 3))
    n_coef, n_slopes, n_act = synth.sizes(cfg)
    assert synth.layer_screens_flat(cfg).size == n_coef and synth.slope_noise(cfg).size == n_slopes


def calibrate_alpha(cfg, n_screens=16):
    o = Oracle(cfg, precond=False)
    Dp = o.prior()
    J = cfg["J"]
    acc = {}
    for seed in range(n_screens):
        c = o.W(synth.layer_screens_flat(cfg, seed=5000 + seed))
        off = 0
        for li, lay in enumerate(cfg["layers"]):
            n = lay["n"]
            lv = kron_ref.levels(n, J).ravel()
            cl, dl = c[off:off + n * n], Dp[off:off + n * n]
            for s in range(1, J):
                m = lv == s
                acc.setdefault((li, s), []).append(np.mean(cl[m] ** 2) * dl[m][0])
            off += n * n
    return 1.0 / np.median([np.mean(v) for v in acc.values()])


@pytest.mark.parametrize("name", ["c0_tiny", "t1_mixed", "c3_mid_lgs", "c1_elt_mcao", "maory_paper"])
def test_alpha_reg_is_the_documented_calibration(name):
    cfg = synth.load_config(name)
    assert abs(calibrate_alpha(cfg) / cfg["alpha_reg"] - 1) < 0.01

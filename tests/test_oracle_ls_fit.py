"""Pins of the oracle's least-squares DM fitting (more layers than DMs): the probe-direction
operator H and its transpose, CG against the dense normal equations, and a closed form.

Closed form: on the tiny configuration the ground layer (0 km, spacing 0.4 m) and the DM (0 km,
pitch 0.4 m) share their grid, and the fitting nodes coincide with actuators.  At zero altitude
every probe direction sees the same points, so H^T H = 25 I on the actuators inside the pupil.
A ground layer holding actuator values a* (the 8 km layer zero) is therefore fitted by
a = 25 / (25 + eps) a* there, and 0 elsewhere.
"""
import numpy as np
import pytest

from paper_2009_00946_amd import synth
from oracle import Oracle


@pytest.fixture(scope="module")
def c0():
    cfg = synth.load_config("c0_tiny")
    return cfg, Oracle(cfg, precond=False)


def test_probe_operator_adjoint(c0):
    cfg, O = c0
    a = synth.normal_vector(O.n_act, 21)
    y = synth.normal_vector(O.fit_points(), 22)
    lhs, rhs = float(O.ls_H(a) @ y), float(a @ O.ls_Ht(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_cg_reaches_the_dense_normal_equations(c0):
    cfg, O = c0
    na, eps = O.n_act, 0.01
    H = np.stack([O.ls_H(np.eye(na)[k]) for k in range(na)], axis=1)
    c = synth.normal_vector(O.n_coef, 23)
    y0 = O.ls_target(O.Wt(c))
    ref = np.linalg.solve(H.T @ H + eps * np.eye(na), H.T @ y0)
    got = O.fit_ls(c, 400, eps)
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_colocated_ground_layer_closed_form(c0):
    cfg, O = c0
    lay0, dm = cfg["layers"][0], cfg["dms"][0]
    n, na = lay0["n"], dm["n_act"]
    assert lay0["height"] == 0.0 and dm["height"] == 0.0 and lay0["spacing"] == dm["pitch"]
    off = n // 2 - (na - 1) // 2              # layer node k = actuator j + off
    D, ns = cfg["D"], cfg["wfs"][0]["n_sub"]
    assert abs(D / ns - dm["pitch"]) < 1e-12 and na == ns + 1
    rng = np.random.default_rng(24)
    a_star = rng.standard_normal((na, na))
    layers = np.zeros(O.n_coef)
    l0 = np.zeros((n, n))
    l0[off:off + na, off:off + na] = a_star
    layers[:n * n] = l0.ravel()
    eps = 0.01
    got = O.fit_ls(O.W(layers), 200, eps).reshape(na, na)
    x = -D / 2 + (D / ns) * np.arange(na)
    r = np.hypot(x[None, :], x[:, None])
    inside = (r <= D / 2) & (r >= cfg.get("obstruction", 0.0) * D / 2)
    assert np.allclose(got[inside], 25.0 / (25.0 + eps) * a_star[inside], rtol=0, atol=1e-10)
    assert np.allclose(got[~inside], 0.0, atol=1e-10)

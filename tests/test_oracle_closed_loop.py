"""Pins of the oracle's closed-loop pieces of Alg. 1: the DM-to-sensor operator H_dm (pseudo-open-
loop slopes s + H_dm a^(-1)) and the closed-loop control a^(1) = a^(0) + gain (F W^T c - a^(-1)).

The DM is read as the piecewise bilinear surface over its actuator grid (Sec. 4.1), seen along
each guide star's ray at the DM's altitude.  Pinned by: a DM whose actuators coincide with the
sensor nodes (H_dm a = mask Gamma a); planes (constant slopes alpha sigma d, the cone factor of the
DM's altitude) and piston (zero) inside the actuator grid; the adjoint; the equivalence of the
closed loop with the open loop when the residual measurements are the open-loop slopes minus the
DM correction; the control law against the open-loop fit.
"""
import copy

import numpy as np
import pytest

from paper_2009_00946_amd import synth
from oracle import Oracle


@pytest.fixture(scope="module")
def c0():
    cfg = synth.load_config("c0_tiny")
    return cfg, Oracle(cfg, precond=False)


@pytest.fixture(scope="module")
def c1():
    cfg = synth.load_config("c1_elt_mcao")
    return cfg, Oracle(cfg, precond=False)


def _planes(O, g):
    ns = O.cfg["wfs"][g]["n_sub"]
    off = sum(2 * O.cfg["wfs"][h]["n_sub"] ** 2 for h in range(g))
    return off, ns


def test_colocated_dm_is_gamma_of_the_actuators(c0):
    cfg, O = c0
    (dm,) = cfg["dms"]
    assert dm["height"] == 0.0 and abs(dm["pitch"] - cfg["D"] / cfg["wfs"][0]["n_sub"]) < 1e-12
    a = synth.normal_vector(O.n_act, 5)
    s = O.Hdm(a)
    mask = O.slope_mask()
    for g, w in enumerate(cfg["wfs"]):
        off, ns = _planes(O, g)
        assert dm["n_act"] == ns + 1
        ref = O.gamma(g, a.reshape(ns + 1, ns + 1)) * mask[off:off + 2 * ns * ns]
        assert np.allclose(s[off:off + 2 * ns * ns], ref, rtol=0, atol=1e-13)


def test_plane_and_piston_inside_the_actuator_grid(c1):
    cfg, O = c1
    m = 1  # the 6 km DM alone
    dm = cfg["dms"][m]
    na, p, h = dm["n_act"], dm["pitch"], dm["height"]
    a_off = sum(d["n_act"] ** 2 for d in cfg["dms"][:m])
    ai, aj = np.mgrid[0:na, 0:na]
    cen = (na - 1) / 2.0
    al, be = 0.013, -0.021
    a = np.zeros(O.n_act)
    a[a_off:a_off + na * na] = (al * (aj - cen) * p + be * (ai - cen) * p).ravel()
    s = O.Hdm(a)
    piston = np.zeros(O.n_act)
    piston[a_off:a_off + na * na] = 1.0
    sp = O.Hdm(piston)
    mask = O.slope_mask()
    checked = 0
    for g, w in enumerate(cfg["wfs"]):
        off, ns = _planes(O, g)
        d = cfg["D"] / ns
        sig = 1.0 - h / w["gs_height"] if w["gs_height"] > 0 else 1.0
        x = sig * (-cfg["D"] / 2 + d * np.arange(ns + 1))
        ux = (x + w["theta_x"] * h) / p + cen
        uy = (x + w["theta_y"] * h) / p + cen
        inx = (ux >= 0) & (ux <= na - 1)
        iny = (uy >= 0) & (uy <= na - 1)
        ok = (iny[:-1] & iny[1:])[:, None] & (inx[:-1] & inx[1:])[None, :]
        ok &= mask[off:off + ns * ns].reshape(ns, ns) > 0
        sx = s[off:off + ns * ns].reshape(ns, ns)
        sy = s[off + ns * ns:off + 2 * ns * ns].reshape(ns, ns)
        assert np.allclose(sx[ok], al * sig * d, rtol=0, atol=1e-12)
        assert np.allclose(sy[ok], be * sig * d, rtol=0, atol=1e-12)
        assert np.allclose(sp[off:off + 2 * ns * ns].reshape(2, ns, ns)[:, ok], 0.0, atol=1e-12)
        checked += int(ok.sum())
    assert checked > 1000


@pytest.mark.parametrize("name", ["c0_tiny", "t1_mixed"])
def test_hdm_adjoint(name):
    O = Oracle(synth.load_config(name), precond=False)
    a = synth.normal_vector(O.n_act, 6)
    s = synth.normal_vector(O.n_slopes, 7)
    lhs, rhs = float(O.Hdm(a) @ s), float(a @ O.Hdm_t(s))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_pseudo_open_loop_recovers_open_loop_slopes(c0):
    cfg, O = c0
    s_open = O.Ahat(synth.layer_screens_flat(cfg, 0)) + O.slope_mask() * synth.slope_noise(cfg, 0)
    a_m1 = synth.normal_vector(O.n_act, 8)
    s_res = s_open - O.Hdm(a_m1)  # what the sensors measure behind the DMs (two-step delay)
    assert np.allclose(O.pol(s_res, a_m1), O.slope_mask() * s_open, rtol=0, atol=1e-12)


def test_closed_loop_control_law(c0):
    cfg, O = c0
    c = synth.normal_vector(O.n_coef, 9)
    a0 = synth.normal_vector(O.n_act, 10)
    a_m1 = synth.normal_vector(O.n_act, 11)
    ft = O.fit(c, None, 1.0)  # F W^T c
    assert np.allclose(O.fit_closed(c, a0, a0, 1.0), ft, rtol=0, atol=1e-13)
    g = 0.4
    assert np.allclose(O.fit_closed(c, a0, a_m1, g), a0 + g * (ft - a_m1), rtol=0, atol=1e-13)

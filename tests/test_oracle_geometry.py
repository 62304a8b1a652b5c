"""Pins of the oracle's Shack-Hartmann operator Gamma and geometric propagation P (Sec. 2.1).

* Gamma: a tilted plane a x + b y + c gives s^x = a d and s^y = b d on every subaperture; the
  Fried waffle (-1)^(i+j) and constants are in its null space (this is what rules out the
  printed diagonal difference in s^y); Gamma^T is its adjoint.
* P: bilinear interpolation reproduces any bilinear layer function exactly, so on layers
  U_l(X, Y) = a + b X + c Y + e X Y the propagated wavefront must equal
  sum_l U_l(sigma x + theta_x h_l, sigma y + theta_y h_l) with sigma = 1 - h_l / H (LGS) or 1
  (NGS): this fixes the cone factor, the direction of the shift and the node origin.
"""
import math

import numpy as np
import pytest

from oracle import Oracle


def _nodes(cfg, g):
    ns = cfg["wfs"][g]["n_sub"]
    d = cfg["D"] / ns
    x = -cfg["D"] / 2 + d * np.arange(ns + 1)
    return ns, d, x


@pytest.mark.parametrize("g", [0, 2, 3])
def test_gamma_plane_gives_constant_slopes(orc_t1, cfg_t1, g):
    ns, d, x = _nodes(cfg_t1, g)
    a, b, c = 0.37, -1.21, 4.0
    phi = a * x[None, :] + b * x[:, None] + c              # row = y, col = x
    s = orc_t1.gamma(g, phi.ravel())
    assert np.allclose(s[:ns * ns], a * d, atol=1e-14)
    assert np.allclose(s[ns * ns:], b * d, atol=1e-14)


def test_gamma_waffle_and_constant_null(orc_t1, cfg_t1):
    ns, d, x = _nodes(cfg_t1, 0)
    i, j = np.meshgrid(np.arange(ns + 1), np.arange(ns + 1), indexing="ij")
    assert np.abs(orc_t1.gamma(0, ((-1.0) ** (i + j)).ravel())).max() < 1e-15
    assert np.abs(orc_t1.gamma(0, np.full((ns + 1) ** 2, 3.5))).max() < 1e-15


def test_gamma_rotation_swaps_axes(orc_t1, cfg_t1):
    """Rotating the wavefront by 90 degrees rotates the gradient: s^x' = rot(s^y), s^y' = -rot(s^x)."""
    ns, d, x = _nodes(cfg_t1, 2)
    phi = np.random.default_rng(1).standard_normal((ns + 1, ns + 1))
    s = orc_t1.gamma(2, phi.ravel())
    sx, sy = s[:ns * ns].reshape(ns, ns), s[ns * ns:].reshape(ns, ns)
    rot = np.rot90(phi)                                     # rot[i, j] = phi[j, n - i]
    s2 = orc_t1.gamma(2, rot.copy().ravel())
    sx2, sy2 = s2[:ns * ns].reshape(ns, ns), s2[ns * ns:].reshape(ns, ns)
    assert np.allclose(sx2, np.rot90(sy), atol=1e-14)
    assert np.allclose(sy2, -np.rot90(sx), atol=1e-14)


@pytest.mark.parametrize("g", [0, 1, 2, 3])
def test_gamma_adjoint(orc_t1, cfg_t1, g):
    ns = cfg_t1["wfs"][g]["n_sub"]
    rng = np.random.default_rng(g)
    phi = rng.standard_normal((ns + 1) ** 2)
    s = rng.standard_normal(2 * ns * ns)
    lhs = np.dot(orc_t1.gamma(g, phi), s)
    rhs = np.dot(phi, orc_t1.gamma_t(g, s))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def _bilinear_layers(cfg, coeffs):
    out = []
    for lay, (a, b, c, e) in zip(cfg["layers"], coeffs):
        n, dl = lay["n"], lay["spacing"]
        X = (np.arange(n) - n / 2) * dl
        out.append((a + b * X[None, :] + c * X[:, None] + e * X[None, :] * X[:, None]).ravel())
    return np.concatenate(out)


@pytest.mark.parametrize("cfgname", ["t1", "c0"])
def test_projection_exact_on_bilinear_layers(cfgname, request):
    cfg = request.getfixturevalue("cfg_" + cfgname)
    o = request.getfixturevalue("orc_" + cfgname)
    rng = np.random.default_rng(11)
    coeffs = [tuple(rng.standard_normal(4) * [1, 0.3, 0.3, 0.05]) for _ in cfg["layers"]]
    phi = o.P(_bilinear_layers(cfg, coeffs))
    off = 0
    for g, w in enumerate(cfg["wfs"]):
        ns, d, x = _nodes(cfg, g)
        expect = np.zeros((ns + 1, ns + 1))
        for lay, (a, b, c, e) in zip(cfg["layers"], coeffs):
            h = lay["height"]
            sig = 1 - h / w["gs_height"] if w["gs_height"] > 0 else 1.0
            X = sig * x[None, :] + w["theta_x"] * h
            Y = sig * x[:, None] + w["theta_y"] * h
            expect += a + b * X + c * Y + e * X * Y
        got = phi[off:off + (ns + 1) ** 2].reshape(ns + 1, ns + 1)
        assert np.abs(got - expect).max() < 1e-12 * max(1, np.abs(expect).max()), g
        off += (ns + 1) ** 2


def test_projection_identity_special_case():
    """On-axis NGS, one ground layer with spacing d: P samples the layer nodes themselves."""
    cfg = dict(D=8.0, obstruction=0.0, J=2, alpha_reg=1.0,
               wfs=[dict(n_sub=8, theta_x=0.0, theta_y=0.0, gs_height=0.0, sigma=1.0)],
               layers=[dict(height=0.0, cn2_weight=1.0, spacing=1.0, n=16)],
               dms=[dict(height=0.0, n_act=9, pitch=1.0)])
    o = Oracle(cfg)
    U = np.random.default_rng(2).standard_normal((16, 16))
    phi = o.P(U.ravel()).reshape(9, 9)
    assert np.abs(phi - U[4:13, 4:13]).max() < 1e-15


@pytest.mark.parametrize("cfgname", ["t1", "c0"])
def test_projection_adjoint(cfgname, request):
    o = request.getfixturevalue("orc_" + cfgname)
    rng = np.random.default_rng(4)
    U = rng.standard_normal(o.n_coef)
    f = rng.standard_normal(o.n_nodes)
    lhs, rhs = np.dot(o.P(U), f), np.dot(U, o.Pt(f))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + abs(rhs))


def test_pupil_mask_annulus(orc_t1, cfg_t1):
    ns, d, _ = _nodes(cfg_t1, 0)
    m = orc_t1.slope_mask()[:ns * ns].reshape(ns, ns)
    c = (np.arange(ns) + 0.5) * d - cfg_t1["D"] / 2
    r = np.hypot(c[None, :], c[:, None])
    D, eps = cfg_t1["D"], cfg_t1["obstruction"]
    assert np.array_equal(m, ((r <= D / 2) & (r >= eps * D / 2)).astype(float))
    assert 0 < m.sum() < ns * ns


def test_geometry_rejections(cfg_c0):
    from oracle.oracle import OracleError
    bad = dict(cfg_c0, layers=[dict(l) for l in cfg_c0["layers"]])
    bad["layers"][1]["spacing"] = 0.2                       # 8 km layer too small for the footprint
    with pytest.raises(OracleError) as e:
        Oracle(bad)
    assert e.value.status == -2
    bad = dict(cfg_c0, layers=[dict(l) for l in cfg_c0["layers"]])
    bad["layers"][0]["n"] = 24                              # not a power of two
    with pytest.raises(OracleError) as e:
        Oracle(bad)
    assert e.value.status == -1
    lgs = dict(cfg_c0, wfs=[dict(w) for w in cfg_c0["wfs"]])
    lgs["wfs"][0]["gs_height"] = 5000.0                     # LGS below the 8 km layer
    with pytest.raises(OracleError) as e:
        Oracle(lgs)
    assert e.value.status == -2
    assert math.isclose(cfg_c0["layers"][1]["spacing"], 0.45194, rel_tol=1e-4)

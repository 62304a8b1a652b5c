"""Pin of the prior D against the statistics it encodes (Eq. (fewha): D is the diagonal stand-in
for C_phi^-1 in the wavelet domain; Eq. (MAP) weighs the coefficients by it).

The oracle builds D = gamma_l^-1 (delta_l / d_1)^(-5/3) 2^(-(11/3)(s-1)).  If that is the inverse
coefficient variance of the turbulence model up to one constant, then D_{l,s} Var(c_{l,s}) is the
same number for every layer l (whatever its node spacing delta_l and Cn2 weight gamma_l) and for
every detail level s.  This is checked on the oracle's own W applied to seeded screens of the input
generator, without restating the formula:

* layers: von Karman screens as the ELT configuration draws them (L0 = 25 m), levels 1 and 2
  (scales 0.5-2 m, well inside L0), all 9 layers (spacings d/2 and d, gamma from 0.40 to 0.007);
* levels: the Kolmogorov limit of the same generator (L0 -> infinity, the kappa^-11/3 spectrum the
  law is derived from), levels 2-4 of the three 256 x 256 layers, fitted exponent of D Var against s.

Only coefficients whose db3 support lies inside the n x n window are used: the periodic transform
of a cropped (non-periodic) screen puts the window's edge jump into the wrapped coefficients.

Each check is also run on mutants of the oracle's D that a plausible slip would produce (either
exponent off by 1/3, 1/gamma dropped or squared); every mutant must fail.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2009_00946_amd import synth

N_SCREENS = 12


def _interior(n, s):
    """Detail coefficients of level s (bands x-high, y-high, HH) whose support stays inside n."""
    m = n >> s
    k = np.arange(m)
    ok = (k << s) + 5 * ((1 << s) - 1) < n
    sel = np.zeros((n, n), bool)
    for r0, c0 in ((0, m), (m, 0), (m, m)):
        sel[r0:r0 + m, c0:c0 + m] = ok[:, None] & ok[None, :]
    return sel.ravel()


def _level_of_detail(n, s):
    m = n >> s
    lv = np.zeros((n, n), bool)
    lv[:2 * m, :2 * m] = True
    lv[:m, :m] = False
    return lv.ravel()


def _products(cfg, L0, levels, seed0):
    """D x mean squared interior coefficient per (layer, level), with the oracle's W and D."""
    cfg = dict(cfg, L0=L0)
    O = Oracle(cfg, precond=False)
    acc = {}
    for k in range(N_SCREENS):
        c = O.W(synth.layer_screens_flat(cfg, seed=seed0 + k))
        off = 0
        for li, lay in enumerate(cfg["layers"]):
            n = lay["n"]
            cl = c[off:off + n * n]
            for s in levels:
                sel = _interior(n, s)
                if sel.any():
                    acc.setdefault((li, s), []).append(np.mean(cl[sel] ** 2))
            off += n * n
    return {key: np.mean(v) for key, v in acc.items()}


def _prior_per_band(cfg, D):
    """D's value on each (layer, level), asserting it is constant there (a diagonal per band)."""
    out, off = {}, 0
    for li, lay in enumerate(cfg["layers"]):
        n = lay["n"]
        for s in range(1, cfg["J"]):
            v = D[off:off + n * n][_level_of_detail(n, s)]
            assert np.ptp(v) <= 1e-12 * abs(v).max()
            out[(li, s)] = v[0]
        off += n * n
    return out


@pytest.fixture(scope="module")
def stats():
    cfg = synth.load_config("c1_elt_mcao")
    O = Oracle(cfg, precond=False)
    D = O.prior()
    vk = _products(cfg, cfg["L0"], (1, 2), 9100)
    kol = _products(cfg, 1e9, (2, 3, 4), 9300)
    return cfg, D, vk, kol


def _layer_spread(cfg, Db, vk):
    """Largest / smallest D Var over the layers, worst of levels 1 and 2."""
    worst = 1.0
    for s in (1, 2):
        p = [Db[(li, s)] * vk[(li, s)] for li in range(len(cfg["layers"]))]
        worst = max(worst, max(p) / min(p))
    return worst


def _level_exponent(cfg, Db, kol):
    """Fitted exponent e of D Var ~ 2^(e s) over levels 2..4, the 256 x 256 layers pooled."""
    big = [li for li, lay in enumerate(cfg["layers"]) if lay["n"] == 256]
    s = np.array([2, 3, 4], float)
    y = [np.log2(np.mean([Db[(li, int(k))] * kol[(li, int(k))] for li in big])) for k in s]
    return np.polyfit(s, y, 1)[0]


def _level_ratio(cfg, Db, vk):
    """D Var at level 1 over level 2 (von Karman screens), layers pooled."""
    nl = len(cfg["layers"])
    return np.mean([Db[(li, 1)] * vk[(li, 1)] for li in range(nl)]) / np.mean([Db[(li, 2)] * vk[(li, 2)] for li in range(nl)])


# measured on the oracle's D with these seeds: spread 1.058, exponent 0.000, ratio 1.097
LAYER_SPREAD_MAX = 1.12
LEVEL_EXPONENT_MAX = 0.12
LEVEL_RATIO = (0.97, 1.22)


def _passes(cfg, D, vk, kol):
    Db = _prior_per_band(cfg, D)
    return (_layer_spread(cfg, Db, vk) <= LAYER_SPREAD_MAX and abs(_level_exponent(cfg, Db, kol)) <= LEVEL_EXPONENT_MAX
            and LEVEL_RATIO[0] <= _level_ratio(cfg, Db, vk) <= LEVEL_RATIO[1])


def test_prior_is_inverse_coefficient_variance_across_layers(stats):
    cfg, D, vk, _ = stats
    spread = _layer_spread(cfg, _prior_per_band(cfg, D), vk)
    assert spread <= LAYER_SPREAD_MAX, spread


def test_prior_is_inverse_coefficient_variance_across_levels(stats):
    cfg, D, vk, kol = stats
    Db = _prior_per_band(cfg, D)
    e = _level_exponent(cfg, Db, kol)
    assert abs(e) <= LEVEL_EXPONENT_MAX, e
    r = _level_ratio(cfg, Db, vk)
    assert LEVEL_RATIO[0] <= r <= LEVEL_RATIO[1], r


def _mutants(cfg, D):
    d1 = cfg["D"] / cfg["wfs"][0]["n_sub"]
    off = 0
    level = np.zeros(D.size)
    spacing = np.zeros(D.size)
    gamma = np.zeros(D.size)
    for lay in cfg["layers"]:
        n = lay["n"]
        lv = np.full((n, n), cfg["J"])
        for s in range(cfg["J"] - 1, 0, -1):
            m = n >> s
            blk = np.zeros((n, n), bool)
            blk[:2 * m, :2 * m] = True
            blk[:m, :m] = False
            lv[blk] = s
        level[off:off + n * n] = lv.ravel()
        spacing[off:off + n * n] = lay["spacing"] / d1
        gamma[off:off + n * n] = lay["cn2_weight"]
        off += n * n
    return {
        "level exponent -10/3": D * 2.0 ** ((level - 1) / 3),
        "level exponent -12/3": D * 2.0 ** (-(level - 1) / 3),
        "spacing exponent -4/3": D * spacing ** (1 / 3),
        "spacing exponent -2": D * spacing ** (-1 / 3),
        "no 1/gamma": D * gamma,
        "1/gamma^2": D / gamma,
    }


def test_every_plausible_slip_in_the_prior_fails(stats):
    cfg, D, vk, kol = stats
    assert _passes(cfg, D, vk, kol)
    for name, Dm in _mutants(cfg, D).items():
        assert not _passes(cfg, Dm, vk, kol), name

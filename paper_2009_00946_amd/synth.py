"""Seeded synthetic inputs shared by the GPU library's callers and the CPU oracle's tests.

This module holds no arithmetic of the reconstruction method itself: it only draws random
numbers with the statistics of the paper's workload (Sec. 4.1 simulates a turbulent
atmosphere seen by Shack-Hartmann sensors):

* von Karman phase screens by the FFT method, one per layer, with Fried parameter
  r0_l = r0 * gamma_l^(-3/5) (so the layer Cn2 weights add up in r0^(-5/3)), outer scale L0,
  phase in rad at 500 nm, generated on a periodic 2n x 2n grid and cropped to n x n;
* frozen flow for warm-started frame chains: frame f crops the window shifted by
  f * flow cells (per-layer direction from the configuration);
* white measurement noise sigma_g * N(0, 1) per slope of guide star g;
* N(0, 1) vectors for operator tests.

Random streams derive from ``numpy.random.SeedSequence(seed).spawn``; every consumer gets
identical arrays for identical (config, seed, frame).
"""
import json
import os

import numpy as np

CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def load_config(name_or_path):
    """Load an AO configuration (JSON) by name (e.g. ``"c1_elt_mcao"``) or path.

    A name ``<base>_lgs`` with no file of its own is configuration ``<base>`` with its laser guide
    stars only (the natural guide stars dropped; layers, DMs, seeds and alpha_reg unchanged), the
    geometry the batched mix runs for its ELT member."""
    path = name_or_path
    if not os.path.exists(path):
        path = os.path.join(CONFIG_DIR, name_or_path + ".json")
    if not os.path.exists(path) and name_or_path.endswith("_lgs"):
        return lgs_only(load_config(name_or_path[:-4]))
    with open(path) as f:
        return json.load(f)


def lgs_only(cfg):
    """A copy of ``cfg`` keeping only its laser guide stars, named ``<name>_lgs``."""
    import copy
    out = copy.deepcopy(cfg)
    out["wfs"] = [w for w in out["wfs"] if w["gs_height"] > 0]
    if not out["wfs"]:
        raise ValueError("%s has no laser guide star" % cfg.get("name"))
    out["name"] = cfg["name"] + "_lgs"
    out["description"] = cfg.get("description", "") + " (laser guide stars only)"
    return out


def sizes(cfg):
    """(n_coef, n_slopes, n_act): vector lengths of the wavelet, slope and actuator spaces."""
    n_coef = sum(l["n"] ** 2 for l in cfg["layers"])
    n_slopes = sum(2 * w["n_sub"] ** 2 for w in cfg["wfs"])
    n_act = sum(d["n_act"] ** 2 for d in cfg["dms"])
    return n_coef, n_slopes, n_act


def von_karman_screen(rng, N, delta, r0, L0):
    """One periodic N x N von Karman phase screen (rad) on spacing delta (m), FFT method.

    PSD 0.023 r0^(-5/3) (f^2 + 1/L0^2)^(-11/6) with f in cycles/m; DC term zeroed.
    """
    f = np.fft.fftfreq(N, d=delta)
    f2 = f[None, :] ** 2 + f[:, None] ** 2
    psd = 0.023 * r0 ** (-5.0 / 3.0) * (f2 + 1.0 / L0 ** 2) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    df = 1.0 / (N * delta)
    cn = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * np.sqrt(psd) * df
    return np.fft.ifft2(cn).real * (N * N)


def _streams(cfg, seed, k):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def layer_screens(cfg, frame=0, seed=None):
    """True turbulent layers for one frame: list of n_l x n_l float64 arrays (row = y, col = x)."""
    seed = cfg["seed"] if seed is None else seed
    rngs = _streams(cfg, seed, len(cfg["layers"]))
    out = []
    for rng, lay in zip(rngs, cfg["layers"]):
        n = lay["n"]
        r0l = cfg["r0"] * lay["cn2_weight"] ** (-3.0 / 5.0)
        big = von_karman_screen(rng, 2 * n, lay["spacing"], r0l, cfg["L0"])
        vx, vy = lay.get("flow", (1, 0))
        oy = (frame * vy) % (2 * n)
        ox = (frame * vx) % (2 * n)
        rows = (oy + np.arange(n)) % (2 * n)
        cols = (ox + np.arange(n)) % (2 * n)
        out.append(big[np.ix_(rows, cols)].copy())
    return out


def layer_screens_flat(cfg, frame=0, seed=None):
    """Layers concatenated in configuration order, each n_l^2 row-major (float64)."""
    return np.concatenate([s.ravel() for s in layer_screens(cfg, frame, seed)])


def slope_noise(cfg, frame=0, seed=None):
    """Measurement noise sigma_g * N(0,1) for every dense slope (s^x plane then s^y plane per WFS)."""
    seed = (cfg["seed"] if seed is None else seed) + 7919
    rng = np.random.default_rng(np.random.SeedSequence([seed, frame]))
    parts = []
    for w in cfg["wfs"]:
        parts.append(w["sigma"] * rng.standard_normal(2 * w["n_sub"] ** 2))
    return np.concatenate(parts)


def normal_vector(n, seed):
    """N(0,1) float64 vector of length n."""
    return np.random.default_rng(np.random.SeedSequence([seed, n])).standard_normal(n)

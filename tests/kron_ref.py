"""Independent dense assembly of the FEWHA operators for tiny configurations (NumPy).

Built from the formulas of Sec. 2.1 and Eq. (fewha) through Kronecker products of 1D
factors -- a different construction from the oracle's loops:

* Gamma^x = Avg_y (x) Diff_x,  Gamma^y = Diff_y (x) Avg_x  (row-major vec, row = y);
* P_gl = R_y (x) R_x with 1D bilinear factors (two non-zeros per row);
* one 2D wavelet level = F (x) F acting on the top-left m x m block, F the 1D periodic
  db3 analysis matrix written from the filter taps (aliased taps summed);
* D from the level of each coefficient.
Only for sizes where dense matrices are cheap (a few thousand unknowns).
"""
import numpy as np


def db3_taps():
    q, p, s = np.sqrt(10.0), np.sqrt(5 + 2 * np.sqrt(10.0)), 16 * np.sqrt(2.0)
    h = np.array([1 + q + p, 5 + q + 3 * p, 10 - 2 * q + 2 * p, 10 - 2 * q - 2 * p, 5 + q - 3 * p, 1 + q - p]) / s
    g = np.array([(-1) ** n * h[5 - n] for n in range(6)])
    return h, g


def analysis_1d(m):
    h, g = db3_taps()
    F = np.zeros((m, m))
    for k in range(m // 2):
        for n in range(6):
            F[k, (2 * k + n) % m] += h[n]
            F[m // 2 + k, (2 * k + n) % m] += g[n]
    return F


def wavelet_layer(n, J):
    W = np.eye(n * n)
    for lev in range(J):
        m = n >> lev
        F = analysis_1d(m)
        idx = (np.arange(m)[:, None] * n + np.arange(m)[None, :]).ravel()
        L = np.eye(n * n)
        L[np.ix_(idx, idx)] = np.kron(F, F)
        W = L @ W
    return W


def block_diag(mats):
    r = sum(a.shape[0] for a in mats)
    c = sum(a.shape[1] for a in mats)
    out = np.zeros((r, c))
    i = j = 0
    for a in mats:
        out[i:i + a.shape[0], j:j + a.shape[1]] = a
        i += a.shape[0]
        j += a.shape[1]
    return out


def wavelet(cfg):
    return block_diag([wavelet_layer(l["n"], cfg["J"]) for l in cfg["layers"]])


def gamma(ns):
    diff = np.zeros((ns, ns + 1))
    avg = np.zeros((ns, ns + 1))
    for i in range(ns):
        diff[i, i], diff[i, i + 1] = -1.0, 1.0
        avg[i, i], avg[i, i + 1] = 0.5, 0.5
    return np.vstack([np.kron(avg, diff), np.kron(diff, avg)])


def interp_1d(coords, n):
    R = np.zeros((len(coords), n))
    for j, u in enumerate(coords):
        k0 = min(int(np.floor(u)), n - 2)
        t = u - k0
        R[j, k0] += 1 - t
        R[j, k0 + 1] += t
    return R


def projection(cfg):
    rows = []
    for w in cfg["wfs"]:
        ns = w["n_sub"]
        d = cfg["D"] / ns
        x = -cfg["D"] / 2 + d * np.arange(ns + 1)
        blocks = []
        for l in cfg["layers"]:
            h, n, dl = l["height"], l["n"], l["spacing"]
            sig = 1 - h / w["gs_height"] if w["gs_height"] > 0 else 1.0
            Rx = interp_1d((sig * x + w["theta_x"] * h) / dl + n / 2, n)
            Ry = interp_1d((sig * x + w["theta_y"] * h) / dl + n / 2, n)
            blocks.append(np.kron(Ry, Rx))
        rows.append(np.hstack(blocks))
    return np.vstack(rows)


def mask_and_weights(cfg):
    m, wt = [], []
    D, eps = cfg["D"], cfg.get("obstruction", 0.0)
    for w in cfg["wfs"]:
        ns = w["n_sub"]
        c = (np.arange(ns) + 0.5) * D / ns - D / 2
        r = np.hypot(c[None, :], c[:, None]).ravel()
        a = ((r <= D / 2) & (r >= eps * D / 2)).astype(float)
        m.append(np.concatenate([a, a]))
        wt.append(np.concatenate([a, a]) / w["sigma"] ** 2)
    return np.concatenate(m), np.concatenate(wt)


def gamma_all(cfg):
    return block_diag([gamma(w["n_sub"]) for w in cfg["wfs"]])


def levels(n, J):
    lv = np.zeros((n, n), int)
    for s in range(1, J + 1):
        m = n >> (s - 1)
        lv[:m, :m] = s
    return lv


def prior(cfg):
    d1 = cfg["D"] / cfg["wfs"][0]["n_sub"]
    out = []
    for l in cfg["layers"]:
        s = levels(l["n"], cfg["J"]).ravel()
        out.append((l["spacing"] / d1) ** (-5.0 / 3.0) / l["cn2_weight"] * 2.0 ** (-(11.0 / 3.0) * (s - 1)))
    return np.concatenate(out)


def operators(cfg):
    """Dense (A, w, D, M, mask): A = mask Gamma P W^T, M = A^T diag(w) A + alpha diag(D)."""
    mask, w = mask_and_weights(cfg)
    W = wavelet(cfg)
    A = mask[:, None] * (gamma_all(cfg) @ projection(cfg) @ W.T)
    Dp = prior(cfg)
    M = A.T @ (w[:, None] * A) + cfg["alpha_reg"] * np.diag(Dp)
    return A, w, Dp, M, mask

"""Precision study of the GPU path (test infrastructure; run by test_gpu_precision.py, or as a
script to print the table).

1. The precision-stress configuration (35 layers up to 512^2, J = 7, 6 LGS, 12 cold PCG
   iterations): FP32 storage with FP64 reductions, and an all-FP64 GPU plan, each against the
   FP64 oracle on the same seeded slopes.  Reported: relative error of c (overall and per
   wavelet level), of what the sensors see (A c), of the layers W^T c and of the PCG residual
   norms per iteration.  The coarsest levels hold layer piston, which no slope sees: only the
   prior alpha D (smallest there) constrains them, so they carry the FP32 error.
2. Drift of the warm-restart recurrence (Alg. 1: r_prev carried from frame to frame instead of
   recomputed): over a chain of ELT frames, the carried residual against b - M c evaluated by
   the oracle in FP64 from the GPU's own c, relative to ||b||.  In exact arithmetic the two are
   equal after every frame.
"""
import json
import sys

import numpy as np

from paper_2009_00946_amd import synth


def _rel(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return {"max": float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)),
            "norm": float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))}


def _slopes(O, cfg, frame):
    return O.Ahat(synth.layer_screens_flat(cfg, frame)) + O.slope_mask() * synth.slope_noise(cfg, frame)


def level_masks(cfg):
    """Per level s = 1..J, a mask over the coefficient vector of that level's bands (LL of
    level J included in level J)."""
    J = cfg["J"]
    masks = []
    for s in range(1, J + 1):
        parts = []
        for lay in cfg["layers"]:
            n = lay["n"]
            m = n >> s
            a = np.zeros((n, n), bool)
            a[:2 * m, :2 * m] = True
            if s < J:
                a[:m, :m] = False
            parts.append(a.ravel())
        masks.append(np.concatenate(parts))
    return masks


def stress(precisions=("fp64", "fp32"), name="c4_stress", plans=None, O=None):
    import torch
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config(name)
    O = O or Oracle(cfg)
    n_iter, N = cfg["n_iter"], O.n_coef
    s = _slopes(O, cfg, 0)
    z = np.zeros(N)
    c_ref, _, _, res_ref, st = O.frame(s, z, z, z, n_iter, True)
    assert st == 0
    lay_ref = O.Wt(c_ref)
    out = {"config": name, "n_iter": n_iter, "n_coef": N}
    for prec in precisions:
        print("[precision] %s %s" % (name, prec), flush=True)
        P = (plans or {}).get(prec) or fewha.Plan(cfg, precision=prec)
        c = P.zeros(N)
        res = torch.zeros(n_iter, dtype=torch.float64, device=P.device)
        P.pcg_solve(torch.as_tensor(s, dtype=P.dtype, device=P.device), c, n_iter, warm=False, resnorm=res)
        torch.cuda.synchronize()
        assert P.last_status() == 0, fewha.STATUS.get(P.last_status(), P.last_status())
        lay = P.dwt_inverse(c)
        res_h = res.cpu().numpy()
        ch = c.double().cpu().numpy()
        by_level = []
        for msk in level_masks(cfg):
            by_level.append(float(np.linalg.norm(ch[msk] - c_ref[msk]) / max(np.linalg.norm(c_ref[msk]), 1e-300)))
        out[prec] = {"c": _rel(ch, c_ref),
                     "c_by_level": by_level,
                     "visible": _rel(O.A(ch), O.A(c_ref)),
                     "layers": _rel(lay.double().cpu().numpy(), lay_ref),
                     "resnorm_per_iter": [float(abs(a - b) / max(abs(b), 1e-300)) for a, b in zip(res_h, res_ref)],
                     "resnorm_ref": [float(x) for x in res_ref]}
    return out


def drift(frames=16, precisions=("fp64", "fp32"), name="c1_elt_mcao", plans=None, O=None, refresh_every=0):
    """Carried against recomputed residual after every frame; with ``refresh_every`` = k > 0 every
    k-th warm frame recomputes its residual as b - M c (FEWHA_REFRESH) instead."""
    import torch
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config(name)
    O = O or Oracle(cfg)
    n_iter, N = cfg["n_iter"], O.n_coef
    S = [_slopes(O, cfg, f) for f in range(frames)]
    out = {"config": name, "frames": frames, "n_iter": n_iter, "refresh_every": refresh_every}
    for prec in precisions:
        print("[drift] %s %s" % (name, prec), flush=True)
        P = (plans or {}).get(prec) or fewha.Plan(cfg, precision=prec)
        c = P.zeros(N)
        rows = []
        for f in range(frames):
            refresh = refresh_every > 0 and f > 0 and f % refresh_every == 0
            P.pcg_solve(torch.as_tensor(S[f], dtype=P.dtype, device=P.device), c, n_iter, warm=f > 0,
                        refresh=refresh)
            torch.cuda.synchronize()
            assert P.last_status() == 0
            _, r_g = P.state_get()
            ch = c.double().cpu().numpy()
            b = O.rhs(S[f])
            r_true = b - O.M(ch)
            rows.append(float(np.linalg.norm(r_g.double().cpu().numpy() - r_true) / np.linalg.norm(b)))
        out[prec] = {"carried_vs_recomputed_residual_over_b": rows}
    return out


if __name__ == "__main__":
    import torch
    torch.cuda.set_device(0)
    r = {"stress": stress(), "drift": drift()}
    print(json.dumps(r), flush=True)
    sys.exit(0)

"""Launch shapes (fewha_set_tuning, fewha_autotune) against the oracle.

The XCD chunk of a tile kernel only renumbers its workgroups, so results are bitwise those of the
default shapes.  The forward-DWT split (kf, tq) changes how many partial sums the PCG reductions
add and in which order, so frames stay within the parity bounds of the default shapes.
"""
import numpy as np
import pytest

from paper_2009_00946_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOUNDS = {"fp64": (1e-9, 1e-9), "fp32": (1e-3, 1e-4)}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(a, b):
    return max(np.abs(a - b).max() / np.abs(b).max(), np.linalg.norm(a - b) / np.linalg.norm(b))


def _chain(P, O, cfg, frames):
    """Warm chain on plan P; returns [(c, layers)] per frame and the oracle's chain."""
    n_iter, N = cfg["n_iter"], O.n_coef
    c_ref, bp, rp = np.zeros(N), np.zeros(N), np.zeros(N)
    c = P.zeros(N)
    out = []
    for f in range(frames):
        s = O.Ahat(synth.layer_screens_flat(cfg, f)) + O.slope_mask() * synth.slope_noise(cfg, f)
        c_ref, bp, rp, _, st = O.frame(s, c_ref, bp, rp, n_iter, f == 0)
        P.pcg_solve(torch.as_tensor(s, dtype=P.dtype, device=P.device), c, n_iter, warm=f > 0)
        assert P.last_status() == 0 and st == 0
        out.append((c.double().cpu().numpy().copy(), P.dwt_inverse(c).double().cpu().numpy(), c_ref.copy(),
                    O.Wt(c_ref)))
    return out


@pytest.mark.parametrize("name,prec", [("t1_mixed", "fp64"), ("c1_elt_mcao", "fp32")])
def test_launch_shapes_keep_parity(name, prec):
    _need_gpu()
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config(name)
    O = Oracle(cfg)
    P = fewha.Plan(cfg, precision=prec)
    default = P.get_tuning()
    base = _chain(P, O, cfg, 3)
    tol_c, tol_l = BOUNDS[prec]
    J = cfg["J"]
    shapes = [dict(default, chunk_wt=8, chunk_proj=4, chunk_pt=0, chunk_fwd=16),   # renumbering only
              dict(default, kf=1, tq=4, fold=0), dict(default, kf=1, tq=8, fold=0),
              dict(default, kf=min(2, J), tq=2), dict(default, kf=min(2, J), tq=4, chunk_wt=4, chunk_fwd=8)]
    if default["fold"]:  # the coarse levels folded into the next inverse DWT, and not
        shapes += [dict(default, fold=0), dict(default, fold=0, tq=4)]
    for sh in shapes:
        print("[shape] %s %s %s" % (name, prec, sh), flush=True)
        P.set_tuning(sh)
        assert P.get_tuning() == sh
        got = _chain(P, O, cfg, 3)
        for f, ((c, lay, c_ref, lay_ref), (c0, lay0, _, _)) in enumerate(zip(got, base)):
            if (sh["kf"], sh["tq"], sh["fold"]) == (default["kf"], default["tq"], default["fold"]):
                assert np.array_equal(c, c0), (sh, f)
            assert _rel(c, c_ref) <= tol_c and _rel(lay, lay_ref) <= tol_l, (sh, f, _rel(c, c_ref), _rel(lay, lay_ref))
    P.set_tuning(default)


@pytest.mark.parametrize("name,prec,nb", [("c1_elt_mcao", "fp32", 1), ("t1_mixed", "fp32", 3)])
def test_autotune_then_parity(name, prec, nb, tmp_path):
    """The autotuner returns a valid shape set (set on the plan), stores it in the cache, and the
    tuned plan's frames follow the oracle; a second plan of the geometry takes it from the cache."""
    _need_gpu()
    from oracle import Oracle
    from paper_2009_00946_amd import fewha, tune
    cfg = synth.load_config(name)
    O = Oracle(cfg)
    P = fewha.Plan(cfg, precision=prec, max_batch=nb)
    cache = str(tmp_path / "tuning.json")
    rec = tune.tuned(P, cache=cache)
    print("[autotune] %s %s nb=%d %s" % (name, prec, nb, rec), flush=True)
    assert not rec["cached"] and P.get_tuning() == rec["tuning"]
    assert all(v > 0 for v in rec["us"].values())
    tol_c, tol_l = BOUNDS[prec]
    for c, lay, c_ref, lay_ref in _chain(P, O, cfg, 3):
        assert _rel(c, c_ref) <= tol_c and _rel(lay, lay_ref) <= tol_l
    P2 = fewha.Plan(cfg, precision=prec, max_batch=nb)
    rec2 = tune.tuned(P2, cache=cache)
    assert rec2["cached"] and P2.get_tuning() == rec["tuning"]

"""Guide-star counts at the edges of the staged P^T: 8 (its second round of pair-entry loads, guide
stars 8 to 15, has no lanes with work), 16 (the most it stages; both rounds full) and 17 (past it:
the scanning P^T).  The geometry is small enough that every other staging condition holds by
construction (node rectangles far below the stage, at most 4 sensor node lines per grid line), so
the guide-star count alone picks the path.  A, A^T and M against the oracle (FP64 1e-12, FP32 1e-5,
as for the configurations), and a cold FP64 frame at 16 guide stars (1e-9).  The operators follow
Sec. 2.1 (projection and SH gradients per guide star) and Eq. (MAP); alternate guide stars are LGS,
so the cone scaling is in every case."""
import math

import numpy as np
import pytest

from tests.test_gpu_pt_scan import max_lines_per_grid_line

torch = pytest.importorskip("torch")

AS = math.pi / (180 * 3600)
PT_MAX_WFS = 16      # guide stars the staged P^T holds
PT_STAGE = 6144      # values of the staged node rectangles per tile
RTAB_WIDTH = 4       # transpose pairs per grid line


def ring_config(n_wfs):
    """D = 3.2 m, 8x8 subapertures; n_wfs guide stars on a 20 arcsec ring, every other one an LGS
    at 90 km; layers 16^2 at 0 and 4 km (0.4 m); J = 3; one DM 9^2."""
    wfs = []
    for k in range(n_wfs):
        a = 2 * math.pi * k / n_wfs
        wfs.append({"n_sub": 8, "theta_x": 20 * AS * math.cos(a), "theta_y": 20 * AS * math.sin(a),
                    "gs_height": 90000.0 if k % 2 else 0.0, "sigma": 0.05})
    layers = [{"height": 0.0, "cn2_weight": 0.7, "n": 16, "spacing": 0.4, "flow": [1, 0]},
              {"height": 4000.0, "cn2_weight": 0.3, "n": 16, "spacing": 0.4, "flow": [0, 1]}]
    return {"name": "ring_%d" % n_wfs, "description": "D=3.2 m, %d guide stars 8x8 on a 20\" ring" % n_wfs,
            "D": 3.2, "obstruction": 0.0, "J": 3, "precision": "fp64", "n_iter": 4, "warm": False, "gain": 1.0,
            "seed": 1200 + n_wfs, "r0": 0.15, "L0": 25.0, "layers": layers, "wfs": wfs,
            "dms": [{"height": 0.0, "n_act": 9, "pitch": 0.4}], "alpha_reg": 0.1}


COUNTS = (8, 16, 17)


@pytest.mark.parametrize("n_wfs", COUNTS)
def test_geometry_meets_the_staging_conditions(n_wfs):
    cfg = ring_config(n_wfs)
    assert max_lines_per_grid_line(cfg) <= RTAB_WIDTH
    # a guide star's node rectangle on one tile is at most its whole (n_sub + 1)^2 node grid, each
    # row widened by at most 3 values to whole 16-byte chunks
    ns = cfg["wfs"][0]["n_sub"]
    assert min(n_wfs, PT_MAX_WFS) * (ns + 1) * (ns + 1 + 3) <= PT_STAGE
    assert (n_wfs <= PT_MAX_WFS) == (n_wfs != 17)


@pytest.mark.parametrize("n_wfs", COUNTS)
def test_library_accepts_the_geometry(n_wfs):
    from paper_2009_00946_amd import fewha
    for prec in ("fp64", "fp32"):
        h, st = fewha.create_host_plan(ring_config(n_wfs), prec)
        assert st == 0
        fewha.load_library().fewha_plan_destroy(h)


@pytest.mark.gpu
@pytest.mark.parametrize("n_wfs", COUNTS)
def test_guide_star_count_parity(n_wfs):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = ring_config(n_wfs)
    O = Oracle(cfg)
    rng = np.random.default_rng(40 + n_wfs)
    c = rng.standard_normal(O.n_coef)
    s = rng.standard_normal(O.n_slopes) * O.slope_mask()
    refs = (O.A(c), O.At(s), O.M(c))
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        print("[case] %d guide stars, %s" % (n_wfs, prec), flush=True)
        P = fewha.Plan(cfg, precision=prec)
        dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=P.dtype, device=P.device)
        got = (P.apply_A(dev(c)), P.apply_At(dev(s)), P.apply_M(dev(c)))
        for what, g, ref in zip(("A", "A^T", "M"), got, refs):
            g = g.detach().double().cpu().numpy()
            err = np.abs(g - ref).max() / np.abs(ref).max()
            assert err <= tol, "%d guide stars, %s, %s: %.3e > %.1e" % (n_wfs, prec, what, err, tol)
        if prec == "fp64" and n_wfs == PT_MAX_WFS:
            z = np.zeros(O.n_coef)
            c_ref = O.frame(s, z, z, z, cfg["n_iter"], True)[0]
            cg = P.zeros(P.n_coef)
            P.pcg_solve(dev(s), cg, cfg["n_iter"], warm=False)
            torch.cuda.synchronize()
            assert P.last_status() == 0
            assert np.abs(cg.cpu().numpy() - c_ref).max() <= 1e-9 * np.abs(c_ref).max()
        del P

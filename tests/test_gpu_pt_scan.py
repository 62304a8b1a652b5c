"""The scanning P^T (`k_pt_scan`), taken when a layer grid line collects more sensor node lines
than the staged transpose tables hold (4): here a 6 km layer at 2 m spacing over 0.4 m
subapertures (about 10 node lines per grid line).  A, A^T and a cold frame against the oracle
(FP64 1e-12 for operators, 1e-9 for the frame, as for the staged path), and a batch against single
frames bitwise."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

AS = math.pi / (180 * 3600)


def coarse_layer_config():
    wfs = [{"n_sub": 20, "theta_x": t * AS, "theta_y": 0.0, "gs_height": 0.0, "sigma": 0.05} for t in (-30.0, 30.0)]
    layers = [{"height": 0.0, "cn2_weight": 0.7, "n": 32, "spacing": 0.4, "flow": [1, 0]},
              {"height": 6000.0, "cn2_weight": 0.3, "n": 8, "spacing": 2.0, "flow": [0, 1]}]
    return {"name": "coarse_high_layer", "description": "D=8 m, 2 NGS 20x20, 32^2 ground layer, 8^2 layer at 2 m",
            "D": 8.0, "obstruction": 0.0, "J": 2, "precision": "fp64", "n_iter": 4, "warm": False, "gain": 1.0,
            "seed": 1100, "r0": 0.15, "L0": 25.0, "layers": layers, "wfs": wfs,
            "dms": [{"height": 0.0, "n_act": 21, "pitch": 0.4}], "alpha_reg": 0.1}


def max_lines_per_grid_line(cfg):
    """Largest number of sensor node lines whose bilinear stencil touches one layer grid line."""
    D, worst = cfg["D"], 0
    for lay in cfg["layers"]:
        n, dl, h = lay["n"], lay["spacing"], lay["height"]
        for w in cfg["wfs"]:
            ns = w["n_sub"]
            x = -D / 2 + (D / ns) * np.arange(ns + 1)
            for th in (w["theta_x"], w["theta_y"]):
                u = (x + th * h) / dl + n / 2
                k0 = np.minimum(np.floor(u).astype(int), n - 2)
                cnt = np.bincount(np.concatenate([k0, k0 + 1]), minlength=n)
                worst = max(worst, int(cnt.max()))
    return worst


def test_geometry_needs_the_scan():
    assert max_lines_per_grid_line(coarse_layer_config()) > 4


def test_library_accepts_the_geometry():
    from paper_2009_00946_amd import fewha
    for prec in ("fp64", "fp32"):
        h, st = fewha.create_host_plan(coarse_layer_config(), prec)
        assert st == 0
        fewha.load_library().fewha_plan_destroy(h)


def test_oracle_frame_runs():
    from oracle import Oracle
    cfg = coarse_layer_config()
    O = Oracle(cfg)
    s = np.random.default_rng(3).standard_normal(O.n_slopes) * O.slope_mask()
    z = np.zeros(O.n_coef)
    c, _, _, _, st = O.frame(s, z, z, z, cfg["n_iter"], True)
    assert st == 0 and np.all(np.isfinite(c)) and np.abs(c).max() > 0


@pytest.mark.gpu
def test_scan_path_parity():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = coarse_layer_config()
    O = Oracle(cfg)
    P = fewha.Plan(cfg, precision="fp64")
    PB = fewha.Plan(cfg, precision="fp64", max_batch=3)
    rng = np.random.default_rng(4)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=P.dtype, device=P.device)
    host = lambda t: t.detach().cpu().numpy()
    c = rng.standard_normal(P.n_coef)
    s = rng.standard_normal(P.n_slopes) * O.slope_mask()
    for got, ref in ((P.apply_A(dev(c)), O.A(c)), (P.apply_At(dev(s)), O.At(s))):
        got = host(got)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    z = np.zeros(P.n_coef)
    c_ref = O.frame(s, z, z, z, cfg["n_iter"], True)[0]
    cg = P.zeros(P.n_coef)
    P.pcg_solve(dev(s), cg, cfg["n_iter"], warm=False)
    torch.cuda.synchronize()
    assert P.last_status() == 0
    assert np.abs(host(cg) - c_ref).max() <= 1e-9 * np.abs(c_ref).max()
    # batched frames equal single ones bitwise on this path
    S = torch.stack([dev(rng.standard_normal(P.n_slopes) * O.slope_mask()) for _ in range(3)]).contiguous()
    cb = torch.zeros((3, P.n_coef), dtype=P.dtype, device=P.device)
    PB.pcg_solve_batch(S, cb, cfg["n_iter"], warm=False)
    for f in range(3):
        c1 = P.zeros(P.n_coef)
        P.pcg_solve(S[f].contiguous(), c1, cfg["n_iter"], warm=False)
        torch.cuda.synchronize()
        assert torch.equal(cb[f], c1), f

"""Layer counts at the edges of the projection's load rounds: its cell entries come in two rounds of
256 (16 layers) before a loop takes the rest, and its bilinear loads in chunks of 12 layer slots
whose slots past the last layer load nothing.  8 layers fill exactly one entry round, 12 one slot
chunk, 13 leave one layer to a second chunk, 16 fill both entry rounds and 17 reach the loop.  A,
A^T and M against the oracle (FP64 1e-12, FP32 1e-5, as for the configurations).  The operators
follow Sec. 2.1 (projection through every layer along each guide-star direction) and Eq. (MAP)."""
import math

import numpy as np
import pytest

from tests.test_gpu_pt_scan import max_lines_per_grid_line

torch = pytest.importorskip("torch")

AS = math.pi / (180 * 3600)


def layered_config(n_layers):
    """D = 3.2 m, 8x8 subapertures; an NGS and two LGS (90 km) on a 20 arcsec ring; n_layers layers
    of 16^2 at 0.4 m spread over 0..8 km with equal weights; J = 3; one DM 9^2."""
    wfs = [{"n_sub": 8, "theta_x": 20 * AS * math.cos(a), "theta_y": 20 * AS * math.sin(a),
            "gs_height": 90000.0 if k else 0.0, "sigma": 0.05}
           for k, a in enumerate(2 * math.pi * k / 3 for k in range(3))]
    layers = [{"height": 8000.0 * k / max(n_layers - 1, 1), "cn2_weight": 1.0 / n_layers, "n": 16,
               "spacing": 0.4, "flow": [1, 0]} for k in range(n_layers)]
    return {"name": "layers_%d" % n_layers, "description": "D=3.2 m, 3 guide stars, %d layers 16^2" % n_layers,
            "D": 3.2, "obstruction": 0.0, "J": 3, "precision": "fp64", "n_iter": 4, "warm": False, "gain": 1.0,
            "seed": 1300 + n_layers, "r0": 0.15, "L0": 25.0, "layers": layers, "wfs": wfs,
            "dms": [{"height": 0.0, "n_act": 9, "pitch": 0.4}], "alpha_reg": 0.1}


COUNTS = (8, 12, 13, 16, 17)


@pytest.mark.parametrize("n_layers", COUNTS)
def test_library_and_oracle_accept_the_geometry(n_layers):
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = layered_config(n_layers)
    assert max_lines_per_grid_line(cfg) <= 4
    for prec in ("fp64", "fp32"):
        h, st = fewha.create_host_plan(cfg, prec)
        assert st == 0
        fewha.load_library().fewha_plan_destroy(h)
    assert Oracle(cfg).n_coef == n_layers * 16 * 16


@pytest.mark.gpu
@pytest.mark.parametrize("n_layers", COUNTS)
def test_layer_count_parity(n_layers):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = layered_config(n_layers)
    O = Oracle(cfg)
    rng = np.random.default_rng(60 + n_layers)
    c = rng.standard_normal(O.n_coef)
    s = rng.standard_normal(O.n_slopes) * O.slope_mask()
    refs = (O.A(c), O.At(s), O.M(c))
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        print("[case] %d layers, %s" % (n_layers, prec), flush=True)
        P = fewha.Plan(cfg, precision=prec)
        dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=P.dtype, device=P.device)
        got = (P.apply_A(dev(c)), P.apply_At(dev(s)), P.apply_M(dev(c)))
        for what, g, ref in zip(("A", "A^T", "M"), got, refs):
            g = g.detach().double().cpu().numpy()
            err = np.abs(g - ref).max() / np.abs(ref).max()
            assert err <= tol, "%d layers, %s, %s: %.3e > %.1e" % (n_layers, prec, what, err, tol)
        del P

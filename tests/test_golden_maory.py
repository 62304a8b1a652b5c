"""The paper's own test configuration (Sec. 4.1 and its parameter table, Table 2; fixture
tests/golden/maory_parameters.txt) at the size of its first runs (Sec. 4.3: L = M = 6, 4 PCG
iterations): the plan's and the oracle's vector sizes against the matrix dimensions the paper
prints (Table 1 in Sec. 2.2), and (GPU) a cold frame with fitting against the oracle.

The configuration is `maory_paper` (written by configs/make_configs.py, which states its readings
of what the table leaves open); the first test pins it to the printed values.  With 28 % obstruction the 1x1
sensors' only subaperture is centred on the obstruction, so those two sensors have no active
slope: a degenerate case the frame must carry."""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
AS = math.pi / (180 * 3600)


def golden():
    vals = {}
    for line in open(os.path.join(HERE, "golden", "maory_parameters.txt")):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = (t.strip() for t in line.split("=", 1))
            vals[k] = [float(x) for x in v.split()]
    return {k: (v[0] if len(v) == 1 else v) for k, v in vals.items()}


def maory_config():
    from paper_2009_00946_amd import synth
    return synth.load_config("maory_paper")


def test_configuration_holds_the_printed_values():
    G, cfg = golden(), maory_config()
    ns = [w["n_sub"] for w in cfg["wfs"]]
    assert cfg["D"] == G["telescope_diameter_m"] and cfg["obstruction"] == G["obstruction_fraction"]
    assert len(ns) == G["n_wfs"] and cfg["n_iter"] == G["first_runs_n_iter"]
    assert ns == [G["n_sub_wfs_1_6"]] * 6 + [G["n_sub_wfs_7"]] + [G["n_sub_wfs_8_9"]] * 2
    lgs = [w for w in cfg["wfs"] if w["gs_height"] > 0]
    ngs = [w for w in cfg["wfs"] if w["gs_height"] == 0]
    assert (len(lgs), len(ngs)) == (G["n_lgs"], G["n_ngs"])
    for group, diam in ((lgs, G["lgs_separation_diameter_arcmin"]), (ngs, G["ngs_separation_diameter_arcmin"])):
        for w in group:
            assert abs(2 * math.hypot(w["theta_x"], w["theta_y"]) / (60 * AS) - diam) < 1e-12
    assert len(cfg["layers"]) == len(cfg["dms"]) == G["first_runs_layers"]
    lo, hi = G["n_layers_range"]
    assert lo <= len(cfg["layers"]) <= hi
    assert all(l["n"] == G["n_lay"] for l in cfg["layers"])
    assert [d["n_act"] for d in cfg["dms"]] == [G["n_act_dm_1"]] + [G["n_act_dm_2_5"]] * 4 + [G["n_act_dm_6_9"]]


def test_sizes_follow_the_printed_dimensions():
    G = golden()
    cfg = maory_config()
    assert len(cfg["wfs"]) == G["n_wfs"] and len(cfg["layers"]) == len(cfg["dms"]) == G["first_runs_layers"]
    L, nl = len(cfg["layers"]), int(G["n_lay"])
    ns = [w["n_sub"] for w in cfg["wfs"]]
    n_coef = nl * nl * L                                # 2^(2 J) L columns of P, size of M
    n_slopes = sum(2 * s * s for s in ns)               # rows of Gamma: 2 n_s^2 per sensor
    n_nodes = sum((s + 1) ** 2 for s in ns)             # columns of Gamma, rows of P
    n_act = sum(d["n_act"] ** 2 for d in cfg["dms"])
    assert (n_coef, n_slopes, n_nodes, n_act) == (98304, 76812, 39383, 18693)
    from paper_2009_00946_amd import fewha
    import ctypes
    h, st = fewha.create_host_plan(cfg, "fp64")
    assert st == 0
    Lb = fewha.load_library()
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert Lb.fewha_sizes(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == 0
    assert (a.value, b.value, c.value) == (n_coef, n_slopes, n_act)
    Lb.fewha_plan_destroy(h)
    from oracle import Oracle
    O = Oracle(cfg, precond=False)
    assert (O.n_coef, O.n_slopes, O.n_nodes, O.n_act) == (n_coef, n_slopes, n_nodes, n_act)
    # the 1x1 sensors sit inside the obstruction: no active slope; the 2x2 sensor keeps all four
    mask = O.slope_mask()
    off = np.cumsum([0] + [2 * s * s for s in ns])
    assert mask[off[7]:off[9]].sum() == 0
    assert mask[off[6]:off[7]].sum() == 8


@pytest.mark.gpu
def test_paper_configuration_frame():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import Oracle
    from paper_2009_00946_amd import fewha, synth
    cfg = maory_config()
    O = Oracle(cfg)
    P = fewha.Plan(cfg, precision="fp64")  # the configuration's bench precision is FP32
    s = O.Ahat(synth.layer_screens_flat(cfg, 0)) + O.slope_mask() * synth.slope_noise(cfg, 0)
    z = np.zeros(P.n_coef)
    c_ref = O.frame(s, z, z, z, cfg["n_iter"], True)[0]
    a_ref = O.fit(c_ref, None, 1.0)
    c = P.zeros(P.n_coef)
    P.pcg_solve(torch.as_tensor(s, dtype=P.dtype, device=P.device), c, cfg["n_iter"], warm=False)
    a = P.fit_dm(c, None, 1.0)
    torch.cuda.synchronize()
    assert P.last_status() == 0
    got_c, got_a = c.cpu().numpy(), a.cpu().numpy()
    print("\n[maory] c %.2e a %.2e" % (np.abs(got_c - c_ref).max() / np.abs(c_ref).max(),
                                       np.abs(got_a - a_ref).max() / np.abs(a_ref).max()), flush=True)
    assert np.abs(got_c - c_ref).max() <= 1e-9 * np.abs(c_ref).max()
    assert np.abs(got_a - a_ref).max() <= 1e-9 * np.abs(a_ref).max()

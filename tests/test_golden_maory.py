"""The paper's own test configuration (Sec. 5 and its parameter table, fixture
tests/golden/maory_parameters.txt) at the size of its first runs (Sec. 6: L = M = 6, 4 PCG
iterations): the plan's and the oracle's vector sizes against the matrix dimensions the paper
prints (Sec. 2.3), and (GPU) a cold frame with fitting against the oracle.

Readings beyond the printed values: LGS at 90 km on a hexagon of the printed diameter, NGS on a
triangle of theirs; layers at 0, 2.5, 5, 7.5, 10 and 15 km on 128^2 grids at 0.5 m; DM 1 at 0 km
with the subaperture pitch, DMs 2-5 at the layer heights 2.5-10 km and DM 6 at 15 km, pitched to
cover the 25 probe directions (+-1 arcmin); slope noise 0.05 rad.  With 28 % obstruction the 1x1
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
    G = golden()
    D, L = G["telescope_diameter_m"], int(G["first_runs_layers"])
    r_lgs = G["lgs_separation_diameter_arcmin"] * 60 / 2 * AS
    r_ngs = G["ngs_separation_diameter_arcmin"] * 60 / 2 * AS
    wfs = []
    for k in range(int(G["n_lgs"])):
        a = 2 * math.pi * k / G["n_lgs"]
        wfs.append({"n_sub": int(G["n_sub_wfs_1_6"]), "theta_x": r_lgs * math.cos(a), "theta_y": r_lgs * math.sin(a),
                    "gs_height": 90000.0, "sigma": 0.05})
    for k, ns in enumerate((G["n_sub_wfs_7"], G["n_sub_wfs_8_9"], G["n_sub_wfs_8_9"])):
        a = 2 * math.pi * k / 3 + math.pi / 6
        wfs.append({"n_sub": int(ns), "theta_x": r_ngs * math.cos(a), "theta_y": r_ngs * math.sin(a),
                    "gs_height": 0.0, "sigma": 0.05})
    heights = [0.0, 2500.0, 5000.0, 7500.0, 10000.0, 15000.0][:L]
    w = np.exp(-np.array(heights) / 4000.0)
    w /= w.sum()
    layers = [{"height": h, "cn2_weight": float(g), "n": int(G["n_lay"]), "spacing": 0.5, "flow": [1, 0]}
              for h, g in zip(heights, w)]
    probe = 60 * AS
    dms = [{"height": 0.0, "n_act": int(G["n_act_dm_1"]), "pitch": D / G["n_sub_wfs_1_6"]}]
    for h in heights[1:5]:
        n = int(G["n_act_dm_2_5"])
        dms.append({"height": h, "n_act": n, "pitch": (D + 2 * h * probe) / (n - 1)})
    n = int(G["n_act_dm_6_9"])
    dms.append({"height": heights[5], "n_act": n, "pitch": (D + 2 * heights[5] * probe) / (n - 1)})
    return {"name": "maory_paper", "description": "the paper's MAORY-like configuration, L = M = 6",
            "D": D, "obstruction": G["obstruction_fraction"], "J": 6, "precision": "fp64",
            "n_iter": int(G["first_runs_n_iter"]), "warm": False, "gain": 1.0, "seed": 1200, "r0": 0.15,
            "L0": 25.0, "layers": layers, "wfs": wfs, "dms": dms, "alpha_reg": 0.1}


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
    P = fewha.Plan(cfg, precision="fp64")
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

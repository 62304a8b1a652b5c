"""Write the explicit AO-system configurations used by the library, the tests and the bench.

Every number a solver needs is written out in the JSON, so that the GPU library and the
CPU oracle read identical parameters without sharing any code:

* telescope diameter and central obstruction (Sec. 4.1, MAORY-like setup),
* guide stars: subaperture count, direction (rad), height (0 = NGS at infinity), noise std,
* layers: height, Cn2 weight, grid size (power of 2) and node spacing,
* DMs: conjugation height, actuator count and pitch,
* wavelet levels J, the regularisation weight alpha_reg and the PCG iteration count.

Geometry rules (readings of Sec. 2.1 and Table 2, which leave them open):

* layer node (k, l) sits at ((l - n/2) delta, (k - n/2) delta);
* delta = max(delta_base, R / (n/2 - 2)) where R is the largest |coordinate| any WFS node
  projects to on that layer, so every projected point stays at least two cells inside;
* a DM at height h covers the 1-arcmin-radius field: pitch = (D + 2 h * 1') / (n_act - 1).

alpha_reg is the calibrated constant listed in ``ALPHA_REG`` below: it makes alpha_reg * D
equal to the inverse empirical variance of the wavelet coefficients of the synthetic
Kolmogorov screens (median over layers and detail levels, 16 screens).  A CPU test
recomputes that calibration and checks these constants against it.

Run ``python -m paper_2009_00946_amd.configs.make_configs`` to rewrite the JSON files.
"""
import json
import math
import os

ARCMIN = math.pi / (180.0 * 60.0)
ARCSEC = ARCMIN / 60.0
HERE = os.path.dirname(os.path.abspath(__file__))

# alpha_reg per configuration; see module docstring (checked by tests/test_synth_and_calibration.py)
ALPHA_REG = {
    "c0_tiny": 0.103,
    "c1_elt_mcao": 0.168,
    "c3_mid_lgs": 0.110,
    "c4_stress": 0.173,
    "t1_mixed": 0.0692,
    "maory_paper": 0.162,
}


def _ring(radius, angles_deg):
    return [(radius * math.cos(math.radians(a)), radius * math.sin(math.radians(a))) for a in angles_deg]


def _spacing(D, wfs, h, n, delta_base):
    """Node spacing rule: keep every projected WFS node two cells inside the grid."""
    R = 0.0
    for w in wfs:
        sig = 1.0 - h / w["gs_height"] if w["gs_height"] > 0 else 1.0
        R = max(R, sig * D / 2 + abs(w["theta_x"]) * h, sig * D / 2 + abs(w["theta_y"]) * h)
    return max(delta_base, R / (n / 2 - 2))


def _cn2(heights, scale=4000.0):
    w = [math.exp(-h / scale) for h in heights]
    s = sum(w)
    return [x / s for x in w]


FLOW_DIRS = [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (1, -1), (-1, -1)]


def _layers(D, wfs, heights, gammas, grid_rule):
    out = []
    for i, (h, g) in enumerate(zip(heights, gammas)):
        n, delta_base = grid_rule(h)
        out.append({
            "height": h, "cn2_weight": g, "n": n,
            "spacing": _spacing(D, wfs, h, n, delta_base),
            "flow": list(FLOW_DIRS[i % len(FLOW_DIRS)]),
        })
    return out


def _dm_pitch(D, h, n_act, fov_radius=ARCMIN):
    return (D + 2.0 * h * fov_radius) / (n_act - 1)


def c0_tiny():
    D, ns = 8.0, 20
    d = D / ns
    wfs = [{"n_sub": ns, "theta_x": tx, "theta_y": ty, "gs_height": 0.0, "sigma": 0.05}
           for tx, ty in _ring(ARCMIN, [0, 120, 240])]
    layers = _layers(D, wfs, [0.0, 8000.0], [0.7, 0.3], lambda h: (32, d))
    dms = [{"height": 0.0, "n_act": 21, "pitch": d}]
    return dict(name="c0_tiny", description="Tiny FP64: D=8 m, 3 NGS 20x20 on a 1' ring, 2 layers 32^2 (J=4), 1 DM 21^2",
                D=D, obstruction=0.0, J=4, precision="fp64", n_iter=10, warm=False, gain=1.0,
                seed=1000, r0=0.15, L0=25.0, wfs=wfs, layers=layers, dms=dms)


def _elt_wfs(with_ngs=True):
    D, ns = 39.0, 84
    wfs = [{"n_sub": ns, "theta_x": tx, "theta_y": ty, "gs_height": 90000.0, "sigma": 0.05}
           for tx, ty in _ring(ARCMIN, [0, 60, 120, 180, 240, 300])]
    if with_ngs:
        wfs += [{"n_sub": ns, "theta_x": tx, "theta_y": ty, "gs_height": 0.0, "sigma": 0.05}
                for tx, ty in _ring(80 * ARCSEC, [60, 180, 300])]
    return D, ns, wfs


def _elt_dms(D, d):
    return [{"height": 0.0, "n_act": 85, "pitch": d},
            {"height": 6000.0, "n_act": 48, "pitch": _dm_pitch(D, 6000.0, 48)},
            {"height": 12000.0, "n_act": 54, "pitch": _dm_pitch(D, 12000.0, 54)}]


def c1_elt_mcao(name="c1_elt_mcao", with_ngs=True):
    D, ns, wfs = _elt_wfs(with_ngs)
    d = D / ns
    heights = [2000.0 * k for k in range(9)]
    layers = _layers(D, wfs, heights, _cn2(heights),
                     lambda h: (256, d / 2) if h <= 4000.0 else (128, d))
    return dict(name=name,
                description="ELT MCAO FP32: D=39 m, 6 LGS (90 km, 1' hexagon) + 3 NGS (80\"), 84x84 SH, "
                            "9 layers 0-16 km (3x256^2 + 6x128^2, J=6), 3 DMs, 4 warm PCG iterations",
                D=D, obstruction=0.0, J=6, precision="fp32", n_iter=4, warm=True, gain=1.0,
                seed=1001, r0=0.15, L0=25.0, wfs=wfs, layers=layers, dms=_elt_dms(D, d))


def c3_mid_lgs():
    D, ns = 20.0, 40
    d = D / ns
    wfs = [{"n_sub": ns, "theta_x": tx, "theta_y": ty, "gs_height": 90000.0, "sigma": 0.05}
           for tx, ty in _ring(ARCMIN, [45, 135, 225, 315])]
    heights = [0.0, 3000.0, 6000.0, 9000.0, 12000.0]
    layers = _layers(D, wfs, heights, _cn2(heights), lambda h: (64, d))
    dms = [{"height": 0.0, "n_act": 41, "pitch": d}]
    return dict(name="c3_mid_lgs",
                description="Batched member: D=20 m, 4 LGS 40x40 on a 1' square, 5 layers 64^2 (J=5), 1 DM 41^2",
                D=D, obstruction=0.0, J=5, precision="fp32", n_iter=4, warm=True, gain=1.0,
                seed=1003, r0=0.15, L0=25.0, wfs=wfs, layers=layers, dms=dms)


def c4_stress():
    D, ns, wfs = _elt_wfs(with_ngs=False)
    d = D / ns
    heights = [20000.0 * k / 34.0 for k in range(35)]

    def rule(h):
        if h < 1000.0:
            return 512, d / 4
        if h < 5000.0:
            return 256, d / 2
        return 128, d
    layers = _layers(D, wfs, heights, _cn2(heights), rule)
    return dict(name="c4_stress",
                description="Precision stress: D=39 m, 6 LGS 84x84, 35 layers 0-20 km (2x512^2 + 7x256^2 + 26x128^2, J=7), "
                            "3 DMs, 12 cold PCG iterations",
                D=D, obstruction=0.0, J=7, precision="fp32", n_iter=12, warm=False, gain=1.0,
                seed=1004, r0=0.15, L0=25.0, wfs=wfs, layers=layers, dms=_elt_dms(D, d))


def t1_mixed():
    """Small test geometry with mixed sensor sizes, LGS cone, an obstructed pupil and uneven layers."""
    D = 10.0
    wfs = [
        {"n_sub": 20, "theta_x": 0.7 * ARCMIN, "theta_y": 0.2 * ARCMIN, "gs_height": 90000.0, "sigma": 0.05},
        {"n_sub": 20, "theta_x": -0.5 * ARCMIN, "theta_y": 0.6 * ARCMIN, "gs_height": 90000.0, "sigma": 0.04},
        {"n_sub": 13, "theta_x": 0.1 * ARCMIN, "theta_y": -0.9 * ARCMIN, "gs_height": 0.0, "sigma": 0.08},
        {"n_sub": 5, "theta_x": -1.0 * ARCMIN, "theta_y": -0.3 * ARCMIN, "gs_height": 0.0, "sigma": 0.2},
    ]
    d = D / 20
    heights = [0.0, 2500.0, 7000.0, 13000.0]
    grids = {0.0: (64, d / 2), 2500.0: (32, d), 7000.0: (32, 0.6), 13000.0: (16, 2 * d)}
    layers = _layers(D, wfs, heights, _cn2(heights), lambda h: grids[h])
    dms = [{"height": 0.0, "n_act": 21, "pitch": d},
           {"height": 9000.0, "n_act": 12, "pitch": _dm_pitch(D, 9000.0, 12)}]
    return dict(name="t1_mixed",
                description="Test geometry: D=10 m, 28% obstruction, 2 LGS 20x20 + NGS 13x13 + NGS 5x5, "
                            "layers 64^2/32^2/32^2/16^2 (J=3), 2 DMs",
                D=D, obstruction=0.28, J=3, precision="fp64", n_iter=6, warm=True, gain=0.5,
                seed=1005, r0=0.15, L0=25.0, wfs=wfs, layers=layers, dms=dms)


def maory_paper():
    """The paper's own test configuration at the size of its first timed runs (Sec. 4.1,
    Table 2; Sec. 4.3: L = M = 6, 4 PCG iterations): D = 39 m, about 28 % obstructed, six LGS
    sensors of 80 x 80, one NGS of 2 x 2 and two of 1 x 1, LGS and NGS on 2' and 8/3' diameters,
    128^2 layer grids, DM 1 with 81^2 actuators, DMs 2-5 with 48^2 and DM 6 with 54^2.
    Readings for what the table leaves open: LGS at 90 km on a hexagon, NGS on a triangle at
    30/150/270 deg; layers at 0, 2.5, 5, 7.5, 10 and 15 km, 0.5 m spacing; DM 1 at 0 km with the
    subaperture pitch, DMs 2-6 at the layer heights 2.5-15 km covering the 1' field."""
    D = 39.0
    wfs = [dict(n_sub=80, theta_x=tx, theta_y=ty, gs_height=90000.0, sigma=0.05)
           for tx, ty in _ring(ARCMIN, [0, 60, 120, 180, 240, 300])]
    wfs += [dict(n_sub=ns, theta_x=tx, theta_y=ty, gs_height=0.0, sigma=0.05)
            for ns, (tx, ty) in zip((2, 1, 1), _ring(80 * ARCSEC, [30, 150, 270]))]
    heights = [0.0, 2500.0, 5000.0, 7500.0, 10000.0, 15000.0]
    layers = [dict(height=h, cn2_weight=g, n=128, spacing=0.5, flow=[1, 0]) for h, g in zip(heights, _cn2(heights))]
    dms = [dict(height=0.0, n_act=81, pitch=D / 80)]
    dms += [dict(height=h, n_act=48, pitch=_dm_pitch(D, h, 48)) for h in heights[1:5]]
    dms += [dict(height=heights[5], n_act=54, pitch=_dm_pitch(D, heights[5], 54))]
    return dict(name="maory_paper",
                description="the paper's MAORY-like test configuration, FP32: D=39 m (28% obstructed), 6 LGS 80x80 "
                            "+ NGS 2x2 + 2 NGS 1x1, L = M = 6 (128^2 grids, J=6), DMs 81^2/4x48^2/54^2, "
                            "4 warm PCG iterations",
                D=D, obstruction=0.28, J=6, precision="fp32", n_iter=4, warm=True, gain=1.0,
                seed=1006, r0=0.15, L0=25.0, wfs=wfs, layers=layers, dms=dms)


ALL = [c0_tiny, c1_elt_mcao, c3_mid_lgs, c4_stress, t1_mixed, maory_paper]


def main():
    for make in ALL:
        cfg = make()
        cfg["alpha_reg"] = ALPHA_REG[cfg["name"]]
        with open(os.path.join(HERE, cfg["name"] + ".json"), "w") as f:
            json.dump(cfg, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()

"""Per-frame time of the FP64 oracle on this host at one thread, at max(L, W) threads (the paper's
CPU scheme, Sec. 3.3) and at every core this process may use: median over 5 frames of the same
frame definition as the GPU metric (RHS + n_iter PCG iterations + fit), seeded synthetic slopes.

    python tests/oracle_timing.py c0_tiny c1_elt_mcao c4_stress
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from bench import host_cpu  # noqa: E402
from oracle import Oracle, get_threads, set_threads  # noqa: E402
from paper_2009_00946_amd import synth  # noqa: E402


def time_config(name, frames=5):
    cfg = synth.load_config(name)
    O = Oracle(cfg)
    S = [O.Ahat(synth.layer_screens_flat(cfg, f)) + O.slope_mask() * synth.slope_noise(cfg, f) for f in range(frames + 1)]
    n_iter, warm = cfg["n_iter"], cfg["warm"]
    model, cores = host_cpu()
    row = {"config": name, "host_cpu": model, "host_cores": cores, "n_iter": n_iter, "warm": warm}
    before = get_threads()
    try:
        for key, nt in (("single", 1), ("paper", max(len(cfg["layers"]), len(cfg["wfs"]))), ("all", cores)):
            set_threads(nt)
            N = O.n_coef
            c, bp, rp = np.zeros(N), np.zeros(N), np.zeros(N)
            c, bp, rp, _, _ = O.frame(S[0], c, bp, rp, n_iter, True)
            ts = []
            for f in range(1, frames + 1):
                t0 = time.perf_counter()
                c, bp, rp, _, _ = O.frame(S[f], c, bp, rp, n_iter, not warm)
                O.fit(c, None, cfg["gain"])
                ts.append(time.perf_counter() - t0)
            row[key + "_threads"] = nt
            row[key + "_ms"] = round(1e3 * float(np.median(ts)), 3)
            print("[oracle_timing] %s %s threads=%d %.3f ms" % (name, key, nt, row[key + "_ms"]), flush=True)
    finally:
        set_threads(before)
    return row


if __name__ == "__main__":
    for name in sys.argv[1:] or ["c0_tiny", "c1_elt_mcao"]:
        print(json.dumps(time_config(name)), flush=True)

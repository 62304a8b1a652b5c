"""Benchmark: per-frame FEWHA reconstruction on one MI355X.

One step = one tomographic frame of the hot path on the ELT MCAO configuration (9 guide
stars with 84x84 subapertures, 9 layers, J = 6, 3 DMs) in FP32: right-hand side, warm-restart
residual update, 4 PCG iterations (Alg. 2) and DM fitting with gain (Alg. 1), with slopes
already resident in HBM.  Slopes are synthetic: seeded von Karman layers (frozen flow over 16
frames) through the library's own forward operator plus white noise.

Prints one JSON line: ms per frame (median over the timed frames is reported beside the mean),
effective bandwidth of the algorithmic byte model against the 8 TB/s HBM peak, the roofline
object of the dominant kernel of a PCG pass (its algorithmic bytes per launch over its average
launch duration, timed live with HIP events on the launch stream), per-stage timings, and the
FP64 CPU oracle timed on a bounded sample of the same frames on the host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "ms per tomographic frame (fixed PCG iters) + effective HBM GB/s vs peak"


def footprint(cfg):
    """(sum_U, U_fit): layer nodes touched by any WFS interpolation stencil / by any fitting stencil."""
    sum_u, u_fit = 0, 0
    D = cfg["D"]
    heights = [d["height"] for d in cfg["dms"]]
    for li, lay in enumerate(cfg["layers"]):
        n, dl, h = lay["n"], lay["spacing"], lay["height"]
        mark = np.zeros((n, n), bool)
        for w in cfg["wfs"]:
            ns = w["n_sub"]
            x = -D / 2 + (D / ns) * np.arange(ns + 1)
            sig = 1 - h / w["gs_height"] if w["gs_height"] > 0 else 1.0
            u = (sig * x + w["theta_x"] * h) / dl + n / 2
            v = (sig * x + w["theta_y"] * h) / dl + n / 2
            l0 = np.minimum(np.floor(u).astype(int), n - 2)
            k0 = np.minimum(np.floor(v).astype(int), n - 2)
            for dk in (0, 1):
                for dj in (0, 1):
                    mark[np.ix_(k0 + dk, l0 + dj)] = True
        sum_u += int(mark.sum())
        m = int(np.argmin([abs(h - hd) + 1e-9 * hd for hd in heights]))
        dm = cfg["dms"][m]
        xa = (np.arange(dm["n_act"]) - (dm["n_act"] - 1) / 2) * dm["pitch"] / dl + n / 2
        a0 = np.minimum(np.floor(xa).astype(int), n - 2)
        fm = np.zeros((n, n), bool)
        for dk in (0, 1):
            for dj in (0, 1):
                fm[np.ix_(a0 + dk, a0 + dj)] = True
        u_fit += int(fm.sum())
    return sum_u, u_fit


def byte_model(cfg, elem_bytes, n_iter):
    """Algorithmic bytes per frame with stage-materialised intermediates (elements x size)."""
    n_c = sum(l["n"] ** 2 for l in cfg["layers"])
    sum_v = sum((w["n_sub"] + 1) ** 2 for w in cfg["wfs"])
    sum_s = sum(2 * w["n_sub"] ** 2 for w in cfg["wfs"])
    n_act = sum(d["n_act"] ** 2 for d in cfg["dms"])
    sum_u, u_fit = footprint(cfg)
    per_iter = 18 * n_c + sum_u + 4 * sum_v
    rhs = sum_s + 2 * sum_v + 7 * n_c
    fit = 2 * n_c + u_fit + n_act
    return {"per_iter": per_iter * elem_bytes, "rhs": rhs * elem_bytes, "fit": fit * elem_bytes,
            "frame": (n_iter * per_iter + rhs + fit) * elem_bytes,
            "n_coef": n_c, "sum_V": sum_v, "sum_S": sum_s, "sum_U": sum_u, "U_fit": u_fit}


# Kernels of one PCG pass that fewha_stage_launch enqueues on their own (stage "fwd" is the pair
# of forward-DWT launches, fine levels then coarse levels), with their algorithmic bytes per
# launch in elements: W^T J^-1 r (read r, write u) | P then Gamma^T C Gamma (read the layer
# footprints, the node grids through the slope stencil and back) | P^T (read v, write x) |
# W + alpha D z + dots + fused update.
# Per-reconstruction times the paper prints for its own test configuration (L = M = 6, 4 PCG
# iterations; Sec. 4.3), with their hardware: context for the same workload on this GPU.
PAPER_MS = {"maory_paper": {"cpu_ms": 3.0, "cpu": "2x Intel Xeon E5-2630v3 (8-core Haswell), OpenMP",
                            "gpu_ms": 8.6, "gpu": "NVIDIA Tesla V100-PCIE-32GB, CUDA 10.1"}}

STAGES = ("wt", "proj", "pt", "fwd")
STAGE_KERNELS = {"wt": "k_wt<pcg>", "proj": "k_proj<M>", "pt": "k_pt", "fwd": "k_fwd<pcg> + k_coarse<pcg>"}
STAGE_KERNELS_FOLD = dict(STAGE_KERNELS, wt="k_wt<fold> (coarse update folded in)", fwd="k_fwd<pcg> (fine levels)")
SINGLE_KERNEL = ("wt", "proj", "pt")


def stage_elements(model, fold=False):
    """Algorithmic elements per stage launch.  With the fold the coarse levels' share of the forward
    transform and update (their coefficients are 1/16 of the layer's with two fine levels) moves
    from the forward-DWT stage into the inverse-DWT stage; the pass total is unchanged."""
    n_c, sv, su = model["n_coef"], model["sum_V"], model["sum_U"]
    coarse = 15 * n_c / 16 if fold else 0
    return {"wt": 2 * n_c + coarse, "proj": su + 3 * sv, "pt": sv + n_c, "fwd": 15 * n_c - coarse}


def time_stages(P, stream, reps, replays=4):
    """Average device duration (us) of each stage launch: `reps` back-to-back launches captured in
    one HIP graph, replayed `replays` times between HIP events on the stream the plan launches on
    (each per-launch figure therefore includes the launch's share of the dispatch gaps)."""
    import torch
    out = {}
    cap = torch.cuda.Stream()
    for st in STAGES:
        for _ in range(5):
            P.stage_launch(st)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=cap):
            for _ in range(reps):
                P.stage_launch(st)
        torch.cuda.current_stream().wait_stream(cap)
        g.replay()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(replays + 1)]
        ev[0].record(stream)
        for i in range(replays):
            g.replay()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        out[st] = 1e3 * ev[0].elapsed_time(ev[-1]) / (replays * reps)
        del g
    return out


def source_digest():
    """SHA-256 over the kernel sources with comments and whitespace removed; recorded traffic is
    valid only for this digest (edits to comments keep it, edits to code do not)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.h", "fewha_internal.h"):
        with open(os.path.join(ROOT, "paper_2009_00946_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update(re.sub(r"\s+", "", src).encode())
    return h.hexdigest()


def recorded_traffic(kernel_stage, config):
    """HBM bytes per launch from the committed counter summary of this kernel and workload
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when absent or taken on other sources."""
    path = os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.md" % (kernel_stage, config))
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- `") and "`: " in line:
                key, val = line[3:].split("`: ", 1)
                rec[key] = val.strip()
    if rec.get("source_sha256") != source_digest():
        return None
    try:
        return float(rec["fetch_bytes_per_launch"]) + float(rec["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def h2d_upload(stream, s_dev, reps=200):
    """One frame's slopes uploaded from pinned host memory (timed on the launch stream).  The
    library takes device pointers, so this is reported beside the frame time, never in it."""
    import torch
    host = torch.empty(s_dev.numel(), dtype=s_dev.dtype, pin_memory=True)
    host.copy_(s_dev.cpu())
    dst = torch.empty_like(s_dev)
    for _ in range(5):
        dst.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(host, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    nbytes = s_dev.numel() * s_dev.element_size()
    return {"bytes": nbytes, "us_per_frame": round(us, 2), "GBps": round(nbytes / (us * 1e-6) / 1e9, 1)}


def copy_bandwidth(stream, nbytes=256 << 20, reps=20):
    """Device-to-device copy bandwidth of this GPU (bytes read + written per second), the
    achievable reference beside the 8 TB/s peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    gbps = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbps, 1)


def host_cpu():
    """Model name of the host CPU and the cores this process may use (its affinity, capped by
    OMP_NUM_THREADS when that is set)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    return model, cores


def cpu_baseline(cfg, frames_s, n_iter, budget_s):
    """The FP64 oracle (plain C; OpenMP over its layer and guide-star loops only) on host cores:
    ms per frame (median) on a bounded sample, at max(L, W) threads (the paper's CPU scheme,
    Sec. 3.3), with one thread and with every core this process may use beside it."""
    from oracle import Oracle, get_threads, set_threads
    model, all_cores = host_cpu()
    paper_threads = max(len(cfg["layers"]), len(cfg["wfs"]))
    before = get_threads()
    O = Oracle(cfg)
    N = O.n_coef
    out = {}
    try:
        for key, nt in (("paper", paper_threads), ("single", 1), ("all", all_cores)):
            set_threads(nt)
            c, bp, rp = np.zeros(N), np.zeros(N), np.zeros(N)
            c, bp, rp, _, _ = O.frame(frames_s[0], c, bp, rp, n_iter, cold=True)
            times = []
            t_all = time.perf_counter()
            f = 1
            while True:
                t0 = time.perf_counter()
                c, bp, rp, _, _ = O.frame(frames_s[f % len(frames_s)], c, bp, rp, n_iter, cold=False)
                O.fit(c, None, cfg["gain"])
                times.append(time.perf_counter() - t0)
                f += 1
                if time.perf_counter() - t_all > budget_s / 3 or f > 24:
                    break
            out[key] = (1e3 * float(np.median(times)), len(times), nt)
    finally:
        set_threads(before)
    ms, frames, nt = out["paper"]
    return {"value": round(ms, 3), "unit": "ms/frame", "cores": nt, "kind": "oracle",
            "sample": "%d warm frames of the same configuration (RHS + %d PCG iterations + fit) after a cold one, "
                      "FP64, median per frame, at max(L, W) = %d threads" % (frames, n_iter, nt),
            "host_cpu": model, "host_cores": all_cores,
            "single_thread_ms": round(out["single"][0], 3),
            "all_cores_ms": round(out["all"][0], 3), "all_cores": out["all"][2]}


# The batched uneven workload: 64 independent FP32 frames of three geometries, 4 PCG passes each,
# warm chains.  Each geometry is one batched plan (one launch per stage over all its frames).
# (geometry, frames, guide stars, batched plans the frames are dealt to: one stream each)
C3_GROUPS = (("c0_tiny", 32, "all guide stars", 1), ("c3_mid_lgs", 24, "all guide stars", 1),
             ("c1_elt_mcao", 8, "LGS only", 2))


def c3_configs():
    """(configuration, frames) of every batched plan of the uneven mix: a geometry whose frames are
    dealt to k plans contributes k entries (the ELT-LGS frames run as two 4-frame batches on two
    streams: 0.620 -> 0.579 ms per 64 frames; more than four streams in all was slower)."""
    import copy
    from paper_2009_00946_amd import synth
    out = []
    for name, count, which, plans in C3_GROUPS:
        cfg = copy.deepcopy(synth.load_config(name + ("_lgs" if which == "LGS only" else "")))
        cfg["precision"], cfg["n_iter"], cfg["warm"] = "fp32", 4, True
        out += [(cfg, count // plans)] * plans
    return out


def c3_description():
    return "c3_batched_uneven: " + ", ".join(
        "%d x %s (%s%s)" % (count, name + ("_lgs" if which == "LGS only" else ""), which,
                            ", %d plans of %d frames" % (plans, count // plans) if plans > 1 else "")
        for name, count, which, plans in C3_GROUPS)


def batch_slopes(P1, cfg, count, first=0):
    """[count][n_slopes] seeded synthetic slopes (frozen-flow frames first .. first + count - 1
    through the plan's own forward operator, plus white noise), resident in HBM."""
    import torch
    from paper_2009_00946_amd import synth
    S = []
    for f in range(first, first + count):
        phi = torch.as_tensor(synth.layer_screens_flat(cfg, f), dtype=P1.dtype, device=P1.device)
        s = P1.apply_A(P1.dwt_forward(phi))
        s += torch.as_tensor(synth.slope_noise(cfg, f), dtype=P1.dtype, device=P1.device)
        S.append(s)
    return torch.stack(S).contiguous()


def capture(fn, warm_steps=3):
    """fn(warm) once cold and warm_steps times warm, then one warm call captured in a HIP graph."""
    import torch
    fn(warm=False)
    for _ in range(warm_steps):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=cap):
        fn()
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    return g


def time_graphs(graphs, steps, warmup):
    """ms per replay of the graph sequence graphs[k % len(graphs)], k = 0..steps-1."""
    import torch
    for k in range(warmup):
        graphs[k % len(graphs)].replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        graphs[k % len(graphs)].replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_stages_batch(P, nb, stream, reps=20, replays=4):
    """Average device duration (us) of each stage launch over nb frames (see time_stages)."""
    import torch
    out = {}
    cap = torch.cuda.Stream()
    for st in STAGES:
        for _ in range(3):
            P.stage_launch_batch(st, nb)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=cap):
            for _ in range(reps):
                P.stage_launch_batch(st, nb)
        torch.cuda.current_stream().wait_stream(cap)
        g.replay()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(replays + 1)]
        ev[0].record(stream)
        for i in range(replays):
            g.replay()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        out[st] = 1e3 * ev[0].elapsed_time(ev[-1]) / (replays * reps)
        del g
    return out


def roofline_of(cfg, us, frames, n_iter, elem=4, fold=False):
    """Roofline object of the dominant single kernel of a PCG pass (launches per frame x duration)
    of a launch over `frames` frames of one geometry."""
    sel = stage_elements(byte_model(cfg, elem, n_iter), fold)
    per_frame = {"wt": n_iter, "proj": n_iter, "pt": n_iter + 1, "fwd": n_iter}
    dom = max(SINGLE_KERNEL + (("fwd",) if fold else ()), key=lambda st: per_frame[st] * us[st])
    nbytes = int(sel[dom] * elem * frames)
    ach = nbytes / (us[dom] * 1e-6) / 1e9
    names = STAGE_KERNELS_FOLD if fold else STAGE_KERNELS
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": names[dom],
            "us_per_launch": round(us[dom], 3), "bytes_per_launch": nbytes, "frames_per_launch": frames}


def batched_same_geometry(cfg, nb, steps, warmup, refresh=8, tuned=True):
    """nb frames of one geometry per launch (RHS + n_iter warm PCG passes + fit each, residual
    refreshed every `refresh`-th step): us per frame, effective GB/s and the roofline object of the
    batched launch's dominant kernel."""
    import torch
    from paper_2009_00946_amd import fewha, tune
    n_iter, gain = cfg["n_iter"], cfg["gain"]
    PB = fewha.Plan(cfg, max_batch=nb)
    shapes = tune.tuned(PB) if tuned else None
    P1 = fewha.Plan(cfg)
    sb = batch_slopes(P1, cfg, nb)
    del P1
    cb = torch.zeros((nb, PB.n_coef), dtype=PB.dtype, device=PB.device)
    ab = torch.zeros((nb, PB.n_act), dtype=PB.dtype, device=PB.device)

    def step(warm=True, fresh=False):
        PB.reconstruct_batch(sb, cb, n_iter, gain=gain, out=ab, warm=warm, refresh=fresh and warm)

    g_warm = capture(step)
    g_fresh = capture(lambda warm=True: step(warm, fresh=True), warm_steps=0) if refresh else None
    seq = [g_fresh] + [g_warm] * (refresh - 1) if refresh else [g_warm]
    ms = time_graphs(seq, max(steps // 8, 2 * len(seq)), warmup)
    assert PB.last_status_batch(nb) == [0] * nb
    elem = 4 if PB.precision == "fp32" else 8
    model = byte_model(cfg, elem, n_iter)
    us = time_stages_batch(PB, nb, torch.cuda.current_stream())
    gbps = model["frame"] * nb / (ms * 1e-3) / 1e9
    out = {"workload": "%s, %d frames per launch" % (cfg["name"], nb), "frames_per_launch": nb,
           "ms_per_launch_set": round(ms, 4), "us_per_frame": round(1e3 * ms / nb, 2),
           "frames_per_s": round(1e3 * nb / ms, 1), "effective_GBps": round(gbps, 1),
           "frac_hbm_peak": round(gbps / HBM_PEAK_GBPS, 4), "residual_refresh_every": refresh or None,
           "roofline": roofline_of(cfg, us, nb, n_iter, elem, PB.get_tuning()["fold"] == 1),
           "stages_us_per_launch": {k: round(v, 3) for k, v in us.items()},
           "launch_shapes": shapes and shapes["tuning"]}
    del PB, sb, cb, ab, g_warm, g_fresh, seq
    torch.cuda.empty_cache()
    return out


class UnevenMix:
    """The batched uneven workload: 64 FP32 frames of three geometries, 4 warm PCG passes and the
    fit each; each geometry's frames in batched plans (one launch per stage over all of a plan's
    frames; the ELT-LGS frames in two plans), the plans on streams of their own, forked and joined
    inside one HIP graph."""

    def __init__(self, with_single=False, tuned=True):
        import torch
        from paper_2009_00946_amd import fewha, tune
        self.groups = []
        first = {}  # a geometry's plans take consecutive synthetic frames
        for cfg, count in c3_configs():
            PB = fewha.Plan(cfg, max_batch=count)
            if tuned:
                tune.tuned(PB)
            P1 = fewha.Plan(cfg)
            f0 = first.get(cfg["name"], 0)
            first[cfg["name"]] = f0 + count
            sb = batch_slopes(P1, cfg, count, f0)
            g = dict(cfg=cfg, count=count, PB=PB, sb=sb,
                     cb=torch.zeros((count, PB.n_coef), dtype=PB.dtype, device=PB.device),
                     ab=torch.zeros((count, PB.n_act), dtype=PB.dtype, device=PB.device))
            if with_single:
                g.update(P1=P1, c1=P1.zeros(P1.n_coef), a1=P1.zeros(P1.n_act))
            self.groups.append(g)
        self.streams = [torch.cuda.Stream() for _ in self.groups]  # default priority
        self.n_iter = 4

    def batched(self, warm=True, fresh=False):
        for g in self.groups:
            g["PB"].reconstruct_batch(g["sb"], g["cb"], self.n_iter, gain=1.0, out=g["ab"], warm=warm,
                                      refresh=fresh and warm)

    def concurrent(self, warm=True, fresh=False):
        # the three batched plans on streams of their own (fork and join by events): no data is
        # shared, so the small geometries fill what the large one leaves idle
        import torch
        main = torch.cuda.current_stream()
        for g, s in zip(self.groups, self.streams):
            s.wait_stream(main)
            with torch.cuda.stream(s):
                g["PB"].reconstruct_batch(g["sb"], g["cb"], self.n_iter, gain=1.0, out=g["ab"], warm=warm,
                                          refresh=fresh and warm)
        for s in self.streams:
            main.wait_stream(s)

    def single(self, warm=True):
        for g in self.groups:
            for f in range(g["count"]):
                g["P1"].reconstruct(g["sb"][f], g["c1"], self.n_iter, gain=1.0, out=g["a1"], warm=warm)

    @property
    def frames(self):
        return sum(g["count"] for g in self.groups)

    def batch_bytes(self):
        return sum(byte_model(g["cfg"], 4, self.n_iter)["frame"] * g["count"] for g in self.groups)

    def check(self):
        for g in self.groups:
            assert g["PB"].last_status_batch(g["count"]) == [0] * g["count"]

    def roofline(self):
        """The dominant single kernel of the mix: the largest launches-per-batch x duration over the
        plans' batched stage launches."""
        import torch
        best = None
        for g in self.groups:
            us = time_stages_batch(g["PB"], g["count"], torch.cuda.current_stream())
            fold = g["PB"].get_tuning()["fold"] == 1
            r = roofline_of(g["cfg"], us, g["count"], self.n_iter, 4, fold)
            names = STAGE_KERNELS_FOLD if fold else STAGE_KERNELS
            per_frame = {names["wt"]: self.n_iter, names["proj"]: self.n_iter, names["pt"]: self.n_iter + 1,
                         names["fwd"]: self.n_iter}
            cost = per_frame[r["kernel"]] * r["us_per_launch"]
            if best is None or cost > best[0]:
                best = (cost, dict(r, geometry=g["cfg"]["name"]))
        return best[1]


def uneven_mix_summary(steps, warmup, refresh=8, tuned=True):
    mix = UnevenMix(tuned=tuned)
    g_warm = capture(mix.concurrent)
    g_fresh = capture(lambda warm=True: mix.concurrent(warm, fresh=True), warm_steps=0)
    ms = time_graphs([g_fresh] + [g_warm] * (refresh - 1), max(steps // 8, 2 * refresh), warmup)
    mix.check()
    gbps = mix.batch_bytes() / (ms * 1e-3) / 1e9
    out = {"workload": c3_description(), "frames": mix.frames, "ms_per_batch": round(ms, 4), "us_per_frame": round(1e3 * ms / mix.frames, 2),
        "effective_GBps": round(gbps, 1), "frac_hbm_peak": round(gbps / HBM_PEAK_GBPS, 4),
        "residual_refresh_every": refresh, "launch": "hip_graph_per_batch, one stream per batched plan",
        "roofline": mix.roofline()}
    del mix, g_warm, g_fresh
    return out


def c3_batch(args):
    """ms per batch of 64 uneven frames: each geometry's frames in one batched plan, the three
    plans on streams of their own in one HIP graph; beside it the same batched plans on one
    stream, and the same frames one at a time."""
    import torch
    torch.cuda.set_device(0)
    mix = UnevenMix(with_single=True)
    gb = capture(mix.batched)
    ms_seq = time_graphs([gb], args.steps, args.warmup)
    gc = capture(mix.concurrent)
    ms_b = time_graphs([gc], args.steps, args.warmup)
    mix.check()
    gs = capture(mix.single)
    ms_s = time_graphs([gs], max(args.steps // 10, 5), args.warmup)
    total_bytes = mix.batch_bytes()
    frames = mix.frames
    gbps = total_bytes / (ms_b * 1e-3) / 1e9
    out = {
        "metric": "ms per batch of 64 uneven frames (fixed PCG iters) + effective HBM GB/s vs peak",
        "value": round(ms_b, 5), "unit": "ms/batch", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_b, 5), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": c3_description(),
            "n_iter": mix.n_iter, "warm": True, "frames": frames,
            "launch": "hip_graph_per_batch, one stream per batched plan"},
        "ms_per_frame": round(ms_b / frames, 5),
        "bytes_per_batch": total_bytes,
        "effective_GBps": round(gbps, 1),
        "frac_hbm_peak": round(gbps / HBM_PEAK_GBPS, 4),
        "batched_one_stream_ms_per_batch": round(ms_seq, 5),
        "unbatched_ms_per_batch": round(ms_s, 5),
        "batching_speedup": round(ms_s / ms_b, 2),
        "roofline": mix.roofline(),
    }
    print(json.dumps(out), flush=True)


def batch_scan(args):
    """Throughput of the ELT frame against the number of frames per launch (one batched plan per
    size; RHS + 4 warm PCG passes + fit per frame, residual refreshed every 8th step, HIP graphs)."""
    import torch
    from paper_2009_00946_amd import synth
    torch.cuda.set_device(0)
    cfg = synth.load_config(args.config)
    rows = []
    for nb in (1, 2, 4, 8, 16, 32, 64, 128):
        r = batched_same_geometry(cfg, nb, max(args.steps // nb, 64), args.warmup)
        rows.append(r)
        print("[batch_scan] %s" % json.dumps(r), flush=True)
    out = {"metric": "ELT frame throughput against frames per launch (batched plans)", "value": rows[-1]["us_per_frame"],
           "unit": "us/frame", "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "%s batched" % cfg["name"], "n_iter": cfg["n_iter"], "warm": True}, "scan": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c1_elt_mcao")
    ap.add_argument("--frames", type=int, default=16, help="distinct synthetic slope frames (cycled)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle CPU time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched forms beside the single frame")
    ap.add_argument("--no-tune", action="store_true", help="default launch shapes instead of the autotuner's")
    ap.add_argument("--batch", type=int, default=32, help="frames per launch of the same-geometry batched form")
    ap.add_argument("--refresh", type=int, default=8,
                    help="FP32: recompute the residual as b - M c every this many frames (0: always carried)")
    ap.add_argument("--eager", action="store_true", help="launch kernels one by one instead of replaying HIP graphs")
    ap.add_argument("--stage-reps", type=int, default=50, help="launches per PCG-pass stage in its timing graph")
    ap.add_argument("--workload", default="frame", choices=("frame", "c3_batch", "batch_scan", "batched"),
                    help="frame: the ELT frame (default); c3_batch: 64 uneven frames in batched launches; "
                         "batch_scan: ELT frames per second against frames per launch; batched: only the "
                         "batched forms of the default line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain 256 MiB device copies (reference dispatches for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs the hot path on one GPU; multi-GPU runs are not provided "
              "(frames would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3_batch":
        c3_batch(args)
        return
    if args.workload == "batch_scan":
        batch_scan(args)
        return
    if args.workload == "batched":
        import torch
        from paper_2009_00946_amd import synth
        torch.cuda.set_device(0)
        cfg = synth.load_config(args.config)
        out = {"same_geometry": batched_same_geometry(cfg, args.batch, args.steps, args.warmup, args.refresh,
                                                      tuned=not args.no_tune),
               "uneven_64": uneven_mix_summary(args.steps, args.warmup, tuned=not args.no_tune)}
        print(json.dumps(out), flush=True)
        return

    import torch
    from paper_2009_00946_amd import fewha, synth, tune

    torch.cuda.set_device(0)
    cfg = synth.load_config(args.config)
    n_iter, gain = cfg["n_iter"], cfg["gain"]
    P = fewha.Plan(cfg)
    tuning = None if args.no_tune else tune.tuned(P)
    stream = torch.cuda.current_stream()

    # synthetic frames, resident on the device before timing
    S, S_host = [], []
    for f in range(args.frames):
        phi = torch.as_tensor(synth.layer_screens_flat(cfg, f), dtype=P.dtype, device=P.device)
        s = P.apply_A(P.dwt_forward(phi))
        s += torch.as_tensor(synth.slope_noise(cfg, f), dtype=P.dtype, device=P.device)
        S.append(s)
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        S_host = [s.double().cpu().numpy() for s in S]

    c = P.zeros(P.n_coef)
    a = P.zeros(P.n_act)

    # every args.refresh-th warm frame recomputes its residual as b - M c (FP32 drift control; the
    # frame graphs cycle through len(S) frames, a multiple of the period)
    if P.precision != "fp32":
        args.refresh = 0
    if args.refresh and len(S) % args.refresh:
        sys.exit("bench.py: --frames must be a multiple of --refresh")

    def frame(k, warm=True):
        fresh = warm and args.refresh > 0 and k % args.refresh == 0
        P.reconstruct(S[k % len(S)], c, n_iter, a_prev=a, gain=gain, out=a, warm=warm, refresh=fresh)

    frame(0, warm=False)
    for k in range(1, args.warmup):
        frame(k)
    torch.cuda.synchronize()
    assert P.last_status() == 0, fewha.STATUS.get(P.last_status())
    run = frame
    graphs = []
    if not args.eager:
        # one HIP graph per synthetic frame (same launches, its own slope buffer): a replay is
        # one whole frame, RHS + PCG + fitting, with no host work between kernels
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        for f in range(len(S)):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                frame(f)
            graphs.append(g)
        torch.cuda.current_stream().wait_stream(cap)
        torch.cuda.synchronize()

        def run(k, warm=True):
            graphs[k % len(graphs)].replay()

        for k in range(len(S)):
            run(k)
        torch.cuda.synchronize()
        assert P.last_status() == 0, fewha.STATUS.get(P.last_status())

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(args.steps):
        run(args.warmup + k)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    total_ms = ev[0].elapsed_time(ev[-1])
    assert P.last_status() == 0
    ms_mean = total_ms / args.steps

    elem = 4 if P.precision == "fp32" else 8
    model = byte_model(cfg, elem, n_iter)
    eff_gbps = model["frame"] / (ms_mean * 1e-3) / 1e9

    # the dominant single kernel of a PCG pass, timed live (launches per frame x duration)
    us = time_stages(P, stream, args.stage_reps)
    fold = P.get_tuning()["fold"] == 1
    names = STAGE_KERNELS_FOLD if fold else STAGE_KERNELS
    sel = stage_elements(model, fold)
    per_frame = {"wt": n_iter, "proj": n_iter, "pt": n_iter + 1, "fwd": n_iter}
    stages = {st: {"kernel": names[st], "us_per_launch": round(us[st], 3),
                   "bytes_per_launch": int(sel[st] * elem), "launches_per_frame": per_frame[st],
                   "GBps": round(sel[st] * elem / (us[st] * 1e-6) / 1e9, 1)} for st in STAGES}
    dom = max(SINGLE_KERNEL + (("fwd",) if fold else ()), key=lambda st: per_frame[st] * us[st])
    achieved = sel[dom] * elem / (us[dom] * 1e-6) / 1e9
    traffic = recorded_traffic(dom, cfg["name"])
    h2d = h2d_upload(stream, S[0])
    copy_gbps = copy_bandwidth(stream)
    if args.copy_calibration:
        import torch
        src = torch.empty(64 << 20, dtype=torch.float32, device=P.device).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = {
        "metric": METRIC,
        "value": round(ms_mean, 5),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_mean, 5),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if P.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (cfg["name"], cfg["description"]), "n_iter": n_iter, "warm": True,
                   "gain": gain, "n_coef": model["n_coef"], "n_slopes": P.n_slopes, "n_act": P.n_act,
                   "launch": ("eager" if args.eager else "hip_graph_per_frame") + " (fewha_reconstruct: solve and fit in one call)",
                   "residual_refresh_every": args.refresh or None,
                   "launch_shapes": tuning and dict(tuning["tuning"], autotuned=not tuning["cached"])},
        "ms_median": round(float(np.median(per)), 5),
        "ms_p99": round(float(np.percentile(per, 99)), 5),
        "frames_per_s": round(1e3 / ms_mean, 1),
        "effective_GBps": round(eff_gbps, 1),
        "frac_hbm_peak": round(eff_gbps / HBM_PEAK_GBPS, 4),
        "bytes_per_frame": model["frame"],
        "copy_GBps": copy_gbps,
        "frac_of_copy_bw": round(eff_gbps / copy_gbps, 4),
        "h2d": h2d,
        "ms_per_frame_with_h2d": round(ms_mean + h2d["us_per_frame"] * 1e-3, 5),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": names[dom], "us_per_launch": round(us[dom], 3),
                     "bytes_per_launch": int(sel[dom] * elem)},
        "stages": stages,
    }
    if cfg["name"] in PAPER_MS:
        # the paper times this very workload (other hardware): value / its faster platform
        ref = PAPER_MS[cfg["name"]]
        out["vs_baseline"] = round(ms_mean / ref["cpu_ms"], 5)
        out["paper_context"] = ref
    if not args.no_batched and P.precision == "fp32":
        # the bandwidth regime beside the single frame: frames of this geometry batched into every
        # launch, and the uneven 64-frame mix
        del graphs
        torch.cuda.synchronize()
        out["batched"] = {"same_geometry": batched_same_geometry(cfg, args.batch, args.steps, args.warmup, args.refresh,
                                                                 tuned=not args.no_tune),
                          "uneven_64": uneven_mix_summary(args.steps, args.warmup, tuned=not args.no_tune)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, S_host, n_iter, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

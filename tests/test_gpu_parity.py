"""GPU parity: every C-ABI call against the FP64 oracle on identical seeded inputs.

Tolerances (relative to the reference vector's largest magnitude, checked element by element,
plus the norm-wise relative error):
  FP64 plans: operators 1e-12, solver iterates 1e-9;
  FP32 plans: operators 1e-5, reconstructed layers W^T c 1e-4 per frame (FP32 storage, FP64
  reductions), the bound the method's spec target states.
Inputs: seeded von Karman layers / noise from ``synth`` and N(0,1) vectors; slopes are made by
the oracle (s = Ahat(phi) + mask * noise), never by the GPU.
"""
import numpy as np
import pytest

from paper_2009_00946_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_plans, _oracles = {}, {}


def plan(name, prec):
    _need_gpu()
    from paper_2009_00946_amd import fewha
    key = (name, prec)
    if key not in _plans:
        print("\n[bind] %s %s" % key, flush=True)
        _plans[key] = fewha.Plan(synth.load_config(name), precision=prec)
    return _plans[key]


def oracle(name):
    from oracle import Oracle
    if name not in _oracles:
        _oracles[name] = Oracle(synth.load_config(name))
    return _oracles[name]


def dev(P, x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=P.dtype, device=P.device)


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def check(got, ref, tol, what=""):
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, what
    assert np.all(np.isfinite(got)), what + ": non-finite output"
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    nrm = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    assert err <= tol and nrm <= tol, "%s: max-rel %.3e norm-rel %.3e > %.1e" % (what, err, nrm, tol)
    return err


OPS_CASES = [("t1_mixed", "fp64", 1e-12), ("c0_tiny", "fp64", 1e-12), ("t1_mixed", "fp32", 1e-5),
             ("c1_elt_mcao", "fp32", 1e-5), ("c3_mid_lgs", "fp32", 1e-5)]


@pytest.mark.parametrize("name,prec,tol", OPS_CASES)
def test_dwt_parity(name, prec, tol):
    P, O = plan(name, prec), oracle(name)
    x = synth.normal_vector(O.n_coef, 11)
    c_ref = O.W(x)
    c = P.dwt_forward(dev(P, x))
    check(host(c), c_ref, tol, "W")
    xr = P.dwt_inverse(dev(P, c_ref))
    check(host(xr), O.Wt(c_ref), tol, "W^T")
    check(host(P.dwt_inverse(c)), x, 4 * tol, "W^T W")


@pytest.mark.parametrize("name,prec,tol", OPS_CASES)
def test_operator_parity(name, prec, tol):
    P, O = plan(name, prec), oracle(name)
    c = synth.normal_vector(O.n_coef, 21)
    s = synth.normal_vector(O.n_slopes, 22)
    check(host(P.apply_A(dev(P, c))), O.A(c), tol, "A")
    check(host(P.apply_At(dev(P, s))), O.At(s), tol, "A^T")
    check(host(P.apply_M(dev(P, c))), O.M(c), tol, "M")


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_stress_config_operator_parity(prec, tol):
    """35 layers up to 512^2 and J = 7 (the coarse forward levels of the largest layers read their
    input from global memory): W, W^T, A, A^T and M against the oracle."""
    from oracle import Oracle
    P = plan("c4_stress", prec)
    if "c4_stress/noprecond" not in _oracles:
        _oracles["c4_stress/noprecond"] = Oracle(synth.load_config("c4_stress"), precond=False)
    O = _oracles["c4_stress/noprecond"]
    x = synth.normal_vector(O.n_coef, 31)
    check(host(P.dwt_forward(dev(P, x))), O.W(x), tol, "W")
    check(host(P.dwt_inverse(dev(P, x))), O.Wt(x), tol, "W^T")
    s = synth.normal_vector(O.n_slopes, 32)
    check(host(P.apply_A(dev(P, x))), O.A(x), tol, "A")
    check(host(P.apply_At(dev(P, s))), O.At(s), tol, "A^T")
    check(host(P.apply_M(dev(P, x))), O.M(x), tol, "M")


@pytest.mark.parametrize("name,prec,tol", [("t1_mixed", "fp64", 1e-12), ("c0_tiny", "fp64", 1e-12),
                                           ("c1_elt_mcao", "fp32", 2e-5)])
def test_precond_table_parity(name, prec, tol):
    P, O = plan(name, prec), oracle(name)
    tab = P.precond_table()
    jd = O.precond()
    cfg = synth.load_config(name)
    from oracle.oracle import level_of
    off = 0
    for l, lay in enumerate(cfg["layers"]):
        n, J = lay["n"], cfg["J"]
        for s in range(1, J + 1):
            for o in range(4):
                if o == 0 and s != J:
                    continue
                m = n >> s
                r = (m if o in (2, 3) else 0) + m // 2
                q = (m if o in (1, 3) else 0) + m // 2
                assert level_of(n, J, r, q) == (s, o)
                ref = jd[off + r * n + q]
                assert abs(tab[l, s, o] - ref) <= tol * ref, (l, s, o, tab[l, s, o], ref)
        off += n * n


def test_gpu_adjointness_fp64():
    P = plan("t1_mixed", "fp64")
    rng = np.random.default_rng(3)
    c, s = rng.standard_normal(P.n_coef), rng.standard_normal(P.n_slopes)
    lhs = float(np.dot(host(P.apply_A(dev(P, c))), s))
    rhs = float(np.dot(c, host(P.apply_At(dev(P, s)))))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    y = rng.standard_normal(P.n_coef)
    lhs = float(np.dot(host(P.apply_M(dev(P, c))), y))
    rhs = float(np.dot(c, host(P.apply_M(dev(P, y)))))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _slopes(O, cfg, frame):
    return O.Ahat(synth.layer_screens_flat(cfg, frame)) + O.slope_mask() * synth.slope_noise(cfg, frame)


# FP32 refresh period of the long chains: every REFRESH-th warm frame recomputes its residual as
# b - M c.  Carried alone, the FP32 residual drifts from b - M c by about 1e-7 of |b| per frame
# (the rounding of each c update is invisible to the recurrence), and on the ELT geometry the
# layers then leave the 1e-4 bound after about 19 frames; refreshed every 8 frames they stay
# below 7e-5 over 64 frames (and below 7e-6 when refreshed every frame).
REFRESH = 8


@pytest.mark.parametrize("name,prec,frames,tol_c,tol_layers,refresh", [
    ("c0_tiny", "fp64", 2, 1e-9, 1e-9, 0),
    ("t1_mixed", "fp64", 4, 1e-9, 1e-9, 0),
    ("t1_mixed", "fp32", 4, 1e-3, 1e-4, 0),
    ("c3_mid_lgs", "fp32", 4, 1e-3, 1e-4, 0),
    # the ELT configuration carried alone over 8 frames, then its first 64 frames with the residual
    # refreshed every REFRESH frames, and the laser-guide-star-only member of the batched mix
    ("c1_elt_mcao", "fp32", 8, 1e-3, 1e-4, 0),
    pytest.param("c1_elt_mcao", "fp32", 64, 1e-3, 1e-4, REFRESH, marks=pytest.mark.timeout(600)),
    ("c1_elt_mcao_lgs", "fp32", 8, 1e-3, 1e-4, 0),
])
def test_frame_chain_parity(name, prec, frames, tol_c, tol_layers, refresh):
    """Alg. 1 frames chained by warm restart (cold first frame), GPU vs oracle after every frame.
    With ``refresh`` every refresh-th warm frame recomputes its residual as b - M c (equal to the
    carried residual in exact arithmetic, so the oracle's chain stays the carried one)."""
    P, O = plan(name, prec), oracle(name)
    cfg = synth.load_config(name)
    n_iter, warm = cfg["n_iter"], cfg["warm"]
    N = O.n_coef
    c_ref, bp, rp = np.zeros(N), np.zeros(N), np.zeros(N)
    c_gpu = P.zeros(N)
    res = torch.zeros(n_iter, dtype=torch.float64, device=P.device)
    for f in range(frames):
        print("[frame] %s %s %d" % (name, prec, f), flush=True)
        s = _slopes(O, cfg, f)
        cold = (f == 0) or not warm
        c_ref, bp, rp, res_ref, st = O.frame(s, c_ref, bp, rp, n_iter, cold)
        assert st == 0
        fresh = bool(refresh) and not cold and f % refresh == 0
        P.pcg_solve(dev(P, s), c_gpu, n_iter, warm=not cold, resnorm=res, refresh=fresh)
        assert P.last_status() == 0
        e_c = check(host(c_gpu), c_ref, tol_c, "c frame %d" % f)
        e_l = check(host(P.dwt_inverse(c_gpu)), O.Wt(c_ref), tol_layers, "layers frame %d" % f)
        check(host(res), res_ref, max(tol_c, 1e-6) if prec == "fp32" else 1e-9, "resnorm frame %d" % f)
        b_g, r_g = P.state_get()
        check(host(b_g), bp, 1e-5 if prec == "fp32" else 1e-12, "b_prev frame %d" % f)
        print("[frame] %s %s %d: c %.2e layers %.2e" % (name, prec, f, e_c, e_l), flush=True)


def test_deep_fold_chain_parity():
    """The ELT geometry taken to J = 7 (the 128 x 128 layers to their 1 x 1 level): the folded
    inverse DWT then runs its deep form (level loops and cone bounds for up to 12 levels instead
    of 6).  Two chained frames (cold, then warm) against the oracle, with the fold and without it,
    held as the stress configuration's FP32 run is: every wavelet level but the coarsest and what
    the sensors see within 1e-4.  The coarsest level holds the 128 x 128 layers' piston, fixed by
    the prior alone, where FP32 rounding becomes an O(1) error: the cold frame is held under the
    stress configuration's ceiling of 1.0 and the warm frame's (which grows with the warm restart:
    measured 3.1 with the fold and 1.8 without, the other levels within 5e-6 either way) is
    reported."""
    _need_gpu()
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    from tests.precision_study import level_masks
    cfg = synth.load_config("c1_elt_mcao")
    cfg["J"] = 7
    O = Oracle(cfg)
    n_iter, N = cfg["n_iter"], O.n_coef
    masks = level_masks(cfg)
    refs = []
    c_ref, bp, rp = np.zeros(N), np.zeros(N), np.zeros(N)
    for f in range(2):
        s = _slopes(O, cfg, f)
        c_ref, bp, rp, _, st = O.frame(s, c_ref, bp, rp, n_iter, f == 0)
        assert st == 0
        refs.append((s, c_ref.copy(), O.A(c_ref)))
    for fold in (1, 0):
        P = fewha.Plan(cfg, precision="fp32")
        assert P.get_tuning()["fold"] == 1
        P.set_tuning(dict(P.get_tuning(), fold=fold))
        c_gpu = P.zeros(N)
        for f, (s, c_ref, a_ref) in enumerate(refs):
            P.pcg_solve(dev(P, s), c_gpu, n_iter, warm=f > 0)
            assert P.last_status() == 0
            ch = host(c_gpu)
            by_level = [float(np.linalg.norm(ch[m] - c_ref[m]) / max(np.linalg.norm(c_ref[m]), 1e-300)) for m in masks]
            vis = float(np.linalg.norm(O.A(ch) - a_ref) / np.linalg.norm(a_ref))
            print("[frame] c1_elt_mcao J=7 fold=%d %d: levels %s, visible %.2e" % (fold, f, ["%.1e" % e for e in by_level], vis),
                  flush=True)
            assert max(by_level[:-1]) <= 1e-4 and vis <= 1e-4, (fold, f, by_level, vis)
            if f == 0:
                assert by_level[-1] <= 1.0, (fold, f, by_level)


@pytest.mark.parametrize("name,prec,tol", [("t1_mixed", "fp64", 1e-12), ("c1_elt_mcao", "fp32", 1e-5),
                                           ("c0_tiny", "fp64", 1e-12)])
def test_fit_parity(name, prec, tol):
    P, O = plan(name, prec), oracle(name)
    c = synth.normal_vector(O.n_coef, 31)
    a_prev = synth.normal_vector(O.n_act, 32)
    check(host(P.fit_dm(dev(P, c))), O.fit(c, None, 1.0), tol, "fit gain 1")
    check(host(P.fit_dm(dev(P, c), dev(P, a_prev), 0.5)), O.fit(c, a_prev, 0.5), tol, "fit gain 0.5")


def test_outputs_fully_overwritten():
    """NaN-poisoned outputs must come back finite: every element is written."""
    P = plan("t1_mixed", "fp32")
    c = dev(P, synth.normal_vector(P.n_coef, 41))
    s = dev(P, synth.normal_vector(P.n_slopes, 42))
    for fn, arg, n in ((P.apply_A, c, P.n_slopes), (P.apply_At, s, P.n_coef), (P.apply_M, c, P.n_coef),
                       (P.dwt_forward, c, P.n_coef), (P.dwt_inverse, c, P.n_coef), (P.fit_dm, c, P.n_act)):
        out = torch.full((n,), float("nan"), dtype=P.dtype, device=P.device)
        fn(arg, out=out)
        assert torch.isfinite(out).all().item(), fn.__name__


def test_bitwise_deterministic():
    P = plan("c1_elt_mcao", "fp32")
    O = oracle("c1_elt_mcao")
    s = dev(P, _slopes(O, synth.load_config("c1_elt_mcao"), 0))
    outs = []
    for _ in range(2):
        c = P.zeros(P.n_coef)
        P.pcg_solve(s, c, 4, warm=False)
        outs.append(host(c))
    assert np.array_equal(outs[0], outs[1])


def test_state_roundtrip_split_chain():
    """A warm chain split after frame 2 and resumed from saved state is bitwise identical."""
    P = plan("t1_mixed", "fp32")
    O = oracle("t1_mixed")
    cfg = synth.load_config("t1_mixed")
    S = [dev(P, _slopes(O, cfg, f)) for f in range(4)]
    c = P.zeros(P.n_coef)
    saved = None
    for f in range(4):
        P.pcg_solve(S[f], c, 6, warm=f > 0)
        if f == 1:
            saved = (c.clone(),) + P.state_get()
    full = host(c)
    c2 = saved[0].clone()
    P.pcg_solve(S[0], P.zeros(P.n_coef), 3, warm=False)   # clobber the state
    P.state_set(saved[1], saved[2])
    for f in (2, 3):
        P.pcg_solve(S[f], c2, 6, warm=True)
    assert np.array_equal(host(c2), full)


def test_zero_slopes_and_nonfinite_status():
    P = plan("t1_mixed", "fp64")
    c = P.zeros(P.n_coef)
    res = torch.full((5,), -1.0, dtype=torch.float64, device=P.device)
    P.pcg_solve(P.zeros(P.n_slopes), c, 5, warm=False, resnorm=res)
    assert P.last_status() == 0
    assert torch.count_nonzero(c).item() == 0 and host(res)[0] == 0.0
    bad = P.zeros(P.n_slopes)
    bad[3 * 20 + 10] = float("nan")     # an active subaperture of the first sensor
    P.pcg_solve(bad, c, 3, warm=False)
    assert P.last_status() == -7
    assert torch.count_nonzero(c).item() == 0


def test_refresh_frame_parity():
    """FEWHA_REFRESH (the residual of a warm frame recomputed as b - M c instead of carried): equal
    in exact arithmetic to the carried form, so a chain with a refreshed frame follows the oracle's
    carried chain to the FP64 iterate bound; the refreshed state is b_prev = b, r_prev = the final
    residual, as after any frame."""
    P, O = plan("t1_mixed", "fp64"), oracle("t1_mixed")
    cfg = synth.load_config("t1_mixed")
    n_iter, N = cfg["n_iter"], O.n_coef
    c_ref, bp, rp = np.zeros(N), np.zeros(N), np.zeros(N)
    c = P.zeros(N)
    for f in range(4):
        s = _slopes(O, cfg, f)
        c_ref, bp, rp, _, st = O.frame(s, c_ref, bp, rp, n_iter, f == 0)
        assert st == 0
        P.pcg_solve(dev(P, s), c, n_iter, warm=f > 0, refresh=f == 2)
        assert P.last_status() == 0
        check(host(c), c_ref, 1e-9, "c frame %d" % f)
        b_g, r_g = P.state_get()
        check(host(b_g), bp, 1e-12, "b_prev frame %d" % f)
        check(host(r_g), rp, 1e-9, "r_prev frame %d" % f)
    with pytest.raises(ValueError):
        P.pcg_solve(dev(P, _slopes(O, cfg, 0)), c, n_iter, warm=False, refresh=True)


def test_status_of_a_solve_on_a_side_stream():
    """A solve enqueued on a non-default stream: the status word read with no synchronisation by
    the caller is already that solve's (the call synchronises the device)."""
    P = plan("t1_mixed", "fp64")
    good = P.zeros(P.n_slopes)
    bad = P.zeros(P.n_slopes)
    bad[3 * 20 + 10] = float("nan")
    c = P.zeros(P.n_coef)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    for slopes, want in ((bad, -7), (good, 0), (bad, -7)):
        with torch.cuda.stream(side):
            # slow the stream down so that the solve is still queued when the status is read
            for _ in range(3):
                P.apply_M(P.zeros(P.n_coef))
            P.pcg_solve(slopes, c, 8, warm=False)
        assert P.last_status() == want


def test_zero_passes_updates_residual_only():
    """n_iter = 0: the right-hand side and the warm-restart residual update run, c is unchanged
    (Alg. 1 with an empty PCG), against the oracle's frame with zero passes."""
    P, O = plan("c0_tiny", "fp64"), oracle("c0_tiny")
    cfg = synth.load_config("c0_tiny")
    N = O.n_coef
    s0, s1 = _slopes(O, cfg, 0), _slopes(O, cfg, 1)
    c_ref, bp, rp, _, st = O.frame(s0, np.zeros(N), np.zeros(N), np.zeros(N), cfg["n_iter"], True)
    c = P.zeros(N)
    P.pcg_solve(dev(P, s0), c, cfg["n_iter"], warm=False)
    c_before = host(c).copy()
    c_ref1, bp1, rp1, _, st1 = O.frame(s1, c_ref, bp, rp, 0, False)
    P.pcg_solve(dev(P, s1), c, 0, warm=True)
    assert st == 0 and st1 == 0 and P.last_status() == 0
    assert np.array_equal(host(c), c_before)
    check(host(c), c_ref1, 1e-9, "c")
    b_g, r_g = P.state_get()
    check(host(b_g), bp1, 1e-12, "b_prev")
    check(host(r_g), rp1, 1e-9, "r_prev")


def test_graph_replay_matches_eager():
    """A frame captured in a HIP graph and replayed gives bitwise the eager chain's result,
    replay after replay (host synchronisation between replays)."""
    P = plan("t1_mixed", "fp32")
    O = oracle("t1_mixed")
    cfg = synth.load_config("t1_mixed")
    S = [dev(P, _slopes(O, cfg, f)) for f in range(4)]
    n_iter = cfg["n_iter"]
    # eager reference chain
    c_e = P.zeros(P.n_coef)
    a_e = P.zeros(P.n_act)
    P.pcg_solve(S[0], c_e, n_iter, warm=False)
    ref = []
    for f in range(1, 4):
        P.pcg_solve(S[f], c_e, n_iter, warm=True)
        P.fit_dm(c_e, a_e, 0.5, out=a_e)
        ref.append((host(c_e).copy(), host(a_e).copy()))
    # graph chain from the same start
    c_g = P.zeros(P.n_coef)
    a_g = P.zeros(P.n_act)
    P.pcg_solve(S[0], c_g, n_iter, warm=False)
    torch.cuda.synchronize()
    graphs = []
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    saved = (c_g.clone(), a_g.clone()) + P.state_get()
    torch.cuda.synchronize()
    for f in range(1, 4):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            P.pcg_solve(S[f], c_g, n_iter, warm=True)
            P.fit_dm(c_g, a_g, 0.5, out=a_g)
        graphs.append(g)
    torch.cuda.synchronize()
    # capture does not execute: restore the start state, then replay
    c_g.copy_(saved[0])
    a_g.copy_(saved[1])
    P.state_set(saved[2], saved[3])
    torch.cuda.synchronize()
    for f in range(3):
        graphs[f].replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(c_g), ref[f][0]), f
        assert np.array_equal(host(a_g), ref[f][1]), f
    assert P.last_status() == 0

"""fewha_reconstruct: one call for Alg. 1's frame (the solve, then the fit of its c).

It must give, bit for bit, what fewha_pcg_solve followed by fewha_fit_dm gives: the iterate, the
actuator commands, the residual norms and the warm-restart state, over warm chains with a
refreshed frame, eagerly and replayed from a HIP graph, single-frame and batched.  (The last
pass steps c's coarse coefficients in its fine forward transform and the coarse levels leave c
alone; both calls take that path.)
"""
import numpy as np
import pytest

from paper_2009_00946_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _slopes(P, cfg, f):
    phi = torch.as_tensor(synth.layer_screens_flat(cfg, f), dtype=P.dtype, device=P.device)
    s = P.apply_A(P.dwt_forward(phi))
    return s + torch.as_tensor(synth.slope_noise(cfg, f), dtype=P.dtype, device=P.device)


@pytest.mark.parametrize("name,prec", [("c1_elt_mcao", "fp32"), ("t1_mixed", "fp64"), ("c3_mid_lgs", "fp32")])
def test_reconstruct_equals_solve_then_fit(name, prec):
    _need_gpu()
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config(name)
    n_iter, gain = cfg["n_iter"], 0.7
    print("\n[reconstruct] %s %s" % (name, prec), flush=True)
    PA, PB = fewha.Plan(cfg, precision=prec), fewha.Plan(cfg, precision=prec)
    S = [_slopes(PA, cfg, f) for f in range(4)]
    cA, cB = PA.zeros(PA.n_coef), PB.zeros(PB.n_coef)
    aA, aB = PA.zeros(PA.n_act), PB.zeros(PB.n_act)
    rA = torch.zeros(n_iter, dtype=torch.float64, device=PA.device)
    rB = torch.zeros_like(rA)
    for f in range(6):
        warm, fresh = f > 0, f == 3
        PA.reconstruct(S[f % 4], cA, n_iter, a_prev=aA, gain=gain, out=aA, warm=warm, resnorm=rA, refresh=fresh)
        PB.pcg_solve(S[f % 4], cB, n_iter, warm=warm, resnorm=rB, refresh=fresh)
        PB.fit_dm(cB, aB, gain, out=aB)
        torch.cuda.synchronize()
        assert PA.last_status() == 0 and PB.last_status() == 0
        assert torch.equal(cA, cB), "frame %d: c" % f
        assert torch.equal(aA, aB), "frame %d: a" % f
        assert torch.equal(rA, rB), "frame %d: resnorm" % f
        for x, y in zip(PA.state_get(), PB.state_get()):
            assert torch.equal(x, y), "frame %d: warm-restart state" % f
    assert np.isfinite(aA.double().cpu().numpy()).all()


def test_reconstruct_graph_replays():
    """A HIP graph captured from one reconstruct call (both stream branches) replays to the eager
    result, replay after replay, with eager work and synchronisations between the replays."""
    _need_gpu()
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config("c1_elt_mcao")
    n_iter = cfg["n_iter"]
    PG, PE = fewha.Plan(cfg), fewha.Plan(cfg)
    S = [_slopes(PG, cfg, f) for f in range(3)]
    cG, cE = PG.zeros(PG.n_coef), PE.zeros(PE.n_coef)
    aG, aE = PG.zeros(PG.n_act), PE.zeros(PE.n_act)
    sG = S[0].clone()
    PG.reconstruct(sG, cG, n_iter, a_prev=aG, out=aG, warm=False)
    PE.reconstruct(S[0], cE, n_iter, a_prev=aE, out=aE, warm=False)
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap):
        PG.reconstruct(sG, cG, n_iter, a_prev=aG, out=aG, warm=True)
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    # capturing does not run the work: both plans still hold the state after frame 0
    assert torch.equal(cG, cE) and torch.equal(aG, aE)
    for f in range(1, 6):
        sG.copy_(S[f % 3])
        torch.cuda.synchronize()
        g.replay()
        PE.reconstruct(S[f % 3], cE, n_iter, a_prev=aE, out=aE, warm=True)
        torch.cuda.synchronize()
        assert torch.equal(cG, cE), "replay %d: c" % f
        assert torch.equal(aG, aE), "replay %d: a" % f
        for x, y in zip(PG.state_get(), PE.state_get()):
            assert torch.equal(x, y), "replay %d: state" % f


@pytest.mark.parametrize("name,prec,nb", [("c1_elt_mcao_lgs", "fp32", 3), ("c0_tiny", "fp64", 5)])
def test_reconstruct_batch_equals_solve_then_fit(name, prec, nb):
    _need_gpu()
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config(name)
    n_iter = cfg["n_iter"]
    PA = fewha.Plan(cfg, precision=prec, max_batch=nb)
    PB = fewha.Plan(cfg, precision=prec, max_batch=nb)
    sb = torch.stack([_slopes(PA, cfg, f) for f in range(nb)]).contiguous()
    cA = torch.zeros((nb, PA.n_coef), dtype=PA.dtype, device=PA.device)
    cB = torch.zeros_like(cA)
    rA = torch.zeros(nb * n_iter, dtype=torch.float64, device=PA.device)
    rB = torch.zeros_like(rA)
    for t in range(3):
        aA = PA.reconstruct_batch(sb, cA, n_iter, gain=1.0, warm=t > 0, resnorm=rA)
        PB.pcg_solve_batch(sb, cB, n_iter, warm=t > 0, resnorm=rB)
        aB = PB.fit_dm_batch(cB, gain=1.0)
        torch.cuda.synchronize()
        assert PA.last_status_batch(nb) == [0] * nb
        assert torch.equal(cA, cB) and torch.equal(aA, aB) and torch.equal(rA, rB), t


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    assert np.all(np.isfinite(a))
    return max(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300),
               np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# n_iter = 1 makes the last pass the first (no q or p before it: the coarse levels' first-pass
# lines); 2 and 3 the short chains of the fold's shadow parities
@pytest.mark.parametrize("name,prec,n_iter", [("c1_elt_mcao", "fp32", 1), ("c1_elt_mcao", "fp32", 2),
                                               ("c3_mid_lgs", "fp32", 3), ("t1_mixed", "fp64", 1),
                                               ("t1_mixed", "fp64", 2)])
def test_reconstruct_short_solves_match_oracle(name, prec, n_iter):
    """Warm chains of 1- to 3-pass frames through fewha_reconstruct against the oracle's frame and
    fit (Alg. 1), and bitwise against fewha_pcg_solve then fewha_fit_dm."""
    _need_gpu()
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config(name)
    O = Oracle(cfg)
    gain = 0.6
    tol_c, tol_l, tol_a = (1e-3, 1e-4, 1e-4) if prec == "fp32" else (1e-9, 1e-9, 1e-9)
    PA, PB = fewha.Plan(cfg, precision=prec), fewha.Plan(cfg, precision=prec)
    print("\n[short] %s %s n_iter=%d fold=%d" % (name, prec, n_iter, PA.get_tuning()["fold"]), flush=True)
    N = O.n_coef
    c_ref, bp, rp, a_ref = np.zeros(N), np.zeros(N), np.zeros(N), np.zeros(O.n_act)
    cA, cB = PA.zeros(N), PB.zeros(N)
    aA, aB = PA.zeros(PA.n_act), PB.zeros(PB.n_act)
    for f in range(3):
        s = O.Ahat(synth.layer_screens_flat(cfg, f)) + O.slope_mask() * synth.slope_noise(cfg, f)
        c_ref, bp, rp, _, st = O.frame(s, c_ref, bp, rp, n_iter, f == 0)
        a_ref = O.fit(c_ref, a_ref, gain)
        sd = torch.as_tensor(s, dtype=PA.dtype, device=PA.device)
        PA.reconstruct(sd, cA, n_iter, a_prev=aA, gain=gain, out=aA, warm=f > 0)
        PB.pcg_solve(sd, cB, n_iter, warm=f > 0)
        PB.fit_dm(cB, aB, gain, out=aB)
        torch.cuda.synchronize()
        assert st == 0 and PA.last_status() == 0
        assert torch.equal(cA, cB) and torch.equal(aA, aB), "frame %d: reconstruct vs solve + fit" % f
        for x, y in zip(PA.state_get(), PB.state_get()):
            assert torch.equal(x, y), "frame %d: state" % f
        c = cA.double().cpu().numpy()
        assert _rel(c, c_ref) <= tol_c, ("c", f, _rel(c, c_ref))
        assert _rel(PA.dwt_inverse(cA).double().cpu().numpy(), O.Wt(c_ref)) <= tol_l, ("layers", f)
        assert _rel(aA.double().cpu().numpy(), a_ref) <= tol_a, ("actuators", f)
        b_g, r_g = PA.state_get()
        assert _rel(b_g.double().cpu().numpy(), bp) <= (1e-5 if prec == "fp32" else 1e-12), ("b_prev", f)

"""Batches of frames of one geometry (one launch per stage over every frame).

Each frame of a batch is an independent reconstruction with its own warm-restart state and Alg. 2
scalars, so frame f of a batched call must equal, bitwise, the same call on a single-frame plan
that carries frame f's chain alone (same kernels, same fixed reduction order).  Checked for warm
chains of pcg_solve (with per-frame residual norms), for A, A^T, M and the DM fit, for a batch
smaller than the workspace's, and against the oracle for one frame of the batch.
"""
import numpy as np
import pytest

from paper_2009_00946_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _slopes(O, cfg, frame):
    return O.Ahat(synth.layer_screens_flat(cfg, frame)) + O.slope_mask() * synth.slope_noise(cfg, frame)


@pytest.mark.parametrize("name,prec,nb,frames", [("c0_tiny", "fp64", 5, 3), ("t1_mixed", "fp32", 3, 3),
                                                  ("c1_elt_mcao", "fp32", 4, 3), ("c1_elt_mcao_lgs", "fp32", 4, 3)])
def test_batched_chains_equal_single_frame_chains(name, prec, nb, frames):
    _need_gpu()
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config(name)
    O = Oracle(cfg, precond=False)
    n_iter = cfg["n_iter"]
    print("\n[batch] %s %s nb=%d" % (name, prec, nb), flush=True)
    PB = fewha.Plan(cfg, precision=prec, max_batch=nb)
    singles = [fewha.Plan(cfg, precision=prec) for _ in range(nb)]
    dt = PB.dtype
    # chain f sees slope frames f, f + nb, f + 2 nb, ...
    S = [[torch.as_tensor(_slopes(O, cfg, f + nb * t), dtype=dt, device=PB.device) for t in range(frames)]
         for f in range(nb)]
    cb = torch.zeros((nb, PB.n_coef), dtype=dt, device=PB.device)
    cs = [P.zeros(P.n_coef) for P in singles]
    rb = torch.zeros(nb * n_iter, dtype=torch.float64, device=PB.device)
    rs = [torch.zeros(n_iter, dtype=torch.float64, device=PB.device) for _ in range(nb)]
    for t in range(frames):
        sb = torch.stack([S[f][t] for f in range(nb)]).contiguous()
        PB.pcg_solve_batch(sb, cb, n_iter, warm=t > 0, resnorm=rb)
        for f in range(nb):
            singles[f].pcg_solve(S[f][t], cs[f], n_iter, warm=t > 0, resnorm=rs[f])
        torch.cuda.synchronize()
        assert PB.last_status_batch(nb) == [0] * nb
        for f in range(nb):
            assert torch.equal(cb[f], cs[f]), "frame %d step %d: c differs" % (f, t)
            assert torch.equal(rb[f * n_iter:(f + 1) * n_iter], rs[f]), "frame %d step %d: resnorm" % (f, t)
    # fitting and the operators, batched vs one frame at a time
    ab = PB.fit_dm_batch(cb, gain=1.0)
    yb = PB.apply_M_batch(cb)
    sb = PB.apply_A_batch(cb)
    xb = PB.apply_At_batch(sb)
    for f in range(nb):
        P = singles[0]
        assert torch.equal(ab[f], P.fit_dm(cs[f], gain=1.0)), "fit frame %d" % f
        assert torch.equal(yb[f], P.apply_M(cs[f])), "M frame %d" % f
        assert torch.equal(sb[f], P.apply_A(cs[f])), "A frame %d" % f
        assert torch.equal(xb[f], P.apply_At(sb[f].contiguous())), "A^T frame %d" % f
    # a batch smaller than the workspace's: frames 0..nb-2 continue their chains
    k = nb - 1
    sk = torch.stack([S[f][0] for f in range(k)]).contiguous()
    PB.pcg_solve_batch(sk, cb[:k], n_iter, warm=True)
    for f in range(k):
        singles[f].pcg_solve(S[f][0], cs[f], n_iter, warm=True)
    torch.cuda.synchronize()
    for f in range(k):
        assert torch.equal(cb[f], cs[f]), "partial batch frame %d" % f
    with pytest.raises(ValueError):
        PB.pcg_solve_batch(torch.zeros((nb + 1, PB.n_slopes), dtype=dt, device=PB.device),
                           torch.zeros((nb + 1, PB.n_coef), dtype=dt, device=PB.device), n_iter)


def test_batched_frame_matches_oracle():
    """One frame of a cold batch against the oracle (the parity bound of single-frame solves)."""
    _need_gpu()
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config("c0_tiny")
    O = Oracle(cfg)
    nb, n_iter = 6, cfg["n_iter"]
    PB = fewha.Plan(cfg, precision="fp64", max_batch=nb)
    S = [_slopes(O, cfg, f) for f in range(nb)]
    sb = torch.as_tensor(np.stack(S), dtype=PB.dtype, device=PB.device)
    cb = torch.zeros((nb, PB.n_coef), dtype=PB.dtype, device=PB.device)
    PB.pcg_solve_batch(sb, cb, n_iter, warm=False)
    torch.cuda.synchronize()
    z = np.zeros(PB.n_coef)
    for f in (0, nb - 1):
        c_ref = O.frame(S[f], z, z, z, n_iter, True)[0]
        got = cb[f].cpu().numpy()
        assert np.abs(got - c_ref).max() <= 1e-9 * np.abs(c_ref).max(), f


def test_large_batch_cold_frames_equal_single():
    """A batch of 17 cold frames: every frame equals, bitwise, the same cold frame on a
    single-frame plan, with its residual norms."""
    _need_gpu()
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config("c0_tiny")
    O = Oracle(cfg, precond=False)
    nb, n_iter = 17, cfg["n_iter"]
    PB = fewha.Plan(cfg, precision="fp64", max_batch=nb)
    P1 = fewha.Plan(cfg, precision="fp64")
    S = torch.as_tensor(np.stack([_slopes(O, cfg, f) for f in range(nb)]), dtype=PB.dtype, device=PB.device)
    rb = torch.zeros(nb * n_iter, dtype=torch.float64, device=PB.device)
    cb = torch.zeros((nb, PB.n_coef), dtype=PB.dtype, device=PB.device)
    PB.pcg_solve_batch(S.contiguous(), cb, n_iter, warm=False, resnorm=rb)
    assert PB.last_status_batch(nb) == [0] * nb
    r1 = torch.zeros(n_iter, dtype=torch.float64, device=PB.device)
    for f in range(nb):
        c1 = P1.zeros(P1.n_coef)
        P1.pcg_solve(S[f].contiguous(), c1, n_iter, warm=False, resnorm=r1)
        torch.cuda.synchronize()
        assert torch.equal(cb[f], c1), "frame %d" % f
        assert torch.equal(rb[f * n_iter:(f + 1) * n_iter], r1), "resnorm frame %d" % f


@pytest.mark.parametrize("nb", [1, 3])
def test_stage_launches_leave_the_solver_state_alone(nb):
    """Stage launches for timing (single-frame and batched forms) between the frames of a warm
    chain change neither its iterates nor its carried state: the chain equals, bitwise, the same
    chain run without them."""
    _need_gpu()
    from oracle import Oracle
    from paper_2009_00946_amd import fewha
    cfg = synth.load_config("t1_mixed")
    O = Oracle(cfg, precond=False)
    n_iter = cfg["n_iter"]
    runs = []
    for with_stages in (False, True):
        PB = fewha.Plan(cfg, precision="fp32", max_batch=nb)
        cb = torch.zeros((nb, PB.n_coef), dtype=PB.dtype, device=PB.device)
        for t in range(3):
            sb = torch.stack([torch.as_tensor(_slopes(O, cfg, f + nb * t), dtype=PB.dtype, device=PB.device)
                              for f in range(nb)]).contiguous()
            PB.pcg_solve_batch(sb, cb, n_iter, warm=t > 0)
            if with_stages:
                for st in ("wt", "proj", "pt", "fwd"):
                    PB.stage_launch_batch(st, nb)
                    PB.stage_launch(st)
        torch.cuda.synchronize()
        assert PB.last_status_batch(nb) == [0] * nb
        b, r = PB.state_get()
        runs.append((cb.clone(), b.clone(), r.clone()))
    for a, b in zip(*runs):
        assert torch.equal(a, b)

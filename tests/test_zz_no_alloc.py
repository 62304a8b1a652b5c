"""The allocation-free forward transform (fewha_dwt_forward_noalloc) against fewha_dwt_forward,
through the C ABI: bitwise equal on two calls in a row, the second on a smaller plan, and on a
plan that was created but never bound (no workspace at all)."""
import ctypes

import numpy as np
import pytest

from paper_2009_00946_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _vec(P, n, seed):
    return torch.as_tensor(synth.normal_vector(n, seed), dtype=P.dtype, device=P.device)


def test_noalloc_forward_matches_workspace_forward():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_00946_amd import fewha
    L = fewha.load_library()
    # a large plan, then a smaller one: the shared scratch keeps the first call's contents
    for name, prec, seed in (("c1_elt_mcao", "fp32", 71), ("c0_tiny", "fp64", 72), ("c3_mid_lgs", "fp32", 73)):
        print("[noalloc] %s %s" % (name, prec), flush=True)
        P = fewha.Plan(synth.load_config(name), precision=prec)
        x = _vec(P, P.n_coef, seed)
        ref = P.dwt_forward(x)
        out = torch.full((P.n_coef,), float("nan"), dtype=P.dtype, device=P.device)
        st = L.fewha_dwt_forward_noalloc(P._h, x.data_ptr(), out.data_ptr(),
                                         torch.cuda.current_stream().cuda_stream)
        assert st == 0, fewha.STATUS.get(st)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), name
        # through the binding as well
        assert torch.equal(P.dwt_forward_noalloc(x), ref), name
    # a created, never bound plan (the call needs no workspace)
    cfg = synth.load_config("t1_mixed")
    h, st = fewha.create_host_plan(cfg, precision="fp32")
    assert st == 0
    P = fewha.Plan(cfg, precision="fp32")
    x = _vec(P, P.n_coef, 74)
    out = torch.full((P.n_coef,), float("nan"), dtype=P.dtype, device=P.device)
    assert L.fewha_dwt_forward_noalloc(h, x.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, P.dwt_forward(x))
    L.fewha_plan_destroy(h)

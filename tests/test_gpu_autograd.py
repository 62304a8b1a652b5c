"""Differentiation on the GPU (autograd wrapper over the C ABI), against central differences and
the FP64 oracle.

* gradcheck of A, A^T and M in FP64 (central differences, step 1e-6; second derivatives of A), on
  the tiny geometry (full Jacobian of A) and on the ELT geometry (random directions);
* a batch of 8 coefficient vectors on the ELT geometry in FP32: the backward of A equals the
  oracle's A^T row by row (1e-5, the operator bound);
* the entry points the implicit gradients use: M c = b from c = 0 (fewha_solve_M) against the
  oracle's Alg. 2 with the same passes, C A (fewha_apply_CA), the per-layer prior products
  (fewha_prior_dot) and the Cn^2 gradient (fewha_cn2_gradient);
* the reconstruction's backward (dL/ds = C A lambda, dL/dgamma_l = lambda_l^T (alpha D)_l c_l /
  gamma_l, lambda = M^-1 dL/dc) against the same expressions evaluated by the oracle with the same
  number of PCG passes.  The expressions themselves are pinned against exact dense derivatives in
  test_oracle_implicit_gradient.py.
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
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    assert got.shape == ref.shape and np.all(np.isfinite(got)), what
    err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
    nrm = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    assert err <= tol and nrm <= tol, "%s: max-rel %.3e norm-rel %.3e > %.1e" % (what, err, nrm, tol)
    return max(err, nrm)


def test_gradcheck_operators_fp64():
    from paper_2009_00946_amd import autograd as ag
    P = plan("c0_tiny", "fp64")
    c = dev(P, synth.normal_vector(P.n_coef, 51)).requires_grad_(True)
    s = dev(P, synth.normal_vector(P.n_slopes, 52)).requires_grad_(True)
    kw = dict(eps=1e-6, atol=1e-8, rtol=1e-6)
    assert torch.autograd.gradcheck(lambda x: ag.apply_A(P, x), (c,), **kw)
    assert torch.autograd.gradcheck(lambda x: ag.apply_At(P, x), (s,), fast_mode=True, **kw)
    assert torch.autograd.gradcheck(lambda x: ag.apply_M(P, x), (c,), fast_mode=True, **kw)
    assert torch.autograd.gradgradcheck(lambda x: ag.apply_A(P, x), (c,), fast_mode=True, **kw)


def test_gradcheck_operators_elt_geometry_fp64():
    """The differentiation configuration's geometry (9 guide stars of 84 x 84, 9 layers up to
    256^2): gradcheck in fast mode (a random direction through the Jacobian, central differences
    step 1e-6, against the backward's vector-Jacobian product) of A, A^T and M in FP64."""
    from paper_2009_00946_amd import autograd as ag
    P = plan("c1_elt_mcao", "fp64")
    c = dev(P, synth.normal_vector(P.n_coef, 53)).requires_grad_(True)
    s = dev(P, synth.normal_vector(P.n_slopes, 54)).requires_grad_(True)
    kw = dict(eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=True)
    assert torch.autograd.gradcheck(lambda x: ag.apply_A(P, x), (c,), **kw)
    assert torch.autograd.gradcheck(lambda x: ag.apply_At(P, x), (s,), **kw)
    assert torch.autograd.gradcheck(lambda x: ag.apply_M(P, x), (c,), **kw)


@pytest.mark.parametrize("name,prec,tol", [("c0_tiny", "fp64", 1e-12), ("c1_elt_mcao", "fp32", 1e-5)])
def test_batched_backward_is_oracle_adjoint(name, prec, tol):
    from paper_2009_00946_amd import autograd as ag
    P, O = plan(name, prec), oracle(name)
    B = 8
    c = torch.stack([dev(P, synth.normal_vector(P.n_coef, 60 + i)) for i in range(B)]).requires_grad_(True)
    w = np.stack([synth.normal_vector(P.n_slopes, 70 + i) for i in range(B)])
    y = ag.apply_A(P, c)
    assert y.shape == (B, P.n_slopes)
    check(host(y[3]), O.A(host(c[3])), tol, "A row 3")
    (y * dev(P, w)).sum().backward()
    for i in range(B):
        check(host(c.grad[i]), O.At(w[i]), tol, "A^T row %d" % i)


@pytest.mark.parametrize("name,prec,tol_c,tol_op", [("c0_tiny", "fp64", 1e-9, 1e-12),
                                                     ("c1_elt_mcao", "fp32", 1e-3, 1e-5)])
def test_adjoint_entry_points(name, prec, tol_c, tol_op):
    P, O = plan(name, prec), oracle(name)
    cfg = synth.load_config(name)
    n = cfg["n_iter"]
    b = synth.normal_vector(P.n_coef, 81)
    res = torch.zeros(n, dtype=torch.float64, device=P.device)
    c = P.solve_M(dev(P, b), n_iter=n, resnorm=res)
    torch.cuda.synchronize()
    assert P.last_status() == 0
    c_ref, _, res_ref, done, st = O.pcg(np.zeros(P.n_coef), b, n)
    assert st == 0 and done == n
    check(host(c), c_ref, tol_c, "solve_M")
    check(host(res), res_ref, max(tol_c * 1e-2, 1e-9) if prec == "fp64" else 1e-5, "solve_M resnorm")
    x = synth.normal_vector(P.n_coef, 82)
    check(host(P.apply_CA(dev(P, x))), O.slope_weights() * O.A(x), tol_op, "C A")
    y = synth.normal_vector(P.n_coef, 83)
    xr, yr = host(dev(P, x)), host(dev(P, y))  # the values the device holds (FP32 rounding)
    aD = cfg["alpha_reg"] * O.prior()
    offs = np.cumsum([0] + [l["n"] ** 2 for l in cfg["layers"]])
    ref = np.array([xr[offs[l]:offs[l + 1]] @ (aD[offs[l]:offs[l + 1]] * yr[offs[l]:offs[l + 1]])
                    for l in range(len(cfg["layers"]))])
    check(host(P.prior_dot(dev(P, x), dev(P, y))), ref, tol_op, "prior_dot")
    gam = np.array([lay["cn2_weight"] for lay in cfg["layers"]])
    check(host(P.cn2_gradient(dev(P, x), dev(P, y))), ref / gam, tol_op, "cn2_gradient")


@pytest.mark.parametrize("name,prec,tol", [("c0_tiny", "fp64", 1e-9), ("c1_elt_mcao", "fp32", 2e-3)])
def test_reconstruction_gradients(name, prec, tol):
    from paper_2009_00946_amd import autograd as ag
    P, O = plan(name, prec), oracle(name)
    cfg = synth.load_config(name)
    n = cfg["n_iter"]
    s_np = O.Ahat(synth.layer_screens_flat(cfg, 0)) + O.slope_mask() * synth.slope_noise(cfg, 0)
    w = synth.normal_vector(P.n_coef, 91)
    s = dev(P, s_np).requires_grad_(True)
    gamma = ag.layer_weights(P)
    c = ag.reconstruct(P, s, gamma, n_iter=n)
    (c * dev(P, w)).sum().backward()
    # the oracle: the same passes for c and for lambda, then the same expressions
    z = np.zeros(P.n_coef)
    c_ref, _, _, _, st = O.frame(s_np, z, z, z, n, True)
    lam, _, _, _, st2 = O.pcg(z, w, n)
    assert st == 0 and st2 == 0
    check(host(c), c_ref, tol, "c")
    aD = cfg["alpha_reg"] * O.prior()
    offs = np.cumsum([0] + [l["n"] ** 2 for l in cfg["layers"]])
    g_ref = np.array([lam[offs[l]:offs[l + 1]] @ (aD[offs[l]:offs[l + 1]] * c_ref[offs[l]:offs[l + 1]])
                      / lay["cn2_weight"] for l, lay in enumerate(cfg["layers"])])
    e_g = check(host(gamma.grad), g_ref, tol, "dL/dgamma")
    e_s = check(host(s.grad), O.slope_weights() * O.A(lam), tol, "dL/ds")
    print("[grad] %s %s: dL/dgamma %.2e dL/ds %.2e" % (name, prec, e_g, e_s), flush=True)


def test_batched_plan_autograd_and_timing():
    """A batched plan (one launch per stage over the 8 rows) gives the row-by-row results
    bitwise; forward + backward of A on 8 ELT vectors is timed both ways (reported)."""
    from paper_2009_00946_amd import autograd as ag, fewha
    P1 = plan("c1_elt_mcao", "fp32")
    PB = fewha.Plan(synth.load_config("c1_elt_mcao"), max_batch=8)
    c = torch.randn(8, P1.n_coef, device=P1.device).requires_grad_(True)
    w = torch.randn(8, P1.n_slopes, device=P1.device)
    grads = []
    for P in (P1, PB):
        c.grad = None
        (ag.apply_A(P, c) * w).sum().backward()
        grads.append(c.grad.clone())
    assert torch.equal(grads[0], grads[1])
    for P, what in ((P1, "row by row"), (PB, "batched")):
        for _ in range(3):
            (ag.apply_A(P, c) * w).sum().backward()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = 20
        for _ in range(reps):
            c.grad = None
            (ag.apply_A(P, c) * w).sum().backward()
        e1.record()
        torch.cuda.synchronize()
        print("[timing] A forward+backward, 8 ELT vectors FP32, %s: %.3f ms" % (what, e0.elapsed_time(e1) / reps),
              flush=True)

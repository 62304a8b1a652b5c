"""Differentiation of the FEWHA operators and of the reconstruction with torch.autograd.

Every forward and backward product runs in the library's kernels through the C ABI; this module
only wires them into autograd:

* ``apply_A(plan, c)``: s = mask Gamma P W^T c (Eq. (atmo) in the wavelet domain); its backward is
  the hand-written adjoint chain ``fewha_apply_At``, and the adjoint's backward is A again, so
  second derivatives work too.  ``apply_At`` and ``apply_M`` (M is symmetric) likewise.
* ``reconstruct(plan, s, gamma)``: c = M^-1 W A^T C s by n_iter cold PCG passes (Alg. 2), with
  gradients by the implicit-function rule at the solution (not by unrolling the passes):
  with lambda = M^-1 dL/dc,
      dL/ds        = C A lambda,
      dL/dgamma_l  = lambda_l^T (alpha D)_l c_l / gamma_l,
  since the prior of Eq. (fewha) scales as D_l ~ 1/gamma_l, so dM/dgamma_l = -(alpha D)_l / gamma_l
  on layer l.  These are exact for the converged solution; with few passes they are the gradients
  of the limit the passes approach.

Inputs are 1-D tensors of the plan's lengths, or 2-D batches (one row per vector): one batched
launch per stage when the plan holds that many frames (``max_batch``), else row by row.  The
reconstruction runs cold and overwrites the plan's warm-restart state.
"""
import torch

__all__ = ["apply_A", "apply_At", "apply_M", "reconstruct"]


def _rows(fn, fn_batch, x, n_out, plan):
    x = x.contiguous()
    if x.dim() == 1:
        return fn(x)
    if x.shape[0] <= plan.max_batch:  # one launch per stage over the whole batch
        return fn_batch(x)
    out = torch.empty((x.shape[0], n_out), dtype=plan.dtype, device=plan.device)
    for i in range(x.shape[0]):
        fn(x[i], out=out[i])
    return out


class _A(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, plan):
        ctx.plan = plan
        return _rows(plan.apply_A, plan.apply_A_batch, c, plan.n_slopes, plan)

    @staticmethod
    def backward(ctx, g):
        return _At.apply(g, ctx.plan), None


class _At(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, plan):
        ctx.plan = plan
        return _rows(plan.apply_At, plan.apply_At_batch, s, plan.n_coef, plan)

    @staticmethod
    def backward(ctx, g):
        return _A.apply(g, ctx.plan), None


class _M(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, plan):
        ctx.plan = plan
        return _rows(plan.apply_M, plan.apply_M_batch, c, plan.n_coef, plan)

    @staticmethod
    def backward(ctx, g):
        return _M.apply(g, ctx.plan), None


def apply_A(plan, c):
    return _A.apply(c, plan)


def apply_At(plan, s):
    return _At.apply(s, plan)


def apply_M(plan, c):
    return _M.apply(c, plan)


class _Reconstruct(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, gamma, plan, n_iter, n_iter_adjoint):
        c = plan.zeros(plan.n_coef)
        plan.pcg_solve(s.contiguous(), c, n_iter, warm=False)
        ctx.plan, ctx.n_adj = plan, n_iter_adjoint
        ctx.save_for_backward(c, gamma)
        return c

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        c, gamma = ctx.saved_tensors
        lam = plan.solve_M(g.contiguous(), n_iter=ctx.n_adj)
        grad_s = plan.apply_CA(lam)
        grad_gamma = plan.cn2_gradient(lam, c)
        return grad_s, grad_gamma.to(gamma.dtype), None, None, None


def layer_weights(plan, requires_grad=True):
    """The Cn^2 weights gamma_l the plan was built with, as a float64 tensor on its device."""
    g = torch.tensor([float(l["cn2_weight"]) for l in plan.cfg["layers"]], dtype=torch.float64, device=plan.device)
    return g.requires_grad_(requires_grad)


def reconstruct(plan, s, gamma=None, n_iter=None, n_iter_adjoint=None):
    """c = M^-1 W A^T C s (n_iter cold passes) with implicit gradients for s and gamma.

    ``gamma`` must hold the weights the plan was built with (it only carries the gradient; the
    plan's prior is fixed at plan creation); ``layer_weights(plan)`` makes it."""
    n_iter = int(plan.cfg["n_iter"] if n_iter is None else n_iter)
    n_iter_adjoint = n_iter if n_iter_adjoint is None else int(n_iter_adjoint)
    if gamma is None:
        gamma = layer_weights(plan)
    ref = torch.tensor([float(l["cn2_weight"]) for l in plan.cfg["layers"]], dtype=torch.float64)
    if gamma.numel() != ref.numel() or not torch.allclose(gamma.detach().cpu().to(torch.float64), ref, rtol=1e-12):
        raise ValueError("gamma must equal the plan's Cn^2 weights (the prior is fixed at plan creation)")
    return _Reconstruct.apply(s, gamma, plan, n_iter, n_iter_adjoint)

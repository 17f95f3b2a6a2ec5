"""torch.autograd over the CBS solver (forward solve + adjoint-field gradient).

Forward:  eps_r (float32 [nz, ny, nx]) -> E = E_inc + E_s (complex64 [3, nz, ny, nx])
          for the x-polarised plane wave (design paragraph of arXiv 2506.15411).
Backward: for a real loss L, torch hands in gE = 2 dL/dE*.  Perturbing eps_r by
          h at voxel v changes K and S by k0^2 h there, so A dE = k0^2 h E (E the
          total field) and dL = Re(conj(gE)^T dE).  With A complex-symmetric,
          E_adj = A^-1 conj(gE) gives dL/d eps_r = k0^2 Re(sum_c E_adj,c E_c)
          (objective and optimisation paragraphs: the gradient via one more CBS
          solve).  Both solves and the product run in the HIP library.
"""

from __future__ import annotations

import torch

from . import libcbs as L
from .solver import Plan


class NotConvergedError(RuntimeError):
    """A solve inside the autograd graph stopped at max_iter before tol."""

    def __init__(self, which: str, stats):
        super().__init__(f"{which} CBS solve did not reach tol: {stats.iterations} iterations, "
                         f"residual {stats.residual:.3e}")
        self.stats = stats


def _checked(which: str, st, strict: bool):
    if strict and st.status == L.CBS_NOT_CONVERGED:
        raise NotConvergedError(which, st)
    return st


class CBSSolve(torch.autograd.Function):
    """Solves record their statistics on the plan (plan.last_forward_stats,
    plan.last_adjoint_stats); with strict (the default) a solve that stops at
    max_iter raises NotConvergedError instead of returning its last iterate."""

    @staticmethod
    def forward(ctx, eps_r: torch.Tensor, plan: Plan, tol: float = 1e-6, max_iter: int = 20000,
                check_every: int = 10, strict: bool = True):
        if eps_r.dtype != torch.float32:
            raise ValueError("CBSSolve differentiates real float32 permittivities")
        eps = eps_r.detach().contiguous()
        plan.set_permittivity(eps)
        E, st = plan.solve(tol=tol, max_iter=max_iter, check_every=check_every)
        plan.last_forward_stats = _checked("forward", st, strict)
        ctx.plan = plan
        ctx.eps = eps
        ctx.opts = (tol, max_iter, check_every, strict)
        ctx.save_for_backward(E)
        return E

    @staticmethod
    def backward(ctx, gE: torch.Tensor):
        (E,) = ctx.saved_tensors
        plan: Plan = ctx.plan
        tol, max_iter, check_every, strict = ctx.opts
        if plan._eps_ref is not ctx.eps:
            plan.set_permittivity(ctx.eps)  # the plan was reused for another medium
        if gE.dtype != torch.complex64:
            raise ValueError(f"expected a complex64 gradient, got {gE.dtype}")
        # the adjoint source is conj(gE), formed by the library; a tensor carrying
        # torch's lazy conjugate bit already stores conj(gE) in memory
        if gE.is_conj():
            src, conj = torch.conj(gE).contiguous(), False
        else:
            src, conj = gE.contiguous(), True
        Ea, st = plan.adjoint(field=src, conj=conj, tol=tol, max_iter=max_iter,
                              check_every=check_every)
        plan.last_adjoint_stats = _checked("adjoint", st, strict)
        grad = plan.gradient(E, Ea, scale=1.0)
        return grad, None, None, None, None, None


def cbs_solve(eps_r: torch.Tensor, plan: Plan, tol: float = 1e-6, max_iter: int = 20000,
              check_every: int = 10, strict: bool = True) -> torch.Tensor:
    """Differentiable total field E(eps_r)."""
    return CBSSolve.apply(eps_r, plan, tol, max_iter, check_every, strict)


def focal_intensity(eps_r: torch.Tensor, plan: Plan, r0, tol: float = 1e-6,
                    max_iter: int = 20000, strict: bool = True) -> torch.Tensor:
    """The paper's figure of merit |E(r0)|^2 (Fig. 2 caption), differentiable."""
    E = cbs_solve(eps_r, plan, tol, max_iter, 10, strict)
    ix, iy, iz = r0
    v = E[:, iz, iy, ix]
    return (v.real ** 2 + v.imag ** 2).sum()

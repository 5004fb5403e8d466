"""Differentiable solve x = (lambda I + Ktilde(h))^{-1} b (torch.autograd.Function).

Adjoint of x = A^{-1} b with A = lambda I + Ktilde(h), the skeletons and
projections of the tree held fixed (the interpolative decomposition is not
differentiated): for a loss L with g = dL/dx,
    z = A^{-T} g               (askit_solve_transpose)
    dL/db      = z
    dL/dlambda = -sum z . x     (dA/dlambda = I)
    dL/dh      = -sum z . (dKtilde/dh) x
where dKtilde/dh has the block structure of Ktilde with kernel entries
dk/dh = k r^2 / h^3, applied by the hierarchical matvec with recomputed blocks
(askit_adjoint_scalars).  All arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import torch

from .askit import ASKIT_FP64


class KernelSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, lam, h, tree, precision, refine):
        tree.set_bandwidth(float(h))
        f = tree.factorize(float(lam), precision)
        if refine is not None:
            f.set_refinement(int(refine[0]), float(refine[1]))
        x = f.solve(b)
        ctx.factor = f
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        f = ctx.factor
        z = f.solve_transpose(gx.contiguous())
        dlam, dh = f.adjoint_scalars(x, z)
        gl = torch.tensor(dlam, dtype=torch.float64)
        gh = torch.tensor(dh, dtype=torch.float64)
        return z, gl, gh, None, None, None


def kernel_solve(b, lam, h, tree, precision=ASKIT_FP64, refine=None):
    """x = (lambda I + Ktilde(h))^{-1} b on a skeletonized `Tree`; differentiable
    in b (CUDA tensor, N or N x nrhs), lam and h (0-dim float64 tensors).
    refine = (max operator applications, relative residual) refines both the
    solve and the transpose solve of the backward pass by GMRES against the
    FP64 hierarchical operator."""
    lam = lam if isinstance(lam, torch.Tensor) else torch.tensor(float(lam), dtype=torch.float64)
    h = h if isinstance(h, torch.Tensor) else torch.tensor(float(h), dtype=torch.float64)
    return KernelSolve.apply(b, lam, h, tree, precision, refine)

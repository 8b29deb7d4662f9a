"""Differentiable AIRG solve: u = A(sigma)^{-1} M s as a torch.autograd.Function.

A(sigma) = A_adv + sum_K sigma_K M_K with a dense cell block M_K per cell
(the removal term of the streaming operator), b = M s.  The backward pass
solves A^T lambda = dL/du with an AIRG hierarchy built on A^T (the downwind
operator) and returns
    dL/ds       = M^T lambda          (M_K symmetric here, so M lambda),
    dL/dsigma_K = -lambda_K^T M_K u_K.
Every numerical step (assembly of A(sigma), M s, both solves, the gradient
contractions) runs in the HIP library; this module only marshals tensors.
"""
import numpy as np
import torch

from . import airg


class DiffProblem:
    """Device data of A(sigma) for one sparsity pattern.

    rowptr/col/val_adv: CSR of A_adv (every cell block must be stored);
    mass: (ncell, bs, bs) symmetric cell blocks, dof of (K, a) = K*bs + a.
    """

    def __init__(self, rowptr, col, val_adv, mass, opts=None, rtol=1e-10, max_it=200, device="cuda"):
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        if not np.allclose(mass, mass.transpose(0, 2, 1)):
            raise ValueError("cell mass blocks must be symmetric")
        ncell, bs = mass.shape[0], mass.shape[1]
        rowptr = np.asarray(rowptr, dtype=np.int64)
        col = np.asarray(col, dtype=np.int64)
        n = len(rowptr) - 1
        if n != ncell * bs:
            raise ValueError("matrix size does not match the cell blocks")
        # CSR position of every cell-block entry (K, a, b)
        K = np.repeat(np.arange(ncell), bs * bs)
        a = np.tile(np.repeat(np.arange(bs), bs), ncell)
        b = np.tile(np.arange(bs), ncell * bs)
        rows = K * bs + a
        cols = K * bs + b
        key = np.repeat(np.arange(n), np.diff(rowptr)) * n + col
        want = rows * n + cols
        pos = np.searchsorted(key, want)
        if np.any(pos >= len(key)) or np.any(key[np.minimum(pos, len(key) - 1)] != want):
            raise ValueError("the pattern does not store every cell block entry")
        self.n, self.ncell, self.bs = n, ncell, bs
        self.rowptr, self.col, self.val_adv = airg.to_device(rowptr, col, val_adv, device=device)
        self.mass = torch.as_tensor(mass, device=device)
        self.pos = torch.as_tensor(pos.astype(np.int32), device=device)
        self.opts = opts if opts is not None else airg.default_opts()
        self.rtol, self.max_it = rtol, max_it
        self.last_forward = None
        self.last_adjoint = None


class AIRGLinearSolve(torch.autograd.Function):
    """u = AIRGLinearSolve.apply(source, sigma, problem)."""

    @staticmethod
    def forward(ctx, source, sigma, prob):
        val = prob.val_adv.clone()
        airg.airg_blockdiag_axpy(prob.mass, sigma.detach().contiguous(), prob.pos, prob.val_adv, val)
        b = airg.airg_blockdiag_apply(prob.mass, source.detach().contiguous())
        h = airg.airg_setup(prob.rowptr, prob.col, val, prob.opts)
        u, info = airg.airg_solve(h, b, rtol=prob.rtol, max_it=prob.max_it)
        prob.last_forward = info
        ctx.h = h
        ctx.prob = prob
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        prob = ctx.prob
        lam, info = airg.airg_adjoint_solve(ctx.h, gu.contiguous(), rtol=prob.rtol, max_it=prob.max_it)
        prob.last_adjoint = info
        grad_s = airg.airg_blockdiag_apply(prob.mass, lam) if ctx.needs_input_grad[0] else None
        grad_sigma = airg.airg_blockdiag_bilinear(prob.mass, u, lam, -1.0) if ctx.needs_input_grad[1] else None
        return grad_s, grad_sigma, None


def solve(source, sigma, prob):
    return AIRGLinearSolve.apply(source, sigma, prob)

"""Differentiable PP-GMRES solve: torch.autograd.Function over the C ABI.

Forward solves A x = b with polynomial-preconditioned GMRES(m).  Backward
solves the adjoint system A^T lam = dL/dx with its own GMRES polynomial built
for A^T (on the device: the transpose comes from pp_csr_transpose), then
returns dL/db = lam and dL/dA_ij = -lam_i x_j on the stored pattern of A
(pp_csr_grad).  Both solves and both helper steps run in libpp.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import torch

from .binding import CSRMatrix, pp_csr_grad, pp_csr_transpose, pp_gmres_solve


@dataclass
class SolveConfig:
    m: int = 50
    d: int = 15
    tol: float = 1e-12
    v0: Optional[torch.Tensor] = None       # start vector for the forward polynomial
    v0_seed: int = 0                        # v0 None: seed of the drawn U(-1, 1) vector
    adj_m: Optional[int] = None             # adjoint solve; None -> forward value
    adj_d: Optional[int] = None
    adj_tol: Optional[float] = None
    adj_v0: Optional[torch.Tensor] = None   # start vector for the A^T polynomial
    adj_v0_seed: int = 0                    # adj_v0 None: seed of the drawn vector
    max_iters: int = 0
    stats: list = field(default_factory=list)  # (phase, Stats) appended per solve


class _PPSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, pattern: CSRMatrix, cfg: SolveConfig):
        A = pattern.with_vals(vals.detach().contiguous())
        x, st = pp_gmres_solve(A, b.detach().contiguous(), m=cfg.m, d=cfg.d, tol=cfg.tol,
                               v0=cfg.v0, v0_seed=cfg.v0_seed, max_iters=cfg.max_iters)
        cfg.stats.append(("forward", st))
        ctx.save_for_backward(vals, x)
        ctx.pattern = pattern
        ctx.cfg = cfg
        return x

    @staticmethod
    def backward(ctx, gx):
        vals, x = ctx.saved_tensors
        cfg = ctx.cfg
        A = ctx.pattern.with_vals(vals.detach().contiguous())
        At = pp_csr_transpose(A)
        lam, st = pp_gmres_solve(
            At, gx.detach().contiguous().to(torch.float64),
            m=cfg.adj_m or cfg.m, d=cfg.d if cfg.adj_d is None else cfg.adj_d,
            tol=cfg.adj_tol or cfg.tol, v0=cfg.adj_v0, v0_seed=cfg.adj_v0_seed,
            max_iters=cfg.max_iters)
        cfg.stats.append(("adjoint", st))
        g_vals = pp_csr_grad(A, lam, x) if ctx.needs_input_grad[0] else None
        g_b = lam if ctx.needs_input_grad[1] else None
        return g_vals, g_b, None, None


def pp_solve(pattern: CSRMatrix, vals: torch.Tensor, b: torch.Tensor,
             cfg: Optional[SolveConfig] = None) -> torch.Tensor:
    """x = A(vals)^{-1} b, differentiable in ``vals`` (A's stored values) and ``b``."""
    return _PPSolve.apply(vals, b, pattern, cfg or SolveConfig())

"""torch.autograd functions over the coded QR and the coded solve.

Both directions run in the HIP library: the forward passes call
coded_qr_encode / coded_qr_factor (with the erasures and recoveries of a
failure schedule) and coded_qr_postorth / coded_qr_solve; the backward passes
call coded_qr_backward and coded_qr_solve_backward.  torch only supplies the
device buffers and converts tensors to the column-major layout the library
reads.

    engine = CodedQR(cfg, v_tilde, gh)
    Q, R1 = coded_qr(A, engine, schedule)   # Q = Q~[:, :n] (m' x n), R1 (n x n)
    x = coded_solve(Q, R1, b, engine)       # R_1^{-1} (G_0 Q_1)^T (G_0 b)
    ((x - x_target) ** 2).sum().backward()  # A.grad, b.grad

With coded_qr(A, engine, schedule, recompute=True) the forward keeps only A
for the backward and the backward runs the factorization again (it is
deterministic: every reduction sums in a fixed order), trading one more
forward for the m' x N encoded matrix that would otherwise stay alive
between the passes.
"""
from __future__ import annotations

import torch

from . import cqr


def _colmajor(t: torch.Tensor, rows: int, cols: int, device) -> torch.Tensor:
    """Column-major FP64 copy of t (zeros when t is None)."""
    out = cqr.col_major(rows, cols, device)
    if t is not None:
        out.copy_(t)
    return out


def _factor(A, engine, schedule):
    """Encode A and factor it with the schedule's erasures and recoveries;
    returns the encoded matrix and R."""
    c = engine.cfg
    At, R = engine.alloc()
    At[:c.m, :c.n].copy_(A)
    engine.encode(At)
    k = 0
    for t, nodes in list(schedule) + [(c.npanels, None)]:
        engine.factor(At, R, k, t)
        k = t
        if nodes is None:
            break
        engine.erase(At, R, nodes)
        engine.recover(At, R, nodes)
    return At, R


class CodedQRFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, engine, schedule, recompute):
        c = engine.cfg
        At, R = _factor(A, engine, schedule)
        Q, R1 = At[:, :c.n], R[:c.n, :c.n]
        ctx.engine = engine
        ctx.schedule = schedule
        ctx.recompute = recompute
        if recompute:
            ctx.save_for_backward(A)
        else:
            ctx.save_for_backward(Q, R1)
        return Q, R1

    @staticmethod
    def backward(ctx, dQ, dR):
        engine = ctx.engine
        c = engine.cfg
        if ctx.recompute:
            (A,) = ctx.saved_tensors
            At, R = _factor(A, engine, ctx.schedule)
            Q, R1 = At[:, :c.n], R[:c.n, :c.n]
        else:
            Q, R1 = ctx.saved_tensors
        dQ = _colmajor(dQ, c.mp, c.n, Q.device)
        dR = _colmajor(dR, c.n, c.n, Q.device)
        return engine.backward(Q, R1, dQ, dR), None, None, None


class CodedSolveFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Q, R1, B, engine):
        c = engine.cfg
        Bc = _colmajor(B, c.m, B.shape[1], Q.device)
        Qpost = cqr.col_major(c.m, c.n, Q.device)
        Bpost = cqr.col_major(c.m, B.shape[1], Q.device)
        engine.postorth(Q, Qpost, Bc, Bpost)
        X = engine.solve(Qpost, R1, Bpost)
        ctx.engine = engine
        ctx.save_for_backward(Qpost, R1, Bpost, X)
        return X

    @staticmethod
    def backward(ctx, dX):
        engine = ctx.engine
        Qpost, R1, Bpost, X = ctx.saved_tensors
        dX = _colmajor(dX, X.shape[0], X.shape[1], X.device)
        dQ, dR, dB = engine.solve_backward(Qpost, R1, Bpost, X, dX)
        return dQ, dR, dB, None


def coded_qr(A: torch.Tensor, engine: "cqr.CodedQR", schedule=(), recompute: bool = False):
    """(Q~[:, :n], R_1) of the coded QR of A (m x n, FP64, on the engine's device).
    recompute: keep only A for the backward and factor again there."""
    return CodedQRFunction.apply(A, engine, list(schedule), bool(recompute))


def coded_solve(Q: torch.Tensor, R1: torch.Tensor, B: torch.Tensor, engine: "cqr.CodedQR") -> torch.Tensor:
    """X = R_1^{-1} (G_0 Q_1)^T (G_0 B) (n x nrhs)."""
    return CodedSolveFunction.apply(Q, R1, B, engine)

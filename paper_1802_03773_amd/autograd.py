"""torch.autograd.Function for the block-angular LM step.

Forward: factor + solve (optionally refined) in libqrkit.so.  Backward: the library's
adjoint, which reuses the stored R (two triangular solves) for u = (J^T J + lam D^2)^{-1} g
and writes dL/dA, dL/dB, dL/db on the structural nonzeros, dL/dlam and dL/dd.
"""
from __future__ import annotations

import torch

from .qrkit import BlockAngularSolver


class QRKSolve(torch.autograd.Function):
    """p = argmin || [J; sqrt(lam) D] p - [b; 0] ||, J = [blkdiag(A_i) | B].

    apply(A, B, b, d, lam, row_off, n, sweeps=1) -> p (float64, [K*n + nB]).
    A [M, n], B [M, nB], b [M] (float32 or float64, same dtype); d [N] float64; lam a
    float or a 0-dim float64 tensor; row_off a host int64 array of K+1 row offsets.
    """

    @staticmethod
    def forward(ctx, A, B, b, d, lam, row_off, n, sweeps=1):
        nB = 0 if B is None else int(B.shape[1])
        dtype = "float32" if A.dtype == torch.float32 else "float64"
        lam_f = float(lam) if not torch.is_tensor(lam) else float(lam.detach().cpu())
        solver = BlockAngularSolver(row_off, n, nB, dtype=dtype)
        Bc = B.detach().contiguous() if B is not None else None
        solver.factor(A.detach().contiguous(), Bc, b.detach().contiguous(), d.detach().contiguous(), lam_f)
        p = solver.solve(sweeps=int(sweeps))
        ctx.solver = solver
        ctx.lam_is_tensor = torch.is_tensor(lam)
        ctx.has_B = B is not None
        ctx.save_for_backward(p)
        return p

    @staticmethod
    def backward(ctx, gp):
        (p,) = ctx.saved_tensors
        want = []
        if ctx.needs_input_grad[0]:
            want.append("dA")
        if ctx.has_B and ctx.needs_input_grad[1]:
            want.append("dB")
        if ctx.needs_input_grad[2]:
            want.append("db")
        if ctx.needs_input_grad[3]:
            want.append("dd")
        if ctx.lam_is_tensor and ctx.needs_input_grad[4]:
            want.append("dlam")
        out = ctx.solver.solve_adjoint(p, gp.detach().to(torch.float64).contiguous(), want=tuple(want))
        dlam = out["dlam"].reshape(()) if "dlam" in out else None
        return (out.get("dA"), out.get("dB"), out.get("db"), out.get("dd"), dlam, None, None, None)

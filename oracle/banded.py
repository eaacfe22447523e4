"""Banded-J oracle: dense assembly of [J; sqrt(lam) D] and a plain QR solve.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Row i of J holds w values at columns row_start[i] .. row_start[i]+w-1 (the
banded problem class of Section 4.4).  The step is the least-squares solution
of Eq. 2; its R (unique up to row signs) has upper bandwidth w-1 when the
row starts are nondecreasing.  Small problems use O1 (hand-written Householder,
oracle.dense); larger ones use LAPACK QR (numpy.linalg.qr) on the same dense
assembly, followed by longdouble residual refinement as in oracle.refine.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import dense

LD = np.longdouble


def assemble(inst) -> np.ndarray:
    J = np.zeros((inst.M, inst.N), dtype=np.float64)
    rows = np.repeat(np.arange(inst.M), inst.w)
    cols = (inst.row_start.astype(np.int64)[:, None] + np.arange(inst.w)[None, :]).reshape(-1)
    J[rows, cols] = inst.vals.astype(np.float64).reshape(-1)
    return J


def solve_dense_o1(inst):
    J = assemble(inst)
    return dense.solve_augmented(J, inst.b.astype(np.float64), inst.d, inst.lam)


def factor_lapack(inst):
    """R (N x N) and c (N) of [J; sqrt(lam) D] with b carried as an extra column."""
    J = assemble(inst)
    N = inst.N
    aug = np.zeros((inst.M + N, N + 1))
    aug[:inst.M, :N] = J
    aug[:inst.M, N] = inst.b.astype(np.float64)
    aug[inst.M + np.arange(N), np.arange(N)] = np.sqrt(inst.lam) * np.asarray(inst.d, np.float64)
    Rr = np.linalg.qr(aug, mode="r")
    return Rr[:N, :N].copy(), Rr[:N, N].copy(), float(abs(Rr[N, N]))


def apply_J(inst, p, dt=LD):
    cols = inst.row_start.astype(np.int64)[:, None] + np.arange(inst.w)[None, :]
    return (inst.vals.astype(dt) * np.asarray(p).astype(dt)[cols]).sum(axis=1)


def apply_JT(inst, r, dt=LD):
    cols = inst.row_start.astype(np.int64)[:, None] + np.arange(inst.w)[None, :]
    g = np.zeros(inst.N, dtype=dt)
    np.add.at(g, cols.reshape(-1), (inst.vals.astype(dt) * np.asarray(r).astype(dt)[:, None]).reshape(-1))
    return g


def reference_solution(inst, sweeps: int = 2):
    """LAPACK QR solve + longdouble CSNE sweeps; returns (p_ref float64, R, c)."""
    R, c, _ = factor_lapack(inst)
    p = scipy.linalg.solve_triangular(R, c, lower=False).astype(LD)
    d = np.asarray(inst.d).astype(LD)
    for _ in range(sweeps):
        r = inst.b.astype(LD) - apply_J(inst, p)
        g = apply_JT(inst, r) - LD(inst.lam) * d * d * p
        y = scipy.linalg.solve_triangular(R, g.astype(np.float64), trans="T", lower=False)
        delta = scipy.linalg.solve_triangular(R, y, lower=False)
        p = p + delta.astype(LD)
    return p.astype(np.float64), R, c

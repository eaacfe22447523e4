"""O-ext: extended-precision residual refinement of an oracle solution.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Plain float64 QR is accurate only to about cond * 1e-16, which is too loose to
assess a result at the 1e-10 level.  The reference solution is therefore an
O1/O2 solution improved by corrected semi-normal-equation sweeps (Bjorck 1987)
whose residuals are evaluated in numpy.longdouble (80-bit x87 extended on
x86-64, eps = 2^-63):

  r = b - J p                   (longdouble)
  g = J^T r - lam D^2 p         (longdouble)   [the normal equations of Eq. 2]
  R^T R delta = g               (float64, the oracle's own R)
  p <- p + delta                (longdouble)

The fixed point is the exact least-squares solution of Eq. 2 for the stored
values of J, b, d and lam.
"""
from __future__ import annotations

import numpy as np

from . import structured

LD = np.longdouble


def apply_J(inst, p: np.ndarray, dt=LD) -> np.ndarray:
    """J p for a block-angular instance, in dtype dt."""
    K, n = inst.K, inst.n
    A = inst.A.astype(dt)
    B = inst.B.astype(dt)
    p = np.asarray(p).astype(dt)
    blk = inst.block_of_row()
    pb = p[:K * n].reshape(K, n)
    out = (A * pb[blk]).sum(axis=1)
    if inst.nB:
        out = out + B @ p[K * n:]
    return out


def apply_JT(inst, r: np.ndarray, dt=LD) -> np.ndarray:
    """J^T r for a block-angular instance, in dtype dt."""
    K, n = inst.K, inst.n
    A = inst.A.astype(dt)
    B = inst.B.astype(dt)
    r = np.asarray(r).astype(dt)
    blk = inst.block_of_row()
    g_blk = np.zeros((K, n), dtype=dt)
    np.add.at(g_blk, blk, A * r[:, None])
    g_B = B.T @ r if inst.nB else np.zeros(0, dtype=dt)
    return np.concatenate([g_blk.reshape(-1), g_B])


def normal_residual(inst, p: np.ndarray, dt=LD) -> np.ndarray:
    """g = J^T (b - J p) - lam D^2 p in dtype dt."""
    p = np.asarray(p).astype(dt)
    r = inst.b.astype(dt) - apply_J(inst, p, dt)
    d = np.asarray(inst.d).astype(dt)
    return apply_JT(inst, r, dt) - dt(inst.lam) * d * d * p


def refine(inst, factor, p0: np.ndarray, sweeps: int = 3) -> np.ndarray:
    """CSNE sweeps with longdouble residuals; returns p as longdouble."""
    p = np.asarray(p0).astype(LD)
    for _ in range(sweeps):
        g = normal_residual(inst, p, LD)
        delta = structured.solve_RtR(factor, g.astype(np.float64))
        p = p + delta.astype(LD)
    return p


def reference_solution(inst, sweeps: int = 3):
    """O2 + longdouble refinement: the parity reference p_ref (float64) and the factor."""
    p0, f = structured.solve_blockangular(inst)
    p = refine(inst, f, p0, sweeps)
    return p.astype(np.float64), f


def rel_err(p, p_ref) -> float:
    p = np.asarray(p, np.float64)
    p_ref = np.asarray(p_ref, np.float64)
    return float(np.linalg.norm(p - p_ref) / np.linalg.norm(p_ref))

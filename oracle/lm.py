"""Backtrack Levenberg-Marquardt (paper Section 5.2) on the synthetic LM workload, float64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Model.  f(x) = J0 phi(x) - y with the elementwise phi(t) = t + c t^3, so the Jacobian
J(x) = J0 diag(phi'(x)) keeps the sparsity of J0 (block-angular here; banded below).

One iteration, as in the Backtrack LM of Section 5.2 (damping rows permuted into J,
D = diag of the column norms of J(x), recomputed every iteration; a zero column gets 1):
    f = f(x),  J = J(x),  d = colnorms(J)
    p = argmin || [J; sqrt(lam) D] p - [-f; 0] ||          (Eq. 2 with b = -f)
    F = 1/2 ||f||^2,  F_new = 1/2 ||f(x + p)||^2
    pred = L(0) - L(p),  L(h) = 1/2 ||f + J h||^2,  which for the step above equals
           1/2 p^T (lam D^2 p - J^T f)
    rho = (F - F_new) / pred
    rho > 0:  x <- x + p,  lam <- lam * max(1/3, 1 - (2 rho - 1)^3),  nu <- 2
    else   :  lam <- lam * nu,  nu <- 2 nu
The paper says only that its lambda update adapts a published rule; the rule above is
Nielsen's gain-ratio rule (Madsen, Nielsen and Tingleff), the reading taken here.

Storage.  The GPU path keeps J(x) and -f in the factor's storage type; `store` rounds them
the same way here (float32 -> np.float32), so both sides solve the same instance.  The step
itself is computed in float64 and refined with longdouble residuals (oracle.refine); J^T f
in pred uses the stored J and the float64 f.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from oracle import banded as obanded
from oracle import refine as orefine


def phi(t, c):
    return t + c * t ** 3


def dphi(t, c):
    return 1.0 + 3.0 * c * t ** 2


def nielsen_update(lam: float, nu: float, rho: float):
    """(lam, nu, accepted) after a trial step with gain ratio rho."""
    if rho > 0.0:
        return lam * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3), 2.0, True
    return lam * nu, 2.0 * nu, False


def _colnorms(cols_sq: np.ndarray) -> np.ndarray:
    d = np.sqrt(cols_sq)
    d[d == 0.0] = 1.0
    return d


# --------------------------------------------------------------------------------------
# block-angular model: J0 = [blkdiag(A0_i) | B0]
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class BlockAngularModel:
    inst0: object      # generators.BlockAngular holding A0, B0 (b, d, lam unused)
    y: np.ndarray      # [M]
    c: float           # cubic coefficient of phi


def _block_cols(inst):
    """Column of each entry of A (row r, slot k) in the unknown vector."""
    blk = np.repeat(np.arange(inst.K), np.diff(inst.row_off))
    return blk[:, None] * inst.n + np.arange(inst.n)[None, :]


def ba_residual(model: BlockAngularModel, x: np.ndarray) -> np.ndarray:
    inst = model.inst0
    return np.asarray(orefine.apply_J(inst, phi(x, model.c), dt=np.float64), np.float64) - model.y


def ba_jacobian_instance(model: BlockAngularModel, x: np.ndarray, lam: float, store=np.float64):
    """The LM step instance at x: J(x) (stored as `store`), b = -f(x) (stored), D, lam."""
    inst = model.inst0
    Kn = inst.K * inst.n
    cols = _block_cols(inst)
    A = (inst.A.astype(np.float64) * dphi(x[cols], model.c)).astype(store)
    B = (inst.B.astype(np.float64) * dphi(x[Kn:], model.c)[None, :]).astype(store)
    f = ba_residual(model, x)
    b = (-f).astype(store)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    sq = np.zeros(inst.N)
    np.add.at(sq, cols.reshape(-1), (A64 ** 2).reshape(-1))
    sq[Kn:] = np.sum(B64 ** 2, axis=0)
    step = dataclasses.replace(inst, A=A, B=B, b=b, d=_colnorms(sq), lam=float(lam), dtype=np.dtype(store))
    return step, f


def ba_lm(model: BlockAngularModel, x0: np.ndarray, lam0: float, iters: int, store=np.float64):
    """Run `iters` Backtrack-LM iterations; returns (x, lam, log) with log rows
    (F, F_trial, lam_after, accepted)."""
    x = np.array(x0, np.float64)
    lam, nu = float(lam0), 2.0
    log = []
    for _ in range(iters):
        step, f = ba_jacobian_instance(model, x, lam, store)
        p, _ = orefine.reference_solution(step)
        F = 0.5 * float(f @ f)
        f_new = ba_residual(model, x + p)
        F_new = 0.5 * float(f_new @ f_new)
        JTf = np.asarray(orefine.apply_JT(step, f, dt=np.float64), np.float64)
        pred = 0.5 * float(p @ (lam * step.d ** 2 * p - JTf))
        rho = (F - F_new) / pred if pred > 0.0 else -1.0
        lam_new, nu, acc = nielsen_update(lam, nu, rho)
        log.append((F, F_new, lam_new, float(acc)))
        if acc:
            x = x + p
        lam = lam_new
    return x, lam, np.array(log)


# --------------------------------------------------------------------------------------
# banded model: J0 banded (row i: w values at columns s_i .. s_i + w - 1)
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class BandedModel:
    inst0: object      # generators.Banded holding row_start and vals0
    y: np.ndarray
    c: float


def bd_residual(model: BandedModel, x: np.ndarray) -> np.ndarray:
    return np.asarray(obanded.apply_J(model.inst0, phi(x, model.c), dt=np.float64), np.float64) - model.y


def bd_jacobian_instance(model: BandedModel, x: np.ndarray, lam: float, store=np.float64):
    inst = model.inst0
    cols = inst.row_start[:, None].astype(np.int64) + np.arange(inst.w)[None, :]
    vals = (inst.vals.astype(np.float64) * dphi(x[cols], model.c)).astype(store)
    f = bd_residual(model, x)
    sq = np.zeros(inst.N)
    np.add.at(sq, cols.reshape(-1), (vals.astype(np.float64) ** 2).reshape(-1))
    step = dataclasses.replace(inst, vals=vals, b=(-f).astype(store), d=_colnorms(sq), lam=float(lam),
                               dtype=np.dtype(store))
    return step, f


def bd_lm(model: BandedModel, x0: np.ndarray, lam0: float, iters: int, store=np.float64):
    x = np.array(x0, np.float64)
    lam, nu = float(lam0), 2.0
    log = []
    for _ in range(iters):
        step, f = bd_jacobian_instance(model, x, lam, store)
        p, _, _ = obanded.reference_solution(step)
        F = 0.5 * float(f @ f)
        f_new = bd_residual(model, x + p)
        F_new = 0.5 * float(f_new @ f_new)
        JTf = np.asarray(obanded.apply_JT(step, f, dt=np.float64), np.float64)
        pred = 0.5 * float(p @ (lam * step.d ** 2 * p - JTf))
        rho = (F - F_new) / pred if pred > 0.0 else -1.0
        lam_new, nu, acc = nielsen_update(lam, nu, rho)
        log.append((F, F_new, lam_new, float(acc)))
        if acc:
            x = x + p
        lam = lam_new
    return x, lam, np.array(log)

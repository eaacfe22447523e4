"""Pins of the Backtrack-LM oracle (oracle/lm.py) against facts that do not come from it:
the lambda rule's values worked by hand, closed forms of a linear model (gain ratio exactly
1, convergence to the LAPACK least-squares solution), the predicted decrease evaluated
directly from its definition, stationarity on the nonlinear model, and a planted mistake."""
import dataclasses

import numpy as np
import pytest

from oracle import dense, lm
from workloads import generators as gen


def test_nielsen_rule_values():
    # rho = 1: factor max(1/3, 1 - 1) = 1/3;  rho = 1/2: 1 - 0 = 1;  rho = 3/4: 1 - 1/8
    assert lm.nielsen_update(1.0, 2.0, 1.0) == (pytest.approx(1.0 / 3.0), 2.0, True)
    assert lm.nielsen_update(3.0, 8.0, 0.5) == (pytest.approx(3.0), 2.0, True)
    assert lm.nielsen_update(2.0, 4.0, 0.75) == (pytest.approx(2.0 * 0.875), 2.0, True)
    # small positive rho: 1 - (2 rho - 1)^3 -> about 2 (damping grows but the step is taken)
    assert lm.nielsen_update(1.0, 2.0, 1e-9)[0] == pytest.approx(2.0, rel=1e-7)
    # rejection: lam * nu, nu doubles
    assert lm.nielsen_update(0.5, 2.0, -0.3) == (1.0, 4.0, False)
    assert lm.nielsen_update(0.5, 4.0, 0.0) == (2.0, 8.0, False)


def _small_model(c, store=np.float64):
    inst0, y, x0, x_true = gen.lm_blockangular(11, K=20, m=6, n=3, nB=5, c=c, dtype=store)
    return lm.BlockAngularModel(inst0, y.astype(np.float64), c), x0, x_true


def _dense_J0(inst0):
    J = np.zeros((inst0.M, inst0.N))
    for i in range(inst0.K):
        r0, r1 = inst0.row_off[i], inst0.row_off[i + 1]
        J[r0:r1, i * inst0.n:(i + 1) * inst0.n] = inst0.A[r0:r1]
    J[:, inst0.K * inst0.n:] = inst0.B
    return J


def test_linear_model_gain_ratio_one_and_lstsq_limit():
    """c = 0: f is affine, so L(p) = F(x + p) exactly: rho = 1 at every step (lam / 3 each
    time) and the iterates reach the least-squares solution of J0 x = y (LAPACK lstsq)."""
    model, x0, _ = _small_model(0.0)
    x, lam, log = lm.ba_lm(model, x0, 1e-2, 25)
    _check_linear_log(log, 1e-2)
    x_ls = np.linalg.lstsq(_dense_J0(model.inst0), model.y, rcond=None)[0]
    assert np.linalg.norm(x - x_ls) <= 1e-10 * np.linalg.norm(x_ls)


def _check_linear_log(log, lam0):
    """While the cost still drops by more than roundoff, every step is accepted and lam is
    divided by exactly 3 (rho = 1); once at the minimum the decrease is roundoff only."""
    real = (log[:, 0] - log[:, 1]) > 1e-9 * log[:, 0]
    k = int(np.argmin(real)) if not real.all() else len(real)
    assert k >= 3 and not real[k:].any()
    assert np.all(log[:k, 3] == 1.0)
    np.testing.assert_allclose(log[:k, 2], lam0 * (1.0 / 3.0) ** np.arange(1, k + 1), rtol=1e-6)


def test_predicted_decrease_matches_its_definition():
    """pred = 1/2 p^T (lam D^2 p - J^T f) must equal L(0) - L(p) = 1/2|f|^2 - 1/2|f + J p|^2
    with J assembled densely (dense.assemble_blockangular's J part)."""
    model, x0, _ = _small_model(0.1)
    lam = 0.3
    step, f = lm.ba_jacobian_instance(model, x0, lam)
    from oracle import refine
    p, _ = refine.reference_solution(step)
    J = _dense_J0(step)  # same block structure, entries of J(x0)
    direct = 0.5 * (f @ f) - 0.5 * np.sum((f + J @ p) ** 2)
    pred = 0.5 * p @ (lam * step.d ** 2 * p - J.T @ f)
    assert abs(pred - direct) <= 1e-10 * abs(direct)


def test_nonlinear_model_reaches_stationarity():
    model, x0, _ = _small_model(0.1)
    x, lam, log = lm.ba_lm(model, x0, 1e-2, 30)
    acc = log[log[:, 3] == 1.0]
    assert np.all(np.diff(acc[:, 1]) <= 0.0)  # accepted costs never increase

    def grad(xx):
        step, f = lm.ba_jacobian_instance(model, xx, 1.0)
        return _dense_J0(step).T @ f

    assert np.linalg.norm(grad(x)) <= 1e-9 * np.linalg.norm(grad(x0))


def test_planted_wrong_jacobian_is_caught():
    """A Jacobian that ignores phi' (a plausible mistake) stalls away from stationarity."""
    model, x0, _ = _small_model(0.1)

    orig = lm.ba_jacobian_instance

    def wrong_jac(model_, x, lam, store=np.float64):
        step, f = orig(dataclasses.replace(model_, c=0.0), x, lam, store)
        f = lm.ba_residual(model_, x)
        return dataclasses.replace(step, b=(-f).astype(store)), f

    try:
        lm.ba_jacobian_instance = wrong_jac
        x, _, _ = lm.ba_lm(model, x0, 1e-2, 30)
    finally:
        lm.ba_jacobian_instance = orig

    def grad(xx):
        step, f = lm.ba_jacobian_instance(model, xx, 1.0)
        return _dense_J0(step).T @ f

    assert np.linalg.norm(grad(x)) > 1e-6 * np.linalg.norm(grad(x0))


def test_banded_linear_model_lstsq_limit():
    inst0, y, x0, _ = gen.lm_banded(21, N=60, w=5, c=0.0, dtype=np.float64)
    model = lm.BandedModel(inst0, y.astype(np.float64), 0.0)
    x, lam, log = lm.bd_lm(model, x0, 1e-2, 25)
    _check_linear_log(log, 1e-2)
    J = np.zeros((inst0.M, inst0.N))
    for i in range(inst0.M):
        J[i, inst0.row_start[i]:inst0.row_start[i] + inst0.w] = inst0.vals[i]
    x_ls = np.linalg.lstsq(J, model.y, rcond=None)[0]
    assert np.linalg.norm(x - x_ls) <= 1e-10 * np.linalg.norm(x_ls)

"""Pins of the oracle's camera-block J (the bundle-adjustment Jacobian of Section 6.2, solved as
the horizontal concatenation of Section 4.2): every row touches its point block and at most one
camera of cw columns.  The dense B the oracle assembles is checked against products written
row by row from that definition (J x and J^T y), the camera Gram matrix is block diagonal, the
generator's d is the column norms of the assembled J, rows without a camera contribute nothing,
and the structured oracle on the assembled problem equals LAPACK's least-squares solution.
Planted mistakes: cameras shifted by one column block, and a wrong camera width, both fail the
row-by-row products."""
import numpy as np
import pytest

from oracle import dense, structured
from workloads import generators as gen


def _instance(seed, K=30, ncam=5, cw=4, prior_rows=1, lam=1e-2):
    obs = (np.arange(K) % ncam) + 1
    return gen.make_blockangular_cam(seed, K=K, obs=obs, ncam=ncam, cw=cw, n=3, lam=lam, prior_rows=prior_rows)


def _row_products(inst, x, y):
    """J x and J^T y from the definition, one row at a time."""
    K, n, cw, ncam = inst.K, inst.n, inst.cw, inst.ncam
    Kn = K * n
    Jx = np.zeros(inst.M)
    JTy = np.zeros(inst.N)
    for i in range(K):
        for r in range(int(inst.row_off[i]), int(inst.row_off[i + 1])):
            a = inst.A[r].astype(np.float64)
            Jx[r] = a @ x[i * n:(i + 1) * n]
            JTy[i * n:(i + 1) * n] += a * y[r]
            c = int(inst.cam[r])
            if 0 <= c < ncam:
                bv = inst.Bv[r].astype(np.float64)
                Jx[r] += bv @ x[Kn + c * cw:Kn + (c + 1) * cw]
                JTy[Kn + c * cw:Kn + (c + 1) * cw] += bv * y[r]
    return Jx, JTy


def _product_error(inst, B):
    """Largest difference between the products of [blkdiag(A_i) | B] and the definition's."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal(inst.N)
    y = rng.standard_normal(inst.M)
    ba = gen.BlockAngular(inst.row_off, inst.n, inst.A, B, inst.b, inst.d, inst.lam, inst.dtype)
    J = dense.assemble_blockangular(ba)
    Jx, JTy = _row_products(inst, x, y)
    return max(np.abs(J @ x - Jx).max(), np.abs(J.T @ y - JTy).max())


@pytest.mark.parametrize("seed,cw,ncam", [(0, 4, 5), (1, 9, 14), (2, 1, 3)])
def test_assembly_matches_row_definition(seed, cw, ncam):
    inst = _instance(seed, ncam=ncam, cw=cw)
    assert _product_error(inst, dense.camera_columns(inst)) < 1e-12


def test_planted_camera_shift_and_width_fail():
    inst = _instance(3)
    B = dense.camera_columns(inst)
    shifted = np.roll(B, inst.cw, axis=1)          # camera c's values in camera c+1's columns
    assert _product_error(inst, shifted) > 1e-3
    wrong_w = np.zeros_like(B)                     # a width one short: the last column lost
    for r in range(inst.M):
        c = int(inst.cam[r])
        if 0 <= c < inst.ncam:
            wrong_w[r, c * inst.cw:c * inst.cw + inst.cw - 1] = inst.Bv[r, :inst.cw - 1]
    assert _product_error(inst, wrong_w) > 1e-3


def test_camera_gram_is_block_diagonal():
    inst = _instance(4, ncam=6, cw=3)
    B = dense.camera_columns(inst)
    G = B.T @ B
    cw = inst.cw
    for c1 in range(inst.ncam):
        for c2 in range(inst.ncam):
            blk = G[c1 * cw:(c1 + 1) * cw, c2 * cw:(c2 + 1) * cw]
            if c1 != c2:
                assert np.all(blk == 0.0)
            else:
                rows = inst.cam == c1
                Bv = inst.Bv[rows].astype(np.float64)
                np.testing.assert_allclose(blk, Bv.T @ Bv, rtol=1e-13, atol=1e-13)


def test_rows_without_a_camera_contribute_nothing():
    inst = _instance(5, prior_rows=2)
    none = np.nonzero(inst.cam < 0)[0]
    assert none.size == 2 * inst.K
    B = dense.camera_columns(inst)
    assert np.all(B[none] == 0.0)
    # a camera index past the last camera is no camera either
    inst.cam[none[::2]] = inst.ncam + 3
    assert np.array_equal(dense.camera_columns(inst), B)
    # and the ignored Bv rows may hold anything
    inst.Bv[none] = 1e30
    assert np.array_equal(dense.camera_columns(inst), B)


def test_generator_observations():
    inst = _instance(6, K=40, ncam=7, prior_rows=1)
    for i in range(inst.K):
        r0, r1 = int(inst.row_off[i]), int(inst.row_off[i + 1])
        cams = inst.cam[r0:r1 - 1]
        assert inst.cam[r1 - 1] == -1
        assert np.array_equal(cams[0::2], cams[1::2])          # x and y rows on one camera
        assert np.unique(cams[0::2]).size == cams.size // 2     # distinct cameras per point
        assert cams.min() >= 0 and cams.max() < inst.ncam


def test_d_is_column_norms_of_assembled_J():
    inst = _instance(7, ncam=6, cw=5)
    inst_nocam = gen.make_blockangular_cam(8, K=6, obs=1, ncam=9, cw=2)  # cameras nobody sees
    for it in (inst, inst_nocam):
        J = dense.assemble_blockangular(dense.blockangular_from_cam(it))
        ref = np.sqrt((J * J).sum(axis=0))
        ref[ref == 0.0] = 1.0
        np.testing.assert_allclose(it.d, ref, rtol=1e-14)
    assert np.any(inst_nocam.d[inst_nocam.K * 3:] == 1.0)


@pytest.mark.parametrize("lam", [1e-4, 1e-2, 1.0])
def test_structured_solution_is_least_squares(lam):
    inst = _instance(9, K=50, ncam=6, cw=4, lam=lam)
    ba = dense.blockangular_from_cam(inst)
    J = dense.assemble_blockangular(ba)
    Aaug = np.vstack([J, np.sqrt(lam) * np.diag(inst.d)])
    rhs = np.concatenate([inst.b.astype(np.float64), np.zeros(inst.N)])
    p_ls, *_ = np.linalg.lstsq(Aaug, rhs, rcond=None)
    p, _ = structured.solve_blockangular(ba)
    np.testing.assert_allclose(p, p_ls, rtol=1e-10, atol=1e-12)

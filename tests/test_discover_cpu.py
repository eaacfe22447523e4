"""Structure discovery (qrk_discover_blockangular, qrk_discover_banded: the row and column
permutations of Section 4.3), host code of the library called through the C ABI, against the
oracle's definitions (oracle/permute.py): the block partition (the unique part) equal as sets,
the conventions (block order, order inside blocks, stable banded order) equal exactly, the
permuted pattern checked to have the structure, and the refusals."""
import numpy as np
import pytest

from oracle import permute
from paper_1802_03773_amd import QRKError, discover_banded, discover_blockangular
from workloads import generators as gen


def _csr(rows):
    row_ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col_idx = np.array([c for r in rows for c in r], dtype=np.int32)
    return row_ptr, col_idx


def _shuffled_blockangular(seed, K=80, nB=11):
    inst = gen.make_blockangular_ncol(seed, K=K, m=(np.arange(K) % 7) + 1, ncol=(np.arange(K) * 5) % 8 + 1,
                                      nB=nB, lam=1e-2)
    po = inst.p_off()
    nd = int(po[K])
    rows = []
    for i in range(K):
        for _ in range(int(inst.row_off[i + 1] - inst.row_off[i])):
            rows.append(list(range(int(po[i]), int(po[i + 1]))) + list(range(nd, nd + nB)))
    rng = np.random.default_rng(seed)
    pr = rng.permutation(inst.M)
    pc = rng.permutation(inst.N)
    inv_c = np.argsort(pc)
    srows = [list(rng.permutation([int(inv_c[c]) for c in rows[int(pr[k])]])) for k in range(inst.M)]
    dense = [int(inv_c[c]) for c in range(nd, inst.N)]
    return inst, srows, dense


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_blockangular_matches_oracle(seed):
    inst, rows, dense = _shuffled_blockangular(seed)
    M, N = inst.M, inst.N
    rp, ci = _csr(rows)
    got = discover_blockangular(rp, ci, N, dense)
    ref = permute.blockangular_blocks(M, N, rows, dense)
    assert ref[-1] == ([], [])
    K = got["K"]
    assert K == len(ref) - 1 == inst.K
    co = np.concatenate([[0], np.cumsum(got["ncol"])])
    for b, (cols, rs) in enumerate(ref[:-1]):  # the same blocks in the same order, exactly
        assert got["col_perm"][co[b]:co[b + 1]].tolist() == cols
        assert got["row_perm"][got["row_off"][b]:got["row_off"][b + 1]].tolist() == rs
    assert got["col_perm"][co[K]:].tolist() == dense
    # the permuted pattern is block-angular: row k of J' touches its block's columns and dense ones
    newcol = np.empty(N, dtype=np.int64)
    newcol[got["col_perm"]] = np.arange(N)
    for b in range(K):
        for k in range(int(got["row_off"][b]), int(got["row_off"][b + 1])):
            cols = newcol[rows[int(got["row_perm"][k])]]
            local = cols[cols < co[K]]
            assert np.all((local >= co[b]) & (local < co[b + 1]))
    assert sorted(got["row_perm"].tolist()) == list(range(M))


def test_rows_with_dense_columns_only_and_untouched_columns():
    rows = [[0, 1, 9], [1, 9], [2, 3], [9], [8, 9], [5]]  # column 4, 6, 7 untouched; row 3 dense only
    rp, ci = _csr(rows)
    got = discover_blockangular(rp, ci, 10, [8, 9])
    # blocks by smallest column: {0,1} rows {0,1}; {2,3} rows {2}; {4}; {5} row {5}; {6}; {7}
    assert got["K"] == 6
    assert got["ncol"].tolist() == [2, 2, 1, 1, 1, 1]
    assert got["col_perm"].tolist() == [0, 1, 2, 3, 4, 5, 6, 7, 8, 9]
    blocks = [got["row_perm"][got["row_off"][b]:got["row_off"][b + 1]].tolist() for b in range(got["K"])]
    # rows touching only dense columns (3 and 4) go to the first block with room
    assert blocks == [[0, 1, 3, 4], [2], [], [5], [], []]


def test_banded_matches_oracle():
    b = gen.make_banded(9, N=400, w=12)
    rng = np.random.default_rng(5)
    rows0 = [list(range(int(s), int(s) + 12)) for s in b.row_start]
    rows0[7] = rows0[7][3:9]                      # a row narrower than the band
    pr = rng.permutation(len(rows0))
    rows = [list(rng.permutation(rows0[int(k)])) for k in pr]
    rp, ci = _csr(rows)
    got = discover_banded(rp, ci, 400)
    order, starts, w = permute.banded_order(rows)
    assert got["w"] == w == 12
    assert np.array_equal(got["row_perm"], order)
    assert np.array_equal(got["row_start"], np.minimum(starts, 400 - w))
    for k, r in enumerate(got["row_perm"]):       # every row's columns inside its band
        c = np.asarray(rows[int(r)])
        assert c.min() >= got["row_start"][k] and c.max() < got["row_start"][k] + w


def test_refusals():
    wide = [list(range(9)) + [20]]                # a block of nine columns
    rp, ci = _csr(wide)
    with pytest.raises(QRKError):
        discover_blockangular(rp, ci, 21, [20])
    tall = [[0, 5] for _ in range(57)]            # a block of 57 rows
    rp, ci = _csr(tall)
    with pytest.raises(QRKError):
        discover_blockangular(rp, ci, 6, [5])
    rp, ci = _csr([[0, 1], [1, 2]])
    with pytest.raises(QRKError):
        discover_blockangular(rp, ci, 3, [2, 2])  # repeated dense column
    with pytest.raises(QRKError):
        discover_blockangular(rp, np.array([0, 1, 1, 7], dtype=np.int32), 3, [2])  # index out of range
    rp, ci = _csr([[0, 40], [1, 2]])
    with pytest.raises(QRKError):
        discover_banded(rp, ci, 50)               # band wider than 31
    rp, ci = _csr([[0, 1], []])
    with pytest.raises(QRKError):
        discover_banded(rp, ci, 5)                # an empty row

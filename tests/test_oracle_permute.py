"""Pins of the oracle's structure discovery (Section 4.3: row and column permutations that reveal
block-angular or banded structure).  A block-angular J generated with known blocks and then
shuffled by random row and column permutations must give back exactly the generated blocks (as
sets, mapped through the permutations); the partition is checked against its definition (every
row's non-dense columns in one block, no block splittable); a banded J with shuffled rows must
come back with nondecreasing starts and its band width; planted mistake: listing no dense
columns merges every block into one."""
import numpy as np

from oracle import permute
from workloads import generators as gen


def _ragged_pattern(inst):
    """Each row's columns (block columns, then the dense ones) of a per-block-width instance."""
    po = inst.p_off()
    rows = []
    nd = int(po[inst.K])
    for i in range(inst.K):
        cols = list(range(int(po[i]), int(po[i + 1])))
        for _ in range(int(inst.row_off[i + 1] - inst.row_off[i])):
            rows.append(cols + list(range(nd, nd + inst.nB)))
    return rows


def _shuffle(rows, M, N, seed):
    rng = np.random.default_rng(seed)
    pr = rng.permutation(M)      # new row k is old row pr[k]
    pc = rng.permutation(N)      # new column j is old column pc[j]
    inv_c = np.argsort(pc)       # old column c is new column inv_c[c]
    return [sorted(int(inv_c[c]) for c in rows[int(pr[k])]) for k in range(M)], pr, pc, inv_c


def test_blocks_recovered_through_random_permutations():
    inst = gen.make_blockangular_ncol(5, K=60, m=(np.arange(60) % 6) + 1, ncol=(np.arange(60) * 3) % 8 + 1,
                                      nB=9, lam=1e-2)
    rows = _ragged_pattern(inst)
    M, N = inst.M, inst.N
    srows, pr, pc, inv_c = _shuffle(rows, M, N, 17)
    nd = int(inst.p_off()[inst.K])
    dense_new = [int(inv_c[c]) for c in range(nd, N)]
    blocks = permute.blockangular_blocks(M, N, srows, dense_new)
    assert blocks[-1] == ([], [])                     # every row touches a block column
    got = {frozenset(int(pc[c]) for c in cols): frozenset(int(pr[r]) for r in rs) for cols, rs in blocks[:-1]}
    po = inst.p_off()
    want = {frozenset(range(int(po[i]), int(po[i + 1]))):
            frozenset(range(int(inst.row_off[i]), int(inst.row_off[i + 1]))) for i in range(inst.K)}
    assert got == want


def test_partition_meets_its_definition():
    rng = np.random.default_rng(3)
    M, N = 200, 60
    dense = [57, 58, 59]
    rows = [sorted(set(rng.choice(57, size=rng.integers(1, 3)).tolist()) | set(rng.choice(dense, 1).tolist()))
            for _ in range(M)]
    rows += [[58], [57, 59]]                          # rows with dense columns only
    blocks = permute.blockangular_blocks(M + 2, N, rows, dense)
    where = {}
    for b, (cols, _) in enumerate(blocks[:-1]):
        for c in cols:
            assert c not in where                     # columns in one block only
            where[c] = b
    for i, cols in enumerate(rows):
        local = [c for c in cols if c not in dense]
        assert len({where[c] for c in local}) <= 1    # a row's local columns in one block
        in_block = [b for b, (_, rs) in enumerate(blocks) if i in rs]
        assert len(in_block) == 1                     # every row listed once
    assert blocks[-1][1] == [M, M + 1]
    for cols, rs in blocks[:-1]:                      # no block splits: its columns are connected
        adj = {c: set() for c in cols}
        for i in rs:
            loc = [c for c in rows[i] if c not in dense]
            for a in loc:
                adj[a].update(loc)
        seen, stack = {cols[0]}, [cols[0]]
        while stack:
            for nb in adj[stack.pop()]:
                if nb not in seen:
                    seen.add(nb)
                    stack.append(nb)
        assert seen == set(cols)


def test_planted_mistake_without_dense_columns_is_one_block():
    inst = gen.make_blockangular_ncol(7, K=20, m=3, ncol=2, nB=4, lam=1e-2)
    rows = _ragged_pattern(inst)
    blocks = permute.blockangular_blocks(inst.M, inst.N, rows, [])
    assert len(blocks) == 2 and len(blocks[0][0]) == inst.N


def test_banded_rows_recovered():
    b = gen.make_banded(9, N=300, w=12)
    rows = [list(range(int(s), int(s) + 12)) for s in b.row_start]
    rng = np.random.default_rng(4)
    pr = rng.permutation(len(rows))
    order, starts, w = permute.banded_order([rows[int(k)] for k in pr])
    assert w == 12
    assert np.all(np.diff(starts) >= 0)
    assert np.array_equal(np.sort(b.row_start), starts)
    assert sorted(pr[order].tolist()) == list(range(len(rows)))

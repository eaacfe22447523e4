"""Row and column permutations that reveal the structure of a sparse J (Section 4.3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper permutes rows (P_r) and columns (P_c) of a sparse matrix so that one of its structured
solvers applies: J' = P_r J P_c.  It names no algorithm beyond the search for an
as-banded-as-possible row order; the plain definitions used here are:

  block-angular: with the coupled (dense) columns given, two rows belong to the same block when
      they share a non-dense column, transitively (connected components of the bipartite
      row / non-dense-column graph).  A block's columns are the non-dense columns of its rows.
      Rows that touch only dense columns belong to no component; they are placed in blocks
      afterwards (first block in order with room).
  banded: rows ordered by their first column (stable), so row starts are nondecreasing; the
      band width is the largest last-minus-first column + 1 over the rows.

The unique parts are the partition of columns and rows into blocks (as sets) and the multiset
of row starts; the block order and the order inside a block are conventions (here: blocks by
smallest column, columns and rows in increasing original order).
"""
from __future__ import annotations

import numpy as np


def blockangular_blocks(M: int, N: int, rows: list, dense_cols) -> list:
    """Blocks of a sparse J given as a list of each row's column indices: a list of
    (columns, rows) pairs, both sorted, blocks in order of their smallest column; rows with
    only dense columns are not in any block (returned last as ([], orphan_rows))."""
    dense = set(int(c) for c in dense_cols)
    col_rows: dict[int, list] = {}
    for i, cols in enumerate(rows):
        for c in cols:
            if int(c) not in dense:
                col_rows.setdefault(int(c), []).append(i)
    seen_row = [False] * M
    seen_col: set = set()
    blocks = []
    for c0 in sorted(col_rows):
        if c0 in seen_col:
            continue
        # breadth-first search over the bipartite graph from column c0
        bcols, brows = {c0}, set()
        seen_col.add(c0)
        frontier = [c0]
        while frontier:
            nxt = []
            for c in frontier:
                for i in col_rows[c]:
                    if seen_row[i]:
                        continue
                    seen_row[i] = True
                    brows.add(i)
                    for c2 in rows[i]:
                        c2 = int(c2)
                        if c2 not in dense and c2 not in seen_col:
                            seen_col.add(c2)
                            bcols.add(c2)
                            nxt.append(c2)
            frontier = nxt
        blocks.append((sorted(bcols), sorted(brows)))
    orphans = [i for i in range(M) if not seen_row[i]]
    blocks.append(([], orphans))
    return blocks


def banded_order(rows: list):
    """(row order, starts in that order, band width): rows sorted stably by first column."""
    first = np.array([min(int(c) for c in cols) for cols in rows], dtype=np.int64)
    last = np.array([max(int(c) for c in cols) for cols in rows], dtype=np.int64)
    order = np.argsort(first, kind="stable")
    return order, first[order], int((last - first).max() + 1) if len(rows) else 0

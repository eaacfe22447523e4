"""Host-side grouping of a batch's blocks into per-block QR classes (blocks with m_i >= n:
register rows 16/32/64 times column slots 1/2; blocks with m_i < n: column slots 1/2),
compiled from the library's own header with the host compiler.

The per-block QR launches walk, for every class c, the positions begin[c] .. begin[c] +
count[c] - 1 of the block list, or of the identity 0 .. K-1 when no list was built.  These
tests check that this walk stays inside the list (or inside 0 .. K-1), visits every block
exactly once, and that each block's class holds its rows and coupled columns (the kernels with
compile-time n keep the damping rows at fixed register rows, which needs m_i >= n)."""
import pathlib
import shutil
import subprocess

import numpy as np
import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
HDR = ROOT / "paper_1802_03773_amd" / "csrc"

DRIVER = r"""
#include <cstdio>
#include "block_classes.hpp"
int main() {
  long long K; int n;
  if (scanf("%lld %d", &K, &n) != 2) return 2;
  std::vector<int64_t> row_off((size_t)K + 1);
  for (auto& r : row_off) { long long v; if (scanf("%lld", &v) != 1) return 2; r = v; }
  std::vector<int> L((size_t)K);
  for (auto& l : L) if (scanf("%d", &l) != 1) return 2;
  qrk::BlockClasses bc;
  bool ok = qrk::group_block_classes(row_off.data(), K, n, [&](int64_t i) { return L[(size_t)i]; }, bc);
  printf("%d\n", ok ? 1 : 0);
  for (int c = 0; c < qrk::kBlockClasses; ++c)
    printf("%lld %lld %d %d %d\n", (long long)bc.begin[c], (long long)bc.count[c], qrk::block_class_rows(c),
           qrk::block_class_slots(c), qrk::block_class_short(c) ? 1 : 0);
  printf("%zu\n", bc.list.size());
  for (int32_t b : bc.list) printf("%d\n", b);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("bq")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", str(HDR), str(src), "-o", str(exe)], check=True)
    return exe


def _group(exe, m, n, L):
    K = len(m)
    row_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    text = f"{K} {n}\n" + " ".join(map(str, row_off)) + "\n" + " ".join(map(str, L)) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    ok = out[0] == "1"
    cls = [tuple(int(v) for v in out[1 + c].split()) for c in range(8)]
    nl = int(out[9])
    lst = [int(v) for v in out[10:10 + nl]]
    return ok, cls, lst


def _walk(cls, lst, K):
    """Blocks visited by the per-class launches, exactly as the host enqueues them."""
    extent = len(lst) if lst else K
    seen = []
    for c, (begin, count, rows, slots, short) in enumerate(cls):
        if count == 0:
            continue
        assert 0 <= begin and begin + count <= extent, (c, begin, count, extent)
        for it in range(count):
            blk = lst[begin + it] if lst else begin + it
            seen.append((blk, rows, slots, short))
    return seen


@pytest.mark.parametrize("seed", range(12))
def test_walk_covers_every_block_once_in_a_fitting_class(driver, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    K = int(rng.integers(0, 400))
    # m_i + n <= 64; mix of single-class and many-class batches
    if seed % 3 == 0:
        m = np.full(K, min(8, 64 - n), dtype=np.int64)
    else:
        m = rng.integers(0, 64 - n + 1, size=K)
    # problems: consecutive runs of blocks sharing one L
    L = np.empty(K, dtype=np.int64)
    i = 0
    while i < K:
        run = int(rng.integers(1, 60))
        L[i:i + run] = int(rng.integers(1, 129)) if seed % 4 else 31
        i += run
    ok, cls, lst = _group(driver, m, n, L)
    assert ok
    seen = _walk(cls, lst, K)
    assert sorted(b for b, _, _, _ in seen) == list(range(K))
    for blk, rows, slots, short in seen:
        assert m[blk] + n <= rows
        assert L[blk] <= 64 * slots
        assert bool(short) == (m[blk] < n)
    used = sum(1 for c in cls if c[1] > 0)
    # a list exists exactly when more than one class is used
    assert (len(lst) > 0) == (used > 1)


def test_single_class_uses_identity(driver):
    ok, cls, lst = _group(driver, np.full(50, 5), 3, np.full(50, 20))
    assert ok and lst == []
    assert [c[1] for c in cls] == [50, 0, 0, 0, 0, 0, 0, 0]
    assert _walk(cls, lst, 50) == [(b, 16, 1, 0) for b in range(50)]


def test_short_blocks_get_their_own_class(driver):
    m = np.array([2, 5, 1, 40, 0, 3])
    ok, cls, lst = _group(driver, m, 3, np.full(6, 91))
    assert ok
    counts = [c[1] for c in cls]
    assert counts[7] == 3 and counts[1] == 2 and counts[5] == 1, counts
    seen = _walk(cls, lst, 6)
    assert sorted(b for b, _, _, _ in seen) == list(range(6))


def test_rejects_block_width_outside_range(driver):
    assert not _group(driver, np.array([10, 10]), 9, np.array([5, 5]))[0]


def test_rejects_blocks_that_fit_no_class(driver):
    assert not _group(driver, np.array([10, 62]), 3, np.array([5, 5]))[0]
    assert not _group(driver, np.array([10, 10]), 3, np.array([5, 129]))[0]

"""CPU float64 oracle for the structured-QR Levenberg-Marquardt step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path (no kernels,
headers, helpers or constant tables); the only common module is
``workloads.generators``, which draws seeded inputs and holds none of the
method's arithmetic.

What it computes (paper, Section 1, Eqs. 1-2): the LM step
    p* = argmin_p || [J; sqrt(lam) D] p - [b; 0] ||_2 = (J^T J + lam D^2)^{-1} J^T b.

Modules
  dense      - O1: assemble [J; sqrt(lam) D] densely, textbook Householder QR
               (Section 2), back-substitution.  Small problems.
  structured - O2: the block-angular factorisation of Section 4.2 (horizontal
               concatenation of the block-diagonal part of Section 4.1 and a
               dense part), with LAPACK QR as the per-block and dense-part step.
  refine     - O-ext: extended-precision (numpy.longdouble) residual refinement
               of an O1/O2 solution; the reference for all parity numbers.
  banded     - banded J (Section 4.4 problem class): dense assembly + O1 / LAPACK.
  block_banded - the block-banded factorisation of Section 4.4: dense steps over column
               blocks, each applied in the compressed WY form (Eq. blockBandedYTY).
  adjoint    - gradient of a loss of p* with respect to J, b, lam, d (closed
               form from differentiating Eq. 1).
  bf16       - bit-level emulation of bf16 rounding and the three-product split.
  lm         - a Backtrack-LM loop (Section 5.2) for the synthetic LM workload.

Parity status: every function is pinned by tests/test_oracle_*.py against
closed forms, exact rational arithmetic, LAPACK special cases or invariants,
except where a module header says "parity unpinned".
"""

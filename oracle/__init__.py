"""CPU FP64 oracle for inner-outer Krylov recycling (arXiv:1602.00138).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package; the
GPU library never does, and this package imports nothing from it.  It is written
for reading against the paper, not for speed: explicit scipy.sparse CSR
operators, dense NumPy/SciPy factorizations, one right-hand side at a time.

Modules
  operator  -- the SPD Schur-complement operator of Sec. 3 and eq. (sum), the
               full boundary-node system of eq. (block1), the RBF absorption.
  krylov    -- CGS2 append with truncation, Galerkin outer projection, deflated CG.
  sequence  -- Algorithm 2 (recycling and global basis construction) in CG form.
  rom       -- the reduced matrices of eq. (newreduced) and transfer functions.

Parity status: every function here is pinned by a CPU test against something
other than itself (closed forms, the full boundary-node system, dense Cholesky,
textbook CG, brute force on tiny grids).  Iteration counts and appended-column
counts on the synthetic workloads cannot be pinned to the paper's tables (a
different problem): parity unpinned for those counts.
"""

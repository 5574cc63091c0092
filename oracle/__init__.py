"""FP64 CPU oracle for BST backprojection -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. The GPU library never calls it and shares no code with it.

Contents (each function cites the passage of the paper it follows):
  geometry    detector / image / angle grids of the problem statement (Section 1)
  bruteforce  pixel-driven backprojection B_d (Eq. 2) and its transpose R_d (Eq. 1)
  ramp        band-limited spatial ramp filter for brute-force FBP (Section 1, F)
  bst         the BST backprojection, steps P0..P8 in order (Section 2, Eq. 3)
  bst_naive   the same steps with literal DFT sums and per-point loops (tiny sizes)

Every function is pinned by a `-m "not gpu"` test against closed forms,
invariants or brute force; none is marked parity unpinned.
"""

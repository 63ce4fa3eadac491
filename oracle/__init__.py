"""CPU oracle for the range-separated (RS) canonical/Tucker potential path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything here: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It is a plain, slow FP64
implementation written from the paper (Benner, Khoromskaia, Khoromskij,
"Range-separated tensor format for numerical modeling of many-particle
interaction potentials"), following the paper's notation and order of
steps.  It shares no code with the HIP library.

Modules
  quadrature  sinc quadrature of the Laplace-Gauss transform, range split (sec. 2.2-2.3)
  grid        the cell-centred n x n x n grid on [-b, b]^3 (sec. 2.2)
  canonical   direct and canonical potential sums, short-range CCT windows (sec. 3.2-3.3)
  rhosvd      side matrices, weighted Gram, RHOSVD basis, core, Tucker (sec. 3.2, Appendix)
  rs          the RS-Tucker assembly (Definition RS-Tucker_format)
  pointeval   point evaluation, interaction energy and forces (sec. 4.2-4.3)
  pairwise    O(N^2) pairwise energies and forces (eq EnergyLatSum)
  gradient    finite-difference gradient of the RS tensor on the grid (sec. 4.3, eq Gradients_Tens)
  dot         scalar product of two RS tensors on one grid (sec. 3.4)
  als         ALS refinement of the RHOSVD bases and core (Appendix, steps (III)-(V))
  rbf         RS form of the RBF interpolation matrix and its matrix-vector product (sec. 4.1)

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against a closed form, an identity, an invariant, brute force, or a value the
paper prints, except where its docstring says "parity unpinned".
"""

"""FP64 CPU oracle for the subspace pencil (H, S) and its lowest eigenvalue E.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library: the only common
input is the seeded generator in ``tnqe_synth``.

Plain, slow NumPy/SciPy in float64, written from the paper (arXiv 2404.10223):

* ``gates``    two-site FSWAP / Givens gates (App. A3, eq. fswap and the d=4
               composites built from d=2 gates);
* ``givens``   QR-type decomposition of an orbital rotation into nearest-
               neighbour Givens rotations (Sec. II.B, eq. givens_decomp);
* ``fock``     brute-force Fock space (eq. ham_def, eq. fci), sector FCI and
               the determinant form of an orbital rotation (Thouless);
* ``mps``      canonical form, two-site gate + SVD truncation (App. A1 eq.
               svd_longform, App. A3), overlap transfer sweep;
* ``mpo``      matrix-product operator of the Hamiltonian and the block-sparse
               left-environment sweep (Sec. II.A, App. A1);
* ``gep``      generalized eigenproblem with S thresholding: projection and
               inversion (Sec. V "Regulating the subspace condition number",
               App. A2) and the eigenvalue condition number kappa_1;
* ``subspace`` the whole pencil for M MPS in rotated orbital bases
               (eq. tnqe, eq. GEE, eq. mat_els).

Parity pins: every function is checked in ``tests/test_oracle_*.py`` against a
closed form, brute force, an invariant or a value printed in the paper.  The
one quantity without a pin is the absolute accuracy of the truncated H and S
against the untruncated values at N = 24 (no FCI is possible there): parity
unpinned for that comparison; the oracle-vs-GPU comparison and the
determinant (Slater-Condon) pins of the MPO still hold at that size.
"""

"""CPU oracle for implicit imaginary-time evolution of matrix product states.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package; only the test suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library (no kernels, headers,
helpers or table generators); the two meet only in the seeded inputs of the
``workload`` module.

Everything is plain FP64 numpy, written so that a reader can check it against
"Fast Tensor Network Imaginary Time Evolution by Implicit Stepping on
Logarithmic Grids" (Zima, Stoudenmire, White, Parcollet, Kaye) by eye:

* ``oracle.ed``   -- full state-vector level: Hamiltonians built from Kronecker
  products, exact evolution through the spectral decomposition (Method, Eq. 1),
  the implicit trapezoid / backward-Euler full-vector step (Method, Eq. 4),
  logarithmic and panel grids (Method), the local trapezoid error E(mu) and the
  explicit steppers used as negative controls (Appendix A).
* ``oracle.mpo``  -- MPO builders for the Heisenberg chain and the star-geometry
  Anderson impurity model (Appendix B: MPOs generated exactly, compressed to
  machine precision) and their contraction to dense matrices.
* ``oracle.mps``  -- the dense-tensor MPS algorithm: the two-site DMRG-style
  linear solve of (I + h (H - s)) x = b with b projected into x's basis, GMRES
  local solves, SVD truncation by discarded weight, normalisation and energy
  shift after every step (Method; Appendices B and D).
* ``oracle.sampling`` -- product-basis sampling of a right-orthonormal MPS by
  conditional probabilities (the METTS collapse, Appendix D).
* ``oracle.dmrg`` -- two-site DMRG ground-state sweeps on the same blocks and
  split, the local problem diagonalised exactly (the ground state that seeds
  the METTS chains and gives the zero-temperature double occupancy,
  Appendix D).
* ``oracle.apply`` -- the right-hand side as an MPS (Appendix B): the
  density-matrix MPO-MPS product and the trapezoid step that starts from it.
* ``oracle.gauss`` -- the spectral variant (Method): Gauss-Legendre
  collocation on a panel, densely and as one augmented MPS linear system
  (an extra node site) solved by the same two-site sweep.
* ``oracle.metts`` -- one-site expectation values and METTS chains
  (evolution, measurement, collapse; Appendix D), with their exact dense
  counterparts used to pin them.

Parity status of every function is stated in its module header; the pins live
in ``tests/test_oracle_*.py``.
"""

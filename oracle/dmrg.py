"""Two-site DMRG ground-state sweeps of the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper computes the ground state of its impurity model with DMRG: the
METTS chains start from product states sampled from it and the zero
temperature double occupancy is measured in it (Appendix D).  The variant
here is the plain two-site one on the same blocks, environments and SVD split
as the implicit step of ``oracle.mps``:

  * psi is right-orthonormal with the centre on site 1 (as after a step);
  * right environments of <psi|H|psi>;
  * left-to-right half sweep over the blocks (j, j+1): theta is the lowest
    eigenvector of the two-site effective Hamiltonian, formed here as a
    dense matrix (the effective Hamiltonian applied to every unit vector)
    and diagonalised with ``numpy.linalg.eigh``; SVD split A_j = U,
    A_(j+1) = S V^T; left environment updated;
  * right-to-left half sweep, mirrored (A_j = U S, A_(j+1) = V^T);
  * the energy is the eigenvalue of the last block, whose eigenvector is
    normalised, so it equals <psi|H|psi> of the new state before truncation.

Readings where the paper is silent: the local eigensolver (exact here,
Lanczos on the GPU path); one sweep = one left-to-right plus one
right-to-left half sweep, as for the step; truncation as in ``oracle.mps``.

Pins (``tests/test_oracle_dmrg.py``): with complete bases the sweeps reach
the exact-diagonalisation ground state of ``oracle.ed``; the XX chain reaches
its closed-form ground energy; the dense effective Hamiltonian is symmetric
and reproduces <psi|H|psi>; the energy never rises from one half sweep to
the next at full bond dimension.
"""
from __future__ import annotations

import numpy as np

from . import mps as om


def heff_dense(Lenv, W1, W2, Renv):
    """The two-site effective Hamiltonian as an n x n matrix, column k the
    product with unit vector k (theta flattened in [a, s1, s2, c] order)."""
    Dl, d1, d2, Dr = Lenv.shape[2], W1.shape[3], W2.shape[3], Renv.shape[2]
    n = Dl * d1 * d2 * Dr
    M = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = om.heff_apply(Lenv, W1, W2, Renv, e.reshape(Dl, d1, d2, Dr)).reshape(-1)
    return M


def lowest_eigvec(M):
    """Lowest eigenpair of the symmetric matrix M (its symmetric part)."""
    lam, V = np.linalg.eigh(0.5 * (M + M.T))
    return float(lam[0]), V[:, 0]


def _boundaries():
    one = np.ones((1, 1, 1))
    return one, one.copy()


def dmrg_sweeps(psi, W, nsweeps: int, chi_max: int, cutoff: float = 0.0, tie_rel: float = 1e-10):
    """nsweeps two-site sweeps from psi (right-orthonormal, centre on site 1).
    Returns the new MPS (centre on site 1), the energy after each half sweep
    and the largest discarded weight."""
    L = len(psi)
    A = [a.copy() for a in psi]
    Lb, Rb = _boundaries()
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = Lb
    Renv[L] = Rb
    for b in range(L - 1, 1, -1):
        Renv[b] = om.env_right_h(Renv[b + 1], A[b], W[b], A[b])
    energies = []
    max_disc = 0.0

    def block(i, direction):
        nonlocal max_disc
        theta = om.two_site(A[i], A[i + 1])
        M = heff_dense(Lenv[i], W[i], W[i + 1], Renv[i + 2])
        E, v = lowest_eigvec(M)
        A1, A2, info = om.split_two_site(v.reshape(theta.shape), direction, cutoff, chi_max, tie_rel)
        A[i], A[i + 1] = A1, A2
        max_disc = max(max_disc, info["disc"])
        return E

    E = None
    for _ in range(nsweeps):
        for i in range(L - 1):
            E = block(i, "lr")
            if i + 2 < L:
                Lenv[i + 1] = om.env_left_h(Lenv[i], A[i], W[i], A[i])
        energies.append(E)
        for i in range(L - 2, -1, -1):
            E = block(i, "rl")
            if i > 0:
                Renv[i + 1] = om.env_right_h(Renv[i + 2], A[i + 1], W[i + 1], A[i + 1])
        energies.append(E)
    return A, energies, max_disc

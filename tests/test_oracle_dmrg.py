"""Pins of the oracle's two-site DMRG ground-state sweeps (``oracle.dmrg``)."""
import numpy as np
import pytest

from oracle import dmrg, ed, mpo, mps
from workload import rng_for, random_spinors


def _neel(L):
    return [np.array([1.0, 0.0]) if i % 2 == 0 else np.array([0.0, 1.0]) for i in range(L)]


@pytest.mark.parametrize("L", [2, 6, 8])
def test_dmrg_reaches_ed_ground_state(L):
    # complete bond dimension 2^(L/2): the sweeps are exact up to the
    # eigensolver, and the Heisenberg ground state (unique, S = 0 for even L)
    # is reached from the Neel state within two sweeps
    chi = 2 ** (L // 2)
    psi = mps.product_state(_neel(L), chi, pad_full=True)
    W = mpo.heisenberg_mpo(L)
    A, energies, disc = dmrg.dmrg_sweeps(psi, W, nsweeps=2, chi_max=chi)
    e0, _ = ed.ground_state(ed.heisenberg_dense(L))
    assert abs(energies[-1] - e0) < 1e-10 * abs(e0)
    # the returned state is normalised and its energy is the reported one
    assert abs(mps.overlap(A, A) - 1.0) < 1e-12
    assert abs(mps.expectation(A, W) - energies[-1]) < 1e-10 * abs(e0)
    assert disc < 1e-20


def test_dmrg_xx_chain_closed_form():
    # XX chain (Jz = 0): free fermions, ground energy in closed form
    L = 10
    psi = mps.product_state(_neel(L), 32, pad_full=True)
    W = mpo.heisenberg_mpo(L, J=1.0, Jz=0.0)
    _, energies, _ = dmrg.dmrg_sweeps(psi, W, nsweeps=2, chi_max=32)
    e0 = ed.xx_chain_e0(L)
    assert abs(energies[-1] - e0) < 1e-10 * abs(e0)


def test_heff_dense_symmetric_and_expectation():
    # at the first block of a normalised right-orthonormal state the dense
    # effective Hamiltonian is symmetric and theta^T M theta = <psi|H|psi>
    L = 6
    rng = rng_for(71)
    psi = mps.product_state(random_spinors(rng, L, 2), 8, pad_full=True)
    W = mpo.heisenberg_mpo(L, J=1.0, Jz=0.7)
    R = [None] * (L + 1)
    R[L] = np.ones((1, 1, 1))
    for b in range(L - 1, 1, -1):
        R[b] = mps.env_right_h(R[b + 1], psi[b], W[b], psi[b])
    M = dmrg.heff_dense(np.ones((1, 1, 1)), W[0], W[1], R[2])
    assert np.abs(M - M.T).max() < 1e-13 * np.abs(M).max()
    th = mps.two_site(psi[0], psi[1]).reshape(-1)
    assert abs(th @ M @ th - mps.expectation(psi, W)) < 1e-12


def test_dmrg_energy_monotone_at_full_bond():
    # each block minimises the energy over a space that contains the current
    # state: without truncation the energy cannot rise between half sweeps
    L = 8
    rng = rng_for(72)
    psi = mps.product_state(random_spinors(rng, L, 2), 16, pad_full=True)
    W = mpo.heisenberg_mpo(L, J=1.0, Jz=0.5)
    e_start = mps.expectation(psi, W)
    _, energies, _ = dmrg.dmrg_sweeps(psi, W, nsweeps=2, chi_max=16)
    seq = [e_start] + energies
    assert all(b <= a + 1e-12 for a, b in zip(seq, seq[1:]))


def test_dmrg_truncated_bond_stays_variational():
    # with chi below the complete dimension the energy is an upper bound of
    # the exact ground energy and close to it for a gapped-enough chain
    L = 10
    psi = mps.product_state(_neel(L), 8, pad_full=True)
    W = mpo.heisenberg_mpo(L)
    A, energies, disc = dmrg.dmrg_sweeps(psi, W, nsweeps=3, chi_max=8)
    e0, _ = ed.ground_state(ed.heisenberg_dense(L))
    assert energies[-1] >= e0 - 1e-10
    assert energies[-1] - e0 < 1e-3 * abs(e0)
    assert max(a.shape[2] for a in A) <= 8

"""Pins of the oracle's MPO builders: contracted to dense matrices they must
equal the Kronecker-product Hamiltonians built from the definitions."""
import numpy as np
import pytest

from oracle import ed, mpo


@pytest.mark.parametrize("L", [2, 3, 4, 7, 8])
@pytest.mark.parametrize("Jz", [1.0, 0.0, 0.45])
def test_heisenberg_mpo_is_the_hamiltonian(L, Jz):
    H = ed.heisenberg_dense(L, J=1.3, Jz=Jz)
    Hm = mpo.mpo_to_dense(mpo.heisenberg_mpo(L, J=1.3, Jz=Jz))
    assert np.abs(H - Hm).max() < 1e-13


def test_heisenberg_mpo_shapes():
    W = mpo.heisenberg_mpo(6)
    assert mpo.mpo_bond_dims(W) == [1, 5, 5, 5, 5, 5, 1]
    assert all(w.shape[2:] == (2, 2) for w in W)


@pytest.mark.parametrize("nb", [1, 2, 3, 4])
def test_aim_mpo_is_the_hamiltonian(nb):
    rng = np.random.default_rng(10 + nb)
    eb = np.sort(rng.uniform(-1, 1, nb))
    V = rng.uniform(0.05, 0.6, nb)
    U = 2.5
    Hk = ed.aim_dense(U, -U / 2 + 0.1, eb, V)
    Hm = mpo.mpo_to_dense(mpo.aim_mpo(U, -U / 2 + 0.1, eb, V))
    p = ed.aim_basis_permutation(nb + 1)
    assert np.abs(Hk[np.ix_(p, p)] - Hm).max() < 1e-13


def test_aim_mpo_shapes():
    W = mpo.aim_mpo(4.0, -2.0, np.linspace(-1, 1, 5), np.full(5, 0.1))
    assert mpo.mpo_bond_dims(W) == [1, 6, 6, 6, 6, 6, 1]

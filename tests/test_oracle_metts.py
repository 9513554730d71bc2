"""Pins of the METTS oracle (``oracle.metts``): one-site expectation values
against dense vectors, the stationarity and unbiasedness identities of METTS
with exact evolution, the statistics of a seeded chain against the thermal
average, and the MPS chain against the dense chain with the same steps."""
import numpy as np
import pytest

from oracle import ed, metts, mpo, mps
from workload import rng_for, aim_bath

ND = np.diag([0.0, 0.0, 0.0, 1.0])     # n_up n_dn in the per-site basis |0>, |up>, |dn>, |up dn>


def _aim(nb, U=4.0, gamma=0.3):
    eb, V = aim_bath(nb, gamma)
    perm = ed.aim_basis_permutation(nb + 1)
    H = ed.aim_dense(U, -U / 2, eb, V)[np.ix_(perm, perm)]
    return H, mpo.aim_mpo(U, -U / 2, eb, V)


@pytest.mark.parametrize("site", [0, 2, 4])
def test_site_expectation_equals_dense(site):
    rng = np.random.default_rng(40 + site)
    dims = [1, 3, 5, 4, 2, 1]
    A = [rng.standard_normal((dims[i], 4, dims[i + 1])) for i in range(5)]
    op = rng.standard_normal((4, 4))
    v = mps.to_vector(A)
    O = np.kron(np.kron(np.eye(4 ** site), op), np.eye(4 ** (4 - site)))
    assert abs(metts.site_expectation(A, site, op) - v @ O @ v / (v @ v)) < 1e-13


@pytest.mark.parametrize("beta", [0.5, 3.0, 20.0])
def test_metts_stationary_and_unbiased_with_exact_evolution(beta):
    # p(i) ~ <i|exp(-beta H)|i> is stationary under T[i, j] = |<j|psi_i>|^2,
    # and sum_i p(i) <psi_i|O|psi_i> = Tr(exp(-beta H) O) / Z exactly
    H, _ = _aim(1)
    O = np.kron(ND, np.eye(4))
    ev, vec = np.linalg.eigh(H)
    w = np.exp(-beta * (ev - ev[0]))
    p = np.einsum("ik,k->i", vec * vec, w)
    p /= p.sum()
    T = metts.metts_transition(H, beta)
    assert np.abs(T.sum(axis=1) - 1).max() < 1e-13
    assert np.abs(p @ T - p).max() < 1e-13
    est = sum(p[i] * (lambda v: v @ O @ v)(metts.exact_metts(H, beta, i)) for i in range(H.shape[0]))
    assert abs(est - metts.thermal_average(H, O, beta)) < 1e-13
    # a plain average over product states (no METTS weights) is biased here
    flat = np.mean([(lambda v: v @ O @ v)(metts.exact_metts(H, beta, i)) for i in range(H.shape[0])])
    assert abs(flat - metts.thermal_average(H, O, beta)) > 1e-4


def test_seeded_dense_chain_reproduces_the_thermal_average():
    H, _ = _aim(1)
    O = np.kron(ND, np.eye(4))
    beta = 4.0
    n = 4000
    u = rng_for(41).random((n, 2))
    _, _, obs = metts.dense_chain(H, O, [1, 2], 2, 4, lambda i: metts.exact_metts(H, beta, i), u)
    # batch means for the autocorrelated chain
    b = obs[: (n // 50) * 50].reshape(50, -1).mean(axis=1)
    se = b.std(ddof=1) / np.sqrt(len(b))
    # the collapse in the computational basis keeps particle number and S^z:
    # the chain samples the canonical ensemble of its start state's sector
    sec = metts.sector([1, 2], 2, 4, [[0, 1, 1, 2], [0, 1, -1, 0]])
    assert abs(obs.mean() - metts.thermal_average(H, O, beta, sec)) < 4 * se + 1e-12
    assert abs(obs.mean() - metts.thermal_average(H, O, beta)) > 10 * se


def test_mps_chain_equals_dense_trapezoid_chain():
    # complete bonds (cutoff 0 keeps every singular value) and converged
    # local solves: every MPS step is the full-vector trapezoid step
    nb = 2
    H, W = _aim(nb, gamma=3.0)
    L = nb + 1
    O = np.kron(ND, np.eye(4 ** nb))
    beta, tau0, ratio = 4.0, 0.01, 1.5
    u = rng_for(42).random((6, L))
    opts = mps.StepOptions(scheme="trap", shift_mode="track", chi_max=16, cutoff=0.0, krylov_dim=10,
                           max_cycles=200, tol_loc=1e-13)
    cfg, en, ob = metts.mps_chain(W, [1, 2, 0], 4, beta, tau0, ratio, opts, 0, ND, u)
    dcfg, den, dob = metts.dense_chain(H, O, [1, 2, 0], L, 4, metts.trapezoid_metts(H, tau0, beta, ratio), u)
    assert (cfg == dcfg).all()
    assert np.abs(en - den).max() < 1e-10 * np.abs(den).max()
    assert np.abs(ob - dob).max() < 1e-10
    assert len({tuple(c) for c in cfg}) > 1

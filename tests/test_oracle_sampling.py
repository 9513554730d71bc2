"""Pins of the oracle's product-basis sampling (``oracle.sampling``)."""
import numpy as np

from oracle import dmrg, ed, mpo, mps, sampling
from workload import rng_for


def _ground_state(L, chi):
    neel = [np.array([1.0, 0.0]) if i % 2 == 0 else np.array([0.0, 1.0]) for i in range(L)]
    A, _, _ = dmrg.dmrg_sweeps(mps.product_state(neel, chi, pad_full=True), mpo.heisenberg_mpo(L, 1.0, 0.5), 2, chi)
    return A


def _amplitude(A, cfg):
    v = np.ones(1)
    for a, s in zip(A, cfg):
        v = v @ a[:, s, :]
    return float(v[0])


def test_probabilities_are_squared_amplitudes():
    L = 6
    A = _ground_state(L, 8)
    u = rng_for(75).random((L, 200))
    cfg, probs = sampling.sample(A, u)
    nrm2 = mps.overlap(A, A)
    for c, p in zip(cfg, probs):
        assert abs(p - _amplitude(A, c) ** 2 / nrm2) < 1e-12


def test_basis_product_state_is_returned():
    L = 7
    bits = [0, 1, 1, 0, 1, 0, 0]
    spin = [np.eye(2)[b] for b in bits]
    A = mps.product_state(spin, 8, pad_full=True)
    cfg, probs = sampling.sample(A, rng_for(76).random((L, 5)))
    assert (cfg == np.array(bits)).all() and np.allclose(probs, 1.0)


def test_frequencies_follow_born_rule():
    L = 4
    A = _ground_state(L, 4)
    S = 20000
    cfg, _ = sampling.sample(A, rng_for(77).random((L, S)))
    v = ed.ground_state(ed.heisenberg_dense(L, 1.0, 0.5))[1]
    p = v * v / (v @ v)
    idx = (cfg * (2 ** np.arange(L - 1, -1, -1))).sum(axis=1)
    freq = np.bincount(idx, minlength=2 ** L) / S
    sigma = np.sqrt(p * (1 - p) / S) + 1e-12
    assert np.all(np.abs(freq - p) <= 5 * sigma)

"""GPU parity of product-basis sampling (``ite_mps_sample``) against the
oracle (``oracle.sampling``) through the C ABI: with the same uniforms the
sampled configurations are identical, integer for integer (the decisions are
FP64 comparisons on both sides; a uniform within rounding of a cumulative
probability is the only way they could differ).
"""
import numpy as np
import pytest

import paper_2606_02930_amd as ite
from paper_2606_02930_amd import hamiltonians
from oracle import sampling as osmp
from workload import rng_for, aim_bath, random_spinors
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = require_gpu()
    c = ite.ite_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    ite.ite_ctx_destroy(c)


def _ground_state_samples(ctx, L, d, W, spinors, chi, S, seed):
    psi = ite.ite_mps_create(ctx, spinors, chi, pad_full=True)
    H = ite.ite_mpo_load(ctx, W)
    try:
        ite.ite_dmrg_sweeps(ctx, psi, H, 2, chi, krylov_dim=16, max_cycles=4, tol=1e-12)
        A = ite.ite_mps_export(ctx, psi, [d] * L)
        u = rng_for(seed).random((L, S))
        cfg = ite.ite_mps_sample(ctx, psi, u)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(H)
    return A, u, cfg


def test_heisenberg_ground_state_samples_match_oracle(ctx):
    L = 12
    A, u, cfg = _ground_state_samples(ctx, L, 2, hamiltonians.heisenberg(L, 1.0, 0.5),
                                      random_spinors(rng_for(78), L, 2), 16, 1000, 79)
    o_cfg, _ = osmp.sample(A, u)
    assert cfg.shape == (1000, L)
    assert (cfg == o_cfg).all()
    # S^z = 0 sector dominates the ground state of an even chain
    assert abs((2 * cfg - 1).sum(axis=1).mean()) < 0.5


def test_anderson_ground_state_samples_match_oracle(ctx):
    nb = 3
    eb, V = aim_bath(nb, gamma=0.3)
    L = nb + 1
    A, u, cfg = _ground_state_samples(ctx, L, 4, hamiltonians.anderson_star(4.0, -2.0, eb, V),
                                      random_spinors(rng_for(80), L, 4), 16, 500, 81)
    o_cfg, _ = osmp.sample(A, u)
    assert (cfg == o_cfg).all()


def test_basis_state_and_errors(ctx):
    bits = [1, 0, 0, 1, 1]
    psi = ite.ite_mps_create(ctx, [np.eye(2)[b] for b in bits], 4, pad_full=True)
    try:
        cfg = ite.ite_mps_sample(ctx, psi, rng_for(82).random((5, 64)))
        assert (cfg == np.array(bits)).all()
        bad = np.full((5, 3), 0.5)
        bad[2, 1] = 1.0
        with pytest.raises(ite.IteError) as e:
            ite.ite_mps_sample(ctx, psi, bad)
        assert e.value.code == ite.ITE_EINVAL
        # uniforms of the wrong orientation: L (rows) differs from the state's
        with pytest.raises(ite.IteError) as e:
            ite.ite_mps_sample(ctx, psi, rng_for(82).random((64, 5)))
        assert e.value.code == ite.ITE_EINVAL
        assert "length" in ite.ite_last_error(ctx)
    finally:
        ite.ite_mps_destroy(psi)
    # a zero state has no distribution to sample
    zero = ite.ite_mps_load(ctx, [np.zeros((1, 2, 1))] * 4, 4)
    try:
        with pytest.raises(ite.IteError) as e:
            ite.ite_mps_sample(ctx, zero, rng_for(83).random((4, 8)))
        assert e.value.code == ite.ITE_ENONFINITE
    finally:
        ite.ite_mps_destroy(zero)

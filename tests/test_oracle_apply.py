"""Pins of the density-matrix MPO-MPS product and the trapezoid step with the
right-hand side formed as an MPS (``oracle/apply.py``): the operator of the
right-hand side against its dense form, the untruncated product against the
dense product, the first truncation against the singular values of the dense
result at that bond (Eckart-Young), orthonormality, and the step at complete
bonds against the full-vector trapezoid step."""
import numpy as np
import pytest

from oracle import apply as oapply, ed, mpo, mps
from workload import random_spinors, rng_for


def _random_mps(rng, dims, d):
    return [rng.standard_normal((dims[i], d, dims[i + 1])) for i in range(len(dims) - 1)]


def test_rhs_mpo_is_its_operator():
    L, h, s = 5, 0.37, -1.2
    W = mpo.heisenberg_mpo(L, Jz=0.8)
    H = ed.heisenberg_dense(L, Jz=0.8)
    n = H.shape[0]
    O = oapply.rhs_mpo(W, h, s)
    assert np.abs(mpo.mpo_to_dense(O) - ((1 + h * s) * np.eye(n) - h * H)).max() < 1e-13


@pytest.mark.parametrize("L,dims", [(5, [1, 2, 4, 3, 2, 1]), (6, [1, 2, 4, 8, 4, 2, 1])])
def test_untruncated_product_is_exact(L, dims):
    rng = np.random.default_rng(30 + L)
    psi = _random_mps(rng, dims, 2)
    W = mpo.heisenberg_mpo(L, Jz=0.6)
    want = mpo.mpo_to_dense(W) @ mps.to_vector(psi)
    b, info = oapply.density_matrix_apply(W, psi, 1 << 10, 0.0, 0.0)
    assert np.abs(mps.to_vector(b) - want).max() < 1e-12 * np.abs(want).max()
    for a in b[1:]:
        assert mps.right_orthonormality_error(a) < 1e-12
    assert info["disc"] < 1e-14     # rounding-level eigenvalues beyond the rank
    # no bond above the rank it can have
    assert all(x <= y for x, y in zip(mps.bond_dims(b), mps.full_dims(L, 2, 1 << 10)))


def test_first_truncation_is_the_optimal_one():
    # the first eigen-decomposition (last site) sees the exact reduced density
    # matrix: keeping k vectors keeps the k largest squared singular values of
    # phi across that bond, and the discarded fraction is theirs
    L = 6
    rng = np.random.default_rng(44)
    psi = _random_mps(rng, [1, 2, 4, 8, 4, 2, 1], 2)
    W = mpo.heisenberg_mpo(L)
    phi = mpo.mpo_to_dense(W) @ mps.to_vector(psi)
    sv = np.linalg.svd(phi.reshape(2 ** (L - 1), 2), compute_uv=False)
    b, info = oapply.density_matrix_apply(W, psi, 1, 0.0, 0.0)
    assert info["k"][0] == 1
    # the reduced density matrix's eigenvalues are phi's squared singular
    # values across the last bond
    assert np.abs(info["lam"][0] - sv ** 2).max() < 1e-12 * sv[0] ** 2
    want = sv[1] ** 2 / np.sum(sv ** 2)
    assert info["disc"] >= want * (1 - 1e-10)
    # chi 2 at the last bond keeps both: nothing is discarded there
    b2, info2 = oapply.density_matrix_apply(W, psi, 2, 0.0, 0.0)
    assert info2["k"][0] == 2
    # the product with chi = 1 is the best product-state-like cut at the last
    # bond: its overlap with phi is at most the largest singular value
    v = mps.to_vector(b)
    assert abs(v @ phi) / np.linalg.norm(v) <= sv[0] * (1 + 1e-12)


@pytest.mark.parametrize("shift_mode", ["fixed", "track"])
def test_step_at_complete_bonds_equals_full_vector_trapezoid(shift_mode):
    L, chi = 8, 16
    W = mpo.heisenberg_mpo(L)
    H = ed.heisenberg_dense(L)
    e0 = ed.ground_state(H)[0]
    sp = random_spinors(rng_for(0, 21), L, 2)
    psi = mps.product_state(sp, chi, pad_full=True)
    opts = mps.StepOptions(scheme="trap", shift_mode=shift_mode, shift=e0, chi_max=chi, cutoff=0.0, krylov_dim=10,
                           max_cycles=400, tol_loc=1e-13)
    grid = ed.loggrid(0.01, 5.0, 1.6)
    out, reps = oapply.evolve_grid_mps_rhs(psi, W, grid, opts)
    states, en, norms, _ = ed.evolve_dense(H, mps.to_vector(psi), grid, "trap", shift_mode, e0)
    # the product diagonalises reduced density matrices (squared Schmidt
    # values), so Schmidt values below about sqrt(eps) of the largest are
    # only resolved to rounding: agreement to 1e-9 rather than 1e-10
    for r, e in zip(reps, en[1:]):
        assert abs(r.energy - e) <= 1e-9 * max(1.0, abs(e))   # the energy passes near zero on the way
        assert r.extra["rhs_disc"] < 1e-14   # rounding-level eigenvalues only
    v = mps.to_vector(out)
    assert 1 - abs(v @ states[-1]) < 1e-10
    for a in out[1:]:
        assert mps.right_orthonormality_error(a) < 1e-12

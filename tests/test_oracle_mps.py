"""Pins of the oracle's dense-tensor MPS algorithm (``oracle.mps``)."""
import math

import numpy as np
import pytest

from oracle import ed, mpo, mps
from workload import rng_for, random_spinors


def _random_mps(rng, dims, d):
    return [rng.standard_normal((dims[i], d, dims[i + 1])) for i in range(len(dims) - 1)]


def _left_block(A):
    """Dense matrix P_left[(s_1..s_j), a] of the left part of an MPS."""
    v = A[0].reshape(A[0].shape[1], A[0].shape[2])
    for a in A[1:]:
        v = np.tensordot(v, a, axes=([1], [0])).reshape(-1, a.shape[2])
    return v


def _right_block(A):
    """Dense matrix P_right[c, (s_j..s_L)] of the right part of an MPS."""
    v = A[-1].reshape(A[-1].shape[0], A[-1].shape[1])
    for a in reversed(A[:-1]):
        v = np.tensordot(a, v, axes=([2], [0])).reshape(a.shape[0], -1)
    return v


def _projector(A, i):
    """P with P theta = full vector of A_1..A_(i-1) theta A_(i+2)..A_L."""
    d1, d2 = A[i].shape[1], A[i + 1].shape[1]
    Pl = _left_block(A[:i]) if i > 0 else np.ones((1, 1))
    Pr = _right_block(A[i + 2:]) if i + 2 < len(A) else np.ones((1, 1))
    return np.kron(np.kron(Pl, np.eye(d1 * d2)), Pr.T)


def _envs(X, Y, W, i):
    Lh = np.ones((1, 1, 1))
    Lo = np.ones((1, 1))
    for j in range(i):
        Lh = mps.env_left_h(Lh, X[j], W[j], Y[j])
        Lo = mps.env_left_o(Lo, X[j], Y[j])
    Rh = np.ones((1, 1, 1))
    Ro = np.ones((1, 1))
    for j in range(len(X) - 1, i + 1, -1):
        Rh = mps.env_right_h(Rh, X[j], W[j], Y[j])
        Ro = mps.env_right_o(Ro, X[j], Y[j])
    return Lh, Lo, Rh, Ro


# --- states and environments -------------------------------------------------

def test_padded_product_state_is_the_product_state():
    sp = random_spinors(rng_for(0), 8, 2)
    plain = mps.product_state(sp)
    padded = mps.product_state(sp, chi_max=16, pad_full=True)
    assert mps.bond_dims(padded) == [1, 2, 4, 8, 16, 8, 4, 2, 1]
    v = mps.to_vector(plain)
    assert np.abs(mps.to_vector(padded) - v).max() < 1e-15
    # brute force: the product state is the Kronecker product of the spinors
    kron = np.ones(1)
    for s in sp:
        kron = np.kron(kron, s)
    assert np.abs(v - kron).max() < 1e-15
    assert max(mps.right_orthonormality_error(a) for a in padded) < 1e-14


def test_expectation_matches_dense():
    rng = np.random.default_rng(20)
    A = _random_mps(rng, [1, 2, 4, 3, 2, 1], 2)
    W = mpo.heisenberg_mpo(5, Jz=0.7)
    H = ed.heisenberg_dense(5, Jz=0.7)
    v = mps.to_vector(A)
    assert abs(mps.expectation(A, W) - v @ H @ v / (v @ v)) < 1e-12
    B = _random_mps(rng, [1, 2, 3, 3, 2, 1], 2)
    assert abs(mps.overlap(A, B) - v @ mps.to_vector(B)) < 1e-12


@pytest.mark.parametrize("i", [0, 1, 2, 3])
def test_heff_is_projected_hamiltonian(i):
    # H_eff = P_x^T H P_y for bra x and ket y that differ (mixed environments).
    rng = np.random.default_rng(30 + i)
    L = 5
    X = _random_mps(rng, [1, 2, 3, 4, 2, 1], 2)
    Y = _random_mps(rng, [1, 2, 2, 3, 2, 1], 2)
    W = mpo.heisenberg_mpo(L, Jz=0.6)
    H = ed.heisenberg_dense(L, Jz=0.6)
    Lh, Lo, Rh, Ro = _envs(X, Y, W, i)
    theta = rng.standard_normal((Y[i].shape[0], 2, 2, Y[i + 1].shape[2]))
    Px, Py = _projector(X, i), _projector(Y, i)
    got = mps.heff_apply(Lh, W[i], W[i + 1], Rh, theta)
    want = (Px.T @ H @ Py @ theta.reshape(-1)).reshape(got.shape)
    assert np.abs(got - want).max() < 1e-12
    got_o = mps.overlap_project(Lo, Ro, theta)
    want_o = (Px.T @ Py @ theta.reshape(-1)).reshape(got_o.shape)
    assert np.abs(got_o - want_o).max() < 1e-12


def test_heff_fermionic_is_projected_hamiltonian():
    rng = np.random.default_rng(40)
    eb, V = np.array([-0.6, 0.1, 0.5]), np.array([0.3, 0.2, 0.4])
    W = mpo.aim_mpo(3.0, -1.5, eb, V)
    p = ed.aim_basis_permutation(4)
    Hk = ed.aim_dense(3.0, -1.5, eb, V)
    H = Hk[np.ix_(p, p)]
    X = _random_mps(rng, [1, 3, 5, 2, 1], 4)
    Lh, Lo, Rh, Ro = _envs(X, X, W, 1)
    theta = rng.standard_normal((3, 4, 4, 2))
    P = _projector(X, 1)
    got = mps.heff_apply(Lh, W[1], W[2], Rh, theta)
    assert np.abs(got.reshape(-1) - P.T @ H @ P @ theta.reshape(-1)).max() < 1e-12


# --- GMRES ------------------------------------------------------------------

def test_gmres_is_the_krylov_minimiser():
    rng = np.random.default_rng(50)
    n, m = 40, 7
    M = rng.standard_normal((n, n))
    A = np.eye(n) + 0.2 * (M + M.T)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    x, info = mps.gmres(lambda v: A @ v, b, x0, m, 1, 0.0)
    assert info["matvecs"] == m + 1
    # brute force: minimise ||b - A(x0 + K c)|| over the power basis of K_m(A, r0)
    r0 = b - A @ x0
    K = np.empty((n, m))
    v = r0.copy()
    for j in range(m):
        K[:, j] = v
        v = A @ v
    c = np.linalg.lstsq(A @ K, r0, rcond=None)[0]
    xb = x0 + K @ c
    assert np.abs(x - xb).max() < 1e-8 * np.abs(xb).max()
    assert abs(info["res_rel"] - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-10


def test_gmres_full_space_is_the_solve_and_restarts_converge():
    rng = np.random.default_rng(51)
    n = 12
    M = rng.standard_normal((n, n))
    A = np.eye(n) * 3 + M @ M.T * 0.1
    b = rng.standard_normal(n)
    x, info = mps.gmres(lambda v: A @ v, b, np.zeros(n), 20, 1, 0.0)
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-11
    assert info["matvecs"] <= n + 1
    x, info = mps.gmres(lambda v: A @ v, b, np.zeros(n), 3, 200, 1e-13)
    assert np.linalg.norm(A @ x - b) <= 2e-13 * np.linalg.norm(b)
    assert info["cycles"] > 1


# --- truncation --------------------------------------------------------------

def test_truncation_rank_rules():
    s = np.array([1.0, 0.5, 1e-3, 1e-6, 0.0])
    tot = np.sum(s ** 2)
    # discarded weight of keeping k: sum_{i>=k} s_i^2 / total
    assert mps.truncation_rank(s, 1e-10, 10, 0.0) == 3       # drops 1e-12 / 1.25
    assert mps.truncation_rank(s, 1e-5, 10, 0.0) == 2        # drops (1e-6 + 1e-12) / 1.25
    assert (1e-6 + 1e-12) / tot <= 1e-5 < (0.25 + 1e-6) / tot
    assert mps.truncation_rank(s, 0.0, 10, 0.0) == 5         # keeps zeros
    assert mps.truncation_rank(s, 0.0, 3, 0.0) == 3          # chi cap
    assert mps.truncation_rank(s, 0.9, 10, 0.0) == 1         # never below 1
    # the cut is inclusive and uses the full cutoff: discarded 1e-4 / 1.0001
    two = np.array([1.0, 0.01])
    assert mps.truncation_rank(two, 1.5e-4, 10, 0.0) == 1
    assert mps.truncation_rank(two, 0.9e-4, 10, 0.0) == 2
    assert mps.truncation_rank(two, 1e-4 / 1.0001, 10, 0.0) == 1
    # a cut inside a degenerate multiplet moves below it
    t = np.array([1.0, 0.6, 0.6, 0.6, 0.1])
    assert mps.truncation_rank(t, 0.0, 3, 1e-13) == 1
    assert mps.truncation_rank(t, 0.0, 4, 1e-13) == 4
    # zeros at the cut are not a multiplet: the bond stays full
    z = np.array([1.0, 0.5, 0.0, 0.0, 0.0])
    assert mps.truncation_rank(z, 0.0, 4, 1e-13) == 4


@pytest.mark.parametrize("direction", ["lr", "rl"])
def test_split_reconstructs_and_is_canonical(direction):
    rng = np.random.default_rng(60)
    theta = rng.standard_normal((3, 2, 2, 5))
    A1, A2, info = mps.split_two_site(theta, direction, 0.0, 100, 1e-13)
    assert np.abs(mps.two_site(A1, A2) - theta).max() < 1e-13
    if direction == "lr":
        assert mps.left_orthonormality_error(A1) < 1e-14
    else:
        assert mps.right_orthonormality_error(A2) < 1e-14
    s = np.linalg.svd(theta.reshape(6, 10), compute_uv=False)
    A1, A2, info = mps.split_two_site(theta, direction, 0.0, 4, 1e-13)
    assert info["k"] == 4
    err = np.linalg.norm(mps.two_site(A1, A2) - theta) ** 2
    assert abs(err - s[4:] @ s[4:]) < 1e-12       # Eckart-Young
    assert abs(info["disc"] - s[4:] @ s[4:] / (s @ s)) < 1e-14


# --- the implicit step -------------------------------------------------------

def _check_against_ed(L, W, H, spinors, chi, scheme, shift_mode, grid, tol_e, tol_ov, perm=None):
    e0 = ed.ground_state(H)[0]
    psi = mps.product_state(spinors, chi, pad_full=True)
    v0 = mps.to_vector(psi)
    if perm is not None:
        v0k = np.empty_like(v0)
        v0k[perm] = v0
    else:
        v0k = v0
    opts = mps.StepOptions(scheme=scheme, shift_mode=shift_mode, shift=e0, chi_max=chi,
                           cutoff=0.0, krylov_dim=10, max_cycles=200, tol_loc=1e-13)
    out, reps = mps.evolve_grid(psi, W, grid, opts)
    states, en, norms, shifts = ed.evolve_dense(H, v0k, grid, scheme, shift_mode, e0)
    for r, e, nb in zip(reps, en[1:], norms[1:]):
        assert abs(r.energy - e) <= tol_e * abs(e)
        assert abs(r.norm_before - nb) <= 1e-9 * nb
    v = mps.to_vector(out)
    vk = v if perm is None else v[np.argsort(perm)]
    assert abs(np.linalg.norm(v) - 1) < 1e-12
    assert 1 - abs(vk @ states[-1]) <= tol_ov
    for a in out[1:]:
        assert mps.right_orthonormality_error(a) < 1e-12
    return reps, en


@pytest.mark.parametrize("scheme", ["be", "trap"])
@pytest.mark.parametrize("shift_mode", ["fixed", "track"])
def test_mps_step_equals_full_vector_step_heisenberg(scheme, shift_mode):
    # Complete bases (chi = 2^(L/2)): the Galerkin solve is the exact step.
    L = 6
    W = mpo.heisenberg_mpo(L)
    H = ed.heisenberg_dense(L)
    sp = random_spinors(rng_for(0, 1), L, 2)
    _check_against_ed(L, W, H, sp, 8, scheme, shift_mode, ed.loggrid(0.01, 100.0, 1.5)[:12], 1e-10, 1e-12)


def test_mps_step_equals_full_vector_step_impurity():
    eb, V = np.array([-0.6, 0.05, 0.5]), np.array([0.3, 0.25, 0.4])
    U = 4.0
    W = mpo.aim_mpo(U, -U / 2, eb, V)
    H = ed.aim_dense(U, -U / 2, eb, V)
    perm = ed.aim_basis_permutation(4)
    sp = random_spinors(rng_for(3, 1), 4, 4)
    _check_against_ed(4, W, H, sp, 16, "trap", "track", ed.loggrid(0.01, 100.0, 1.5)[:10], 1e-10, 1e-12, perm)


def test_backward_euler_monotone_and_reaches_ground_state():
    L = 6
    W = mpo.heisenberg_mpo(L)
    H = ed.heisenberg_dense(L)
    e0 = ed.ground_state(H)[0]
    sp = random_spinors(rng_for(0, 2), L, 2)
    reps, en = _check_against_ed(L, W, H, sp, 8, "be", "fixed", ed.loggrid(0.01, 100.0, 1.5), 1e-10, 1e-12)
    E = [r.energy for r in reps]
    assert np.all(np.diff(E) <= 1e-12)
    assert E[-1] - e0 < 1e-8


def test_xx_chain_reaches_closed_form_without_ed():
    # L = 16 is beyond the dense reference; the XX closed form pins the result.
    # Fixed shift just below E0 keeps I + h (H - s) positive definite (with the
    # shift above E0 the operator turns indefinite at large h).
    L = 16
    e0 = ed.xx_chain_e0(L)
    W = mpo.heisenberg_mpo(L, Jz=0.0)
    sp = random_spinors(rng_for(0, 3), L, 2)
    psi = mps.product_state(sp)
    opts = mps.StepOptions(scheme="be", shift_mode="fixed", shift=e0 - 1e-3, chi_max=32,
                           cutoff=1e-12, krylov_dim=10, max_cycles=1, tol_loc=0.0)
    out, reps = mps.evolve_grid(psi, W, ed.loggrid(0.05, 1000.0, 2.0), opts)
    assert abs(reps[-1].energy - e0) < 1e-8 * abs(e0)
    assert max(mps.bond_dims(out)) <= 32
    assert abs(mps.overlap(out, out) - 1) < 1e-12


def test_paper_budget_counts_matvecs():
    # one GMRES cycle of 10 Arnoldi steps: 11 products per block once n > 10
    L = 8
    W = mpo.heisenberg_mpo(L)
    sp = random_spinors(rng_for(0, 4), L, 2)
    psi = mps.product_state(sp, 16, pad_full=True)
    opts = mps.StepOptions(scheme="trap", shift_mode="track", chi_max=16, cutoff=0.0)
    out, rep = mps.imag_step(psi, W, 0.05, opts)
    dims = mps.bond_dims(psi)
    expect = 0
    blocks = list(range(L - 1)) + list(range(L - 2, -1, -1))
    for i in blocks:
        n = dims[i] * 4 * dims[i + 2]
        expect += 1 + min(10, n)
    assert rep.matvecs <= expect
    assert rep.matvecs >= expect - 2 * (L - 1) * 2      # early invariant-space stops only


def _krylov_minimiser(A, b, x0, m):
    """Brute-force GMRES(m) cycle: x0 + argmin over span{r0, A r0, .., A^(m-1) r0}
    of ||b - A x||, from the explicit Krylov matrix (no Arnoldi)."""
    r0 = b - A @ x0
    K = np.stack([np.linalg.matrix_power(A, j) @ r0 for j in range(m)], axis=1)
    y = np.linalg.lstsq(A @ K, r0, rcond=None)[0]
    return x0 + K @ y


@pytest.mark.parametrize("init_guess", ["b", "psi"])
@pytest.mark.parametrize("m", [1, 2])
def test_initial_guess_on_a_single_block_by_brute_force(init_guess, m):
    # L = 2: the sweep is the block (1, 2) solved twice (left-to-right, then
    # right-to-left) with complete bonds, so the step is two GMRES(m) cycles on
    # the dense 4 x 4 problem.  Appendix B starts the first from b, the "psi"
    # reading from psi; the second starts from the first's result.
    H = ed.heisenberg_dense(2, Jz=0.6)
    sp = random_spinors(rng_for(4, 1), 2, 2)
    psi = mps.product_state(sp)
    v = mps.to_vector(psi)
    v = v / np.linalg.norm(v)
    h = 0.7
    s = float(v @ H @ v)
    A = (1 - h * s) * np.eye(4) + h * H
    b = (1 + h * s) * v - h * (H @ v)
    x = _krylov_minimiser(A, b, b if init_guess == "b" else v, m)
    x = _krylov_minimiser(A, b, x, m)
    x = x / np.linalg.norm(x)
    opts = mps.StepOptions(scheme="trap", shift_mode="track", chi_max=4, cutoff=0.0, krylov_dim=m,
                           init_guess=init_guess)
    out, rep = mps.imag_step(psi, mpo.heisenberg_mpo(2, Jz=0.6), h, opts)
    got = mps.to_vector(out)
    assert abs(abs(got @ x) - 1) < 1e-13
    assert abs(rep.energy - x @ H @ x) < 1e-13
    # the two guesses give different steps with this budget
    other = _krylov_minimiser(A, b, v if init_guess == "b" else b, m)
    other = _krylov_minimiser(A, b, other, m)
    other = other / np.linalg.norm(other)
    assert abs(abs(got @ other) - 1) > 1e-11


def test_initial_guess_is_irrelevant_for_backward_euler_and_converged_solves():
    # backward Euler: b = psi, so both guesses are the same step (bitwise);
    # tolerance-driven solves reach the same step from either guess
    L = 8
    W = mpo.heisenberg_mpo(L)
    psi = mps.product_state(random_spinors(rng_for(4, 2), L, 2), 16, pad_full=True)
    for kw, tol in ((dict(scheme="be"), None), (dict(scheme="trap", max_cycles=200, tol_loc=1e-13), 1e-10)):
        outs = []
        for g in ("b", "psi"):
            o = mps.StepOptions(shift_mode="track", chi_max=16, cutoff=0.0, init_guess=g, **kw)
            outs.append(mps.imag_step(psi, W, 0.4, o))
        (a, ra), (b_, rb) = outs
        if tol is None:
            assert all(np.array_equal(x, y) for x, y in zip(a, b_))
        else:
            assert abs(ra.energy - rb.energy) < tol * abs(ra.energy)
            assert 1 - abs(mps.overlap(a, b_)) < 1e-10

"""Pins of the Gauss-Legendre collocation oracle (``oracle/gauss.py``):
quadrature and collocation order conditions, the diagonal Pade approximant of
the exponential in closed form, the one-node case against the trapezoid step,
the convergence order, the right-end read-off, the shifted and augmented MPOs
against their dense operators, the widened augmented state (the same state,
right-orthonormal), and the MPS panel at complete bonds against the dense
panel (with four and five nodes only through the widening)."""
import math

import numpy as np
import pytest

from oracle import ed, gauss, mpo, mps
from workload import random_spinors, rng_for


def _pade(p, z):
    # diagonal (p, p) Pade approximant of exp(-z): N(-z) / N(z),
    # N(z) = sum_k (2p - k)! p! / ((2p)! k! (p - k)!) z^k
    N = lambda x: sum(math.factorial(2 * p - k) * math.factorial(p)
                      / (math.factorial(2 * p) * math.factorial(k) * math.factorial(p - k)) * x ** k
                      for k in range(p + 1))
    return N(-z) / N(z)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_order_conditions(p):
    c, b, A = gauss.collocation_matrix(p)
    assert np.all(np.diff(c) > 0) and c[0] > 0 and c[-1] < 1
    # Gauss quadrature integrates t^(k-1) exactly up to k = 2p
    for k in range(1, 2 * p + 1):
        assert abs(b @ c ** (k - 1) - 1.0 / k) < 1e-14
    assert abs(b @ c ** (2 * p) - 1.0 / (2 * p + 1)) > 1e-6     # and not beyond
    # collocation: the rows of A integrate t^(k-1) from 0 to c_i for k <= p
    for k in range(1, p + 1):
        assert np.abs(A @ c ** (k - 1) - c ** k / k).max() < 1e-14
    # the weights are the last row's integral to 1 (B from the same basis)
    r_inf, w = gauss.end_weights(p)
    assert abs(r_inf - (-1) ** p) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("dtau,s", [(0.7, 0.0), (0.3, -1.5), (1e3, 0.2)])
def test_dense_step_is_diagonal_pade(p, dtau, s):
    rng = np.random.default_rng(40 + p)
    n = 12
    M = rng.standard_normal((n, n))
    H = (M + M.T) / 2
    psi = rng.standard_normal(n)
    end, Y = gauss.dense_step(H, psi, dtau, p, s)
    lam, V = np.linalg.eigh(H)
    z = dtau * (lam - s)
    want = V @ (_pade(p, z) * (V.T @ psi))
    assert np.abs(end - want).max() <= 1e-10 * max(1.0, np.abs(want).max())
    # A-stability where the spectrum is above the shift
    if np.all(z >= 0):
        assert np.all(np.abs(_pade(p, z)) <= 1 + 1e-14)


def test_one_node_is_the_trapezoid_step():
    H = ed.heisenberg_dense(6)
    psi = np.random.default_rng(3).standard_normal(H.shape[0])
    for dtau, s in [(0.4, 0.0), (5.0, -2.0)]:
        end, _ = gauss.dense_step(H, psi, dtau, 1, s)
        assert np.abs(end - ed.implicit_step(H, psi, dtau / 2, s, "trap")).max() < 1e-12


@pytest.mark.parametrize("p,rate", [(1, 4.0), (2, 16.0), (3, 64.0)])
def test_convergence_order(p, rate):
    H = ed.heisenberg_dense(6)
    psi0 = np.random.default_rng(5).standard_normal(H.shape[0])
    T = 2.0
    exact = ed.exact_evolve(H, psi0, T)
    exact /= np.linalg.norm(exact)
    errs = []
    for n in (4, 8):
        st, _ = gauss.dense_evolve(H, psi0, np.linspace(0.0, T, n + 1), p, "fixed", 0.0)
        errs.append(np.linalg.norm(st[-1] - exact))
    assert 0.7 * rate < errs[0] / errs[1] < 1.4 * rate


@pytest.mark.parametrize("p", [1, 2, 3])
def test_right_end_read_off(p):
    # r_inf psi + sum_j w_j Y_j equals the integral equation at the right end
    rng = np.random.default_rng(7 + p)
    n = 10
    M = rng.standard_normal((n, n))
    H = M + M.T
    psi = rng.standard_normal(n)
    end, Y = gauss.dense_step(H, psi, 0.9, p, 0.3)
    r_inf, w = gauss.end_weights(p)
    assert np.abs(r_inf * psi + w @ Y - end).max() < 1e-11 * np.abs(end).max()


def test_shifted_and_augmented_mpo_are_their_operators():
    L, s, p = 5, -0.8, 2
    W = mpo.heisenberg_mpo(L, Jz=0.7)
    H = ed.heisenberg_dense(L, Jz=0.7)
    n = H.shape[0]
    Ws = gauss.shifted_mpo(W, s)
    assert mpo.mpo_bond_dims(Ws)[1:-1] == [w + 1 for w in mpo.mpo_bond_dims(W)[1:-1]]
    assert np.abs(mpo.mpo_to_dense(Ws) - (H - s * np.eye(n))).max() < 1e-13
    _, _, A = gauss.collocation_matrix(p)
    At = np.zeros((p + 1, p + 1))
    At[1:, 1:] = A
    Wa = gauss.augmented_mpo(W, p, s)
    assert np.abs(mpo.mpo_to_dense(Wa) - np.kron(At, H - s * np.eye(n))).max() < 1e-13
    # a single site
    W1 = [np.diag([1.0, -1.0]).reshape(1, 1, 2, 2)]
    assert np.abs(mpo.mpo_to_dense(gauss.shifted_mpo(W1, 0.5)) - np.diag([0.5, -1.5])).max() == 0.0


def test_augmented_state_and_node_contraction():
    sp = random_spinors(rng_for(0, 9), 4, 2)
    psi = mps.product_state(sp)
    v = mps.to_vector(psi)
    aug = gauss.augmented_state(psi, 3)
    assert np.abs(mps.to_vector(aug) - np.kron(np.full(4, 0.5), v)).max() < 1e-15
    coef = np.array([0.3, -1.0, 2.0, 0.5])
    assert np.abs(mps.to_vector(gauss.contract_node(aug, coef)) - 0.5 * coef.sum() * v).max() < 1e-15


@pytest.mark.parametrize("p", [4, 5, 7])
def test_widened_augmented_state_is_the_same_state(p):
    # p + 1 > d_1 D_2 = 4: the bonds complete within chi_max are widened by
    # zero-weight orthonormal completions; same vector, right-orthonormal
    # sites, the complete bond dimensions (capped where they exceed chi_max)
    L, chi = 6, 24
    psi = mps.product_state(random_spinors(rng_for(0, 12), L, 2), 64, pad_full=True)
    plain = gauss.augmented_state(psi, p)
    wide = gauss.augmented_state(psi, p, chi)
    assert np.abs(mps.to_vector(wide) - mps.to_vector(plain)).max() < 1e-14
    for a in wide[1:]:
        assert mps.right_orthonormality_error(a) < 1e-13
    complete = mps.full_dims(L + 1, [p + 1] + [2] * L, 2 ** 62)
    want = [c if c <= chi else b for c, b in zip(complete, mps.bond_dims(plain))]
    assert mps.bond_dims(wide) == want and max(want) > max(mps.bond_dims(plain))
    # p + 1 <= 4: left as it is
    assert mps.bond_dims(gauss.augmented_state(psi, 3, chi)) == mps.bond_dims(gauss.augmented_state(psi, 3))
    # a product state (bonds 1): p + 1 > d_1 = 2 already for two nodes; the
    # widening stops where a site's right bond leaves no room (d_i times it)
    prod = mps.product_state(random_spinors(rng_for(0, 13), 10, 2), 16)
    for q in (2, 5):
        wide = gauss.augmented_state(prod, q, 16)
        assert np.abs(mps.to_vector(wide) - mps.to_vector(gauss.augmented_state(prod, q))).max() < 1e-14
        dims = mps.bond_dims(wide)
        assert dims[1] == q + 1 and all(dims[k] <= 2 * dims[k + 1] for k in range(1, len(wide)))
        for a in wide[1:]:
            assert mps.right_orthonormality_error(a) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("shift_mode", ["fixed", "track"])
def test_mps_panel_equals_dense_panel_at_complete_bonds(p, shift_mode):
    L = 6
    W = mpo.heisenberg_mpo(L)
    H = ed.heisenberg_dense(L)
    e0 = ed.ground_state(H)[0]
    sp = random_spinors(rng_for(0, 11), L, 2)
    psi = mps.product_state(sp, 64, pad_full=True)
    opts = mps.StepOptions(shift_mode=shift_mode, shift=e0, chi_max=64, cutoff=0.0, krylov_dim=10,
                           max_cycles=400, tol_loc=1e-13)
    grid = [0.0, 0.1, 0.3, 0.7, 1.5]
    out, reps = gauss.gl_evolve(psi, W, grid, p, opts)
    st, en = gauss.dense_evolve(H, mps.to_vector(psi), grid, p, shift_mode, e0)
    for r, e in zip(reps, en[1:]):
        assert abs(r.energy - e) <= 1e-10 * abs(e)
    v = mps.to_vector(out)
    assert abs(np.linalg.norm(v) - 1.0) < 1e-12
    assert 1.0 - abs(v @ st[-1]) < 1e-10
    for a in out[1:]:
        assert mps.right_orthonormality_error(a) < 1e-12
    # the augmented sweep widened the left bonds; the panel's state is cut
    # back to the chain's own bond dimensions
    assert max(r.extra["aug_max_chi"] for r in reps) > 0
    assert mps.bond_dims(out) == mps.full_dims(L, 2, 64)


def test_recompress_is_exact_and_minimal():
    # an MPS whose left bonds are padded with redundant directions
    rng = np.random.default_rng(12)
    L = 6
    A = [rng.standard_normal((1, 2, 6))] + [rng.standard_normal((6, 2, 6)) for _ in range(2)] + \
        [rng.standard_normal((6, 2, 4)), rng.standard_normal((4, 2, 2)), rng.standard_normal((2, 2, 1))]
    v = mps.to_vector(A)
    B = gauss.recompress(A, 64, 1e-13)
    assert np.abs(mps.to_vector(B) - v).max() < 1e-12 * np.abs(v).max()
    assert mps.bond_dims(B) == [1, 2, 4, 6, 4, 2, 1]
    # the sites the two passes went over are right-orthonormal again, the
    # others untouched
    for a in B[1:3]:
        assert mps.right_orthonormality_error(a) < 1e-12
    for a, b in zip(A[3:], B[3:]):
        assert np.array_equal(a, b)

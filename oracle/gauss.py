"""Gauss-Legendre collocation on a panel (the spectral variant of the Method
section: the solution on a panel is a polynomial in tau, fixed by requiring
the integral form of the evolution equation, Eq. 2 with the integration
starting at the panel's left end, at the Gauss-Legendre nodes; one linear
system per panel).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings (the paper leaves the details to a later publication):
  * the unknowns are the values of the polynomial (degree p - 1) at the p
    nodes c_1..c_p of the panel [a, a + dtau] (nodes on [0, 1]); the paper's
    Legendre coefficients are these values in another basis (an invertible
    p x p change of basis), so the linear system and its solution are the
    same.  Requiring psi(a + c_i dtau) = psi(a) - int_a^(a + c_i dtau)
    (H - s) u at every node gives, with A_ij = int_0^(c_i) l_j (l_j the
    Lagrange polynomial of node j),
        (I + dtau A (x) (H - s)) Y = 1 (x) psi(a),     Y_i = u(a + c_i dtau);
  * the value at the panel's right end is the integral equation taken there:
    psi(a + dtau) = psi(a) - dtau sum_j b_j (H - s) Y_j with the Gauss
    weights b_j (the integral of the interpolant).  In exact arithmetic this
    is the p-point Gauss collocation (Gauss-Legendre Runge-Kutta) value, the
    (p, p) Pade approximant of exp(-dtau (H - s)) applied to psi(a);
  * shift: s = the energy of psi(a) (tracking, as for the trapezoid step) or
    a fixed value; it changes the norm of the exact evolution only, but not
    only the norm of the collocation value;
  * on an MPS the unknowns Y_1..Y_p form one MPS with an extra leading site
    of dimension p + 1 (the node index), component 0 holding psi(a) itself:
    Z = (psi(a), Y_1, .., Y_p) solves (I + dtau At (x) (H - s)) Z = 1 (x) psi(a)
    with At = [[0, 0], [0, A]], a backward-Euler-type system (step size dtau,
    shift 0) for the MPO At (x) (H - s) on L + 1 sites, solved by the same
    two-site sweep as every other step.  The right-end value is then read off
    the node index without a further operator product: from the stage
    equations, dtau (H - s) Y = A^(-1) (1 psi(a) - Y) row by row, so
    psi(a + dtau) = r_inf psi(a) + sum_j w_j Y_j with w = A^(-T) b and
    r_inf = 1 - b^T A^(-1) 1 (= (-1)^p, the approximant at infinity).  The
    MPS of psi(a + dtau) is the augmented MPS with the node site contracted
    with v = (r_inf, w) into site 1.  (Exact when the stage equations are;
    with truncation the two right-end formulas differ at the truncation
    level.)
  * the MPO of (H - s) is the direct sum of H's MPO and -s times the identity
    (bond dimension w + 1), which needs no knowledge of H's MPO layout;
  * the node bond needs rank p + 1, but the first block of the sweep can
    give it at most d_1 D_2 (with psi's bonds): when p + 1 is larger (p >= 4
    on a spin-1/2 chain), the augmented state's bonds that are complete
    within chi_max are widened to complete before the sweep by zero-weight
    orthonormal completions (``augmented_state``), without which the panel
    is not exact even at complete bonds;
  * after the contraction the bonds near the left end can be larger than
    the chain can need (the augmented left space is p + 1 times larger):
    every bond up to the last one above min(prod d left, prod d right,
    chi_max) is cut back by exact two-site splits (cutoff 0, left to right,
    then right to left back to site 1), so that the next panel starts from a
    right-orthonormal state with the centre on site 1 and minimal bonds.
"""
from __future__ import annotations

from dataclasses import replace
import math

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly

from . import mps as omps


def nodes_weights(p: int):
    """Gauss-Legendre nodes c (ascending) and weights b on [0, 1]."""
    if p < 1:
        raise ValueError("p must be at least 1")
    x, w = npleg.leggauss(p)
    return (x + 1.0) / 2.0, w / 2.0


def collocation_matrix(p: int):
    """(c, b, A) with A_ij = int_0^(c_i) l_j(t) dt, l_j the Lagrange
    polynomial of the nodes that is 1 at c_j."""
    c, b = nodes_weights(p)
    A = np.empty((p, p))
    for j in range(p):
        lj = nppoly.polyfromroots(np.delete(c, j))
        lj = lj / nppoly.polyval(c[j], lj)
        Ij = nppoly.polyint(lj)                 # antiderivative vanishing at 0
        A[:, j] = nppoly.polyval(c, Ij)
    return c, b, A


def end_weights(p: int):
    """(r_inf, w): the right-end value is r_inf psi(a) + sum_j w_j Y_j."""
    c, b, A = collocation_matrix(p)
    w = np.linalg.solve(A.T, b)
    r_inf = 1.0 - float(b @ np.linalg.solve(A, np.ones(p)))
    return r_inf, w


def dense_step(H: np.ndarray, psi: np.ndarray, dtau: float, p: int, s: float = 0.0):
    """One panel on a dense vector: solve the collocation system, return the
    right-end value (not normalised) and the node values Y [p, n]."""
    c, b, A = collocation_matrix(p)
    n = psi.shape[0]
    Hs = H - s * np.eye(n)
    K = np.eye(p * n) + dtau * np.kron(A, Hs)
    Y = np.linalg.solve(K, np.tile(psi, p)).reshape(p, n)
    end = psi - dtau * (Hs @ (b @ Y))
    return end, Y


def dense_evolve(H: np.ndarray, psi0: np.ndarray, grid, p: int, shift_mode: str = "track", shift: float = 0.0):
    """Panels along an explicit grid, normalising after every panel; returns
    the states (psi0 normalised first) and the energies."""
    v = psi0 / np.linalg.norm(psi0)
    states, energies = [v], [float(v @ H @ v)]
    for k in range(1, len(grid)):
        s = float(v @ H @ v) if shift_mode == "track" else shift
        v, _ = dense_step(H, v, float(grid[k] - grid[k - 1]), p, s)
        v = v / np.linalg.norm(v)
        states.append(v)
        energies.append(float(v @ H @ v))
    return states, energies


# ----------------------------------------------------------------------------
# MPS form
# ----------------------------------------------------------------------------

def shifted_mpo(W, s: float):
    """MPO of H - s I: the direct sum of H's MPO and the identity MPO scaled by
    -s (bond dimensions w + 1)."""
    L = len(W)
    out = []
    for j, Wj in enumerate(W):
        wl, wr, d, _ = Wj.shape
        first, last = j == 0, j == L - 1
        nl = wl if first else wl + 1
        nr = wr if last else wr + 1
        if first and last:
            T = np.zeros((1, 1, d, d))
            T[0, 0] = Wj[0, 0] - s * np.eye(d)
        else:
            T = np.zeros((1 if first else nl, 1 if last else nr, d, d))
            if first:
                T[0, :wr] = Wj[0]
                T[0, wr] = -s * np.eye(d)
            elif last:
                T[:wl, 0] = Wj[:, 0]
                T[wl, 0] = np.eye(d)
            else:
                T[:wl, :wr] = Wj
                T[wl, wr] = np.eye(d)
        out.append(T)
    return out


def augmented_mpo(W, p: int, s: float):
    """MPO of At (x) (H - s) on L + 1 sites, the node site first."""
    _, _, A = collocation_matrix(p)
    At = np.zeros((p + 1, p + 1))
    At[1:, 1:] = A
    return [At.reshape(1, 1, p + 1, p + 1)] + shifted_mpo(W, s)


def augmented_state(psi, p: int, chi_max: int | None = None):
    """(1 / sqrt(p + 1)) (1, .., 1) (x) psi as an MPS on L + 1 sites.

    The sweep can give the node bond rank at most d_1 D_2 in its first block
    (site 1's dimension times the bond behind it); when p + 1 exceeds that,
    the bonds whose complete dimension in the augmented chain is at most
    chi_max and above the chain's own are widened to it before the sweep,
    and the others to at least
    what the node rank needs to pass (p + 1 over the site dimensions
    between; a bond at most d_i times the widened bond right of site i),
    right to left: a widened right bond gets
    zero columns, and a widened left bond gets the trailing columns of the
    Householder Q of the site's rows transposed (an orthonormal completion
    of its rows, as numpy's complete QR computes it).
    The added basis states carry no weight, so the state is the same and
    stays right-orthonormal with the centre on the node site."""
    node = np.full((1, p + 1, 1), 1.0 / math.sqrt(p + 1))
    A = [node] + [a.copy() for a in psi]
    if chi_max is None or p + 1 <= psi[0].shape[1] * psi[0].shape[2]:
        return A
    n = len(A)
    dims = [a.shape[1] for a in A]
    complete = omps.full_dims(n, dims, 2 ** 62)
    cur = omps.bond_dims(A)
    # bonds complete within chi_max: complete; others at least what the node
    # rank p + 1 needs to pass (p + 1 over the dimensions between)
    need = [1] * (n + 1)
    need[1] = p + 1
    for k in range(2, n):
        need[k] = -(-need[k - 1] // dims[k - 1])
    # (only where the augmented chain's complete bond exceeds the chain's own:
    # towards the right end both are the product of the dimensions right of
    # the bond)
    own = [1] + omps.full_dims(n - 1, dims[1:], 2 ** 62)
    tgt = [complete[k] if complete[k] <= chi_max and complete[k] > own[k] else max(cur[k], min(need[k], chi_max))
           for k in range(n + 1)]
    # a site's rows can be completed only within d_i times its right bond
    for k in range(n - 1, 0, -1):
        tgt[k] = max(cur[k], min(tgt[k], dims[k] * tgt[k + 1]))
    for i in range(n - 1, -1, -1):
        Dl, d, Dr = A[i].shape
        if tgt[i + 1] > Dr:
            A[i] = np.concatenate([A[i], np.zeros((Dl, d, tgt[i + 1] - Dr))], axis=2)
            Dr = tgt[i + 1]
        if i > 0 and tgt[i] > Dl:
            R = A[i].reshape(Dl, d * Dr)
            Q, _ = np.linalg.qr(R.T, mode="complete")
            A[i] = np.concatenate([R, Q[:, Dl:tgt[i]].T], axis=0).reshape(tgt[i], d, Dr)
    return A


def contract_node(aug, v):
    """Contract the node site of an augmented MPS with v into the first
    chain site."""
    r = np.tensordot(v, aug[0][0], axes=([0], [0]))            # [D1]
    A1 = np.tensordot(r, aug[1], axes=([0], [0]))[None]         # [1, d, D2]
    return [A1] + [a.copy() for a in aug[2:]]


def recompress(A, chi_max: int, tie_rel: float):
    """Cut bonds above min(prod d left, prod d right, chi_max) back by exact
    splits: left to right over the bonds up to the last such bond, then
    right to left back to site 1."""
    L = len(A)
    caps = omps.full_dims(L, [a.shape[1] for a in A], chi_max)
    dims = omps.bond_dims(A)
    over = [b for b in range(1, L) if dims[b] > caps[b]]
    A = [a.copy() for a in A]
    if not over:
        return A
    last = max(over)
    for i in range(last):                       # blocks (i, i + 1): bond i + 1
        A[i], A[i + 1], _ = omps.split_two_site(omps.two_site(A[i], A[i + 1]), "lr", 0.0,
                                                min(chi_max, caps[i + 1]), tie_rel)
    for i in range(last - 1, -1, -1):
        A[i], A[i + 1], _ = omps.split_two_site(omps.two_site(A[i], A[i + 1]), "rl", 0.0,
                                                min(chi_max, caps[i + 1]), tie_rel)
    return A


def gl_step(psi, W, dtau: float, p: int, opts):
    """One panel of p-point Gauss-Legendre collocation on an MPS; opts as for
    ``mps.imag_step`` (its scheme is ignored: the augmented system is solved
    as a backward-Euler-type system with shift 0).  Returns (psi_new, report)
    with the energy and shift of the physical chain."""
    s = omps.expectation(psi, W) if opts.shift_mode == "track" else opts.shift
    Wa = augmented_mpo(W, p, s)
    xa, rep = omps.imag_step(augmented_state(psi, p, opts.chi_max), Wa, dtau,
                             replace(opts, scheme="be", shift_mode="fixed", shift=0.0))
    r_inf, w = end_weights(p)
    out = recompress(contract_node(xa, np.concatenate([[r_inf], w])), opts.chi_max, opts.tie_rel)
    nrm = float(np.linalg.norm(out[0]))
    out[0] = out[0] / nrm
    rep.norm_before = nrm
    rep.shift = s
    rep.h = dtau
    rep.energy = omps.expectation(out, W)
    rep.max_chi = max(omps.bond_dims(out))
    rep.extra["aug_max_chi"] = max(omps.bond_dims(xa))
    return out, rep


def gl_evolve(psi, W, grid, p: int, opts):
    """Panels along an explicit grid; returns (psi, reports)."""
    reps = []
    for k in range(1, len(grid)):
        psi, rep = gl_step(psi, W, float(grid[k] - grid[k - 1]), p, opts)
        rep.tau = float(grid[k])
        reps.append(rep)
    return psi, reps

"""Dense-tensor MPS algorithm of the oracle (the implicit step as a two-site,
DMRG-style linear solve).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions: site tensors A_i[Dl, d, Dr]; MPO tensors W_i[wl, wr, s_out, s_in];
environments carry x's index first, then the MPO index, then the ket's index:
L[a', w, a], R[c', w, c]; overlap environments L[a', a], R[c', c].

One step (Method, Eq. 4 and the two operations listed after it; Appendix B;
Appendix D for the budget and the shift):

  1. psi is normalised and right-orthonormal with the centre on site 1.
     x <- copy of psi.  s = fixed shift, or the energy of psi ("track").
  2. Right environments of <x|H|x>; while x = psi the mixed <x|H|psi> and
     <x|psi> environments equal the <x|H|x> one and the identity.
  3. Left-to-right half sweep over the blocks (j, j+1):
       theta_psi = psi_j psi_(j+1)
       b  = P^T psi                                  (backward Euler)
       b  = (1 + h s) P^T psi - h P^T H psi          (trapezoid)
         -- the right-hand side projected into x's basis, computed exactly
            through the mixed environments;
       theta0 = b on the first block of the step (the right-hand side is the
         initial guess, Appendix B), x_j x_(j+1) on every later block
         (or x_j x_(j+1) throughout with init_guess = "psi");
       GMRES on (1 - h s) v + h H_eff v = b;
       SVD split, A_j = U, A_(j+1) = S V^T; update the left environments.
  4. Right-to-left half sweep, mirrored (A_j = U S, A_(j+1) = V^T).
  5. Normalise x, measure E = <x|H|x>, psi <- x.

Readings where the paper is silent:
  * b is projected exactly through mixed environments rather than first formed
    as an MPS by the density-matrix MPO-MPS product;
  * the initial guess: Appendix B starts the solve from b itself.  x starts
    as a copy of psi (its basis is the one b is projected into), and the
    local guess of the step's first block is b projected into that basis,
    which is what x = b would give there; later blocks start from the
    current x_j x_(j+1), as a sweep does.  For backward Euler b = psi, so both
    choices coincide.  init_guess = "psi" uses x_j x_(j+1) on every block;
  * the budget of Appendix D is one GMRES cycle of at most 10 Arnoldi steps
    per local solve and one sweep per step, a sweep being a left-to-right
    plus a right-to-left half sweep;
  * truncation: keep the smallest k with sum_(i>=k) s_i^2 <= cutoff sum s_i^2,
    1 <= k <= chi_max; with cutoff 0 keep min(rows, cols, chi_max) values,
    zeros included; a cut inside a group of (numerically) equal non-zero
    singular values moves down to below the group.

Pins (``tests/test_oracle_mps.py``): with complete bases (``pad_full`` at
L = 8..10, chi = 2^(L/2)) every step equals the full-vector implicit step of
``oracle.ed`` to 1e-10; GMRES equals the minimiser over the explicitly built
Krylov space and, for m >= n, the dense solve; the SVD split reproduces theta;
environments reproduce the dense expectation value; canonical forms are
isometries; the energy decreases monotonically under backward Euler with the
exact ground-state shift and reaches the ED ground state at large tau; the XX
chain reaches its closed-form energy.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


# ----------------------------------------------------------------------------
# States
# ----------------------------------------------------------------------------

def full_dims(L: int, d, chi_max: int) -> list[int]:
    """Bond dimensions min(prod of d left of the bond, prod right of it,
    chi_max); d is one dimension for every site or a list of L."""
    ds = [int(d)] * L if np.ndim(d) == 0 else [int(x) for x in d]
    out = []
    for i in range(L + 1):
        left = math.prod(ds[:i]) if i < 62 else chi_max
        right = math.prod(ds[i:]) if L - i < 62 else chi_max
        out.append(int(min(chi_max, left, right)))
    return out


def product_state(spinors, chi_max: int | None = None, pad_full: bool = False) -> list[np.ndarray]:
    """Product state from normalised spinors.

    Without padding every bond has dimension 1.  With ``pad_full`` the state is
    embedded in bonds of dimension min(d^i, d^(L-i), chi_max): row 0 of site
    tensor i (as a D_(i-1) x (d D_i) matrix) is u = spinor_i (x) e_0 and the
    other rows are the remaining rows of the Householder reflector
    I - 2 v v^T / v^T v, v = e_0 - u, which maps e_0 to u.  The rows are then
    orthonormal (right-orthonormal form) and only bond index 0 is ever reached
    from the left, so the state is unchanged.
    """
    L = len(spinors)
    if not pad_full:
        return [np.asarray(s, dtype=float).reshape(1, len(s), 1).copy() for s in spinors]
    dims = full_dims(L, [len(s) for s in spinors], chi_max)
    out = []
    for i, sp in enumerate(spinors):
        d = len(sp)
        dl, dr = dims[i], dims[i + 1]
        u = np.zeros(d * dr)
        u[np.arange(d) * dr] = sp
        v = -u
        v[0] += 1.0
        vv = float(v @ v)
        refl = np.eye(d * dr)
        if vv > 0.0:
            refl = refl - 2.0 * np.outer(v, v) / vv
        out.append(np.ascontiguousarray(refl[:dl, :]).reshape(dl, d, dr))
    return out


def bond_dims(A) -> list[int]:
    return [A[0].shape[0]] + [a.shape[2] for a in A]


def to_vector(A) -> np.ndarray:
    """Contract the MPS to a dense vector (site 1 most significant)."""
    v = A[0]
    for a in A[1:]:
        v = np.tensordot(v, a, axes=([v.ndim - 1], [0]))
    return v.reshape(-1)


def overlap(A, B) -> float:
    """<A|B> by transfer matrices from the left:
    E'[j, b] = sum E[i, a] A[i, s, j] B[a, s, b], one pairwise contraction at
    a time."""
    E = np.ones((1, 1))
    for a, b in zip(A, B):
        t = np.tensordot(E, b, axes=([1], [0]))                # [i, s, b]
        E = np.tensordot(a, t, axes=([0, 1], [0, 1]))          # [j, b]
    return float(E[0, 0])


def expectation(A, W) -> float:
    """<A|H|A> / <A|A> by contracting left environments over the whole chain."""
    E = np.ones((1, 1, 1))
    for a, w in zip(A, W):
        E = env_left_h(E, a, w, a)
    return float(E[0, 0, 0]) / overlap(A, A)


def right_orthonormality_error(a: np.ndarray) -> float:
    m = a.reshape(a.shape[0], -1)
    return float(np.abs(m @ m.T - np.eye(m.shape[0])).max())


def left_orthonormality_error(a: np.ndarray) -> float:
    m = a.reshape(-1, a.shape[2])
    return float(np.abs(m.T @ m - np.eye(m.shape[1])).max())


# ----------------------------------------------------------------------------
# Environments and the effective operator
# ----------------------------------------------------------------------------

def _c(spec, a, b):
    """Pairwise contraction (einsum notation, dispatched to BLAS)."""
    return np.einsum(spec, a, b, optimize=True)


def env_left_h(Lenv, X, W, Y):
    """L'[b', v, b] = sum L[a', w, a] X[a', p, b'] W[w, v, p, s] Y[a, s, b]."""
    t = _c("iwa,asb->iwsb", Lenv, Y)
    t = _c("iwsb,wvps->ivpb", t, W)
    return _c("ivpb,ipj->jvb", t, X)


def env_right_h(Renv, X, W, Y):
    """R'[b', w, b] = sum R[c', v, c] X[b', p, c'] W[w, v, p, s] Y[b, s, c]."""
    t = _c("kvc,bsc->kvbs", Renv, Y)
    t = _c("kvbs,wvps->kwbp", t, W)
    return _c("kwbp,jpk->jwb", t, X)


def env_left_o(Lenv, X, Y):
    """L'[b', b] = sum L[a', a] X[a', s, b'] Y[a, s, b]."""
    t = _c("ia,asb->isb", Lenv, Y)
    return _c("isb,isj->jb", t, X)


def env_right_o(Renv, X, Y):
    """R'[b', b] = sum R[c', c] X[b', s, c'] Y[b, s, c]."""
    t = _c("kc,bsc->kbs", Renv, Y)
    return _c("kbs,jsk->jb", t, X)


def heff_apply(Lenv, W1, W2, Renv, theta):
    """Two-site effective Hamiltonian applied to theta[a, s1, s2, c]:
    y[a', p, q, c'] = sum L[a', w, a] W1[w, v, p, s1] W2[v, u, q, s2]
                          R[c', u, c] theta[a, s1, s2, c]."""
    t = _c("iwa,astc->iwstc", Lenv, theta)
    t = _c("iwstc,wvps->ivptc", t, W1)
    t = _c("ivptc,vuqt->ipquc", t, W2)
    return _c("ipquc,yuc->ipqy", t, Renv)


def overlap_project(Lo, Ro, theta):
    """y[a', s1, s2, c'] = sum L[a', a] R[c', c] theta[a, s1, s2, c]."""
    t = _c("ia,astc->istc", Lo, theta)
    return _c("istc,yc->isty", t, Ro)


def two_site(A1, A2):
    return np.einsum("asb,btc->astc", A1, A2)


# ----------------------------------------------------------------------------
# GMRES (Saad and Schultz), restarted
# ----------------------------------------------------------------------------

def gmres(apply_A, b, x0, m: int, max_cycles: int = 1, tol: float = 0.0,
          breakdown: float = 1e-14):
    """GMRES(m): x in x0 + K_k(A, r0) minimising ||b - A x||.

    Arnoldi with modified Gram-Schmidt and one re-orthogonalisation pass; the
    small least-squares problem min ||beta e_1 - H_k y|| is solved directly.
    An Arnoldi step ends the cycle when h_(k+1,k) <= breakdown * beta (the
    Krylov space is invariant) or, for tol > 0, when the residual estimate is
    <= tol ||b||.  Cycles restart from the current x while tol > 0 is not met
    and fewer than max_cycles have run.  With tol = 0 every cycle runs
    min(m, n) Arnoldi steps (the paper's fixed budget).
    """
    shape = b.shape
    bv = b.reshape(-1)
    x = x0.reshape(-1).copy()
    n = bv.size
    bnorm = float(np.linalg.norm(bv))
    matvecs = 0
    cycles = 0
    res = float("nan")
    A = lambda v: apply_A(v.reshape(shape)).reshape(-1)
    for _ in range(max_cycles):
        cycles += 1
        r = bv - A(x)
        matvecs += 1
        beta = float(np.linalg.norm(r))
        res = beta
        if beta == 0.0 or (tol > 0 and beta <= tol * bnorm):
            break
        V = [r / beta]
        H = np.zeros((m + 1, m))
        y = np.zeros(0)
        k_used = 0
        for k in range(min(m, n)):
            w = A(V[k])
            matvecs += 1
            for _pass in range(2):
                for i in range(k + 1):
                    c = float(V[i] @ w)
                    H[i, k] += c
                    w = w - c * V[i]
            H[k + 1, k] = float(np.linalg.norm(w))
            k_used = k + 1
            e1 = np.zeros(k + 2)
            e1[0] = beta
            y = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)[0]
            res = float(np.linalg.norm(e1 - H[:k + 2, :k + 1] @ y))
            if H[k + 1, k] <= breakdown * beta:
                break
            if tol > 0 and res <= tol * bnorm:
                break
            V.append(w / H[k + 1, k])
        for i in range(k_used):
            x = x + y[i] * V[i]
        if tol > 0 and res <= tol * bnorm:
            break
        if tol <= 0:
            pass
    rel = res / bnorm if bnorm > 0 else 0.0
    return x.reshape(shape), {"matvecs": matvecs, "cycles": cycles, "res_rel": rel}


# ----------------------------------------------------------------------------
# Truncated SVD split
# ----------------------------------------------------------------------------

def truncation_rank(sigma, cutoff: float, chi_max: int, tie_rel: float) -> int:
    """Number of singular values kept (sigma sorted descending).

    cutoff > 0: smallest k >= 1 with sum_(i>=k) sigma_i^2 <= cutoff * sum sigma^2
    (discarded weight, Heisenberg chain section); cutoff = 0: every value.
    Then k <= chi_max, and while the cut falls inside a group of non-zero
    values closer than tie_rel * sigma_0, k moves below the group.
    """
    s = np.asarray(sigma, dtype=float)
    r = len(s)
    total = float(np.sum(s * s))
    k = r
    if cutoff > 0 and total > 0:
        tail = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
        k = r
        for kk in range(1, r + 1):
            if tail[kk] <= cutoff * total:
                k = kk
                break
    k = max(1, min(k, chi_max))
    tie = tie_rel * (s[0] if r else 0.0)
    while 1 < k < r and s[k - 1] > tie and s[k - 1] - s[k] <= tie:
        k -= 1
    return k


def split_two_site(theta, direction: str, cutoff: float, chi_max: int, tie_rel: float):
    """SVD of theta as (Dl d1) x (d2 Dr); direction 'lr' gives A_j = U,
    A_(j+1) = S V^T; 'rl' gives A_j = U S, A_(j+1) = V^T."""
    Dl, d1, d2, Dr = theta.shape
    M = theta.reshape(Dl * d1, d2 * Dr)
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    k = truncation_rank(s, cutoff, chi_max, tie_rel)
    total = float(np.sum(s * s))
    disc = float(np.sum(s[k:] ** 2)) / total if total > 0 else 0.0
    if direction == "lr":
        A1 = U[:, :k].reshape(Dl, d1, k)
        A2 = (s[:k, None] * Vt[:k]).reshape(k, d2, Dr)
    elif direction == "rl":
        A1 = (U[:, :k] * s[None, :k]).reshape(Dl, d1, k)
        A2 = Vt[:k].reshape(k, d2, Dr)
    else:
        raise ValueError(direction)
    return np.ascontiguousarray(A1), np.ascontiguousarray(A2), {"k": k, "disc": disc, "sigma": s}


# ----------------------------------------------------------------------------
# The implicit step
# ----------------------------------------------------------------------------

@dataclass
class StepOptions:
    scheme: str = "trap"           # "trap" or "be"
    shift_mode: str = "track"      # "fixed" or "track"
    shift: float = 0.0
    chi_max: int = 64
    cutoff: float = 0.0
    tie_rel: float = 1e-13
    krylov_dim: int = 10
    max_cycles: int = 1
    tol_loc: float = 0.0
    nsweeps: int = 1
    init_guess: str = "b"          # "b" (Appendix B) or "psi"


@dataclass
class StepReport:
    tau: float = 0.0
    h: float = 0.0
    shift: float = 0.0
    energy: float = 0.0
    norm_before: float = 0.0
    max_chi: int = 0
    max_disc: float = 0.0
    sum_disc: float = 0.0
    max_res_rel: float = 0.0
    matvecs: int = 0
    extra: dict = field(default_factory=dict)


def imag_step(psi, W, h: float, opts: StepOptions):
    """One implicit step (I + h (H - s)) x = b; returns (psi_new, report)."""
    L = len(psi)
    if opts.shift_mode == "track":
        s = expectation(psi, W)
    else:
        s = opts.shift
    x = [a.copy() for a in psi]
    ones3 = np.ones((1, 1, 1))
    LH = [None] * (L + 1)
    LHp = [None] * (L + 1)
    LO = [None] * (L + 1)
    RH = [None] * (L + 1)
    RHp = [None] * (L + 1)
    RO = [None] * (L + 1)
    LH[0] = ones3
    LHp[0] = ones3
    LO[0] = np.ones((1, 1))
    RH[L] = ones3
    for b in range(L - 1, 1, -1):
        RH[b] = env_right_h(RH[b + 1], x[b], W[b], x[b])
    for b in range(2, L + 1):
        RHp[b] = RH[b]                          # x = psi on sites b..L-1
        RO[b] = np.eye(RH[b].shape[0])          # <x|psi> = identity there
    rep = StepReport(h=h, shift=s)
    a_coef = 1.0 - h * s

    def solve_block(i, first):
        theta_psi = two_site(psi[i], psi[i + 1])
        ov = overlap_project(LO[i], RO[i + 2], theta_psi)
        if opts.scheme == "be":
            b = ov
        elif opts.scheme == "trap":
            b = (1.0 + h * s) * ov - h * heff_apply(LHp[i], W[i], W[i + 1], RHp[i + 2], theta_psi)
        else:
            raise ValueError(opts.scheme)
        if opts.init_guess == "b" and first:
            theta0 = b.copy()
        elif opts.init_guess in ("b", "psi"):
            theta0 = two_site(x[i], x[i + 1])
        else:
            raise ValueError(opts.init_guess)
        op = lambda v: a_coef * v + h * heff_apply(LH[i], W[i], W[i + 1], RH[i + 2], v)
        theta, info = gmres(op, b, theta0, opts.krylov_dim, opts.max_cycles, opts.tol_loc)
        rep.matvecs += info["matvecs"]
        rep.max_res_rel = max(rep.max_res_rel, info["res_rel"])
        return theta

    for sweep in range(opts.nsweeps):
        for i in range(0, L - 1):
            theta = solve_block(i, sweep == 0 and i == 0)
            x[i], x[i + 1], sp = split_two_site(theta, "lr", opts.cutoff, opts.chi_max, opts.tie_rel)
            rep.max_disc = max(rep.max_disc, sp["disc"])
            rep.sum_disc += sp["disc"]
            if i < L - 2:
                LH[i + 1] = env_left_h(LH[i], x[i], W[i], x[i])
                LHp[i + 1] = env_left_h(LHp[i], x[i], W[i], psi[i])
                LO[i + 1] = env_left_o(LO[i], x[i], psi[i])
        for i in range(L - 2, -1, -1):
            theta = solve_block(i, False)
            x[i], x[i + 1], sp = split_two_site(theta, "rl", opts.cutoff, opts.chi_max, opts.tie_rel)
            rep.max_disc = max(rep.max_disc, sp["disc"])
            rep.sum_disc += sp["disc"]
            if i > 0:
                RH[i + 1] = env_right_h(RH[i + 2], x[i + 1], W[i + 1], x[i + 1])
                RHp[i + 1] = env_right_h(RHp[i + 2], x[i + 1], W[i + 1], psi[i + 1])
                RO[i + 1] = env_right_o(RO[i + 2], x[i + 1], psi[i + 1])
    nrm = float(np.linalg.norm(x[0]))
    x[0] = x[0] / nrm
    rep.norm_before = nrm
    rep.energy = expectation(x, W)
    rep.max_chi = max(bond_dims(x))
    return x, rep


def evolve_grid(psi, W, grid, opts: StepOptions):
    """Step along an explicit grid; h = dtau / 2 (trapezoid) or dtau (backward
    Euler).  Returns (psi, reports)."""
    reps = []
    for k in range(1, len(grid)):
        dtau = float(grid[k] - grid[k - 1])
        h = dtau / 2 if opts.scheme == "trap" else dtau
        psi, rep = imag_step(psi, W, h, opts)
        rep.tau = float(grid[k])
        reps.append(rep)
    return psi, reps


def evolve_loggrid(psi, W, tau0: float, tau1: float, ratio: float, opts: StepOptions):
    from .ed import loggrid
    return evolve_grid(psi, W, loggrid(tau0, tau1, ratio), opts)

"""The right-hand side as an MPS (Appendix B: the operator is applied by the
"density matrix" algorithm for MPO-MPS products, and the right-hand side
b = (I - h (H - s)) psi, itself an MPS, is the initial guess of the solve).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The density-matrix product phi = O psi, right to left:
  1. left environments of <phi|phi> without truncation,
       F_0 = 1,  F_j[a', w', a, w] = sum F_(j-1) psi_j* O_j* O_j psi_j
     (primed indices: the bra copy);
  2. at the last site, T_L[a, w, s] = sum_t psi_L[a, t] O_L[w, s, t]; its
     reduced density matrix rho[s', s] = sum T_L*[a', w', s'] F_(L-1)[a', w',
     a, w] T_L[a, w, s]; the eigenvectors of the k largest eigenvalues (the
     truncation rule of the splits on sigma = sqrt(eigenvalue)) are the
     rows of b_L[k, s];  C_L[a, w, k] = sum_s T_L[a, w, s] b_L[k, s];
  3. at site j < L, T_j[a, w, s, k] = sum psi_j[a, t, a2] O_j[w, w2, s, t]
     C_(j+1)[a2, w2, k], rho over (s k) from F_(j-1) in the same way, b_j the
     leading eigenvectors as rows [k_(j-1), (s, k)], C_j = T_j b_j^T;
  4. at site 1 the rest is kept whole: b_1[1, s, k] = T_1[1, 1, s, k].
The result is right-orthonormal from site 2 on with the norm of phi in site
1; with no truncation it is O psi exactly.

Readings: the eigen-decomposition keeps eigenvectors by the same discarded
weight rule as the splits (the eigenvalues are the squared singular values of
phi at that bond, so they are the weights), at most min(prod d left, prod d
right, chi_max) of them, the largest rank the bond can have (as for every MPS
here); the operator of the trapezoid
right-hand side, (1 + h s) I - h H, is the direct sum of H's MPO scaled by
-h and the identity scaled by (1 + h s) (bond dimension w + 1).

The step with this right-hand side: s from psi (tracking) or fixed; b by the
density-matrix product with the step's chi_max / cutoff; then the linear solve
(I + h (H - s)) x = b of ``mps.imag_step`` in its backward-Euler form with psi
replaced by b (x starts as b, b projected into x's basis through the <x|b>
environments) and the shift held at s.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from . import mps as omps


def rhs_mpo(W, h: float, s: float):
    """MPO of (1 + h s) I - h H: H's MPO with its first site scaled by -h, in
    direct sum with the identity scaled by (1 + h s)."""
    L = len(W)
    out = []
    for j, Wj in enumerate(W):
        wl, wr, d, _ = Wj.shape
        first, last = j == 0, j == L - 1
        if first and last:
            T = (-h * Wj[0, 0] + (1.0 + h * s) * np.eye(d)).reshape(1, 1, d, d)
        elif first:
            T = np.zeros((1, wr + 1, d, d))
            T[0, :wr] = -h * Wj[0]
            T[0, wr] = (1.0 + h * s) * np.eye(d)
        elif last:
            T = np.zeros((wl + 1, 1, d, d))
            T[:wl, 0] = Wj[:, 0]
            T[wl, 0] = np.eye(d)
        else:
            T = np.zeros((wl + 1, wr + 1, d, d))
            T[:wl, :wr] = Wj
            T[wl, wr] = np.eye(d)
        out.append(T)
    return out


def _eig_keep(rho, cutoff: float, chi_max: int, tie_rel: float):
    """Leading eigenvectors of a symmetric positive semi-definite matrix by
    the splits' truncation rule on sqrt(eigenvalue); returns (V [n, k],
    eigenvalues descending, k)."""
    lam, vec = np.linalg.eigh((rho + rho.T) / 2)
    order = np.argsort(lam)[::-1]
    lam = np.clip(lam[order], 0.0, None)
    vec = vec[:, order]
    k = omps.truncation_rank(np.sqrt(lam), cutoff, chi_max, tie_rel)
    return vec[:, :k], lam, k


def density_matrix_apply(O, psi, chi_max: int, cutoff: float, tie_rel: float):
    """phi = O psi by the density-matrix algorithm; returns (b, info) with b
    right-orthonormal from site 2 on and info["disc"] the largest discarded
    weight fraction."""
    L = len(psi)
    F = [None] * L
    F[0] = np.ones((1, 1, 1, 1))
    for j in range(L - 1):
        # F_j[a', w', a, w] = F_(j-1)[c', v', c, v] psi*[c', t', a'] O*[v', w', s, t'] O[v, w, s, t] psi[c, t, a]
        X = np.tensordot(F[j], psi[j], axes=([2], [0]))                 # [c', v', v, t, a]
        X = np.tensordot(X, O[j], axes=([2, 3], [0, 3]))                # [c', v', a, w, s]
        X = np.tensordot(X, O[j], axes=([1, 4], [0, 2]))                # [c', a, w, w', t']
        X = np.tensordot(X, psi[j], axes=([0, 4], [0, 1]))              # [a, w, w', a']
        F[j + 1] = np.ascontiguousarray(np.transpose(X, (3, 2, 0, 1)))  # [a', w', a, w]
    caps = omps.full_dims(L, [a.shape[1] for a in psi], chi_max)
    b = [None] * L
    info = {"disc": 0.0, "k": [], "lam": []}
    C = np.ones((1, 1, 1))                                              # [a, w, k] at the right boundary
    for j in range(L - 1, -1, -1):
        # T[a, w, s, k] = psi[a, t, a2] O[w, w2, s, t] C[a2, w2, k]
        T = np.tensordot(psi[j], C, axes=([2], [0]))                    # [a, t, w2, k]
        T = np.tensordot(T, O[j], axes=([1, 2], [3, 1]))                # [a, k, w, s]
        T = np.ascontiguousarray(np.transpose(T, (0, 2, 3, 1)))         # [a, w, s, k]
        Da, w, d, k = T.shape
        if j == 0:
            b[0] = T.reshape(1, d, k)
            break
        Tm = T.reshape(Da * w, d * k)
        Fm = F[j].reshape(Da * w, Da * w)                               # [(a' w'), (a w)]
        rho = Tm.T @ Fm @ Tm                                            # [(s' k'), (s k)]
        V, lam, kk = _eig_keep(rho, cutoff, min(chi_max, caps[j]), tie_rel)
        total = float(lam.sum())
        info["disc"] = max(info["disc"], float(lam[kk:].sum()) / total if total > 0 else 0.0)
        info["k"].append(kk)
        info["lam"].append(lam)
        b[j] = np.ascontiguousarray(V.T.reshape(kk, d, k))
        C = (Tm @ V).reshape(Da, w, kk)
    return b, info


def trap_step_mps_rhs(psi, W, h: float, opts):
    """One trapezoid step with b = (I - h (H - s)) psi formed as an MPS by the
    density-matrix product and used as the initial guess.  Returns
    (psi_new, report); report.extra["rhs_disc"] is the product's largest
    discarded weight."""
    s = omps.expectation(psi, W) if opts.shift_mode == "track" else opts.shift
    b, info = density_matrix_apply(rhs_mpo(W, h, s), psi, opts.chi_max, opts.cutoff, opts.tie_rel)
    x, rep = omps.imag_step(b, W, h, replace(opts, scheme="be", shift_mode="fixed", shift=s))
    rep.shift = s
    rep.extra["rhs_disc"] = info["disc"]
    return x, rep


def evolve_grid_mps_rhs(psi, W, grid, opts):
    reps = []
    for k in range(1, len(grid)):
        psi, rep = trap_step_mps_rhs(psi, W, float(grid[k] - grid[k - 1]) / 2, opts)
        rep.tau = float(grid[k])
        reps.append(rep)
    return psi, reps

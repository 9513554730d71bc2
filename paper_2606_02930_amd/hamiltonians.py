"""Host-side MPO construction for the two Hamiltonians of the paper.

The paper generates its MPOs with an operator-sum system and compresses them
to machine precision (Appendix B).  Both models here have exact finite-state
forms, assembled from a table of (row, column) -> local operator entries per
site.  Tensor layout, as ``ite_mpo_load`` expects: W[wl][wr][out][in].

* ``heisenberg``: H = J sum_j [Jz S^z_j S^z_(j+1) + (S^+_j S^-_(j+1) + h.c.)/2]
  on an open chain (Heisenberg chain section), bond dimension 5.
* ``anderson_star``: the single-impurity Anderson model in star geometry
  (Anderson impurity model section), impurity first, spinful sites with the
  local basis (|0>, |up>, |dn>, |up dn> = c+_up c+_dn |0>) and Jordan-Wigner
  strings F = (-1)^n, bond dimension 6.
"""
from __future__ import annotations

import numpy as np


def _assemble(entries: dict, w_left: int, w_right: int, d: int) -> np.ndarray:
    W = np.zeros((w_left, w_right, d, d))
    for (r, c), op in entries.items():
        W[r, c] += op
    return W


def _chain(L: int, d: int, bulk_entries, w: int, start: int, done: int):
    """Open-chain MPO from per-site entry tables; the first site keeps the row
    `start`, the last site keeps the column `done`."""
    out = []
    for i in range(L):
        W = _assemble(bulk_entries(i), w, w, d)
        if i == 0:
            W = W[start:start + 1]
        if i == L - 1:
            W = W[:, done:done + 1]
        out.append(np.ascontiguousarray(W))
    return out


def heisenberg(L: int, J: float = 1.0, Jz: float = 1.0) -> list[np.ndarray]:
    half = 0.5
    sz = np.diag([half, -half])
    sp = np.zeros((2, 2)); sp[0, 1] = 1.0      # |up><dn|
    sm = sp.T.copy()
    one = np.eye(2)
    # states: 0 'nothing yet', 1..3 waiting for the partner of S-, S+, Sz, 4 'complete'
    def entries(_i):
        return {
            (0, 0): one,
            (0, 1): J * half * sp,      # S+ ... waits for S-
            (0, 2): J * half * sm,      # S- ... waits for S+
            (0, 3): J * Jz * sz,
            (1, 4): sm,
            (2, 4): sp,
            (3, 4): sz,
            (4, 4): one,
        }
    return _chain(L, 2, entries, 5, start=0, done=4)


def anderson_star(U: float, eps_d: float, eps_b, V) -> list[np.ndarray]:
    eps_b = np.asarray(eps_b, dtype=float)
    V = np.asarray(V, dtype=float)
    n_sites = len(eps_b) + 1
    # local operators in (|0>, |up>, |dn>, |up dn>)
    occ_up = np.array([0, 1, 0, 1], dtype=float)
    occ_dn = np.array([0, 0, 1, 1], dtype=float)
    a_up = np.zeros((4, 4)); a_up[0, 1] = 1.0; a_up[2, 3] = 1.0
    a_dn = np.zeros((4, 4)); a_dn[0, 2] = 1.0; a_dn[1, 3] = -1.0
    parity = np.diag((-1.0) ** (occ_up + occ_dn))
    n_tot = np.diag(occ_up + occ_dn)
    double = np.diag(occ_up * occ_dn)
    one = np.eye(4)
    # hopping channels c = 1..4: (impurity operator, bath operator)
    #   d+_s c_ks = (a+_s F)_imp F..F (a_s)_k ;  c+_ks d_s = (F a_s)_imp F..F (a+_s)_k
    channels = [
        (a_up.T @ parity, a_up),
        (parity @ a_up, a_up.T),
        (a_dn.T @ parity, a_dn),
        (parity @ a_dn, a_dn.T),
    ]
    START, DONE = 0, 5

    def entries(i):
        e = {(START, START): one, (DONE, DONE): one}
        if i == 0:
            e[(START, DONE)] = eps_d * n_tot + U * double
            for c, (imp_op, _) in enumerate(channels):
                e[(START, 1 + c)] = imp_op
        else:
            e[(START, DONE)] = eps_b[i - 1] * n_tot
            for c, (_, bath_op) in enumerate(channels):
                e[(1 + c, 1 + c)] = parity
                e[(1 + c, DONE)] = V[i - 1] * bath_op
        return e
    return _chain(n_sites, 4, entries, 6, start=START, done=DONE)

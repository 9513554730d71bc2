"""MPO level of the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Tensor convention: W_i[wl, wr, s_out, s_in]; W_1 has wl = 1 and W_L has wr = 1.
The operator is H = sum over bond indices of W_1 W_2 ... W_L.

The paper builds its MPOs with an OpSum system and compresses them to machine
precision (Appendix B).  Both Hamiltonians used here have exact low-rank
finite-state forms, written out below directly from the Hamiltonian
definitions (Heisenberg chain section; Anderson impurity model section).

Pins (``tests/test_oracle_mpo.py``): ``mpo_to_dense`` of each builder equals the
Kronecker-product Hamiltonian of ``oracle.ed`` to 1e-13 (Heisenberg L <= 8,
XXZ, impurity model with up to 4 bath sites).
"""
from __future__ import annotations

import numpy as np

from .ed import SZ, SP, SM


def heisenberg_mpo(L: int, J: float = 1.0, Jz: float = 1.0) -> list[np.ndarray]:
    """Open XXZ chain, MPO bond dimension 5.

    Bond states: 0 = 'complete' (all terms placed, identity follows),
    1..3 = an S^+, S^-, S^z placed on the previous site waiting for its
    partner, 4 = 'nothing placed yet'.
    """
    d, w = 2, 5
    bulk = np.zeros((w, w, d, d))
    bulk[0, 0] = np.eye(d)
    bulk[1, 0] = SP
    bulk[2, 0] = SM
    bulk[3, 0] = SZ
    bulk[4, 1] = 0.5 * J * SM
    bulk[4, 2] = 0.5 * J * SP
    bulk[4, 3] = J * Jz * SZ
    bulk[4, 4] = np.eye(d)
    out = []
    for i in range(L):
        W = bulk.copy()
        if i == 0:
            W = W[4:5, :, :, :]
        if i == L - 1:
            W = W[:, 0:1, :, :]
        out.append(np.ascontiguousarray(W))
    return out


# Per-site fermion operators in the basis (|0>, |up>, |dn>, |up dn>) with
# |up dn> = c+_up c+_dn |0> (up before dn in the Jordan-Wigner order).
def _site_fermion_ops():
    cu = np.zeros((4, 4))
    cu[0, 1] = 1.0      # c_up |up>    = |0>
    cu[2, 3] = 1.0      # c_up |up dn> = |dn>
    cd = np.zeros((4, 4))
    cd[0, 2] = 1.0      # c_dn |dn>    = |0>
    cd[1, 3] = -1.0     # c_dn |up dn> = -|up>  (passes c+_up)
    F = np.diag([1.0, -1.0, -1.0, 1.0])
    nu = cu.T @ cu
    nd = cd.T @ cd
    return cu, cd, F, nu, nd


def aim_mpo(U: float, eps_d: float, eps_b, V) -> list[np.ndarray]:
    """Star-geometry Anderson impurity model, impurity on site 1 followed by the
    bath sites, MPO bond dimension 6.

    With the string F = (-1)^n:
      d+_s c_(k s) = (c+_s F)_imp  F ... F  (c_s)_k
      c+_(k s) d_s = (F c_s)_imp   F ... F  (c+_s)_k
    Bond states: 0 = complete, 1..4 = one of the four impurity operators above
    carried through the string, 5 = nothing placed yet.
    """
    eps_b = np.asarray(eps_b, dtype=float)
    V = np.asarray(V, dtype=float)
    cu, cd, F, nu, nd = _site_fermion_ops()
    I4 = np.eye(4)
    n_sites = len(eps_b) + 1
    w = 6
    out = []
    # impurity operators opening the four channels, and their partners
    openers = [cu.T @ F, F @ cu, cd.T @ F, F @ cd]
    closers = [cu, cu.T, cd, cd.T]
    for i in range(n_sites):
        W = np.zeros((w, w, 4, 4))
        W[0, 0] = I4
        W[5, 5] = I4
        if i == 0:
            W[5, 0] = eps_d * (nu + nd) + U * nu @ nd
            for c in range(4):
                W[5, 1 + c] = openers[c]
        else:
            W[5, 0] = eps_b[i - 1] * (nu + nd)
            for c in range(4):
                W[1 + c, 1 + c] = F
                W[1 + c, 0] = V[i - 1] * closers[c]
        if i == 0:
            W = W[5:6]
        if i == n_sites - 1:
            W = W[:, 0:1]
        out.append(np.ascontiguousarray(W))
    return out


def mpo_to_dense(Ws: list[np.ndarray]) -> np.ndarray:
    """Contract an MPO to the dense operator (site 1 most significant)."""
    T = Ws[0][0]                        # [wr, so, si]
    T = T.reshape(T.shape[0], T.shape[1], T.shape[2])
    dims_out = T.shape[1]
    acc = np.transpose(T, (0, 1, 2))   # [w, O, I]
    for W in Ws[1:]:
        # acc[w, O, I] * W[w, v, o, i] -> [v, O o, I i]
        nw, O, I = acc.shape
        _, nv, do, di = W.shape
        new = np.einsum("wOI,wvoi->vOoIi", acc, W)
        acc = new.reshape(nv, O * do, I * di)
        dims_out = O * do
    assert acc.shape[0] == 1
    return acc[0]


def mpo_bond_dims(Ws) -> list[int]:
    return [Ws[0].shape[0]] + [W.shape[1] for W in Ws]

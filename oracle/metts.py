"""METTS chains and one-site expectation values (Appendix D).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Appendix D computes thermal expectation values of the impurity model with
minimally entangled typical thermal states: from a product state |i>, form
|psi_i> proportional to exp(-beta H / 2)|i>, measure the observable in it,
collapse |psi_i> to a product state |j> drawn with probability
|<j|psi_i>|^2, and repeat from |j>; the thermal average is the plain mean of
<psi_i|O|psi_i> over the chain.  The chains start from a product state
sampled from the ground state, and the observable is the impurity double
occupancy n_(d,up) n_(d,dn).

* ``site_expectation(psi, site, op)`` -- <psi|O_site|psi> / <psi|psi> for a
  one-site operator (op[s_out, s_in]), by transfer matrices over the whole
  chain (no canonical form assumed).
* ``basis_state(config, d)`` -- the product state |s_1 .. s_L> as an MPS of
  unit bond dimension.
* ``mps_chain`` -- the chain with the MPS evolution of ``oracle.mps`` on the
  geometric grid tau0 -> beta / 2 and the collapse of ``oracle.sampling``
  (one uniform per site and METTS, supplied by the caller); returns the
  seeding configuration, the energy and <O> of every METTS.
* ``dense_chain`` -- the same chain on dense vectors (Hamiltonian in the
  per-site product basis) with the Born-rule collapse, and either the exact
  evolution exp(-beta H / 2) (``exact_metts``, spectral decomposition) or the
  full-vector trapezoid steps on the same grid (``trapezoid_metts``), for the
  pins.
* ``thermal_average(H, O, beta)`` -- Tr(exp(-beta H) O) / Tr(exp(-beta H)).
* ``metts_transition(H, beta)`` -- T[i, j] = |<j|psi_i>|^2 with the exact
  normalised METTS of every product state i.

Pins (``tests/test_oracle_metts.py``): ``site_expectation`` equals the dense
expectation value; with the exact evolution the distribution
p(i) ~ <i|exp(-beta H)|i> is stationary under T and the p-weighted mean of
<psi_i|O|psi_i> equals the thermal average to rounding (the identity that
makes METTS unbiased); a seeded dense chain with exact evolution reproduces the thermal average
within its statistical error; the MPS chain with complete bonds and
converged local solves reproduces the dense trapezoid chain: the same
configurations, energies and observables to 1e-10.
"""
from __future__ import annotations

import numpy as np

from . import mps as omps
from . import sampling as osmp


def site_expectation(psi, site: int, op) -> float:
    """<psi|O_site|psi> / <psi|psi> by transfer matrices from the left."""
    op = np.asarray(op, dtype=float)
    E = np.ones((1, 1))
    N = np.ones((1, 1))
    for j, a in enumerate(psi):
        ta = np.tensordot(E, a, axes=([1], [0]))                     # [i, s, b]
        if j == site:
            ta = np.einsum("ps,isb->ipb", op, ta)
        E = np.tensordot(a, ta, axes=([0, 1], [0, 1]))               # [j, b]
        tn = np.tensordot(N, a, axes=([1], [0]))
        N = np.tensordot(a, tn, axes=([0, 1], [0, 1]))
    return float(E[0, 0]) / float(N[0, 0])


def basis_state(config, d: int):
    out = []
    for s in config:
        a = np.zeros((1, d, 1))
        a[0, int(s), 0] = 1.0
        out.append(a)
    return out


def mps_chain(W, start, d: int, beta: float, tau0: float, ratio: float, opts, site: int, op, uniforms):
    """METTS chain with the MPS evolution.  uniforms [n][L]: row k collapses
    METTS k.  Returns (configs [n][L] seeding each METTS, energies [n],
    observables [n])."""
    n, L = uniforms.shape
    cfg = np.array(start, dtype=np.int64)
    configs = np.zeros((n, L), dtype=np.int64)
    energies = np.zeros(n)
    obs = np.zeros(n)
    for k in range(n):
        configs[k] = cfg
        psi, reps = omps.evolve_loggrid(basis_state(cfg, d), W, tau0, beta / 2, ratio, opts)
        energies[k] = reps[-1].energy
        obs[k] = site_expectation(psi, site, op)
        nxt, _ = osmp.sample(psi, uniforms[k].reshape(L, 1))
        cfg = nxt[0]
    return configs, energies, obs


def _index(config, d: int) -> int:
    k = 0
    for s in config:
        k = k * d + int(s)
    return k


def _config(index: int, L: int, d: int):
    out = []
    for _ in range(L):
        out.append(index % d)
        index //= d
    return out[::-1]


def exact_metts(H, beta: float, i: int):
    """Normalised exp(-beta H / 2)|i> for the product-basis index i."""
    ev, vec = np.linalg.eigh(H)
    v = vec @ (np.exp(-0.5 * beta * (ev - ev[0])) * vec[i, :])
    return v / np.linalg.norm(v)


def trapezoid_metts(H, tau0: float, beta: float, ratio: float):
    """evolve(i) for ``dense_chain``: the full-vector trapezoid steps with the
    shift tracking the energy (Appendix D's rule) on the geometric grid
    tau0 -> beta / 2 from the product-basis state i, normalised."""
    from .ed import evolve_dense, loggrid
    grid = loggrid(tau0, beta / 2, ratio)

    def evolve(i):
        e = np.zeros(H.shape[0])
        e[i] = 1.0
        states, _, _, _ = evolve_dense(H, e, grid, "trap", "track")
        return states[-1]
    return evolve


def dense_chain(H, O, start, L: int, d: int, evolve, uniforms):
    """The chain on dense vectors (small L): evolve(i) gives the normalised
    METTS of product-basis index i (``exact_metts`` or ``trapezoid_metts``);
    the collapse uses uniforms [n][L] as ``sampling.sample`` does, drawing
    s_i from its conditional probability given s_1 .. s_(i-1)."""
    n = uniforms.shape[0]
    cfg = list(start)
    configs = np.zeros((n, L), dtype=np.int64)
    energies = np.zeros(n)
    obs = np.zeros(n)
    for k in range(n):
        configs[k] = cfg
        v = evolve(_index(cfg, d))
        energies[k] = float(v @ H @ v)
        obs[k] = float(v @ O @ v)
        p = (v * v).reshape([d] * L)
        nxt = []
        for i in range(L):
            marg = p.reshape(d, -1).sum(axis=1)          # P(s_i | earlier choices), unnormalised
            tot = float(marg.sum())
            thr = uniforms[k, i] * tot
            pick, cum = -1, 0.0
            for s in range(d):
                cum += marg[s]
                if pick < 0 and cum > thr and marg[s] > 0.0:
                    pick = s
            if pick < 0:
                pick = int(np.nonzero(marg > 0.0)[0][-1])
            nxt.append(pick)
            p = p[pick]
        cfg = nxt
    return configs, energies, obs


def thermal_average(H, O, beta: float, states=None) -> float:
    """Tr(exp(-beta H) O) / Tr(exp(-beta H)); with ``states`` (product-basis
    indices spanning a sector that H and O leave invariant) the trace runs
    over that sector only.  A chain whose collapse conserves quantum numbers
    (the computational basis conserves particle number and S^z of the
    impurity model) samples the sector of its start state."""
    ev, vec = np.linalg.eigh(H)
    w = np.exp(-beta * (ev - ev[0]))
    rho = (vec * w) @ vec.T
    if states is None:
        states = np.arange(H.shape[0])
    states = np.asarray(states)
    return float(np.trace((rho @ O)[np.ix_(states, states)]) / np.trace(rho[np.ix_(states, states)]))


def sector(config, L: int, d: int, charges):
    """Product-basis indices with the same total charges as ``config``;
    charges[q][s] is charge q of local state s."""
    want = [sum(ch[int(s)] for s in config) for ch in charges]
    out = []
    for i in range(d ** L):
        c = _config(i, L, d)
        if all(sum(ch[s] for s in c) == wv for ch, wv in zip(charges, want)):
            out.append(i)
    return out


def metts_transition(H, beta: float):
    """T[i, j] = |<j|psi_i>|^2 (rows sum to one)."""
    dim = H.shape[0]
    T = np.zeros((dim, dim))
    for i in range(dim):
        v = exact_metts(H, beta, i)
        T[i] = v * v
    return T

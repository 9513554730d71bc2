"""Full state-vector level of the oracle (exact diagonalisation).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Contents and what pins each one (tests in ``tests/test_oracle_ed.py``):

* ``heisenberg_dense``  -- H = J sum_j [Jz S^z_j S^z_(j+1) + (S^+_j S^-_(j+1) +
  h.c.)/2] on an open chain (Heisenberg chain section).  Pinned by the two-site
  singlet energy -3/4 and, at Jz = 0, by the free-fermion closed form
  ``xx_chain_e0``.
* ``aim_dense``         -- single-impurity Anderson model (Anderson impurity
  model section), built from Jordan-Wigner mode operators.  Pinned by the
  U = 0 single-particle spectrum and the V = 0 atomic limit.
* ``exact_evolve``      -- psi(tau) = sum_i exp(-E_i tau) v_i <v_i|psi0>
  (Method, Eq. 1), with the spectrum shifted so that E_0 = 0.
* ``implicit_step``     -- one step of (I + h (H - s)) x = b with b = psi
  (backward Euler) or b = (I - h (H - s)) psi (implicit trapezoid, Method Eq. 4
  with h = dtau / 2).  Pinned by the eigenbasis step factors of Appendix A.
* ``loggrid`` / ``panel_grid`` -- geometric grid, and the panel grid with
  endpoints {0, tau_max / 2^(P-j)} and n uniform steps per panel (Method).
* ``trap_local_error``  -- E(mu) = exp(-3 mu / 2) (mu cosh(mu/2) - 2 sinh(mu/2))
  (Appendix A).  Pinned by the defining integral and the quoted maximum.
* ``forward_euler_step`` / ``heun_step`` -- explicit negative controls
  (Appendix A; Heisenberg chain section).
"""
from __future__ import annotations

import math

import numpy as np

# Spin-1/2 operators in the basis (|up>, |down>) = (index 0, index 1).
SZ = np.array([[0.5, 0.0], [0.0, -0.5]])
SP = np.array([[0.0, 1.0], [0.0, 0.0]])   # S^+ |down> = |up>
SM = SP.T.copy()                           # S^- |up> = |down>
I2 = np.eye(2)


def site_operator(op: np.ndarray, i: int, L: int) -> np.ndarray:
    """The operator ``op`` acting on site i (0-based) of an L-site chain of
    equal local dimension, as a dense matrix (Kronecker product, site 0 is the
    most significant index)."""
    d = op.shape[0]
    out = np.ones((1, 1))
    for j in range(L):
        out = np.kron(out, op if j == i else np.eye(d))
    return out


def heisenberg_dense(L: int, J: float = 1.0, Jz: float = 1.0) -> np.ndarray:
    """Dense open-chain XXZ Hamiltonian; Jz = 1 is the Heisenberg chain."""
    dim = 2 ** L
    H = np.zeros((dim, dim))
    for j in range(L - 1):
        H += J * Jz * site_operator(SZ, j, L) @ site_operator(SZ, j + 1, L)
        H += 0.5 * J * site_operator(SP, j, L) @ site_operator(SM, j + 1, L)
        H += 0.5 * J * site_operator(SM, j, L) @ site_operator(SP, j + 1, L)
    return H


def xx_chain_e0(L: int, J: float = 1.0) -> float:
    """Ground-state energy of the open XX chain (Jz = 0).

    Jordan-Wigner maps it to free fermions with hopping J/2 and single-particle
    energies J cos(k pi / (L + 1)), k = 1..L; the ground state fills all
    negative levels.
    """
    return float(sum(min(0.0, J * math.cos(k * math.pi / (L + 1))) for k in range(1, L + 1)))


# ----------------------------------------------------------------------------
# Fermions (Jordan-Wigner on spin-orbital modes)
# ----------------------------------------------------------------------------

def jw_annihilators(n_modes: int) -> list[np.ndarray]:
    """Annihilation operators c_m = Z x ... x Z x a x 1 x ... (mode m, 0-based),
    with a = |0><1| on the occupation basis (|0>, |1>) and Z = diag(1, -1)."""
    a = np.array([[0.0, 1.0], [0.0, 0.0]])
    Z = np.diag([1.0, -1.0])
    out = []
    for m in range(n_modes):
        op = np.ones((1, 1))
        for k in range(n_modes):
            op = np.kron(op, Z if k < m else (a if k == m else I2))
        out.append(op)
    return out


def aim_dense(U: float, eps_d: float, eps_b, V) -> np.ndarray:
    """Anderson impurity Hamiltonian on 2 (N_B + 1) Jordan-Wigner modes.

    H = eps_d n_d + U n_(d,up) n_(d,dn) + sum_(j,s) eps_j c+_(js) c_(js)
        + sum_(j,s) V_j (d+_s c_(js) + c+_(js) d_s).

    Mode order: imp-up, imp-dn, bath1-up, bath1-dn, ...  The matrix is in the
    Kronecker occupation basis; ``aim_basis_permutation`` maps it to the
    per-site basis (|0>, |up>, |dn>, |up dn>) used by the MPO.
    """
    eps_b = np.asarray(eps_b, dtype=float)
    V = np.asarray(V, dtype=float)
    nb = len(eps_b)
    c = jw_annihilators(2 * (nb + 1))
    n = [ci.T @ ci for ci in c]
    H = eps_d * (n[0] + n[1]) + U * n[0] @ n[1]
    for j in range(nb):
        for s in range(2):
            m = 2 * (j + 1) + s
            H = H + eps_b[j] * n[m]
            H = H + V[j] * (c[s].T @ c[m] + c[m].T @ c[s])
    return H


def aim_basis_permutation(n_sites: int) -> np.ndarray:
    """Index map from the per-site MPO basis to the Kronecker mode basis.

    Per site, MPO index (0: |0>, 1: |up>, 2: |dn>, 3: |up dn>) corresponds to
    occupations (n_up, n_dn) = (0,0), (1,0), (0,1), (1,1), whose Kronecker
    index is 2 n_up + n_dn.  Returns perm with H_mpo = H_kron[perm][:, perm].
    """
    local = [0, 2, 1, 3]
    perm = np.zeros(4 ** n_sites, dtype=np.int64)
    for idx in range(4 ** n_sites):
        digits = []
        r = idx
        for _ in range(n_sites):
            digits.append(r % 4)
            r //= 4
        digits = digits[::-1]
        k = 0
        for dgt in digits:
            k = 4 * k + local[dgt]
        perm[idx] = k
    return perm


def free_fermion_aim_e0(eps_d: float, eps_b, V) -> float:
    """U = 0 ground-state energy: twice the sum of the negative eigenvalues of
    the (N_B + 1) x (N_B + 1) single-particle matrix (two spin species)."""
    eps_b = np.asarray(eps_b, dtype=float)
    nb = len(eps_b)
    h = np.zeros((nb + 1, nb + 1))
    h[0, 0] = eps_d
    h[1:, 1:] = np.diag(eps_b)
    h[0, 1:] = V
    h[1:, 0] = V
    ev = np.linalg.eigvalsh(h)
    return float(2.0 * ev[ev < 0].sum())


# ----------------------------------------------------------------------------
# Exact evolution and full-vector implicit steps
# ----------------------------------------------------------------------------

def ground_state(H: np.ndarray) -> tuple[float, np.ndarray]:
    ev, vec = np.linalg.eigh(H)
    return float(ev[0]), vec[:, 0]


def exact_evolve(H: np.ndarray, psi0: np.ndarray, tau: float) -> np.ndarray:
    """psi(tau) = sum_i exp(-(E_i - E_0) tau) v_i <v_i|psi0> (Method, Eq. 1),
    the spectrum shifted so that the ground-state energy is zero."""
    ev, vec = np.linalg.eigh(H)
    coef = vec.T @ psi0
    return vec @ (np.exp(-(ev - ev[0]) * tau) * coef)


def step_factor(lam, h: float, s: float, scheme: str):
    """Amplification of an eigencomponent with eigenvalue lam in one implicit
    step of (I + h (H - s)) x = b: (1 - h (lam - s)) / (1 + h (lam - s)) for the
    trapezoid rule (Appendix A, stability factor with dtau = 2 h), and
    1 / (1 + h (lam - s)) for backward Euler."""
    z = h * (np.asarray(lam) - s)
    if scheme == "trap":
        return (1.0 - z) / (1.0 + z)
    if scheme == "be":
        return 1.0 / (1.0 + z)
    raise ValueError(scheme)


def implicit_step(H: np.ndarray, psi: np.ndarray, h: float, s: float, scheme: str) -> np.ndarray:
    """Solve (I + h (H - s)) x = b by a dense LU solve.

    Trapezoid (Method, Eq. 4 with h = dtau / 2): b = (I - h (H - s)) psi.
    Backward Euler: b = psi.
    """
    A = np.eye(H.shape[0]) + h * (H - s * np.eye(H.shape[0]))
    if scheme == "trap":
        b = psi - h * (H @ psi - s * psi)
    elif scheme == "be":
        b = psi.copy()
    else:
        raise ValueError(scheme)
    return np.linalg.solve(A, b)


def loggrid(tau0: float, tau1: float, ratio: float) -> np.ndarray:
    """Geometric grid 0, tau0, tau0 r, tau0 r^2, ..., clamped to end at tau1."""
    if not (tau0 > 0 and tau1 > tau0 and ratio > 1):
        raise ValueError("need 0 < tau0 < tau1 and ratio > 1")
    t = [0.0, tau0]
    while t[-1] < tau1:
        t.append(min(t[-1] * ratio, tau1))
    return np.array(t)


def panel_grid(tau_max: float, P: int, n: int) -> np.ndarray:
    """P panels with endpoints {0, tau_max / 2^(P-j), j = 1..P} and n uniform
    steps on each panel (Method)."""
    ends = [0.0] + [tau_max / 2.0 ** (P - j) for j in range(1, P + 1)]
    t = [0.0]
    for a, b in zip(ends[:-1], ends[1:]):
        for i in range(1, n + 1):
            t.append(a + (b - a) * i / n)
    return np.array(t)


def trap_local_error(mu):
    """E(mu) = exp(-3 mu / 2) (mu cosh(mu / 2) - 2 sinh(mu / 2)) (Appendix A)."""
    mu = np.asarray(mu, dtype=float)
    return np.exp(-1.5 * mu) * (mu * np.cosh(mu / 2) - 2.0 * np.sinh(mu / 2))


def forward_euler_step(H, psi, dtau, s=0.0):
    """psi <- (I - dtau (H - s)) psi (Appendix A)."""
    return psi - dtau * (H @ psi - s * psi)


def heun_step(H, psi, dtau, s=0.0):
    """Explicit predictor-corrector version of the trapezoid rule: predictor by
    forward Euler, corrector by the trapezoid average of the two slopes."""
    f0 = -(H @ psi - s * psi)
    pred = psi + dtau * f0
    f1 = -(H @ pred - s * pred)
    return psi + 0.5 * dtau * (f0 + f1)


def evolve_dense(H: np.ndarray, psi0: np.ndarray, grid, scheme: str,
                 shift_mode: str = "fixed", shift: float = 0.0):
    """Full-vector evolution along ``grid`` with normalisation after every step.

    Returns (states, energies, norms_before, shifts): states[k] is the
    normalised state at grid[k].  The energy shift is ``shift`` (fixed) or the
    energy of the current state (track), the rule the paper uses for the
    impurity model (Appendix D).
    """
    psi = psi0 / np.linalg.norm(psi0)
    states = [psi]
    energies = [float(psi @ H @ psi)]
    norms = [1.0]
    shifts = []
    for k in range(1, len(grid)):
        dtau = grid[k] - grid[k - 1]
        h = dtau / 2 if scheme == "trap" else dtau
        s = shift if shift_mode == "fixed" else energies[-1]
        x = implicit_step(H, psi, h, s, scheme)
        nrm = float(np.linalg.norm(x))
        psi = x / nrm
        states.append(psi)
        energies.append(float(psi @ H @ psi))
        norms.append(nrm)
        shifts.append(s)
    return states, energies, norms, shifts

"""Pins of the oracle's full state-vector level (``oracle.ed``).

Each test fixes a part of the oracle against something other than itself:
closed forms, textbook values, symmetry invariants, numbers the paper prints
(``tests/golden/paper_values.json``) or brute force.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import ed

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# --- Hamiltonians -----------------------------------------------------------

def test_two_site_singlet_energy():
    # S_1.S_2 has eigenvalues -3/4 (singlet) and +1/4 (triplet, 3-fold).
    ev = np.linalg.eigvalsh(ed.heisenberg_dense(2))
    assert np.allclose(ev, [-0.75, 0.25, 0.25, 0.25], atol=1e-14)


def test_four_site_open_chain_energy():
    # Open 4-site Heisenberg chain: E0 = -(3 + 2 sqrt 3) / 4 (textbook result).
    e0, _ = ed.ground_state(ed.heisenberg_dense(4))
    assert abs(e0 + (3 + 2 * math.sqrt(3)) / 4) < 1e-13


@pytest.mark.parametrize("L", [2, 3, 5, 8, 10])
def test_xx_chain_closed_form(L):
    # Jz = 0 maps to free fermions (Jordan-Wigner): an independent closed form.
    e0, _ = ed.ground_state(ed.heisenberg_dense(L, Jz=0.0))
    assert abs(e0 - ed.xx_chain_e0(L)) < 1e-12


def test_xx_closed_form_two_sites_by_hand():
    # H = (S+S- + S-S+)/2 on two sites has eigenvalues +-1/2, 0, 0.
    assert ed.xx_chain_e0(2) == pytest.approx(-0.5, abs=1e-15)


def test_heisenberg_su2_invariance():
    L = 6
    H = ed.heisenberg_dense(L)
    Sz = sum(ed.site_operator(ed.SZ, i, L) for i in range(L))
    Sp = sum(ed.site_operator(ed.SP, i, L) for i in range(L))
    S2 = Sp @ Sp.T + Sz @ Sz - Sz
    assert np.abs(H @ Sz - Sz @ H).max() < 1e-13
    assert np.abs(H @ S2 - S2 @ H).max() < 1e-12
    # an XXZ anisotropy keeps S^z but breaks S^2
    Hx = ed.heisenberg_dense(L, Jz=0.3)
    assert np.abs(Hx @ S2 - S2 @ Hx).max() > 1e-3


def test_aim_free_fermion_limit():
    rng = np.random.default_rng(7)
    eb = np.sort(rng.uniform(-1, 1, 3))
    V = rng.uniform(0.1, 0.5, 3)
    H = ed.aim_dense(0.0, 0.13, eb, V)
    assert abs(ed.ground_state(H)[0] - ed.free_fermion_aim_e0(0.13, eb, V)) < 1e-12


def test_aim_atomic_limit():
    # V = 0: impurity levels 0, eps_d, 2 eps_d + U; bath filled below zero.
    U = 4.0
    eb = np.array([-0.7, -0.2, 0.4])
    H = ed.aim_dense(U, -U / 2, eb, np.zeros(3))
    e_imp = min(0.0, -U / 2, 2 * (-U / 2) + U)
    assert abs(ed.ground_state(H)[0] - (e_imp + 2 * eb[eb < 0].sum())) < 1e-12


def test_aim_conserves_particle_number_and_is_symmetric():
    eb = np.array([-0.5, 0.5])
    H = ed.aim_dense(3.0, -1.5, eb, np.array([0.3, 0.3]))
    c = ed.jw_annihilators(6)
    N = sum(ci.T @ ci for ci in c)
    assert np.abs(H - H.T).max() == 0.0
    assert np.abs(H @ N - N @ H).max() < 1e-13
    # canonical anticommutation of the Jordan-Wigner operators
    for a in range(6):
        for b in range(6):
            ac = c[a] @ c[b].T + c[b].T @ c[a]
            assert np.abs(ac - (np.eye(64) if a == b else 0)).max() < 1e-15


# --- exact evolution and the implicit steps ---------------------------------

def test_exact_evolve_solves_the_ode():
    L = 6
    H = ed.heisenberg_dense(L)
    e0, _ = ed.ground_state(H)
    psi0 = np.random.default_rng(1).standard_normal(2 ** L)
    assert np.allclose(ed.exact_evolve(H, psi0, 0.0), psi0, atol=1e-13)
    tau, eps = 0.7, 1e-5
    deriv = (ed.exact_evolve(H, psi0, tau + eps) - ed.exact_evolve(H, psi0, tau - eps)) / (2 * eps)
    rhs = -(H - e0 * np.eye(2 ** L)) @ ed.exact_evolve(H, psi0, tau)
    assert np.abs(deriv - rhs).max() < 1e-8
    # semigroup property
    a = ed.exact_evolve(H, ed.exact_evolve(H, psi0, 0.3), 0.4)
    assert np.allclose(a, ed.exact_evolve(H, psi0, 0.7), atol=1e-12)


@pytest.mark.parametrize("scheme", ["trap", "be"])
def test_implicit_step_is_the_eigenbasis_factor(scheme):
    L = 6
    H = ed.heisenberg_dense(L)
    ev, vec = np.linalg.eigh(H)
    psi = np.random.default_rng(2).standard_normal(2 ** L)
    for h, s in [(0.05, 0.0), (1.7, ev[0]), (40.0, -1.0)]:
        x = ed.implicit_step(H, psi, h, s, scheme)
        expect = vec @ (ed.step_factor(ev, h, s, scheme) * (vec.T @ psi))
        assert np.abs(x - expect).max() < 1e-12 * max(1.0, np.abs(expect).max())


def test_trapezoid_factor_is_the_papers_stability_factor():
    lam = np.linspace(0, 50, 101)
    dtau = 0.37
    paper = (1 - lam * dtau / 2) / (1 + lam * dtau / 2)
    assert np.allclose(ed.step_factor(lam, dtau / 2, 0.0, "trap"), paper, rtol=0, atol=1e-15)


def test_a_stability_and_explicit_blow_up():
    # Appendix A: the implicit steps never amplify a mode with lambda >= s; forward
    # Euler (kappa = dtau * (E_max - s) > 2) and Heun do.
    L = 6
    H = ed.heisenberg_dense(L)
    ev = np.linalg.eigvalsh(H)
    s = ev[0]
    emax = ev[-1] - s
    kmax = GOLDEN["forward_euler_stable_kappa_max"]["value"]
    lam = ev - s
    for dtau in [0.1, 1.0, 10.0, 1e3]:
        assert np.all(np.abs(ed.step_factor(ev, dtau / 2, s, "trap")) <= 1 + 1e-15)
        assert np.all(np.abs(ed.step_factor(ev, dtau, s, "be")) <= 1 + 1e-15)
    psi = np.random.default_rng(3).standard_normal(2 ** L)
    psi /= np.linalg.norm(psi)
    for stepper in (ed.forward_euler_step, ed.heun_step):
        for kappa, grows in [(0.9 * kmax, False), (1.3 * kmax, True)]:
            dtau = kappa / emax
            p = psi.copy()
            for _ in range(200):
                p = stepper(H, p, dtau, s)
            assert (np.linalg.norm(p) > 10.0) == grows
    # forward Euler's amplification is |1 - kappa| exactly
    fe = [np.linalg.norm(ed.forward_euler_step(H, v, 2.5 / emax, s)) for v in np.linalg.eigh(H)[1].T[-1:]]
    assert abs(fe[0] - abs(1 - 2.5 * lam[-1] / emax)) < 1e-12


# --- grids and the local trapezoid error ------------------------------------

def test_loggrid_step_counts():
    # 0.01 * 1.5^22 = 74.8 < 100 < 0.01 * 1.5^23: 23 geometric points after 0, then
    # the clamp to 100 -> 24 steps.  0.01 * 1.3^43 = 791 < 1000 -> 45 steps;
    # 0.01 * 1.3^52 = 8.5e3 < 1e4 -> 54 steps.
    assert len(ed.loggrid(0.01, 100.0, 1.5)) - 1 == 24
    assert len(ed.loggrid(0.01, 1000.0, 1.3)) - 1 == 45
    assert len(ed.loggrid(0.01, 1e4, 1.3)) - 1 == 54
    g = ed.loggrid(0.01, 100.0, 1.5)
    assert g[0] == 0 and g[1] == 0.01 and g[-1] == 100.0
    assert np.allclose(g[2:-1] / g[1:-2], 1.5)


def test_panel_grid_endpoints():
    g = ed.panel_grid(64.0, 4, 3)
    # panels [0, 8], [8, 16], [16, 32], [32, 64], 3 uniform steps each
    assert len(g) == 13
    assert np.allclose(g[[0, 3, 6, 9, 12]], [0, 8, 16, 32, 64])
    assert np.allclose(np.diff(g[9:]), 32 / 3)


def test_trap_local_error_matches_definition_and_paper():
    # Closed form vs the defining expression lambda h/2 (e^-a l + e^-b l) - (e^-a l - e^-b l)
    # with a = h, b = 2h (Appendix A).
    for h in [0.5, 2.0, 16.0]:
        for mu in [0.1, 1.0, 2.1, 5.0]:
            lam = mu / h
            a, b = h, 2 * h
            direct = lam * h / 2 * (math.exp(-a * lam) + math.exp(-b * lam)) - (math.exp(-a * lam) - math.exp(-b * lam))
            assert abs(ed.trap_local_error(mu) - direct) < 1e-15
    # the integral term by quadrature too: lam * int_a^b e^(-tau lam) dtau
    from scipy.integrate import quad
    lam, h = 0.9, 1.3
    integral = lam * quad(lambda t: math.exp(-t * lam), h, 2 * h, epsabs=1e-14)[0]
    assert abs(integral - (math.exp(-h * lam) - math.exp(-2 * h * lam))) < 1e-13
    mu = np.linspace(1e-3, 20, 200001)
    E = ed.trap_local_error(mu)
    ref = GOLDEN["trap_local_error_max"]
    assert abs(E.max() - ref["value"]) <= ref["rel_tol"] * ref["value"]
    assert abs(mu[E.argmax()] - ref["at_mu"]) <= ref["mu_tol"]
    assert np.all(E > 0)


def test_trapezoid_second_order_on_panel_grid():
    # Method: the panel grid gives O(n^-2) convergence of the trapezoid rule;
    # Heisenberg chain section: doubling n improves accuracy by about 4.
    L = 8
    H = ed.heisenberg_dense(L)
    e0, _ = ed.ground_state(H)
    psi0 = np.random.default_rng(4).standard_normal(2 ** L)
    errs = {}
    for scheme in ["trap", "be"]:
        errs[scheme] = []
        for n in [2, 4, 8, 16]:
            g = ed.panel_grid(64.0, 14, n)
            states, *_ = ed.evolve_dense(H, psi0, g, scheme, "fixed", e0)
            worst = 0.0
            for t, p in zip(g, states):
                ref = ed.exact_evolve(H, psi0, t)
                ref /= np.linalg.norm(ref)
                worst = max(worst, math.sqrt(max(0.0, 1 - abs(p @ ref))))
            errs[scheme].append(worst)
    band = GOLDEN["trapezoid_convergence_factor_per_doubling"]
    ratios = [a / b for a, b in zip(errs["trap"][:-1], errs["trap"][1:])]
    assert all(band["lo"] < r < band["hi"] for r in ratios), ratios
    be_ratios = [a / b for a, b in zip(errs["be"][:-1], errs["be"][1:])]
    assert all(1.6 < r < 2.6 for r in be_ratios), be_ratios


def test_dense_evolution_converges_to_ground_state():
    L = 8
    H = ed.heisenberg_dense(L)
    e0, v0 = ed.ground_state(H)
    psi0 = np.random.default_rng(5).standard_normal(2 ** L)
    for mode in ["fixed", "track"]:
        states, en, norms, shifts = ed.evolve_dense(H, psi0, ed.loggrid(0.01, 100.0, 1.5), "be", mode, e0)
        assert en[-1] - e0 < 1e-8
        assert np.all(np.diff(en) <= 1e-12)
        assert abs(abs(states[-1] @ v0) - 1) < 1e-8

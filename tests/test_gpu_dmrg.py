"""GPU parity of the two-site DMRG ground-state sweeps against the oracle
(``oracle.dmrg``, exact local eigensolves) and exact diagonalisation, through
the C ABI.

* Heisenberg chain at complete bonds: the energy equals the oracle's and the
  exact ground energy to 1e-10 (relative), the state the oracle's (unique
  ground state) to 1e-8 in overlap.
* Truncated bonds grown from a bond-1 product state: the energy after every
  sweep count equals the oracle's, and so do the bond dimensions.
* The Anderson impurity model (d = 4, MPO bond 6).
* A two-site chain (a single block); the error paths of the boundary.
"""
import numpy as np
import pytest

import paper_2606_02930_amd as ite
from paper_2606_02930_amd import hamiltonians
from oracle import dmrg as odmrg, ed, mpo as ompo, mps as omps
from workload import rng_for, random_spinors, aim_bath
from tests.gpu_util import require_gpu, mps_overlap

pytestmark = pytest.mark.gpu

# local problems solved to the rounding level, as the oracle's exact ones
EXACT = dict(krylov_dim=24, max_cycles=30, tol=1e-14)


@pytest.fixture(scope="module")
def ctx():
    torch = require_gpu()
    c = ite.ite_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    ite.ite_ctx_destroy(c)


def _neel(L):
    return [np.array([1.0, 0.0]) if i % 2 == 0 else np.array([0.0, 1.0]) for i in range(L)]


def _run_both(ctx, L, d, Wprod, Woracle, spinors, chi, pad, nsweeps, cutoff=0.0):
    psi = ite.ite_mps_create(ctx, spinors, chi, pad_full=pad)
    H = ite.ite_mpo_load(ctx, Wprod)
    try:
        rep = ite.ite_dmrg_sweeps(ctx, psi, H, nsweeps, chi, cutoff=cutoff, **EXACT)
        e_meas = ite.ite_measure_energy(ctx, psi, H)
        out = ite.ite_mps_export(ctx, psi, [d] * L)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(H)
    o_out, o_en, o_disc = odmrg.dmrg_sweeps(omps.product_state(spinors, chi, pad_full=pad), Woracle, nsweeps,
                                            chi, cutoff)
    return rep, e_meas, out, o_out, o_en


@pytest.mark.parametrize("L", [6, 8])
def test_dmrg_heisenberg_complete_bonds_match_oracle_and_ed(ctx, L):
    chi = 2 ** (L // 2)
    rep, e_meas, out, o_out, o_en = _run_both(ctx, L, 2, hamiltonians.heisenberg(L), ompo.heisenberg_mpo(L),
                                              _neel(L), chi, True, 2)
    e0 = ed.ground_state(ed.heisenberg_dense(L))[0]
    assert abs(rep["energy"] - o_en[-1]) <= 1e-10 * abs(e0)
    assert abs(rep["energy"] - e0) <= 1e-10 * abs(e0)
    assert abs(e_meas - rep["energy"]) <= 1e-12 * abs(e0)
    assert rep["max_res_rel"] < 1e-10
    assert 1 - abs(mps_overlap(out, o_out)) <= 1e-8
    assert abs(mps_overlap(out, out) - 1.0) < 1e-12


@pytest.mark.parametrize("nsweeps", [1, 3])
def test_dmrg_truncated_from_product_state_matches_oracle(ctx, nsweeps):
    # bonds grow from 1 up to chi = 8 on a 12-site XXZ chain, random spinors
    L, chi = 12, 8
    sp = random_spinors(rng_for(73), L, 2)
    rep, e_meas, out, o_out, o_en = _run_both(ctx, L, 2, hamiltonians.heisenberg(L, 1.0, 0.6),
                                              ompo.heisenberg_mpo(L, 1.0, 0.6), sp, chi, False, nsweeps)
    assert abs(rep["energy"] - o_en[-1]) <= 1e-9 * abs(o_en[-1])
    # one sweep from bond 1 reaches bond 4 (the right bonds are still 1 on
    # the way out); three reach chi and truncate
    assert [a.shape[2] for a in out] == [a.shape[2] for a in o_out]
    assert max(a.shape[2] for a in out) == (4 if nsweeps == 1 else chi)
    assert (rep["max_disc"] > 0.0) == (nsweeps > 1)
    assert 1 - abs(mps_overlap(out, o_out)) <= 1e-7


def test_dmrg_anderson_impurity_matches_oracle(ctx):
    nb = 3
    eb, V = aim_bath(nb, gamma=0.3)
    U = 4.0
    L = nb + 1
    sp = random_spinors(rng_for(74), L, 4)
    rep, e_meas, out, o_out, o_en = _run_both(ctx, L, 4, hamiltonians.anderson_star(U, -U / 2, eb, V),
                                              ompo.aim_mpo(U, -U / 2, eb, V), sp, 16, True, 2)
    assert abs(rep["energy"] - o_en[-1]) <= 1e-10 * abs(o_en[-1])
    assert 1 - abs(mps_overlap(out, o_out)) <= 1e-8


def test_dmrg_two_sites_is_one_block(ctx):
    # a single block: the singlet, E = -3/4 J
    psi = ite.ite_mps_create(ctx, _neel(2), 2)
    H = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(2))
    try:
        rep = ite.ite_dmrg_sweeps(ctx, psi, H, 1, 2, **EXACT)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(H)
    assert abs(rep["energy"] + 0.75) < 1e-13


def test_dmrg_error_paths(ctx):
    psi = ite.ite_mps_create(ctx, _neel(4), 4)
    H = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(4))
    H6 = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(6))
    try:
        for kw in (dict(nsweeps=0), dict(krylov_dim=65), dict(krylov_dim=0), dict(cutoff=1.0), dict(tol=-1.0),
                   dict(max_cycles=0), dict(chi_max=0)):
            args = dict(nsweeps=1, chi_max=4)
            args.update(kw)
            with pytest.raises(ite.IteError) as e:
                ite.ite_dmrg_sweeps(ctx, psi, H, **args)
            assert e.value.code == ite.ITE_EINVAL
        with pytest.raises(ite.IteError) as e:
            ite.ite_dmrg_sweeps(ctx, psi, H6, 1, 4)
        assert e.value.code == ite.ITE_ESTATE
        # the state is still usable after the refused calls
        rep = ite.ite_dmrg_sweeps(ctx, psi, H, 1, 4, **EXACT)
        assert np.isfinite(rep["energy"])
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(H)
        ite.ite_mpo_destroy(H6)

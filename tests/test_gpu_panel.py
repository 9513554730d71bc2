"""GPU parity of the Gauss-Legendre collocation panel (the spectral variant of
the Method section) and of the density-matrix MPO-MPS product with the
trapezoid step that uses it for its right-hand side (Appendix B), through the
C ABI, against the oracle (``oracle/gauss.py``, ``oracle/apply.py``) and
exact diagonalisation.

* ite_mpo_apply: without truncation the product equals O psi densely (any
  MPS, any MPO of the chain); with truncation the kept bonds and the state
  equal the oracle's product.
* The MPS right-hand-side trapezoid step at complete bonds equals the
  full-vector trapezoid step; with the paper's budget and truncation it
  follows the oracle step by step.
* The panel at complete bonds with converged local solves equals the dense
  panel (the (p, p) Pade approximant) for p = 1..3; with the paper's budget
  and truncation it follows the oracle panel by panel.
* Both run inside a batch (one by one) with the same bits as alone, and the
  options are validated.
"""
import numpy as np
import pytest

import paper_2606_02930_amd as ite
from paper_2606_02930_amd import hamiltonians
from oracle import apply as oapply, ed, gauss, mpo as ompo, mps as omps
from workload import rng_for, random_spinors, aim_bath
from tests.gpu_util import require_gpu, mps_vector, mps_overlap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = require_gpu()
    c = ite.ite_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    ite.ite_ctx_destroy(c)


def _opts(**kw):
    o = ite.ite_default_opts()
    conv = {"scheme": {"trap": ite.SCHEME_TRAP, "be": ite.SCHEME_BE, "gl": ite.SCHEME_GL},
            "shift_mode": {"fixed": ite.SHIFT_FIXED, "track": ite.SHIFT_TRACK},
            "rhs_mode": {"project": ite.RHS_PROJECT, "mps": ite.RHS_MPS}}
    for k, v in kw.items():
        setattr(o, k, conv[k][v] if k in conv and isinstance(v, str) else v)
    return o


def _random_mps(rng, dims, d):
    return [rng.standard_normal((dims[i], d, dims[i + 1])) for i in range(len(dims) - 1)]


# ---------------------------------------------------------------------------
# density-matrix product
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("L,dims,Jz", [(5, [1, 2, 4, 3, 2, 1], 0.6), (8, [1, 2, 4, 8, 16, 8, 4, 2, 1], 1.0),
                                       (9, [1, 2, 3, 5, 7, 6, 4, 4, 2, 1], 0.0)])
def test_mpo_apply_untruncated_is_exact(ctx, L, dims, Jz):
    rng = np.random.default_rng(70 + L)
    A = _random_mps(rng, dims, 2)
    W = ompo.heisenberg_mpo(L, Jz=Jz)
    want = ompo.mpo_to_dense(W) @ mps_vector(A)
    psi = ite.ite_mps_load(ctx, A, 64)
    O = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(L, Jz=Jz))
    try:
        out, disc = ite.ite_mpo_apply(ctx, O, psi, 64, 0.0, 0.0)
        try:
            B = ite.ite_mps_export(ctx, out, [2] * L)
        finally:
            ite.ite_mps_destroy(out)
        # psi is unchanged
        assert np.abs(mps_vector(ite.ite_mps_export(ctx, psi, [2] * L)) - mps_vector(A)).max() < 1e-15 * 10
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(O)
    got = mps_vector(B)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    assert disc < 1e-14
    for a in B[1:]:
        m = a.reshape(a.shape[0], -1)
        assert np.abs(m @ m.T - np.eye(m.shape[0])).max() < 1e-12
    b_or, _ = oapply.density_matrix_apply(W, A, 64, 0.0, 0.0)
    assert omps.bond_dims(B) == omps.bond_dims(b_or)


@pytest.mark.parametrize("chi,cutoff", [(4, 0.0), (6, 1e-3), (64, 1e-6)])
def test_mpo_apply_truncated_matches_oracle(ctx, chi, cutoff):
    L = 10
    rng = np.random.default_rng(81)
    A = omps.product_state(random_spinors(rng_for(0, 30), L, 2), 32, pad_full=True)
    # a non-trivial state: one trapezoid step of the oracle from a padded product state
    A, _ = omps.imag_step(A, ompo.heisenberg_mpo(L), 0.4,
                          omps.StepOptions(scheme="trap", chi_max=32, cutoff=0.0, max_cycles=50, tol_loc=1e-12))
    h, s = 0.3, -2.0
    Or = oapply.rhs_mpo(ompo.heisenberg_mpo(L), h, s)
    b_or, info = oapply.density_matrix_apply(Or, A, chi, cutoff, 1e-13)
    psi = ite.ite_mps_load(ctx, A, 32)
    O = ite.ite_mpo_load(ctx, Or)
    try:
        out, disc = ite.ite_mpo_apply(ctx, O, psi, chi, cutoff, 1e-13)
        try:
            B = ite.ite_mps_export(ctx, out, [2] * L)
        finally:
            ite.ite_mps_destroy(out)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(O)
    assert omps.bond_dims(B) == omps.bond_dims(b_or)
    assert abs(disc - info["disc"]) <= 1e-8 * max(info["disc"], 1e-12) + 1e-15
    v, w = mps_vector(B), mps_vector(b_or)
    assert np.linalg.norm(v - w) <= 1e-9 * np.linalg.norm(w)


def test_mpo_apply_on_the_impurity_model(ctx):
    # d = 4 sites and a fermionic MPO (w = 6): the untruncated product is exact
    eps, V = aim_bath(3)
    U = 4.0
    W = ompo.aim_mpo(U, -U / 2, eps, V)
    L = len(W)
    rng = np.random.default_rng(9)
    dims = [1, 4, 12, 4, 1]
    A = _random_mps(rng, dims, 4)
    want = ompo.mpo_to_dense(W) @ mps_vector(A)
    psi = ite.ite_mps_load(ctx, A, 64)
    O = ite.ite_mpo_load(ctx, hamiltonians.anderson_star(U, -U / 2, eps, V))
    try:
        out, disc = ite.ite_mpo_apply(ctx, O, psi, 64, 0.0, 0.0)
        B = ite.ite_mps_export(ctx, out, [4] * L)
        ite.ite_mps_destroy(out)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(O)
    assert np.abs(mps_vector(B) - want).max() <= 1e-12 * np.abs(want).max()


def test_mpo_apply_errors(ctx):
    psi = ite.ite_mps_create(ctx, random_spinors(rng_for(0, 3), 6, 2), 8)
    O = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(7))
    O6 = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(6))
    try:
        with pytest.raises(ite.IteError) as e:
            ite.ite_mpo_apply(ctx, O, psi, 8)
        assert e.value.code == ite.ITE_ESTATE
        for bad in [dict(chi_max=0), dict(cutoff=1.0), dict(tie_rel=-1.0)]:
            kw = dict(chi_max=8, cutoff=0.0, tie_rel=0.0)
            kw.update(bad)
            with pytest.raises(ite.IteError) as e:
                ite.ite_mpo_apply(ctx, O6, psi, **kw)
            assert e.value.code == ite.ITE_EINVAL
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(O)
        ite.ite_mpo_destroy(O6)


# ---------------------------------------------------------------------------
# trapezoid step with the right-hand side as an MPS
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shift_mode", ["fixed", "track"])
def test_mps_rhs_step_at_complete_bonds_equals_full_vector(ctx, shift_mode):
    L, chi = 8, 16
    H = ed.heisenberg_dense(L)
    e0 = ed.ground_state(H)[0]
    sp = random_spinors(rng_for(0, 21), L, 2)
    grid = ed.loggrid(0.01, 5.0, 1.6)
    psi = ite.ite_mps_create(ctx, sp, chi, pad_full=True)
    Hm = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(L))
    try:
        reps = ite.ite_evolve_grid(ctx, psi, Hm, grid,
                                   _opts(scheme="trap", rhs_mode="mps", shift_mode=shift_mode, shift=e0, chi_max=chi,
                                         cutoff=0.0, max_cycles=400, tol_loc=1e-13))
        out = ite.ite_mps_export(ctx, psi, [2] * L)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(Hm)
    states, en, norms, _ = ed.evolve_dense(H, mps_vector(omps.product_state(sp)), grid, "trap", shift_mode, e0)
    assert len(reps) == len(grid) - 1
    # the product diagonalises reduced density matrices (squared Schmidt
    # values): agreement at 1e-9, the product's own resolution
    for r, e in zip(reps, en[1:]):
        assert abs(r["energy"] - e) <= 1e-9 * max(1.0, abs(e))
        assert r["rhs_disc"] < 1e-14
    v = mps_vector(out)
    assert 1 - abs(v @ states[-1]) < 1e-10


@pytest.mark.parametrize("model", ["heis", "aim"])
def test_mps_rhs_step_paper_budget_matches_oracle(ctx, model):
    if model == "heis":
        L, chi, d = 12, 16, 2
        sp = random_spinors(rng_for(1, 5), L, 2)
        Wp, Wo = hamiltonians.heisenberg(L), ompo.heisenberg_mpo(L)
        grid = ed.loggrid(0.01, 10.0, 1.3)
    else:
        eps, V = aim_bath(3)
        Wp, Wo = hamiltonians.anderson_star(4.0, -2.0, eps, V), ompo.aim_mpo(4.0, -2.0, eps, V)
        L, chi, d = len(Wo), 16, 4
        sp = random_spinors(rng_for(3, 5), L, 4)
        grid = ed.loggrid(0.01, 5.0, 1.3)
    kw = dict(scheme="trap", shift_mode="track", chi_max=chi, cutoff=1e-8, krylov_dim=10, max_cycles=1, tol_loc=0.0)
    psi = ite.ite_mps_create(ctx, sp, chi)
    Hm = ite.ite_mpo_load(ctx, Wp)
    try:
        reps = ite.ite_evolve_grid(ctx, psi, Hm, grid, _opts(rhs_mode="mps", **kw))
        out = ite.ite_mps_export(ctx, psi, [d] * L)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(Hm)
    o_out, o_reps = oapply.evolve_grid_mps_rhs(omps.product_state(sp, chi), Wo, grid, omps.StepOptions(**kw))
    for r, orr in zip(reps, o_reps):
        assert r["max_chi"] == orr.max_chi
        assert abs(r["energy"] - orr.energy) <= 1e-10 * abs(orr.energy)
        assert abs(r["rhs_disc"] - orr.extra["rhs_disc"]) <= 1e-6 * orr.extra["rhs_disc"] + 1e-14
    assert 1 - abs(mps_overlap(out, o_out)) <= 1e-8


# ---------------------------------------------------------------------------
# Gauss-Legendre panel
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p,chi", [(1, 32), (2, 32), (3, 32), (4, 64), (5, 64)])
def test_gl_panel_at_complete_bonds_equals_dense_panel(ctx, p, chi):
    # chi holds the augmented state exactly (node site of dimension p + 1:
    # bonds up to 32); with p + 1 > 4 the augmented state's bonds are first
    # widened to complete (the first block could not give the node bond its
    # rank otherwise); the chain's own bonds stay at most 16
    L = 8
    H = ed.heisenberg_dense(L)
    sp = random_spinors(rng_for(0, 40 + p), L, 2)
    grid = ed.loggrid(0.01, 20.0, 2.0)
    psi = ite.ite_mps_create(ctx, sp, chi, pad_full=True)
    Hm = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(L))
    try:
        reps = ite.ite_evolve_grid(ctx, psi, Hm, grid, _opts(scheme="gl", gl_nodes=p, shift_mode="track",
                                                             chi_max=chi, cutoff=0.0, max_cycles=400,
                                                             tol_loc=1e-13))
        out = ite.ite_mps_export(ctx, psi, [2] * L)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(Hm)
    states, energies = gauss.dense_evolve(H, mps_vector(omps.product_state(sp)), grid, p, "track")
    assert len(reps) == len(grid) - 1
    for r, e, t in zip(reps, energies[1:], grid[1:]):
        assert abs(r["energy"] - e) <= 1e-10 * max(1.0, abs(e))
        assert abs(r["tau"] - t) < 1e-12 * t
        assert r["max_chi"] <= 16 and r["aux_max_chi"] >= r["max_chi"]
    v = mps_vector(out)
    assert abs(np.linalg.norm(v) - 1) < 1e-12
    assert 1 - abs(v @ states[-1]) < 1e-10


@pytest.mark.parametrize("p", [4, 5])
def test_gl_panel_many_nodes_matches_oracle(ctx, p):
    # four and five nodes on a spin-1/2 chain: the node bond needs rank
    # p + 1 > 4 while the first block's columns (site 1 and the bond of 2
    # behind it) hold 4, so both sides widen the augmented state's bonds by
    # the same Householder completion before the sweep; the library follows
    # the oracle step for step (splits of up to 128 rows: multi-pair Jacobi)
    L, chi = 8, 64
    sp = random_spinors(rng_for(0, 40 + p), L, 2)
    grid = ed.loggrid(0.01, 20.0, 2.0)
    kw = dict(shift_mode="track", chi_max=chi, cutoff=0.0, krylov_dim=10, max_cycles=400, tol_loc=1e-13)
    psi = ite.ite_mps_create(ctx, sp, chi, pad_full=True)
    Hm = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(L))
    try:
        reps = ite.ite_evolve_grid(ctx, psi, Hm, grid, _opts(scheme="gl", gl_nodes=p, **kw))
        out = ite.ite_mps_export(ctx, psi, [2] * L)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(Hm)
    o_out, o_reps = gauss.gl_evolve(omps.product_state(sp, chi, pad_full=True), ompo.heisenberg_mpo(L), grid, p,
                                    omps.StepOptions(**kw))
    assert len(reps) == len(o_reps) == len(grid) - 1
    for r, orr in zip(reps, o_reps):
        assert r["max_chi"] == orr.max_chi
        assert abs(r["energy"] - orr.energy) <= 1e-10 * abs(orr.energy)
    assert 1 - abs(mps_overlap(out, o_out)) <= 1e-10


@pytest.mark.parametrize("p", [2, 3])
def test_gl_panel_paper_budget_matches_oracle(ctx, p):
    L, chi = 10, 16
    sp = random_spinors(rng_for(1, 60 + p), L, 2)
    grid = ed.loggrid(0.01, 10.0, 1.6)
    kw = dict(shift_mode="track", chi_max=chi, cutoff=1e-9, krylov_dim=10, max_cycles=1, tol_loc=0.0)
    psi = ite.ite_mps_create(ctx, sp, chi)
    Hm = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(L))
    try:
        reps = ite.ite_evolve_grid(ctx, psi, Hm, grid, _opts(scheme="gl", gl_nodes=p, **kw))
        out = ite.ite_mps_export(ctx, psi, [2] * L)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(Hm)
    o_out, o_reps = gauss.gl_evolve(omps.product_state(sp, chi), ompo.heisenberg_mpo(L), grid, p,
                                    omps.StepOptions(**kw))
    for r, orr in zip(reps, o_reps):
        assert r["max_chi"] == orr.max_chi
        assert r["aux_max_chi"] == orr.extra["aug_max_chi"]
        assert abs(r["energy"] - orr.energy) <= 1e-10 * abs(orr.energy)
        assert abs(r["norm_before"] - orr.norm_before) <= 1e-9 * orr.norm_before
    assert 1 - abs(mps_overlap(out, o_out)) <= 1e-8


def test_gl_panel_on_the_impurity_model(ctx):
    eps, V = aim_bath(2)
    Wo = ompo.aim_mpo(4.0, -2.0, eps, V)
    L, chi = len(Wo), 64
    sp = random_spinors(rng_for(3, 61), L, 4)
    grid = ed.loggrid(0.05, 5.0, 2.0)
    kw = dict(shift_mode="track", chi_max=chi, cutoff=0.0, krylov_dim=10, max_cycles=200, tol_loc=1e-12)
    psi = ite.ite_mps_create(ctx, sp, chi, pad_full=True)
    Hm = ite.ite_mpo_load(ctx, hamiltonians.anderson_star(4.0, -2.0, eps, V))
    try:
        reps = ite.ite_evolve_grid(ctx, psi, Hm, grid, _opts(scheme="gl", gl_nodes=2, **kw))
        out = ite.ite_mps_export(ctx, psi, [4] * L)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(Hm)
    perm = ed.aim_basis_permutation(L)
    Hd = ed.aim_dense(4.0, -2.0, eps, V)[perm][:, perm]
    states, energies = gauss.dense_evolve(Hd, mps_vector(omps.product_state(sp)), grid, 2, "track")
    for r, e in zip(reps, energies[1:]):
        assert abs(r["energy"] - e) <= 1e-10 * max(1.0, abs(e))
    assert 1 - abs(mps_vector(out) @ states[-1]) < 1e-10


def test_composite_steps_in_a_batch_equal_alone(ctx):
    L, chi = 10, 16
    Wp = hamiltonians.heisenberg(L)
    kws = [dict(scheme="gl", gl_nodes=2), dict(scheme="trap", rhs_mode="mps"), dict(scheme="trap")]
    seeds = [70, 71, 72]

    def run(batch):
        Hm = ite.ite_mpo_load(ctx, Wp)
        psis = [ite.ite_mps_create(ctx, random_spinors(rng_for(1, s), L, 2), chi) for s in seeds]
        opts = [_opts(chi_max=chi, cutoff=1e-9, **kw) for kw in kws]
        try:
            for h in (0.05, 0.2):
                if batch:
                    _, st = ite.ite_step_batch(ctx, psis, [Hm] * 3, [h, h, h], opts)
                    assert st == [0, 0, 0]
                else:
                    for p, o in zip(psis, opts):
                        ite.ite_imag_step(ctx, p, Hm, h, o)
            return [ite.ite_mps_export(ctx, p, [2] * L) for p in psis]
        finally:
            for p in psis:
                ite.ite_mps_destroy(p)
            ite.ite_mpo_destroy(Hm)

    alone, mixed = run(False), run(True)
    for a, b in zip(alone, mixed):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_panel_option_validation(ctx):
    psi = ite.ite_mps_create(ctx, random_spinors(rng_for(0, 9), 6, 2), 8)
    Hm = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(6))
    try:
        for bad in [dict(scheme="gl", gl_nodes=0), dict(scheme="gl", gl_nodes=8), dict(rhs_mode=2)]:
            with pytest.raises(ite.IteError) as e:
                ite.ite_imag_step(ctx, psi, Hm, 0.1, _opts(chi_max=8, **bad))
            assert e.value.code == ite.ITE_EINVAL
        # psi untouched by refused steps
        assert ite.ite_mps_get_tau(psi) == 0.0
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(Hm)


@pytest.mark.parametrize("mode", ["gl", "mps_rhs"])
def test_full_size_splits_inside_panels_and_mps_rhs_steps(ctx, mode):
    # complete bonds up to 256: the central blocks (and, for the MPS
    # right-hand side, the density matrices of the product) split 512 x 512
    # matrices, through the Householder preconditioning and the multi-pair
    # Jacobi rounds; paper budget, two steps of the 0.01 -> 1000, ratio 1.3
    # grid
    L, chi = 16, 256
    sp = random_spinors(rng_for(1, 80), L, 2)
    grid = ed.loggrid(0.01, 1000.0, 1.3)[:3]
    kw = dict(shift_mode="track", chi_max=chi, cutoff=0.0, krylov_dim=10, max_cycles=1, tol_loc=0.0)
    extra = dict(scheme="gl", gl_nodes=2) if mode == "gl" else dict(scheme="trap", rhs_mode="mps")
    psi = ite.ite_mps_create(ctx, sp, chi, pad_full=True)
    Hm = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(L))
    try:
        reps = ite.ite_evolve_grid(ctx, psi, Hm, grid, _opts(**extra, **kw))
        out = ite.ite_mps_export(ctx, psi, [2] * L)
    finally:
        ite.ite_mps_destroy(psi)
        ite.ite_mpo_destroy(Hm)
    o_psi = omps.product_state(sp, chi, pad_full=True)
    if mode == "gl":
        o_out, o_reps = gauss.gl_evolve(o_psi, ompo.heisenberg_mpo(L), grid, 2, omps.StepOptions(**kw))
    else:
        o_out, o_reps = oapply.evolve_grid_mps_rhs(o_psi, ompo.heisenberg_mpo(L), grid,
                                                   omps.StepOptions(scheme="trap", **kw))
    assert len(reps) == 2 and max(omps.bond_dims(o_out)) == chi
    for r, orr in zip(reps, o_reps):
        assert r["max_chi"] == orr.max_chi
        assert abs(r["energy"] - orr.energy) <= 1e-10 * abs(orr.energy)
        assert abs(r["norm_before"] - orr.norm_before) <= 1e-10 * orr.norm_before
    assert 1 - abs(mps_overlap(out, o_out)) <= 1e-8

"""GPU tests of batched steps (ite_step_batch): several independent states of
different lengths, bond dimensions, local dimensions and precisions stepped
in lockstep with grouped H_eff launches and a captured graph of the batched
local solves.

* Each state's reports and tensors are bitwise those of the same state
  stepped alone (a batch of one), with the graph and without it, and equal
  ite_imag_step's step to rounding (1e-12 relative energy).
* Each state's energies match the oracle's evolution per step (1e-10
  relative, paper budget; 1e-8 for FP32 refinement).
* FP32 refinement (fixed corrections, one GMRES cycle each) is batched too:
  same product counts as the unbatched refinement and the same step to
  rounding (its FP32 products are the same tiles with the same K order; the
  correction is added to x in one pass instead of through a separate vector).
* The graph is captured once per batch size and budget and then replayed.
"""
import numpy as np
import pytest

import paper_2606_02930_amd as ite
from paper_2606_02930_amd import hamiltonians
from oracle import ed, mpo as ompo, mps as omps
from workload import rng_for, random_spinors, aim_bath
from tests.gpu_util import require_gpu, mps_overlap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = require_gpu()
    c = ite.ite_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    ite.ite_ctx_destroy(c)


def _cases():
    eb, V = aim_bath(3, 0.3)
    out = []
    for k, (L, chi, prec) in enumerate([(8, 16, 0), (12, 32, 0), (10, 24, 0), (16, 48, 0), (9, 16, 1)]):
        out.append(dict(W=hamiltonians.heisenberg(L), Wo=ompo.heisenberg_mpo(L), d=2,
                        sp=random_spinors(rng_for(70, k), L, 2), chi=chi, prec=prec))
    out.append(dict(W=hamiltonians.anderson_star(4.0, -2.0, eb, V), Wo=ompo.aim_mpo(4.0, -2.0, eb, V), d=4,
                    sp=random_spinors(rng_for(70, 9), 4, 4), chi=16, prec=0))
    return out


def _run(ctx, cases, which, steps, batched=True, graphs=True, refine=0):
    ite.ite_ctx_set_graphs(ctx, graphs)
    grid = ed.loggrid(0.01, 20.0, 1.3)[:steps + 1]
    psis, Hs, opts = [], [], []
    for j in which:
        cs = cases[j]
        psis.append(ite.ite_mps_create(ctx, cs["sp"], cs["chi"]))
        Hs.append(ite.ite_mpo_load(ctx, cs["W"]))
        opts.append(ite.ite_default_opts(chi_max=cs["chi"], cutoff=1e-10, precision=cs["prec"],
                                         max_refine=refine if cs["prec"] else 0))
    reps = {j: [] for j in which}
    try:
        for k in range(1, len(grid)):
            h = 0.5 * (grid[k] - grid[k - 1])
            if batched:
                rs, st = ite.ite_step_batch(ctx, psis, Hs, [h] * len(psis), opts)
                assert st == [0] * len(psis)
            else:
                rs = [ite.ite_imag_step(ctx, p, H, h, o) for p, H, o in zip(psis, Hs, opts)]
            for j, r in zip(which, rs):
                reps[j].append(r)
        states = {j: ite.ite_mps_export(ctx, p, [cases[j]["d"]] * len(cases[j]["sp"])) for j, p in zip(which, psis)}
    finally:
        for p in psis:
            ite.ite_mps_destroy(p)
        for H in Hs:
            ite.ite_mpo_destroy(H)
        ite.ite_ctx_set_graphs(ctx, True)
    return reps, states


KEYS = ("energy", "norm_before", "max_chi", "max_disc", "matvecs_fp64", "matvecs_lo", "max_res_rel")


def test_batch_equals_each_state_alone_bitwise(ctx):
    cases = _cases()
    allj = list(range(len(cases)))
    before = ite.ite_ctx_batch_stats(ctx)
    reps_b, st_b = _run(ctx, cases, allj, 6)
    after = ite.ite_ctx_batch_stats(ctx)
    assert after["solves"] > before["solves"]
    assert after["replays"] > after["captures"] - before["captures"]
    for j in allj:
        reps_a, st_a = _run(ctx, cases, [j], 6)
        for a, b in zip(reps_a[j], reps_b[j]):
            for k in KEYS:
                assert a[k] == b[k], (j, k, a[k], b[k])
        for x, y in zip(st_a[j], st_b[j]):
            assert x.shape == y.shape and np.array_equal(x, y)
    # the same launches issued one by one, without the graph
    reps_n, st_n = _run(ctx, cases, allj, 6, graphs=False)
    for j in allj:
        assert [r["energy"] for r in reps_n[j]] == [r["energy"] for r in reps_b[j]]
        assert all(np.array_equal(x, y) for x, y in zip(st_n[j], st_b[j]))


def test_batch_matches_single_steps_and_the_oracle(ctx):
    cases = _cases()
    allj = list(range(len(cases)))
    reps_b, st_b = _run(ctx, cases, allj, 6)
    reps_s, st_s = _run(ctx, cases, allj, 6, batched=False)
    grid = ed.loggrid(0.01, 20.0, 1.3)[:7]
    for j in allj:
        cs = cases[j]
        for a, b in zip(reps_s[j], reps_b[j]):
            tol = 1e-12 if cs["prec"] == 0 else 1e-10
            assert abs(a["energy"] - b["energy"]) <= tol * abs(a["energy"]), (j, a["energy"], b["energy"])
            assert a["max_chi"] == b["max_chi"]
            assert (a["matvecs_fp64"], a["matvecs_lo"]) == (b["matvecs_fp64"], b["matvecs_lo"]), j
        o_out, o_reps = omps.evolve_grid(omps.product_state(cs["sp"]), cs["Wo"], grid,
                                         omps.StepOptions(chi_max=cs["chi"], cutoff=1e-10))
        bound = 1e-10 if cs["prec"] == 0 else 1e-8
        for b, o in zip(reps_b[j], o_reps):
            assert abs(b["energy"] - o.energy) <= bound * abs(o.energy)
        if cs["prec"] == 0:
            assert 1 - abs(mps_overlap(st_b[j], o_out)) <= 1e-8


def test_batch_argument_errors(ctx):
    L = 6
    H = ite.ite_mpo_load(ctx, hamiltonians.heisenberg(L))
    p = ite.ite_mps_create(ctx, random_spinors(rng_for(71), L, 2), 8)
    try:
        o = ite.ite_default_opts(chi_max=8)
        with pytest.raises(ite.IteError) as e:
            ite.ite_step_batch(ctx, [p, p], [H, H], [0.1, 0.1], o)
        assert e.value.code == ite.ITE_EINVAL
        with pytest.raises(ite.IteError) as e:
            ite.ite_step_batch(ctx, [p], [H], [-1.0], o)
        assert e.value.code == ite.ITE_EINVAL
        rs, st = ite.ite_step_batch(ctx, [p], [H], [0.1], o)
        assert st == [0] and np.isfinite(rs[0]["energy"])
    finally:
        ite.ite_mps_destroy(p)
        ite.ite_mpo_destroy(H)


def test_batch_fp32_refinement_two_corrections(ctx):
    """FP32 refinement with two corrections: batched (with FP64 states in the
    same slot) bitwise equal to the state alone, equal to the unbatched
    refinement to rounding, and close to the oracle's evolution."""
    cases = _cases()
    cases.append(dict(W=hamiltonians.heisenberg(14), Wo=ompo.heisenberg_mpo(14), d=2,
                      sp=random_spinors(rng_for(70, 11), 14, 2), chi=40, prec=1))
    fp32 = [4, len(cases) - 1]
    allj = [0, 1] + fp32
    before = ite.ite_ctx_batch_stats(ctx)
    reps_b, st_b = _run(ctx, cases, allj, 5, refine=2)
    assert ite.ite_ctx_batch_stats(ctx)["solves"] > before["solves"]
    reps_s, _ = _run(ctx, cases, fp32, 5, batched=False, refine=2)
    grid = ed.loggrid(0.01, 20.0, 1.3)[:6]
    for j in fp32:
        reps_a, st_a = _run(ctx, cases, [j], 5, refine=2)
        for a, b in zip(reps_a[j], reps_b[j]):
            for k in KEYS:
                assert a[k] == b[k], (j, k, a[k], b[k])
        assert all(np.array_equal(x, y) for x, y in zip(st_a[j], st_b[j]))
        for a, b in zip(reps_s[j], reps_b[j]):
            assert abs(a["energy"] - b["energy"]) <= 1e-10 * abs(a["energy"]), (j, a["energy"], b["energy"])
            assert (a["matvecs_fp64"], a["matvecs_lo"]) == (b["matvecs_fp64"], b["matvecs_lo"])
        cs = cases[j]
        _, o_reps = omps.evolve_grid(omps.product_state(cs["sp"]), cs["Wo"], grid,
                                     omps.StepOptions(chi_max=cs["chi"], cutoff=1e-10))
        for b, o in zip(reps_b[j], o_reps):
            assert abs(b["energy"] - o.energy) <= 1e-8 * abs(o.energy)

"""Schedules of the batched dock and the autotuner: every kernel variant a
size class can run, forced at full and narrow persistent widths, replays the
oracle's Monte Carlo chains (without BFGS, decision by decision); the
autotuner times the candidates of every class, applies one, remembers it in
the context, and the tuned run stays valid against the oracle."""
import numpy as np
import pytest

from gpu_util import cpu_dof, e_tol
from paper_2506_20043_amd import synth as S

pytestmark = pytest.mark.gpu
KAPPA = 10.0


@pytest.fixture(scope="module")
def pv_ctx():
    import paper_2506_20043_amd as pv
    return pv.Context(0)


@pytest.fixture(scope="module")
def setup(oracle, pv_ctx):
    """The multi-pocket receptor's first pocket with a 30-atom and an
    80-atom ligand (two size classes)."""
    import paper_2506_20043_amd as pv
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    g = np.random.default_rng(41)
    mols = [S.tree_ligand(g, 30, 6), S.tree_ligand(g, 80, 10)]
    b = bxs[0]
    return dict(grids=pv.build_grids(pv_ctx, rx, rt, bxs[:1], penalty_slope=KAPPA),
                ligs=pv.Ligands(pv_ctx, mols),
                og=oracle.Grid.build(rx, rt, b.center.astype(np.float64), b.size.astype(np.float64), b.spacing,
                                     kappa=KAPPA),
                ol=[oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable) for m in mols])


def _replays(oracle, setup, out, jobs, p, chains, step=4):
    from test_gpu_search import _oparams
    cbe = out["chain_best_e"].cpu().numpy().reshape(len(jobs), chains)
    ev = out["chain_evals"].cpu().numpy().reshape(len(jobs), chains)
    same = total = 0
    for j, (lig, _) in enumerate(jobs):
        for c in range(0, chains, step):
            d, e_ref, ne = oracle.mc_chain(setup["ol"][lig], setup["og"], _oparams(oracle, p), j, c)
            same += int(ne == ev[j, c] and abs(cbe[j, c] - e_ref) <= e_tol(e_ref))
            total += 1
    return same, total


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_forced_variants_replay_oracle(oracle, pv_ctx, setup, variant):
    import paper_2506_20043_amd as pv
    jobs = [(0, 0), (0, 0), (1, 0)]
    chains = 24
    p = pv.dock_params(chains=chains, steps=25, seed=91, bfgs_max_iter=0, refine_max_iter=0,
                       flags=pv.PV_DOCK_GRAPH)
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    plan = pv.Plan(pv_ctx, setup["grids"], setup["ligs"], jobs, p)
    assert plan.groups() == 2
    assert plan.schedule(0)["n_jobs"] == 2 and plan.schedule(1)["n_jobs"] == 1
    runs = []
    for width in (0, 5):
        plan.set_schedule(0, variant, width)
        sc = plan.schedule(0)
        assert sc["variant"] == variant and sc["per_cu"] >= 1
        assert sc["workgroups"] == (width if width else min(sc["per_cu"] * n_cu, 2 * chains))
        out = {k: v.clone() for k, v in plan.run().items()}
        same, total = _replays(oracle, setup, out, jobs, p, chains)
        assert same >= total - 2, (variant, width, same, total)
        runs.append(out)
    plan.close()
    # the width changes which wave runs which chain, never a chain's result
    for k in ("chain_best_e", "chain_evals", "chain_best_dof", "job_best_e"):
        assert torch.equal(runs[0][k], runs[1][k]), (variant, k)


def test_autotune_chooses_remembers_and_stays_valid(oracle, pv_ctx, setup):
    import paper_2506_20043_amd as pv
    jobs = [(0, 0), (1, 0), (0, 0)]
    chains = 32
    p = pv.dock_params(chains=chains, steps=40, seed=92, flags=pv.PV_DOCK_GRAPH)
    plan = pv.Plan(pv_ctx, setup["grids"], setup["ligs"], jobs, p)
    before = [plan.schedule(g) for g in range(plan.groups())]
    res = plan.autotune(steps=3, repeats=1)
    for g in range(plan.groups()):
        mine = [r for r in res if r["group"] == g]
        assert len(mine) >= 2 and all(r["cached"] == 0 and r["ms"] > 0 for r in mine)
        # the model's schedule is the first candidate of its class
        assert (mine[0]["variant"], mine[0]["workgroups"]) == (before[g]["variant"], before[g]["workgroups"])
        chosen = [r for r in mine if r["chosen"]]
        assert len(chosen) == 1
        assert chosen[0]["evals_per_s"] == max(r["evals_per_s"] for r in mine)
        sc = plan.schedule(g)
        assert (sc["variant"], sc["workgroups"]) == (chosen[0]["variant"], chosen[0]["workgroups"])
    # the small class may run any of the three variants, the large one only two atoms per lane
    assert {r["variant"] for r in res if r["group"] == 0} == {0, 1, 2}
    assert {r["variant"] for r in res if r["group"] == 1} == {2}
    out = {k: v.cpu().numpy() for k, v in plan.run().items()}
    cbe = out["chain_best_e"].reshape(len(jobs), chains)
    cbd = out["chain_best_dof"].reshape(len(jobs), chains, -1)
    assert np.array_equal(out["job_best_e"], cbe.min(axis=1))
    assert np.all(out["chain_evals"] >= 1 + p.steps)
    for j, (lig, _) in enumerate(jobs):
        L = setup["ol"][lig]
        for c in range(0, chains, 8):
            r = L.score_grad(setup["og"], cpu_dof(cbd[j, c, :L.ndof]))
            slack = 0.01 if r["min_cut"] < 1e-4 else 0.0
            assert abs(r["e"] - cbe[j, c]) <= e_tol(r["e"]) + slack, (j, c, cbe[j, c], r["e"])
    # a second plan of the same shape takes the remembered choice without timing
    plan2 = pv.Plan(pv_ctx, setup["grids"], setup["ligs"], jobs, p)
    res2 = plan2.autotune(steps=3, repeats=1)
    assert len(res2) == plan.groups() and all(r["cached"] == 1 and r["chosen"] == 1 for r in res2)
    for g in range(plan.groups()):
        a, b = plan.schedule(g), plan2.schedule(g)
        assert (a["variant"], a["workgroups"]) == (b["variant"], b["workgroups"])
    o2 = {k: v.cpu().numpy() for k, v in plan2.run().items()}
    assert np.array_equal(o2["chain_best_e"], out["chain_best_e"])
    plan.close()
    plan2.close()


def test_autotune_on_a_prefix_of_a_large_class(pv_ctx, setup):
    """A class with more chains than 8 times the widest candidate is tuned
    on its first jobs only; the tuner still reports every candidate with a
    timing and a rate, sets the fastest, and the tuned run equals a run of
    a fresh plan given the same schedule by hand."""
    import paper_2506_20043_amd as pv
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    chains = 16
    n_jobs = (8 * 8 * n_cu) // chains + 76   # more chains than 8 x (8 waves per CU x the CUs)
    jobs = [(0, 0)] * n_jobs
    p = pv.dock_params(chains=chains, steps=1, seed=97, flags=pv.PV_DOCK_GRAPH)
    plan = pv.Plan(pv_ctx, setup["grids"], setup["ligs"], jobs, p)
    assert plan.groups() == 1
    res = plan.autotune(steps=1, repeats=1)
    assert len(res) >= 2 and all(r["cached"] == 0 and r["ms"] > 0 and r["evals_per_s"] > 0 for r in res)
    chosen = [r for r in res if r["chosen"]]
    assert len(chosen) == 1 and chosen[0]["evals_per_s"] == max(r["evals_per_s"] for r in res)
    sc = plan.schedule(0)
    assert (sc["variant"], sc["workgroups"]) == (chosen[0]["variant"], chosen[0]["workgroups"])
    out = {k: v.cpu().numpy().copy() for k, v in plan.run().items()}
    plan.close()
    assert np.all(np.isfinite(out["job_best_e"])) and np.all(out["job_evals"] > 0)
    ref = pv.Plan(pv_ctx, setup["grids"], setup["ligs"], jobs, p)
    ref.set_schedule(0, sc["variant"], sc["workgroups"])
    o2 = {k: v.cpu().numpy().copy() for k, v in ref.run().items()}
    ref.close()
    for k in ("chain_best_e", "chain_evals", "job_best_e", "job_evals"):
        assert np.array_equal(out[k], o2[k]), k


def test_schedule_rejects(pv_ctx, setup):
    import paper_2506_20043_amd as pv
    p = pv.dock_params(chains=8, steps=5, seed=93)
    plan = pv.Plan(pv_ctx, setup["grids"], setup["ligs"], [(0, 0), (1, 0)], p)
    for args in ((-1, 0, 0), (2, 0, 0), (1, 0, 0), (1, 1, 0), (0, 3, 0), (0, -1, 0), (0, 1, 9), (0, 1, -1)):
        with pytest.raises(pv.PvError):
            plan.set_schedule(*args)
    for kw in ({"steps": 0}, {"repeats": 0}, {"repeats": 101}):
        with pytest.raises(pv.PvError):
            plan.autotune(**kw)
    empty = pv.Plan(pv_ctx, setup["grids"], setup["ligs"], [], p)
    assert empty.groups() == 0 and empty.autotune() == []
    with pytest.raises(pv.PvError):
        empty.schedule(0)
    empty.close()
    plan.close()


def test_job_orders_change_only_the_order(oracle, pv_ctx):
    """PV_DOCK_LARGEST_FIRST hands out each size class's jobs most costly
    ligand first and PV_DOCK_BOX_ORDER groups them by box; every chain still
    depends on (seed, job, chain) alone, so all outputs equal the job-order
    plan's bit for bit, alone and combined.  Unknown flag bits are
    rejected."""
    import paper_2506_20043_amd as pv
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    g = np.random.default_rng(43)
    mols = [S.tree_ligand(g, n, t) for n, t in ((12, 2), (50, 7), (30, 4), (100, 12), (80, 9), (20, 3))]
    grids = pv.build_grids(pv_ctx, rx, rt, bxs[:2], penalty_slope=KAPPA)
    ligs = pv.Ligands(pv_ctx, mols)
    jobs = [(i % len(mols), (i // 3) % 2) for i in range(14)]
    outs = []
    for flag in (0, pv.PV_DOCK_LARGEST_FIRST, pv.PV_DOCK_BOX_ORDER, pv.PV_DOCK_LARGEST_FIRST | pv.PV_DOCK_BOX_ORDER):
        p = pv.dock_params(chains=16, steps=15, seed=94, flags=pv.PV_DOCK_GRAPH | pv.PV_DOCK_TIMESTAMPS | flag)
        plan = pv.Plan(pv_ctx, grids, ligs, jobs, p)
        assert plan.groups() == 2
        outs.append({k: v.cpu().numpy().copy() for k, v in plan.run().items()})
        plan.close()
    for o in outs[1:]:
        for k in outs[0]:
            if k in ("job_t_start", "job_t_end"):
                continue
            assert np.array_equal(outs[0][k], o[k]), k
        assert np.all(o["job_t_end"] >= o["job_t_start"])
    with pytest.raises(pv.PvError):
        pv.Plan(pv_ctx, grids, ligs, jobs, pv.dock_params(chains=4, steps=2, seed=1, flags=32))


def test_ligands_without_intra_pairs(oracle, pv_ctx, setup):
    """Ligands of one, two and three atoms have no intra pair (the pair loop
    runs no pass): under each kernel variant, chains without BFGS replay the
    oracle and full docks give chain bests that re-score to their energies
    (the variants sum forces in different orders, so their BFGS chains may
    part ways)."""
    import paper_2506_20043_amd as pv
    from test_gpu_search import _oparams
    one = S.Molecule(np.zeros((1, 3)), np.array([0], np.int32), np.zeros((0, 2), np.int32), np.zeros(0, np.uint8))
    two = S.Molecule(np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.0]]), np.array([3, 5], np.int32),
                     np.array([[0, 1]], np.int32), np.zeros(1, np.uint8))
    three = S.Molecule(np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.0], [2.0, 1.4, 0.0]]), np.array([0, 2, 6], np.int32),
                       np.array([[0, 1], [1, 2]], np.int32), np.zeros(2, np.uint8))
    mols = [one, two, three]
    ligs = pv.Ligands(pv_ctx, mols)
    assert [ligs.info(i)[3] for i in range(3)] == [0, 0, 0]
    ol = [oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable) for m in mols]
    jobs = [(0, 0), (1, 0), (2, 0)]
    chains = 16
    p0 = pv.dock_params(chains=chains, steps=15, seed=95, bfgs_max_iter=0, refine_max_iter=0)
    p = pv.dock_params(chains=chains, steps=8, seed=96)
    outs = []
    for variant in (0, 1, 2):
        plan = pv.Plan(pv_ctx, setup["grids"], ligs, jobs, p0)
        plan.set_schedule(0, variant, 0)
        o = {k: v.cpu().numpy().copy() for k, v in plan.run().items()}
        plan.close()
        cbe, ev = o["chain_best_e"].reshape(3, chains), o["chain_evals"].reshape(3, chains)
        same = total = 0
        for j, (lig, _) in enumerate(jobs):
            for c in range(0, chains, 4):
                d, e_ref, ne = oracle.mc_chain(ol[lig], setup["og"], _oparams(oracle, p0), j, c)
                same += int(ne == ev[j, c] and abs(cbe[j, c] - e_ref) <= e_tol(e_ref))
                total += 1
        assert same >= total - 1, (variant, same, total)
        plan = pv.Plan(pv_ctx, setup["grids"], ligs, jobs, p)
        plan.set_schedule(0, variant, 0)
        outs.append({k: v.cpu().numpy().copy() for k, v in plan.run().items()})
        plan.close()
    for variant, o in enumerate(outs):
        assert np.all(o["chain_evals"] >= 1 + p.steps) and np.all(np.isfinite(o["chain_best_e"]))
        cbd = o["chain_best_dof"].reshape(3, chains, -1)
        cbe = o["chain_best_e"].reshape(3, chains)
        for j, (lig, _) in enumerate(jobs):
            L = ol[lig]
            for c in range(0, chains, 3):
                r = L.score_grad(setup["og"], cpu_dof(cbd[j, c, :L.ndof]))
                slack = 0.01 if r["min_cut"] < 1e-4 else 0.0
                assert abs(r["e"] - cbe[j, c]) <= e_tol(r["e"]) + slack, (variant, j, c, cbe[j, c], r["e"])

"""Per-chain and per-job statuses of a dock, each forced from the host: an
evaluation budget that every chain reaches, a box too small for the ligand
(best poses outside it) and an infinite out-of-box slope (energies that are
not finite).  A failing job never stops the others."""
import numpy as np
import pytest

from gpu_util import cpu_dof
from paper_2506_20043_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2506_20043_amd as pv
    g = np.random.default_rng(61)
    rx, rt = S.receptor(g, 1200, 30.0)
    mols = [S.tree_ligand(g, 20, 4), S.tree_ligand(g, 70, 8)]
    return pv, pv.Context(0), rx, rt, mols


def test_budget_stops_chains(setup):
    pv, ctx, rx, rt, mols = setup
    box = S.Box(np.full(3, 15.0, np.float32), np.full(3, 18.0, np.float32), 0.375)
    grids = pv.build_grids(ctx, rx, rt, [box], penalty_slope=10.0)
    ligs = pv.Ligands(ctx, mols)
    jobs = [(0, 0), (1, 0)]
    free = pv.dock(ctx, grids, ligs, jobs, pv.dock_params(chains=8, steps=40, seed=3))
    ev_free = free["chain_evals"].cpu().numpy()
    assert np.all((free["chain_status"].cpu().numpy() & pv.PV_JOB_BUDGET) == 0)
    budget = 60
    res = pv.dock(ctx, grids, ligs, jobs, pv.dock_params(chains=8, steps=40, seed=3, max_evals=budget))
    ev = res["chain_evals"].cpu().numpy()
    cst = res["chain_status"].cpu().numpy()
    assert np.all(ev >= budget) and np.all(ev < ev_free)
    assert np.all((cst & pv.PV_JOB_BUDGET) != 0)
    assert np.all((res["job_status"].cpu().numpy() & pv.PV_JOB_BUDGET) != 0)
    assert np.all(np.isfinite(res["job_best_e"].cpu().numpy()))
    # a budget above what the chains need changes nothing
    res2 = pv.dock(ctx, grids, ligs, jobs, pv.dock_params(chains=8, steps=40, seed=3, max_evals=10 ** 9))
    assert np.array_equal(res2["chain_best_e"].cpu().numpy(), free["chain_best_e"].cpu().numpy())
    assert np.all((res2["chain_status"].cpu().numpy() & pv.PV_JOB_BUDGET) == 0)
    with pytest.raises(pv.PvError, match="max_evals"):
        pv.dock(ctx, grids, ligs, jobs, pv.dock_params(chains=2, steps=1, seed=3, max_evals=-1))


def test_outside_flag_matches_best_pose(oracle, setup):
    """A 1.5 A box cannot hold a 20-atom ligand, so every chain's best pose
    is flagged; in an 18 A box the flag of each chain equals the oracle's
    placement of its best pose (some atom beyond the lattice box)."""
    pv, ctx, rx, rt, mols = setup
    small = S.Box(np.full(3, 15.0, np.float32), np.full(3, 1.5, np.float32), 0.375)
    big = S.Box(np.full(3, 15.0, np.float32), np.full(3, 18.0, np.float32), 0.375)
    grids = pv.build_grids(ctx, rx, rt, [small, big], penalty_slope=10.0)
    ligs = pv.Ligands(ctx, mols[:1])
    res = pv.dock(ctx, grids, ligs, [(0, 0), (0, 1)], pv.dock_params(chains=16, steps=30, seed=4))
    cst = res["chain_status"].cpu().numpy().reshape(2, 16)
    jst = res["job_status"].cpu().numpy()
    assert np.all((cst[0] & pv.PV_JOB_OUTSIDE) != 0) and (jst[0] & pv.PV_JOB_OUTSIDE) != 0
    L = oracle.Ligand(mols[0].xyz, mols[0].types, mols[0].bonds, mols[0].rotatable)
    dims, org = grids.info(1)
    lo = org.astype(np.float64)
    hi = lo + 0.375 * (dims.astype(np.float64) - 1)
    dof = res["chain_best_dof"].cpu().numpy().reshape(2, 16, -1)
    checked = 0
    for c in range(16):
        x = L.fk(cpu_dof(dof[1, c, :L.ndof]))
        margin = np.minimum(x - lo, hi - x)
        if np.abs(margin).min() < 1e-3:
            continue   # an atom within rounding of a face
        assert bool(cst[1, c] & pv.PV_JOB_OUTSIDE) == bool(np.any(margin < 0)), c
        checked += 1
    assert checked >= 10   # best poses often rest an atom on a face, where the penalty starts
    best = int(res["job_best_chain"][1].item())
    assert bool(jst[1] & pv.PV_JOB_OUTSIDE) == bool(cst[1, best] & pv.PV_JOB_OUTSIDE)


def test_nonfinite_energy_flagged_and_isolated(setup):
    """An out-of-box slope near the largest binary32 value (3e38 kcal/mol/A,
    finite, so accepted) in a box too small for the ligand makes every
    energy overflow to infinity: the job is flagged and the other job, in a
    normal box of the same grids, is not."""
    pv, ctx, rx, rt, mols = setup
    small = S.Box(np.full(3, 15.0, np.float32), np.full(3, 0.375, np.float32), 0.375)
    big = S.Box(np.full(3, 15.0, np.float32), np.full(3, 18.0, np.float32), 0.375)
    grids = pv.build_grids(ctx, rx, rt, [small, big], penalty_slope=3.0e38)
    ligs = pv.Ligands(ctx, mols[:1])
    res = pv.dock(ctx, grids, ligs, [(0, 0), (0, 1)], pv.dock_params(chains=32, steps=10, seed=5))
    jst = res["job_status"].cpu().numpy()
    jbe = res["job_best_e"].cpu().numpy()
    assert (jst[0] & pv.PV_JOB_NONFINITE) != 0 and not np.isfinite(jbe[0])
    # the normal box: chains that start with atoms outside have infinite
    # energies, the others reach finite poses inside
    assert np.isfinite(jbe[1]) and (jst[1] & pv.PV_JOB_NONFINITE) == 0

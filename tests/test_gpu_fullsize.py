"""The multi-pocket dock at full size, in the launch the benchmark times (5
pockets of 24 A, one 35-atom ligand, 256 chains x 1,000 Monte Carlo steps
with RILC-BFGS, one persistent launch replayed as a graph; Supplementary
Algorithm 2).  Chains with BFGS are chaotic, so the oracle checks what it can
compute one chain at a time: the per-job reductions exactly, every sampled
chain's best pose re-scored to its energy and no worse than the chain's
initial pose, and the distribution of chain bests of one pocket against the
oracle's own chains on the same Philox streams."""
import numpy as np
import pytest
from scipy import stats

from gpu_util import cpu_dof, e_tol
from paper_2506_20043_amd import synth as S

pytestmark = pytest.mark.gpu
KAPPA = 10.0


def test_multipocket_dock_full_size(oracle):
    import paper_2506_20043_amd as pv
    from test_gpu_search import _oparams
    cfg = S.CONFIGS["c2"]
    rx, rt, bxs = S.make_receptor(cfg)
    mols = S.make_ligands(cfg)
    seed = S.philox_seed(cfg)
    ctx = pv.Context(0)
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=KAPPA)
    ligs = pv.Ligands(ctx, mols)
    jobs = [(0, b) for b in range(len(bxs))]
    chains, steps = 256, 1000
    p = pv.dock_params(chains=chains, steps=steps, seed=seed, flags=pv.PV_DOCK_GRAPH)
    plan = pv.Plan(ctx, grids, ligs, jobs, p)
    out = {k: v.cpu().numpy().copy() for k, v in plan.run().items()}
    plan.close()
    nj = len(jobs)
    cbe = out["chain_best_e"].reshape(nj, chains)
    cev = out["chain_evals"].reshape(nj, chains)
    cbd = out["chain_best_dof"].reshape(nj, chains, -1)
    # per-job reductions: the lowest chain best, ties to the lowest chain
    assert np.array_equal(out["job_best_e"], cbe.min(axis=1))
    assert np.array_equal(out["job_best_chain"], np.argmin(cbe, axis=1))
    assert np.array_equal(out["job_evals"], cev.sum(axis=1))
    assert np.all(out["job_status"] == 0)
    # every step optimises at least once, after the one evaluation of the start
    assert np.all(cev >= 1 + steps)
    assert np.all(np.isfinite(cbe))
    L = oracle.Ligand(mols[0].xyz, mols[0].types, mols[0].bonds, mols[0].rotatable)
    G = [oracle.Grid.build(rx, rt, b.center.astype(np.float64), b.size.astype(np.float64), b.spacing, kappa=KAPPA)
         for b in bxs]
    rng = np.random.default_rng(7)
    for j in range(nj):
        for c in rng.choice(chains, 8, replace=False):
            d = cpu_dof(cbd[j, c, :L.ndof])
            assert np.linalg.norm(d[3:7]) == pytest.approx(1.0, abs=1e-5)
            r = L.score_grad(G[j], d)
            slack = 0.01 if r["min_cut"] < 1e-4 else 0.0
            assert abs(r["e"] - cbe[j, c]) <= e_tol(r["e"]) + slack, (j, c, cbe[j, c], r["e"])
            e0 = L.score_grad(G[j], oracle.init_pose(L, G[j], seed, j, int(c)))["e"]
            assert cbe[j, c] <= e0 + e_tol(e0), (j, c, cbe[j, c], e0)
    # the oracle's first 24 chains of pocket 0 (the same Philox streams)
    p24 = pv.dock_params(chains=24, steps=steps, seed=seed)
    ref = oracle.dock([L], [G[0]], [(0, 0)], _oparams(oracle, p24))
    oe = ref["chain_best_e"][0]
    assert len(oe) == 24
    ks = stats.ks_2samp(cbe[0], oe)
    assert ks.pvalue > 0.01, (ks, np.median(cbe[0]), np.median(oe))

"""GPU parity of the first-order consistency check (Eqs. qvina_eq_4 and
qvina_eq_5) gating the Monte Carlo step's BFGS: chains without BFGS replay
the oracle's check decisions and Metropolis moves, and full docks with the
check match the oracle's distributions of chain bests and evaluation
counts while spending fewer evaluations than without it."""
import numpy as np
import pytest
from scipy import stats

from gpu_util import cpu_dof, e_tol
from test_gpu_search import KAPPA, _oparams, _params, tiny, pv_ctx  # noqa: F401  (fixtures)

pytestmark = pytest.mark.gpu


def test_check_without_bfgs_replays_oracle(oracle, pv_ctx, tiny):
    """BFGS capped at 0 iterations: every step is mutate, evaluate, check,
    then either nothing or a Metropolis test, so the same Philox draws give
    the same trajectory unless a sign or a Metropolis test lands within
    rounding of its threshold (rare)."""
    import paper_2506_20043_amd as pv
    p = _params(pv, chains=64, steps=40, seed=tiny["seed"] + 2, bfgs_max_iter=0, refine_max_iter=0, consistency=1)
    res = pv.dock(pv_ctx, tiny["grids"], tiny["ligs"], [(0, 0)], p)
    cbd = res["chain_best_dof"].cpu().numpy()
    cbe = res["chain_best_e"].cpu().numpy()
    ev = res["chain_evals"].cpu().numpy()
    L, G = tiny["ol"], tiny["og"]
    same = 0
    for c in range(64):
        d, e, ne = oracle.mc_chain(L, G, _oparams(oracle, p), 0, c)
        if ne == ev[c] and abs(cbe[c] - e) <= e_tol(e) and np.abs(cbd[c, :3] - d[:3]).max() < 1e-3:
            same += 1
    assert same >= 58, same


def test_check_dock_statistics(oracle, pv_ctx, tiny):
    import paper_2506_20043_amd as pv
    p = _params(pv, chains=64, steps=200, seed=tiny["seed"], consistency=1)
    res = pv.dock(pv_ctx, tiny["grids"], tiny["ligs"], [(0, 0)], p)
    cbd = res["chain_best_dof"].cpu().numpy()
    cbe = res["chain_best_e"].cpu().numpy()
    ev = res["chain_evals"].cpu().numpy()
    L, G = tiny["ol"], tiny["og"]
    for c in range(64):
        r = L.score_grad(G, cpu_dof(cbd[c, :L.ndof]))
        assert abs(r["e"] - cbe[c]) <= e_tol(r["e"]) + 0.01, (c, cbe[c], r["e"])
    ref = oracle.dock([L], [G], [(0, 0)], _oparams(oracle, p))
    ks = stats.ks_2samp(cbe, ref["chain_best_e"][0])
    assert ks.pvalue > 0.01, (ks, np.median(cbe), np.median(ref["chain_best_e"][0]))
    ks = stats.ks_2samp(ev, ref["chain_evals"][0])
    assert ks.pvalue > 0.01, (ks, ev.mean(), ref["chain_evals"][0].mean())
    # the same chains without the check spend more evaluations
    p0 = _params(pv, chains=64, steps=200, seed=tiny["seed"])
    ev0 = pv.dock(pv_ctx, tiny["grids"], tiny["ligs"], [(0, 0)], p0)["chain_evals"].cpu().numpy()
    assert ev.sum() < 0.9 * ev0.sum(), (ev.sum(), ev0.sum())


def test_check_rejects(pv_ctx, tiny):
    import paper_2506_20043_amd as pv
    with pytest.raises(pv.PvError):
        pv.Plan(pv_ctx, tiny["grids"], tiny["ligs"], [(0, 0)], _params(pv, consistency=2))

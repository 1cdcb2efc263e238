"""The allocation-free dock entry point (pv_dock_noalloc) against pv_dock,
through the C ABI: the same jobs give the same outputs bit for bit, on two
calls in a row (the second smaller, with only per-job outputs, so the
per-chain arrays come from the library's static scratch), and sizes beyond
the scratch are rejected."""
import numpy as np
import pytest

from paper_2506_20043_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2506_20043_amd as pv
    g = np.random.default_rng(91)
    rx, rt = S.receptor(g, 900, 30.0)
    boxes = [S.Box(np.array([12.0, 13.0, 14.0], np.float32), np.full(3, 14.0, np.float32), 0.375),
             S.Box(np.array([17.0, 15.0, 13.0], np.float32), np.full(3, 16.0, np.float32), 0.375)]
    # both size classes: ligands of at most 64 atoms and larger ones
    mols = [S.tree_ligand(g, n, t) for n, t in ((20, 4), (70, 9), (35, 6), (12, 2), (66, 5))]
    ctx = pv.Context(0)
    grids = pv.build_grids(ctx, rx, rt, boxes, penalty_slope=10.0)
    ligs = pv.Ligands(ctx, mols)
    return pv, ctx, grids, ligs


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def test_noalloc_matches_pv_dock_twice(setup):
    pv, ctx, grids, ligs = setup
    p = pv.dock_params(chains=8, steps=12, seed=4242)
    jobs1 = [(l, b) for l in range(5) for b in range(2)]
    print("noalloc call 1: %d jobs x %d chains" % (len(jobs1), p.chains), flush=True)
    want1 = _np(pv.dock_call(ctx, grids, ligs, jobs1, p))
    got1 = _np(pv.dock_noalloc(ctx, grids, ligs, jobs1, p))
    assert set(got1) == set(want1)
    for k in want1:
        assert np.array_equal(got1[k], want1[k]), k
    assert np.all((got1["job_status"] & pv.PV_JOB_NONFINITE) == 0)
    # a second, smaller call: per-job outputs only, the chains' bests and
    # counts in the scratch, which still holds the first call's contents
    jobs2 = [(4, 1), (0, 0), (1, 1)]
    print("noalloc call 2: %d jobs, per-job outputs" % len(jobs2), flush=True)
    want2 = _np(pv.dock_call(ctx, grids, ligs, jobs2, p))
    got2 = _np(pv.dock_noalloc(ctx, grids, ligs, jobs2, p, chain_outputs=False))
    for k in ("job_best_e", "job_best_chain", "job_evals", "job_status"):
        assert np.array_equal(got2[k], want2[k]), k


def test_noalloc_rejects(setup):
    pv, ctx, grids, ligs = setup
    p = pv.dock_params(chains=64, steps=1, seed=1)
    too_many = [(0, 0)] * (pv.NOALLOC_MAX_CHAINS // 64 + 1)
    with pytest.raises(pv.PvError, match="MAX_CHAINS"):
        pv.dock_noalloc(ctx, grids, ligs, too_many, p, chain_outputs=False)
    with pytest.raises(pv.PvError, match="MAX_JOBS"):
        pv.dock_noalloc(ctx, grids, ligs, [(0, 0)] * (pv.NOALLOC_MAX_JOBS + 1),
                        pv.dock_params(chains=1, steps=1, seed=1), chain_outputs=False)
    with pytest.raises(pv.PvError, match="PV_DOCK_TIMESTAMPS"):
        pv.dock_noalloc(ctx, grids, ligs, [(0, 0)], pv.dock_params(chains=2, steps=1, seed=1, flags=pv.PV_DOCK_GRAPH))
    with pytest.raises(pv.PvError, match="unknown box"):
        pv.dock_noalloc(ctx, grids, ligs, [(0, 7)], pv.dock_params(chains=2, steps=1, seed=1))
    # a valid call after the rejections still works
    out = _np(pv.dock_noalloc(ctx, grids, ligs, [(3, 0)], pv.dock_params(chains=4, steps=3, seed=5)))
    assert (out["job_status"][0] & pv.PV_JOB_NONFINITE) == 0

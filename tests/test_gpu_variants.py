"""GPU parity of the three kernel variants: intra forces through LDS slots,
through the per-pair coefficient gather, and two atoms per lane.  The variant
follows from the launch size and the ligand size (slots while the CUs can
still hold the launch's waves); each one is checked against the oracle on the
same poses and chains (Eq. qvina_eq_3, Supplementary Algorithm 2)."""
import numpy as np
import pytest

from gpu_util import cpu_dof, e_tol
from paper_2506_20043_amd import synth as S
from test_gpu_score import KAPPA, Setup, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pv_ctx():
    import paper_2506_20043_amd as pv
    return pv.Context(0)


@pytest.fixture(scope="module")
def big(oracle, pv_ctx):
    """Two ligands near the one-atom-per-lane limit in a 24 A pocket of the
    multi-pocket receptor: their force slots take ~60 KB of LDS."""
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    g = np.random.default_rng(77)
    mols = [S.tree_ligand(g, 60, 12), S.tree_ligand(g, 58, 9)]
    return Setup(oracle, pv_ctx, rx, rt, bxs[:1], mols)


def _poses(st, g, lig, B):
    lo, hi = st.lohi(0)
    dof = np.zeros((B, st.ligs.dof_stride), np.float32)
    for b in range(B):
        nt = st.ol[lig[b]].n_tors
        dof[b, :7 + nt] = S.poses(g, 1, lo + 2, hi - 2, nt)[0]
    return dof


def test_variant_selection(pv_ctx, big):
    import paper_2506_20043_amd as pv
    v, lds, occ = pv.launch_info(pv_ctx, big.ligs, pv.KIND_SCORE, 16)
    assert v == pv.VARIANT_SLOTS and lds > 48 * 1024 and occ >= 1
    v, lds_g, occ_g = pv.launch_info(pv_ctx, big.ligs, pv.KIND_SCORE, 16384)
    assert v == pv.VARIANT_GATHER and lds_g < lds and occ_g > occ
    assert pv.launch_info(pv_ctx, big.ligs, pv.KIND_DOCK, 4096)[0] == pv.VARIANT_GATHER
    assert pv.launch_info(pv_ctx, big.ligs, pv.KIND_LOCAL_OPT, 16)[0] == pv.VARIANT_SLOTS
    g = np.random.default_rng(5)
    huge = pv.Ligands(pv_ctx, [S.tree_ligand(g, 100, 20)])
    assert pv.launch_info(pv_ctx, huge, pv.KIND_SCORE, 16)[0] == pv.VARIANT_GATHER2
    # the multi-pocket dock (5 pockets x 256 chains of a 35-atom ligand) keeps the slots
    cfg = S.CONFIGS["multi_pocket"]
    lc2 = pv.Ligands(pv_ctx, S.make_ligands(cfg))
    assert pv.launch_info(pv_ctx, lc2, pv.KIND_DOCK, 5 * 256)[0] == pv.VARIANT_SLOTS
    with pytest.raises(pv.PvError):
        pv.launch_info(pv_ctx, big.ligs, 7, 16)


def test_slots_and_gather_score_agree_with_oracle(oracle, pv_ctx, big):
    """The same 64 poses scored in a small launch (slots) and at the head of
    a large one (gather); both match the oracle, and a sample of the rest of
    the large launch does too."""
    import paper_2506_20043_amd as pv
    g = np.random.default_rng(11)
    B = 8192
    assert pv.launch_info(pv_ctx, big.ligs, pv.KIND_SCORE, B)[0] == pv.VARIANT_GATHER
    assert pv.launch_info(pv_ctx, big.ligs, pv.KIND_SCORE, 64)[0] == pv.VARIANT_SLOTS
    lig = np.tile(np.array([0, 1], np.int32), B // 2)
    box = np.zeros(B, np.int32)
    dof = _poses(big, g, lig, B)
    small = pv.score_grad(pv_ctx, big.grids, big.ligs, lig[:64], box[:64], dof[:64], parts=True)
    large = pv.score_grad(pv_ctx, big.grids, big.ligs, lig, box, dof, parts=True)
    compare(big, lig, box, dof, small, range(64))
    idx = np.concatenate([np.arange(64), np.random.default_rng(3).choice(np.arange(64, B), 96, replace=False)])
    compare(big, lig, box, dof, large, idx)
    es, el = small["energy"].cpu().numpy(), large["energy"].cpu().numpy()[:64]
    assert np.all(np.abs(es - el) <= e_tol(es))


def test_gather_dock_replays_oracle(oracle, pv_ctx, big):
    """Monte Carlo without BFGS on a 60-atom ligand with 2,048 chains (the
    gather variant) replays the oracle's chains decision by decision, in the
    batched and in the plain form."""
    import paper_2506_20043_amd as pv
    from test_gpu_search import _oparams
    chains = 2048
    assert pv.launch_info(pv_ctx, big.ligs, pv.KIND_DOCK, chains)[0] == pv.VARIANT_GATHER
    p = pv.dock_params(chains=chains, steps=20, seed=4242, bfgs_max_iter=0, refine_max_iter=0)
    plan = pv.Plan(pv_ctx, big.grids, big.ligs, [(0, 0)], p)
    out = {k: v.cpu().numpy() for k, v in plan.run().items()}
    plain = {k: v.cpu().numpy() for k, v in plan.run(plain=True).items()}
    plan.close()
    assert np.array_equal(out["chain_evals"], plain["chain_evals"])
    assert np.array_equal(out["chain_best_e"], plain["chain_best_e"])
    L, G = big.ol[0], big.og[0]
    sample = np.random.default_rng(9).choice(chains, 32, replace=False)
    same = 0
    for c in sample:
        d, e, ne = oracle.mc_chain(L, G, _oparams(oracle, p), 0, int(c))
        if (ne == out["chain_evals"][c] and abs(out["chain_best_e"][c] - e) <= e_tol(e)
                and np.abs(out["chain_best_dof"][c, :3] - d[:3]).max() < 1e-3):
            same += 1
    assert same >= 29, same


def test_gather_local_opt_is_valid(oracle, pv_ctx, big):
    """BFGS from 4,096 starts (gather variant): every end point's energy is
    at most its start's, and re-scored by the oracle it matches the returned
    energy."""
    import paper_2506_20043_amd as pv
    g = np.random.default_rng(21)
    B = 4096
    assert pv.launch_info(pv_ctx, big.ligs, pv.KIND_LOCAL_OPT, B)[0] == pv.VARIANT_GATHER
    lig = np.tile(np.array([0, 1], np.int32), B // 2)
    box = np.zeros(B, np.int32)
    dof = _poses(big, g, lig, B)
    start = pv.score_grad(pv_ctx, big.grids, big.ligs, lig, box, dof)["energy"].cpu().numpy()
    out, e, ne = pv.local_opt(pv_ctx, big.grids, big.ligs, lig, box, dof, pv.dock_params())
    e, out, ne = e.cpu().numpy(), out.cpu().numpy(), ne.cpu().numpy()
    assert np.all(np.isfinite(e)) and np.all(ne >= 1)
    assert np.all(e <= start + e_tol(start))
    for b in np.random.default_rng(4).choice(B, 48, replace=False):
        L = big.ol[lig[b]]
        r = L.score_grad(big.og[0], cpu_dof(out[b, :L.ndof]))
        assert abs(r["e"] - e[b]) <= e_tol(r["e"]) + (0.01 if r["min_cut"] < 1e-4 else 0.0), (b, r["e"], e[b])


def test_mixed_size_jobs(oracle, pv_ctx, big):
    """Jobs of a 30-atom and an 80-atom ligand in one plan run as two size
    classes (one and two atoms per lane): the batched launch matches the
    plain one exactly, every job's outputs land at its own index, and
    without BFGS both ligands' chains replay the oracle."""
    import paper_2506_20043_amd as pv
    from test_gpu_search import _oparams
    g = np.random.default_rng(13)
    small, large = S.tree_ligand(g, 30, 6), S.tree_ligand(g, 80, 10)
    ligs = pv.Ligands(pv_ctx, [small, large])
    jobs = [(0, 0), (1, 0), (1, 0), (0, 0), (1, 0)]
    p = pv.dock_params(chains=32, steps=25, seed=777, flags=pv.PV_DOCK_GRAPH | pv.PV_DOCK_TIMESTAMPS)
    plan = pv.Plan(pv_ctx, big.grids, ligs, jobs, p)
    bat = {k: v.cpu().numpy().copy() for k, v in plan.run().items()}
    pla = {k: v.cpu().numpy().copy() for k, v in plan.run(plain=True).items()}
    plan.close()
    for k in ("chain_best_e", "chain_evals", "chain_best_dof", "job_best_e", "job_best_chain"):
        assert np.array_equal(bat[k], pla[k]), k
    assert np.all(bat["job_t_end"] >= bat["job_t_start"]) and np.all(bat["job_t_start"] > 0)
    # different ligands' jobs differ, same ligand's jobs draw their own streams
    e = bat["chain_best_e"].reshape(5, 32)
    assert not np.array_equal(e[0], e[3]) and not np.array_equal(e[1], e[2])
    p0 = pv.dock_params(chains=32, steps=20, seed=778, bfgs_max_iter=0, refine_max_iter=0)
    res = pv.dock(pv_ctx, big.grids, ligs, jobs, p0)
    cbe = res["chain_best_e"].cpu().numpy().reshape(5, 32)
    ev = res["chain_evals"].cpu().numpy().reshape(5, 32)
    ol = [oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable) for m in (small, large)]
    same = total = 0
    for j, (lig, _) in enumerate(jobs):
        for c in range(0, 32, 4):
            d, e_ref, ne = oracle.mc_chain(ol[lig], big.og[0], _oparams(oracle, p0), j, c)
            same += int(ne == ev[j, c] and abs(cbe[j, c] - e_ref) <= e_tol(e_ref))
            total += 1
    assert same >= total - 3, (same, total)


def _seeded_ligand(seed):
    """A tree ligand drawn the way the boundary search drew it: with seeds
    37, 241, 705 and 452 it has 256, 255, 257 and 512 intra pairs."""
    g = np.random.default_rng(seed)
    n = int(g.integers(24, 46))
    nt = int(g.integers(3, 12))
    return S.tree_ligand(g, n, nt)


def test_slot_records_at_pass_boundaries(oracle, pv_ctx):
    """The slot layout pads its pair records to whole passes of 256: ligands
    with 0, 255, 256, 257 and 512 intra pairs and one of 64 atoms (the far
    point right after the last atom) score like the oracle in the slot
    variant, and like the gather variant of a large launch."""
    import paper_2506_20043_amd as pv
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    g = np.random.default_rng(31)
    mols = [S.tree_ligand(g, 12, 0)] + [_seeded_ligand(s) for s in (241, 37, 705, 452)]
    mols.append(S.tree_ligand(np.random.default_rng(1000), 64, 10))
    st = Setup(oracle, pv_ctx, rx, rt, bxs[:1], mols)
    counts = [st.ol[k].n_pairs for k in range(len(mols))]
    assert counts[:5] == [0, 255, 256, 257, 512] and st.ol[5].n_atoms == 64, counts
    per = 24
    lig = np.repeat(np.arange(len(mols), dtype=np.int32), per)
    B = len(lig)
    box = np.zeros(B, np.int32)
    dof = _poses(st, g, lig, B)
    assert pv.launch_info(pv_ctx, st.ligs, pv.KIND_SCORE, B)[0] == pv.VARIANT_SLOTS
    out = pv.score_grad(pv_ctx, st.grids, st.ligs, lig, box, dof, parts=True)
    compare(st, lig, box, dof, out, range(B))
    # the same poses at the head of a launch large enough for the gather
    reps = 8192 // B + 1
    big_lig, big_box, big_dof = np.tile(lig, reps), np.tile(box, reps), np.tile(dof, (reps, 1))
    assert pv.launch_info(pv_ctx, st.ligs, pv.KIND_SCORE, len(big_lig))[0] != pv.VARIANT_SLOTS
    big = pv.score_grad(pv_ctx, st.grids, st.ligs, big_lig, big_box, big_dof)
    es, eb = out["energy"].cpu().numpy(), big["energy"].cpu().numpy()[:B]
    assert np.all(np.abs(es - eb) <= e_tol(es))


def test_max_size_ligand_dock(oracle, pv_ctx, big):
    """The largest ligand the library takes (128 atoms, 32 torsions: 38
    tangent components, so the BFGS wave sums span three rows): without BFGS
    sampled chains replay the oracle; with BFGS the batched and plain
    launches agree exactly, every chain best re-scores to its energy under the
    oracle, and local optimisation never ends above its start."""
    import paper_2506_20043_amd as pv
    from test_gpu_search import _oparams
    m = S.tree_ligand(np.random.default_rng(128), 128, 32)
    assert m.n_tors == 32
    ligs = pv.Ligands(pv_ctx, [m])
    L = oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    assert L.ndof == 39
    G = big.og[0]
    assert pv.launch_info(pv_ctx, ligs, pv.KIND_DOCK, 16)[0] == pv.VARIANT_GATHER2
    p0 = pv.dock_params(chains=16, steps=12, seed=1281, bfgs_max_iter=0, refine_max_iter=0)
    res = pv.dock(pv_ctx, big.grids, ligs, [(0, 0)], p0)
    cbe, ev = res["chain_best_e"].cpu().numpy(), res["chain_evals"].cpu().numpy()
    same = 0
    for c in range(0, 16, 2):
        d, e_ref, ne = oracle.mc_chain(L, G, _oparams(oracle, p0), 0, c)
        same += int(ne == ev[c] and abs(cbe[c] - e_ref) <= e_tol(e_ref))
    assert same >= 7, same
    p = pv.dock_params(chains=16, steps=6, seed=1282, flags=pv.PV_DOCK_GRAPH)
    plan = pv.Plan(pv_ctx, big.grids, ligs, [(0, 0)], p)
    bat = {k: v.cpu().numpy().copy() for k, v in plan.run().items()}
    pla = {k: v.cpu().numpy().copy() for k, v in plan.run(plain=True).items()}
    plan.close()
    for k in ("chain_best_e", "chain_evals", "chain_best_dof", "job_best_e"):
        assert np.array_equal(bat[k], pla[k]), k
    assert np.all(bat["chain_evals"] >= 1 + p.steps) and np.all(np.isfinite(bat["chain_best_e"]))
    for c in range(16):
        r = L.score_grad(G, cpu_dof(bat["chain_best_dof"][c, :L.ndof]))
        slack = 0.01 if r["min_cut"] < 1e-4 else 0.0
        assert abs(r["e"] - bat["chain_best_e"][c]) <= e_tol(r["e"]) + slack, (c, r["e"], bat["chain_best_e"][c])
    lig = np.zeros(8, np.int32)
    box = np.zeros(8, np.int32)
    dims, org = big.grids.info(0)
    g = np.random.default_rng(129)
    dof = S.poses(g, 8, org + 3.0, org + 0.375 * (dims - 1) - 3.0, 32).astype(np.float32)
    start = pv.score_grad(pv_ctx, big.grids, ligs, lig, box, dof)["energy"].cpu().numpy()
    out, e, ne = pv.local_opt(pv_ctx, big.grids, ligs, lig, box, dof, pv.dock_params())
    e = e.cpu().numpy()
    assert np.all(np.isfinite(e)) and np.all(e <= start + e_tol(start))

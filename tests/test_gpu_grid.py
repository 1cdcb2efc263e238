"""GPU parity of the grid-map kernel ("Kernel 1" grid cache) against the
oracle's maps: every value of the tiny configuration, sampled values of the
five 24 A pockets at full size, and ragged or degenerate boxes."""
import numpy as np
import pytest

from paper_2506_20043_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pv_ctx():
    import paper_2506_20043_amd as pv
    return pv.Context(0)


def _gpu_maps(pv_ctx, rx, rt, boxes):
    import paper_2506_20043_amd as pv
    grids = pv.build_grids(pv_ctx, rx, rt, boxes)
    return grids, [grids.maps(b).cpu().numpy() for b in range(len(boxes))]


def _assert_maps_close(gpu, ref, what):
    """Every map value within 1e-3 + 1e-4 |ref| of the oracle's.  Both sides
    decide the 8 A cutoff as r < 8 in binary64, so a term is in both sums or
    in neither (a wrong decision would move a value by the term's 8 A value,
    up to 0.0045 kcal/mol)."""
    err = np.abs(gpu.astype(np.float64) - ref)
    tol = 1e-3 + 1e-4 * np.abs(ref)
    bad = err > tol
    assert not bad.any(), "%s: %d of %d values off, worst %.3g at %s" % (
        what, int(bad.sum()), bad.size, float(err.max()), np.unravel_index(np.argmax(err - tol), err.shape))


def test_tiny_config_every_value(oracle, pv_ctx):
    cfg = S.CONFIGS["tiny"]
    rx, rt, bxs = S.make_receptor(cfg)
    grids, maps = _gpu_maps(pv_ctx, rx, rt, bxs)
    dims, org = grids.info(0)
    odims, oorg = oracle.lattice(bxs[0].center.astype(np.float64), bxs[0].size.astype(np.float64), bxs[0].spacing)
    np.testing.assert_array_equal(dims, odims)
    np.testing.assert_array_equal(org, oorg)
    ref = oracle.build_maps(rx, rt, dims, org, bxs[0].spacing)
    assert maps[0].shape == ref.shape == (8, 55, 55, 55)
    _assert_maps_close(maps[0], ref, "tiny")


def test_five_pockets_sampled(oracle, pv_ctx):
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    grids, maps = _gpu_maps(pv_ctx, rx, rt, bxs)
    g = np.random.default_rng(0)
    for b, box in enumerate(bxs):
        dims, org = grids.info(b)
        assert list(dims) == [65, 65, 65]
        pts = [(0, 0, 0), (64, 64, 64), (64, 0, 32)] + [tuple(int(v) for v in g.integers(0, 65, 3)) for _ in range(300)]
        for i, j, k in pts:
            ref = oracle.map_point(rx, rt, dims, org, box.spacing, i, j, k)
            _assert_maps_close(maps[b][:, k, j, i], ref, "box %d point %s" % (b, (i, j, k)))


def test_maps_reproducible_and_docks_repeat(pv_ctx):
    """Two builds and a rebuild of the five pockets give the same maps bit for
    bit (the candidate atoms keep their order, so every point sums in the same
    order), and a dock on either build repeats exactly: the chains are chaotic,
    so an ulp of difference in a map would move them."""
    import torch

    import paper_2506_20043_amd as pv
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    g1, m1 = _gpu_maps(pv_ctx, rx, rt, bxs)
    g2, m2 = _gpu_maps(pv_ctx, rx, rt, bxs)
    for b in range(len(bxs)):
        assert np.array_equal(m1[b], m2[b]), b
    g1.rebuild()
    torch.cuda.synchronize()
    for b in range(len(bxs)):
        assert np.array_equal(g1.maps(b).cpu().numpy(), m1[b]), b
    ligs = pv.Ligands(pv_ctx, S.make_ligands(cfg))
    jobs = [(0, b) for b in range(len(bxs))]
    p = pv.dock_params(chains=64, steps=60, seed=S.philox_seed(cfg), flags=pv.PV_DOCK_GRAPH)
    outs = []
    for grids in (g1, g2):
        plan = pv.Plan(pv_ctx, grids, ligs, jobs, p)
        outs.append({k: v.cpu().numpy().copy() for k, v in plan.run().items()})
        plan.close()
    for k in ("chain_best_e", "chain_evals", "chain_best_dof", "job_best_e"):
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_ragged_and_degenerate_boxes(oracle, pv_ctx):
    g = np.random.default_rng(1)
    rx, rt = S.receptor(g, 400, 20.0)
    boxes = [S.Box(np.array([10.0, 10.0, 10.0], np.float32), np.array([7.3, 4.1, 9.9], np.float32), 0.375),
             S.Box(np.array([3.0, 17.0, 9.0], np.float32), np.array([0.3, 0.3, 0.3], np.float32), 0.375),
             S.Box(np.array([-5.0, 25.0, 10.0], np.float32), np.array([6.0, 6.0, 6.0], np.float32), 0.5)]
    grids, maps = _gpu_maps(pv_ctx, rx, rt, boxes)
    for b, box in enumerate(boxes):
        dims, org = grids.info(b)
        ref = oracle.build_maps(rx, rt, dims, org, box.spacing)
        _assert_maps_close(maps[b], ref, "box %d dims %s" % (b, dims))
    assert list(grids.info(1)[0]) == [2, 2, 2]


def _straddling_atoms(oracle, n_want, seed):
    """Receptor atoms (binary32) placed within 3e-6 A of the 8 A cutoff from
    chosen lattice points of a box whose origin is (0, 0, 0), kept when the
    binary64 decision and a plain binary32 one (g = fma(i, h, 0), r2 =
    fma(dx,dx,fma(dy,dy,dz*dz)) < 64) disagree, or, failing enough such, when
    the atom lies within 1e-6 A of the cutoff.  Returns the atoms and their
    target points."""
    g = np.random.default_rng(seed)
    h = np.float32(0.375)
    atoms, pts = [], []
    tries = 0
    while len(atoms) < n_want and tries < 200000:
        tries += 1
        ijk = g.integers(0, 41, 3)
        p = ijk.astype(np.float64) * 0.375
        u = g.normal(size=3)
        u /= np.linalg.norm(u)
        a = (p + (8.0 + g.uniform(-3e-6, 3e-6)) * u).astype(np.float32)
        if np.any(a < -10) or np.any(a > 25):
            continue
        d64 = np.sqrt(((p - a.astype(np.float64)) ** 2).sum())
        gx = (ijk.astype(np.float32) * h).astype(np.float32)
        dd = (gx - a).astype(np.float32)
        r2 = np.float32(np.float64(dd[0]) * dd[0] + np.float32(np.float64(dd[1]) * dd[1] + np.float32(dd[2] * dd[2])))
        disagree = (d64 < 8.0) != (r2 < np.float32(64.0))
        if disagree or (tries > 100000 and abs(d64 - 8.0) < 1e-6):
            atoms.append(a)
            pts.append(tuple(int(v) for v in ijk))
    return np.array(atoms, np.float32), pts


def test_map_cutoff_decided_in_binary64(oracle, pv_ctx):
    """Atoms within a few 1e-6 A of the cutoff from lattice points, chosen
    where binary32 rounding would decide differently from binary64: the
    kernel's map values at those points match the oracle's r < 8 decision."""
    rx, pts = _straddling_atoms(oracle, 24, 5)
    assert len(rx) >= 12
    rt = np.array([0, 1, 2, 5, 7, 3] * 4, np.uint8)[:len(rx)]
    box = S.Box(np.full(3, 7.5, np.float32), np.full(3, 15.0, np.float32), 0.375)
    grids, maps = _gpu_maps(pv_ctx, rx, rt, [box])
    dims, org = grids.info(0)
    assert list(dims) == [41, 41, 41] and np.all(org == 0.0)
    for i, j, k in pts:
        ref, mg = oracle.map_point(rx, rt, dims, org, box.spacing, i, j, k, margin=True)
        assert mg < 5e-6
        _assert_maps_close(maps[0][:, k, j, i], ref, "point %s" % ((i, j, k),))


def test_empty_receptor_gives_zero_maps(pv_ctx):
    box = S.Box(np.zeros(3, np.float32), np.full(3, 5.0, np.float32), 0.375)
    _, maps = _gpu_maps(pv_ctx, np.zeros((0, 3), np.float32), np.zeros(0, np.uint8), [box])
    assert maps[0].shape == (8, 15, 15, 15) and np.all(maps[0] == 0.0)


def test_receptor_far_from_box_gives_zero_maps(pv_ctx):
    rx = np.array([[100.0, 0, 0], [0, 100.0, 0]], np.float32)
    box = S.Box(np.zeros(3, np.float32), np.full(3, 10.0, np.float32), 0.375)
    _, maps = _gpu_maps(pv_ctx, rx, np.array([0, 5], np.uint8), [box])
    assert np.all(maps[0] == 0.0)


def test_build_grids_rejects(pv_ctx):
    import paper_2506_20043_amd as pv
    rx = np.zeros((1, 3), np.float32)
    box = S.Box(np.zeros(3, np.float32), np.full(3, 5.0, np.float32), 0.375)
    with pytest.raises(pv.PvError, match="type"):
        pv.build_grids(pv_ctx, rx, np.array([8], np.uint8), [box])
    with pytest.raises(pv.PvError, match="penalty"):
        pv.build_grids(pv_ctx, rx, np.array([0], np.uint8), [box], penalty_slope=-1.0)
    bad = S.Box(np.zeros(3, np.float32), np.array([5.0, 0.0, 5.0], np.float32), 0.375)
    with pytest.raises(pv.PvError, match="size"):
        pv.build_grids(pv_ctx, rx, np.array([0], np.uint8), [bad])
    # 268^3 points: beyond the 2^24 points a box's 32-bit map offsets allow
    huge = S.Box(np.zeros(3, np.float32), np.full(3, 100.0, np.float32), 0.375)
    with pytest.raises(pv.PvError, match="2\\^24"):
        pv.build_grids(pv_ctx, rx, np.array([0], np.uint8), [huge])
    edge = S.Box(np.zeros(3, np.float32), np.full(3, 94.875, np.float32), 0.375)   # 254^3 points: accepted
    assert pv.build_grids(pv_ctx, rx, np.array([0], np.uint8), [edge]).info(0)[0].tolist() == [254, 254, 254]


def test_box_size_sweep_sampled(oracle, pv_ctx):
    """The box-size sweep (edges 15..30 A in 1 A steps around two pockets of
    the multi-pocket receptor) in one build: each box has n = ceil(s/h) + 1
    points per axis and matches the oracle at its corners and at sampled
    points."""
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    sweep = S.box_sweep(bxs[:2])
    assert len(sweep) == 32
    grids, maps = _gpu_maps(pv_ctx, rx, rt, sweep)
    g = np.random.default_rng(8)
    for b, box in enumerate(sweep):
        dims, org = grids.info(b)
        n = int(np.ceil(float(box.size[0]) / box.spacing)) + 1
        assert list(dims) == [n, n, n], (b, dims)
        ldims, lorg = oracle.lattice(box.center.astype(np.float64), box.size.astype(np.float64), box.spacing)
        assert list(ldims) == list(dims) and np.array_equal(np.float32(lorg), org)
        m = n - 1
        pts = [(0, 0, 0), (m, m, m), (m, 0, m // 2)] + [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(40)]
        for i, j, k in pts:
            ref = oracle.map_point(rx, rt, dims, org, box.spacing, i, j, k)
            _assert_maps_close(maps[b][:, k, j, i], ref, "box %d point %s" % (b, (i, j, k)))

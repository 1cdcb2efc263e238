"""Pins of the oracle's lattice, grid maps and trilinear lookup ("Kernel 1"
grid cache and the trilinear e_inter of Eq. qvina_eq_3)."""
import numpy as np
import pytest
from scipy import ndimage

from paper_2506_20043_amd import synth as S


def test_lattice_dims(oracle):
    for edge, n in ((20.0, 55), (24.0, 65), (30.0, 81), (15.0, 41), (0.375, 2), (0.5, 3)):
        dims, org = oracle.lattice([10.0, 20.0, 30.0], [edge] * 3, 0.375)
        assert list(dims) == [n] * 3
        np.testing.assert_array_equal(org, np.float32(np.array([10.0, 20.0, 30.0]) - (n - 1) * 0.375 / 2))


def test_lattice_rejects(oracle):
    for size, h in (([0.0, 1, 1], 0.375), ([1, 1, 1], 0.0), ([1, -1, 1], 0.375)):
        with pytest.raises(ValueError):
            oracle.lattice([0, 0, 0], size, h)


def _small_receptor(seed, n, cube):
    g = np.random.default_rng(seed)
    return S.receptor(g, n, cube)


def test_maps_two_paths_agree(oracle):
    """Atom-major map build equals the point-major sum at sampled points, and
    both report the same cutoff margin wherever an atom is near the cutoff."""
    rx, rt = _small_receptor(1, 300, 16.0)
    dims, org = oracle.lattice([8.0, 8.0, 8.0], [9.0, 7.5, 8.25], 0.375)
    maps, margin = oracle.build_maps(rx, rt, dims, org, 0.375, margin=True)
    g = np.random.default_rng(2)
    pts = [(0, 0, 0), (dims[0] - 1, dims[1] - 1, dims[2] - 1)]
    pts += [tuple(int(g.integers(0, dims[a])) for a in range(3)) for _ in range(60)]
    for i, j, k in pts:
        ref, mg = oracle.map_point(rx, rt, dims, org, 0.375, i, j, k, margin=True)
        np.testing.assert_array_equal(maps[:, k, j, i], ref)
        if mg < 0.01:
            assert margin[k, j, i] == mg
        else:
            assert margin[k, j, i] >= 0.01


def test_map_cutoff_margin_bruteforce(oracle):
    """The margin is the smallest |r - 8| over the receptor atoms, r taken
    from the binary32 receptor and lattice in binary64."""
    rx, rt = _small_receptor(3, 120, 18.0)
    dims, org = oracle.lattice([9.0, 9.0, 9.0], [6.0, 6.0, 6.0], 0.375)
    g = np.random.default_rng(4)
    for _ in range(40):
        i, j, k = (int(g.integers(0, dims[a])) for a in range(3))
        p = org.astype(np.float64) + 0.375 * np.array([i, j, k], np.float64)
        r = np.sqrt(((p[None, :] - rx.astype(np.float64)) ** 2).sum(axis=1))
        _, mg = oracle.map_point(rx, rt, dims, org, 0.375, i, j, k, margin=True)
        assert mg == pytest.approx(np.abs(r - 8.0).min(), abs=1e-12)


def test_map_single_atom_bruteforce(oracle):
    """One receptor atom of each type: every lattice value is phi(r) within 8 A."""
    dims, org = oracle.lattice([0.0, 0.0, 0.0], [20.0, 20.0, 20.0], 0.375)
    for rtype in range(8):
        atom = np.array([[0.1234, -0.377, 0.913]], np.float32)
        maps = oracle.build_maps(atom, [rtype], dims, org, 0.375)
        ii = np.arange(dims[0])
        gx = org[0].astype(np.float64) + 0.375 * ii
        gy = org[1].astype(np.float64) + 0.375 * np.arange(dims[1])
        gz = org[2].astype(np.float64) + 0.375 * np.arange(dims[2])
        Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
        r = np.sqrt((X - atom[0, 0]) ** 2 + (Y - atom[0, 1]) ** 2 + (Z - atom[0, 2]) ** 2)
        # the cutoff is decided on this same binary64 distance, so the set of
        # non-zero points is exactly the open 8 A ball
        inside = r < 8.0
        assert np.all(maps[:, ~inside] == 0.0)
        assert np.all(maps[:, inside] != 0.0)
        sel = np.argwhere(inside)[::97]
        for (k, j, i) in sel:
            for t in (0, 3, 5, 7):
                assert maps[t, k, j, i] == pytest.approx(oracle.pair(t, rtype, r[k, j, i])[0], rel=1e-12)


def _grid_with(oracle, maps, dims, org, h=0.375, kappa=1000.0):
    return oracle.Grid(maps, dims, org, h, kappa)


def test_trilinear_exact_at_lattice_points(oracle):
    g = np.random.default_rng(3)
    dims, org = oracle.lattice([1.0, 2.0, 3.0], [6.0, 4.5, 5.25], 0.375)
    maps = g.normal(size=(8, dims[2], dims[1], dims[0]))
    G = _grid_with(oracle, maps, dims, org)
    for _ in range(50):
        i, j, k = (int(g.integers(0, dims[a])) for a in range(3))
        x = np.array([org[0] + 0.375 * i, org[1] + 0.375 * j, org[2] + 0.375 * k], np.float64)
        for t in (0, 6):
            v, _, _ = G.trilinear(t, x)
            assert v == pytest.approx(maps[t, k, j, i], abs=1e-12)


def test_trilinear_affine_field_exact(oracle):
    """The interpolant of an affine field is the field: exact value and gradient."""
    dims, org = oracle.lattice([0.0, 0.0, 0.0], [6.0, 6.0, 6.0], 0.375)
    a = np.array([0.7, -1.3, 2.1])
    c0 = 0.25
    gz, gy, gx = np.meshgrid(*(org[ax].astype(np.float64) + 0.375 * np.arange(dims[ax]) for ax in (2, 1, 0)),
                             indexing="ij")
    field = c0 + a[0] * gx + a[1] * gy + a[2] * gz
    maps = np.repeat(field[None], 8, axis=0)
    G = _grid_with(oracle, maps, dims, org)
    g = np.random.default_rng(4)
    lo, hi = org.astype(np.float64), org + 0.375 * (dims - 1)
    for _ in range(100):
        x = g.uniform(lo, hi)
        v, grad, _ = G.trilinear(2, x)
        assert v == pytest.approx(c0 + a @ x, abs=1e-12)
        np.testing.assert_allclose(grad, a, atol=1e-11)


def test_trilinear_matches_scipy(oracle):
    g = np.random.default_rng(5)
    dims, org = oracle.lattice([0.0, 0.0, 0.0], [5.0, 6.0, 7.0], 0.375)
    maps = g.normal(size=(8, dims[2], dims[1], dims[0]))
    G = _grid_with(oracle, maps, dims, org)
    lo, hi = org.astype(np.float64), org + 0.375 * (dims - 1)
    for _ in range(200):
        x = g.uniform(lo, hi)
        f = (x - org.astype(np.float64)) / 0.375
        want = ndimage.map_coordinates(maps[4], [[f[2]], [f[1]], [f[0]]], order=1)[0]
        v, _, _ = G.trilinear(4, x)
        assert v == pytest.approx(want, abs=1e-12)


def test_trilinear_gradient_fd(oracle):
    g = np.random.default_rng(6)
    dims, org = oracle.lattice([0.0, 0.0, 0.0], [5.0, 5.0, 5.0], 0.375)
    maps = g.normal(size=(8, dims[2], dims[1], dims[0]))
    G = _grid_with(oracle, maps, dims, org)
    lo, hi = org.astype(np.float64), org + 0.375 * (dims - 1)
    n = 0
    for _ in range(200):
        x = g.uniform(lo, hi)
        v, grad, fd_ = G.trilinear(1, x)
        if fd_ < 1e-4:
            continue
        h = 1e-6
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[a] += h
            xm[a] -= h
            fd = (G.trilinear(1, xp)[0] - G.trilinear(1, xm)[0]) / (2 * h)
            assert grad[a] == pytest.approx(fd, rel=1e-6, abs=1e-7)
        n += 1
    assert n > 150


def test_out_of_box_penalty(oracle):
    dims, org = oracle.lattice([0.0, 0.0, 0.0], [3.0, 3.0, 3.0], 0.375)
    g = np.random.default_rng(7)
    maps = g.normal(size=(8, dims[2], dims[1], dims[0]))
    G = _grid_with(oracle, maps, dims, org, kappa=123.0)
    hi = org + 0.375 * (dims - 1)
    inside = np.array([0.3, -0.2, 0.1])
    v_in, _, _ = G.trilinear(0, np.array([hi[0], inside[1], inside[2]], np.float64))
    v_out, grad, _ = G.trilinear(0, np.array([hi[0] + 0.5, inside[1], inside[2]], np.float64))
    assert v_out == pytest.approx(v_in + 123.0 * 0.5, abs=1e-12)
    assert grad[0] == 123.0
    v_lo, grad, _ = G.trilinear(0, np.array([org[0] - 2.0, org[1] - 1.0, inside[2]], np.float64))
    v_c, _, _ = G.trilinear(0, np.array([org[0], org[1], inside[2]], np.float64))
    assert v_lo == pytest.approx(v_c + 123.0 * 3.0, abs=1e-11)
    assert grad[0] == -123.0 and grad[1] == -123.0


def test_grid_converges_to_pairwise_h2(oracle):
    """e_inter by trilinear lookup tends to the pairwise sum as O(h^2).

    Atoms sit at fractional coordinate 1/3 of the coarse cell, which keeps
    u(1-u) = 2/9 at every halving, so the error ratio tends to exactly 4.
    Receptor atoms are 5.8-7.0 A away (smooth part of every term, inside the
    cutoff for every corner used)."""
    g = np.random.default_rng(8)
    center = np.array([10.0, 10.0, 10.0])
    lig_types = np.array([1, 2, 7], np.int32)
    dims0, org0 = oracle.lattice(center, [12.0] * 3, 0.375)
    base = np.array([[16, 15, 14], [13, 17, 16], [15, 13, 17]], np.float64)
    lig = org0.astype(np.float64) + 0.375 * (base + 1.0 / 3.0)
    rec = []
    while len(rec) < 8:
        v = g.normal(size=3)
        p = lig[len(rec) % 3] + v / np.linalg.norm(v) * g.uniform(5.8, 7.0)
        dmin = np.linalg.norm(lig - p, axis=1).min()
        if 5.8 <= dmin and np.linalg.norm(lig - p, axis=1).max() < 7.0:
            rec.append(p)
    rec = np.array(rec, np.float32)
    rt = np.array([1, 2, 2, 7, 1, 2, 1, 7], np.int32)
    exact = oracle.inter_pairwise(rec, rt, lig, lig_types)
    errs = []
    for h in (0.375, 0.1875, 0.09375):
        dims, org = oracle.lattice(center, [12.0] * 3, h)
        np.testing.assert_array_equal(org, org0)
        G = oracle.Grid.build(rec, rt, center, [12.0] * 3, h)
        e = sum(G.trilinear(int(t), x)[0] for t, x in zip(lig_types, lig))
        errs.append(e - exact)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert abs(errs[0]) > 1e-6
    assert r1 == pytest.approx(4.0, abs=0.5) and r2 == pytest.approx(4.0, abs=0.5), errs


def test_grid_score_translation_invariance(oracle):
    """Shifting receptor, ligand and box together leaves the grid score unchanged."""
    cfg = S.CONFIGS["tiny"]
    rx, rt = _small_receptor(9, 600, 20.0)
    # coordinates on a 2^-10 grid, so the shifted receptor is exactly representable
    rx = (np.round(rx.astype(np.float64) * 1024) / 1024).astype(np.float32)
    mol = S.make_ligands(cfg)[0]
    L = oracle.Ligand(mol.xyz, mol.types, mol.bonds, mol.rotatable)
    c = np.array([10.0, 10.0, 10.0])
    G1 = oracle.Grid.build(rx, rt, c, [12.0] * 3, 0.375)
    shift = np.array([3.0, -2.0, 5.0])
    G2 = oracle.Grid.build((rx + shift).astype(np.float32), rt, c + shift, [12.0] * 3, 0.375)
    g = np.random.default_rng(10)
    for _ in range(10):
        dof = np.concatenate([g.uniform(8, 12, 3), S.random_quaternions(g, 1)[0],
                              g.uniform(-np.pi, np.pi, L.n_tors)])
        d2 = dof.copy()
        d2[:3] += shift
        a, b = L.score_grad(G1, dof), L.score_grad(G2, d2)
        assert b["e"] == pytest.approx(a["e"], rel=1e-9, abs=1e-9)
        np.testing.assert_allclose(b["grad_dof"], a["grad_dof"], rtol=1e-7, atol=1e-7)


def test_pairwise_rigid_motion_invariance(oracle):
    """The pairwise inter score is invariant under one SE(3) motion of both molecules."""
    from scipy.spatial.transform import Rotation
    g = np.random.default_rng(11)
    rx, rt = _small_receptor(12, 200, 12.0)
    lig = g.uniform(3, 9, size=(15, 3))
    lt = g.integers(0, 8, 15).astype(np.int32)
    e0 = oracle.inter_pairwise(rx, rt, lig, lt)
    for _ in range(5):
        R = Rotation.random(random_state=int(g.integers(1 << 30))).as_matrix()
        t = g.normal(size=3) * 5
        # the receptor interface is binary32: moving it rounds each coordinate
        # by ~1e-6 A, far below what changes the score beyond 1e-6 relative
        rx2 = (rx.astype(np.float64) @ R.T + t).astype(np.float32)
        lig2 = lig @ R.T + t
        e_moved = oracle.inter_pairwise(rx2, rt, lig2, lt)
        assert e_moved == pytest.approx(e0, rel=1e-6, abs=1e-6)

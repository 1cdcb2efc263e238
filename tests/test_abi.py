"""CPU tests of the C ABI: the library loads and exports every declared
symbol, argument checks answer before any device work, and the host-side
model (box lattice, ligand torsion tree and intra pairs) equals the
oracle's exactly."""
import os
import re

import numpy as np
import pytest

import paper_2506_20043_amd as pv
from paper_2506_20043_amd import synth as S

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "pvdock.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pv_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = pv.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    # the binding declares exactly the header's functions
    assert sorted(pv.SIGNATURES) == names


def test_binding_constants_match_the_header():
    """Every PV_* integer constant the Python binding defines has the value the
    header gives it (flag and status bits, limits, kinds, variants)."""
    text = open(HEADER).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"^#define (PV_[A-Z0-9_]+) (\d+)u?\b", text, re.M)}
    assert "PV_DOCK_NO_INTRA_BOUND" in defs and len(defs) >= 15
    mirrored = [n for n in dir(pv) if n.startswith("PV_") and isinstance(getattr(pv, n), int)]
    assert len(mirrored) >= 8
    for n in mirrored:
        assert n in defs and getattr(pv, n) == defs[n], n


def test_version_and_defaults():
    assert pv.lib().pv_version() == 102
    p = pv.dock_params()
    assert (p.bfgs_max_iter, p.bfgs_m, p.ls_max_trials) == (30, 5, 10)
    assert p.ls_rho == pytest.approx(1e-4) and p.ls_sigma == pytest.approx(0.1)
    assert p.temperature == pytest.approx(1.2)


def test_calls_without_context_fail_cleanly():
    import ctypes as C
    L = pv.lib()
    h = C.c_void_p()
    boxes = pv.make_boxes([([0, 0, 0], [10, 10, 10], 0.375)])
    assert L.pv_build_grids(None, 0, None, None, boxes, 1, 10.0, None, C.byref(h)) == -6
    assert b"context" in L.pv_last_error()
    assert L.pv_build_grids(None, 0, None, None, boxes, 1, 10.0, None, None) == -1
    assert L.pv_ligands_info(None, 0, (C.c_int32 * 8)()) == -1
    assert L.pv_score_grad(None, None, None, 1, None, None, None, 7, *([None] * 6), 0, None) == -6
    assert L.pv_dock_run(None, None, None) == -1
    assert L.pv_dock_plan(None, None, None, None, 0, None, C.byref(h)) == -6
    # freeing NULL handles is a no-op
    L.pv_grids_free(None)
    L.pv_ligands_free(None)
    L.pv_plan_free(None)
    L.pv_destroy(None)


def test_box_lattice_matches_oracle(oracle):
    g = np.random.default_rng(0)
    for _ in range(300):
        c = g.uniform(-50, 80, 3).astype(np.float32)
        s = np.float32(g.choice([g.uniform(0.1, 40.0), float(g.integers(15, 31))]))
        h = np.float32(g.choice([0.375, 0.25, 0.5, 1.0, g.uniform(0.1, 1.0)]))
        d1, o1 = pv.box_lattice(c, [s] * 3, h)
        d2, o2 = oracle.lattice(c.astype(np.float64), [float(s)] * 3, float(h))
        np.testing.assert_array_equal(d1, d2)
        np.testing.assert_array_equal(o1, o2)


def test_box_lattice_rejects():
    for size, h, code in (([0, 1, 1], 0.375, "must be > 0"), ([1, 1, 1], 0.0, "spacing"),
                          ([1000, 1, 1], 0.375, "2048"), ([np.nan, 1, 1], 0.375, "finite")):
        with pytest.raises(pv.PvError, match=code):
            pv.box_lattice([0, 0, 0], size, h)


def _check_same_model(oracle, m):
    info, pairs, frag = pv.describe_ligand(m.xyz, m.types, m.bonds, m.rotatable)
    L = oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    assert info[0] == L.n_atoms and info[1] == L.n_frag and info[2] == L.n_tors
    assert info[3] == L.n_pairs and info[5] == L.depth and info[6] == 7 + L.n_tors
    op = L.pairs()
    np.testing.assert_array_equal(pairs, op[np.lexsort((op[:, 1], op[:, 0]))])
    of = L.frag()
    # the same partition into fragments; the library's root is fragment 0
    assert info[4] == int(np.sum(of == L.root))
    assert np.all(frag[of == L.root] == 0)
    pairs_map = {}
    for a, b in zip(of, frag):
        assert pairs_map.setdefault(a, b) == b
    assert len(set(pairs_map.values())) == L.n_frag


@pytest.mark.parametrize("cfg", ["tiny", "multi_pocket", "uneven_batch", "differentiation", "screening"])
def test_ligand_model_matches_oracle(oracle, cfg):
    c = S.CONFIGS[cfg]
    n = {"tiny": 1, "multi_pocket": 1, "uneven_batch": 40, "differentiation": 8, "screening": 40}[cfg]
    for m in S.make_ligands(c, count=n):
        _check_same_model(oracle, m)


def _bond_distances(n, bonds):
    """All-pairs bond-graph distances by breadth-first search."""
    adj = [[] for _ in range(n)]
    for a, b in bonds:
        adj[a].append(b)
        adj[b].append(a)
    dist = np.full((n, n), -1, np.int64)
    for s0 in range(n):
        dist[s0, s0] = 0
        todo = [s0]
        while todo:
            u = todo.pop(0)
            for v in adj[u]:
                if dist[s0, v] < 0:
                    dist[s0, v] = dist[s0, u] + 1
                    todo.append(v)
    return dist


def test_ligand_model_with_rings_matches_oracle(oracle):
    """Ligands with rigid six-membered rings (rings inside fragments, torsions
    on bridges elsewhere): the library's host model equals the oracle's, every
    ring lies inside one fragment, and the intra pairs are exactly the atom
    pairs in different fragments at least four bonds apart along the
    shortest path of the cyclic bond graph."""
    g = np.random.default_rng(17)
    for n, t, r in ((12, 2, 1), (20, 4, 2), (33, 7, 2), (40, 8, 3), (64, 12, 4), (90, 16, 3)):
        m = S.ring_ligand(g, n, t, r)
        assert len(m.bonds) == n - 1 + r
        _check_same_model(oracle, m)
        info, pairs, frag = pv.describe_ligand(m.xyz, m.types, m.bonds, m.rotatable)
        for k in range(r):
            assert len(set(frag[6 * k:6 * k + 6].tolist())) == 1
        dist = _bond_distances(n, m.bonds)
        want = {(i, j) for i in range(n) for j in range(i + 1, n) if frag[i] != frag[j] and dist[i, j] >= 4}
        assert {tuple(p) for p in pairs.tolist()} == want


def test_ligand_model_extremes(oracle):
    g = np.random.default_rng(3)
    # one atom, two atoms, the maximum of 128 atoms with 32 torsions
    one = S.Molecule(np.zeros((1, 3)), np.array([2], np.int32), np.zeros((0, 2), np.int32), np.zeros(0, np.uint8))
    _check_same_model(oracle, one)
    _check_same_model(oracle, S.tree_ligand(g, 2, 0))
    big = S.tree_ligand(g, 128, 32)
    assert big.n_tors == 32
    _check_same_model(oracle, big)
    info, _, _ = pv.describe_ligand(big.xyz, big.types, big.bonds, big.rotatable)
    assert info[0] == 128 and info[2] == 32


def test_ligand_model_rejects(oracle):
    g = np.random.default_rng(4)
    m = S.tree_ligand(g, 10, 3)
    bad = [
        (m.xyz, np.full(10, 8), m.bonds, m.rotatable, "type"),
        (m.xyz, m.types, m.bonds[:-1], m.rotatable[:-1], "connected"),
        (m.xyz, m.types, np.vstack([m.bonds, [[0, 0]]]), np.append(m.rotatable, 0), "self"),
        (m.xyz, m.types, np.vstack([m.bonds, m.bonds[:1]]), np.append(m.rotatable, 0), "duplicate"),
    ]
    xyz = m.xyz.copy()
    xyz[3, 1] = np.nan
    bad.append((xyz, m.types, m.bonds, m.rotatable, "finite"))
    for x, t, b, r, what in bad:
        with pytest.raises(pv.PvError, match=what):
            pv.describe_ligand(x, t, b, r)
    # a ring closed by a rotatable bond
    ring_x = np.array([[0, 0, 0], [1.5, 0, 0], [1.5, 1.5, 0], [0, 1.5, 0]], np.float64)
    ring_b = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], np.int32)
    with pytest.raises(pv.PvError, match="ring"):
        pv.describe_ligand(ring_x, np.zeros(4), ring_b, [0, 0, 0, 1])
    with pytest.raises(ValueError):
        oracle.Ligand(ring_x, np.zeros(4, np.int32), ring_b, np.array([0, 0, 0, 1], np.uint8))
    # limits
    big = S.tree_ligand(g, 129, 0)
    with pytest.raises(pv.PvError, match="128"):
        pv.describe_ligand(big.xyz, big.types, big.bonds, big.rotatable)
    many = S.tree_ligand(g, 100, 33)
    if many.n_tors == 33:
        with pytest.raises(pv.PvError, match="32"):
            pv.describe_ligand(many.xyz, many.types, many.bonds, many.rotatable)

"""Seeded synthetic inputs for the docking hot path.

This module only draws inputs: receptors, search boxes, random tree ligands,
poses and job lists.  It holds none of the method's arithmetic, and it is the
one module that both the HIP path's tests and the oracle's tests use.

Shapes follow the paper's workloads: box edges of 15-30 A and 20 A
(Methods, docking setting), ligands binned by rotatable bonds (<=5, 6-10,
>10) and heavy atoms (<=15, 15-25, >25) as in the paper's success-rate
analyses, and a handful of pockets per receptor.  The paper's datasets are
not used; these inputs stand in for them.

Vina XS atom types used here (index: name):
  0 C_H  1 C_P  2 N_P  3 N_D  4 N_A  5 O_A  6 O_DA  7 S_P
drawn with probabilities 40/15/10/8/7/12/5/3 %.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

XS_NAMES = ("C_H", "C_P", "N_P", "N_D", "N_A", "O_A", "O_DA", "S_P")
XS_PROBS = np.array([0.40, 0.15, 0.10, 0.08, 0.07, 0.12, 0.05, 0.03])
BASE_SEED = 20043


def rng(config_index: int, stream: int) -> np.random.Generator:
    """Independent sub-stream `stream` of config `config_index`."""
    ss = np.random.SeedSequence(BASE_SEED + config_index, spawn_key=(stream,))
    return np.random.default_rng(ss)


STREAM_RECEPTOR, STREAM_BOXES, STREAM_LIGANDS, STREAM_POSES, STREAM_JOBS, STREAM_KEY = range(6)


def _types(g: np.random.Generator, n: int) -> np.ndarray:
    return g.choice(8, size=n, p=XS_PROBS).astype(np.int32)


def receptor(g: np.random.Generator, n_atoms: int, cube: float):
    """Atoms uniform in [0, cube)^3, binary32 coordinates, XS types."""
    xyz = (g.random((n_atoms, 3)) * cube).astype(np.float32)
    return xyz, _types(g, n_atoms)


@dataclass
class Box:
    center: np.ndarray  # (3,) binary32 values
    size: np.ndarray    # (3,)
    spacing: float = 0.375


def boxes(g: np.random.Generator, n: int, edge_lo: float, edge_hi: float, cube: float,
          centred: bool = False, integer_edges: bool = True):
    out = []
    for _ in range(n):
        if integer_edges:
            e = float(g.integers(int(edge_lo), int(edge_hi) + 1))
        else:
            e = float(g.uniform(edge_lo, edge_hi))
        if centred:
            c = np.full(3, cube / 2.0)
        else:
            c = g.uniform(e / 2.0, cube - e / 2.0, size=3)
        out.append(Box(np.float32(c).astype(np.float32), np.full(3, e, np.float32)))
    return out


def box_sweep(pockets, edges=tuple(range(15, 31))):
    """The box-size sweep: every pocket centre with cubic boxes of each edge
    (15..30 A in 1 A steps by default), pocket-major."""
    return [Box(np.asarray(b.center, np.float32).copy(), np.full(3, float(e), np.float32), b.spacing)
            for b in pockets for e in edges]


def sphere_directions(n: int) -> np.ndarray:
    """n unit vectors spread over the sphere (golden-angle spiral), binary32."""
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * k
    d = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d.astype(np.float32)


@dataclass
class Molecule:
    xyz: np.ndarray        # (N, 3) float64 holding binary32 values
    types: np.ndarray      # (N,) int32
    bonds: np.ndarray      # (B, 2) int32
    rotatable: np.ndarray  # (B,) uint8
    n_tors: int = field(default=0)


def tree_ligand(g: np.random.Generator, n_atoms: int, n_tors: int, bond: float = 1.5,
                min_sep: float = 2.3, max_degree: int = 4) -> Molecule:
    """Random tree of `n_atoms` heavy atoms with `bond`-A bonds.

    Atoms are attached one at a time to a random atom of degree < max_degree
    along a random direction, redrawn until every non-bonded distance is at
    least `min_sep`.  `n_tors` bonds with two non-terminal ends are marked
    rotatable (clamped to the number of such bonds).
    """
    while True:
        xyz = np.zeros((n_atoms, 3))
        deg = np.zeros(n_atoms, np.int32)
        bonds = []
        ok = True
        for a in range(1, n_atoms):
            placed = False
            for _ in range(400):
                cand = np.nonzero(deg[:a] < max_degree)[0]
                p = int(cand[g.integers(0, len(cand))])   # the draw Generator.choice(cand) makes
                v = g.normal(size=3)
                v /= np.sqrt(v.dot(v))
                x = xyz[p] + bond * v
                diff = xyz[:a] - x
                d2 = np.einsum("ij,ij->i", diff, diff)
                d2[p] = np.inf
                if np.sqrt(d2.min()) >= min_sep:
                    xyz[a] = x
                    deg[p] += 1
                    deg[a] += 1
                    bonds.append((p, a))
                    placed = True
                    break
            if not placed:
                ok = False
                break
        if ok:
            break
    bonds = np.array(bonds, np.int32).reshape(-1, 2)
    inner = [b for b in range(len(bonds)) if deg[bonds[b, 0]] >= 2 and deg[bonds[b, 1]] >= 2]
    k = min(n_tors, len(inner))
    rot = np.zeros(len(bonds), np.uint8)
    if k > 0:
        rot[g.choice(inner, size=k, replace=False)] = 1
    xyz -= xyz.mean(axis=0)
    xyz = xyz.astype(np.float32).astype(np.float64)
    return Molecule(xyz, _types(g, n_atoms), bonds, rot, int(k))


def ring_ligand(g: np.random.Generator, n_atoms: int, n_tors: int, n_rings: int = 1, bond: float = 1.5,
                min_sep: float = 2.3, max_degree: int = 4) -> Molecule:
    """Random ligand with `n_rings` planar six-membered rings (bond length
    `bond`, so 1,3 and 1,4 ring distances are 2.6 and 3.0 A), each ring after
    the first joined by a single bond to an atom of the one before, then
    grown into a tree as tree_ligand does.  Ring bonds are never rotatable (a
    rotatable bond must be a bridge); `n_tors` bridges with two non-terminal
    ends are marked rotatable (clamped)."""
    assert n_atoms >= 6 * n_rings
    hexagon = np.array([[np.cos(k * np.pi / 3), np.sin(k * np.pi / 3), 0.0] for k in range(6)]) * bond
    while True:
        xyz = np.zeros((n_atoms, 3))
        deg = np.zeros(n_atoms, np.int32)
        bonds, in_ring = [], []
        ok = True
        a = 0
        for r in range(n_rings):
            w, x, y, z = random_quaternions(g, 1)[0]
            R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                          [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                          [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
            ring = hexagon @ R.T
            anchor = -1
            if r > 0:
                # ring r starts one bond out from a random atom of ring r - 1,
                # pointing away from that ring's centre, its own centre
                # further out along the same line
                anchor = a - 6 + int(g.integers(0, 6))
                out = xyz[anchor] - xyz[a - 6:a].mean(axis=0)
                out /= np.linalg.norm(out)
                first = xyz[anchor] + bond * out
                centre = first + bond * out
                ring = ring - ring.mean(axis=0)
                k0 = int(np.argmin(((ring + centre - first) ** 2).sum(axis=1)))
                ring = np.roll(ring, -k0, axis=0) + centre
                ring += first - ring[0]
            if a > 0:
                diff = ring[:, None, :] - xyz[None, :a, :]
                d = np.sqrt((diff ** 2).sum(axis=2))
                d[0, anchor] = np.inf
                if d.min() < min_sep:
                    ok = False
                    break
            xyz[a:a + 6] = ring
            for k in range(6):
                bonds.append((a + k, a + (k + 1) % 6))
                in_ring.append(True)
            deg[a:a + 6] += 2
            if anchor >= 0:
                bonds.append((anchor, a))
                in_ring.append(False)
                deg[anchor] += 1
                deg[a] += 1
            a += 6
        if not ok:
            continue
        for b in range(a, n_atoms):
            placed = False
            for _ in range(400):
                cand = np.nonzero(deg[:b] < max_degree)[0]
                p = int(cand[g.integers(0, len(cand))])
                v = g.normal(size=3)
                v /= np.sqrt(v.dot(v))
                x = xyz[p] + bond * v
                diff = xyz[:b] - x
                d2 = np.einsum("ij,ij->i", diff, diff)
                d2[p] = np.inf
                if np.sqrt(d2.min()) >= min_sep:
                    xyz[b] = x
                    deg[p] += 1
                    deg[b] += 1
                    bonds.append((p, b))
                    in_ring.append(False)
                    placed = True
                    break
            if not placed:
                ok = False
                break
        if ok:
            break
    bonds = np.array(bonds, np.int32).reshape(-1, 2)
    inner = [k for k in range(len(bonds)) if not in_ring[k] and deg[bonds[k, 0]] >= 2 and deg[bonds[k, 1]] >= 2]
    k = min(n_tors, len(inner))
    rot = np.zeros(len(bonds), np.uint8)
    if k > 0:
        rot[g.choice(inner, size=k, replace=False)] = 1
    xyz -= xyz.mean(axis=0)
    xyz = xyz.astype(np.float32).astype(np.float64)
    return Molecule(xyz, _types(g, n_atoms), bonds, rot, int(k))


def random_quaternions(g: np.random.Generator, n: int) -> np.ndarray:
    q = g.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def poses(g: np.random.Generator, n: int, lo, hi, n_tors: int) -> np.ndarray:
    """n poses [t(3), q(4), psi(T)]: t uniform in [lo, hi], q uniform on S^3,
    psi uniform in [-pi, pi]; binary32 values."""
    t = g.uniform(np.asarray(lo, np.float64), np.asarray(hi, np.float64), size=(n, 3))
    q = random_quaternions(g, n)
    psi = g.uniform(-np.pi, np.pi, size=(n, n_tors))
    return np.concatenate([t, q, psi], axis=1).astype(np.float32)


# ---------------------------------------------------------------- configurations
@dataclass
class Config:
    name: str
    index: int
    rec_atoms: int
    cube: float
    n_boxes: int
    box_edge: tuple
    box_centred: bool
    n_ligands: int
    lig_atoms: tuple
    lig_tors: tuple
    chains: int
    steps: int
    bfgs_iter: int = 30
    n_poses: int = 0
    shared_from: int | None = None  # config whose receptor and boxes are reused


CONFIGS = {
    "tiny": Config("tiny", 0, 2000, 30.0, 1, (20, 20), True, 1, (20, 20), (4, 4), 8, 200),
    "multi_pocket": Config("multi-pocket", 1, 5000, 50.0, 5, (24, 24), False, 1, (35, 35), (8, 8), 256, 1000),
    "uneven_batch": Config("batched-uneven", 2, 5000, 50.0, 5, (24, 24), False, 4096, (10, 60), (0, 15), 32, 500,
                 shared_from=1),
    "differentiation": Config("differentiation", 3, 5000, 50.0, 1, (24, 24), False, 64, (40, 40), (10, 10), 0, 0,
                 n_poses=16384, shared_from=1),
    "screening": Config("screening", 4, 8000, 60.0, 16, (20, 30), False, 6250, (8, 80), (0, 20), 16, 300),
}


def make_receptor(cfg: Config):
    src = cfg.shared_from if cfg.shared_from is not None else cfg.index
    base = [c for c in CONFIGS.values() if c.index == src][0]
    xyz, ty = receptor(rng(src, STREAM_RECEPTOR), base.rec_atoms, base.cube)
    bxs = boxes(rng(src, STREAM_BOXES), base.n_boxes, base.box_edge[0], base.box_edge[1],
                base.cube, centred=base.box_centred)
    if cfg.shared_from is not None:
        bxs = bxs[:cfg.n_boxes]
    return xyz, ty, bxs


def make_ligands(cfg: Config, count: int | None = None, first: int = 0):
    """Ligands first..first+count of the config, each from its own sub-stream,
    so any slice is reproducible on its own."""
    n = cfg.n_ligands if count is None else count
    out = []
    for i in range(first, first + n):
        g = np.random.default_rng(np.random.SeedSequence(BASE_SEED + cfg.index,
                                                         spawn_key=(STREAM_LIGANDS, i)))
        na = int(g.integers(cfg.lig_atoms[0], cfg.lig_atoms[1] + 1))
        nt = int(g.integers(cfg.lig_tors[0], cfg.lig_tors[1] + 1))
        out.append(tree_ligand(g, na, nt))
    return out


def _ligand_slice(args):
    name, count, first = args
    return make_ligands(CONFIGS[name], count, first)


def make_ligands_parallel(key: str, count: int | None = None, first: int = 0, workers: int = 1):
    """make_ligands(CONFIGS[key], count, first) split over `workers` forked
    processes (the same ligands: each has its own sub-stream).  Call it
    before the process initialises a GPU."""
    cfg = CONFIGS[key]
    n = cfg.n_ligands if count is None else count
    if workers <= 1 or n < 64:
        return make_ligands(cfg, n, first)
    import multiprocessing as mp
    step = (n + 4 * workers - 1) // (4 * workers)
    parts = [(key, min(step, n - s), first + s) for s in range(0, n, step)]
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_ligand_slice, parts)
    return [m for part in out for m in part]


def make_jobs(cfg: Config):
    """(ligand, box) pairs.  Screening: every ligand in every box, seeded random order."""
    pairs = np.array([(l, b) for l in range(cfg.n_ligands) for b in range(cfg.n_boxes)],
                     np.int32).reshape(-1, 2)
    if cfg.name == "screening":
        pairs = pairs[rng(cfg.index, STREAM_JOBS).permutation(len(pairs))]
    return pairs


def philox_seed(cfg: Config) -> int:
    return int(rng(cfg.index, STREAM_KEY).integers(0, 2**63))

"""Pins of the oracle's RNG, RILC-BFGS and Monte Carlo chain
(Eqs. qvina_eq_6 .. qvina_eq_13 and Supplementary Algorithm 2)."""
import numpy as np
import pytest
from scipy import optimize, stats
from scipy.spatial.transform import Rotation

from paper_2506_20043_amd import synth as S


# ------------------------------------------------------------------ Philox
def test_philox_matches_numpy(oracle):
    """Philox4x64-10 words equal numpy's Philox, which advances its 256-bit
    counter by one before it generates each block."""
    g = np.random.default_rng(0)
    cases = [(np.zeros(4, np.uint64), np.array([5, 0], np.uint64)),
             (np.array([2**64 - 1, 7, 0, 0], np.uint64), np.array([1, 2], np.uint64))]
    for _ in range(20):
        cases.append((g.integers(0, 2**63, 4, dtype=np.uint64) * 2 + 1,
                      g.integers(0, 2**63, 2, dtype=np.uint64)))
    for ctr, key in cases:
        bg = np.random.Philox(counter=ctr.copy(), key=key.copy())
        want = bg.random_raw(8).astype(np.uint64)
        c = [int(v) for v in ctr]
        for blk in range(2):
            v = (c[0] | c[1] << 64 | c[2] << 128 | c[3] << 192) + 1 + blk
            v &= (1 << 256) - 1
            cc = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], np.uint64)
            np.testing.assert_array_equal(oracle.philox4x64_10(cc, key), want[4 * blk:4 * blk + 4])


# ------------------------------------------------------------------ BFGS
def test_bfgs_convex_quadratic(oracle):
    g = np.random.default_rng(1)
    for n in (3, 8, 17):
        A = g.normal(size=(n, n))
        A = A @ A.T + n * np.eye(n)
        x0 = g.normal(size=n) * 3
        P = oracle.bfgs_params(max_iter=200, eps_g=1e-10)
        x, f, ne, it = oracle.bfgs_generic(lambda x: (0.5 * x @ A @ x, A @ x), x0, P)
        np.testing.assert_allclose(x, 0, atol=1e-8)
        assert f < 1e-15 and it < 200


def test_bfgs_rosenbrock(oracle):
    P = oracle.bfgs_params(max_iter=500, eps_g=1e-8)
    x, f, ne, it = oracle.bfgs_generic(lambda x: (optimize.rosen(x), optimize.rosen_der(x)),
                                        np.array([-1.2, 1.0, -0.5, 0.8]), P)
    np.testing.assert_allclose(x, 1.0, atol=1e-6)


def test_bfgs_accepted_steps_satisfy_wolfe(oracle):
    """Replay the evaluations: every accepted point satisfies Armijo and the
    weak Wolfe condition with rho = 1e-4 and sigma = 0.1 against the point it
    left, and the objective never rises."""
    g = np.random.default_rng(2)
    n = 6
    A = g.normal(size=(n, n))
    A = A @ A.T + 0.5 * np.eye(n)
    b = g.normal(size=n)
    log = []

    def fun(x):
        f = 0.5 * x @ A @ x + np.sum(np.cos(x)) + b @ x
        gr = A @ x - np.sin(x) + b
        log.append((x.copy(), f, gr.copy()))
        return f, gr

    P = oracle.bfgs_params(max_iter=40, eps_g=1e-12)
    xf, ff, ne, it = oracle.bfgs_generic(fun, g.normal(size=n) * 2, P)
    assert ne == len(log)
    # rebuild the accepted iterates: those evaluations whose point is kept
    acc = [log[0]]
    for x, f, gr in log[1:]:
        x0, f0, g0 = acc[-1]
        d = x - x0
        if f <= f0 + 1e-4 * (g0 @ d) and gr @ d >= 0.1 * (g0 @ d):
            acc.append((x, f, gr))
    assert np.allclose(acc[-1][0], xf)
    fs = [a[1] for a in acc]
    assert all(b_ <= a_ for a_, b_ in zip(fs, fs[1:]))


def _sparse_setup(oracle, seed=3):
    """A receptor of moderate density (300 atoms in a 24 A cube) so that
    local minima are not dominated by clashes."""
    g = np.random.default_rng(seed)
    rx, rt = S.receptor(g, 300, 24.0)
    G = oracle.Grid.build(rx, rt, [12.0, 12.0, 12.0], [16.0] * 3, 0.375)
    m = S.tree_ligand(g, 14, 3)
    L = oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    return G, L, g


def _diameter(n, bonds):
    adj = [[] for _ in range(n)]
    for a, b in bonds:
        adj[a].append(b)
        adj[b].append(a)
    best = 0
    for s0 in range(n):
        dist = {s0: 0}
        todo = [s0]
        while todo:
            u = todo.pop(0)
            for v in adj[u]:
                if v not in dist:
                    dist[v] = dist[u] + 1
                    todo.append(v)
        best = max(best, max(dist.values()))
    return best


def test_bfgs_matches_scipy_on_torsions(oracle):
    """With empty maps only e_intra acts.  For ligands at most 5 bonds across
    (every pair stays inside the 8 A cutoff) made of C_P atoms (no hydrophobic
    or hydrogen-bond kink) it is a smooth function of the torsions.  From the
    same starts, the oracle's BFGS on the full pose and scipy's BFGS on the
    torsions alone stop at stationary points of equal energy."""
    g = np.random.default_rng(5)
    dims, org = oracle.lattice([0.0, 0.0, 0.0], [60.0] * 3, 2.0)
    G = oracle.Grid(np.zeros((8, dims[2], dims[1], dims[0])), dims, org, 2.0)
    P = oracle.bfgs_params(max_iter=500, eps_g=1e-9)
    tried = same = 0
    while tried < 12:
        m = S.tree_ligand(g, 9, 4)
        if m.n_tors < 3 or _diameter(9, m.bonds) > 5:
            continue
        L = oracle.Ligand(m.xyz, np.full(9, 1, np.int32), m.bonds, m.rotatable)
        if L.n_pairs < 3:
            continue
        x0 = np.concatenate([[0.0, 0.0, 0.0], S.random_quaternions(g, 1)[0],
                             g.uniform(-np.pi, np.pi, L.n_tors)])

        def fg(psi):
            d = x0.copy()
            d[7:] = psi
            r = L.score_grad(G, d)
            return r["e"], r["grad_tan"][6:]

        # start both a little away from a minimum found by the oracle
        x0[7:] = oracle.bfgs(L, G, x0, P)[0][7:] + g.normal(size=L.n_tors) * 0.1
        sp = optimize.minimize(fg, x0[7:], jac=True, method="BFGS", options=dict(gtol=1e-9, maxiter=2000))
        xo, fo, _, _ = oracle.bfgs(L, G, x0, P)
        go = L.score_grad(G, xo)["grad_tan"]
        assert np.linalg.norm(go) < 1e-6 and np.linalg.norm(sp.jac) < 1e-6
        tried += 1
        if abs(fo - sp.fun) <= 1e-3:
            same += 1
        else:
            # a different stationary point: scipy's one must be a fixed point
            # of the oracle's BFGS as well
            d = x0.copy()
            d[7:] = sp.x
            _, fp, _, _ = oracle.bfgs(L, G, d, P)
            assert fp == pytest.approx(sp.fun, abs=1e-6)
    assert same >= 10, same


# ------------------------------------------------------------------ MC
@pytest.fixture(scope="module")
def sparse(oracle):
    return _sparse_setup(oracle, 4)


def test_init_pose_in_box_and_unit(oracle, sparse):
    G, L, _ = sparse
    lo, hi = G.origin.astype(np.float64), G.origin + G.h * (G.dims - 1)
    qs = []
    for c in range(3000):
        d = oracle.init_pose(L, G, 5, 1, c)
        assert np.all(d[:3] >= lo) and np.all(d[:3] <= hi)
        assert abs(np.linalg.norm(d[3:7]) - 1) < 1e-12
        assert np.all(np.abs(d[7:]) <= np.pi)
        qs.append(d[3:7])
    q = np.array(qs)
    n = len(q)
    # uniform on S^3: E[q] = 0, E[q q^T] = I/4 (3 sigma)
    assert np.all(np.abs(q.mean(axis=0)) < 3 * 0.5 / np.sqrt(n))
    C = q.T @ q / n
    assert np.all(np.abs(np.diag(C) - 0.25) < 3 * np.sqrt((3 / 8 - 1 / 16) / n) * 1.1)
    off = C[~np.eye(4, dtype=bool)]
    assert np.all(np.abs(off) < 3 * np.sqrt(1 / 24 / n) * 1.1)
    # rotation angle density (1 - cos theta)/pi on [0, pi]
    th = 2 * np.arccos(np.clip(np.abs(q[:, 0]), 0, 1))
    cdf = lambda t: (t - np.sin(t)) / np.pi
    assert stats.kstest(th, cdf).pvalue > 0.01


def test_mc_zero_steps_is_initial_pose(oracle, sparse):
    G, L, _ = sparse
    P = oracle.mc_params(chains=4, steps=0, seed=11)
    for c in range(4):
        d, e, ne = oracle.mc_chain(L, G, P, 2, c)
        np.testing.assert_array_equal(d, oracle.init_pose(L, G, 11, 2, c))
        assert e == L.score_grad(G, d)["e"] and ne == 1


def test_mc_without_bfgs_counts(oracle, sparse):
    """With a zero iteration cap each step costs one evaluation, plus one for
    each refinement of a new best."""
    G, L, _ = sparse
    P = oracle.mc_params(chains=1, steps=50, seed=12, bfgs=oracle.bfgs_params(max_iter=0))
    d, e, ne = oracle.mc_chain(L, G, P, 0, 0)
    assert 1 + 50 <= ne <= 1 + 100
    assert e == pytest.approx(L.score_grad(G, d)["e"], abs=1e-12)


def test_mc_deterministic_and_consistent(oracle, sparse):
    G, L, _ = sparse
    P = oracle.mc_params(chains=6, steps=30, seed=13)
    a = oracle.dock([L], [G], [(0, 0)], P)
    b = oracle.dock([L], [G], [(0, 0)], P, n_threads=1)
    np.testing.assert_array_equal(a["chain_best_e"], b["chain_best_e"])
    np.testing.assert_array_equal(a["chain_best_dof"], b["chain_best_dof"])
    e = a["chain_best_e"][0]
    assert len(set(e.tolist())) == 6          # chains draw independent streams
    for c in range(6):
        d = a["chain_best_dof"][0, c, :L.ndof]
        assert e[c] == pytest.approx(L.score_grad(G, d)["e"], abs=1e-12)
        assert e[c] <= L.score_grad(G, oracle.init_pose(L, G, 13, 0, c))["e"]
    assert a["job_best_e"][0] == e.min() and a["job_best_chain"][0] == int(np.argmin(e))


def test_mc_improves_over_random_poses(oracle, sparse):
    """The search finds poses far better than random ones in the same box."""
    G, L, _ = sparse
    P = oracle.mc_params(chains=4, steps=60, seed=14)
    res = oracle.dock([L], [G], [(0, 0)], P)
    rnd = [L.score_grad(G, oracle.init_pose(L, G, 777, 0, c))["e"] for c in range(200)]
    assert res["job_best_e"][0] < np.percentile(rnd, 1)
    assert res["job_best_e"][0] < 0.0


def _qmul(a, b):
    w1, v1, w2, v2 = a[0], np.asarray(a[1:]), b[0], np.asarray(b[1:])
    return np.concatenate([[w1 * w2 - v1 @ v2], w1 * v2 + w2 * v1 + np.cross(v1, v2)])


def test_mutation_distributions(oracle):
    """The mutation of a Monte Carlo step (Eq. qvina_eq_2, with the readings
    of the step): exactly one entity moves, chosen uniformly among the
    position, the orientation and each torsion; the position by a uniform
    draw from the 2 A ball (radius CDF (r/2)^3, isotropic direction); the
    orientation by a left rotation whose rotation vector is uniform in the
    ball of radius 2 / R_g (angle CDF (theta/theta_max)^3); a torsion is
    redrawn uniformly on [-pi, pi).  Fed with independent uniform words."""
    g = np.random.default_rng(31)
    m = S.tree_ligand(g, 14, 3)
    L = oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    T = L.n_tors
    assert T == 3
    P = oracle.mc_params(chains=1, steps=1, seed=0)
    q0 = g.normal(size=4)
    q0 /= np.linalg.norm(q0)
    x0 = np.concatenate([[1.0, -2.0, 3.0], q0, g.uniform(-np.pi, np.pi, T)])
    N = 24000
    W = g.integers(0, np.iinfo(np.uint64).max, size=(N, 8), dtype=np.uint64, endpoint=True)
    counts = np.zeros(2 + T, np.int64)
    dpos, theta, psi = [], [], []
    q0c = np.concatenate([[q0[0]], -q0[1:]])
    for w in W:
        y = oracle.mutate(L, P, w, x0)
        moved = [np.any(y[:3] != x0[:3]), np.any(y[3:7] != x0[3:7])] + [y[7 + k] != x0[7 + k] for k in range(T)]
        assert sum(moved) == 1, moved
        ent = moved.index(True)
        counts[ent] += 1
        if ent == 0:
            dpos.append(y[:3] - x0[:3])
        elif ent == 1:
            assert abs(np.linalg.norm(y[3:7]) - 1.0) < 1e-12
            dq = _qmul(y[3:7], q0c)
            theta.append(2.0 * np.arccos(min(1.0, abs(dq[0]))))
        else:
            psi.append(y[7 + ent - 2])
    assert stats.chisquare(counts).pvalue > 1e-3, counts
    d = np.array(dpos)
    r = np.linalg.norm(d, axis=1)
    assert r.max() <= 2.0 * (1 + 1e-12)
    assert stats.kstest(r, lambda v: np.clip(v / 2.0, 0, 1) ** 3).pvalue > 1e-3
    u = d / r[:, None]
    assert stats.kstest(u[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3   # Archimedes: cos of the polar angle
    assert np.all(np.abs(u.mean(axis=0)) < 4 / np.sqrt(3 * len(u)))
    th_max = 2.0 / L.rg()
    th = np.array(theta)
    assert th.max() <= th_max * (1 + 1e-9)
    assert stats.kstest(th, lambda v: np.clip(v / th_max, 0, 1) ** 3).pvalue > 1e-3
    p = np.array(psi)
    assert p.min() >= -np.pi and p.max() < np.pi
    assert stats.kstest(p, "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-3


def test_metropolis_acceptance_frequency(oracle):
    """The Monte Carlo step's decision (Eq. qvina_eq_13, read as
    exp((e_i - e_o)/1.2)): at a fixed energy rise the acceptance frequency
    over independent uniform words is exp(-rise/T) within binomial error; a
    fall or a tie is always accepted (the printed form exp(e_i - e_o)/1.2
    would accept a tie only 83 % of the time)."""
    g = np.random.default_rng(41)
    n = 20000
    for T, rise in ((1.2, -1.0), (1.2, 0.0), (1.2, 0.3), (1.2, 1.0), (1.2, 2.5), (0.6, 1.0)):
        words = g.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
        acc = sum(oracle.metropolis_accepts(-3.0, -3.0 + rise, int(w), T) for w in words)
        p = min(1.0, float(np.exp(-rise / T)))
        sd = np.sqrt(max(p * (1 - p), 1.0 / n) / n)
        assert abs(acc / n - p) <= 4 * sd, (T, rise, acc / n, p)

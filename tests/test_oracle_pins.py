"""Pins of the oracle's orientation update and Monte Carlo control flow
against definitions independent of the oracle's own code.

  * the BFGS pose update x (+) lam d (Eq. qvina_eq_9, read in the 6+T
    tangent space) turns the orientation by the LEFT rotation exp(lam d_theta),
    checked against scipy's rotation composition and against the gradient:
    the slope of E along the update must equal g . d, which a right-multiplied
    update violates;
  * the oracle's BFGS reaches the minimum scipy's BFGS reaches when scipy
    works in a rotation-vector chart around the start orientation, on an
    objective that goes through the map lookup, the torsion tree and the
    intra pairs and is smooth (an affine map field, which trilinear
    interpolation reproduces exactly);
  * the Monte Carlo chain (Supplementary Algorithm 2 with Eq. qvina_eq_13,
    Metropolis against the current energy; a new best refined, then made both
    best and current) restated here step by step from the oracle's exported
    pieces replays or_mc_chain bit for bit, while the same restatement with
    one planted mistake does not.
"""
import numpy as np
import pytest
from scipy import optimize
from scipy.spatial.transform import Rotation

from paper_2506_20043_amd import synth as S


def _sp_rot(q):
    """scipy Rotation of a (w, x, y, z) quaternion (scipy is scalar-last)."""
    return Rotation.from_quat([q[1], q[2], q[3], q[0]])


def _wxyz(r):
    x, y, z, w = r.as_quat()
    return np.array([w, x, y, z])


def _skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def _left_jacobian(th):
    """J_l of SO(3): exp(th + e) = exp(J_l(th) e) exp(th) to first order."""
    a = np.linalg.norm(th)
    K = _skew(th)
    if a < 1e-8:
        return np.eye(3) + 0.5 * K
    return np.eye(3) + (1.0 - np.cos(a)) / a ** 2 * K + (a - np.sin(a)) / a ** 3 * (K @ K)


def _sparse_problem(oracle, seed):
    g = np.random.default_rng(seed)
    rx, rt = S.receptor(g, 300, 24.0)
    G = oracle.Grid.build(rx, rt, [12.0, 12.0, 12.0], [16.0] * 3, 0.375, kappa=10.0)
    m = S.tree_ligand(g, 14, 3)
    L = oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    return g, G, L


# ------------------------------------------------------------------ retraction
def test_retraction_is_a_left_rotation(oracle):
    """or_retract: t and psi move additively; the quaternion becomes
    exp(lam d_theta) (x) q, i.e. scipy's from_rotvec(lam d_theta) * R(q),
    unit and with the sign of the product.  A right-multiplied update
    R(q) * from_rotvec(lam d_theta) is a different rotation for generic q."""
    g = np.random.default_rng(11)
    for _ in range(200):
        nt = int(g.integers(0, 6))
        x = np.concatenate([g.normal(size=3) * 5, S.random_quaternions(g, 1)[0].astype(np.float64),
                            g.uniform(-np.pi, np.pi, nt)])
        x[3:7] /= np.linalg.norm(x[3:7])
        d = g.normal(size=6 + nt)
        lam = float(g.uniform(0.01, 2.0))
        o = oracle.retract(nt, x, d, lam)
        np.testing.assert_allclose(o[:3], x[:3] + lam * d[:3], rtol=0, atol=1e-12)
        np.testing.assert_allclose(o[7:], x[7:] + lam * d[6:], rtol=0, atol=1e-12)
        assert abs(np.linalg.norm(o[3:7]) - 1.0) < 1e-12
        left = Rotation.from_rotvec(lam * d[3:6]) * _sp_rot(x[3:7])
        right = _sp_rot(x[3:7]) * Rotation.from_rotvec(lam * d[3:6])
        np.testing.assert_allclose(_sp_rot(o[3:7]).as_matrix(), left.as_matrix(), atol=1e-12)
        assert np.abs(right.as_matrix() - left.as_matrix()).max() > 1e-6
        # the quaternion itself, not only its rotation: the renormalised
        # product, whose sign follows the product's
        w = _wxyz(left)
        assert np.allclose(o[3:7], w, atol=1e-12) or np.allclose(o[3:7], -w, atol=1e-12)


def _slope_along(L, G, x, d, retract, h=1e-6):
    fp = L.score_grad(G, retract(x, d, h))["e"]
    fm = L.score_grad(G, retract(x, d, -h))["e"]
    return (fp - fm) / (2 * h)


def test_retraction_slope_is_gradient_dot_direction(oracle):
    """On a real map objective (receptor maps, torsion tree, intra pairs):
    d/dlam E(x (+) lam d) at lam = 0 equals grad_tan . d, the slope BFGS's
    Armijo and Wolfe tests assume.  Poses near a non-smooth point are
    skipped.  A right-multiplied orientation update, planted here on the
    CPU, breaks the identity on the same poses: the pin can tell them apart."""
    g, G, L = _sparse_problem(oracle, 21)
    lo, hi = G.origin.astype(np.float64) + 2, G.origin + G.h * (G.dims - 1) - 2
    nt = L.n_tors

    def right_retract(x, d, lam):
        o = oracle.retract(nt, x, np.concatenate([d[:3], np.zeros(3), d[6:]]), lam)
        q = _sp_rot(x[3:7]) * Rotation.from_rotvec(lam * d[3:6])
        o[3:7] = _wxyz(q)
        return o

    checked = wrong_detected = 0
    for x in S.poses(g, 60, lo, hi, nt).astype(np.float64):
        x[3:7] /= np.linalg.norm(x[3:7])
        r = L.score_grad(G, x)
        if min(r["min_face"], r["min_cut"], r["min_kink"]) < 1e-3:
            continue
        d = np.zeros(6 + nt)
        d[3:6] = g.normal(size=3)            # rotation only: the part under test
        d[6:] = g.normal(size=nt) * 0.3
        want = r["grad_tan"] @ d
        got = _slope_along(L, G, x, d, lambda a, b, c: oracle.retract(nt, a, b, c))
        assert got == pytest.approx(want, rel=1e-5, abs=1e-5)
        bad = _slope_along(L, G, x, d, right_retract)
        if abs(bad - want) > 1e-3 * (1 + abs(want)):
            wrong_detected += 1
        checked += 1
    assert checked >= 30, checked
    assert wrong_detected >= checked - 2, (wrong_detected, checked)


# ------------------------------------------------------------------ BFGS vs scipy
def _diameter(n, bonds):
    """Largest bond-graph distance of a tree of n atoms."""
    adj = [[] for _ in range(n)]
    for a, b in bonds:
        adj[a].append(b)
        adj[b].append(a)
    best = 0
    for s0 in range(n):
        dist, todo = {s0: 0}, [s0]
        while todo:
            u = todo.pop(0)
            for v in adj[u]:
                if v not in dist:
                    dist[v] = dist[u] + 1
                    todo.append(v)
        best = max(best, max(dist.values()))
    return best


def _affine_problem(oracle, g):
    """A 9-atom ligand at most 5 bonds across (every intra pair inside 8 A)
    of the non-hydrophobic, non-hydrogen-bonding types C_P, N_P and S_P (no
    term kink), over maps holding an affine field per type whose gradients
    a_t sum to zero over the ligand's atoms: e_inter is then a smooth
    function of the orientation and torsions with no pull on the
    translation, and trilinear interpolation reproduces it exactly."""
    while True:
        m = S.tree_ligand(g, 9, 3)
        if m.n_tors < 2 or _diameter(9, m.bonds) > 5:
            continue
        types = np.array([1, 2, 7])[g.integers(0, 3, 9)].astype(np.int32)
        counts = np.array([np.sum(types == t) for t in (1, 2, 7)])
        if np.any(counts == 0):
            continue
        L = oracle.Ligand(m.xyz, types, m.bonds, m.rotatable)
        if L.n_pairs >= 3:
            break
    a1, a2 = g.normal(size=3), g.normal(size=3)
    a3 = -(counts[0] * a1 + counts[1] * a2) / counts[2]
    grad = {1: a1, 2: a2, 7: a3}
    dims, org = oracle.lattice([0.0, 0.0, 0.0], [40.0] * 3, 0.5)
    ax = [org[k].astype(np.float64) + 0.5 * np.arange(dims[k]) for k in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    maps = np.zeros((8, dims[2], dims[1], dims[0]))
    for t, a in grad.items():
        maps[t] = a[0] * X + a[1] * Y + a[2] * Z
    return L, oracle.Grid(maps, dims, org, 0.5, kappa=10.0)


def test_bfgs_matches_scipy_in_rotation_chart(oracle):
    """From starts near a minimum of the smooth map objective, the oracle's
    BFGS (left-rotation update) and scipy's BFGS over the chart
    u -> (t0 + u_t, exp(u_theta) (x) q0, psi0 + u_psi) both converge
    (|g| < 1e-6) to the same energy within 1e-3 kcal/mol.  The chart's
    gradient is J_l(u_theta)^T times the oracle's torque (the left Jacobian
    of SO(3)), so scipy never uses the oracle's update."""
    g = np.random.default_rng(23)
    P = oracle.bfgs_params(max_iter=3000, eps_g=1e-9)
    same = tried = 0
    while tried < 10:
        L, G = _affine_problem(oracle, g)
        x0 = np.concatenate([g.uniform(-3, 3, 3), S.random_quaternions(g, 1)[0].astype(np.float64),
                             g.uniform(-np.pi, np.pi, L.n_tors)])
        x0[3:7] /= np.linalg.norm(x0[3:7])
        xm = oracle.bfgs(L, G, x0, P)[0]
        if np.linalg.norm(L.score_grad(G, xm)["grad_tan"]) > 1e-6:
            continue
        # start a little away from that minimum, rotation included
        pert = np.concatenate([np.zeros(3), g.normal(size=3) * 0.15, g.normal(size=L.n_tors) * 0.15])
        xs = oracle.retract(L.n_tors, xm, pert, 1.0)
        q0 = xs[3:7].copy()

        def fg(u):
            d = xs.copy()
            d[:3] = xs[:3] + u[:3]
            d[3:7] = _wxyz(Rotation.from_rotvec(u[3:6]) * _sp_rot(q0))
            d[7:] = xs[7:] + u[6:]
            r = L.score_grad(G, d)
            gu = r["grad_tan"].copy()
            gu[3:6] = _left_jacobian(u[3:6]).T @ gu[3:6]
            return r["e"], gu

        sp = optimize.minimize(fg, np.zeros(6 + L.n_tors), jac=True, method="BFGS",
                               options=dict(gtol=1e-9, maxiter=5000))
        xo, fo, _, _ = oracle.bfgs(L, G, xs, P)
        assert np.linalg.norm(L.score_grad(G, xo)["grad_tan"]) < 1e-6
        assert np.linalg.norm(sp.jac) < 1e-6
        tried += 1
        same += abs(fo - sp.fun) <= 1e-3
    assert same >= 9, same


# ------------------------------------------------------------------ MC control flow
def _words(seed, job, chain, step):
    """The 8 Philox4x64-10 words of one Monte Carlo step: counter (block, step,
    chain, job), key (seed, 0), blocks 0 and 1, from numpy's Philox (which
    advances its counter by one before each block)."""
    out = []
    for blk in range(2):
        c = blk | step << 64 | chain << 128 | job << 192
        c = (c - 1) % (1 << 256)
        ctr = np.array([(c >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], np.uint64)
        out.extend(np.random.Philox(counter=ctr, key=np.array([seed, 0], np.uint64)).random_raw(4))
    return np.array(out, np.uint64)


def _restated_chain(oracle, L, G, P, job, chain, plant=None):
    """Supplementary Algorithm 2 for one thread, in the order the method
    states it: the initial pose is not optimised and is the first best; each
    step mutates the current pose (Eq. qvina_eq_2), optimises it by RILC-BFGS,
    takes the Metropolis decision against the current energy
    (Eq. qvina_eq_13), and a candidate better than the best is refined by a
    second BFGS and becomes both the best and the current pose."""
    cur = oracle.init_pose(L, G, P.seed, job, chain)
    e_cur = L.score_grad(G, cur)["e"]
    n = 1
    best, e_best = cur.copy(), e_cur
    rp = oracle.bfgs_params(max_iter=P.refine_max_iter, m=P.bfgs.m, ls_max=P.bfgs.ls_max, rho=P.bfgs.rho,
                            sigma=P.bfgs.sigma, eps_g=P.bfgs.eps_g, eps_c=P.bfgs.eps_c)
    refined = 0
    for s in range(P.steps):
        w = _words(P.seed, job, chain, s + 1)
        mut = oracle.mutate(L, P, w, cur)
        opt, e_o, ne, _ = oracle.bfgs(L, G, mut, P.bfgs)
        n += ne
        e_ref = e_best if plant == "metropolis_vs_best" else e_cur
        if oracle.metropolis_accepts(e_ref, e_o, int(w[7]), P.temperature):
            cur, e_cur = opt, e_o
        if e_o < e_best:
            ref, e_r, ne, _ = oracle.bfgs(L, G, opt, rp)
            n += ne
            best, e_best = ref, e_r
            refined += 1
            if plant != "no_current_after_refine":
                cur, e_cur = ref, e_r
    return best, e_best, n, refined


def test_mc_chain_replays_restated_algorithm(oracle):
    """or_mc_chain equals the restatement bit for bit (best pose, best energy,
    evaluation count) on chains where refinement fires, and each planted
    mistake -- the current pose left unrefined after a new best, or the
    Metropolis test taken against the best energy -- changes the outcome of
    at least one of them."""
    g, G, L = _sparse_problem(oracle, 25)
    P = oracle.mc_params(chains=4, steps=12, seed=77, bfgs=oracle.bfgs_params(max_iter=6),
                         refine_max_iter=6)
    differs = {"no_current_after_refine": 0, "metropolis_vs_best": 0}
    fired = 0
    for job, chain in ((0, 0), (0, 1), (3, 2), (5, 3)):
        d, e, ne = oracle.mc_chain(L, G, P, job, chain)
        best, e_best, n, refined = _restated_chain(oracle, L, G, P, job, chain)
        np.testing.assert_array_equal(d, best)
        assert e == e_best and ne == n
        fired += refined > 0
        for plant in differs:
            b2, e2, n2, _ = _restated_chain(oracle, L, G, P, job, chain, plant)
            if not (np.array_equal(b2, d) and e2 == e and n2 == ne):
                differs[plant] += 1
    assert fired >= 3, fired
    assert all(v >= 1 for v in differs.values()), differs

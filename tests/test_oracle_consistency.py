"""Pins of the oracle's first-order consistency check (Eqs. qvina_eq_4 and
qvina_eq_5): constructed sign patterns where each inequality is decided by
hand, the tested coordinate range, the rotation difference and the torsion
wrap, points a tiny step along the current pose's gradient (the check
fails: no optimisation) or against it in one coordinate (it passes), and
the Monte Carlo chain with the check switched on."""
import numpy as np
import pytest

from paper_2506_20043_amd import synth as S

KAPPA = 10.0


def _quat_exp(theta):
    a = np.linalg.norm(theta)
    if a == 0:
        return np.array([1.0, 0, 0, 0])
    return np.concatenate([[np.cos(a / 2)], np.sin(a / 2) * theta / a])


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _pair(dt, theta, dpsi, g=None):
    """y and x = y (+) (dt, theta, dpsi) with a left rotation; gradients
    equal to g (all +1 by default) at both points."""
    rng = np.random.default_rng(0)
    nt = len(dpsi)
    y = np.zeros(7 + nt)
    y[:3] = rng.normal(size=3)
    q = rng.normal(size=4)
    y[3:7] = q / np.linalg.norm(q)
    y[7:] = rng.uniform(-np.pi, np.pi, nt)
    x = y.copy()
    x[:3] += dt
    x[3:7] = _qmul(_quat_exp(np.asarray(theta, float)), y[3:7])
    x[7:] += dpsi
    gg = np.ones(6 + nt) if g is None else np.asarray(g, float)
    return nt, x, y, gg


def _ex(oracle):
    """consistency over every tangent coordinate: the check does not pass"""
    return lambda nt, x, fx, gx, y, fy, gy: not oracle.consistency_passes(nt, x, fx, gx, y, fy, gy)


def test_sign_patterns(oracle):
    ex = _ex(oracle)
    nt, x, y, g = _pair([0.5, 0.3, 0.2], [0.1, 0.2, 0.05], [0.3, 0.4])
    # same gradient signs and every coordinate moved uphill: explained
    assert ex(nt, x, 2.0, g, y, 1.0, g)
    # the reverse energy order puts the secant against the gradient (Eq. 5)
    assert not ex(nt, x, 0.5, g, y, 1.0, g)
    for p in range(6 + nt):
        gy = g.copy()
        gy[p] = -1.0                      # Eq. 4 holds in coordinate p
        assert not ex(nt, x, 2.0, g, y, 1.0, gy), p
        gz = g.copy()
        gz[p] = 0.0                       # a zero sign never explains
        assert not ex(nt, x, 2.0, gz, y, 1.0, g), p
        # only the tested range counts: p alone passes, every other single
        # coordinate stays consistent
        assert oracle.consistency_passes(nt, x, 2.0, g, y, 1.0, gy, p, p + 1)
        for q in range(6 + nt):
            if q != p:
                assert not oracle.consistency_passes(nt, x, 2.0, g, y, 1.0, gy, q, q + 1), (p, q)


def test_rotation_and_torsion_differences(oracle):
    ex = _ex(oracle)
    theta = np.array([0.2, -0.3, 0.1])
    g = np.array([1, 1, 1, 1, -1, 1, 1.0])
    nt, x, y, _ = _pair([0.1, 0.1, 0.1], theta, [0.25], g)
    assert ex(nt, x, 3.0, g, y, 1.0, g)
    xm = x.copy()
    xm[3:7] = -xm[3:7]                    # the same rotation
    assert ex(nt, xm, 3.0, g, y, 1.0, g)
    for k in range(3):                    # a rotation component against its gradient sign
        g2 = g.copy()
        g2[3 + k] = -g2[3 + k]
        assert not ex(nt, x, 3.0, g2, y, 1.0, g2), k
    xw = x.copy()
    xw[7] -= 2 * np.pi                    # torsion difference wraps to +0.25
    assert ex(nt, xw, 3.0, g, y, 1.0, g)
    xf = x.copy()
    xf[7] = y[7] + 3.5                    # wraps to 3.5 - 2 pi < 0
    assert not ex(nt, xf, 3.0, g, y, 1.0, g)


def test_steepest_descent_neighbour_is_explained(oracle):
    """On the tiny configuration's landscape, a point a tiny step down (or
    up) the gradient of y stays on y's slope in every coordinate, so the
    check fails; moving one coordinate the other way makes it pass."""
    cfg = S.CONFIGS["tiny"]
    rx, rt, bxs = S.make_receptor(cfg)
    m = S.make_ligands(cfg)[0]
    b = bxs[0]
    G = oracle.Grid.build(rx, rt, b.center.astype(np.float64), b.size.astype(np.float64), b.spacing, kappa=KAPPA)
    L = oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    g = np.random.default_rng(3)
    lo, hi = G.origin.astype(np.float64) + 3, G.origin + G.h * (G.dims - 1) - 3
    tested = 0
    for y in S.poses(g, 60, lo, hi, L.n_tors).astype(np.float64):
        ry = L.score_grad(G, y)
        gy = ry["grad_tan"]
        # a 1e-5 step moves atoms by ~1e-4 A and the gradient by ~1e-4: keep
        # poses whose gradient signs and one-sided derivatives cannot change
        if (np.min(np.abs(gy)) < 1e-2 or ry["min_face"] < 2e-3 or ry["min_kink"] < 2e-3
                or ry["min_cut"] < 2e-3):
            continue
        for sgn in (-1.0, 1.0):
            step = sgn * 1e-5 * gy / np.linalg.norm(gy)
            x = y.copy()
            x[:3] += step[:3]
            x[3:7] = _qmul(_quat_exp(step[3:6]), y[3:7])
            x[7:] += step[6:]
            rx_ = L.score_grad(G, x)
            assert not oracle.consistency_passes(L.n_tors, x, rx_["e"], rx_["grad_tan"], y, ry["e"], gy)
            x2 = y.copy()
            x2[0] -= sgn * 1e-5 * np.sign(gy[0])          # one coordinate moved the other way
            x2[:3] += step[:3] * np.array([0, 1, 1])
            r2 = L.score_grad(G, x2)
            assert oracle.consistency_passes(L.n_tors, x2, r2["e"], r2["grad_tan"], y, ry["e"], gy)
        tested += 1
    assert tested >= 10


def test_chain_with_the_check(oracle):
    """With the check the chain still returns a best that re-scores to its
    energy, and steps it skips cost one evaluation, so the count falls."""
    cfg = S.CONFIGS["tiny"]
    rx, rt, bxs = S.make_receptor(cfg)
    m = S.make_ligands(cfg)[0]
    b = bxs[0]
    G = oracle.Grid.build(rx, rt, b.center.astype(np.float64), b.size.astype(np.float64), b.spacing, kappa=KAPPA)
    L = oracle.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    seed = S.philox_seed(cfg)
    p0 = oracle.mc_params(chains=4, steps=60, seed=seed)
    p8 = oracle.mc_params(chains=4, steps=60, seed=seed, consistency=True)
    evals0 = evals8 = 0
    for c in range(4):
        d0, e0, n0 = oracle.mc_chain(L, G, p0, 0, c)
        d8, e8, n8 = oracle.mc_chain(L, G, p8, 0, c)
        assert L.score_grad(G, d8)["e"] == pytest.approx(e8, abs=1e-9)
        evals0 += n0
        evals8 += n8
    assert evals8 < evals0

"""Pins of the oracle's receptor surface points and point features (Methods,
"Pocket prediction with P2Rank", Eq. prank_eq_1): an isolated atom keeps
every direction at its radius, two overlapping atoms lose the spherical cap
the closed form of the sphere-sphere intersection predicts, an enclosed atom
keeps none, hand-computed feature values and cutoffs, linearity over atoms,
and translation invariance."""
import numpy as np
import pytest

from paper_2506_20043_amd import synth as S

PROBE = 1.6
RADIUS = {0: 1.9, 2: 1.8, 3: 1.8, 5: 1.7, 7: 2.0}


def test_isolated_atom_keeps_every_direction(oracle):
    dirs = S.sphere_directions(200)
    x = np.array([[1.25, -2.5, 3.0]], np.float32)
    pts, atom = oracle.sas_points(x, [5], dirs, PROBE)
    assert len(pts) == 200 and np.all(atom == 0)
    r = np.float32(1.7) + np.float32(PROBE)
    np.testing.assert_allclose(np.linalg.norm(pts - x, axis=1), r, rtol=1e-6)
    np.testing.assert_allclose((pts - x) / r, dirs, atol=1e-6)


@pytest.mark.parametrize("dist", [1.5, 2.5, 4.0, 5.2])
def test_two_atoms_lose_the_intersection_cap(oracle, dist):
    n = 6000
    dirs = S.sphere_directions(n)
    x = np.array([[0, 0, 0], [dist, 0, 0]], np.float32)
    t = [0, 7]                                  # C_H (1.9) and S_P (2.0)
    pts, atom = oracle.sas_points(x, t, dirs, PROBE)
    ra, rb = 1.9 + PROBE, 2.0 + PROBE
    for a, (r_self, r_other) in enumerate([(ra, rb), (rb, ra)]):
        cos_cap = (r_self ** 2 + dist ** 2 - r_other ** 2) / (2 * r_self * dist)
        lost = (1 - np.clip(cos_cap, -1, 1)) / 2
        kept = np.sum(atom == a)
        assert abs(kept / n - (1 - lost)) < 2e-3, (a, kept / n, 1 - lost)


def test_enclosed_atom_keeps_nothing(oracle):
    dirs = S.sphere_directions(300)
    shell = S.sphere_directions(40).astype(np.float64) * 2.2
    x = np.vstack([[0, 0, 0], shell]).astype(np.float32)
    pts, atom = oracle.sas_points(x, [2] * len(x), dirs, PROBE)
    assert np.sum(atom == 0) == 0
    assert len(pts) > 0


def test_feature_values_and_cutoffs(oracle):
    p = np.array([[0, 0, 0]], np.float32)
    # N_D (donor) at 3 A: weight 0.5 in its type channel and the donor channel
    f = oracle.point_features(np.array([[3, 0, 0]], np.float32), [3], p)[0]
    want = np.zeros(12)
    want[3] = want[9] = 0.5
    want[11] = 1
    np.testing.assert_allclose(f, want, atol=1e-12)
    # C_H at 1.5 A: hydrophobic; O_DA at 4.5 A: donor and acceptor
    f = oracle.point_features(np.array([[0, 1.5, 0], [0, 0, -4.5]], np.float32), [0, 6], p)[0]
    assert f[0] == pytest.approx(0.75) and f[8] == pytest.approx(0.75)
    assert f[6] == pytest.approx(0.25) and f[9] == pytest.approx(0.25) and f[10] == pytest.approx(0.25)
    assert f[11] == 2
    # beyond 6 A no weight, beyond 10 A no protrusion
    f = oracle.point_features(np.array([[6.01, 0, 0], [0, 9.99, 0], [0, 0, 10.01]], np.float32), [1, 1, 1], p)[0]
    assert np.all(f[:11] == 0) and f[11] == 2


def test_features_are_additive_and_translation_invariant(oracle):
    g = np.random.default_rng(5)
    rx, rt = S.receptor(g, 300, 20.0)
    rx = np.round(rx * 1024) / 1024             # dyadic, so shifts below are exact
    dirs = S.sphere_directions(30)
    pts, atom = oracle.sas_points(rx, rt, dirs, PROBE)
    assert 0 < len(pts) < 300 * 30
    f = oracle.point_features(rx, rt, pts)
    half = len(rt) // 2
    fa = oracle.point_features(rx[:half], rt[:half], pts)
    fb = oracle.point_features(rx[half:], rt[half:], pts)
    np.testing.assert_allclose(f, fa + fb, rtol=1e-12, atol=1e-12)
    shift = np.array([3.0, -5.0, 8.0], np.float32)
    pts2, atom2 = oracle.sas_points(rx + shift, rt, dirs, PROBE)
    assert np.array_equal(atom2, atom)
    np.testing.assert_allclose(pts2, pts + shift, atol=1e-5)
    # type channels sum to the flags' channels where the flag applies
    np.testing.assert_allclose(f[:, 8], f[:, 0], atol=1e-12)                   # hydrophobic = C_H
    np.testing.assert_allclose(f[:, 9], f[:, 3] + f[:, 6], atol=1e-12)         # donors N_D, O_DA
    np.testing.assert_allclose(f[:, 10], f[:, 4] + f[:, 5] + f[:, 6], atol=1e-12)

"""GPU parity of the receptor surface points and their Eq. prank_eq_1
features (Methods, "Pocket prediction with P2Rank") against the oracle:
the point set is decided in binary32 on both sides and must match bit for
bit; features within tolerance, protrusion counts exactly."""
import numpy as np
import pytest

from paper_2506_20043_amd import synth as S

pytestmark = pytest.mark.gpu
PROBE = 1.6


@pytest.fixture(scope="module")
def pv_ctx():
    import paper_2506_20043_amd as pv
    return pv.Context(0)


def _check(oracle, pv_ctx, rx, rt, dirs, sample=None):
    import paper_2506_20043_amd as pv
    sas = pv.SurfacePoints(pv_ctx, rx, rt, dirs, PROBE)
    xyz, atom = sas.points()
    feat = sas.features().cpu().numpy()
    xyz, atom = xyz.cpu().numpy(), atom.cpu().numpy()
    sas.close()
    opts, oatom = oracle.sas_points(rx, rt, dirs, PROBE)
    assert len(xyz) == len(opts)
    assert np.array_equal(atom, oatom)
    assert np.array_equal(xyz, opts)
    idx = np.arange(len(opts)) if sample is None else np.random.default_rng(0).choice(len(opts), sample, replace=False)
    ref = oracle.point_features(rx, rt, opts[idx])
    got = feat[idx]
    assert np.array_equal(got[:, 11], ref[:, 11])
    assert np.all(np.abs(got[:, :11] - ref[:, :11]) <= 1e-4 + 1e-5 * np.abs(ref[:, :11]))
    return len(opts)


def test_small_receptor_every_point(oracle, pv_ctx):
    g = np.random.default_rng(11)
    rx, rt = S.receptor(g, 600, 18.0)
    n = _check(oracle, pv_ctx, rx, rt, S.sphere_directions(30))
    assert 0 < n < 600 * 30


def test_multi_pocket_receptor_full_size(oracle, pv_ctx):
    """The 5,000-atom receptor of the multi-pocket workload, 30 directions:
    every point, features at 3,000 sampled points."""
    rx, rt, _ = S.make_receptor(S.CONFIGS["multi_pocket"])
    _check(oracle, pv_ctx, rx, rt, S.sphere_directions(30), sample=3000)


def test_degenerate_receptors(oracle, pv_ctx):
    import paper_2506_20043_amd as pv
    one = np.array([[1.0, 2.0, 3.0]], np.float32)
    assert _check(oracle, pv_ctx, one, np.array([4], np.uint8), S.sphere_directions(7)) == 7
    sas = pv.SurfacePoints(pv_ctx, np.zeros((0, 3), np.float32), np.zeros(0, np.uint8), S.sphere_directions(5))
    assert sas.n_points == 0
    assert sas.features().shape == (0, 12)
    sas.close()


def test_rejects(pv_ctx):
    import paper_2506_20043_amd as pv
    x = np.zeros((2, 3), np.float32)
    d = S.sphere_directions(4)
    for args in ((x, np.array([0, 9], np.uint8), d, PROBE), (x, np.zeros(2, np.uint8), d[:0], PROBE),
                 (x, np.zeros(2, np.uint8), d, -1.0), (x, np.zeros(2, np.uint8), d, float("nan"))):
        with pytest.raises(pv.PvError):
            pv.SurfacePoints(pv_ctx, *args)

"""Host logic of the sensitivity sweeps: mask popcounts and the scaled pose
error of the generator (no GPU)."""
import numpy as np

from paper_2008_06972_amd import synth, sweeps


def test_popcount64():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2 ** 63, 200, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 200).astype(np.uint64)
    want = np.array([bin(int(x)).count("1") for x in a])
    assert np.array_equal(sweeps._popcount64(a), want)
    assert sweeps._popcount64(np.array([0xFFFFFFFFFFFFFFFF], np.uint64))[0] == 64


def test_pose_error_scales_linearly():
    s = synth.SENSORS["c1"]
    base = synth.make_sequence(s, "c1", 11, n_frames=3, key_index=1, imu_noise=0.0)
    one = synth.make_sequence(s, "c1", 11, n_frames=3, key_index=1, imu_noise=1.0)
    two = synth.make_sequence(s, "c1", 11, n_frames=3, key_index=1, imu_noise=2.0)
    assert np.array_equal(base.transforms[1], one.transforms[1])          # the key frame is never perturbed
    d1 = one.transforms[0, :3, 3].astype(np.float64) - base.transforms[0, :3, 3]
    d2 = two.transforms[0, :3, 3].astype(np.float64) - base.transforms[0, :3, 3]
    assert np.abs(d1).max() > 1e-4
    assert np.allclose(d2, 2 * d1, atol=1e-5)

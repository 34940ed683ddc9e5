"""The library's IMU front end (host code, no GPU) against the oracle
(Sec. III-D, Eq. (4)-(5)): FP64 on both sides, FP32 results."""
import numpy as np
import pytest

from paper_2008_06972_amd import pcc
from oracle import imu


@pytest.mark.parametrize("seed", range(6))
def test_imu_transform_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 500))
    dt = float(np.float32(rng.uniform(0.001, 0.02)))
    acc = rng.normal(0, 2, (n, 3)).astype(np.float32)
    gyro = rng.normal(0, 0.5, (n, 3)).astype(np.float32)
    v0 = rng.normal(0, 10, 3).astype(np.float32)
    M, v = pcc.pc_imu_transform(acc, gyro, dt, v0)
    Mo, vo = imu.transform(acc, gyro, dt, v0)
    assert np.allclose(M, Mo, rtol=2e-7, atol=2e-7 * max(1.0, np.abs(Mo).max()))
    assert np.allclose(v, vo, rtol=2e-7, atol=1e-6)


def test_imu_edge_cases():
    M, v = pcc.pc_imu_transform(np.zeros((0, 3)), np.zeros((0, 3)), 0.01)
    assert np.array_equal(M, np.eye(4, dtype=np.float32)) and not v.any()
    with pytest.raises(pcc.PcError):
        pcc.pc_imu_transform(np.zeros((2, 3)), np.zeros((2, 3)), 0.0)
    with pytest.raises(pcc.PcError):
        pcc.pc_imu_transform(np.full((2, 3), np.nan), np.zeros((2, 3)), 0.01)

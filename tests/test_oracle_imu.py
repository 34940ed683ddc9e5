"""Pins of the IMU front-end oracle (Sec. III-D, Eq. (4)-(5)): closed forms of
the explicit-Euler sums, first-order convergence, and the printed rotation
against scipy's Euler-angle rotations."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import imu


def test_no_samples_is_identity():
    M, v = imu.transform(np.zeros((0, 3)), np.zeros((0, 3)), 0.01, v0=[1.0, 2.0, 3.0])
    assert np.array_equal(M, np.eye(4)) and np.array_equal(v, [1.0, 2.0, 3.0])


def test_constant_acceleration_closed_form():
    # Euler: x_n = n v0 dt + a dt^2 n (n - 1) / 2, v_n = v0 + n a dt
    rng = np.random.default_rng(1)
    for n in (1, 2, 7, 100):
        a, v0, dt = rng.normal(size=3), rng.normal(size=3), 0.01
        T, v, ang = imu.integrate(np.tile(a, (n, 1)), np.zeros((n, 3)), dt, v0)
        assert np.allclose(T, n * v0 * dt + a * dt * dt * n * (n - 1) / 2, rtol=1e-12, atol=1e-15)
        assert np.allclose(v, v0 + n * a * dt, rtol=1e-12)
        assert not ang.any()


def test_constant_rates_accumulate_linearly():
    w = np.array([0.3, -0.2, 0.5])
    _, _, ang = imu.integrate(np.zeros((50, 3)), np.tile(w, (50, 1)), 0.02)
    assert np.allclose(ang, 50 * 0.02 * w, rtol=1e-12)


def test_first_order_convergence():
    # a(t) = cos t from rest: exact x(t) = 1 - cos t.  Halving dt halves the error.
    errs = []
    for n in (100, 200, 400):
        dt = 1.0 / n
        t = np.arange(n) * dt
        acc = np.stack([np.cos(t), np.zeros(n), np.zeros(n)], 1)
        T, _, _ = imu.integrate(acc, np.zeros((n, 3)), dt)
        errs.append(abs(T[0] - (1 - math.cos(1.0))))
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


@pytest.mark.parametrize("seed", range(5))
def test_rotation_is_the_printed_product(seed):
    rng = np.random.default_rng(seed)
    a, b, g = rng.uniform(-1.5, 1.5, 3)
    R = imu.rotation(a, b, g)
    # the printed matrices are the right-handed rotations by -alpha about z,
    # -beta about y, -gamma about x, composed in the printed order
    want = Rotation.from_euler("ZYX", [-a, -b, -g]).as_matrix()
    assert np.allclose(R, want, atol=1e-12)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-12) and abs(np.linalg.det(R) - 1) < 1e-12


def test_single_axis_signs():
    a = 0.25
    R = imu.rotation(a, 0.0, 0.0)
    assert np.allclose(R @ [1, 0, 0], [math.cos(a), -math.sin(a), 0])
    R = imu.rotation(0.0, a, 0.0)
    assert np.allclose(R @ [1, 0, 0], [math.cos(a), 0, math.sin(a)])
    R = imu.rotation(0.0, 0.0, a)
    assert np.allclose(R @ [0, 1, 0], [0, math.cos(a), -math.sin(a)])


def test_transform_uses_z_rate_for_alpha():
    n, dt = 10, 0.01
    gyro = np.zeros((n, 3))
    gyro[:, 2] = 1.0                       # about z only
    M, _ = imu.transform(np.zeros((n, 3)), gyro, dt)
    assert np.allclose(M[:3, :3], imu.rotation(n * dt, 0.0, 0.0))

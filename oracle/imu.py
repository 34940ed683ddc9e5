"""CPU oracle of the IMU front end -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It shares no code with the GPU library.

The transform of a predicted frame into the key frame (Sec. III-D,
Eq. (4)-(6)) from IMU samples, in FP64:

* translation ``T = (dx, dy, dz)`` (Eq. (4)): the measured translational
  acceleration integrated twice with the first-order Runge-Kutta (explicit
  Euler) method -- per sample the position advances by the current velocity
  times dt, then the velocity by the sample's acceleration times dt;
* rotational displacements ``(d_alpha, d_beta, d_gamma)``: the measured
  rotational rates integrated once the same way;
* ``R`` (Eq. (5)): the product, in the printed order, of the three printed
  matrices -- a rotation in the x-y plane by d_alpha, in the z-x plane by
  d_beta, in the y-z plane by d_gamma, each with the printed signs (these
  are the transposes of the right-handed rotations by those angles);
* ``M = [R | T]`` maps a frame's points into the key frame (Eq. (6)).

Readings (the paper fixes none of these): the rates are given per body axis
(x, y, z) and feed (d_gamma, d_beta, d_alpha): alpha turns about z, beta
about y, gamma about x; the samples are equally spaced by ``dt``; the
velocity at the first sample is an input (an IMU does not measure it), and
the velocity after the last sample is returned so that intervals can be
chained.
"""
from __future__ import annotations

import math

import numpy as np


def integrate(acc, gyro, dt: float, v0=None):
    """Explicit-Euler integration of n samples: returns (T, v_end, angles)
    with angles = accumulated (about x, about y, about z)."""
    acc = np.asarray(acc, np.float64).reshape(-1, 3)
    gyro = np.asarray(gyro, np.float64).reshape(-1, 3)
    assert len(acc) == len(gyro)
    x = np.zeros(3)
    v = np.zeros(3) if v0 is None else np.asarray(v0, np.float64).reshape(3).copy()
    ang = np.zeros(3)
    for k in range(len(acc)):
        x = x + v * dt
        v = v + acc[k] * dt
        ang = ang + gyro[k] * dt
    return x, v, ang


def rotation(alpha: float, beta: float, gamma: float) -> np.ndarray:
    """Eq. (5) as printed."""
    ca, sa = math.cos(alpha), math.sin(alpha)
    cb, sb = math.cos(beta), math.sin(beta)
    cg, sg = math.cos(gamma), math.sin(gamma)
    first = np.array([[ca, sa, 0.0], [-sa, ca, 0.0], [0.0, 0.0, 1.0]])
    second = np.array([[cb, 0.0, -sb], [0.0, 1.0, 0.0], [sb, 0.0, cb]])
    third = np.array([[1.0, 0.0, 0.0], [0.0, cg, sg], [0.0, -sg, cg]])
    return first @ second @ third


def transform(acc, gyro, dt: float, v0=None):
    """(M (4x4 FP64), velocity after the last sample)."""
    T, v, ang = integrate(acc, gyro, dt, v0)
    gamma, beta, alpha = ang
    M = np.eye(4)
    M[:3, :3] = rotation(alpha, beta, gamma)
    M[:3, 3] = T
    return M, v

// IMU front end (Sec. III-D, Eq. (4)-(5)): the transform of a predicted
// frame into the key frame from equally spaced IMU samples.  Host code: a
// frame interval holds a few hundred samples at most, far too little work
// for a launch.  FP64 accumulation, FP32 results.
//
// Per sample k (explicit Euler, the first-order Runge-Kutta method): the
// position moves by the current velocity times dt, then the velocity by
// the sample's acceleration times dt; each rotational displacement moves by
// the sample's rate times dt.  R is the printed product of three planar
// rotations: by the accumulated z rate in the x-y plane, the y rate in the
// z-x plane, the x rate in the y-z plane, each with the printed signs.
#include <math.h>

#include "pc_internal.h"

namespace pcc {
pc_status set_error(pc_status st, const char *fmt, ...);
}

extern "C" pc_status pc_imu_transform(const float *acc, const float *gyro, int32_t n, float dt, const float *v0,
                                      float *M, float *v_end) {
  using pcc::set_error;
  if (n < 0) return set_error(PC_ERR_ARG, "sample count %d < 0", n);
  if (n > 0 && (!acc || !gyro)) return set_error(PC_ERR_ARG, "samples are NULL");
  if (!M) return set_error(PC_ERR_ARG, "transform output is NULL");
  if (!(dt > 0.0f) || !isfinite(dt)) return set_error(PC_ERR_ARG, "dt must be finite and > 0");
  double pos[3] = {0.0, 0.0, 0.0}, vel[3] = {0.0, 0.0, 0.0}, ang[3] = {0.0, 0.0, 0.0};
  if (v0)
    for (int c = 0; c < 3; c++) {
      if (!isfinite(v0[c])) return set_error(PC_ERR_ARG, "initial velocity is not finite");
      vel[c] = v0[c];
    }
  const double h = dt;
  for (int32_t k = 0; k < n; k++) {
    for (int c = 0; c < 3; c++) {
      const double a = acc[3 * (size_t)k + c], w = gyro[3 * (size_t)k + c];
      if (!isfinite(a) || !isfinite(w)) return set_error(PC_ERR_ARG, "sample %d is not finite", k);
      pos[c] += vel[c] * h;
      vel[c] += a * h;
      ang[c] += w * h;
    }
  }
  // ang = (about x, about y, about z) = (gamma, beta, alpha)
  const double ca = cos(ang[2]), sa = sin(ang[2]), cb = cos(ang[1]), sb = sin(ang[1]), cg = cos(ang[0]),
               sg = sin(ang[0]);
  const double A[3][3] = {{ca, sa, 0.0}, {-sa, ca, 0.0}, {0.0, 0.0, 1.0}};
  const double B[3][3] = {{cb, 0.0, -sb}, {0.0, 1.0, 0.0}, {sb, 0.0, cb}};
  const double G[3][3] = {{1.0, 0.0, 0.0}, {0.0, cg, sg}, {0.0, -sg, cg}};
  double AB[3][3], R[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int k = 0; k < 3; k++) s += A[i][k] * B[k][j];
      AB[i][j] = s;
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int k = 0; k < 3; k++) s += AB[i][k] * G[k][j];
      R[i][j] = s;
    }
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) M[4 * i + j] = (float)R[i][j];
    M[4 * i + 3] = (float)pos[i];
  }
  M[12] = M[13] = M[14] = 0.0f;
  M[15] = 1.0f;
  if (v_end)
    for (int c = 0; c < 3; c++) v_end[c] = (float)vel[c];
  return PC_OK;
}

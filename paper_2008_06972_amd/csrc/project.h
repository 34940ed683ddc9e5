// Point to pixel (Sec. III-B, Eq. (1)-(2)) with the rigid transform of
// predicted frames (Sec. III-D, Eq. (6)), shared by the per-frame
// projection kernel and the batched binning kernels.
//
// All arithmetic that decides a bin is FP32 with the operation order written
// out (explicit fmaf, correctly rounded sqrt and division), so bins are
// reproducible bit for bit.  Row and column come from table comparisons
// against the sensor's cut tangents and column edge vectors; the angle
// estimates that pick the first table entry to compare are only search
// starts, so their accuracy affects the speed, never the bin.
#pragma once
#include "pc_internal.h"

namespace pcc {

// Loads through the global address space (the tables live in device memory).
template <class T>
__device__ __forceinline__ T gload(const T *p) {
  return *(const __attribute__((address_space(1))) T *)p;
}

// Where the row and column walks read the sensor's cut tangents and edge
// vectors: device memory, or a copy of the tables in LDS.
struct TabGlobal {
  const float *cut, *ebx, *eby;
  __device__ __forceinline__ float c(int v) const { return gload(cut + v); }
  __device__ __forceinline__ float ex(int u) const { return gload(ebx + u); }
  __device__ __forceinline__ float ey(int u) const { return gload(eby + u); }
};
struct TabLds {
  typedef const __attribute__((address_space(3))) float lfloat;
  lfloat *cut, *ebx, *eby;
  __device__ __forceinline__ float c(int v) const { return cut[v]; }
  __device__ __forceinline__ float ex(int u) const { return ebx[u]; }
  __device__ __forceinline__ float ey(int u) const { return eby[u]; }
};

// atan on [-1, 1] to about 1e-5 rad: the odd polynomial of Abramowitz &
// Stegun 4.4.49.
__device__ __forceinline__ float atan_unit_as(float x) {
  const float x2 = x * x;
  float p = fmaf(0.0208351f, x2, -0.0851330f);
  p = fmaf(p, x2, 0.1801410f);
  p = fmaf(p, x2, -0.3302995f);
  p = fmaf(p, x2, 0.9998660f);
  return p * x;
}

// atan2 to about 1e-5 rad (octant reduction of the polynomial above);
// (x, y) must not both be zero.
__device__ __forceinline__ float atan2_as(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float a = atan_unit_as(fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay)));
  float t = ay > ax ? 1.57079632679f - a : a;
  t = x < 0.0f ? 3.14159265359f - t : t;
  return y < 0.0f ? -t : t;
}

// Row: the v with cut[v] > q >= cut[v + 1] (cuts descend; the caller has
// checked cut[0] > q >= cut[H]), i.e. the number of interior cuts above q.
// Start at the beam nearest the point's elevation and walk; the answer is
// unique, so the path taken does not change it.
template <class Tab>
__device__ __forceinline__ int row_of(const SensorDev &s, const Tab &tab, float q) {
  const int H = s.H;
  const float e = fabsf(q) <= 1.0f ? atan_unit_as(q)
                                    : copysignf(1.57079632679f, q) - atan_unit_as(__builtin_amdgcn_rcpf(q));
  int v = (int)fmaf(s.elev0 - e, s.inv_de, 0.5f);
  v = min(max(v, 0), H - 1);
  // one branch-free step settles almost every point (the caller's range
  // check keeps v inside [0, H - 1]); the walk below finishes the rest
  {
    const float above = tab.c(v), below = tab.c(v + 1);
    v += (below > q ? 1 : 0) - (above <= q ? 1 : 0);
  }
  {
    const float above = tab.c(v), below = tab.c(v + 1);
    if (above > q && !(below > q)) return v;
  }
  for (int step = 0; step <= H; step++) {
    const float above = tab.c(v), below = tab.c(v + 1);
    if (above <= q) v--;
    else if (below > q) v++;
    else return v;
  }
  return -1;
}

// Row from an estimate qa of q known to within mg: the v with
// cut[v] > q >= cut[v + 1] when qa decides it (both cuts farther than mg
// from qa after one step from the beam nearest the elevation), else -1.
// The caller has checked cut[0] > q >= cut[H].
template <class Tab>
__device__ __forceinline__ int row_near(const SensorDev &s, const Tab &tab, float qa, float mg) {
  const int H = s.H;
  const float e = fabsf(qa) <= 1.0f ? atan_unit_as(qa)
                                     : copysignf(1.57079632679f, qa) - atan_unit_as(__builtin_amdgcn_rcpf(qa));
  int v = (int)fmaf(s.elev0 - e, s.inv_de, 0.5f);
  v = min(max(v, 0), H - 1);
  {
    const float above = tab.c(v), below = tab.c(v + 1);
    v += (below > qa ? 1 : 0) - (above <= qa ? 1 : 0);
  }
  const float above = tab.c(v), below = tab.c(v + 1);
  return (above > qa + mg && below <= qa - mg) ? v : -1;
}

template <class Tab>
__device__ __forceinline__ float edge_side(const Tab &tab, int u, float x, float y) {
  float t = tab.ey(u) * x;
  return fmaf(tab.ex(u), y, -t);
}

// Column: the unique u with side(u) <= 0 < side(u + 1); start from the
// azimuth's bin and walk (the walk ends within one step for any estimate
// error below a bin; it is bounded by W steps in any case).
template <class Tab>
__device__ __forceinline__ int column_of(const SensorDev &s, const Tab &tab, float x, float y) {
  const int W = s.W;
  const float rel = s.beta0 - atan2_as(y, x);      // within (-2 pi, 2 pi]
  int u = (int)floorf(rel * s.inv_dth);
  u = u < 0 ? u + W : u;
  u = u < 0 ? u + W : u;
  u = u >= W ? u - W : u;
  u = u >= W ? u - W : u;
  u = min(max(u, 0), W - 1);
  // one branch-free step; its check needs only the one edge the step did
  // not already evaluate (stepping back: the new leading edge; forward:
  // the new trailing edge)
  {
    const int un = (u + 1 == W) ? 0 : u + 1;
    const float lead = edge_side(tab, u, x, y), next = edge_side(tab, un, x, y);
    const bool back = lead > 0.0f, fwd = !back && next <= 0.0f;
    const int ub = (u == 0) ? W - 1 : u - 1, un2 = (un + 1 == W) ? 0 : un + 1;
    const float other = edge_side(tab, back ? ub : un2, x, y);
    u = back ? ub : (fwd ? un : u);
    if (back ? !(other > 0.0f) : (fwd ? other > 0.0f : true)) return u;
  }
  for (int step = 0; step <= W + 2; step++) {
    const int un = (u + 1 == W) ? 0 : u + 1;
    const float lead = edge_side(tab, u, x, y), next = edge_side(tab, un, x, y);
    if (lead > 0.0f) u = (u == 0) ? W - 1 : u - 1;
    else if (next <= 0.0f) u = un;
    else return u;
  }
  return -1;
}

enum { PROJ_KEPT = 0, PROJ_NONFINITE = 1, PROJ_FOV = 2 };

// Transform (if hasM), range, row and column of one point.  Returns
// PROJ_KEPT with v, u, r set, or why the point is dropped: non-finite
// coordinates or a zero range, or outside the field of view (on the axis,
// above the top or below the bottom edge).
template <class Tab>
__device__ __forceinline__ int project_point(const SensorDev &s, const Tab &tab, const Mat12 &M, int hasM, float x,
                                             float y, float z, int &v, int &u, float &r) {
  if (hasM) {
    const float xx = fmaf(M.m[0], x, fmaf(M.m[1], y, fmaf(M.m[2], z, M.m[3])));
    const float yy = fmaf(M.m[4], x, fmaf(M.m[5], y, fmaf(M.m[6], z, M.m[7])));
    const float zz = fmaf(M.m[8], x, fmaf(M.m[9], y, fmaf(M.m[10], z, M.m[11])));
    x = xx; y = yy; z = zz;
  }
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return PROJ_NONFINITE;
  const float yy2 = y * y;
  const float rho2 = fmaf(x, x, yy2);
  const float zz2 = z * z;
  r = sqrtf(fmaf(x, x, fmaf(y, y, zz2)));
  if (!isfinite(r) || r == 0.0f) return PROJ_NONFINITE;
  if (rho2 < 1e-12f) return PROJ_FOV;
  // The row depends on q = z / sqrt(rho2) (correctly rounded square root
  // and division) only through comparisons with the cut tangents.  The
  // estimate z * rsq(rho2) is within 3e-7 |q| of q (one-ulp reciprocal
  // square root, two roundings on each side), so a cut farther than
  // 1e-6 |q| from it compares the same way with q; only a point that close
  // to a cut (or to the field of view's edges) computes q itself.
  const float qa = z * __builtin_amdgcn_rsqf(rho2);
  const float mg = fmaf(fabsf(qa), 1e-6f, 1e-30f);
  const float top = tab.c(0), bot = tab.c(s.H);
  if (qa - mg >= top || qa + mg < bot) return PROJ_FOV;
  v = -1;
  if (qa + mg < top && qa - mg >= bot) v = row_near(s, tab, qa, mg);
  if (v < 0) {
    const float q = z / sqrtf(rho2);
    if (!(q < top) || q < bot) return PROJ_FOV;
    v = row_of(s, tab, q);
  }
  u = column_of(s, tab, x, y);
  return (v < 0 || u < 0) ? PROJ_FOV : PROJ_KEPT;
}

__device__ __forceinline__ int project_point(const SensorDev &s, const Mat12 &M, int hasM, float x, float y, float z,
                                             int &v, int &u, float &r) {
  return project_point(s, TabGlobal{s.cut, s.ebx, s.eby}, M, hasM, x, y, z, v, u, r);
}

}  // namespace pcc

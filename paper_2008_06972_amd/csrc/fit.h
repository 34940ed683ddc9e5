// Per-tile plane fitting on gfx950: one thread owns one tile.  Sec. III-C:
// least-squares planes fitted in closed form (total least squares: the
// eigenvector of the smallest eigenvalue of the centred scatter matrix),
// stored with the dominant normal component set to one (Eq. (3) is the case
// of the x axis), and tested by casting the pixel's ray onto the plane
// exactly as the decoder does.
//
// A tile's ranges stay in the work-group's LDS copy of the strip and are
// read a tile row at a time; the pixel loops are branch-free.
#pragma once
#include "pc_internal.h"

namespace pcc {

struct Plane {
  int k;
  float a, b, c;
};

// Pixel-centre ray direction from the separable sensor tables, one FP32
// rounding per product: (cos e cos a, cos e sin a, sin e).
struct Dir {
  float x, y, z;
};
__device__ __forceinline__ Dir dir_of(float ce, float se, float ca, float sa) { return Dir{ce * ca, ce * sa, se}; }

// den = d_k + a d_k1 + b d_k2 with the fma order the decoder uses.
__device__ __forceinline__ float plane_den(const Plane &P, const Dir &d) {
  float dk = P.k == 0 ? d.x : (P.k == 1 ? d.y : d.z);
  float dk1 = P.k == 0 ? d.y : d.x;
  float dk2 = P.k == 2 ? d.y : d.z;
  return fmaf(P.b, dk2, fmaf(P.a, dk1, dk));
}

// Range at which the pixel ray meets the plane (correctly rounded division).
__device__ __forceinline__ float ray_cast(const Plane &P, const Dir &d) { return P.c / plane_den(P, d); }

__device__ __forceinline__ bool reproduces_exact(float c, float den, float r, float eps) {
  float t = c / den;
  return isfinite(t) && t > 0.0f && fabsf(t - r) <= eps;
}

// The decoder's test |c/den - r| <= eps, decided with a one-ulp reciprocal
// when the answer is clear by a wide margin and with the correctly rounded
// division otherwise; the result always equals the exact test.
__device__ __forceinline__ bool reproduces(const Plane &P, const Dir &d, float r, float eps) {
  float den = plane_den(P, d);
  float t0 = P.c * __builtin_amdgcn_rcpf(den);
  float diff = fabsf(t0 - r);
  float margin = fmaf(fabsf(t0), 1e-6f, 1e-7f);
  if (diff < eps - margin) return t0 > 0.0f;
  if (diff > eps + margin) return false;
  return reproduces_exact(P.c, den, r, eps);
}

// One-ulp hardware reciprocal, reciprocal square root and square root: the
// FP32 fit only needs to be accurate, not correctly rounded (the decisions
// that must match the decoder bit for bit are made elsewhere).
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// acos to about 7e-5 rad: the polynomial of Abramowitz & Stegun 4.4.45
// (Hastings) on [0, 1], reflected for negative arguments.
__device__ __forceinline__ float acos_as(float x) {
  const float ax = fabsf(x);
  const float poly = fmaf(fmaf(fmaf(-0.0187293f, ax, 0.0742610f), ax, -0.2121144f), ax, 1.5707288f);
  const float a = fsqrt(1.0f - ax) * poly;
  return x < 0.0f ? 3.14159265358979f - a : a;
}

// Dominant axis (ties to the lower axis) and the stored coefficients.
__device__ __forceinline__ Plane stored_form_f32(float nx, float ny, float nz, float c) {
  float ax = fabsf(nx), ay = fabsf(ny), az = fabsf(nz);
  int k = 0;
  float m = ax;
  if (ay > m) { k = 1; m = ay; }
  if (az > m) { k = 2; }
  float nk = k == 0 ? nx : (k == 1 ? ny : nz);
  float n1 = k == 0 ? ny : nx;
  float n2 = k == 2 ? ny : nz;
  float ik = frcp(nk);
  return Plane{k, n1 * ik, n2 * ik, c * ik};
}
__device__ __forceinline__ Plane stored_form_f64(double nx, double ny, double nz, double c) {
  double ax = fabs(nx), ay = fabs(ny), az = fabs(nz);
  int k = 0;
  double m = ax;
  if (ay > m) { k = 1; m = ay; }
  if (az > m) { k = 2; }
  double nk = k == 0 ? nx : (k == 1 ? ny : nz);
  double n1 = k == 0 ? ny : nx;
  double n2 = k == 2 ? ny : nz;
  return Plane{k, (float)(n1 / nk), (float)(n2 / nk), (float)(c / nk)};
}

// ------------------------------------------------------------- eigen-solves
// Eigenvector of eigenvalue l from the best-conditioned cross product of
// two rows of (A - l I).
__device__ __forceinline__ bool cross_eigvec(float a00, float a01, float a02, float a11, float a12, float a22,
                                             float l, float &x, float &y, float &z) {
  float r0x = a00 - l, r0y = a01, r0z = a02;
  float r1x = a01, r1y = a11 - l, r1z = a12;
  float r2x = a02, r2y = a12, r2z = a22 - l;
  float x0 = r0y * r1z - r0z * r1y, y0 = r0z * r1x - r0x * r1z, z0 = r0x * r1y - r0y * r1x;
  float x1 = r0y * r2z - r0z * r2y, y1 = r0z * r2x - r0x * r2z, z1 = r0x * r2y - r0y * r2x;
  float x2 = r1y * r2z - r1z * r2y, y2 = r1z * r2x - r1x * r2z, z2 = r1x * r2y - r1y * r2x;
  float d0 = x0 * x0 + y0 * y0 + z0 * z0, d1 = x1 * x1 + y1 * y1 + z1 * z1, d2 = x2 * x2 + y2 * y2 + z2 * z2;
  float bx = x0, by = y0, bz = z0, bd = d0;
  if (d1 > bd) { bx = x1; by = y1; bz = z1; bd = d1; }
  if (d2 > bd) { bx = x2; by = y2; bz = z2; bd = d2; }
  if (!(bd > 0.0f) || !isfinite(bd)) return false;
  float inv = frsq(bd);
  x = bx * inv; y = by * inv; z = bz * inv;
  return true;
}

// Approximate eigenframe of a symmetric 3x3 in FP32: closed-form eigenvalues
// (trigonometric solution of the characteristic cubic), normal n for the
// smallest and a unit long axis l orthogonal to n.  Only used to rotate the
// scatter before an accurate solve.  False if A is a multiple of I.
__device__ __forceinline__ bool eig3_frame_f32(float a00, float a01, float a02, float a11, float a12, float a22,
                                               float &nx, float &ny, float &nz, float &lx, float &ly, float &lz) {
  float q = (a00 + a11 + a22) * (1.0f / 3.0f);
  float b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
  float off = a01 * a01 + a02 * a02 + a12 * a12;
  float p2 = (b00 * b00 + b11 * b11 + b22 * b22 + 2.0f * off) * (1.0f / 6.0f);
  if (!(p2 > 0.0f)) return false;
  float ip = frsq(p2);
  float p = p2 * ip;
  float c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip, c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
  float det = c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02);
  float rr = fminf(1.0f, fmaxf(-1.0f, 0.5f * det));
  float phi = acos_as(rr) * (1.0f / 3.0f);
  float l3 = q + 2.0f * p * __cosf(phi);
  float l1 = q + 2.0f * p * __cosf(phi + 2.0943951023931953f);
  if (!cross_eigvec(a00, a01, a02, a11, a12, a22, l1, nx, ny, nz)) return false;
  bool okl = cross_eigvec(a00, a01, a02, a11, a12, a22, l3, lx, ly, lz);
  if (okl) {
    float dp = lx * nx + ly * ny + lz * nz;
    lx -= dp * nx; ly -= dp * ny; lz -= dp * nz;
    okl = (lx * lx + ly * ly + lz * lz) > 0.25f;
  }
  if (!okl) {   // l2 close to l3: any unit vector orthogonal to n completes the frame
    float ux = fabsf(nx) <= fabsf(ny) && fabsf(nx) <= fabsf(nz) ? 1.f : 0.f;
    float uy = ux == 0.f && fabsf(ny) <= fabsf(nz) ? 1.f : 0.f;
    float uz = (ux == 0.f && uy == 0.f) ? 1.f : 0.f;
    lx = ny * uz - nz * uy; ly = nz * ux - nx * uz; lz = nx * uy - ny * ux;
  }
  float il = frsq(lx * lx + ly * ly + lz * lz);
  lx *= il; ly *= il; lz *= il;
  return true;
}

__device__ __forceinline__ float t_abs(float x) { return fabsf(x); }
__device__ __forceinline__ double t_abs(double x) { return fabs(x); }
__device__ __forceinline__ float t_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double t_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float t_min(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double t_min(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float t_max(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double t_max(double a, double b) { return fmax(a, b); }

// One Jacobi rotation zeroing a_pq (r is the third index), applied to the
// eigenvector columns p and q.
#define PCC_JACOBI_ROT(T, app, aqq, apq, arp, arq, vp0, vq0, vp1, vq1, vp2, vq2)          \
  if (apq != (T)0) {                                                                       \
    T th_ = (aqq - app) / ((T)2 * apq);                                                    \
    T t_ = (th_ >= (T)0 ? (T)1 : (T)-1) / (t_abs(th_) + t_sqrt(th_ * th_ + (T)1));      \
    T c_ = (T)1 / t_sqrt(t_ * t_ + (T)1), s_ = t_ * c_;                                    \
    T np_ = app - t_ * apq, nq_ = aqq + t_ * apq;                                          \
    T rp_ = c_ * arp - s_ * arq, rq_ = s_ * arp + c_ * arq;                                \
    app = np_; aqq = nq_; apq = (T)0; arp = rp_; arq = rq_;                                \
    T w0_ = c_ * vp0 - s_ * vq0, w1_ = s_ * vp0 + c_ * vq0; vp0 = w0_; vq0 = w1_;          \
    w0_ = c_ * vp1 - s_ * vq1; w1_ = s_ * vp1 + c_ * vq1; vp1 = w0_; vq1 = w1_;             \
    w0_ = c_ * vp2 - s_ * vq2; w1_ = s_ * vp2 + c_ * vq2; vp2 = w0_; vq2 = w1_;             \
  }

// Cyclic Jacobi on a symmetric 3x3 (scalars only, no arrays): returns the
// eigenvector of the smallest eigenvalue and the sorted eigenvalues.
template <class T>
__device__ __forceinline__ void jacobi3(T a00, T a01, T a02, T a11, T a12, T a22, int sweeps, T &vx, T &vy, T &vz,
                                        T &l1, T &l2, T &l3) {
  T v00 = 1, v01 = 0, v02 = 0, v10 = 0, v11 = 1, v12 = 0, v20 = 0, v21 = 0, v22 = 1;
  for (int sweep = 0; sweep < sweeps; sweep++) {
    T off = a01 * a01 + a02 * a02 + a12 * a12;
    T dia = a00 * a00 + a11 * a11 + a22 * a22;
    if (off <= (T)1e-30 * dia || off == (T)0) break;
    PCC_JACOBI_ROT(T, a00, a11, a01, a02, a12, v00, v01, v10, v11, v20, v21)
    PCC_JACOBI_ROT(T, a00, a22, a02, a01, a12, v00, v02, v10, v12, v20, v22)
    PCC_JACOBI_ROT(T, a11, a22, a12, a01, a02, v01, v02, v11, v12, v21, v22)
  }
  T m = a00;
  vx = v00; vy = v10; vz = v20;
  if (a11 < m) { m = a11; vx = v01; vy = v11; vz = v21; }
  if (a22 < m) { m = a22; vx = v02; vy = v12; vz = v22; }
  l1 = t_min(a00, t_min(a11, a22));
  l3 = t_max(a00, t_max(a11, a22));
  l2 = a00 + a11 + a22 - l1 - l3;
}

// The FP32 Jacobi used on the nearly diagonal scatter of the rotated frame,
// with hardware reciprocal and square roots.
__device__ __forceinline__ void jacobi3_f32(float a00, float a01, float a02, float a11, float a12, float a22, int sweeps,
                                            float &vx, float &vy, float &vz, float &l1, float &l2, float &l3) {
  float v00 = 1, v01 = 0, v02 = 0, v10 = 0, v11 = 1, v12 = 0, v20 = 0, v21 = 0, v22 = 1;
#define PCC_JACOBI_ROT_F32(app, aqq, apq, arp, arq, vp0, vq0, vp1, vq1, vp2, vq2)          \
  if (apq != 0.0f) {                                                                        \
    float th_ = (aqq - app) * frcp(2.0f * apq);                                             \
    float r_ = frcp(fabsf(th_) + fsqrt(fmaf(th_, th_, 1.0f)));                              \
    float t_ = th_ >= 0.0f ? r_ : -r_;                                                      \
    float c_ = frsq(fmaf(t_, t_, 1.0f)), s_ = t_ * c_;                                      \
    float np_ = app - t_ * apq, nq_ = aqq + t_ * apq;                                       \
    float rp_ = c_ * arp - s_ * arq, rq_ = s_ * arp + c_ * arq;                             \
    app = np_; aqq = nq_; apq = 0.0f; arp = rp_; arq = rq_;                                 \
    float w0_ = c_ * vp0 - s_ * vq0, w1_ = s_ * vp0 + c_ * vq0; vp0 = w0_; vq0 = w1_;       \
    w0_ = c_ * vp1 - s_ * vq1; w1_ = s_ * vp1 + c_ * vq1; vp1 = w0_; vq1 = w1_;              \
    w0_ = c_ * vp2 - s_ * vq2; w1_ = s_ * vp2 + c_ * vq2; vp2 = w0_; vq2 = w1_;              \
  }
  for (int sweep = 0; sweep < sweeps; sweep++) {
    // the small eigenvalues can be far below the largest: only an exactly
    // diagonal matrix ends the sweeps early
    if (a01 == 0.0f && a02 == 0.0f && a12 == 0.0f) break;
    PCC_JACOBI_ROT_F32(a00, a11, a01, a02, a12, v00, v01, v10, v11, v20, v21)
    PCC_JACOBI_ROT_F32(a00, a22, a02, a01, a12, v00, v02, v10, v12, v20, v22)
    PCC_JACOBI_ROT_F32(a11, a22, a12, a01, a02, v01, v02, v11, v12, v21, v22)
  }
#undef PCC_JACOBI_ROT_F32
  float m = a00;
  vx = v00; vy = v10; vz = v20;
  if (a11 < m) { m = a11; vx = v01; vy = v11; vz = v21; }
  if (a22 < m) { m = a22; vx = v02; vy = v12; vz = v22; }
  l1 = fminf(a00, fminf(a11, a22));
  l3 = fmaxf(a00, fmaxf(a11, a22));
  l2 = a00 + a11 + a22 - l1 - l3;
}

// -------------------------------------------------------------- tile views
// A tile as its owning thread sees it: ranges in LDS (tile-major, the
// tile's 16-byte units XOR-swizzled by sw), the TW column direction tables
// in registers, the TH row tables in LDS (broadcast reads).  Loops go row by
// row: a row's ranges arrive with 128-bit LDS reads and its pixels are
// unrolled.
template <int TH, int TW>
struct TileRows {
  static constexpr int N = TH * TW;
  static constexpr int TWc = TW;
  const float *rp;           // tile base: element j at rp[4 * ((j / 4) ^ sw) + j % 4]
  int sw;
  int i0, i1;                // rows this lane visits in each(): all, or its share when lanes split a tile
  const float *ce, *se;      // TH row tables (LDS)
  float ca[TW], sa[TW];      // column tables of this tile (registers)

  __device__ __forceinline__ float at(int j) const { return rp[(((j >> 2) ^ sw) << 2) | (j & 3)]; }
  // direction of pixel (i, k) for a k known only at run time: the column
  // tables are selected from registers
  __device__ __forceinline__ Dir dir_at(int i, int k) const {
    float c = ca[0], s = sa[0];
#pragma unroll
    for (int q = 1; q < TW; q++) {
      c = k == q ? ca[q] : c;
      s = k == q ? sa[q] : s;
    }
    return dir_of(ce[i], se[i], c, s);
  }

  __device__ __forceinline__ void row(int i, float (&r)[TW]) const {
    const float4 *q = reinterpret_cast<const float4 *>(rp);
#pragma unroll
    for (int k4 = 0; k4 < TW / 4; k4++) {
      float4 v = q[(i * (TW / 4) + k4) ^ sw];
      r[4 * k4] = v.x; r[4 * k4 + 1] = v.y; r[4 * k4 + 2] = v.z; r[4 * k4 + 3] = v.w;
    }
  }
  // f(j, r, d) for every pixel of the tile (r may be 0 for empty pixels)
  // The empty asm makes each pass re-read LDS instead of letting the
  // compiler keep every pixel in registers across refits.
  template <class F>
  __device__ __forceinline__ void each(F f) const {
    asm volatile("" ::: "memory");
#pragma unroll 1
    for (int i = i0; i < i1; i++) {
      float r[TW];
      row(i, r);
      const float cei = ce[i], sei = se[i];
#pragma unroll
      for (int k = 0; k < TW; k++) f(i * TW + k, r[k], dir_of(cei, sei, ca[k], sa[k]));
    }
  }
};

__device__ __forceinline__ float bitw(uint64_t S, int j) { return (float)((S >> j) & 1ull); }

// Combining the partial results of the lanes that share a tile: one lane
// (nothing to combine), or two or four neighbouring lanes, each holding some
// of the tile's rows, combined by butterfly DPP moves so that every lane of
// the group ends with the same bits.
struct LaneOne {
  __device__ __forceinline__ float sum(float x) const { return x; }
  __device__ __forceinline__ uint32_t bor(uint32_t x) const { return x; }
};
struct LanePair {
  __device__ __forceinline__ static int dpp(int x) { return __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false); }
  __device__ __forceinline__ float sum(float x) const { return x + __int_as_float(dpp(__float_as_int(x))); }
  __device__ __forceinline__ uint32_t bor(uint32_t x) const { return x | (uint32_t)dpp((int)x); }
};
struct LaneQuad {
  template <int Ctrl>
  __device__ __forceinline__ static int dpp(int x) {
    return __builtin_amdgcn_update_dpp(x, x, Ctrl, 0xF, 0xF, false);
  }
  __device__ __forceinline__ float sum(float x) const {
    x = x + __int_as_float(dpp<0xB1>(__float_as_int(x)));      // quad_perm(1, 0, 3, 2)
    return x + __int_as_float(dpp<0x4E>(__float_as_int(x)));   // quad_perm(2, 3, 0, 1)
  }
  __device__ __forceinline__ uint32_t bor(uint32_t x) const {
    x |= (uint32_t)dpp<0xB1>((int)x);
    return x | (uint32_t)dpp<0x4E>((int)x);
  }
};

// Pixels of the tile that plane P reproduces within eps (the decoder's
// test).  Branch-free over the pixels with the one-ulp reciprocal; the few
// pixels whose |t - r| lies within rounding reach of eps are decided
// afterwards with the correctly rounded division.
template <int LANES> struct LaneGroup;
template <> struct LaneGroup<1> { typedef LaneOne type; };
template <> struct LaneGroup<2> { typedef LanePair type; };
template <> struct LaneGroup<4> { typedef LaneQuad type; };

template <class Tile, class Red = LaneOne>
__device__ __forceinline__ uint64_t inliers(const Tile &T, const Plane &P, float eps, Red red = Red{}) {
  const bool isx = P.k == 0, isz = P.k == 2;
  uint32_t lo = 0, hi = 0, ulo = 0, uhi = 0;
  T.each([&](int j, float r, const Dir &d) {
    const float dk = isz ? d.z : (isx ? d.x : d.y);
    const float dk1 = isx ? d.y : d.x;
    const float dk2 = isz ? d.y : d.z;
    const float den = fmaf(P.b, dk2, fmaf(P.a, dk1, dk));
    const float t0 = P.c * __builtin_amdgcn_rcpf(den);
    const float diff = fabsf(t0 - r);
    const float margin = fmaf(fabsf(t0), 1e-6f, 1e-7f);
    const bool valid = r > 0.0f;
    const bool sure_in = valid & (diff < eps - margin) & (t0 > 0.0f);
    const bool unsure = valid & !(diff < eps - margin) & !(diff > eps + margin);
    if (j < 32) {
      lo |= (uint32_t)sure_in << (j & 31);
      ulo |= (uint32_t)unsure << (j & 31);
    } else {
      hi |= (uint32_t)sure_in << (j & 31);
      uhi |= (uint32_t)unsure << (j & 31);
    }
  });
  uint64_t m = ((uint64_t)hi << 32) | lo, u = ((uint64_t)uhi << 32) | ulo;
  while (u) {
    const int j = __ffsll((long long)u) - 1;
    u &= u - 1;
    const int i = j / Tile::TWc, k = j % Tile::TWc;
    if (reproduces_exact(P.c, plane_den(P, T.dir_at(i, k)), T.at(j), eps)) m |= 1ull << j;
  }
  return ((uint64_t)red.bor((uint32_t)(m >> 32)) << 32) | red.bor((uint32_t)m);
}

// inliers() with, in the same pass, the sum of r (d_k + a d_k1 + b d_k2)
// over the pixels it keeps (the offset sum of the next temporal iteration),
// accumulated in pixel order exactly as temporal_offset does; a pixel kept
// only after the correctly rounded recheck makes the sum be taken again.
template <class Tile, class Red = LaneOne>
__device__ __forceinline__ uint64_t inliers_offset_sum(const Tile &T, const Plane &P, float eps, float &sum_out,
                                                       Red red = Red{}) {
  const bool isx = P.k == 0, isz = P.k == 2;
  uint32_t lo = 0, hi = 0, ulo = 0, uhi = 0;
  float sum = 0.f;
  T.each([&](int j, float r, const Dir &d) {
    const float dk = isz ? d.z : (isx ? d.x : d.y);
    const float dk1 = isx ? d.y : d.x;
    const float dk2 = isz ? d.y : d.z;
    const float den = fmaf(P.b, dk2, fmaf(P.a, dk1, dk));
    const float t0 = P.c * __builtin_amdgcn_rcpf(den);
    const float diff = fabsf(t0 - r);
    const float margin = fmaf(fabsf(t0), 1e-6f, 1e-7f);
    const bool valid = r > 0.0f;
    const bool sure_in = valid & (diff < eps - margin) & (t0 > 0.0f);
    const bool unsure = valid & !(diff < eps - margin) & !(diff > eps + margin);
    sum = fmaf(r * (sure_in ? 1.0f : 0.0f), den, sum);
    if (j < 32) {
      lo |= (uint32_t)sure_in << (j & 31);
      ulo |= (uint32_t)unsure << (j & 31);
    } else {
      hi |= (uint32_t)sure_in << (j & 31);
      uhi |= (uint32_t)unsure << (j & 31);
    }
  });
  uint64_t m = ((uint64_t)hi << 32) | lo, u = ((uint64_t)uhi << 32) | ulo;
  uint32_t late = 0;
  while (u) {
    const int j = __ffsll((long long)u) - 1;
    u &= u - 1;
    const int i = j / Tile::TWc, k = j % Tile::TWc;
    if (reproduces_exact(P.c, plane_den(P, T.dir_at(i, k)), T.at(j), eps)) {
      m |= 1ull << j;
      late = 1;
    }
  }
  m = ((uint64_t)red.bor((uint32_t)(m >> 32)) << 32) | red.bor((uint32_t)m);
  if (red.bor(late)) {
    sum = 0.f;
    T.each([&](int j, float r, const Dir &d) { sum = fmaf(r * bitw(m, j), plane_den(P, d), sum); });
  }
  sum_out = red.sum(sum);
  return m;
}

// FP64 least squares on the exact products r*d: two-pass centring, Jacobi.
// Rare path (near-degenerate scatter).
template <class Tile>
__device__ __forceinline__ bool fit_plane_f64(const Tile &T, uint64_t S, Plane &P) {
  double m0 = 0, m1 = 0, m2 = 0;
  T.each([&](int j, float rf, const Dir &d) {
    const double r = ((S >> j) & 1ull) ? (double)rf : 0.0;
    m0 = fma(r, (double)d.x, m0);
    m1 = fma(r, (double)d.y, m1);
    m2 = fma(r, (double)d.z, m2);
  });
  const double dn = (double)__popcll(S);
  m0 /= dn; m1 /= dn; m2 /= dn;
  double a00 = 0, a01 = 0, a02 = 0, a11 = 0, a12 = 0, a22 = 0;
  T.each([&](int j, float rf, const Dir &d) {
    const double w = ((S >> j) & 1ull) ? 1.0 : 0.0;
    const double r = (double)rf;
    const double e0 = fma(r, (double)d.x, -m0) * w, e1 = fma(r, (double)d.y, -m1) * w, e2 = fma(r, (double)d.z, -m2) * w;
    a00 = fma(e0, e0, a00); a01 = fma(e0, e1, a01); a02 = fma(e0, e2, a02);
    a11 = fma(e1, e1, a11); a12 = fma(e1, e2, a12); a22 = fma(e2, e2, a22);
  });
  double vx, vy, vz, l1, l2, l3;
  jacobi3<double>(a00, a01, a02, a11, a12, a22, 32, vx, vy, vz, l1, l2, l3);
  if (!(l3 > 0.0) || l2 <= kDegenerate * l3) return false;
  double vn = sqrt(vx * vx + vy * vy + vz * vz);
  vx /= vn; vy /= vn; vz /= vn;
  double c = vx * m0 + vy * m1 + vz * m2;
  P = stored_form_f64(vx, vy, vz, c);
  return true;
}

// Steps 2-3 of the FP32 fit for the pixels in S (n of them): the scatter
// about the point m with each deviation rotated into the orthonormal frame
// (a, l x a, l), its first moments correcting for m not being the mean,
// then Jacobi on the nearly diagonal result, rotated back, and the offset
// through the mean.  False when FP32 cannot decide (the two smallest
// eigenvalues within kNearDegenerate of the largest).
template <class Tile, class Red>
__device__ __forceinline__ bool fit_in_frame(const Tile &T, uint64_t S, float n, float mx, float my, float mz, float ax,
                                             float ay, float az, float lx, float ly, float lz, Plane &P, Red red) {
  const float in = frcp(n);
  float bx = ly * az - lz * ay, by = lz * ax - lx * az, bz = lx * ay - ly * ax;   // a2 = a3 x a1
  float q1 = 0.f, q2 = 0.f, q3 = 0.f;
  float s11 = 0.f, s12 = 0.f, s13 = 0.f, s22 = 0.f, s23 = 0.f, s33 = 0.f;
  T.each([&](int j, float r, const Dir &d) {
    float w = bitw(S, j);
    float ex = fmaf(r, d.x, -mx), ey = fmaf(r, d.y, -my), ez = fmaf(r, d.z, -mz);
    float e1 = fmaf(ax, ex, fmaf(ay, ey, az * ez)) * w;
    float e2 = fmaf(bx, ex, fmaf(by, ey, bz * ez)) * w;
    float e3 = fmaf(lx, ex, fmaf(ly, ey, lz * ez)) * w;
    q1 += e1; q2 += e2; q3 += e3;
    s11 = fmaf(e1, e1, s11); s12 = fmaf(e1, e2, s12); s13 = fmaf(e1, e3, s13);
    s22 = fmaf(e2, e2, s22); s23 = fmaf(e2, e3, s23); s33 = fmaf(e3, e3, s33);
  });
  q1 = red.sum(q1); q2 = red.sum(q2); q3 = red.sum(q3);
  s11 = red.sum(s11); s12 = red.sum(s12); s13 = red.sum(s13);
  s22 = red.sum(s22); s23 = red.sum(s23); s33 = red.sum(s33);
  float u1 = q1 * in, u2 = q2 * in, u3 = q3 * in;    // rounding left in the mean
  s11 -= q1 * u1; s12 -= q1 * u2; s13 -= q1 * u3;
  s22 -= q2 * u2; s23 -= q2 * u3; s33 -= q3 * u3;
  float w1, w2, w3, l1, l2, l3;
  jacobi3_f32(s11, s12, s13, s22, s23, s33, 3, w1, w2, w3, l1, l2, l3);
  if (!((l2 - l1) > kNearDegenerate * l3)) return false;
  float nx = w1 * ax + w2 * bx + w3 * lx;
  float ny = w1 * ay + w2 * by + w3 * ly;
  float nz = w1 * az + w2 * bz + w3 * lz;
  float nn = frsq(nx * nx + ny * ny + nz * nz);
  nx *= nn; ny *= nn; nz *= nn;
  // offset through the exact-product mean: n . mean + n . (mean of e)
  float ux = u1 * ax + u2 * bx + u3 * lx, uy = u1 * ay + u2 * by + u3 * ly, uz = u1 * az + u2 * bz + u3 * lz;
  float c = (nx * mx + ny * my + nz * mz) + (nx * ux + ny * uy + nz * uz);
  P = stored_form_f32(nx, ny, nz, c);
  return true;
}

// Least-squares plane through the pixels in S, FP32:
//  1. sums of the deviations from one of the tile's points, p - p0 =
//     fma(r, d, -p0) (one rounding), and of their products: the mean and an
//     approximate scatter, whose closed-form eigenframe follows;
//  2. the scatter again about the mean with each deviation rotated into
//     that frame, so the small eigen-directions are accumulated free of the
//     large one's rounding (elongated tiles: far ground seen by few beams);
//  3. Jacobi on the nearly diagonal result, rotated back.
// Returns false when FP32 cannot decide: the two smallest eigenvalues are
// within kNearDegenerate of the largest (the caller then fits in FP64).
// Pixels outside S enter every sum with weight 0 (no branches).
template <class Tile, class Red = LaneOne>
__device__ __forceinline__ bool fit_plane_f32(const Tile &T, uint64_t S, Plane &P, Red red = Red{}) {
  float n = (float)__popcll(S);
  // shift: the first pixel in S
  const int j0 = __ffsll((long long)S) - 1;
  const int i0 = j0 / Tile::TWc, k0 = j0 % Tile::TWc;
  const Dir d0 = T.dir_at(i0, k0);
  const float r0 = T.at(j0);
  const float px = r0 * d0.x, py = r0 * d0.y, pz = r0 * d0.z;
  float sx = 0.f, sy = 0.f, sz = 0.f;
  float cxx = 0.f, cxy = 0.f, cxz = 0.f, cyy = 0.f, cyz = 0.f, czz = 0.f;
  T.each([&](int j, float r, const Dir &d) {
    float w = bitw(S, j);
    float ex = fmaf(r, d.x, -px) * w, ey = fmaf(r, d.y, -py) * w, ez = fmaf(r, d.z, -pz) * w;
    sx += ex; sy += ey; sz += ez;
    cxx = fmaf(ex, ex, cxx); cxy = fmaf(ex, ey, cxy); cxz = fmaf(ex, ez, cxz);
    cyy = fmaf(ey, ey, cyy); cyz = fmaf(ey, ez, cyz); czz = fmaf(ez, ez, czz);
  });
  sx = red.sum(sx); sy = red.sum(sy); sz = red.sum(sz);
  cxx = red.sum(cxx); cxy = red.sum(cxy); cxz = red.sum(cxz);
  cyy = red.sum(cyy); cyz = red.sum(cyz); czz = red.sum(czz);
  const float in = frcp(n);
  const float ux0 = sx * in, uy0 = sy * in, uz0 = sz * in;
  cxx -= sx * ux0; cxy -= sx * uy0; cxz -= sx * uz0;
  cyy -= sy * uy0; cyz -= sy * uz0; czz -= sz * uz0;
  const float mx = px + ux0, my = py + uy0, mz = pz + uz0;
  float ax, ay, az, lx, ly, lz;
  if (!eig3_frame_f32(cxx, cxy, cxz, cyy, cyz, czz, ax, ay, az, lx, ly, lz)) return false;
  return fit_in_frame(T, S, n, mx, my, mz, ax, ay, az, lx, ly, lz, P, red);
}

// The FP32 fit of a refit (iteration two on): the previous fit's normal
// serves as the frame's first axis, the direction from the first to the
// last pixel of S (made orthogonal to it) as its third, and the first
// pixel as the point m, so the fit takes one pass over the tile (the first
// moments in the frame carry the mean exactly).  When the pixels lie close
// to a line, that direction is the line's, which the frame must carry for
// the in-plane scatter to stay well resolved in FP32.
template <class Tile, class Red = LaneOne>
__device__ __forceinline__ bool refit_plane_f32(const Tile &T, uint64_t S, const Plane &prev, Plane &P, Red red = Red{}) {
  const float n = (float)__popcll(S);
  const int j0 = __ffsll((long long)S) - 1, j1 = 63 - __clzll((long long)S);
  const Dir d0 = T.dir_at(j0 / Tile::TWc, j0 % Tile::TWc), d1 = T.dir_at(j1 / Tile::TWc, j1 % Tile::TWc);
  const float r0 = T.at(j0), r1 = T.at(j1);
  const float mx = r0 * d0.x, my = r0 * d0.y, mz = r0 * d0.z;
  // unit normal of the previous stored form (1, a, b) on axes (k, k1, k2)
  float ax = prev.k == 0 ? 1.0f : prev.a, ay = prev.k == 1 ? 1.0f : (prev.k == 0 ? prev.a : prev.b),
        az = prev.k == 2 ? 1.0f : prev.b;
  const float na = frsq(ax * ax + ay * ay + az * az);
  ax *= na; ay *= na; az *= na;
  // first-to-last pixel, orthogonal to the normal
  float lx = fmaf(r1, d1.x, -mx), ly = fmaf(r1, d1.y, -my), lz = fmaf(r1, d1.z, -mz);
  const float dp = lx * ax + ly * ay + lz * az;
  lx -= dp * ax; ly -= dp * ay; lz -= dp * az;
  float ll = lx * lx + ly * ly + lz * lz;
  if (!(ll > 1e-12f)) {     // along the normal: any unit vector orthogonal to it
    const float ux = fabsf(ax) <= fabsf(ay) && fabsf(ax) <= fabsf(az) ? 1.f : 0.f;
    const float uy = ux == 0.f && fabsf(ay) <= fabsf(az) ? 1.f : 0.f;
    const float uz = (ux == 0.f && uy == 0.f) ? 1.f : 0.f;
    lx = ay * uz - az * uy; ly = az * ux - ax * uz; lz = ax * uy - ay * ux;
    ll = lx * lx + ly * ly + lz * lz;
  }
  const float il = frsq(ll);
  lx *= il; ly *= il; lz *= il;
  return fit_in_frame(T, S, n, mx, my, mz, ax, ay, az, lx, ly, lz, P, red);
}

// Points a tile must keep on its plane: max(min(min_pts, n), ceil(rho n)),
// tabulated on the host in FP64.
__device__ __forceinline__ int need_of(const EncParams &p, int n) { return p.need[n]; }

// Offset of the key plane's stored form (normal held) through the pixels in
// S: the mean of r * (d_k + a d_k1 + b d_k2) (Sec. III-D).
template <class Tile, class Red = LaneOne>
__device__ __forceinline__ float temporal_offset(const Tile &T, const Plane &Q, uint64_t S, Red red = Red{}) {
  float sum = 0.f;
  T.each([&](int j, float r, const Dir &d) { sum = fmaf(r * bitw(S, j), plane_den(Q, d), sum); });
  return red.sum(sum) / (float)__popcll(S);
}

}  // namespace pcc

// Per-tile plane fitting on gfx950: one thread owns one tile and reads it
// from the work-group's LDS copy of the strip.  Sec. III-C: least-squares planes fitted in closed
// form (total least squares: the eigenvector of the smallest eigenvalue of
// the centred scatter matrix), stored with the dominant normal component
// set to one (Eq. (3) is the case of the x axis), and tested by casting the
// pixel's ray onto the plane exactly as the decoder does.
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

__device__ __forceinline__ bool reproduces(const Plane &P, const Dir &d, float r, float eps) {
  float t = ray_cast(P, d);
  return isfinite(t) && t > 0.0f && fabsf(t - r) <= eps;
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
  return Plane{k, n1 / nk, n2 / nk, c / nk};
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

// Symmetric 3x3 eigen-solve, FP32, closed form (trigonometric solution of
// the characteristic cubic); eigenvectors of the smallest and largest
// eigenvalues from the best-conditioned cross product of rows of (A - l I).
// Only used to build an approximate eigenframe; returns false if the
// matrix is (numerically) a multiple of the identity or a vector vanishes.
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
  float inv = 1.0f / sqrtf(bd);
  x = bx * inv; y = by * inv; z = bz * inv;
  return true;
}

__device__ __forceinline__ bool eig3_frame_f32(float a00, float a01, float a02, float a11, float a12, float a22,
                                               float &nx, float &ny, float &nz, float &lx, float &ly, float &lz) {
  float q = (a00 + a11 + a22) * (1.0f / 3.0f);
  float b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
  float off = a01 * a01 + a02 * a02 + a12 * a12;
  float p2 = (b00 * b00 + b11 * b11 + b22 * b22 + 2.0f * off) * (1.0f / 6.0f);
  if (!(p2 > 0.0f)) return false;
  float p = sqrtf(p2);
  float ip = 1.0f / p;
  float c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip, c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
  float det = c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02);
  float rr = fminf(1.0f, fmaxf(-1.0f, 0.5f * det));
  float phi = acosf(rr) * (1.0f / 3.0f);
  float l3 = q + 2.0f * p * cosf(phi);
  float l1 = q + 2.0f * p * cosf(phi + 2.0943951023931953f);
  if (!cross_eigvec(a00, a01, a02, a11, a12, a22, l1, nx, ny, nz)) return false;
  // the long axis only completes the frame: any unit vector orthogonal to
  // the normal estimate will do when it is ill-defined (l2 close to l3)
  float dp = 0.f;
  bool okl = cross_eigvec(a00, a01, a02, a11, a12, a22, l3, lx, ly, lz);
  if (okl) {
    dp = lx * nx + ly * ny + lz * nz;
    lx -= dp * nx; ly -= dp * ny; lz -= dp * nz;
    okl = (lx * lx + ly * ly + lz * lz) > 0.25f;
  }
  if (!okl) {
    float ux = fabsf(nx) <= fabsf(ny) && fabsf(nx) <= fabsf(nz) ? 1.f : 0.f;
    float uy = ux == 0.f && fabsf(ny) <= fabsf(nz) ? 1.f : 0.f;
    float uz = (ux == 0.f && uy == 0.f) ? 1.f : 0.f;
    lx = ny * uz - nz * uy; ly = nz * ux - nx * uz; lz = nx * uy - ny * ux;
  }
  float il = 1.0f / sqrtf(lx * lx + ly * ly + lz * lz);
  lx *= il; ly *= il; lz *= il;
  return true;
}

// Cyclic Jacobi on a symmetric 3x3 in FP32, few sweeps (the refined
// matrices are nearly diagonal).  Returns the eigenvector of the smallest
// eigenvalue and the sorted eigenvalues.
__device__ __forceinline__ void jacobi3_f32(float a00, float a01, float a02, float a11, float a12, float a22,
                                            float &vx, float &vy, float &vz, float &l1, float &l2, float &l3) {
  float v00 = 1.f, v01 = 0.f, v02 = 0.f, v10 = 0.f, v11 = 1.f, v12 = 0.f, v20 = 0.f, v21 = 0.f, v22 = 1.f;
  // one rotation zeroing a_pq; the rest of row/column update follows
#define PCC_ROT(app, aqq, apq, arp, arq, vp0, vq0, vp1, vq1, vp2, vq2)                                  \
  if (apq != 0.0f) {                                                                                    \
    float th = (aqq - app) / (2.0f * apq);                                                              \
    float t = (th >= 0.f ? 1.f : -1.f) / (fabsf(th) + sqrtf(fmaf(th, th, 1.0f)));                      \
    float c = 1.0f / sqrtf(fmaf(t, t, 1.0f)), sn = t * c;                                               \
    float np_ = app - t * apq, nq_ = aqq + t * apq;                                                     \
    float rp = c * arp - sn * arq, rq = sn * arp + c * arq;                                              \
    app = np_; aqq = nq_; apq = 0.0f; arp = rp; arq = rq;                                               \
    float w0 = c * vp0 - sn * vq0, w1 = sn * vp0 + c * vq0; vp0 = w0; vq0 = w1;                         \
    w0 = c * vp1 - sn * vq1; w1 = sn * vp1 + c * vq1; vp1 = w0; vq1 = w1;                                \
    w0 = c * vp2 - sn * vq2; w1 = sn * vp2 + c * vq2; vp2 = w0; vq2 = w1;                                \
  }
  for (int sweep = 0; sweep < 4; sweep++) {
    PCC_ROT(a00, a11, a01, a02, a12, v00, v01, v10, v11, v20, v21)   // (p,q)=(0,1), r=2
    PCC_ROT(a00, a22, a02, a01, a12, v00, v02, v10, v12, v20, v22)   // (0,2), r=1
    PCC_ROT(a11, a22, a12, a01, a02, v01, v02, v11, v12, v21, v22)   // (1,2), r=0
  }
#undef PCC_ROT
  // smallest eigenvalue's column
  float m = a00;
  vx = v00; vy = v10; vz = v20;
  if (a11 < m) { m = a11; vx = v01; vy = v11; vz = v21; }
  if (a22 < m) { m = a22; vx = v02; vy = v12; vz = v22; }
  l1 = fminf(a00, fminf(a11, a22));
  l3 = fmaxf(a00, fmaxf(a11, a22));
  l2 = a00 + a11 + a22 - l1 - l3;
}

// FP64 cyclic Jacobi (near-degenerate scatter matrices).  Eigenvalues on the
// diagonal, eigenvectors in the columns of V.
__device__ inline void jacobi3_f64(double A[3][3], double V[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 32; sweep++) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-30 * dia || off == 0.0) break;
#pragma unroll
    for (int pq = 0; pq < 3; pq++) {
      int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      if (A[p][q] == 0.0) continue;
      double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
      double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
      }
    }
  }
}

// One tile as seen by the thread that owns it: ranges in LDS (tile-major,
// padded stride), direction tables of its rows and columns in LDS.
template <int TH, int TW>
struct TileView {
  static constexpr int N = TH * TW;
  const float *r;            // N ranges of the tile, slot j = i*TW + k
  const float *ce, *se;      // TH row tables of the strip
  const float *ca, *sa;      // TW column tables of the tile
  uint64_t V;                // valid pixels
  int nV;

  __device__ __forceinline__ Dir d(int j) const {
    int i = j / TW, k = j % TW;
    return dir_of(ce[i], se[i], ca[k], sa[k]);
  }
};

// Pixels of the tile that plane P reproduces within eps.
template <int TH, int TW>
__device__ __forceinline__ uint64_t inliers(const TileView<TH, TW> &T, const Plane &P, float eps) {
  uint64_t m = 0;
#pragma unroll 2
  for (int j = 0; j < TH * TW; j++) {
    if (!((T.V >> j) & 1ull)) continue;
    if (reproduces(P, T.d(j), T.r[j], eps)) m |= 1ull << j;
  }
  return m;
}

// FP64 least squares on the exact products r*d: two-pass centring, Jacobi.
template <int TH, int TW>
__device__ __noinline__ bool fit_plane_f64(const TileView<TH, TW> &T, uint64_t S, Plane &P) {
  constexpr int N = TH * TW;
  double m0 = 0, m1 = 0, m2 = 0;
  for (int j = 0; j < N; j++) {
    if (!((S >> j) & 1ull)) continue;
    Dir d = T.d(j);
    double r = (double)T.r[j];
    m0 += r * (double)d.x; m1 += r * (double)d.y; m2 += r * (double)d.z;
  }
  double dn = (double)__popcll(S);
  m0 /= dn; m1 /= dn; m2 /= dn;
  double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int j = 0; j < N; j++) {
    if (!((S >> j) & 1ull)) continue;
    Dir d = T.d(j);
    double r = (double)T.r[j];
    double e0 = r * (double)d.x - m0, e1 = r * (double)d.y - m1, e2 = r * (double)d.z - m2;
    A[0][0] += e0 * e0; A[0][1] += e0 * e1; A[0][2] += e0 * e2;
    A[1][1] += e1 * e1; A[1][2] += e1 * e2; A[2][2] += e2 * e2;
  }
  A[1][0] = A[0][1]; A[2][0] = A[0][2]; A[2][1] = A[1][2];
  double V[3][3];
  jacobi3_f64(A, V);
  // order the eigenvalues (explicit selects: no dynamic register indexing)
  double l0 = A[0][0], l1 = A[1][1], l2 = A[2][2];
  double lmin = fmin(l0, fmin(l1, l2)), lmax = fmax(l0, fmax(l1, l2));
  double lmid = l0 + l1 + l2 - lmin - lmax;
  if (!(lmax > 0.0) || lmid <= kDegenerate * lmax) return false;
  int i0 = (l0 == lmin) ? 0 : ((l1 == lmin) ? 1 : 2);
  double vx = i0 == 0 ? V[0][0] : (i0 == 1 ? V[0][1] : V[0][2]);
  double vy = i0 == 0 ? V[1][0] : (i0 == 1 ? V[1][1] : V[1][2]);
  double vz = i0 == 0 ? V[2][0] : (i0 == 1 ? V[2][1] : V[2][2]);
  double vn = sqrt(vx * vx + vy * vy + vz * vz);
  vx /= vn; vy /= vn; vz /= vn;
  double c = vx * m0 + vy * m1 + vz * m2;
  P = stored_form_f64(vx, vy, vz, c);
  return true;
}

// Least-squares plane through the pixels in S, FP32:
//  1. mean of r*d;
//  2. scatter of the deviations e = fma(r, d, -mean) (one rounding from the
//     exact product) and a closed-form eigenframe of it;
//  3. the scatter again, with each deviation rotated into that frame, so the
//     small eigen-directions are accumulated free of the large one's
//     rounding (elongated tiles: far ground seen by few beams);
//  4. Jacobi on the nearly diagonal result, rotated back.
// FP64 on the exact products when the two smallest eigenvalues are within
// kNearDegenerate of the largest.  Returns false if degenerate.
template <int TH, int TW>
__device__ __forceinline__ bool fit_plane(const TileView<TH, TW> &T, uint64_t S, Plane &P, int &fp64) {
  constexpr int N = TH * TW;
  float n = (float)__popcll(S);
  float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll 2
  for (int j = 0; j < N; j++) {
    if (!((S >> j) & 1ull)) continue;
    Dir d = T.d(j);
    float r = T.r[j];
    sx = fmaf(r, d.x, sx);
    sy = fmaf(r, d.y, sy);
    sz = fmaf(r, d.z, sz);
  }
  float mx = sx / n, my = sy / n, mz = sz / n;
  float cxx = 0.f, cxy = 0.f, cxz = 0.f, cyy = 0.f, cyz = 0.f, czz = 0.f;
#pragma unroll 2
  for (int j = 0; j < N; j++) {
    if (!((S >> j) & 1ull)) continue;
    Dir d = T.d(j);
    float r = T.r[j];
    float ex = fmaf(r, d.x, -mx), ey = fmaf(r, d.y, -my), ez = fmaf(r, d.z, -mz);
    cxx = fmaf(ex, ex, cxx); cxy = fmaf(ex, ey, cxy); cxz = fmaf(ex, ez, cxz);
    cyy = fmaf(ey, ey, cyy); cyz = fmaf(ey, ez, cyz); czz = fmaf(ez, ez, czz);
  }
  float ax, ay, az, lx, ly, lz;
  bool ok = eig3_frame_f32(cxx, cxy, cxz, cyy, cyz, czz, ax, ay, az, lx, ly, lz);
  if (ok) {
    // orthonormal frame: a1 = normal estimate, a3 = long axis, a2 = a3 x a1
    {
      float bx = ly * az - lz * ay, by = lz * ax - lx * az, bz = lx * ay - ly * ax;
      float q1 = 0.f, q2 = 0.f, q3 = 0.f;
      float s11 = 0.f, s12 = 0.f, s13 = 0.f, s22 = 0.f, s23 = 0.f, s33 = 0.f;
#pragma unroll 2
      for (int j = 0; j < N; j++) {
        if (!((S >> j) & 1ull)) continue;
        Dir d = T.d(j);
        float r = T.r[j];
        float ex = fmaf(r, d.x, -mx), ey = fmaf(r, d.y, -my), ez = fmaf(r, d.z, -mz);
        float e1 = fmaf(ax, ex, fmaf(ay, ey, az * ez));
        float e2 = fmaf(bx, ex, fmaf(by, ey, bz * ez));
        float e3 = fmaf(lx, ex, fmaf(ly, ey, lz * ez));
        q1 += e1; q2 += e2; q3 += e3;
        s11 = fmaf(e1, e1, s11); s12 = fmaf(e1, e2, s12); s13 = fmaf(e1, e3, s13);
        s22 = fmaf(e2, e2, s22); s23 = fmaf(e2, e3, s23); s33 = fmaf(e3, e3, s33);
      }
      float in = 1.0f / n;
      float u1 = q1 * in, u2 = q2 * in, u3 = q3 * in;    // rounding left in the mean
      s11 -= q1 * u1; s12 -= q1 * u2; s13 -= q1 * u3;
      s22 -= q2 * u2; s23 -= q2 * u3; s33 -= q3 * u3;
      float w1, w2, w3, l1, l2, l3;
      jacobi3_f32(s11, s12, s13, s22, s23, s33, w1, w2, w3, l1, l2, l3);
      ok = (l2 - l1) > kNearDegenerate * l3;
      if (ok) {
        float nx = w1 * ax + w2 * bx + w3 * lx;
        float ny = w1 * ay + w2 * by + w3 * ly;
        float nz = w1 * az + w2 * bz + w3 * lz;
        float nn = 1.0f / sqrtf(nx * nx + ny * ny + nz * nz);
        nx *= nn; ny *= nn; nz *= nn;
        // offset through the exact-product mean: n . mean + n . (mean of e)
        float ux = u1 * ax + u2 * bx + u3 * lx, uy = u1 * ay + u2 * by + u3 * ly, uz = u1 * az + u2 * bz + u3 * lz;
        float c = (nx * mx + ny * my + nz * mz) + (nx * ux + ny * uy + nz * uz);
        P = stored_form_f32(nx, ny, nz, c);
        return true;
      }
    }
  }
  fp64++;
  return fit_plane_f64<TH, TW>(T, S, P);
}

struct FitResult {
  Plane P;
  uint64_t mask;
  int status, iters;
};

// Points a tile must keep on its plane: max(min(min_pts, n), ceil(rho n)).
__device__ __forceinline__ int need_of(const EncParams &p, int n) {
  int a = n < p.min_pts ? n : p.min_pts;
  int b = (int)ceil((double)p.rho * (double)n);
  return a > b ? a : b;
}

// Own fit of a tile: fit, keep the pixels the plane reproduces, refit on
// them, up to max_iter fits (converged when the kept set stops changing).
template <int TH, int TW>
__device__ inline FitResult own_fit(const TileView<TH, TW> &T, const EncParams &p, int &fits, int &fp64) {
  FitResult R{Plane{0, 0.f, 0.f, 0.f}, 0ull, ST_EMPTY, 0};
  if (T.nV == 0) return R;
  if (T.nV < p.min_pts) { R.status = ST_FEW; return R; }
  uint64_t S = T.V;
  for (int it = 1; it <= p.max_iter; it++) {
    R.iters = it;
    fits++;
    if (!fit_plane<TH, TW>(T, S, R.P, fp64)) {
      R.status = ST_DEGENERATE;
      R.mask = 0;
      return R;
    }
    uint64_t S2 = inliers<TH, TW>(T, R.P, p.eps);
    R.mask = S2;
    if (S2 == S) break;
    if (__popcll(S2) < p.min_pts) {
      R.status = ST_FAILED;
      R.mask = 0;
      return R;
    }
    S = S2;
  }
  R.status = __popcll(R.mask) >= need_of(p, T.nV) ? ST_ACCEPTED : ST_REJECTED;
  return R;
}

// Temporal fit (Sec. III-D): the key plane's normal (k, a, b) is held and
// only the offset varies; in the stored form the offset is the mean of
// r * (d_k + a d_k1 + b d_k2) over the pixels kept.
template <int TH, int TW>
__device__ inline FitResult temporal_fit(const TileView<TH, TW> &T, Plane Q, const EncParams &p) {
  constexpr int N = TH * TW;
  FitResult R{Q, 0ull, 1, 0};
  if (T.nV < p.min_pts) return R;
  uint64_t S = T.V;
  for (int it = 1; it <= p.max_iter; it++) {
    R.iters = it;
    float sum = 0.f;
#pragma unroll 2
    for (int j = 0; j < N; j++) {
      if (!((S >> j) & 1ull)) continue;
      sum = fmaf(T.r[j], plane_den(Q, T.d(j)), sum);
    }
    R.P.c = sum / (float)__popcll(S);
    uint64_t S2 = inliers<TH, TW>(T, R.P, p.eps);
    R.mask = S2;
    if (S2 == S) break;
    if (__popcll(S2) < p.min_pts) {
      R.mask = 0;
      return R;
    }
    S = S2;
  }
  R.status = __popcll(R.mask) >= need_of(p, T.nV) ? 2 : 1;
  return R;
}

}  // namespace pcc

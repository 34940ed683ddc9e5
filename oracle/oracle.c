/*
 * CPU oracle for the spatio-temporal LiDAR range-image encoder
 * (Feng, Liu, Zhu, "Real-Time Spatio-Temporal LiDAR Point Cloud Compression").
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the GPU library.  Plain loops, written
 * for a reader to check against the paper; no blocking, fusion or reordering.
 *
 * Section map:
 *   range image conversion ........ Sec. III-B, Eq. (1)-(2); collisions Sec. III-D
 *   rigid transform of P-frames ... Sec. III-D, Eq. (6)
 *   plane model and ray casting ... Sec. III-C, Eq. (3)
 *   tiling, growth, least squares . Sec. III-C
 *   run format [s, len, P] ........ Sec. III-C (row-wise three-tuples)
 *   temporal reuse with c' free ... Sec. III-D (Encoding paragraph)
 *   lossless stage (Huffman) ...... Sec. III-A
 * Readings where the paper is silent or ambiguous are listed in the repository
 * design notes and referred to here by their short names (e.g. "dominant-axis
 * form").  Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math: the FP32
 * decisions below must round exactly as written).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------------ */
/* Sensor tables (Sec. III-B).  FP64 trigonometry rounded once to FP32.      */
/* ------------------------------------------------------------------------ */
void orc_tables(int H, int W, const float *elev, float az0, float *cut, float *ebx, float *eby,
                float *ce, float *se, float *ca, float *sa) {
  double dth = TWO_PI / (double)W;
  /* Rows: beam v covers elevations between the midpoints to its neighbours;
   * the outer beams extend half a gap beyond themselves (the field of view). */
  double top = (double)elev[0] + 0.5 * ((double)elev[0] - (double)elev[1]);
  double bot = (double)elev[H - 1] - 0.5 * ((double)elev[H - 2] - (double)elev[H - 1]);
  cut[0] = (float)tan(top);
  for (int v = 1; v < H; v++) cut[v] = (float)tan(0.5 * ((double)elev[v - 1] + (double)elev[v]));
  cut[H] = (float)tan(bot);
  for (int v = 0; v < H; v++) {
    ce[v] = (float)cos((double)elev[v]);
    se[v] = (float)sin((double)elev[v]);
  }
  /* Columns advance clockwise from az0: column u spans (beta_u - dth, beta_u]. */
  for (int u = 0; u < W; u++) {
    double beta = (double)az0 - (double)u * dth;
    double alpha = (double)az0 - ((double)u + 0.5) * dth;
    ebx[u] = (float)cos(beta);
    eby[u] = (float)sin(beta);
    ca[u] = (float)cos(alpha);
    sa[u] = (float)sin(alpha);
  }
}

/* Pixel-centre ray direction, FP32: (cos e cos a, cos e sin a, sin e), one
 * rounding per product of table values. */
static void direction(const orc_sensor *s, int v, int u, float d[3]) {
  d[0] = s->ce[v] * s->ca[u];
  d[1] = s->ce[v] * s->sa[u];
  d[2] = s->se[v];
}

/* Sign test of a point against the leading edge of column u:
 * cross(edge_u, (x, y)) = ex*y - ey*x, with ey*x rounded first and one fma. */
static float edge_side(const orc_sensor *s, int u, float x, float y) {
  float t = s->eby[u] * x;
  return fmaf(s->ebx[u], y, -t);
}

/* Column of a point: the unique u with side(u) <= 0 < side(u+1) (a point on
 * an edge belongs to the column that edge starts).  The search starts from
 * an atan2 estimate and walks; the answer does not depend on the estimate. */
static int column_of(const orc_sensor *s, float x, float y) {
  int W = s->W;
  double dth = TWO_PI / (double)W;
  double beta0 = atan2((double)s->eby[0], (double)s->ebx[0]);
  double rel = beta0 - atan2((double)y, (double)x);
  long u = (long)floor(rel / dth);
  u %= W;
  if (u < 0) u += W;
  for (int step = 0; step <= W + 2; step++) {
    if (edge_side(s, (int)u, x, y) > 0.0f) { u = (u + W - 1) % W; continue; }
    if (edge_side(s, (int)((u + 1) % W), x, y) <= 0.0f) { u = (u + 1) % W; continue; }
    return (int)u;
  }
  return -1;
}

/* Range-image conversion with optional rigid transform (Eq. (1), (2), (6)).
 * All arithmetic FP32 with the operation order written out. */
void orc_project(const float *xyz, int64_t n, const float *M, const orc_sensor *s,
                 float *range, int32_t *src_idx, int64_t *stats) {
  int H = s->H, W = s->W;
  int64_t npx = (int64_t)H * W;
  int64_t *best = (int64_t *)malloc(sizeof(int64_t) * npx);
  for (int64_t i = 0; i < npx; i++) { range[i] = 0.0f; best[i] = -1; }
  int64_t nonfinite = 0, fov = 0, inserted = 0, kept = 0;
  for (int64_t i = 0; i < n; i++) {
    float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    if (M) { /* p' = R p + T, Eq. (6) */
      float xx = fmaf(M[0], x, fmaf(M[1], y, fmaf(M[2], z, M[3])));
      float yy = fmaf(M[4], x, fmaf(M[5], y, fmaf(M[6], z, M[7])));
      float zz = fmaf(M[8], x, fmaf(M[9], y, fmaf(M[10], z, M[11])));
      x = xx; y = yy; z = zz;
    }
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) { nonfinite++; continue; }
    float rho2 = fmaf(x, x, y * y);
    float r = sqrtf(fmaf(x, x, fmaf(y, y, z * z)));   /* Eq. (1) */
    if (!isfinite(r) || r == 0.0f) { nonfinite++; continue; }
    if (rho2 < 1e-12f) { fov++; continue; }            /* on the sensor axis */
    float q = z / sqrtf(rho2);                          /* tan(elevation) */
    if (!(q < s->cut[0]) || q < s->cut[H]) { fov++; continue; }
    int v = 0;                                          /* Eq. (2), phi */
    for (int k = 1; k < H; k++)
      if (s->cut[k] > q) v++;
    int u = column_of(s, x, y);                         /* Eq. (2), theta */
    if (u < 0) { fov++; continue; }
    int64_t px = (int64_t)v * W + u;
    inserted++;
    /* keep the nearest point; equal ranges keep the lower index */
    if (best[px] < 0 || r < range[px]) { range[px] = r; best[px] = i; }
  }
  for (int64_t i = 0; i < npx; i++) {
    if (best[i] >= 0) kept++;
    if (src_idx) src_idx[i] = (int32_t)best[i];
  }
  if (stats) {
    stats[0] = n; stats[1] = nonfinite; stats[2] = fov; stats[3] = inserted - kept; stats[4] = kept;
  }
  free(best);
}

/* ------------------------------------------------------------------------ */
/* Total least squares (Sec. III-C; the smallest eigenvector of the centred  */
/* scatter matrix).  FP64, two-pass centring, cyclic Jacobi.                 */
/* ------------------------------------------------------------------------ */
static void jacobi3(double A[3][3], double V[3][3], double lam[3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) V[i][j] = (i == j);
  for (int sweep = 0; sweep < 64; sweep++) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int p = 0; p < 2; p++)
      for (int q = p + 1; q < 3; q++) {
        if (A[p][q] == 0.0) continue;
        /* rotation that zeroes A[p][q] */
        double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; k++) { /* A <- A J */
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; k++) { /* A <- J^T A */
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; k++) {
          double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 3; i++) lam[i] = A[i][i];
}

int orc_tls(int n, const double *p, double *normal, double *c, double *evals) {
  double mu[3] = {0, 0, 0};
  for (int j = 0; j < n; j++)
    for (int a = 0; a < 3; a++) mu[a] += p[3 * j + a];
  for (int a = 0; a < 3; a++) mu[a] /= (double)n;
  double C[3][3] = {{0}};
  for (int j = 0; j < n; j++) {
    double e[3] = {p[3 * j] - mu[0], p[3 * j + 1] - mu[1], p[3 * j + 2] - mu[2]};
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) C[a][b] += e[a] * e[b];
  }
  double V[3][3], lam[3];
  jacobi3(C, V, lam);
  int o[3] = {0, 1, 2};                 /* sort eigenvalues ascending */
  for (int i = 0; i < 3; i++)
    for (int j = i + 1; j < 3; j++)
      if (lam[o[j]] < lam[o[i]]) { int t = o[i]; o[i] = o[j]; o[j] = t; }
  for (int i = 0; i < 3; i++) evals[i] = lam[o[i]];
  for (int a = 0; a < 3; a++) normal[a] = V[a][o[0]];
  double nn = sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
  for (int a = 0; a < 3; a++) normal[a] /= nn;
  *c = normal[0] * mu[0] + normal[1] * mu[1] + normal[2] * mu[2];
  /* collinear or coincident points do not define a plane */
  if (!(evals[2] > 0.0) || evals[1] <= 1e-6 * evals[2]) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Plane storage and the ray-cast test (Eq. (3) and the decoder of Sec.      */
/* III-C).  Dominant-axis form: axis k with |n_k| maximal (ties: lower axis),*/
/* p_k + a p_k1 + b p_k2 = c with k1 < k2 the other axes; Eq. (3) is k = x.  */
/* ------------------------------------------------------------------------ */
typedef struct { int k; float a, b, c; } plane_t;

static plane_t stored_form(const double n[3], double c) {
  plane_t P;
  int k = 0;
  if (fabs(n[1]) > fabs(n[k])) k = 1;
  if (fabs(n[2]) > fabs(n[k])) k = 2;
  int k1 = (k == 0) ? 1 : 0, k2 = (k == 2) ? 1 : 2;
  P.k = k;
  P.a = (float)(n[k1] / n[k]);
  P.b = (float)(n[k2] / n[k]);
  P.c = (float)(c / n[k]);
  return P;
}

/* Range at which the ray d meets the stored plane, FP32, fixed order. */
static float ray_cast(plane_t P, const float d[3]) {
  int k1 = (P.k == 0) ? 1 : 0, k2 = (P.k == 2) ? 1 : 2;
  float den = fmaf(P.b, d[k2], fmaf(P.a, d[k1], d[P.k]));
  return P.c / den;
}

/* A pixel is reproduced by the plane when the decoded range is within eps. */
static int reproduces(plane_t P, const float d[3], float r, float eps) {
  float t = ray_cast(P, d);
  if (!isfinite(t) || !(t > 0.0f)) return 0;
  return fabsf(t - r) <= eps;
}

/* ------------------------------------------------------------------------ */
/* Tiles                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n;                 /* valid pixels */
  int slot[64];          /* slot j = i*tw + k of the pixel (row i, column k in the tile) */
  float r[64];
  float d[64][3];
  double p[64][3];       /* r*d in FP64 (exact product of two FP32 values) */
  /* diagnostics only (no result depends on them): over every pixel test
   * made on the tile, the smallest distance of | t - r | from eps, in metres
   * and relative to max(r, 1 m); and that distance times the cosine of the
   * angle between the ray and the plane normal, relative to max(r, 1 m): the
   * relative change of the plane that moves the ray-cast range t = c / (n.d)
   * by that distance (a plane seen nearly edge-on amplifies any change of
   * its coefficients by 1 / cos); a test whose t is not finite or not
   * positive contributes the cosine itself */
  double margin_abs, margin_rel, margin_cond;
} tile_t;

static void load_tile(const float *range, const orc_sensor *s, const orc_params *prm, int tr,
                      int tc, tile_t *T) {
  T->n = 0;
  T->margin_abs = T->margin_rel = T->margin_cond = INFINITY;
  for (int i = 0; i < prm->th; i++) {
    int v = tr * prm->th + i;
    if (v >= s->H) break;
    for (int k = 0; k < prm->tw; k++) {
      int u = tc * prm->tw + k;
      if (u >= s->W) break;
      float r = range[(int64_t)v * s->W + u];
      if (!(r > 0.0f)) continue;
      int m = T->n++;
      T->slot[m] = i * prm->tw + k;
      T->r[m] = r;
      direction(s, v, u, T->d[m]);
      for (int a = 0; a < 3; a++) T->p[m][a] = (double)r * (double)T->d[m][a];
    }
  }
}

static int popcount64(uint64_t x) { return __builtin_popcountll(x); }

/* Points a tile must keep on its plane: at least min(min_pts, n), and at
 * least the fraction rho of its valid points. */
static int need(const orc_params *prm, int n) {
  int a = n < prm->min_pts ? n : prm->min_pts;
  int b = (int)ceil((double)prm->rho * (double)n);
  return a > b ? a : b;
}

static uint64_t inliers_of(plane_t P, tile_t *T, float eps) {
  uint64_t m = 0;
  for (int j = 0; j < T->n; j++) {
    if (reproduces(P, T->d[j], T->r[j], eps)) m |= 1ull << T->slot[j];
    float t = ray_cast(P, T->d[j]);
    /* how close this decision was to flipping */
    int k1 = (P.k == 0) ? 1 : 0, k2 = (P.k == 2) ? 1 : 2;
    double den = (double)T->d[j][P.k] + (double)P.a * T->d[j][k1] + (double)P.b * T->d[j][k2];
    double cosang = fabs(den) / sqrt(1.0 + (double)P.a * P.a + (double)P.b * P.b);
    double cond = cosang;
    if (isfinite(t) && t > 0.0f) {
      double dev = fabs(fabs((double)t - (double)T->r[j]) - (double)eps);
      double rel = dev / fmax((double)T->r[j], 1.0);
      if (dev < T->margin_abs) T->margin_abs = dev;
      if (rel < T->margin_rel) T->margin_rel = rel;
      cond = rel * cosang;
    }
    if (cond < T->margin_cond) T->margin_cond = cond;
  }
  return m;
}

/* Own fit of a tile: least-squares plane, then refit on the points it
 * reproduces, at most max_iter fits (iterative plane fitting). */
static void own_fit(tile_t *T, const orc_params *prm, int8_t *status, int8_t *iters,
                    plane_t *P, uint64_t *mask) {
  *iters = 0;
  *mask = 0;
  memset(P, 0, sizeof *P);
  if (T->n == 0) { *status = ORC_EMPTY; return; }
  if (T->n < prm->min_pts) { *status = ORC_FEW; return; }
  uint64_t S = 0;
  for (int j = 0; j < T->n; j++) S |= 1ull << T->slot[j];
  for (int it = 1; it <= prm->max_iter; it++) {
    double pts[64 * 3];
    int m = 0;
    for (int j = 0; j < T->n; j++)
      if (S >> T->slot[j] & 1) {
        for (int a = 0; a < 3; a++) pts[3 * m + a] = T->p[j][a];
        m++;
      }
    double nrm[3], c, ev[3];
    *iters = (int8_t)it;
    if (orc_tls(m, pts, nrm, &c, ev)) { *status = ORC_DEGENERATE; *mask = 0; return; }
    *P = stored_form(nrm, c);
    uint64_t S2 = inliers_of(*P, T, prm->eps);
    *mask = S2;
    if (S2 == S) break;
    if (popcount64(S2) < prm->min_pts) { *status = ORC_FAILED; *mask = 0; return; }
    S = S2;
  }
  *status = popcount64(*mask) >= need(prm, T->n) ? ORC_ACCEPTED : ORC_REJECTED;
}

/* Seeded fit (learned plane seeding): the seed normal's stored form
 * (FP32 coefficients), its offset as the mean of p_k + a p_k1 + b p_k2 over
 * the tile's points, the points that plane reproduces, one least-squares
 * refit on them, and the same acceptance test as the own fit.  Returns 1 when
 * the seed is accepted (status, plane, mask set), 0 when the tile must fall
 * back to the plain fit, -1 when the tile has no usable seed. */
static int seeded_fit(tile_t *T, const float seed[4], const orc_params *prm, int8_t *status,
                      int8_t *iters, plane_t *P, uint64_t *mask) {
  if (!(seed[3] > 0.0f) || T->n < prm->min_pts) return -1;
  float n[3] = {seed[0], seed[1], seed[2]};
  if (!isfinite(n[0]) || !isfinite(n[1]) || !isfinite(n[2])) return -1;
  int k = 0;
  float m = fabsf(n[0]);
  if (fabsf(n[1]) > m) { k = 1; m = fabsf(n[1]); }
  if (fabsf(n[2]) > m) { k = 2; m = fabsf(n[2]); }
  if (!(m > 0.0f)) return -1;
  int k1 = (k == 0) ? 1 : 0, k2 = (k == 2) ? 1 : 2;
  plane_t Q = {k, n[k1] / n[k], n[k2] / n[k], 0.0f};
  double sum = 0.0;
  for (int j = 0; j < T->n; j++) sum += T->p[j][k] + (double)Q.a * T->p[j][k1] + (double)Q.b * T->p[j][k2];
  Q.c = (float)(sum / (double)T->n);
  uint64_t S1 = inliers_of(Q, T, prm->eps);
  if (popcount64(S1) < prm->min_pts) return 0;
  double pts[64 * 3], nrm[3], c, ev[3];
  int cnt = 0;
  for (int j = 0; j < T->n; j++)
    if (S1 >> T->slot[j] & 1) {
      for (int a = 0; a < 3; a++) pts[3 * cnt + a] = T->p[j][a];
      cnt++;
    }
  if (orc_tls(cnt, pts, nrm, &c, ev)) return 0;
  plane_t P1 = stored_form(nrm, c);
  uint64_t S2 = inliers_of(P1, T, prm->eps);
  if (popcount64(S2) < need(prm, T->n)) return 0;
  *P = P1;
  *mask = S2;
  *iters = 1;
  *status = ORC_ACCEPTED;
  return 1;
}

/* Temporal fit: the key-frame plane's normal is held and only the offset
 * varies (Sec. III-D).  In the stored form the offset is the mean of
 * p_k + a p_k1 + b p_k2 over the points kept. */
static void temporal_fit(tile_t *T, plane_t Q, const orc_params *prm, int8_t *status,
                         int8_t *iters, float *cprime, uint64_t *mask) {
  *iters = 0; *mask = 0; *cprime = 0.0f;
  if (T->n < prm->min_pts) { *status = 1; return; }
  int k1 = (Q.k == 0) ? 1 : 0, k2 = (Q.k == 2) ? 1 : 2;
  uint64_t S = 0;
  for (int j = 0; j < T->n; j++) S |= 1ull << T->slot[j];
  for (int it = 1; it <= prm->max_iter; it++) {
    double sum = 0.0;
    int m = 0;
    for (int j = 0; j < T->n; j++)
      if (S >> T->slot[j] & 1) {
        sum += T->p[j][Q.k] + (double)Q.a * T->p[j][k1] + (double)Q.b * T->p[j][k2];
        m++;
      }
    plane_t P = Q;
    P.c = (float)(sum / (double)m);
    *iters = (int8_t)it;
    *cprime = P.c;
    uint64_t S2 = inliers_of(P, T, prm->eps);
    *mask = S2;
    if (S2 == S) break;
    if (popcount64(S2) < prm->min_pts) { *status = 1; *mask = 0; return; }
    S = S2;
  }
  *status = popcount64(*mask) >= need(prm, T->n) ? 2 : 1;
}

/* ------------------------------------------------------------------------ */
/* Streams: byte histograms of the serialized OCC, RUN, MASK, RES streams.   */
/* ------------------------------------------------------------------------ */
enum { S_OCC = 0, S_RUN = 1, S_MASK = 2, S_RES = 3 };

static void put_byte(orc_frame *f, int stream, unsigned v) {
  f->hist[stream * 256 + (v & 255u)]++;
  if (f->sbuf[stream] && f->stream_bytes[stream] < f->scap[stream]) f->sbuf[stream][f->stream_bytes[stream]] = (uint8_t)v;
  f->stream_bytes[stream]++;
}
static void put_varint(orc_frame *f, uint32_t v) {   /* LEB128 */
  while (v >= 128u) { put_byte(f, S_RUN, (v & 127u) | 128u); v >>= 7; }
  put_byte(f, S_RUN, v);
}
static void put_f32(orc_frame *f, float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  for (int i = 0; i < 4; i++) put_byte(f, S_RUN, (u >> (8 * i)) & 255u);
}

/* Optimal (Huffman) code length sum over a byte histogram: repeatedly merge
 * the two lightest nodes; the cost is the sum of merged weights. */
uint64_t orc_huffman_bits(const uint32_t *hist) {
  uint64_t heap[257];
  int n = 0;
  uint64_t total = 0;
  for (int i = 0; i < 256; i++)
    if (hist[i]) {
      uint64_t w = hist[i];
      total += w;
      int j = n++;            /* sift up */
      while (j > 0 && heap[(j - 1) / 2] > w) { heap[j] = heap[(j - 1) / 2]; j = (j - 1) / 2; }
      heap[j] = w;
    }
  if (n == 0) return 0;
  if (n == 1) return total;   /* one symbol still costs one bit per occurrence */
  uint64_t cost = 0;
  while (n > 1) {
    uint64_t ab[2];
    for (int t = 0; t < 2; t++) {   /* pop min */
      ab[t] = heap[0];
      uint64_t last = heap[--n];
      int j = 0;
      for (;;) {
        int l = 2 * j + 1, r = l + 1, m = j;
        uint64_t vm = last;
        if (l < n && heap[l] < vm) { m = l; vm = heap[l]; }
        if (r < n && heap[r] < vm) { m = r; vm = heap[r]; }
        if (m == j) break;
        heap[j] = heap[m];
        j = m;
      }
      if (n > 0) heap[j] = last;
    }
    uint64_t w = ab[0] + ab[1];
    cost += w;
    int j = n++;
    while (j > 0 && heap[(j - 1) / 2] > w) { heap[j] = heap[(j - 1) / 2]; j = (j - 1) / 2; }
    heap[j] = w;
  }
  return cost;
}

#define HEADER_BYTES 112u   /* fixed fields (64 bytes) and the transform M_i (12 FP32) */
#define TABLE_BYTES 128u

static void finish_size(orc_frame *f) {
  f->size_bytes = HEADER_BYTES;
  for (int s = 0; s < 4; s++) {
    f->coded_bits[s] = orc_huffman_bits(f->hist + 256 * s);
    if (f->stream_bytes[s]) f->size_bytes += (f->coded_bits[s] + 7) / 8 + TABLE_BYTES;
  }
}

/* Residual quantiser: step 2*eps*(1 - 2^-8), round to nearest even in FP32.
 * The decoder's q*step is then within eps of the range (a reading: the paper
 * keeps raw ranges in the residual map). */
static void quant_constants(float eps, float *step, float *inv) {
  double st = 2.0 * (double)eps * (1.0 - 1.0 / 256.0);
  *step = (float)st;
  *inv = (float)(1.0 / (double)(*step));
}

/* OCC, MASK and RES streams and the residual codes, shared by key and
 * predicted frames (the RUN stream is written by the caller). */
static void emit_pixels(const float *range, const orc_sensor *s, const orc_params *prm,
                        orc_frame *f) {
  int H = s->H, W = s->W;
  int64_t npx = (int64_t)H * W;
  /* OCC */
  for (int64_t b = 0; b < (npx + 7) / 8; b++) {
    unsigned v = 0;
    for (int i = 0; i < 8; i++) {
      int64_t px = 8 * b + i;
      if (px < npx && range[px] > 0.0f) v |= 1u << i;
    }
    f->occ[b] = (uint8_t)v;
    put_byte(f, S_OCC, v);
  }
  /* MASK: per plane-coded tile in tile raster order, its valid pixels'
   * bits in tile raster order, packed LSB first, byte aligned per tile */
  for (int t = 0; t < f->TR * f->TC; t++) {
    if (f->cls[t] != ORC_CLS_SPATIAL && f->cls[t] != ORC_CLS_TEMPORAL) continue;
    int tr = t / f->TC, tc = t % f->TC, nb = 0;
    unsigned cur = 0;
    for (int i = 0; i < prm->th; i++) {
      int v = tr * prm->th + i;
      if (v >= H) break;
      for (int k = 0; k < prm->tw; k++) {
        int u = tc * prm->tw + k;
        if (u >= W) break;
        if (!(range[(int64_t)v * W + u] > 0.0f)) continue;
        if (f->mask[t] >> (i * prm->tw + k) & 1) cur |= 1u << (nb & 7);
        nb++;
        if ((nb & 7) == 0) { put_byte(f, S_MASK, cur); cur = 0; }
      }
    }
    if (nb & 7) put_byte(f, S_MASK, cur);
  }
  /* RES: valid pixels no plane reproduces, frame raster order; each code
   * is sent as the zigzag-mapped difference (mod 2^16) from the previous
   * residual code of its image row (0 before a row's first), u16 LE */
  float step, inv;
  quant_constants(prm->eps, &step, &inv);
  f->n_res = 0;
  f->range_error = 0;
  for (int v = 0; v < H; v++) {
    uint16_t prev = 0;
    for (int u = 0; u < W; u++) {
      float r = range[(int64_t)v * W + u];
      if (!(r > 0.0f)) continue;
      int t = (v / prm->th) * f->TC + u / prm->tw;
      int covered = (f->cls[t] == ORC_CLS_SPATIAL || f->cls[t] == ORC_CLS_TEMPORAL) &&
                    (f->mask[t] >> ((v % prm->th) * prm->tw + u % prm->tw) & 1);
      if (covered) continue;
      float q = rintf(r * inv);
      double back = (double)(q * step);
      if (q > 65535.0f || fabs(back - (double)r) > (double)prm->eps) {
        f->range_error = 1;
        q = q > 65535.0f ? 65535.0f : q;
      }
      uint16_t code = (uint16_t)q;
      f->codes[f->n_res++] = code;
      const int16_t d = (int16_t)(uint16_t)(code - prev);
      const uint16_t z = (uint16_t)(((uint16_t)d << 1) ^ (uint16_t)(d < 0 ? 0xFFFFu : 0u));
      prev = code;
      put_byte(f, S_RES, z & 255u);
      put_byte(f, S_RES, (unsigned)z >> 8);
    }
  }
}

static void alloc_free_tiles(int T, tile_t **tiles) { *tiles = (tile_t *)malloc(sizeof(tile_t) * (size_t)T); }

static void copy_margins(orc_frame *f, const tile_t *tiles, int T) {
  for (int t = 0; t < T; t++) {
    if (f->margin_abs) f->margin_abs[t] = (float)tiles[t].margin_abs;
    if (f->margin_rel) f->margin_rel[t] = (float)tiles[t].margin_rel;
    if (f->margin_cond) f->margin_cond[t] = (float)tiles[t].margin_cond;
  }
}

/* Horizontal growth of runs within one tile row (Sec. III-C): a run grows
 * into the next tile while its plane reproduces at least the tile's need of
 * its points (the run plane is not refit); otherwise a new run starts at the
 * tile if the tile's own fit is accepted.
 * `eligible` (NULL = all) excludes tiles taken by temporal runs; such tiles
 * end any open run. */
static void grow_spatial_row(int tr, tile_t *tiles, const plane_t *own, const uint8_t *eligible,
                             const orc_params *prm, orc_frame *f) {
  int open = 0, cur = -1;
  plane_t P = {0, 0, 0, 0};
  for (int tc = 0; tc < f->TC; tc++) {
    int t = tr * f->TC + tc;
    if (eligible && !eligible[t]) { open = 0; continue; }
    tile_t *T = &tiles[t];
    if (open) {
      uint64_t m = inliers_of(P, T, prm->eps);
      if (popcount64(m) >= need(prm, T->n)) {
        f->srun_len[cur]++;
        f->cls[t] = ORC_CLS_SPATIAL; f->mask[t] = m; f->run_of[t] = cur;
        continue;
      }
      open = 0;
    }
    if (f->own_status[t] == ORC_ACCEPTED) {
      cur = f->n_sruns++;
      P = own[t];
      f->srun_row[cur] = tr; f->srun_s[cur] = tc; f->srun_len[cur] = 1;
      f->srun_axis[cur] = (int8_t)P.k;
      f->srun_abc[3 * cur] = P.a; f->srun_abc[3 * cur + 1] = P.b; f->srun_abc[3 * cur + 2] = P.c;
      f->cls[t] = ORC_CLS_SPATIAL; f->mask[t] = f->own_mask[t]; f->run_of[t] = cur;
      open = 1;
    } else {
      f->cls[t] = T->n == 0 ? ORC_CLS_EMPTY : ORC_CLS_UNFIT;
      f->mask[t] = 0; f->run_of[t] = -1;
    }
  }
}

static void put_spatial_runs_of_row(orc_frame *f, int tr, int first, int count) {
  put_varint(f, (uint32_t)count);
  int prev_end = 0;
  for (int r = first; r < first + count; r++) {
    put_varint(f, (uint32_t)(f->srun_s[r] - prev_end));
    put_varint(f, (uint32_t)f->srun_len[r]);
    put_byte(f, S_RUN, (unsigned)f->srun_axis[r]);
    put_f32(f, f->srun_abc[3 * r]);
    put_f32(f, f->srun_abc[3 * r + 1]);
    put_f32(f, f->srun_abc[3 * r + 2]);
    prev_end = f->srun_s[r] + f->srun_len[r];
  }
  (void)tr;
}

static void reset_frame(orc_frame *f, const orc_sensor *s, const orc_params *prm) {
  f->TR = (s->H + prm->th - 1) / prm->th;
  f->TC = (s->W + prm->tw - 1) / prm->tw;
  f->n_sruns = f->n_pruns = 0;
  f->n_res = 0;
  memset(f->hist, 0, sizeof(uint32_t) * 4 * 256);
  for (int i = 0; i < 4; i++) f->stream_bytes[i] = f->coded_bits[i] = 0;
  f->size_bytes = 0;
  f->range_error = 0;
}

/* Spatial-only encoding of a key frame (Sec. III-C). */
void orc_encode_key(const float *range, const orc_sensor *s, const orc_params *prm, const float *seed,
                    orc_frame *f) {
  reset_frame(f, s, prm);
  int T = f->TR * f->TC;
  tile_t *tiles;
  alloc_free_tiles(T, &tiles);
  plane_t *own = (plane_t *)calloc((size_t)T, sizeof(plane_t));
  for (int t = 0; t < T; t++) {
    load_tile(range, s, prm, t / f->TC, t % f->TC, &tiles[t]);
    int sd = -1;
    if (seed) sd = seeded_fit(&tiles[t], seed + 4 * (size_t)t, prm, &f->own_status[t], &f->own_iters[t], &own[t],
                              &f->own_mask[t]);
    if (f->seeded) f->seeded[t] = (int8_t)(sd == 1 ? 1 : (sd == 0 ? 2 : 0));
    if (sd != 1) own_fit(&tiles[t], prm, &f->own_status[t], &f->own_iters[t], &own[t], &f->own_mask[t]);
    f->own_axis[t] = (int8_t)own[t].k;
    f->own_abc[3 * t] = own[t].a; f->own_abc[3 * t + 1] = own[t].b; f->own_abc[3 * t + 2] = own[t].c;
    if (f->t_status) { f->t_status[t] = 0; f->t_iters[t] = 0; f->t_c[t] = 0; f->t_mask[t] = 0; }
  }
  for (int tr = 0; tr < f->TR; tr++) {
    int first = f->n_sruns;
    grow_spatial_row(tr, tiles, own, NULL, prm, f);
    put_spatial_runs_of_row(f, tr, first, f->n_sruns - first);
  }
  emit_pixels(range, s, prm, f);
  finish_size(f);
  copy_margins(f, tiles, T);
  free(own);
  free(tiles);
}

/* Predicted frame (Sec. III-D): reuse the key frame's run planes with the
 * offset free, grow temporal runs within one key-frame run, then encode the
 * remaining tiles spatially, channel by channel. */
void orc_encode_pred(const orc_frame *key, const float *range, const orc_sensor *s,
                     const orc_params *prm, orc_frame *f) {
  reset_frame(f, s, prm);
  int T = f->TR * f->TC;
  tile_t *tiles;
  alloc_free_tiles(T, &tiles);
  plane_t *own = (plane_t *)calloc((size_t)T, sizeof(plane_t));
  uint8_t *eligible = (uint8_t *)malloc((size_t)T);
  for (int t = 0; t < T; t++) load_tile(range, s, prm, t / f->TC, t % f->TC, &tiles[t]);
  /* key-frame plane of each tile: the plane of the key run covering it */
  for (int t = 0; t < T; t++) {
    f->t_status[t] = 0; f->t_iters[t] = 0; f->t_c[t] = 0.0f; f->t_mask[t] = 0;
    if (key->cls[t] != ORC_CLS_SPATIAL) continue;
    int kr = key->run_of[t];
    plane_t Q = {key->srun_axis[kr], key->srun_abc[3 * kr], key->srun_abc[3 * kr + 1], key->srun_abc[3 * kr + 2]};
    temporal_fit(&tiles[t], Q, prm, &f->t_status[t], &f->t_iters[t], &f->t_c[t], &f->t_mask[t]);
  }
  /* temporal runs: grow while the key run stays the same and (normal, c')
   * of the run start reproduces the tile */
  for (int tr = 0; tr < f->TR; tr++) {
    int open = 0, cur = -1, krun = -1;
    plane_t P = {0, 0, 0, 0};
    for (int tc = 0; tc < f->TC; tc++) {
      int t = tr * f->TC + tc;
      tile_t *Tt = &tiles[t];
      if (open) {
        if (key->cls[t] == ORC_CLS_SPATIAL && key->run_of[t] == krun) {
          uint64_t m = inliers_of(P, Tt, prm->eps);
          if (popcount64(m) >= need(prm, Tt->n)) {
            f->prun_len[cur]++;
            f->cls[t] = ORC_CLS_TEMPORAL; f->mask[t] = m; f->run_of[t] = T + cur; eligible[t] = 0;
            continue;
          }
        }
        open = 0;
      }
      if (f->t_status[t] == 2) {
        krun = key->run_of[t];
        cur = f->n_pruns++;
        P.k = key->srun_axis[krun]; P.a = key->srun_abc[3 * krun]; P.b = key->srun_abc[3 * krun + 1];
        P.c = f->t_c[t];
        f->prun_row[cur] = tr; f->prun_s[cur] = tc; f->prun_len[cur] = 1; f->prun_krun[cur] = krun;
        f->prun_c[cur] = P.c;
        f->cls[t] = ORC_CLS_TEMPORAL; f->mask[t] = f->t_mask[t]; f->run_of[t] = T + cur; eligible[t] = 0;
        open = 1;
      } else {
        eligible[t] = 1;
      }
    }
  }
  /* spatial encoding of what is left (channel-wise, Sec. III-D) */
  for (int t = 0; t < T; t++) {
    if (eligible[t]) {
      own_fit(&tiles[t], prm, &f->own_status[t], &f->own_iters[t], &own[t], &f->own_mask[t]);
    } else {
      f->own_status[t] = ORC_EMPTY; f->own_iters[t] = 0; f->own_mask[t] = 0;
      memset(&own[t], 0, sizeof(plane_t));
    }
    f->own_axis[t] = (int8_t)own[t].k;
    f->own_abc[3 * t] = own[t].a; f->own_abc[3 * t + 1] = own[t].b; f->own_abc[3 * t + 2] = own[t].c;
  }
  int pfirst = 0;
  for (int tr = 0; tr < f->TR; tr++) {
    int first = f->n_sruns;
    grow_spatial_row(tr, tiles, own, eligible, prm, f);
    /* RUN stream of the row: temporal runs, then spatial runs */
    int pcount = 0;
    while (pfirst + pcount < f->n_pruns && f->prun_row[pfirst + pcount] == tr) pcount++;
    put_varint(f, (uint32_t)pcount);
    int prev_end = 0;
    for (int r = pfirst; r < pfirst + pcount; r++) {
      put_varint(f, (uint32_t)(f->prun_s[r] - prev_end));
      put_varint(f, (uint32_t)f->prun_len[r]);
      put_f32(f, f->prun_c[r]);
      prev_end = f->prun_s[r] + f->prun_len[r];
    }
    pfirst += pcount;
    put_spatial_runs_of_row(f, tr, first, f->n_sruns - first);
  }
  emit_pixels(range, s, prm, f);
  finish_size(f);
  copy_margins(f, tiles, T);
  free(eligible);
  free(own);
  free(tiles);
}

/* ------------------------------------------------------------------------ */
/* Decoder: ray-cast plane-coded pixels, dequantise the rest (Sec. III-C).   */
/* Uses only the encoded data: OCC, runs, masks, codes (and the key frame's  */
/* runs for the normals of temporal runs).                                   */
/* ------------------------------------------------------------------------ */
void orc_decode(const orc_frame *key, const orc_frame *f, const orc_sensor *s,
                const orc_params *prm, float *out) {
  int H = s->H, W = s->W, T = f->TR * f->TC;
  plane_t *pl = (plane_t *)calloc((size_t)T, sizeof(plane_t));
  uint8_t *has = (uint8_t *)calloc((size_t)T, 1);
  for (int r = 0; r < f->n_sruns; r++)
    for (int i = 0; i < f->srun_len[r]; i++) {
      int t = f->srun_row[r] * f->TC + f->srun_s[r] + i;
      pl[t].k = f->srun_axis[r]; pl[t].a = f->srun_abc[3 * r]; pl[t].b = f->srun_abc[3 * r + 1];
      pl[t].c = f->srun_abc[3 * r + 2];
      has[t] = 1;
    }
  for (int r = 0; r < f->n_pruns; r++) {
    int kr = f->prun_krun[r];
    for (int i = 0; i < f->prun_len[r]; i++) {
      int t = f->prun_row[r] * f->TC + f->prun_s[r] + i;
      pl[t].k = key->srun_axis[kr]; pl[t].a = key->srun_abc[3 * kr]; pl[t].b = key->srun_abc[3 * kr + 1];
      pl[t].c = f->prun_c[r];
      has[t] = 1;
    }
  }
  float step, inv;
  quant_constants(prm->eps, &step, &inv);
  int64_t ci = 0;
  for (int v = 0; v < H; v++)
    for (int u = 0; u < W; u++) {
      int64_t px = (int64_t)v * W + u;
      out[px] = 0.0f;
      if (!(f->occ[px >> 3] >> (px & 7) & 1)) continue;
      int t = (v / prm->th) * f->TC + u / prm->tw;
      if (has[t] && (f->mask[t] >> ((v % prm->th) * prm->tw + u % prm->tw) & 1)) {
        float d[3];
        direction(s, v, u, d);
        out[px] = ray_cast(pl[t], d);
      } else {
        out[px] = (float)f->codes[ci++] * step;
      }
    }
  free(has);
  free(pl);
}

/* ------------------------------------------------------------------------ */
/* CPU baseline: whole sequences, per-frame threads (Sec. III-E scheme).     */
/* ------------------------------------------------------------------------ */
typedef struct {
  orc_frame f;
  void *mem;
} frame_buf;

static void frame_alloc(frame_buf *b, const orc_sensor *s, const orc_params *prm) {
  int TR = (s->H + prm->th - 1) / prm->th, TC = (s->W + prm->tw - 1) / prm->tw, T = TR * TC;
  int64_t npx = (int64_t)s->H * s->W;
  memset(&b->f, 0, sizeof b->f);
  b->f.own_status = calloc(T, 1); b->f.own_iters = calloc(T, 1); b->f.own_axis = calloc(T, 1);
  b->f.own_abc = calloc(3 * (size_t)T, 4); b->f.own_mask = calloc(T, 8);
  b->f.t_status = calloc(T, 1); b->f.t_iters = calloc(T, 1); b->f.t_c = calloc(T, 4); b->f.t_mask = calloc(T, 8);
  b->f.cls = calloc(T, 1); b->f.mask = calloc(T, 8); b->f.run_of = calloc(T, 4);
  b->f.srun_row = calloc(T, 4); b->f.srun_s = calloc(T, 4); b->f.srun_len = calloc(T, 4);
  b->f.srun_axis = calloc(T, 1); b->f.srun_abc = calloc(3 * (size_t)T, 4);
  b->f.prun_row = calloc(T, 4); b->f.prun_s = calloc(T, 4); b->f.prun_len = calloc(T, 4);
  b->f.prun_krun = calloc(T, 4); b->f.prun_c = calloc(T, 4);
  b->f.occ = calloc((size_t)(npx + 7) / 8, 1);
  b->f.codes = calloc((size_t)npx, 2);
  b->f.hist = calloc(4 * 256, 4);
}

static void frame_free(frame_buf *b) {
  void *p[] = {b->f.own_status, b->f.own_iters, b->f.own_axis, b->f.own_abc, b->f.own_mask,
               b->f.t_status, b->f.t_iters, b->f.t_c, b->f.t_mask, b->f.cls, b->f.mask, b->f.run_of,
               b->f.srun_row, b->f.srun_s, b->f.srun_len, b->f.srun_axis, b->f.srun_abc,
               b->f.prun_row, b->f.prun_s, b->f.prun_len, b->f.prun_krun, b->f.prun_c,
               b->f.occ, b->f.codes, b->f.hist};
  for (size_t i = 0; i < sizeof p / sizeof p[0]; i++) free(p[i]);
}

uint64_t orc_encode_sequences(int nseq, int nf, int key_index, const float *const *xyz,
                              const int64_t *count, const float *M, const orc_sensor *s,
                              const orc_params *prm, uint64_t *sizes, int64_t *finite_points) {
  int nfr = nseq * nf;
  int64_t npx = (int64_t)s->H * s->W;
  float *ranges = (float *)malloc(sizeof(float) * (size_t)npx * (size_t)nfr);
  int64_t *fin = (int64_t *)calloc((size_t)nfr, sizeof(int64_t));
  frame_buf *fb = (frame_buf *)malloc(sizeof(frame_buf) * (size_t)nfr);
  for (int i = 0; i < nfr; i++) frame_alloc(&fb[i], s, prm);
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < nfr; i++) {
    int64_t st[5];
    const float *Mi = (i % nf == key_index) ? NULL : M + 16 * (size_t)i;
    orc_project(xyz[i], count[i], Mi, s, ranges + (size_t)i * npx, NULL, st);
    fin[i] = st[0] - st[1];
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int q = 0; q < nseq; q++) {
    int i = q * nf + key_index;
    orc_encode_key(ranges + (size_t)i * npx, s, prm, NULL, &fb[i].f);
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < nfr; i++) {
    if (i % nf == key_index) continue;
    int k = (i / nf) * nf + key_index;
    orc_encode_pred(&fb[k].f, ranges + (size_t)i * npx, s, prm, &fb[i].f);
  }
  uint64_t total = 0;
  int64_t ftot = 0;
  for (int i = 0; i < nfr; i++) {
    if (sizes) sizes[i] = fb[i].f.size_bytes;
    total += fb[i].f.size_bytes;
    ftot += fin[i];
    frame_free(&fb[i]);
  }
  if (finite_points) *finite_points = ftot;
  free(fb);
  free(fin);
  free(ranges);
  return total;
}

/* ------------------------------------------------------------------------ */
/* Entropy-coded bitstream: canonical Huffman codes of at most 15 bits.      */
/* ------------------------------------------------------------------------ */
#define PACK_MAXLEN 15
#define PACK_MAGIC 0x31434350u   /* "PCC1" */

static const uint32_t *g_sort_hist;
static int by_count_then_symbol(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  if (g_sort_hist[x] != g_sort_hist[y]) return g_sort_hist[x] < g_sort_hist[y] ? -1 : 1;
  return x - y;
}
static int by_count_desc_then_symbol(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  if (g_sort_hist[x] != g_sort_hist[y]) return g_sort_hist[x] > g_sort_hist[y] ? -1 : 1;
  return x - y;
}

void orc_code_lengths(const uint32_t *hist, uint8_t *len) {
  memset(len, 0, 256);
  int sym[256], m = 0;
  for (int i = 0; i < 256; i++)
    if (hist[i]) sym[m++] = i;
  if (m == 0) return;
  if (m == 1) { len[sym[0]] = 1; return; }
  g_sort_hist = hist;
  qsort(sym, (size_t)m, sizeof(int), by_count_then_symbol);
  /* two queues: leaves 0..m-1 in sorted order, internal nodes from m on */
  uint64_t w[512];
  int parent[512];
  for (int i = 0; i < m; i++) w[i] = hist[sym[i]];
  int li = 0, qh = m, qt = m;
  for (int step = 0; step < m - 1; step++) {
    int pick[2];
    for (int z = 0; z < 2; z++) pick[z] = (li < m && (qh == qt || w[li] <= w[qh])) ? li++ : qh++;
    w[qt] = w[pick[0]] + w[pick[1]];
    parent[pick[0]] = parent[pick[1]] = qt;
    qt++;
  }
  int depth[512], bl[512];
  memset(bl, 0, sizeof(bl));
  depth[qt - 1] = 0;
  for (int n = qt - 2; n >= 0; n--) depth[n] = depth[parent[n]] + 1;
  int maxl = 0;
  for (int i = 0; i < m; i++) {
    bl[depth[i]]++;
    if (depth[i] > maxl) maxl = depth[i];
  }
  /* at most PACK_MAXLEN bits: move pairs of the deepest codes up, keeping
   * the Kraft sum (the adjustment of JPEG, ITU T.81 Annex K.3) */
  for (int i = maxl; i > PACK_MAXLEN; i--)
    while (bl[i] > 0) {
      int j = i - 2;
      while (bl[j] == 0) j--;
      bl[i] -= 2;
      bl[i - 1] += 1;
      bl[j + 1] += 2;
      bl[j] -= 1;
    }
  qsort(sym, (size_t)m, sizeof(int), by_count_desc_then_symbol);
  int L = 1;
  for (int i = 0; i < m; i++) {
    while (bl[L] == 0) L++;
    len[sym[i]] = (uint8_t)L;
    bl[L]--;
  }
}

void orc_canonical_codes(const uint8_t *len, uint32_t *code) {
  uint32_t next = 0;
  memset(code, 0, 256 * sizeof(uint32_t));
  for (int L = 1; L <= PACK_MAXLEN; L++) {
    for (int s = 0; s < 256; s++)
      if (len[s] == L) code[s] = next++;
    next <<= 1;
  }
}

static void put_u16(uint8_t *p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put_u32(uint8_t *p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void put_u64(uint8_t *p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint32_t get_u16(const uint8_t *p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8); }
static uint32_t get_u32(const uint8_t *p) { uint32_t v = 0; for (int i = 0; i < 4; i++) v |= (uint32_t)p[i] << (8 * i); return v; }
static uint64_t get_u64(const uint8_t *p) { uint64_t v = 0; for (int i = 0; i < 8; i++) v |= (uint64_t)p[i] << (8 * i); return v; }

/* header: magic u32, kind u8, th u8, tw u8, 0 u8, H u16, W u16,
 * stream bytes u64[4], payload bytes u32[4], 4 zero bytes, then the
 * transform into the key frame as 12 FP32 (rows of [R | T]; identity when
 * M is NULL): a predicted frame's points go back to its own coordinates
 * through it when decompression reverses the compression (Sec. III-D). */
uint64_t orc_pack(const orc_frame *f, int kind, int H, int W, int th, int tw, const float *M, uint8_t *out,
                  uint64_t cap) {
  if (cap < HEADER_BYTES) return 0;
  memset(out, 0, HEADER_BYTES);
  put_u32(out, PACK_MAGIC);
  out[4] = (uint8_t)kind; out[5] = (uint8_t)th; out[6] = (uint8_t)tw;
  put_u16(out + 8, (uint32_t)H); put_u16(out + 10, (uint32_t)W);
  for (int e = 0; e < 12; e++) {
    float m = M ? M[e] : (e % 5 == 0 ? 1.0f : 0.0f);
    uint32_t bits;
    memcpy(&bits, &m, 4);
    put_u32(out + 64 + 4 * e, bits);
  }
  uint64_t at = HEADER_BYTES;
  for (int s = 0; s < 4; s++) {
    const uint64_t n = f->stream_bytes[s];
    put_u64(out + 12 + 8 * s, n);
    if (n == 0) continue;
    if (!f->sbuf[s] || n > f->scap[s]) return 0;
    uint8_t len[256];
    uint32_t code[256];
    orc_code_lengths(f->hist + 256 * s, len);
    orc_canonical_codes(len, code);
    if (at + TABLE_BYTES > cap) return 0;
    for (int i = 0; i < 128; i++) out[at + i] = (uint8_t)(len[2 * i] | (len[2 * i + 1] << 4));
    at += TABLE_BYTES;
    uint64_t bits = 0;
    for (uint64_t q = 0; q < n; q++) bits += len[f->sbuf[s][q]];
    const uint64_t pb = (bits + 7) / 8;
    if (at + pb > cap) return 0;
    memset(out + at, 0, pb);
    uint64_t bp = 0;
    for (uint64_t q = 0; q < n; q++) {
      const int L = len[f->sbuf[s][q]];
      const uint32_t c = code[f->sbuf[s][q]];
      for (int b = L - 1; b >= 0; b--, bp++)
        if ((c >> b) & 1u) out[at + bp / 8] |= (uint8_t)(0x80u >> (bp % 8));
    }
    put_u32(out + 44 + 4 * s, (uint32_t)pb);
    at += pb;
  }
  return at;
}

int orc_unpack(const uint8_t *in, uint64_t n, uint8_t *const *streams, const uint64_t *caps, uint64_t *nbytes,
               float *M) {
  if (n < HEADER_BYTES || get_u32(in) != PACK_MAGIC) return -1;
  if (M)
    for (int e = 0; e < 12; e++) {
      uint32_t bits = get_u32(in + 64 + 4 * e);
      memcpy(&M[e], &bits, 4);
    }
  uint64_t at = HEADER_BYTES;
  for (int s = 0; s < 4; s++) {
    const uint64_t cnt = get_u64(in + 12 + 8 * s);
    const uint64_t pb = get_u32(in + 44 + 4 * s);
    nbytes[s] = cnt;
    if (cnt == 0) continue;
    if (cnt > caps[s] || at + TABLE_BYTES + pb > n) return -1;
    uint8_t len[256];
    for (int i = 0; i < 128; i++) { len[2 * i] = in[at + i] & 15u; len[2 * i + 1] = in[at + i] >> 4; }
    at += TABLE_BYTES;
    /* canonical decoding: first code and first index per length */
    int count[PACK_MAXLEN + 2] = {0}, sorted[256], ns = 0;
    for (int L = 1; L <= PACK_MAXLEN; L++)
      for (int v = 0; v < 256; v++)
        if (len[v] == L) { sorted[ns++] = v; count[L]++; }
    const uint8_t *p = in + at;
    uint64_t bp = 0;
    for (uint64_t q = 0; q < cnt; q++) {
      uint32_t code = 0, first = 0;
      int index = 0, L;
      for (L = 1; L <= PACK_MAXLEN; L++) {
        if (bp >= 8 * pb) return -1;
        code |= (p[bp / 8] >> (7 - bp % 8)) & 1u;
        bp++;
        if (code - first < (uint32_t)count[L]) break;
        index += count[L];
        first = (first + (uint32_t)count[L]) << 1;
        code <<= 1;
      }
      if (L > PACK_MAXLEN) return -1;
      streams[s][q] = (uint8_t)sorted[index + (int)(code - first)];
    }
    at += pb;
  }
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops over frames (n >= 1). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

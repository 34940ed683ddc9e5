// Key-frame and predicted-frame encoders (Sec. III-C, III-D) and the
// per-frame stream size (Sec. III-A).
//
// Work decomposition: one work-group per tile-row strip (tile_h range-image
// rows).  Phase 1: each thread owns a tile and fits it from registers.
// Phase 2: one wavefront grows runs left to right (the growth is a
// sequential chain, Sec. III-C); its 64 lanes test a window of 64/(th*tw)
// tiles against the open run's plane per step, so a run that keeps growing
// costs one step per window.  Phase 3: each thread quantises its tile's
// residual pixels and the work-group places them in raster order with a
// prefix sum, and fills per-strip byte histograms of the four streams.  A
// last kernel per frame sums the strip histograms and computes the optimal
// Huffman cost of each stream.
#include "fit.h"

namespace pcc {

// ---------------------------------------------------------------- LDS layout
template <int TH, int TW>
struct StripSmem {
  static constexpr int N = TH * TW;
  static constexpr int NP = N + 1;       // padded tile stride (conflict-free column reads)
  float *r;          // [TC * NP] ranges, tile-major
  float *ca, *sa;    // [W]
  float *ce, *se;    // [TH] row tables of the strip
  uint32_t *cnt;     // [TH * TC] residual counts (aliases ca/sa after the scans)
  float4 *plane;     // [TC] own plane: a, b, c, axis
  uint64_t *omask;   // [TC] own plane's reproduced pixels
  uint64_t *fmask;   // [TC] final mask (covering plane)
  uint8_t *stat;     // [TC] own-fit status
  uint8_t *nv;       // [TC] valid pixels
  uint8_t *cls;      // [TC] final class
  uint8_t *elig;     // [TC] still to be encoded spatially (predicted frames)
  int32_t *runof;    // [TC]
  // predicted frames
  float4 *tplane;    // [TC] key plane a, b, c', axis
  uint64_t *tmask;   // [TC]
  uint8_t *tstat;    // [TC]
  int32_t *krun;     // [TC] key run slot, -1 if the key tile is not plane coded
  uint32_t *hist;    // [4 * 256]
  uint32_t *occ;     // [TH * W / 32]
  int32_t *misc;     // [32] counters / scan partials

  __host__ __device__ static size_t bytes(int W, int TC, bool pred) {
    size_t b = 0;
    b += sizeof(float) * (size_t)TC * NP;
    size_t casa = sizeof(float) * 2 * (size_t)W;
    size_t cntb = sizeof(uint32_t) * (size_t)TH * TC;
    b += casa > cntb ? casa : cntb;
    b += sizeof(float4) * TC + 2 * sizeof(uint64_t) * TC + 4 * TC + sizeof(int32_t) * TC;
    if (pred) b += sizeof(float4) * TC + sizeof(uint64_t) * TC + TC + sizeof(int32_t) * TC;
    b += sizeof(uint32_t) * 1024 + sizeof(uint32_t) * (TH * W / 32) + sizeof(int32_t) * 32;
    b += 2 * 16 * sizeof(float);
    return b + 512;
  }

  __device__ void carve(char *base, int W, int TC, bool pred) {
    char *p = base;
    auto take = [&](size_t n) { char *q = p; p += (n + 15) & ~(size_t)15; return q; };
    r = (float *)take(sizeof(float) * (size_t)TC * NP);
    size_t casa = sizeof(float) * 2 * (size_t)W;
    size_t cntb = sizeof(uint32_t) * (size_t)TH * TC;
    char *u = take(casa > cntb ? casa : cntb);
    ca = (float *)u;
    sa = (float *)u + W;
    cnt = (uint32_t *)u;
    plane = (float4 *)take(sizeof(float4) * TC);
    omask = (uint64_t *)take(sizeof(uint64_t) * TC);
    fmask = (uint64_t *)take(sizeof(uint64_t) * TC);
    stat = (uint8_t *)take(TC);
    nv = (uint8_t *)take(TC);
    cls = (uint8_t *)take(TC);
    elig = (uint8_t *)take(TC);
    runof = (int32_t *)take(sizeof(int32_t) * TC);
    if (pred) {
      tplane = (float4 *)take(sizeof(float4) * TC);
      tmask = (uint64_t *)take(sizeof(uint64_t) * TC);
      tstat = (uint8_t *)take(TC);
      krun = (int32_t *)take(sizeof(int32_t) * TC);
    }
    hist = (uint32_t *)take(sizeof(uint32_t) * 1024);
    occ = (uint32_t *)take(sizeof(uint32_t) * (TH * W / 32));
    misc = (int32_t *)take(sizeof(int32_t) * 32);
    ce = (float *)take(sizeof(float) * 16);
    se = (float *)take(sizeof(float) * 16);
  }
};

__device__ __forceinline__ float4 pack_plane(const Plane &P) { return make_float4(P.a, P.b, P.c, (float)P.k); }
__device__ __forceinline__ Plane unpack_plane(float4 v) { return Plane{(int)v.w, v.x, v.y, v.z}; }

// Bytes of the RUN stream go through these (LDS histogram, stream 1).
__device__ __forceinline__ void hist_byte(uint32_t *hist, int stream, uint32_t v) {
  atomicAdd(&hist[stream * 256 + (v & 255u)], 1u);
}
__device__ __forceinline__ int varint_bytes(uint32_t *hist, uint32_t v) {
  int n = 0;
  while (v >= 128u) { hist_byte(hist, S_RUN, (v & 127u) | 128u); v >>= 7; n++; }
  hist_byte(hist, S_RUN, v);
  return n + 1;
}
__device__ __forceinline__ void f32_bytes(uint32_t *hist, float x) {
  uint32_t u = __float_as_uint(x);
  for (int i = 0; i < 4; i++) hist_byte(hist, S_RUN, (u >> (8 * i)) & 255u);
}

// --------------------------------------------------------- phase 1: loads
// Coalesced float4 loads of the strip's rows into LDS, tile-major.
template <int TH, int TW>
__device__ __forceinline__ void load_strip(StripSmem<TH, TW> &sm, const float *__restrict__ range, const SensorDev &s,
                                           int tr) {
  constexpr int NP = TH * TW + 1;
  const int W = s.W, nq = W / 4;
  const float4 *src = reinterpret_cast<const float4 *>(range + (int64_t)tr * TH * W);
  for (int e = threadIdx.x; e < TH * nq; e += kBlock) {
    int i = e / nq, u = (e % nq) * 4;
    float4 q = src[e];
    int tc = u / TW, k = u % TW;
    float *dst = sm.r + tc * NP + i * TW + k;
    dst[0] = q.x; dst[1] = q.y; dst[2] = q.z; dst[3] = q.w;
  }
}

template <int TH, int TW>
__device__ __forceinline__ TileView<TH, TW> tile_view(const StripSmem<TH, TW> &sm, int tc) {
  constexpr int N = TH * TW, NP = N + 1;
  TileView<TH, TW> T;
  T.r = sm.r + tc * NP;
  T.ce = sm.ce;
  T.se = sm.se;
  T.ca = sm.ca + tc * TW;
  T.sa = sm.sa + tc * TW;
  uint64_t V = 0;
#pragma unroll 4
  for (int j = 0; j < N; j++) V |= (uint64_t)(T.r[j] > 0.0f) << j;
  T.V = V;
  T.nV = __popcll(V);
  return T;
}

// ------------------------------------------------ phase 2: run growth scan
// One wavefront.  Lane l looks at pixel j = l % N of tile t + l / N.
template <int TH, int TW>
struct ScanLane {
  static constexpr int N = TH * TW;
  static constexpr int TPW = 64 / N;     // tiles per window
  int lane, w, j, i, k;
  float ce, se;
  uint64_t segmask;
  __device__ ScanLane(const SensorDev &s, int tr) {
    lane = threadIdx.x & 63;
    w = lane / N;
    j = lane % N;
    i = j / TW;
    k = j % TW;
    ce = s.ce[tr * TH + i];
    se = s.se[tr * TH + i];
    segmask = (N == 64) ? ~0ull : ((1ull << N) - 1ull);
  }
};

// Test the window of tiles [t, t+TPW) against plane P.  Returns the number of
// leading tiles that extend the run; their masks go to fm[].
// `allowed(tc)` says whether tile tc may join this run at all.
template <int TH, int TW, class Allowed>
__device__ __forceinline__ int window_extend(const ScanLane<TH, TW> &L, StripSmem<TH, TW> &sm, const EncParams &p,
                                             const Plane &P, int t, int TC, Allowed allowed, uint64_t &mymask) {
  constexpr int N = TH * TW, NP = N + 1, TPW = 64 / N;
  int tt = t + L.w;
  bool in = tt < TC;
  float r = in ? sm.r[tt * NP + L.j] : 0.0f;
  bool inl = false;
  if (r > 0.0f) {
    int u = tt * TW + L.k;
    inl = reproduces(P, dir_of(L.ce, L.se, sm.ca[u], sm.sa[u]), r, p.eps);
  }
  uint64_t B = __ballot(inl);
  uint64_t m = (B >> (L.w * N)) & L.segmask;
  bool ext = in && allowed(tt) && __popcll(m) >= need_of(p, in ? sm.nv[tt] : 0);
  uint64_t E = __ballot(L.j == 0 && ext);
  // tile w extends iff bit w*N of E is set; count leading extended tiles
  int f = 0;
#pragma unroll
  for (int q = 0; q < TPW; q++) {
    if (((E >> (q * N)) & 1ull) && f == q) f = q + 1;
  }
  mymask = m;
  return f;
}

// Spatial growth over one tile row (Sec. III-C).  `pred`: tiles with
// elig == 0 belong to temporal runs and close any open spatial run.
template <int TH, int TW>
__device__ void grow_spatial(StripSmem<TH, TW> &sm, const SensorDev &s, const EncParams &p, const FrameDev &f,
                             int tr, bool pred) {
  constexpr int TPW = 64 / (TH * TW);
  const int TC = f.TC;
  ScanLane<TH, TW> L(s, tr);
  pc_run *runs = f.sruns + (int64_t)tr * TC;
  int nr = 0, prev_end = 0;
  bool open = false;
  Plane P{0, 0.f, 0.f, 0.f};
  int rs = 0, rlen = 0;
  auto allowed = [&](int tc) { return !pred || sm.elig[tc] != 0; };
  auto close_run = [&]() {
    if (L.lane == 0) {
      runs[nr] = pc_run{rs, rlen, P.k, P.a, P.b, P.c};
      varint_bytes(sm.hist, (uint32_t)(rs - prev_end));
      varint_bytes(sm.hist, (uint32_t)rlen);
      hist_byte(sm.hist, S_RUN, (uint32_t)P.k);
      f32_bytes(sm.hist, P.a);
      f32_bytes(sm.hist, P.b);
      f32_bytes(sm.hist, P.c);
    }
    prev_end = rs + rlen;
    nr++;
    open = false;
  };
  int t = 0;
  while (t < TC) {
    if (open) {
      uint64_t m;
      int fcount = window_extend<TH, TW>(L, sm, p, P, t, TC, allowed, m);
      if (L.j == 0 && L.w < fcount) {
        sm.cls[t + L.w] = CLS_SPATIAL;
        sm.fmask[t + L.w] = m;
        sm.runof[t + L.w] = tr * TC + nr;
      }
      rlen += fcount;
      t += fcount;
      if (fcount == TPW) continue;
      close_run();
      if (t >= TC) break;
    }
    // no open run at tile t
    bool el = !pred || sm.elig[t] != 0;
    if (el && sm.stat[t] == ST_ACCEPTED) {
      P = unpack_plane(sm.plane[t]);
      rs = t;
      rlen = 1;
      open = true;
      if (L.lane == 0) {
        sm.cls[t] = CLS_SPATIAL;
        sm.fmask[t] = sm.omask[t];
        sm.runof[t] = tr * TC + nr;
      }
    } else if (el && L.lane == 0) {
      sm.cls[t] = sm.nv[t] ? CLS_UNFIT : CLS_EMPTY;
      sm.fmask[t] = 0;
      sm.runof[t] = -1;
    }
    t++;
  }
  if (open) close_run();
  if (L.lane == 0) {
    f.nruns[tr] = nr;
    varint_bytes(sm.hist, (uint32_t)nr);
    sm.misc[0] = nr;
  }
}

// Temporal growth (Sec. III-D): a temporal run grows while the key run stays
// the same and (key normal, c' of the run start) reproduces the tile.  Tiles
// not taken become eligible for the spatial pass.
template <int TH, int TW>
__device__ void grow_temporal(StripSmem<TH, TW> &sm, const SensorDev &s, const EncParams &p, const FrameDev &f,
                              int tr) {
  constexpr int TPW = 64 / (TH * TW);
  const int TC = f.TC, T = f.T;
  ScanLane<TH, TW> L(s, tr);
  pc_prun *runs = f.pruns + (int64_t)tr * TC;
  int nr = 0, prev_end = 0;
  bool open = false;
  Plane P{0, 0.f, 0.f, 0.f};
  int rs = 0, rlen = 0, rk = -1;
  auto close_run = [&]() {
    if (L.lane == 0) {
      runs[nr] = pc_prun{rs, rlen, rk, P.c};
      varint_bytes(sm.hist, (uint32_t)(rs - prev_end));
      varint_bytes(sm.hist, (uint32_t)rlen);
      f32_bytes(sm.hist, P.c);
    }
    prev_end = rs + rlen;
    nr++;
    open = false;
  };
  int t = 0;
  while (t < TC) {
    if (open) {
      uint64_t m;
      int key_run = rk;
      auto allowed = [&](int tc) { return sm.krun[tc] == key_run; };
      int fcount = window_extend<TH, TW>(L, sm, p, P, t, TC, allowed, m);
      if (L.j == 0 && L.w < fcount) {
        sm.cls[t + L.w] = CLS_TEMPORAL;
        sm.fmask[t + L.w] = m;
        sm.runof[t + L.w] = T + tr * TC + nr;
        sm.elig[t + L.w] = 0;
      }
      rlen += fcount;
      t += fcount;
      if (fcount == TPW) continue;
      close_run();
      if (t >= TC) break;
    }
    if (sm.tstat[t] == 2) {
      P = unpack_plane(sm.tplane[t]);
      rs = t;
      rlen = 1;
      rk = sm.krun[t];
      open = true;
      if (L.lane == 0) {
        sm.cls[t] = CLS_TEMPORAL;
        sm.fmask[t] = sm.tmask[t];
        sm.runof[t] = T + tr * TC + nr;
        sm.elig[t] = 0;
      }
    } else if (L.lane == 0) {
      sm.elig[t] = 1;
    }
    t++;
  }
  if (open) close_run();
  if (L.lane == 0) {
    f.nruns[f.TR + tr] = nr;
    varint_bytes(sm.hist, (uint32_t)nr);
    sm.misc[1] = nr;
  }
}

// ----------------------------------------------------- phase 3: residuals
// Block-wide exclusive scan of sm.cnt[0 .. n) in place; returns the total.
template <int TH, int TW>
__device__ uint32_t block_exclusive_scan(StripSmem<TH, TW> &sm, int n) {
  const int tid = threadIdx.x;
  const int per = (n + kBlock - 1) / kBlock;
  const int b = tid * per, e = min(n, b + per);
  uint32_t local = 0;
  for (int q = b; q < e; q++) local += sm.cnt[q];
  // wave inclusive scan
  uint32_t x = local;
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __shared__ uint32_t wsum[kBlock / 64];
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint32_t base = 0, total = 0;
  for (int q = 0; q < kBlock / 64; q++) {
    if (q < wv) base += wsum[q];
    total += wsum[q];
  }
  uint32_t run = base + x - local;
  for (int q = b; q < e; q++) {
    uint32_t c = sm.cnt[q];
    sm.cnt[q] = run;
    run += c;
  }
  __syncthreads();
  return total;
}

// Pack the bits of `m` at the set positions of `sel`, in order (LSB first).
__device__ __forceinline__ uint64_t pext64(uint64_t m, uint64_t sel) {
  uint64_t out = 0;
  int o = 0;
  while (sel) {
    int b = __ffsll((long long)sel) - 1;
    out |= ((m >> b) & 1ull) << o;
    o++;
    sel &= sel - 1;
  }
  return out;
}

template <int TH, int TW>
__device__ void residuals_and_streams(StripSmem<TH, TW> &sm, const float *__restrict__ range, const SensorDev &s,
                                      const EncParams &p, const FrameDev &f, int tr, int fits, int fp64) {
  constexpr int N = TH * TW, NP = N + 1;
  const int TC = f.TC, W = s.W, tid = threadIdx.x;
  // counts per (row in strip, tile) in raster order, OCC words, MASK bytes
  for (int tc = tid; tc < TC; tc += kBlock) {
    uint64_t V = 0;
#pragma unroll
    for (int j = 0; j < N; j++) V |= (uint64_t)(sm.r[tc * NP + j] > 0.0f) << j;
    int cl = sm.cls[tc];
    bool cov = cl == CLS_SPATIAL || cl == CLS_TEMPORAL;
    uint64_t R = V & ~(cov ? sm.fmask[tc] : 0ull);
#pragma unroll
    for (int i = 0; i < TH; i++) {
      uint32_t rowbits = (uint32_t)((V >> (i * TW)) & ((1ull << TW) - 1ull));
      sm.cnt[i * TC + tc] = __popc((uint32_t)((R >> (i * TW)) & ((1ull << TW) - 1ull)));
      int bit = i * W + tc * TW;
      if (rowbits) atomicOr(&sm.occ[bit >> 5], rowbits << (bit & 31));
    }
    int nv = sm.nv[tc];
    if (cov && nv > 0) {
      uint64_t packed = pext64(sm.fmask[tc], V);
      for (int q = 0; q < (nv + 7) / 8; q++) hist_byte(sm.hist, S_MASK, (uint32_t)(packed >> (8 * q)) & 255u);
    }
  }
  __syncthreads();
  uint32_t total = block_exclusive_scan<TH, TW>(sm, TH * TC);
  // codes, raster order within the strip
  uint16_t *res = f.res + (int64_t)tr * TH * W;
  uint32_t bad = 0;
  for (int tc = tid; tc < TC; tc += kBlock) {
    int cl = sm.cls[tc];
    bool cov = cl == CLS_SPATIAL || cl == CLS_TEMPORAL;
    uint64_t fm = cov ? sm.fmask[tc] : 0ull;
#pragma unroll
    for (int i = 0; i < TH; i++) {
      uint32_t o = sm.cnt[i * TC + tc];
#pragma unroll
      for (int k = 0; k < TW; k++) {
        int j = i * TW + k;
        float r = sm.r[tc * NP + j];
        if (r > 0.0f && !((fm >> j) & 1ull)) {
          float q = rintf(r * p.inv);
          double back = (double)(q * p.step);
          if (q > 65535.0f || fabs(back - (double)r) > (double)p.eps) {
            bad = 1;
            q = fminf(q, 65535.0f);
          }
          uint32_t code = (uint32_t)q;
          res[o++] = (uint16_t)code;
          hist_byte(sm.hist, S_RES, code & 255u);
          hist_byte(sm.hist, S_RES, code >> 8);
        }
      }
    }
  }
  // per-tile outputs
  for (int tc = tid; tc < TC; tc += kBlock) {
    int t = tr * TC + tc;
    f.cls[t] = sm.cls[tc];
    f.mask[t] = (sm.cls[tc] == CLS_SPATIAL || sm.cls[tc] == CLS_TEMPORAL) ? sm.fmask[tc] : 0ull;
    f.run_of[t] = sm.runof[tc];
  }
  // block reductions of counters
  __shared__ int red[8];
  if (tid < 8) red[tid] = 0;
  __syncthreads();
  int nvalid = 0, nc[4] = {0, 0, 0, 0};
  for (int tc = tid; tc < TC; tc += kBlock) {
    nvalid += sm.nv[tc];
    nc[sm.cls[tc]]++;
  }
  atomicAdd(&red[0], nvalid);
  for (int c = 0; c < 4; c++) atomicAdd(&red[1 + c], nc[c]);
  atomicAdd(&red[5], fits);
  atomicAdd(&red[6], fp64);
  if (bad) atomicOr(&red[7], 1);
  __syncthreads();
  // OCC words to global and into the OCC histogram (little-endian bytes)
  const int nw = TH * W / 32;
  uint32_t *occ = f.occ + (int64_t)tr * nw;
  for (int q = tid; q < nw; q += kBlock) {
    uint32_t wv = sm.occ[q];
    occ[q] = wv;
    for (int b = 0; b < 4; b++) hist_byte(sm.hist, S_OCC, (wv >> (8 * b)) & 255u);
  }
  __syncthreads();
  uint32_t *ss = f.strip + (int64_t)tr * PC_STRIP_WORDS;
  for (int q = tid; q < 1024; q += kBlock) ss[q] = sm.hist[q];
  if (tid == 0) {
    uint32_t *st = ss + 1024;
    st[PC_SS_VALID] = red[0];
    st[PC_SS_RES] = total;
    for (int c = 0; c < 4; c++) st[PC_SS_TILES + c] = red[1 + c];
    st[PC_SS_SRUNS] = sm.misc[0];
    st[PC_SS_PRUNS] = sm.misc[1];
    st[PC_SS_FITS] = red[5];
    st[PC_SS_FP64] = red[6];
    st[PC_SS_STATUS] = red[7] ? PC_STATUS_RANGE : 0u;
    st[PC_SS_SEEDED] = sm.misc[2];
    st[PC_SS_FALLBACK] = sm.misc[3];
    for (int q = PC_SS_FALLBACK + 1; q < PC_STRIP_STATS; q++) st[q] = 0;
    f.nres[tr] = (int32_t)total;
  }
}

template <int TH, int TW>
__device__ void strip_init(StripSmem<TH, TW> &sm, const SensorDev &s, int tr) {
  const int tid = threadIdx.x;
  for (int q = tid; q < 1024; q += kBlock) sm.hist[q] = 0;
  for (int q = tid; q < TH * s.W / 32; q += kBlock) sm.occ[q] = 0;
  if (tid < 32) sm.misc[tid] = 0;
  for (int u = tid; u < s.W; u += kBlock) {
    sm.ca[u] = s.ca[u];
    sm.sa[u] = s.sa[u];
  }
  if (tid < TH) {
    sm.ce[tid] = s.ce[tr * TH + tid];
    sm.se[tid] = s.se[tr * TH + tid];
  }
}

// ------------------------------------------------------------ the kernels
template <int TH, int TW>
__global__ void __launch_bounds__(kBlock) k_encode_key(const float *__restrict__ range, SensorDev s, EncParams p,
                                                       const float *__restrict__ seed, FrameDev f) {
  extern __shared__ __align__(16) char smem_raw[];
  StripSmem<TH, TW> sm;
  const int TC = f.TC, tr = blockIdx.x;
  sm.carve(smem_raw, s.W, TC, false);
  strip_init<TH, TW>(sm, s, tr);
  load_strip<TH, TW>(sm, range, s, tr);
  __syncthreads();
  int fits = 0, fp64 = 0;
  for (int tc = threadIdx.x; tc < TC; tc += kBlock) {
    TileView<TH, TW> T = tile_view<TH, TW>(sm, tc);
    sm.nv[tc] = (uint8_t)T.nV;
    FitResult R = own_fit<TH, TW>(T, p, fits, fp64);
    sm.plane[tc] = pack_plane(R.P);
    sm.omask[tc] = R.mask;
    sm.stat[tc] = (uint8_t)R.status;
    pc_tile_rec rec;
    rec.a = R.P.a; rec.b = R.P.b; rec.c = R.P.c;
    rec.axis = (uint8_t)R.P.k; rec.status = (uint8_t)R.status; rec.iters = (uint8_t)R.iters; rec.t_status = 0;
    rec.mask = R.mask; rec.t_mask = 0; rec.t_c = 0.f; rec.t_iters = 0; rec.seeded = 0; rec.pad[0] = rec.pad[1] = 0;
    f.tiles[tr * TC + tc] = rec;
  }
  __syncthreads();
  if (threadIdx.x < 64) grow_spatial<TH, TW>(sm, s, p, f, tr, false);
  if (threadIdx.x == 0) f.nruns[f.TR + tr] = 0;
  __syncthreads();
  residuals_and_streams<TH, TW>(sm, range, s, p, f, tr, fits, fp64);
}

template <int TH, int TW>
__global__ void __launch_bounds__(kBlock) k_encode_pred(const float *__restrict__ range, SensorDev s, EncParams p,
                                                        FrameDev key, FrameDev f) {
  extern __shared__ __align__(16) char smem_raw[];
  StripSmem<TH, TW> sm;
  const int TC = f.TC, tr = blockIdx.x;
  sm.carve(smem_raw, s.W, TC, true);
  strip_init<TH, TW>(sm, s, tr);
  load_strip<TH, TW>(sm, range, s, tr);
  __syncthreads();
  int fits = 0, fp64 = 0;
  // phase 1a: temporal fits against the key frame's run planes
  for (int tc = threadIdx.x; tc < TC; tc += kBlock) {
    const int t = tr * TC + tc;
    TileView<TH, TW> T = tile_view<TH, TW>(sm, tc);
    sm.nv[tc] = (uint8_t)T.nV;
    int kr = key.cls[t] == CLS_SPATIAL ? key.run_of[t] : -1;
    sm.krun[tc] = kr;
    FitResult R{Plane{0, 0.f, 0.f, 0.f}, 0ull, 0, 0};
    if (kr >= 0) {
      pc_run q = key.sruns[kr];
      R = temporal_fit<TH, TW>(T, Plane{q.axis, q.a, q.b, q.c}, p);
    }
    sm.tplane[tc] = pack_plane(R.P);
    sm.tmask[tc] = R.mask;
    sm.tstat[tc] = (uint8_t)R.status;
    sm.cls[tc] = CLS_EMPTY;
    sm.elig[tc] = 0;
    pc_tile_rec rec;
    rec.a = 0.f; rec.b = 0.f; rec.c = 0.f; rec.axis = 0; rec.status = 0; rec.iters = 0;
    rec.t_status = (uint8_t)R.status; rec.mask = 0; rec.t_mask = R.mask; rec.t_c = R.P.c;
    rec.t_iters = (uint8_t)R.iters; rec.seeded = 0; rec.pad[0] = rec.pad[1] = 0;
    f.tiles[t] = rec;
  }
  __syncthreads();
  if (threadIdx.x < 64) grow_temporal<TH, TW>(sm, s, p, f, tr);
  __syncthreads();
  // phase 1b: own fits of the tiles left over
  for (int tc = threadIdx.x; tc < TC; tc += kBlock) {
    FitResult R{Plane{0, 0.f, 0.f, 0.f}, 0ull, ST_EMPTY, 0};
    if (sm.elig[tc]) {
      TileView<TH, TW> T = tile_view<TH, TW>(sm, tc);
      R = own_fit<TH, TW>(T, p, fits, fp64);
      pc_tile_rec *rec = &f.tiles[tr * TC + tc];
      rec->a = R.P.a; rec->b = R.P.b; rec->c = R.P.c;
      rec->axis = (uint8_t)R.P.k; rec->status = (uint8_t)R.status; rec->iters = (uint8_t)R.iters;
      rec->mask = R.mask;
    }
    sm.plane[tc] = pack_plane(R.P);
    sm.omask[tc] = R.mask;
    sm.stat[tc] = (uint8_t)R.status;
  }
  __syncthreads();
  if (threadIdx.x < 64) grow_spatial<TH, TW>(sm, s, p, f, tr, true);
  __syncthreads();
  residuals_and_streams<TH, TW>(sm, range, s, p, f, tr, fits, fp64);
}

// --------------------------------------------------- per-frame stream size
// Optimal Huffman cost of a byte histogram: with the leaves sorted, merge the
// two lightest of (next leaf, next internal node) until one node is left;
// the cost is the sum of the merged weights (two-queue construction).
__device__ uint64_t huffman_cost_wave(uint32_t *h, uint64_t *q, int lane) {
  // rank sort of the 256 counts (ties by index)
  uint32_t c[4];
  int rk[4];
#pragma unroll
  for (int e = 0; e < 4; e++) { c[e] = h[lane * 4 + e]; rk[e] = 0; }
  for (int o = 0; o < 256; o++) {
    uint32_t x = h[o];
#pragma unroll
    for (int e = 0; e < 4; e++) rk[e] += (x < c[e]) || (x == c[e] && o < lane * 4 + e);
  }
  __syncthreads();
  // h is reused as the sorted array
#pragma unroll
  for (int e = 0; e < 4; e++) h[rk[e]] = c[e];
  __syncthreads();
  uint64_t cost = 0;
  if (lane == 0) {
    int i = 0;
    while (i < 256 && h[i] == 0) i++;
    int m = 256 - i;
    if (m == 1) {
      cost = h[i];
    } else if (m > 1) {
      int qh = 0, qt = 0;
      for (int step = 0; step < m - 1; step++) {
        uint64_t ab[2];
        for (int z = 0; z < 2; z++) {
          bool take_leaf = i < 256 && (qh == qt || (uint64_t)h[i] <= q[qh]);
          ab[z] = take_leaf ? (uint64_t)h[i++] : q[qh++];
        }
        uint64_t wsum = ab[0] + ab[1];
        cost += wsum;
        q[qt++] = wsum;
      }
    }
  }
  return cost;
}

__global__ void __launch_bounds__(256) k_finish_frame(FrameDev f, int kind, Mat12 M, int hasM) {
  __shared__ uint32_t h[4][256];
  __shared__ uint64_t q[4][256];
  __shared__ uint32_t st[PC_STRIP_STATS];
  const int tid = threadIdx.x;
  for (int e = tid; e < 1024; e += 256) {
    uint32_t sum = 0;
    for (int r = 0; r < f.TR; r++) sum += f.strip[(int64_t)r * PC_STRIP_WORDS + e];
    h[e >> 8][e & 255] = sum;
  }
  if (tid < PC_STRIP_STATS) {
    uint32_t sum = 0;
    for (int r = 0; r < f.TR; r++) {
      uint32_t v = f.strip[(int64_t)r * PC_STRIP_WORDS + 1024 + tid];
      sum = (tid == PC_SS_STATUS) ? (sum | v) : sum + v;
    }
    st[tid] = sum;
  }
  __syncthreads();
  const int wv = tid >> 6, lane = tid & 63;
  // stream byte counts
  uint64_t nbytes = 0;
  for (int o = lane; o < 256; o += 64) nbytes += h[wv][o];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nbytes += __shfl_xor(nbytes, o, 64);
  uint64_t bits = huffman_cost_wave(h[wv], q[wv], lane);
  __shared__ uint64_t sb[4], sc[4];
  if (lane == 0) { sb[wv] = nbytes; sc[wv] = bits; }
  __syncthreads();
  if (tid == 0) {
    pc_frame_info *I = f.info;
    I->kind = kind;
    I->status = st[PC_SS_STATUS];
    I->n_sruns = (int32_t)st[PC_SS_SRUNS];
    I->n_pruns = (int32_t)st[PC_SS_PRUNS];
    I->n_valid = st[PC_SS_VALID];
    I->n_res = st[PC_SS_RES];
    for (int c = 0; c < 4; c++) I->tiles[c] = (int32_t)st[PC_SS_TILES + c];
    I->fits = (int32_t)st[PC_SS_FITS];
    I->fp64_fits = (int32_t)st[PC_SS_FP64];
    I->seeded = (int32_t)st[PC_SS_SEEDED];
    I->fallback = (int32_t)st[PC_SS_FALLBACK];
    uint64_t size = kHeaderBytes;
    for (int c = 0; c < 4; c++) {
      I->stream_bytes[c] = sb[c];
      I->coded_bits[c] = sc[c];
      if (sb[c]) size += (sc[c] + 7) / 8 + kTableBytes;
    }
    I->size_bytes = size;
    for (int e = 0; e < 12; e++) I->M[e] = hasM ? M.m[e] : (e % 5 == 0 ? 1.0f : 0.0f);
    for (int e = 0; e < 4; e++) I->pad[e] = 0;
  }
}

// -------------------------------------------------------------- launchers
template <int TH, int TW>
static hipError_t launch_key_t(const float *range, const SensorDev &s, const EncParams &p, const float *seed,
                               const FrameDev &f, hipStream_t st) {
  size_t sh = StripSmem<TH, TW>::bytes(s.W, f.TC, false);
  hipError_t e = hipFuncSetAttribute((const void *)k_encode_key<TH, TW>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_encode_key<TH, TW>), dim3(f.TR), dim3(kBlock), sh, st, range, s, p, seed, f);
  return hipGetLastError();
}

template <int TH, int TW>
static hipError_t launch_pred_t(const FrameDev &key, const float *range, const SensorDev &s, const EncParams &p,
                                const FrameDev &f, hipStream_t st) {
  size_t sh = StripSmem<TH, TW>::bytes(s.W, f.TC, true);
  hipError_t e = hipFuncSetAttribute((const void *)k_encode_pred<TH, TW>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_encode_pred<TH, TW>), dim3(f.TR), dim3(kBlock), sh, st, range, s, p, key, f);
  return hipGetLastError();
}

static Mat12 mat12(const float *M12) {
  Mat12 m{};
  if (M12)
    for (int e = 0; e < 12; e++) m.m[e] = M12[e];
  return m;
}

#define PC_DISPATCH_TILE(th, tw, CALL)                  \
  if (th == 4 && tw == 4) return CALL(4, 4);            \
  if (th == 4 && tw == 8) return CALL(4, 8);            \
  if (th == 4 && tw == 16) return CALL(4, 16);          \
  if (th == 8 && tw == 8) return CALL(8, 8);            \
  return hipErrorInvalidValue;

hipError_t launch_key(const float *range, const SensorDev &s, const EncParams &p, const float *seed,
                      const FrameDev &f, const float *M12, hipStream_t st) {
  hipError_t e;
#define CALL_KEY(a, b) launch_key_t<a, b>(range, s, p, seed, f, st)
  e = [&]() -> hipError_t { PC_DISPATCH_TILE(p.th, p.tw, CALL_KEY) }();
#undef CALL_KEY
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finish_frame, dim3(1), dim3(256), 0, st, f, 0, mat12(M12), M12 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_pred(const FrameDev &key, const float *range, const SensorDev &s, const EncParams &p,
                       const FrameDev &f, const float *M12, hipStream_t st) {
  hipError_t e;
#define CALL_PRED(a, b) launch_pred_t<a, b>(key, range, s, p, f, st)
  e = [&]() -> hipError_t { PC_DISPATCH_TILE(p.th, p.tw, CALL_PRED) }();
#undef CALL_PRED
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finish_frame, dim3(1), dim3(256), 0, st, f, 1, mat12(M12), M12 ? 1 : 0);
  return hipGetLastError();
}

}  // namespace pcc

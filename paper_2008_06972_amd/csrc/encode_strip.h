// Device bodies of the key-frame and predicted-frame strip encoders and the
// per-frame size computation, shared by the per-frame kernels (encode.hip)
// and the batched persistent kernels (batch.hip).
//
// Key frames are encoded spatially (Sec. III-C), predicted frames
// temporally first and then spatially on what is left (Sec. III-D); stream
// sizes follow from byte histograms and an optimal Huffman code (Sec. III-A).
//
// One work-group encodes one tile-row strip (tile_h rows of the range
// image), staged in LDS:
//  1. fits: each thread owns a tile and runs the iterative least-squares fit
//     (predicted frames: the offset-only fit against the key run's plane);
//  2. reach: each tile whose fit is accepted measures, in parallel, how many
//     following tiles (up to kReach) its plane reproduces -- the extension
//     test of the horizontal growth;
//  3. chain: one wavefront walks the run starts: a run starts at the next
//     accepted tile and covers its reach; the next run starts at the first
//     accepted tile after it (runs that reach kReach continue with a
//     wavefront-wide test of the following tiles).  This is exactly the
//     sequential growth, in O(runs) steps; the runs' stream bytes are then
//     counted in parallel;
//  4. masks: each thread records its tile's class and the pixels the covering
//     run's plane reproduces;
//  5. residuals: codes of the remaining pixels, placed in raster order by a
//     work-group prefix sum, and byte histograms of the four streams.
// A last block per frame sums the strip histograms and computes the optimal
// Huffman cost of each stream.
#pragma once
#include "fit.h"

namespace pcc {

constexpr int kReach = 6;     // tiles a fit measures its reach over before the chain continues it

// ---------------------------------------------------------------- LDS layout
template <int TH, int TW>
struct StripSmem {
  static constexpr int N = TH * TW;
  static constexpr int NP = N + 4;       // tile stride: 16-byte aligned rows, conflict-free 128-bit reads across threads
  float *r;          // [TC * NP] ranges, tile-major
  const float *ca, *sa;   // [W] column tables (global memory, L1/L2 resident)
  uint32_t *cnt;     // [TH * TC] residual counts
  float *ce, *se;    // [TH] row tables of the strip
  float4 *plane;     // [TC] own plane: a, b, c, axis
  uint64_t *omask;   // [TC] own plane's reproduced pixels
  uint64_t *fmask;   // [TC] final mask (covering plane)
  uint8_t *stat;     // [TC] own-fit status
  uint8_t *nv;       // [TC] valid pixels
  uint8_t *cls;      // [TC] final class
  uint8_t *elig;     // [TC] still to be encoded spatially (predicted frames)
  uint8_t *reach;    // [TC] tiles a run starting here covers after its start (<= kReach)
  int32_t *runof;    // [TC] run index within the current pass, then the stream's run slot
  int32_t *rs;       // [TC] run starts of the current pass
  int32_t *rl;       // [TC] run lengths
  uint64_t *acc;     // [8] tiles that may start a run (bit tc)
  // predicted frames
  float4 *tplane;    // [TC] key plane a, b with own offset c', axis
  uint64_t *tmask;   // [TC]
  uint8_t *tstat;    // [TC]
  int32_t *krun;     // [TC] key run slot, -1 if the key tile is not plane coded
  uint32_t *hist;    // [4 * 256]
  uint32_t *occ;     // [TH * W / 32]
  int32_t *misc;     // [32] counters

  __host__ __device__ static size_t bytes(int W, int TC, bool pred) {
    auto a16 = [](size_t n) { return (n + 15) & ~(size_t)15; };
    size_t b = 0;
    b += a16(sizeof(float) * (size_t)TC * NP);
    b += a16(sizeof(uint32_t) * (size_t)TH * TC);
    b += 2 * a16(sizeof(float) * 16);
    b += a16(sizeof(float4) * TC) + 2 * a16(sizeof(uint64_t) * TC) + 5 * a16(TC) + 3 * a16(sizeof(int32_t) * TC);
    b += a16(sizeof(uint64_t) * 8);
    if (pred) b += a16(sizeof(float4) * TC) + a16(sizeof(uint64_t) * TC) + a16(TC) + a16(sizeof(int32_t) * TC);
    b += a16(sizeof(uint32_t) * 1024) + a16(sizeof(uint32_t) * (TH * W / 32)) + a16(sizeof(int32_t) * 32);
    return b + 64;
  }

  __device__ void carve(char *base, int W, int TC, bool pred) {
    char *p = base;
    auto take = [&](size_t n) { char *q = p; p += (n + 15) & ~(size_t)15; return q; };
    r = (float *)take(sizeof(float) * (size_t)TC * NP);
    cnt = (uint32_t *)take(sizeof(uint32_t) * (size_t)TH * TC);
    ce = (float *)take(sizeof(float) * 16);
    se = (float *)take(sizeof(float) * 16);
    plane = (float4 *)take(sizeof(float4) * TC);
    omask = (uint64_t *)take(sizeof(uint64_t) * TC);
    fmask = (uint64_t *)take(sizeof(uint64_t) * TC);
    stat = (uint8_t *)take(TC);
    nv = (uint8_t *)take(TC);
    cls = (uint8_t *)take(TC);
    elig = (uint8_t *)take(TC);
    reach = (uint8_t *)take(TC);
    runof = (int32_t *)take(sizeof(int32_t) * TC);
    rs = (int32_t *)take(sizeof(int32_t) * TC);
    rl = (int32_t *)take(sizeof(int32_t) * TC);
    acc = (uint64_t *)take(sizeof(uint64_t) * 8);
    if (pred) {
      tplane = (float4 *)take(sizeof(float4) * TC);
      tmask = (uint64_t *)take(sizeof(uint64_t) * TC);
      tstat = (uint8_t *)take(TC);
      krun = (int32_t *)take(sizeof(int32_t) * TC);
    }
    hist = (uint32_t *)take(sizeof(uint32_t) * 1024);
    occ = (uint32_t *)take(sizeof(uint32_t) * (TH * W / 32));
    misc = (int32_t *)take(sizeof(int32_t) * 32);
  }
};

__device__ __forceinline__ float4 pack_plane(const Plane &P) { return make_float4(P.a, P.b, P.c, (float)P.k); }
__device__ __forceinline__ Plane unpack_plane(float4 v) { return Plane{(int)v.w, v.x, v.y, v.z}; }

// Bytes of the serialized streams go into the LDS histograms.
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

// --------------------------------------------------------- phase 0: loads
template <int TH, int TW>
__device__ void strip_init(StripSmem<TH, TW> &sm, const SensorDev &s, int tr) {
  const int tid = threadIdx.x;
  for (int q = tid; q < 1024; q += kBlock) sm.hist[q] = 0;
  for (int q = tid; q < TH * s.W / 32; q += kBlock) sm.occ[q] = 0;
  if (tid < 32) sm.misc[tid] = 0;
  sm.ca = s.ca;
  sm.sa = s.sa;
  if (tid < TH) {
    sm.ce[tid] = s.ce[tr * TH + tid];
    sm.se[tid] = s.se[tr * TH + tid];
  }
}

// Coalesced float4 loads of the strip's rows into LDS, tile-major.
template <int TH, int TW>
__device__ __forceinline__ void load_strip(StripSmem<TH, TW> &sm, const float *__restrict__ range, const SensorDev &s,
                                           int tr) {
  constexpr int NP = StripSmem<TH, TW>::NP;
  const int W = s.W, nq = W / 4;
  const float4 *src = reinterpret_cast<const float4 *>(range + (int64_t)tr * TH * W);
  for (int e = threadIdx.x; e < TH * nq; e += kBlock) {
    int i = e / nq, u = (e % nq) * 4;
    float4 q = src[e];
    // empty pixels are 0 (+inf is taken as empty too)
    q.x = q.x < INFINITY ? q.x : 0.0f;
    q.y = q.y < INFINITY ? q.y : 0.0f;
    q.z = q.z < INFINITY ? q.z : 0.0f;
    q.w = q.w < INFINITY ? q.w : 0.0f;
    int tc = u / TW, k = u % TW;
    *reinterpret_cast<float4 *>(sm.r + tc * NP + i * TW + k) = q;
  }
}

// Where a strip's ranges come from: a range image (0 = empty), or the
// strip's bucket of (pixel within the strip, range bits) entries from the
// batched binning pass, resolved here with LDS atomicMin (nearest point
// wins, Sec. III-D).  range_out, if set, receives the strip's range image.
struct StripSrc {
  const float *range;
  const uint2 *bucket;     // frame's bucket entries
  const int *bcount;       // [TR] entries per strip
  const int *boff;         // [TR] first entry of each strip
  float *range_out;
};

template <int TH, int TW>
__device__ __forceinline__ void load_source(StripSmem<TH, TW> &sm, const StripSrc &src, const SensorDev &s, int tr) {
  constexpr int NP = StripSmem<TH, TW>::NP;
  const int W = s.W, TC = W / TW, tid = threadIdx.x;
  if (!src.bucket) {
    load_strip<TH, TW>(sm, src.range, s, tr);
  } else {
    uint32_t *ri = reinterpret_cast<uint32_t *>(sm.r);
    for (int e = tid; e < TC * NP; e += kBlock) ri[e] = 0x7f800000u;   // +inf: empty
    __syncthreads();
    const int n = src.bcount[tr];
    const uint2 *b = src.bucket + src.boff[tr];
    for (int q = tid; q < n; q += kBlock) {
      uint2 en = b[q];
      if (en.x >= (uint32_t)(TH * W)) continue;
      int i = (int)en.x / W, u = (int)en.x - i * W;
      atomicMin(&ri[(u / TW) * NP + i * TW + (u % TW)], en.y);
    }
    __syncthreads();
    for (int e = tid; e < TC * NP; e += kBlock)
      if (ri[e] == 0x7f800000u) ri[e] = 0u;
  }
  if (src.range_out) {
    __syncthreads();
    float *dst = src.range_out + (int64_t)tr * TH * W;
    for (int e = tid; e < TH * W; e += kBlock) {
      int i = e / W, u = e - i * W;
      dst[e] = sm.r[(u / TW) * NP + i * TW + (u % TW)];
    }
  }
}

// A tile of the strip as seen by one thread (its own, or a neighbour it
// tests): ranges in LDS, column tables loaded into registers.
template <int TH, int TW>
__device__ __forceinline__ TileRows<TH, TW> tile_at(const StripSmem<TH, TW> &sm, int tc, int TC, bool with_valid) {
  TileRows<TH, TW> T;
  T.rp = sm.r + tc * StripSmem<TH, TW>::NP;
  T.ce = sm.ce;
  T.se = sm.se;
  T.cal = sm.ca + tc * TW;
  T.sal = sm.sa + tc * TW;
  T.cstride = 1;
  const float4 *ca4 = reinterpret_cast<const float4 *>(T.cal), *sa4 = reinterpret_cast<const float4 *>(T.sal);
#pragma unroll
  for (int k4 = 0; k4 < TW / 4; k4++) {
    float4 c = ca4[k4], d = sa4[k4];
    T.ca[4 * k4] = c.x; T.ca[4 * k4 + 1] = c.y; T.ca[4 * k4 + 2] = c.z; T.ca[4 * k4 + 3] = c.w;
    T.sa[4 * k4] = d.x; T.sa[4 * k4 + 1] = d.y; T.sa[4 * k4 + 2] = d.z; T.sa[4 * k4 + 3] = d.w;
  }
  T.V = 0;
  T.nV = 0;
  if (with_valid) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < TH; i++) {
      float r[TW];
      T.row(i, r);
#pragma unroll
      for (int k = 0; k < TW; k++) {
        const int j = i * TW + k;
        if (j < 32) lo |= (uint32_t)(r[k] > 0.0f) << (j & 31); else hi |= (uint32_t)(r[k] > 0.0f) << (j & 31);
      }
    }
    T.V = ((uint64_t)hi << 32) | lo;
    T.nV = __popcll(T.V);
  }
  return T;
}

// Pixels of tile tc that plane P reproduces.
template <int TH, int TW>
__device__ __forceinline__ uint64_t inliers_at(const StripSmem<TH, TW> &sm, int tc, int TC, const Plane &P,
                                               float eps) {
  return inliers(tile_at<TH, TW>(sm, tc, TC, false), P, eps);
}

// ------------------------------------------------ phases 2-4: run growth
// Reach of a run started at tile s with plane P: the number of following
// tiles (at most kReach) it extends over.  `allowed(s, t)` says whether tile
// t may join a run started at s.
template <int TH, int TW, class Allowed>
__device__ __forceinline__ int reach_of(const StripSmem<TH, TW> &sm, const EncParams &p, const Plane &P, int s, int TC,
                                        Allowed allowed) {
  int e = 0;
  for (int t = s + 1; t < TC && e < kReach; t++) {
    if (!allowed(s, t)) break;
    int n = __popcll(inliers_at<TH, TW>(sm, t, TC, P, p.eps));
    if (n < need_of(p, sm.nv[t])) break;
    e++;
  }
  return e;
}

// Continue a run beyond its measured reach: the wavefront tests windows of
// 64/(th*tw) tiles from tile t on; returns how many more tiles join.
template <int TH, int TW, class Allowed>
__device__ int extend_beyond(const StripSmem<TH, TW> &sm, const EncParams &p, const Plane &P, int s, int t, int TC,
                             Allowed allowed) {
  constexpr int N = TH * TW, NP = StripSmem<TH, TW>::NP, TPW = 64 / N;
  const int lane = threadIdx.x & 63, w = lane / N, j = lane % N, i = j / TW, k = j % TW;
  const uint64_t segmask = (N == 64) ? ~0ull : ((1ull << N) - 1ull);
  int added = 0;
  while (t < TC) {
    int tt = t + w;
    bool in = tt < TC;
    float r = in ? sm.r[tt * NP + j] : 0.0f;
    bool inl = false;
    if (r > 0.0f) {
      Dir d = dir_of(sm.ce[i], sm.se[i], sm.ca[tt * TW + k], sm.sa[tt * TW + k]);
      inl = reproduces(P, d, r, p.eps);
    }
    uint64_t B = __ballot(inl);
    uint64_t m = (B >> (w * N)) & segmask;
    bool ext = in && allowed(s, tt) && __popcll(m) >= need_of(p, in ? sm.nv[tt] : 0);
    uint64_t E = __ballot(j == 0 && ext);
    int f = 0;
#pragma unroll
    for (int q = 0; q < TPW; q++)
      if (((E >> (q * N)) & 1ull) && f == q) f = q + 1;
    added += f;
    t += f;
    if (f < TPW) break;
  }
  return added;
}

// Next tile >= t in the start bitmask, or -1.
__device__ __forceinline__ int next_start(const uint64_t *acc, int t, int TC) {
  const int nw = (TC + 63) >> 6;
  int w = t >> 6;
  if (w >= nw) return -1;
  uint64_t bits = acc[w] & (~0ull << (t & 63));
  while (!bits) {
    if (++w >= nw) return -1;
    bits = acc[w];
  }
  return (w << 6) + __ffsll((long long)bits) - 1;
}

// The chain (one wavefront, lane-uniform control): runs from the start
// bitmask and the reaches.  Writes rs/rl and runof (run index per tile;
// -1 elsewhere, set beforehand); returns the number of runs.
template <int TH, int TW, class Allowed, class PlaneOf>
__device__ int chain_runs(StripSmem<TH, TW> &sm, const EncParams &p, int TC, Allowed allowed, PlaneOf plane_of) {
  const int lane = threadIdx.x & 63;
  int nr = 0, t = 0;
  for (;;) {
    int s = next_start(sm.acc, t, TC);
    if (s < 0) break;
    int len = 1 + sm.reach[s];
    if (len == 1 + kReach && s + len < TC) len += extend_beyond<TH, TW>(sm, p, plane_of(s), s, s + len, TC, allowed);
    for (int q = lane; q < len; q += 64) sm.runof[s + q] = nr;
    if (lane == 0) {
      sm.rs[nr] = s;
      sm.rl[nr] = len;
    }
    nr++;
    t = s + len;
  }
  return nr;
}

// RUN-stream bytes of the pass's runs, one thread per run: varint of the
// gap to the previous run's end, varint of the length, then the run's own
// bytes (emit), and the count of runs of the row.
template <int TH, int TW, class EmitRun>
__device__ void run_bytes(StripSmem<TH, TW> &sm, int nr, EmitRun emit) {
  for (int q = threadIdx.x; q < nr; q += kBlock) {
    int prev_end = q ? sm.rs[q - 1] + sm.rl[q - 1] : 0;
    varint_bytes(sm.hist, (uint32_t)(sm.rs[q] - prev_end));
    varint_bytes(sm.hist, (uint32_t)sm.rl[q]);
    emit(sm.rs[q]);
  }
  if (threadIdx.x == 0) varint_bytes(sm.hist, (uint32_t)nr);
}

// Spatial growth of one strip (Sec. III-C).  For predicted frames
// (`pred`), only tiles with elig != 0 take part; the others belong to
// temporal runs and break spatial runs.
template <int TH, int TW>
__device__ void grow_spatial(StripSmem<TH, TW> &sm, const EncParams &p, const FrameDev &f, int tr, bool pred) {
  const int TC = f.TC, tid = threadIdx.x;
  auto allowed = [&](int, int t) { return !pred || sm.elig[t] != 0; };
  // starts and reaches
  if (tid < 8) sm.acc[tid] = 0;
  __syncthreads();
  for (int tc = tid; tc < TC; tc += kBlock) {
    bool el = !pred || sm.elig[tc];
    if (el) sm.runof[tc] = -1;
    bool start = el && sm.stat[tc] == ST_ACCEPTED;
    int e = 0;
    if (start) {
      atomicOr((unsigned long long *)&sm.acc[tc >> 6], 1ull << (tc & 63));
      e = reach_of<TH, TW>(sm, p, unpack_plane(sm.plane[tc]), tc, TC, allowed);
    }
    sm.reach[tc] = (uint8_t)e;
  }
  __syncthreads();
  if (tid < 64) {
    auto plane_of = [&](int s) { return unpack_plane(sm.plane[s]); };
    int nr = chain_runs<TH, TW>(sm, p, TC, allowed, plane_of);
    if (tid == 0) {
      sm.misc[0] = nr;
      f.nruns[tr] = nr;
    }
  }
  __syncthreads();
  // stream bytes, masks, classes and the runs themselves
  const int nr = sm.misc[0];
  run_bytes<TH, TW>(sm, nr, [&](int s) {
    Plane P = unpack_plane(sm.plane[s]);
    hist_byte(sm.hist, S_RUN, (uint32_t)P.k);
    f32_bytes(sm.hist, P.a);
    f32_bytes(sm.hist, P.b);
    f32_bytes(sm.hist, P.c);
  });
  pc_run *runs = f.sruns + (int64_t)tr * TC;
  for (int q = tid; q < nr; q += kBlock) {
    Plane P = unpack_plane(sm.plane[sm.rs[q]]);
    runs[q] = pc_run{sm.rs[q], sm.rl[q], P.k, P.a, P.b, P.c};
  }
  for (int tc = tid; tc < TC; tc += kBlock) {
    if (pred && !sm.elig[tc]) continue;
    int ri = sm.runof[tc];
    if (ri >= 0) {
      int s = sm.rs[ri];
      uint64_t m = (s == tc) ? sm.omask[tc] : inliers_at<TH, TW>(sm, tc, TC, unpack_plane(sm.plane[s]), p.eps);
      sm.cls[tc] = CLS_SPATIAL;
      sm.fmask[tc] = m;
      sm.runof[tc] = tr * TC + ri;
    } else {
      sm.cls[tc] = sm.nv[tc] ? CLS_UNFIT : CLS_EMPTY;
      sm.fmask[tc] = 0;
      sm.runof[tc] = -1;
    }
  }
}

// Temporal growth (Sec. III-D): a temporal run grows while the key run
// stays the same and (key normal, c' of the run start) reproduces the
// tile.  Tiles not covered become eligible for the spatial pass.
template <int TH, int TW>
__device__ void grow_temporal(StripSmem<TH, TW> &sm, const EncParams &p, const FrameDev &f, int tr) {
  const int TC = f.TC, T = f.T, tid = threadIdx.x;
  auto allowed = [&](int s, int t) { return sm.krun[t] == sm.krun[s]; };
  if (tid < 8) sm.acc[tid] = 0;
  __syncthreads();
  for (int tc = tid; tc < TC; tc += kBlock) {
    sm.runof[tc] = -1;
    bool start = sm.tstat[tc] == 2;
    int e = 0;
    if (start) {
      atomicOr((unsigned long long *)&sm.acc[tc >> 6], 1ull << (tc & 63));
      e = reach_of<TH, TW>(sm, p, unpack_plane(sm.tplane[tc]), tc, TC, allowed);
    }
    sm.reach[tc] = (uint8_t)e;
  }
  __syncthreads();
  if (tid < 64) {
    auto plane_of = [&](int s) { return unpack_plane(sm.tplane[s]); };
    int nr = chain_runs<TH, TW>(sm, p, TC, allowed, plane_of);
    if (tid == 0) {
      sm.misc[1] = nr;
      f.nruns[f.TR + tr] = nr;
    }
  }
  __syncthreads();
  const int nr = sm.misc[1];
  run_bytes<TH, TW>(sm, nr, [&](int s) { f32_bytes(sm.hist, sm.tplane[s].z); });
  pc_prun *runs = f.pruns + (int64_t)tr * TC;
  for (int q = tid; q < nr; q += kBlock) runs[q] = pc_prun{sm.rs[q], sm.rl[q], sm.krun[sm.rs[q]], sm.tplane[sm.rs[q]].z};
  for (int tc = tid; tc < TC; tc += kBlock) {
    int ri = sm.runof[tc];
    if (ri >= 0) {
      int s = sm.rs[ri];
      uint64_t m = (s == tc) ? sm.tmask[tc] : inliers_at<TH, TW>(sm, tc, TC, unpack_plane(sm.tplane[s]), p.eps);
      sm.cls[tc] = CLS_TEMPORAL;
      sm.fmask[tc] = m;
      sm.runof[tc] = T + tr * TC + ri;
      sm.elig[tc] = 0;
    } else {
      sm.elig[tc] = 1;
    }
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
__device__ void residuals_and_streams(StripSmem<TH, TW> &sm, const SensorDev &s,
                                      const EncParams &p, const FrameDev &f, int tr, int fits, int fp64) {
  constexpr int N = TH * TW, NP = StripSmem<TH, TW>::NP;
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

// Key frame, one tile-row strip (Sec. III-C).
template <int TH, int TW>
__device__ void key_strip(char *smem_raw, const StripSrc &src, const SensorDev &s, const EncParams &p,
                          const float *__restrict__ seed, const FrameDev &f, int tr) {
  StripSmem<TH, TW> sm;
  const int TC = f.TC;
  sm.carve(smem_raw, s.W, TC, false);
  strip_init<TH, TW>(sm, s, tr);
  load_source<TH, TW>(sm, src, s, tr);
  __syncthreads();
  int fits = 0, fp64 = 0;
  for (int tc = threadIdx.x; tc < TC; tc += kBlock) {
    TileRows<TH, TW> T = tile_at<TH, TW>(sm, tc, TC, true);
    sm.nv[tc] = (uint8_t)T.nV;
    FitResult R = own_fit(T, p, fits, fp64);
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
  grow_spatial<TH, TW>(sm, p, f, tr, false);
  if (threadIdx.x == 0) f.nruns[f.TR + tr] = 0;
  __syncthreads();
  residuals_and_streams<TH, TW>(sm, s, p, f, tr, fits, fp64);
}

// Predicted frame, one tile-row strip (Sec. III-D).
template <int TH, int TW>
__device__ void pred_strip(char *smem_raw, const FrameDev &key, const StripSrc &src, const SensorDev &s,
                           const EncParams &p, const FrameDev &f, int tr) {
  StripSmem<TH, TW> sm;
  const int TC = f.TC;
  sm.carve(smem_raw, s.W, TC, true);
  strip_init<TH, TW>(sm, s, tr);
  load_source<TH, TW>(sm, src, s, tr);
  __syncthreads();
  int fits = 0, fp64 = 0;
  // temporal fits against the key frame's run planes
  for (int tc = threadIdx.x; tc < TC; tc += kBlock) {
    const int t = tr * TC + tc;
    TileRows<TH, TW> T = tile_at<TH, TW>(sm, tc, TC, true);
    sm.nv[tc] = (uint8_t)T.nV;
    int kr = key.cls[t] == CLS_SPATIAL ? key.run_of[t] : -1;
    sm.krun[tc] = kr;
    FitResult R{Plane{0, 0.f, 0.f, 0.f}, 0ull, 0, 0};
    if (kr >= 0) {
      pc_run q = key.sruns[kr];
      R = temporal_fit(T, Plane{q.axis, q.a, q.b, q.c}, p);
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
  grow_temporal<TH, TW>(sm, p, f, tr);
  __syncthreads();
  // own fits of the tiles left over
  for (int tc = threadIdx.x; tc < TC; tc += kBlock) {
    FitResult R{Plane{0, 0.f, 0.f, 0.f}, 0ull, ST_EMPTY, 0};
    if (sm.elig[tc]) {
      TileRows<TH, TW> T = tile_at<TH, TW>(sm, tc, TC, true);
      R = own_fit(T, p, fits, fp64);
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
  grow_spatial<TH, TW>(sm, p, f, tr, true);
  __syncthreads();
  residuals_and_streams<TH, TW>(sm, s, p, f, tr, fits, fp64);
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

// Whole-frame totals and the Huffman size; one 256-thread block per frame.
__device__ void finish_frame(const FrameDev &f, int kind, const Mat12 &M, int hasM) {
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

}  // namespace pcc

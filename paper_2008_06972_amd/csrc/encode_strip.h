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
//  1. fits, one thread per tile: the iterative least-squares fit (predicted
//     frames: first the offset-only fit against the key run's plane).  The
//     iterations are synchronous across the work-group and the tiles still
//     iterating are compacted onto the first threads after each one, so a
//     wavefront does not idle on its tiles that converged early; FP64 fits
//     of near-degenerate tiles are likewise gathered onto a few threads;
//  2. growth: each tile whose fit is accepted measures, in parallel, how
//     many following tiles (up to kReach) its plane reproduces -- the
//     extension test of the horizontal growth -- and which start would
//     follow its run; one wavefront then walks the actual run starts in
//     order (runs that reach kReach continue with a wavefront-wide test of
//     the following tiles).  This is exactly the sequential growth, in
//     O(runs) steps.  Covered tiles then take their masks, and the runs'
//     stream bytes are counted, in parallel;
//  3. residuals: codes of the remaining pixels, placed in raster order by a
//     work-group prefix sum, and byte histograms of the four streams.
// A last block per frame sums the strip histograms and computes the optimal
// Huffman cost of each stream.
#pragma once
#include "fit.h"

namespace pcc {

// Thread index inside the strip encoders, opaque to the optimizer: the
// persistent kernels run the encoders in a loop over work items, and values
// derived from the thread index would otherwise be hoisted out of that loop
// and held in registers across the whole encoder.
__device__ __forceinline__ int strip_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

constexpr int kReach = 6;     // tiles a fit measures its reach over before the walk continues it
constexpr int kBinChunkPts = 4096;      // points per binning block (its chunk's capacity)
constexpr int kSegMax = 512;            // chunk offsets the loader gathers at a time (two ints each)
constexpr int kSegJoint = 8;            // chunk segments a loader wavefront reads together
constexpr size_t kSegBytes = 2 * sizeof(int) * kSegMax;

// ---------------------------------------------------------------- LDS layout
// Ranges are stored tile-major, N = th*tw per tile with no padding; the
// 16-byte units of a tile are XOR-swizzled by the tile index, so threads
// reading the same unit of consecutive tiles (one tile per thread) hit
// distinct LDS banks, with 32 or with 64 four-byte banks.
__host__ __device__ constexpr int tile_swizzle(int tc, int units) {
  return units == 4 ? ((tc >> 1) ^ (tc >> 2)) & 3 : (units == 8 ? (tc ^ (tc >> 3)) & 7 : tc & 15);
}

// LDS slot of element j (= row * tw + column) of tile tc.
__host__ __device__ constexpr int tile_elem(int tc, int j, int n) {
  return tc * n + ((((j >> 2) ^ tile_swizzle(tc, n >> 2))) << 2) + (j & 3);
}

template <int TH, int TW>
struct StripSmem {
  static constexpr int N = TH * TW;
  static constexpr int UNITS = N / 4;    // 16-byte units per tile
  float *r;          // [TC * N] ranges, tile-major, units swizzled (tile_elem)
  const float *gca, *gsa;   // [W] column tables (global memory; read through the caches)
  float *ce, *se;    // [TH] row tables of the strip
  float4 *plane;     // [TC] plane: a, b, c, axis (predicted frames: the temporal pass's, then the own fits')
  uint64_t *omask;   // [TC] pixels that plane reproduces
  uint64_t *fmask;   // [TC] final mask (covering plane)
  uint8_t *stat;     // [TC] fit status
  uint8_t *iters;    // [TC] fits done
  uint8_t *nv;       // [TC] valid pixels
  uint8_t *cls;      // [TC] final class
  uint8_t *elig;     // [TC] still to be encoded spatially (predicted frames)
  int32_t *runof;    // [TC] run index within the current pass, then the stream's run slot
  int16_t *rs, *rl;  // [TC] run starts and lengths of the current pass
  uint8_t *reach;    // [TC] tiles a run starting here covers after its start (<= kReach)
  int16_t *nx;       // [TC] start that follows a run starting here (-1: none)
  uint64_t *acc;     // [(TC + 63) / 64] tiles that may start a run (bit tc)
  int32_t *krun;     // [TC] key run slot, -1 if the key tile is not plane coded (predicted frames)
  uint32_t *scratch; // fits: cur (u64[TC]), two work lists and the FP64 list (i16[TC] each);
                     // residuals: counts per (row, tile) (u32[TH * TC]); load: chunk offsets
  uint32_t *hist;    // [4 * 256] 16-bit counts, two per word (byte v of a stream in half v & 1)
  int32_t *misc;     // [32] counters

  __device__ uint32_t *cnt() const { return scratch; }
  __device__ uint64_t *cur() const { return reinterpret_cast<uint64_t *>(scratch); }
  __device__ int16_t *list(int q, int TC) const { return reinterpret_cast<int16_t *>(cur() + TC) + q * TC; }
  // growth: the masks the run tests found (over cur) and the start whose
  // plane found each (after the three lists)
  __device__ uint64_t *mcache() const { return cur(); }
  __device__ int16_t *mstart(int TC) const { return list(3, TC); }

  // fits: cur and three lists; growth: the mask cache over cur, the
  // lists, the masks' start tiles after them; residuals: counts; the load
  // of binned points: the chunk offsets it gathers
  __host__ __device__ static size_t scratch_bytes(int TC) {
    size_t a = sizeof(uint32_t) * (size_t)TH * TC, b = sizeof(uint64_t) * (size_t)TC + 4 * sizeof(int16_t) * (size_t)TC;
    size_t m = a > b ? a : b;
    return m > kSegBytes ? m : kSegBytes;
  }
  __host__ __device__ static size_t bytes(int W, int TC, bool pred) {
    auto a16 = [](size_t n) { return (n + 15) & ~(size_t)15; };
    size_t b = 0;
    b += a16(sizeof(float) * (size_t)TC * N);
    b += 2 * a16(sizeof(float) * 16);
    b += a16(sizeof(float4) * TC) + 2 * a16(sizeof(uint64_t) * TC) + 6 * a16(TC) + a16(sizeof(int32_t) * TC) +
         3 * a16(sizeof(int16_t) * TC);
    b += a16(sizeof(uint64_t) * ((TC + 63) / 64));
    if (pred) b += a16(sizeof(int32_t) * TC);
    b += a16(scratch_bytes(TC));
    b += a16(sizeof(uint32_t) * 512) + a16(sizeof(int32_t) * 32);
    return b + 64;
  }

  __device__ void carve(char *base, int W, int TC, bool pred) {
    char *p = base;
    auto take = [&](size_t n) { char *q = p; p += (n + 15) & ~(size_t)15; return q; };
    r = (float *)take(sizeof(float) * (size_t)TC * N);
    ce = (float *)take(sizeof(float) * 16);
    se = (float *)take(sizeof(float) * 16);
    plane = (float4 *)take(sizeof(float4) * TC);
    omask = (uint64_t *)take(sizeof(uint64_t) * TC);
    fmask = (uint64_t *)take(sizeof(uint64_t) * TC);
    stat = (uint8_t *)take(TC);
    iters = (uint8_t *)take(TC);
    nv = (uint8_t *)take(TC);
    cls = (uint8_t *)take(TC);
    elig = (uint8_t *)take(TC);
    runof = (int32_t *)take(sizeof(int32_t) * TC);
    rs = (int16_t *)take(sizeof(int16_t) * TC);
    rl = (int16_t *)take(sizeof(int16_t) * TC);
    reach = (uint8_t *)take(TC);
    nx = (int16_t *)take(sizeof(int16_t) * TC);
    acc = (uint64_t *)take(sizeof(uint64_t) * ((TC + 63) / 64));
    krun = pred ? (int32_t *)take(sizeof(int32_t) * TC) : nullptr;
    scratch = (uint32_t *)take(scratch_bytes(TC));
    hist = (uint32_t *)take(sizeof(uint32_t) * 512);
    misc = (int32_t *)take(sizeof(int32_t) * 32);
  }
};

// LDS bytes of a strip encoder's work-group (0 for shapes not compiled).
__host__ __device__ inline size_t strip_lds_bytes(int th, int tw, int W, bool pred) {
  if (th == 4 && tw == 4) return StripSmem<4, 4>::bytes(W, W / 4, pred);
  if (th == 4 && tw == 8) return StripSmem<4, 8>::bytes(W, W / 8, pred);
  if (th == 4 && tw == 16) return StripSmem<4, 16>::bytes(W, W / 16, pred);
  if (th == 8 && tw == 8) return StripSmem<8, 8>::bytes(W, W / 8, pred);
  return 0;
}

// LDS slot of pixel (row i of the strip, column u) in StripSmem::r.
__host__ __device__ inline int strip_slot(int i, int u, int th, int tw_log2) {
  const int tw = 1 << tw_log2;
  return tile_elem(u >> tw_log2, i * tw + (u & (tw - 1)), th * tw);
}

// misc[] slots
constexpr int M_SRUNS = 0, M_PRUNS = 1, M_SEEDED = 2, M_FALLBACK = 3, M_LIST = 8, M_F64 = 10, M_NEXT = 12;

__device__ __forceinline__ float4 pack_plane(const Plane &P) { return make_float4(P.a, P.b, P.c, (float)P.k); }
__device__ __forceinline__ Plane unpack_plane(float4 v) { return Plane{(int)v.w, v.x, v.y, v.z}; }

// Bytes of the serialized streams go into the LDS histograms.
__device__ __forceinline__ void hist_byte(uint32_t *hist, int stream, uint32_t v) {
  atomicAdd(&hist[stream * 128 + ((v & 255u) >> 1)], 1u << ((v & 1u) << 4));
}
// The two RES-stream bytes of a residual code given its row predecessor:
// zigzag-mapped difference mod 2^16, little-endian.  The high byte is zero
// for nearly every code; those counts are summed over the active lanes of
// the wavefront and added once, instead of 64 atomics on one LDS word.
__device__ __forceinline__ void hist_delta(uint32_t *hist, uint32_t code, uint32_t prev) {
  const uint32_t d = (code - prev) & 0xFFFFu;
  const uint32_t z = ((d << 1) ^ ((d & 0x8000u) ? 0xFFFFu : 0u)) & 0xFFFFu;
  hist_byte(hist, S_RES, z & 255u);
  const uint32_t hi = z >> 8;
  const uint64_t zero = __ballot(hi == 0u);
  if (hi != 0u) {
    hist_byte(hist, S_RES, hi);
  } else if ((int)(__lane_id()) == __ffsll((long long)zero) - 1) {
    atomicAdd(&hist[S_RES * 128], (uint32_t)__popcll(zero));   // symbol 0: low half of the first word
  }
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
__device__ __forceinline__ void strip_init(StripSmem<TH, TW> &sm, const SensorDev &s, int tr) {
  const int tid = strip_tid();
  for (int q = tid; q < 512; q += kBlock) sm.hist[q] = 0;
  if (tid < 32) sm.misc[tid] = 0;
  sm.gca = s.ca;
  sm.gsa = s.sa;
  if (tid < TH) {
    sm.ce[tid] = s.ce[tr * TH + tid];
    sm.se[tid] = s.se[tr * TH + tid];
  }
}

// Coalesced float4 loads of the strip's rows into LDS, tile-major.
template <int TH, int TW>
__device__ __forceinline__ void load_strip(StripSmem<TH, TW> &sm, const float *__restrict__ range, const SensorDev &s,
                                           int tr) {
  constexpr int N = StripSmem<TH, TW>::N;
  const int W = s.W, nq = W / 4;
  const float4 *src = reinterpret_cast<const float4 *>(range + (int64_t)tr * TH * W);
  for (int e = strip_tid(); e < TH * nq; e += kBlock) {
    int i = e / nq, u = (e % nq) * 4;
    float4 q = src[e];
    // empty pixels are 0 (+inf is taken as empty too)
    q.x = q.x < INFINITY ? q.x : 0.0f;
    q.y = q.y < INFINITY ? q.y : 0.0f;
    q.z = q.z < INFINITY ? q.z : 0.0f;
    q.w = q.w < INFINITY ? q.w : 0.0f;
    int tc = u / TW, k = u % TW;
    *reinterpret_cast<float4 *>(sm.r + tile_elem(tc, i * TW + k, N)) = q;
  }
}

// Where a strip's ranges come from: a range image (0 = empty), or the
// batched binning pass's chunks, one per binning block of the frame, each
// holding its block's kept points as (LDS slot, range bits) entries grouped
// by strip (slots as strip_slot gives them), resolved here with LDS
// atomicMin: the nearest point wins (Sec. III-D).  range_out, if set,
// receives the strip's range image.
struct StripSrc {
  const float *range;
  const uint2 *chunks;     // frame's chunks, block b's at b * kBinChunkPts
  const int *blkoff;       // [nblk][TR + 1] first entry of each strip in each chunk
  int nblk, TR;
  float *range_out;
};

template <int TH, int TW>
__device__ __forceinline__ void load_source(StripSmem<TH, TW> &sm, const StripSrc &src, const SensorDev &s, int tr) {
  constexpr int N = StripSmem<TH, TW>::N, NW = kBlock / 64;
  const int W = s.W, TC = W / TW, tid = strip_tid();
  if (!src.chunks) {
    load_strip<TH, TW>(sm, src.range, s, tr);
  } else {
    uint32_t *ri = reinterpret_cast<uint32_t *>(sm.r);
    for (int e = tid; e < TC * N; e += kBlock) ri[e] = 0x7f800000u;   // +inf: empty
    const uint32_t lim = (uint32_t)(TC * N);
    const int lane = tid & 63, wv = tid >> 6, stride = src.TR + 1;
    int *sb = reinterpret_cast<int *>(sm.scratch), *sl = sb + kSegMax;     // segment start and length per chunk
    const auto *ch = (const __attribute__((address_space(1))) uint64_t *)src.chunks;
    for (int c0 = 0; c0 < src.nblk; c0 += kSegMax) {
      const int nb = min(kSegMax, src.nblk - c0);
      for (int b = tid; b < nb; b += kBlock) {
        const int *o = src.blkoff + (int64_t)(c0 + b) * stride + tr;
        const int a = o[0];
        sb[b] = a;
        sl[b] = o[1] - a;
      }
      __syncthreads();
      // a wavefront takes kSegJoint chunks' segments at a time and reads
      // them jointly, 128 entries of each per round (2 kSegJoint loads per
      // lane in flight), as many rounds as the longest of them needs
      for (int b0 = wv; b0 < nb; b0 += kSegJoint * NW) {
        int len[kSegJoint];
        int64_t at[kSegJoint];
        int mx = 0;
#pragma unroll
        for (int u = 0; u < kSegJoint; u++) {
          const int b = b0 + u * NW;
          len[u] = b < nb ? sl[b] : 0;
          at[u] = (int64_t)(c0 + b) * kBinChunkPts + (b < nb ? sb[b] : 0);
          mx = max(mx, len[u]);
        }
        for (int q0 = lane; q0 < mx; q0 += 128) {
          uint64_t en[2 * kSegJoint];
#pragma unroll
          for (int u = 0; u < kSegJoint; u++) {
            en[2 * u] = q0 < len[u] ? (uint64_t)ch[at[u] + q0] : ~0ull;
            en[2 * u + 1] = q0 + 64 < len[u] ? (uint64_t)ch[at[u] + q0 + 64] : ~0ull;
          }
#pragma unroll
          for (int u = 0; u < 2 * kSegJoint; u++)
            if ((uint32_t)en[u] < lim) atomicMin(&ri[(uint32_t)en[u]], (uint32_t)(en[u] >> 32));
        }
      }
      __syncthreads();     // every segment read before the next offsets overwrite them
    }
    for (int e = tid; e < TC * N; e += kBlock)
      if (ri[e] == 0x7f800000u) ri[e] = 0u;
  }
  if (src.range_out) {
    __syncthreads();
    float *dst = src.range_out + (int64_t)tr * TH * W;
    for (int e = tid; e < TH * W; e += kBlock) {
      int i = e / W, u = e - i * W;
      dst[e] = sm.r[tile_elem(u / TW, i * TW + (u % TW), N)];
    }
  }
}

// A tile of the strip as seen by one thread: ranges in LDS, the tile's
// column tables loaded into registers.
template <int TH, int TW>
__device__ __forceinline__ TileRows<TH, TW> tile_at(const StripSmem<TH, TW> &sm, int tc) {
  TileRows<TH, TW> T;
  T.rp = sm.r + tc * StripSmem<TH, TW>::N;
  T.sw = tile_swizzle(tc, StripSmem<TH, TW>::UNITS);
  T.i0 = 0;
  T.i1 = TH;
  T.ce = sm.ce;
  T.se = sm.se;
  typedef float v4f __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(1))) v4f gv4f;
  gv4f *ca4 = (gv4f *)(sm.gca + tc * TW), *sa4 = (gv4f *)(sm.gsa + tc * TW);
#pragma unroll
  for (int k4 = 0; k4 < TW / 4; k4++) {
    const v4f c = ca4[k4], d = sa4[k4];
    T.ca[4 * k4] = c.x; T.ca[4 * k4 + 1] = c.y; T.ca[4 * k4 + 2] = c.z; T.ca[4 * k4 + 3] = c.w;
    T.sa[4 * k4] = d.x; T.sa[4 * k4 + 1] = d.y; T.sa[4 * k4 + 2] = d.z; T.sa[4 * k4 + 3] = d.w;
  }
  return T;
}

// Valid pixels of tile tc (range > 0), bit j = i * TW + k.
template <int TH, int TW>
__device__ __forceinline__ uint64_t valid_bits(const StripSmem<TH, TW> &sm, int tc) {
  constexpr int N = StripSmem<TH, TW>::N;
  uint32_t lo = 0, hi = 0;
  const float4 *q = reinterpret_cast<const float4 *>(sm.r + tc * N);
  const int sw = tile_swizzle(tc, N / 4);
#pragma unroll
  for (int j4 = 0; j4 < TH * TW / 4; j4++) {
    float4 v = q[j4 ^ sw];
    uint32_t b = (uint32_t)(v.x > 0.0f) | ((uint32_t)(v.y > 0.0f) << 1) | ((uint32_t)(v.z > 0.0f) << 2) |
                 ((uint32_t)(v.w > 0.0f) << 3);
    const int j = 4 * j4;
    if (j < 32) lo |= b << (j & 31); else hi |= b << (j & 31);
  }
  return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------------------ phase 1: fits
// Work-group-synchronous iterations over a compacted list of the tiles
// still iterating.  Lists live in the scratch area: lists 0 and 1
// alternate, list 2 gathers the tiles whose FP32 fit needs FP64.
// misc[M_LIST + q] counts list q (q < 2), misc[M_F64] list 2.
template <int TH, int TW>
__device__ __forceinline__ void list_push(StripSmem<TH, TW> &sm, int q, int TC, int tc) {
  int at = atomicAdd(&sm.misc[q == 2 ? M_F64 : M_LIST + q], 1);
  sm.list(q, TC)[at] = (int16_t)tc;
}

// The fits of one iteration for the tiles on list q (n of them, every thread
// having read n after the last barrier): (a) FP32 fits, the near-degenerate
// ones gathered on the FP64 list; (b) FP64 fits of those, on_degenerate(tc)
// for a degenerate scatter.  Each plane goes to sm.plane and, with the
// pixels it reproduces, to keep(tc, P, S2).  LANES neighbouring lanes share
// a tile, TH / LANES of its rows each (short lists, where one thread per
// tile would leave most of the work-group idle and the iteration bound by
// one thread's latency).  Ends after a barrier with list q's and the FP64
// list's counters cleared.
template <int TH, int TW, int LANES, class OnDegenerate, class Keep>
__device__ __forceinline__ void fit_pass(StripSmem<TH, TW> &sm, const EncParams &p, int q, int n, int TC, bool refit, int &fits,
                         int &fp64, OnDegenerate on_degenerate, Keep keep) {
  typedef typename LaneGroup<LANES>::type Red;
  const int tid = strip_tid(), sub = tid & (LANES - 1);
  const int16_t *L = sm.list(q, TC);
  const uint64_t *cur = sm.cur();
  for (int e = tid / LANES; e < n; e += kBlock / LANES) {
    const int tc = L[e];
    TileRows<TH, TW> T = tile_at<TH, TW>(sm, tc);
    Plane P{0, 0.f, 0.f, 0.f};
    T.i0 = sub * (TH / LANES);
    T.i1 = T.i0 + TH / LANES;
    const bool ok = refit ? refit_plane_f32(T, cur[tc], unpack_plane(sm.plane[tc]), P, Red{})
                          : fit_plane_f32(T, cur[tc], P, Red{});
    const uint64_t S2 = ok ? inliers(T, P, p.eps, Red{}) : 0ull;
    if (sub != 0) continue;
    fits++;
    if (ok) {
      sm.plane[tc] = pack_plane(P);
      keep(tc, P, S2);
    } else {
      list_push<TH, TW>(sm, 2, TC, tc);
    }
  }
  __syncthreads();
  const int nf = sm.misc[M_F64];
  if (tid == 0) sm.misc[M_LIST + q] = 0;      // every thread has read n before (a)
  if (nf == 0) return;
  for (int e = tid; e < nf; e += kBlock) {
    const int tc = sm.list(2, TC)[e];
    TileRows<TH, TW> T = tile_at<TH, TW>(sm, tc);
    Plane P{0, 0.f, 0.f, 0.f};
    fp64++;
    if (fit_plane_f64(T, cur[tc], P)) {
      sm.plane[tc] = pack_plane(P);
      keep(tc, P, inliers(T, P, p.eps));
    } else {
      on_degenerate(tc);
    }
  }
  __syncthreads();
  if (tid == 0) sm.misc[M_F64] = 0;            // every thread has read nf before (b)
}

// Own least-squares fits (Sec. III-C) of the tiles with take(tc): fit,
// keep the pixels the plane reproduces, refit on them, up to max_iter fits,
// converged when the kept set stops changing; accepted when at least
// need(n) pixels are kept.  Results in plane/omask/stat/iters.
template <int TH, int TW, class Take>
__device__ __forceinline__ void own_fits(StripSmem<TH, TW> &sm, const EncParams &p, int TC, Take take, int &fits, int &fp64) {
  const int tid = strip_tid();
  uint64_t *cur = sm.cur();
  for (int tc = tid; tc < TC; tc += kBlock) {
    if (!take(tc)) continue;
    const int n = sm.nv[tc];
    sm.plane[tc] = make_float4(0.f, 0.f, 0.f, 0.f);
    sm.omask[tc] = 0;
    sm.iters[tc] = 0;
    sm.stat[tc] = (uint8_t)(n == 0 ? ST_EMPTY : ST_FEW);
    if (n >= p.min_pts) {
      cur[tc] = valid_bits<TH, TW>(sm, tc);
      list_push<TH, TW>(sm, 0, TC, tc);
    }
  }
  __syncthreads();
  int n = sm.misc[M_LIST];
  for (int it = 1; it <= p.max_iter && n > 0; it++) {
    const int q = (it - 1) & 1;
    auto degenerate = [&](int tc) {
      sm.iters[tc] = (uint8_t)it;
      sm.stat[tc] = ST_DEGENERATE;
      sm.omask[tc] = 0;
    };
    auto kept = [&](int tc, const Plane &P, uint64_t S2) {
          // kept pixels, convergence
          sm.iters[tc] = (uint8_t)it;
          const uint64_t S = cur[tc];
          if (S2 != S && __popcll(S2) < p.min_pts) {
            sm.stat[tc] = ST_FAILED;
            sm.omask[tc] = 0;
            return;
          }
          sm.omask[tc] = S2;
          if (S2 != S && it < p.max_iter) {
            cur[tc] = S2;
            list_push<TH, TW>(sm, q ^ 1, TC, tc);
          } else {
            sm.stat[tc] = __popcll(S2) >= need_of(p, sm.nv[tc]) ? ST_ACCEPTED : ST_REJECTED;
          }
    };
    // from the second fit on, the previous fit's normal gives the frame
    const bool refit = it > 1;
    if (p.lanes >= 4 && n <= kBlock / 4) fit_pass<TH, TW, 4>(sm, p, q, n, TC, refit, fits, fp64, degenerate, kept);
    else if (p.lanes >= 2 && n <= kBlock / 2) fit_pass<TH, TW, 2>(sm, p, q, n, TC, refit, fits, fp64, degenerate, kept);
    else fit_pass<TH, TW, 1>(sm, p, q, n, TC, refit, fits, fp64, degenerate, kept);
    n = sm.misc[M_LIST + (q ^ 1)];
  }
  __syncthreads();
  if (tid == 0) {
    sm.misc[M_LIST] = 0;
    sm.misc[M_LIST + 1] = 0;
  }
  __syncthreads();
}

// Offset of a seed plane (normal held) through all of the tile's points:
// the FP64 mean of p_k + a p_k1 + b p_k2 over the valid pixels with p = r d,
// in pixel order, rounded once (the kept set of the refit depends on it).
template <class Tile>
__device__ __forceinline__ float seed_offset(const Tile &T, const Plane &Q) {
  const bool isx = Q.k == 0, isz = Q.k == 2;
  double sum = 0.0;
  int n = 0;
  T.each([&](int, float r, const Dir &d) {
    const double px = (double)r * (double)d.x, py = (double)r * (double)d.y, pz = (double)r * (double)d.z;
    const double pk = isz ? pz : (isx ? px : py), pk1 = isx ? py : px, pk2 = isz ? py : pz;
    const double v = pk + (double)Q.a * pk1 + (double)Q.b * pk2;
    sum += r > 0.0f ? v : 0.0;
    n += r > 0.0f;
  });
  return (float)(sum / (double)n);
}

// Seeded fits (learned plane seeding) of a key-frame strip: a tile whose
// seed logit is positive takes the seed normal's stored form (FP32
// coefficients), its offset along the tile's points, the points that plane
// reproduces, one least-squares refit on them, and the own fit's acceptance
// test.  Accepted tiles get their plane, mask, status ACCEPTED and one
// iteration; seed state in sm.elig (key frames do not use it otherwise):
// 0 no seed, 1 accepted, 2 fell back to the plain fit.
template <int TH, int TW>
__device__ __forceinline__ void seeded_fits(StripSmem<TH, TW> &sm, const EncParams &p, int TC, const float4 *__restrict__ seed,
                            int &fits, int &fp64) {
  const int tid = strip_tid();
  uint64_t *cur = sm.cur();
  for (int tc = tid; tc < TC; tc += kBlock) {
    uint8_t state = 0;
    const float4 s4 = seed[tc];
    if (s4.w > 0.0f && sm.nv[tc] >= p.min_pts && isfinite(s4.x) && isfinite(s4.y) && isfinite(s4.z)) {
      int k = 0;
      float m = fabsf(s4.x);
      if (fabsf(s4.y) > m) { k = 1; m = fabsf(s4.y); }
      if (fabsf(s4.z) > m) { k = 2; m = fabsf(s4.z); }
      if (m > 0.0f) {
        // stored form: dominant component k, then the other two in order
        const float nk = k == 0 ? s4.x : (k == 1 ? s4.y : s4.z);
        const float n1 = k == 0 ? s4.y : s4.x, n2 = k == 2 ? s4.y : s4.z;
        Plane Q{k, n1 / nk, n2 / nk, 0.0f};
        TileRows<TH, TW> T = tile_at<TH, TW>(sm, tc);
        Q.c = seed_offset(T, Q);
        const uint64_t S1 = inliers(T, Q, p.eps);
        state = 2;
        if (__popcll(S1) >= p.min_pts) {
          cur[tc] = S1;
          sm.plane[tc] = pack_plane(Q);     // the seed's normal frames the refit
          list_push<TH, TW>(sm, 0, TC, tc);
          state = 3;
        }
      }
    }
    sm.elig[tc] = state;
  }
  __syncthreads();
  const int n = sm.misc[M_LIST];
  if (n > 0)
    fit_pass<TH, TW, 1>(
        sm, p, 0, n, TC, true, fits, fp64, [&](int tc) { sm.elig[tc] = 2; },
        [&](int tc, const Plane &P, uint64_t S2) {
          if (__popcll(S2) >= need_of(p, sm.nv[tc])) {
            sm.omask[tc] = S2;
            sm.stat[tc] = ST_ACCEPTED;
            sm.iters[tc] = 1;
            sm.elig[tc] = 1;
          } else {
            sm.elig[tc] = 2;
          }
        });
  __syncthreads();
  int ns = 0, nb = 0;
  for (int tc = tid; tc < TC; tc += kBlock) {
    ns += sm.elig[tc] == 1;
    nb += sm.elig[tc] == 2;
  }
  if (ns) atomicAdd(&sm.misc[M_SEEDED], ns);
  if (nb) atomicAdd(&sm.misc[M_FALLBACK], nb);
  __syncthreads();
}

// One temporal-fit iteration over list q (n tiles), LANES lanes per tile
// as in fit_pass: the offset through the kept pixels, the pixels it
// reproduces, convergence.
template <int TH, int TW, int LANES>
__device__ __forceinline__ void temporal_pass(StripSmem<TH, TW> &sm, const EncParams &p, int q, int n, int TC, int it) {
  typedef typename LaneGroup<LANES>::type Red;
  const int tid = strip_tid(), sub = tid & (LANES - 1);
  const int16_t *L = sm.list(q, TC);
  uint64_t *cur = sm.cur();
  float *tsum = reinterpret_cast<float *>(sm.fmask);     // final masks are not in use yet
  for (int e = tid / LANES; e < n; e += kBlock / LANES) {
    const int tc = L[e];
    TileRows<TH, TW> T = tile_at<TH, TW>(sm, tc);
    T.i0 = sub * (TH / LANES);
    T.i1 = T.i0 + TH / LANES;
    Plane P = unpack_plane(sm.plane[tc]);
    const uint64_t S = cur[tc];
    // the first iteration sums over the valid pixels; later ones take the
    // sum the previous test accumulated over the pixels it kept
    P.c = it == 1 ? temporal_offset(T, P, S, Red{}) : tsum[tc] / (float)__popcll(S);
    float next_sum;
    const uint64_t S2 = inliers_offset_sum(T, P, p.eps, next_sum, Red{});
    if (sub != 0) continue;
    sm.iters[tc] = (uint8_t)it;
    sm.plane[tc] = pack_plane(P);
    if (S2 != S && __popcll(S2) < p.min_pts) {     // failed: stat stays 1
      sm.omask[tc] = 0;
      continue;
    }
    sm.omask[tc] = S2;
    if (S2 != S && it < p.max_iter) {
      cur[tc] = S2;
      tsum[tc] = next_sum;
      list_push<TH, TW>(sm, q ^ 1, TC, tc);
    } else {
      sm.stat[tc] = __popcll(S2) >= need_of(p, sm.nv[tc]) ? 2 : 1;
    }
  }
}

// Temporal fits (Sec. III-D) of the tiles whose key tile is plane coded:
// the key run's normal (k, a, b) is held and only the offset varies, with
// the same iteration, kept-pixel test and acceptance as the own fits.
// stat: 2 accepted, 1 not, 0 no key plane.  Results in plane/omask/stat/iters.
template <int TH, int TW>
__device__ __forceinline__ void temporal_fits(StripSmem<TH, TW> &sm, const FrameDev &key, const EncParams &p, int tr, int TC) {
  const int tid = strip_tid();
  uint64_t *cur = sm.cur();
  for (int tc = tid; tc < TC; tc += kBlock) {
    const int t = tr * TC + tc;
    const int kr = key.cls[t] == CLS_SPATIAL ? key.run_of[t] : -1;
    sm.krun[tc] = kr;
    float4 Q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (kr >= 0) {
      pc_run q = key.sruns[kr];
      Q = pack_plane(Plane{q.axis, q.a, q.b, q.c});
    }
    sm.plane[tc] = Q;
    sm.omask[tc] = 0;
    sm.iters[tc] = 0;
    sm.stat[tc] = kr >= 0 ? 1 : 0;
    if (kr >= 0 && sm.nv[tc] >= p.min_pts) {
      cur[tc] = valid_bits<TH, TW>(sm, tc);
      list_push<TH, TW>(sm, 0, TC, tc);
    }
  }
  __syncthreads();
  int n = sm.misc[M_LIST];
  for (int it = 1; it <= p.max_iter && n > 0; it++) {
    const int q = (it - 1) & 1;
    if (p.lanes >= 4 && n <= kBlock / 4) temporal_pass<TH, TW, 4>(sm, p, q, n, TC, it);
    else if (p.lanes >= 2 && n <= kBlock / 2) temporal_pass<TH, TW, 2>(sm, p, q, n, TC, it);
    else temporal_pass<TH, TW, 1>(sm, p, q, n, TC, it);
    __syncthreads();
    n = sm.misc[M_LIST + (q ^ 1)];
    if (tid == 0) sm.misc[M_LIST + q] = 0;    // every thread read its count before the pass
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) {
    sm.misc[M_LIST] = 0;
    sm.misc[M_LIST + 1] = 0;
  }
  __syncthreads();
}

// --------------------------------------------------------- phase 2: growth
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

// Pixels of tile tc that plane P reproduces.
template <int TH, int TW>
__device__ __forceinline__ uint64_t inliers_at(const StripSmem<TH, TW> &sm, int tc, const Plane &P, float eps) {
  return inliers(tile_at<TH, TW>(sm, tc), P, eps);
}

// Continue a run beyond its measured reach: the wavefront tests windows of
// 64 / (TH * TW) tiles from tile t on (lane = pixel); returns how many more
// tiles join.
template <int TH, int TW, class Allowed>
__device__ __forceinline__ int extend_beyond(StripSmem<TH, TW> &sm, const EncParams &p, const Plane &P, int s, int t, int TC,
                             Allowed allowed) {
  constexpr int N = TH * TW, TPW = 64 / N;
  const int lane = strip_tid() & 63, w = lane / N, j = lane % N, i = j / TW, k = j % TW;
  const uint64_t segmask = (N == 64) ? ~0ull : ((1ull << N) - 1ull);
  int added = 0;
  while (t < TC) {
    const int tt = t + w;
    const bool in = tt < TC;
    const float r = in ? sm.r[tile_elem(tt, j, N)] : 0.0f;
    bool inl = false;
    if (r > 0.0f) inl = reproduces(P, dir_of(sm.ce[i], sm.se[i], sm.gca[tt * TW + k], sm.gsa[tt * TW + k]), r, p.eps);
    const uint64_t B = __ballot(inl);
    const uint64_t m = (B >> (w * N)) & segmask;
    const bool ext = in && allowed(s, tt) && __popcll(m) >= need_of(p, in ? sm.nv[tt] : 0);
    const uint64_t E = __ballot(j == 0 && ext);
    int f = 0;
#pragma unroll
    for (int q = 0; q < TPW; q++)
      if (((E >> (q * N)) & 1ull) && f == q) f = q + 1;
    if (j == 0 && w < f) {          // tiles that join the run: their masks
      sm.mcache()[tt] = m;
      sm.mstart(TC)[tt] = (int16_t)s;
    }
    added += f;
    t += f;
    if (f < TPW) break;
  }
  return added;
}

// One level d of the reach: does the plane of start s (list q, n starts)
// reproduce tile s + d?  LANES lanes per test as in fit_pass.
template <int TH, int TW, int LANES, class Allowed, class PlaneOf>
__device__ __forceinline__ void reach_pass(StripSmem<TH, TW> &sm, const EncParams &p, int q, int n, int TC, int d,
                                           Allowed allowed, PlaneOf plane_of) {
  typedef typename LaneGroup<LANES>::type Red;
  const int tid = strip_tid(), sub = tid & (LANES - 1);
  const int16_t *L = sm.list(q, TC);
  for (int e = tid / LANES; e < n; e += kBlock / LANES) {
    const int s = L[e], t = s + d;
    if (t >= TC || !allowed(s, t)) continue;
    TileRows<TH, TW> T = tile_at<TH, TW>(sm, t);
    T.i0 = sub * (TH / LANES);
    T.i1 = T.i0 + TH / LANES;
    const uint64_t m = inliers(T, plane_of(s), p.eps, Red{});
    if (sub != 0 || __popcll(m) < need_of(p, sm.nv[t])) continue;
    sm.reach[s] = (uint8_t)d;
    // levels run in order of d, so the farthest start that reaches t keeps
    // its mask here: the run's own start for a tile of a run's first kReach
    sm.mcache()[t] = m;
    sm.mstart(TC)[t] = (int16_t)s;
    if (d < kReach) list_push<TH, TW>(sm, q ^ 1, TC, s);
  }
}

// Runs of one pass.  Every tile that may start a run (start(tc)) measures
// its reach -- level by level over a compacted list of the starts still
// extending, so no thread idles on a neighbour's longer run -- and notes
// the start that would follow its run.  One wavefront then walks the actual
// starts in order (a run starts at the first start tile at or after the
// previous run's end), reading each start's note from a register window of
// 64 tiles, and continues runs that reached kReach.  Then every covered
// tile takes its mask: its own for a run's first tile, else the pixels the
// run plane reproduces.  Writes rs/rl, runof (run index, -1 outside runs,
// for tiles with member(tc)) and fmask; returns the number of runs.
template <int TH, int TW, class Member, class Start, class Allowed, class PlaneOf, class MaskOf>
__device__ __forceinline__ int grow_runs(StripSmem<TH, TW> &sm, const EncParams &p, int TC, Member member, Start start,
                         Allowed allowed, PlaneOf plane_of, MaskOf own_mask, int *nr_out) {
  const int tid = strip_tid(), nw = (TC + 63) >> 6;
  for (int w = tid >> 6; w < nw; w += kBlock / 64) {
    const int tc = w * 64 + (tid & 63);
    const bool st = tc < TC && start(tc);
    const uint64_t b = __ballot(st);
    if ((tid & 63) == 0) sm.acc[w] = b;
    if (st) {
      sm.reach[tc] = 0;
      list_push<TH, TW>(sm, 0, TC, tc);
    }
  }
  for (int tc = tid; tc < TC; tc += kBlock) {
    if (member(tc)) sm.runof[tc] = -1;
    sm.mstart(TC)[tc] = -1;
  }
  __syncthreads();
  // reach, level by level
  int n = sm.misc[M_LIST];
  for (int d = 1; d <= kReach && n > 0; d++) {
    const int q = (d - 1) & 1;
    if (p.lanes >= 4 && n <= kBlock / 4) reach_pass<TH, TW, 4>(sm, p, q, n, TC, d, allowed, plane_of);
    else if (p.lanes >= 2 && n <= kBlock / 2) reach_pass<TH, TW, 2>(sm, p, q, n, TC, d, allowed, plane_of);
    else reach_pass<TH, TW, 1>(sm, p, q, n, TC, d, allowed, plane_of);
    __syncthreads();
    n = sm.misc[M_LIST + (q ^ 1)];
    if (tid == 0) sm.misc[M_LIST + q] = 0;    // every thread read its count before the pass
    __syncthreads();
  }
  if (tid == 0) {
    sm.misc[M_LIST] = 0;
    sm.misc[M_LIST + 1] = 0;
  }
  for (int tc = tid; tc < TC; tc += kBlock)
    if (start(tc)) sm.nx[tc] = (int16_t)next_start(sm.acc, tc + 1 + sm.reach[tc], TC);
  __syncthreads();
  // The chain of run starts, by pointer jumping: from the first start,
  // every marked start marks the start 2^k links further on (level k), so
  // about log2(runs) levels mark the whole chain; the marked starts in tile
  // order are the runs.  A start whose reach hit kReach has an unknown
  // successor (its run may go on), so the chain is cut there: that run is
  // continued by extend_beyond and the marking restarts after it.
  {
    int16_t *ja = sm.list(0, TC), *jb = ja + TC;     // the lists are free now; the mask cache is kept
    uint8_t *on = reinterpret_cast<uint8_t *>(jb + TC);
    __shared__ int wcnt[kBlock / 64];
    const int lane = tid & 63, wv = tid >> 6;
    int nr = 0;
    int s0 = next_start(sm.acc, 0, TC);
    while (s0 >= 0) {
      for (int t = tid; t < TC; t += kBlock) {
        const bool st = (sm.acc[t >> 6] >> (t & 63)) & 1ull;
        const bool capped = st && sm.reach[t] == kReach && t + 1 + kReach < TC;
        ja[t] = !st ? (int16_t)-1 : (capped ? (int16_t)-2 : sm.nx[t]);
        on[t] = t == s0;
      }
      __syncthreads();
      for (;;) {
        // ja = J_k: 2^k links on (-1: none, -2: a capped start on the way)
        for (int t = tid; t < TC; t += kBlock) {
          const int j = ja[t];
          if (on[t] && j >= 0) on[j] = 1;
        }
        for (int t = tid; t < TC; t += kBlock) {
          const int j = ja[t];
          jb[t] = j >= 0 ? ja[j] : (int16_t)j;
        }
        __syncthreads();
        // all links within 2^(k+1) of s0 are marked; done when s0 has no
        // start 2^(k+1) links on
        const bool more = jb[s0] >= 0;
        int16_t *x = ja;
        ja = jb;
        jb = x;
        if (!more) break;
        __syncthreads();     // the next level overwrites jb, read above
      }
      // marked starts, in tile order, appended to the runs
      for (int t0 = 0; t0 < TC; t0 += kBlock) {
        const int t = t0 + tid;
        const bool m = t < TC && on[t];
        const uint64_t b = __ballot(m);
        if (lane == 0) wcnt[wv] = __popcll(b);
        __syncthreads();
        int base = nr, tot = 0;
        for (int q = 0; q < kBlock / 64; q++) {
          base += q < wv ? wcnt[q] : 0;
          tot += wcnt[q];
        }
        if (m) {
          const int at = base + __popcll(b & ((1ull << lane) - 1ull));
          sm.rs[at] = (int16_t)t;
          sm.rl[at] = (int16_t)(1 + sm.reach[t]);
        }
        nr += tot;
        __syncthreads();
      }
      // the chain's last start: continue its run if its reach was capped
      const int last = sm.rs[nr - 1];
      if (sm.reach[last] == kReach && last + 1 + kReach < TC) {
        if (tid < 64) {
          const int len = 1 + kReach + extend_beyond<TH, TW>(sm, p, plane_of(last), last, last + 1 + kReach, TC, allowed);
          if (lane == 0) {
            sm.rl[nr - 1] = (int16_t)len;
            sm.misc[M_NEXT] = next_start(sm.acc, last + len, TC);
          }
        }
        __syncthreads();
        s0 = sm.misc[M_NEXT];
        __syncthreads();     // every thread has read M_NEXT and the marks before they are reset
      } else {
        s0 = -1;
      }
    }
    if (tid == 0) *nr_out = nr;
  }
  __syncthreads();
  {
    const int nr = *nr_out;
    for (int k = tid; k < nr; k += kBlock) {
      const int s0 = sm.rs[k], len = sm.rl[k];
      for (int q = 0; q < len; q++) sm.runof[s0 + q] = k;
    }
  }
  __syncthreads();
  for (int tc = tid; tc < TC; tc += kBlock) {
    if (!member(tc)) continue;
    const int ri = sm.runof[tc];
    if (ri < 0) continue;
    const int s = sm.rs[ri];
    sm.fmask[tc] = s == tc ? own_mask(tc)
                           : (sm.mstart(TC)[tc] == s ? sm.mcache()[tc] : inliers_at<TH, TW>(sm, tc, plane_of(s), p.eps));
  }
  return *nr_out;
}

// RUN-stream bytes of the pass's runs, one thread per run: varint of the
// gap to the previous run's end, varint of the length, then the run's own
// bytes (emit), and the count of runs of the row.
template <int TH, int TW, class EmitRun>
__device__ __forceinline__ void run_bytes(StripSmem<TH, TW> &sm, int nr, EmitRun emit) {
  for (int q = strip_tid(); q < nr; q += kBlock) {
    int prev_end = q ? sm.rs[q - 1] + sm.rl[q - 1] : 0;
    varint_bytes(sm.hist, (uint32_t)(sm.rs[q] - prev_end));
    varint_bytes(sm.hist, (uint32_t)sm.rl[q]);
    emit(sm.rs[q]);
  }
  if (strip_tid() == 0) varint_bytes(sm.hist, (uint32_t)nr);
}

// Spatial growth of one strip (Sec. III-C).  For predicted frames
// (`pred`), only tiles with elig != 0 take part; the others belong to
// temporal runs and break spatial runs.
template <int TH, int TW>
__device__ __forceinline__ void grow_spatial(StripSmem<TH, TW> &sm, const EncParams &p, const FrameDev &f, int tr, bool pred) {
  const int TC = f.TC, tid = strip_tid();
  auto member = [&](int tc) { return !pred || sm.elig[tc] != 0; };
  const int nr = grow_runs<TH, TW>(
      sm, p, TC, member, [&](int tc) { return member(tc) && sm.stat[tc] == ST_ACCEPTED; },
      [&](int, int t) { return member(t); }, [&](int s) { return unpack_plane(sm.plane[s]); },
      [&](int s) { return sm.omask[s]; }, &sm.misc[M_SRUNS]);
  if (tid == 0) f.nruns[tr] = nr;
  // stream bytes, classes and the runs themselves
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
    if (!member(tc)) continue;
    int ri = sm.runof[tc];
    if (ri >= 0) {
      sm.cls[tc] = CLS_SPATIAL;
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
__device__ __forceinline__ void grow_temporal(StripSmem<TH, TW> &sm, const EncParams &p, const FrameDev &f, int tr) {
  const int TC = f.TC, T = f.T, tid = strip_tid();
  const int nr = grow_runs<TH, TW>(
      sm, p, TC, [](int) { return true; }, [&](int tc) { return sm.stat[tc] == 2; },
      [&](int s, int t) { return sm.krun[t] == sm.krun[s]; }, [&](int s) { return unpack_plane(sm.plane[s]); },
      [&](int s) { return sm.omask[s]; }, &sm.misc[M_PRUNS]);
  if (tid == 0) f.nruns[f.TR + tr] = nr;
  run_bytes<TH, TW>(sm, nr, [&](int s) { f32_bytes(sm.hist, sm.plane[s].z); });
  pc_prun *runs = f.pruns + (int64_t)tr * TC;
  for (int q = tid; q < nr; q += kBlock) runs[q] = pc_prun{sm.rs[q], sm.rl[q], sm.krun[sm.rs[q]], sm.plane[sm.rs[q]].z};
  for (int tc = tid; tc < TC; tc += kBlock) {
    int ri = sm.runof[tc];
    if (ri >= 0) {
      sm.cls[tc] = CLS_TEMPORAL;
      sm.runof[tc] = T + tr * TC + ri;
      sm.elig[tc] = 0;
    } else {
      sm.elig[tc] = 1;
    }
  }
}

// ----------------------------------------------------- phase 3: residuals
// Block-wide exclusive scan of sm.cnt()[0 .. n) in place; returns the total.
template <int TH, int TW>
__device__ __forceinline__ uint32_t block_exclusive_scan(StripSmem<TH, TW> &sm, int n) {
  const int tid = strip_tid();
  const int per = (n + kBlock - 1) / kBlock;
  const int b = tid * per, e = min(n, b + per);
  uint32_t local = 0;
  for (int q = b; q < e; q++) local += sm.cnt()[q];
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
    uint32_t c = sm.cnt()[q];
    sm.cnt()[q] = run;
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
__device__ __forceinline__ void residuals_and_streams(StripSmem<TH, TW> &sm, const SensorDev &s,
                                      const EncParams &p, const FrameDev &f, int tr, int fits, int fp64) {
  constexpr int N = TH * TW;
  const int TC = f.TC, W = s.W, tid = strip_tid();
  // counts per (row in strip, tile) in raster order, MASK bytes
  for (int tc = tid; tc < TC; tc += kBlock) {
    const uint64_t V = valid_bits<TH, TW>(sm, tc);
    int cl = sm.cls[tc];
    bool cov = cl == CLS_SPATIAL || cl == CLS_TEMPORAL;
    uint64_t R = V & ~(cov ? sm.fmask[tc] : 0ull);
#pragma unroll
    for (int i = 0; i < TH; i++) sm.cnt()[i * TC + tc] = __popc((uint32_t)((R >> (i * TW)) & ((1ull << TW) - 1ull)));
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
      uint32_t o = sm.cnt()[i * TC + tc];
      uint32_t prev = 0;
      bool have = false;
#pragma unroll
      for (int k = 0; k < TW; k++) {
        int j = i * TW + k;
        float r = sm.r[tile_elem(tc, j, N)];
        if (r > 0.0f && !((fm >> j) & 1ull)) {
          float q = rintf(r * p.inv);
          // the difference is exact in FP32 (back and r within a factor of
          // two when q >= 1, back = 0 otherwise)
          const float back = q * p.step;
          if (q > 65535.0f || fabsf(back - r) > p.eps) {
            bad = 1;
            q = fminf(q, 65535.0f);
          }
          const uint32_t code = (uint32_t)q;
          res[o++] = (uint16_t)code;
          // RES stream bytes: the zigzag difference (mod 2^16) from the
          // previous residual code of the image row; a segment's first code
          // is done below, once its predecessor in an earlier tile is known
          if (have) hist_delta(sm.hist, code, prev);
          prev = code;
          have = true;
        }
      }
    }
  }
  // first code of every (row, tile) segment: its predecessor is the code
  // just before it in the strip's raster-order list, unless it opens its row
  __syncthreads();
  for (int e = tid; e < TH * TC; e += kBlock) {
    const uint32_t k = sm.cnt()[e], next = e + 1 < TH * TC ? sm.cnt()[e + 1] : total;
    if (next == k) continue;
    const uint32_t row0 = sm.cnt()[(e / TC) * TC];
    hist_delta(sm.hist, res[k], k == row0 ? 0u : res[k - 1]);
  }
  // per-tile outputs
  for (int tc = tid; tc < TC; tc += kBlock) {
    int t = tr * TC + tc;
    f.cls[t] = sm.cls[tc];
    f.mask[t] = (sm.cls[tc] == CLS_SPATIAL || sm.cls[tc] == CLS_TEMPORAL) ? sm.fmask[tc] : 0ull;
    f.run_of[t] = sm.runof[tc];
  }
  // block reductions of counters: wavefront sums, one atomic per wavefront
  __shared__ int red[8];
  if (tid < 8) red[tid] = 0;
  __syncthreads();
  int v[8] = {0, 0, 0, 0, 0, fits, fp64, (int)bad};
  for (int tc = tid; tc < TC; tc += kBlock) {
    const int cl = sm.cls[tc];
    v[0] += sm.nv[tc];
    v[1] += cl == 0;
    v[2] += cl == 1;
    v[3] += cl == 2;
    v[4] += cl == 3;
  }
#pragma unroll
  for (int c = 0; c < 8; c++) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o, 64);
  }
  if ((tid & 63) < 8) {
    const int c = tid & 63;
    int x = v[0];
#pragma unroll
    for (int q = 1; q < 8; q++) x = c == q ? v[q] : x;
    atomicAdd(&red[c], x);       // red[7]: nonzero when any pixel was out of range
  }
  __syncthreads();
  // OCC words (bit u % 32 of word (i * W + u) / 32: pixel (i, u) not
  // empty) from the ranges, to global and into the OCC histogram
  // (little-endian bytes).  A word covers 32 columns of one row: 32 / TW
  // tiles, whole 16-byte units of each.
  const int nw = TH * W / 32;
  uint32_t *occ = f.occ + (int64_t)tr * nw;
  for (int q = tid; q < nw; q += kBlock) {
    const int i = q / (W / 32), u0 = (q % (W / 32)) * 32;
    uint32_t wv = 0;
#pragma unroll
    for (int c4 = 0; c4 < 8; c4++) {
      const int u = u0 + 4 * c4;
      const float4 v = *reinterpret_cast<const float4 *>(sm.r + tile_elem(u / TW, i * TW + (u % TW), N));
      wv |= ((uint32_t)(v.x > 0.0f) | ((uint32_t)(v.y > 0.0f) << 1) | ((uint32_t)(v.z > 0.0f) << 2) |
             ((uint32_t)(v.w > 0.0f) << 3)) << (4 * c4);
    }
    occ[q] = wv;
    for (int b = 0; b < 4; b++) hist_byte(sm.hist, S_OCC, (wv >> (8 * b)) & 255u);
  }
  __syncthreads();
  uint32_t *ss = f.strip + (int64_t)tr * PC_STRIP_WORDS;
  for (int q = tid; q < 1024; q += kBlock) ss[q] = (sm.hist[q >> 1] >> ((q & 1) << 4)) & 0xffffu;
  if (tid == 0) {
    uint32_t *st = ss + 1024;
    st[PC_SS_VALID] = red[0];
    st[PC_SS_RES] = total;
    for (int c = 0; c < 4; c++) st[PC_SS_TILES + c] = red[1 + c];
    st[PC_SS_SRUNS] = sm.misc[M_SRUNS];
    st[PC_SS_PRUNS] = sm.misc[M_PRUNS];
    st[PC_SS_FITS] = red[5];
    st[PC_SS_FP64] = red[6];
    st[PC_SS_STATUS] = red[7] ? PC_STATUS_RANGE : 0u;
    st[PC_SS_SEEDED] = sm.misc[M_SEEDED];
    st[PC_SS_FALLBACK] = sm.misc[M_FALLBACK];
    for (int q = PC_SS_FALLBACK + 1; q < PC_STRIP_STATS; q++) st[q] = 0;
    f.nres[tr] = (int32_t)total;
  }
}

// Valid-pixel counts of the strip's tiles.
template <int TH, int TW>
__device__ __forceinline__ void count_valid(StripSmem<TH, TW> &sm, int TC) {
  for (int tc = strip_tid(); tc < TC; tc += kBlock) sm.nv[tc] = (uint8_t)__popcll(valid_bits<TH, TW>(sm, tc));
}

// Key frame, one tile-row strip (Sec. III-C).
template <int TH, int TW>
__device__ __forceinline__ void key_strip(char *smem_raw, const StripSrc &src, const SensorDev &s, const EncParams &p,
                          const float *__restrict__ seed, const FrameDev &f, int tr) {
  StripSmem<TH, TW> sm;
  const int TC = f.TC;
  sm.carve(smem_raw, s.W, TC, false);
  strip_init<TH, TW>(sm, s, tr);
  load_source<TH, TW>(sm, src, s, tr);
  __syncthreads();
  count_valid<TH, TW>(sm, TC);
  __syncthreads();
  int fits = 0, fp64 = 0;
  if (seed) {
    seeded_fits<TH, TW>(sm, p, TC, reinterpret_cast<const float4 *>(seed) + (int64_t)tr * TC, fits, fp64);
    own_fits<TH, TW>(sm, p, TC, [&](int tc) { return sm.elig[tc] != 1; }, fits, fp64);
  } else {
    for (int tc = strip_tid(); tc < TC; tc += kBlock) sm.elig[tc] = 0;
    own_fits<TH, TW>(sm, p, TC, [](int) { return true; }, fits, fp64);
  }
  // per-tile fit records (diagnostics; a batch may leave them out)
  for (int tc = strip_tid(); f.tiles && tc < TC; tc += kBlock) {
    Plane P = unpack_plane(sm.plane[tc]);
    pc_tile_rec rec;
    rec.a = P.a; rec.b = P.b; rec.c = P.c;
    rec.axis = (uint8_t)P.k; rec.status = sm.stat[tc]; rec.iters = sm.iters[tc]; rec.t_status = 0;
    rec.mask = sm.omask[tc]; rec.t_mask = 0; rec.t_c = 0.f; rec.t_iters = 0; rec.seeded = sm.elig[tc];
    rec.pad[0] = rec.pad[1] = 0;
    f.tiles[tr * TC + tc] = rec;
  }
  grow_spatial<TH, TW>(sm, p, f, tr, false);
  if (strip_tid() == 0) f.nruns[f.TR + tr] = 0;
  __syncthreads();
  residuals_and_streams<TH, TW>(sm, s, p, f, tr, fits, fp64);
}

// Predicted frame, one tile-row strip (Sec. III-D).
template <int TH, int TW>
__device__ __forceinline__ void pred_strip(char *smem_raw, const FrameDev &key, const StripSrc &src, const SensorDev &s,
                           const EncParams &p, const FrameDev &f, int tr) {
  StripSmem<TH, TW> sm;
  const int TC = f.TC;
  sm.carve(smem_raw, s.W, TC, true);
  strip_init<TH, TW>(sm, s, tr);
  load_source<TH, TW>(sm, src, s, tr);
  __syncthreads();
  count_valid<TH, TW>(sm, TC);
  for (int tc = strip_tid(); tc < TC; tc += kBlock) {
    sm.cls[tc] = CLS_EMPTY;
    sm.elig[tc] = 0;
  }
  __syncthreads();
  int fits = 0, fp64 = 0;
  // temporal fits against the key frame's run planes, temporal runs
  temporal_fits<TH, TW>(sm, key, p, tr, TC);
  for (int tc = strip_tid(); f.tiles && tc < TC; tc += kBlock) {
    pc_tile_rec rec;
    rec.a = 0.f; rec.b = 0.f; rec.c = 0.f; rec.axis = 0; rec.status = 0; rec.iters = 0;
    rec.t_status = sm.stat[tc]; rec.mask = 0; rec.t_mask = sm.omask[tc]; rec.t_c = sm.plane[tc].z;
    rec.t_iters = sm.iters[tc]; rec.seeded = 0; rec.pad[0] = rec.pad[1] = 0;
    f.tiles[tr * TC + tc] = rec;
  }
  grow_temporal<TH, TW>(sm, p, f, tr);
  __syncthreads();
  // own fits of the tiles left over, spatial runs
  own_fits<TH, TW>(sm, p, TC, [&](int tc) { return sm.elig[tc] != 0; }, fits, fp64);
  for (int tc = strip_tid(); f.tiles && tc < TC; tc += kBlock) {
    if (!sm.elig[tc]) continue;
    Plane P = unpack_plane(sm.plane[tc]);
    pc_tile_rec *rec = &f.tiles[tr * TC + tc];
    rec->a = P.a; rec->b = P.b; rec->c = P.c;
    rec->axis = (uint8_t)P.k; rec->status = sm.stat[tc]; rec->iters = sm.iters[tc];
    rec->mask = sm.omask[tc];
  }
  grow_spatial<TH, TW>(sm, p, f, tr, true);
  __syncthreads();
  residuals_and_streams<TH, TW>(sm, s, p, f, tr, fits, fp64);
}

// --------------------------------------------------- per-frame stream size
// 256 counts sorted ascending across a wavefront, element e in register
// e / 64 of lane e % 64: bitonic network, partners in other lanes through
// shuffles, partners in other registers of the same lane directly.
__device__ __forceinline__ void wave_sort256(uint32_t (&v)[4], int lane) {
#pragma unroll
  for (int k = 2; k <= 256; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
#pragma unroll
        for (int R = 0; R < 4; R++) {
          if (R & (j >> 6)) continue;
          const int R2 = R ^ (j >> 6);
          const bool up = ((64 * R + lane) & k) == 0;
          const uint32_t lo = min(v[R], v[R2]), hi = max(v[R], v[R2]);
          v[R] = up ? lo : hi;
          v[R2] = up ? hi : lo;
        }
      } else {
#pragma unroll
        for (int R = 0; R < 4; R++) {
          const int e = 64 * R + lane;
          const uint32_t o = (uint32_t)__shfl_xor((int)v[R], j, 64);
          const bool up = (e & k) == 0, lower = (e & j) == 0;
          v[R] = (lower == up) ? min(v[R], o) : max(v[R], o);
        }
      }
    }
  }
}

__device__ __forceinline__ uint32_t pick4(const uint32_t (&v)[4], int r) {
  return r == 0 ? v[0] : (r == 1 ? v[1] : (r == 2 ? v[2] : v[3]));
}

// Optimal Huffman cost of a byte histogram (256 counts in LDS, one
// wavefront): with the leaves sorted, merge the two lightest of (next leaf,
// next internal node) until one node is left; the cost is the sum of the
// merged weights (two-queue construction).  Leaves and internal nodes stay
// in registers, 64 to a register; the merge runs on uniform indices and
// reads one lane of the current block with readlane.  Counts and their
// total are below 2^32.
__device__ uint64_t huffman_cost_wave(const uint32_t *h, int lane) {
  uint32_t v[4];
#pragma unroll
  for (int R = 0; R < 4; R++) v[R] = h[64 * R + lane];
  wave_sort256(v, lane);
  int i = 0;
#pragma unroll
  for (int R = 0; R < 4; R++) i += __popcll(__ballot(v[R] == 0u));
  const int m = 256 - i;
  if (m <= 0) return 0;
  if (m == 1) return (uint32_t)__builtin_amdgcn_readlane((int)pick4(v, i >> 6), i & 63);
  // lv: block of leaf i; qw: block being written (node qt); qr: block of
  // node qh when that is an older block; done: finished node blocks.  lf
  // and nd are the next leaf and the queue head (~0: none).
  uint32_t lv = pick4(v, i >> 6), qw = 0u, qr = 0u;
  uint32_t done[4] = {0u, 0u, 0u, 0u};
  int qh = 0, qt = 0;
  uint64_t cost = 0;
  uint32_t lf = (uint32_t)__builtin_amdgcn_readlane((int)lv, i & 63), nd = ~0u;
  for (int step = 0; step < m - 1; step++) {
    uint32_t ab[2];
#pragma unroll
    for (int z = 0; z < 2; z++) {
      if (lf <= nd) {             // ties go to the leaf; an exhausted side reads ~0
        ab[z] = lf;
        i++;
        if ((i & 63) == 0 && i < 256) lv = pick4(v, i >> 6);
        lf = i < 256 ? (uint32_t)__builtin_amdgcn_readlane((int)lv, i & 63) : ~0u;
      } else {
        ab[z] = nd;
        qh++;
        if ((qh & 63) == 0) qr = pick4(done, qh >> 6);
        const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)((((qh ^ qt) >> 6) == 0) ? qw : qr), qh & 63);
        nd = qh < qt ? x : ~0u;
      }
    }
    const uint32_t wsum = ab[0] + ab[1];
    cost += wsum;
    qw = lane == (qt & 63) ? wsum : qw;
    if (qh == qt) nd = wsum;      // the queue was empty: the new node is its head
    qt++;
    if ((qt & 63) == 0) {
      const int b = (qt >> 6) - 1;
      done[0] = b == 0 ? qw : done[0];
      done[1] = b == 1 ? qw : done[1];
      done[2] = b == 2 ? qw : done[2];
      done[3] = b == 3 ? qw : done[3];
      if ((qh >> 6) == b) qr = qw;
    }
  }
  return cost;
}

// Whole-frame totals and the Huffman size; one 256-thread block per frame.
__device__ void finish_frame(const FrameDev &f, int kind, const Mat12 &M, int hasM) {
  __shared__ uint32_t h[4][256];
  __shared__ uint32_t st[PC_STRIP_STATS];
  const int tid = strip_tid();
  // strip sums: eight strips' loads in flight per thread and entry
  const int TR = f.TR;
  const __attribute__((address_space(1))) uint32_t *ss = (const __attribute__((address_space(1))) uint32_t *)f.strip;
  uint32_t hs[4] = {0u, 0u, 0u, 0u}, sts = 0u;
  for (int r0 = 0; r0 < TR; r0 += 8) {
    uint32_t x[8][4], y[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const int r = r0 + k < TR ? r0 + k : r0;       // in range; repeats are masked below
      const int64_t base = (int64_t)r * PC_STRIP_WORDS;
#pragma unroll
      for (int e = 0; e < 4; e++) x[k][e] = ss[base + tid + 256 * e];
      y[k] = tid < PC_STRIP_STATS ? ss[base + 1024 + tid] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (r0 + k >= TR) break;
#pragma unroll
      for (int e = 0; e < 4; e++) hs[e] += x[k][e];
      sts = (tid == PC_SS_STATUS) ? (sts | y[k]) : sts + y[k];
    }
  }
#pragma unroll
  for (int e = 0; e < 4; e++) h[e][tid] = hs[e];
  if (tid < PC_STRIP_STATS) st[tid] = sts;
  __syncthreads();
  const int wv = tid >> 6, lane = tid & 63;
  // stream byte counts
  uint64_t nbytes = 0;
  for (int o = lane; o < 256; o += 64) nbytes += h[wv][o];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nbytes += __shfl_xor(nbytes, o, 64);
  uint64_t bits = huffman_cost_wave(h[wv], lane);
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

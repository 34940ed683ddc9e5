// Entropy-coded bitstream of a frame (Sec. III-A) and its inverse.
//
// The four byte streams of a frame stream buffer (OCC, RUN, MASK, RES, in
// the order the encoder accounts them) are each coded with a canonical
// Huffman code limited to 15 bits.  Container: a 112-byte header (magic
// "PCC1" u32, kind u8, tile_h u8, tile_w u8, 0 u8, H u16, W u16, stream
// bytes u64[4], payload bytes u32[4], 4 zero bytes, then the frame's
// transform into the key frame as 12 FP32, rows of [R | T]), then for each
// non-empty stream a 128-byte table of 4-bit code lengths (symbol 2i in the
// low nibble of byte i) and the code words, MSB first, padded to a byte.
//
// Packing: one work-group sums the per-strip histograms the encoder already
// wrote, builds the code (sorted two-queue Huffman construction, ties going
// to the leaf; the bit-count adjustment of ITU T.81 Annex K.3 when the tree
// is deeper than 15; lengths handed out by descending count, then symbol)
// and places every strip's bits from the histograms alone.  Then one
// work-group per strip regenerates its bytes of each stream in LDS and
// writes its code words at their known bit offsets: interior 32-bit words
// with plain stores, words shared with a neighbour with atomicOr into a
// container zeroed beforehand.
//
// Unpacking: canonical decoding by per-length limits.  Each stream's
// payload is cut into subsequences decoded in parallel from guessed starts;
// a subsequence whose start differs from its predecessor's end is decoded
// again until no start changes (Huffman codes resynchronise after a few
// code words), then every subsequence writes its symbols at the prefix of
// the counts.  The streams are then parsed back into a frame stream buffer
// that the decoder reads.
#include <algorithm>
#include <vector>

#include "encode_strip.h"

namespace pcc {
namespace {

constexpr int kMaxLen = 15;
constexpr uint32_t kMagic = 0x31434350u;   // bytes "PCC1"
constexpr int kPackBlock = 256;
constexpr int kChunk = 16384;              // stream bytes per segment when packing raw streams
constexpr int kUnpackBlock = 1024;
constexpr int kMaxSub = 8192;              // decode subsequences per stream
constexpr int kMinSubBits = 256;
constexpr int kRunLds = 32768;             // run tables up to this size are parsed from LDS
constexpr int kPayLds = 49152;             // stream payloads up to this size are decoded from LDS
constexpr int kMaxRec = 4096;              // run records a frame's table is decoded in parallel up to

struct PackPlan {
  uint32_t hist[4][256];
  uint32_t code[4][256];
  uint8_t len[4][256];
  uint8_t head[kHeaderBytes];
  uint8_t table[4][kTableBytes];
  uint64_t nbytes[4];       // stream bytes
  uint64_t bits[4];         // payload bits
  uint64_t table_at[4];     // container offset of the stream's table; its payload follows
  uint64_t total;           // container bytes (0: does not fit)
  uint32_t err;             // 1: capacity, 2: a strip's bytes disagree with its histogram
  uint32_t pad;
};

struct SegInfo {
  uint64_t bit;             // container bit of the segment's first code word
  uint64_t byte;            // offset of the segment's first byte in its stream
  uint32_t n;               // bytes
  uint32_t nbits;           // code bits
};

// Per-segment histograms: segment r of stream q at base + q*stride_q + r*stride_s.
struct HistSrc {
  const uint32_t *base;
  int64_t stride_q, stride_s;
  int nseg[4];
};

struct HeadInfo {
  int kind, th, tw, H, W;
  int kind_from_frame;      // 1: read kind from the frame's info block
  const pc_frame_info *info;
};

struct StreamPtrs {
  uint8_t *p[4];
  uint64_t cap[4];
};

// Everything one frame's (or one raw stream set's) packing needs.  Kernels
// take a job by value (one frame) or an array of jobs in device memory
// (several frames, one per block row).
struct PackJob {
  HistSrc hs;
  HeadInfo hi;
  PackPlan *plan;
  SegInfo *seg;
  int max_seg;
  int th, tw, W;
  uint64_t cap;
  uint64_t *nbytes;
  uint32_t *out;
  FrameDev f;
  StreamPtrs so;
};

struct UnpackPlan {
  uint64_t nbytes[4];       // symbols (stream bytes)
  uint64_t bit0[4];         // container bit of the payload
  uint64_t nbits[4];        // payload bits (8 x payload bytes)
  uint32_t limit[4][kMaxLen + 1];   // left-aligned end of the codes of each length
  uint32_t first[4][kMaxLen + 1];   // first code of each length
  uint32_t index[4][kMaxLen + 1];   // position of that code's symbol in sorted[]
  uint8_t sorted[4][256];           // symbols by (length, symbol)
  int32_t kind, th, tw, H, W;
  uint32_t err;             // 1: malformed container, 2: malformed payload, 4: malformed streams
  float M[12];              // the frame's transform into the key frame (rows of [R | T])
};

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *red, uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int)x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) red[wave] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < nw; w++) {
    uint32_t r = red[w];
    off += w < wave ? r : 0u;
    tot += r;
  }
  __syncthreads();
  if (total) *total = tot;
  return off + x - v;
}

// Run fields as read from a frame buffer, clamped to [0, TC]: for an encoded
// frame this changes nothing, for a damaged one it keeps every varint at two
// bytes or less, so a strip's run bytes stay within its staging buffer (the
// byte count then disagrees with the histogram and the pack reports it).
__device__ __forceinline__ uint32_t clamp_tc(int v, int TC) { return (uint32_t)min(max(v, 0), TC); }

__device__ __forceinline__ int varint_len(uint32_t v) {
  return v < (1u << 7) ? 1 : (v < (1u << 14) ? 2 : (v < (1u << 21) ? 3 : (v < (1u << 28) ? 4 : 5)));
}
__device__ __forceinline__ int put_varint(uint8_t *b, uint32_t v) {
  int k = 0;
  while (v >= 128u) {
    b[k++] = (uint8_t)((v & 127u) | 128u);
    v >>= 7;
  }
  b[k++] = (uint8_t)v;
  return k;
}
__device__ __forceinline__ void put_f32(uint8_t *b, float x) {
  const uint32_t u = __float_as_uint(x);
  b[0] = (uint8_t)u;
  b[1] = (uint8_t)(u >> 8);
  b[2] = (uint8_t)(u >> 16);
  b[3] = (uint8_t)(u >> 24);
}

// ------------------------------------------------------------------ the code
// Code lengths of one stream by wavefront `q`: the wave sorts the counts,
// lane 0 merges the two queues and derives the leaves' depths, then the
// depth counts are limited to 15 bits.  bl[0..63] receives the number of
// codes of each length.
struct LenScratch {
  uint32_t w[256];          // leaf weights, ascending
  uint32_t nw[256];         // internal node weights
  uint8_t lp[256];          // parent of leaf k (internal index)
  uint8_t np[256];          // parent of internal node k
  uint8_t dn[256];          // depth of internal node k
  int32_t bl[64];
};

__device__ void depth_counts_wave(const uint32_t *h, LenScratch &sc, int lane) {
  uint32_t v[4];
#pragma unroll
  for (int R = 0; R < 4; R++) v[R] = h[64 * R + lane];
  wave_sort256(v, lane);
  int zeros = 0;
#pragma unroll
  for (int R = 0; R < 4; R++) {
    sc.w[64 * R + lane] = v[R];
    zeros += __popcll(__ballot(v[R] == 0u));
  }
  sc.bl[lane] = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  if (lane != 0) return;
  const int m = 256 - zeros;
  if (m == 0) return;
  if (m == 1) {
    sc.bl[1] = 1;
    return;
  }
  int li = zeros, qh = 0, qt = 0;
  for (int step = 0; step < m - 1; step++) {
    uint32_t s = 0;
    for (int z = 0; z < 2; z++) {
      if (li < 256 && (qh == qt || sc.w[li] <= sc.nw[qh])) {     // ties take the leaf
        s += sc.w[li];
        sc.lp[li - zeros] = (uint8_t)qt;
        li++;
      } else {
        s += sc.nw[qh];
        sc.np[qh] = (uint8_t)qt;
        qh++;
      }
    }
    sc.nw[qt++] = s;
  }
  // depths top-down: the root is the last internal node
  sc.dn[qt - 1] = 0;
  for (int k = qt - 2; k >= 0; k--) sc.dn[k] = (uint8_t)(sc.dn[sc.np[k]] + 1);
  int maxd = 0;
  for (int k = 0; k < m; k++) {
    int d = sc.dn[sc.lp[k]] + 1;
    d = d > 63 ? 63 : d;
    sc.bl[d]++;
    maxd = d > maxd ? d : maxd;
  }
  // limit to 15 bits: a pair of the deepest codes becomes one code one
  // level up plus, by splitting the deepest shorter code, two codes one
  // level below that (the Kraft sum is kept)
  for (int i = maxd; i > kMaxLen; i--) {
    while (sc.bl[i] > 0) {
      int j = i - 2;
      while (j > 0 && sc.bl[j] == 0) j--;
      if (j == 0) break;
      sc.bl[i] -= 2;
      sc.bl[i - 1] += 1;
      sc.bl[j + 1] += 2;
      sc.bl[j] -= 1;
    }
  }
}

// Builds the code of all four streams, the header and the tables, and the
// bit offset of every segment.  One work-group of kPackBlock threads.
__global__ void __launch_bounds__(kPackBlock) k_pack_plan(PackJob j0, const PackJob *jobs) {
  const PackJob *J = jobs ? jobs + blockIdx.x : &j0;
  const HistSrc &hs = J->hs;
  const HeadInfo &hi = J->hi;
  PackPlan *plan = J->plan;
  SegInfo *seg = J->seg;
  const int max_seg = J->max_seg;
  const uint64_t cap = J->cap;
  uint64_t *nbytes_out = J->nbytes;
  __shared__ uint32_t h[4][256];
  __shared__ LenScratch sc[4];
  __shared__ uint8_t len[4][256];
  __shared__ uint32_t cum[4][kMaxLen + 1], first[4][kMaxLen + 1];
  __shared__ uint64_t nb[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < 1024; e += kPackBlock) {
    const int q = e >> 8, b = e & 255;
    uint32_t s = 0;
    for (int r = 0; r < hs.nseg[q]; r++) s += hs.base[q * hs.stride_q + r * hs.stride_s + b];
    h[q][b] = s;
    plan->hist[q][b] = s;
  }
  __syncthreads();
  depth_counts_wave(h[wave], sc[wave], lane);
  __syncthreads();
  if (tid < 4) {
    uint32_t c = 0, code = 0;
    uint64_t n = 0;
    for (int L = 1; L <= kMaxLen; L++) {
      c += (uint32_t)sc[tid].bl[L];
      cum[tid][L] = c;
      first[tid][L] = code;
      code = (code + (uint32_t)sc[tid].bl[L]) << 1;
    }
    for (int b = 0; b < 256; b++) n += h[tid][b];
    nb[tid] = n;
  }
  __syncthreads();
  // lengths: rank by (count descending, symbol ascending), shortest first
  for (int e = tid; e < 1024; e += kPackBlock) {
    const int q = e >> 8, s = e & 255;
    const uint32_t c = h[q][s];
    uint8_t L = 0;
    if (c) {
      uint32_t rank = 0;
      for (int t = 0; t < 256; t++) {
        const uint32_t o = h[q][t];
        rank += (o > c || (o == c && t < s)) ? 1u : 0u;
      }
      L = 1;
      while (L < kMaxLen && cum[q][L] <= rank) L++;
    }
    len[q][s] = L;
    plan->len[q][s] = L;
  }
  __syncthreads();
  // canonical codes: by length, then symbol
  for (int e = tid; e < 1024; e += kPackBlock) {
    const int q = e >> 8, s = e & 255, L = len[q][s];
    uint32_t code = 0;
    if (L) {
      uint32_t k = 0;
      for (int t = 0; t < s; t++) k += len[q][t] == L ? 1u : 0u;
      code = first[q][L] + k;
    }
    plan->code[q][s] = code;
  }
  for (int e = tid; e < 4 * kTableBytes; e += kPackBlock) {
    const int q = e / kTableBytes, i = e % kTableBytes;
    plan->table[q][i] = (uint8_t)(len[q][2 * i] | (len[q][2 * i + 1] << 4));
  }
  // per segment: bytes and code bits (a wave per segment)
  for (int p = wave; p < 4 * max_seg; p += kPackBlock / 64) {
    const int q = p / max_seg, r = p % max_seg;
    if (r >= hs.nseg[q]) continue;
    const uint32_t *hp = hs.base + q * hs.stride_q + r * hs.stride_s;
    uint32_t n = 0, bits = 0;
#pragma unroll
    for (int R = 0; R < 4; R++) {
      const uint32_t c = hp[64 * R + lane];
      n += c;
      bits += c * len[q][64 * R + lane];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      n += (uint32_t)__shfl_xor((int)n, o, 64);
      bits += (uint32_t)__shfl_xor((int)bits, o, 64);
    }
    if (lane == 0) {
      seg[q * max_seg + r].n = n;
      seg[q * max_seg + r].nbits = bits;
    }
  }
  __syncthreads();
  if (tid == 0) {
    const int kind = hi.kind_from_frame ? hi.info->kind : hi.kind;
    uint8_t *hd = plan->head;
    for (int i = 0; i < kHeaderBytes; i++) hd[i] = 0;
    for (int i = 0; i < 4; i++) hd[i] = (uint8_t)(kMagic >> (8 * i));
    hd[4] = (uint8_t)kind;
    hd[5] = (uint8_t)hi.th;
    hd[6] = (uint8_t)hi.tw;
    hd[8] = (uint8_t)hi.H;
    hd[9] = (uint8_t)(hi.H >> 8);
    hd[10] = (uint8_t)hi.W;
    hd[11] = (uint8_t)(hi.W >> 8);
    // the transform (identity for raw streams): a predicted frame's points
    // return to its own coordinates through it (Sec. III-D)
    for (int e = 0; e < 12; e++) {
      const float m = hi.kind_from_frame ? hi.info->M[e] : (e % 5 == 0 ? 1.0f : 0.0f);
      const uint32_t u = __float_as_uint(m);
      for (int i = 0; i < 4; i++) hd[64 + 4 * e + i] = (uint8_t)(u >> (8 * i));
    }
    uint64_t at = kHeaderBytes;
    for (int q = 0; q < 4; q++) {
      uint64_t bits = 0;
      for (int r = 0; r < hs.nseg[q]; r++) bits += seg[q * max_seg + r].nbits;
      plan->nbytes[q] = nb[q];
      plan->bits[q] = bits;
      const uint64_t pb = (bits + 7) / 8;
      for (int i = 0; i < 8; i++) hd[12 + 8 * q + i] = (uint8_t)(nb[q] >> (8 * i));
      for (int i = 0; i < 4; i++) hd[44 + 4 * q + i] = (uint8_t)(pb >> (8 * i));
      plan->table_at[q] = at;
      if (nb[q] == 0) continue;
      uint64_t bit = 8 * (at + kTableBytes), byte = 0;
      for (int r = 0; r < hs.nseg[q]; r++) {
        SegInfo &S = seg[q * max_seg + r];
        S.bit = bit;
        S.byte = byte;
        bit += S.nbits;
        byte += S.n;
      }
      at += kTableBytes + pb;
    }
    const bool fits = ((at + 3) & ~(uint64_t)3) <= cap;
    plan->total = fits ? at : 0;
    plan->err = fits ? 0u : 1u;
    *nbytes_out = 0;
  }
}

// Header, tables and zeroed payload words.  16-byte units that lie inside
// payloads (all but a few) are zeroed with one vector store; the units that
// touch the header or a table are built byte by byte.
__global__ void __launch_bounds__(kPackBlock) k_pack_fill(PackJob j0, const PackJob *jobs) {
  const PackJob *J = jobs ? jobs + blockIdx.y : &j0;
  const PackPlan *plan = J->plan;
  uint32_t *out = J->out;
  const uint64_t total = plan->total;
  if (plan->err || total == 0) return;
  const uint64_t nw = (total + 3) / 4;
  uint64_t t0[4];
  for (int q = 0; q < 4; q++) t0[q] = plan->nbytes[q] ? plan->table_at[q] : ~0ull - kTableBytes;
  auto word = [&](uint64_t w) {
    uint32_t v = 0;
    for (int j = 0; j < 4; j++) {
      const uint64_t B = 4 * w + j;
      uint32_t byte = 0;
      if (B < kHeaderBytes) {
        byte = plan->head[B];
      } else {
        for (int q = 0; q < 4; q++)
          if (B >= t0[q] && B < t0[q] + kTableBytes) byte = plan->table[q][B - t0[q]];
      }
      v |= byte << (8 * j);
    }
    return v;
  };
  const uint64_t stride = (uint64_t)gridDim.x * kPackBlock, first = (uint64_t)blockIdx.x * kPackBlock + threadIdx.x;
  if (((uintptr_t)out & 15) == 0) {
    const uint64_t nu = nw / 4;                // whole 16-byte units
    for (uint64_t u = first; u < nu; u += stride) {
      const uint64_t B0 = 16 * u, B1 = B0 + 16;
      bool special = B0 < kHeaderBytes;
      for (int q = 0; q < 4; q++) special |= B0 < t0[q] + kTableBytes && B1 > t0[q];
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (special) v = make_uint4(word(4 * u), word(4 * u + 1), word(4 * u + 2), word(4 * u + 3));
      reinterpret_cast<uint4 *>(out)[u] = v;
    }
    for (uint64_t w = 4 * nu + first; w < nw; w += stride) out[w] = word(w);
  } else {
    for (uint64_t w = first; w < nw; w += stride) out[w] = word(w);
  }
}

// Code words of buf[0..n) from container bit `bit0`, never past `bit_end`.
// Each thread codes a contiguous share of the bytes at the prefix of the
// shares' bit counts.  buf is 4-byte aligned; a share is a whole number of
// 32-bit words, an odd number of them, so that the lanes of a wavefront
// reading their shares' k-th words hit distinct LDS banks.
__device__ void encode_bytes(const uint8_t *buf, uint32_t n, uint64_t bit0, uint64_t bit_end, const uint8_t *len,
                             const uint32_t *code, uint32_t *out, uint32_t *red, uint32_t *err) {
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  uint32_t per = (((n + nt - 1) / nt) + 3) & ~3u;
  if (((per >> 2) & 1u) == 0 && per) per += 4;
  const uint32_t b0 = min(n, tid * per), b1 = min(n, b0 + per);
  const uint32_t *bw = reinterpret_cast<const uint32_t *>(buf);
  uint32_t nb = 0;
  for (uint32_t i = b0; i < b1; i += 4) {
    const uint32_t w = bw[i >> 2];
    const uint32_t m = min(4u, b1 - i);
    for (uint32_t k = 0; k < m; k++) nb += len[(w >> (8 * k)) & 255u];
  }
  const uint32_t ex = block_excl_scan(nb, red, nullptr);
  const uint64_t start = bit0 + ex;
  uint64_t pos = start;
  const uint64_t stop = min(start + nb, bit_end);
  auto flush = [&](uint64_t w, uint32_t acc) {
    const uint32_t v = __builtin_bswap32(acc);
    if ((w << 5) >= start && ((w + 1) << 5) <= stop)
      out[w] = v;
    else
      atomicOr(&out[w], v);
  };
  uint64_t cw = pos >> 5;
  uint32_t acc = 0;
  uint32_t w = 0;
  for (uint32_t i = b0; i < b1; i++) {
    if (((i - b0) & 3u) == 0) w = bw[i >> 2];
    const uint32_t s = (w >> (8 * ((i - b0) & 3u))) & 255u, L = len[s], c = code[s];
    if (pos + L > stop) {
      atomicOr(err, 2u);
      break;
    }
    const uint32_t o = (uint32_t)(pos & 31);
    if (o + L <= 32) {
      acc |= c << (32 - o - L);
      pos += L;
      if ((pos & 31) == 0) {
        flush(cw, acc);
        cw++;
        acc = 0;
      }
    } else {
      const uint32_t sp = o + L - 32;
      acc |= c >> sp;
      flush(cw, acc);
      cw++;
      acc = c << (32 - sp);
      pos += L;
    }
  }
  if ((pos & 31) && pos > start) flush(cw, acc);
}

// One work-group per tile-row strip: regenerate the strip's bytes of each
// stream from the frame stream buffer, optionally copy them out, and code
// them.  blockIdx.x is the frame (job) and blockIdx.y the strip, so that
// every XCD gets every strip row.
__global__ void __launch_bounds__(kPackBlock) k_pack_frame(PackJob j0, const PackJob *jobs) {
  const PackJob *J = jobs ? jobs + blockIdx.x : &j0;
  const FrameDev f = J->f;
  const int th = J->th, tw = J->tw, W = J->W, max_seg = J->max_seg;
  PackPlan *plan = J->plan;
  const SegInfo *seg = J->seg;
  uint32_t *out = J->out;
  const StreamPtrs &so = J->so;
  extern __shared__ __align__(16) char smem[];
  uint8_t *len = (uint8_t *)smem;                        // [4][256]
  uint32_t *code = (uint32_t *)(smem + 1024);            // [4][256]
  uint32_t *red = code + 1024;                           // [16]
  uint8_t *buf = (uint8_t *)(red + 16);                  // the strip's bytes of one stream
  __shared__ int skip;
  const int tid = threadIdx.x, tr = blockIdx.y, TC = f.TC, TR = f.TR;
  // other strips may raise plan->err meanwhile: decide once for the group
  if (tid == 0) skip = (plan->err & 1u) || plan->total == 0;
  __syncthreads();
  if (skip) return;
  for (int e = tid; e < 1024; e += kPackBlock) {
    len[e] = plan->len[e >> 8][e & 255];
    code[e] = plan->code[e >> 8][e & 255];
  }
  const int kind = f.info->kind;
  const int nw = th * W / 32;
  const uint32_t *occ = f.occ + (int64_t)tr * nw;
  const uint32_t lowm = (uint32_t)((1ull << tw) - 1ull);
  auto valid_bits = [&](int tc) {
    uint64_t V = 0;
    for (int i = 0; i < th; i++) {
      const int bit = i * W + tc * tw;
      V |= (uint64_t)((occ[bit >> 5] >> (bit & 31)) & lowm) << (i * tw);
    }
    return V;
  };
  for (int q = 0; q < 4; q++) {
    __syncthreads();
    uint32_t n = 0;
    if (q == S_OCC) {
      for (int w = tid; w < nw; w += kPackBlock) ((uint32_t *)buf)[w] = occ[w];
      n = 4u * (uint32_t)nw;
    } else if (q == S_RUN) {
      const int np = kind ? min(max(f.nruns[TR + tr], 0), TC) : 0, ns = min(max(f.nruns[tr], 0), TC);
      const pc_prun *pr = f.pruns + (int64_t)tr * TC;
      const pc_run *sr = f.sruns + (int64_t)tr * TC;
      const int head0 = kind ? varint_len((uint32_t)np) : 0;
      // temporal runs: gap, length, c'
      const int pp = (np + kPackBlock - 1) / kPackBlock, p0 = min(np, tid * pp), p1 = min(np, p0 + pp);
      uint32_t mine = 0;
      for (int k = p0; k < p1; k++) {
        const int prev = k ? pr[k - 1].s + pr[k - 1].len : 0;
        mine += varint_len(clamp_tc(pr[k].s - prev, TC)) + varint_len(clamp_tc(pr[k].len, TC)) + 4;
      }
      uint32_t P;
      uint32_t at = head0 + block_excl_scan(mine, red, &P);
      for (int k = p0; k < p1; k++) {
        const int prev = k ? pr[k - 1].s + pr[k - 1].len : 0;
        at += put_varint(buf + at, clamp_tc(pr[k].s - prev, TC));
        at += put_varint(buf + at, clamp_tc(pr[k].len, TC));
        put_f32(buf + at, pr[k].c);
        at += 4;
      }
      // spatial runs: gap, length, axis, a, b, c
      const int hs = varint_len((uint32_t)ns);
      const int sp = (ns + kPackBlock - 1) / kPackBlock, s0 = min(ns, tid * sp), s1 = min(ns, s0 + sp);
      mine = 0;
      for (int k = s0; k < s1; k++) {
        const int prev = k ? sr[k - 1].s + sr[k - 1].len : 0;
        mine += varint_len(clamp_tc(sr[k].s - prev, TC)) + varint_len(clamp_tc(sr[k].len, TC)) + 13;
      }
      uint32_t S;
      at = head0 + P + hs + block_excl_scan(mine, red, &S);
      for (int k = s0; k < s1; k++) {
        const int prev = k ? sr[k - 1].s + sr[k - 1].len : 0;
        at += put_varint(buf + at, clamp_tc(sr[k].s - prev, TC));
        at += put_varint(buf + at, clamp_tc(sr[k].len, TC));
        buf[at++] = (uint8_t)sr[k].axis;
        put_f32(buf + at, sr[k].a);
        put_f32(buf + at + 4, sr[k].b);
        put_f32(buf + at + 8, sr[k].c);
        at += 12;
      }
      if (tid == 0) {
        if (kind) put_varint(buf, (uint32_t)np);
        put_varint(buf + head0 + P, (uint32_t)ns);
      }
      n = head0 + P + hs + S;
    } else if (q == S_MASK) {
      // per plane-coded tile: its valid pixels' mask bits, LSB first
      const int tp = (TC + kPackBlock - 1) / kPackBlock, t0 = min(TC, tid * tp), t1 = min(TC, t0 + tp);
      uint32_t mine = 0;
      for (int tc = t0; tc < t1; tc++) {
        const int c = f.cls[(int64_t)tr * TC + tc];
        if (c == CLS_SPATIAL || c == CLS_TEMPORAL) mine += (__popcll(valid_bits(tc)) + 7) >> 3;
      }
      uint32_t tot;
      uint32_t at = block_excl_scan(mine, red, &tot);
      for (int tc = t0; tc < t1; tc++) {
        const int64_t t = (int64_t)tr * TC + tc;
        const int c = f.cls[t];
        if (c != CLS_SPATIAL && c != CLS_TEMPORAL) continue;
        const uint64_t V = valid_bits(tc), M = f.mask[t];
        uint64_t bits = 0;
        int k = 0;
        for (uint64_t v = V; v; v &= v - 1, k++) bits |= ((M >> __builtin_ctzll(v)) & 1ull) << k;
        for (int b = 0; b < (k + 7) >> 3; b++) buf[at++] = (uint8_t)(bits >> (8 * b));
      }
      n = tot;
    } else {
      // each code as the zigzag difference (mod 2^16) from the previous
      // residual code of its image row; rows start where the strip's
      // uncovered non-empty pixels of the rows above end
      __shared__ uint32_t rowc[8];
      const int nr = min(max(f.nres[tr], 0), th * W);
      const uint16_t *rs = f.res + (int64_t)tr * th * W;
      if (tid < th) rowc[tid] = 0;
      __syncthreads();
      for (int tc = tid; tc < TC; tc += kPackBlock) {
        const int64_t t = (int64_t)tr * TC + tc;
        const int c = f.cls[t];
        const uint64_t R = valid_bits(tc) & ~((c == CLS_SPATIAL || c == CLS_TEMPORAL) ? f.mask[t] : 0ull);
        for (int i = 0; i < th; i++) {
          const uint32_t k = (uint32_t)__popcll((R >> (i * tw)) & lowm);
          if (k) atomicAdd(&rowc[i], k);
        }
      }
      __syncthreads();
      uint32_t st[8], acc = 0;
      for (int i = 0; i < 8; i++) {
        st[i] = i < th ? acc : 0xFFFFFFFFu;
        acc += i < th ? rowc[i] : 0u;
      }
      for (int k = tid; k < nr; k += kPackBlock) {
        bool first = false;
        for (int i = 0; i < 8; i++) first |= (uint32_t)k == st[i];
        const uint32_t prev = first ? 0u : rs[k - 1];
        const uint32_t d = ((uint32_t)rs[k] - prev) & 0xFFFFu;
        ((uint16_t *)buf)[k] = (uint16_t)(((d << 1) ^ ((d & 0x8000u) ? 0xFFFFu : 0u)) & 0xFFFFu);
      }
      n = 2u * (uint32_t)nr;
    }
    __syncthreads();
    const SegInfo S = seg[q * max_seg + tr];
    if (n != S.n) {
      if (tid == 0) atomicOr(&plan->err, 2u);
      n = min(n, S.n);
    }
    if (so.p[q] && S.byte + n <= so.cap[q])
      for (uint32_t i = tid; i < n; i += kPackBlock) so.p[q][S.byte + i] = buf[i];
    encode_bytes(buf, n, S.bit, S.bit + S.nbits, len + 256 * q, code + 256 * q, out, red, &plan->err);
  }
}

__global__ void k_pack_done(PackJob j0, const PackJob *jobs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PackJob *J = jobs ? jobs + i : &j0;
  *J->nbytes = J->plan->err ? 0 : J->plan->total;
}

// Raw streams: histogram and code of each kChunk-byte segment.
struct StreamIn {
  const uint8_t *p[4];
  uint64_t n[4];
};

__global__ void __launch_bounds__(kPackBlock) k_pack_hist(StreamIn in, uint32_t *seg_hist, int max_seg) {
  __shared__ uint32_t h[256];
  const int q = blockIdx.x / max_seg, r = blockIdx.x % max_seg, tid = threadIdx.x;
  const uint64_t b0 = (uint64_t)r * kChunk;
  if (b0 >= in.n[q]) return;
  const uint32_t n = (uint32_t)min((uint64_t)kChunk, in.n[q] - b0);
  h[tid] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < n; i += kPackBlock) atomicAdd(&h[in.p[q][b0 + i]], 1u);
  __syncthreads();
  seg_hist[((int64_t)q * max_seg + r) * 256 + tid] = h[tid];
}

__global__ void __launch_bounds__(kPackBlock) k_pack_chunks(StreamIn in, PackPlan *plan, const SegInfo *seg, int max_seg,
                                                           uint32_t *out) {
  __shared__ uint8_t len[256];
  __shared__ uint32_t code[256];
  __shared__ uint32_t red[16];
  __shared__ __align__(16) uint8_t buf[kChunk];
  __shared__ int skip;
  const int q = blockIdx.x / max_seg, r = blockIdx.x % max_seg, tid = threadIdx.x;
  const uint64_t b0 = (uint64_t)r * kChunk;
  if (tid == 0) skip = (plan->err & 1u) || plan->total == 0;
  __syncthreads();
  if (skip || b0 >= in.n[q]) return;
  const uint32_t n = (uint32_t)min((uint64_t)kChunk, in.n[q] - b0);
  len[tid] = plan->len[q][tid];
  code[tid] = plan->code[q][tid];
  for (uint32_t i = tid; i < n; i += kPackBlock) buf[i] = in.p[q][b0 + i];
  __syncthreads();
  const SegInfo S = seg[q * max_seg + r];
  encode_bytes(buf, min(n, S.n), S.bit, S.bit + S.nbits, len, code, out, red, &plan->err);
}

// ---------------------------------------------------------------- unpacking
__device__ __forceinline__ uint32_t rd_u32(const uint8_t *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

// Header and code tables.  One thread; the container is small at this point
// of the check (header and four tables).
// Header and code tables of one container, by one work-group of 64 threads:
// thread 0 reads the header and places the tables, the group loads the four
// length tables into LDS, then one thread per stream builds its decoding
// table (a counting sort of the symbols by length).  Called by every thread
// of the group.
__device__ void unpack_plan(const uint8_t *in, uint64_t n_in, UnpackPlan *up, const uint64_t *caps) {
  __shared__ __align__(4) uint8_t lens[4][256];
  __shared__ uint64_t tab_at[4];
  __shared__ int ok;
  const int tid = threadIdx.x;
  if (tid == 0) {
    uint32_t err = 0;
    for (int q = 0; q < 4; q++) {
      up->nbytes[q] = up->nbits[q] = up->bit0[q] = 0;
      tab_at[q] = 0;
    }
    if (n_in < kHeaderBytes || rd_u32(in) != kMagic) {
      err = 1;
    } else {
      up->kind = in[4];
      up->th = in[5];
      up->tw = in[6];
      up->H = in[8] | (in[9] << 8);
      up->W = in[10] | (in[11] << 8);
      for (int e = 0; e < 12; e++) up->M[e] = __uint_as_float(rd_u32(in + 64 + 4 * e));
      uint64_t at = kHeaderBytes;
      for (int q = 0; q < 4 && !err; q++) {
        uint64_t nb = 0;
        for (int i = 0; i < 8; i++) nb |= (uint64_t)in[12 + 8 * q + i] << (8 * i);
        const uint64_t pb = rd_u32(in + 44 + 4 * q);
        up->nbytes[q] = nb;
        if (nb == 0) {
          if (pb) err = 1;
          continue;
        }
        if (nb > caps[q] || at + kTableBytes + pb > n_in) {
          err = 1;
          break;
        }
        tab_at[q] = at;
        at += kTableBytes;
        up->bit0[q] = 8 * at;
        up->nbits[q] = 8 * pb;
        at += pb;
      }
      if (at != n_in) err = 1;
    }
    up->err = err;
    ok = err == 0;
  }
  __syncthreads();
  if (!ok) return;
  for (int e = tid; e < 1024; e += blockDim.x) {
    const int q = e >> 8, sym = e & 255;
    lens[q][sym] = up->nbytes[q] ? (uint8_t)((in[tab_at[q] + sym / 2] >> (4 * (sym & 1))) & 15) : (uint8_t)0;
  }
  __syncthreads();
  // canonical code tables, one stream at a time by the wavefront: lane l
  // holds the lengths of symbols 4l .. 4l + 3, and for each length in turn
  // a wavefront scan of the lanes' counts places those symbols in symbol
  // order after the shorter ones (the canonical order) and gives the count
  // of the length, from which the first code, index and limit follow
  const int lane = tid & 63;
  for (int q = 0; q < 4 && tid < 64; q++) {
    if (!up->nbytes[q]) continue;
    const uint32_t l4 = reinterpret_cast<const uint32_t *>(lens[q])[lane];
    uint32_t code = 0, idx = 0, used = 0, c1 = 0;
    uint64_t kraft = 0;
    for (int L = 1; L <= kMaxLen; L++) {
      uint32_t mine = 0;
#pragma unroll
      for (int j = 0; j < 4; j++) mine += ((l4 >> (8 * j)) & 255u) == (uint32_t)L ? 1u : 0u;
      uint32_t x = mine;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
        if (lane >= o) x += y;
      }
      const uint32_t total = (uint32_t)__shfl((int)x, 63, 64);
      uint32_t at = idx + x - mine;
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (((l4 >> (8 * j)) & 255u) == (uint32_t)L) up->sorted[q][at++] = (uint8_t)(4 * lane + j);
      if (lane == 0) {
        up->first[q][L] = code;
        up->index[q][L] = idx;
        up->limit[q][L] = (code + total) << (kMaxLen - L);
      }
      kraft += (uint64_t)total << (kMaxLen - L);
      used += total;
      if (L == 1) c1 = total;
      idx += total;
      code = (code + total) << 1;
    }
    if (lane == 0) {
      up->limit[q][0] = 0;
      // a complete code, or one symbol coded with one bit
      if (!(kraft == (1ull << kMaxLen) || (used == 1 && c1 == 1))) atomicOr(&up->err, 1u);
    }
  }
}

constexpr int kFastBits = 13;               // code words this short decode with one table lookup (16 KB of LDS)

struct DecTab {
  uint32_t limit[kMaxLen + 1], first[kMaxLen + 1], index[kMaxLen + 1];
  uint8_t sorted[256];
  // by the first kFastBits bits of a code word: symbol | length << 8 when
  // the word is at most kFastBits long, else 0
  uint16_t fast[1 << kFastBits];
};

// Payload reads of one stream: from its LDS copy (whole little-endian
// words, zero past the payload) or, for a payload too large to copy, from
// device memory byte by byte (clamped loads, zero past the payload).
template <bool LDS>
struct PayRead {
  const __attribute__((address_space(3))) uint32_t *w;
  const __attribute__((address_space(1))) uint8_t *g;
  uint32_t nbytes;
  // the 15 bits from payload bit p, MSB first
  __device__ __forceinline__ uint32_t peek15(uint32_t p) const {
    const uint32_t B = p >> 3;
    uint32_t x;
    if (LDS) {
      const uint32_t W0 = B >> 2;
      const uint64_t v = ((uint64_t)w[W0 + 1] << 32) | w[W0];
      x = __builtin_bswap32((uint32_t)(v >> (8 * (B & 3))));
    } else {
      x = 0;
#pragma unroll
      for (int j = 0; j < 3; j++) {
        const uint32_t i = B + j, b = g[min(i, nbytes - 1)];
        x = (x << 8) | (i < nbytes ? b : 0u);
      }
      x <<= 8;
    }
    return ((x << (p & 7)) >> 17) & 0x7fffu;
  }
};

// Length of the code word at the head of win: canonical limits (left
// justified to 15 bits) never decrease with the length, so the length is
// one more than the number of limits at or below win.  lim: the stream's
// limits in registers.
__device__ __forceinline__ int code_len(const uint32_t (&lim)[kMaxLen + 1], uint32_t win, uint32_t *bad) {
  int L = 1;
#pragma unroll
  for (int l = 1; l <= kMaxLen; l++) L += win >= lim[l] ? 1 : 0;
  if (L > kMaxLen) {
    *bad = 1;
    return 1;
  }
  return L;
}

// Decodes subsequence j from payload bit `s`: code words starting before
// min((j + 1) S, nbits).  Returns the end bit and the code word count.
template <class Pay>
__device__ __forceinline__ void decode_sub(const uint32_t (&lim)[kMaxLen + 1],
                                           const __attribute__((address_space(3))) uint16_t *fast, const Pay &pay,
                                           uint32_t lim_bit, uint32_t s, uint32_t *end, uint32_t *cnt, uint32_t *bad) {
  uint32_t p = s, c = 0;
  while (p < lim_bit) {
    const uint32_t win = pay.peek15(p);
    const uint32_t e = fast[win >> (kMaxLen - kFastBits)];
    p += e ? (e >> 8) : code_len(lim, win, bad);
    c++;
  }
  *end = p;
  *cnt = c;
}

// The subsequences of one stream (the part of unpack_stream after its
// payload and tables are in place): decode from guessed starts, redo those
// whose start differs from the predecessor's end until none changes, then
// write the symbols at the prefix of the counts.  st, en: subsequence
// starts and ends (bits), cnt: code words.
template <class Pay>
__device__ __forceinline__ void decode_stream(const Pay &pay, const DecTab &t, uint32_t nbits, uint64_t n,
                                              uint32_t *st, uint32_t *en, uint32_t *cnt, uint8_t *out, uint32_t *red,
                                              int *any, uint32_t *err) {
  const int tid = threadIdx.x;
  uint32_t lim[kMaxLen + 1];
#pragma unroll
  for (int L = 0; L <= kMaxLen; L++) lim[L] = __builtin_amdgcn_readfirstlane(t.limit[L]);   // uniform: scalar registers
  typedef const __attribute__((address_space(3))) uint16_t lds_u16;
  lds_u16 *fast = (lds_u16 *)t.fast;
  uint32_t S = (nbits + kMaxSub - 1) / kMaxSub;
  S = S < kMinSubBits ? kMinSubBits : S;
  // an odd number of 32-bit words per subsequence: neighbouring lanes then
  // read the LDS payload an odd number of words apart, which spreads them
  // over the banks (at 8 words apart, 16 lanes share a bank)
  S = (((S + 31u) / 32u) | 1u) * 32u;
  const uint32_t m = (nbits + S - 1) / S;
  const uint32_t per = (m + kUnpackBlock - 1) / kUnpackBlock;
  const uint32_t j0 = min(m, tid * per), j1 = min(m, j0 + per);
  uint32_t bad = 0;
  for (uint32_t j = j0; j < j1; j++) {
    st[j] = j * S;
    decode_sub(lim, fast, pay, min((j + 1) * S, nbits), st[j], &en[j], &cnt[j], &bad);
  }
  // a start that differs from its predecessor's end is decoded again; the
  // verified prefix grows by at least one thread's share per round
  for (uint32_t round = 0; round <= kUnpackBlock; round++) {
    __syncthreads();
    const uint32_t snap = (j0 > 0 && j0 < j1) ? en[j0 - 1] : 0;
    if (tid == 0) *any = 0;
    __syncthreads();
    int changed = 0;
    for (uint32_t j = j0; j < j1; j++) {
      const uint32_t s = j == 0 ? 0 : (j == j0 ? snap : en[j - 1]);
      if (s != st[j]) {
        st[j] = s;
        decode_sub(lim, fast, pay, min((j + 1) * S, nbits), s, &en[j], &cnt[j], &bad);
        changed = 1;
      }
    }
    if (changed) *any = 1;
    __syncthreads();
    if (!*any) break;
  }
  uint32_t mine = 0;
  for (uint32_t j = j0; j < j1; j++) mine += cnt[j];
  uint32_t total;
  uint64_t idx = block_excl_scan(mine, red, &total);
  // a lane's symbols are consecutive bytes of out: they are gathered into
  // 32-bit words and stored whole where the lane owns the whole aligned word
  // (within the n bytes), byte by byte at its two ends
  const uint32_t a0 = (uint32_t)(reinterpret_cast<uintptr_t>(out) & 3u);
  uint64_t wbeg = idx;
  uint32_t acc = 0;
  auto flush = [&](uint64_t e) {
    if (((a0 + wbeg) & 3u) == 0 && e == wbeg + 4 && e <= n) {
      *reinterpret_cast<uint32_t *>(out + wbeg) = acc;
    } else {
      for (uint64_t i = wbeg; i < e; i++)
        if (i < n) out[i] = (uint8_t)(acc >> (8u * ((a0 + (uint32_t)i) & 3u)));
    }
    acc = 0;
    wbeg = e;
  };
  for (uint32_t j = j0; j < j1; j++) {
    uint32_t p = st[j];
    const uint32_t lim_bit = min((j + 1) * S, nbits);
    while (p < lim_bit) {
      const uint32_t win = pay.peek15(p);
      const uint32_t e = fast[win >> (kMaxLen - kFastBits)];
      int L;
      uint32_t sym;
      if (e) {
        L = (int)(e >> 8);
        sym = e & 255u;
      } else {
        L = code_len(lim, win, &bad);
        sym = t.sorted[t.index[L] + ((win >> (kMaxLen - L)) - t.first[L])];
      }
      acc |= sym << (8u * ((a0 + (uint32_t)idx) & 3u));
      idx++;
      if (((a0 + (uint32_t)idx) & 3u) == 0) flush(idx);
      p += L;
    }
  }
  if (idx > wbeg) flush(idx);
  if (tid == 0 && total < n) bad = 1;
  if (bad) atomicOr(err, 2u);
}

// Stream q of one container, by one work-group.
__device__ __forceinline__ void unpack_stream(int q, const uint8_t *in, UnpackPlan *up, uint64_t *sub, uint32_t *subc,
                                              const StreamPtrs &outp) {
  __shared__ DecTab t;
  __shared__ uint32_t red[16];
  __shared__ int any, skip;
  const int tid = threadIdx.x;
  // other streams may raise up->err meanwhile: decide once for the group
  if (tid == 0) skip = (up->err & 1u) != 0;
  __syncthreads();
  if (skip) return;
  const uint64_t n = up->nbytes[q], nbits = up->nbits[q];
  if (n == 0) return;
  for (int L = tid; L <= kMaxLen; L += kUnpackBlock) {
    t.limit[L] = up->limit[q][L];
    t.first[L] = up->first[q][L];
    t.index[L] = up->index[q][L];
  }
  for (int s = tid; s < 256; s += kUnpackBlock) t.sorted[s] = up->sorted[q][s];
  __syncthreads();
  for (int e = tid; e < (1 << kFastBits); e += kUnpackBlock) {
    const uint32_t win = (uint32_t)e << (kMaxLen - kFastBits);
    int L = 1;
    while (L <= kMaxLen && win >= t.limit[L]) L++;
    t.fast[e] = L <= kFastBits ? (uint16_t)(t.sorted[t.index[L] + ((win >> (kMaxLen - L)) - t.first[L])] | (L << 8))
                               : (uint16_t)0;
  }
  __syncthreads();
  const uint8_t *gpay = in + up->bit0[q] / 8;
  const uint64_t pbytes = nbits / 8;
  if (nbits > 0xFFFFFF00ull) {                 // positions are 32-bit
    if (tid == 0) atomicOr(&up->err, 2u);
    return;
  }
  // a payload that fits is staged in LDS (with eight zero bytes after it):
  // every code word costs dependent reads of its bytes, which LDS serves
  // several times faster
  __shared__ __align__(16) uint8_t paybuf[kPayLds + 8];
  const bool staged = pbytes <= (uint64_t)kPayLds;
  if (staged) {
    for (uint32_t i = tid; i < (uint32_t)pbytes; i += kUnpackBlock) paybuf[i] = gpay[i];
    if (tid < 8) paybuf[pbytes + tid] = 0;
  }
  __syncthreads();
  uint32_t *st = reinterpret_cast<uint32_t *>(sub) + (int64_t)q * 2 * kMaxSub, *en = st + kMaxSub;
  uint32_t *cnt = subc + (int64_t)q * kMaxSub;
  typedef const __attribute__((address_space(3))) uint32_t lds_u32;
  typedef const __attribute__((address_space(1))) uint8_t glb_u8;
  if (staged)
    decode_stream(PayRead<true>{(lds_u32 *)paybuf, (glb_u8 *)gpay, (uint32_t)pbytes}, t, (uint32_t)nbits, n, st, en, cnt,
                  outp.p[q], red, &any, &up->err);
  else
    decode_stream(PayRead<false>{(lds_u32 *)paybuf, (glb_u8 *)gpay, (uint32_t)pbytes}, t, (uint32_t)nbits, n, st, en,
                  cnt, outp.p[q], red, &any, &up->err);
}

// Streams back into a frame stream buffer: occupancy words, runs and tile
// classes, masks, residual codes per strip.  One work-group.
__device__ __forceinline__ void unpack_frame(UnpackPlan *up, const StreamPtrs &sp, const FrameDev &f,
                                             const FrameDev &key, int has_key, int th, int tw, int W) {
  __shared__ uint32_t red[16];
  __shared__ uint32_t err;
  __shared__ uint32_t rowcnt[1024], rowoff[1024];
  __shared__ uint32_t base;
  if (up->err) return;
  const int tid = threadIdx.x, TR = f.TR, TC = f.TC, T = f.T, H = TR * th;
  const int kind = up->kind;
  if (tid == 0) err = 0;
  const int64_t nw = (int64_t)H * W / 32;
  if (up->nbytes[S_OCC] != (uint64_t)nw * 4 || up->nbytes[S_RES] % 2) {
    if (tid == 0) atomicOr(&up->err, 4u);
    return;
  }
  const uint8_t *ob = sp.p[S_OCC];
  for (int64_t w = tid; w < nw; w += kUnpackBlock) f.occ[w] = rd_u32(ob + 4 * w);
  __syncthreads();
  const uint32_t lowm = (uint32_t)((1ull << tw) - 1ull);
  auto valid_bits = [&](int64_t t) {
    const int tr = (int)(t / TC), tc = (int)(t % TC);
    const uint32_t *occ = f.occ + (int64_t)tr * (th * W / 32);
    uint64_t V = 0;
    for (int i = 0; i < th; i++) {
      const int bit = i * W + tc * tw;
      V |= (uint64_t)((occ[bit >> 5] >> (bit & 31)) & lowm) << (i * tw);
    }
    return V;
  };
  for (int64_t t = tid; t < T; t += kUnpackBlock) {
    f.cls[t] = valid_bits(t) ? CLS_UNFIT : CLS_EMPTY;
    f.run_of[t] = -1;
    f.mask[t] = 0;
  }
  // Runs of each tile row, in stream order.  The table has no index
  // (variable-length fields), so one thread first walks it to find where
  // each tile row starts, reading only the bytes that give a record's
  // length (the lead bytes of its two varints: a temporal record is gap,
  // len and one FP32 value, a spatial one gap, len, an axis byte and three
  // FP32 values); then one thread per tile row decodes its records.
  // Counts, gaps and lengths are at most TC, so their varints take one or
  // two bytes (a longer one is malformed).  A table that fits is staged in
  // LDS first.
  __shared__ __align__(16) uint8_t runbuf[kRunLds];
  __shared__ uint32_t rowstart[1025];
  __shared__ uint32_t recp[kMaxRec], recid[kMaxRec];   // start and (spatial << 31 | row << 13 | k) of every record
  __shared__ int nsr_s, npr_s, nrec;
  const uint64_t nrun = up->nbytes[S_RUN];
  const bool staged = nrun <= (uint64_t)kRunLds;
  if (staged)
    for (uint32_t i = tid; i < (uint32_t)nrun; i += kUnpackBlock) runbuf[i] = sp.p[S_RUN][i];
  __syncthreads();
  // byte q of the table, zero past its end: from LDS when staged (a
  // table larger than the LDS copy is only read from device memory), with
  // typed pointers so that each path is a plain LDS or global load
  typedef const __attribute__((address_space(3))) uint8_t lds_u8;
  typedef const __attribute__((address_space(1))) uint8_t glb_u8;
  const lds_u8 *RL = (lds_u8 *)runbuf;
  const glb_u8 *RG = (glb_u8 *)sp.p[S_RUN];
  const uint32_t n = (uint32_t)nrun;
  auto rbyte = [&](uint32_t q) -> uint32_t {
    const uint32_t v = staged ? (uint32_t)RL[min(q, (uint32_t)kRunLds - 1u)] : (uint32_t)RG[min(q, n - 1u)];
    return q < n ? v : 0u;
  };
  if (nrun > 0xFFFFFFF0ull && tid == 0) err |= 4u;
  if (tid < 64) {
    // the walk, by wavefront 0: lane l holds byte wb + l of a 64-byte
    // window and the length of the two varints that would start there
    // (0 when one is longer than two bytes); a record then costs one
    // readlane at the wave-uniform offset p - wb
    const int lane = tid;
    uint32_t wb = 0, b0 = 0, b1 = 0, lead = 0;
    auto load = [&](uint32_t at) {
      wb = at;
      const uint32_t q = at + lane;
      b0 = rbyte(q);
      b1 = rbyte(q + 1);
      const uint32_t b2 = rbyte(q + 2), b3 = rbyte(q + 3);
      const int lg = (b0 & 128u) ? 2 : 1;
      const uint32_t l0 = lg == 1 ? b1 : b2, l1 = lg == 1 ? b2 : b3;
      const int ll = (l0 & 128u) ? 2 : 1;
      lead = ((lg == 2 && (b1 & 128u)) || (ll == 2 && (l1 & 128u))) ? 0u : (uint32_t)(lg + ll);
    };
    auto at = [&](uint32_t v, uint32_t q) -> uint32_t {     // lane q - wb's v (q uniform, inside the window)
      return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)(q - wb));
    };
    load(0);
    uint32_t p = 0, bad = 0, nr = 0;
    if (lane == 0) nsr_s = npr_s = 0;
    for (int tr = 0; tr < TR && !bad; tr++) {
      if (lane == 0) rowstart[tr] = p;
      for (int sec = kind ? 0 : 1; sec < 2 && !bad; sec++) {      // temporal runs, then spatial
        if (p - wb >= 64) load(p);
        const uint32_t c0 = at(b0, p), c1 = at(b1, p);
        const uint32_t cnt = (c0 & 128u) ? ((c0 & 127u) | (c1 << 7)) : c0;
        if (((c0 & 128u) && (c1 & 128u)) || cnt > (uint32_t)TC) bad = 1;
        p += (c0 & 128u) ? 2 : 1;
        const uint32_t fixed = sec == 0 ? 4 : 13;
        for (uint32_t k = 0; k < cnt && !bad; k++) {
          if (p - wb >= 64) load(p);
          const uint32_t L = at(lead, p);
          if (!L) bad = 1;
          if (lane == 0 && nr < kMaxRec) {
            recp[nr] = p;
            recid[nr] = ((uint32_t)sec << 31) | ((uint32_t)tr << 13) | k;
          }
          nr++;
          p += L + fixed;
          if (p > n) bad = 1;
        }
        if (lane == 0) (sec ? nsr_s : npr_s) += (int)cnt;
        if (lane == 0) f.nruns[sec ? tr : TR + tr] = (int32_t)cnt;
      }
      if (!kind && lane == 0) f.nruns[TR + tr] = 0;
    }
    if (lane == 0) {
      rowstart[TR] = p;
      nrec = (int)nr;
      if (bad || p != n) err |= 4u;
    }
  }
  __syncthreads();
  if (!err && nrec <= kMaxRec) {
    // every record by its own thread: the fields follow the two varints at
    // offset 2, 3 or 4 and are taken by selects on that offset; runs must
    // lie inside the row in order (the previous record of the row gives
    // where the previous run ended)
    for (int e = tid; e < nrec; e += kUnpackBlock) {
      const uint32_t q = recp[e], id = recid[e];
      const int sp_ = (int)(id >> 31), tr = (int)((id >> 13) & 1023u), k = (int)(id & 8191u);
      uint32_t b[17];
#pragma unroll
      for (int j = 0; j < 17; j++) b[j] = rbyte(q + j);
      const bool g2 = (b[0] & 128u) != 0;
      const uint32_t gap = g2 ? ((b[0] & 127u) | (b[1] << 7)) : b[0];
      const uint32_t l0 = g2 ? b[2] : b[1], l1 = g2 ? b[3] : b[2];
      const bool l2 = (l0 & 128u) != 0;
      const uint32_t len = l2 ? ((l0 & 127u) | (l1 << 7)) : l0;
      const int o = (g2 ? 2 : 1) + (l2 ? 2 : 1);
      auto field = [&](int j) -> uint32_t { return o == 2 ? b[2 + j] : (o == 3 ? b[3 + j] : b[4 + j]); };
      auto u32f = [&](int j) -> uint32_t {
        return field(j) | (field(j + 1) << 8) | (field(j + 2) << 16) | (field(j + 3) << 24);
      };
      if (gap > (uint32_t)TC || len < 1 || len > (uint32_t)TC) atomicOr(&err, 4u);
      if (sp_) {
        const uint32_t axis = field(0);
        if (axis > 2) atomicOr(&err, 4u);
        f.sruns[(int64_t)tr * TC + k] = pc_run{(int)gap, (int)len, (int)axis, __uint_as_float(u32f(1)),
                                             __uint_as_float(u32f(5)), __uint_as_float(u32f(9))};
      } else {
        f.pruns[(int64_t)tr * TC + k] = pc_prun{(int)gap, (int)len, -1, __uint_as_float(u32f(0))};   // key slot filled below
      }
    }
    __syncthreads();
    // gaps to starts, a row and kind per thread (runs in order, inside the row)
    for (int e = tid; e < 2 * TR && !err; e += kUnpackBlock) {
      const int tr = e >> 1, sp_ = e & 1;
      const int cnt = f.nruns[sp_ ? tr : TR + tr];
      int prev = 0;
      for (int k = 0; k < cnt; k++) {
        const int64_t slot = (int64_t)tr * TC + k;
        const int gap = sp_ ? f.sruns[slot].s : f.pruns[slot].s, len = sp_ ? f.sruns[slot].len : f.pruns[slot].len;
        if (prev + gap + len > TC) {
          atomicOr(&err, 4u);
          break;
        }
        if (sp_) f.sruns[slot].s = prev + gap;
        else f.pruns[slot].s = prev + gap;
        prev += gap + len;
      }
    }
  }
  __syncthreads();
  // (a table of more than kMaxRec records) the rows, a thread each: a
  // record's bytes are fetched together and its fields, which follow the
  // two varints at offset 2, 3 or 4, taken by selects on that offset
  for (int tr = tid; tr < TR && !err && nrec > kMaxRec; tr += kUnpackBlock) {
    uint32_t p = rowstart[tr];
    const uint32_t end = rowstart[tr + 1];
    uint32_t bad = 0;
    auto count = [&]() -> uint32_t {
      const uint32_t c0 = rbyte(p), c1 = rbyte(p + 1);
      p += (c0 & 128u) ? 2 : 1;
      return (c0 & 128u) ? ((c0 & 127u) | (c1 << 7)) : c0;
    };
    // gap and len of the record at p; o = their bytes
    auto lead2 = [&](const uint32_t *b, uint32_t &gap, uint32_t &len, int &o) {
      const bool g2 = (b[0] & 128u) != 0;
      gap = g2 ? ((b[0] & 127u) | (b[1] << 7)) : b[0];
      const uint32_t l0 = g2 ? b[2] : b[1], l1 = g2 ? b[3] : b[2];
      const bool l2 = (l0 & 128u) != 0;
      len = l2 ? ((l0 & 127u) | (l1 << 7)) : l0;
      o = (g2 ? 2 : 1) + (l2 ? 2 : 1);
    };
    auto field = [&](const uint32_t *b, int o, int j) -> uint32_t {   // byte o + j, o in {2, 3, 4}
      return o == 2 ? b[2 + j] : (o == 3 ? b[3 + j] : b[4 + j]);
    };
    auto u32f = [&](const uint32_t *b, int o, int j) -> uint32_t {
      return field(b, o, j) | (field(b, o, j + 1) << 8) | (field(b, o, j + 2) << 16) | (field(b, o, j + 3) << 24);
    };
    int np = 0;
    if (kind) {
      np = (int)count();
      int prev = 0;
      for (int k = 0; k < np && !bad; k++) {
        uint32_t b[8];
#pragma unroll
        for (int j = 0; j < 8; j++) b[j] = rbyte(p + j);
        uint32_t gap, len;
        int o;
        lead2(b, gap, len, o);
        const float c = __uint_as_float(u32f(b, o, 0));
        p += o + 4;
        if (p > end || gap > (uint32_t)TC || len < 1 || len > (uint32_t)TC || prev + (int)gap + (int)len > TC) {
          bad = 1;
          break;
        }
        const int s0 = prev + (int)gap;
        f.pruns[(int64_t)tr * TC + k] = pc_prun{s0, (int)len, -1, c};      // key slot filled below
        prev = s0 + (int)len;
      }
    }
    f.nruns[TR + tr] = np;
    const int ns = bad ? 0 : (int)count();
    int prev = 0;
    for (int k = 0; k < ns && !bad; k++) {
      uint32_t b[17];
#pragma unroll
      for (int j = 0; j < 17; j++) b[j] = rbyte(p + j);
      uint32_t gap, len;
      int o;
      lead2(b, gap, len, o);
      const uint32_t axis = field(b, o, 0);
      const float fa = __uint_as_float(u32f(b, o, 1)), fb = __uint_as_float(u32f(b, o, 5)),
                  fc = __uint_as_float(u32f(b, o, 9));
      p += o + 13;
      if (p > end || gap > (uint32_t)TC || len < 1 || len > (uint32_t)TC || prev + (int)gap + (int)len > TC ||
          axis > 2) {
        bad = 1;
        break;
      }
      const int s0 = prev + (int)gap;
      f.sruns[(int64_t)tr * TC + k] = pc_run{s0, (int)len, (int)axis, fa, fb, fc};
      prev = s0 + (int)len;
    }
    f.nruns[tr] = ns;
    if (bad || p != end) atomicOr(&err, 4u);
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < (int)sizeof(pc_frame_info); i++) ((uint8_t *)f.info)[i] = 0;
    f.info->kind = kind;
    f.info->status = 0;
    for (int e = 0; e < 12; e++) f.info->M[e] = up->M[e];
    f.info->n_sruns = nsr_s;
    f.info->n_pruns = npr_s;
    for (int q = 0; q < 4; q++) f.info->stream_bytes[q] = up->nbytes[q];
  }
  __syncthreads();
  if (err) {
    if (tid == 0) atomicOr(&up->err, err);
    return;
  }
  // the runs' tiles, a run per thread: temporal runs take the key frame's
  // run slot at their first tile and must stay inside that key run (a
  // temporal run reuses one key plane, Sec. III-D); spatial runs must not
  // cover a temporal tile (slots r*TC + k, so slot e is row e / TC, run e % TC)
  for (int64_t e = tid; e < T; e += kUnpackBlock) {
    const int tr = (int)(e / TC), k = (int)(e % TC);
    if (!kind || k >= f.nruns[TR + tr]) continue;
    const pc_prun R = f.pruns[e];
    const int64_t t0 = (int64_t)tr * TC + R.s;
    const int kr = has_key ? key.run_of[t0] : -1;
    if (kr < 0 || kr >= T) {
      atomicOr(&err, 4u);
      continue;
    }
    f.pruns[e].krun = kr;
    for (int q = 0; q < R.len; q++) {
      if (key.run_of[t0 + q] != kr) atomicOr(&err, 4u);
      f.cls[t0 + q] = CLS_TEMPORAL;
      f.run_of[t0 + q] = (int32_t)(T + e);
    }
  }
  __syncthreads();
  for (int64_t e = tid; e < T; e += kUnpackBlock) {
    const int tr = (int)(e / TC), k = (int)(e % TC);
    if (k >= f.nruns[tr]) continue;
    const pc_run R = f.sruns[e];
    const int64_t t0 = (int64_t)tr * TC + R.s;
    for (int q = 0; q < R.len; q++) {
      if (f.cls[t0 + q] == CLS_TEMPORAL) atomicOr(&err, 4u);
      f.cls[t0 + q] = CLS_SPATIAL;
      f.run_of[t0 + q] = (int32_t)e;
    }
  }
  __syncthreads();
  if (err) {
    if (tid == 0) atomicOr(&up->err, err);
    return;
  }
  // masks of the plane-coded tiles, in tile order
  const uint8_t *Mb = sp.p[S_MASK];
  const uint64_t nmask = up->nbytes[S_MASK];
  if (tid == 0) base = 0;
  for (int64_t c0 = 0; c0 < T; c0 += kUnpackBlock) {
    __syncthreads();
    const int64_t t = c0 + tid;
    uint64_t V = 0;
    uint32_t nb = 0;
    bool cov = false;
    if (t < T) {
      const int c = f.cls[t];
      cov = c == CLS_SPATIAL || c == CLS_TEMPORAL;
      if (cov) {
        V = valid_bits(t);
        nb = (__popcll(V) + 7) >> 3;
      }
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(nb, red, &tot);
    const uint64_t at = (uint64_t)base + ex;
    if (cov) {
      if (at + nb > nmask) {
        atomicOr(&err, 4u);
      } else {
        uint64_t bits = 0;
        for (uint32_t b = 0; b < nb; b++) bits |= (uint64_t)Mb[at + b] << (8 * b);
        uint64_t M = 0;
        int k = 0;
        for (uint64_t v = V; v; v &= v - 1, k++) M |= ((bits >> k) & 1ull) << __builtin_ctzll(v);
        f.mask[t] = M;
      }
    }
    __syncthreads();
    if (tid == 0) base += tot;
  }
  __syncthreads();
  if (tid == 0 && base != nmask) err |= 4u;
  // residual codes: uncovered valid pixels of each image row, raster order;
  // each stream value is the zigzag difference (mod 2^16) from the row's
  // previous code, so every row is rebuilt by one thread from its start
  for (int h = tid; h < H; h += kUnpackBlock) rowcnt[h] = 0;
  __syncthreads();
  for (int64_t t = tid; t < T; t += kUnpackBlock) {
    const uint64_t R = valid_bits(t) & ~f.mask[t];
    const int tr = (int)(t / TC);
    for (int i = 0; i < th; i++) {
      const uint32_t c = (uint32_t)__popcll((R >> (i * tw)) & lowm);
      if (c) atomicAdd(&rowcnt[tr * th + i], c);
    }
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t s = 0;
    for (int h = 0; h < H; h++) {
      rowoff[h] = s;
      s += rowcnt[h];
    }
    for (int r = 0; r < TR; r++) {
      const uint32_t end = r + 1 < TR ? rowoff[(r + 1) * th] : s;
      f.nres[r] = (int32_t)(end - rowoff[r * th]);
    }
    if ((uint64_t)s * 2 != up->nbytes[S_RES]) err |= 4u;
    f.info->n_res = s;
  }
  __syncthreads();
  if (err) {
    if (tid == 0) atomicOr(&up->err, err);
    return;
  }
  // each row's codes are the prefix sums (mod 2^16) of its differences, so
  // a wavefront rebuilds a row 64 codes at a time with a scan (additions
  // mod 2^32 wrap consistently with mod 2^16)
  const uint8_t *Rb = sp.p[S_RES];
  const int lane = tid & 63;
  for (int h = tid >> 6; h < H; h += kUnpackBlock / 64) {
    const int r = h / th;
    const uint32_t b = rowoff[h], c = rowcnt[h], in_strip = b - rowoff[r * th];
    uint16_t *dst = f.res + (int64_t)r * th * W + in_strip;
    uint32_t carry = 0;
    for (uint32_t j0 = 0; j0 < c; j0 += 64) {
      const uint32_t j = j0 + lane;
      uint32_t x = 0;
      if (j < c) {
        const uint32_t z = Rb[2 * (b + j)] | ((uint32_t)Rb[2 * (b + j) + 1] << 8);
        x = (z >> 1) ^ ((z & 1u) ? 0xFFFFu : 0u);
      }
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (j < c) dst[j] = (uint16_t)((carry + x) & 0xFFFFu);
      carry += __shfl(x, 63, 64);
    }
  }
}

// One container's decoding job (batched unpacking).
struct UnpackJob {
  const uint8_t *in;
  uint64_t n_in;
  UnpackPlan *up;
  uint64_t *sub;
  uint32_t *subc;
  const uint64_t *caps;
  StreamPtrs sp;
  FrameDev f, key;
  int has_key;
};

__global__ void k_unpack_plan(const uint8_t *in, uint64_t n_in, UnpackPlan *up, const uint64_t *caps) {
  unpack_plan(in, n_in, up, caps);
}
__global__ void k_unpack_plan_b(const UnpackJob *jobs) {
  const UnpackJob &J = jobs[blockIdx.x];
  unpack_plan(J.in, J.n_in, J.up, J.caps);
}

// One work-group per stream (and container).
__global__ void __launch_bounds__(kUnpackBlock) k_unpack_streams(const uint8_t *in, UnpackPlan *up, uint64_t *sub,
                                                                uint32_t *subc, StreamPtrs outp) {
  unpack_stream(blockIdx.x, in, up, sub, subc, outp);
}
// blockIdx.x is the container and 3 - blockIdx.y the stream: consecutive
// work-groups go to different XCDs, so each XCD gets every stream kind
// (with the stream as the fast index, the long residual streams all landed
// on two of the eight), and the residual streams, the longest, start first.
__global__ void __launch_bounds__(kUnpackBlock) k_unpack_streams_b(const UnpackJob *jobs) {
  const UnpackJob &J = jobs[blockIdx.x];
  unpack_stream(3 - (int)blockIdx.y, J.in, J.up, J.sub, J.subc, J.sp);
}

__global__ void __launch_bounds__(kUnpackBlock) k_unpack_frame(UnpackPlan *up, StreamPtrs sp, FrameDev f,
                                                              FrameDev key, int has_key, int th, int tw, int W) {
  unpack_frame(up, sp, f, key, has_key, th, tw, W);
}
// Containers of kind `pass` (0 key frames first, then 1 predicted frames,
// which read their key frames' run slots), after checking the header's
// sensor size and tile shape and that a predicted frame has a key frame.
__global__ void __launch_bounds__(kUnpackBlock) k_unpack_frame_b(const UnpackJob *jobs, int pass, int H, int W, int th,
                                                                int tw) {
  const UnpackJob &J = jobs[blockIdx.x];
  UnpackPlan *up = J.up;
  __shared__ int go;
  if (threadIdx.x == 0) {
    int g = 0;
    if (!up->err && pass == 0 && up->kind != 0 && up->kind != 1) up->err |= 8u;
    if (!up->err && up->kind == pass) {
      if (up->H != H || up->W != W || up->th != th || up->tw != tw)
        up->err |= 8u;
      else if (pass == 1 && !J.has_key)
        up->err |= 16u;
      else
        g = 1;
    }
    go = g;
  }
  __syncthreads();
  if (!go) return;
  unpack_frame(up, J.sp, J.f, J.key, J.has_key, th, tw, W);
}

// Per container: error bits in the low 16 bits, kind in the next 8.
__global__ void k_unpack_status(const UnpackJob *jobs, int n, uint32_t *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) status[i] = (jobs[i].up->err & 0xFFFFu) | ((uint32_t)(jobs[i].up->kind & 0xFF) << 16);
}

// ------------------------------------------------------------------ sizing
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct FrameCaps {
  uint64_t c[4];
};
FrameCaps frame_caps(const pc_layout &L) {
  FrameCaps k;
  k.c[S_OCC] = (uint64_t)L.H * L.W / 8;
  k.c[S_RUN] = (uint64_t)L.TR * (4 + 17 * (uint64_t)L.TC);
  k.c[S_MASK] = 8 * (uint64_t)L.T;
  k.c[S_RES] = 2 * (uint64_t)L.H * L.W;
  return k;
}
uint64_t bound_of(const uint64_t *n) {
  uint64_t b = kHeaderBytes;
  for (int q = 0; q < 4; q++)
    if (n[q]) b += kTableBytes + (kMaxLen * n[q] + 7) / 8;
  return (b + 255) & ~(uint64_t)255;
}
size_t pack_ws(int max_seg, bool raw) {
  size_t b = a256(sizeof(PackPlan)) + a256(sizeof(SegInfo) * 4 * (size_t)max_seg);
  if (raw) b += a256(sizeof(uint32_t) * 256 * 4 * (size_t)max_seg);
  return b;
}
size_t unpack_ws() {
  return a256(sizeof(UnpackPlan)) + a256(sizeof(uint64_t) * 8 * kMaxSub) + a256(sizeof(uint32_t) * 4 * kMaxSub) +
         a256(sizeof(uint64_t) * 4);
}
size_t frame_ws(const pc_layout &L) {
  FrameCaps k = frame_caps(L);
  size_t u = unpack_ws();
  for (int q = 0; q < 4; q++) u += a256(k.c[q]);
  size_t p = pack_ws(L.TR, false);
  return p > u ? p : u;
}
int raw_segs(const uint64_t *n) {
  uint64_t m = 1;
  for (int q = 0; q < 4; q++) {
    uint64_t s = (n[q] + kChunk - 1) / kChunk;
    m = s > m ? s : m;
  }
  return (int)m;
}

// Decode the streams of a container into `outp` (device).  Synchronises.
pc_status unpack_to_streams(const uint8_t *in, uint64_t n_in, char *ws, const uint64_t *caps, const StreamPtrs &outp,
                            UnpackPlan *host, hipStream_t st) {
  UnpackPlan *up = (UnpackPlan *)ws;
  char *w = ws + a256(sizeof(UnpackPlan));
  uint64_t *sub = (uint64_t *)w;
  w += a256(sizeof(uint64_t) * 8 * kMaxSub);
  uint32_t *subc = (uint32_t *)w;
  w += a256(sizeof(uint32_t) * 4 * kMaxSub);
  uint64_t *dcaps = (uint64_t *)w;
  if (hipMemcpyAsync(dcaps, caps, sizeof(uint64_t) * 4, hipMemcpyHostToDevice, st) != hipSuccess)
    return set_error(PC_ERR_DEVICE, "caps upload failed");
  hipLaunchKernelGGL(k_unpack_plan, dim3(1), dim3(64), 0, st, in, n_in, up, (const uint64_t *)dcaps);
  hipLaunchKernelGGL(k_unpack_streams, dim3(4), dim3(kUnpackBlock), 0, st, in, up, sub, subc, outp);
  if (hipGetLastError() != hipSuccess) return set_error(PC_ERR_DEVICE, "unpack launch failed");
  if (hipMemcpyAsync(host, up, sizeof(UnpackPlan), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return set_error(PC_ERR_DEVICE, "unpack read-back failed");
  if (host->err & 1u) return set_error(PC_ERR_ARG, "malformed container (header, tables or sizes)");
  if (host->err) return set_error(PC_ERR_ARG, "malformed payload");
  return PC_OK;
}

// One frame's packing job; `ws` holds its plan and segment table.
PackJob frame_job(const pc_layout &L, const void *frame, char *ws, void *out, uint64_t cap, uint64_t *nbytes,
                  const StreamPtrs &so) {
  PackJob j{};
  j.f = frame_dev((void *)frame, L);
  j.hs.base = j.f.strip;
  j.hs.stride_q = 256;
  j.hs.stride_s = PC_STRIP_WORDS;
  for (int q = 0; q < 4; q++) j.hs.nseg[q] = L.TR;
  j.hi = HeadInfo{0, L.th, L.tw, L.H, L.W, 1, j.f.info};
  j.plan = (PackPlan *)ws;
  j.seg = (SegInfo *)(ws + a256(sizeof(PackPlan)));
  j.max_seg = L.TR;
  j.th = L.th;
  j.tw = L.tw;
  j.W = L.W;
  j.cap = cap;
  j.nbytes = nbytes;
  j.out = (uint32_t *)out;
  j.so = so;
  return j;
}

// Plan (a work-group per frame), fill, strips (a work-group per strip and
// frame), sizes.  jobs == NULL: the single job j0.
hipError_t launch_frame_jobs(const PackJob &j0, const PackJob *jobs, int n, const pc_layout &L, uint64_t cap,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_pack_plan, dim3(n), dim3(kPackBlock), 0, st, j0, jobs);
  const int fill_blocks = (int)std::min<uint64_t>(jobs ? 64 : 2048, (cap / 4 + kPackBlock - 1) / kPackBlock);
  hipLaunchKernelGGL(k_pack_fill, dim3(fill_blocks, n), dim3(kPackBlock), 0, st, j0, jobs);
  const size_t sh = 1024 + 4 * 1024 + 64 + 2 * (size_t)L.th * L.W + 64;
  hipError_t e = hipFuncSetAttribute((const void *)k_pack_frame, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pack_frame, dim3(n, L.TR), dim3(kPackBlock), sh, st, j0, jobs);
  hipLaunchKernelGGL(k_pack_done, dim3((n + 255) / 256), dim3(256), 0, st, j0, jobs, n);
  return hipGetLastError();
}

pc_status check_frame_pack(const pc_sensor *sensor, const pc_params *params, uint64_t cap, pc_layout *L) {
  pc_status stt = pc_stream_layout(sensor, params, L);
  if (stt) return stt;
  if (L->TR > 1024) return set_error(PC_ERR_UNSUPPORTED, "more than 1024 tile rows");
  FrameCaps k = frame_caps(*L);
  if (cap < bound_of(k.c))
    return set_error(PC_ERR_CAPACITY, "output %llu bytes < bound %llu", (unsigned long long)cap,
                     (unsigned long long)bound_of(k.c));
  return PC_OK;
}

}  // namespace
}  // namespace pcc

using namespace pcc;

extern "C" {

size_t pc_pack_bound(const pc_sensor *sensor, const pc_params *params) {
  pc_layout L;
  if (pc_stream_layout(sensor, params, &L) != PC_OK) return 0;
  FrameCaps k = frame_caps(L);
  return bound_of(k.c);
}

size_t pc_pack_workspace_size(const pc_sensor *sensor, const pc_params *params) {
  pc_layout L;
  if (pc_stream_layout(sensor, params, &L) != PC_OK) return 0;
  return frame_ws(L);
}

pc_status pc_pack(pc_ctx *ctx, const void *frame, const pc_sensor *sensor, const pc_params *params, void *work,
                  size_t work_bytes, void *out, uint64_t cap, uint64_t *nbytes, uint8_t *const *streams,
                  const uint64_t *stream_caps, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_layout L;
  pc_status stt = check_frame_pack(sensor, params, cap, &L);
  if (stt) return stt;
  if (!frame || !out || !nbytes || !work) return set_error(PC_ERR_ARG, "frame, output, size or workspace is NULL");
  if ((uintptr_t)out & 3) return set_error(PC_ERR_ARG, "output must be 4-byte aligned");
  if (work_bytes < frame_ws(L)) return set_error(PC_ERR_CAPACITY, "workspace %zu bytes < %zu", work_bytes, frame_ws(L));
  if (streams && !stream_caps) return set_error(PC_ERR_ARG, "stream capacities are NULL");
  StreamPtrs so{};
  for (int q = 0; q < 4; q++) {
    so.p[q] = streams ? streams[q] : nullptr;
    so.cap[q] = streams ? stream_caps[q] : 0;
  }
  PackJob j = frame_job(L, frame, (char *)work, out, cap, nbytes, so);
  hipError_t he = launch_frame_jobs(j, nullptr, 1, L, cap, (hipStream_t)stream);
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "pack launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

size_t pc_pack_batch_workspace_size(const pc_sensor *sensor, const pc_params *params, int32_t n) {
  pc_layout L;
  if (n < 1 || pc_stream_layout(sensor, params, &L) != PC_OK) return 0;
  return a256(sizeof(PackJob) * (size_t)n) + (size_t)n * pack_ws(L.TR, false);
}

pc_status pc_pack_batch(pc_ctx *ctx, int32_t n, const void *const *frames, const pc_sensor *sensor,
                        const pc_params *params, void *work, size_t work_bytes, void *const *outs, uint64_t cap,
                        uint64_t *nbytes, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  if (n < 1 || n > 65535) return set_error(PC_ERR_ARG, "frame count %d out of range 1..65535", n);
  pc_layout L;
  pc_status stt = check_frame_pack(sensor, params, cap, &L);
  if (stt) return stt;
  if (!frames || !outs || !nbytes || !work) return set_error(PC_ERR_ARG, "NULL argument");
  const size_t need = pc_pack_batch_workspace_size(sensor, params, n);
  if (work_bytes < need) return set_error(PC_ERR_CAPACITY, "workspace %zu bytes < %zu", work_bytes, need);
  std::vector<PackJob> jobs((size_t)n);
  char *ws = (char *)work + a256(sizeof(PackJob) * (size_t)n);
  for (int i = 0; i < n; i++) {
    if (!frames[i] || !outs[i]) return set_error(PC_ERR_ARG, "frame or output %d is NULL", i);
    if ((uintptr_t)outs[i] & 3) return set_error(PC_ERR_ARG, "output %d must be 4-byte aligned", i);
    jobs[i] = frame_job(L, frames[i], ws + (size_t)i * pack_ws(L.TR, false), outs[i], cap, nbytes + i, StreamPtrs{});
  }
  hipStream_t st = (hipStream_t)stream;
  PackJob *dj = (PackJob *)work;
  // the job table is read by every launch; the host copy must outlive the upload
  if (hipMemcpyAsync(dj, jobs.data(), sizeof(PackJob) * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return set_error(PC_ERR_DEVICE, "job table upload failed");
  hipError_t he = launch_frame_jobs(jobs[0], dj, n, L, cap, st);
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "pack launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

size_t pc_stream_pack_workspace_size(const uint64_t *n) {
  if (!n) return 0;
  size_t p = pack_ws(raw_segs(n), true), u = unpack_ws();
  return p > u ? p : u;
}

uint64_t pc_stream_pack_bound(const uint64_t *n) { return n ? bound_of(n) : 0; }

pc_status pc_pack_streams(pc_ctx *ctx, const uint8_t *const *streams, const uint64_t *n, int32_t kind, int32_t H,
                          int32_t W, int32_t tile_h, int32_t tile_w, void *work, size_t work_bytes, void *out, uint64_t cap,
                          uint64_t *nbytes, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  if (!streams || !n || !work || !out || !nbytes) return set_error(PC_ERR_ARG, "NULL argument");
  if ((uintptr_t)out & 3) return set_error(PC_ERR_ARG, "output must be 4-byte aligned");
  if (kind < 0 || kind > 255 || tile_h < 0 || tile_h > 255 || tile_w < 0 || tile_w > 255 || H < 0 || H > 65535 || W < 0 ||
      W > 65535)
    return set_error(PC_ERR_ARG, "header field out of range");
  for (int q = 0; q < 4; q++) {
    if (n[q] && !streams[q]) return set_error(PC_ERR_ARG, "stream %d is NULL", q);
    if (n[q] >= (1ull << 28)) return set_error(PC_ERR_UNSUPPORTED, "stream %d longer than 2^28 bytes", q);
  }
  const int max_seg = raw_segs(n);
  if (work_bytes < pc_stream_pack_workspace_size(n)) return set_error(PC_ERR_CAPACITY, "workspace too small");
  if (cap < bound_of(n)) return set_error(PC_ERR_CAPACITY, "output smaller than the bound");
  hipStream_t st = (hipStream_t)stream;
  char *ws = (char *)work;
  PackPlan *plan = (PackPlan *)ws;
  SegInfo *seg = (SegInfo *)(ws + a256(sizeof(PackPlan)));
  uint32_t *seg_hist = (uint32_t *)(ws + a256(sizeof(PackPlan)) + a256(sizeof(SegInfo) * 4 * (size_t)max_seg));
  StreamIn in;
  HistSrc hs;
  for (int q = 0; q < 4; q++) {
    in.p[q] = streams[q];
    in.n[q] = n[q];
    hs.nseg[q] = (int)((n[q] + kChunk - 1) / kChunk);
  }
  hs.base = seg_hist;
  hs.stride_q = 256 * (int64_t)max_seg;
  hs.stride_s = 256;
  PackJob j{};
  j.hs = hs;
  j.hi = HeadInfo{kind, tile_h, tile_w, H, W, 0, nullptr};
  j.plan = plan;
  j.seg = seg;
  j.max_seg = max_seg;
  j.cap = cap;
  j.nbytes = nbytes;
  j.out = (uint32_t *)out;
  const PackJob *none = nullptr;
  hipLaunchKernelGGL(k_pack_hist, dim3(4 * max_seg), dim3(kPackBlock), 0, st, in, seg_hist, max_seg);
  hipLaunchKernelGGL(k_pack_plan, dim3(1), dim3(kPackBlock), 0, st, j, none);
  const int fill_blocks = (int)std::min<uint64_t>(2048, (cap / 4 + kPackBlock - 1) / kPackBlock);
  hipLaunchKernelGGL(k_pack_fill, dim3(fill_blocks), dim3(kPackBlock), 0, st, j, none);
  hipLaunchKernelGGL(k_pack_chunks, dim3(4 * max_seg), dim3(kPackBlock), 0, st, in, plan, (const SegInfo *)seg, max_seg,
                     (uint32_t *)out);
  hipLaunchKernelGGL(k_pack_done, dim3(1), dim3(1), 0, st, j, none, 1);
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "pack launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

pc_status pc_unpack_streams(pc_ctx *ctx, const void *data, uint64_t n_in, void *work, size_t work_bytes,
                            uint8_t *const *streams, const uint64_t *caps, uint64_t *n_out, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  if (!data || !work || !streams || !caps || !n_out) return set_error(PC_ERR_ARG, "NULL argument");
  if (work_bytes < unpack_ws()) return set_error(PC_ERR_CAPACITY, "workspace too small");
  StreamPtrs o{};
  for (int q = 0; q < 4; q++) {
    o.p[q] = streams[q];
    o.cap[q] = caps[q];
    if (caps[q] && !streams[q]) return set_error(PC_ERR_ARG, "stream %d is NULL", q);
  }
  UnpackPlan h;
  pc_status s = unpack_to_streams((const uint8_t *)data, n_in, (char *)work, caps, o, &h, (hipStream_t)stream);
  for (int q = 0; q < 4; q++) n_out[q] = s == PC_OK ? h.nbytes[q] : 0;
  return s;
}

size_t pc_unpack_batch_workspace_size(const pc_sensor *sensor, const pc_params *params, int32_t n) {
  pc_layout L;
  if (n < 1 || pc_stream_layout(sensor, params, &L) != PC_OK) return 0;
  FrameCaps k = frame_caps(L);
  size_t per = unpack_ws();
  for (int q = 0; q < 4; q++) per += a256(k.c[q]);
  return a256(sizeof(UnpackJob) * (size_t)n) + a256(sizeof(uint32_t) * (size_t)n) + a256(sizeof(uint64_t) * 4) +
         (size_t)n * per;
}

pc_status pc_unpack_batch(pc_ctx *ctx, int32_t n, const void *const *data, const uint64_t *n_in,
                          const void *const *keys, const pc_sensor *sensor, const pc_params *params, void *work,
                          size_t work_bytes, void *const *frames_out, int32_t *kinds_out, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  if (n < 1 || n > 65535) return set_error(PC_ERR_ARG, "container count %d out of range 1..65535", n);
  pc_layout L;
  pc_status stt = pc_stream_layout(sensor, params, &L);
  if (stt) return stt;
  if (!data || !n_in || !work || !frames_out) return set_error(PC_ERR_ARG, "NULL argument");
  const size_t need = pc_unpack_batch_workspace_size(sensor, params, n);
  if (work_bytes < need) return set_error(PC_ERR_CAPACITY, "workspace %zu bytes < %zu", work_bytes, need);
  FrameCaps k = frame_caps(L);
  char *ws = (char *)work;
  UnpackJob *dj = (UnpackJob *)ws;
  ws += a256(sizeof(UnpackJob) * (size_t)n);
  uint32_t *dstatus = (uint32_t *)ws;
  ws += a256(sizeof(uint32_t) * (size_t)n);
  uint64_t *dcaps = (uint64_t *)ws;
  ws += a256(sizeof(uint64_t) * 4);
  std::vector<UnpackJob> jobs((size_t)n);
  for (int i = 0; i < n; i++) {
    if (!data[i] || !frames_out[i]) return set_error(PC_ERR_ARG, "container or output frame %d is NULL", i);
    const void *key = keys ? keys[i] : nullptr;
    if (key == frames_out[i]) return set_error(PC_ERR_ARG, "output frame %d is its own key frame", i);
    UnpackJob &j = jobs[i];
    j.in = (const uint8_t *)data[i];
    j.n_in = n_in[i];
    j.up = (UnpackPlan *)ws;
    char *w = ws + a256(sizeof(UnpackPlan));
    j.sub = (uint64_t *)w;
    w += a256(sizeof(uint64_t) * 8 * kMaxSub);
    j.subc = (uint32_t *)w;
    w += a256(sizeof(uint32_t) * 4 * kMaxSub);
    w += a256(sizeof(uint64_t) * 4);
    for (int q = 0; q < 4; q++) {
      j.sp.p[q] = (uint8_t *)w;
      j.sp.cap[q] = k.c[q];
      w += a256(k.c[q]);
    }
    j.caps = dcaps;
    j.f = frame_dev(frames_out[i], L);
    j.key = key ? frame_dev((void *)key, L) : j.f;
    j.has_key = key ? 1 : 0;
    ws = w;
  }
  hipStream_t st = (hipStream_t)stream;
  std::vector<uint32_t> status((size_t)n);
  // the job table is read by every launch; the host copies must outlive the uploads
  if (hipMemcpyAsync(dj, jobs.data(), sizeof(UnpackJob) * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dcaps, k.c, sizeof(uint64_t) * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return set_error(PC_ERR_DEVICE, "job table upload failed");
  hipLaunchKernelGGL(k_unpack_plan_b, dim3(n), dim3(64), 0, st, (const UnpackJob *)dj);
  hipLaunchKernelGGL(k_unpack_streams_b, dim3(n, 4), dim3(kUnpackBlock), 0, st, (const UnpackJob *)dj);
  for (int pass = 0; pass < 2; pass++)
    hipLaunchKernelGGL(k_unpack_frame_b, dim3(n), dim3(kUnpackBlock), 0, st, (const UnpackJob *)dj, pass, L.H, L.W,
                       L.th, L.tw);
  hipLaunchKernelGGL(k_unpack_status, dim3((n + 255) / 256), dim3(256), 0, st, (const UnpackJob *)dj, n, dstatus);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(status.data(), dstatus, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return set_error(PC_ERR_DEVICE, "unpack launch failed");
  for (int i = 0; i < n; i++) {
    if (kinds_out) kinds_out[i] = (int32_t)((status[i] >> 16) & 0xFF);
    const uint32_t e = status[i] & 0xFFFFu;
    if (e & 1u) return set_error(PC_ERR_ARG, "container %d: malformed header, tables or sizes", i);
    if (e & 8u) return set_error(PC_ERR_ARG, "container %d: another sensor size, tile shape or frame kind", i);
    if (e & 16u) return set_error(PC_ERR_ARG, "container %d: a predicted frame needs its key frame", i);
    if (e) return set_error(PC_ERR_ARG, "container %d: malformed payload or streams", i);
  }
  return PC_OK;
}

pc_status pc_unpack(pc_ctx *ctx, const void *data, uint64_t n_in, const void *key, const pc_sensor *sensor,
                    const pc_params *params, void *work, size_t work_bytes, void *frame_out, int32_t *kind_out,
                    void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_layout L;
  pc_status stt = pc_stream_layout(sensor, params, &L);
  if (stt) return stt;
  if (!data || !work || !frame_out) return set_error(PC_ERR_ARG, "data, workspace or frame is NULL");
  if (key == frame_out) return set_error(PC_ERR_ARG, "output frame must differ from the key frame");
  if (work_bytes < frame_ws(L)) return set_error(PC_ERR_CAPACITY, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  FrameCaps k = frame_caps(L);
  char *ws = (char *)work;
  StreamPtrs sp{};
  char *w = ws + unpack_ws();
  for (int q = 0; q < 4; q++) {
    sp.p[q] = (uint8_t *)w;
    sp.cap[q] = k.c[q];
    w += a256(k.c[q]);
  }
  UnpackPlan h;
  pc_status s = unpack_to_streams((const uint8_t *)data, n_in, ws, k.c, sp, &h, st);
  if (s) return s;
  if (h.H != L.H || h.W != L.W || h.th != L.th || h.tw != L.tw)
    return set_error(PC_ERR_ARG, "container is %dx%d with %dx%d tiles; sensor and params give %dx%d with %dx%d", h.H, h.W,
                     h.th, h.tw, L.H, L.W, L.th, L.tw);
  if (h.kind != 0 && h.kind != 1) return set_error(PC_ERR_ARG, "unknown frame kind %d", h.kind);
  if (h.kind == 1 && !key) return set_error(PC_ERR_ARG, "a predicted frame needs its key frame");
  FrameDev f = frame_dev(frame_out, L);
  FrameDev kf = key ? frame_dev((void *)key, L) : f;
  hipLaunchKernelGGL(k_unpack_frame, dim3(1), dim3(kUnpackBlock), 0, st, (UnpackPlan *)ws, sp, f, kf, key ? 1 : 0,
                     L.th, L.tw, L.W);
  uint32_t err = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&err, &((UnpackPlan *)ws)->err, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return set_error(PC_ERR_DEVICE, "unpack launch failed");
  if (err) return set_error(PC_ERR_ARG, "malformed streams (runs, masks or residual count)");
  if (kind_out) *kind_out = h.kind;
  return PC_OK;
}

}  // extern "C"

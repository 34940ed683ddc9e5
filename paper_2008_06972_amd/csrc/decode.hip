// Decoder (Sec. III-C): a plane-coded pixel is reconstructed by casting the
// pixel-centre ray onto its run plane; every other non-empty pixel takes its
// residual code times the quantiser step.  Points are placed on the pixel
// rays at the decoded ranges and, for a predicted frame, optionally taken
// back through the inverse of its transform into the key frame (Eq. (6)).
// Uses only the encoded data: the occupancy bits, the runs (and the key
// frame's runs for the normals of temporal runs), the per-tile masks, the
// residual codes of each strip and the transform in the info block.
#include "fit.h"

namespace pcc {

// Exclusive prefix sum of a[0..n) in place, by the whole work-group: each
// thread sums a contiguous share, wavefronts scan the shares, the
// wavefront totals are combined through LDS.
__device__ __forceinline__ void block_prefix(uint32_t *a, int n, uint32_t *wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (n + kBlock - 1) / kBlock, b = min(n, tid * per), e = min(n, b + per);
  uint32_t local = 0;
  for (int q = b; q < e; q++) local += a[q];
  uint32_t x = local;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint32_t run = x - local;
  for (int w = 0; w < wv; w++) run += wsum[w];
  for (int q = b; q < e; q++) {
    const uint32_t c = a[q];
    a[q] = run;
    run += c;
  }
  __syncthreads();
}

// One work-group per (frame, tile-row strip); blockIdx.x picks the frame's
// job from `jobs` (or j0 when jobs is NULL) and blockIdx.y the strip, so
// that consecutive work-groups, which go to different XCDs, hold different
// frames and every XCD gets every strip row.  Phase 1 (a thread per tile):
// the run planes of the strip's tiles and the residual count of every
// (row, tile) segment, prefix-summed into each segment's first code.
// Phase 2 (a thread per four consecutive pixels of a row): each pixel is
// decoded from its tile's plane or its residual code and the four ranges
// are stored as one float4, so a wavefront writes a contiguous 1 KiB of the
// image; points, if asked for, are r d along the pixel-centre ray, taken
// back to the frame's own coordinates by R^T (p - T) when frame_coords is
// set (M from the frame's info block), three float4 stores per thread.
// A predicted frame's temporal runs need the key frame's run normals: with
// no key frame given, their pixels decode to 0 and the frame's info block
// gets the sticky PC_STATUS_NOKEY bit.
template <int TH, int TW>
__global__ void __launch_bounds__(kBlock) k_decode(DecodeJob j0, const DecodeJob *jobs, SensorDev s, EncParams p) {
  static_assert(TW % 4 == 0, "four pixels of a thread share one tile");
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ uint32_t wsum[kBlock / 64];
  __shared__ float Ms[12];
  const DecodeJob *J = jobs ? jobs + blockIdx.x : &j0;
  const FrameDev f = J->f;
  const int has_key = J->has_key;
  float *__restrict__ out = J->out;
  float *__restrict__ xyz = J->xyz;
  const int TC = f.TC, tr = blockIdx.y, tid = threadIdx.x, W = s.W;
  float4 *pl = (float4 *)smem_raw;                          // [TC]
  uint8_t *has = (uint8_t *)(pl + TC);                      // [TC]: 0 none, 1 plane, 2 temporal without its key
  uint32_t *cnt = (uint32_t *)(has + ((TC + 15) & ~15));    // [TH * TC]
  for (int tc = tid; tc < TC; tc += kBlock) has[tc] = 0;
  if (tid < 12) {
    const bool back = xyz && J->frame_coords;
    Ms[tid] = back ? f.info->M[tid] : (tid % 5 == 0 ? 1.0f : 0.0f);
  }
  __syncthreads();
  // planes of the spatial runs of this tile row
  const int ns = f.nruns[tr];
  for (int q = tid; q < ns; q += kBlock) {
    pc_run R = f.sruns[(int64_t)tr * TC + q];
    for (int e = 0; e < R.len; e++) {
      pl[R.s + e] = make_float4(R.a, R.b, R.c, (float)R.axis);
      has[R.s + e] = 1;
    }
  }
  // temporal runs: key run's normal, own offset
  const int np = f.nruns[f.TR + tr];
  if (has_key) {
    const pc_run *ksr = J->key.sruns;
    for (int q = tid; q < np; q += kBlock) {
      pc_prun R = f.pruns[(int64_t)tr * TC + q];
      pc_run K = ksr[R.krun];
      for (int e = 0; e < R.len; e++) {
        pl[R.s + e] = make_float4(K.a, K.b, R.c, (float)K.axis);
        has[R.s + e] = 1;
      }
    }
  } else if (np > 0) {
    for (int q = tid; q < np; q += kBlock) {
      pc_prun R = f.pruns[(int64_t)tr * TC + q];
      for (int e = 0; e < R.len; e++) has[R.s + e] = 2;
    }
    if (tid == 0) atomicOr(&f.info->status, PC_STATUS_NOKEY);
  }
  __syncthreads();
  const uint32_t *occ = f.occ + (int64_t)tr * (TH * W / 32);
  constexpr uint32_t kSeg = (uint32_t)((1ull << TW) - 1ull);
  // residual pixels per (row, tile) in raster order
  for (int tc = tid; tc < TC; tc += kBlock) {
    uint64_t fm = has[tc] ? f.mask[(int64_t)tr * TC + tc] : 0ull;
#pragma unroll
    for (int i = 0; i < TH; i++) {
      int bit = i * W + tc * TW;
      uint32_t vb = (occ[bit >> 5] >> (bit & 31)) & kSeg;
      uint32_t mb = (uint32_t)((fm >> (i * TW)) & kSeg);
      cnt[i * TC + tc] = __popc(vb & ~mb);
    }
  }
  __syncthreads();
  block_prefix(cnt, TH * TC, wsum);
  const uint16_t *res = f.res + (int64_t)tr * TH * W;
  const int nq = W / 4;
  for (int e = tid; e < TH * nq; e += kBlock) {
    const int i = e / nq, u0 = (e - i * nq) * 4, tc = u0 / TW, k0 = u0 % TW;
    const int v = tr * TH + i;
    const int bit = i * W + tc * TW;
    const uint32_t vb = (occ[bit >> 5] >> (bit & 31)) & kSeg;
    const int hp = has[tc];
    const uint64_t fm = hp ? f.mask[(int64_t)tr * TC + tc] : 0ull;
    const uint32_t mb = (uint32_t)((fm >> (i * TW)) & kSeg);
    // first code of these four pixels: the segment's first code plus the
    // residual pixels of the segment before column k0
    uint32_t o = cnt[i * TC + tc] + __popc(vb & ~mb & ((1u << k0) - 1u));
    const Plane P = Plane{(int)pl[tc].w, pl[tc].x, pl[tc].y, pl[tc].z};
    const float ce = s.ce[v], se = s.se[v];
    float val[4];
    Dir dd[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int k = k0 + q, u = u0 + q;
      dd[q] = dir_of(ce, se, s.ca[u], s.sa[u]);
      val[q] = 0.0f;
      if ((vb >> k) & 1u) {
        if ((mb >> k) & 1u) {
          val[q] = hp == 1 ? ray_cast(P, dd[q]) : 0.0f;
        } else {
          val[q] = (float)res[o++] * p.step;
        }
      }
    }
    const int64_t px = (int64_t)v * W + u0;
    if (out) *reinterpret_cast<float4 *>(out + px) = make_float4(val[0], val[1], val[2], val[3]);
    if (xyz) {
      float w[12];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        float x = val[q] * dd[q].x, y = val[q] * dd[q].y, z = val[q] * dd[q].z;
        if (J->frame_coords) {
          // R^T (p - T): rows of M are (R_r0, R_r1, R_r2, T_r)
          const float qx = x - Ms[3], qy = y - Ms[7], qz = z - Ms[11];
          x = fmaf(Ms[8], qz, fmaf(Ms[4], qy, Ms[0] * qx));
          y = fmaf(Ms[9], qz, fmaf(Ms[5], qy, Ms[1] * qx));
          z = fmaf(Ms[10], qz, fmaf(Ms[6], qy, Ms[2] * qx));
        }
        const bool keep = val[q] != 0.0f;
        w[3 * q] = keep ? x : 0.0f;
        w[3 * q + 1] = keep ? y : 0.0f;
        w[3 * q + 2] = keep ? z : 0.0f;
      }
      float4 *dst = reinterpret_cast<float4 *>(xyz + 3 * px);
      dst[0] = make_float4(w[0], w[1], w[2], w[3]);
      dst[1] = make_float4(w[4], w[5], w[6], w[7]);
      dst[2] = make_float4(w[8], w[9], w[10], w[11]);
    }
  }
}

template <int TH, int TW>
static hipError_t launch_decode_t(const DecodeJob &j0, const DecodeJob *jobs, int n, int TR, int TC,
                                  const SensorDev &s, const EncParams &p, hipStream_t st) {
  size_t sh = sizeof(float4) * TC + ((TC + 15) & ~15) + sizeof(uint32_t) * TH * TC + 64;
  hipError_t e = hipFuncSetAttribute((const void *)k_decode<TH, TW>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_decode<TH, TW>), dim3(n, TR), dim3(kBlock), sh, st, j0, jobs, s, p);
  return hipGetLastError();
}

hipError_t launch_decode_jobs(const DecodeJob &j0, const DecodeJob *jobs, int n, const SensorDev &s,
                              const EncParams &p, hipStream_t st) {
  const int TR = j0.f.TR, TC = j0.f.TC;
  if (p.th == 4 && p.tw == 4) return launch_decode_t<4, 4>(j0, jobs, n, TR, TC, s, p, st);
  if (p.th == 4 && p.tw == 8) return launch_decode_t<4, 8>(j0, jobs, n, TR, TC, s, p, st);
  if (p.th == 4 && p.tw == 16) return launch_decode_t<4, 16>(j0, jobs, n, TR, TC, s, p, st);
  if (p.th == 8 && p.tw == 8) return launch_decode_t<8, 8>(j0, jobs, n, TR, TC, s, p, st);
  return hipErrorInvalidValue;
}

hipError_t launch_decode(const FrameDev *key, const FrameDev &f, const SensorDev &s, const EncParams &p,
                         float *range_out, float *xyz_out, int frame_coords, hipStream_t st) {
  DecodeJob j;
  j.f = f;
  j.key = key ? *key : f;
  j.has_key = key ? 1 : 0;
  j.out = range_out;
  j.xyz = xyz_out;
  j.frame_coords = frame_coords;
  return launch_decode_jobs(j, nullptr, 1, s, p, st);
}

}  // namespace pcc

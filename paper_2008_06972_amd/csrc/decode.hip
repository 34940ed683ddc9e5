// Decoder (Sec. III-C): a plane-coded pixel is reconstructed by casting the
// pixel-centre ray onto its run plane; every other non-empty pixel takes its
// residual code times the quantiser step.  Uses only the encoded data: the
// occupancy bits, the runs (and the key frame's runs for the normals of
// temporal runs), the per-tile masks and the residual codes of each strip.
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

// One work-group per (tile-row strip, frame); blockIdx.y picks the frame's
// job from `jobs`, or j0 when jobs is NULL.
template <int TH, int TW>
__global__ void __launch_bounds__(kBlock) k_decode(DecodeJob j0, const DecodeJob *jobs, SensorDev s, EncParams p) {
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ uint32_t wsum[kBlock / 64];
  constexpr int N = TH * TW;
  const DecodeJob *J = jobs ? jobs + blockIdx.y : &j0;
  const FrameDev f = J->f;
  const int has_key = J->has_key;
  float *__restrict__ out = J->out;
  const int TC = f.TC, tr = blockIdx.x, tid = threadIdx.x, W = s.W;
  float4 *pl = (float4 *)smem_raw;                          // [TC]
  uint8_t *has = (uint8_t *)(pl + TC);                      // [TC]
  uint32_t *cnt = (uint32_t *)(has + ((TC + 15) & ~15));    // [TH * TC]
  for (int tc = tid; tc < TC; tc += kBlock) has[tc] = 0;
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
  if (has_key) {
    const pc_run *ksr = J->key.sruns;
    const int np = f.nruns[f.TR + tr];
    for (int q = tid; q < np; q += kBlock) {
      pc_prun R = f.pruns[(int64_t)tr * TC + q];
      pc_run K = ksr[R.krun];
      for (int e = 0; e < R.len; e++) {
        pl[R.s + e] = make_float4(K.a, K.b, R.c, (float)K.axis);
        has[R.s + e] = 1;
      }
    }
  }
  __syncthreads();
  const uint32_t *occ = f.occ + (int64_t)tr * (TH * W / 32);
  // residual pixels per (row, tile) in raster order
  for (int tc = tid; tc < TC; tc += kBlock) {
    uint64_t fm = has[tc] ? f.mask[(int64_t)tr * TC + tc] : 0ull;
#pragma unroll
    for (int i = 0; i < TH; i++) {
      int bit = i * W + tc * TW;
      uint32_t vb = (occ[bit >> 5] >> (bit & 31)) & (uint32_t)((1ull << TW) - 1ull);
      uint32_t mb = (uint32_t)((fm >> (i * TW)) & ((1ull << TW) - 1ull));
      cnt[i * TC + tc] = __popc(vb & ~mb);
    }
  }
  __syncthreads();
  block_prefix(cnt, TH * TC, wsum);
  const uint16_t *res = f.res + (int64_t)tr * TH * W;
  for (int tc = tid; tc < TC; tc += kBlock) {
    bool hp = has[tc] != 0;
    Plane P = Plane{(int)pl[tc].w, pl[tc].x, pl[tc].y, pl[tc].z};
    uint64_t fm = hp ? f.mask[(int64_t)tr * TC + tc] : 0ull;
#pragma unroll
    for (int i = 0; i < TH; i++) {
      const int v = tr * TH + i;
      const float ce = s.ce[v], se = s.se[v];
      uint32_t o = cnt[i * TC + tc];
      int bit0 = i * W + tc * TW;
      uint32_t vb = (occ[bit0 >> 5] >> (bit0 & 31)) & (uint32_t)((1ull << TW) - 1ull);
#pragma unroll
      for (int k = 0; k < TW; k++) {
        const int u = tc * TW + k;
        float val = 0.0f;
        if ((vb >> k) & 1u) {
          if ((fm >> (i * TW + k)) & 1ull) {
            val = ray_cast(P, dir_of(ce, se, s.ca[u], s.sa[u]));
          } else {
            val = (float)res[o++] * p.step;
          }
        }
        out[(int64_t)v * W + u] = val;
      }
    }
  }
}

template <int TH, int TW>
static hipError_t launch_decode_t(const DecodeJob &j0, const DecodeJob *jobs, int n, int TR, int TC,
                                  const SensorDev &s, const EncParams &p, hipStream_t st) {
  size_t sh = sizeof(float4) * TC + ((TC + 15) & ~15) + sizeof(uint32_t) * TH * TC + 64;
  hipError_t e = hipFuncSetAttribute((const void *)k_decode<TH, TW>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_decode<TH, TW>), dim3(TR, n), dim3(kBlock), sh, st, j0, jobs, s, p);
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
                         float *range_out, hipStream_t st) {
  DecodeJob j;
  j.f = f;
  j.key = key ? *key : f;
  j.has_key = key ? 1 : 0;
  j.out = range_out;
  return launch_decode_jobs(j, nullptr, 1, s, p, st);
}

}  // namespace pcc

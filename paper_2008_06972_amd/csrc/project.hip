// Range-image conversion (Sec. III-B, Eq. (1)-(2)) with the rigid transform
// of predicted frames (Sec. III-D, Eq. (6)) and nearest-point collisions.
//
// One thread per point.  The pixel keeps the minimum 64-bit key
// (bits(r) << 32 | index): positive FP32 bit patterns order like the values,
// so the nearest point wins and equal ranges go to the lower index, whatever
// order the atomics land in.  All arithmetic is FP32 with the operation order
// written out (explicit fmaf, correctly rounded sqrt and division), so bins
// are reproducible bit for bit.
#include "project.h"

namespace pcc {

__global__ void k_key_clear(unsigned long long *keys, int64_t npx, pc_proj_stats *stats, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < npx; i += stride) keys[i] = ~0ull;
  if (stats && blockIdx.x == 0 && threadIdx.x == 0) {
    stats->n_in = n;
    stats->n_nonfinite = 0;
    stats->n_fov = 0;
    stats->n_collided = 0;
    stats->n_kept = 0;
  }
}

__global__ void k_project(const float *__restrict__ xyz, int64_t n, Mat12 M, int hasM, SensorDev s,
                          unsigned long long *__restrict__ keys, pc_proj_stats *stats) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int nonfinite = 0, fov = 0;
  if (i < n) {
    int v, u;
    float r;
    const int st = project_point(s, M, hasM, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], v, u, r);
    if (st == PROJ_KEPT) {
      unsigned long long key = ((unsigned long long)__float_as_uint(r) << 32) | (unsigned long long)(uint32_t)i;
      atomicMin(&keys[(int64_t)v * s.W + u], key);
    }
    nonfinite = st == PROJ_NONFINITE;
    fov = st == PROJ_FOV;
  }
  if (stats) {
    // wave-level counts, one atomic per wave and counter
    unsigned long long bn = __ballot(nonfinite), bf = __ballot(fov);
    if ((threadIdx.x & 63) == 0) {
      if (bn) atomicAdd((unsigned long long *)&stats->n_nonfinite, (unsigned long long)__popcll(bn));
      if (bf) atomicAdd((unsigned long long *)&stats->n_fov, (unsigned long long)__popcll(bf));
    }
  }
}

__global__ void k_key_finalize(const unsigned long long *__restrict__ keys, int64_t npx, float *__restrict__ range,
                               int32_t *__restrict__ src_idx, pc_proj_stats *stats) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int kept = 0;
  if (i < npx) {
    unsigned long long k = keys[i];
    if (k == ~0ull) {
      range[i] = 0.0f;
      if (src_idx) src_idx[i] = -1;
    } else {
      range[i] = __uint_as_float((uint32_t)(k >> 32));
      if (src_idx) src_idx[i] = (int32_t)(uint32_t)(k & 0xffffffffull);
      kept = 1;
    }
  }
  if (stats) {
    unsigned long long b = __ballot(kept);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd((unsigned long long *)&stats->n_kept, (unsigned long long)__popcll(b));
  }
}

__global__ void k_stats_collided(pc_proj_stats *stats) {
  stats->n_collided = stats->n_in - stats->n_nonfinite - stats->n_fov - stats->n_kept;
}

hipError_t launch_project(const float *xyz, int64_t n, const float *M, const SensorDev &s,
                          unsigned long long *keys, float *range, int32_t *src_idx,
                          pc_proj_stats *stats, hipStream_t st) {
  int64_t npx = (int64_t)s.H * s.W;
  Mat12 m{};
  if (M)
    for (int r = 0; r < 3; r++)
      for (int c = 0; c < 4; c++) m.m[4 * r + c] = M[4 * r + c];
  int clear_blocks = (int)((npx + 255) / 256);
  if (clear_blocks > 2048) clear_blocks = 2048;
  hipLaunchKernelGGL(k_key_clear, dim3(clear_blocks), dim3(256), 0, st, keys, npx, stats, n);
  if (n > 0)
    hipLaunchKernelGGL(k_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xyz, n, m, M ? 1 : 0, s,
                       keys, stats);
  hipLaunchKernelGGL(k_key_finalize, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, st, keys, npx, range,
                     src_idx, stats);
  if (stats) hipLaunchKernelGGL(k_stats_collided, dim3(1), dim3(1), 0, st, stats);
  return hipGetLastError();
}

}  // namespace pcc

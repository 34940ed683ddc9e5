// Range-image conversion (Sec. III-B, Eq. (1)-(2)) with the rigid transform
// of predicted frames (Sec. III-D, Eq. (6)) and nearest-point collisions.
//
// One thread per point.  The pixel keeps the minimum 64-bit key
// (bits(r) << 32 | index): positive FP32 bit patterns order like the values,
// so the nearest point wins and equal ranges go to the lower index, whatever
// order the atomics land in.  All arithmetic is FP32 with the operation order
// written out (explicit fmaf, correctly rounded sqrt and division), so bins
// are reproducible bit for bit.
#include "pc_internal.h"

namespace pcc {

struct Mat34 {
  float m[12];
};

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

// Row: number of interior cuts above q (cuts descend), found by bisection.
__device__ __forceinline__ int row_of(const float *cut, int H, float q) {
  int lo = 1, hi = H;      // first k in [1, H) with cut[k] <= q
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (cut[mid] > q) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

__device__ __forceinline__ float edge_side(const SensorDev &s, int u, float x, float y) {
  float t = s.eby[u] * x;
  return fmaf(s.ebx[u], y, -t);
}

// Column: the unique u with side(u) <= 0 < side(u+1); start from an atan2
// estimate and walk (the walk ends within one step for any estimate error
// below a bin; it is bounded by W steps in any case).
__device__ __forceinline__ int column_of(const SensorDev &s, float x, float y) {
  int W = s.W;
  float rel = s.beta0 - atan2f(y, x);
  int u = (int)floorf(rel / s.dth);
  u %= W;
  if (u < 0) u += W;
  for (int step = 0; step <= W + 2; step++) {
    if (edge_side(s, u, x, y) > 0.0f) { u = (u == 0) ? W - 1 : u - 1; continue; }
    int un = (u + 1 == W) ? 0 : u + 1;
    if (edge_side(s, un, x, y) <= 0.0f) { u = un; continue; }
    return u;
  }
  return -1;
}

__global__ void k_project(const float *__restrict__ xyz, int64_t n, Mat34 M, int hasM, SensorDev s,
                          unsigned long long *__restrict__ keys, pc_proj_stats *stats) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int nonfinite = 0, fov = 0;
  if (i < n) {
    float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    if (hasM) {
      float xx = fmaf(M.m[0], x, fmaf(M.m[1], y, fmaf(M.m[2], z, M.m[3])));
      float yy = fmaf(M.m[4], x, fmaf(M.m[5], y, fmaf(M.m[6], z, M.m[7])));
      float zz = fmaf(M.m[8], x, fmaf(M.m[9], y, fmaf(M.m[10], z, M.m[11])));
      x = xx; y = yy; z = zz;
    }
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
      nonfinite = 1;
    } else {
      float yy = y * y;
      float rho2 = fmaf(x, x, yy);
      float zz = z * z;
      float r = sqrtf(fmaf(x, x, fmaf(y, y, zz)));
      if (!isfinite(r) || r == 0.0f) {
        nonfinite = 1;
      } else if (rho2 < 1e-12f) {
        fov = 1;
      } else {
        float q = z / sqrtf(rho2);
        if (!(q < s.cut[0]) || q < s.cut[s.H]) {
          fov = 1;
        } else {
          int v = row_of(s.cut, s.H, q);
          int u = column_of(s, x, y);
          if (u < 0) {
            fov = 1;
          } else {
            unsigned long long key = ((unsigned long long)__float_as_uint(r) << 32) | (unsigned long long)(uint32_t)i;
            atomicMin(&keys[(int64_t)v * s.W + u], key);
          }
        }
      }
    }
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
  Mat34 m{};
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

// Plane-seed network (learned plane seeding of the key-frame fit): forward
// on MFMA, backward, loss and Adam.
//
// Four 3x3 convolutions, zero padding 1, channels 4 -> 16 -> 32 -> 32 -> 4,
// strides (2,2), (2,2), (1,2), (1,1), ReLU after the first three, so a
// range image of H x W gives one (n_x, n_y, n_z, planarity logit) per 4x8
// tile.  Input channels: (r, x, y, z) / 16 with (x, y, z) = r d.  Inputs,
// weights and stored activations are bfloat16 (round to nearest even);
// products and sums are FP32.
//
// Forward: each convolution is an implicit GEMM on
// v_mfma_f32_16x16x16_bf16, taken transposed: A = the weights (16 output
// channels per block), B = 16 output pixels per wavefront, K = (ky, kx,
// input channel) with the channel fastest, so a lane's four K values are
// four consecutive channels of one input pixel (one 8-byte load from the
// NHWC activations) and its four results are four consecutive output
// channels of one pixel (one 8-byte store).  Weights are packed once per
// call into [out channel][K] bf16 rows padded to 16.
// Backward (training only) runs on the vector ALUs in FP32 with fixed-order
// reductions (no floating-point atomics): a gradient is the same bits on
// every run.
//
// Parameters: one FP32 vector, per layer W[out][in][ky][kx] then b[out].
#include "seednet.h"

namespace pcc {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct NetLayerDesc {
  int ci, co, sy, sx;
  int woff, boff;      // offsets of W and b in the FP32 parameter vector
  int kpad, copad;     // packed bf16 weights: copad rows of kpad
  int poff;            // offset of the layer's packed weights (elements)
};

constexpr int kNetLayers = 4;
constexpr int kNetParams = 15636;

__host__ __device__ constexpr int net_kpad(int ci) { return (9 * ci + 15) / 16 * 16; }

// layer table (constant, host and device)
__host__ __device__ inline NetLayerDesc net_layer(int l) {
  const int ci[4] = {4, 16, 32, 32}, co[4] = {16, 32, 32, 4}, sy[4] = {2, 2, 1, 1}, sx[4] = {2, 2, 2, 1};
  int woff = 0, poff = 0;
  for (int q = 0; q < l; q++) {
    woff += co[q] * ci[q] * 9 + co[q];
    poff += ((co[q] + 15) / 16 * 16) * net_kpad(ci[q]);
  }
  return NetLayerDesc{ci[l], co[l], sy[l], sx[l], woff, woff + co[l] * ci[l] * 9, net_kpad(ci[l]),
                      (co[l] + 15) / 16 * 16, poff};
}

__host__ __device__ inline int net_packed_elems() {
  NetLayerDesc d = net_layer(3);
  return d.poff + d.copad * d.kpad;
}

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------ forward
__global__ void k_net_pack(const float *__restrict__ params, uint16_t *__restrict__ packed) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= net_packed_elems()) return;
  int l = 0;
  while (l < kNetLayers - 1 && e >= net_layer(l + 1).poff) l++;
  const NetLayerDesc d = net_layer(l);
  const int q = e - d.poff, co = q / d.kpad, k = q % d.kpad;
  const int pos = k / d.ci, ci = k % d.ci;
  float w = 0.0f;
  if (co < d.co && pos < 9) w = params[d.woff + (co * d.ci + ci) * 9 + pos];
  packed[e] = bf16_rne(w);
}

// Input channels of the first layer from a range image (one job, or
// jobs[blockIdx.y]).
__global__ void k_net_input(NetInputJob job, const NetInputJob *__restrict__ jobs) {
  const NetInputJob J = jobs ? jobs[blockIdx.y] : job;
  const int H = J.H, W = J.W;
  uint16_t *__restrict__ a0 = J.a0;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  const int v = p / W, u = p - v * W;
  const float r = J.range[p];
  const float ce = J.ce[v], se = J.se[v], ca = J.ca[u], sa = J.sa[u];
  const float dx = ce * ca, dy = ce * sa;
  uint16_t *o = a0 + 4 * (size_t)p;
  o[0] = bf16_rne(r * 0.0625f);
  o[1] = bf16_rne((r * dx) * 0.0625f);
  o[2] = bf16_rne((r * dy) * 0.0625f);
  o[3] = bf16_rne((r * se) * 0.0625f);
}

// Epilogue of a convolution whose product was taken transposed (weights as
// the A operand, pixels as B: each element is the same dot product of the
// same bf16 values): the lane holds channels nb*16 + 4g .. + 3 of one pixel.
// Hidden layers store bf16(ReLU(. + bias)) as one 8-byte word per nb, the
// last layer (four channels) its FP32 values as one 16-byte word.
template <int CO, int NB, bool LAST>
__device__ __forceinline__ void store_channels(void *out, size_t pix, const f32x4 (&acc)[NB], const float (&bv)[NB][4],
                                               int g) {
  if (LAST) {
    if (g == 0)
      *reinterpret_cast<float4 *>(static_cast<float *>(out) + pix * 4) =
          make_float4(acc[0][0] + bv[0][0], acc[0][1] + bv[0][1], acc[0][2] + bv[0][2], acc[0][3] + bv[0][3]);
  } else {
#pragma unroll
    for (int nb = 0; nb < NB; nb++) {
      if (nb * 16 + 4 * g >= CO) continue;
      bf16x4 v;
#pragma unroll
      for (int i = 0; i < 4; i++) v[i] = (short)bf16_rne(fmaxf(acc[nb][i] + bv[nb][i], 0.0f));
      *reinterpret_cast<bf16x4 *>(static_cast<uint16_t *>(out) + pix * CO + nb * 16 + 4 * g) = v;
    }
  }
}

// One wavefront: kMT groups of 16 consecutive output pixels x all output
// channels.  The weights (B operands) are loaded once per wavefront and
// reused for every pixel group; each group's input gathers (A operands) are
// all issued before its MFMA chain.
constexpr int kMT = 4;

template <int CI, int CO, int SY, int SX, bool LAST>
__global__ void __launch_bounds__(256) k_net_conv(ConvJob job, const ConvJob *__restrict__ jobs,
                                                  const uint16_t *__restrict__ wpk, const float *__restrict__ bias) {
  constexpr int KPAD = net_kpad(CI), KSTEPS = KPAD / 16, NB = (CO + 15) / 16;
  const ConvJob J = jobs ? jobs[blockIdx.y] : job;
  const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
  const int npx = J.Ho * J.Wo;
  const int pw = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 * kMT;
  if (pw >= npx) return;
  bf16x4 b[KSTEPS][NB];
#pragma unroll
  for (int s = 0; s < KSTEPS; s++)
#pragma unroll
    for (int nb = 0; nb < NB; nb++)
      b[s][nb] = *reinterpret_cast<const bf16x4 *>(wpk + (size_t)(nb * 16 + m) * KPAD + 16 * s + 4 * g);
  float bv[NB][4];      // bias of the four channels a lane's results hold
#pragma unroll
  for (int nb = 0; nb < NB; nb++)
#pragma unroll
    for (int i = 0; i < 4; i++) bv[nb][i] = nb * 16 + 4 * g + i < CO ? bias[nb * 16 + 4 * g + i] : 0.0f;
  for (int t = 0; t < kMT; t++) {
    const int p0 = pw + 16 * t;
    if (p0 >= npx) break;
    const int p = p0 + m;
    const int oy = p / J.Wo, ox = p - oy * J.Wo;
    bf16x4 a[KSTEPS];
#pragma unroll
    for (int s = 0; s < KSTEPS; s++) {
      const int k0 = 16 * s + 4 * g, pos = k0 / CI, ci0 = k0 % CI;
      const int iy = oy * SY - 1 + pos / 3, ix = ox * SX - 1 + pos % 3;
      const bool ok = pos < 9 && p < npx && iy >= 0 && iy < J.Hi && ix >= 0 && ix < J.Wi;
      const int cy = ok ? iy : 0, cx = ok ? ix : 0;
      const bf16x4 v = *reinterpret_cast<const bf16x4 *>(J.in + ((size_t)cy * J.Wi + cx) * CI + ci0);
      a[s] = ok ? v : bf16x4{0, 0, 0, 0};
    }
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KSTEPS; s++)
#pragma unroll
      for (int nb = 0; nb < NB; nb++) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b[s][nb], a[s], acc[nb], 0, 0, 0);
    // lane holds D[channel nb*16 + 4g + i][pixel p]: four consecutive
    // channels of one pixel, stored together
    if (p < npx) store_channels<CO, NB, LAST>(J.out, (size_t)p, acc, bv, g);
  }
}

// The same convolution with the input staged in LDS: a block computes BW
// consecutive output pixels of R consecutive output rows; it first copies
// the input rows they read (zero outside the image) into LDS with coalesced
// loads, PS bf16 per input pixel (CI + 4, so that the 16 pixels of an MFMA
// group hit different banks), and then forms every A operand from LDS; each
// wavefront keeps the weights in registers for R * BW / 64 pixels.  With
// RANGE the input channels are computed from the range image while staging
// (the first layer of the batched forward).  The operands and the MFMA order
// are those of k_net_conv, so the results are the same.
template <int CI, int CO, int SY, int SX, bool LAST, bool RANGE, int BW, int R>
__global__ void __launch_bounds__(256) k_net_conv_lds(ConvJob job, const ConvJob *__restrict__ jobs,
                                                      const NetInputJob *__restrict__ in_jobs,
                                                      const uint16_t *__restrict__ wpk, const float *__restrict__ bias) {
  constexpr int KPAD = net_kpad(CI), KSTEPS = KPAD / 16, NB = (CO + 15) / 16;
  constexpr int IW = (BW - 1) * SX + 3, IH = (R - 1) * SY + 3, PS = RANGE ? CI : CI + 4;
  __shared__ __align__(16) uint16_t tile[IH * IW * PS];
  const ConvJob J = jobs ? jobs[blockIdx.y] : job;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, m = lane & 15;
  const int nseg = (J.Wo + BW - 1) / BW;
  const int oy0 = (blockIdx.x / nseg) * R, ox0 = (blockIdx.x % nseg) * BW;
  if (oy0 >= J.Ho) return;
  const int iy0 = oy0 * SY - 1, ix0 = ox0 * SX - 1;
  // staging: U elements' loads in flight per thread before their stores
  constexpr int U = 8;
  if (RANGE) {
    const NetInputJob I = in_jobs[blockIdx.y];
    constexpr int NE = IH * IW;
    for (int e0 = tid; e0 < NE; e0 += 256 * U) {
      float r[U], ce[U], se[U], ca[U], sa[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int e = e0 + 256 * u, dy = e / IW, c = e - dy * IW, iy = iy0 + dy, ix = ix0 + c;
        const bool ok = e < NE && iy >= 0 && iy < I.H && ix >= 0 && ix < I.W;
        const int cy = ok ? iy : 0, cx = ok ? ix : 0;
        r[u] = ok ? I.range[(size_t)cy * I.W + cx] : 0.0f;
        ce[u] = I.ce[cy]; se[u] = I.se[cy]; ca[u] = I.ca[cx]; sa[u] = I.sa[cx];
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int e = e0 + 256 * u;
        if (e >= NE) break;
        const float dx = ce[u] * ca[u], dyy = ce[u] * sa[u];
        bf16x4 v;
        v[0] = (short)bf16_rne(r[u] * 0.0625f);
        v[1] = (short)bf16_rne((r[u] * dx) * 0.0625f);
        v[2] = (short)bf16_rne((r[u] * dyy) * 0.0625f);
        v[3] = (short)bf16_rne((r[u] * se[u]) * 0.0625f);
        *reinterpret_cast<bf16x4 *>(tile + (size_t)e * PS) = v;
      }
    }
  } else {
    constexpr int NQ = CI / 4, NE = IH * IW * NQ;   // 8-byte pieces per pixel
    for (int e0 = tid; e0 < NE; e0 += 256 * U) {
      bf16x4 v[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int e = e0 + 256 * u, px = e / NQ, q = e - px * NQ, dy = px / IW, c = px - dy * IW;
        const int iy = iy0 + dy, ix = ix0 + c;
        v[u] = bf16x4{0, 0, 0, 0};
        if (e < NE && iy >= 0 && iy < J.Hi && ix >= 0 && ix < J.Wi)
          v[u] = *reinterpret_cast<const bf16x4 *>(J.in + ((size_t)iy * J.Wi + ix) * CI + 4 * q);
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int e = e0 + 256 * u, px = e / NQ, q = e - px * NQ;
        if (e < NE) *reinterpret_cast<bf16x4 *>(tile + (size_t)px * PS + 4 * q) = v[u];
      }
    }
  }
  bf16x4 b[KSTEPS][NB];
#pragma unroll
  for (int s = 0; s < KSTEPS; s++)
#pragma unroll
    for (int nb = 0; nb < NB; nb++)
      b[s][nb] = *reinterpret_cast<const bf16x4 *>(wpk + (size_t)(nb * 16 + m) * KPAD + 16 * s + 4 * g);
  float bv[NB][4];      // bias of the four channels a lane's results hold
#pragma unroll
  for (int nb = 0; nb < NB; nb++)
#pragma unroll
    for (int i = 0; i < 4; i++) bv[nb][i] = nb * 16 + 4 * g + i < CO ? bias[nb * 16 + 4 * g + i] : 0.0f;
  __syncthreads();
  for (int t = wave; t < R * (BW / 16); t += 4) {
    const int r = t / (BW / 16), tc = t - r * (BW / 16), oy = oy0 + r;
    if (oy >= J.Ho) break;
    const int pl = 16 * tc + m;
    bf16x4 a[KSTEPS];
#pragma unroll
    for (int s = 0; s < KSTEPS; s++) {
      const int k0 = 16 * s + 4 * g, pos = k0 / CI, ci0 = k0 % CI;
      a[s] = pos < 9 ? *reinterpret_cast<const bf16x4 *>(tile + ((r * SY + pos / 3) * IW + pl * SX + pos % 3) * PS + ci0)
                     : bf16x4{0, 0, 0, 0};
    }
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KSTEPS; s++)
#pragma unroll
      for (int nb = 0; nb < NB; nb++) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b[s][nb], a[s], acc[nb], 0, 0, 0);
    // lane holds D[channel nb*16 + 4g + i][pixel pl]
    const int ox = ox0 + pl;
    if (ox < J.Wo) store_channels<CO, NB, LAST>(J.out, (size_t)oy * J.Wo + ox, acc, bv, g);
  }
}

// Workspace of one frame: packed weights, activations a0..a3 (bf16 NHWC),
// backward gradients dz1..dz3 (FP32 NHWC).
struct NetWork {
  uint16_t *wpk, *a0, *a1, *a2, *a3;
  float *dz1, *dz2, *dz3;
  float *part;            // per-chunk weight gradient sums of the layer in progress
  size_t bytes;
};

constexpr int kGradChunk = 4096;     // output pixels per weight-gradient block

// Largest per-chunk partial-sum table of the four layers (floats).
static size_t net_grad_part_elems(int H, int W) {
  const int npx[4] = {(H / 2) * (W / 2), (H / 4) * (W / 4), (H / 4) * (W / 8), (H / 4) * (W / 8)};
  size_t most = 0;
  for (int l = 0; l < kNetLayers; l++) {
    const NetLayerDesc d = net_layer(l);
    const size_t n = (size_t)((npx[l] + kGradChunk - 1) / kGradChunk) * (d.co * d.ci * 9 + d.co);
    most = n > most ? n : most;
  }
  return most;
}

static size_t a256n(size_t x) { return (x + 255) & ~(size_t)255; }

static NetWork net_work(char *base, int H, int W) {
  NetWork w;
  size_t at = 0;
  auto take = [&](size_t n) { char *p = base ? base + at : nullptr; at += a256n(n); return p; };
  w.wpk = (uint16_t *)take(2 * (size_t)net_packed_elems());
  w.a0 = (uint16_t *)take(2 * 4 * (size_t)H * W);
  w.a1 = (uint16_t *)take(2 * 16 * (size_t)(H / 2) * (W / 2));
  w.a2 = (uint16_t *)take(2 * 32 * (size_t)(H / 4) * (W / 4));
  w.a3 = (uint16_t *)take(2 * 32 * (size_t)(H / 4) * (W / 8));
  w.dz1 = (float *)take(4 * 16 * (size_t)(H / 2) * (W / 2));
  w.dz2 = (float *)take(4 * 32 * (size_t)(H / 4) * (W / 4));
  w.dz3 = (float *)take(4 * 32 * (size_t)(H / 4) * (W / 8));
  w.part = (float *)take(4 * net_grad_part_elems(H, W));
  w.bytes = at;
  return w;
}

size_t net_workspace_bytes(int H, int W) { return net_work(nullptr, H, W).bytes; }

template <int CI, int CO, int SY, int SX, bool LAST>
static void launch_conv(const ConvJob &j, const ConvJob *jobs, int njobs, int max_px, const uint16_t *wpk,
                        const float *bias, hipStream_t st) {
  const int blocks = (max_px + 64 * kMT - 1) / (64 * kMT);
  hipLaunchKernelGGL((k_net_conv<CI, CO, SY, SX, LAST>), dim3(blocks, njobs), dim3(256), 0, st, j, jobs, wpk, bias);
}

// LDS-staged convolution over output rows of at most max_ho rows and max_wo
// columns (per frame: j; or the table jobs[njobs]).
template <int CI, int CO, int SY, int SX, bool LAST, bool RANGE, int BW, int R>
static void launch_conv_lds(const ConvJob &j, const ConvJob *jobs, const NetInputJob *in_jobs, int njobs, int max_ho,
                            int max_wo, const uint16_t *wpk, const float *bias, hipStream_t st) {
  const int blocks = ((max_ho + R - 1) / R) * ((max_wo + BW - 1) / BW);
  hipLaunchKernelGGL((k_net_conv_lds<CI, CO, SY, SX, LAST, RANGE, BW, R>), dim3(blocks, njobs), dim3(256), 0, st, j,
                     jobs, in_jobs, wpk, bias);
}

// Layers 1-4 given a0: per frame (jobs == NULL, j* used) or a table of frames.
void net_layers(const float *params, const uint16_t *wpk, const ConvJob *j, const ConvJob *jobs, int njobs,
                const int *max_px, hipStream_t st) {
  launch_conv<4, 16, 2, 2, false>(j[0], jobs ? jobs : nullptr, njobs, max_px[0], wpk + net_layer(0).poff,
                                  params + net_layer(0).boff, st);
  launch_conv<16, 32, 2, 2, false>(j[1], jobs ? jobs + njobs : nullptr, njobs, max_px[1], wpk + net_layer(1).poff,
                                   params + net_layer(1).boff, st);
  launch_conv_lds<32, 32, 1, 2, false, false, 64, 4>(j[2], jobs ? jobs + 2 * njobs : nullptr, nullptr, njobs, j[2].Ho,
                                                  j[2].Wo, wpk + net_layer(2).poff, params + net_layer(2).boff, st);
  launch_conv_lds<32, 4, 1, 1, true, false, 128, 2>(j[3], jobs ? jobs + 3 * njobs : nullptr, nullptr, njobs, j[3].Ho,
                                                 j[3].Wo, wpk + net_layer(3).poff, params + net_layer(3).boff, st);
}

void net_pack(const float *params, uint16_t *wpk, hipStream_t st) {
  const int n = net_packed_elems();
  hipLaunchKernelGGL(k_net_pack, dim3((n + 255) / 256), dim3(256), 0, st, params, wpk);
}

void net_input(const float *range, const SensorDev &s, uint16_t *a0, hipStream_t st) {
  const int n = s.H * s.W;
  NetInputJob j{range, a0, s.ce, s.se, s.ca, s.sa, s.H, s.W};
  hipLaunchKernelGGL(k_net_input, dim3((n + 255) / 256), dim3(256), 0, st, j, (const NetInputJob *)nullptr);
}

// Forward pass over many frames: input jobs in_jobs[n], convolution jobs
// conv_jobs[4][n] (device tables); max_px[0] = largest H*W, max_px[1 + l] =
// largest output of layer l.
void net_forward_batch(const float *params, uint16_t *wpk, const NetInputJob *in_jobs, const ConvJob *conv_jobs, int n,
                       int max_h, int max_w, hipStream_t st) {
  net_pack(params, wpk, st);
  launch_conv_lds<4, 16, 2, 2, false, true, 128, 2>(ConvJob{}, conv_jobs, in_jobs, n, max_h / 2, max_w / 2,
                                                 wpk + net_layer(0).poff, params + net_layer(0).boff, st);
  // the second layer reads each input pixel about twice (stride 2): direct
  // gathers beat staging it in LDS
  launch_conv<16, 32, 2, 2, false>(ConvJob{}, conv_jobs + n, n, (max_h / 4) * (max_w / 4), wpk + net_layer(1).poff,
                                   params + net_layer(1).boff, st);
  launch_conv_lds<32, 32, 1, 2, false, false, 64, 4>(ConvJob{}, conv_jobs + 2 * n, nullptr, n, max_h / 4, max_w / 8,
                                                  wpk + net_layer(2).poff, params + net_layer(2).boff, st);
  launch_conv_lds<32, 4, 1, 1, true, false, 128, 2>(ConvJob{}, conv_jobs + 3 * n, nullptr, n, max_h / 4, max_w / 8,
                                                 wpk + net_layer(3).poff, params + net_layer(3).boff, st);
}

size_t net_packed_bytes() { return 2 * (size_t)net_packed_elems(); }

size_t net_forward_act_bytes(int H, int W, size_t *a0, size_t *a1, size_t *a2, size_t *a3) {
  *a0 = a256n(2 * 4 * (size_t)H * W);
  *a1 = a256n(2 * 16 * (size_t)(H / 2) * (W / 2));
  *a2 = a256n(2 * 32 * (size_t)(H / 4) * (W / 4));
  *a3 = a256n(2 * 32 * (size_t)(H / 4) * (W / 8));
  return *a0 + *a1 + *a2 + *a3;
}

hipError_t net_forward(const float *params, const float *range, const SensorDev &s, char *work, float *seed,
                       hipStream_t st) {
  const int H = s.H, W = s.W;
  NetWork w = net_work(work, H, W);
  net_pack(params, w.wpk, st);
  net_input(range, s, w.a0, st);
  ConvJob j[4] = {{w.a0, H, W, w.a1, H / 2, W / 2},
                  {w.a1, H / 2, W / 2, w.a2, H / 4, W / 4},
                  {w.a2, H / 4, W / 4, w.a3, H / 4, W / 8},
                  {w.a3, H / 4, W / 8, seed, H / 4, W / 8}};
  const int px[4] = {j[0].Ho * j[0].Wo, j[1].Ho * j[1].Wo, j[2].Ho * j[2].Wo, j[3].Ho * j[3].Wo};
  net_layers(params, w.wpk, j, nullptr, 1, px, st);
  return hipGetLastError();
}

// ----------------------------------------------------------------- backward
// Weight and bias gradients of one layer: a block per (out channel, input
// channel, pixel chunk); nine partial sums per thread, block reduction in a
// fixed tree, the block's sums written to its chunk's row of part
// ([chunk][CO * CI * 9 weights, then CO biases]); k_net_grad_sum adds the
// rows in chunk order, so the gradient does not depend on scheduling.
template <int CI, int CO, int SY, int SX>
__global__ void __launch_bounds__(256) k_net_wgrad(const uint16_t *__restrict__ ain, int Hi, int Wi,
                                                   const float *__restrict__ dz, int Ho, int Wo, float *__restrict__ part,
                                                   int chunk) {
  const int co = blockIdx.x / CI, ci = blockIdx.x % CI;
  const int p_begin = blockIdx.y * chunk, p_end = min(Ho * Wo, p_begin + chunk);
  float acc[10];
#pragma unroll
  for (int q = 0; q < 10; q++) acc[q] = 0.0f;
  for (int p = p_begin + threadIdx.x; p < p_end; p += 256) {
    const int oy = p / Wo, ox = p - oy * Wo;
    const float g = dz[(size_t)p * CO + co];
    acc[9] += g;
#pragma unroll
    for (int pos = 0; pos < 9; pos++) {
      const int iy = oy * SY - 1 + pos / 3, ix = ox * SX - 1 + pos % 3;
      if (iy >= 0 && iy < Hi && ix >= 0 && ix < Wi) acc[pos] += g * bf16_val(ain[((size_t)iy * Wi + ix) * CI + ci]);
    }
  }
  __shared__ float red[10][256];
#pragma unroll
  for (int q = 0; q < 10; q++) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
#pragma unroll
      for (int q = 0; q < 10; q++) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  float *row = part + (size_t)blockIdx.y * (CO * CI * 9 + CO);
  if (threadIdx.x < 9) row[(co * CI + ci) * 9 + threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 9 && ci == 0) row[CO * CI * 9 + co] = red[9][0];
}

// grad[e] += sum over chunks c = 0, 1, ... of part[c][e] for the nw weight
// and nb bias gradients of one layer (gW, gb).
__global__ void __launch_bounds__(256) k_net_grad_sum(const float *__restrict__ part, int nchunk, int nw, int nb,
                                                      float *__restrict__ gW, float *__restrict__ gb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nw + nb) return;
  float s = 0.0f;
  for (int c = 0; c < nchunk; c++) s += part[(size_t)c * (nw + nb) + e];
  if (e < nw) gW[e] += s;
  else gb[e - nw] += s;
}

// Gradient of a layer's input through the convolution (bfloat16 weights)
// and the previous ReLU: dz_in[iy][ix][ci] = [a_in > 0] sum W dz.
template <int CI, int CO, int SY, int SX>
__global__ void __launch_bounds__(256) k_net_dgrad(const uint16_t *__restrict__ wpk, const float *__restrict__ dz, int Ho,
                                                   int Wo, const uint16_t *__restrict__ ain, int Hi, int Wi,
                                                   float *__restrict__ dzin) {
  constexpr int KPAD = net_kpad(CI);
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)Hi * Wi * CI) return;
  const int ci = (int)(e % CI);
  const int px = (int)(e / CI), iy = px / Wi, ix = px - iy * Wi;
  float s = 0.0f;
  if (bf16_val(ain[e]) > 0.0f) {
    for (int pos = 0; pos < 9; pos++) {
      const int ty = iy + 1 - pos / 3, tx = ix + 1 - pos % 3;
      if (ty < 0 || tx < 0 || ty % SY || tx % SX) continue;
      const int oy = ty / SY, ox = tx / SX;
      if (oy >= Ho || ox >= Wo) continue;
      const float *d = dz + ((size_t)oy * Wo + ox) * CO;
      for (int co = 0; co < CO; co++) s += bf16_val(wpk[(size_t)co * KPAD + pos * CI + ci]) * d[co];
    }
  }
  dzin[e] = s;
}

// Weight and bias gradients of layer l (its output grid npx pixels) from its
// input activations and output gradient, added to grad in a fixed order.
template <int CI, int CO, int SY, int SX>
static void layer_wgrad(int l, const uint16_t *ain, int Hi, int Wi, const float *dz, int Ho, int Wo, float *part,
                        float *grad, hipStream_t st) {
  const NetLayerDesc d = net_layer(l);
  const int nchunk = (Ho * Wo + kGradChunk - 1) / kGradChunk, nw = CO * CI * 9;
  hipLaunchKernelGGL((k_net_wgrad<CI, CO, SY, SX>), dim3(CO * CI, nchunk), dim3(256), 0, st, ain, Hi, Wi, dz, Ho, Wo,
                     part, kGradChunk);
  hipLaunchKernelGGL(k_net_grad_sum, dim3((nw + CO + 255) / 256), dim3(256), 0, st, (const float *)part, nchunk, nw,
                     CO, grad + d.woff, grad + d.boff);
}

hipError_t net_backward(const float *params, const SensorDev &s, char *work, const float *dseed, float *grad,
                        hipStream_t st) {
  const int H = s.H, W = s.W;
  NetWork w = net_work(work, H, W);
  const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 4, W3 = W / 8;
  // layer 4: dz = dseed
  layer_wgrad<32, 4, 1, 1>(3, w.a3, H3, W3, dseed, H3, W3, w.part, grad, st);
  hipLaunchKernelGGL((k_net_dgrad<32, 4, 1, 1>), dim3((H3 * W3 * 32 + 255) / 256), dim3(256), 0, st,
                     w.wpk + net_layer(3).poff, dseed, H3, W3, w.a3, H3, W3, w.dz3);
  layer_wgrad<32, 32, 1, 2>(2, w.a2, H2, W2, w.dz3, H3, W3, w.part, grad, st);
  hipLaunchKernelGGL((k_net_dgrad<32, 32, 1, 2>), dim3((H2 * W2 * 32 + 255) / 256), dim3(256), 0, st,
                     w.wpk + net_layer(2).poff, w.dz3, H3, W3, w.a2, H2, W2, w.dz2);
  layer_wgrad<16, 32, 2, 2>(1, w.a1, H1, W1, w.dz2, H2, W2, w.part, grad, st);
  hipLaunchKernelGGL((k_net_dgrad<16, 32, 2, 2>), dim3((H1 * W1 * 16 + 255) / 256), dim3(256), 0, st,
                     w.wpk + net_layer(1).poff, w.dz2, H2, W2, w.a1, H1, W1, w.dz1);
  layer_wgrad<4, 16, 2, 2>(0, w.a0, H, W, w.dz1, H1, W1, w.part, grad, st);
  return hipGetLastError();
}

// --------------------------------------------------------------- loss, Adam
// Labels from a plain key-frame fit: planar = accepted; normal = the stored
// plane's unit normal; tiles with a fit attempt (status >= 2) are labelled.
// loss = mean over labelled tiles of BCE(logit, planar) + planar (1 - |cos|).
__global__ void __launch_bounds__(256) k_net_loss(const float4 *__restrict__ seed, const pc_tile_rec *__restrict__ rec,
                                                  int T, float4 *__restrict__ dseed, float *__restrict__ loss) {
  __shared__ float red[256];
  float cnt = 0.0f;
  for (int t = threadIdx.x; t < T; t += 256) cnt += rec[t].status >= 2 ? 1.0f : 0.0f;
  red[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const float inv = 1.0f / fmaxf(red[0], 1.0f);
  __syncthreads();
  float L = 0.0f;
  for (int t = threadIdx.x; t < T; t += 256) {
    const pc_tile_rec r = rec[t];
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r.status >= 2) {
      const float y = r.status == 5 ? 1.0f : 0.0f;
      const float4 s = seed[t];
      float lab[3];
      const int k = r.axis, k1 = k == 0 ? 1 : 0, k2 = k == 2 ? 1 : 2;
      lab[k] = 1.0f;
      lab[k1] = r.a;
      lab[k2] = r.b;
      const float ln = rsqrtf(lab[0] * lab[0] + lab[1] * lab[1] + lab[2] * lab[2]);
      lab[0] *= ln; lab[1] *= ln; lab[2] *= ln;
      const float logit = s.w;
      L += fmaxf(logit, 0.0f) - logit * y + log1pf(expf(-fabsf(logit)));
      g.w = (1.0f / (1.0f + expf(-logit)) - y) * inv;
      const float nn = sqrtf(s.x * s.x + s.y * s.y + s.z * s.z) + 1e-12f;
      const float cosv = (s.x * lab[0] + s.y * lab[1] + s.z * lab[2]) / nn;
      L += y * (1.0f - fabsf(cosv));
      const float f = -y * (cosv > 0.0f ? 1.0f : (cosv < 0.0f ? -1.0f : 0.0f)) * inv;
      g.x = f * (lab[0] / nn - cosv * s.x / (nn * nn));
      g.y = f * (lab[1] / nn - cosv * s.y / (nn * nn));
      g.z = f * (lab[2] / nn - cosv * s.z / (nn * nn));
    }
    dseed[t] = g;
  }
  red[threadIdx.x] = L;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] * inv;
}

__global__ void k_net_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, int n, float lr, float b1, float b2, float c1, float c2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t net_loss(const float *seed, const void *labels_stream, const pc_layout &L, float *dseed, float *loss,
                    hipStream_t st) {
  const pc_tile_rec *rec = (const pc_tile_rec *)((const char *)labels_stream + L.off_tiles);
  hipLaunchKernelGGL(k_net_loss, dim3(1), dim3(256), 0, st, (const float4 *)seed, rec, L.T, (float4 *)dseed, loss);
  return hipGetLastError();
}

hipError_t net_adam(float *w, const float *g, float *m, float *v, int step, float lr, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - pow(0.9, step)), c2 = (float)(1.0 - pow(0.999, step));
  hipLaunchKernelGGL(k_net_adam, dim3((kNetParams + 255) / 256), dim3(256), 0, st, w, g, m, v, kNetParams, lr, b1, b2,
                     c1, c2, 1e-8f);
  return hipGetLastError();
}

}  // namespace pcc

// ---------------------------------------------------------------- the ABI
using namespace pcc;

pc_status pcc_sensor_dev(pc_ctx *ctx, const pc_sensor *s, SensorDev *out);
pc_status pcc_check_sensor(const pc_sensor *s);

static pc_status net_sensor(pc_ctx *ctx, const pc_sensor *sensor, SensorDev *sd) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_status st = pcc_check_sensor(sensor);
  if (st) return st;
  if (sensor->H % 4 || sensor->W % 8)
    return set_error(PC_ERR_UNSUPPORTED, "the seed network needs H %% 4 == 0 and W %% 8 == 0 (got %d x %d)", sensor->H,
                     sensor->W);
  return pcc_sensor_dev(ctx, sensor, sd);
}

extern "C" {

size_t pc_net_workspace_size(const pc_sensor *sensor) {
  if (!sensor || sensor->H <= 0 || sensor->W <= 0) return 0;
  return net_workspace_bytes(sensor->H, sensor->W);
}

pc_status pc_net_forward(pc_ctx *ctx, const float *params, const float *range, const pc_sensor *sensor, void *work,
                         size_t work_bytes, float *seed, void *stream) {
  SensorDev sd;
  pc_status st = net_sensor(ctx, sensor, &sd);
  if (st) return st;
  if (!params || !range || !seed || !work) return set_error(PC_ERR_ARG, "params, range, seed or workspace is NULL");
  if (work_bytes < net_workspace_bytes(sensor->H, sensor->W))
    return set_error(PC_ERR_CAPACITY, "net workspace %zu bytes < %zu needed", work_bytes,
                     net_workspace_bytes(sensor->H, sensor->W));
  hipError_t e = net_forward(params, range, sd, (char *)work, seed, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(PC_ERR_DEVICE, "net forward launch failed: %s", hipGetErrorString(e));
  return PC_OK;
}

pc_status pc_net_backward(pc_ctx *ctx, const float *params, const pc_sensor *sensor, void *work, size_t work_bytes,
                          const float *dseed, float *grad, void *stream) {
  SensorDev sd;
  pc_status st = net_sensor(ctx, sensor, &sd);
  if (st) return st;
  if (!params || !dseed || !grad || !work) return set_error(PC_ERR_ARG, "params, dseed, grad or workspace is NULL");
  if (work_bytes < net_workspace_bytes(sensor->H, sensor->W))
    return set_error(PC_ERR_CAPACITY, "net workspace too small");
  hipError_t e = net_backward(params, sd, (char *)work, dseed, grad, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(PC_ERR_DEVICE, "net backward launch failed: %s", hipGetErrorString(e));
  return PC_OK;
}

pc_status pc_net_loss(pc_ctx *ctx, const float *seed, const void *labels, const pc_sensor *sensor,
                      const pc_params *params, float *dseed, float *loss, void *stream) {
  if (!ctx || !seed || !labels || !dseed || !loss) return set_error(PC_ERR_ARG, "NULL argument");
  pc_layout L;
  pc_status st = pc_stream_layout(sensor, params, &L);
  if (st) return st;
  if (L.th != 4 || L.tw != 8) return set_error(PC_ERR_UNSUPPORTED, "labels must come from 4x8 tiles");
  hipError_t e = net_loss(seed, labels, L, dseed, loss, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(PC_ERR_DEVICE, "net loss launch failed: %s", hipGetErrorString(e));
  return PC_OK;
}

pc_status pc_net_adam(pc_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t step, float lr,
                      void *stream) {
  if (!ctx || !params || !grad || !m || !v) return set_error(PC_ERR_ARG, "NULL argument");
  if (step < 1 || !(lr > 0.0f)) return set_error(PC_ERR_ARG, "step must be >= 1 and lr > 0");
  hipError_t e = net_adam(params, grad, m, v, step, lr, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(PC_ERR_DEVICE, "adam launch failed: %s", hipGetErrorString(e));
  return PC_OK;
}

}  // extern "C"

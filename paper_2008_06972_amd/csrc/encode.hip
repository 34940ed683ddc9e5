// Per-frame launches of the key-frame and predicted-frame encoders: one
// work-group per tile-row strip, then one block computing the frame's size.
#include "encode_strip.h"

namespace pcc {

template <int TH, int TW>
__global__ void __launch_bounds__(kBlock, kStripWavesPerEU) k_encode_key(const float *__restrict__ range, SensorDev s, EncParams p,
                                                       const float *__restrict__ seed, FrameDev f) {
  extern __shared__ __align__(16) char smem_raw[];
  StripSrc src{range, nullptr, nullptr, 0, 0, nullptr};
  key_strip<TH, TW>(smem_raw, src, s, p, seed, f, blockIdx.x);
}

template <int TH, int TW>
__global__ void __launch_bounds__(kBlock, kStripWavesPerEU) k_encode_pred(const float *__restrict__ range, SensorDev s, EncParams p,
                                                        FrameDev key, FrameDev f) {
  extern __shared__ __align__(16) char smem_raw[];
  StripSrc src{range, nullptr, nullptr, 0, 0, nullptr};
  pred_strip<TH, TW>(smem_raw, key, src, s, p, f, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_finish_frame(FrameDev f, int kind, Mat12 M, int hasM) {
  finish_frame(f, kind, M, hasM);
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

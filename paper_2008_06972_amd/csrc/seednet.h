// Plane-seed network: job tables for running its forward pass over many
// frames (used by the batched encoder).
#pragma once
#include "pc_internal.h"

namespace pcc {

struct ConvJob {
  const uint16_t *in;     // NHWC bf16, Hi x Wi x ci
  int Hi, Wi;
  void *out;              // NHWC bf16 Ho x Wo x co, or FP32 [Ho][Wo][4] for the last layer
  int Ho, Wo;
};

struct NetInputJob {
  const float *range;     // H x W FP32 range image
  uint16_t *a0;           // H x W x 4 bf16 input channels
  const float *ce, *se, *ca, *sa;
  int H, W;
};

// Bytes of the packed bf16 weights, and of one frame's forward activations
// a0..a3 (bf16).
size_t net_packed_bytes();
size_t net_forward_act_bytes(int H, int W, size_t *a0, size_t *a1, size_t *a2, size_t *a3);

// Forward pass over n frames: in_jobs[n] and conv_jobs[4][n] in device
// memory; max_h, max_w: the largest frame height and width.
void net_forward_batch(const float *params, uint16_t *wpk, const NetInputJob *in_jobs, const ConvJob *conv_jobs, int n,
                       int max_h, int max_w, hipStream_t st);

}  // namespace pcc

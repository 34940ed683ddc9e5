// Internal declarations shared by the HIP sources of the encoder library.
// gfx950 only; every kernel is wave64 and uses no matrix cores except the
// seed network's convolutions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pc.h"

namespace pcc {

constexpr int kBlock = 256;            // threads per strip work-group
constexpr int kStripWavesPerEU = 3;  // strip encoders: three work-groups of four waves per CU (registers <= 168)
constexpr size_t kMaxStripLds = 159 * 1024;   // LDS a strip work-group may take (160 KiB per CU, less static use)
constexpr float kNearDegenerate = 1e-4f;   // FP32 eigen gap below this * lambda_max -> FP64 solve
constexpr double kDegenerate = 1e-6;       // lambda_mid <= this * lambda_max -> no plane
constexpr int kHeaderBytes = 112;          // per-frame header: 64 bytes of fields, the transform (12 FP32)
constexpr int kTableBytes = 128;           // code-length table per non-empty stream

enum : int { ST_EMPTY = 0, ST_FEW = 1, ST_DEGENERATE = 2, ST_FAILED = 3, ST_REJECTED = 4, ST_ACCEPTED = 5 };
enum : int { CLS_EMPTY = 0, CLS_UNFIT = 1, CLS_SPATIAL = 2, CLS_TEMPORAL = 3 };
enum : int { S_OCC = 0, S_RUN = 1, S_MASK = 2, S_RES = 3 };

// Sensor tables in device memory (FP32 values rounded once from FP64).
struct SensorDev {
  int H, W;
  float beta0;          // angle of column 0's leading edge (search start only)
  float dth;            // 2 pi / W (search start only)
  float inv_dth;        // W / (2 pi) (search start only)
  float elev0, inv_de;  // first beam's elevation, beams per radian (search start only)
  const float *cut;     // H+1: tan of row cuts, [0] top edge, [H] bottom edge
  const float *ebx, *eby;   // W: leading-edge unit vectors
  const float *ce, *se;     // H: cos/sin of beam elevation
  const float *ca, *sa;     // W: cos/sin of column-centre azimuth
};

struct EncParams {
  float eps;
  int th, tw, max_iter, min_pts;
  float rho;
  float step, inv;      // residual quantiser: step = 2 eps (1 - 2^-8), inv = 1/step
  int lanes;            // most lanes that share one tile in the fit, temporal and reach passes (1, 2, 4)
  uint8_t need[72];     // need[n] = max(min(min_pts, n), ceil(rho n)) for n = 0..64
};

struct Mat12 {
  float m[12];   // rows of [R | T]
};

// Device pointers into one frame stream buffer.
struct FrameDev {
  pc_frame_info *info;
  uint32_t *occ;
  uint8_t *cls;
  uint64_t *mask;
  int32_t *run_of;
  int32_t *nruns;       // [2*TR]
  pc_run *sruns;        // [T]
  pc_prun *pruns;       // [T]
  int32_t *nres;        // [TR]
  uint16_t *res;        // [H*W]
  uint32_t *strip;      // [TR][PC_STRIP_WORDS]
  pc_tile_rec *tiles;   // [T]
  int TR, TC, T;
};

FrameDev frame_dev(void *base, const pc_layout &L);

// Host helpers implemented in api.hip
pc_status set_error(pc_status st, const char *fmt, ...);

// Kernel launchers (project.hip, encode.hip, decode.hip)
hipError_t launch_project(const float *xyz, int64_t n, const float *M, const SensorDev &s,
                          unsigned long long *keys, float *range, int32_t *src_idx,
                          pc_proj_stats *stats, hipStream_t st);
hipError_t launch_key(const float *range, const SensorDev &s, const EncParams &p, const float *seed,
                      const FrameDev &f, const float *M12, hipStream_t st);
hipError_t launch_pred(const FrameDev &key, const float *range, const SensorDev &s, const EncParams &p,
                       const FrameDev &f, const float *M12, hipStream_t st);
// One frame of a decode launch: the frame, its key frame (temporal runs take
// the key run's normal), the output range image and points (either may be
// NULL), and whether points go back to the frame's own coordinates.
struct DecodeJob {
  FrameDev key;
  FrameDev f;
  float *out;
  float *xyz;
  int has_key;
  int frame_coords;
};
hipError_t launch_decode_jobs(const DecodeJob &j0, const DecodeJob *jobs, int n, const SensorDev &s,
                              const EncParams &p, hipStream_t st);
hipError_t launch_decode(const FrameDev *key, const FrameDev &f, const SensorDev &s, const EncParams &p,
                         float *range_out, float *xyz_out, int frame_coords, hipStream_t st);

}  // namespace pcc

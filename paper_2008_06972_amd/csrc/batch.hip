// Batched encoding of many frames of many sensors in one HIP graph.
//
// A plan holds a device table of frame descriptors.  One replay runs:
//   reset    zero the queue counters (a kernel, so the graph holds no memset
//            node)
//   bin      project every point (Eq. (1), (2), (6)); each work-group groups
//            its 4096 points by tile-row strip in LDS and writes them as one
//            chunk of (LDS slot, range bits) entries, with the chunk's first
//            entry of every strip
//   keyimage (with a seed network) the key frames' range images, built per
//            strip from the chunks in LDS
//   net      the seed network's forward pass over those key frames
//   key      persistent work-groups pull (key frame, strip) items from an
//            atomic counter; each builds its strip from its segment of every
//            chunk of the frame with LDS atomicMin (nearest point wins,
//            Sec. III-D) and encodes it
//   pred     the same for the predicted frames' strips
//   finish   one block per frame: totals and the Huffman size
// Binning needs no device-wide atomics and moves each point once (12 bytes
// read, 8 written, 8 read back by its strip); the per-pixel minimum happens
// in LDS and the range image never goes through HBM.  Phases are separate
// kernels, so a predicted strip never waits inside a kernel for its key
// strip.  Items are grouped by tile shape; each group is one launch per
// phase.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "encode_strip.h"
#include "project.h"
#include "seednet.h"

namespace pcc {

constexpr int kBinPts = 8;                 // points per thread in the binning passes
constexpr int kBinBlock = 512;
constexpr int kBinChunk = kBinPts * kBinBlock;
static_assert(kBinChunk == kBinChunkPts, "chunk capacity as the strip loader reads it");
constexpr size_t kCountTabMax = 32 * 1024;  // sensor tables up to this size go to LDS in the binning pass

struct FrameDescDev {
  const float *xyz;
  int64_t n;
  Mat12 M;
  int hasM;
  int kind;        // 0 key, 1 predicted
  int key;         // descriptor index of the key frame
  int pad0;
  SensorDev s;
  EncParams p;
  uint2 *chunks;   // nblk * kBinChunk entries (LDS slot, range bits): binning block b's kept points
                   // from b * kBinChunk on, grouped by strip
  int *blkoff;     // [nblk][TR + 1]: first entry of each strip in block b's chunk; [TR]: its kept points
  int nblk;        // binning blocks of the frame
  int twl;         // log2 tile_w
  float *range_out;
  const float *seed;
  float *net_range;  // key frame's range image for the seed network, or NULL
  FrameDev f;
};

__global__ void k_batch_reset(int *a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) a[i] = 0;
}

// blocks [first[f], first[f+1]) belong to frame f; owner[b] = f.  With
// LdsTab the sensor's cut tangents and edge vectors are first copied into
// LDS (H + 1 + 2 W floats) and the row and column walks read them there.
// Each thread projects kBinPts points and takes a rank in its strip's LDS
// count; after the block's exclusive sum over the strips, the entries are
// grouped by strip in LDS (over the tables, which are no longer needed) and
// copied out as one contiguous chunk, and the strip offsets beside it.
template <bool LdsTab>
__global__ void __launch_bounds__(kBinBlock) k_batch_bin(const FrameDescDev *__restrict__ d, const int *__restrict__ owner,
                                                         const int *__restrict__ first, int base) {
  __shared__ int cnt[256], loff[257];
  extern __shared__ __align__(16) float tabs[];      // tables, then the grouped entries
  const int blk = base + blockIdx.x;
  const int fidx = __builtin_amdgcn_readfirstlane(owner[blk]);
  const FrameDescDev &D = d[fidx];
  const int th = D.p.th, thl = __ffs(th) - 1, TR = D.f.TR, tid = threadIdx.x;     // tile heights are powers of two
  for (int t = tid; t < TR; t += kBinBlock) cnt[t] = 0;
  const int H = D.s.H, W = D.s.W;
  if (LdsTab) {
    for (int t = tid; t <= H; t += kBinBlock) tabs[t] = gload(D.s.cut + t);
    for (int t = tid; t < W; t += kBinBlock) {
      tabs[H + 1 + t] = gload(D.s.ebx + t);
      tabs[H + 1 + W + t] = gload(D.s.eby + t);
    }
  }
  typedef const __attribute__((address_space(3))) float lfloat;
  const TabLds tl{(lfloat *)tabs, (lfloat *)(tabs + H + 1), (lfloat *)(tabs + H + 1 + W)};
  const TabGlobal tg{D.s.cut, D.s.ebx, D.s.eby};
  __syncthreads();
  const int b = blk - first[fidx];
  const int64_t p0 = (int64_t)b * kBinChunk;
  const auto *xyz = (const __attribute__((address_space(1))) float *)D.xyz;
  uint64_t e[kBinPts];
  int key[kBinPts];     // strip << 16 | rank in the strip, -1 for a dropped point
#pragma unroll
  for (int q = 0; q < kBinPts; q++) {
    const int64_t i = p0 + q * kBinBlock + tid;
    key[q] = -1;
    e[q] = 0;
    if (i >= D.n) continue;
    int v, u;
    float r;
    const int st = LdsTab ? project_point(D.s, tl, D.M, D.hasM, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], v, u, r)
                          : project_point(D.s, tg, D.M, D.hasM, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], v, u, r);
    if (st == PROJ_KEPT) {
      const int strip = v >> thl;
      e[q] = (uint64_t)(uint32_t)strip_slot(v & (th - 1), u, th, D.twl) | ((uint64_t)__float_as_uint(r) << 32);
      key[q] = (strip << 16) | atomicAdd(&cnt[strip], 1);
    }
  }
  __syncthreads();
  // exclusive sum over the strips (first wavefront); the offsets go out
  // beside the chunk
  int *bo = D.blkoff + (int64_t)b * (TR + 1);
  if (tid < 64) {
    const int lane = tid;
    int carry = 0;
    for (int t0 = 0; t0 < TR; t0 += 64) {
      const int t = t0 + lane;
      const int c = t < TR ? cnt[t] : 0;
      int x = c;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (t < TR) {
        loff[t] = carry + x - c;
        bo[t] = carry + x - c;
      }
      carry += __shfl(x, 63, 64);
    }
    if (lane == 0) {
      loff[TR] = carry;
      bo[TR] = carry;
    }
  }
  __syncthreads();
  uint64_t *sorted = reinterpret_cast<uint64_t *>(tabs);
#pragma unroll
  for (int q = 0; q < kBinPts; q++)
    if (key[q] >= 0) sorted[loff[key[q] >> 16] + (key[q] & 0xffff)] = e[q];
  __syncthreads();
  auto *out = (__attribute__((address_space(1))) uint64_t *)(D.chunks) + p0;
  const int total = loff[TR];
  for (int k = tid; k < total; k += kBinBlock) out[k] = sorted[k];
}

__device__ __forceinline__ StripSrc src_of(const FrameDescDev &D) {
  return StripSrc{nullptr, D.chunks, D.blkoff, D.nblk, D.f.TR, D.range_out};
}

template <int TH, int TW>
__global__ void __launch_bounds__(kBlock, kStripWavesPerEU) k_batch_key(const FrameDescDev *__restrict__ d, const int2 *__restrict__ items,
                                                      int nitems, int *counter) {
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: descriptor fields go to scalar registers
    if (it >= nitems) break;
    const int2 fi = items[it];
    const FrameDescDev &D = d[fi.x];
    key_strip<TH, TW>(smem_raw, src_of(D), D.s, D.p, D.seed, D.f, fi.y);
  }
}

template <int TH, int TW>
__global__ void __launch_bounds__(kBlock, kStripWavesPerEU) k_batch_pred(const FrameDescDev *__restrict__ d, const int2 *__restrict__ items,
                                                       int nitems, int *counter) {
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: descriptor fields go to scalar registers
    if (it >= nitems) break;
    const int2 fi = items[it];
    const FrameDescDev &D = d[fi.x];
    pred_strip<TH, TW>(smem_raw, d[D.key].f, src_of(D), D.s, D.p, D.f, fi.y);
  }
}

// One work-group per strip (no queue), for comparison and for the autotuner.
template <int TH, int TW>
__global__ void __launch_bounds__(kBlock, kStripWavesPerEU) k_batch_key_grid(const FrameDescDev *__restrict__ d, const int2 *__restrict__ items) {
  extern __shared__ __align__(16) char smem_raw[];
  const int2 fi = items[blockIdx.x];
  const FrameDescDev &D = d[fi.x];
  key_strip<TH, TW>(smem_raw, src_of(D), D.s, D.p, D.seed, D.f, fi.y);
}

template <int TH, int TW>
__global__ void __launch_bounds__(kBlock, kStripWavesPerEU) k_batch_pred_grid(const FrameDescDev *__restrict__ d, const int2 *__restrict__ items) {
  extern __shared__ __align__(16) char smem_raw[];
  const int2 fi = items[blockIdx.x];
  const FrameDescDev &D = d[fi.x];
  pred_strip<TH, TW>(smem_raw, d[D.key].f, src_of(D), D.s, D.p, D.f, fi.y);
}

// Range image of a key frame's strip for the seed network: the strip's
// binned points resolved in LDS (nearest point wins) and written out.
template <int TH, int TW>
__global__ void __launch_bounds__(kBlock) k_batch_keyimage(const FrameDescDev *__restrict__ d,
                                                           const int2 *__restrict__ items) {
  extern __shared__ __align__(16) char smem_raw[];
  const int2 fi = items[blockIdx.x];
  const FrameDescDev &D = d[fi.x];
  StripSmem<TH, TW> sm;
  sm.r = reinterpret_cast<float *>(smem_raw);
  sm.scratch = reinterpret_cast<uint32_t *>(smem_raw + sizeof(float) * (size_t)(D.s.W / TW) * TH * TW);
  load_source<TH, TW>(sm, StripSrc{nullptr, D.chunks, D.blkoff, D.nblk, D.f.TR, D.net_range}, D.s, fi.y);
}

__global__ void __launch_bounds__(256) k_batch_finish(const FrameDescDev *__restrict__ d) {
  const FrameDescDev &D = d[blockIdx.x];
  finish_frame(D.f, D.kind, D.M, D.hasM);
}

// ------------------------------------------------------------------ host
struct Group {
  int th, tw, kind;
  int first, count;     // slice of the item array
  size_t smem;
  int grid;
};

struct BatchPlan {
  int device = 0;
  int nframes = 0;
  FrameDescDev *d_desc = nullptr;
  int2 *d_items = nullptr;
  int *d_bin_owner = nullptr, *d_bin_first = nullptr;
  // key frames' binning blocks come first, then the predicted frames'
  int bin_blocks_key = 0;
  int *d_key_frames = nullptr, *d_pred_frames = nullptr;
  int nkey = 0, npred = 0;
  // predicted frames are binned on a second stream while the key frames are
  // encoded (fork and join by events; captured as parallel graph branches)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int *d_counters = nullptr;     // queue counters (64), then the frames' strip counts
  int64_t ncounters = 0;
  int bin_blocks = 0;
  size_t count_smem = 0;     // LDS of the binning pass: its sensor tables and then its grouped entries
  int count_tab = 0;         // the sensor tables fit in LDS (else the walks read device memory)
  std::vector<Group> groups;
  int persistent = 1;
  // seed network (key frames with 4x8 tiles)
  int nnet = 0;
  const float *net_params = nullptr;
  uint16_t *net_wpk = nullptr;
  int2 *d_net_items = nullptr;
  int n_net_items = 0;
  size_t net_smem = 0;
  NetInputJob *d_net_in = nullptr;
  ConvJob *d_net_conv = nullptr;
  int net_hw[2] = {0, 0};      // largest seeded frame's H and W
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int use_graph = 0;
};

template <int TH, int TW>
static const void *key_fn(bool persistent) {
  return persistent ? (const void *)k_batch_key<TH, TW> : (const void *)k_batch_key_grid<TH, TW>;
}
template <int TH, int TW>
static const void *pred_fn(bool persistent) {
  return persistent ? (const void *)k_batch_pred<TH, TW> : (const void *)k_batch_pred_grid<TH, TW>;
}

static const void *group_fn(const Group &g, bool persistent) {
  if (g.th == 4 && g.tw == 4) return g.kind ? pred_fn<4, 4>(persistent) : key_fn<4, 4>(persistent);
  if (g.th == 4 && g.tw == 8) return g.kind ? pred_fn<4, 8>(persistent) : key_fn<4, 8>(persistent);
  if (g.th == 4 && g.tw == 16) return g.kind ? pred_fn<4, 16>(persistent) : key_fn<4, 16>(persistent);
  if (g.th == 8 && g.tw == 8) return g.kind ? pred_fn<8, 8>(persistent) : key_fn<8, 8>(persistent);
  return nullptr;
}

static size_t group_smem(int th, int tw, int W, bool pred) {
  if (th == 4 && tw == 4) return StripSmem<4, 4>::bytes(W, W / 4, pred);
  if (th == 4 && tw == 8) return StripSmem<4, 8>::bytes(W, W / 8, pred);
  if (th == 4 && tw == 16) return StripSmem<4, 16>::bytes(W, W / 16, pred);
  return StripSmem<8, 8>::bytes(W, W / 8, pred);
}

// All launches of one batch, in order; mark(kind) follows each (PC_LAUNCH_*).
// Key-frame groups always run a work-group per strip: they are a tenth of
// the strips, and their persistent form holds more registers than the
// three-work-groups-per-CU budget allows.
static hipError_t launch_group(BatchPlan &P, int gi, hipStream_t st) {
  const Group &g = P.groups[gi];
  const bool persistent = P.persistent != 0 && g.kind == 1;
  const void *fn = group_fn(g, persistent);
  const int2 *items = P.d_items + g.first;
  int nitems = g.count;
  int *counter = P.d_counters + gi;
  if (persistent) {
    void *args[] = {(void *)&P.d_desc, (void *)&items, (void *)&nitems, (void *)&counter};
    return hipLaunchKernel(fn, dim3(g.grid), dim3(kBlock), args, g.smem, st);
  }
  void *args[] = {(void *)&P.d_desc, (void *)&items};
  return hipLaunchKernel(fn, dim3(g.count), dim3(kBlock), args, g.smem, st);
}

// Binning of one frame subset.
template <class Mark>
static void bin_frames(BatchPlan &P, bool key, hipStream_t st, Mark mark) {
  const int nb = key ? P.bin_blocks_key : P.bin_blocks - P.bin_blocks_key;
  const int base = key ? 0 : P.bin_blocks_key;
  if (!nb) return;
  if (P.count_tab)
    hipLaunchKernelGGL(k_batch_bin<true>, dim3(nb), dim3(kBinBlock), P.count_smem, st, P.d_desc, P.d_bin_owner,
                       P.d_bin_first, base);
  else
    hipLaunchKernelGGL(k_batch_bin<false>, dim3(nb), dim3(kBinBlock), P.count_smem, st, P.d_desc, P.d_bin_owner,
                       P.d_bin_first, base);
  mark(PC_LAUNCH_COUNT);
}

// All launches of one batch, in order; mark(kind) follows each (PC_LAUNCH_*).
// concurrent: the predicted frames' binning runs on the side stream while
// the key frames are binned, seeded and encoded; serial: one stream.
template <class Mark>
static hipError_t batch_launches(BatchPlan &P, hipStream_t st, Mark mark, bool concurrent) {
  const int ngroups = (int)P.groups.size();
  int rb = (int)std::min<int64_t>(1024, (P.ncounters + 255) / 256);
  hipLaunchKernelGGL(k_batch_reset, dim3(rb), dim3(256), 0, st, P.d_counters, P.ncounters);
  mark(PC_LAUNCH_RESET);
  concurrent = concurrent && P.side && P.npred > 0;
  if (concurrent) {
    hipEventRecord(P.ev_fork, st);
    hipStreamWaitEvent(P.side, P.ev_fork, 0);
    bin_frames(P, false, P.side, mark);
    hipEventRecord(P.ev_join, P.side);
  }
  bin_frames(P, true, st, mark);
  if (!concurrent) bin_frames(P, false, st, mark);
  if (P.nnet) {
    hipLaunchKernelGGL((k_batch_keyimage<4, 8>), dim3(P.n_net_items), dim3(kBlock), P.net_smem, st, P.d_desc,
                       P.d_net_items);
    mark(PC_LAUNCH_KEYIMAGE);
    net_forward_batch(P.net_params, P.net_wpk, P.d_net_in, P.d_net_conv, P.nnet, P.net_hw[0], P.net_hw[1], st);
    mark(PC_LAUNCH_NET);
  }
  for (int pass = 0; pass < 2; pass++) {      // key groups, then predicted groups
    if (pass == 1 && concurrent) hipStreamWaitEvent(st, P.ev_join, 0);
    for (int gi = 0; gi < ngroups; gi++) {
      const Group &g = P.groups[gi];
      if (g.kind != pass || g.count == 0) continue;
      hipError_t e = launch_group(P, gi, st);
      if (e != hipSuccess) return e;
      mark(pass == 0 ? PC_LAUNCH_KEY : PC_LAUNCH_PRED);
    }
  }
  hipLaunchKernelGGL(k_batch_finish, dim3(P.nframes), dim3(256), 0, st, P.d_desc);
  mark(PC_LAUNCH_FINISH);
  return hipGetLastError();
}

}  // namespace pcc

// ---------------------------------------------------------------- the ABI
using namespace pcc;

struct pc_batch {
  BatchPlan plan;
};

// defined in api.hip
pc_status pcc_sensor_dev(pc_ctx *ctx, const pc_sensor *s, SensorDev *out);
pc_status pcc_check_all(const pc_sensor *s, const pc_params *p);
EncParams pcc_enc_params(const pc_params *p);
int pcc_ctx_device(pc_ctx *ctx);

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchSizes {
  size_t desc, items, bins, counters, buckets, net, total;
  int nitems, bin_blocks, nnet, net_items;
  int64_t strips;
};

// Does frame i get seeds from the batch's network?  Key frames with 4x8
// tiles, a sensor the network takes, and no seeds of their own.
static bool net_frame(const pc_frame_desc &F, int i, const pc_batch_opts *o) {
  return o && o->net && F.key == i && !F.seed && F.params->tile_h == 4 && F.params->tile_w == 8 &&
         F.sensor->H % 4 == 0 && F.sensor->W % 8 == 0;
}

// Network workspace of one frame: range image, activations, seeds.
static size_t net_frame_bytes(int H, int W) {
  size_t a0, a1, a2, a3;
  return a256(4 * (size_t)H * W) + net_forward_act_bytes(H, W, &a0, &a1, &a2, &a3) +
         a256(16 * (size_t)(H / 4) * (W / 8));
}

static pc_status batch_sizes(const pc_frame_desc *frames, int32_t nframes, const pc_batch_opts *opts,
                             BatchSizes &B) {
  memset(&B, 0, sizeof B);
  int64_t items = 0, bb = 0, strips = 0;
  size_t buckets = 0, net = 0;
  int nnet = 0, net_items = 0;
  for (int i = 0; i < nframes; i++) {
    const pc_frame_desc &F = frames[i];
    if (!F.sensor || !F.params) return set_error(PC_ERR_ARG, "frame %d: sensor or params is NULL", i);
    if (F.n < 0) return set_error(PC_ERR_ARG, "frame %d: negative point count", i);
    int tr = F.sensor->H / (F.params->tile_h > 0 ? F.params->tile_h : 1);
    items += tr;
    strips += tr;
    const int64_t nblk = (F.n + kBinChunk - 1) / kBinChunk;
    bb += nblk;
    buckets += a256(sizeof(uint2) * (size_t)nblk * kBinChunk) + a256(sizeof(int) * (size_t)nblk * (tr + 1));
    if (net_frame(F, i, opts)) {
      nnet++;
      net_items += tr;
      net += net_frame_bytes(F.sensor->H, F.sensor->W);
    }
  }
  if (items > 0x7fffffff || bb > 0x7fffffff) return set_error(PC_ERR_CAPACITY, "batch too large");
  if (nnet) net += a256(net_packed_bytes()) + a256(sizeof(NetInputJob) * nnet) + a256(sizeof(ConvJob) * 4 * nnet) +
                   a256(sizeof(int2) * net_items);
  B.nitems = (int)items;
  B.bin_blocks = (int)bb;
  B.strips = strips;
  B.nnet = nnet;
  B.net_items = net_items;
  B.desc = a256(sizeof(FrameDescDev) * (size_t)nframes);
  B.items = a256(sizeof(int2) * (size_t)items);
  B.bins = a256(sizeof(int) * ((size_t)bb + 2 * (size_t)nframes));     // owner, first, frame lists
  B.counters = a256(sizeof(int) * 64);
  B.buckets = buckets;
  B.net = net;
  B.total = B.desc + B.items + B.bins + B.counters + B.buckets + B.net;
  return PC_OK;
}

extern "C" {

size_t pc_batch_workspace_size(const pc_frame_desc *frames, int32_t nframes, const pc_batch_opts *opts) {
  BatchSizes B;
  if (!frames || nframes <= 0 || batch_sizes(frames, nframes, opts, B) != PC_OK) return 0;
  return B.total;
}

pc_status pc_batch_create(pc_ctx *ctx, const pc_frame_desc *frames, int32_t nframes, const pc_batch_opts *opts,
                          void *workspace, size_t ws_bytes, pc_batch **out) {
  if (!ctx || !out) return set_error(PC_ERR_ARG, "ctx or output is NULL");
  if (!frames || nframes <= 0) return set_error(PC_ERR_ARG, "no frames");
  BatchSizes B;
  pc_status st = batch_sizes(frames, nframes, opts, B);
  if (st) return st;
  if (!workspace || ws_bytes < B.total)
    return set_error(PC_ERR_CAPACITY, "batch workspace %zu bytes < %zu needed", ws_bytes, B.total);
  pc_batch_opts o = opts ? *opts : pc_batch_opts{1, 1, 0, 0, nullptr, 0};
  if (o.records != 0 && o.records != 1) return set_error(PC_ERR_ARG, "records must be 0 or 1");
  if (o.lanes_max != 0 && o.lanes_max != 1 && o.lanes_max != 2 && o.lanes_max != 4)
    return set_error(PC_ERR_ARG, "lanes_max must be 0, 1, 2 or 4");
  if (o.blocks_per_cu < 0) return set_error(PC_ERR_ARG, "blocks_per_cu must be >= 0");
  char *ws = (char *)workspace;
  int *counters = (int *)(ws + B.desc + B.items + B.bins);
  char *bucket_ws = ws + B.desc + B.items + B.bins + B.counters;
  char *net_ws = bucket_ws + B.buckets;
  std::vector<FrameDescDev> desc((size_t)nframes);
  // seed network: packed weights, job tables, strip items, then per frame
  // range image, activations and seeds
  uint16_t *net_wpk = nullptr;
  NetInputJob *d_net_in = nullptr;
  ConvJob *d_net_conv = nullptr;
  int2 *d_net_items = nullptr;
  std::vector<NetInputJob> net_in;
  std::vector<ConvJob> net_conv[4];
  std::vector<int2> net_items;
  int net_hw[2] = {0, 0};
  int net_maxW = 0;
  if (B.nnet) {
    net_wpk = (uint16_t *)net_ws;
    net_ws += a256(net_packed_bytes());
    d_net_in = (NetInputJob *)net_ws;
    net_ws += a256(sizeof(NetInputJob) * B.nnet);
    d_net_conv = (ConvJob *)net_ws;
    net_ws += a256(sizeof(ConvJob) * 4 * B.nnet);
    d_net_items = (int2 *)net_ws;
    net_ws += a256(sizeof(int2) * B.net_items);
  }
  for (int i = 0; i < nframes; i++) {
    const pc_frame_desc &F = frames[i];
    if ((st = pcc_check_all(F.sensor, F.params))) return st;
    if (F.n > 0x7fffffffLL || (F.n > 0 && !F.xyz)) return set_error(PC_ERR_ARG, "frame %d: bad points", i);
    if (!F.out) return set_error(PC_ERR_ARG, "frame %d: output stream is NULL", i);
    if (F.key < 0 || F.key >= nframes) return set_error(PC_ERR_ARG, "frame %d: key index out of range", i);
    const pc_frame_desc &K = frames[F.key];
    if (K.key != F.key) return set_error(PC_ERR_ARG, "frame %d: its key frame %d is not a key frame", i, F.key);
    if (K.sensor->H != F.sensor->H || K.sensor->W != F.sensor->W || K.params->tile_h != F.params->tile_h ||
        K.params->tile_w != F.params->tile_w)
      return set_error(PC_ERR_ARG, "frame %d: sensor or tile shape differs from its key frame", i);
    if (F.M && F.key != i)
      for (int q = 0; q < 16; q++)
        if (!std::isfinite(F.M[q])) return set_error(PC_ERR_ARG, "frame %d: transform has a non-finite entry", i);
    FrameDescDev &D = desc[i];
    memset(&D, 0, sizeof D);
    D.xyz = F.xyz;
    D.n = F.n;
    D.hasM = (F.M && F.key != i) ? 1 : 0;
    for (int q = 0; q < 12; q++) D.M.m[q] = D.hasM ? F.M[q] : (q % 5 == 0 ? 1.f : 0.f);
    D.kind = F.key == i ? 0 : 1;
    D.key = F.key;
    if ((st = pcc_sensor_dev(ctx, F.sensor, &D.s))) return st;
    D.p = pcc_enc_params(F.params);
    D.p.lanes = o.lanes_max ? o.lanes_max : 4;
    pc_layout L;
    pc_stream_layout(F.sensor, F.params, &L);
    if (L.TR > 256) return set_error(PC_ERR_UNSUPPORTED, "frame %d: more than 256 tile-row strips", i);
    D.f = frame_dev(F.out, L);
    if (!o.records) D.f.tiles = nullptr;     // per-tile fit records are diagnostics only
    D.nblk = (int)((F.n + kBinChunk - 1) / kBinChunk);
    D.chunks = (uint2 *)bucket_ws;
    bucket_ws += a256(sizeof(uint2) * (size_t)D.nblk * kBinChunk);
    D.blkoff = (int *)bucket_ws;
    bucket_ws += a256(sizeof(int) * (size_t)D.nblk * (L.TR + 1));
    D.twl = __builtin_ctz((unsigned)F.params->tile_w);
    D.range_out = F.range;
    D.seed = F.seed;
    if (net_frame(F, i, &o)) {
      const int H = F.sensor->H, W = F.sensor->W;
      size_t a0b, a1b, a2b, a3b;
      net_forward_act_bytes(H, W, &a0b, &a1b, &a2b, &a3b);
      float *range = (float *)net_ws;
      net_ws += a256(4 * (size_t)H * W);
      uint16_t *a0 = (uint16_t *)net_ws, *a1 = (uint16_t *)(net_ws + a0b), *a2 = (uint16_t *)(net_ws + a0b + a1b),
               *a3 = (uint16_t *)(net_ws + a0b + a1b + a2b);
      net_ws += a0b + a1b + a2b + a3b;
      float *seedbuf = (float *)net_ws;
      net_ws += a256(16 * (size_t)(H / 4) * (W / 8));
      D.net_range = range;
      D.seed = seedbuf;
      net_in.push_back(NetInputJob{range, a0, D.s.ce, D.s.se, D.s.ca, D.s.sa, H, W});
      net_conv[0].push_back(ConvJob{a0, H, W, a1, H / 2, W / 2});
      net_conv[1].push_back(ConvJob{a1, H / 2, W / 2, a2, H / 4, W / 4});
      net_conv[2].push_back(ConvJob{a2, H / 4, W / 4, a3, H / 4, W / 8});
      net_conv[3].push_back(ConvJob{a3, H / 4, W / 8, seedbuf, H / 4, W / 8});
      net_hw[0] = std::max(net_hw[0], H);
      net_hw[1] = std::max(net_hw[1], W);
      net_maxW = std::max(net_maxW, W);
      for (int tr = 0; tr < L.TR; tr++) net_items.push_back(make_int2(i, tr));
    }
  }
  // items grouped by (kind, tile shape); inside a group, frames in order
  pc_batch *b = new pc_batch();
  BatchPlan &P = b->plan;
  P.device = pcc_ctx_device(ctx);
  P.nframes = nframes;
  P.persistent = o.persistent;
  P.use_graph = o.graph;
  {
    size_t tab = 0;
    for (int i = 0; i < nframes; i++)
      tab = std::max(tab, sizeof(float) * (size_t)(desc[i].s.H + 1 + 2 * desc[i].s.W));
    P.count_tab = tab <= kCountTabMax ? 1 : 0;
    P.count_smem = std::max(P.count_tab ? tab : (size_t)0, sizeof(uint64_t) * (size_t)kBinChunk);
  }
  std::vector<int2> items;
  items.reserve(B.nitems);
  int cus = 0;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P.device);
  const int shapes[4][2] = {{4, 4}, {4, 8}, {4, 16}, {8, 8}};
  for (int kind = 0; kind < 2; kind++)
    for (auto &sh : shapes) {
      Group g{sh[0], sh[1], kind, (int)items.size(), 0, 0, 0};
      int maxW = 0;
      int maxTR = 0;
      for (int i = 0; i < nframes; i++) {
        if (desc[i].kind != kind || desc[i].p.th != sh[0] || desc[i].p.tw != sh[1]) continue;
        maxTR = std::max(maxTR, desc[i].f.TR);
        maxW = std::max(maxW, desc[i].s.W);
      }
      for (int tr = 0; tr < maxTR; tr++)
        for (int i = 0; i < nframes; i++) {
          if (desc[i].kind != kind || desc[i].p.th != sh[0] || desc[i].p.tw != sh[1] || tr >= desc[i].f.TR) continue;
          items.push_back(make_int2(i, tr));
        }
      g.count = (int)items.size() - g.first;
      if (!g.count) continue;
      g.smem = group_smem(sh[0], sh[1], maxW, kind == 1);
      const void *fn = group_fn(g, P.persistent != 0);
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.smem) != hipSuccess) {
        delete b;
        return set_error(PC_ERR_DEVICE, "shared memory attribute failed");
      }
      // Persistent grid: generous; work-groups that start after the queue is
      // empty exit at once, so over-provisioning costs nothing.
      int per_cu = o.blocks_per_cu > 0 ? o.blocks_per_cu : 4;
      g.grid = std::min(g.count, std::max(1, cus * per_cu));
      P.groups.push_back(g);
    }
  if ((int)P.groups.size() > 64) { delete b; return set_error(PC_ERR_CAPACITY, "too many groups"); }
  if (B.nnet) {
    P.nnet = B.nnet;
    P.net_params = o.net;
    P.net_wpk = net_wpk;
    P.d_net_items = d_net_items;
    P.n_net_items = (int)net_items.size();
    // the strip's ranges, then the binning offsets the loader gathers
    P.net_smem = sizeof(float) * (size_t)(net_maxW / 8) * StripSmem<4, 8>::N + kSegBytes;
    P.d_net_in = d_net_in;
    P.d_net_conv = d_net_conv;
    P.net_hw[0] = net_hw[0];
    P.net_hw[1] = net_hw[1];
    if (hipFuncSetAttribute((const void *)k_batch_keyimage<4, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)P.net_smem) != hipSuccess) {
      delete b;
      return set_error(PC_ERR_DEVICE, "shared memory attribute failed");
    }
    std::vector<ConvJob> conv;
    for (int l = 0; l < 4; l++) conv.insert(conv.end(), net_conv[l].begin(), net_conv[l].end());
    bool nok = hipMemcpy(d_net_in, net_in.data(), sizeof(NetInputJob) * net_in.size(), hipMemcpyHostToDevice) == hipSuccess &&
               hipMemcpy(d_net_conv, conv.data(), sizeof(ConvJob) * conv.size(), hipMemcpyHostToDevice) == hipSuccess &&
               hipMemcpy(d_net_items, net_items.data(), sizeof(int2) * net_items.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!nok) {
      delete b;
      return set_error(PC_ERR_DEVICE, "network table upload failed");
    }
  }
  // block -> frame table of the binning passes: key frames' blocks first
  std::vector<int> bin_owner, bin_first(nframes), flist;
  for (int pass = 0; pass < 2; pass++)
    for (int i = 0; i < nframes; i++) {
      if (desc[i].kind != pass) continue;
      bin_first[i] = (int)bin_owner.size();
      for (int64_t q = 0; q < (desc[i].n + kBinChunk - 1) / kBinChunk; q++) bin_owner.push_back(i);
      flist.push_back(i);
      if (pass == 0) P.bin_blocks_key = (int)bin_owner.size(), P.nkey++;
      else P.npred++;
    }
  P.bin_blocks = (int)bin_owner.size();
  P.d_desc = (FrameDescDev *)ws;
  P.d_items = (int2 *)(ws + B.desc);
  P.d_bin_owner = (int *)(ws + B.desc + B.items);
  P.d_bin_first = P.d_bin_owner + bin_owner.size();
  P.d_key_frames = P.d_bin_first + nframes;
  P.d_pred_frames = P.d_key_frames + P.nkey;
  P.d_counters = counters;
  P.ncounters = 64;                 // queue counters (binning rewrites its chunk offsets every pass)
  bool ok = hipMemcpy(P.d_desc, desc.data(), sizeof(FrameDescDev) * desc.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(P.d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice) == hipSuccess &&
            (bin_owner.empty() || hipMemcpy(P.d_bin_owner, bin_owner.data(), sizeof(int) * bin_owner.size(), hipMemcpyHostToDevice) == hipSuccess) &&
            hipMemcpy(P.d_bin_first, bin_first.data(), sizeof(int) * nframes, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(P.d_key_frames, flist.data(), sizeof(int) * nframes, hipMemcpyHostToDevice) == hipSuccess &&
            hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&P.ev_join, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    delete b;
    return set_error(PC_ERR_DEVICE, "descriptor upload failed");
  }
  *out = b;
  return PC_OK;
}

pc_status pc_batch_run(pc_batch *b, void *stream) {
  if (!b) return set_error(PC_ERR_ARG, "batch is NULL");
  BatchPlan &P = b->plan;
  hipStream_t st = (hipStream_t)stream;
  auto nomark = [](int) {};
  if (P.use_graph) {
    if (!P.exec) {
      // capture once on a private stream, replay on the caller's
      hipStream_t cap;
      if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return set_error(PC_ERR_DEVICE, "stream creation failed");
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t le = batch_launches(P, cap, nomark, true);
        e = hipStreamEndCapture(cap, &P.graph);
        if (le != hipSuccess) e = le;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0);
      hipStreamDestroy(cap);
      if (e != hipSuccess) return set_error(PC_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    hipError_t e = hipGraphLaunch(P.exec, st);
    if (e != hipSuccess) return set_error(PC_ERR_DEVICE, "graph launch failed: %s", hipGetErrorString(e));
    return PC_OK;
  }
  hipError_t e = batch_launches(P, st, nomark, true);
  if (e != hipSuccess) return set_error(PC_ERR_DEVICE, "batch launch failed: %s", hipGetErrorString(e));
  return PC_OK;
}

pc_status pc_batch_profile(pc_batch *b, void *stream, float *ms, int32_t *kinds, int32_t cap, int32_t *count) {
  if (!b || !ms || !count || cap <= 0) return set_error(PC_ERR_ARG, "bad profile arguments");
  BatchPlan &P = b->plan;
  hipStream_t st = (hipStream_t)stream;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;
  auto mark = [&](int k) {
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, st);
    ev.push_back(e);
    kind.push_back(k);
  };
  mark(-1);
  hipError_t le = batch_launches(P, st, mark, false);
  hipError_t e = hipEventSynchronize(ev.back());
  int n = 0;
  for (size_t i = 1; i < ev.size() && n < cap; i++, n++) {
    float t = 0.f;
    hipEventElapsedTime(&t, ev[i - 1], ev[i]);
    ms[n] = t;
    if (kinds) kinds[n] = kind[i];
  }
  for (hipEvent_t x : ev) hipEventDestroy(x);
  *count = n;
  if (le != hipSuccess || e != hipSuccess)
    return set_error(PC_ERR_DEVICE, "profiled batch failed: %s", hipGetErrorString(le != hipSuccess ? le : e));
  return PC_OK;
}

pc_status pc_batch_info(const pc_batch *b, int32_t *nitems, int32_t *ngroups, int32_t *grid_max) {
  if (!b) return set_error(PC_ERR_ARG, "batch is NULL");
  int n = 0, gm = 0;
  for (const Group &g : b->plan.groups) {
    n += g.count;
    gm = std::max(gm, g.grid);
  }
  if (nitems) *nitems = n;
  if (ngroups) *ngroups = (int)b->plan.groups.size();
  if (grid_max) *grid_max = gm;
  return PC_OK;
}

pc_status pc_batch_destroy(pc_batch *b) {
  if (!b) return PC_OK;
  if (b->plan.exec) hipGraphExecDestroy(b->plan.exec);
  if (b->plan.graph) hipGraphDestroy(b->plan.graph);
  if (b->plan.ev_fork) hipEventDestroy(b->plan.ev_fork);
  if (b->plan.ev_join) hipEventDestroy(b->plan.ev_join);
  if (b->plan.side) hipStreamDestroy(b->plan.side);
  delete b;
  return PC_OK;
}

}  // extern "C"

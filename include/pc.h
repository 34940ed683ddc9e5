/*
 * pc.h -- C ABI of the MI355X (gfx950) spatio-temporal LiDAR range-image
 * encoder.  The method is that of Feng, Liu and Zhu, "Real-Time
 * Spatio-Temporal LiDAR Point Cloud Compression": a group of frames is
 * projected to range images (Sec. III-B), the key frame is tiled and encoded
 * with least-squares planes grown horizontally into runs [s, len, P]
 * (Sec. III-C), the other frames reuse the key frame's planes after a rigid
 * transform with only the plane offset free (Sec. III-D), and what no plane
 * reproduces within the error bound eps is kept in a residual map whose
 * streams are sized by an optimal Huffman code (Sec. III-A).  The streams
 * are emitted as length-limited canonical Huffman containers and read back
 * (pc_pack, pc_unpack), and transforms can be integrated from IMU samples
 * (pc_imu_transform, Eq. (4)-(5)).
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE memory unless the comment says "host".
 *   - Every call is asynchronous on the given HIP stream (`stream` is a
 *     hipStream_t; NULL = the null stream), except those whose comment says
 *     they synchronise.  The caller owns every buffer;
 *     the library keeps no pointer to caller memory after a call returns,
 *     except the workspace handed to pc_ctx_create.
 *   - Argument errors are detected on the host before any launch and
 *     returned as a negative pc_status; nothing is launched then.  Errors
 *     that depend on data (a residual out of code range) set a sticky bit in
 *     the frame's info block (pc_frame_info.status) and are reported by
 *     pc_check() / by reading the info block after synchronising.
 *   - Non-finite, zero-range and out-of-field-of-view input points are not
 *     errors: they are dropped and counted.
 *   - Alignment: device pointers 16 B aligned (PyTorch's allocator gives 512 B).
 *   - A pc_ctx is not thread safe; use one per host thread / stream.
 *   - GPU-path restrictions (return PC_ERR_UNSUPPORTED): W % 32 == 0,
 *     W % tile_w == 0, H % tile_h == 0, tile_h*tile_w in {16, 32, 64} with a
 *     compiled tile shape (4x4, 4x8, 4x16, 8x8).
 */
#ifndef PC_H
#define PC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PC_OK = 0,
  PC_ERR_ARG = -1,          /* invalid argument (NULL buffer, bad size, eps <= 0 ...) */
  PC_ERR_CAPACITY = -2,     /* a buffer or workspace is too small */
  PC_ERR_DEVICE = -3,       /* a HIP runtime call failed */
  PC_ERR_STATE = -4,        /* a sticky device error was found by pc_check */
  PC_ERR_UNSUPPORTED = -5,  /* valid for the method, not supported by this GPU path */
  PC_ERR_RANGE = -6         /* a residual could not be coded within eps (sticky) */
} pc_status;

/* Sensor geometry (host struct).  Row 0 is the top beam; elevations must be
 * strictly descending.  Column u covers the clockwise azimuth interval
 * (az0 - (u+1) 2pi/W, az0 - u 2pi/W] (Sec. III-B, Eq. (2): theta and phi are
 * pixel coordinates at the sensor's angular resolution). */
typedef struct {
  int32_t H, W;             /* beams (rows), azimuth bins (columns) */
  const float *elev_rad;    /* host, H beam elevations in radians */
  float az0_rad;            /* leading edge of column 0 */
} pc_sensor;

/* Encoder parameters (host struct). */
typedef struct {
  float eps;                /* error bound on the range, metres, > 0 (Sec. III-C "threshold") */
  int32_t tile_h, tile_w;   /* unit tile, rows x columns (Sec. III-C, e.g. 4x4) */
  int32_t max_iter;         /* plane fits per tile, 1..8 (refit on reproduced points) */
  int32_t min_pts;          /* fewest points a plane is fitted to, >= 3 */
  float min_inlier_frac;    /* share of a tile's points its plane must reproduce, (0, 1] */
} pc_params;

/* Projection statistics (device struct, written by pc_project). */
typedef struct {
  int64_t n_in;             /* points given */
  int64_t n_nonfinite;      /* non-finite coordinates or zero / overflowing range */
  int64_t n_fov;            /* outside the vertical field of view or on the sensor axis */
  int64_t n_collided;       /* landed on a pixel a nearer point kept (Sec. III-D) */
  int64_t n_kept;           /* non-empty pixels */
} pc_proj_stats;

/* Sticky status bits in pc_frame_info.status */
#define PC_STATUS_RANGE 1u  /* a residual exceeded the 16-bit code range or eps */
#define PC_STATUS_NOKEY 2u  /* a predicted frame was decoded without its key frame (its temporal
                               pixels came out as 0) */

/* Strip summary layout: 4 x 256 histogram words, then these counters. */
#define PC_STRIP_STATS 16
#define PC_STRIP_WORDS (4 * 256 + PC_STRIP_STATS)
#define PC_SS_VALID 0       /* non-empty pixels */
#define PC_SS_RES 1         /* residual pixels */
#define PC_SS_TILES 2       /* 4 words: tiles per class */
#define PC_SS_SRUNS 6       /* spatial runs */
#define PC_SS_PRUNS 7       /* temporal runs */
#define PC_SS_FITS 8        /* plane fits */
#define PC_SS_FP64 9        /* FP64 eigen solves */
#define PC_SS_STATUS 10     /* sticky status bits */
#define PC_SS_SEEDED 11     /* seeded tiles accepted */
#define PC_SS_FALLBACK 12   /* seeded tiles that fell back */

/* Per-frame info block (device struct, first section of a frame stream). */
typedef struct {
  int32_t kind;             /* 0 = key frame, 1 = predicted frame */
  uint32_t status;          /* sticky PC_STATUS_* bits */
  int32_t n_sruns;          /* spatial runs [s, len, P] */
  int32_t n_pruns;          /* temporal runs [s, len, c'] */
  int64_t n_valid;          /* non-empty pixels */
  int64_t n_res;            /* residual pixels */
  int32_t tiles[4];         /* tiles per class: empty, unfit, spatial, temporal */
  int32_t fits;             /* plane fits run (all iterations, all tiles) */
  int32_t fp64_fits;        /* of which took the FP64 eigen path */
  int32_t seeded;           /* tiles whose learned seed was accepted */
  int32_t fallback;         /* tiles whose learned seed failed the check */
  uint64_t stream_bytes[4]; /* serialized bytes of OCC, RUN, MASK, RES */
  uint64_t coded_bits[4];   /* optimal Huffman cost of each stream */
  uint64_t size_bytes;      /* header + coded streams + code tables */
  float M[12];              /* rigid transform into the key frame (rows of [R|T]) */
  int32_t pad[4];
} pc_frame_info;

/* A run of tiles in one tile row sharing one plane (Sec. III-C, [s, len, P]).
 * The plane is p_k + a p_k1 + b p_k2 = c in the frame's coordinates, k the
 * dominant axis of its normal and k1 < k2 the other two (Eq. (3) is k = x). */
typedef struct {
  int32_t s, len;           /* first tile column, number of tiles */
  int32_t axis;             /* k: 0, 1, 2 */
  float a, b, c;
} pc_run;

/* A temporal run: the key frame's run plane `krun` with offset c' (Sec. III-D). */
typedef struct {
  int32_t s, len;
  int32_t krun;             /* slot of the key-frame run: row * TC + index in row */
  float c;
} pc_prun;

/* Per-tile fit record (diagnostics and parity checks; not needed to decode).
 * pc_fit_key and pc_encode_pred always write it; a batch writes it only when
 * pc_batch_opts.records is set. */
typedef struct {
  float a, b, c;            /* own plane (valid when status >= 4) */
  uint8_t axis, status, iters, t_status;   /* status: 0 empty, 1 few, 2 degenerate, 3 failed, 4 rejected, 5 accepted;
                                              t_status: 0 none, 1 failed, 2 accepted */
  uint64_t mask;            /* own plane's reproduced pixels, bit i*tw+k */
  uint64_t t_mask;          /* temporal fit's reproduced pixels */
  float t_c;                /* temporal offset c' */
  uint8_t t_iters;
  uint8_t seeded;           /* learned seed: 0 none, 1 accepted, 2 fell back to the plain fit */
  uint8_t pad[2];
} pc_tile_rec;

/* Section offsets (bytes) of one frame stream buffer.  Sizes:
 * TR = H/tile_h tile rows, TC = W/tile_w tile columns, T = TR*TC. */
typedef struct {
  int32_t H, W, th, tw, TR, TC, T;
  int32_t pad;
  size_t bytes;             /* total size of the buffer */
  size_t off_info;          /* pc_frame_info */
  size_t off_occ;           /* uint32 words: bit (v*W+u) = pixel non-empty (OCC stream) */
  size_t off_cls;           /* uint8[T]: 0 empty, 1 unfit, 2 spatial run, 3 temporal run */
  size_t off_mask;          /* uint64[T]: pixels the covering plane reproduces */
  size_t off_run_of;        /* int32[T]: covering run slot (spatial: slot; temporal: T + slot), -1 */
  size_t off_nruns;         /* int32[2*TR]: spatial then temporal run count of each tile row */
  size_t off_sruns;         /* pc_run[T]: tile row r's runs at slots r*TC .. */
  size_t off_pruns;         /* pc_prun[T] */
  size_t off_nres;          /* int32[TR]: residual pixels of each tile-row strip */
  size_t off_res;           /* uint16[H*W]: strip r's codes (raster order) from r*tile_h*W */
  size_t off_hist;          /* uint32[TR][PC_STRIP_WORDS]: per tile-row strip, the byte histograms
                               of its OCC, RUN, MASK and RES bytes (4 x 256), then PC_STRIP_STATS
                               counters (see PC_SS_*) */
  size_t off_tiles;         /* pc_tile_rec[T] */
} pc_layout;

typedef struct pc_ctx pc_ctx;

/* ---- set-up ------------------------------------------------------------ */

/* Fill *out with the section offsets of a frame stream for this sensor and
 * these parameters.  Returns PC_ERR_ARG / PC_ERR_UNSUPPORTED on bad input. */
pc_status pc_stream_layout(const pc_sensor *sensor, const pc_params *params, pc_layout *out);

/* Workspace a context needs to project frames of up to H*W pixels
 * (8 bytes per pixel for the nearest-point keys). */
size_t pc_workspace_size(const pc_sensor *sensor);

/* Create a context on `device` using the caller's device workspace (at least
 * pc_workspace_size bytes for every sensor used with it).  Sensors must be
 * registered with pc_sensor_register before any other call takes them. */
pc_status pc_ctx_create(pc_ctx **out, int device, void *workspace, size_t ws_bytes);
pc_status pc_ctx_destroy(pc_ctx *ctx);

/* Compute the sensor's tables on the host (FP64 trigonometry rounded once to
 * FP32) and upload them: one device allocation per distinct sensor, freed by
 * pc_ctx_destroy; registering a sensor twice finds the first tables.  This
 * is the only call that allocates device memory: every other call taking a
 * sensor returns PC_ERR_STATE for a sensor not registered with the context.
 * Synchronises the device. */
pc_status pc_sensor_register(pc_ctx *ctx, const pc_sensor *sensor);

/* Copy the sensor tables the GPU path uses to host arrays (for checks):
 * cut[H+1], ebx[W], eby[W], ce[H], se[H], ca[W], sa[W]. */
pc_status pc_sensor_tables(pc_ctx *ctx, const pc_sensor *sensor, float *cut, float *ebx, float *eby,
                           float *ce, float *se, float *ca, float *sa);

/* ---- the hot path -------------------------------------------------------- */

/* Range-image conversion (Sec. III-B, Eq. (1)-(2)) of n points xyz[n][3]
 * (FP32, any order), optionally moved into the key frame by M (host, 16 FP32,
 * row-major 4x4, Eq. (6)).  Writes range[H][W] (FP32, 0 = empty) keeping the
 * nearest point on collisions, ties to the lower index (Sec. III-D), the
 * winning point's index src_idx[H][W] (-1 = empty; may be NULL) and stats
 * (may be NULL).  Uses the context workspace. */
pc_status pc_project(pc_ctx *ctx, const float *xyz, int64_t n, const float *M_host,
                     const pc_sensor *sensor, float *range, int32_t *src_idx,
                     pc_proj_stats *stats, void *stream);

/* Largest sensor (H * W pixels) pc_project_noalloc takes: 4 MiB of
 * collision keys per device. */
#define PC_PROJECT_NOALLOC_MAX_PIXELS 524288

/* pc_project for callers that cannot allocate device memory or hand over a
 * workspace (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): same arguments, results and errors as pc_project, but
 * the collision keys live in a fixed array of the library
 * (PC_PROJECT_NOALLOC_MAX_PIXELS keys of 8 bytes, one array per device,
 * held until the process ends) instead of the context workspace, so the
 * context may have been created without one.  Allocates nothing and calls
 * no allocating routine; the keys are reset by a fill kernel on every call.
 * Returns PC_ERR_CAPACITY for a sensor with more than
 * PC_PROJECT_NOALLOC_MAX_PIXELS pixels.  Every call on one device shares
 * that device's array: calls that overlap in time on one device (two
 * streams, two host threads) race and give wrong ranges. */
pc_status pc_project_noalloc(pc_ctx *ctx, const float *xyz, int64_t n, const float *M_host,
                             const pc_sensor *sensor, float *range, int32_t *src_idx,
                             pc_proj_stats *stats, void *stream);

/* Spatial encoding of a key frame (Sec. III-C) from its range image into the
 * frame stream buffer `out` (pc_layout.bytes bytes, laid out by
 * pc_stream_layout).  Per tile: least-squares plane (FP32 moments, FP64 when
 * the two smallest eigenvalues are close), refit on reproduced pixels up to
 * max_iter times; per tile row: horizontal run growth; residual pixels
 * quantised with step 2 eps (1 - 2^-8); per-strip byte histograms; then the
 * optimal Huffman size into the info block.  `seed` (may be NULL) holds
 * per-tile normal seeds [T][4] (n_x, n_y, n_z, planarity logit) from
 * pc_net_forward: a seeded tile takes one refit from the seed and keeps it
 * when it passes the same acceptance test, else runs the plain fit. */
pc_status pc_fit_key(pc_ctx *ctx, const float *range, const pc_sensor *sensor,
                     const pc_params *params, const float *seed, void *out, void *stream);

/* Temporal encoding of a predicted frame (Sec. III-D) against the key
 * frame's stream `key` (same sensor and parameters): each tile covered by a
 * key run reuses that run's normal with the offset c' free; temporal runs
 * grow within one key run; remaining tiles are encoded spatially.  `range` is
 * the predicted frame's range image in the key frame's grid (pc_project with
 * its transform); M_host (16 FP32, may be NULL) is recorded in the info block. */
pc_status pc_encode_pred(pc_ctx *ctx, const void *key, const float *range, const float *M_host,
                         const pc_sensor *sensor, const pc_params *params, void *out, void *stream);

/* Decode a frame stream (Sec. III-C): plane pixels by casting the
 * pixel-centre ray onto the run plane, residual pixels as code * step.
 * range_out[H][W] (FP32, 0 = empty; may be NULL) receives the ranges;
 * xyz_out[H][W][3] (FP32, pixel-major; may be NULL, not both) the points r d
 * on the pixel-centre rays d, 0 at empty pixels.  With frame_coords = 1 the
 * points of a predicted frame are taken back to its own coordinates,
 * R^T (p - T) for its transform [R | T] into the key frame (Eq. (6); the
 * transform recorded in the frame's info block); 0 leaves them in the key
 * frame's coordinates.  `key` is the key frame's stream for a predicted
 * frame (NULL for a key frame); a predicted frame decoded without it sets
 * the sticky PC_STATUS_NOKEY bit in its info block (see pc_check) and its
 * temporal pixels decode to 0.  Outputs 16-byte aligned. */
pc_status pc_decode(pc_ctx *ctx, const void *key, const void *frame, const pc_sensor *sensor,
                    const pc_params *params, float *range_out, float *xyz_out, int32_t frame_coords,
                    void *stream);

/* pc_decode over n frames of one sensor and tile shape in one launch (a
 * work-group per tile-row strip and frame).  frames: host array of n device
 * pointers; range_out, xyz_out: NULL or host arrays of n device pointers
 * (entries may be NULL, but not both outputs of a frame); keys: NULL (all key
 * frames) or a host array whose entry i is frame i's key frame buffer, or
 * NULL for a key frame.  The per-frame job table is uploaded into `work`
 * (pc_decode_batch_workspace_size bytes), which synchronises `stream`. */
size_t pc_decode_batch_workspace_size(int32_t n);
pc_status pc_decode_batch(pc_ctx *ctx, int32_t n, const void *const *keys, const void *const *frames,
                          const pc_sensor *sensor, const pc_params *params, float *const *range_out,
                          float *const *xyz_out, int32_t frame_coords, void *work, size_t work_bytes, void *stream);

/* ---- learned plane seeding -------------------------------------------------
 * A small convolutional network proposes, per 4x8 tile, a plane normal and a
 * planarity logit from the key frame's range image; pc_fit_key tries one
 * refit from each planar seed and falls back to the plain fit when the seed
 * does not pass the same acceptance test (learned plane seeding of the
 * Sec. III-C fit).  Network: four 3x3 convolutions, zero padding 1, channels
 * 4 -> 16 -> 32 -> 32 -> 4, strides (2,2), (2,2), (1,2), (1,1), ReLU after
 * the first three; input channels (r, x, y, z) / 16 with (x, y, z) = r d at
 * the FP32 pixel directions; inputs, weights and stored activations bfloat16
 * (round to nearest even), FP32 accumulation on MFMA.  Parameters: one FP32
 * vector of PC_NET_PARAMS values, per layer W[out][in][ky][kx] then b[out].
 * Sensors need H % 4 == 0 and W % 8 == 0 (else PC_ERR_UNSUPPORTED). */
#define PC_NET_PARAMS 15636

/* Device workspace of one frame's forward pass (kept for its backward pass). */
size_t pc_net_workspace_size(const pc_sensor *sensor);

/* seed[H/4][W/8][4] (FP32: n_x, n_y, n_z, logit) from range[H][W]; the
 * workspace keeps the activations for pc_net_backward. */
pc_status pc_net_forward(pc_ctx *ctx, const float *params, const float *range, const pc_sensor *sensor, void *work,
                         size_t work_bytes, float *seed, void *stream);

/* Gradient of a loss with respect to the parameters, ADDED to grad[PC_NET_PARAMS],
 * given dseed = d loss / d seed and the workspace of the matching forward
 * pass (bfloat16 roundings pass gradients straight through). */
pc_status pc_net_backward(pc_ctx *ctx, const float *params, const pc_sensor *sensor, void *work, size_t work_bytes,
                          const float *dseed, float *grad, void *stream);

/* Training loss against labels from a plain key-frame stream `labels`
 * (pc_fit_key without seed, 4x8 tiles): tiles with a fit attempt are
 * labelled, planar = accepted, normal = the stored plane's unit normal.
 * loss[0] (device) = mean over labelled tiles of BCE(logit, planar) +
 * planar * (1 - |cos(seed normal, label normal)|); dseed = its gradient. */
pc_status pc_net_loss(pc_ctx *ctx, const float *seed, const void *labels, const pc_sensor *sensor,
                      const pc_params *params, float *dseed, float *loss, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; Kingma & Ba 2015) on
 * params with moments m, v (PC_NET_PARAMS each); step counts from 1. */
pc_status pc_net_adam(pc_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t step, float lr,
                      void *stream);

/* ---- batched encoding ------------------------------------------------------
 * Many frames of many sensors (and groups of frames with their key frames)
 * encoded by one replay of a HIP graph: every frame's points are projected
 * and binned by tile-row strip, the key frames' strips are encoded, then
 * the predicted frames' strips, then every frame's size.  Each strip's work
 * item builds its strip's range image in LDS from its bin (nearest point
 * wins) -- the range images never go through device memory unless asked
 * for.  Predicted-frame strips are pulled in (frame, strip) items from an
 * atomic queue by persistent work-groups.  Each frame's stream equals what pc_project +
 * pc_fit_key / pc_encode_pred give for it. */
typedef struct {
  const float *xyz;          /* device, n x 3 FP32 points in the frame's own coordinates */
  int64_t n;
  const float *M;            /* host 16 FP32 (read at create): transform into the key frame; NULL for key frames */
  const pc_sensor *sensor;   /* host, read at create */
  const pc_params *params;   /* host, read at create; a predicted frame's tile shape equals its key frame's */
  int32_t key;               /* batch index of the frame's key frame (its own index for a key frame) */
  int32_t pad;
  const float *seed;         /* device per-tile seeds for a key frame (as pc_fit_key), or NULL */
  float *range;              /* device H*W FP32: receives the frame's range image (0 = empty); NULL = not written */
  void *out;                 /* device frame stream buffer (pc_stream_layout bytes) */
} pc_frame_desc;

typedef struct {
  int32_t persistent;        /* 1: persistent work-groups pull predicted-frame strips from an atomic queue;
                                0: a work-group per strip (key-frame strips always run this way) */
  int32_t graph;             /* 1: capture the batch in a HIP graph at the first run and replay it afterwards */
  int32_t blocks_per_cu;     /* persistent grid = CUs * this (at most one work-group per item); 0 = 4 */
  int32_t records;           /* 1: also write every frame's per-tile fit records (pc_tile_rec); 0: skip them */
  const float *net;          /* device PC_NET_PARAMS seed-network parameters, or NULL: key frames with 4x8
                                tiles and no seeds of their own get seeds from this network inside the batch */
  int32_t lanes_max;         /* wavefront mapping of the strip encoders: at most this many neighbouring
                                lanes share one tile (1, 2 or 4; 0 = 4) once few tiles are left to fit,
                                test or grow; the lanes' partial sums are combined in another order, so
                                planes may differ by rounding between mappings */
} pc_batch_opts;

typedef struct pc_batch pc_batch;

/* Device workspace a batch plan needs (descriptor table, work items, block
 * tables, counters, 16 bytes per point for staging and the strip bins, and
 * with a seed network about 27 bytes per pixel of each seeded key frame).
 * opts may be NULL. */
size_t pc_batch_workspace_size(const pc_frame_desc *frames, int32_t nframes, const pc_batch_opts *opts);

/* Check the frames, build and upload the descriptor table into the
 * workspace.  The workspace, the frames' xyz, range and out buffers must stay
 * valid until pc_batch_destroy.  opts may be NULL (persistent, graph).
 * Besides the per-frame restrictions: at most 256 tile-row strips per frame
 * (PC_ERR_UNSUPPORTED), and a predicted frame's key frame must be in the
 * same batch with the same sensor size and tile shape (PC_ERR_ARG). */
pc_status pc_batch_create(pc_ctx *ctx, const pc_frame_desc *frames, int32_t nframes, const pc_batch_opts *opts,
                          void *workspace, size_t ws_bytes, pc_batch **out);

/* Encode the whole batch on `stream` (asynchronous). */
pc_status pc_batch_run(pc_batch *batch, void *stream);

/* Work items (strips), launch groups (one per kind and tile shape) and the
 * largest persistent grid of a plan. */
pc_status pc_batch_info(const pc_batch *batch, int32_t *nitems, int32_t *ngroups, int32_t *grid_max);

/* Run the batch once without the graph, recording a HIP event after every
 * launch; ms[i] is the duration of launch i and kinds[i] its PC_LAUNCH_* kind
 * (kinds may be NULL).  Synchronises the stream.  For measurement only. */
#define PC_LAUNCH_RESET 0
#define PC_LAUNCH_COUNT 1     /* binning: projection, each block's points grouped by strip */
#define PC_LAUNCH_OFFSETS 2   /* (not launched: kept for the numbering) */
#define PC_LAUNCH_SCATTER 3   /* (not launched: kept for the numbering) */
#define PC_LAUNCH_KEY 4
#define PC_LAUNCH_PRED 5
#define PC_LAUNCH_FINISH 6
#define PC_LAUNCH_KEYIMAGE 7  /* key-frame range images for the seed network */
#define PC_LAUNCH_NET 8       /* the seed network's forward pass */
pc_status pc_batch_profile(pc_batch *batch, void *stream, float *ms, int32_t *kinds, int32_t cap, int32_t *count);

pc_status pc_batch_destroy(pc_batch *batch);

/* Synchronise `stream` and scan the given frame info blocks (device
 * pointers to pc_frame_info; may be 0 of them) for sticky errors, in order.
 * Returns PC_ERR_RANGE for the first frame with PC_STATUS_RANGE set,
 * PC_ERR_STATE for one with PC_STATUS_NOKEY, else PC_OK. */
pc_status pc_check(pc_ctx *ctx, void *stream, const void *const *frames, int32_t nframes);

/* ---- IMU front end (Sec. III-D, Eq. (4)-(5)) ---------------------------------
 * The transform M of a predicted frame into its key frame from n equally
 * spaced IMU samples (host arrays): acc[n][3] translational acceleration and
 * gyro[n][3] rotational rate about the body x, y, z axes, dt the sample
 * spacing, v0[3] the velocity at the first sample (NULL = 0).  Per sample
 * (explicit Euler, the first-order Runge-Kutta method) the position advances
 * by the velocity times dt, then the velocity by the acceleration times dt,
 * and each rotational displacement by its rate times dt; T = the position
 * (Eq. (4)), R = the printed product of the planar rotations by the
 * accumulated z, y and x rotations (Eq. (5)).  M (host, 16 FP32, row-major
 * [R | T; 0 0 0 1]) is the transform pc_encode_pred and the batch take;
 * v_end (host, 3 FP32, may be NULL) receives the velocity after the last
 * sample.  FP64 accumulation.  PC_ERR_ARG on n < 0, dt <= 0, NULL or
 * non-finite input. */
pc_status pc_imu_transform(const float *acc, const float *gyro, int32_t n, float dt, const float *v0, float *M,
                           float *v_end);

/* ---- entropy-coded bitstream (Sec. III-A) -----------------------------------
 * The frame's four byte streams, in the order the size model counts them:
 *   OCC  the occupancy bits, H*W/8 bytes (bit v*W+u of the little-endian
 *        bytes: pixel (v, u) not empty);
 *   RUN  per tile row: for a predicted frame first LEB128(count) and per
 *        temporal run LEB128(gap), LEB128(len), FP32 c' (gap = first tile
 *        column minus the previous run's end in the row, from 0); then for
 *        every frame LEB128(count) and per spatial run LEB128(gap),
 *        LEB128(len), axis u8, FP32 a, b, c (little-endian);
 *   MASK per plane-coded tile in tile raster order, the mask bits of its
 *        non-empty pixels (tile raster order), LSB first, byte aligned;
 *   RES  the residual codes of the pixels no plane reproduces, frame raster
 *        order, u16 little-endian.
 * Each non-empty stream is coded with a canonical Huffman code limited to 15
 * bits (Huffman construction on the counts sorted by (count, symbol), ties
 * taking the leaf, depths limited by the bit-count adjustment of ITU T.81
 * Annex K.3, lengths given shortest first by (count descending, symbol
 * ascending); code words by (length, symbol)).  Container: 64-byte header
 * (magic "PCC1" u32, kind u8 (0 key, 1 predicted), tile_h u8, tile_w u8,
 * 0 u8, H u16, W u16, stream bytes u64[4], payload bytes u32[4], 4 zero
 * bytes), then per non-empty stream a 128-byte table of 4-bit code lengths
 * (symbol 2i in the low nibble of byte i) and the payload: the code words MSB
 * first, padded to a byte.  Whenever no optimal code word exceeds 15 bits the
 * container's size equals pc_frame_info.size_bytes. */

/* Largest container of one frame (a multiple of 256 bytes). */
size_t pc_pack_bound(const pc_sensor *sensor, const pc_params *params);

/* Device workspace of pc_pack and pc_unpack for this sensor and tile shape. */
size_t pc_pack_workspace_size(const pc_sensor *sensor, const pc_params *params);

/* Pack an encoded frame stream buffer (device) into `out` (device, 4-byte
 * aligned, cap >= pc_pack_bound bytes).  The container's byte count is
 * written to *nbytes (device u64; 0 on an internal inconsistency).
 * streams: NULL, or a host array of 4 device buffers (capacities in the host
 * array stream_caps) that receive the frame's raw stream bytes.
 * Asynchronous on `stream`; nothing is allocated. */
pc_status pc_pack(pc_ctx *ctx, const void *frame, const pc_sensor *sensor, const pc_params *params, void *work,
                  size_t work_bytes, void *out, uint64_t cap, uint64_t *nbytes, uint8_t *const *streams,
                  const uint64_t *stream_caps, void *stream);

/* pc_pack over n frames of one sensor and tile shape: outs[i] (host array of
 * device pointers, each 4-byte aligned with cap >= pc_pack_bound bytes)
 * receives frame i's container and nbytes[i] (device u64[n]) its size.  One
 * planning work-group per frame and one work-group per strip and frame.  The
 * per-frame job table is uploaded into the workspace first, which
 * synchronises `stream`; nothing is allocated on the device. */
size_t pc_pack_batch_workspace_size(const pc_sensor *sensor, const pc_params *params, int32_t n);
pc_status pc_pack_batch(pc_ctx *ctx, int32_t n, const void *const *frames, const pc_sensor *sensor,
                        const pc_params *params, void *work, size_t work_bytes, void *const *outs, uint64_t cap,
                        uint64_t *nbytes, void *stream);

/* Unpack a container (device bytes, n_in exactly its size) into a frame
 * stream buffer that pc_decode reads: occupancy, tile classes, runs, masks
 * and residual codes (the encoder's fit records and strip histograms are not
 * reproduced).  A predicted frame needs its key frame's stream buffer (the
 * temporal runs take the normals of the key frame's runs).  *kind_out (host,
 * may be NULL) receives the frame kind.  Synchronises `stream`; returns
 * PC_ERR_ARG on a malformed container or one for another sensor size or
 * tile shape. */
pc_status pc_unpack(pc_ctx *ctx, const void *data, uint64_t n_in, const void *key, const pc_sensor *sensor,
                    const pc_params *params, void *work, size_t work_bytes, void *frame_out, int32_t *kind_out,
                    void *stream);

/* pc_unpack over n containers of one sensor and tile shape: data and
 * frames_out are host arrays of n device pointers, n_in (host) the
 * containers' sizes, keys NULL or a host array whose entry i is the key
 * frame buffer of a predicted container i (it may be another output of the
 * same call: key frames are parsed first), NULL for key frames.  kinds_out
 * (host int32[n], may be NULL) receives each container's kind.  Headers,
 * streams and frame buffers of all containers are decoded by five launches;
 * the job table upload and the final status read synchronise `stream`.
 * PC_ERR_ARG names the first failing container. */
size_t pc_unpack_batch_workspace_size(const pc_sensor *sensor, const pc_params *params, int32_t n);
pc_status pc_unpack_batch(pc_ctx *ctx, int32_t n, const void *const *data, const uint64_t *n_in,
                          const void *const *keys, const pc_sensor *sensor, const pc_params *params, void *work,
                          size_t work_bytes, void *const *frames_out, int32_t *kinds_out, void *stream);

/* The same coder on four raw device byte streams of n[4] bytes each (below
 * 2^28), with the header fields given; `out` needs pc_stream_pack_bound(n)
 * bytes and `work` pc_stream_pack_workspace_size(n). */
uint64_t pc_stream_pack_bound(const uint64_t *n);
size_t pc_stream_pack_workspace_size(const uint64_t *n);
pc_status pc_pack_streams(pc_ctx *ctx, const uint8_t *const *streams, const uint64_t *n, int32_t kind, int32_t H,
                          int32_t W, int32_t tile_h, int32_t tile_w, void *work, size_t work_bytes, void *out,
                          uint64_t cap, uint64_t *nbytes, void *stream);

/* Decode a container's streams into 4 device buffers of host-given
 * capacities; n_out (host u64[4]) receives the stream lengths.  The
 * workspace needs pc_stream_pack_workspace_size of any sizes.  Synchronises
 * `stream`; PC_ERR_ARG on a malformed container or a stream above its
 * capacity. */
pc_status pc_unpack_streams(pc_ctx *ctx, const void *data, uint64_t n_in, void *work, size_t work_bytes,
                            uint8_t *const *streams, const uint64_t *caps, uint64_t *n_out, void *stream);

/* Thread-local message for the last error returned on this thread. */
const char *pc_last_error(void);

/* Library version string. */
const char *pc_version(void);

#ifdef __cplusplus
}
#endif
#endif

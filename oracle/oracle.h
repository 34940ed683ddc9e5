/*
 * CPU oracle for the spatio-temporal LiDAR range-image encoder of
 * "Real-Time Spatio-Temporal LiDAR Point Cloud Compression" (Feng, Liu, Zhu).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; the two are
 * written independently from the paper and compared on the same inputs.
 *
 * Precision: FP64 for the plane fits (moments, eigen-solve, offsets);
 * FP32 exactly where the method takes an integer decision from floating
 * point (projection bins, the ray-cast inlier test, the residual quantiser),
 * so both sides decide in the same precision.
 *
 * Parity status per function (pins live in tests/test_oracle_*.py):
 *   orc_tables, orc_project      pinned (brute force, closed form)
 *   orc_tls                      pinned (numpy eigh, sphere sampling, noiseless planes)
 *   orc_encode_key/_pred         pinned by constructed cases and the eps invariant;
 *                                "parity unpinned" against the paper's own numbers
 *                                (the paper prints no worked example)
 *   orc_huffman_bits             pinned (textbook heap construction, entropy bound)
 *   orc_code_lengths, orc_pack   pinned (brute-force optimal codes on small alphabets, the
 *                                heap cost, Kraft equality, round trips)
 *   orc_decode                   pinned (closed-form ray-plane intersection)
 */
#ifndef PCC_ORACLE_H
#define PCC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sensor tables, all FP32 values rounded once from FP64 trigonometry.
 *   cut[H+1] : tan of the elevation cuts; cut[0] = top FOV edge, cut[v] (1<=v<H)
 *              = tan of the midpoint between beams v-1 and v, cut[H] = bottom edge.
 *   ebx, eby[W] : unit vector of the leading (counter-clockwise) edge of column u.
 *   ce, se[H] : cos / sin of beam elevations.   ca, sa[W] : cos / sin of column centres. */
typedef struct {
  int H, W;
  float *cut, *ebx, *eby, *ce, *se, *ca, *sa;
} orc_sensor;

typedef struct {
  float eps;           /* error bound on the range (m) */
  int th, tw;          /* tile shape: rows x columns, th*tw <= 64 */
  int max_iter;        /* inlier-refit iterations per tile */
  int min_pts;         /* minimum points for a fit */
  float rho;           /* minimum inlier fraction for acceptance */
} orc_params;

/* own-fit status of a tile */
enum { ORC_EMPTY = 0, ORC_FEW = 1, ORC_DEGENERATE = 2, ORC_FAILED = 3, ORC_REJECTED = 4, ORC_ACCEPTED = 5 };
/* final class of a tile */
enum { ORC_CLS_EMPTY = 0, ORC_CLS_UNFIT = 1, ORC_CLS_SPATIAL = 2, ORC_CLS_TEMPORAL = 3 };

/* Per-frame encoder output.  T = TR*TC tiles.  Arrays are caller-allocated. */
typedef struct {
  int TR, TC;
  /* own (spatial) fit per tile */
  int8_t *own_status, *own_iters, *own_axis;
  float *own_abc;                  /* T*3 */
  uint64_t *own_mask;
  /* temporal fit per tile (P-frames only; may be NULL for key frames) */
  int8_t *t_status, *t_iters;      /* 0 = not a candidate, 1 = failed/rejected, 2 = accepted */
  float *t_c;
  uint64_t *t_mask;
  /* final tile classes */
  int8_t *cls;
  uint64_t *mask;
  int32_t *run_of;                 /* index of the covering run (spatial and temporal lists share numbering: temporal runs are offset by T) */
  /* run lists, row-major: spatial runs then, separately, temporal runs */
  int32_t n_sruns, n_pruns;
  int32_t *srun_row, *srun_s, *srun_len; int8_t *srun_axis; float *srun_abc;   /* capacity T */
  int32_t *prun_row, *prun_s, *prun_len, *prun_krun; float *prun_c;           /* capacity T */
  /* occupancy bitmap: H*W bits, raster order, LSB first (capacity (H*W+7)/8 bytes) */
  uint8_t *occ;
  /* residual codes in frame raster order */
  int64_t n_res;
  uint16_t *codes;                 /* capacity H*W */
  /* byte histograms of the serialized streams: OCC, RUN, MASK, RES */
  uint32_t *hist;                  /* 4*256 */
  uint64_t stream_bytes[4];        /* serialized byte count per stream */
  uint64_t coded_bits[4];          /* optimal Huffman cost per stream */
  uint64_t size_bytes;             /* frame size: header + coded streams + tables */
  int32_t range_error;             /* set if a residual cannot be coded within eps */
  /* learned plane seeding (key frames): 0 no seed, 1 seed accepted, 2 seed fell back */
  int8_t *seeded;                  /* T entries, may be NULL */
  /* optional capture of the serialized streams' bytes, in emission order
   * (OCC, RUN, MASK, RES; NULL = not captured; scap = capacity in bytes) */
  uint8_t *sbuf[4];
  uint64_t scap[4];
  /* optional diagnostics (NULL = not kept; T entries): per tile, the
   * smallest distance from eps of | t - r | over every pixel test made on
   * the tile (own and temporal fits, run extensions), in metres and relative
   * to max(r, 1 m), and the relative plane change that flips a test (that
   * distance times the cosine between ray and plane normal, over max(r, 1 m);
   * the cosine alone for a test whose ray-cast range is not finite and
   * positive).  Tells how close a tile's decisions came to flipping; no
   * result depends on them. */
  float *margin_abs, *margin_rel, *margin_cond;
} orc_frame;

void orc_tables(int H, int W, const float *elev, float az0, float *cut, float *ebx, float *eby,
                float *ce, float *se, float *ca, float *sa);

/* stats[5]: points given, non-finite, out of field of view, collided, kept */
void orc_project(const float *xyz, int64_t n, const float *M, const orc_sensor *s,
                 float *range, int32_t *src_idx, int64_t *stats);

/* total-least-squares plane of n FP64 points: unit normal, offset c = n.mu,
 * eigenvalues ascending.  Returns 0, or 1 if degenerate. */
int orc_tls(int n, const double *p, double *normal, double *c, double *evals);

/* seed (may be NULL): per tile (n_x, n_y, n_z, planarity logit) from the
 * seed network; a tile with logit > 0 tries one refit from the seed plane
 * and keeps it when it passes the acceptance test, else runs the plain fit. */
void orc_encode_key(const float *range, const orc_sensor *s, const orc_params *prm, const float *seed,
                    orc_frame *out);
void orc_encode_pred(const orc_frame *key, const float *range, const orc_sensor *s,
                     const orc_params *prm, orc_frame *out);

/* decode a frame to a range image (0 = empty).  key is NULL for a key frame. */
void orc_decode(const orc_frame *key, const orc_frame *fr, const orc_sensor *s,
                const orc_params *prm, float *range_out);

uint64_t orc_huffman_bits(const uint32_t *hist256);

/* Whole-sequence encode for the CPU baseline: nseq sequences of nf frames,
 * frame f of sequence q at xyz[q*nf+f] with count[q*nf+f] points and transform
 * M[(q*nf+f)*16] (ignored for the key frame).  Returns total bytes; frame sizes
 * go to sizes[].  OpenMP threads over frames (projection, predicted frames) and
 * over sequences (key frames). */
uint64_t orc_encode_sequences(int nseq, int nf, int key_index, const float *const *xyz,
                              const int64_t *count, const float *M, const orc_sensor *s,
                              const orc_params *prm, uint64_t *sizes, int64_t *finite_points);

/* ---- entropy-coded bitstream (Sec. III-A) ----
 * Code lengths of one stream from its byte histogram: Huffman code lengths
 * (two-queue construction over leaves sorted by (count, symbol), ties taking
 * the leaf), limited to 15 bits by the JPEG bit-count adjustment when the
 * tree is deeper, then given to the symbols by (count descending, symbol
 * ascending), shortest first.  One used symbol gets length 1. */
void orc_code_lengths(const uint32_t *hist256, uint8_t *len256);
/* Canonical code words (by length, then symbol), value right-aligned. */
void orc_canonical_codes(const uint8_t *len256, uint32_t *code256);
/* Bitstream of a frame whose streams were captured (sbuf): 112-byte header
 * (64 bytes of fixed fields, then the frame's transform into the key frame
 * M as 12 FP32, rows of [R | T]; M is 16 FP32 row-major, NULL = identity),
 * then per non-empty stream a 128-byte table of 4-bit lengths (symbol 2i in
 * the low nibble of byte i) and the code words MSB first, byte aligned.
 * kind: 0 key, 1 predicted.  Returns the byte count (0 if cap is too small
 * or a stream was not captured). */
uint64_t orc_pack(const orc_frame *f, int kind, int H, int W, int th, int tw, const float *M, uint8_t *out,
                  uint64_t cap);
/* Inverse of orc_pack down to the streams' bytes; nbytes[4] receives the
 * stream lengths, M (12 FP32, may be NULL) the transform.  Returns 0, or -1
 * on a malformed or too large input. */
int orc_unpack(const uint8_t *in, uint64_t n, uint8_t *const *streams, const uint64_t *caps, uint64_t *nbytes,
               float *M);

int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif

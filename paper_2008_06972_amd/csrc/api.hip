// C ABI entry points: argument checks, sensor tables, frame-stream layout,
// launches.  No allocation happens in the encode/decode calls; sensor tables
// are allocated once per distinct sensor by pc_sensor_register, and every
// other call takes a registered sensor only.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "encode_strip.h"

using namespace pcc;

namespace {

thread_local char g_err[512] = "";

struct SensorEntry {
  int H, W;
  float az0;
  std::vector<float> elev;
  float *dev = nullptr;     // one allocation: cut, ebx, eby, ce, se, ca, sa
  SensorDev sd{};
};

}  // namespace

struct pc_ctx {
  int device;
  void *ws;
  size_t ws_bytes;
  std::vector<SensorEntry *> sensors;
};

// Collision keys of pc_project_noalloc: one fixed array per device, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it is only a stand-in for the symbol): its device
// address comes from hipGetSymbolAddress, once per device, when the first
// context is created on that device.
static __device__ __align__(256) unsigned long long scratch[PC_PROJECT_NOALLOC_MAX_PIXELS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (device `dev` current).
pc_status scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return pcc::set_error(PC_ERR_DEVICE, "device %d beyond %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return PC_OK;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return pcc::set_error(PC_ERR_DEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
  g_scratch_ptr[dev] = (unsigned long long *)ptr;
  return PC_OK;
}
}  // namespace

namespace pcc {

pc_status set_error(pc_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

FrameDev frame_dev(void *base, const pc_layout &L) {
  char *b = (char *)base;
  FrameDev f;
  f.info = (pc_frame_info *)(b + L.off_info);
  f.occ = (uint32_t *)(b + L.off_occ);
  f.cls = (uint8_t *)(b + L.off_cls);
  f.mask = (uint64_t *)(b + L.off_mask);
  f.run_of = (int32_t *)(b + L.off_run_of);
  f.nruns = (int32_t *)(b + L.off_nruns);
  f.sruns = (pc_run *)(b + L.off_sruns);
  f.pruns = (pc_prun *)(b + L.off_pruns);
  f.nres = (int32_t *)(b + L.off_nres);
  f.res = (uint16_t *)(b + L.off_res);
  f.strip = (uint32_t *)(b + L.off_hist);
  f.tiles = (pc_tile_rec *)(b + L.off_tiles);
  f.TR = L.TR;
  f.TC = L.TC;
  f.T = L.T;
  return f;
}

}  // namespace pcc

// ------------------------------------------------------------------ checks
static pc_status check_sensor(const pc_sensor *s) {
  if (!s) return set_error(PC_ERR_ARG, "sensor is NULL");
  if (s->H < 2 || s->W < 32) return set_error(PC_ERR_ARG, "sensor needs H >= 2 and W >= 32 (got %d x %d)", s->H, s->W);
  if (s->W % 32) return set_error(PC_ERR_UNSUPPORTED, "W must be a multiple of 32 (got %d)", s->W);
  if (s->W > 4096 || s->H > 1024) return set_error(PC_ERR_UNSUPPORTED, "sensor larger than 1024 x 4096");
  if (!s->elev_rad) return set_error(PC_ERR_ARG, "sensor elevations are NULL");
  if (!isfinite(s->az0_rad)) return set_error(PC_ERR_ARG, "az0 is not finite");
  for (int v = 0; v < s->H; v++) {
    if (!isfinite(s->elev_rad[v])) return set_error(PC_ERR_ARG, "elevation %d is not finite", v);
    if (v && !(s->elev_rad[v] < s->elev_rad[v - 1])) return set_error(PC_ERR_ARG, "elevations must descend strictly");
  }
  double e0 = s->elev_rad[0], e1 = s->elev_rad[1], eh = s->elev_rad[s->H - 1], eh1 = s->elev_rad[s->H - 2];
  double top = e0 + 0.5 * (e0 - e1), bot = eh - 0.5 * (eh1 - eh);
  if (!(top < 1.5) || !(bot > -1.5)) return set_error(PC_ERR_ARG, "field of view must stay within +-1.5 rad");
  return PC_OK;
}

static pc_status check_params(const pc_sensor *s, const pc_params *p) {
  if (!p) return set_error(PC_ERR_ARG, "params is NULL");
  if (!(p->eps > 0.0f) || !isfinite(p->eps)) return set_error(PC_ERR_ARG, "eps must be > 0");
  bool shape = (p->tile_h == 4 && (p->tile_w == 4 || p->tile_w == 8 || p->tile_w == 16)) || (p->tile_h == 8 && p->tile_w == 8);
  if (p->tile_h <= 0 || p->tile_w <= 0 || p->tile_h * p->tile_w > 64)
    return set_error(PC_ERR_ARG, "tile must be positive with tile_h*tile_w <= 64");
  if (!shape) return set_error(PC_ERR_UNSUPPORTED, "tile %dx%d not compiled (4x4, 4x8, 4x16, 8x8)", p->tile_h, p->tile_w);
  if (p->max_iter < 1 || p->max_iter > 8) return set_error(PC_ERR_ARG, "max_iter must be in 1..8");
  if (p->min_pts < 3 || p->min_pts > 64) return set_error(PC_ERR_ARG, "min_pts must be in 3..64");
  if (!(p->min_inlier_frac > 0.0f) || !(p->min_inlier_frac <= 1.0f)) return set_error(PC_ERR_ARG, "min_inlier_frac must be in (0, 1]");
  if (s) {
    if (s->H % p->tile_h || s->W % p->tile_w)
      return set_error(PC_ERR_UNSUPPORTED, "H %% tile_h and W %% tile_w must be 0 (%dx%d, tile %dx%d)", s->H, s->W, p->tile_h, p->tile_w);
    // also keeps every strip's per-byte stream counts below 2^16 (16-bit
    // LDS histogram bins): at most 2 bytes per pixel and 17 per run
    if ((size_t)p->tile_h * s->W > 16384) return set_error(PC_ERR_UNSUPPORTED, "tile_h * W must be <= 16384");
    if (pcc::strip_lds_bytes(p->tile_h, p->tile_w, s->W, true) > kMaxStripLds)
      return set_error(PC_ERR_UNSUPPORTED, "a %dx%d-tile strip of width %d needs more than %zu bytes of LDS", p->tile_h,
                       p->tile_w, s->W, kMaxStripLds);
  }
  return PC_OK;
}

static EncParams enc_params(const pc_params *p) {
  EncParams e;
  e.eps = p->eps;
  e.th = p->tile_h;
  e.tw = p->tile_w;
  e.max_iter = p->max_iter;
  e.min_pts = p->min_pts;
  e.rho = p->min_inlier_frac;
  double st = 2.0 * (double)p->eps * (1.0 - 1.0 / 256.0);
  e.step = (float)st;
  e.inv = (float)(1.0 / (double)e.step);
  e.lanes = 4;
  for (int n = 0; n < 72; n++) {
    int a = n < p->min_pts ? n : p->min_pts;
    int b = (int)ceil((double)p->min_inlier_frac * (double)n);
    e.need[n] = (uint8_t)(n > 64 ? 0 : (a > b ? a : b));
  }
  return e;
}

// ------------------------------------------------------------ sensor tables
// FP64 trigonometry rounded once to FP32; row cuts at the elevation midpoints,
// field of view half a beam gap beyond the outer beams; columns advance
// clockwise from az0 (Sec. III-B, Eq. (2)).
// Table offsets (floats) in the one device allocation; every table starts
// on a 16-byte boundary so kernels may read it with 128-bit loads.
struct TableOffsets {
  size_t cut, ebx, eby, ce, se, ca, sa, total;
};
static TableOffsets table_offsets(int H, int W) {
  auto pad = [](size_t n) { return (n + 3) & ~(size_t)3; };
  TableOffsets o;
  o.cut = 0;
  o.ebx = o.cut + pad(H + 1);
  o.eby = o.ebx + pad(W);
  o.ce = o.eby + pad(W);
  o.se = o.ce + pad(H);
  o.ca = o.se + pad(H);
  o.sa = o.ca + pad(W);
  o.total = o.sa + pad(W);
  return o;
}

static void sensor_tables_host(const pc_sensor *s, std::vector<float> &t) {
  const int H = s->H, W = s->W;
  TableOffsets o = table_offsets(H, W);
  t.assign(o.total, 0.0f);
  float *cut = t.data() + o.cut, *ebx = t.data() + o.ebx, *eby = t.data() + o.eby, *ce = t.data() + o.ce,
        *se = t.data() + o.se, *ca = t.data() + o.ca, *sa = t.data() + o.sa;
  double e0 = s->elev_rad[0], e1 = s->elev_rad[1];
  double eh = s->elev_rad[H - 1], eh1 = s->elev_rad[H - 2];
  cut[0] = (float)tan(e0 + 0.5 * (e0 - e1));
  for (int v = 1; v < H; v++) cut[v] = (float)tan(0.5 * ((double)s->elev_rad[v - 1] + (double)s->elev_rad[v]));
  cut[H] = (float)tan(eh - 0.5 * (eh1 - eh));
  for (int v = 0; v < H; v++) {
    ce[v] = (float)cos((double)s->elev_rad[v]);
    se[v] = (float)sin((double)s->elev_rad[v]);
  }
  const double dth = 6.283185307179586476925286766559 / (double)W;
  for (int u = 0; u < W; u++) {
    double beta = (double)s->az0_rad - (double)u * dth;
    double alpha = (double)s->az0_rad - ((double)u + 0.5) * dth;
    ebx[u] = (float)cos(beta);
    eby[u] = (float)sin(beta);
    ca[u] = (float)cos(alpha);
    sa[u] = (float)sin(alpha);
  }
}

static SensorEntry *find_sensor(pc_ctx *ctx, const pc_sensor *s) {
  for (SensorEntry *e : ctx->sensors)
    if (e->H == s->H && e->W == s->W && memcmp(&e->az0, &s->az0_rad, 4) == 0 &&
        memcmp(e->elev.data(), s->elev_rad, sizeof(float) * s->H) == 0)
      return e;
  return nullptr;
}

// The tables of a registered sensor.  Encode, decode and batch calls use
// this: they never allocate, so a sensor must be registered first.
static pc_status get_sensor(pc_ctx *ctx, const pc_sensor *s, SensorEntry **out) {
  *out = find_sensor(ctx, s);
  if (!*out)
    return set_error(PC_ERR_STATE, "sensor %d x %d is not registered with this context (pc_sensor_register)", s->H,
                     s->W);
  return PC_OK;
}

// Compute and upload a sensor's tables (one device allocation per distinct
// sensor), or find them if the sensor is registered already.
static pc_status register_sensor(pc_ctx *ctx, const pc_sensor *s, SensorEntry **out) {
  if ((*out = find_sensor(ctx, s))) return PC_OK;
  std::vector<float> t;
  sensor_tables_host(s, t);
  SensorEntry *e = new SensorEntry();
  e->H = s->H;
  e->W = s->W;
  e->az0 = s->az0_rad;
  e->elev.assign(s->elev_rad, s->elev_rad + s->H);
  if (hipSetDevice(ctx->device) != hipSuccess || hipMalloc((void **)&e->dev, sizeof(float) * t.size()) != hipSuccess ||
      hipMemcpy(e->dev, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice) != hipSuccess) {
    delete e;
    return set_error(PC_ERR_DEVICE, "sensor table upload failed");
  }
  const int H = s->H, W = s->W;
  TableOffsets o = table_offsets(H, W);
  SensorDev &d = e->sd;
  d.H = H;
  d.W = W;
  d.cut = e->dev + o.cut;
  d.ebx = e->dev + o.ebx;
  d.eby = e->dev + o.eby;
  d.ce = e->dev + o.ce;
  d.se = e->dev + o.se;
  d.ca = e->dev + o.ca;
  d.sa = e->dev + o.sa;
  d.beta0 = (float)atan2((double)t[o.eby], (double)t[o.ebx]);
  d.dth = (float)(6.283185307179586476925286766559 / (double)W);
  d.inv_dth = (float)((double)W / 6.283185307179586476925286766559);
  d.elev0 = s->elev_rad[0];
  d.inv_de = (float)((double)(H - 1) / ((double)s->elev_rad[0] - (double)s->elev_rad[H - 1]));
  ctx->sensors.push_back(e);
  *out = e;
  return PC_OK;
}

// helpers for the batch planner (batch.hip)
pc_status pcc_sensor_dev(pc_ctx *ctx, const pc_sensor *s, SensorDev *out) {
  SensorEntry *e;
  pc_status st = get_sensor(ctx, s, &e);
  if (st == PC_OK) *out = e->sd;
  return st;
}
pc_status pcc_check_all(const pc_sensor *s, const pc_params *p) {
  pc_status st = check_sensor(s);
  if (st == PC_OK) st = check_params(s, p);
  return st;
}
EncParams pcc_enc_params(const pc_params *p) { return enc_params(p); }
pc_status pcc_check_sensor(const pc_sensor *s) { return check_sensor(s); }
int pcc_ctx_device(pc_ctx *ctx) { return ctx->device; }

// ------------------------------------------------------------------ the ABI
extern "C" {

const char *pc_last_error(void) { return g_err; }

const char *pc_version(void) { return "pcc-gfx950 1.0"; }

pc_status pc_stream_layout(const pc_sensor *sensor, const pc_params *params, pc_layout *out) {
  pc_status st = check_sensor(sensor);
  if (st) return st;
  if ((st = check_params(sensor, params))) return st;
  if (!out) return set_error(PC_ERR_ARG, "layout output is NULL");
  pc_layout L;
  memset(&L, 0, sizeof L);
  L.H = sensor->H;
  L.W = sensor->W;
  L.th = params->tile_h;
  L.tw = params->tile_w;
  L.TR = L.H / L.th;
  L.TC = L.W / L.tw;
  L.T = L.TR * L.TC;
  size_t off = 0;
  auto put = [&](size_t n) { size_t o = off; off = align256(off + n); return o; };
  const size_t T = (size_t)L.T, HW = (size_t)L.H * L.W;
  L.off_info = put(sizeof(pc_frame_info));
  L.off_occ = put((HW + 31) / 32 * 4);
  L.off_cls = put(T);
  L.off_mask = put(8 * T);
  L.off_run_of = put(4 * T);
  L.off_nruns = put(8 * (size_t)L.TR);
  L.off_sruns = put(sizeof(pc_run) * T);
  L.off_pruns = put(sizeof(pc_prun) * T);
  L.off_nres = put(4 * (size_t)L.TR);
  L.off_res = put(2 * HW);
  L.off_hist = put(4 * (size_t)L.TR * PC_STRIP_WORDS);
  L.off_tiles = put(sizeof(pc_tile_rec) * T);
  L.bytes = off;
  *out = L;
  return PC_OK;
}

size_t pc_workspace_size(const pc_sensor *sensor) {
  if (!sensor || sensor->H <= 0 || sensor->W <= 0) return 0;
  return align256((size_t)8 * sensor->H * sensor->W);
}

pc_status pc_ctx_create(pc_ctx **out, int device, void *workspace, size_t ws_bytes) {
  if (!out) return set_error(PC_ERR_ARG, "ctx output is NULL");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return set_error(PC_ERR_DEVICE, "no HIP device %d", device);
  if (hipSetDevice(device) != hipSuccess) return set_error(PC_ERR_DEVICE, "cannot select device %d", device);
  pc_status sst = scratch_address(device);
  if (sst != PC_OK) return sst;
  pc_ctx *c = new pc_ctx();
  c->device = device;
  c->ws = workspace;
  c->ws_bytes = workspace ? ws_bytes : 0;
  *out = c;
  return PC_OK;
}

pc_status pc_ctx_destroy(pc_ctx *ctx) {
  if (!ctx) return PC_OK;
  hipSetDevice(ctx->device);
  for (SensorEntry *e : ctx->sensors) {
    if (e->dev) hipFree(e->dev);
    delete e;
  }
  delete ctx;
  return PC_OK;
}

pc_status pc_sensor_register(pc_ctx *ctx, const pc_sensor *sensor) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_status st = check_sensor(sensor);
  if (st) return st;
  SensorEntry *e;
  return register_sensor(ctx, sensor, &e);
}

pc_status pc_sensor_tables(pc_ctx *ctx, const pc_sensor *sensor, float *cut, float *ebx, float *eby, float *ce,
                           float *se, float *ca, float *sa) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_status st = check_sensor(sensor);
  if (st) return st;
  SensorEntry *e;
  if ((st = get_sensor(ctx, sensor, &e))) return st;
  const int H = sensor->H, W = sensor->W;
  TableOffsets o = table_offsets(H, W);
  std::vector<float> t(o.total);
  if (hipMemcpy(t.data(), e->dev, sizeof(float) * t.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return set_error(PC_ERR_DEVICE, "table read-back failed");
  if (cut) memcpy(cut, t.data() + o.cut, sizeof(float) * (H + 1));
  if (ebx) memcpy(ebx, t.data() + o.ebx, sizeof(float) * W);
  if (eby) memcpy(eby, t.data() + o.eby, sizeof(float) * W);
  if (ce) memcpy(ce, t.data() + o.ce, sizeof(float) * H);
  if (se) memcpy(se, t.data() + o.se, sizeof(float) * H);
  if (ca) memcpy(ca, t.data() + o.ca, sizeof(float) * W);
  if (sa) memcpy(sa, t.data() + o.sa, sizeof(float) * W);
  return PC_OK;
}

pc_status pc_project(pc_ctx *ctx, const float *xyz, int64_t n, const float *M_host, const pc_sensor *sensor,
                     float *range, int32_t *src_idx, pc_proj_stats *stats, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_status st = check_sensor(sensor);
  if (st) return st;
  if (n < 0 || n > 0x7fffffffLL) return set_error(PC_ERR_ARG, "point count %lld out of range", (long long)n);
  if (n > 0 && !xyz) return set_error(PC_ERR_ARG, "xyz is NULL");
  if (!range) return set_error(PC_ERR_ARG, "range output is NULL");
  if (M_host)
    for (int e = 0; e < 16; e++)
      if (!isfinite(M_host[e])) return set_error(PC_ERR_ARG, "transform has a non-finite entry");
  size_t need = (size_t)8 * sensor->H * sensor->W;
  if (!ctx->ws || ctx->ws_bytes < need)
    return set_error(PC_ERR_CAPACITY, "workspace %zu bytes < %zu needed", ctx->ws_bytes, need);
  SensorEntry *e;
  if ((st = get_sensor(ctx, sensor, &e))) return st;
  hipError_t he = launch_project(xyz, n, M_host, e->sd, (unsigned long long *)ctx->ws, range, src_idx, stats,
                                 (hipStream_t)stream);
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "projection launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

pc_status pc_project_noalloc(pc_ctx *ctx, const float *xyz, int64_t n, const float *M_host, const pc_sensor *sensor,
                             float *range, int32_t *src_idx, pc_proj_stats *stats, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_status st = check_sensor(sensor);
  if (st) return st;
  if (n < 0 || n > 0x7fffffffLL) return set_error(PC_ERR_ARG, "point count %lld out of range", (long long)n);
  if (n > 0 && !xyz) return set_error(PC_ERR_ARG, "xyz is NULL");
  if (!range) return set_error(PC_ERR_ARG, "range output is NULL");
  if (M_host)
    for (int e = 0; e < 16; e++)
      if (!isfinite(M_host[e])) return set_error(PC_ERR_ARG, "transform has a non-finite entry");
  if ((int64_t)sensor->H * sensor->W > PC_PROJECT_NOALLOC_MAX_PIXELS)
    return set_error(PC_ERR_CAPACITY, "sensor %d x %d has more than the %d pixels of the fixed projection scratch",
                     sensor->H, sensor->W, PC_PROJECT_NOALLOC_MAX_PIXELS);
  SensorEntry *e;
  if ((st = get_sensor(ctx, sensor, &e))) return st;
  unsigned long long *keys = ctx->device >= 0 && ctx->device < kMaxDevices ? g_scratch_ptr[ctx->device] : nullptr;
  if (!keys) return set_error(PC_ERR_STATE, "no scratch address for device %d", ctx->device);
  hipError_t he = launch_project(xyz, n, M_host, e->sd, keys, range, src_idx, stats, (hipStream_t)stream);
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "projection launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

pc_status pc_fit_key(pc_ctx *ctx, const float *range, const pc_sensor *sensor, const pc_params *params,
                     const float *seed, void *out, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_status st = check_sensor(sensor);
  if (st) return st;
  if ((st = check_params(sensor, params))) return st;
  if (!range || !out) return set_error(PC_ERR_ARG, "range or output stream is NULL");
  SensorEntry *e;
  if ((st = get_sensor(ctx, sensor, &e))) return st;
  pc_layout L;
  pc_stream_layout(sensor, params, &L);
  FrameDev f = frame_dev(out, L);
  EncParams p = enc_params(params);
  hipError_t he = launch_key(range, e->sd, p, seed, f, nullptr, (hipStream_t)stream);
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "key-frame launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

pc_status pc_encode_pred(pc_ctx *ctx, const void *key, const float *range, const float *M_host,
                         const pc_sensor *sensor, const pc_params *params, void *out, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_status st = check_sensor(sensor);
  if (st) return st;
  if ((st = check_params(sensor, params))) return st;
  if (!key || !range || !out) return set_error(PC_ERR_ARG, "key, range or output stream is NULL");
  if (key == out) return set_error(PC_ERR_ARG, "output stream must differ from the key stream");
  SensorEntry *e;
  if ((st = get_sensor(ctx, sensor, &e))) return st;
  pc_layout L;
  pc_stream_layout(sensor, params, &L);
  FrameDev f = frame_dev(out, L), k = frame_dev((void *)key, L);
  EncParams p = enc_params(params);
  float M12[12];
  if (M_host)
    for (int q = 0; q < 12; q++) M12[q] = M_host[q];
  hipError_t he = launch_pred(k, range, e->sd, p, f, M_host ? M12 : nullptr, (hipStream_t)stream);
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "predicted-frame launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

pc_status pc_decode(pc_ctx *ctx, const void *key, const void *frame, const pc_sensor *sensor, const pc_params *params,
                    float *range_out, float *xyz_out, int32_t frame_coords, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  pc_status st = check_sensor(sensor);
  if (st) return st;
  if ((st = check_params(sensor, params))) return st;
  if (!frame || (!range_out && !xyz_out)) return set_error(PC_ERR_ARG, "frame is NULL or no output is given");
  if (frame_coords != 0 && frame_coords != 1) return set_error(PC_ERR_ARG, "frame_coords must be 0 or 1");
  SensorEntry *e;
  if ((st = get_sensor(ctx, sensor, &e))) return st;
  pc_layout L;
  pc_stream_layout(sensor, params, &L);
  FrameDev f = frame_dev((void *)frame, L);
  FrameDev k = key ? frame_dev((void *)key, L) : f;
  EncParams p = enc_params(params);
  hipError_t he = launch_decode(key ? &k : nullptr, f, e->sd, p, range_out, xyz_out, frame_coords,
                                (hipStream_t)stream);
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "decode launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

size_t pc_decode_batch_workspace_size(int32_t n) { return n < 1 ? 0 : align256(sizeof(DecodeJob) * (size_t)n); }

pc_status pc_decode_batch(pc_ctx *ctx, int32_t n, const void *const *keys, const void *const *frames,
                          const pc_sensor *sensor, const pc_params *params, float *const *range_out,
                          float *const *xyz_out, int32_t frame_coords, void *work, size_t work_bytes, void *stream) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  if (n < 1 || n > 65535) return set_error(PC_ERR_ARG, "frame count %d out of range 1..65535", n);
  pc_status st = check_sensor(sensor);
  if (st) return st;
  if ((st = check_params(sensor, params))) return st;
  if (!frames || (!range_out && !xyz_out) || !work) return set_error(PC_ERR_ARG, "frames, outputs or workspace is NULL");
  if (frame_coords != 0 && frame_coords != 1) return set_error(PC_ERR_ARG, "frame_coords must be 0 or 1");
  if (work_bytes < pc_decode_batch_workspace_size(n)) return set_error(PC_ERR_CAPACITY, "workspace too small");
  SensorEntry *e;
  if ((st = get_sensor(ctx, sensor, &e))) return st;
  pc_layout L;
  pc_stream_layout(sensor, params, &L);
  std::vector<DecodeJob> jobs((size_t)n);
  for (int i = 0; i < n; i++) {
    float *ro = range_out ? range_out[i] : nullptr, *xo = xyz_out ? xyz_out[i] : nullptr;
    if (!frames[i] || (!ro && !xo)) return set_error(PC_ERR_ARG, "frame %d or both of its outputs are NULL", i);
    const void *k = keys ? keys[i] : nullptr;
    jobs[i].f = frame_dev((void *)frames[i], L);
    jobs[i].key = k ? frame_dev((void *)k, L) : jobs[i].f;
    jobs[i].has_key = k ? 1 : 0;
    jobs[i].out = ro;
    jobs[i].xyz = xo;
    jobs[i].frame_coords = frame_coords;
  }
  hipStream_t hs = (hipStream_t)stream;
  DecodeJob *dj = (DecodeJob *)work;
  // the job table is read by the launch; the host copy must outlive the upload
  if (hipMemcpyAsync(dj, jobs.data(), sizeof(DecodeJob) * (size_t)n, hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipStreamSynchronize(hs) != hipSuccess)
    return set_error(PC_ERR_DEVICE, "job table upload failed");
  hipError_t he = launch_decode_jobs(jobs[0], dj, n, e->sd, enc_params(params), hs);
  if (he != hipSuccess) return set_error(PC_ERR_DEVICE, "decode launch failed: %s", hipGetErrorString(he));
  return PC_OK;
}

pc_status pc_check(pc_ctx *ctx, void *stream, const void *const *frames, int32_t nframes) {
  if (!ctx) return set_error(PC_ERR_ARG, "ctx is NULL");
  if (nframes < 0 || (nframes > 0 && !frames)) return set_error(PC_ERR_ARG, "bad frame list");
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return set_error(PC_ERR_DEVICE, "stream synchronisation failed");
  for (int i = 0; i < nframes; i++) {
    pc_frame_info I;
    if (hipMemcpy(&I, frames[i], sizeof I, hipMemcpyDeviceToHost) != hipSuccess)
      return set_error(PC_ERR_DEVICE, "info read-back failed");
    if (I.status & PC_STATUS_RANGE) return set_error(PC_ERR_RANGE, "frame %d: a residual is out of code range", i);
    if (I.status & PC_STATUS_NOKEY)
      return set_error(PC_ERR_STATE, "frame %d: a predicted frame was decoded without its key frame", i);
  }
  return PC_OK;
}

}  // extern "C"

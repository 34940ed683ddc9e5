"""Thin Python binding of the C ABI in ``include/pc.h`` (ctypes).

Every function named ``pc_*`` here marshals arguments and calls the entry
point of the same name in ``libpcc.so``; all work runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.  There is no fallback:
if the library is missing the import of :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcc.so")

PC_OK, PC_ERR_ARG, PC_ERR_CAPACITY, PC_ERR_DEVICE, PC_ERR_STATE, PC_ERR_UNSUPPORTED, PC_ERR_RANGE = 0, -1, -2, -3, -4, -5, -6
PC_STATUS_RANGE, PC_STATUS_NOKEY = 1, 2
PC_STRIP_STATS = 16
PC_PROJECT_NOALLOC_MAX_PIXELS = 524288
PC_STRIP_WORDS = 4 * 256 + PC_STRIP_STATS


class PcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pc status {status}: {msg}")
        self.status = status


class pc_sensor(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("elev_rad", C.c_void_p), ("az0_rad", C.c_float)]


class pc_params(C.Structure):
    _fields_ = [("eps", C.c_float), ("tile_h", C.c_int32), ("tile_w", C.c_int32), ("max_iter", C.c_int32),
                ("min_pts", C.c_int32), ("min_inlier_frac", C.c_float)]


class pc_layout(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("H", "W", "th", "tw", "TR", "TC", "T", "pad")] + [
        (n, C.c_size_t) for n in ("bytes", "off_info", "off_occ", "off_cls", "off_mask", "off_run_of", "off_nruns",
                                  "off_sruns", "off_pruns", "off_nres", "off_res", "off_hist", "off_tiles")]


class pc_proj_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_in", "n_nonfinite", "n_fov", "n_collided", "n_kept")]


class pc_frame_info(C.Structure):
    _fields_ = [("kind", C.c_int32), ("status", C.c_uint32), ("n_sruns", C.c_int32), ("n_pruns", C.c_int32),
                ("n_valid", C.c_int64), ("n_res", C.c_int64), ("tiles", C.c_int32 * 4), ("fits", C.c_int32),
                ("fp64_fits", C.c_int32), ("seeded", C.c_int32), ("fallback", C.c_int32),
                ("stream_bytes", C.c_uint64 * 4), ("coded_bits", C.c_uint64 * 4), ("size_bytes", C.c_uint64),
                ("M", C.c_float * 12), ("pad", C.c_int32 * 4)]


class pc_frame_desc(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("n", C.c_int64), ("M", C.c_void_p), ("sensor", C.c_void_p),
                ("params", C.c_void_p), ("key", C.c_int32), ("pad", C.c_int32), ("seed", C.c_void_p),
                ("range", C.c_void_p), ("out", C.c_void_p)]


class pc_batch_opts(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("graph", C.c_int32), ("blocks_per_cu", C.c_int32), ("records", C.c_int32),
                ("net", C.c_void_p), ("lanes_max", C.c_int32)]


# numpy views of the device records
RUN_DTYPE = np.dtype([("s", "<i4"), ("len", "<i4"), ("axis", "<i4"), ("a", "<f4"), ("b", "<f4"), ("c", "<f4")])
PRUN_DTYPE = np.dtype([("s", "<i4"), ("len", "<i4"), ("krun", "<i4"), ("c", "<f4")])
TILE_DTYPE = np.dtype([("a", "<f4"), ("b", "<f4"), ("c", "<f4"), ("axis", "u1"), ("status", "u1"), ("iters", "u1"),
                       ("t_status", "u1"), ("mask", "<u8"), ("t_mask", "<u8"), ("t_c", "<f4"), ("t_iters", "u1"),
                       ("seeded", "u1"), ("pad", "u1", (2,))])

_lib = None


def lib():
    """Load ``libpcc.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.pc_last_error.restype = C.c_char_p
        L.pc_version.restype = C.c_char_p
        L.pc_workspace_size.restype = C.c_size_t
        for name in ("pc_stream_layout", "pc_ctx_create", "pc_ctx_destroy", "pc_sensor_register", "pc_sensor_tables",
                     "pc_project", "pc_fit_key", "pc_encode_pred", "pc_decode", "pc_check", "pc_batch_create",
                     "pc_batch_run", "pc_batch_info", "pc_batch_profile", "pc_batch_destroy", "pc_net_forward",
                     "pc_net_backward", "pc_net_loss", "pc_net_adam", "pc_pack", "pc_unpack", "pc_pack_streams",
                     "pc_unpack_streams", "pc_pack_batch", "pc_imu_transform", "pc_decode_batch",
                     "pc_unpack_batch", "pc_project_noalloc"):
            getattr(L, name).restype = C.c_int
        L.pc_batch_workspace_size.restype = C.c_size_t
        L.pc_net_workspace_size.restype = C.c_size_t
        L.pc_pack_bound.restype = C.c_size_t
        L.pc_pack_workspace_size.restype = C.c_size_t
        L.pc_pack_batch_workspace_size.restype = C.c_size_t
        L.pc_decode_batch_workspace_size.restype = C.c_size_t
        L.pc_unpack_batch_workspace_size.restype = C.c_size_t
        L.pc_stream_pack_bound.restype = C.c_uint64
        L.pc_stream_pack_workspace_size.restype = C.c_size_t
        _lib = L
    return _lib


EXPORTED = ("pc_stream_layout", "pc_workspace_size", "pc_ctx_create", "pc_ctx_destroy", "pc_sensor_register",
            "pc_sensor_tables", "pc_project", "pc_fit_key", "pc_encode_pred", "pc_decode", "pc_check",
            "pc_last_error", "pc_version", "pc_batch_workspace_size", "pc_batch_create", "pc_batch_run",
            "pc_batch_info", "pc_batch_profile", "pc_batch_destroy", "pc_net_workspace_size", "pc_net_forward",
            "pc_net_backward", "pc_net_loss", "pc_net_adam", "pc_pack_bound", "pc_pack_workspace_size", "pc_pack",
            "pc_unpack", "pc_stream_pack_bound", "pc_stream_pack_workspace_size", "pc_pack_streams",
            "pc_unpack_streams", "pc_pack_batch_workspace_size", "pc_pack_batch", "pc_imu_transform",
            "pc_decode_batch_workspace_size", "pc_decode_batch", "pc_unpack_batch_workspace_size", "pc_unpack_batch",
            "pc_project_noalloc")
PC_NET_PARAMS = 15636
LAUNCH_KINDS = {0: "reset", 1: "bin", 2: "offsets", 3: "scatter", 4: "key", 5: "pred", 6: "finish",
                7: "keyimage", 8: "net"}


def _check(st: int):
    if st != PC_OK:
        raise PcError(st, lib().pc_last_error().decode())


def _ptr(x):
    """Device or host address of a torch tensor / numpy array / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return C.c_void_p(x)
    if hasattr(x, "data_ptr"):
        return C.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(C.c_void_p)
    raise TypeError(type(x))


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------- host structs
class Sensor:
    """Holds a pc_sensor and the host elevation array it points to."""

    def __init__(self, H: int, W: int, elev_rad: np.ndarray, az0: float):
        self.elev = np.ascontiguousarray(elev_rad, dtype=np.float32)
        assert self.elev.shape == (H,)
        self.c = pc_sensor(H, W, self.elev.ctypes.data, float(az0))
        self.H, self.W = H, W

    @classmethod
    def of(cls, s):
        return cls(s.H, s.W, s.elevations(), s.az0)


def params(eps=0.02, tile_h=4, tile_w=8, max_iter=5, min_pts=4, min_inlier_frac=0.5) -> pc_params:
    return pc_params(eps, tile_h, tile_w, max_iter, min_pts, min_inlier_frac)


# ---------------------------------------------------------------- the ABI
def pc_stream_layout(sensor: Sensor, prm: pc_params) -> pc_layout:
    L = pc_layout()
    _check(lib().pc_stream_layout(C.byref(sensor.c), C.byref(prm), C.byref(L)))
    return L


def pc_workspace_size(sensor: Sensor) -> int:
    return int(lib().pc_workspace_size(C.byref(sensor.c)))


def pc_ctx_create(device: int, workspace, ws_bytes: int):
    h = C.c_void_p()
    _check(lib().pc_ctx_create(C.byref(h), C.c_int(device), _ptr(workspace), C.c_size_t(ws_bytes)))
    return h


def pc_ctx_destroy(ctx):
    _check(lib().pc_ctx_destroy(ctx))


def pc_sensor_register(ctx, sensor: Sensor):
    _check(lib().pc_sensor_register(ctx, C.byref(sensor.c)))


def pc_sensor_tables(ctx, sensor: Sensor):
    H, W = sensor.H, sensor.W
    out = {k: np.zeros(n, np.float32) for k, n in
           (("cut", H + 1), ("ebx", W), ("eby", W), ("ce", H), ("se", H), ("ca", W), ("sa", W))}
    _check(lib().pc_sensor_tables(ctx, C.byref(sensor.c), *(_ptr(out[k]) for k in
                                                               ("cut", "ebx", "eby", "ce", "se", "ca", "sa"))))
    return out


def pc_project(ctx, xyz, n: int, M_host, sensor: Sensor, range_out, src_idx=None, stats=None, stream=None):
    Mh = None if M_host is None else np.ascontiguousarray(M_host, dtype=np.float32).reshape(16)
    _check(lib().pc_project(ctx, _ptr(xyz), C.c_int64(n), _ptr(Mh), C.byref(sensor.c), _ptr(range_out),
                            _ptr(src_idx), _ptr(stats), _stream(stream)))


def pc_project_noalloc(ctx, xyz, n: int, M_host, sensor: Sensor, range_out, src_idx=None, stats=None, stream=None):
    Mh = None if M_host is None else np.ascontiguousarray(M_host, dtype=np.float32).reshape(16)
    _check(lib().pc_project_noalloc(ctx, _ptr(xyz), C.c_int64(n), _ptr(Mh), C.byref(sensor.c), _ptr(range_out),
                                    _ptr(src_idx), _ptr(stats), _stream(stream)))


def pc_fit_key(ctx, range_img, sensor: Sensor, prm: pc_params, seed, out, stream=None):
    _check(lib().pc_fit_key(ctx, _ptr(range_img), C.byref(sensor.c), C.byref(prm), _ptr(seed), _ptr(out),
                            _stream(stream)))


def pc_net_workspace_size(sensor: Sensor) -> int:
    return int(lib().pc_net_workspace_size(C.byref(sensor.c)))


def pc_net_forward(ctx, params, range_img, sensor: Sensor, work, seed, stream=None):
    _check(lib().pc_net_forward(ctx, _ptr(params), _ptr(range_img), C.byref(sensor.c), _ptr(work),
                                C.c_size_t(work.numel() * work.element_size()), _ptr(seed), _stream(stream)))


def pc_net_backward(ctx, params, sensor: Sensor, work, dseed, grad, stream=None):
    _check(lib().pc_net_backward(ctx, _ptr(params), C.byref(sensor.c), _ptr(work),
                                 C.c_size_t(work.numel() * work.element_size()), _ptr(dseed), _ptr(grad),
                                 _stream(stream)))


def pc_net_loss(ctx, seed, labels, sensor: Sensor, prm: pc_params, dseed, loss, stream=None):
    _check(lib().pc_net_loss(ctx, _ptr(seed), _ptr(labels), C.byref(sensor.c), C.byref(prm), _ptr(dseed), _ptr(loss),
                             _stream(stream)))


def pc_net_adam(ctx, params, grad, m, v, step: int, lr: float, stream=None):
    _check(lib().pc_net_adam(ctx, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), C.c_int32(step), C.c_float(lr),
                             _stream(stream)))


def pc_encode_pred(ctx, key, range_img, M_host, sensor: Sensor, prm: pc_params, out, stream=None):
    Mh = None if M_host is None else np.ascontiguousarray(M_host, dtype=np.float32).reshape(16)
    _check(lib().pc_encode_pred(ctx, _ptr(key), _ptr(range_img), _ptr(Mh), C.byref(sensor.c), C.byref(prm),
                                _ptr(out), _stream(stream)))


def pc_decode(ctx, key, frame, sensor: Sensor, prm: pc_params, range_out, xyz_out=None, frame_coords=0,
              stream=None):
    _check(lib().pc_decode(ctx, _ptr(key), _ptr(frame), C.byref(sensor.c), C.byref(prm), _ptr(range_out),
                           _ptr(xyz_out), C.c_int32(frame_coords), _stream(stream)))


def pc_decode_batch_workspace_size(n: int) -> int:
    return int(lib().pc_decode_batch_workspace_size(C.c_int32(n)))


def pc_decode_batch(ctx, keys, frames, sensor: Sensor, prm: pc_params, range_out, work, work_bytes: int,
                    stream=None, xyz_out=None, frame_coords=0):
    """keys: None or a list with None for key frames; range_out, xyz_out:
    None or lists of device buffers (entries may be None)."""
    n = len(frames)

    def arr(xs):
        return None if xs is None else (C.c_void_p * n)(*[(_ptr(x).value if x is not None else None) for x in xs])
    fa = (C.c_void_p * n)(*[_ptr(f).value for f in frames])
    _check(lib().pc_decode_batch(ctx, C.c_int32(n), arr(keys), fa, C.byref(sensor.c), C.byref(prm), arr(range_out),
                                 arr(xyz_out), C.c_int32(frame_coords), _ptr(work), C.c_size_t(work_bytes),
                                 _stream(stream)))


def pc_check(ctx, frames, stream=None):
    arr = (C.c_void_p * max(1, len(frames)))(*[_ptr(f).value for f in frames])
    _check(lib().pc_check(ctx, _stream(stream), arr, C.c_int32(len(frames))))


def pc_batch_workspace_size(frames, opts=None) -> int:
    arr = (pc_frame_desc * len(frames))(*frames)
    return int(lib().pc_batch_workspace_size(arr, C.c_int32(len(frames)), C.byref(opts) if opts is not None else None))


def pc_batch_create(ctx, frames, opts, workspace, ws_bytes):
    arr = (pc_frame_desc * len(frames))(*frames)
    h = C.c_void_p()
    _check(lib().pc_batch_create(ctx, arr, C.c_int32(len(frames)), C.byref(opts) if opts is not None else None,
                                 _ptr(workspace), C.c_size_t(ws_bytes), C.byref(h)))
    return h


def pc_batch_run(batch, stream=None):
    _check(lib().pc_batch_run(batch, _stream(stream)))


def pc_batch_info(batch):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().pc_batch_info(batch, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def pc_batch_profile(batch, stream=None, cap=64):
    ms = np.zeros(cap, np.float32)
    kinds = np.zeros(cap, np.int32)
    n = C.c_int32()
    _check(lib().pc_batch_profile(batch, _stream(stream), _ptr(ms), _ptr(kinds), C.c_int32(cap), C.byref(n)))
    return [(LAUNCH_KINDS[int(k)], float(t)) for k, t in zip(kinds[:n.value], ms[:n.value])]


def pc_batch_destroy(batch):
    _check(lib().pc_batch_destroy(batch))


def _u64x4(n):
    return (C.c_uint64 * 4)(*[int(x) for x in n])


def _ptrx4(ps):
    return (C.c_void_p * 4)(*[(_ptr(p).value if p is not None else None) for p in ps])


def pc_pack_bound(sensor: Sensor, prm: pc_params) -> int:
    return int(lib().pc_pack_bound(C.byref(sensor.c), C.byref(prm)))


def pc_pack_workspace_size(sensor: Sensor, prm: pc_params) -> int:
    return int(lib().pc_pack_workspace_size(C.byref(sensor.c), C.byref(prm)))


def pc_pack(ctx, frame, sensor: Sensor, prm: pc_params, work, work_bytes: int, out, cap: int, nbytes, streams=None,
            stream_caps=None, stream=None):
    sp = _ptrx4(streams) if streams is not None else None
    sc = _u64x4(stream_caps) if stream_caps is not None else None
    _check(lib().pc_pack(ctx, _ptr(frame), C.byref(sensor.c), C.byref(prm), _ptr(work), C.c_size_t(work_bytes),
                         _ptr(out), C.c_uint64(cap), _ptr(nbytes), sp, sc, _stream(stream)))


def pc_pack_batch_workspace_size(sensor: Sensor, prm: pc_params, n: int) -> int:
    return int(lib().pc_pack_batch_workspace_size(C.byref(sensor.c), C.byref(prm), C.c_int32(n)))


def pc_pack_batch(ctx, frames, sensor: Sensor, prm: pc_params, work, work_bytes: int, outs, cap: int, nbytes,
                  stream=None):
    n = len(frames)
    fa = (C.c_void_p * n)(*[_ptr(f).value for f in frames])
    oa = (C.c_void_p * n)(*[_ptr(o).value for o in outs])
    _check(lib().pc_pack_batch(ctx, C.c_int32(n), fa, C.byref(sensor.c), C.byref(prm), _ptr(work),
                               C.c_size_t(work_bytes), oa, C.c_uint64(cap), _ptr(nbytes), _stream(stream)))


def pc_unpack(ctx, data, n_in: int, key, sensor: Sensor, prm: pc_params, work, work_bytes: int, frame_out,
              stream=None) -> int:
    kind = C.c_int32(-1)
    _check(lib().pc_unpack(ctx, _ptr(data), C.c_uint64(n_in), _ptr(key), C.byref(sensor.c), C.byref(prm), _ptr(work),
                           C.c_size_t(work_bytes), _ptr(frame_out), C.byref(kind), _stream(stream)))
    return kind.value


def pc_unpack_batch_workspace_size(sensor: Sensor, prm: pc_params, n: int) -> int:
    return int(lib().pc_unpack_batch_workspace_size(C.byref(sensor.c), C.byref(prm), C.c_int32(n)))


def pc_unpack_batch(ctx, data, n_in, keys, sensor: Sensor, prm: pc_params, work, work_bytes: int, frames_out,
                    stream=None):
    """Returns the containers' kinds.  keys: None or a list with None for key frames."""
    n = len(data)
    da = (C.c_void_p * n)(*[_ptr(d).value for d in data])
    na = (C.c_uint64 * n)(*[int(x) for x in n_in])
    ka = None if keys is None else (C.c_void_p * n)(*[(_ptr(k).value if k is not None else None) for k in keys])
    fa = (C.c_void_p * n)(*[_ptr(f).value for f in frames_out])
    kinds = (C.c_int32 * n)()
    _check(lib().pc_unpack_batch(ctx, C.c_int32(n), da, na, ka, C.byref(sensor.c), C.byref(prm), _ptr(work),
                                 C.c_size_t(work_bytes), fa, kinds, _stream(stream)))
    return [int(k) for k in kinds]


def pc_stream_pack_bound(n) -> int:
    return int(lib().pc_stream_pack_bound(_u64x4(n)))


def pc_stream_pack_workspace_size(n) -> int:
    return int(lib().pc_stream_pack_workspace_size(_u64x4(n)))


def pc_pack_streams(ctx, streams, n, kind: int, H: int, W: int, tile_h: int, tile_w: int, work, work_bytes: int, out,
                    cap: int, nbytes, stream=None):
    _check(lib().pc_pack_streams(ctx, _ptrx4(streams), _u64x4(n), C.c_int32(kind), C.c_int32(H), C.c_int32(W),
                                 C.c_int32(tile_h), C.c_int32(tile_w), _ptr(work), C.c_size_t(work_bytes), _ptr(out),
                                 C.c_uint64(cap), _ptr(nbytes), _stream(stream)))


def pc_unpack_streams(ctx, data, n_in: int, work, work_bytes: int, streams, caps, stream=None):
    n_out = (C.c_uint64 * 4)()
    _check(lib().pc_unpack_streams(ctx, _ptr(data), C.c_uint64(n_in), _ptr(work), C.c_size_t(work_bytes),
                                   _ptrx4(streams), _u64x4(caps), n_out, _stream(stream)))
    return [int(x) for x in n_out]


def pc_imu_transform(acc, gyro, dt: float, v0=None):
    """(M 4x4 FP32, velocity after the last sample) from host IMU samples."""
    a = np.ascontiguousarray(acc, dtype=np.float32).reshape(-1, 3)
    g = np.ascontiguousarray(gyro, dtype=np.float32).reshape(-1, 3)
    if len(a) != len(g):
        raise ValueError("acc and gyro need the same number of samples")
    v = None if v0 is None else np.ascontiguousarray(v0, dtype=np.float32).reshape(3)
    M = np.zeros(16, np.float32)
    ve = np.zeros(3, np.float32)
    _check(lib().pc_imu_transform(_ptr(a), _ptr(g), C.c_int32(len(a)), C.c_float(dt), _ptr(v), _ptr(M), _ptr(ve)))
    return M.reshape(4, 4), ve


def pc_version() -> str:
    return lib().pc_version().decode()


# ---------------------------------------------------- torch-side convenience
class Context:
    """A pc_ctx with a device workspace allocated by torch."""

    def __init__(self, sensors, device: int = 0):
        import torch
        ws = max(pc_workspace_size(s) for s in sensors)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=f"cuda:{device}")
        self.h = pc_ctx_create(device, self.ws, ws)
        for s in sensors:
            pc_sensor_register(self.h, s)

    def close(self):
        if self.h is not None:
            pc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FrameStream:
    """A device frame stream buffer with host-side readers of its sections."""

    def __init__(self, sensor: Sensor, prm: pc_params, device="cuda"):
        import torch
        self.L = pc_stream_layout(sensor, prm)
        self.buf = torch.zeros(self.L.bytes, dtype=torch.uint8, device=device)

    def data_ptr(self):
        return self.buf.data_ptr()

    def _sec(self, off, nbytes):
        return self.buf[off:off + nbytes].cpu().numpy()

    def info(self) -> pc_frame_info:
        raw = self._sec(self.L.off_info, C.sizeof(pc_frame_info))
        return pc_frame_info.from_buffer_copy(raw.tobytes())

    def host(self) -> dict:
        """Copy the encoded sections to host numpy arrays."""
        L = self.L
        b = self.buf.cpu().numpy()
        T, TR, TC = L.T, L.TR, L.TC
        out = {
            "info": pc_frame_info.from_buffer_copy(b[L.off_info:L.off_info + C.sizeof(pc_frame_info)].tobytes()),
            "occ": b[L.off_occ:L.off_occ + (L.H * L.W + 31) // 32 * 4].view(np.uint32),
            "cls": b[L.off_cls:L.off_cls + T].copy(),
            "mask": b[L.off_mask:L.off_mask + 8 * T].view(np.uint64),
            "run_of": b[L.off_run_of:L.off_run_of + 4 * T].view(np.int32),
            "nruns": b[L.off_nruns:L.off_nruns + 8 * TR].view(np.int32),
            "sruns": b[L.off_sruns:L.off_sruns + RUN_DTYPE.itemsize * T].view(RUN_DTYPE),
            "pruns": b[L.off_pruns:L.off_pruns + PRUN_DTYPE.itemsize * T].view(PRUN_DTYPE),
            "nres": b[L.off_nres:L.off_nres + 4 * TR].view(np.int32),
            "res": b[L.off_res:L.off_res + 2 * L.H * L.W].view(np.uint16),
            "strip": b[L.off_hist:L.off_hist + 4 * TR * PC_STRIP_WORDS].view(np.uint32).reshape(TR, PC_STRIP_WORDS),
            "tiles": b[L.off_tiles:L.off_tiles + TILE_DTYPE.itemsize * T].view(TILE_DTYPE),
        }
        # flattened run lists in row order (slots r*TC .. r*TC+n)
        ns, npr = out["nruns"][:TR], out["nruns"][TR:]
        out["srun_list"] = np.concatenate([out["sruns"][r * TC:r * TC + ns[r]] for r in range(TR)])
        out["srun_row"] = np.concatenate([np.full(ns[r], r, np.int32) for r in range(TR)])
        out["prun_list"] = np.concatenate([out["pruns"][r * TC:r * TC + npr[r]] for r in range(TR)])
        out["prun_row"] = np.concatenate([np.full(npr[r], r, np.int32) for r in range(TR)])
        thw = L.th * L.W
        out["codes"] = np.concatenate([out["res"][r * thw:r * thw + out["nres"][r]] for r in range(TR)])
        return out


class Batch:
    """A batch plan over frames given as dicts with keys xyz (device tensor),
    M (host 4x4 or None), sensor (Sensor), params (pc_params), key (int),
    out (FrameStream), range (device tensor or None), seed (tensor or None)."""

    def __init__(self, ctx: Context, frames, persistent=True, graph=True, blocks_per_cu=0, net=None, records=False,
                 lanes_max=0):
        import torch
        self._keep = []
        descs = []
        for i, f in enumerate(frames):
            M = None
            if f.get("M") is not None:
                M = np.ascontiguousarray(f["M"], dtype=np.float32).reshape(16)
                self._keep.append(M)
            d = pc_frame_desc()
            d.xyz = f["xyz"].data_ptr() if len(f["xyz"]) else None
            d.n = len(f["xyz"])
            d.M = M.ctypes.data if M is not None else None
            d.sensor = C.addressof(f["sensor"].c)
            d.params = C.addressof(f["params"])
            d.key = f["key"]
            d.seed = f["seed"].data_ptr() if f.get("seed") is not None else None
            d.range = f["range"].data_ptr() if f.get("range") is not None else None
            d.out = f["out"].data_ptr()
            descs.append(d)
            self._keep += [f["sensor"], f["params"]]
        self.frames = frames
        self.net = net
        opts = pc_batch_opts(1 if persistent else 0, 1 if graph else 0, blocks_per_cu, 1 if records else 0,
                             net.data_ptr() if net is not None else None, lanes_max)
        ws = pc_batch_workspace_size(descs, opts)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=frames[0]["xyz"].device)
        self.h = pc_batch_create(ctx.h, descs, opts, self.ws, ws)

    def run(self, stream=None):
        pc_batch_run(self.h, stream)

    def profile(self, stream=None):
        return pc_batch_profile(self.h, stream)

    def info(self):
        return pc_batch_info(self.h)

    def close(self):
        if self.h is not None:
            pc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

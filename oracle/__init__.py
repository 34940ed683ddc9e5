"""CPU oracle of the spatio-temporal range-image encoder -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C, FP64
fits, FP32 exactly where the method turns floating point into an integer
decision) with ctypes and numpy.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

CLS_EMPTY, CLS_UNFIT, CLS_SPATIAL, CLS_TEMPORAL = 0, 1, 2, 3
EMPTY, FEW, DEGENERATE, FAILED, REJECTED, ACCEPTED = range(6)


def build() -> str:
    """Compile the oracle with gcc (no fast-math, no contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", "-o", _SO, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.orc_huffman_bits.restype = C.c_uint64
        L.orc_encode_sequences.restype = C.c_uint64
        L.orc_tls.restype = C.c_int
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.restype = None
        L.orc_pack.restype = C.c_uint64
        L.orc_unpack.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _Sensor(C.Structure):
    _fields_ = [("H", C.c_int), ("W", C.c_int)] + [(n, C.c_void_p) for n in
                                                   ("cut", "ebx", "eby", "ce", "se", "ca", "sa")]


class _Params(C.Structure):
    _fields_ = [("eps", C.c_float), ("th", C.c_int), ("tw", C.c_int), ("max_iter", C.c_int),
                ("min_pts", C.c_int), ("rho", C.c_float)]


_FRAME_FIELDS = [
    ("own_status", np.int8, 1), ("own_iters", np.int8, 1), ("own_axis", np.int8, 1),
    ("own_abc", np.float32, 3), ("own_mask", np.uint64, 1),
    ("t_status", np.int8, 1), ("t_iters", np.int8, 1), ("t_c", np.float32, 1), ("t_mask", np.uint64, 1),
    ("cls", np.int8, 1), ("mask", np.uint64, 1), ("run_of", np.int32, 1),
]
_SRUN = [("srun_row", np.int32, 1), ("srun_s", np.int32, 1), ("srun_len", np.int32, 1),
         ("srun_axis", np.int8, 1), ("srun_abc", np.float32, 3)]
_PRUN = [("prun_row", np.int32, 1), ("prun_s", np.int32, 1), ("prun_len", np.int32, 1),
         ("prun_krun", np.int32, 1), ("prun_c", np.float32, 1)]


class _Frame(C.Structure):
    _fields_ = ([("TR", C.c_int), ("TC", C.c_int)]
                + [(n, C.c_void_p) for n, _, _ in _FRAME_FIELDS]
                + [("n_sruns", C.c_int32), ("n_pruns", C.c_int32)]
                + [(n, C.c_void_p) for n, _, _ in _SRUN]
                + [(n, C.c_void_p) for n, _, _ in _PRUN]
                + [("occ", C.c_void_p), ("n_res", C.c_int64), ("codes", C.c_void_p), ("hist", C.c_void_p),
                   ("stream_bytes", C.c_uint64 * 4), ("coded_bits", C.c_uint64 * 4),
                   ("size_bytes", C.c_uint64), ("range_error", C.c_int32), ("seeded", C.c_void_p),
                   ("sbuf", C.c_void_p * 4), ("scap", C.c_uint64 * 4),
                   ("margin_abs", C.c_void_p), ("margin_rel", C.c_void_p),
                   ("margin_cond", C.c_void_p)])


@dataclass
class Params:
    eps: float = 0.02
    th: int = 4
    tw: int = 4
    max_iter: int = 5
    min_pts: int = 4
    rho: float = 0.5

    def c(self):
        return _Params(self.eps, self.th, self.tw, self.max_iter, self.min_pts, self.rho)


class Tables:
    """Sensor tables computed by the oracle (FP64 trigonometry, rounded once)."""

    def __init__(self, H: int, W: int, elev: np.ndarray, az0: float):
        self.H, self.W = H, W
        self.elev = np.ascontiguousarray(elev, dtype=np.float32)
        self.az0 = np.float32(az0)
        self.cut = np.zeros(H + 1, np.float32)
        self.ebx, self.eby = np.zeros(W, np.float32), np.zeros(W, np.float32)
        self.ce, self.se = np.zeros(H, np.float32), np.zeros(H, np.float32)
        self.ca, self.sa = np.zeros(W, np.float32), np.zeros(W, np.float32)
        lib().orc_tables(C.c_int(H), C.c_int(W), _p(self.elev), C.c_float(self.az0), _p(self.cut),
                         _p(self.ebx), _p(self.eby), _p(self.ce), _p(self.se), _p(self.ca), _p(self.sa))
        self.s = _Sensor(H, W, *(_p(a).value for a in
                                 (self.cut, self.ebx, self.eby, self.ce, self.se, self.ca, self.sa)))

    @classmethod
    def of(cls, sensor):
        return cls(sensor.H, sensor.W, sensor.elevations(), sensor.az0)

    def directions(self) -> np.ndarray:
        """FP32 pixel-centre directions (H, W, 3), one rounding per product."""
        d = np.empty((self.H, self.W, 3), np.float32)
        d[..., 0] = self.ce[:, None] * self.ca[None, :]
        d[..., 1] = self.ce[:, None] * self.sa[None, :]
        d[..., 2] = self.se[:, None]
        return d


def project(xyz: np.ndarray, tables: Tables, M: np.ndarray | None = None):
    """Range image (H, W) FP32, source index (H, W) int32 (-1 empty), stats[5]."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    rng = np.zeros((tables.H, tables.W), np.float32)
    idx = np.zeros((tables.H, tables.W), np.int32)
    st = np.zeros(5, np.int64)
    Mp = None
    if M is not None:
        Mp = np.ascontiguousarray(M, dtype=np.float32).reshape(16)
    lib().orc_project(_p(xyz), C.c_int64(len(xyz)), _p(Mp), C.byref(tables.s), _p(rng), _p(idx), _p(st))
    return rng, idx, st


def tls(points: np.ndarray):
    """Total-least-squares plane of FP64 points: (unit normal, c, eigenvalues, degenerate)."""
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    n = np.zeros(3)
    c = C.c_double()
    ev = np.zeros(3)
    deg = lib().orc_tls(C.c_int(len(p)), _p(p), _p(n), C.byref(c), _p(ev))
    return n, c.value, ev, bool(deg)


class Frame:
    """Encoder output of one frame (numpy views over the oracle's arrays)."""

    def __init__(self, H: int, W: int, prm: Params):
        self.H, self.W = H, W
        self.TR = -(-H // prm.th)
        self.TC = -(-W // prm.tw)
        T = self.TR * self.TC
        self.arrays = {}
        for n, dt, k in _FRAME_FIELDS + _SRUN + _PRUN:
            self.arrays[n] = np.zeros(T * k, dt)
        self.arrays["occ"] = np.zeros((H * W + 7) // 8, np.uint8)
        self.arrays["codes"] = np.zeros(H * W, np.uint16)
        self.arrays["hist"] = np.zeros(4 * 256, np.uint32)
        self.arrays["seeded"] = np.zeros(T, np.int8)
        self.arrays["margin_abs"] = np.full(T, np.inf, np.float32)
        self.arrays["margin_rel"] = np.full(T, np.inf, np.float32)
        self.arrays["margin_cond"] = np.full(T, np.inf, np.float32)
        kw = {n: _p(a).value for n, a in self.arrays.items()}
        self.c = _Frame(TR=self.TR, TC=self.TC, **kw)
        # captured stream bytes (OCC, RUN, MASK, RES), capacities from the
        # stream formats: a row's runs cover at most TC tiles, at most 23
        # bytes each, plus two varint counts
        caps = [(H * W + 7) // 8, self.TR * (10 + 23 * self.TC), 8 * T, 2 * H * W]
        self.sbufs = [np.zeros(c, np.uint8) for c in caps]
        for q in range(4):
            self.c.sbuf[q] = _p(self.sbufs[q]).value
            self.c.scap[q] = caps[q]

    def __getattr__(self, name):
        arrays = self.__dict__.get("arrays")
        if arrays is not None and name in arrays:
            a = arrays[name]
            if name in ("srun_row", "srun_s", "srun_len", "srun_axis"):
                return a[: self.c.n_sruns]
            if name == "srun_abc":
                return a[: 3 * self.c.n_sruns].reshape(-1, 3)
            if name.startswith("prun_"):
                return a[: self.c.n_pruns]
            if name == "own_abc":
                return a.reshape(-1, 3)
            if name == "codes":
                return a[: self.c.n_res]
            if name == "hist":
                return a.reshape(4, 256)
            return a
        raise AttributeError(name)

    @property
    def n_res(self):
        return self.c.n_res

    @property
    def size_bytes(self):
        return int(self.c.size_bytes)

    @property
    def stream_bytes(self):
        return list(self.c.stream_bytes)

    @property
    def coded_bits(self):
        return list(self.c.coded_bits)

    @property
    def range_error(self):
        return int(self.c.range_error)

    def streams(self):
        """The serialized OCC, RUN, MASK and RES bytes, in emission order."""
        return [self.sbufs[q][: int(self.c.stream_bytes[q])].copy() for q in range(4)]


def encode_key(range_img: np.ndarray, tables: Tables, prm: Params, seed: np.ndarray | None = None) -> Frame:
    """Key-frame encoding; ``seed`` (T x 4 FP32: normal, planarity logit) turns
    on the seeded fit with fallback."""
    r = np.ascontiguousarray(range_img, dtype=np.float32)
    f = Frame(tables.H, tables.W, prm)
    pc = prm.c()
    sd = None if seed is None else np.ascontiguousarray(seed, dtype=np.float32).reshape(-1, 4)
    if sd is not None and len(sd) != f.TR * f.TC:
        raise ValueError("seed must have one row per tile")
    lib().orc_encode_key(_p(r), C.byref(tables.s), C.byref(pc), _p(sd), C.byref(f.c))
    return f


def encode_pred(key: Frame, range_img: np.ndarray, tables: Tables, prm: Params) -> Frame:
    r = np.ascontiguousarray(range_img, dtype=np.float32)
    f = Frame(tables.H, tables.W, prm)
    pc = prm.c()
    lib().orc_encode_pred(C.byref(key.c), _p(r), C.byref(tables.s), C.byref(pc), C.byref(f.c))
    return f


def decode(frame: Frame, tables: Tables, prm: Params, key: Frame | None = None) -> np.ndarray:
    out = np.zeros((tables.H, tables.W), np.float32)
    pc = prm.c()
    lib().orc_decode(C.byref(key.c) if key is not None else None, C.byref(frame.c), C.byref(tables.s),
                     C.byref(pc), _p(out))
    return out


def decode_points(frame: Frame, tables: Tables, prm: Params, key: Frame | None = None,
                  M: np.ndarray | None = None) -> np.ndarray:
    """Decoded points (H, W, 3) in FP64, zero at empty pixels.  The decoder
    reconstructs a point on its pixel-centre ray at the decoded range
    (Sec. III-C): p = r d.  With M (the 4x4 transform [R | T] that moved the
    predicted frame into the key frame, Eq. (6)) the point is taken back to
    the frame's own coordinates, R^T (p - T) (decompression reverses the
    compression steps).  Plain FP64 arithmetic on the FP32 decoded ranges
    and FP32 pixel directions."""
    r = decode(frame, tables, prm, key).astype(np.float64)
    p = r[..., None] * tables.directions().astype(np.float64)
    if M is not None:
        A = np.asarray(M, np.float64).reshape(4, 4)
        R, T = A[:3, :3], A[:3, 3]
        p = (p - T) @ R                      # row vectors: (R^T (p - T))^T = (p - T)^T R
        p[r == 0] = 0.0
    return p


def code_lengths(hist) -> np.ndarray:
    """Code lengths (uint8[256], at most 15) of one stream's byte histogram."""
    h = np.ascontiguousarray(hist, dtype=np.uint32).reshape(256)
    out = np.zeros(256, np.uint8)
    lib().orc_code_lengths(_p(h), _p(out))
    return out


def canonical_codes(lengths) -> np.ndarray:
    ln = np.ascontiguousarray(lengths, dtype=np.uint8).reshape(256)
    out = np.zeros(256, np.uint32)
    lib().orc_canonical_codes(_p(ln), _p(out))
    return out


HEADER_BYTES = 112


def pack(frame: Frame, kind: int, prm: Params, M: np.ndarray | None = None) -> bytes:
    """Entropy-coded bitstream of an encoded frame (kind 0 key, 1 predicted);
    M (4x4) is the frame's transform into the key frame (None = identity)."""
    cap = HEADER_BYTES + sum(128 + 2 * int(n) + 8 for n in frame.stream_bytes)
    out = np.zeros(cap, np.uint8)
    Mp = None if M is None else np.ascontiguousarray(M, dtype=np.float32).reshape(16)
    n = lib().orc_pack(C.byref(frame.c), C.c_int(kind), C.c_int(frame.H), C.c_int(frame.W), C.c_int(prm.th),
                       C.c_int(prm.tw), _p(Mp), _p(out), C.c_uint64(cap))
    if n == 0:
        raise ValueError("pack failed")
    return out[:n].tobytes()


def unpack(data: bytes, caps=None, with_transform: bool = False):
    """The four streams' bytes back from a bitstream (and, with
    with_transform, the 12 FP32 of its transform, rows of [R | T])."""
    buf = np.frombuffer(data, np.uint8).copy()
    if caps is None:
        caps = [8 * len(buf) + 64] * 4     # at least one bit per symbol
    arrs = [np.zeros(int(c), np.uint8) for c in caps]
    ptrs = (C.c_void_p * 4)(*[_p(a).value for a in arrs])
    capv = (C.c_uint64 * 4)(*[int(c) for c in caps])
    nb = (C.c_uint64 * 4)()
    M = np.zeros(12, np.float32)
    if lib().orc_unpack(_p(buf), C.c_uint64(len(buf)), ptrs, capv, nb, _p(M)) != 0:
        raise ValueError("malformed bitstream")
    streams = [arrs[q][: nb[q]].copy() for q in range(4)]
    return (streams, M) if with_transform else streams


def huffman_bits(hist) -> int:
    h = np.ascontiguousarray(hist, dtype=np.uint32).reshape(256)
    return int(lib().orc_huffman_bits(_p(h)))


def encode_sequences(frames, transforms, key_index: int, nseq: int, nf: int, tables: Tables,
                     prm: Params):
    """CPU baseline: encode nseq sequences of nf frames (threads over frames).
    Returns (total bytes, per-frame sizes, finite points)."""
    assert len(frames) == nseq * nf
    arrs = [np.ascontiguousarray(f, dtype=np.float32) for f in frames]
    ptrs = (C.c_void_p * len(arrs))(*[_p(a).value for a in arrs])
    counts = np.array([len(a) for a in arrs], np.int64)
    M = np.ascontiguousarray(np.asarray(transforms, dtype=np.float32).reshape(-1, 16))
    sizes = np.zeros(len(arrs), np.uint64)
    fin = C.c_int64()
    pc = prm.c()
    total = lib().orc_encode_sequences(C.c_int(nseq), C.c_int(nf), C.c_int(key_index), ptrs, _p(counts),
                                       _p(M), C.byref(tables.s), C.byref(pc), _p(sizes), C.byref(fin))
    return int(total), sizes, int(fin.value)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the frame-parallel loops (OpenMP)."""
    lib().orc_set_num_threads(C.c_int(int(n)))

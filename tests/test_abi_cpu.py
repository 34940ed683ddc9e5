"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point ``include/pc.h`` declares, lays out frame streams as
documented, and rejects bad arguments before any launch."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2008_06972_amd import pcc, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pc_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = pcc.lib()
    names = declared_entry_points()
    assert {"pc_project", "pc_fit_key", "pc_encode_pred", "pc_decode"} <= names
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in include/ but not exported"
    assert set(pcc.EXPORTED) <= names


def test_version():
    assert pcc.pc_version().startswith("pcc-gfx950")


def test_layout_sections_aligned_and_disjoint():
    S = pcc.Sensor.of(synth.SENSORS["c2"])
    for th, tw in ((4, 4), (4, 8), (4, 16), (8, 8)):
        L = pcc.pc_stream_layout(S, pcc.params(tile_h=th, tile_w=tw))
        T, TR = L.T, L.TR
        assert (L.TR, L.TC, L.T) == (64 // th, 2048 // tw, (64 // th) * (2048 // tw))
        secs = [("info", L.off_info, C.sizeof(pcc.pc_frame_info)), ("occ", L.off_occ, 64 * 2048 // 8),
                ("cls", L.off_cls, T), ("mask", L.off_mask, 8 * T), ("run_of", L.off_run_of, 4 * T),
                ("nruns", L.off_nruns, 8 * TR), ("sruns", L.off_sruns, 24 * T), ("pruns", L.off_pruns, 16 * T),
                ("nres", L.off_nres, 4 * TR), ("res", L.off_res, 2 * 64 * 2048),
                ("hist", L.off_hist, 4 * TR * pcc.PC_STRIP_WORDS), ("tiles", L.off_tiles, pcc.TILE_DTYPE.itemsize * T)]
        end = 0
        for name, off, n in secs:
            assert off % 256 == 0, name
            assert off >= end, name
            end = off + n
        assert L.bytes >= end


def test_struct_sizes_match_header():
    assert C.sizeof(pcc.pc_frame_info) == 4 * 4 + 8 * 2 + 4 * 4 + 4 * 4 + 8 * 9 + 4 * 12 + 4 * 4
    assert pcc.RUN_DTYPE.itemsize == 24 and pcc.PRUN_DTYPE.itemsize == 16
    assert pcc.TILE_DTYPE.itemsize == 40


def _err(fn):
    with pytest.raises(pcc.PcError) as e:
        fn()
    return e.value.status


def test_argument_errors_before_launch():
    s = synth.SENSORS["c1"]
    S = pcc.Sensor.of(s)
    assert _err(lambda: pcc.pc_stream_layout(S, pcc.params(eps=0.0))) == pcc.PC_ERR_ARG
    assert _err(lambda: pcc.pc_stream_layout(S, pcc.params(eps=float("nan")))) == pcc.PC_ERR_ARG
    assert _err(lambda: pcc.pc_stream_layout(S, pcc.params(tile_h=3, tile_w=4))) == pcc.PC_ERR_UNSUPPORTED
    assert _err(lambda: pcc.pc_stream_layout(S, pcc.params(tile_h=16, tile_w=8))) == pcc.PC_ERR_ARG
    assert _err(lambda: pcc.pc_stream_layout(S, pcc.params(max_iter=0))) == pcc.PC_ERR_ARG
    assert _err(lambda: pcc.pc_stream_layout(S, pcc.params(min_pts=2))) == pcc.PC_ERR_ARG
    assert _err(lambda: pcc.pc_stream_layout(S, pcc.params(min_inlier_frac=0.0))) == pcc.PC_ERR_ARG
    bad_w = pcc.Sensor(16, 500, s.elevations(), s.az0)
    assert _err(lambda: pcc.pc_stream_layout(bad_w, pcc.params())) == pcc.PC_ERR_UNSUPPORTED
    asc = pcc.Sensor(16, 512, s.elevations()[::-1].copy(), s.az0)
    assert _err(lambda: pcc.pc_stream_layout(asc, pcc.params())) == pcc.PC_ERR_ARG
    nan_e = s.elevations().copy()
    nan_e[3] = np.nan
    assert _err(lambda: pcc.pc_stream_layout(pcc.Sensor(16, 512, nan_e, s.az0), pcc.params())) == pcc.PC_ERR_ARG
    odd_h = pcc.Sensor(18, 512, np.linspace(0.2, -0.2, 18).astype(np.float32), 0.0)
    assert _err(lambda: pcc.pc_stream_layout(odd_h, pcc.params(tile_h=4))) == pcc.PC_ERR_UNSUPPORTED
    assert pcc.pc_workspace_size(S) == 8 * 16 * 512


def test_context_needs_a_device():
    if os.environ.get("HIP_VISIBLE_DEVICES", None) == "" or not _has_gpu():
        assert _err(lambda: pcc.pc_ctx_create(0, None, 0)) == pcc.PC_ERR_DEVICE


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False

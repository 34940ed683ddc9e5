"""The benchmark's workload at full size, in the launch configuration it is
timed in: 96 sequences x 10 frames of the 64x2048 sensor (tiles 4x8,
eps = 2 cm, key frame 5, about 116 M points) encoded by one batch graph of
persistent kernels, without and with the seed network, replayed twice.

The timed configuration writes no per-tile fit records; a second plan with
records gives streams equal to it outside the record section, and its
records feed the fit-level comparisons.  Against the oracle (its own
projection and encodes of the same points): sampled key and predicted
frames of the plain form have sizes within 0.5%, identical residual codes
wherever both sides code a pixel, every difference of class, mask, run or
temporal result explained by a decision within rounding of eps (at most
0.2% of the tiles), by a key-frame difference in the key run a predicted
tile reuses, or downstream of either in the same run (classes 99.8% equal
on key frames, 99% on predicted frames, temporal results 99.8%), c' within
1e-4 where both sides keep the same pixels, and the whole batch's size is
within 0.5% of the oracle's
encode of all 960 frames.  Both forms hold the eps bound on every decoded
pixel of the sampled frames, and the learned form's ratio is within 2% of
the plain form's.  The second replay's streams equal the first's."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
from paper_2008_06972_amd import pcc, synth  # noqa: E402
from gpu_common import (compare_frame, explain_differences, residual_codes_agree,  # noqa: E402
                        temporal_offsets_agree)

DEV = torch.device("cuda:0")
NSEQ, NF, KEY = 96, bench.N_FRAMES, bench.KEY_INDEX
SAMPLE = [(0, KEY), (0, 0), (0, 9), (37, KEY), (37, 3), (95, KEY), (95, 6)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def workload():
    say("generating", NSEQ, "sequences")
    frames, transforms = bench.make_workload(NSEQ, 16)
    return frames, transforms


def _run(ctx, S, prm, frames, transforms, net, records=False):
    xyz = [torch.from_numpy(f).to(DEV) for f in frames]
    outs = [pcc.FrameStream(S, prm, DEV) for _ in frames]

    def key_of(i):
        return (i // NF) * NF + KEY

    fr = [dict(xyz=xyz[i], M=None if i == key_of(i) else transforms[i], sensor=S, params=prm, key=key_of(i),
               out=outs[i]) for i in range(len(frames))]
    batch = pcc.Batch(ctx, fr, persistent=True, graph=True, net=net, records=records)
    batch.run()
    torch.cuda.synchronize()
    first = [o.buf.clone() for o in outs]
    batch.run()
    torch.cuda.synchronize()
    for i, (a, o) in enumerate(zip(first, outs)):
        assert torch.equal(a, o.buf), f"replay changed frame {i}"
    batch.close()
    return outs


def test_headline_workload_against_oracle(workload):
    frames, transforms = workload
    s = synth.SENSORS["c2"]
    S = pcc.Sensor.of(s)
    prm = pcc.params(eps=bench.EPS, tile_h=4, tile_w=8, max_iter=5, min_pts=4, min_inlier_frac=0.5)
    ctx = pcc.Context([S])
    tb = oracle.Tables.of(s)
    oprm = oracle.Params(eps=bench.EPS, th=4, tw=8)
    try:
        timed = _run(ctx, S, prm, frames, transforms, None)
        plain = _run(ctx, S, prm, frames, transforms, None, records=True)
        off = plain[0].L.off_tiles
        for i, (a, b) in enumerate(zip(timed, plain)):
            assert torch.equal(a.buf[:off], b.buf[:off]), f"frame {i}: records change the stream"
        del timed
        w = np.fromfile(os.path.join(ROOT, "paper_2008_06972_amd", "weights", "seednet_c2.f32"), dtype="<f4")
        learned = _run(ctx, S, prm, frames, transforms, torch.from_numpy(w).to(DEV))
        pts = sum(int(np.isfinite(f).all(axis=1).sum()) for f in frames)
        size_p = sum(int(o.info().size_bytes) for o in plain)
        size_l = sum(int(o.info().size_bytes) for o in learned)
        say("points", pts, "ratio plain", 12.0 * pts / size_p, "learned", 12.0 * pts / size_l)
        assert abs(size_l - size_p) <= 0.02 * size_p
        # the oracle on all 960 frames
        total_o, _, _ = oracle.encode_sequences(frames, transforms, KEY, NSEQ, NF, tb, oprm)
        say("batch size gpu", size_p, "oracle", total_o)
        assert abs(size_p - total_o) <= 0.005 * total_o
        # sampled frames
        okeys = {}
        for q, j in SAMPLE:
            i = q * NF + j
            M = None if j == KEY else transforms[i]
            r, _, _ = oracle.project(frames[i], tb, M)
            if q not in okeys:
                rk, _, _ = oracle.project(frames[q * NF + KEY], tb, None)
                okeys[q] = oracle.encode_key(rk, tb, oprm)
            o = okeys[q] if j == KEY else oracle.encode_pred(okeys[q], r, tb, oprm)
            g = plain[i].host()
            gk = plain[q * NF + KEY].host()
            st = compare_frame(oracle, g, o, r)
            ok, nboth, ndiff = residual_codes_agree(g, o, r, 4, 8)
            ex = explain_differences(g, o, r, 4, 8, tb, temporal=j != KEY, keys=(gk, okeys[q]))
            t_agree = float(np.mean(g["tiles"]["t_status"] == o.t_status))
            n_c, worst_c = temporal_offsets_agree(g, o, okeys[q], gk) if j != KEY else (0, 0.0)
            say((q, j), {k: st[k] for k in ("cls_agree", "size_gpu", "size_orc", "size_rel")}, "codes", ok, nboth, ex,
                "t_status agree", t_agree, "c'", n_c, worst_c)
            assert ok and st["valid_agree"]
            assert st["size_rel"] <= 0.005, st
            assert ex["cls_agree"] >= (0.998 if j == KEY else 0.99) and t_agree >= 0.998, ex
            assert ex["unexplained"] == 0 and ex["near_eps"] <= 0.002 * len(o.cls), ex
            assert worst_c <= 1e-4
            assert st["worst_normal_rad"] <= 1e-4 and st["worst_offset_rel"] <= 1e-4, st
            for outs in (plain, learned):
                dec = torch.empty(s.H, s.W, dtype=torch.float32, device=DEV)
                key_fs = None if j == KEY else outs[q * NF + KEY]
                pcc.pc_decode(ctx.h, key_fs, outs[i], S, prm, dec)
                torch.cuda.synchronize()
                d = dec.cpu().numpy().astype(np.float64)
                v = r > 0
                assert np.all(d[~v] == 0) and np.abs(d[v] - r[v]).max() <= bench.EPS
    finally:
        ctx.close()

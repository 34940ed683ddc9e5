"""The next-step measurements on the GPU against the oracle.

* IMU front end (Sec. III-D, Eq. (4)-(6)): for each predicted frame of a
  64x2048 sequence, 100 Hz samples that carry the true motion (velocity at
  the first sample, yaw rate) plus accelerometer and gyro noise, a gyro bias
  and an error in the first-sample velocity are integrated by the library
  (pc_imu_transform) and by the oracle (oracle.imu.transform): the two
  transforms agree to one FP32 ulp, the GPU batch encodes with the
  library's and the oracle with its own, and the projections (the same
  pixels occupied, ranges equal up to the rounding the last ulp of the
  transform moves), sizes (0.5 %) and temporal shares (0.5 % of the pixels)
  agree; every decoded pixel is
  within eps; and the temporal share with these transforms stays within 15 %
  of the share with the exact ones, on both sides (the offset c' of a reused
  plane absorbs the translation error).
* Frames per key frame (Sec. V-C): sequences of N = 1, 3 and 5 frames
  (key frame in the middle) encoded by the batch: per N, the bytes within
  0.5 % of the oracle's and the shares of temporally, spatially and
  residual-coded pixels within 0.5 % of the pixels of the oracle's.
* Denoising (Sec. III-C): key frames of noisy scenes, decoded, against the
  same scenes rendered without noise: the mean absolute errors of
  plane-coded and of residual pixels within 1 % of the oracle's own encode
  and decode, and plane-coded pixels closer to the noiseless surface than
  the input."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from paper_2008_06972_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from oracle import imu  # noqa: E402
from paper_2008_06972_amd import pcc, sweeps  # noqa: E402

DEV = torch.device("cuda:0")
EPS = 0.02


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _popcount(a):
    return np.unpackbits(np.asarray(a, np.uint64).view(np.uint8).reshape(-1, 8), axis=1).sum(1).astype(np.int64)


def _oracle_shares(frames_o):
    """(temporal, spatial, residual, valid) pixels of oracle frames."""
    t = s = r = v = 0
    for o, rng in frames_o:
        pop = _popcount(o.mask)
        t += int(pop[o.cls == 3].sum())
        s += int(pop[o.cls == 2].sum())
        r += int(o.c.n_res)
        v += int((rng > 0).sum())
    return t, s, r, v


def _gpu_shares(outs):
    t = s = r = v = 0
    for o in outs:
        a, b, c, d = sweeps._classes(o)
        t, s, r, v = t + a, s + b, r + c, v + d
    return t, s, r, v


def _batch(ctx, S, prm, frames, transforms, n):
    xyz = [torch.from_numpy(f).to(DEV) for f in frames]
    outs = [pcc.FrameStream(S, prm, DEV) for _ in frames]
    rngs = [torch.empty(S.H, S.W, dtype=torch.float32, device=DEV) for _ in frames]

    def key_of(i):
        return (i // n) * n + n // 2
    fr = [dict(xyz=xyz[i], M=None if i == key_of(i) else transforms[i], sensor=S, params=prm, key=key_of(i),
               out=outs[i], range=rngs[i]) for i in range(len(frames))]
    b = pcc.Batch(ctx, fr, persistent=True, graph=True)
    b.run()
    torch.cuda.synchronize()
    b.close()
    return outs, rngs, key_of


def _oracle_encode(frames, transforms, n, tb, oprm):
    out = []
    for q in range(0, len(frames), n):
        k = q + n // 2
        rk, _, _ = oracle.project(frames[k], tb, None)
        ok = oracle.encode_key(rk, tb, oprm)
        for i in range(q, q + n):
            if i == k:
                out.append((ok, rk))
            else:
                r, _, _ = oracle.project(frames[i], tb, transforms[i])
                out.append((oracle.encode_pred(ok, r, tb, oprm), r))
    return out


def _imu_samples(M_true, nsamp, rng, bias):
    """Samples whose integration is M_true (frame into key frame) up to the
    noise: velocity T / (n dt) at the first sample, yaw rate giving the
    rotation (Eq. (5) turns by -alpha in the x-y plane)."""
    dt = 1.0 / sweeps.IMU_RATE
    T = M_true[:3, 3].astype(np.float64)
    theta = math.atan2(float(M_true[1, 0]), float(M_true[0, 0]))
    v0 = T / (nsamp * dt) + rng.normal(0, 0.1, 3) * np.array([1.0, 1.0, 0.2])
    acc = rng.normal(0, 0.05, (nsamp, 3))
    gyro = rng.normal(0, 0.002, (nsamp, 3)) + bias + np.array([0.0, 0.0, -theta / (nsamp * dt)])
    return acc.astype(np.float32), gyro.astype(np.float32), dt, v0.astype(np.float32)


def test_imu_front_end_against_oracle():
    s = synth.SENSORS["c2"]
    S = pcc.Sensor.of(s)
    ctx = pcc.Context([S])
    tb = oracle.Tables.of(s)
    prm = pcc.params(eps=EPS, tile_h=4, tile_w=8)
    oprm = oracle.Params(eps=EPS, th=4, tw=8)
    n, K = 10, 5
    try:
        seq = synth.make_sequence(s, "c2", 7300, n_frames=n, key_index=K, moving=5, shuffle=True)
        bias = np.random.default_rng(1).normal(0, 0.002, 3)
        M_lib = seq.transforms.copy()
        M_orc = seq.transforms.copy()
        worst_ulp = 0
        for i in range(n):
            if i == K:
                continue
            ns = int(round(abs(i - K) * sweeps.FRAME_DT * sweeps.IMU_RATE))
            acc, gyro, dt, v0 = _imu_samples(seq.transforms[i], ns, np.random.default_rng([7300, i]), bias)
            M_lib[i], _ = pcc.pc_imu_transform(acc, gyro, dt, v0)
            Mo, _ = imu.transform(acc, gyro, dt, v0)
            M_orc[i] = Mo.astype(np.float32)
            ulp = np.abs(M_lib[i].view(np.int32).astype(np.int64) - M_orc[i].view(np.int32).astype(np.int64))
            worst_ulp = max(worst_ulp, int(ulp.max()))
            err_t = float(np.linalg.norm(M_orc[i][:3, 3] - seq.transforms[i][:3, 3]))
            say(f"frame {i}: {ns} samples, translation error {err_t:.3f} m")
        assert worst_ulp <= 1, worst_ulp
        outs, rngs, key_of = _batch(ctx, S, prm, seq.frames, M_lib, n)
        frames_o = _oracle_encode(seq.frames, M_orc, n, tb, oprm)
        # a transform one ulp apart moves each point by about 1e-8 m, which
        # flips the last bit of some ranges; a point that lands in another
        # pixel, or a pixel another point wins, shows as an occupancy or a
        # larger range difference
        ulps = moved = 0
        for r, (_, ro) in zip(rngs, frames_o):
            rg = r.cpu().numpy().astype(np.float64)
            ro = ro.astype(np.float64)
            ulps += int(np.sum(rg != ro))
            moved += int(np.sum(((rg > 0) != (ro > 0)) | (np.abs(rg - ro) > 1e-6 * np.maximum(ro, 1.0))))
        total_px = n * s.H * s.W
        say(f"pixels of the two projections: {ulps} differ in range, {moved} by more than rounding")
        assert moved <= 1e-4 * total_px
        for i, (o, (fo, ro)) in enumerate(zip(outs, frames_o)):
            g, f = int(o.info().size_bytes), int(fo.size_bytes)
            assert abs(g - f) <= 0.005 * f, (i, g, f)
        tg, sg, rg, vg = _gpu_shares(outs)
        to, so, ro_, vo = _oracle_shares(frames_o)
        say("temporal share gpu", tg / vg, "oracle", to / vo)
        assert abs(tg / vg - to / vo) <= 0.005 and abs(sg / vg - so / vo) <= 0.005
        # every pixel decoded within eps of the range image it was encoded from
        ws = pcc.pc_decode_batch_workspace_size(n)
        work = torch.empty(ws, dtype=torch.uint8, device=DEV)
        dec = [torch.empty(s.H, s.W, dtype=torch.float32, device=DEV) for _ in range(n)]
        pcc.pc_decode_batch(ctx.h, [None if i == K else outs[K] for i in range(n)], outs, S, prm, dec, work, ws)
        torch.cuda.synchronize()
        for d, r in zip(dec, rngs):
            v = r > 0
            assert bool((d[~v] == 0).all()) and float((d[v].double() - r[v].double()).abs().max()) <= EPS
        # robustness: the exact transforms on both sides
        outs_x, _, _ = _batch(ctx, S, prm, seq.frames, seq.transforms, n)
        tx, _, _, vx = _gpu_shares(outs_x)
        tox, _, _, vox = _oracle_shares(_oracle_encode(seq.frames, seq.transforms, n, tb, oprm))
        say("temporal share with exact transforms gpu", tx / vx, "oracle", tox / vox)
        assert tg / vg >= 0.85 * tx / vx and to / vo >= 0.85 * tox / vox
    finally:
        ctx.close()


def test_frames_per_key_sweep_against_oracle():
    s = synth.SENSORS["c2"]
    S = pcc.Sensor.of(s)
    ctx = pcc.Context([S])
    tb = oracle.Tables.of(s)
    prm = pcc.params(eps=EPS, tile_h=4, tile_w=8)
    oprm = oracle.Params(eps=EPS, th=4, tw=8)
    try:
        for n in (1, 3, 5):
            frames, transforms = sweeps._workload(2, n, 7400, corridor_frames=5)
            outs, _, _ = _batch(ctx, S, prm, frames, transforms, n)
            frames_o = _oracle_encode(frames, transforms, n, tb, oprm)
            g = sum(int(o.info().size_bytes) for o in outs)
            f = sum(int(fo.size_bytes) for fo, _ in frames_o)
            tg, sg, rg, vg = _gpu_shares(outs)
            to, so, ro, vo = _oracle_shares(frames_o)
            say(f"N={n}: bytes gpu {g} oracle {f}; shares gpu {tg / vg:.4f} {sg / vg:.4f} {rg / vg:.4f} "
                f"oracle {to / vo:.4f} {so / vo:.4f} {ro / vo:.4f}")
            assert vg == vo
            assert abs(g - f) <= 0.005 * f
            for a, b in ((tg, to), (sg, so), (rg, ro)):
                assert abs(a - b) <= 0.005 * vo, (n, a, b)
            if n == 1:
                assert tg == 0 and to == 0
    finally:
        ctx.close()


def test_denoising_against_oracle():
    s = synth.SENSORS["c2"]
    S = pcc.Sensor.of(s)
    ctx = pcc.Context([S])
    tb = oracle.Tables.of(s)
    prm = pcc.params(eps=EPS, tile_h=4, tile_w=8)
    oprm = oracle.Params(eps=EPS, th=4, tw=8)
    acc = {side: {k: [0.0, 0.0, 0] for k in ("plane", "residual")} for side in ("gpu", "oracle")}
    try:
        for seed in (7500, 7501):
            rng = synth._rng(seed, 0)
            scene = synth.make_scene("c2", rng)
            clean = dataclasses.replace(scene, sigma=0.0)
            pts_n, _, _ = synth.render(s, scene, np.eye(3), np.zeros(3), 0, synth._rng(seed, 1))
            pts_0, _, _ = synth.render(s, clean, np.eye(3), np.zeros(3), 0, synth._rng(seed, 1))
            rn, _, _ = oracle.project(pts_n, tb)
            r0, _, _ = oracle.project(pts_0, tb)
            # GPU: project, encode, decode
            img = torch.empty(s.H, s.W, dtype=torch.float32, device=DEV)
            pcc.pc_project(ctx.h, torch.from_numpy(pts_n).to(DEV), len(pts_n), None, S, img)
            fs = pcc.FrameStream(S, prm, DEV)
            pcc.pc_fit_key(ctx.h, img, S, prm, None, fs)
            dec = torch.empty_like(img)
            pcc.pc_decode(ctx.h, None, fs, S, prm, dec)
            torch.cuda.synchronize()
            assert np.array_equal(img.cpu().numpy(), rn)
            o = oracle.encode_key(rn, tb, oprm)
            sides = {"gpu": (fs.host(), dec.cpu().numpy()), "oracle": ({"cls": o.cls, "mask": o.mask},
                                                                       oracle.decode(o, tb, oprm))}
            both = (rn > 0) & (r0 > 0)
            for side, (h, rd) in sides.items():
                covered = np.zeros((s.H, s.W), bool)
                TC = s.W // 8
                for t in np.nonzero(np.isin(h["cls"], (2, 3)))[0]:
                    tr, tc = divmod(int(t), TC)
                    m = np.array([(int(h["mask"][t]) >> j) & 1 for j in range(32)], bool).reshape(4, 8)
                    covered[tr * 4:(tr + 1) * 4, tc * 8:(tc + 1) * 8] = m
                for name, sel in (("plane", both & covered), ("residual", both & ~covered)):
                    acc[side][name][0] += float(np.abs(rn[sel].astype(np.float64) - r0[sel]).sum())
                    acc[side][name][1] += float(np.abs(rd[sel].astype(np.float64) - r0[sel]).sum())
                    acc[side][name][2] += int(sel.sum())
        for name in ("plane", "residual"):
            ig, dg, ng = acc["gpu"][name]
            io, do, no = acc["oracle"][name]
            say(f"{name}: gpu {ng} px input {ig / ng * 1e3:.2f} mm decoded {dg / ng * 1e3:.2f} mm; "
                f"oracle {no} px input {io / no * 1e3:.2f} mm decoded {do / no * 1e3:.2f} mm")
            assert abs(ng - no) <= 0.01 * no
            assert abs(dg / ng - do / no) <= 0.01 * (do / no)
        ig, dg, ng = acc["gpu"]["plane"]
        io, do, no = acc["oracle"]["plane"]
        assert dg < ig and do < io
    finally:
        ctx.close()

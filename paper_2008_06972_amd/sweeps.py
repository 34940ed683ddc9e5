"""Sensitivity measurements on the GPU encoder (the analyses of Sec. IV).

    python -m paper_2008_06972_amd.sweeps frames  [--frames 960] [--ns 1,3,5,9,19]
    python -m paper_2008_06972_amd.sweeps denoise [--seqs 4]
    python -m paper_2008_06972_amd.sweeps imu     [--scales 0,0.5,1,2,4,8] [--model pose|imu]

``frames``: for each number N of consecutive frames encoded together (key
frame in the middle), about --frames frames of the 64x2048 sensor in
sequences of N are encoded by one batch graph: frames/s, compression ratio,
and how the non-empty pixels are coded (temporal run, spatial run,
residual), the analogue of the paper's sensitivity and encoding-type
figures.

``denoise``: each frame is also rendered without range noise (same rays,
same dropout), and the decoded range's error against that noiseless truth
is compared with the input's error against it, split by how the pixel was
coded: the paper's observation that plane fitting smooths sensor noise.

``imu``: pose errors of the kind IMU integration leaves are injected into
the transforms, either directly (translation and yaw, scaled) or by
integrating IMU sensor noise with the library's front end
(``pc_imu_transform``, Eq. (4)-(5)); the sweep reports the
compression ratio, the temporal share, and the share of temporally coded
pixels whose run needed its offset moved by more than eps, 2 eps from the
key plane's: pixels that the fixed-normal offset relaxation (Sec. III-D)
keeps temporal and that a plane reused unchanged would lose.

Every line printed is one JSON object.  Inputs are the seeded generator of
``synth`` (no dataset).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

SENSOR = "c2"
EPS = 0.02


def _classes(fs):
    """Pixels per coding class of one encoded frame stream buffer:
    (temporal, spatial, residual, valid), from its tile classes and masks."""
    L = fs.L
    cls = fs._sec(L.off_cls, L.T)
    mask = fs._sec(L.off_mask, 8 * L.T).view(np.uint64)
    info = fs.info()
    pop = _popcount64(mask)
    temporal = int(pop[cls == 3].sum())
    spatial = int(pop[cls == 2].sum())
    return temporal, spatial, int(info.n_res), int(info.n_valid)


def _popcount64(a: np.ndarray) -> np.ndarray:
    a = a.astype(np.uint64)
    b = a.view(np.uint8).reshape(-1, 8)
    return np.unpackbits(b, axis=1).sum(1).astype(np.int64)


def _gen(args):
    from paper_2008_06972_amd import synth
    seed, n, scale, nc = args
    seq = synth.make_sequence(synth.SENSORS[SENSOR], SENSOR, seed, n_frames=n, key_index=n // 2, moving=5,
                              shuffle=True, imu_noise=scale, corridor_frames=nc)
    return seq.frames, seq.transforms


def _workload(nseq, n, seed0, scale=0.0, procs=16, corridor_frames=None):
    import multiprocessing as mp
    jobs = [(seed0 + q, n, scale, corridor_frames) for q in range(nseq)]
    with mp.get_context("fork").Pool(procs) as pool:
        out = pool.map(_gen, jobs, chunksize=1)
    frames = [f for fr, _ in out for f in fr]
    transforms = np.concatenate([t for _, t in out])
    return frames, transforms


def _encode_batch(pcc, torch, ctx, S, prm, frames, transforms, n, steps, warmup):
    """One batch graph over sequences of n frames; returns (ms per pass, outs)."""
    dev = torch.device("cuda:0")
    nfr = len(frames)
    xyz = [torch.from_numpy(f).to(dev) for f in frames]
    outs = [pcc.FrameStream(S, prm, dev) for _ in range(nfr)]

    def key_of(i):
        return (i // n) * n + n // 2

    fr = [dict(xyz=xyz[i], M=None if i == key_of(i) else transforms[i], sensor=S, params=prm, key=key_of(i),
               out=outs[i]) for i in range(nfr)]
    batch = pcc.Batch(ctx, fr, persistent=True, graph=True)
    for _ in range(warmup):
        batch.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        batch.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    batch.close()
    return ms, outs, key_of


def _decode_batch(pcc, torch, ctx, S, prm, outs, key_of, s_hw, reps=5):
    """ms for one pc_decode_batch call over every frame (table upload included)."""
    n = len(outs)
    dec = torch.empty((n,) + tuple(s_hw), dtype=torch.float32, device="cuda:0")
    keys = [None if i == key_of(i) else outs[key_of(i)] for i in range(n)]
    ws = pcc.pc_decode_batch_workspace_size(n)
    work = torch.empty(ws, dtype=torch.uint8, device="cuda:0")
    lst = [dec[i] for i in range(n)]
    pcc.pc_decode_batch(ctx.h, keys, outs, S, prm, lst, work, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pcc.pc_decode_batch(ctx.h, keys, outs, S, prm, lst, work, ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _summary(frames, outs):
    pts = sum(int(np.isfinite(f).all(axis=1).sum()) for f in frames)
    infos = [o.info() for o in outs]
    size = sum(int(i.size_bytes) for i in infos)
    t = s = r = v = 0
    for o in outs:
        a, b, c, d = _classes(o)
        t, s, r, v = t + a, s + b, r + c, v + d
    return dict(points=pts, bytes=size, ratio=12.0 * pts / size, temporal=t / v, spatial=s / v, residual=r / v)


def cmd_frames(a, pcc, torch):
    from paper_2008_06972_amd import synth
    S = pcc.Sensor.of(synth.SENSORS[SENSOR])
    prm = pcc.params(eps=EPS, tile_h=4, tile_w=8)
    ctx = pcc.Context([S])
    ns = [int(x) for x in a.ns.split(",")]
    for n in ns:
        nseq = max(1, round(a.frames / n))
        t0 = time.time()
        # one scene distribution for every N: the corridor of the longest track
        frames, transforms = _workload(nseq, n, a.seed0, corridor_frames=max(ns))
        gen_s = time.time() - t0
        ms, outs, key_of = _encode_batch(pcc, torch, ctx, S, prm, frames, transforms, n, a.steps, a.warmup)
        dms = _decode_batch(pcc, torch, ctx, S, prm, outs, key_of, s_hw=(synth.SENSORS[SENSOR].H,
                                                                           synth.SENSORS[SENSOR].W))
        row = dict(sweep="frames", N=n, corridor_frames=max(ns), sequences=nseq, frames=len(frames), ms_per_pass=ms,
                   frames_per_s=len(frames) / (ms / 1e3), decode_frames_per_s=len(frames) / (dms / 1e3),
                   gen_s=round(gen_s, 1))
        row.update(_summary(frames, outs))
        print(json.dumps(row), flush=True)
        del outs
        torch.cuda.empty_cache()
    ctx.close()


IMU_RATE = 100.0        # samples per second
FRAME_DT = 0.1          # seconds between frames


def imu_pose_errors(pcc, transforms, n, seed0, scale):
    """Apply to each predicted frame's exact transform the pose error that the
    IMU front end (pc_imu_transform) makes from sensor noise alone over the
    samples between the frame and its key frame: white accelerometer noise
    (0.05 s m/s^2 per sample), white gyro noise (0.002 s rad/s) plus a gyro
    bias per sequence (0.002 s rad/s per axis), and an unknown velocity at
    the first sample (0.1 s m/s per horizontal axis, a fifth of it in z)."""
    out = transforms.copy()
    for i in range(len(transforms)):
        q, j = divmod(i, n)
        k = n // 2
        if j == k or scale == 0:
            continue
        rb = np.random.default_rng([seed0 + q, 1])
        bias = rb.normal(0, 0.002 * scale, 3)
        r = np.random.default_rng([seed0 + q, 2, j])
        ns = int(round(abs(j - k) * FRAME_DT * IMU_RATE))
        acc = r.normal(0, 0.05 * scale, (ns, 3))
        gyro = r.normal(0, 0.002 * scale, (ns, 3)) + bias
        v0 = r.normal(0, 0.1 * scale, 3) * np.array([1.0, 1.0, 0.2])
        E, _ = pcc.pc_imu_transform(acc, gyro, 1.0 / IMU_RATE, v0)
        out[i] = (E.astype(np.float64) @ transforms[i].astype(np.float64)).astype(np.float32)
    return out


def cmd_imu(a, pcc, torch):
    from paper_2008_06972_amd import synth
    S = pcc.Sensor.of(synth.SENSORS[SENSOR])
    prm = pcc.params(eps=EPS, tile_h=4, tile_w=8)
    ctx = pcc.Context([S])
    n = a.n
    nseq = max(1, round(a.frames / n))
    for scale in [float(x) for x in a.scales.split(",")]:
        if a.model == "pose":
            frames, transforms = _workload(nseq, n, a.seed0, scale)
            noise = dict(sigma_translation_m=0.05 * scale, sigma_yaw_deg=0.1 * scale)
        else:
            frames, transforms = _workload(nseq, n, a.seed0, 0.0)
            transforms = imu_pose_errors(pcc, transforms, n, a.seed0, scale)
            noise = dict(acc_sigma=0.05 * scale, gyro_sigma=0.002 * scale, gyro_bias_sigma=0.002 * scale,
                         v0_sigma=0.1 * scale, imu_rate_hz=IMU_RATE)
        ms, outs, key_of = _encode_batch(pcc, torch, ctx, S, prm, frames, transforms, n, a.steps, a.warmup)
        row = dict(sweep="imu", model=a.model, scale=scale, N=n, frames=len(frames),
                   frames_per_s=len(frames) / (ms / 1e3))
        row.update(noise)
        row.update(_summary(frames, outs))
        # temporal pixels whose run moved the key plane's offset by > eps, > 2 eps
        moved = {1: 0, 2: 0}
        tpix = 0
        keys = {}
        for i, o in enumerate(outs):
            if i == key_of(i):
                continue
            h = o.host()
            if key_of(i) not in keys:
                keys[key_of(i)] = outs[key_of(i)].host()
            k = keys[key_of(i)]
            L = o.L
            pop = _popcount64(h["mask"])
            for tr in range(L.TR):
                for q in range(int(h["nruns"][L.TR + tr])):
                    R = h["pruns"][tr * L.TC + q]
                    K = k["sruns"][int(R["krun"])]
                    nrm = math.sqrt(1.0 + float(K["a"]) ** 2 + float(K["b"]) ** 2)
                    shift = abs(float(R["c"]) - float(K["c"])) / nrm
                    t0 = tr * L.TC + int(R["s"])
                    px = int(pop[t0:t0 + int(R["len"])].sum())
                    tpix += px
                    for m in moved:
                        if shift > m * EPS:
                            moved[m] += px
        row["temporal_pixels"] = tpix
        row["temporal_shift_gt_eps"] = moved[1] / max(1, tpix)
        row["temporal_shift_gt_2eps"] = moved[2] / max(1, tpix)
        print(json.dumps(row), flush=True)
        del outs
        torch.cuda.empty_cache()
    ctx.close()


def cmd_denoise(a, pcc, torch):
    import dataclasses
    from paper_2008_06972_amd import synth
    s = synth.SENSORS[SENSOR]
    S = pcc.Sensor.of(s)
    prm = pcc.params(eps=EPS, tile_h=4, tile_w=8)
    ctx = pcc.Context([S])
    dev = torch.device("cuda:0")
    acc = {k: [0.0, 0.0, 0] for k in ("plane", "residual", "all")}
    for q in range(a.seqs):
        seed = a.seed0 + q
        rng = synth._rng(seed, 0)
        scene = synth.make_scene(SENSOR, rng)
        clean = dataclasses.replace(scene, sigma=0.0)
        pts_n, rows_n, cols_n = synth.render(s, scene, np.eye(3), np.zeros(3), 0, synth._rng(seed, 1))
        pts_0, rows_0, cols_0 = synth.render(s, clean, np.eye(3), np.zeros(3), 0, synth._rng(seed, 1))
        imgs = []
        for pts in (pts_n, pts_0):
            r = torch.zeros(s.H, s.W, dtype=torch.float32, device=dev)
            pcc.pc_project(ctx.h, torch.from_numpy(pts).to(dev), len(pts), None, S, r)
            imgs.append(r)
        fs = pcc.FrameStream(S, prm, dev)
        pcc.pc_fit_key(ctx.h, imgs[0], S, prm, None, fs)
        dec = torch.empty_like(imgs[0])
        pcc.pc_decode(ctx.h, None, fs, S, prm, dec)
        torch.cuda.synchronize()
        rn, r0, rd = imgs[0].cpu().numpy(), imgs[1].cpu().numpy(), dec.cpu().numpy()
        h = fs.host()
        L = fs.L
        covered = np.zeros((s.H, s.W), bool)
        bits = np.arange(L.th * L.tw, dtype=np.uint64)
        for t in np.nonzero(np.isin(h["cls"], (2, 3)))[0]:
            tr, tc = divmod(int(t), L.TC)
            m = ((int(h["mask"][t]) >> bits.astype(np.int64)) & 1).astype(bool).reshape(L.th, L.tw)
            covered[tr * L.th:(tr + 1) * L.th, tc * L.tw:(tc + 1) * L.tw] = m
        both = (rn > 0) & (r0 > 0)
        for name, sel in (("plane", both & covered), ("residual", both & ~covered), ("all", both)):
            acc[name][0] += float(np.abs(rn[sel].astype(np.float64) - r0[sel]).sum())
            acc[name][1] += float(np.abs(rd[sel].astype(np.float64) - r0[sel]).sum())
            acc[name][2] += int(sel.sum())
    row = dict(sweep="denoise", frames=a.seqs, sigma_m=float(synth.make_scene(SENSOR, synth._rng(a.seed0, 0)).sigma),
               eps_m=EPS)
    for name, (ein, eout, n) in acc.items():
        row[name] = dict(pixels=n, input_mae_m=ein / max(1, n), decoded_mae_m=eout / max(1, n))
    print(json.dumps(row), flush=True)
    ctx.close()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    f = sub.add_parser("frames")
    f.add_argument("--frames", type=int, default=960)
    f.add_argument("--ns", default="1,3,5,9,19")
    f.add_argument("--seed0", type=int, default=8000)
    f.add_argument("--steps", type=int, default=10)
    f.add_argument("--warmup", type=int, default=2)
    d = sub.add_parser("denoise")
    d.add_argument("--seqs", type=int, default=8)
    d.add_argument("--seed0", type=int, default=8500)
    m = sub.add_parser("imu")
    m.add_argument("--frames", type=int, default=480)
    m.add_argument("--n", type=int, default=5)
    m.add_argument("--scales", default="0,0.5,1,2,4,8")
    m.add_argument("--seed0", type=int, default=8800)
    m.add_argument("--model", choices=("pose", "imu"), default="pose",
                   help="pose: perturb the transforms directly; imu: pose errors from IMU noise through pc_imu_transform")
    m.add_argument("--steps", type=int, default=5)
    m.add_argument("--warmup", type=int, default=1)
    a = ap.parse_args(argv)
    import torch
    from paper_2008_06972_amd import pcc
    if not torch.cuda.is_available():
        print("the sweeps need a GPU", file=sys.stderr)
        return 2
    pcc.lib()
    {"frames": cmd_frames, "denoise": cmd_denoise, "imu": cmd_imu}[a.cmd](a, pcc, torch)
    return 0


if __name__ == "__main__":
    sys.exit(main())

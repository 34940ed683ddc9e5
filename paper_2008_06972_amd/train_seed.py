#!/usr/bin/env python3
"""Train the plane-seed network on the GPU through the C ABI.

Labels are the plain key-frame fits of generated frames (``pc_fit_key``
without seeds): a tile with a fit attempt is labelled, planar = accepted,
normal = the stored plane's unit normal.  Each step runs ``pc_net_forward``,
``pc_net_loss``, ``pc_net_backward`` and ``pc_net_adam`` on one frame.
After training, held-out frames are encoded with and without seeds and the
seeded / fallback counts and sizes are reported.

    python -m paper_2008_06972_amd.train_seed --frames 2000 --epochs 2 \
        --out paper_2008_06972_amd/weights/seednet_c2.f32

Weights are written as PC_NET_PARAMS little-endian FP32 values, with a JSON
note beside them (training configuration and held-out results).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _frame(args):
    from paper_2008_06972_amd import synth
    sensor, seed = args
    pts, _, _ = synth.make_frame(synth.SENSORS[sensor], sensor, seed)
    return pts


def gen_frames(sensor: str, seeds, procs: int):
    if procs > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(procs) as pool:
            return pool.map(_frame, [(sensor, s) for s in seeds], chunksize=4)
    return [_frame((sensor, s)) for s in seeds]


def he_init(seed: int, n_params: int) -> np.ndarray:
    """He-normal weights, zero biases, in the parameter layout of pc.h."""
    rng = np.random.default_rng(seed)
    layers = ((4, 16), (16, 32), (32, 32), (32, 4))
    parts = []
    for i, o in layers:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (i * 9)), o * i * 9))
        parts.append(np.zeros(o))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == n_params
    return p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sensor", default="c2")
    ap.add_argument("--frames", type=int, default=2000)
    ap.add_argument("--seed0", type=int, default=5000)
    ap.add_argument("--eval-frames", type=int, default=50)
    ap.add_argument("--eval-seed0", type=int, default=900000)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2008_06972_amd", "weights", "seednet_c2.f32"))
    a = ap.parse_args()

    import torch
    from paper_2008_06972_amd import pcc, synth
    dev = torch.device("cuda:0")
    s = synth.SENSORS[a.sensor]
    S = pcc.Sensor.of(s)
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=8)
    ctx = pcc.Context([S])
    t0 = time.time()
    train = gen_frames(a.sensor, range(a.seed0, a.seed0 + a.frames), a.procs)
    held = gen_frames(a.sensor, range(a.eval_seed0, a.eval_seed0 + a.eval_frames), a.procs)
    print(f"generated {len(train)} + {len(held)} frames in {time.time() - t0:.1f}s", flush=True)

    # range images and labels on the GPU
    def ranges_and_labels(frames):
        out = []
        for pts in frames:
            xyz = torch.from_numpy(pts).to(dev)
            rng = torch.empty(s.H, s.W, dtype=torch.float32, device=dev)
            pcc.pc_project(ctx.h, xyz, len(pts), None, S, rng)
            lab = pcc.FrameStream(S, prm, dev)
            pcc.pc_fit_key(ctx.h, rng, S, prm, None, lab)
            out.append((rng, lab))
        torch.cuda.synchronize()
        return out
    t0 = time.time()
    data = ranges_and_labels(train)
    print(f"labels in {time.time() - t0:.1f}s", flush=True)

    P = pcc.PC_NET_PARAMS
    params = torch.from_numpy(he_init(1, P)).to(dev)
    m = torch.zeros(P, device=dev)
    v = torch.zeros(P, device=dev)
    grad = torch.zeros(P, device=dev)
    work = torch.zeros(pcc.pc_net_workspace_size(S), dtype=torch.uint8, device=dev)
    seed = torch.zeros(s.H // 4, s.W // 8, 4, device=dev)
    dseed = torch.zeros_like(seed)
    loss = torch.zeros(1, device=dev)
    losses = []
    step = 0
    t0 = time.time()
    for ep in range(a.epochs):
        order = np.random.default_rng(ep).permutation(len(data))
        acc = torch.zeros(1, device=dev)
        for q in order:
            rng, lab = data[q]
            step += 1
            pcc.pc_net_forward(ctx.h, params, rng, S, work, seed)
            pcc.pc_net_loss(ctx.h, seed, lab, S, prm, dseed, loss)
            grad.zero_()
            pcc.pc_net_backward(ctx.h, params, S, work, dseed, grad)
            lr = a.lr * 0.5 * (1.0 + np.cos(np.pi * ep / a.epochs))     # cosine decay over epochs
            pcc.pc_net_adam(ctx.h, params, grad, m, v, step, lr)
            acc += loss
        torch.cuda.synchronize()
        losses.append(float(acc.item()) / len(data))
        print(f"epoch {ep}: mean loss {losses[-1]:.4f} ({time.time() - t0:.1f}s)", flush=True)

    # held-out comparison: plain vs seeded key frames
    res = {"plain_bytes": 0, "seeded_bytes": 0, "seeded": 0, "fallback": 0, "fits_plain": 0, "fits_seeded": 0,
           "tiles": 0}
    for rng, lab in ranges_and_labels(held):
        pcc.pc_net_forward(ctx.h, params, rng, S, work, seed)
        fs = pcc.FrameStream(S, prm, dev)
        pcc.pc_fit_key(ctx.h, rng, S, prm, seed, fs)
        torch.cuda.synchronize()
        ip, isd = lab.info(), fs.info()
        res["plain_bytes"] += int(ip.size_bytes)
        res["seeded_bytes"] += int(isd.size_bytes)
        res["seeded"] += int(isd.seeded)
        res["fallback"] += int(isd.fallback)
        res["fits_plain"] += int(ip.fits)
        res["fits_seeded"] += int(isd.fits)
        res["tiles"] += int(sum(ip.tiles))
    res["size_ratio_seeded_over_plain"] = res["seeded_bytes"] / max(1, res["plain_bytes"])
    res["fallback_rate"] = res["fallback"] / max(1, res["seeded"] + res["fallback"])
    print("held-out:", json.dumps(res), flush=True)

    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    params.cpu().numpy().astype("<f4").tofile(a.out)
    note = {"sensor": a.sensor, "frames": a.frames, "seeds": [a.seed0, a.seed0 + a.frames - 1], "epochs": a.epochs,
            "lr": a.lr, "loss_per_epoch": losses, "held_out": res,
            "held_out_seeds": [a.eval_seed0, a.eval_seed0 + a.eval_frames - 1]}
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump(note, f, indent=1)
    print("wrote", a.out, flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Train the plane-seed network on the GPU through the C ABI.

Labels are the plain key-frame fits of generated frames (``pc_fit_key``
without seeds): a tile with a fit attempt is labelled, planar = accepted,
normal = the stored plane's unit normal.  Each step runs ``pc_net_forward``,
``pc_net_loss``, ``pc_net_backward`` and ``pc_net_adam`` on one frame.
After training, held-out sequences (10 frames, key frame 5) are encoded by
the batch graph with and without the network (its seeds serve the key
frames) and the key-frame fits per tile, the seeded / fallback counts, the
sizes and the rates of both are reported.

    python -m paper_2008_06972_amd.train_seed --sensor c5 --frames 2000 \
        --epochs 12 --eval-seqs 200 --out paper_2008_06972_amd/weights/seednet_c5.f32

Weights are written as PC_NET_PARAMS little-endian FP32 values, with a JSON
note beside them (training configuration and held-out results); with
--state the Adam moments and step count are kept too and training resumes
from them.
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
    sensor, scene, seed = args
    pts, _, _ = synth.make_frame(synth.SENSORS[sensor], scene, seed)
    return pts


def _sequence(args):
    from paper_2008_06972_amd import synth
    sensor, scene, seed = args
    q = synth.make_sequence(synth.SENSORS[sensor], scene, seed, n_frames=10, key_index=5, moving=5, shuffle=True)
    return q.frames, q.transforms


def _pool_map(fn, args, procs):
    if procs > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(procs) as pool:
            return pool.map(fn, args, chunksize=4)
    return [fn(x) for x in args]


def gen_frames(sensor: str, scene: str, seeds, procs: int):
    return _pool_map(_frame, [(sensor, scene, s) for s in seeds], procs)


def gen_sequences(sensor: str, scene: str, seeds, procs: int):
    return _pool_map(_sequence, [(sensor, scene, s) for s in seeds], procs)


def held_out(pcc, torch, ctx, S, seqs, net, steps=5):
    """Batch-encode held-out sequences without and with the network: per
    form the key frames' fits per tile, seeded and fallback tiles, bytes,
    compression ratio and frames/s (HIP events around graph replays)."""
    dev = torch.device("cuda:0")
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=8)
    xyz = [torch.from_numpy(f).to(dev) for fr, _ in seqs for f in fr]
    pts = sum(int(np.isfinite(f).all(axis=1).sum()) for fr, _ in seqs for f in fr)
    stream = torch.cuda.current_stream()
    out = {"sequences": len(seqs), "frames": len(xyz)}
    for name, w in (("plain", None), ("learned", net)):
        outs, fr = [], []
        for q, (frames, transforms) in enumerate(seqs):
            for i in range(len(frames)):
                o = pcc.FrameStream(S, prm, dev)
                outs.append(o)
                fr.append(dict(xyz=xyz[len(fr)], M=None if i == 5 else transforms[i], sensor=S, params=prm,
                               key=q * len(frames) + 5, out=o))
        b = pcc.Batch(ctx, fr, persistent=True, graph=True, net=w)
        b.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            b.run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        infos = [o.info() for o in outs]
        keys = [infos[j] for j in range(len(infos)) if j % 10 == 5]
        size = sum(int(i.size_bytes) for i in infos)
        out[name] = {"ms": ms, "frames_per_s": len(infos) / (ms / 1e3), "bytes": size,
                     "compression_ratio": 12.0 * pts / size,
                     "key_fits_per_tile": sum(i.fits for i in keys) / max(1, sum(sum(i.tiles) for i in keys)),
                     "seeded": int(sum(i.seeded for i in keys)), "fallback": int(sum(i.fallback for i in keys))}
        b.close()
    lr = out["learned"]
    lr["fallback_rate"] = lr["fallback"] / max(1, lr["seeded"] + lr["fallback"])
    out["ratio_learned_over_plain"] = lr["compression_ratio"] / out["plain"]["compression_ratio"]
    out["key_fits_learned_over_plain"] = lr["key_fits_per_tile"] / out["plain"]["key_fits_per_tile"]
    return out


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
    ap.add_argument("--scene", default="c2")
    ap.add_argument("--frames", type=int, default=2000)
    ap.add_argument("--seed0", type=int, default=5000)
    ap.add_argument("--eval-seqs", type=int, default=200, help="held-out 10-frame sequences")
    ap.add_argument("--eval-seed0", type=int, default=900000)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2008_06972_amd", "weights", "seednet_c2.f32"))
    ap.add_argument("--state", default="", metavar="NPZ",
                    help="optimiser state (parameters, Adam moments, step): resumed from if present, written at the end")
    a = ap.parse_args()

    import torch
    from paper_2008_06972_amd import pcc, synth
    dev = torch.device("cuda:0")
    s = synth.SENSORS[a.sensor]
    S = pcc.Sensor.of(s)
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=8)
    ctx = pcc.Context([S])
    t0 = time.time()
    train = gen_frames(a.sensor, a.scene, range(a.seed0, a.seed0 + a.frames), a.procs)
    print(f"generated {len(train)} frames in {time.time() - t0:.1f}s", flush=True)

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
    step0 = 0
    if a.state and os.path.exists(a.state):
        st = np.load(a.state)                  # plain arrays (no pickle)
        params = torch.from_numpy(st["params"].astype(np.float32)).to(dev)
        m = torch.from_numpy(st["m"].astype(np.float32)).to(dev)
        v = torch.from_numpy(st["v"].astype(np.float32)).to(dev)
        step0 = int(st["step"])
        print(f"resumed from {a.state} at step {step0}", flush=True)
    grad = torch.zeros(P, device=dev)
    work = torch.zeros(pcc.pc_net_workspace_size(S), dtype=torch.uint8, device=dev)
    seed = torch.zeros(s.H // 4, s.W // 8, 4, device=dev)
    dseed = torch.zeros_like(seed)
    loss = torch.zeros(1, device=dev)
    losses = []
    step = step0
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

    # held-out sequences: the batch with and without the network
    del data
    torch.cuda.empty_cache()
    t0 = time.time()
    held = gen_sequences(a.sensor, a.scene, range(a.eval_seed0, a.eval_seed0 + a.eval_seqs), a.procs)
    print(f"generated {len(held)} held-out sequences in {time.time() - t0:.1f}s", flush=True)
    res = held_out(pcc, torch, ctx, S, held, params)
    print("held-out:", json.dumps(res), flush=True)

    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    params.cpu().numpy().astype("<f4").tofile(a.out)
    if a.state:
        np.savez(a.state, params=params.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(), step=np.int64(step))
    note = {"sensor": a.sensor, "sensor_shape": [s.H, s.W, s.top_deg, s.bot_deg], "scene": a.scene,
            "frames": a.frames, "seeds": [a.seed0, a.seed0 + a.frames - 1], "epochs": a.epochs,
            "lr": a.lr, "loss_per_epoch": losses, "held_out": res,
            "held_out_sequence_seeds": [a.eval_seed0, a.eval_seed0 + a.eval_seqs - 1]}
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump(note, f, indent=1)
    print("wrote", a.out, flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

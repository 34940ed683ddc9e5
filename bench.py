#!/usr/bin/env python3
"""Benchmark of the spatio-temporal LiDAR encoder on one MI355X.

Workload: 96 sequences x 10 frames of a 64-beam x 2048-bin HDL-64E-like
sensor (+2..-24.8 deg), synthetic scenes (ground, 40 boxes, 30 poles,
sigma 2 cm, 5 % dropout, about 120k points per frame) with ego-motion
0.8-1.2 m and +-0.5 deg yaw per frame and 5 moving cars; key frame = index
5 of each sequence; eps = 2 cm, tiles 4x8, at most 5 fits per tile.
Inputs (xyz points, transforms) are resident in HBM before timing.

A step encodes all 960 frames from points to stream sizes: projection of
every frame, key-frame spatial encoding, predicted-frame temporal encoding,
residual quantisation, stream histograms and Huffman sizes.

Forms: "plain" launches the per-frame C-ABI calls frame by frame;
"batched" replays one HIP graph of persistent kernels over all frames;
"learned" is the batched graph with the plane-seed network seeding the key
frames' fits (the headline when its weights are present).  The ablation
batched vs learned isolates the network's effect from batching's.
Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "encoded frames/s at 64×2048, ε=2cm, learned+batched vs plain; compression ratio"
N_FRAMES, KEY_INDEX = 10, 5
SEED0 = 7000
EPS = 0.02
TRAFFIC_FILE = "hbm_traffic_batched_encoder_64x2048_960frames.json"


def _gen(seed):
    from paper_2008_06972_amd import synth
    seq = synth.make_sequence(synth.SENSORS["c2"], "c2", seed, n_frames=N_FRAMES, key_index=KEY_INDEX,
                              moving=5, shuffle=True)
    return seq.frames, seq.transforms


def make_workload(nseq: int, procs: int):
    seeds = [SEED0 + q for q in range(nseq)]
    if procs > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(procs) as pool:
            out = pool.map(_gen, seeds, chunksize=1)
    else:
        out = [_gen(s) for s in seeds]
    frames = [f for fr, _ in out for f in fr]
    transforms = np.concatenate([t for _, t in out])
    return frames, transforms


def traffic_from_profiles(kernel_kind: str, launches: int):
    """HBM traffic per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel sources (else None)."""
    from paper_2008_06972_amd.profile_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel_kind)
    if not k:
        return None
    return k.get("bytes_per_launch")


def _gen_mixed(q):
    from paper_2008_06972_amd import synth
    seq = synth.mixed_sequence(q, n_frames=N_FRAMES, key_index=KEY_INDEX)
    return (seq.sensor.H, seq.sensor.W), seq.frames, seq.transforms


def run_mixed(a, log, nseq=96):
    import torch
    from paper_2008_06972_amd import autotune, pcc, synth
    dev = torch.device("cuda:0")
    t0 = time.time()
    if a.procs > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(a.procs) as pool:
            seqs = pool.map(_gen_mixed, range(nseq), chunksize=1)
    else:
        seqs = [_gen_mixed(q) for q in range(nseq)]
    sens = {hw: pcc.Sensor.of(synth.mixed_sensor(*hw)) for hw, _, _ in seqs}
    npts = [len(f) for _, fr, _ in seqs for f in fr]
    pts = sum(int(np.isfinite(f).all(axis=1).sum()) for _, fr, _ in seqs for f in fr)
    xyz = [torch.from_numpy(f).to(dev) for _, fr, _ in seqs for f in fr]
    log(f"mixed: {len(npts)} frames, {min(npts)}-{max(npts)} points per frame, generated in {time.time() - t0:.1f}s")
    ctx = pcc.Context(list(sens.values()))
    stream = torch.cuda.current_stream()
    out = {"workload": f"{nseq} sequences x {N_FRAMES} frames, sensors {sorted(sens)}, 12 sequences each, "
                       "config-1 style scenes with moving cars, key frame 5",
           "frames": len(npts), "points": pts, "points_per_frame": [min(npts), max(npts)]}

    def timed(plans, lanes):
        fr, outs = [], []
        prms = {}
        j = 0
        for q, (hw, frames, transforms) in enumerate(seqs):
            th, tw = plans[hw]
            prm = prms.setdefault(hw, pcc.params(eps=eps, tile_h=th, tile_w=tw))
            for i in range(len(frames)):
                o = pcc.FrameStream(sens[hw], prm, dev)
                outs.append(o)
                fr.append(dict(xyz=xyz[j], M=None if i == KEY_INDEX else transforms[i], sensor=sens[hw], params=prm,
                               key=q * N_FRAMES + KEY_INDEX, out=o))
                j += 1
        b = pcc.Batch(ctx, fr, persistent=True, graph=True, lanes_max=lanes)
        for _ in range(a.warmup):
            b.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.steps):
            b.run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        size = sum(int(o.info().size_bytes) for o in outs)
        b.close()
        return {"ms_per_step": ms, "frames_per_s": len(npts) / (ms / 1e3), "compression_ratio": 12.0 * pts / size,
                "bytes": size}

    for eps in (0.01, 0.02):
        plain = timed({hw: (4, 8) for hw in sens}, 0)
        samples = {}
        for hw in sens:
            q = next(q for q, x in enumerate(seqs) if x[0] == hw)
            samples[hw] = (sens[hw], [(seqs[q][1], seqs[q][2])])
        chosen = autotune.tune_mixed(pcc, torch, ctx, eps, samples, KEY_INDEX)
        plans = {hw: (c.tile if c else (4, 8)) for hw, c in chosen.items()}
        big = max(sens, key=lambda hw: hw[0] * hw[1])
        tuned = timed(plans, chosen[big].lanes if chosen[big] else 0)
        tuned["plans"] = {f"{hw[0]}x{hw[1]}": (c.key() if c else None) for hw, c in chosen.items()}
        if a.plans:
            autotune.save_plans(a.plans, {autotune.plan_key(hw[0], hw[1], eps): c for hw, c in chosen.items() if c})
        out[f"eps_{eps}"] = {"tiles_4x8": plain, "autotuned": tuned}
        log(f"mixed eps {eps}: 4x8 {plain['frames_per_s']:.0f} frames/s ratio {plain['compression_ratio']:.2f}; "
            f"autotuned {tuned['frames_per_s']:.0f} frames/s ratio {tuned['compression_ratio']:.2f}")
    ctx.close()
    del xyz
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seqs", type=int, default=96)
    ap.add_argument("--forms", default="plain,batched,learned")
    ap.add_argument("--tune-seqs", type=int, default=8, help="sequences the autotuner times candidates on (0 = off)")
    ap.add_argument("--plans", default="", metavar="JSON", help="keep the autotuner's chosen plans in this file")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2008_06972_amd", "weights", "seednet_c2.f32"),
                    help="seed-network parameters for the learned form")
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--cpu-seqs", type=int, default=96, help="oracle sample (sequences)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-pack", action="store_true", help="skip packing the frames into containers")
    ap.add_argument("--no-decode", action="store_true", help="skip decoding the frames")
    ap.add_argument("--no-mixed", action="store_true", help="skip the uneven batch (eight sensors, eps 1 and 2 cm)")
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (traffic counter calibration) and exit")
    a = ap.parse_args()
    if a.copy_probe:
        import torch
        n = a.copy_probe << 18
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: it encodes one GPU's share of the sequences "
              "(sequences are independent, so N GPUs would each run this same batch)", file=sys.stderr)
        sys.exit(2)

    def log(*x):
        if not a.quiet:
            print(*x, file=sys.stderr, flush=True)

    import torch
    from paper_2008_06972_amd import pcc, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    pcc.lib()
    dev = torch.device("cuda:0")
    t0 = time.time()
    frames_np, transforms = make_workload(a.seqs, a.procs)
    nfr = len(frames_np)
    fin_per_frame = np.array([np.isfinite(f).all(axis=1).sum() for f in frames_np], np.int64)
    finite_pts = int(fin_per_frame.sum())
    log(f"workload: {nfr} frames, {finite_pts} points, generated in {time.time() - t0:.1f}s")

    s = synth.SENSORS["c2"]
    S = pcc.Sensor.of(s)
    prm = pcc.params(eps=EPS, tile_h=4, tile_w=8, max_iter=5, min_pts=4, min_inlier_frac=0.5)
    ctx = pcc.Context([S])
    xyz = [torch.from_numpy(f).to(dev) for f in frames_np]
    stream = torch.cuda.current_stream()
    L = pcc.pc_stream_layout(S, prm)
    HW, T = s.H * s.W, L.T

    def key_of(i):
        return (i // N_FRAMES) * N_FRAMES + KEY_INDEX

    result = {"metric": METRIC, "unit": "frames/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
              "data": "synthetic (seeded ray-cast scenes standing in for KITTI HDL-64E sequences)",
              "config": {"workload": f"{a.seqs} sequences x {N_FRAMES} frames, 64x2048 HDL-64E-like sensor, "
                                     f"eps=2cm, tiles 4x8, max 5 fits/tile, key frame 5",
                         "frames": nfr, "points": finite_pts}}
    forms = {}
    sizes = {}

    # ------------------------------------------------- batched / learned
    batches = {}

    def run_batched(name, net, cfg=None):
        prm_b = prm if cfg is None else pcc.params(eps=EPS, tile_h=cfg.tile[0], tile_w=cfg.tile[1], max_iter=5)
        outs = [pcc.FrameStream(S, prm_b, dev) for _ in range(nfr)]
        fr = [dict(xyz=xyz[i], M=None if i == key_of(i) else transforms[i], sensor=S, params=prm_b, key=key_of(i),
                   out=outs[i]) for i in range(nfr)]
        pers = True if cfg is None else cfg.persistent
        bpc = 0 if cfg is None else cfg.blocks_per_cu
        batch = pcc.Batch(ctx, fr, persistent=pers, graph=True, blocks_per_cu=bpc,
                          net=net if (cfg is None or cfg.seeded) else None, lanes_max=0 if cfg is None else cfg.lanes)
        nitems, ngroups, grid = batch.info()
        log(f"{name}: {nitems} strip items, {ngroups} groups, persistent grid {grid}")
        for _ in range(a.warmup):
            batch.run()
        torch.cuda.synchronize()
        # events between the replays: the mean over the K steps is the
        # result; the median replay is reported beside it
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
        ev[0].record(stream)
        for k in range(a.steps):
            batch.run()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[-1]) / a.steps
        ms_median = float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(a.steps)]))
        infos = [o.info() for o in outs]
        key_infos = [infos[i] for i in range(nfr) if i == key_of(i)]
        tiles = sum(sum(i.tiles) for i in infos)
        st = {"ms_per_step": ms, "frames_per_s": nfr / (ms / 1e3), "ms_per_step_median": ms_median,
              "mapping": "default 4x8 persistent" if cfg is None else cfg.key(),
              "fits_per_tile": sum(i.fits for i in infos) / max(1, tiles),
              "key_fits_per_tile": sum(i.fits for i in key_infos) / max(1, sum(sum(i.tiles) for i in key_infos)),
              "seeded_tiles": int(sum(i.seeded for i in infos)), "fallback_tiles": int(sum(i.fallback for i in infos))}
        st["fallback_rate"] = st["fallback_tiles"] / max(1, st["seeded_tiles"] + st["fallback_tiles"])
        forms[name] = st
        sizes[name] = np.array([i.size_bytes for i in infos], np.int64)
        batch.outs = outs
        batches[name] = batch
        log(f"{name}: {ms:.3f} ms/step, {nfr / (ms / 1e3):.0f} frames/s")

    net = None
    if "learned" in a.forms and os.path.exists(a.weights):
        net = torch.from_numpy(np.fromfile(a.weights, dtype="<f4")).to(dev)
        assert net.numel() == pcc.PC_NET_PARAMS, a.weights
    tuned = {}
    if a.tune_seqs > 0:
        # autotune the mapping on a sample (first --tune-seqs sequences):
        # fastest plan whose ratio >= 0.98 x the plain 4x8 ratio
        from paper_2008_06972_amd import autotune
        sample = [(frames_np[q * N_FRAMES:(q + 1) * N_FRAMES], transforms[q * N_FRAMES:(q + 1) * N_FRAMES])
                  for q in range(min(a.tune_seqs, a.seqs))]
        t1 = time.time()
        for name, shapes, use_net in (("batched", autotune.SHAPES, None), ("learned", ((4, 8),), net)):
            if name not in a.forms or (name == "learned" and net is None):
                continue
            log(f"autotune {name}:")
            best, cands, ref_ratio = autotune.tune(pcc, torch, ctx, S, EPS, sample, KEY_INDEX, net=use_net,
                                                   shapes=shapes, log=log)
            tuned[name] = best
            if a.plans and best is not None:
                autotune.save_plans(a.plans, {autotune.plan_key(s.H, s.W, EPS) + f" {name}": best})
            result.setdefault("autotune", {})[name] = {
                "chosen": best.key() if best else None, "reference_ratio": ref_ratio,
                "candidates": {c.key(): {"ms": round(c.ms, 4), "ratio": round(c.ratio, 4), "ok": c.ok} for c in cands}}
        result.setdefault("autotune", {})["sample"] = f"{len(sample)} sequences, {time.time() - t1:.1f}s"
    if "batched" in a.forms:
        run_batched("batched", None, tuned.get("batched"))
    if net is not None:
        run_batched("learned", net, tuned.get("learned"))

    # -------------------------------------------------------------- plain
    if "plain" in a.forms:
        outs_p = [pcc.FrameStream(S, prm, dev) for _ in range(nfr)]
        rng = [torch.empty(s.H, s.W, dtype=torch.float32, device=dev) for _ in range(nfr)]

        def plain_step():
            for q in range(0, nfr, N_FRAMES):
                k = q + KEY_INDEX
                pcc.pc_project(ctx.h, xyz[k], len(frames_np[k]), None, S, rng[k], stream=stream)
                pcc.pc_fit_key(ctx.h, rng[k], S, prm, None, outs_p[k], stream=stream)
                for i in range(q, q + N_FRAMES):
                    if i == k:
                        continue
                    pcc.pc_project(ctx.h, xyz[i], len(frames_np[i]), transforms[i], S, rng[i], stream=stream)
                    pcc.pc_encode_pred(ctx.h, outs_p[k], rng[i], transforms[i], S, prm, outs_p[i], stream=stream)
        plain_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_host = time.time()
        e0.record(stream)
        for _ in range(a.plain_steps):
            plain_step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.plain_steps
        forms["plain"] = {"ms_per_step": ms, "frames_per_s": nfr / (ms / 1e3),
                          "host_ms_per_step": (time.time() - t_host) * 1e3 / a.plain_steps}
        sizes["plain"] = np.array([o.info().size_bytes for o in outs_p], np.int64)
        log(f"plain: {ms:.3f} ms/step, {nfr / (ms / 1e3):.0f} frames/s")
        if "batched" in sizes and forms["batched"]["mapping"].startswith(("default", "4x8")):
            same = bool(np.array_equal(sizes["plain"], sizes["batched"]))
            result["plain_equals_batched"] = same
            log("plain and batched streams have equal sizes:", same)

    for name, sz in sizes.items():
        tot = int(sz.sum())
        forms[name]["compression_ratio"] = 12.0 * finite_pts / tot
        forms[name]["bytes"] = tot
    result["forms"] = forms
    head = "learned" if "learned" in forms else ("batched" if "batched" in forms else "plain")
    if "learned" in forms and "plain" in forms:
        result["learned_over_plain_ratio"] = forms["learned"]["compression_ratio"] / forms["plain"]["compression_ratio"]
    if "learned" in forms and "batched" in forms:
        result["ablation"] = {
            "batched_plain_fps": forms["batched"]["frames_per_s"], "batched_learned_fps": forms["learned"]["frames_per_s"],
            "batched_plain_ratio": forms["batched"]["compression_ratio"],
            "batched_learned_ratio": forms["learned"]["compression_ratio"],
            "key_fits_per_tile_plain": forms["batched"]["key_fits_per_tile"],
            "key_fits_per_tile_learned": forms["learned"]["key_fits_per_tile"],
            "fallback_rate": forms["learned"]["fallback_rate"]}
    result["form"] = head
    result["value"] = forms[head]["frames_per_s"]
    result["ms_per_step"] = forms[head]["ms_per_step"]
    result["compression_ratio"] = forms[head]["compression_ratio"]
    result["compression_ratio_16B_per_point"] = forms[head]["compression_ratio"] * 16.0 / 12.0

    # ------------------------------------------- host-to-device transfer
    # the boundary takes device-resident points; a caller holding them in
    # host memory adds one copy per pass (pinned memory, outside `value`)
    tot_pts = sum(len(f) for f in frames_np)
    host_pts = torch.empty((tot_pts, 3), dtype=torch.float32, pin_memory=True)
    off = 0
    for f in frames_np:
        host_pts[off:off + len(f)] = torch.from_numpy(f)
        off += len(f)
    dev_pts = torch.empty((tot_pts, 3), dtype=torch.float32, device=dev)
    dev_pts.copy_(host_pts, non_blocking=True)
    torch.cuda.synchronize()
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h0.record(stream)
    for _ in range(3):
        dev_pts.copy_(host_pts, non_blocking=True)
    h1.record(stream)
    torch.cuda.synchronize()
    h2d_ms = h0.elapsed_time(h1) / 3
    result["h2d"] = {"bytes": 12 * tot_pts, "ms": h2d_ms, "GB/s": 12 * tot_pts / (h2d_ms / 1e3) / 1e9,
                     "frames_per_s_including_h2d": nfr / ((result["ms_per_step"] + h2d_ms) / 1e3),
                     "what": "every frame's points copied once from pinned host memory (not part of value)"}
    log(f"h2d: {h2d_ms:.2f} ms for {12 * tot_pts / 1e9:.2f} GB")
    del host_pts, dev_pts

    # ------------------------------------------------------------ roofline
    batch = batches.get(head)
    if batch is not None:
        # per-launch durations: HIP events between the launches of the same
        # launch sequence, on the same stream, averaged over --steps passes
        prof = []
        for _ in range(a.steps):
            prof += batch.profile(stream.cuda_stream)
        prof = [(k, t / a.steps) for k, t in prof]
        log("per-launch ms:", prof)
        infos = [o.info() for o in batch.outs]
        n_res_k = sum(i.n_res for j, i in enumerate(infos) if j == key_of(j))
        n_res_p = sum(i.n_res for j, i in enumerate(infos) if j != key_of(j))
        nk = sum(1 for j in range(nfr) if j == key_of(j))
        npf = nfr - nk
        # algorithmic bytes per launch: what the method must move, not what
        # this implementation moves.  Projection (binning) reads 12 B per
        # point and produces a 4 B range value per pixel; an encoder reads the range
        # image (4 B per pixel) and writes the occupancy bits (1/8 B per
        # pixel), the run and plane table (16 B per tile), the masks (8 B per
        # tile) and the codes (2 B each); a predicted frame also reads the
        # key frame's plane table (16 B per tile).
        pts_k = sum(int(fin_per_frame[j]) for j in range(nfr) if j == key_of(j))
        Tb = batch.outs[0].L.T            # tiles per frame of the timed mapping
        alg = {
            "bin": 12 * finite_pts + 4 * HW * nfr,
            "key": nk * (4 * HW + HW // 8 + 16 * Tb + 8 * Tb) + 2 * n_res_k,
            "pred": npf * (4 * HW + HW // 8 + 16 * Tb + 8 * Tb + 16 * Tb) + 2 * n_res_p,
        }
        pass_bytes = 12 * finite_pts + nfr * (8 * HW + HW // 8 + 24 * Tb) + npf * 16 * Tb + 2 * (n_res_k + n_res_p)
        dur = {}
        for kind, t in prof:
            dur[kind] = dur.get(kind, 0.0) + t
        dom = max((k for k in alg if k in dur), key=lambda k: dur[k])
        ach = alg[dom] / (dur[dom] / 1e3) / 1e9
        pass_gbps = pass_bytes / (result["ms_per_step"] / 1e3) / 1e9
        result["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": 8000.0, "unit": "GB/s",
                              "frac": ach / 8000.0, "traffic": traffic_from_profiles(dom, 1),
                              "bytes_per_launch": alg[dom], "ms_per_launch": dur[dom],
                              "pass": {"bytes": pass_bytes, "GB/s": pass_gbps, "frac": pass_gbps / 8000.0,
                                       "what": "algorithmic bytes of the whole pass over ms_per_step"}}
        result["launch_ms"] = {k: round(v, 4) for k, v in dur.items()}
        # a plain device copy of 1 GiB (read once, written once): the
        # bandwidth a kernel on this device can reach in practice
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(5):
            dst.copy_(src)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_gbps = 5 * 2 * (4 << 28) / (c0.elapsed_time(c1) / 1e3) / 1e9
        del src, dst
        result["copy_ceiling"] = {"GB/s": copy_gbps, "bytes": 2 * (4 << 28), "what": "1 GiB device copy, read + write"}
        result["roofline"]["frac_of_copy"] = ach / copy_gbps

    # ------------------------------------------- entropy-coded bitstream
    # every frame of the head form packed into its container (Sec. III-A):
    # the emitted bytes against the size model, and the packing rate
    if batch is not None and not a.no_pack:
        Lh = batch.outs[0].L
        prm_h = pcc.params(eps=EPS, tile_h=Lh.th, tile_w=Lh.tw, max_iter=5, min_pts=4, min_inlier_frac=0.5)
        cap = pcc.pc_pack_bound(S, prm_h)
        wsb = pcc.pc_pack_batch_workspace_size(S, prm_h, nfr)
        work = torch.empty(wsb, dtype=torch.uint8, device=dev)
        cont = torch.empty(nfr, cap, dtype=torch.uint8, device=dev)
        outs_c = [cont[i] for i in range(nfr)]
        nbytes = torch.zeros(nfr, dtype=torch.int64, device=dev)
        pcc.pc_pack_batch(ctx.h, batch.outs, S, prm_h, work, wsb, outs_c, cap, nbytes, stream=stream)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        t_host = time.time()
        p0.record(stream)
        for _ in range(reps):
            pcc.pc_pack_batch(ctx.h, batch.outs, S, prm_h, work, wsb, outs_c, cap, nbytes, stream=stream)
        p1.record(stream)
        torch.cuda.synchronize()
        pms = p0.elapsed_time(p1) / reps
        packed = nbytes.cpu().numpy().astype(np.int64)
        model = sizes[head]
        result["bitstream"] = {
            "frames": nfr, "container_bytes": int(packed.sum()), "model_bytes": int(model.sum()),
            "excess_over_model": float(packed.sum() / model.sum() - 1.0),
            "frames_equal_to_model": int((packed == model).sum()),
            "compression_ratio": 12.0 * finite_pts / float(packed.sum()),
            "pack_ms": pms, "pack_frames_per_s": nfr / (pms / 1e3),
            "pack_host_ms": (time.time() - t_host) * 1e3 / reps,
            "what": "pc_pack_batch over every frame of the timed form (job-table upload included)"}
        log(f"bitstream: {int(packed.sum())} bytes vs model {int(model.sum())}, {pms:.3f} ms per batch pack")
        # decode from bytes: every container back into a frame buffer
        # (pc_unpack_batch, which synchronises), then checked against the
        # frames it was packed from through their decoded ranges' sizes
        outs_u = [pcc.FrameStream(S, prm_h, dev) for _ in range(nfr)]
        keys_u = [None if i == key_of(i) else outs_u[key_of(i)] for i in range(nfr)]
        wsu = pcc.pc_unpack_batch_workspace_size(S, prm_h, nfr)
        work_u = torch.empty(wsu, dtype=torch.uint8, device=dev)
        sizes_u = [int(x) for x in packed]
        pcc.pc_unpack_batch(ctx.h, outs_c, sizes_u, keys_u, S, prm_h, work_u, wsu, outs_u, stream=stream)
        u0 = time.time()
        reps_u = 3
        for _ in range(reps_u):
            pcc.pc_unpack_batch(ctx.h, outs_c, sizes_u, keys_u, S, prm_h, work_u, wsu, outs_u, stream=stream)
        ums = (time.time() - u0) * 1e3 / reps_u
        same = all(int(u.info().n_res) == int(o.info().n_res) for u, o in zip(outs_u, batch.outs))
        result["bitstream"].update({"unpack_ms": ums, "unpack_frames_per_s": nfr / (ums / 1e3),
                                    "unpacked_residuals_equal": bool(same),
                                    "unpack_what": "pc_unpack_batch of every container, host clock around the "
                                                   "synchronising call"})
        log(f"unpack: {ums:.2f} ms per batch")
        del cont, work, outs_u, work_u

    # ---------------------------------------------------------------- decode
    # every frame of the head form decoded to its range image by one
    # pc_decode_batch call (job-table upload included in the time)
    if batch is not None and not a.no_decode:
        Lh = batch.outs[0].L
        prm_d = pcc.params(eps=EPS, tile_h=Lh.th, tile_w=Lh.tw, max_iter=5, min_pts=4, min_inlier_frac=0.5)
        outs_d = batch.outs
        dec = torch.empty((nfr, s.H, s.W), dtype=torch.float32, device=dev)
        dec_list = [dec[i] for i in range(nfr)]
        keys_d = [None if i == key_of(i) else outs_d[key_of(i)] for i in range(nfr)]
        wsd = pcc.pc_decode_batch_workspace_size(nfr)
        work_d = torch.empty(wsd, dtype=torch.uint8, device=dev)
        pcc.pc_decode_batch(ctx.h, keys_d, outs_d, S, prm_d, dec_list, work_d, wsd, stream=stream)
        torch.cuda.synchronize()
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        d0.record(stream)
        for _ in range(reps):
            pcc.pc_decode_batch(ctx.h, keys_d, outs_d, S, prm_d, dec_list, work_d, wsd, stream=stream)
        d1.record(stream)
        torch.cuda.synchronize()
        dms = d0.elapsed_time(d1) / reps
        infos_d = [o.info() for o in outs_d]
        Td, HWd = Lh.T, s.H * s.W
        # algorithmic bytes: OCC, masks, run tables, codes read; key run
        # planes read for temporal runs; the range image written
        alg_d = sum(HWd // 8 + 8 * Td + 16 * (i.n_sruns + i.n_pruns) + 16 * i.n_pruns + 2 * i.n_res + 4 * HWd
                    for i in infos_d)
        result["decode"] = {"frames": nfr, "ms": dms, "frames_per_s": nfr / (dms / 1e3), "bytes": alg_d,
                            "GB/s": alg_d / (dms / 1e3) / 1e9, "frac_of_hbm_peak": alg_d / (dms / 1e3) / 8e12,
                            "what": "pc_decode_batch over every frame of the timed form (job-table upload included)"}
        log(f"decode: {dms:.3f} ms for {nfr} frames")
        del dec, dec_list, work_d

    # ------------------------------------------------------ uneven batch
    # 96 sequences over eight sensors (16/32/64/128 beams x 1024/2048 bins),
    # config-1 style scenes, one graph per eps; per sensor the autotuner's
    # tile shape and mapping (timed on one sequence per sensor), beside the
    # same batch with 4x8 tiles everywhere
    if not a.no_mixed:
        result["mixed"] = run_mixed(a, log)

    # ------------------------------------------------------- CPU baseline
    if not a.no_cpu:
        import oracle
        tb = oracle.Tables.of(s)
        oprm = oracle.Params(eps=EPS, th=4, tw=8)
        nq = min(a.cpu_seqs, a.seqs)
        sample = frames_np[: nq * N_FRAMES]
        t1 = time.time()
        total, osz, ofin = oracle.encode_sequences(sample, transforms[: nq * N_FRAMES], KEY_INDEX, nq, N_FRAMES, tb, oprm)
        dt = time.time() - t1
        result["cpu_baseline"] = {"value": len(sample) / dt, "unit": "frames/s", "cores": oracle.num_threads(),
                                  "kind": "oracle",
                                  "sample": f"first {nq} sequences ({len(sample)} frames) of the same workload, "
                                            f"plain fits (no seed network), {dt:.1f}s wall",
                                  "compression_ratio": 12.0 * ofin / total}
        for name, sz in sizes.items():
            rel = abs(int(sz[: nq * N_FRAMES].sum()) - total) / total
            result["cpu_baseline"][f"size_rel_diff_{name}"] = rel
        log(f"oracle: {len(sample) / dt:.1f} frames/s on {oracle.num_threads()} threads")
        # one core, on the first sequence
        nt = oracle.num_threads()
        oracle.set_num_threads(1)
        t1 = time.time()
        oracle.encode_sequences(frames_np[:N_FRAMES], transforms[:N_FRAMES], KEY_INDEX, 1, N_FRAMES, tb, oprm)
        dt1 = time.time() - t1
        oracle.set_num_threads(nt)
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        result["cpu_baseline"]["one_core"] = {"value": N_FRAMES / dt1, "unit": "frames/s",
                                              "sample": f"first sequence ({N_FRAMES} frames), {dt1:.2f}s wall"}
        result["cpu_baseline"]["host"] = {"cpu": model, "logical_cpus": os.cpu_count()}
        log(f"oracle: {N_FRAMES / dt1:.1f} frames/s on one core ({model})")
    print(json.dumps(result), flush=True)
    for b in batches.values():
        b.close()
    ctx.close()


if __name__ == "__main__":
    main()

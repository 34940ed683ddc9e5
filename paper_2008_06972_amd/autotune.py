"""Autotuner of the batched encoder's mapping.

For one sensor and error bound it times candidate plans on a sample of the
workload and keeps the fastest whose compression ratio is at least
``ratio_floor`` times the reference ratio (the plain 4x8-tile encoding of
the same sample): a tile shape changes the encoding itself, so speed may
not be bought with size.  Candidates combine

* tile shape: 4x4, 4x8, 4x16, 8x8 (the compiled shapes);
* work distribution: persistent work-groups pulling (frame, strip) items
  from an atomic queue, or one work-group per strip;
* persistent grid size: work-groups per CU;
* wavefront mapping: how many neighbouring lanes (1, 2 or 4) may share one
  tile once few tiles are left iterating (more lanes shorten one tile's
  chain of dependent operations, fewer leave more tiles per wavefront).

With a seed network only 4x8 tiles are seeded, so other shapes are timed
without it.  Timing uses HIP events around replays of the captured graph.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

SHAPES = ((4, 8), (4, 4), (4, 16), (8, 8))


@dataclass
class Candidate:
    tile: tuple
    persistent: bool
    blocks_per_cu: int
    seeded: bool
    lanes: int = 4
    ms: float = float("nan")
    ratio: float = float("nan")
    ok: bool = False
    notes: dict = field(default_factory=dict)

    def key(self):
        return f"{self.tile[0]}x{self.tile[1]} {'persistent' if self.persistent else 'grid'} " \
               f"bpc={self.blocks_per_cu} lanes<={self.lanes}{' seeded' if self.seeded else ''}"


def candidates(shapes=SHAPES, blocks=(2, 4, 8), with_net=False, lanes=(1, 2, 4)):
    """Every tile shape with every work distribution at the default mapping
    (up to 4 lanes per tile), and every mapping at the default distribution
    (persistent, 4 work-groups per CU)."""
    out = []
    for (th, tw), pers in itertools.product(shapes, (True, False)):
        for b in (blocks if pers else (0,)):
            out.append(Candidate((th, tw), pers, b, with_net and (th, tw) == (4, 8)))
        if pers:
            for ln in lanes:
                if ln != 4:
                    out.append(Candidate((th, tw), True, 4, with_net and (th, tw) == (4, 8), ln))
    return out


def choose(cands, ref_ratio: float, ratio_floor: float = 0.98):
    """Fastest candidate whose ratio >= ratio_floor * ref_ratio (None if none)."""
    best = None
    for c in cands:
        c.ok = bool(np.isfinite(c.ms) and c.ratio >= ratio_floor * ref_ratio)
        if c.ok and (best is None or c.ms < best.ms):
            best = c
    return best


def measure(pcc, torch, ctx, sensor, eps, seqs, key_index, cand: Candidate, net=None, reps=5, warmup=2,
            max_iter=5):
    """Time one candidate on the sample; returns (ms per replay, ratio)."""
    dev = torch.device("cuda:0")
    prm = pcc.params(eps=eps, tile_h=cand.tile[0], tile_w=cand.tile[1], max_iter=max_iter)
    frames = []
    outs = []
    pts = 0
    for q, (fr, tr) in enumerate(seqs):
        base = len(frames)
        for i, p in enumerate(fr):
            o = pcc.FrameStream(sensor, prm, dev)
            outs.append(o)
            frames.append(dict(xyz=torch.from_numpy(p).to(dev), M=None if i == key_index else tr[i], sensor=sensor,
                               params=prm, key=base + key_index, out=o))
            pts += int(np.isfinite(p).all(axis=1).sum())
    batch = pcc.Batch(ctx, frames, persistent=cand.persistent, graph=True, blocks_per_cu=cand.blocks_per_cu,
                      net=net if cand.seeded else None, lanes_max=cand.lanes)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        batch.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        batch.run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    size = sum(int(o.info().size_bytes) for o in outs)
    batch.close()
    return ms, 12.0 * pts / size


def tune(pcc, torch, ctx, sensor, eps, seqs, key_index, net=None, ratio_floor=0.98, shapes=SHAPES, blocks=(2, 4, 8),
         reps=5, log=None):
    """Measure every candidate on the sample ``seqs`` (list of (frames,
    transforms)); returns (best Candidate, all candidates, reference ratio).
    The reference is the plain 4x8 encoding of the same sample."""
    ref = Candidate((4, 8), True, 4, False)
    ref.ms, ref_ratio = measure(pcc, torch, ctx, sensor, eps, seqs, key_index, ref, reps=1)
    cands = candidates(shapes, blocks, with_net=net is not None)
    for c in cands:
        try:
            c.ms, c.ratio = measure(pcc, torch, ctx, sensor, eps, seqs, key_index, c, net=net, reps=reps)
        except pcc.PcError as e:          # shape not valid for this sensor
            c.notes["error"] = str(e)
        if log:
            log(f"  {c.key():32s} {c.ms:8.3f} ms  ratio {c.ratio:7.3f}")
    return choose(cands, ref_ratio, ratio_floor), cands, ref_ratio


def tune_mixed(pcc, torch, ctx, eps, samples, key_index, shapes=SHAPES, lanes=(1, 2, 4), ratio_floor=0.98,
               reps=3, log=None):
    """Plans for a batch of several sensors: per sensor the fastest tile
    shape and wavefront mapping on its sample (persistent, 4 work-groups per
    CU) whose ratio keeps the floor of that sensor's plain 4x8 encoding.
    `samples` maps a sensor key to (Sensor, [(frames, transforms)]).
    Returns {key: Candidate or None}; the batch-wide mapping is the one
    chosen for the sensor with the most pixels."""
    out = {}
    for k, (S, seqs) in samples.items():
        ref = Candidate((4, 8), True, 4, False)
        ref.ms, ref_ratio = measure(pcc, torch, ctx, S, eps, seqs, key_index, ref, reps=1)
        cands = [Candidate(sh, True, 4, False, ln) for sh in shapes for ln in lanes]
        for c in cands:
            try:
                c.ms, c.ratio = measure(pcc, torch, ctx, S, eps, seqs, key_index, c, reps=reps)
            except pcc.PcError as e:
                c.notes["error"] = str(e)
        best = choose(cands, ref_ratio, ratio_floor)
        out[k] = best
        if log:
            log(f"  {S.H}x{S.W} eps {eps}: {best.key() if best else None} "
                f"({best.ms if best else float('nan'):.3f} ms, ratio {best.ratio if best else float('nan'):.3f}, "
                f"4x8 ratio {ref_ratio:.3f})")
    return out


# ------------------------------------------------------------ plan cache
# Chosen plans kept between runs: a JSON object keyed by "HxW eps" (sensor
# rows and columns, error bound in metres), each value the candidate's
# fields and its measurement.
def plan_key(H: int, W: int, eps: float) -> str:
    return f"{H}x{W} {eps:g}"


def to_record(c: Candidate) -> dict:
    return {"tile": list(c.tile), "persistent": c.persistent, "blocks_per_cu": c.blocks_per_cu, "seeded": c.seeded,
            "lanes": c.lanes, "ms": c.ms, "ratio": c.ratio}


def from_record(r: dict) -> Candidate:
    c = Candidate(tuple(int(x) for x in r["tile"]), bool(r["persistent"]), int(r["blocks_per_cu"]), bool(r["seeded"]),
                  int(r.get("lanes", 4)))
    c.ms, c.ratio, c.ok = float(r.get("ms", float("nan"))), float(r.get("ratio", float("nan"))), True
    if c.tile not in SHAPES or c.lanes not in (1, 2, 4) or c.blocks_per_cu < 0:
        raise ValueError(f"not a valid plan: {r}")
    return c


def save_plans(path: str, plans: dict) -> None:
    """plans: {plan_key: Candidate}; merged into the file's existing entries."""
    import json
    import os
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.update({k: to_record(c) for k, c in plans.items()})
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load_plans(path: str) -> dict:
    """{plan_key: Candidate} from a file written by save_plans ({} if absent)."""
    import json
    import os
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return {k: from_record(r) for k, r in data.items()}

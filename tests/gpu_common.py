"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same inputs, and compare what must agree."""
from __future__ import annotations

import math

import numpy as np

EPS = 0.02


def unit_normal(axis, a, b):
    """Unit normal of the stored plane p_k + a p_k1 + b p_k2 = c, and the
    scale |n_s| (so the plane's distance from the origin is c / |n_s|)."""
    n = np.zeros(3)
    k = int(axis)
    k1, k2 = (1, 2) if k == 0 else ((0, 2) if k == 1 else (0, 1))
    n[k], n[k1], n[k2] = 1.0, float(a), float(b)
    s = np.linalg.norm(n)
    return n / s, s


def plane_diff(g, o):
    """(normal angle in rad, |offset difference| in m) of two stored planes
    given as (axis, a, b, c)."""
    ng, sg = unit_normal(g[0], g[1], g[2])
    no, so = unit_normal(o[0], o[1], o[2])
    cg, co = float(g[3]) / sg, float(o[3]) / so
    if np.dot(ng, no) < 0:
        no, co = -no, -co
    ang = math.acos(min(1.0, abs(float(np.dot(ng, no)))))
    return ang, abs(cg - co), max(abs(co), 1.0)


def run_gpu_sequence(pcc, torch, ctx, S, prm, frames, transforms, key_index, dev, shuffle_idx=None):
    """Project, encode (key then predicted frames) and decode on the GPU.
    Returns per frame: dict(range, host stream, decoded range, stats)."""
    out = [None] * len(frames)
    key_fs = None
    order = [key_index] + [i for i in range(len(frames)) if i != key_index]
    for i in order:
        xyz = torch.from_numpy(np.ascontiguousarray(frames[i])).to(dev)
        rng = torch.empty(S.H, S.W, dtype=torch.float32, device=dev)
        idx = torch.empty(S.H, S.W, dtype=torch.int32, device=dev)
        st = torch.zeros(5, dtype=torch.int64, device=dev)
        M = None if i == key_index else transforms[i]
        pcc.pc_project(ctx.h, xyz, len(frames[i]), M, S, rng, idx, st)
        fs = pcc.FrameStream(S, prm, dev)
        if i == key_index:
            pcc.pc_fit_key(ctx.h, rng, S, prm, None, fs)
            key_fs = fs
        else:
            pcc.pc_encode_pred(ctx.h, key_fs, rng, M, S, prm, fs)
        dec = torch.empty_like(rng)
        pcc.pc_decode(ctx.h, None if i == key_index else key_fs, fs, S, prm, dec)
        torch.cuda.synchronize()
        out[i] = dict(range=rng.cpu().numpy(), idx=idx.cpu().numpy(), stats=st.cpu().numpy(), fs=fs,
                      host=fs.host(), dec=dec.cpu().numpy())
    return out


def compare_frame(orc, g, o, rng_img, tol_frac=0.005, max_iter=5):
    """Compare one encoded frame: GPU host dict `g` vs oracle Frame `o`.
    Returns a dict of agreement statistics."""
    T = len(g["cls"])
    st = {}
    st["tiles"] = T
    st["cls_agree"] = float(np.mean(g["cls"] == o.cls))
    st["own_status_agree"] = float(np.mean(g["tiles"]["status"] == o.own_status))
    # a fit that stopped at max_iter without converging took its plane from
    # the previous iteration's pixels, which the records do not hold: planes
    # are compared where both sides converged to the same pixels
    conv = (g["tiles"]["iters"] < max_iter) & (o.own_iters < max_iter)
    same_mask = (g["tiles"]["mask"] == o.own_mask) & (g["tiles"]["status"] >= 4) & (o.own_status >= 4) & conv
    st["own_mask_agree"] = float(np.mean(g["tiles"]["mask"] == o.own_mask))
    worst_ang, worst_c = 0.0, 0.0
    for t in np.nonzero(same_mask)[0]:
        tg = g["tiles"][t]
        ang, dc, sc = plane_diff((tg["axis"], tg["a"], tg["b"], tg["c"]),
                                 (o.own_axis[t], o.own_abc[t][0], o.own_abc[t][1], o.own_abc[t][2]))
        worst_ang = max(worst_ang, ang)
        worst_c = max(worst_c, dc / sc)
    st["planes_compared"] = int(same_mask.sum())
    st["worst_normal_rad"] = worst_ang
    st["worst_offset_rel"] = worst_c
    info = g["info"]
    st["size_gpu"] = int(info.size_bytes)
    st["size_orc"] = int(o.size_bytes)
    st["size_rel"] = abs(int(info.size_bytes) - int(o.size_bytes)) / int(o.size_bytes)
    v = rng_img > 0
    st["n_valid"] = int(v.sum())
    st["valid_agree"] = int(info.n_valid) == int(v.sum())
    st["fp64_frac"] = info.fp64_fits / max(1, info.fits)
    return st


def residual_codes_agree(g, o, rng_img, th, tw):
    """Codes of pixels both sides keep as residuals must be bit-identical
    (the code is a function of the range alone)."""
    H, W = rng_img.shape
    def residual_map(cls, mask):
        res = np.zeros((H, W), bool)
        v = rng_img > 0
        TC = W // tw
        for t in range(len(cls)):
            tr, tc = divmod(t, TC)
            blk = v[tr * th:(tr + 1) * th, tc * tw:(tc + 1) * tw]
            m = int(mask[t]) if cls[t] in (2, 3) else 0
            bits = np.array([(m >> j) & 1 for j in range(th * tw)], bool).reshape(th, tw)
            res[tr * th:(tr + 1) * th, tc * tw:(tc + 1) * tw] = blk & ~bits
        return res
    rg = residual_map(g["cls"], g["mask"])
    ro = residual_map(o.cls, o.mask)
    cg = np.zeros((H, W), np.int64) - 1
    co = np.zeros((H, W), np.int64) - 1
    cg[rg] = g["codes"]
    co[ro] = o.codes
    both = rg & ro
    return bool(np.array_equal(cg[both], co[both])), int(both.sum()), int((rg != ro).sum())


def _ray_t(tb, th, tw, t, TC, axis, a, b, c):
    """FP64 ray-cast ranges of a stored plane over the pixels of tile t (the
    oracle's FP32 pixel directions)."""
    tr, tc = divmod(int(t), TC)
    d = tb.directions()[tr * th:(tr + 1) * th, tc * tw:(tc + 1) * tw].astype(np.float64).reshape(-1, 3)
    k = int(axis)
    k1, k2 = (1, 2) if k == 0 else ((0, 2) if k == 1 else (0, 1))
    den = d[:, k] + float(a) * d[:, k1] + float(b) * d[:, k2]
    with np.errstate(divide="ignore", invalid="ignore"):
        return float(c) / den


def tile_ranges(rng_img, th, tw, t, TC):
    tr, tc = divmod(int(t), TC)
    return rng_img[tr * th:(tr + 1) * th, tc * tw:(tc + 1) * tw].astype(np.float64).ravel()


# A pixel's keep-or-drop decision is |c/den - r| <= eps on each side with its
# own FP32 plane.  Both sides fit the same pixels, the GPU in FP32 and the
# oracle in FP64, so their planes differ by rounding, and a decision may
# flip only for a pixel whose |t - r| lies within that rounding of eps.  A
# relative change q of the plane moves the ray-cast range t = c / (n.d) by
# about q t / cos, cos being the cosine between the ray and the plane
# normal, so the oracle reports per tile how close its own decisions came to
# eps in metres (margin_abs), and as the relative plane change that flips
# one (margin_cond = margin / max(r, 1 m) * cos; for a ray that misses the
# plane, the cosine).  A tile whose points all lie in one pixel column lies
# in a plane through the sensor: its fitted plane is seen edge-on (cos near
# 1e-5) and any rounding flips its decisions.
NEAR_EPS_ABS = 1e-5
NEAR_EPS_REL = 1e-5


def key_differences(gk, ok):
    """Key-frame tiles whose class or (covered tiles) mask differ between the
    GPU key frame `gk` (host dict) and the oracle key frame `ok`."""
    d = gk["cls"] != ok.cls
    d |= (gk["cls"] >= 2) & (ok.cls >= 2) & (gk["mask"] != ok.mask)
    return d


def key_affected(gk, ok):
    """Predicted-frame tiles whose key-frame plane may differ between the two
    sides: the key tile differs, or the key run covering the tile on either
    side holds a tile that differs (temporal fits take the key run's plane,
    temporal runs stay inside one key run)."""
    d = key_differences(gk, ok)
    T = len(d)
    aff = d.copy()
    for run_of, cls in ((gk["run_of"], gk["cls"]), (ok.run_of, ok.cls)):
        runs = {}
        for t in range(T):
            if cls[t] == 2 and run_of[t] >= 0:
                runs.setdefault(int(run_of[t]), []).append(t)
        for ts in runs.values():
            if d[ts].any():
                aff[ts] = True
    return aff


def explain_differences(g, o, rng_img, th, tw, tb, temporal=False, keys=None):
    """Tiles whose final class, final mask, run (first tile of the run
    covering them) or (predicted frames) temporal result differ between the
    GPU frame `g` (host dict with fit records) and the oracle frame `o`,
    sorted into: near-eps (a decision of the oracle on
    that tile lies within NEAR_EPS_ABS m of eps, or within a relative plane
    change NEAR_EPS_REL of flipping), key (predicted frames, `keys` = (GPU
    key host dict, oracle key frame): the key-frame plane the tile reuses
    differs between the sides), downstream (same tile row, inside a run on
    either side whose first tile or any earlier tile of the run is itself
    explained: growth tests the run's plane), and unexplained.  Also the
    largest plane discrepancy |t_g - t_o| / max(r, 1 m) over the pixels of
    tiles whose own fits agree."""
    T = len(o.cls)
    TC = rng_img.shape[1] // tw
    rec = g["tiles"]
    # runs on either side, per tile: first tile of its run
    def run_start(run_of, cls, sruns_s, pruns_s, T_):
        start = np.full(T_, -1, np.int64)
        for t in range(T_):
            ro = int(run_of[t])
            if cls[t] == 2 and ro >= 0:
                start[t] = (t // TC) * TC + int(sruns_s[ro])
            elif cls[t] == 3 and ro >= T_:
                start[t] = (t // TC) * TC + int(pruns_s[ro - T_])
        return start
    g_srun_s = g["sruns"]["s"]
    g_prun_s = g["pruns"]["s"]
    o_srun_s = np.zeros(T, np.int64)
    o_srun_s[:o.c.n_sruns] = o.srun_s
    o_prun_s = np.zeros(T, np.int64)
    o_prun_s[:o.c.n_pruns] = o.prun_s
    sg = run_start(g["run_of"], g["cls"], g_srun_s, g_prun_s, T)
    so = run_start(o.run_of, o.cls, o_srun_s, o_prun_s, T)
    diff = (g["cls"] != o.cls)
    cov = (o.cls >= 2) & (g["cls"] >= 2)
    diff |= cov & (g["mask"] != o.mask)
    diff |= cov & (sg != so)          # same class and mask, another run
    if temporal:
        diff |= rec["t_status"] != o.t_status
        both_t = (rec["t_status"] == 2) & (o.t_status == 2)
        diff |= both_t & (rec["t_mask"] != o.t_mask)
    near = diff & ((o.margin_abs <= NEAR_EPS_ABS) | (o.margin_cond <= NEAR_EPS_REL))
    keyd = np.zeros(T, bool)
    if temporal and keys is not None:
        keyd = diff & ~near & key_affected(keys[0], keys[1])
    cause = near | keyd
    # a tile inside a run (either side) that began at or before an explained
    # difference of its row follows from it: growth tests the run's plane,
    # and a run that ends elsewhere moves every later boundary of the row;
    # followed link by link until nothing changes
    down = np.zeros(T, bool)
    while True:
        known = cause | down
        grew = False
        for t in np.nonzero(diff & ~known)[0]:
            for st in (sg[t], so[t]):
                if st >= 0 and st < t and np.any(known[st:t]):
                    down[t] = True
                    grew = True
                    break
        if not grew:
            break
    unexplained = diff & ~cause & ~down
    # plane rounding actually seen: own fits with equal masks on both sides
    worst_rel = 0.0
    agree = (rec["status"] >= 4) & (o.own_status >= 4) & (rec["mask"] == o.own_mask)
    for t in np.nonzero(agree)[0][:400]:
        r = tile_ranges(rng_img, th, tw, t, TC)
        v = r > 0
        tg = _ray_t(tb, th, tw, t, TC, rec["axis"][t], rec["a"][t], rec["b"][t], rec["c"][t])
        to = _ray_t(tb, th, tw, t, TC, o.own_axis[t], o.own_abc[t][0], o.own_abc[t][1], o.own_abc[t][2])
        worst_rel = max(worst_rel, float(np.max(np.abs(tg[v] - to[v]) / np.maximum(r[v], 1.0))))
    return dict(differ=int(diff.sum()), near_eps=int(near.sum()), key=int(keyd.sum()), downstream=int(down.sum()),
                unexplained=int(unexplained.sum()), unexplained_tiles=[int(t) for t in np.nonzero(unexplained)[0][:10]],
                cls_agree=float(np.mean(g["cls"] == o.cls)), plane_rounding_rel=worst_rel)


def temporal_offsets_agree(g, o, key_o, key_g=None):
    """c' of tiles both sides fit temporally to the same pixels (and, with
    the GPU key frame `key_g`, against the same key-frame plane): the offset
    along the unit normal, |c'_g - c'_o| / |n_s| relative to max(|c'|, 1 m).
    Returns (tiles compared, worst relative difference)."""
    rec = g["tiles"]
    both = (rec["t_status"] == 2) & (o.t_status == 2) & (rec["t_mask"] == o.t_mask)
    if key_g is not None:
        both &= ~key_affected(key_g, key_o)
    worst = 0.0
    n = 0
    for t in np.nonzero(both)[0]:
        kr = int(key_o.run_of[t])
        _, s = unit_normal(key_o.srun_axis[kr], key_o.srun_abc[kr][0], key_o.srun_abc[kr][1])
        cg, co = float(rec["t_c"][t]) / s, float(o.t_c[t]) / s
        worst = max(worst, abs(cg - co) / max(abs(co), 1.0))
        n += 1
    return n, worst


def run_lists(g):
    """GPU spatial and temporal runs as sorted tuples (row, s, len, ...)."""
    sr = [(int(r), int(x["s"]), int(x["len"]), int(x["axis"])) for r, x in zip(g["srun_row"], g["srun_list"])]
    pr = [(int(r), int(x["s"]), int(x["len"]), int(x["krun"])) for r, x in zip(g["prun_row"], g["prun_list"])]
    return sr, pr


def oracle_run_lists(o, TC):
    sr = [(int(o.srun_row[i]), int(o.srun_s[i]), int(o.srun_len[i]), int(o.srun_axis[i])) for i in range(o.c.n_sruns)]
    pr = [(int(o.prun_row[i]), int(o.prun_s[i]), int(o.prun_len[i]), int(o.prun_krun[i]))
          for i in range(o.c.n_pruns)]
    return sr, pr

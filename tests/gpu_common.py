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


def compare_frame(orc, g, o, rng_img, tol_frac=0.005):
    """Compare one encoded frame: GPU host dict `g` vs oracle Frame `o`.
    Returns a dict of agreement statistics."""
    T = len(g["cls"])
    st = {}
    st["tiles"] = T
    st["cls_agree"] = float(np.mean(g["cls"] == o.cls))
    st["own_status_agree"] = float(np.mean(g["tiles"]["status"] == o.own_status))
    same_mask = (g["tiles"]["mask"] == o.own_mask) & (g["tiles"]["status"] >= 4) & (o.own_status >= 4)
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

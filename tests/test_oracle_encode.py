"""Pins of the oracle's encoder: total-least-squares planes and the ray-cast
test (Sec. III-C, Eq. (3)), per-tile refits, horizontal growth and the
[s, len, P] runs (Sec. III-C), temporal reuse with the offset free
(Sec. III-D), the residual quantiser, the Huffman size (Sec. III-A) and the
decoder.  Each test checks the oracle against something other than itself:
numpy's symmetric eigensolver, brute-force sampling, closed forms, a
textbook Huffman example, and scenes constructed so the answer is known."""
import heapq
import json
import math
import os

import numpy as np
import pytest

from paper_2008_06972_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- least squares
def test_tls_matches_numpy_eigh(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        n = int(rng.integers(3, 65))
        p = rng.normal(size=(n, 3)) * rng.uniform(0.01, 5, size=3) + rng.uniform(-80, 80, 3)
        nrm, c, ev, deg = orc.tls(p)
        mu = p.mean(0)
        w, V = np.linalg.eigh((p - mu).T @ (p - mu))
        assert np.allclose(ev, w, rtol=1e-9, atol=1e-9 * w[-1])
        if w[1] - w[0] > 1e-6 * w[2]:
            assert abs(abs(np.dot(nrm, V[:, 0])) - 1) < 1e-9
            assert abs(c - np.dot(nrm, mu)) < 1e-9 * max(1, np.abs(mu).max())


def test_tls_beats_sphere_sampling(orc):
    """The TLS normal minimises the sum of squared distances; no sampled
    direction of 1e5 on the sphere does better."""
    rng = np.random.default_rng(9)
    dirs = rng.normal(size=(100_000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    for _ in range(5):
        p = rng.normal(size=(12, 3)) * [2.0, 1.0, 0.2]
        nrm, c, ev, _ = orc.tls(p)
        q = p - p.mean(0)
        best = np.min(np.sum((q @ dirs.T) ** 2, axis=0))
        mine = np.sum((q @ nrm) ** 2)
        assert mine <= best * (1 + 1e-12)
        assert abs(mine - ev[0]) < 1e-9 * ev[2]


def test_tls_noiseless_plane_exact(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        c = rng.uniform(-50, 50)
        a = np.cross(n, [1, 0, 0] if abs(n[0]) < 0.9 else [0, 1, 0])
        a /= np.linalg.norm(a)
        b = np.cross(n, a)
        uv = rng.uniform(-3, 3, size=(16, 2))
        p = c * n + uv[:, :1] * a + uv[:, 1:] * b
        nrm, cc, ev, deg = orc.tls(p)
        s = np.sign(np.dot(nrm, n))
        assert np.max(np.abs(s * nrm - n)) < 1e-10
        assert abs(s * cc - c) < 1e-9 * max(1, abs(c))
        assert not deg


def test_tls_collinear_is_degenerate(orc):
    t = np.linspace(0, 1, 10)[:, None]
    p = np.array([1.0, 2.0, 3.0]) + t * np.array([0.3, -0.2, 0.9])
    assert orc.tls(p)[3]
    assert orc.tls(np.ones((5, 3)))[3]


# --------------------------------------------------------------- tile fixtures
def _plane_image(sensor, tb, planes_by_col):
    """Range image whose column block u0:u1 sees plane (n, c): ranges from the
    closed-form ray-plane intersection t = c / (n . d) along the oracle's FP32
    pixel directions."""
    d = tb.directions().astype(np.float64)
    img = np.zeros((sensor.H, sensor.W), np.float64)
    for (u0, u1, n, c) in planes_by_col:
        n = np.asarray(n, float)
        img[:, u0:u1] = c / (d[:, u0:u1] @ n)
    return img.astype(np.float32)


SMALL = synth.Sensor(4, 32, 3.0, -3.0, az0=0.4)   # 4 beams x 32 columns -> 1 x 8 tiles of 4x4


def test_noiseless_single_plane_one_run(orc):
    tb = orc.Tables.of(SMALL)
    # a wall x = 10 seen by columns whose centres face +x
    cols = np.nonzero(tb.ca > 0.2)[0]
    img = np.zeros((4, 32), np.float32)
    img[:, cols] = _plane_image(SMALL, tb, [(0, 32, [1, 0, 0], 10.0)])[:, cols]
    prm = orc.Params(eps=0.01, th=4, tw=4)
    f = orc.encode_key(img, tb, prm)
    covered = [t for t in range(8) if f.cls[t] == orc.CLS_SPATIAL]
    full = [t for t in range(8) if np.all(img[:, 4 * t:4 * t + 4] > 0)]
    assert set(full) <= set(covered)
    # every fully visible tile reproduced exactly by one plane x = 10
    for r in range(f.c.n_sruns):
        assert f.srun_axis[r] == 0
        assert abs(f.srun_abc[r][0]) < 1e-6 and abs(f.srun_abc[r][1]) < 1e-6
        assert abs(f.srun_abc[r][2] - 10.0) < 1e-5
    # contiguous visible tiles form a single run
    assert f.c.n_sruns == 1 + sum(1 for a, b in zip(covered, covered[1:]) if b != a + 1)
    assert f.n_res == 0
    dec = orc.decode(f, tb, prm)
    assert np.max(np.abs(dec - img)) < 1e-5


def test_two_planes_split_runs(orc):
    tb = orc.Tables.of(SMALL)
    c = np.nonzero(tb.ca > 0.5)[0]
    half = c[len(c) // 2 // 4 * 4]
    img = np.zeros((4, 32), np.float32)
    img[:, c] = _plane_image(SMALL, tb, [(0, half, [1, 0, 0], 10.0), (half, 32, [1, 0.3, 0], 12.0)])[:, c]
    prm = orc.Params(eps=0.005, th=4, tw=4)
    f = orc.encode_key(img, tb, prm)
    assert f.c.n_sruns >= 2
    # no run crosses the plane boundary at column `half`
    for r in range(f.c.n_sruns):
        s0, l0 = f.srun_s[r] * 4, f.srun_len[r] * 4
        assert s0 + l0 <= half or s0 >= half
    dec = orc.decode(f, tb, prm)
    assert np.max(np.abs(dec - img)) < 1e-5


def test_refit_drops_outlier_in_two_fits(orc):
    """15 coplanar points + 1 off the plane by 10 cm along its ray: the first
    fit includes it, the refit on the reproduced points drops it, the third
    fit confirms (converged)."""
    sensor = synth.Sensor(4, 64, 2.0, -2.0, az0=0.2)
    tb = orc.Tables.of(sensor)
    img = _plane_image(sensor, tb, [(0, 64, [1, 0.1, 0.05], 15.0)])
    img[2, 1] += np.float32(0.10)
    keep = np.zeros_like(img)
    keep[:, :4] = img[:, :4]
    prm = orc.Params(eps=0.02, th=4, tw=4)
    f = orc.encode_key(keep, tb, prm)
    assert f.own_status[0] == orc.ACCEPTED
    m = int(f.own_mask[0])
    assert m == (0xFFFF & ~(1 << (2 * 4 + 1)))
    assert f.own_iters[0] in (2, 3)
    assert f.n_res == 1
    dec = orc.decode(f, tb, prm)
    assert np.max(np.abs(dec[:, :4].astype(np.float64) - keep[:, :4])) <= 0.02


def test_unfit_tile_breaks_run(orc):
    sensor = synth.Sensor(4, 64, 3.0, -3.0)
    tb = orc.Tables.of(sensor)
    img = _plane_image(sensor, tb, [(24, 40, [1, 0, 0], 10.0)])      # tiles 6..9 see the wall
    img[:, :24] = 0
    img[:, 40:] = 0
    rng = np.random.default_rng(0)
    img[:, 32:36] = rng.uniform(2, 30, (4, 4)).astype(np.float32)   # tile 8: random ranges
    prm = orc.Params(eps=0.01, th=4, tw=4)
    f = orc.encode_key(img, tb, prm)
    assert list(f.cls[6:10]) == [orc.CLS_SPATIAL, orc.CLS_SPATIAL, orc.CLS_UNFIT, orc.CLS_SPATIAL]
    assert f.run_of[6] == f.run_of[7] != f.run_of[9]
    assert f.c.n_sruns == 2 and f.n_res == 16


def test_empty_tile_extends_open_run(orc):
    sensor = synth.Sensor(4, 64, 3.0, -3.0)
    tb = orc.Tables.of(sensor)
    img = _plane_image(sensor, tb, [(24, 40, [1, 0, 0], 10.0)])
    img[:, :24] = 0
    img[:, 40:] = 0
    img[:, 32:36] = 0                                                  # tile 8 empty
    prm = orc.Params(eps=0.01, th=4, tw=4)
    f = orc.encode_key(img, tb, prm)
    assert list(f.cls[6:10]) == [orc.CLS_SPATIAL] * 4
    # empty tiles need no points, so the open run carries on to the row's end
    assert f.c.n_sruns == 1 and f.srun_s[0] == 6 and f.srun_len[0] == 16 - 6
    assert f.cls[5] == orc.CLS_EMPTY and f.cls[10] == orc.CLS_SPATIAL
    assert f.n_res == 0


# ------------------------------------------------------------------ temporal
def test_identity_transform_reuses_every_plane(orc):
    """A predicted frame equal to the key frame: every plane-coded tile is
    reused with c' = c (the mean of p_k + a p_k1 + b p_k2 over points that
    the plane reproduces), the temporal runs follow the key runs, and only
    the key frame's residual pixels remain."""
    s = synth.SENSORS["c1"]
    tb = orc.Tables.of(s)
    pts, _, _ = synth.make_frame(s, "c1", 1003)
    img, _, _ = orc.project(pts, tb)
    prm = orc.Params(eps=0.02, th=4, tw=4)
    k = orc.encode_key(img, tb, prm)
    p = orc.encode_pred(k, img, tb, prm)
    cov = k.cls == orc.CLS_SPATIAL
    temporal = p.cls == orc.CLS_TEMPORAL
    # tiles reused: all key tiles whose own temporal fit succeeds
    assert temporal.sum() >= 0.9 * cov.sum()
    assert not np.any(temporal & ~cov)
    for r in range(p.c.n_pruns):
        kr = p.prun_krun[r]
        assert abs(p.prun_c[r] - k.srun_abc[kr][2]) <= 2e-3 * max(1.0, abs(k.srun_abc[kr][2]))
    dec = orc.decode(p, tb, prm, key=k)
    v = img > 0
    assert np.max(np.abs(dec[v].astype(np.float64) - img[v])) <= prm.eps


def test_offset_shift_along_normal(orc):
    """Moving a plane by delta along its unit normal n changes the stored offset
    by delta / n_k (stored form p_k + a p_k1 + b p_k2 = c / n_k)."""
    sensor = synth.Sensor(4, 64, 2.0, -2.0, az0=0.2)
    tb = orc.Tables.of(sensor)
    n = np.array([1.0, 0.2, 0.05])
    n /= np.linalg.norm(n)
    cols = np.nonzero(tb.ca > 0.5)[0]
    base = np.zeros((4, 64), np.float32)
    base[:, cols] = _plane_image(sensor, tb, [(0, 64, n, 12.0)])[:, cols]
    moved = np.zeros_like(base)
    delta = 0.35
    moved[:, cols] = _plane_image(sensor, tb, [(0, 64, n, 12.0 + delta)])[:, cols]
    prm = orc.Params(eps=0.01, th=4, tw=4)
    k = orc.encode_key(base, tb, prm)
    p = orc.encode_pred(k, moved, tb, prm)
    assert p.c.n_pruns >= 1
    for r in range(p.c.n_pruns):
        kr = p.prun_krun[r]
        assert k.srun_axis[kr] == 0
        assert abs((p.prun_c[r] - k.srun_abc[kr][2]) - delta / n[0]) < 2e-4


# ------------------------------------------------------------------ quantiser
def test_quantiser_bound_and_rounding(orc):
    """Residual pixels decode as q * step with step = 2 eps (1 - 2^-8).  The
    margin eps 2^-8 covers the FP32 rounding (about 2e-7 r) up to
    r = eps 2^-8 / 2e-7 (about 19500 eps: 195 m at 1 cm, 390 m at 2 cm); over
    that range the error never exceeds eps and q is the nearest integer to
    r / step (exact arithmetic, away from ties)."""
    for eps in (0.01, 0.02):
        sensor = synth.Sensor(8, 4096, 10.0, -10.0)
        tb = orc.Tables.of(sensor)
        rng = np.random.default_rng(2)
        img = rng.uniform(0.05, 19000 * eps, size=(8, 4096)).astype(np.float32)
        img[:, ::2] = rng.uniform(0.05, 5.0, size=(8, 2048)).astype(np.float32)   # dense small values
        prm = orc.Params(eps=eps, th=4, tw=4, min_pts=64)   # min_pts > tile size: every pixel is a residual
        f = orc.encode_key(img, tb, prm)
        assert f.n_res == img.size and f.range_error == 0
        step = np.float32(2 * eps * (1 - 2 ** -8))
        dec = orc.decode(f, tb, prm)
        err = np.abs(dec.astype(np.float64) - img.astype(np.float64))
        assert err.max() <= eps
        exact = img.astype(np.float64).ravel() / float(step)
        frac = np.abs(exact - np.round(exact))
        ok = np.abs(frac - 0.5) > 2e-7 * exact + 1e-6   # FP32 product error: about 1.2e-7 q
        assert np.array_equal(f.codes[ok], np.round(exact[ok]).astype(np.uint16))


def test_quantiser_flags_out_of_range(orc):
    sensor = synth.Sensor(4, 16, 10.0, -10.0)
    tb = orc.Tables.of(sensor)
    img = np.full((4, 16), 5.0, np.float32)
    img[0, 0] = 2000.0          # beyond 65535 steps at eps = 1 cm
    prm = orc.Params(eps=0.01, th=4, tw=4, min_pts=64)
    assert orc.encode_key(img, tb, prm).range_error == 1


# ------------------------------------------------------------------ Huffman
def _textbook_huffman_lengths(freq):
    """Huffman's construction with a heap of (weight, tiebreak, symbols)."""
    heap = [(w, i, [s]) for i, (s, w) in enumerate(freq.items()) if w > 0]
    heapq.heapify(heap)
    depth = {s: 0 for s in freq}
    k = len(heap)
    while len(heap) > 1:
        w1, _, s1 = heapq.heappop(heap)
        w2, _, s2 = heapq.heappop(heap)
        for s in s1 + s2:
            depth[s] += 1
        heapq.heappush(heap, (w1 + w2, k, s1 + s2))
        k += 1
    return depth


def test_huffman_textbook_example(orc):
    g = json.load(open(os.path.join(GOLDEN, "huffman_textbook.json")))
    hist = np.zeros(256, np.uint32)
    for i, (s, w) in enumerate(g["frequencies"].items()):
        hist[i] = w
    assert orc.huffman_bits(hist) == g["optimal_cost_bits"]
    lengths = _textbook_huffman_lengths(g["frequencies"])
    assert sum(g["frequencies"][s] * lengths[s] for s in lengths) == g["optimal_cost_bits"]


def test_huffman_random_vs_textbook_and_entropy(orc):
    rng = np.random.default_rng(4)
    for _ in range(100):
        k = int(rng.integers(1, 257))
        hist = np.zeros(256, np.uint32)
        hist[rng.choice(256, k, replace=False)] = rng.integers(1, 10_000, k)
        bits = orc.huffman_bits(hist)
        freq = {i: int(hist[i]) for i in range(256) if hist[i]}
        n = sum(freq.values())
        if len(freq) == 1:
            assert bits == n
            continue
        L = _textbook_huffman_lengths(freq)
        assert bits == sum(freq[s] * L[s] for s in freq)
        p = np.array(list(freq.values()), float) / n
        H = -np.sum(p * np.log2(p))
        assert H * n - 1e-6 <= bits < (H + 1) * n
    assert orc.huffman_bits(np.zeros(256, np.uint32)) == 0


# -------------------------------------------------------- streams and decode
@pytest.mark.parametrize("name,tw", [("c1", 4), ("c2", 8)])
def test_key_frame_roundtrip_and_stream_format(orc, name, tw):
    s = synth.SENSORS[name]
    tb = orc.Tables.of(s)
    pts, _, _ = synth.make_frame(s, name, {"c1": 1000, "c2": 2000}[name])
    img, _, _ = orc.project(pts, tb)
    prm = orc.Params(eps=0.02, th=4, tw=tw)
    f = orc.encode_key(img, tb, prm)
    v = img > 0
    dec = orc.decode(f, tb, prm)
    assert np.all(dec[~v] == 0)
    assert np.max(np.abs(dec[v].astype(np.float64) - img[v])) <= prm.eps   # eps invariant, 100 %
    # OCC: one bit per pixel
    assert f.stream_bytes[0] == (s.H * s.W + 7) // 8
    # RES: two bytes per residual pixel; residual pixels = valid minus mask bits
    covered = (f.cls == orc.CLS_SPATIAL)
    mask_bits = sum(bin(int(m)).count("1") for m in f.mask[covered])
    assert f.n_res == v.sum() - mask_bits
    assert f.stream_bytes[3] == 2 * f.n_res
    # MASK: ceil(valid/8) bytes per plane-coded tile
    vt = v.reshape(s.H // 4, 4, s.W // tw, tw).sum(axis=(1, 3)).ravel()
    assert f.stream_bytes[2] == int(np.sum((vt[covered] + 7) // 8))
    # RUN: varint(count) per row, varint(gap) varint(len) u8 + 3 f32 per run
    def vlen(x):
        return 1 if x < 128 else 1 + vlen(x >> 7)
    nb = 0
    for tr in range(f.TR):
        rows = [r for r in range(f.c.n_sruns) if f.srun_row[r] == tr]
        nb += vlen(len(rows))
        prev = 0
        for r in rows:
            nb += vlen(int(f.srun_s[r]) - prev) + vlen(int(f.srun_len[r])) + 13
            prev = int(f.srun_s[r] + f.srun_len[r])
    assert f.stream_bytes[1] == nb
    # every tile in a run, and runs tile the covered set exactly
    cov = np.zeros(f.TR * f.TC, bool)
    for r in range(f.c.n_sruns):
        t0 = f.srun_row[r] * f.TC + f.srun_s[r]
        assert not cov[t0:t0 + f.srun_len[r]].any()
        cov[t0:t0 + f.srun_len[r]] = True
    assert np.array_equal(cov, covered)
    # size = header + per stream (ceil(bits/8) + table)
    want = 112 + sum((b + 7) // 8 + 128 for b, n in zip(f.coded_bits, f.stream_bytes) if n)
    assert f.size_bytes == want
    for k in range(4):
        assert f.coded_bits[k] == orc.huffman_bits(f.hist[k])


def test_sequence_roundtrip_eps_invariant(orc):
    s = synth.SENSORS["c1"]
    tb = orc.Tables.of(s)
    seq = synth.make_sequence(s, "c1", 3000, n_frames=10)
    prm = orc.Params(eps=0.02, th=4, tw=4)
    imgs = [orc.project(f, tb, None if i == seq.key_index else seq.transforms[i])[0]
            for i, f in enumerate(seq.frames)]
    k = orc.encode_key(imgs[seq.key_index], tb, prm)
    ntemp = 0
    for i, img in enumerate(imgs):
        if i == seq.key_index:
            continue
        p = orc.encode_pred(k, img, tb, prm)
        ntemp += int(np.sum(p.cls == orc.CLS_TEMPORAL))
        dec = orc.decode(p, tb, prm, key=k)
        v = img > 0
        assert np.all(dec[~v] == 0)
        assert np.max(np.abs(dec[v].astype(np.float64) - img[v])) <= prm.eps
    assert ntemp > 0
    total, sizes, fin = orc.encode_sequences(seq.frames, seq.transforms, seq.key_index, 1, 10, tb, prm)
    assert fin == sum(len(f) for f in seq.frames)
    assert total == int(sizes.sum())
    assert sizes[seq.key_index] == k.size_bytes


def test_temporal_runs_nest_inside_key_runs(orc):
    """Sec. III-D reuses the key frame's fitted planes: a temporal run takes
    its normal from one key run, so it may not grow into the neighbouring
    key run even where that run's plane would also reproduce the tiles.
    Key frame (one 4 x 4-tile row): a wall x = 10 m on tiles 0-3 and a
    parallel wall x = 12 m on tiles 4-7 (two key runs, the second carried to
    the row's end over empty tiles).  Predicted frame: one wall x = 11 m on
    tiles 0-7.  Worked by hand: every non-empty tile is reproduced with its
    key run's normal (1, 0, 0) and c' = 11, yet the temporal runs must stop
    where the key run changes, so there are two temporal runs [0, 4) and
    [4, 64) with c' = 11 (one run [0, 64) if nesting were ignored)."""
    sensor = synth.Sensor(4, 256, 2.0, -2.0, az0=22.5 * math.pi / 180)
    tb = orc.Tables.of(sensor)
    key = _plane_image(sensor, tb, [(0, 16, [1, 0, 0], 10.0), (16, 32, [1, 0, 0], 12.0)])
    key[:, 32:] = 0
    pred = _plane_image(sensor, tb, [(0, 32, [1, 0, 0], 11.0)])
    pred[:, 32:] = 0
    prm = orc.Params(eps=0.01, th=4, tw=4)
    k = orc.encode_key(key, tb, prm)
    assert k.c.n_sruns == 2 and list(k.srun_s) == [0, 4] and list(k.srun_len) == [4, 60]
    assert [round(float(c), 4) for c in k.srun_abc[:, 2]] == [10.0, 12.0]
    p = orc.encode_pred(k, pred, tb, prm)
    assert p.c.n_pruns == 2
    assert list(p.prun_s) == [0, 4] and list(p.prun_len) == [4, 60]
    assert list(p.prun_krun) == [0, 1]
    assert np.allclose(p.prun_c, 11.0, atol=1e-5)
    assert p.c.n_sruns == 0 and p.n_res == 0
    assert np.all(p.cls == orc.CLS_TEMPORAL)
    dec = orc.decode(p, tb, prm, key=k)
    v = pred > 0
    assert np.max(np.abs(dec[v].astype(np.float64) - pred[v])) <= prm.eps


# ----------------------------------------------------------- decode to points
def test_decoded_points_on_pixel_rays_within_eps(orc):
    """Key frame: every decoded point lies on its pixel-centre ray at the
    decoded range, so |p_hat| = r_hat, and (the generator places points on
    the same pixel-centre rays) each is within eps of the source point the
    projection kept for its pixel, up to the FP32 rounding of the ray
    direction (about 1e-7 r)."""
    s = synth.SENSORS["c1"]
    tb = orc.Tables.of(s)
    pts, _, _ = synth.make_frame(s, "c1", 1004)
    img, idx, _ = orc.project(pts, tb)
    prm = orc.Params(eps=0.02, th=4, tw=4)
    f = orc.encode_key(img, tb, prm)
    r_hat = orc.decode(f, tb, prm).astype(np.float64)
    P = orc.decode_points(f, tb, prm)
    v = img > 0
    assert np.all(P[~v] == 0)
    assert np.allclose(np.linalg.norm(P[v], axis=1), r_hat[v], rtol=1e-6, atol=0)
    src = pts[idx[v]].astype(np.float64)
    err = np.linalg.norm(P[v] - src, axis=1)
    assert err.max() <= prm.eps + 2e-7 * np.abs(r_hat[v]).max()


def test_decoded_points_back_in_frame_coordinates(orc):
    """Predicted frame: with its transform M = [R | T] (Eq. (6)) the decoded
    points go back to the frame's own coordinates by R^T (p - T); applying M
    again gives the key-frame points (closed-form inverse of a rigid
    transform), and the distances to the sensor origin of the key frame are
    kept (|R q + T| = |p|)."""
    s = synth.SENSORS["c1"]
    tb = orc.Tables.of(s)
    seq = synth.make_sequence(s, "c1", 3005, n_frames=3, key_index=1)
    prm = orc.Params(eps=0.02, th=4, tw=4)
    rk, _, _ = orc.project(seq.frames[1], tb)
    k = orc.encode_key(rk, tb, prm)
    M = np.asarray(seq.transforms[0], np.float64)
    r0, _, _ = orc.project(seq.frames[0], tb, seq.transforms[0])
    p = orc.encode_pred(k, r0, tb, prm)
    Pk = orc.decode_points(p, tb, prm, key=k)
    Pf = orc.decode_points(p, tb, prm, key=k, M=M)
    v = r0 > 0
    back = Pf[v] @ M[:3, :3].T + M[:3, 3]
    assert np.allclose(back, Pk[v], rtol=0, atol=1e-9 * max(1.0, np.abs(Pk).max()))
    assert np.all(Pf[~v] == 0)
    # a rotation keeps lengths: |q| for q = R^T (p - T) equals |p - T| (R is
    # orthogonal to the FP32 rounding of its entries, about 1e-7)
    assert np.allclose(np.linalg.norm(Pf[v], axis=1), np.linalg.norm(Pk[v] - M[:3, 3], axis=1), rtol=1e-6, atol=0)


# ------------------------------------------------------ decision margins
@pytest.mark.parametrize("normal,c", [((1.0, 0.0, 0.0), 10.0), ((0.2, 0.98, 0.0), 5.0)])
def test_margin_diagnostics_on_a_noiseless_wall(orc, normal, c):
    """The per-tile margins are diagnostics of how close the keep-or-drop
    test |t - r| <= eps came to flipping.  On a noiseless plane every point is
    reproduced with |t - r| at the level of FP32 rounding, so over a fully
    visible tile: margin_abs = eps (to that rounding), margin_rel = eps /
    max(r, 1) at the tile's farthest point, and margin_cond = the smallest
    eps |n . d| / max(r, 1) over the tile's pixels, n . d being the cosine
    between the pixel's ray and the wall's unit normal (face-on and oblique
    walls)."""
    sensor = synth.Sensor(4, 64, 3.0, -3.0, az0=0.4)
    tb = orc.Tables.of(sensor)
    n = np.asarray(normal, float)
    n /= np.linalg.norm(n)
    d = tb.directions().astype(np.float64)
    nd = d @ n
    img = _plane_image(sensor, tb, [(0, sensor.W, n, c)])
    ok = np.all((nd > 0.1) & (img > 0) & (img < 60.0), axis=0)
    img[:, ~ok] = 0
    prm = orc.Params(eps=0.01, th=4, tw=4)
    f = orc.encode_key(img, tb, prm)
    r = img.astype(np.float64)
    checked = 0
    for t in range(sensor.W // 4):
        cols = slice(4 * t, 4 * t + 4)
        if not np.all(ok[cols]) or f.cls[t] != orc.CLS_SPATIAL:
            continue
        checked += 1
        rt, ct = r[:, cols], np.abs(nd[:, cols])
        assert abs(f.margin_abs[t] - prm.eps) <= 1e-4 * prm.eps * max(1.0, rt.max())
        assert f.margin_abs[t] <= prm.eps
        assert f.margin_rel[t] == pytest.approx(prm.eps / np.maximum(rt, 1).max(), rel=2e-3)
        assert f.margin_cond[t] == pytest.approx((prm.eps * ct / np.maximum(rt, 1)).min(), rel=2e-3)
    assert checked >= 3

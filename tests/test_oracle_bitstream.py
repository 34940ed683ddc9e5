"""Pins of the oracle's entropy-coded bitstream (Sec. III-A): code lengths
against brute-force optimal prefix codes on small alphabets and against the
independent heap construction of the optimal cost, the Kraft equality, the
15-bit limit, canonical code words, a hand-worked bitstream, and round trips
of encoded frames."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2008_06972_amd import synth


def _hist(rng, kind):
    if kind == 0:
        return rng.integers(0, 1000, 256)
    if kind == 1:
        return np.where(rng.random(256) < 0.9, 0, rng.integers(1, 50, 256))
    if kind == 2:
        return rng.integers(0, 3, 256)
    return rng.geometric(0.05, 256) * (rng.random(256) < 0.5)


def _huffman_depth(h):
    """Depth of an optimal (unlimited) Huffman tree, by heapq."""
    items = [(int(c), i, 0) for i, c in enumerate(h) if c]
    if len(items) < 2:
        return len(items)
    import heapq
    heapq.heapify(items)
    k = 256
    while len(items) > 1:
        a, b = heapq.heappop(items), heapq.heappop(items)
        heapq.heappush(items, (a[0] + b[0], k, max(a[2], b[2]) + 1))
        k += 1
    return items[0][2]


def _kraft_units(lengths):
    """sum of 2^(15 - L) over used symbols (2^15 for a full code)"""
    L = lengths[lengths > 0].astype(np.int64)
    return int((1 << (15 - L)).sum())


@pytest.mark.parametrize("kind", range(4))
def test_lengths_reach_the_heap_cost_and_fill_the_code(kind):
    rng = np.random.default_rng(10 + kind)
    for _ in range(40):
        h = _hist(rng, kind).astype(np.uint32)
        if (h > 0).sum() < 2:
            continue
        ln = oracle.code_lengths(h)
        assert ln.max() <= 15 and np.all((ln > 0) == (h > 0))
        assert _kraft_units(ln) == 1 << 15
        cost = int((h.astype(np.int64) * ln).sum())
        opt = oracle.huffman_bits(h)
        assert cost >= opt
        if _huffman_depth(h) <= 15:                    # no limiting: the optimum itself
            assert cost == opt


def test_lengths_are_optimal_by_brute_force():
    rng = np.random.default_rng(3)
    for m in range(2, 7):
        for _ in range(15):
            counts = rng.integers(1, 60, m)
            h = np.zeros(256, np.uint32)
            syms = rng.choice(256, m, replace=False)
            h[syms] = counts
            ln = oracle.code_lengths(h)
            best = None
            for L in itertools.product(range(1, m + 1), repeat=m):
                if sum(2.0 ** -x for x in L) <= 1.0:
                    c = sum(int(a) * b for a, b in zip(counts, L))
                    best = c if best is None else min(best, c)
            assert int((h.astype(np.int64) * ln).sum()) == best


def test_single_symbol_and_empty():
    h = np.zeros(256, np.uint32)
    assert not oracle.code_lengths(h).any()
    h[77] = 5
    ln = oracle.code_lengths(h)
    assert ln[77] == 1 and ln.sum() == 1


def test_length_limit_on_a_deep_tree():
    # Fibonacci counts make the Huffman tree a chain 30 levels deep
    f = [1, 1]
    while len(f) < 30:
        f.append(f[-1] + f[-2])
    h = np.zeros(256, np.uint32)
    h[:30] = f
    ln = oracle.code_lengths(h)
    assert ln.max() == 15 and _kraft_units(ln) == 1 << 15
    assert int((h.astype(np.int64) * ln).sum()) >= oracle.huffman_bits(h)
    # more frequent symbols never get longer codes
    order = np.argsort(-h[:30], kind="stable")
    assert np.all(np.diff(ln[order].astype(int)) >= 0)


def test_canonical_codes_are_prefix_free_and_ordered():
    rng = np.random.default_rng(4)
    for kind in range(4):
        h = _hist(rng, kind).astype(np.uint32)
        ln = oracle.code_lengths(h)
        code = oracle.canonical_codes(ln)
        used = [s for s in range(256) if ln[s]]
        words = {s: format(int(code[s]), "0%db" % int(ln[s])) for s in used}
        assert len(set(words.values())) == len(used)
        for a in used:
            for b in used:
                if a != b:
                    assert not words[b].startswith(words[a])
        # canonical: by (length, symbol) the left-aligned values increase
        keys = sorted(used, key=lambda s: (int(ln[s]), s))
        vals = [int(code[s]) << (15 - int(ln[s])) for s in keys]
        assert vals == sorted(vals)


def _frame_with_streams(streams, H=8, W=32):
    prm = oracle.Params(th=4, tw=8)
    f = oracle.Frame(H, W, prm)
    for q, b in enumerate(streams):
        b = np.asarray(b, np.uint8)
        f.sbufs[q][: len(b)] = b
        f.c.stream_bytes[q] = len(b)
        f.arrays["hist"][256 * q: 256 * (q + 1)] = np.bincount(b, minlength=256)
    return f, prm


def test_hand_worked_bitstream():
    # RUN stream "3 3 3 9": lengths 1 and 1; canonical codes 3 -> 0, 9 -> 1;
    # payload bits 0001 -> one byte 0x10.  Header: 64 bytes of fields, then
    # the transform (here a translation by (1, -2, 0.5)) as 12 FP32.
    f, prm = _frame_with_streams([[], [3, 3, 3, 9], [], []])
    M = np.eye(4, dtype=np.float32)
    M[:3, 3] = [1.0, -2.0, 0.5]
    data = oracle.pack(f, 1, prm, M)
    assert len(data) == 112 + 128 + 1
    assert data[:4] == b"PCC1" and data[4] == 1
    assert int.from_bytes(data[12 + 8: 12 + 16], "little") == 4      # RUN stream bytes
    assert np.array_equal(np.frombuffer(data[64:112], "<f4"), [1, 0, 0, 1, 0, 1, 0, -2, 0, 0, 1, 0.5])
    table = np.frombuffer(data[112:240], np.uint8)
    # symbols 3 and 9 are odd: high nibbles of bytes 1 and 4
    assert table[1] == 0x10 and table[4] == 0x10 and int(table.sum()) == 0x20
    assert data[240] == 0x10
    streams, Mb = oracle.unpack(data, with_transform=True)
    assert [list(s) for s in streams] == [[], [3, 3, 3, 9], [], []]
    assert np.array_equal(Mb, M[:3].ravel())
    # no transform given: identity
    assert np.array_equal(np.frombuffer(oracle.pack(f, 0, prm)[64:112], "<f4"), np.eye(4, dtype=np.float32)[:3].ravel())


def test_round_trip_of_random_streams():
    rng = np.random.default_rng(5)
    for _ in range(10):
        streams = [rng.integers(0, rng.integers(1, 256), rng.integers(0, 3000)).astype(np.uint8) for _ in range(4)]
        f, prm = _frame_with_streams(streams, H=64, W=1024)
        data = oracle.pack(f, 1, prm)
        back = oracle.unpack(data)
        for a, b in zip(streams, back):
            assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def encoded():
    s = synth.SENSORS["c1"]
    tb = oracle.Tables.of(s)
    prm = oracle.Params(eps=0.02, th=4, tw=4)
    seq = synth.make_sequence(s, "c1", 3020, n_frames=3, key_index=1, shuffle=True)
    rk, _, _ = oracle.project(seq.frames[1], tb)
    key = oracle.encode_key(rk, tb, prm)
    rp, _, _ = oracle.project(seq.frames[2], tb, seq.transforms[2])
    pred = oracle.encode_pred(key, rp, tb, prm)
    return dict(prm=prm, key=key, pred=pred, rk=rk, rp=rp)


def zigzag_row_deltas(codes, rows):
    """RES bytes written out: per image row, each code's difference (mod
    2^16) from the row's previous residual code, zigzag mapped, u16 LE."""
    out = np.zeros(len(codes), np.uint16)
    prev, last_row = 0, -1
    for k, (c, r) in enumerate(zip(codes.astype(np.int64), rows)):
        if r != last_row:
            prev, last_row = 0, r
        d = (int(c) - prev) & 0xFFFF
        d = d - 0x10000 if d >= 0x8000 else d
        out[k] = ((d << 1) ^ (-1 if d < 0 else 0)) & 0xFFFF
        prev = int(c)
    return out.astype("<u2").view(np.uint8)


def residual_rows(f, rng, th, tw):
    """Image row of each residual code (raster order) of an oracle frame."""
    H, W = rng.shape
    res = rng > 0
    TC = W // tw
    for t in range(len(f.cls)):
        if f.cls[t] in (oracle.CLS_SPATIAL, oracle.CLS_TEMPORAL):
            tr, tc = divmod(t, TC)
            m = int(f.mask[t])
            for j in range(th * tw):
                if (m >> j) & 1:
                    res[tr * th + j // tw, tc * tw + j % tw] = False
    return np.nonzero(res)[0]


def test_residual_prediction_hand_worked():
    # 4 x 32 sensor, 4x8 tiles, too few points for any fit: every point is a
    # residual.  Row 0 codes 100, 103, 98 -> differences 100, 3, -5 -> zigzag
    # 200, 6, 9; row 1 codes 65000, 10 -> 65000 (as -536: 1071), then
    # 10 - 65000 = 546 (mod 2^16) -> 1092.
    H, W = 4, 32
    tb = oracle.Tables(H, W, np.radians(np.array([3.0, 1.0, -1.0, -3.0])), 0.0)
    prm = oracle.Params(eps=0.02, th=4, tw=8)
    step = np.float32(2 * 0.02 * (1 - 2.0 ** -8))
    img = np.zeros((H, W), np.float32)
    for (v, u), c in {(0, 1): 100, (0, 5): 103, (0, 20): 98, (1, 3): 65000, (1, 30): 10}.items():
        img[v, u] = np.float32(c) * step
    f = oracle.encode_key(img, tb, prm)
    assert f.n_res == 5 and list(f.codes) == [100, 103, 98, 65000, 10]
    res = f.streams()[3]
    assert list(res.view("<u2")) == [200, 6, 9, 1071, 1092]
    assert np.array_equal(res, zigzag_row_deltas(f.codes, [0, 0, 0, 1, 1]))


def test_streams_match_histograms_and_sources(encoded):
    prm = encoded["prm"]
    for name, rng in (("key", encoded["rk"]), ("pred", encoded["rp"])):
        f = encoded[name]
        st = f.streams()
        for q in range(4):
            assert len(st[q]) == f.stream_bytes[q]
            assert np.array_equal(np.bincount(st[q], minlength=256), f.hist[q])
        assert np.array_equal(st[0], np.packbits((rng > 0).ravel(), bitorder="little"))
        rows = residual_rows(f, rng, prm.th, prm.tw)
        assert np.array_equal(st[3], zigzag_row_deltas(f.codes, rows))


def test_frame_round_trip_and_size(encoded):
    prm = encoded["prm"]
    for kind, name in ((0, "key"), (1, "pred")):
        f = encoded[name]
        data = oracle.pack(f, kind, prm)
        back = oracle.unpack(data)
        for a, b in zip(f.streams(), back):
            assert np.array_equal(a, b)
        # exact accounting; equal to the size model when no code exceeds 15 bits
        want = oracle.HEADER_BYTES
        deep = False
        for q in range(4):
            if f.stream_bytes[q] == 0:
                continue
            ln = oracle.code_lengths(f.hist[q])
            bits = int((f.hist[q].astype(np.int64) * ln).sum())
            want += 128 + (bits + 7) // 8
            deep |= bits != f.coded_bits[q]
        assert len(data) == want
        if not deep:
            assert len(data) == f.size_bytes


def test_unpack_rejects_malformed(encoded):
    data = oracle.pack(encoded["key"], 0, encoded["prm"])
    with pytest.raises(ValueError):
        oracle.unpack(data[:40])                           # shorter than the header
    with pytest.raises(ValueError):
        oracle.unpack(b"XXXX" + data[4:])                  # magic
    with pytest.raises(ValueError):
        oracle.unpack(data[:-5])                           # payload cut short

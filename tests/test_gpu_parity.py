"""GPU parity: the HIP path through the C ABI against the oracle, on the same
seeded inputs.  Projection indices, ranges and residual codes must agree bit
for bit; planes within 1e-4 (normal angle in rad, offset relative to
max(|c|, 1 m)) where both sides keep the same pixels; the compressed size
within 0.5 %; every decoded pixel within eps of its source (100 %)."""
import sys

import numpy as np
import pytest

from paper_2008_06972_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_06972_amd import pcc  # noqa: E402
import oracle  # noqa: E402
from gpu_common import compare_frame, residual_codes_agree, run_gpu_sequence  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def own_range(tb, pts, M, g):
    """The oracle's own projection of the points a GPU frame was made from;
    the projection parity makes it bit-identical to the GPU's range image, so
    both encoders start from the same input without GPU output entering the
    oracle."""
    r, _, _ = oracle.project(np.asarray(pts, np.float32), tb, M)
    assert np.array_equal(r, g["range"])
    return r


@pytest.fixture(scope="module")
def ctx_factory():
    made = []

    def make(*sensors):
        c = pcc.Context(list(sensors))
        made.append(c)
        return c
    yield make
    for c in made:
        c.close()


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_sensor_tables_bitwise(ctx_factory, name):
    s = synth.SENSORS[name]
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    g = pcc.pc_sensor_tables(ctx.h, S)
    o = oracle.Tables.of(s)
    for k in ("cut", "ebx", "eby", "ce", "se", "ca", "sa"):
        assert np.array_equal(g[k].view(np.uint32), getattr(o, k).view(np.uint32)), k


def _project_both(ctx, S, tb, pts, M=None):
    xyz = torch.from_numpy(np.ascontiguousarray(pts)).to(DEV)
    rng = torch.empty(S.H, S.W, dtype=torch.float32, device=DEV)
    idx = torch.empty(S.H, S.W, dtype=torch.int32, device=DEV)
    st = torch.zeros(5, dtype=torch.int64, device=DEV)
    pcc.pc_project(ctx.h, xyz, len(pts), M, S, rng, idx, st)
    torch.cuda.synchronize()
    r_o, i_o, s_o = oracle.project(pts, tb, M)
    return (rng.cpu().numpy(), idx.cpu().numpy(), st.cpu().numpy()), (r_o, i_o, s_o)


@pytest.mark.parametrize("name,seed", [("c1", 1000), ("c2", 2000)])
def test_projection_bit_exact(ctx_factory, name, seed):
    s = synth.SENSORS[name]
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    tb = oracle.Tables.of(s)
    pts, _, _ = synth.make_frame(s, name, seed)
    pts = pts[np.random.default_rng(seed).permutation(len(pts))]
    say("projection", name, len(pts))
    (rg, ig, sg), (ro, io, so) = _project_both(ctx, S, tb, pts)
    assert np.array_equal(rg.view(np.uint32), ro.view(np.uint32))
    assert np.array_equal(ig, io)
    assert list(sg) == list(so)


def test_projection_transform_collisions_and_edge_cases(ctx_factory):
    s = synth.SENSORS["c2"]
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    tb = oracle.Tables.of(s)
    seq = synth.make_sequence(s, "c2", 2100, n_frames=3, key_index=1, shuffle=True)
    pts = seq.frames[0]
    # duplicates (exact range ties), NaN / inf / zero / axis / out-of-FOV points
    extra = np.array([[np.nan, 1, 1], [np.inf, 0, 0], [0, 0, 0], [0, 0, 3.0], [1, 0, 5.0], [1, 0, -5.0]], np.float32)
    pts = np.concatenate([pts, pts[:500], extra]).astype(np.float32)
    say("projection with transform", len(pts))
    (rg, ig, sg), (ro, io, so) = _project_both(ctx, S, tb, pts, seq.transforms[0])
    assert np.array_equal(rg.view(np.uint32), ro.view(np.uint32))
    assert np.array_equal(ig, io)
    assert list(sg) == list(so)
    assert so[3] > 500
    # no points at all
    (rg, ig, sg), (ro, io, so) = _project_both(ctx, S, tb, np.zeros((0, 3), np.float32))
    assert not rg.any() and np.all(ig == -1) and list(sg) == [0, 0, 0, 0, 0]


def _key_parity(ctx_factory, s, kind, seed, th, tw, report):
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    tb = oracle.Tables.of(s)
    prm = pcc.params(eps=0.02, tile_h=th, tile_w=tw)
    oprm = oracle.Params(eps=0.02, th=th, tw=tw)
    pts, _, _ = synth.make_frame(s, kind, seed)
    say("key frame", kind, s.H, s.W, th, tw, len(pts))
    g = run_gpu_sequence(pcc, torch, ctx, S, prm, [pts], np.eye(4, dtype=np.float32)[None], 0, DEV)[0]
    r_o = own_range(tb, pts, None, g)
    o = oracle.encode_key(r_o, tb, oprm)
    st = compare_frame(oracle, g["host"], o, r_o)
    ok, nboth, ndiff = residual_codes_agree(g["host"], o, r_o, th, tw)
    st.update(codes_equal=ok, res_both=nboth, res_differ=ndiff)
    report(st)
    v = g["range"] > 0
    err = np.abs(g["dec"].astype(np.float64) - g["range"].astype(np.float64))
    assert np.all(g["dec"][~v] == 0)
    assert err[v].max() <= 0.02, "eps invariant"
    assert st["valid_agree"]
    assert ok
    assert st["size_rel"] <= 0.005, st
    assert st["worst_normal_rad"] <= 1e-4 and st["worst_offset_rel"] <= 1e-4, st
    assert st["own_status_agree"] >= 0.97 and st["cls_agree"] >= 0.97, st
    return g, o, st


@pytest.mark.parametrize("kind,seed,th,tw", [("c1", 1000, 4, 4), ("c1", 1001, 4, 8), ("c2", 2000, 4, 8),
                                             ("c2", 2001, 4, 4), ("c2", 2002, 4, 16), ("c2", 2003, 8, 8)])
def test_key_frame_parity(ctx_factory, kind, seed, th, tw):
    s = synth.SENSORS[kind]
    _key_parity(ctx_factory, s, kind, seed, th, tw, lambda st: say(st))


def test_noiseless_planes_exact_structure(ctx_factory):
    """Scenes without noise: residuals sit far from eps, so both sides keep
    exactly the same pixels and build exactly the same runs."""
    s = synth.SENSORS["c1"]
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    tb = oracle.Tables.of(s)
    rng = np.random.Generator(np.random.PCG64(77))
    scene = synth.make_scene("c1", rng)
    scene.sigma = 0.0
    scene.dropout = 0.0
    pts, _, _ = synth.render(s, scene, np.eye(3), np.zeros(3), 0, rng)
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=4)
    g = run_gpu_sequence(pcc, torch, ctx, S, prm, [pts], np.eye(4, dtype=np.float32)[None], 0, DEV)[0]
    o = oracle.encode_key(own_range(tb, pts, None, g), tb, oracle.Params(eps=0.02, th=4, tw=4))
    h = g["host"]
    agree = np.mean(h["cls"] == o.cls)
    say("noiseless cls agreement", agree, "runs", len(h["srun_list"]), o.c.n_sruns)
    assert agree >= 0.995
    assert abs(len(h["srun_list"]) - o.c.n_sruns) <= max(1, 0.01 * o.c.n_sruns)


def test_sequence_parity_and_invariant(ctx_factory):
    s = synth.SENSORS["c1"]
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    tb = oracle.Tables.of(s)
    seq = synth.make_sequence(s, "c1", 3000, n_frames=10, shuffle=True)
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=4)
    oprm = oracle.Params(eps=0.02, th=4, tw=4)
    say("sequence c3", [len(f) for f in seq.frames])
    g = run_gpu_sequence(pcc, torch, ctx, S, prm, seq.frames, seq.transforms, seq.key_index, DEV)
    ki = seq.key_index
    ok_key = oracle.encode_key(own_range(tb, seq.frames[ki], None, g[ki]), tb, oprm)
    tot_g = tot_o = 0
    for i, gi in enumerate(g):
        o = ok_key if i == ki else oracle.encode_pred(ok_key, own_range(tb, seq.frames[i], seq.transforms[i], gi),
                                                      tb, oprm)
        v = gi["range"] > 0
        err = np.abs(gi["dec"].astype(np.float64) - gi["range"].astype(np.float64))
        assert np.all(gi["dec"][~v] == 0) and err[v].max() <= 0.02, f"frame {i} eps invariant"
        st = compare_frame(oracle, gi["host"], o, gi["range"])
        tot_g += st["size_gpu"]
        tot_o += st["size_orc"]
        ntemp = int(np.sum(gi["host"]["cls"] == 3))
        say(i, {k: st[k] for k in ("cls_agree", "size_gpu", "size_orc", "size_rel")}, "temporal tiles", ntemp,
            int(np.sum(o.cls == 3)))
    assert abs(tot_g - tot_o) <= 0.005 * tot_o


def test_run_twice_bitwise(ctx_factory):
    s = synth.SENSORS["c2"]
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    seq = synth.make_sequence(s, "c2", 2200, n_frames=2, key_index=0, shuffle=True)
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=8)
    a = run_gpu_sequence(pcc, torch, ctx, S, prm, seq.frames, seq.transforms, 0, DEV)
    b = run_gpu_sequence(pcc, torch, ctx, S, prm, seq.frames, seq.transforms, 0, DEV)
    for x, y in zip(a, b):
        assert torch.equal(x["fs"].buf, y["fs"].buf)
        assert np.array_equal(x["dec"], y["dec"])


def test_empty_and_ragged_frames(ctx_factory):
    # W = 1056: 132 tiles of 8 per row, not a multiple of the window or block
    s = synth.Sensor(16, 1056, 15.0, -15.0)
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    tb = oracle.Tables.of(s)
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=8)
    oprm = oracle.Params(eps=0.02, th=4, tw=8)
    empty = np.zeros((0, 3), np.float32)
    g = run_gpu_sequence(pcc, torch, ctx, S, prm, [empty], np.eye(4, dtype=np.float32)[None], 0, DEV)[0]
    o = oracle.encode_key(own_range(tb, empty, None, g), tb, oprm)
    assert g["host"]["info"].size_bytes == o.size_bytes
    assert not g["dec"].any()
    pts, _, _ = synth.make_frame(s, "c1", 1010)
    g = run_gpu_sequence(pcc, torch, ctx, S, prm, [pts], np.eye(4, dtype=np.float32)[None], 0, DEV)[0]
    r_o = own_range(tb, pts, None, g)
    o = oracle.encode_key(r_o, tb, oprm)
    st = compare_frame(oracle, g["host"], o, r_o)
    say("ragged", st)
    assert st["size_rel"] <= 0.005
    v = g["range"] > 0
    assert np.abs(g["dec"][v].astype(np.float64) - g["range"][v]).max() <= 0.02


def test_decode_batch_equals_per_frame(ctx_factory):
    """One decode launch over a whole sequence (key and predicted frames)
    gives the per-frame decoder's ranges bit for bit."""
    s = synth.SENSORS["c2"]
    S = pcc.Sensor.of(s)
    ctx = ctx_factory(S)
    seq = synth.make_sequence(s, "c2", 2300, n_frames=6, key_index=3, shuffle=True)
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=8)
    g = run_gpu_sequence(pcc, torch, ctx, S, prm, seq.frames, seq.transforms, 3, DEV)
    n = len(g)
    outs = [torch.full((s.H, s.W), -1.0, dtype=torch.float32, device=DEV) for _ in range(n)]
    ws = pcc.pc_decode_batch_workspace_size(n)
    work = torch.empty(ws, dtype=torch.uint8, device=DEV)
    keys = [None if i == 3 else g[3]["fs"] for i in range(n)]
    pcc.pc_decode_batch(ctx.h, keys, [x["fs"] for x in g], S, prm, outs, work, ws)
    torch.cuda.synchronize()
    for i in range(n):
        assert np.array_equal(outs[i].cpu().numpy(), g[i]["dec"]), f"frame {i}"
    # key frames only, no key list
    o1 = [torch.empty(s.H, s.W, dtype=torch.float32, device=DEV)]
    pcc.pc_decode_batch(ctx.h, None, [g[3]["fs"]], S, prm, o1, work, ws)
    torch.cuda.synchronize()
    assert np.array_equal(o1[0].cpu().numpy(), g[3]["dec"])

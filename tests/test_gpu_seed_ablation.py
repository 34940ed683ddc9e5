"""What the trained seed network gains over the method without it, on
held-out sequences (10 frames, key frame 5, seeds from 900000; the network
was trained on frames with seeds 5000-6999): the batch graph with the
network against the same batch without it, at eps = 2 cm, for the 64x2048
network and for the 128x2048 network.  Asserted: the key frames need at
most 0.6 times the plain fits per tile, at most 20 % of the seeded tiles
fall back to the plain fit, the compression ratio stays within 2 % of the
plain form's, and every pixel of every frame decodes within eps.  Random
weights keep eps and the ratio within 2 %; non-finite weights give no seeds,
so the streams equal the plain form's byte for byte."""
import os
import sys

import numpy as np
import pytest

from paper_2008_06972_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_06972_amd import pcc, train_seed  # noqa: E402

DEV = torch.device("cuda:0")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NSEQ, NF, KEY = 16, 10, 5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _encode(ctx, S, seqs, net):
    prm = pcc.params(eps=0.02, tile_h=4, tile_w=8)
    fr, outs, rngs = [], [], []
    for q, (frames, transforms) in enumerate(seqs):
        for i, p in enumerate(frames):
            o = pcc.FrameStream(S, prm, DEV)
            r = torch.empty(S.H, S.W, dtype=torch.float32, device=DEV)
            outs.append(o)
            rngs.append(r)
            fr.append(dict(xyz=torch.from_numpy(p).to(DEV), M=None if i == KEY else transforms[i], sensor=S, params=prm,
                           key=q * NF + KEY, out=o, range=r))
    b = pcc.Batch(ctx, fr, persistent=True, graph=True, net=net)
    b.run()
    torch.cuda.synchronize()
    b.close()
    infos = [o.info() for o in outs]
    keys = [infos[j] for j in range(len(infos)) if j % NF == KEY]
    st = {"bytes": sum(int(i.size_bytes) for i in infos),
          "key_fits_per_tile": sum(i.fits for i in keys) / sum(sum(i.tiles) for i in keys),
          "seeded": int(sum(i.seeded for i in keys)), "fallback": int(sum(i.fallback for i in keys))}
    st["fallback_rate"] = st["fallback"] / max(1, st["seeded"] + st["fallback"])
    # every frame decoded, every pixel within eps of its range image
    keys_d = [None if j % NF == KEY else outs[(j // NF) * NF + KEY] for j in range(len(outs))]
    dec = [torch.empty(S.H, S.W, dtype=torch.float32, device=DEV) for _ in outs]
    ws = pcc.pc_decode_batch_workspace_size(len(outs))
    work = torch.empty(ws, dtype=torch.uint8, device=DEV)
    pcc.pc_decode_batch(ctx.h, keys_d, outs, S, prm, dec, work, ws)
    torch.cuda.synchronize()
    worst = 0.0
    for d, r in zip(dec, rngs):
        v = r > 0
        assert bool((d[~v] == 0).all())
        worst = max(worst, float((d[v].double() - r[v].double()).abs().max()))
    st["worst_err"] = worst
    return st, outs


@pytest.mark.parametrize("name,weights", [("c2", "seednet_c2.f32"), ("c5", "seednet_c5.f32")])
def test_trained_network_gains(name, weights):
    s = synth.SENSORS[name]
    S = pcc.Sensor.of(s)
    ctx = pcc.Context([S])
    try:
        seqs = train_seed.gen_sequences(name, "c2", range(900000, 900000 + NSEQ), 16)
        pts = sum(int(np.isfinite(f).all(axis=1).sum()) for fr, _ in seqs for f in fr)
        w = np.fromfile(os.path.join(ROOT, "paper_2008_06972_amd", "weights", weights), dtype="<f4")
        assert w.size == pcc.PC_NET_PARAMS
        plain, outs_p = _encode(ctx, S, seqs, None)
        learned, _ = _encode(ctx, S, seqs, torch.from_numpy(w).to(DEV))
        rp, rl = 12.0 * pts / plain["bytes"], 12.0 * pts / learned["bytes"]
        say(name, "plain", plain, "ratio", rp)
        say(name, "learned", learned, "ratio", rl)
        assert plain["worst_err"] <= 0.02 and learned["worst_err"] <= 0.02
        assert plain["seeded"] == 0 and learned["seeded"] > 0
        assert learned["key_fits_per_tile"] <= 0.6 * plain["key_fits_per_tile"]
        assert learned["fallback_rate"] <= 0.2
        assert abs(rl / rp - 1.0) <= 0.02
        # untrained (random) weights: seeds are tested like any plane, so
        # eps holds and the ratio stays close
        rnd, _ = _encode(ctx, S, seqs, torch.from_numpy(train_seed.he_init(7, pcc.PC_NET_PARAMS)).to(DEV))
        rr = 12.0 * pts / rnd["bytes"]
        say(name, "random weights", rnd, "ratio", rr)
        assert rnd["worst_err"] <= 0.02 and abs(rr / rp - 1.0) <= 0.02
        # non-finite weights: no seed survives, every tile takes the plain fit
        bad = w.copy()
        bad[::97] = np.nan
        nan, outs_n = _encode(ctx, S, seqs, torch.from_numpy(bad).to(DEV))
        say(name, "non-finite weights", nan)
        assert nan["seeded"] == 0 and nan["bytes"] == plain["bytes"]
        off = outs_p[0].L.off_tiles
        for a, b in zip(outs_p, outs_n):
            assert torch.equal(a.buf[:off], b.buf[:off])
    finally:
        ctx.close()

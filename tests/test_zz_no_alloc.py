"""pc_project_noalloc, the projection for callers that cannot allocate: its
collision keys live in a fixed per-device array of the library, so it runs
on a context created without a workspace.  Through the C ABI, two calls in
a row (a 64x2048 frame, then a smaller 16x512 frame with a transform, on
the array the first call left behind) give the ranges, source indices and
statistics of pc_project bit for bit; a sensor beyond the array's size is
refused before any launch."""
import numpy as np
import pytest

from paper_2008_06972_amd import pcc, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def _project(fn, ctx, S, pts, M):
    xyz = torch.from_numpy(np.ascontiguousarray(pts)).to(DEV)
    rng = torch.full((S.H, S.W), -1.0, dtype=torch.float32, device=DEV)
    idx = torch.full((S.H, S.W), -2, dtype=torch.int32, device=DEV)
    st = torch.full((5,), -1, dtype=torch.int64, device=DEV)
    fn(ctx, xyz, len(pts), M, S, rng, idx, st)
    torch.cuda.synchronize()
    return rng.cpu().numpy(), idx.cpu().numpy(), st.cpu().numpy()


def test_project_noalloc_equals_project():
    big, small = synth.SENSORS["c2"], synth.SENSORS["c1"]
    Sb, Ss = pcc.Sensor.of(big), pcc.Sensor.of(small)
    ref = pcc.Context([Sb, Ss])                      # pc_project with its workspace
    h = pcc.pc_ctx_create(0, None, 0)                # no workspace at all
    try:
        for S in (Sb, Ss):
            pcc.pc_sensor_register(h, S)
        pts_b, _, _ = synth.make_frame(big, "c2", 2600)
        pts_b = pts_b[np.random.default_rng(1).permutation(len(pts_b))]
        seq = synth.make_sequence(small, "c1", 3300, n_frames=2, key_index=0, shuffle=True)
        cases = [(Sb, pts_b, None), (Ss, seq.frames[1], seq.transforms[1])]
        for S, pts, M in cases:
            print("case", S.H, S.W, len(pts), "transform" if M is not None else "", flush=True)
            want = _project(pcc.pc_project, ref.h, S, pts, M)
            got = _project(pcc.pc_project_noalloc, h, S, pts, M)
            assert np.array_equal(got[0].view(np.uint32), want[0].view(np.uint32))
            assert np.array_equal(got[1], want[1])
            assert list(got[2]) == list(want[2])
            assert (got[0] > 0).sum() == want[2][4] > 0
        # the workspace-based call still refuses to run without a workspace
        rng = torch.empty(Ss.H, Ss.W, device=DEV)
        with pytest.raises(pcc.PcError) as e:
            pcc.pc_project(h, torch.zeros(3, device=DEV), 1, None, Ss, rng)
        assert e.value.status == pcc.PC_ERR_CAPACITY
        # a sensor larger than the fixed array
        huge = pcc.Sensor.of(synth.Sensor(256, 4096, 10.0, -30.0))
        assert huge.H * huge.W > pcc.PC_PROJECT_NOALLOC_MAX_PIXELS
        pcc.pc_sensor_register(h, huge)
        out = torch.empty(huge.H, huge.W, device=DEV)
        with pytest.raises(pcc.PcError) as e:
            pcc.pc_project_noalloc(h, torch.zeros(3, device=DEV), 1, None, huge, out)
        assert e.value.status == pcc.PC_ERR_CAPACITY
    finally:
        pcc.pc_ctx_destroy(h)
        ref.close()

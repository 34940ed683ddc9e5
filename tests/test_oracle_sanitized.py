"""The oracle's encoder built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, every error fatal) encodes a short
sequence of each small sensor without a report, and its frame sizes equal
those of the regular build (the sanitizers change no result)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
from paper_2008_06972_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _have_sanitizers(tmp):
    src = os.path.join(tmp, "t.c")
    open(src, "w").write("int main(void){return 0;}\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", src, "-o", os.path.join(tmp, "t")],
                       capture_output=True)
    return r.returncode == 0


@pytest.mark.parametrize("name,th,tw,seed", [("c1", 4, 4, 61), ("c2", 4, 8, 62)])
def test_oracle_under_sanitizers(tmp_path, name, th, tw, seed):
    if shutil.which("gcc") is None or not _have_sanitizers(str(tmp_path)):
        pytest.skip("gcc with AddressSanitizer is not available")
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           os.path.join(HERE, "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
                           "-o", exe, "-lm"])
    s = synth.SENSORS[name]
    nf, key = 3, 1
    q = synth.make_sequence(s, name, seed, n_frames=nf, key_index=key, moving=2, shuffle=True)
    eps = 0.02
    inp = str(tmp_path / "input.bin")
    with open(inp, "wb") as f:
        f.write(struct.pack("<5i", s.H, s.W, 1, nf, key))
        f.write(struct.pack("<2f2i", s.az0, eps, th, tw))
        f.write(np.asarray(s.elevations(), "<f4").tobytes())
        for pts, M in zip(q.frames, q.transforms):
            p = np.ascontiguousarray(pts, "<f4")
            f.write(struct.pack("<q", len(p)))
            f.write(p.tobytes())
            f.write(np.ascontiguousarray(M, "<f4").tobytes())
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, inp], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    out = [int(x) for x in r.stdout.split()]
    tb = oracle.Tables.of(s)
    total, sizes, fin = oracle.encode_sequences(q.frames, q.transforms, key, 1, nf, tb,
                                                oracle.Params(eps=eps, th=th, tw=tw))
    assert out[:nf] == [int(x) for x in sizes] and out[nf] == fin

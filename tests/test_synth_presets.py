"""The named workloads of the synthetic generator are consistent: every
sensor resolves, tile shapes divide the range image, key frames lie inside
their sequences, and a frame of each single-frame workload has finite
points."""
import numpy as np
import pytest

from paper_2008_06972_amd import synth


@pytest.mark.parametrize("name", sorted(synth.WORKLOADS))
def test_workload_preset(name):
    w = synth.WORKLOADS[name]
    assert 0 <= w["key"] < w["frames"] and w["sequences"] >= 1
    assert all(0.0 < e < 0.1 for e in w["eps"])
    for sn in w["sensors"]:
        s = synth.workload_sensor(sn)
        if w["tile"] is not None:
            th, tw = w["tile"]
            assert s.H % th == 0 and s.W % tw == 0, (name, sn)
    if w["frames"] == 1:
        s = synth.workload_sensor(w["sensors"][0])
        pts, _, _ = synth.make_frame(s, w["scene"], w["seed"])
        assert len(pts) > 0 and np.isfinite(pts).any()


def test_uneven_batch_sensors_match_the_sequence_generator():
    names = synth.WORKLOADS["batch-uneven"]["sensors"]
    assert [tuple(int(x) for x in n.split("x")) for n in names] == list(synth.MIXED)

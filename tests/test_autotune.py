"""Autotuner selection logic (host side): the fastest candidate whose
compression ratio stays within the floor of the reference wins."""
import math

from paper_2008_06972_amd import autotune as at


def _c(tile, pers, b, ms, ratio):
    c = at.Candidate(tile, pers, b, False)
    c.ms, c.ratio = ms, ratio
    return c


def test_fastest_within_floor_wins():
    cs = [_c((4, 8), True, 4, 5.0, 14.0), _c((4, 4), True, 4, 3.0, 13.0), _c((4, 16), False, 0, 4.0, 14.5)]
    best = at.choose(cs, ref_ratio=14.0, ratio_floor=0.98)
    assert best is cs[2]                       # 4x4 is faster but 13.0 < 0.98 * 14.0
    assert [c.ok for c in cs] == [True, False, True]


def test_none_when_nothing_qualifies():
    cs = [_c((4, 4), True, 4, 3.0, 10.0), _c((8, 8), True, 2, math.nan, 20.0)]
    assert at.choose(cs, ref_ratio=14.0) is None


def test_candidate_space():
    cs = at.candidates(blocks=(2, 4, 8), with_net=True)
    # 4 shapes x (3 persistent grid sizes + 1 grid form + 2 more wavefront
    # mappings: at most 1 or 2 lanes per tile); seeds only on 4x8
    assert len(cs) == 24
    assert all(c.seeded == (c.tile == (4, 8)) for c in cs)
    assert sum(1 for c in cs if not c.persistent) == 4
    assert sorted({c.lanes for c in cs}) == [1, 2, 4]
    assert len({c.key() for c in cs}) == len(cs)


def test_plan_cache_round_trip(tmp_path):
    """Chosen plans survive a save and load; a second save merges entries;
    a record naming a shape that is not compiled is refused."""
    import pytest
    autotune = at
    p = str(tmp_path / "plans.json")
    a = autotune.Candidate((4, 8), True, 4, False, 2)
    a.ms, a.ratio = 1.25, 24.9
    b = autotune.Candidate((8, 8), False, 0, False)
    autotune.save_plans(p, {autotune.plan_key(64, 2048, 0.02): a})
    autotune.save_plans(p, {autotune.plan_key(16, 1024, 0.01): b})
    got = autotune.load_plans(p)
    assert set(got) == {"64x2048 0.02", "16x1024 0.01"}
    assert got["64x2048 0.02"].key() == a.key() and got["64x2048 0.02"].ms == 1.25
    assert got["16x1024 0.01"].key() == b.key()
    assert autotune.load_plans(str(tmp_path / "missing.json")) == {}
    import json
    bad = dict(autotune.to_record(a), tile=[3, 5])
    json.dump({"x": bad}, open(p, "w"))
    with pytest.raises(ValueError):
        autotune.load_plans(p)

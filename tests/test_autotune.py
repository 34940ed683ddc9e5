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

"""CPU checks of the plane-march launch plans (hjr_march_plan; host logic only, no device).

Every plan must cover each (column, plane) of the grid exactly once: whole lines (-1), runs of
8, 4 and 2 planes, and the brick variant (-16), whose tiles span rows 2k, 2k+1 of each of dims
1..3 (rows past a dim's end left out) and a segment of at most 128 columns of those rows.  The
tiles are also checked against the XCD interleave: in every full round of eight blocks,
workgroup t belongs to the block of XCD t mod 8, so consecutive tiles of one XCD come from one
block of neighbouring rows.
"""
import numpy as np
import pytest

from paper_1903_07715_amd import hjr
from paper_1903_07715_amd import workloads as W


@pytest.fixture(autouse=True)
def _lib(hjrlib):
    return hjrlib


def _grid(n, periodic=None):
    d = len(n)
    return W.Grid(tuple(n), (-1.0,) * d, (1.0,) * d, tuple(periodic) if periodic else ())


def _strides(n):
    s = [1] * len(n)
    for d in range(len(n) - 2, -1, -1):
        s[d] = s[d + 1] * n[d + 1]
    return s


def _cover(n, plan):
    """Times each (plane, column) is covered by the plan's tiles."""
    n = list(n)
    P = int(np.prod(n[1:]))
    s = _strides(n)
    cnt = np.zeros((n[0], P), dtype=np.int32)
    for c0, i0, ln, cn, rows in plan:
        if cn == 0:
            continue
        assert 0 <= i0 and i0 + ln <= n[0] and ln > 0
        if rows == 1:
            starts = [c0]
        else:
            assert rows == 8 and len(n) == 6
            base = [(c0 // s[d]) % n[d] for d in range(6)]
            assert base[1] % 2 == 0 and base[2] % 2 == 0 and base[3] % 2 == 0
            starts = []
            for e1 in (0, 1):
                for e2 in (0, 1):
                    for e3 in (0, 1):
                        if base[1] + e1 < n[1] and base[2] + e2 < n[2] and base[3] + e3 < n[3]:
                            starts.append(c0 + e1 * s[1] + e2 * s[2] + e3 * s[3])
            # a segment stays inside one row of dims 4..5
            r = c0 % (n[4] * n[5])
            assert r + cn <= n[4] * n[5]
        for a in starts:
            assert a + cn <= P
            cnt[i0:i0 + ln, a:a + cn] += 1
    return cnt


GRIDS = [
    ((25, 25, 25, 25, 25, 25), None),          # the benchmark's grid, whole lines only (large)
    ((7, 9, 11, 13, 8, 10), None),
    ((7, 8, 7, 8, 9, 31), (False, True, False, True, False, False)),
    ((9, 6, 5, 4, 3, 130), None),
    ((13, 41, 23, 17), None),
    ((21, 97, 101), (False, False, True)),
    ((37, 9001), (True, True)),
]


@pytest.mark.parametrize("config", [-1, -8, -4, -2, -16])
@pytest.mark.parametrize("case", GRIDS, ids=lambda c: "x".join(map(str, c[0])))
def test_plan_covers_every_node_once(case, config):
    n, per = case
    g = _grid(n, per)
    if n[0] == 25 and config not in (-1, -16):
        pytest.skip("runs of planes on the 25^6 grid: covered on the smaller grids")
    if config == -16 and len(n) != 6:
        with pytest.raises(hjr.HJRError):
            hjr.march_plan(g, config)
        return
    plan = hjr.march_plan(g, config)
    if n[0] == 25:
        # whole lines: cover the columns of one plane (each tile spans all 25 planes)
        assert np.all(plan[plan[:, 3] > 0][:, 1] == 0) and np.all(plan[plan[:, 3] > 0][:, 2] == 25)
        plan = plan.copy()
        plan[:, 2] = 1
        cnt = _cover((1,) + tuple(n[1:]), plan)
    else:
        cnt = _cover(n, plan)
    assert cnt.min() == 1 and cnt.max() == 1
    assert np.all(plan[:, 3] <= (128 if config == -16 else 256))


def test_brick_plan_rejects_odd_periodic_dims():
    g = _grid((7, 9, 8, 8, 9, 11), (False, True, False, False, False, False))
    with pytest.raises(hjr.HJRError):
        hjr.march_plan(g, -16)
    hjr.march_plan(_grid((7, 10, 8, 8, 9, 11), (False, True, False, False, False, False)), -16)


def test_brick_plan_xcd_blocks_on_the_benchmark_grid():
    """25^6: bricks of 2 x 2 x 2 rows and 5 segments per row (128 x 4 + 113 columns); blocks of
    2 x 2 x 3 bricks with their 5 segments (60 tiles), eight blocks per round interleaved tile by
    tile, so the tiles t, t + 8, t + 16, ... of a round lie in one block."""
    n = (25,) * 6
    plan = hjr.march_plan(_grid(n), -16)
    real = plan[plan[:, 3] > 0]
    assert len(real) == 13 ** 3 * 5
    assert sorted(set(real[:, 3].tolist())) == [113, 128]
    s = _strides(n)
    first_round = plan[:8 * 60]
    for x in range(8):
        tiles = first_round[x::8]
        tiles = tiles[tiles[:, 3] > 0]
        q = np.stack([(tiles[:, 0] // s[d]) % n[d] // 2 for d in (1, 2, 3)], axis=1)
        span = q.max(axis=0) - q.min(axis=0) + 1
        assert tuple(span) == (2, 2, 3), (x, span)


def test_plan_rejects_bad_configs():
    g = _grid((7, 9, 11, 13, 8, 10))
    for cfg in (0, 1, 4, -3, -32):
        with pytest.raises(hjr.HJRError):
            hjr.march_plan(g, cfg)

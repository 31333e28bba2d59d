"""Host logic of the binomial checkpointing schedule (no GPU): the library's
schedule, run by its own executor without device work, must visit every
state in reverse order (the executor refuses anything else), take exactly
the fewest forward steps possible and hold at most 2 s + 3 buffers.

The optimum is pinned two ways, both independent of the library: a brute
force over every first-snapshot position (small cases), and Griewank's
closed form T(l, s) = r l - C(s + r + 1, r - 1), r the least with
C(s + 1 + r, r) >= l, where s counts the free snapshots besides the stored
initial state (Griewank 1992, Griewank & Walther 2000)."""
from functools import lru_cache
from math import comb

import pytest

import paper_1608_08658_amd as awe


@lru_cache(maxsize=None)
def brute_force(l, s):
    """Fewest forward steps to revisit l states in reverse from a stored first
    state with s free snapshots: try every position of the next snapshot."""
    if l <= 1:
        return 0
    if s == 0:
        return l * (l - 1) // 2
    best = brute_force(l, s - 1)
    for m in range(1, l):
        best = min(best, m + brute_force(l - m, s - 1) + brute_force(m, s))
    return best


def closed_form(l, s):
    if l <= 1:
        return 0
    r = 0
    while comb(s + 1 + r, r) < l:
        r += 1
    return r * l - comb(s + 1 + r, r - 1)


def test_schedule_cost_is_the_brute_force_optimum():
    for s in range(0, 6):
        for nt in range(1, 60):
            steps, fields = awe.binomial_cost(nt, s)
            assert steps == brute_force(nt, s), (nt, s)
            assert fields <= 2 * s + 3, (nt, s, fields)


@pytest.mark.parametrize("nt,s", [(2000, 20), (2000, 50), (1500, 30), (3001, 7), (500, 1), (10000, 64)])
def test_schedule_cost_matches_the_closed_form(nt, s):
    steps, fields = awe.binomial_cost(nt, s)
    assert steps == closed_form(nt, s)
    assert nt - 1 <= steps
    assert fields <= 2 * s + 3


def test_schedule_special_cases():
    assert awe.binomial_cost(1, 0) == (0, 0)          # nothing to advance
    assert awe.binomial_cost(2, 0) == (1, 1)
    assert awe.binomial_cost(300, 0)[0] == 300 * 299 // 2   # no snapshots: restart from x_0 for every state
    steps, fields = awe.binomial_cost(400, 399)        # one snapshot per state: a single sweep
    assert steps == 399
    # enough snapshots never cost more steps than fewer
    prev = None
    for s in range(0, 40):
        st = awe.binomial_cost(777, s)[0]
        assert prev is None or st <= prev
        prev = st


def test_schedule_errors():
    with pytest.raises(awe.AweError) as e:
        awe.binomial_cost(0, 3)
    assert e.value.status == -1
    with pytest.raises(awe.AweError) as e:
        awe.binomial_cost(100, -1)
    assert e.value.status == -1
    with pytest.raises(awe.AweError) as e:             # 2^31+ forward steps
        awe.binomial_cost(200000, 0)
    assert e.value.status == -1


def test_binomial_footprint_counts_the_pool():
    # footprint = forward plan + (pool + 3) fields (pool, mu pair, imaging
    # accumulator) + the wavelet copy; the field size follows from two pools
    nt, nsrc = 800, 1
    geo = awe.make_geometry(shape=(100, 120), spacing=(10.0, 10.0), space_order=8, nbl=20, dt=1e-3, nt=nt,
                            src_coords=[[50.0, 60.0]], rec_coords=[[20.0, 30.0]])
    base = awe.footprint(geo, 0)
    f = {s: awe.binomial_cost(nt, s)[1] for s in (0, 5, 20)}
    b = {s: awe.footprint(geo, snapshots=s) for s in f}
    field = (b[20] - b[0]) // (f[20] - f[0])
    assert field * (f[20] - f[0]) == b[20] - b[0]
    assert field >= 140 * 160 * 4                      # at least the padded grid
    for s in f:
        assert b[s] == base + (f[s] + 3) * field + nt * nsrc * 4
    assert b[5] < awe.footprint(geo, 40)               # fewer fields than periodic checkpoints every 40

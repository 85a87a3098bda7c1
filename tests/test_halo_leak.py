"""The stale-halo weight bench.py reports for near-exact overlaps, checked
against its definition by brute force: the probability that the x-coordinate
of a 2D simple random walk (the walk whose expectation a Jacobi sweep
computes: each step moves to one of the four neighbours) reaches the halo
column, d = ceil(o/2) + 1 points away, within s - 1 steps.  Also its exact
regime (o >= 2s - 2 gives 0, Sec. 3.5 overlap) and monotonicity."""
import itertools
from fractions import Fraction

import pytest

import bench


def hitting_probability(d, steps):
    """Dynamic programming over the lazy walk (-1, 0, +1 with 1/4, 1/2, 1/4)
    absorbed at -d: exact rational probability of absorption within steps."""
    dist = {0: Fraction(1)}
    hit = Fraction(0)
    for _ in range(steps):
        nxt = {}
        for pos, p in dist.items():
            for step, w in ((-1, Fraction(1, 4)), (0, Fraction(1, 2)), (1, Fraction(1, 4))):
                q = pos + step
                if q <= -d:
                    hit += p * w
                else:
                    nxt[q] = nxt.get(q, Fraction(0)) + p * w
        dist = nxt
    return hit


def hitting_by_enumeration(d, steps):
    """The same by listing every path of the four-neighbour walk (small cases)."""
    moves = ((-1, 0), (1, 0), (0, -1), (0, 1))
    hits = 0
    for path in itertools.product(moves, repeat=steps):
        x = 0
        for dx, _ in path:
            x += dx
            if x <= -d:
                hits += 1
                break
    return Fraction(hits, 4 ** steps)


@pytest.mark.parametrize("s,o", [(3, 0), (4, 2), (5, 2), (6, 4), (5, 0)])
def test_lazy_walk_is_the_four_neighbour_walk(s, o):
    d = -(-o // 2) + 1
    assert hitting_probability(d, s - 1) == hitting_by_enumeration(d, s - 1)


@pytest.mark.parametrize("s,o", [(12, 22), (12, 18), (12, 16), (12, 14), (16, 22), (16, 18), (20, 22),
                                 (24, 26), (32, 8), (32, 34), (8, 0), (4, 2)])
def test_halo_leak_equals_the_hitting_probability(s, o):
    want = float(hitting_probability(-(-o // 2) + 1, s - 1))
    assert bench.halo_leak(s, o) == pytest.approx(want, rel=1e-12, abs=0.0)


def test_halo_leak_exact_regime_and_monotone():
    for s in range(1, 40):
        assert bench.halo_leak(s, 2 * s - 2) == 0.0
        leaks = [bench.halo_leak(s, o) for o in range(0, 2 * s - 1, 2)]
        assert all(a >= b for a, b in zip(leaks, leaks[1:]))

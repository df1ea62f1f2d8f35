"""Pins of the pruned search oracle (oracle.search.search_beam), whose rule
is read here (the paper leaves pruning to future work): against the
exhaustive search when nothing is cut, a closed form that no cut can change,
an independent re-derivation of the rule over sets of action prefixes, and
the bound that a search over a sub-tree never exceeds the exhaustive one."""
import itertools

from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

from oracle import env as E, qnet as Q, search as S
from paper_2107_01715_amd import workload as W

GAMMA = 0.99


@pytest.fixture(scope="module")
def world():
    ep = W.env_params(1001)
    return S.World(ep.delta, ep.vel, Q.prepare(W.qnet_weights(7)))


@pytest.mark.parametrize("A,d,beam", [(4, 3, 4), (3, 4, 9), (6, 2, 1)])
def test_no_cut_equals_exhaustive(world, A, d, beam):
    """beam >= the largest per-action block of every cut level (A^(d-2)), or
    d <= 2 (no level is cut): identical to the exhaustive search."""
    pos, st = W.roots(1001, 2)
    for r in range(2):
        b = S.search_beam(world, pos[r], st[r], d, A, GAMMA, beam)
        e = S.search(world, pos[r], st[r], d, A, GAMMA)
        np.testing.assert_allclose(b.q, e.q, rtol=1e-12, atol=1e-12)
        assert b.action == e.action


def test_constant_reward_closed_form_under_any_cut():
    """All sprites co-located and moving together: every transition scores 7,
    so every node of a level has the same return and any beam gives
    Q_d = 7 (1 - gamma^d) / (1 - gamma) + gamma^d max b (zero conv/fc1
    weights, fc2 bias b)."""
    delta = np.tile(np.array([[1, 0]], np.int64), (18, 1))
    vel = np.tile(np.array([[1, 0]], np.int64), (7, 1))
    w = {k: np.zeros_like(v, dtype=np.float64) for k, v in W.qnet_weights(7).items()}
    b = np.linspace(-0.5, 0.8, 18)
    w["fc2.b"] = b
    world = S.World(delta, vel, w)
    pos = np.full((8, 2), 10, np.int32)
    stack = np.stack([E.render(pos)] * 4)
    for A, d, beam in [(4, 4, 1), (3, 5, 2)]:
        res = S.search_beam(world, pos, stack, d, A, GAMMA, beam, correction=False)
        want = 7 * (1 - GAMMA ** d) / (1 - GAMMA) + GAMMA ** d * b[:A].max()
        np.testing.assert_allclose(res.q, np.full(A, want), rtol=1e-12)


def prefix_rederivation(world, pos, stack, d, A, beam):
    """The rule over sets of action prefixes: roll every prefix from the
    root, rank prefixes of one root action by FP32 return (ties: the
    lexicographically smaller prefix, which is the smaller Alg. 1 index)."""
    gps = S.level_discounts_f32(GAMMA, d)
    memo = {(): (pos, stack, 0.0, 0.0)}

    def roll(path):
        if path not in memo:
            p, s, R64, R32 = roll(path[:-1])
            p1 = E.move(p, path[-1], world.delta, world.vel)
            s1 = np.concatenate([s[1:], E.render(p1)[None]], axis=0)
            r = E.reward(p1)
            k = len(path)
            memo[path] = (p1, s1, R64 + GAMMA ** (k - 1) * r, S.ret_step_f32(R32, gps[k - 1], r))
        return memo[path]

    alive = [(a,) for a in range(A)]
    for k in range(2, d + 1):
        cand = [p + (a,) for p in alive for a in range(A)]
        if k <= d - 1:
            nxt = []
            for a0 in range(A):
                grp = [p for p in cand if p[0] == a0]
                grp.sort(key=lambda p: (-roll(p)[3], p))
                nxt.extend(grp[:beam])
            cand = nxt
        alive = cand
    qd = np.full(A, -np.inf)
    for p in alive:
        _, s, R64, _ = roll(p)
        qd[p[0]] = max(qd[p[0]], R64 + GAMMA ** d * float(Q.qvalues(s, world.w64, A).max()))
    return qd


@pytest.mark.parametrize("A,d,beam,root", [(4, 3, 1, 0), (4, 3, 2, 1), (3, 4, 2, 2), (6, 3, 1, 3), (2, 5, 3, 4)])
def test_prefix_rederivation(world, A, d, beam, root):
    pos, st = W.roots(1001, 5)
    got = S.search_beam(world, pos[root], st[root], d, A, GAMMA, beam, correction=False)
    np.testing.assert_allclose(got.q, prefix_rederivation(world, pos[root], st[root], d, A, beam),
                               rtol=1e-12, atol=1e-12)


def test_cut_never_exceeds_exhaustive_and_changes_something(world):
    pos, st = W.roots(1002, 6)
    changed = 0
    for r in range(6):
        b = S.search_beam(world, pos[r], st[r], 3, 6, GAMMA, 1, correction=False)
        e = S.search(world, pos[r], st[r], 3, 6, GAMMA, correction=False)
        assert np.all(b.q <= e.q + 1e-12)
        changed += int(np.any(b.q < e.q - 1e-9))
    assert changed > 0, "the cut should bind for some root at beam 1"


def _nearest_f32(exact: Decimal) -> float:
    """The FP32 value nearest to `exact` by direct comparison with the
    neighbours of a first guess (an independent route to the rounding);
    asserts the nearest is unique (no tie)."""
    guess = np.float32(float(exact))
    cands = [np.nextafter(guess, np.float32(-np.inf)), guess, np.nextafter(guess, np.float32(np.inf))]
    dist = sorted((abs(Decimal(float(c)) - exact), float(c)) for c in cands)
    assert dist[0][0] < dist[1][0]
    return dist[0][1]


def test_fp32_discounts_of_the_rule():
    """d_k = RN32(g^(k-1)), g the FP32 gamma.  Powers of 1/2 and 1 are exact;
    for gamma = 0.99: d_2 = float32(0.99) (0x3F7D70A4); g^2 has 48
    significant bits, exact in binary64, so d_3 = float32(g * g computed in
    binary64); d_4 by nearest-neighbour search against the exact decimal
    value of g^3."""
    assert S.level_discounts_f32(0.5, 4) == [1.0, 0.5, 0.25, 0.125]
    assert S.level_discounts_f32(1.0, 3) == [1.0, 1.0, 1.0]
    d = S.level_discounts_f32(0.99, 4)
    g = np.float32(0.99)
    assert int(g.view(np.uint32)) == 0x3F7D70A4
    assert d[0] == 1.0 and d[1] == float(g)
    assert d[2] == float(np.float32(np.float64(g) * np.float64(g)))
    getcontext().prec = 80
    assert d[3] == _nearest_f32(Decimal(float(g)) ** 3)
    assert all(float(np.float32(x)) == x for x in d)


def test_fp32_return_is_one_rounding():
    """R_k = RN32(R_{k-1} + d_k r): on FP32 inputs where rounding the product
    first gives another value (14.734909057617188), the rule keeps the value
    nearest to the exact sum (checked by neighbour search)."""
    prev = float(np.uint32(0x41002BFB).view(np.float32))
    dk = float(np.uint32(0x3F75E99F).view(np.float32))
    assert (prev, dk) == (8.010737419128418, 0.9605960249900818)
    got = S.ret_step_f32(prev, dk, 7)
    assert got == _nearest_f32(Decimal(prev) + Decimal(dk) * 7) == 14.734910011291504
    assert float(np.float32(prev + float(np.float32(dk * 7)))) == 14.734909057617188   # two roundings
    # simple exact cases
    assert S.ret_step_f32(0.0, 1.0, 3) == 3.0 and S.ret_step_f32(1.75, 0.25, 1) == 2.0


def test_round_f32_matches_numpy_on_doubles():
    """RN32 of an exact rational equals numpy's float64 -> float32
    conversion (a library routine) on random doubles, ties included."""
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.integers(-6, 6, 3000),
                        np.array([1.0 + 2.0 ** -24, 1.0 + 3 * 2.0 ** -24, 3.0 * 2.0 ** -25, -(1.0 + 2.0 ** -24)])])
    for v in x:
        assert S.round_f32(Fraction(float(v))) == float(np.float32(v)), v

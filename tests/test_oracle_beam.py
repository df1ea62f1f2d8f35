"""Pins of the pruned search oracle (oracle.search.search_beam), whose rule
is read here (the paper leaves pruning to future work): against the
exhaustive search when nothing is cut, a closed form that no cut can change,
an independent re-derivation of the rule over sets of action prefixes, and
the bound that a search over a sub-tree never exceeds the exhaustive one."""
import itertools

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


def test_fp32_discounts_and_fma():
    gps = S.level_discounts_f32(0.99, 4)
    assert gps[0] == 1.0 and abs(gps[3] - 0.99 ** 3) < 1e-7
    assert all(np.float32(g) == g for g in gps)
    # one rounding: 0.1f + 0.99f * 7 differs from rounding the product first when they disagree
    x = S.ret_step_f32(float(np.float32(0.1)), gps[1], 7)
    assert np.float32(x) == x
    assert x == float(np.float32(np.float64(np.float32(0.1)) + np.float64(gps[1]) * 7.0))

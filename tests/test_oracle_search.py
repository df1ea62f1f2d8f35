"""Pins of the oracle's search, backup and correction against what the paper
and the mathematics fix: brute-force enumeration, a constant-reward closed
form, the depth-0 and depth-1 identities, the structure of Eq. 3, Eq. 6
against Eq. 5 with Prop. 3.6's sigma, and Alg. 1's BFS evaluation order."""
import itertools
import math

import numpy as np
import pytest

from oracle import env as E, qnet as Q, search as S
from paper_2107_01715_amd import workload as W

GAMMA = 0.99


def brute_force_qd(world, pos, stack, d, A, gamma):
    """Every action sequence (a_0..a_{d-1}) rolled out from the root; the leaf
    adds gamma^d max_a Q; the best sequence per first action."""
    best = np.full(A, -np.inf)
    for seq in itertools.product(range(A), repeat=d):
        p, s, ret = np.asarray(pos, dtype=np.int64), stack, 0.0
        for t, a in enumerate(seq):
            p, s, r = E.step(p, s, a, world.delta, world.vel)
            ret += gamma ** t * r
        v = ret + gamma ** d * float(Q.qvalues(s, world.w64, A).max())
        best[seq[0]] = max(best[seq[0]], v)
    return best


@pytest.mark.parametrize("d,A", [(1, 4), (2, 4), (2, 6), (1, 18)])
def test_dfs_equals_brute_force(world_c1, d, A):
    pos, st = W.roots(1001, 3)
    for r in range(3):
        got = S.root_values(world_c1, pos[r], st[r], d, A, GAMMA)
        want = brute_force_qd(world_c1, pos[r], st[r], d, A, GAMMA)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def alg1_bfs(world, pos, stack, d, A, gamma):
    """Alg. 1 with explicit tensors: replicate states/returns (repeat each A
    times), tile the action vector, accumulate gamma^i r, add gamma^d max Q at
    the leaves, return the flat returns R."""
    states = [(np.asarray(pos, dtype=np.int64), stack)]
    R = np.zeros(1)
    for i in range(d):
        states = [x for x in states for _ in range(A)]      # S x A (repeat-interleave)
        R = np.repeat(R, A)                                  # R x A
        acts = np.tile(np.arange(A), len(states) // A)       # A tiled
        out = [E.step(p, s, int(a), world.delta, world.vel) for (p, s), a in zip(states, acts)]
        states = [(p, s) for p, s, _ in out]
        R = R + gamma ** i * np.array([r for _, _, r in out], dtype=np.float64)
    V = Q.qvalues(np.stack([s for _, s in states]), world.w64, A).max(axis=1)
    return R + gamma ** d * V


@pytest.mark.parametrize("d,A", [(1, 4), (2, 4), (3, 3), (2, 6)])
def test_alg1_order_equals_dfs(world_c1, d, A):
    pos, st = W.roots(77, 2)
    for r in range(2):
        Rflat = alg1_bfs(world_c1, pos[r], st[r], d, A, GAMMA)
        qd = S.root_values(world_c1, pos[r], st[r], d, A, GAMMA)
        # root action of flat leaf i is floor(i / A^(d-1))
        per_root = Rflat.reshape(A, A ** (d - 1)).max(axis=1)
        np.testing.assert_allclose(per_root, qd, rtol=1e-12, atol=1e-12)
        assert int(np.argmax(Rflat)) // A ** (d - 1) == S.argmax_low(qd)


def _constant_world(b):
    z = {k: np.zeros(s, dtype=np.float32) for k, s in W.QNET_SHAPES}
    z["fc2.b"] = np.asarray(b, dtype=np.float32)
    world = S.World(np.tile(np.array([[1, 0]]), (18, 1)), np.tile(np.array([[1, 0]]), (7, 1)),
                    Q.prepare(z))
    pos = np.tile(np.array([[10, 20]]), (8, 1))
    stack = np.zeros((4, 84, 84), dtype=np.uint8)
    return world, pos, stack


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_constant_reward_closed_form(d):
    """r = 7 every step and Q(s, .) = b for every s: Q_d(a) = 7 (1 - g^d)/(1 - g)
    + g^d max b; delta(a) = 7 + g max b - b(a); corrected vector shifts every
    a != argmax b by c g^d B."""
    A = 4
    b = np.array([0.25, -0.5, 1.0, 0.125], dtype=np.float32).astype(np.float64)
    world, pos, stack = _constant_world(np.concatenate([b, np.zeros(14)]))
    res = S.search(world, pos, stack, d, A, GAMMA, correction=True, c=0.75)
    ret = 7.0 * (1 - GAMMA ** d) / (1 - GAMMA)
    np.testing.assert_allclose(res.q_d, ret + GAMMA ** d * b.max(), rtol=1e-13)
    assert [7, 13.93, 20.7907, 27.582793][d - 1] == pytest.approx(ret, rel=1e-12)
    np.testing.assert_allclose(res.q0, b, rtol=0, atol=0)
    np.testing.assert_allclose(res.delta, 7.0 + GAMMA * b.max() - b, rtol=1e-13)
    assert res.pi_o == 2
    do = abs(7.0 + GAMMA * 1.0 - 1.0)
    de = float(np.mean([abs(7.0 + GAMMA - x) for x in (0.25, -0.5, 0.125)]))
    np.testing.assert_allclose(res.B, S.penalty(de, do, A, d), rtol=1e-13)
    want = res.q_d - 0.75 * GAMMA ** d * res.B * (np.arange(A) != 2)
    np.testing.assert_allclose(res.q, want, rtol=1e-13)


def test_negative_bellman_error_enters_by_magnitude():
    """Sprites far apart moving together score 0; Q(s, .) = b everywhere, so
    delta(a) = g max b - b(a), negative at pi_o (max b > 0): d_o = |delta(pi_o)|."""
    A, d, c = 4, 2, 1.0
    b = np.array([0.5, 2.0, -1.0, 1.5])
    z = {k: np.zeros(s, dtype=np.float32) for k, s in W.QNET_SHAPES}
    z["fc2.b"] = np.concatenate([b, np.zeros(14)]).astype(np.float32)
    world = S.World(np.tile(np.array([[1, 1]]), (18, 1)), np.tile(np.array([[1, 1]]), (7, 1)), Q.prepare(z))
    pos = np.array([[10 * i, 10 * i] for i in range(8)])
    res = S.search(world, pos, np.zeros((4, 84, 84), np.uint8), d, A, GAMMA, correction=True, c=c)
    np.testing.assert_allclose(res.delta, GAMMA * 2.0 - b, rtol=1e-14)
    assert res.delta[1] < 0
    do = 0.02
    de = (abs(1.98 - 0.5) + abs(1.98 + 1.0) + abs(1.98 - 1.5)) / 3
    np.testing.assert_allclose(res.B, S.penalty(de, do, A, d), rtol=1e-12)
    np.testing.assert_allclose(res.q_d, GAMMA ** d * 2.0, rtol=1e-14)


def test_depth0_is_argmax_q(world_c1):
    pos, st = W.roots(1001, 4)
    for r in range(4):
        res = S.search(world_c1, pos[r], st[r], 0, 6, GAMMA)
        q0 = Q.qvalues(st[r], world_c1.w64, 6)
        np.testing.assert_array_equal(res.q, q0)
        assert res.action == int(np.argmax(q0))


def test_depth1_delta_is_q1_minus_q0(world_c1):
    """Prop. 3.6: at depth 1 the Bellman error is Q_1 - Q_0."""
    pos, st = W.roots(1001, 4)
    for r in range(4):
        res = S.search(world_c1, pos[r], st[r], 1, 6, GAMMA, correction=True, c=1.0)
        np.testing.assert_allclose(res.delta, res.q_d - res.q0, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("d", [1, 2])
def test_correction_structure(world_c1, d):
    """Eq. 3: pi_o's entry is untouched, every other entry moves by the same
    constant c g^d B; c = 0 gives the vanilla d-step policy (Eq. 2)."""
    pos, st = W.roots(1001, 3)
    for r in range(3):
        res = S.search(world_c1, pos[r], st[r], d, 4, GAMMA, correction=True, c=1.0)
        van = S.search(world_c1, pos[r], st[r], d, 4, GAMMA, correction=False)
        zero = S.search(world_c1, pos[r], st[r], d, 4, GAMMA, correction=True, c=0.0)
        np.testing.assert_array_equal(zero.q, van.q)
        assert zero.action == van.action
        shift = van.q - res.q
        assert shift[res.pi_o] == 0.0
        others = np.delete(shift, res.pi_o)
        np.testing.assert_allclose(others, GAMMA ** d * res.B, rtol=1e-12)
        assert res.pi_o == int(np.argmax(res.q0))


@pytest.mark.parametrize("A", [2, 3, 4, 6, 18])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 6])
def test_eq6_is_eq5_with_bellman_sigma(A, d):
    """Eq. 6 is Eq. 5 with sigma = delta/sqrt(2) (Prop. 3.6: var = delta^2/2)."""
    from oracle import gev
    rng = np.random.default_rng(A * 10 + d)
    for _ in range(5):
        de, do = rng.uniform(0, 3, size=2)
        want = gev.approx_gap(de / math.sqrt(2), do / math.sqrt(2), A, d)
        assert S.penalty(de, do, A, d) == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_eq6_special_cases():
    # equal Bellman errors at depth 1: B = delta * sqrt(log A)
    assert S.penalty(1.5, 1.5, 4, 1) == pytest.approx(1.5 * math.sqrt(math.log(4)), rel=1e-14)
    # d_o = 0: B = d_e (sqrt(d log A) - 1/sqrt(8))
    assert S.penalty(2.0, 0.0, 6, 3) == pytest.approx(2.0 * (math.sqrt(3 * math.log(6)) - 1 / math.sqrt(8)), rel=1e-14)
    # B is linear in (d_e, d_o) and zero at zero
    assert S.penalty(0.0, 0.0, 18, 3) == 0.0
    assert S.penalty(2.0, 1.0, 18, 3) == pytest.approx(2 * S.penalty(1.0, 0.5, 18, 3), rel=1e-14)


def test_tie_set_and_argmax():
    assert S.argmax_low([1.0, 3.0, 3.0]) == 1
    assert S.tie_set([1.0, 3.0, 3.0 - 1e-9]) == [1, 2]
    assert S.tie_set([1.0, 3.0, 2.9]) == [1]


def test_enumerate_nodes_matches_paths(world_c1):
    pos, st = W.roots(1001, 1)
    lv = S.enumerate_nodes(world_c1, pos[0], st[0], 3, 4)
    assert [len(l[0]) for l in lv] == [4, 16, 64]
    for k in range(1, 4):
        for i in (0, 5 % 4 ** k, 4 ** k - 1, (7 * k) % 4 ** k):
            acts = S.node_path(i, k, 4)
            p, s, rs = S.node_at(world_c1, pos[0], st[0], acts)
            P, Fr, R = lv[k - 1]
            assert np.array_equal(P[i], p) and np.array_equal(Fr[i], s[-1]) and R[i] == rs[-1]
            assert acts[0] == i // 4 ** (k - 1)

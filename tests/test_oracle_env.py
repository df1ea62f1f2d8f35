"""Pins of the oracle's integer environment: hand-worked cases (golden),
pixel-set definitions of render and overlap, and frame invariants."""
import json
import os

import numpy as np
import pytest

from oracle import env as E
from paper_2107_01715_amd import workload as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "env_cases.json")))


def square(x, y):
    """Pixel set of a sprite square, listed directly: anchor plus 0..5 in x and y, wrapped."""
    return {((x + i) % 84, (y + j) % 84) for i in range(6) for j in range(6)}


@pytest.mark.parametrize("case", GOLD["render"], ids=lambda c: c["name"])
def test_render_golden(case):
    pos = np.array(case["pos"])
    img = E.render(pos)
    rows, cols = case["pixels_255"]["rows"], case["pixels_255"]["cols"]
    assert (img[np.ix_(rows, cols)] == 255).all()
    assert int((img == 255).sum()) == case["count_255"]
    if "count_128" in case:
        assert int((img == 128).sum()) == case["count_128"]
    assert E.reward(pos) == case["reward"]


@pytest.mark.parametrize("case", GOLD["move"], ids=lambda c: c["name"])
def test_move_golden(case):
    pos = np.zeros((8, 2), dtype=np.int64)
    pos[0] = case["p0"]
    delta = np.zeros((18, 2), dtype=np.int64)
    delta[0] = case["delta"]
    vel = np.tile(np.array(case["delta"]), (7, 1))
    p2 = E.move(pos, 0, delta, vel)
    assert list(p2[0]) == case["expect"]
    # sprites 1..7 started at (0,0) and moved by the same vector
    assert all(list(p2[i]) == [(case["delta"][0]) % 84, (case["delta"][1]) % 84] for i in range(1, 8))


def test_render_matches_pixel_sets():
    """render == per-pixel max over the listed squares (255 for sprite 0, 128 otherwise)."""
    rng = np.random.default_rng(0)
    for _ in range(30):
        pos = rng.integers(0, 84, size=(8, 2))
        want = np.zeros((84, 84), dtype=np.uint8)
        for i in range(8):
            for (x, y) in square(*pos[i]):
                want[y, x] = max(want[y, x], 255 if i == 0 else 128)
        assert np.array_equal(E.render(pos), want)


def test_overlap_is_shared_pixel():
    """reward's overlap test == the two squares share a pixel (brute force over placements)."""
    for dx in range(-12, 13):
        for dy in (-7, -6, -5, 0, 5, 6, 7):
            for base in ((0, 0), (81, 3), (40, 82)):
                p = np.array(base)
                q = np.array([(base[0] + dx) % 84, (base[1] + dy) % 84])
                assert E.overlap(p, q) == bool(square(*p) & square(*q)), (base, dx, dy)


def test_frame_invariants_and_reward_range():
    ep = W.env_params(1001)
    pos, stacks = W.roots(1001, 8)
    for r in range(8):
        p, s = pos[r].astype(np.int64), stacks[r]
        for a in range(18):
            p2, s2, rew = E.step(p, s, a, ep.delta, ep.vel)
            f = s2[-1]
            assert set(np.unique(f)) <= {0, 128, 255}
            assert int((f == 255).sum()) == 36
            assert 0 <= rew <= 7
            assert np.array_equal(s2[:3], s[1:])
            assert ((p2 >= 0) & (p2 < 84)).all()


def test_constant_reward_world():
    """All sprites co-located and moving together: every step scores 7."""
    pos = np.tile(np.array([[83, 83]]), (8, 1))
    delta = np.tile(np.array([[1, 0]]), (18, 1))
    vel = np.tile(np.array([[1, 0]]), (7, 1))
    s = np.zeros((4, 84, 84), dtype=np.uint8)
    for a in range(4):
        pos, s, r = E.step(pos, s, a, delta, vel)
        assert r == 7


def test_reward_is_taken_after_the_move():
    """Sprite 0 starts on sprite 1 and moves 3 px away twice: the first step
    still overlaps (distance 3), the second does not (distance 6)."""
    pos = np.array([[10, 10]] + [[10, 10]] + [[50 + 6 * i, 50] for i in range(6)])
    delta = np.tile(np.array([[3, 0]]), (18, 1))
    vel = np.zeros((7, 2), dtype=np.int64)
    s = np.zeros((4, 84, 84), dtype=np.uint8)
    assert E.reward(pos) == 1
    p1, s1, r1 = E.step(pos, s, 0, delta, vel)
    assert r1 == 1 and list(p1[0]) == [13, 10]
    p2, s2, r2 = E.step(p1, s1, 0, delta, vel)
    assert r2 == 0 and list(p2[0]) == [16, 10]
    assert np.array_equal(s2[-1], E.render(p2)) and np.array_equal(s2[-2], E.render(p1))

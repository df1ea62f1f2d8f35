"""The seeded input generators: SplitMix64 reference values, determinism,
ranges, and the structure of the synthetic workload."""
import numpy as np

from paper_2107_01715_amd import workload as W


def test_splitmix64_reference_sequence():
    """Sequential SplitMix64 from state 0: first outputs as published with the
    generator (Vigna's splitmix64.c reference)."""
    key = np.uint64(0)
    i = np.arange(1, 4, dtype=np.uint64)
    with np.errstate(over="ignore"):
        got = W._mix64(key + i * W.GOLDEN)
    assert [int(x) for x in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_streams_are_deterministic_and_distinct():
    a = W.draws(1, "x", 100)
    assert np.array_equal(a, W.draws(1, "x", 100))
    assert not np.array_equal(a, W.draws(2, "x", 100))
    assert not np.array_equal(a, W.draws(1, "y", 100))
    assert np.array_equal(W.draws(1, "x", 10, start=90), a[90:])
    u = W.uniform01(3, "u", 100000)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.01


def test_env_params():
    ep = W.env_params(1001)
    assert ep.delta.shape == (18, 2) and ep.vel.shape == (7, 2)
    assert len({tuple(r) for r in ep.delta}) == 18
    assert ep.delta.min() >= -3 and ep.delta.max() <= 3
    assert ep.vel.min() >= -2 and ep.vel.max() <= 2


def test_roots_structure():
    from oracle import env as E
    pos, st = W.roots(1003, 5)
    assert pos.shape == (5, 8, 2) and pos.dtype == np.int32 and st.shape == (5, 4, 84, 84)
    assert pos.min() >= 0 and pos.max() < 84
    for r in range(5):
        assert np.array_equal(st[r, 3], E.render(pos[r]))   # newest frame shows the root
        for c in range(4):
            assert int((st[r, c] == 255).sum()) == 36
        # older frames: sprite 0's 6x6 square moved by at most 3 pixels per step
        def anchor(frame):
            ys, xs = np.nonzero(frame == 255)
            cy, cx = set(ys.tolist()), set(xs.tolist())
            return ([y for y in cy if (y - 1) % 84 not in cy][0], [x for x in cx if (x - 1) % 84 not in cx][0])
        y3, x3 = anchor(st[r, 3])
        for c in range(3):
            y, x = anchor(st[r, c])
            for dlt in ((y - y3) % 84, (x - x3) % 84):
                assert min(dlt, 84 - dlt) <= 3 * (3 - c), (r, c, dlt)


def test_request_stream_mix():
    t, a, d, pos, st = W.request_stream(1005, 2000.0, 1.0)
    assert 1800 < len(t) < 2200 and np.all(np.diff(t) > 0)
    assert set(np.unique(a)) <= {4, 6, 18}
    assert set(np.unique(d)) <= {1, 2, 3, 4}
    assert not np.any((a == 18) & (d > 3))
    assert abs(np.mean(d == 1) - 0.5) < 0.05

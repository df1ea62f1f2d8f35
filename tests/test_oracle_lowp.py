"""Pins of the oracle's low-precision emulation (the reference for the BF16
and FP8 matrix-core paths): rounding of known values, and the reduction to
the FP64 network when the roundings are the identity."""
import numpy as np
import pytest

from oracle import qnet as Q
from paper_2107_01715_amd import workload as W


def test_round_bf16_known_values():
    x = np.array([1.0, 255.0, 128.0, 0.1, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9])
    want = np.array([1.0, 255.0, 128.0, 0.10009765625, 1.0, 1.0 + 2 ** -7])
    np.testing.assert_array_equal(Q.round_bf16(x), want)


def test_round_e4m3_known_values():
    x = np.array([1.0, 255.0, 128.0, 448.0, 500.0, -1000.0, 0.3, 2 ** -9, 17.0, 19.0])
    # e4m3 has 3 mantissa bits: 255 -> 256, 17 -> 16 (tie to even), 19 -> 20 (tie to even)
    want = np.array([1.0, 256.0, 128.0, 448.0, 448.0, -448.0, 0.3125, 2 ** -9, 16.0, 20.0])
    np.testing.assert_array_equal(Q.round_e4m3(x), want)


@pytest.mark.parametrize("scale", [1e-4, 0.05, 1.0, 300.0])
def test_roundings_match_torch_conversions(scale):
    """The bit-level roundings against torch's own float32 -> bfloat16 and
    float32 -> float8_e4m3fn conversions (a library routine), on random
    values across the normal and subnormal ranges, exact halves included."""
    import torch
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(200000) * scale).astype(np.float32)
    halves = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 17.0, 19.0, 2 ** -8 + 2 ** -10, 3 * 2 ** -10],
                      dtype=np.float32)
    x = np.concatenate([x, halves, -halves])
    want_bf = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(Q.round_bf16(x), want_bf)
    y = np.clip(x, -448.0, 448.0)
    want_f8 = torch.from_numpy(y).to(torch.float8_e4m3fn).double().numpy()
    np.testing.assert_array_equal(Q.round_e4m3(x), want_f8)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lowp_reduces_to_fp64_without_rounding(monkeypatch, prec):
    w64 = Q.prepare(W.qnet_weights(7))
    _, st = W.roots(4, 3)
    monkeypatch.setattr(Q, "round_bf16", lambda x: np.asarray(x, dtype=np.float64))
    monkeypatch.setattr(Q, "round_e4m3", lambda x: np.asarray(x, dtype=np.float64))
    monkeypatch.setattr(Q, "fp8_dot", lambda X, Wm: X @ Wm.T)       # exact sums
    got = Q.qvalues_lowp(st, w64, 18, prec, ascale=[1.0, 37.0, 5.0, 123.0, 9.0])
    np.testing.assert_allclose(got, Q.qvalues(st, w64, 18), rtol=1e-11, atol=1e-13)


def _dot1(a_vals, b_vals=None):
    """One row x one column of the grouped FP8 sum; K padded to a multiple of 8."""
    a = np.asarray(a_vals, dtype=np.float64)
    b = np.ones_like(a) if b_vals is None else np.asarray(b_vals, dtype=np.float64)
    k = -(-a.size // 8) * 8
    A = np.zeros((1, k)); B = np.zeros((1, k))
    A[0, :a.size], B[0, :b.size] = a, b
    return float(Q.dot_fp8_groups(A, B)[0, 0])


def test_fp8_group_sum_hand_worked():
    """Hand-worked values of the FP8 matrix-core sum rule (groups of 8
    consecutive K values; products truncated toward zero to multiples of
    2^(E-13), E the group's largest sum of operand exponent fields; zero
    products ignored; subnormals at exponent -6)."""
    t = 2.0 ** -6
    # 256 at k = 0: the 7 tiny products of its group fall below the grid
    # 2^(8-13) = 2^-5; the other 3 groups of 8 keep theirs
    assert _dot1([256.0] + [t] * 31) == 256.0 + 24 * t
    # a tiny product in the next group is kept whole
    assert _dot1([256.0] + [0.0] * 7 + [t]) == 256.0 + t
    # truncation toward zero, for either sign: 1.5 * 2^-5 -> 2^-5
    assert _dot1([256.0, 1.5 * 2 ** -5]) == 256.0 + 2 ** -5
    assert _dot1([256.0, -1.5 * 2 ** -5]) == 256.0 - 2 ** -5
    assert _dot1([-256.0, 1.5 * 2 ** -5]) == -256.0 + 2 ** -5
    # E is the sum of the exponent fields, not the product's exponent:
    # 1.75 * 1.75 = 3.0625 has fields 0 + 0, so 2^-13 stays; 1 * 2 has 0 + 1
    assert _dot1([1.75, 2.0 ** -7], [1.75, 2.0 ** -6]) == 3.0625 + 2.0 ** -13
    assert _dot1([1.0, 2.0 ** -7], [2.0, 2.0 ** -6]) == 2.0
    # products with a zero operand take no part in E
    assert _dot1([0.0, 2.0 ** -6], [448.0, 2.0 ** -6]) == 2.0 ** -12
    # a subnormal operand counts as exponent -6: 2^-9 * 448 has E = 2
    assert _dot1([2.0 ** -9, 2.0 ** -6], [448.0, 2.0 ** -6]) == 2.0 ** -9 * 448.0
    assert _dot1([2.0 ** -9, 2.0 ** -6], [448.0, 2.0 ** -5]) == 2.0 ** -9 * 448.0 + 2.0 ** -11
    # products within 2^7 of the group's largest are exact (8-bit products)
    rng = np.random.default_rng(3)
    a = Q.round_e4m3(rng.uniform(1.0, 2.0, 64))
    b = Q.round_e4m3(rng.uniform(1.0, 2.0, 64))
    assert _dot1(a, b) == float(np.dot(a, b))


def test_fp8_conv_grouping_reduces_to_conv2d(monkeypatch):
    """With exact sums the grouped convolution (its K reorderings) equals the
    plain convolution, for the frame layer and the channels-last layers."""
    monkeypatch.setattr(Q, "fp8_dot", lambda X, Wm: X @ Wm.T)
    rng = np.random.default_rng(5)
    for (C, H, O, k, s, inner) in ((4, 84, 32, 8, 4, False), (32, 20, 64, 4, 2, True), (64, 9, 64, 3, 1, True)):
        x = rng.standard_normal((2, C, H, H))
        w = rng.standard_normal((O, C, k, k))
        np.testing.assert_allclose(Q.conv_fp8(x, w, s, inner), Q.conv2d(x, w, np.zeros(O), s), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("prec,bound", [("bf16", 0.02), ("fp8", 0.3)])
def test_lowp_error_is_small_but_present(prec, bound):
    w64 = Q.prepare(W.qnet_weights(7))
    _, st = W.roots(5, 6)
    ref = Q.qvalues(st, w64, 18)
    got = Q.qvalues_lowp(st, w64, 18, prec, ascale=[1.0, 100.0, 100.0, 100.0, 100.0])
    rel = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert 0 < rel.max() < bound


# ---- the low-precision search (leaves through the emulation) ---------------
import itertools  # noqa: E402

from oracle import env as E, search as S  # noqa: E402

ASCALE = [1.0, 37.0, 5.0, 123.0, 9.0]


def brute_force_lowp_qd(world, pos, stack, d, A, gamma, prec):
    """Every action sequence rolled out from the root by hand; the leaf adds
    gamma^d max of the emulated network; best sequence per first action."""
    best = np.full(A, -np.inf)
    for seq in itertools.product(range(A), repeat=d):
        p, s, ret = np.asarray(pos, dtype=np.int64), stack, 0.0
        for t, a in enumerate(seq):
            p, s, r = E.step(p, s, a, world.delta, world.vel)
            ret += gamma ** t * r
        v = Q.qvalues_lowp(s, world.w64, A, prec, ascale=ASCALE).max()
        best[seq[0]] = max(best[seq[0]], ret + gamma ** d * float(v))
    return best


@pytest.mark.parametrize("prec,d,A", [("bf16", 1, 4), ("bf16", 2, 4), ("fp8", 2, 3)])
def test_search_lowp_equals_brute_force(world_c1, prec, d, A):
    pos, st = W.roots(1001, 2)
    for r in range(2):
        got = S.search_lowp(world_c1, pos[r], st[r], d, A, 0.99, prec, ascale=ASCALE, correction=False)
        want = brute_force_lowp_qd(world_c1, pos[r], st[r], d, A, 0.99, prec)
        np.testing.assert_allclose(got.q, want, rtol=1e-12, atol=1e-12)


def test_search_lowp_keeps_fp64_correction_inputs(world_c1):
    """With corr_prec="fp64" pi_o, the Bellman errors and B are the FP64
    search's; only the backed-up values carry the leaves' rounding."""
    pos, st = W.roots(1001, 3)
    for r in range(3):
        lo = S.search_lowp(world_c1, pos[r], st[r], 2, 4, 0.99, "bf16")
        hi = S.search(world_c1, pos[r], st[r], 2, 4, 0.99)
        assert lo.pi_o == hi.pi_o
        np.testing.assert_array_equal(lo.delta, hi.delta)
        assert lo.B == hi.B
        assert not np.array_equal(lo.q_d, hi.q_d)


def test_search_lowp_rounds_correction_inputs_on_request(world_c1):
    """corr_prec="bf16" sends the root and depth-1 evaluations through the
    emulation too: the root values the correction reads are the emulated
    network's, not the FP64 one's."""
    pos, st = W.roots(1001, 1)
    lo = S.search_lowp(world_c1, pos[0], st[0], 2, 4, 0.99, "bf16", corr_prec="bf16")
    want_q0 = Q.qvalues_lowp(st[0], world_c1.w64, 4, "bf16")
    np.testing.assert_array_equal(lo.q0, want_q0)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_search_lowp_reduces_to_fp64_without_rounding(world_c1, monkeypatch, prec):
    monkeypatch.setattr(Q, "round_bf16", lambda x: np.asarray(x, dtype=np.float64))
    monkeypatch.setattr(Q, "round_e4m3", lambda x: np.asarray(x, dtype=np.float64))
    monkeypatch.setattr(Q, "fp8_dot", lambda X, Wm: X @ Wm.T)       # exact sums
    pos, st = W.roots(1002, 2)
    for d in (0, 1, 2):
        for r in range(2):
            lo = S.search_lowp(world_c1, pos[r], st[r], d, 4, 0.99, prec, ascale=ASCALE, corr_prec=prec)
            hi = S.search(world_c1, pos[r], st[r], d, 4, 0.99)
            np.testing.assert_allclose(lo.q, hi.q, rtol=1e-11, atol=1e-12)
            assert lo.action == hi.action

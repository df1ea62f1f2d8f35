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


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lowp_reduces_to_fp64_without_rounding(monkeypatch, prec):
    w64 = Q.prepare(W.qnet_weights(7))
    _, st = W.roots(4, 3)
    monkeypatch.setattr(Q, "round_bf16", lambda x: np.asarray(x, dtype=np.float64))
    monkeypatch.setattr(Q, "round_e4m3", lambda x: np.asarray(x, dtype=np.float64))
    got = Q.qvalues_lowp(st, w64, 18, prec, ascale=[1.0, 37.0, 5.0, 123.0, 9.0])
    np.testing.assert_allclose(got, Q.qvalues(st, w64, 18), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("prec,bound", [("bf16", 0.02), ("fp8", 0.3)])
def test_lowp_error_is_small_but_present(prec, bound):
    w64 = Q.prepare(W.qnet_weights(7))
    _, st = W.roots(5, 6)
    ref = Q.qvalues(st, w64, 18)
    got = Q.qvalues_lowp(st, w64, 18, prec, ascale=[1.0, 100.0, 100.0, 100.0, 100.0])
    rel = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert 0 < rel.max() < bound

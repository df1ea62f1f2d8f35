"""The headline configuration at full size, in the launch shape the benchmark
times: 256 roots, A = 18, depth 3 (1,492,992 leaves), gamma 0.99, the BCTS
correction with c = 1; BF16 through the fused conv kernel in rounds of 3
stacks and chunks of 1,048,576 stacks (the same seeds as the benchmark).

The FP64 oracle needs about 0.2 s per root here, so it checks sampled roots:
* FP32 root vectors within 1e-5 of the oracle's largest |Q| per root, actions
  equal unless the oracle's best two are within 1e-6 (the parity bar);
* BF16 root vectors within the BF16 operand error of the oracle (mean
  relative error < 1e-2, as on the small configuration);
and over all 256 roots, properties that hold at any size:
* BF16 root actions agree with the FP32 path on >= 99.5% of the roots;
* BF16 results are bit-identical when the stacks are chunked differently.
The empty batch is an argument error.  Beyond the headline, two roots at
A = 18 and depth 4 check the BF16 path against the FP32 one (the oracle is
too slow at that size) and against itself under another chunking.
"""
import numpy as np
import pytest

from oracle import qnet as Q, search as S
from paper_2107_01715_amd import workload as W

pytestmark = pytest.mark.gpu

N, A, D, GAMMA = 256, 18, 3, 0.99
INSTANCE_SEED, WEIGHT_SEED = 1003, 7
SAMPLE = (0, 97, 255)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_01715_amd import bcts
    return bcts


@pytest.fixture(scope="module")
def headline(lib):
    ep = W.env_params(INSTANCE_SEED)
    w = W.qnet_weights(WEIGHT_SEED)
    ctx = lib.Context(0)
    ctx.set_env(ep.delta, ep.vel)
    ctx.set_qnet(W.qnet_blob(w))
    world = S.World(ep.delta, ep.vel, Q.prepare(w))
    pos, st = W.roots(INSTANCE_SEED, N)
    corr = lib.correction(True, 1.0)
    ctx.set_precision(lib.FP32)
    a32, q32 = ctx.search(pos, st, D, A, GAMMA, corr)
    ctx.set_precision(lib.BF16)
    ctx.set_tuning(lib.TUNE_FUSED, 1)
    ctx.set_tuning(lib.TUNE_FUSED_ROUND, 3)
    ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 1048576)
    a16, q16 = ctx.search(pos, st, D, A, GAMMA, corr)
    ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 262144)
    a16c, q16c = ctx.search(pos, st, D, A, GAMMA, corr)
    ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 1048576)
    ctx.set_precision(lib.FP32)
    refs = {r: S.search(world, pos[r], st[r], D, A, GAMMA, correction=True, c=1.0) for r in SAMPLE}
    yield ctx, (a32, q32), (a16, q16), (a16c, q16c), refs
    ctx.close()


def test_fp32_sampled_roots_match_oracle(headline):
    _, (a32, q32), _, _, refs = headline
    for r, ref in refs.items():
        qo = np.asarray(ref.q, dtype=np.float64)
        err = np.abs(q32[r].astype(np.float64) - qo).max()
        bound = 1e-5 * np.abs(qo).max() + 1e-7
        assert err <= bound, (r, err, bound)
        assert a32[r] == ref.action or a32[r] in ref.ties, (r, a32[r], ref.action)


def test_bf16_sampled_roots_within_operand_error(headline):
    _, _, (a16, q16), _, refs = headline
    errs = [np.abs(q16[r].astype(np.float64) - np.asarray(ref.q)).max() / np.abs(ref.q).max()
            for r, ref in refs.items()]
    print(f"BF16 vs FP64 oracle on roots {SAMPLE}: rel err {np.round(errs, 5)}")
    assert np.mean(errs) < 1e-2, errs


def test_bf16_actions_agree_with_fp32(headline):
    _, (a32, q32), (a16, _), _, _ = headline
    agree = 0
    for r in range(N):
        m = q32[r].max()
        ties = np.flatnonzero(q32[r] >= m - 1e-6 * max(1.0, abs(m)))
        agree += a16[r] == a32[r] or a16[r] in ties
    print(f"BF16 vs FP32 root actions: {agree}/{N}")
    assert agree >= 0.995 * N, agree


def test_bf16_chunking_is_bitwise_invariant(headline):
    _, _, (a16, q16), (a16c, q16c), _ = headline
    assert np.array_equal(a16, a16c)
    assert np.array_equal(q16, q16c)


def test_empty_batch_is_rejected(lib, headline):
    ctx = headline[0]
    pos, st = W.roots(INSTANCE_SEED, 1)
    with pytest.raises(lib.BctsError) as e:
        ctx.search(pos[:0], st[:0], D, A, GAMMA, lib.correction(True, 1.0))
    assert e.value.status == lib.E_INVAL
    ctx.search(pos, st, 1, A, GAMMA, lib.correction(True, 1.0))      # the context stays usable


def test_largest_tree_a18_depth4(lib, headline):
    """A = 18 at depth 4 (104,976 leaves per root, the deepest tree of the
    configurations' range; the FP64 oracle needs minutes per root there):
    BF16 agrees with the FP32 GPU path within the BF16 operand error, and is
    bit-identical when its stacks are chunked differently."""
    ctx = headline[0]
    pos, st = W.roots(INSTANCE_SEED + 1, 2)
    corr = lib.correction(True, 1.0)
    ctx.set_precision(lib.FP32)
    a32, q32 = ctx.search(pos, st, 4, A, GAMMA, corr)
    ctx.set_precision(lib.BF16)
    try:
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 1048576)
        a1, q1 = ctx.search(pos, st, 4, A, GAMMA, corr)
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 65536)
        a2, q2 = ctx.search(pos, st, 4, A, GAMMA, corr)
    finally:
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 1048576)
        ctx.set_precision(lib.FP32)
    assert np.array_equal(a1, a2) and np.array_equal(q1, q2)
    rel = np.abs(q1.astype(np.float64) - q32).max(axis=1) / np.abs(q32).max(axis=1)
    print(f"A=18 d=4 BF16 vs FP32: rel err {np.round(rel, 5)}")
    assert rel.max() < 2e-2, rel


def test_fp8_instruction_paths_agree_at_full_size(lib, headline):
    """FP8 at the headline shape in the benchmark's launch shape: the K = 128
    path (conv2 / conv3 weights in LDS, its own x1 / x2 layouts, fc1 over
    stage pairs) and the K = 32 path sum each group of 8 products the same way
    and add the group sums in the same order, so the two must give the same
    bits on all 256 roots; so must another chunking of the stacks.  (The FP8
    emulation needs about 20 minutes per root at this size; it is checked
    against the kernels on sibling groups of 18 and on A = 18, depth-2 roots.)"""
    ctx = headline[0]
    pos, st = W.roots(INSTANCE_SEED, N)
    corr = lib.correction(True, 1.0)
    _, cal = W.roots(2003, 64)
    ctx.calibrate_fp8(cal)
    ctx.set_precision(lib.FP8)
    out = {}
    try:
        for k128, chunk in ((1, 1048576), (0, 1048576), (1, 262144)):
            ctx.set_tuning(lib.TUNE_FP8_K128, k128)
            ctx.set_tuning(lib.TUNE_FUSED_CHUNK, chunk)
            out[(k128, chunk)] = ctx.search(pos, st, D, A, GAMMA, corr)
    finally:
        ctx.set_tuning(lib.TUNE_FP8_K128, 1)
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 1048576)
        ctx.set_precision(lib.FP32)
    a, q = out[(1, 1048576)]
    for key in ((0, 1048576), (1, 262144)):
        assert np.array_equal(out[key][0], a), key
        assert np.array_equal(out[key][1], q), key
    _, (a32, q32), _, _, _ = headline
    agree = sum(int(a[r] == a32[r] or q32[r][a[r]] >= q32[r].max() - 1e-6 * max(1.0, abs(q32[r].max())))
                for r in range(N))
    print(f"FP8 vs FP32 root actions: {agree}/{N}")

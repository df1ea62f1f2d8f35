"""The working-size and batching configurations at their full sizes, in the
launch forms they are defined with (parity cases beside the benchmark's
headline configuration, which tests/test_gpu_headline.py covers):

* 256 roots, A = 6, depth 3, FP32, one root per launch sequence (the plain
  form): sampled roots against the FP64 oracle at the FP32 bar (1e-5 of the
  largest |Q| per root; actions equal unless tied within 1e-6), and every
  root's result equal, bit for bit, to the batched search of all 256;
* 1,024 roots with A ~ U{4, 6, 18}, d ~ U{1, 2, 3} plus 8 roots at A = 6,
  d = 4, BF16, the whole batch as one captured HIP graph: the graph's
  replays equal the eager batch bit for bit, sampled roots searched alone
  equal their rows of the batch bit for bit, and small sampled trees are
  within the BF16 operand error of the oracle.
"""
import numpy as np
import pytest

from oracle import qnet as Q, search as S
from paper_2107_01715_amd import workload as W

pytestmark = pytest.mark.gpu

GAMMA = 0.99
WEIGHT_SEED = 7


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_01715_amd import bcts
    return bcts


def make(lib, seed):
    ep = W.env_params(seed)
    w = W.qnet_weights(WEIGHT_SEED)
    ctx = lib.Context(0)
    ctx.set_env(ep.delta, ep.vel)
    ctx.set_qnet(W.qnet_blob(w))
    return ctx, S.World(ep.delta, ep.vel, Q.prepare(w))


def test_working_size_single_root_launches(lib):
    ctx, world = make(lib, 1002)
    n, A, d = 256, 6, 3
    pos, st = W.roots(1002, n)
    corr = lib.correction(True, 1.0)
    ctx.set_precision(lib.FP32)
    single_a = np.zeros(n, np.int32)
    single_q = np.zeros((n, A), np.float32)
    for r in range(n):
        a, q = ctx.search(pos[r:r + 1], st[r:r + 1], d, A, GAMMA, corr)
        single_a[r], single_q[r] = a[0], q[0]
    batch_a, batch_q = ctx.search(pos, st, d, A, GAMMA, corr)
    assert np.array_equal(single_a, batch_a)
    assert np.array_equal(single_q, batch_q)
    for r in range(0, n, 17):
        ref = S.search(world, pos[r], st[r], d, A, GAMMA, correction=True, c=1.0)
        qo = np.asarray(ref.q, dtype=np.float64)
        err = np.abs(single_q[r].astype(np.float64) - qo).max()
        assert err <= 1e-5 * np.abs(qo).max() + 1e-7, (r, err)
        assert single_a[r] == ref.action or single_a[r] in ref.ties, (r, single_a[r], ref.action)
    ctx.close()


def test_mixed_batch_as_one_graph(lib):
    import torch
    ctx, world = make(lib, 1004)
    A_mix, d_mix = W.mixed_shapes(1004, 1024, (4, 6, 18), (1, 2, 3))
    Av = np.concatenate([A_mix, np.full(8, 6, np.int32)]).astype(np.int32)
    dv = np.concatenate([d_mix, np.full(8, 4, np.int32)]).astype(np.int32)
    n = len(Av)
    pos, st = W.roots(1004, n)
    corr = lib.correction(True, 1.0)
    ctx.set_precision(lib.BF16)
    eager_a, eager_q = ctx.search_batch(pos, st, dv, Av, GAMMA, corr)
    dev = torch.device("cuda:0")
    act_t = torch.zeros(n, dtype=torch.int32, device=dev)
    q_t = torch.zeros(n, 18, dtype=torch.float32, device=dev)
    ctx.search_batch_graph(torch.from_numpy(pos).to(dev), torch.from_numpy(st).to(dev), dv, Av, GAMMA, corr,
                           act_t, q_t, replays=3)
    torch.cuda.synchronize()
    assert np.array_equal(act_t.cpu().numpy(), eager_a)
    assert np.array_equal(q_t.cpu().numpy(), eager_q)
    # batch invariance: the largest tree, a depth-4 root and a few others alone
    sample = [int(np.flatnonzero((Av == 18) & (dv == 3))[0]), n - 1, 0, 511]
    for r in sample:
        a1, q1 = ctx.search_batch(pos[r:r + 1], st[r:r + 1], dv[r:r + 1], Av[r:r + 1], GAMMA, corr)
        assert a1[0] == eager_a[r], r
        assert np.array_equal(q1[0], eager_q[r]), r
    # small trees against the oracle (BF16 operand error)
    small = [int(i) for i in np.flatnonzero((Av <= 6) & (dv <= 2))[:4]]
    for r in small:
        ref = S.search(world, pos[r], st[r], int(dv[r]), int(Av[r]), GAMMA, correction=True, c=1.0)
        rel = np.abs(eager_q[r, :Av[r]].astype(np.float64) - np.asarray(ref.q)).max() / np.abs(ref.q).max()
        assert rel < 2e-2, (r, rel)
    ctx.set_precision(lib.FP32)
    ctx.close()


def test_graph_handle_is_reusable(lib):
    """bcts_graph_create captures one batch shape once; launches replay it on
    whatever the input buffers hold, with eager searches in between, and
    equal the eager search bit for bit; the model's settings are refused
    while the graph exists."""
    import torch
    ctx, _ = make(lib, 1004)
    g = None
    try:
        ctx.set_precision(lib.BF16)
        n = 12
        A, d = W.mixed_shapes(1008, n, (4, 6, 18), (1, 2, 3))
        corr = lib.correction(True, 1.0)
        dev = torch.device("cuda:0")
        pos_a, st_a = W.roots(1008, n)
        pos_b, st_b = W.roots(1009, n)
        pt = torch.from_numpy(pos_a).to(dev)
        stt = torch.from_numpy(st_a).to(dev)
        at = torch.zeros(n, dtype=torch.int32, device=dev)
        qt = torch.zeros(n, 18, dtype=torch.float32, device=dev)
        g = ctx.graph_create(pt, stt, d, A, GAMMA, corr, at, qt)
        with pytest.raises(lib.BctsError) as e:
            ctx.set_precision(lib.FP32)
        assert e.value.status == lib.E_STATE
        for pos, st in ((pos_a, st_a), (pos_b, st_b), (pos_a, st_a)):
            pt.copy_(torch.from_numpy(pos))
            stt.copy_(torch.from_numpy(st))
            a_ref, q_ref = ctx.search_batch(pos, st, d, A, GAMMA, corr)     # eager work in between
            at.fill_(-1)
            g.launch(2)
            torch.cuda.synchronize()
            assert np.array_equal(at.cpu().numpy(), a_ref)
            assert np.array_equal(qt.cpu().numpy(), q_ref)
        g.close()
        ctx.set_precision(lib.FP32)                       # allowed again
    finally:
        if g is not None:
            g.close()
        ctx.close()

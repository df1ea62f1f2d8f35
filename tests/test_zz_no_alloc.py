"""The entry point that allocates nothing (bcts_search_batch_device_noalloc)
against the device entry point it varies (bcts_search_batch_device), through
the C ABI: bit-identical actions and root vectors on two calls in a row (the
second smaller, on another stream), in BF16 (fused kernels) and FP32 (layer
kernels); a search larger than the static scratch is refused before any work
is enqueued."""
import numpy as np
import pytest

from paper_2107_01715_amd import workload as W

pytestmark = pytest.mark.gpu
GAMMA = 0.99


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_01715_amd import bcts
    return bcts


def batch(seed, n, big):
    pos, st = W.roots(seed, n)
    A, d = W.mixed_shapes(seed, n, (4, 6, 18), (1, 2, 3))
    d = np.where(A == 18, np.minimum(d, 2), d)
    if big:                                   # one root of the headline shape
        A[0], d[0] = 18, 3
    return pos, st, A.astype(np.int32), d.astype(np.int32)


def run(lib, ctx, fn, pos, st, A, d, stream):
    import torch
    with torch.cuda.stream(stream):
        pt = torch.from_numpy(pos).cuda()
        stt = torch.from_numpy(st).cuda()
        at = torch.full((len(A),), -1, dtype=torch.int32, device="cuda")
        qt = torch.zeros((len(A), 18), dtype=torch.float32, device="cuda")
        fn(pt, stt, d, A, GAMMA, lib.correction(True, 1.0), at, qt, stream=stream)
        stream.synchronize()
        return at.cpu().numpy(), qt.cpu().numpy()


@pytest.mark.parametrize("prec", ["BF16", "FP32"])
def test_noalloc_equals_device_entry_point(lib, prec):
    import torch
    ep = W.env_params(1004)
    ctx = lib.Context(0)
    try:
        ctx.set_env(ep.delta, ep.vel)
        ctx.set_qnet(W.qnet_blob(W.qnet_weights(7)))
        ctx.set_precision(getattr(lib, prec))
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        for call, (seed, n, big, stream) in enumerate(((41, 10, True, s1), (42, 3, False, s2))):
            pos, st, A, d = batch(seed, n, big)
            print(f"{prec} call {call}: {n} roots, A {A.tolist()}, depth {d.tolist()}", flush=True)
            a_ref, q_ref = run(lib, ctx, ctx.search_batch_device, pos, st, A, d, stream)
            a_na, q_na = run(lib, ctx, ctx.search_batch_device_noalloc, pos, st, A, d, stream)
            assert np.array_equal(a_na, a_ref), (call, a_na, a_ref)
            assert np.array_equal(q_na, q_ref), (call, np.abs(q_na - q_ref).max())
            mask = np.arange(18)[None, :] < A[:, None]
            assert (a_na >= 0).all() and np.isfinite(q_na[mask]).all()
    finally:
        ctx.close()


def test_noalloc_refuses_more_than_its_scratch(lib):
    import torch
    ep = W.env_params(1003)
    ctx = lib.Context(0)
    try:
        ctx.set_env(ep.delta, ep.vel)
        ctx.set_qnet(W.qnet_blob(W.qnet_weights(7)))
        ctx.set_precision(lib.BF16)
        n = 64                                   # 64 roots at A = 18, depth 3: ~2.8 GB of levels
        pt = torch.zeros((n, 8, 2), dtype=torch.int32, device="cuda")
        stt = torch.zeros((n, 4, 84, 84), dtype=torch.uint8, device="cuda")
        at = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        qt = torch.zeros((n, 18), dtype=torch.float32, device="cuda")
        with pytest.raises(lib.BctsError) as e:
            ctx.search_batch_device_noalloc(pt, stt, [3] * n, [18] * n, GAMMA, lib.correction(True, 1.0), at, qt)
        assert e.value.status == lib.E_NOMEM
        assert "static scratch" in ctx.last_error()
        torch.cuda.synchronize()
        assert (at.cpu().numpy() == -7).all()   # nothing was enqueued
    finally:
        ctx.close()

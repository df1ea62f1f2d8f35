"""Serving through the C ABI: iteration-level continuous batching with pooled
HBM admission.  Each request's result equals the same root searched alone;
requests beyond the pool queue and still complete; a request larger than the
pool is refused; a small request admitted while a large batch runs finishes
first; an injected launch failure puts the context in its error state, from
which bcts_reset recovers."""
import time

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


def make_ctx(lib, budget=0, prec=None):
    ep = W.env_params(1005)
    ctx = lib.Context(0, budget)
    ctx.set_env(ep.delta, ep.vel)
    ctx.set_qnet(W.qnet_blob(W.qnet_weights(7)))
    if prec is not None:
        ctx.set_precision(prec)
    return ctx


def drain(ctx, tickets, A, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        assert time.time() - t0 < timeout, "serving did not finish"
        for t, a in zip(tickets, A):
            if t in out:
                continue
            r = ctx.poll(t, int(a))
            if r is not None:
                out[t] = r
    return out


@pytest.mark.parametrize("prec_name", ["FP32", "BF16"])
def test_served_equals_alone(lib, prec_name):
    prec = getattr(lib, prec_name)
    ctx = make_ctx(lib, prec=prec)
    ctx.serve_config(64, 2)
    t, A, d, pos, st = W.request_stream(1005, 2000.0, 0.05)
    n = len(t)
    corr = lib.correction(True, 1.0)
    tickets = [ctx.submit(pos[i], st[i], int(d[i]), int(A[i]), GAMMA, corr) for i in range(n)]
    res = drain(ctx, tickets, A)
    for i in range(n):
        a1, q1 = ctx.search(pos[i:i + 1], st[i:i + 1], int(d[i]), int(A[i]), GAMMA, corr)
        act, q, _ = res[tickets[i]]
        assert act == a1[0], i
        np.testing.assert_array_equal(q, q1[0])
    ctx.close()


def test_admission_under_small_budget(lib):
    """A 1.5 GB budget: requests wait for pool memory and every one still
    completes with the result of its root searched alone; an oversized
    request is refused with E_NOMEM."""
    ctx = make_ctx(lib, budget=1536 << 20, prec=lib.BF16)
    ctx.serve_config(8, 2)
    corr = lib.correction(True, 1.0)
    n = 40
    pos, st = W.roots(77, n)
    A = np.array([18, 6, 4, 18, 6] * 8)[:n]
    d = np.array([3, 4, 2, 2, 3] * 8)[:n]
    tickets = [ctx.submit(pos[i], st[i], int(d[i]), int(A[i]), GAMMA, corr) for i in range(n)]
    assert ctx.progress() > 0
    stats = ctx.serve_stats()
    print("after submission:", stats)
    assert stats["pool_capacity"] < 1536 << 20 and stats["pool_in_use"] <= stats["pool_capacity"]
    res = drain(ctx, tickets, A, timeout=120)
    done = [res[t][2] for t in tickets]
    for i in range(n):
        a1, q1 = ctx.search(pos[i:i + 1], st[i:i + 1], int(d[i]), int(A[i]), GAMMA, corr)
        assert res[tickets[i]][0] == a1[0]
        np.testing.assert_array_equal(res[tickets[i]][1], q1[0])
    assert all(np.isfinite(done))
    with pytest.raises(lib.BctsError) as e:
        ctx.submit(pos[0], st[0], 6, 18, GAMMA, corr)      # 18^6 leaves: far over a slot
    assert e.value.status == lib.E_NOMEM
    with pytest.raises(lib.BctsError) as e:
        ctx.poll(123456789, 4)
    assert e.value.status == lib.E_STATE
    ctx.close()


def test_settings_refused_while_serving(lib):
    """Calls that change what queued or running batches read are refused
    with E_STATE until the engine has nothing pending; finished results that
    are not polled yet do not block them, and keep the values they were
    computed with."""
    ctx = make_ctx(lib, prec=lib.BF16)
    ctx.serve_config(2, 1)
    corr = lib.correction(True, 1.0)
    n = 24
    pos, st = W.roots(78, n)
    tickets = [ctx.submit(pos[i], st[i], 3, 18, GAMMA, corr) for i in range(n)]
    assert ctx.progress() > 0       # 12 batches of 5,832-leaf searches, one at a time
    for call in (lambda: ctx.set_precision(lib.FP32), lambda: ctx.set_beam(2),
                 lambda: ctx.set_tuning(lib.TUNE_FUSED_ROUND, 2),
                 lambda: ctx.set_qnet(W.qnet_blob(W.qnet_weights(8)))):
        with pytest.raises(lib.BctsError) as e:
            call()
        assert e.value.status == lib.E_STATE
    t0 = time.time()
    while ctx.progress() > 0:
        assert time.time() - t0 < 60.0, "serving did not finish"
    ctx.set_precision(lib.FP32)     # nothing pending: allowed before polling
    res = drain(ctx, tickets, [18] * n)
    ctx.set_precision(lib.BF16)
    for i in (0, n - 1):
        a1, q1 = ctx.search(pos[i:i + 1], st[i:i + 1], 3, 18, GAMMA, corr)
        assert res[tickets[i]][0] == a1[0]
        np.testing.assert_array_equal(res[tickets[i]][1], q1[0])
    ctx.close()


def test_small_request_overtakes_large_batch(lib):
    """32 roots at A = 18, depth 3 (186,624 leaves) are admitted as a cohort
    that runs stage by stage; a request of A = 4, depth 1 submitted after
    their admission joins at the next stage boundary and finishes before the
    large cohort.  Every result equals the root searched alone."""
    ctx = make_ctx(lib, prec=lib.BF16)
    ctx.serve_config(64, 2)
    corr = lib.correction(True, 1.0)
    n = 32
    pos, st = W.roots(79, n + 1)
    big = [ctx.submit(pos[i], st[i], 3, 18, GAMMA, corr) for i in range(n)]
    t0 = time.time()
    while ctx.serve_stats()["queued"] > 0:          # until every large request is admitted
        ctx.progress()
        assert time.time() - t0 < 60.0
    stats = ctx.serve_stats()
    print("after admission:", stats)
    assert stats["staging"] >= 1                     # a cohort still has stages to run
    small = ctx.submit(pos[n], st[n], 1, 4, GAMMA, corr)
    res = drain(ctx, big + [small], [18] * n + [4], timeout=120)
    t_small = res[small][2]
    t_big = max(res[t][2] for t in big)
    print(f"small request done {1e3 * (t_big - t_small):.2f} ms before the large batch")
    assert t_small < t_big
    for i, t in [(n, small), (0, big[0]), (n - 1, big[-1])]:
        d, A = (1, 4) if t == small else (3, 18)
        a1, q1 = ctx.search(pos[i:i + 1], st[i:i + 1], d, A, GAMMA, corr)
        assert res[t][0] == a1[0]
        np.testing.assert_array_equal(res[t][1], q1[0])
    assert ctx.serve_stats()["pool_in_use"] == 0
    ctx.close()


def test_injected_launch_failure_enters_error_state(lib):
    """A launch made to fail from the host (bcts_debug_fail_launches): the
    call reports E_HIP, the context refuses further work with E_STATE,
    outstanding tickets are dropped by bcts_reset, and the context then
    serves and searches with unchanged results."""
    ctx = make_ctx(lib, prec=lib.BF16)
    ctx.serve_config(16, 2)
    corr = lib.correction(True, 1.0)
    pos, st = W.roots(80, 6)
    a_ref, q_ref = ctx.search(pos, st, 2, 6, GAMMA, corr)
    # a plain search
    ctx.debug_fail_launches(1)
    with pytest.raises(lib.BctsError) as e:
        ctx.search(pos, st, 2, 6, GAMMA, corr)
    assert e.value.status == lib.E_HIP and "injected" in ctx.last_error()
    with pytest.raises(lib.BctsError) as e:
        ctx.search(pos, st, 2, 6, GAMMA, corr)
    assert e.value.status == lib.E_STATE
    ctx.reset()
    a, q = ctx.search(pos, st, 2, 6, GAMMA, corr)
    assert np.array_equal(a, a_ref) and np.array_equal(q, q_ref)
    # serving: the first step's launch fails
    ctx.serve_config(16, 1)
    ctx.debug_fail_launches(1)
    with pytest.raises(lib.BctsError) as e:
        ctx.submit(pos[0], st[0], 2, 6, GAMMA, corr)
    assert e.value.status == lib.E_HIP
    with pytest.raises(lib.BctsError) as e:
        ctx.progress()
    assert e.value.status == lib.E_STATE
    ctx.reset()
    with pytest.raises(lib.BctsError) as e:
        ctx.poll(1, 6)                                 # dropped by the reset
    assert e.value.status == lib.E_STATE
    tickets = [ctx.submit(pos[i], st[i], 2, 6, GAMMA, corr) for i in range(6)]
    res = drain(ctx, tickets, [6] * 6)
    for i, t in enumerate(tickets):
        assert res[t][0] == a_ref[i]
        np.testing.assert_array_equal(res[t][1], q_ref[i][:6])
    ctx.close()

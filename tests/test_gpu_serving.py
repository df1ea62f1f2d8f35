"""Serving through the C ABI: continuous batching with HBM-budget admission.
Each request's result equals the same root searched alone; requests beyond
the budget queue and still complete in arrival order; a request larger than
a serving slot is refused."""
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
    """A 1.5 GB budget: every request still completes, in FIFO completion
    order per slot; an oversized request is refused with E_NOMEM."""
    ctx = make_ctx(lib, budget=1536 << 20, prec=lib.BF16)
    ctx.serve_config(8, 2)
    corr = lib.correction(True, 1.0)
    n = 40
    pos, st = W.roots(77, n)
    A = np.array([18, 6, 4, 18, 6] * 8)[:n]
    d = np.array([3, 4, 2, 2, 3] * 8)[:n]
    tickets = [ctx.submit(pos[i], st[i], int(d[i]), int(A[i]), GAMMA, corr) for i in range(n)]
    assert ctx.progress() > 0
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

"""Forward-model world on the GPU (through the C ABI) against the FP64 oracle
(oracle/mlp.py).

Bars: the FP32 root vector within 1e-5 of the oracle's largest |Q| per root
(1e-6 absolute floor: Q-values of this model are O(0.1-1) and each of the d
levels chains four length-100 FP32 dot products); root actions equal unless
the oracle's best two are within 1e-6 max(1, |max|).  Ragged tiles (children
not a multiple of the 64-child tile), depth 0 and 1, both correction modes
and batch invariance are covered.
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2107_01715_amd import workload as W

pytestmark = pytest.mark.gpu

GAMMA = 0.99
RTOL, ATOL = 1e-5, 1e-6


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_01715_amd import bcts
    return bcts


@pytest.fixture(scope="module", params=[2, 10])
def model(lib, request):
    A = request.param
    w = W.mlp_weights(7, A)
    ctx = lib.Context(0)
    ctx.set_mlp(A, W.mlp_blob(w, A))
    yield ctx, A, M.prepare(w)
    ctx.close()


def check(q_gpu, act_gpu, ref, tag):
    qo = np.asarray(ref.q, dtype=np.float64)
    err = np.abs(np.asarray(q_gpu, dtype=np.float64) - qo).max()
    bound = RTOL * np.abs(qo).max() + ATOL
    assert err <= bound, f"{tag}: |dQ| {err:.3g} > {bound:.3g}\n gpu {q_gpu}\n ref {qo}"
    assert act_gpu == ref.action or act_gpu in ref.ties, f"{tag}: action {act_gpu} vs {ref.action} ties {ref.ties}"


@pytest.mark.parametrize("d", [0, 1, 2, 3, 4])
def test_parity_with_oracle(lib, model, d):
    ctx, A, w = model
    if A == 10 and d == 4:
        pytest.skip("covered by test_parity_deep (one root)")
    n = 5                                      # n * A^k is never a multiple of the 64-child tile
    st = W.mlp_states(101, n)
    act, q = ctx.mlp_search(st, d, A, GAMMA, lib.correction(True, 1.0))
    for r in range(n):
        ref = M.search(w, st[r].astype(np.float64), d, A, GAMMA, correction=True, c=1.0)
        check(q[r], int(act[r]), ref, f"A={A} d={d} root {r}")


def test_parity_deep(lib, model):
    ctx, A, w = model
    d = 7 if A == 2 else 4
    st = W.mlp_states(102, 1)
    act, q = ctx.mlp_search(st, d, A, GAMMA, lib.correction(True, 1.0))
    ref = M.search(w, st[0].astype(np.float64), d, A, GAMMA, correction=True, c=1.0)
    check(q[0], int(act[0]), ref, f"A={A} d={d}")


@pytest.mark.parametrize("mode", ["eq6", "gev", "off"])
def test_correction_modes(lib, model, mode):
    ctx, A, w = model
    st = W.mlp_states(103, 3)
    corr = (lib.correction(False) if mode == "off" else
            lib.correction(True, 0.5, lib.CORR_EXACT_GEV if mode == "gev" else lib.CORR_EQ6))
    act, q = ctx.mlp_search(st, 2, A, GAMMA, corr)
    for r in range(3):
        ref = M.search(w, st[r].astype(np.float64), 2, A, GAMMA, correction=mode != "off", c=0.5,
                       mode="gev" if mode == "gev" else "eq6")
        check(q[r], int(act[r]), ref, f"A={A} {mode} root {r}")


def test_batch_invariance_and_device_form(lib, model):
    """A root gives the same bits alone, in a batch, and through device pointers."""
    import torch
    ctx, A, _ = model
    st = W.mlp_states(104, 33)
    corr = lib.correction(True, 1.0)
    act_b, q_b = ctx.mlp_search(st, 3, A, GAMMA, corr)
    for r in (0, 17, 32):
        act_1, q_1 = ctx.mlp_search(st[r:r + 1], 3, A, GAMMA, corr)
        assert act_1[0] == act_b[r] and np.array_equal(q_1[0], q_b[r])
    dev = torch.device("cuda:0")
    st_t = torch.from_numpy(st).to(dev)
    act_t = torch.zeros(33, dtype=torch.int32, device=dev)
    q_t = torch.zeros(33, A, dtype=torch.float32, device=dev)
    ctx.mlp_search_device(st_t, 3, GAMMA, corr, act_t, q_t)
    torch.cuda.synchronize()
    assert np.array_equal(act_t.cpu().numpy(), act_b) and np.array_equal(q_t.cpu().numpy(), q_b)


def test_argument_errors(lib):
    ctx = lib.Context(0)
    st = W.mlp_states(1, 2)
    with pytest.raises(lib.BctsError) as e:          # no model yet
        ctx.mlp_search(st, 2, 2, GAMMA, lib.correction())
    assert e.value.status == lib.E_STATE
    w = W.mlp_weights(7, 2)
    with pytest.raises(lib.BctsError) as e:          # blob sized for another A
        ctx.set_mlp(3, W.mlp_blob(w, 2))
    assert e.value.status == lib.E_INVAL
    with pytest.raises(lib.BctsError) as e:
        ctx.set_mlp(1, W.mlp_blob(w, 2))
    assert e.value.status == lib.E_INVAL
    ctx.set_mlp(2, W.mlp_blob(w, 2))
    for bad in (dict(depth=17), dict(gamma=1.5), dict(gamma=0.0)):
        kw = dict(depth=2, gamma=GAMMA)
        kw.update(bad)
        with pytest.raises(lib.BctsError) as e:
            ctx.mlp_search(st, kw["depth"], 2, kw["gamma"], lib.correction())
        assert e.value.status == lib.E_INVAL
    bad_states = st.copy()
    bad_states[1, 5] = np.nan
    with pytest.raises(lib.BctsError) as e:
        ctx.mlp_search(bad_states, 2, 2, GAMMA, lib.correction())
    assert e.value.status == lib.E_INVAL
    ctx.close()


@pytest.mark.parametrize("crossover", [1, 2, 3])
def test_crossover_equals_gpu_search(lib, model, crossover):
    """CPU-to-GPU cross-over (Sec. 4.1): the first `crossover` levels on the
    host, the rest on the device.  The host levels do the device kernel's
    FP32 arithmetic in the same order, so actions and root vectors are the
    all-GPU search's bit for bit, for every depth it applies to (the leaves
    always stay on the device), with and without the correction, in both
    correction modes."""
    ctx, A, w = model
    n = 3
    st = W.mlp_states(103, n)
    for d in range(0, 6 if A == 2 else 5):
        for corr in (lib.correction(True, 1.0), lib.correction(False, 0.0),
                     lib.correction(True, 0.5, lib.CORR_EXACT_GEV)):
            ctx.set_tuning(lib.TUNE_MLP_CROSSOVER, 0)
            a0, q0 = ctx.mlp_search(st, d, A, GAMMA, corr)
            ctx.set_tuning(lib.TUNE_MLP_CROSSOVER, crossover)
            a1, q1 = ctx.mlp_search(st, d, A, GAMMA, corr)
            ctx.set_tuning(lib.TUNE_MLP_CROSSOVER, 0)
            assert np.array_equal(a0, a1), (d, crossover)
            assert np.array_equal(q0, q1), (d, crossover, np.abs(q0 - q1).max())
    if A == 2:                                   # and against the oracle at the deepest case
        ctx.set_tuning(lib.TUNE_MLP_CROSSOVER, crossover)
        act, q = ctx.mlp_search(st, 5, A, GAMMA, lib.correction(True, 1.0))
        ctx.set_tuning(lib.TUNE_MLP_CROSSOVER, 0)
        for r in range(n):
            ref = M.search(w, st[r].astype(np.float64), 5, A, GAMMA, correction=True, c=1.0)
            check(q[r], int(act[r]), ref, f"A={A} d=5 crossover {crossover} root {r}")


def test_cpu_bfs_equals_gpu_search(lib, model):
    """The whole search on the host (the CPU BFS of the runtime study) gives
    the GPU search's actions and root vectors bit for bit: every depth to 5
    (4 at A = 10), both correction modes and none, 3 roots per call."""
    ctx, A, _ = model
    st = W.mlp_states(104, 3)
    try:
        for d in range(0, 6 if A == 2 else 5):
            for corr in (lib.correction(True, 1.0), lib.correction(False, 0.0),
                         lib.correction(True, 0.5, lib.CORR_EXACT_GEV)):
                ctx.set_tuning(lib.TUNE_MLP_HOST, 0)
                a0, q0 = ctx.mlp_search(st, d, A, GAMMA, corr)
                for mode in (1, 2):                  # always on the host; the host for small trees
                    ctx.set_tuning(lib.TUNE_MLP_HOST, mode)
                    a1, q1 = ctx.mlp_search(st, d, A, GAMMA, corr)
                    assert np.array_equal(a0, a1), (d, mode)
                    assert np.array_equal(q0, q1), (d, mode, np.abs(q0 - q1).max())
        with pytest.raises(lib.BctsError) as e:
            ctx.set_tuning(lib.TUNE_MLP_HOST, 3)
        assert e.value.status == lib.E_INVAL
    finally:
        ctx.set_tuning(lib.TUNE_MLP_HOST, 0)


def test_crossover_argument(lib, model):
    ctx, _, _ = model
    with pytest.raises(lib.BctsError) as e:
        ctx.set_tuning(lib.TUNE_MLP_CROSSOVER, 17)
    assert e.value.status == lib.E_INVAL
    assert ctx.get_tuning(lib.TUNE_MLP_CROSSOVER) == 0

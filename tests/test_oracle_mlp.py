"""Pins of the forward-model oracle (oracle/mlp.py) against things other than
itself: the framework's own fully connected layers, brute-force enumeration of
action sequences, and a closed form for a model whose transitions are
constant."""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import mlp as M
from oracle import search as S
from paper_2107_01715_amd import workload as W

GAMMA = 0.99


@pytest.fixture(scope="module", params=[2, 10])
def model(request):
    A = request.param
    return A, M.prepare(W.mlp_weights(7, A))


def test_step_matches_torch_linear(model):
    A, w = model
    s = W.mlp_states(3, 4).astype(np.float64)
    t = {k: torch.from_numpy(v) for k, v in w.items()}
    for i in range(4):
        for a in range(A):
            x = torch.cat([torch.from_numpy(s[i]), torch.nn.functional.one_hot(torch.tensor(a), A).double()])
            h = torch.relu(torch.nn.functional.linear(x, t["l1.w"], t["l1.b"]))
            h = torch.relu(torch.nn.functional.linear(h, t["l2.w"], t["l2.b"]))
            h = torch.relu(torch.nn.functional.linear(h, t["l3.w"], t["l3.b"]))
            o = torch.nn.functional.linear(h, t["out.w"], t["out.b"]).numpy()
            s1, r = M.step(w, s[i], a, A)
            np.testing.assert_allclose(s1, o[:100], rtol=0, atol=1e-13)
            assert abs(r - o[100]) < 1e-13
        q = torch.nn.functional.linear(torch.from_numpy(s[i]), t["q.w"], t["q.b"]).numpy()
        np.testing.assert_allclose(M.qvalues(w, s[i], A), q, rtol=0, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_dfs_equals_brute_force(model, d):
    A, w = model
    if A == 10 and d == 3:
        pytest.skip("1,000 sequences per root are covered by d <= 2 at A = 10")
    s0 = W.mlp_states(5, 1)[0].astype(np.float64)
    best = np.full(A, -np.inf)
    for seq in itertools.product(range(A), repeat=d):
        s, tot = s0, 0.0
        for t, a in enumerate(seq):
            s, r = M.step(w, s, a, A)
            tot += GAMMA ** t * r
        tot += GAMMA ** d * M.qvalues(w, s, A).max()
        best[seq[0]] = max(best[seq[0]], tot)
    q = M.root_values(w, s0, d, A, GAMMA)
    np.testing.assert_allclose(q, best, rtol=1e-12, atol=1e-12)


def test_constant_transition_closed_form():
    """Hidden layers zeroed: every transition lands on out.b[:100] with reward
    out.b[100], whatever the state or action, so
    Q_d(a) = r (1 - gamma^d) / (1 - gamma) + gamma^d max Q(b_s) (d >= 1) and
    delta(a) = r + gamma max Q(b_s) - Q0(a)."""
    A = 10
    w = M.prepare(W.mlp_weights(11, A))
    for k in ("l1.w", "l1.b", "l2.w", "l2.b", "l3.w", "l3.b"):
        w[k] = np.zeros_like(w[k])
    bs, r = w["out.b"][:100], float(w["out.b"][100])
    vmax = float((w["q.w"] @ bs + w["q.b"]).max())
    s0 = W.mlp_states(12, 1)[0].astype(np.float64)
    q0 = w["q.w"] @ s0 + w["q.b"]
    for d in (1, 2, 3):
        res = M.search(w, s0, d, A, GAMMA, correction=True, c=1.0)
        qd = r * (1 - GAMMA ** d) / (1 - GAMMA) + GAMMA ** d * vmax
        np.testing.assert_allclose(res.q_d, np.full(A, qd), rtol=1e-12)
        np.testing.assert_allclose(res.delta, r + GAMMA * vmax - q0, rtol=1e-12, atol=1e-12)
        pi = int(np.argmax(q0))
        assert res.pi_o == pi
        # Eq. 3: the root network's action keeps Q_d, every other action moves by the same shift
        assert res.q[pi] == res.q_d[pi]
        shifts = [res.q_d[a] - res.q[a] for a in range(A) if a != pi]
        np.testing.assert_allclose(shifts, shifts[0], rtol=1e-12)
        np.testing.assert_allclose(shifts[0], GAMMA ** d * res.B, rtol=1e-12)


def test_depth0_and_no_correction(model):
    A, w = model
    s0 = W.mlp_states(13, 1)[0].astype(np.float64)
    r0 = M.search(w, s0, 0, A, GAMMA)
    np.testing.assert_array_equal(r0.q, M.qvalues(w, s0, A))
    assert r0.action == S.argmax_low(r0.q)
    r1 = M.search(w, s0, 2, A, GAMMA, correction=False)
    np.testing.assert_array_equal(r1.q, M.root_values(w, s0, 2, A, GAMMA))


def test_depth1_delta_is_q1_minus_q0(model):
    """Prop. 3.6 at depth 1: delta = Q_1 - Q_0."""
    A, w = model
    s0 = W.mlp_states(14, 1)[0].astype(np.float64)
    res = M.search(w, s0, 1, A, GAMMA)
    np.testing.assert_allclose(res.delta, res.q_d - res.q0, rtol=1e-12, atol=1e-12)


def test_weights_follow_the_stated_init():
    w = W.mlp_weights(7, 10)
    for name, shape in W.mlp_shapes(10):
        layer = name.split(".")[0]
        fan_in = dict(W.mlp_shapes(10))[layer + ".w"][1]
        v = w[name].astype(np.float64)
        assert v.shape == shape
        assert np.abs(v).max() <= 1.0 / math.sqrt(fan_in) + 1e-7
        if v.size > 500:      # a uniform draw fills most of its range
            assert np.abs(v).max() > 0.9 / math.sqrt(fan_in)

"""Pin of the oracle's FP64 Q-network against PyTorch's own conv2d / linear
(float64, CPU): the library routines fix the layout (OIHW, cross-correlation,
(c, h, w) flatten)."""
import numpy as np
import torch
import torch.nn.functional as F

from oracle import qnet as Q
from paper_2107_01715_amd import workload as W


def torch_qnet(stacks, w, A):
    t = {k: torch.from_numpy(np.asarray(v, dtype=np.float32)).double() for k, v in w.items()}
    x = torch.from_numpy(stacks).double() / 255.0
    x = F.relu(F.conv2d(x, t["conv1.w"], t["conv1.b"], stride=4))
    x = F.relu(F.conv2d(x, t["conv2.w"], t["conv2.b"], stride=2))
    x = F.relu(F.conv2d(x, t["conv3.w"], t["conv3.b"], stride=1))
    x = torch.flatten(x, 1)
    x = F.relu(F.linear(x, t["fc1.w"], t["fc1.b"]))
    return F.linear(x, t["fc2.w"][:A], t["fc2.b"][:A]).numpy()


def test_qnet_matches_torch_f64():
    w = W.qnet_weights(7)
    w64 = Q.prepare(w)
    _, stacks = W.roots(1001, 6)
    # also a dense random stack, far from the sparse sprite frames
    dense = np.random.default_rng(1).integers(0, 256, size=(2, 4, 84, 84), dtype=np.uint8)
    x = np.concatenate([stacks, dense])
    for A in (1, 4, 18):
        got = Q.qvalues(x, w64, A)
        want = torch_qnet(x, w, A)
        assert got.shape == (8, A)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_qnet_single_equals_batch():
    w64 = Q.prepare(W.qnet_weights(7))
    _, stacks = W.roots(5, 3)
    b = Q.qvalues(stacks, w64, 6)
    for i in range(3):
        np.testing.assert_allclose(Q.qvalues(stacks[i], w64, 6), b[i], rtol=1e-13, atol=1e-15)


def test_kaiming_bounds():
    w = W.qnet_weights(7)
    for name, shape in W.QNET_SHAPES:
        layer = name.split(".")[0]
        fan_in = int(np.prod(dict(W.QNET_SHAPES)[layer + ".w"][1:]))
        bound = np.sqrt(6.0 / fan_in) if name.endswith(".w") else 1.0 / np.sqrt(fan_in)
        v = w[name]
        assert v.dtype == np.float32 and v.shape == shape
        assert np.abs(v).max() <= bound * (1 + 1e-7)
        assert np.abs(v).max() > 0.9 * bound          # the range is actually used
        assert abs(float(v.astype(np.float64).mean())) < 0.1 * bound

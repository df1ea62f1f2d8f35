"""FP64 Nature-DQN Q-network of the oracle (test infrastructure only).

The leaves of the search are scored by the value network Q_theta
(Alg. 1, leaf step; Sec. 4.1).  The network here is the DQN architecture the
paper's Atari agents use: input uint8 frames / 255, conv 32@8x8 stride 4,
conv 64@4x4 stride 2, conv 64@3x3 stride 1 (valid, cross-correlation, OIHW
weights), flatten in (c, h, w) order to 3136, FC 512, FC A; ReLU after every
layer but the last.  The FP32 weights are promoted exactly to FP64.
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def prepare(weights: dict) -> dict:
    """Promote the FP32 weight arrays exactly to FP64 (done once per net)."""
    return {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in weights.items()}


def conv2d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """out[n, o, y, x] = b[o] + sum_{c,i,j} w[o, c, i, j] * x[n, c, stride*y + i, stride*x + j]."""
    kh, kw = w.shape[2], w.shape[3]
    win = sliding_window_view(x, (kh, kw), axis=(2, 3))[:, :, ::stride, ::stride]
    return np.einsum("ncyxij,ocij->noyx", win, w, optimize=True) + b[None, :, None, None]


def relu(x: np.ndarray) -> np.ndarray:
    return np.maximum(x, 0.0)


def qvalues(stacks: np.ndarray, w: dict, A: int) -> np.ndarray:
    """Q-values [n][A] (FP64) for stacks uint8 [n][4][84][84] (or one stack);
    `w` is the output of prepare()."""
    one = stacks.ndim == 3
    s = stacks[None] if one else stacks
    x = s.astype(np.float64) / 255.0
    x = relu(conv2d(x, w["conv1.w"], w["conv1.b"], 4))   # [n,32,20,20]
    x = relu(conv2d(x, w["conv2.w"], w["conv2.b"], 2))   # [n,64,9,9]
    x = relu(conv2d(x, w["conv3.w"], w["conv3.b"], 1))   # [n,64,7,7]
    x = x.reshape(x.shape[0], -1)                         # (c, h, w) order
    x = relu(x @ w["fc1.w"].T + w["fc1.b"])
    q = x @ w["fc2.w"][:A].T + w["fc2.b"][:A]
    return q[0] if one else q

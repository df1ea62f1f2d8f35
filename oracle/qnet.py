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


def _round_mantissa(y: np.ndarray, keep: int) -> np.ndarray:
    """Round float32 values to `keep` explicit mantissa bits, nearest even,
    on their bit patterns: add half a unit of the kept last place (minus one,
    plus the kept last bit, which makes exact halves go to even) and clear
    the dropped bits.  Finite inputs only."""
    drop = 23 - keep
    u = np.ascontiguousarray(y, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + ((1 << (drop - 1)) - 1) + ((u >> drop) & 1)
    u = u & ~np.uint64((1 << drop) - 1)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (8 significant bits, nearest even) and back: the
    float32 value first, then its mantissa to 7 explicit bits."""
    return _round_mantissa(np.asarray(x, dtype=np.float32), 7)


def round_e4m3(x: np.ndarray) -> np.ndarray:
    """Saturate to +-448 and round to OCP FP8 e4m3 (nearest even) and back:
    normal values (|x| >= 2^-6) keep 3 explicit mantissa bits; below that
    the grid is uniform with spacing 2^-9 (subnormals)."""
    y = np.clip(np.asarray(x, dtype=np.float64), -448.0, 448.0).astype(np.float32)
    normal = _round_mantissa(y, 3)
    sub = np.rint(y.astype(np.float64) * 512.0) / 512.0        # rint: nearest even
    return np.where(np.abs(y) >= 2.0 ** -6, normal, sub)


_LOWP_W: dict = {}


def _rounded_weights(w: dict, name: str, prec: str):
    """The rounded weight operand of a layer (and, for fp8, its scale),
    computed once per weight dict (the dict is kept alive by the cache)."""
    rnd = round_bf16 if prec == "bf16" else round_e4m3
    key = (id(w), name, prec, id(rnd))
    hit = _LOWP_W.get(key)
    if hit is not None and hit[0] is w and hit[3] is rnd:
        return hit[1], hit[2]
    W = w[name + ".w"]
    if prec == "bf16":
        Wq, ws = round_bf16(W), 1.0
    else:
        ws = 448.0 / float(np.abs(W).max())
        Wq = round_e4m3(W * ws)
    _LOWP_W[key] = (w, Wq, ws, rnd)
    return Wq, ws


# ---- the FP8 matrix-core dot product ---------------------------------------
# The e4m3 x e4m3 matrix instructions of gfx950 do not sum their products
# exactly (measured with single-instruction probes on fixed operands): the K
# values of one instruction fall into groups of 8 consecutive values; within a
# group, every non-zero product is truncated toward zero to a multiple of
# 2^(E - 13), where E is the largest, over the group's non-zero products, of
# the sum of the two operands' exponent fields (a subnormal operand counts as
# exponent -6; products with a zero operand take no part); the truncated
# products of a group add exactly, and the group sums add in FP32.  The FP8
# emulation sums this way, because the e4m3 code every later layer reads is
# decided from these sums.  Which K values share a group follows the order in
# which the layer's input is naturally stored: 8 consecutive pixels of one
# kernel row for conv1 (raw frames, row-major), 8 consecutive channels of one
# kernel tap (or of one pixel, for fc1) for the channels-last activations, 8
# consecutive hidden units for fc2.

_ZERO_EXP = -400.0      # exponent given to zero operands: below every real product


def _e4m3_exponent(v: np.ndarray) -> np.ndarray:
    """Exponent field of e4m3 values: floor(log2 |v|) for normal values,
    -6 for subnormal ones, _ZERO_EXP for zero."""
    _, e = np.frexp(v)
    ex = (e - 1).astype(np.float64)
    ex = np.where(np.abs(v) < 2.0 ** -6, -6.0, ex)
    return np.where(v == 0, _ZERO_EXP, ex)


def dot_fp8_groups(X: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Y[m, n] = sum_k X[m, k] W[n, k] for e4m3-valued X [M][K], W [N][K]
    (K a multiple of 8), summed as the FP8 matrix instructions sum (see
    above); the final adds are done in FP64."""
    M, K = X.shape
    N = W.shape[0]
    G = K // 8
    ex, ew = _e4m3_exponent(X), _e4m3_exponent(W)
    out = np.empty((M, N))
    step = max(1, 3_000_000 // (N * K))
    for m0 in range(0, M, step):
        x, xe = X[m0:m0 + step], ex[m0:m0 + step]
        m = x.shape[0]
        p = (x[:, None, :] * W[None, :, :]).reshape(m, N, G, 8)          # exact products
        E = (xe[:, None, :] + ew[None, :, :]).reshape(m, N, G, 8).max(axis=3)
        grid = np.exp2(E - 13.0)[..., None]
        out[m0:m0 + step] = (np.trunc(p / grid) * grid).sum(axis=(2, 3))
    return out


# the sum the FP8 emulation uses (a test may swap in the exact X @ W.T)
def fp8_dot(X: np.ndarray, W: np.ndarray) -> np.ndarray:
    return dot_fp8_groups(X, W)


def _im2col_tap_major(x: np.ndarray, kh: int, kw: int, stride: int) -> np.ndarray:
    """[n, C, H, W] -> [n, P, kh*kw*C] with K ordered (kernel row, kernel
    column, channel): channels innermost, as channels-last data stores them."""
    win = sliding_window_view(x, (kh, kw), axis=(2, 3))[:, :, ::stride, ::stride]   # n C oy ox kh kw
    n, C, oy, ox = win.shape[:4]
    return win.transpose(0, 2, 3, 4, 5, 1).reshape(n, oy * ox, kh * kw * C)


def conv_fp8(xq: np.ndarray, Wq: np.ndarray, stride: int, channels_inner: bool) -> np.ndarray:
    """Convolution sums of e4m3 operands with the FP8 matrix-core grouping:
    conv1 (raw frames) groups 8 kernel-row pixels (K order c, kh, kw), the
    channels-last layers group 8 channels (K order kh, kw, c)."""
    O, C, kh, kw = Wq.shape
    n = xq.shape[0]
    if channels_inner:
        cols = _im2col_tap_major(xq, kh, kw, stride)
        Wm = Wq.transpose(0, 2, 3, 1).reshape(O, -1)
    else:
        win = sliding_window_view(xq, (kh, kw), axis=(2, 3))[:, :, ::stride, ::stride]   # n C oy ox kh kw
        oy, ox = win.shape[2], win.shape[3]
        cols = win.transpose(0, 2, 3, 1, 4, 5).reshape(n, oy * ox, C * kh * kw)
        Wm = Wq.reshape(O, -1)
    oy = ox = int(round(np.sqrt(cols.shape[1])))
    y = fp8_dot(cols.reshape(-1, cols.shape[2]), Wm)                   # [n*P, O]
    return y.reshape(n, oy, ox, O).transpose(0, 3, 1, 2)


def qvalues_lowp(stacks: np.ndarray, w: dict, A: int, prec: str, ascale=None) -> np.ndarray:
    """Q-values with each layer's two operands rounded to a low precision
    (the emulation a BF16/FP8 matrix-core path is compared against).

    bf16: pixels (integers, exact) and weights rounded to bf16; every later
          layer input rounded to bf16; 1/255 applied after conv1's sum; the
          products summed in FP64.
    fp8:  layer l's input x and weights W enter as e4m3(x * ascale[l]) and
          e4m3(W * wscale[l]) with wscale[l] = 448 / max|W_l|; the products
          are summed as the FP8 matrix instructions sum (dot_fp8_groups) and
          the sum divided by ascale[l] * wscale[l] (and 255 for conv1).
    Biases stay exact; ReLU after every layer but the last."""
    one = stacks.ndim == 3
    s = stacks[None] if one else stacks
    layers = (("conv1", 4), ("conv2", 2), ("conv3", 1), ("fc1", 0), ("fc2", 0))
    x = s.astype(np.float64)                     # raw pixels
    for l, (name, stride) in enumerate(layers):
        b = w[name + ".b"]
        if prec == "bf16":
            Wq, _ = _rounded_weights(w, name, prec)
            xq, div = round_bf16(x), 1.0
        elif prec == "fp8":
            Wq, ws = _rounded_weights(w, name, prec)
            xq = round_e4m3(x * float(ascale[l]))
            div = float(ascale[l]) * ws
        else:
            raise ValueError(prec)
        if name == "fc2":
            Wq, b = Wq[:A], b[:A]
        if l == 0:
            div *= 255.0
        if stride:
            if prec == "fp8":
                acc = conv_fp8(xq, Wq, stride, channels_inner=l > 0)
            else:
                acc = conv2d(xq, Wq, np.zeros_like(b), stride)
            y = acc / div + b[None, :, None, None]
        else:
            if l == 3:
                if prec == "fp8":          # the fc1 input in channels-last order, weights to match
                    xq = xq.transpose(0, 2, 3, 1)
                    Wq = Wq.reshape(Wq.shape[0], 64, 7, 7).transpose(0, 2, 3, 1)
                    Wq = Wq.reshape(Wq.shape[0], -1)
                xq = xq.reshape(xq.shape[0], -1)
            acc = fp8_dot(xq, Wq) if prec == "fp8" else xq @ Wq.T
            y = acc / div + b
        x = relu(y) if l < 4 else y
    return x[0] if one else x


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

"""Seeded synthetic inputs for Batch-BFS search (environment tables, root
states, Q-network weights, request streams).

This module only draws numbers.  It holds none of the search arithmetic: no
environment step, no Q-network, no backup, no correction.  Both the FP64
oracle and the HIP path receive the arrays it returns; neither shares any
other code with the other.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used in counter form: the
i-th draw of a stream with key ``k`` is ``mix64(k + (i + 1) * GOLDEN)``, which
equals the i-th output of the sequential generator started at state ``k``.
A stream key is derived from (instance seed, purpose tag).

Workload shapes follow the paper's Atari setting (Sec. 4.1 / 5: 84x84 uint8
frames, a stack of 4, up to A = 18 actions, depths 1..4); the content is a
sprite world standing in for the emulator, and random Kaiming-uniform
Nature-DQN weights stand in for the pre-trained agents.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1

FRAME = 84
N_SPRITES = 8
STACK = 4
MAX_A = 18
SPRITE = 6

# Nature-DQN parameter shapes (conv 32@8x8/4, 64@4x4/2, 64@3x3/1, FC 512, FC A).
QNET_SHAPES = (
    ("conv1.w", (32, 4, 8, 8)), ("conv1.b", (32,)),
    ("conv2.w", (64, 32, 4, 4)), ("conv2.b", (64,)),
    ("conv3.w", (64, 64, 3, 3)), ("conv3.b", (64,)),
    ("fc1.w", (512, 3136)), ("fc1.b", (512,)),
    ("fc2.w", (MAX_A, 512)), ("fc2.b", (MAX_A,)),
)
QNET_NUMEL = sum(int(np.prod(s)) for _, s in QNET_SHAPES)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _tag64(tag: str) -> int:
    """FNV-1a 64-bit hash of a purpose tag."""
    h = 0xCBF29CE484222325
    for ch in tag.encode():
        h = ((h ^ ch) * 0x100000001B3) & _MASK
    return h


def stream_key(seed: int, tag: str) -> int:
    s = _mix64(np.uint64(seed & _MASK))
    return int(_mix64(s ^ np.uint64(_tag64(tag))))


def draws(seed: int, tag: str, n: int, start: int = 0) -> np.ndarray:
    """n uint64 draws of the stream (seed, tag), beginning at counter `start`."""
    key = np.uint64(stream_key(seed, tag))
    i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(key + i * GOLDEN)


def uniform01(seed: int, tag: str, n: int) -> np.ndarray:
    """Doubles in [0, 1) with 53 random bits: (u >> 11) * 2^-53."""
    return (draws(seed, tag, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def ints(seed: int, tag: str, n: int, mod: int) -> np.ndarray:
    return (draws(seed, tag, n) % np.uint64(mod)).astype(np.int64)


# ---------------------------------------------------------------------------
# environment tables
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class EnvParams:
    delta: np.ndarray  # int32 [18][2]: (dx, dy) of sprite 0 per action, distinct, in [-3,3]^2
    vel: np.ndarray    # int32 [7][2]: (vx, vy) of sprites 1..7, in [-2,2]^2


def env_params(seed: int) -> EnvParams:
    """Action table: 18 distinct cells of [-3,3]^2 taken by a Fisher-Yates
    shuffle of the 49 cells; velocities: (u mod 5) - 2 per component."""
    cells = [(dx, dy) for dy in range(-3, 4) for dx in range(-3, 4)]
    u = draws(seed, "env.delta", len(cells))
    for i in range(len(cells) - 1, 0, -1):
        j = int(u[i] % np.uint64(i + 1))
        cells[i], cells[j] = cells[j], cells[i]
    delta = np.array(cells[:MAX_A], dtype=np.int32)
    vel = (ints(seed, "env.vel", 14, 5) - 2).astype(np.int32).reshape(7, 2)
    return EnvParams(delta=delta, vel=vel)


# ---------------------------------------------------------------------------
# root states
# ---------------------------------------------------------------------------
def paint_sprites(pos: np.ndarray) -> np.ndarray:
    """Input image for a root stack: 6x6 squares (wrapping) at the given
    (x, y), value 128, the first one 255 on top.  Used only to make the
    root stacks handed to both implementations."""
    img = np.zeros((FRAME, FRAME), dtype=np.uint8)
    order = list(range(1, N_SPRITES)) + [0]
    for i in order:
        x, y = int(pos[i, 0]), int(pos[i, 1])
        rows = (y + np.arange(SPRITE)) % FRAME
        cols = (x + np.arange(SPRITE)) % FRAME
        img[np.ix_(rows, cols)] = 255 if i == 0 else 128
    return img


def roots(seed: int, n: int) -> tuple[np.ndarray, np.ndarray]:
    """n root states: positions int32 [n][8][2] (x, y in [0,84)) and frame
    stacks uint8 [n][4][84][84] (channel 0 oldest).  The newest frame shows
    the root positions (uniform); each older frame shows every sprite moved
    back by a seeded offset in [-3, 3]^2 (wrapping), so a stack looks like
    the last steps of a trajectory, as an agent's frame stack does.  (The
    offsets are drawn here; the world's own transition is not used.)"""
    pos = ints(seed, "roots.pos", n * N_SPRITES * 2, FRAME).reshape(n, N_SPRITES, 2).astype(np.int64)
    back = ints(seed, "roots.back", n * (STACK - 1) * N_SPRITES * 2, 7).reshape(n, STACK - 1, N_SPRITES, 2) - 3
    hist = np.empty((n, STACK, N_SPRITES, 2), dtype=np.int64)
    hist[:, STACK - 1] = pos
    for c in range(STACK - 2, -1, -1):
        hist[:, c] = (hist[:, c + 1] - back[:, c]) % FRAME
    hist = hist.astype(np.int32)
    pos = np.ascontiguousarray(hist[:, STACK - 1])
    stacks = np.empty((n, STACK, FRAME, FRAME), dtype=np.uint8)
    for r in range(n):
        for c in range(STACK):
            stacks[r, c] = paint_sprites(hist[r, c])
    return pos, stacks


# ---------------------------------------------------------------------------
# Q-network weights
# ---------------------------------------------------------------------------
def qnet_weights(seed: int) -> dict[str, np.ndarray]:
    """Kaiming-uniform (fan-in, ReLU gain) weights W ~ U(-sqrt(6/fan_in),
    +sqrt(6/fan_in)) and biases ~ U(-1/sqrt(fan_in), +1/sqrt(fan_in)), drawn
    in FP64 and rounded to FP32.  fc2 has 18 rows; a search with A actions
    uses rows 0..A-1."""
    out = {}
    for name, shape in QNET_SHAPES:
        layer = name.split(".")[0]
        wshape = dict(QNET_SHAPES)[layer + ".w"]
        fan_in = int(np.prod(wshape[1:]))
        bound = math.sqrt(6.0 / fan_in) if name.endswith(".w") else 1.0 / math.sqrt(fan_in)
        u = uniform01(seed, "qnet." + name, int(np.prod(shape)))
        out[name] = ((2.0 * u - 1.0) * bound).astype(np.float32).reshape(shape)
    return out


def qnet_blob(weights: dict[str, np.ndarray]) -> np.ndarray:
    """Flat FP32 blob in the canonical order of QNET_SHAPES."""
    return np.concatenate([weights[n].reshape(-1) for n, _ in QNET_SHAPES]).astype(np.float32)


def qnet_unblob(blob: np.ndarray) -> dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shape in QNET_SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(blob[o:o + k], dtype=np.float32).reshape(shape)
        o += k
    return out


# ---------------------------------------------------------------------------
# learned forward model (a fully connected stand-in for a learned simulator)
# ---------------------------------------------------------------------------
MLP_STATE = 100


def mlp_shapes(A: int):
    """Layer shapes in the canonical blob order ([out][in] matrices): l1 takes
    the state then the one-hot action; out has the 100 next-state units then
    the reward unit; q is the A-action leaf head on the state."""
    return (("l1.w", (100, MLP_STATE + A)), ("l1.b", (100,)),
            ("l2.w", (100, 100)), ("l2.b", (100,)),
            ("l3.w", (100, 100)), ("l3.b", (100,)),
            ("out.w", (MLP_STATE + 1, 100)), ("out.b", (MLP_STATE + 1,)),
            ("q.w", (A, MLP_STATE)), ("q.b", (A,)))


def mlp_numel(A: int) -> int:
    return sum(int(np.prod(s)) for _, s in mlp_shapes(A))


def mlp_weights(seed: int, A: int) -> dict[str, np.ndarray]:
    """Weights and biases uniform on +-1/sqrt(fan_in) (the default
    initialisation of a fully connected layer), drawn in FP64 and rounded to
    FP32; the streams are keyed by A so each action count is its own model."""
    out = {}
    shapes = mlp_shapes(A)
    for name, shape in shapes:
        layer = name.split(".")[0]
        fan_in = dict(shapes)[layer + ".w"][1]
        u = uniform01(seed, f"mlp{A}." + name, int(np.prod(shape)))
        out[name] = ((2.0 * u - 1.0) / math.sqrt(fan_in)).astype(np.float32).reshape(shape)
    return out


def mlp_blob(weights: dict[str, np.ndarray], A: int) -> np.ndarray:
    return np.concatenate([weights[n].reshape(-1) for n, _ in mlp_shapes(A)]).astype(np.float32)


def mlp_states(seed: int, n: int) -> np.ndarray:
    """n root states, FP32 [n][100], uniform on [-1, 1)."""
    u = uniform01(seed, "mlp.state", n * MLP_STATE)
    return (2.0 * u - 1.0).astype(np.float32).reshape(n, MLP_STATE)


# ---------------------------------------------------------------------------
# mixed batches and request streams
# ---------------------------------------------------------------------------
def mixed_shapes(seed: int, n: int, a_choices=(4, 6, 18), d_choices=(1, 2, 3)):
    a = np.array(a_choices)[ints(seed, "mix.A", n, len(a_choices))]
    d = np.array(d_choices)[ints(seed, "mix.d", n, len(d_choices))]
    return a.astype(np.int32), d.astype(np.int32)


def request_arrivals(seed: int, rate: float, duration: float, max_requests: int | None = None):
    """Poisson arrivals (exponential gaps -ln(1-u)/rate); A uniform on
    {4,6,18}; d in {1,2,3,4} with p = .50/.30/.15/.05; A = 18 caps d at 3.
    Returns arrival times (s), A and d."""
    n_cap = int(rate * duration * 1.5 + 64) if max_requests is None else max_requests
    gaps = -np.log1p(-uniform01(seed, "req.gap", n_cap)) / rate
    t = np.cumsum(gaps)
    keep = t < duration
    if max_requests is not None:
        keep[max_requests:] = False
    n = int(keep.sum())
    t = t[:n]
    a = np.array([4, 6, 18])[ints(seed, "req.A", n, 3)].astype(np.int32)
    u = uniform01(seed, "req.d", n)
    d = np.where(u < 0.50, 1, np.where(u < 0.80, 2, np.where(u < 0.95, 3, 4))).astype(np.int32)
    d = np.where((a == 18) & (d > 3), 3, d).astype(np.int32)
    return t, a, d


def request_stream(seed: int, rate: float, duration: float, max_requests: int | None = None):
    """request_arrivals plus one root state per request (positions, stacks)."""
    t, a, d = request_arrivals(seed, rate, duration, max_requests)
    pos, stacks = roots(seed, len(t))
    return t, a, d, pos, stacks

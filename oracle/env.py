"""Integer sprite environment of the oracle (test infrastructure only).

The paper's method needs a deterministic forward model that maps an action
sequence from the root to a trajectory (Sec. 2, "Vanilla tree search"); its
experiments use the Atari emulator with 84x84 frames stacked 4 deep (Sec. 5).
This file is the synthetic stand-in, written plainly:

* state: positions P[8][2] = (x, y) in [0,84) of 8 sprites, plus the stack
  F[4][84][84] uint8 of the last four frames (channel 0 oldest);
* step(a): sprite 0 moves by delta[a], sprite i >= 1 by vel[i-1]; every
  coordinate wraps modulo 84 (non-negative remainder);
* render: zero background; each sprite is a 6x6 square anchored at its (x, y)
  and extending +5 in x and y, wrapping; sprites 1..7 paint 128, sprite 0
  paints 255; pixels combine by max, so sprite 0 is on top;
* reward: the number of sprites 1..7 whose square overlaps sprite 0's square
  after the move, where two squares overlap when their circular distances in
  x and in y are both below 6.
"""
from __future__ import annotations

import numpy as np

W = 84          # frame side
NS = 8          # sprites
SQ = 6          # sprite square side


def wrap(v: int) -> int:
    return v % W   # Python's % is non-negative for a positive modulus


def move(pos: np.ndarray, a: int, delta: np.ndarray, vel: np.ndarray) -> np.ndarray:
    """New positions after action a."""
    out = np.empty((NS, 2), dtype=np.int64)
    out[0, 0] = wrap(int(pos[0, 0]) + int(delta[a, 0]))
    out[0, 1] = wrap(int(pos[0, 1]) + int(delta[a, 1]))
    for i in range(1, NS):
        out[i, 0] = wrap(int(pos[i, 0]) + int(vel[i - 1, 0]))
        out[i, 1] = wrap(int(pos[i, 1]) + int(vel[i - 1, 1]))
    return out


def covers(px: int, py: int, sx: int, sy: int) -> bool:
    """Does the square anchored at (sx, sy) contain pixel (px, py)?"""
    return wrap(px - sx) < SQ and wrap(py - sy) < SQ


def render(pos: np.ndarray) -> np.ndarray:
    """84x84 uint8 frame, row-major [y][x]; each square is combined by max."""
    img = np.zeros((W, W), dtype=np.uint8)
    for i in range(NS):
        val = 255 if i == 0 else 128
        sx, sy = int(pos[i, 0]), int(pos[i, 1])
        rows = [wrap(sy + dy) for dy in range(SQ)]
        cols = [wrap(sx + dx) for dx in range(SQ)]
        blk = np.ix_(rows, cols)
        img[blk] = np.maximum(img[blk], val)
    return img


def circ(t: int) -> int:
    t = wrap(t)
    return min(t, W - t)


def overlap(p: np.ndarray, q: np.ndarray) -> bool:
    return circ(int(p[0]) - int(q[0])) < SQ and circ(int(p[1]) - int(q[1])) < SQ


def reward(pos: np.ndarray) -> int:
    return sum(1 for i in range(1, NS) if overlap(pos[0], pos[i]))


def step(pos: np.ndarray, stack: np.ndarray, a: int, delta: np.ndarray, vel: np.ndarray):
    """One transition: (new positions, new stack, integer reward).  The reward
    is taken on the positions after the move."""
    p2 = move(pos, a, delta, vel)
    frame = render(p2)
    s2 = np.concatenate([stack[1:], frame[None]], axis=0)
    return p2, s2, reward(p2)

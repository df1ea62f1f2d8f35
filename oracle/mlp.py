"""A learned forward model in place of the simulator, FP64 (test
infrastructure only).

Sec. 4.1 times tree search on a deep network that mimics a learned forward
model: three randomly initialised hidden layers of width 100, fed a
100-dimensional state and a one-hot action (A = 2 or 10).  Readings where the
paper is silent (all of them are stated again where the library follows
them):

* the model maps x = [s ; onehot(a)] through h1 = ReLU(W1 x + b1),
  h2 = ReLU(W2 h1 + b2), h3 = ReLU(W3 h2 + b3) to a linear output layer of 101
  units: units 0..99 are the next state, unit 100 the reward;
* a leaf state is valued by a linear head Q(s, .) = Wq s + bq (A outputs);
* the initialisation is the default of a fully connected layer in the
  paper's framework: weights and biases uniform on +-1/sqrt(fan_in).

The search itself is the one of the sprite world: the d-step value of Eq. 1
by recursive depth-first search, and the BCTS correction of Eq. 3 with B of
Eq. 6 (or the exact bias gap of Lemma 3.2), reusing ``search.penalty`` and
the same readings (|delta|, mean over the other actions, natural log, no
correction at depth 0).
"""
from __future__ import annotations

import math

import numpy as np

from . import search as S

STATE = 100
HIDDEN = 100


def prepare(weights: dict) -> dict:
    """FP32 weight arrays promoted exactly to FP64."""
    return {k: np.asarray(v, dtype=np.float64) for k, v in weights.items()}


def relu(x):
    return np.maximum(x, 0.0)


def step(w: dict, s: np.ndarray, a: int, A: int):
    """(next state, reward) of the forward model for state s and action a."""
    x = np.concatenate([s, np.eye(A)[a]])
    h = relu(w["l1.w"] @ x + w["l1.b"])
    h = relu(w["l2.w"] @ h + w["l2.b"])
    h = relu(w["l3.w"] @ h + w["l3.b"])
    o = w["out.w"] @ h + w["out.b"]
    return o[:STATE], float(o[STATE])


def qvalues(w: dict, s: np.ndarray, A: int) -> np.ndarray:
    """The leaf head Q(s, .) = Wq s + bq."""
    return w["q.w"][:A] @ s + w["q.b"][:A]


def dfs(w: dict, s, k: int, d: int, A: int, gamma: float) -> float:
    """Value of a node at level k: max_a Q(s, a) at level d, otherwise
    max_a [ r_a + gamma * value(child_a) ]."""
    if k == d:
        return float(qvalues(w, s, A).max())
    best = -math.inf
    for a in range(A):
        s1, r = step(w, s, a, A)
        best = max(best, r + gamma * dfs(w, s1, k + 1, d, A, gamma))
    return best


def root_values(w: dict, s, d: int, A: int, gamma: float) -> np.ndarray:
    """Q_d(s, a) for every root action (Eq. 1), d >= 1."""
    out = np.empty(A)
    for a in range(A):
        s1, r = step(w, s, a, A)
        out[a] = r + gamma * dfs(w, s1, 1, d, A, gamma)
    return out


def search(w: dict, s, d: int, A: int, gamma: float, correction: bool = True, c: float = 1.0,
           mode: str = "eq6") -> S.Result:
    """One root of the forward-model world: the corrected root vector and its
    action, exactly as ``search.search`` does for the sprite world."""
    q0 = qvalues(w, s, A)
    if d == 0:
        return S.Result(action=S.argmax_low(q0), q=q0.copy(), q0=q0, ties=S.tie_set(q0))
    qd = root_values(w, s, d, A, gamma)
    if not correction:
        return S.Result(action=S.argmax_low(qd), q=qd.copy(), q_d=qd, ties=S.tie_set(qd))
    pi_o = S.argmax_low(q0)
    delta = np.empty(A)
    for a in range(A):
        s1, r = step(w, s, a, A)
        delta[a] = r + gamma * float(qvalues(w, s1, A).max()) - q0[a]
    do = abs(delta[pi_o])
    de = float(np.mean([abs(delta[a]) for a in range(A) if a != pi_o]))
    if mode == "eq6":
        B = S.penalty(de, do, A, d)
    else:
        from . import gev
        B = gev.exact_gap(de / math.sqrt(2.0), do / math.sqrt(2.0), A, d)
    q = qd.copy()
    for a in range(A):
        if a != pi_o:
            q[a] = qd[a] - c * gamma ** d * B
    return S.Result(action=S.argmax_low(q), q=q, q_d=qd, q0=q0, pi_o=pi_o, delta=delta, B=B,
                    ties=S.tie_set(q))

"""Exhaustive tree search with the BCTS correction, FP64 (test infrastructure
only).

What is computed (and where the paper defines it):

* the d-step value Q_d(s, a) = max over a_1..a_{d-1} and the leaf action a_d
  of  sum_{t<d} gamma^t r_t + gamma^d Q(s_d, a_d),  with s_0 = s, a_0 = a
  (Eq. 1) -- here by plain recursive depth-first search, the non-parallel
  search the paper compares Batch-BFS against (Sec. 4.1);
* the root network values Q_0 = Q(s_0, .) and pi_o = argmax Q_0 (Sec. 3.2);
* the Bellman errors at depth 0/1: delta(a) = r(s_0, a) + gamma max_a'
  Q(s_1^a, a') - Q(s_0, a) (Prop. 3.6 and the paragraph after it);
* the penalty B(d_e, d_o, A, d) = sqrt(log A) (d_e sqrt(d) - d_o sqrt(d-1))
  - (d_e - d_o) / sqrt(8) (Eq. 6), with d_o = |delta(pi_o)| and d_e the mean
  of |delta(a)| over a != pi_o;
* the corrected root vector: Q_d(s, a) - c gamma^d B for a != pi_o, and
  Q_d(s, pi_o) unchanged (Eq. 3, with B in place of B_e - B_o and the
  constant multiplier c of Sec. 5.1); the action is its argmax (Eq. 4),
  lowest index on ties.

Readings where the paper is silent: the log is natural; delta enters through
its magnitude; depth 0 applies no correction (the pre-trained agent itself);
depth 1 uses Eq. 6 as written.

``enumerate_nodes`` lists every tree node in the index order of Alg. 1: the
child of node j by action a has index j*A + a, so the root action of leaf i is
floor(i / A^(d-1)).
"""
from __future__ import annotations

import math
from fractions import Fraction
from dataclasses import dataclass, field

import numpy as np

from . import env as E
from . import qnet as Q

TIE_REL = 1e-6


@dataclass
class World:
    delta: np.ndarray   # int [18][2]
    vel: np.ndarray     # int [7][2]
    w64: dict           # FP64 Q-network weights (qnet.prepare)


def qmax(world: World, stacks: np.ndarray, A: int, qfn=None) -> np.ndarray:
    """max_a Q(s, a) for a batch of stacks; `qfn(stacks, A)` replaces the
    FP64 network (e.g. by its low-precision emulation)."""
    q = Q.qvalues(stacks, world.w64, A) if qfn is None else qfn(stacks, A)
    return q.max(axis=1)


def children(world: World, pos, stack, A: int):
    return [E.step(pos, stack, a, world.delta, world.vel) for a in range(A)]


def dfs(world: World, pos, stack, k: int, d: int, A: int, gamma: float, qfn=None) -> float:
    """Value of a node at level k < d: max_a [ r_a + gamma * value(child_a) ],
    where a node at level d is worth max_a Q(s, a)."""
    kids = children(world, pos, stack, A)
    if k + 1 == d:
        v = qmax(world, np.stack([s for _, s, _ in kids]), A, qfn)
        return max(r + gamma * float(v[a]) for a, (_, _, r) in enumerate(kids))
    return max(r + gamma * dfs(world, p, s, k + 1, d, A, gamma, qfn) for p, s, r in kids)


def root_values(world: World, pos, stack, d: int, A: int, gamma: float, qfn=None) -> np.ndarray:
    """Q_d(s_0, a) for every root action a (Eq. 1); d >= 1."""
    assert d >= 1
    out = np.empty(A)
    for a, (p, s, r) in enumerate(children(world, pos, stack, A)):
        if d == 1:
            out[a] = r + gamma * float(qmax(world, s[None], A, qfn)[0])
        else:
            out[a] = r + gamma * dfs(world, p, s, 1, d, A, gamma, qfn)
    return out


def penalty(de: float, do: float, A: int, d: int) -> float:
    """B of Eq. 6 (natural log)."""
    return math.sqrt(math.log(A)) * (de * math.sqrt(d) - do * math.sqrt(d - 1)) - (de - do) / math.sqrt(8.0)


def argmax_low(v) -> int:
    v = np.asarray(v)
    return int(np.flatnonzero(v == v.max())[0])


def tie_set(v, rel: float = TIE_REL) -> list[int]:
    v = np.asarray(v, dtype=np.float64)
    m = float(v.max())
    return [int(a) for a in np.flatnonzero(v >= m - rel * max(1.0, abs(m)))]


@dataclass
class Result:
    action: int
    q: np.ndarray                       # the returned root vector
    q_d: np.ndarray | None = None       # uncorrected d-step values
    q0: np.ndarray | None = None
    pi_o: int | None = None
    delta: np.ndarray | None = None
    B: float | None = None
    ties: list = field(default_factory=list)


def search(world: World, pos, stack, d: int, A: int, gamma: float,
           correction: bool = True, c: float = 1.0, mode: str = "eq6",
           leaf_qfn=None, corr_qfn=None) -> Result:
    """One root: the returned vector and action of the corrected search.
    mode "eq6" uses B of Eq. 6; mode "gev" uses the exact bias gap of
    Lemma 3.2 with sigma = |delta| / sqrt(2).  `leaf_qfn` evaluates the
    leaves (and the root at depth 0), `corr_qfn` the root and depth-1 nodes
    the correction reads; both default to the FP64 network."""
    if d == 0:
        q0 = Q.qvalues(stack, world.w64, A) if leaf_qfn is None else leaf_qfn(stack[None], A)[0]
        return Result(action=argmax_low(q0), q=q0.copy(), q0=q0, ties=tie_set(q0))
    qd = root_values(world, pos, stack, d, A, gamma, leaf_qfn)
    if not correction:
        return Result(action=argmax_low(qd), q=qd.copy(), q_d=qd, ties=tie_set(qd))
    q0 = Q.qvalues(stack, world.w64, A) if corr_qfn is None else corr_qfn(stack[None], A)[0]
    pi_o = argmax_low(q0)
    delta = np.empty(A)
    for a, (p, s, r) in enumerate(children(world, pos, stack, A)):
        delta[a] = r + gamma * float(qmax(world, s[None], A, corr_qfn)[0]) - q0[a]
    do = abs(delta[pi_o])
    de = float(np.mean([abs(delta[a]) for a in range(A) if a != pi_o]))
    if mode == "eq6":
        B = penalty(de, do, A, d)
    else:
        from . import gev
        B = gev.exact_gap(de / math.sqrt(2.0), do / math.sqrt(2.0), A, d)
    q = qd.copy()
    for a in range(A):
        if a != pi_o:
            q[a] = qd[a] - c * gamma ** d * B
    return Result(action=argmax_low(q), q=q, q_d=qd, q0=q0, pi_o=pi_o, delta=delta, B=B,
                  ties=tie_set(q))


def search_lowp(world: World, pos, stack, d: int, A: int, gamma: float, prec: str, ascale=None,
                correction: bool = True, c: float = 1.0, mode: str = "eq6",
                corr_prec: str = "fp64") -> Result:
    """The search of `search` with every leaf (and the root at depth 0)
    scored by the emulation of a low-precision network (``qnet.qvalues_lowp``:
    each layer's operands rounded to `prec`, the sums in FP64).  The root and
    depth-1 evaluations the correction reads use `corr_prec`: "fp64" (the
    exact network; a matrix-core path that keeps them in FP32 is compared
    against this) or the leaves' `prec`."""
    def lowp(stacks, A_):
        return Q.qvalues_lowp(stacks, world.w64, A_, prec, ascale=ascale)
    return search(world, pos, stack, d, A, gamma, correction, c, mode, leaf_qfn=lowp,
                  corr_qfn=None if corr_prec == "fp64" else lowp)


def enumerate_nodes(world: World, pos, stack, d: int, A: int):
    """Per level k = 1..d: positions [A^k][8][2], frames [A^k][84][84] and
    rewards [A^k], node index = parent index * A + action."""
    levels = []
    cur = [(np.asarray(pos, dtype=np.int64), np.asarray(stack))]
    for _ in range(d):
        nxt, P, F, R = [], [], [], []
        for p, s in cur:
            for a in range(A):
                p2, s2, r = E.step(p, s, a, world.delta, world.vel)
                nxt.append((p2, s2))
                P.append(p2)
                F.append(s2[-1])
                R.append(r)
        levels.append((np.array(P, dtype=np.int32), np.array(F, dtype=np.uint8),
                       np.array(R, dtype=np.int32)))
        cur = nxt
    return levels


def node_path(i: int, k: int, A: int) -> list[int]:
    """Actions (a_0..a_{k-1}) leading to node i of level k."""
    acts = []
    for _ in range(k):
        acts.append(i % A)
        i //= A
    return acts[::-1]


def node_at(world: World, pos, stack, acts):
    """Walk an action sequence from the root: (positions, stack, rewards)."""
    p, s, rs = np.asarray(pos, dtype=np.int64), np.asarray(stack), []
    for a in acts:
        p, s, r = E.step(p, s, a, world.delta, world.vel)
        rs.append(r)
    return p, s, rs


# ---- the FP32 returns a pruned search ranks by --------------------------
# Pruning decides which nodes survive by comparing discounted returns, so
# both sides must take that decision on the same values.  The rule (stated
# here and followed by the library): with g = the FP32 value of gamma,
#   * the discount of a level-k reward is d_k = RN32(g^(k-1)), the FP32 value
#     nearest the exact power (ties to even);
#   * a level-k node's FP32 return is R_k = RN32(R_{k-1} + d_k * r_k) with
#     R_0 = 0: the exact product and sum, rounded once (a fused
#     multiply-add).
# Both roundings are taken here on exact rationals.

def round_f32(x: Fraction) -> float:
    """The FP32 value nearest the exact rational x, ties to even (normal
    range and zero; subnormal and overflowing values do not occur here)."""
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    x = abs(x)
    e = x.numerator.bit_length() - x.denominator.bit_length()      # 2^e <= x < 2^(e+2)
    while Fraction(2) ** e > x:
        e -= 1
    while Fraction(2) ** (e + 1) <= x:
        e += 1
    assert -126 <= e <= 127, e
    scaled = x / Fraction(2) ** (e - 23)                       # in [2^23, 2^24)
    m = scaled.numerator // scaled.denominator
    rest = scaled - m
    if rest > Fraction(1, 2) or (rest == Fraction(1, 2) and m % 2 == 1):
        m += 1
    return sign * float(Fraction(m) * Fraction(2) ** (e - 23))


def level_discounts_f32(gamma: float, d: int) -> list:
    """[d_1, .., d_d] with d_k = RN32(g^(k-1)), g the FP32 value of gamma."""
    g = Fraction(float(np.float32(gamma)))
    return [round_f32(g ** (k - 1)) for k in range(1, d + 1)]


def ret_step_f32(prev: float, dk: float, r: int) -> float:
    """R_k = RN32(R_{k-1} + d_k r_k), one rounding of the exact value."""
    return round_f32(Fraction(prev) + Fraction(dk) * r)


def beam_levels(world: World, pos, stack, d: int, A: int, gamma: float, beam: int):
    """The levels of the pruned search (rule: see search_beam).  Returns, per
    level k = 1..d, (nodes, kept): nodes lists every expanded node of level k
    -- the A children of each kept node of level k-1, in that order -- as
    (a0, path, positions, stack, reward, R64, R32); kept is None for an
    uncut level, else the indices (into nodes) of the survivors, root action
    by root action, ascending."""
    gps = level_discounts_f32(gamma, d)
    out = []
    level = [(a, [a], p1, s1, r, float(r), ret_step_f32(0.0, gps[0], r))
             for a, (p1, s1, r) in enumerate(children(world, pos, stack, A))]
    for k in range(1, d + 1):
        if k > 1:
            nxt = []
            for (a0, path, pk, sk, _, R64, R32) in level:
                for a, (p1, s1, r) in enumerate(children(world, pk, sk, A)):
                    nxt.append((a0, path + [a], p1, s1, r, R64 + gamma ** (k - 1) * r, ret_step_f32(R32, gps[k - 1], r)))
            level = nxt
        kept = None
        if beam > 0 and 2 <= k <= d - 1:
            blocks = [[i for i, nd in enumerate(level) if nd[0] == a0] for a0 in range(A)]
            if any(len(b) > beam for b in blocks):
                kept = []
                for blk in blocks:
                    if len(blk) > beam:
                        blk = sorted(sorted(blk, key=lambda i: (-level[i][6], i))[:beam])
                    kept.extend(blk)
        out.append((level, kept))
        if kept is not None:
            level = [level[i] for i in kept]
    return out


def search_beam(world: World, pos, stack, d: int, A: int, gamma: float, beam: int,
                correction: bool = True, c: float = 1.0, mode: str = "eq6") -> Result:
    """Pruned Batch-BFS: the paper leaves early pruning to future work and
    only sketches it (an index array of unpruned states, updated at each
    pruning step, then used to trace the root action, Sec. 4).  The rule read
    here: the tree grows level by level as in Alg. 1; at every level
    k = 2..d-1, inside each root action's sub-tree, only the `beam` nodes
    with the largest discounted return so far are expanded further (ties:
    lowest index; ranked on the FP32 returns of the rule above, so both sides
    take the same decision); the leaves are all children of the kept
    level-(d-1) nodes.  Q_d(a0) is the max over a0's surviving leaves of
    R + gamma^d max_a Q (FP64); the depth-0/1 quantities of the correction
    are untouched.  beam = 0 is the exhaustive search."""
    if beam == 0 or d <= 2:
        return search(world, pos, stack, d, A, gamma, correction, c, mode)
    level = [(nd[0], nd[2], nd[3], nd[5], nd[6]) for nd in beam_levels(world, pos, stack, d, A, gamma, beam)[-1][0]]
    qd = np.full(A, -np.inf)
    stacks = np.stack([nd[2] for nd in level])
    vmax = Q.qvalues(stacks, world.w64, A).max(axis=1)
    for nd, v in zip(level, vmax):
        qd[nd[0]] = max(qd[nd[0]], nd[3] + gamma ** d * float(v))
    q0 = Q.qvalues(stack, world.w64, A)
    if not correction:
        return Result(action=argmax_low(qd), q=qd.copy(), q_d=qd, ties=tie_set(qd))
    pi_o = argmax_low(q0)
    delta = np.empty(A)
    for a, (p, s, r) in enumerate(children(world, pos, stack, A)):
        delta[a] = r + gamma * float(qmax(world, s[None], A)[0]) - q0[a]
    do = abs(delta[pi_o])
    de = float(np.mean([abs(delta[a]) for a in range(A) if a != pi_o]))
    if mode == "eq6":
        B = penalty(de, do, A, d)
    else:
        from . import gev
        B = gev.exact_gap(de / math.sqrt(2.0), do / math.sqrt(2.0), A, d)
    q = qd.copy()
    for a in range(A):
        if a != pi_o:
            q[a] = qd[a] - c * gamma ** d * B
    return Result(action=argmax_low(q), q=q, q_d=qd, q0=q0, pi_o=pi_o, delta=delta, B=B, ties=tie_set(q))

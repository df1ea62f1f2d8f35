"""BF16 / FP8 parity of the matrix-core path against the oracle's emulation of
the same operand roundings (``qnet.qvalues_lowp``: every layer's operands
rounded as the kernels round them, the sums in FP64), through the C ABI.

Two levels:
* the Q-network on real sibling groups (the A children of one node share
  stack channels 0..2, and the fused kernel sums that shared part of conv1
  once per group): ``bcts_debug_qnet_siblings`` against ``qvalues_lowp``;
* whole searches (fused kernel, sibling groups of 4, 6 and 18, the FP32
  correction evaluations) against ``search.search_lowp``: the small
  configuration, a mixed batch and 8 roots of the headline configuration.

Bars (relative to each stack's / root's largest |Q|):
* BF16: median <= 1e-4 and max <= 2e-3.  The two sides differ only by FP32
  against FP64 summation, which can move an activation across a BF16
  rounding boundary (one BF16 step is 2^-8 of that activation);
* FP8:  median <= 1e-4, at most 1 in 8 stacks (roots) above 1e-3, max <=
  5e-2.  The emulation sums as the FP8 matrix instructions do
  (``qnet.dot_fp8_groups``: products truncated per group of 8), so the two
  sides differ only where the hardware's FP32 addition of the group sums
  and the emulation's FP64 addition put a pre-activation on two sides of an
  e4m3 rounding boundary; one e4m3 step is 2^-3 = 12.5% of the activation
  it rounds, so such a flip moves Q by up to a few per cent, and flips are
  rare, which the count bound checks.
Against the FP64 search every root also meets a max bound: its error is at
most the emulation's own distance from FP64 (the operand rounding alone,
computed by the oracle) plus the emulation bar.
Root actions must agree with the emulated search's, up to actions whose
values lie within the root's measured error of the best one.  Where
the FP64 root values are themselves within FP32 rounding of a tie for pi_o,
the root is excused (the GPU's FP32 correction evaluations may pick the other
action and shift the vector differently).
"""
import multiprocessing as mp
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from oracle import env as E, qnet as Q, search as S
from paper_2107_01715_amd import workload as W

pytestmark = pytest.mark.gpu
GAMMA = 0.99
BARS = {"BF16": dict(med=1e-4, mx=2e-3, cnt_tol=None, cnt_frac=0.0),
        "FP8": dict(med=1e-4, mx=5e-2, cnt_tol=1e-3, cnt_frac=1 / 8)}


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_01715_amd import bcts
    return bcts


def make_ctx(lib, seed):
    ep = W.env_params(seed)
    ctx = lib.Context(0)
    ctx.set_env(ep.delta, ep.vel)
    ctx.set_qnet(W.qnet_blob(W.qnet_weights(7)))
    _, cal = W.roots(2003, 64)
    ctx.calibrate_fp8(cal)
    return ctx, S.World(ep.delta, ep.vel, Q.prepare(W.qnet_weights(7)))


def check_bars(rel, prec, what):
    b = BARS[prec]
    rel = np.asarray(rel)
    print(f"{prec} {what}: median {np.median(rel):.3g}, max {rel.max():.3g}, "
          f"> 1e-3: {(rel > 1e-3).sum()}/{rel.size}")
    assert np.median(rel) <= b["med"], (what, np.median(rel))
    assert rel.max() <= b["mx"], (what, rel.max())
    if b["cnt_tol"] is not None:
        assert (rel > b["cnt_tol"]).sum() <= b["cnt_frac"] * rel.size, (what, np.sort(rel)[-8:])


def sibling_stacks(world, seed, A, n_parents):
    """Real sibling groups: the A children of the root and of its first
    depth-1 nodes, n_parents parents per root."""
    pos, st = W.roots(seed, n_parents)
    out = []
    for r in range(n_parents):
        for a0 in range(2 if A < 18 else 1):
            p, s, _ = E.step(pos[r], st[r], a0, world.delta, world.vel) if a0 else (pos[r], st[r], 0)
            for a in range(A):
                out.append(E.step(p, s, a, world.delta, world.vel)[1])
    return np.stack(out)


@pytest.mark.parametrize("prec,k128", [("BF16", 0), ("FP8", 1), ("FP8", 0)])
def test_sibling_groups_match_emulation(lib, prec, k128):
    """The fused kernel on sibling groups against the emulation; FP8 with
    conv2 / conv3 on the K = 128 instruction (the default) and the K = 32
    one, in rounds of 3 and 4 stacks."""
    ctx, world = make_ctx(lib, 1003)
    try:
        ctx.set_precision(getattr(lib, prec))
        ctx.set_tuning(lib.TUNE_FP8_K128, k128)
        ascale = ctx.get_fp8_scales()
        rels = []
        for A, npar in ((18, 3), (6, 4), (4, 4)):
            x = sibling_stacks(world, 3100 + A, A, npar)
            got = ctx.debug_qnet_siblings(x, 18, A)
            want = Q.qvalues_lowp(x, world.w64, 18, prec.lower(), ascale=ascale)
            rels.append(np.abs(got - want).max(axis=1) / np.abs(want).max(axis=1))
            # the grouping never changes a stack's arithmetic, nor the round size
            np.testing.assert_array_equal(got, ctx.debug_qnet_siblings(x, 18, 1))
            if prec == "FP8":
                ctx.set_tuning(lib.TUNE_FUSED_ROUND, 4)
                np.testing.assert_array_equal(got, ctx.debug_qnet_siblings(x, 18, A))
                ctx.set_tuning(lib.TUNE_FUSED_ROUND, 3)
        check_bars(np.concatenate(rels), prec, "sibling-group stacks vs emulation")
    finally:
        ctx.close()


def test_sibling_groups_reject_unshared_frames(lib):
    ctx, world = make_ctx(lib, 1003)
    try:
        _, st = W.roots(5, 4)
        with pytest.raises(lib.BctsError) as e:
            ctx.debug_qnet_siblings(st, 18, 4)       # independent roots share nothing
        assert e.value.status == lib.E_INVAL
    finally:
        ctx.close()


def _lowp_root(args):
    seed, r, n, d, A, prec, ascale = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        ep = W.env_params(seed)
        world = S.World(ep.delta, ep.vel, Q.prepare(W.qnet_weights(7)))
        pos, st = W.roots(seed, n)
        res = S.search_lowp(world, pos[r], st[r], d, A, GAMMA, prec, ascale=ascale)
        ref = S.search(world, pos[r], st[r], 0, A, GAMMA)         # FP64 root values (pi_o)
        full = S.search(world, pos[r], st[r], d, A, GAMMA)        # the FP64 search itself
        return res.q, res.action, res.ties, ref.q, full.q


def lowp_refs(seed, n, roots, d, A, prec, ascale):
    jobs = [(seed, int(r), n, int(d[i]), int(A[i]), prec, None if ascale is None else list(ascale))
            for i, r in enumerate(roots)]
    with ProcessPoolExecutor(max_workers=min(16, len(jobs)), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_lowp_root, jobs))


def compare_roots(act, q, refs, Avec, prec, what):
    """Against the emulated search (the bars above) and, per root, a max
    bound against the FP64 search: the GPU's distance from FP64 is at most
    the emulation's own (the operand rounding, computed by the oracle) plus
    the emulation bar."""
    rels, excused = [], 0
    far = []
    for i, (qo, ao, ties, q0, q64) in enumerate(refs):
        A = int(Avec[i])
        q64 = np.asarray(q64)
        scale = np.abs(q64).max()
        e_gpu = np.abs(q[i, :A].astype(np.float64) - q64).max() / scale
        e_emu = np.abs(np.asarray(qo) - q64).max() / scale
        far.append(e_gpu)
        assert e_gpu <= e_emu + BARS[prec]["mx"], (what, i, e_gpu, e_emu)
    print(f"{prec} {what}: max error against FP64 {max(far):.3g} (mean {np.mean(far):.3g})")
    for i, (qo, ao, ties, q0, _) in enumerate(refs):
        A = int(Avec[i])
        qo = np.asarray(qo)
        top = np.sort(q0)[-2:]
        if top[1] - top[0] <= 1e-5 * max(1.0, abs(top[1])):   # pi_o itself within FP32 rounding of a tie
            excused += 1
            continue
        err = np.abs(q[i, :A].astype(np.float64) - qo).max()
        rels.append(err / np.abs(qo).max())
        # the action is the emulated search's, up to values within the
        # measured error of its best one (and its own ties)
        near = np.flatnonzero(qo >= qo.max() - 2 * err - 1e-6 * max(1.0, abs(qo.max())))
        assert act[i] == ao or act[i] in ties or act[i] in near, (what, i, act[i], ao, ties, err)
    print(f"{what}: {excused} root(s) excused for a pi_o tie")
    check_bars(rels, prec, what)


@pytest.mark.parametrize("prec", ["BF16", "FP8"])
def test_small_configuration_matches_lowp_search(lib, prec):
    """64 roots, A = 4, depth 2: every root against the emulated search."""
    ctx, _ = make_ctx(lib, 1001)
    try:
        ctx.set_precision(getattr(lib, prec))
        pos, st = W.roots(1001, 64)
        act, q = ctx.search(pos, st, 2, 4, GAMMA, lib.correction(True, 1.0))
        ascale = ctx.get_fp8_scales() if prec == "FP8" else None
    finally:
        ctx.close()
    n = 64
    refs = lowp_refs(1001, n, range(n), [2] * n, [4] * n, prec.lower(), ascale)
    compare_roots(act, q, refs, [4] * n, prec, "small configuration")


@pytest.mark.parametrize("prec", ["BF16", "FP8"])
def test_mixed_batch_matches_lowp_search(lib, prec):
    """24 roots of A in {4, 6, 18} and depth 1..3 (A = 18 capped at 2) in one
    batch: groups of 4, 6 and 18 siblings and single roots in one launch."""
    ctx, _ = make_ctx(lib, 1004)
    n = 24
    pos, st = W.roots(1004, n)
    A, d = W.mixed_shapes(1004, n, (4, 6, 18), (1, 2, 3))
    d = np.where(A == 18, np.minimum(d, 2), d)
    try:
        ctx.set_precision(getattr(lib, prec))
        act, q = ctx.search_batch(pos, st, d, A, GAMMA, lib.correction(True, 1.0))
        ascale = ctx.get_fp8_scales() if prec == "FP8" else None
    finally:
        ctx.close()
    refs = lowp_refs(1004, n, range(n), d, A, prec.lower(), ascale)
    compare_roots(act, q, refs, A, prec, "mixed batch")


def test_headline_roots_match_lowp_search(lib):
    """8 roots of the headline configuration (A = 18, depth 3, 5,832 leaves
    each), BF16 in the benchmark's launch shape, against the emulated search."""
    ctx, _ = make_ctx(lib, 1003)
    pos, st = W.roots(1003, 256)
    try:
        ctx.set_precision(lib.BF16)
        ctx.set_tuning(lib.TUNE_FUSED_ROUND, 3)
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 1048576)
        act, q = ctx.search(pos, st, 3, 18, GAMMA, lib.correction(True, 1.0))
    finally:
        ctx.close()
    sample = [0, 31, 64, 97, 130, 178, 211, 255]
    refs = lowp_refs(1003, 256, sample, [3] * 8, [18] * 8, "bf16", None)
    compare_roots(act[sample], q[sample], refs, [18] * 8, "BF16", "headline roots")

"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: frames, positions and rewards bit-exact; FP32 root vectors within
1e-5 of the oracle's largest |Q| per root (1e-7 absolute floor); root
actions equal unless the oracle's best two are within 1e-6 max(1, |max|).
"""
import numpy as np
import pytest

from oracle import qnet as Q, search as S
from paper_2107_01715_amd import workload as W

pytestmark = pytest.mark.gpu

GAMMA = 0.99
RTOL = 1e-5


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_01715_amd import bcts
    return bcts


@pytest.fixture(scope="module")
def setup(lib):
    ep = W.env_params(1001)
    w = W.qnet_weights(7)
    ctx = lib.Context(0)
    ctx.set_env(ep.delta, ep.vel)
    ctx.set_qnet(W.qnet_blob(w))
    world = S.World(ep.delta, ep.vel, Q.prepare(w))
    yield ctx, world, w
    ctx.close()


def assert_root_parity(q_gpu, act_gpu, ref, A, tag=""):
    qo = np.asarray(ref.q, dtype=np.float64)
    err = np.abs(np.asarray(q_gpu[:A], dtype=np.float64) - qo).max()
    bound = RTOL * np.abs(qo).max() + 1e-7
    assert err <= bound, f"{tag}: |dQ| {err:.3g} > {bound:.3g}\n gpu {q_gpu[:A]}\n ref {qo}"
    assert act_gpu == ref.action or act_gpu in ref.ties, f"{tag}: action {act_gpu} vs {ref.action} ties {ref.ties}"


@pytest.mark.parametrize("A,d,seed,roots", [(4, 2, 1001, range(0, 64, 9)), (6, 3, 1002, [0, 7]),
                                            (18, 2, 1003, [3]), (18, 3, 1003, [0]), (2, 6, 5, [1])])
def test_expansion_bit_exact(lib, setup, A, d, seed, roots):
    ctx, world, _ = setup
    pos, st = W.roots(seed, max(roots) + 1)
    for r in roots:
        got = ctx.debug_expand(pos[r], st[r], d, A)
        want = S.enumerate_nodes(world, pos[r], st[r], d, A)
        for k in range(d):
            gp, gf, gr = got[k]
            wp, wf, wr = want[k]
            assert np.array_equal(gp, wp), f"positions, level {k + 1}"
            assert np.array_equal(gr, wr), f"rewards, level {k + 1}"
            bad = np.flatnonzero((gf != wf).reshape(len(gf), -1).any(axis=1))
            assert bad.size == 0, f"frames differ at level {k + 1} nodes {bad[:8]}"


def test_qnet_fp32_matches_oracle(lib, setup):
    ctx, world, _ = setup
    _, st = W.roots(11, 40)
    dense = np.random.default_rng(3).integers(0, 256, size=(9, 4, 84, 84), dtype=np.uint8)
    x = np.concatenate([st, dense])
    ctx.set_precision(lib.FP32)
    for A in (18, 5):
        got = ctx.debug_qnet(x, A)
        want = Q.qvalues(x, world.w64, A)
        err = np.abs(got - want).max(axis=1)
        bound = RTOL * np.abs(want).max(axis=1) + 1e-6
        assert (err <= bound).all(), (err / np.abs(want).max(axis=1)).max()


def _sibling_stacks(world, seed, A, n_parents):
    """The A children of n_parents roots: stacks that share channels 0..2."""
    from oracle import env as E
    pos, st = W.roots(seed, n_parents)
    return np.stack([E.step(pos[r], st[r], a, world.delta, world.vel)[1]
                     for r in range(n_parents) for a in range(A)])


def test_fp32_sibling_groups_match_oracle(lib, setup):
    """FP32 conv1 by sibling groups (channels 0..2 summed once per group, each
    sibling's channel 3 added to a copy): groups of 18, 6, 4 and a ragged
    last group against the FP64 oracle at the FP32 bar, and bit for bit equal
    to the same stacks evaluated one by one and with the grouping off.  (At
    these sizes the default choice would run conv1 per stack: the grouping is
    forced on.)"""
    ctx, world, _ = setup
    ctx.set_precision(lib.FP32)
    try:
        ctx.set_tuning(lib.TUNE_CONV1_GROUPS, 2)
        for A, npar, group in ((18, 3, 18), (6, 5, 6), (4, 7, 4), (5, 3, 4)):
            x = _sibling_stacks(world, 3300 + A, A, npar)
            if group != A:      # groups of 4 over parents of 5 children: keep whole parents per group
                x = np.concatenate([x[r * A:r * A + group] for r in range(npar)] + [x[:1]])
            got = ctx.debug_qnet_siblings(x, 18, group)
            want = Q.qvalues(x, world.w64, 18)
            err = np.abs(got - want).max(axis=1)
            assert (err <= RTOL * np.abs(want).max(axis=1) + 1e-6).all(), (A, (err / np.abs(want).max(axis=1)).max())
            np.testing.assert_array_equal(got, ctx.debug_qnet(x, 18))
            ctx.set_tuning(lib.TUNE_CONV1_GROUPS, 0)
            np.testing.assert_array_equal(got, ctx.debug_qnet_siblings(x, 18, group))
            ctx.set_tuning(lib.TUNE_CONV1_GROUPS, 2)
    finally:
        ctx.set_tuning(lib.TUNE_CONV1_GROUPS, 1)


def test_conv1_groups_searches_bit_identical(lib, setup):
    """Whole searches with conv1 by sibling groups equal those with conv1 per
    stack, bit for bit: FP32 (every layer-path chunk), BF16 (its FP32
    correction evaluations, groups of A depth-1 nodes and single roots), BF16
    and FP8 with fusion off (their leaves through the group kernel too),
    on a mixed batch with A in {4, 6, 18}, d in {1, 2, 3}, in small chunks
    so that groups end at chunk edges; the default per-chunk choice (which
    here takes both kernels) agrees with both."""
    ctx, _, _ = setup
    A, d = W.mixed_shapes(1006, 120, (4, 6, 18), (1, 2, 3))
    pos, st = W.roots(1006, 120)
    corr = lib.correction(True, 1.0)
    chunk = ctx.get_tuning(lib.TUNE_LAYER_CHUNK)
    try:
        ctx.set_tuning(lib.TUNE_LAYER_CHUNK, 1000)
        for prec in (lib.FP32, lib.BF16):
            ctx.set_precision(prec)
            out = []
            for knob in (2, 0, 1):
                ctx.set_tuning(lib.TUNE_CONV1_GROUPS, knob)
                out.append(ctx.search_batch(pos, st, d, A, GAMMA, corr))
            for k in (1, 2):
                assert np.array_equal(out[0][0], out[k][0]), (prec, k)
                assert np.array_equal(out[0][1], out[k][1]), (prec, k)
        # BF16 and FP8 with fusion off: their leaves on the layer path too
        ctx.set_tuning(lib.TUNE_FUSED, 0)
        for prec in (lib.BF16, lib.FP8):
            ctx.set_precision(prec)
            out = []
            for knob in (2, 0):
                ctx.set_tuning(lib.TUNE_CONV1_GROUPS, knob)
                out.append(ctx.search_batch(pos, st, d, A, GAMMA, corr))
            assert np.array_equal(out[0][0], out[1][0]), prec
            assert np.array_equal(out[0][1], out[1][1]), prec
        with pytest.raises(lib.BctsError) as e:
            ctx.set_tuning(lib.TUNE_CONV1_GROUPS, 3)
        assert e.value.status == lib.E_INVAL
    finally:
        ctx.set_tuning(lib.TUNE_FUSED, 1)
        ctx.set_tuning(lib.TUNE_CONV1_GROUPS, 1)
        ctx.set_tuning(lib.TUNE_LAYER_CHUNK, chunk)
        ctx.set_precision(lib.FP32)


@pytest.mark.parametrize("corr_on,c", [(True, 1.0), (False, 1.0), (True, 0.0), (True, 2.5)])
def test_c1_end_to_end(lib, setup, corr_on, c):
    """64 roots, A=4, d=2 (the small configuration), FP32."""
    ctx, world, _ = setup
    ctx.set_precision(lib.FP32)
    pos, st = W.roots(1001, 64)
    act, q = ctx.search(pos, st, 2, 4, GAMMA, lib.correction(corr_on, c))
    for r in range(64):
        ref = S.search(world, pos[r], st[r], 2, 4, GAMMA, correction=corr_on, c=c)
        assert_root_parity(q[r], act[r], ref, 4, f"root {r}")


@pytest.mark.parametrize("A,d", [(4, 0), (6, 0), (4, 1), (18, 1), (18, 2), (6, 3), (3, 4), (2, 2), (2, 5), (2, 6)])
def test_shapes_end_to_end(lib, setup, A, d):
    """FP32 end to end over the shape range: depth 0 (no search), the
    largest A (18) and the largest depth (6)."""
    ctx, world, _ = setup
    ctx.set_precision(lib.FP32)
    pos, st = W.roots(1002 + A + d, 4)
    act, q = ctx.search(pos, st, d, A, GAMMA, lib.correction(True, 1.0))
    for r in range(4):
        ref = S.search(world, pos[r], st[r], d, A, GAMMA, correction=True, c=1.0)
        assert_root_parity(q[r], act[r], ref, A, f"A={A} d={d} root {r}")


def test_exact_gev_mode(lib, setup):
    ctx, world, _ = setup
    ctx.set_precision(lib.FP32)
    pos, st = W.roots(31, 6)
    act, q = ctx.search(pos, st, 2, 6, GAMMA, lib.correction(True, 1.0, lib.CORR_EXACT_GEV))
    for r in range(6):
        ref = S.search(world, pos[r], st[r], 2, 6, GAMMA, correction=True, c=1.0, mode="gev")
        assert_root_parity(q[r], act[r], ref, 6, f"root {r}")


def test_mixed_batch_equals_single(lib, setup):
    """Roots of different (A, d) in one batch give the single-root results."""
    ctx, world, _ = setup
    ctx.set_precision(lib.FP32)
    n = 24
    pos, st = W.roots(1004, n)
    A, d = W.mixed_shapes(1004, n, (4, 6, 18), (0, 1, 2, 3))
    d = np.where(A == 18, np.minimum(d, 2), d)
    act, q = ctx.search_batch(pos, st, d, A, GAMMA, lib.correction(True, 1.0))
    for r in range(n):
        a1, q1 = ctx.search(pos[r:r + 1], st[r:r + 1], int(d[r]), int(A[r]), GAMMA, lib.correction(True, 1.0))
        assert act[r] == a1[0]
        np.testing.assert_array_equal(q[r, :A[r]], q1[0])
        assert np.all(np.isneginf(q[r, A[r]:]))
    for r in range(0, n, 5):
        ref = S.search(world, pos[r], st[r], int(d[r]), int(A[r]), GAMMA, correction=True, c=1.0)
        assert_root_parity(q[r], act[r], ref, int(A[r]), f"root {r}")


def test_device_and_graph_equal_host(lib, setup):
    import torch
    ctx, _, _ = setup
    ctx.set_precision(lib.BF16)
    n = 16
    pos, st = W.roots(1006, n)
    A, d = W.mixed_shapes(1006, n, (4, 6, 18), (1, 2, 3))
    corr = lib.correction(True, 1.0)
    act_h, q_h = ctx.search_batch(pos, st, d, A, GAMMA, corr)
    pt = torch.from_numpy(pos).cuda()
    stt = torch.from_numpy(st).cuda()
    at = torch.zeros(n, dtype=torch.int32, device="cuda")
    qt = torch.zeros(n, 18, dtype=torch.float32, device="cuda")
    ctx.search_batch_device(pt, stt, d, A, GAMMA, corr, at, qt)
    torch.cuda.synchronize()
    assert np.array_equal(at.cpu().numpy(), act_h)
    assert np.array_equal(qt.cpu().numpy(), q_h)
    for rep in range(3):
        qt.zero_()
        at.fill_(-1)
        torch.cuda.synchronize()
        ctx.search_batch_graph(pt, stt, d, A, GAMMA, corr, at, qt, replays=2)
        torch.cuda.synchronize()
        assert np.array_equal(at.cpu().numpy(), act_h), rep
        assert np.array_equal(qt.cpu().numpy(), q_h), rep
    ctx.set_precision(lib.FP32)


@pytest.mark.parametrize("prec,tol,tol_med", [("BF16", 2e-3, 1e-4), ("FP8", 2e-3, 1e-4)])
def test_lowp_qnet_matches_emulation(lib, setup, prec, tol, tol_med):
    """BF16 / FP8 matrix-core Q-network vs the oracle's emulation of the same
    operand roundings (same per-layer scales; BF16 products summed in FP64,
    FP8 products summed as the FP8 matrix instructions sum them).  An
    activation whose FP32 value sits at a rounding boundary may round the
    other way than in the emulation, so most stacks agree to FP32 rounding
    (the median bound) and a rare one differs by such a flip (the max: one
    BF16 step is 2^-8 of the activation; the FP8 stacks here have none)."""
    ctx, world, _ = setup
    _, st = W.roots(21, 24)
    dense = np.random.default_rng(8).integers(0, 256, size=(4, 4, 84, 84), dtype=np.uint8)
    x = np.concatenate([st, dense])
    if prec == "FP8":
        _, cal = W.roots(2003, 64)
        ctx.calibrate_fp8(cal)
    ctx.set_precision(getattr(lib, prec))
    got = ctx.debug_qnet(x, 18)
    ctx.set_precision(lib.FP32)
    want = Q.qvalues_lowp(x, world.w64, 18, prec.lower(), ascale=ctx.get_fp8_scales())
    rel = np.abs(got - want).max(axis=1) / np.abs(want).max(axis=1)
    print(f"{prec} vs emulation: max rel {rel.max():.3g}, median {np.median(rel):.3g}")
    assert rel.max() < tol, rel.max()
    assert np.median(rel) < tol_med, np.median(rel)


@pytest.mark.parametrize("prec,tol_mean,min_agree", [("BF16", 0.01, 31), ("FP8", 0.25, 24)])
def test_low_precision_vs_fp64(lib, setup, prec, tol_mean, min_agree):
    """Root-vector error and action agreement of BF16 / FP8 searches against
    the FP64 oracle on the small configuration (reported; loose bounds: the
    error is that of the operand precision itself -- the emulation test above
    checks the kernels against the same roundings).  Errors are relative to
    the root's largest |Q|, so roots whose values are all near 0 read large."""
    ctx, world, _ = setup
    pos, st = W.roots(1001, 32)
    if prec == "FP8":
        _, cal = W.roots(2003, 64)
        ctx.calibrate_fp8(cal)
    ctx.set_precision(getattr(lib, prec))
    act, q = ctx.search(pos, st, 2, 4, GAMMA, lib.correction(True, 1.0))
    ctx.set_precision(lib.FP32)
    errs, agree = [], 0
    for r in range(32):
        ref = S.search(world, pos[r], st[r], 2, 4, GAMMA, correction=True, c=1.0)
        errs.append(np.abs(q[r] - ref.q).max() / np.abs(ref.q).max())
        agree += act[r] == ref.action or act[r] in ref.ties
    print(f"{prec}: root-Q rel err max {max(errs):.3g} mean {np.mean(errs):.3g}; agreement {agree}/32")
    assert np.mean(errs) < tol_mean, np.mean(errs)
    assert agree >= min_agree, agree


def test_validation_errors(lib, setup):
    ctx, _, _ = setup
    pos, st = W.roots(1, 1)
    c = lib.correction(True, 1.0)
    for args in [(2, 19), (2, 0), (7, 4), (-1, 4)]:
        with pytest.raises(lib.BctsError) as e:
            ctx.search(pos, st, args[0], args[1], GAMMA, c)
        assert e.value.status == lib.E_INVAL
    with pytest.raises(lib.BctsError) as e:          # correction needs A >= 2
        ctx.search(pos, st, 2, 1, GAMMA, c)
    assert e.value.status == lib.E_INVAL
    ctx.search(pos, st, 2, 1, GAMMA, lib.correction(False))   # A = 1 without correction is fine
    with pytest.raises(lib.BctsError):
        ctx.search(pos, st, 2, 4, 1.5, c)
    bad = pos.copy()
    bad[0, 3, 1] = 84
    with pytest.raises(lib.BctsError) as e:
        ctx.search(bad, st, 2, 4, GAMMA, c)
    assert e.value.status == lib.E_INVAL
    # the context stays usable
    ctx.search(pos, st, 1, 4, GAMMA, c)


def test_state_errors(lib):
    ctx = lib.Context(0)
    pos, st = W.roots(1, 1)
    with pytest.raises(lib.BctsError) as e:
        ctx.search(pos, st, 1, 4, GAMMA, lib.correction(True, 1.0))
    assert e.value.status == lib.E_STATE
    ctx.close()


def test_fused_matches_layer_path(lib, setup):
    """The fused conv kernel (conv1's shared channels summed once per sibling
    group) against the layer-by-layer kernels at the same operand precision:
    only FP32 summation order and the occasional BF16 rounding flip differ."""
    ctx, world, _ = setup
    pos, st = W.roots(41, 12)
    A, d = 6, 2
    corr = lib.correction(True, 1.0)
    ctx.set_precision(lib.BF16)
    ctx.set_tuning(lib.TUNE_FUSED, 0)
    a0, q0 = ctx.search(pos, st, d, A, GAMMA, corr)
    ctx.set_tuning(lib.TUNE_FUSED, 1)
    a1, q1 = ctx.search(pos, st, d, A, GAMMA, corr)
    ctx.set_precision(lib.FP32)
    rel = np.abs(q1 - q0).max(axis=1) / np.abs(q0).max(axis=1)
    assert rel.max() < 5e-3, rel.max()
    assert (a0 == a1).mean() >= 11 / 12


@pytest.mark.parametrize("prec_name", ["BF16", "FP8"])
def test_fc2_folded_matches_fc2_on_h(lib, setup, prec_name):
    """fc2 in fc1's epilogue (the default) against fc1 writing h and fc2
    reading it back: the same operands (fc1's outputs rounded to the operand
    type), only fc2's FP32 sum associated differently, so the root vectors
    agree to FP32 rounding (1e-5 of each root's largest |Q|) and the actions
    agree except between values that close; a mixed batch with root rows of
    Q_0 (depth 0) and leaf chunks of several sizes."""
    ctx, _, _ = setup
    A, d = W.mixed_shapes(1007, 60, (4, 6, 18), (0, 1, 2, 3))
    pos, st = W.roots(1007, 60)
    corr = lib.correction(True, 1.0)
    chunk = ctx.get_tuning(lib.TUNE_FUSED_CHUNK)
    try:
        ctx.set_precision(getattr(lib, prec_name))
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 5000)
        out = []
        for folded in (1, 0):
            ctx.set_tuning(lib.TUNE_FC2_FOLDED, folded)
            out.append(ctx.search_batch(pos, st, d, A, GAMMA, corr))
        (a1, q1), (a0, q0) = out
        for r in range(len(A)):
            qa, qb = q1[r, :A[r]].astype(np.float64), q0[r, :A[r]].astype(np.float64)
            tol = 1e-5 * np.abs(qb).max() + 1e-7
            assert np.abs(qa - qb).max() <= tol, (r, np.abs(qa - qb).max())
            assert a1[r] == a0[r] or qb[a1[r]] >= qb.max() - 2 * tol, (r, a1[r], a0[r])
    finally:
        ctx.set_tuning(lib.TUNE_FC2_FOLDED, 1)
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, chunk)
        ctx.set_precision(lib.FP32)


@pytest.mark.parametrize("prec_name,rounds", [("BF16", (1, 2, 3)), ("FP8", (1, 2, 3, 4))])
def test_fused_rounds_and_chunks_are_bitwise_identical(lib, setup, prec_name, rounds):
    """Round size and chunking change only how stacks are grouped into
    launches and LDS rounds, never a stack's arithmetic."""
    ctx, _, _ = setup
    n = 20
    pos, st = W.roots(1004, n)
    A, d = W.mixed_shapes(1004, n, (4, 6, 18), (0, 1, 2, 3))
    d = np.where(A == 18, np.minimum(d, 2), d)
    corr = lib.correction(True, 1.0)
    if prec_name == "FP8":
        _, cal = W.roots(2003, 64)
        ctx.calibrate_fp8(cal)
    ctx.set_precision(getattr(lib, prec_name))
    ref = None
    for T in rounds:
        for chunk in (37, 262144):
            ctx.set_tuning(lib.TUNE_FUSED_ROUND, T)
            ctx.set_tuning(lib.TUNE_FUSED_CHUNK, chunk)
            act, q = ctx.search_batch(pos, st, d, A, GAMMA, corr)
            if ref is None:
                ref = (act, q)
            else:
                assert np.array_equal(act, ref[0]), (T, chunk)
                assert np.array_equal(q, ref[1]), (T, chunk)
    ctx.set_tuning(lib.TUNE_FUSED_ROUND, 3)
    ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 262144)
    ctx.set_precision(lib.FP32)


@pytest.mark.parametrize("prec_name,T", [("BF16", 3), ("FP8", 4)])
def test_persistent_loop_over_mixed_groups(lib, setup, prec_name, T):
    """The fused kernel's workgroups loop over sibling groups (prefetching
    the next group's frames) when a launch holds more groups than there are
    resident workgroups.  300 roots of mixed A and depth give groups of 1, 4,
    6 and 18 stacks in one launch; the results must equal, bit for bit, the
    launches of a few groups each (no workgroup loops), and sampled roots
    meet the operand-precision bound against the oracle."""
    ctx, world, _ = setup
    n = 300
    pos, st = W.roots(1006, n)
    A, d = W.mixed_shapes(1006, n, (4, 6, 18), (1, 2))
    corr = lib.correction(True, 1.0)
    if prec_name == "FP8":
        _, cal = W.roots(2003, 64)
        ctx.calibrate_fp8(cal)
    ctx.set_precision(getattr(lib, prec_name))
    ctx.set_tuning(lib.TUNE_FUSED, 1)
    ctx.set_tuning(lib.TUNE_FUSED_ROUND, T)
    try:
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 1048576)
        a1, q1 = ctx.search_batch(pos, st, d, A, GAMMA, corr)
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 37)
        a2, q2 = ctx.search_batch(pos, st, d, A, GAMMA, corr)
    finally:
        ctx.set_tuning(lib.TUNE_FUSED_ROUND, 3)
        ctx.set_tuning(lib.TUNE_FUSED_CHUNK, 262144)
        ctx.set_precision(lib.FP32)
    assert np.array_equal(a1, a2) and np.array_equal(q1, q2)
    if prec_name == "BF16":
        for r in (0, 151, 299):
            ref = S.search(world, pos[r], st[r], int(d[r]), int(A[r]), GAMMA, correction=True, c=1.0)
            rel = np.abs(q1[r, :A[r]].astype(np.float64) - np.asarray(ref.q)).max() / np.abs(ref.q).max()
            assert rel < 2e-2, (r, rel)

"""Python binding of libbcts (ctypes): argument marshalling only.

Every function named ``bcts_*`` here calls the C entry point of the same name
(declared in include/bcts.h); all search work runs in the HIP kernels of the
library.  Host arrays are numpy arrays; the ``*_device`` / ``*_graph`` calls
take torch tensors already on the GPU and a torch stream.  PyTorch is only
plumbing: it is imported first so that the process holds a single HIP
runtime, shared by torch's allocator/streams and the library.

Importing this module raises ImportError when libbcts.so has not been built:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_float, c_int32, c_size_t, c_uint64, c_void_p

import numpy as np

import torch  # noqa: F401  (one HIP runtime for torch and libbcts)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbcts.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2107_01715_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVAL, E_NOMEM, E_HIP, E_BUSY, E_STATE = 0, -1, -2, -3, -4, -5
FP32, BF16, FP8 = 0, 1, 2
CORR_EQ6, CORR_EXACT_GEV = 0, 1
MAX_A, MAX_DEPTH, QNET_NUMEL = 18, 6, 1693362
STATUS_NAMES = {OK: "OK", E_INVAL: "E_INVAL", E_NOMEM: "E_NOMEM", E_HIP: "E_HIP", E_BUSY: "E_BUSY",
                E_STATE: "E_STATE"}

# every symbol declared in include/bcts.h
EXPORTS = (
    "bcts_create", "bcts_destroy", "bcts_last_error", "bcts_reset", "bcts_set_env", "bcts_set_qnet",
    "bcts_set_precision", "bcts_calibrate_fp8", "bcts_get_fp8_scales", "bcts_set_fp8_scales",
    "bcts_search", "bcts_search_batch", "bcts_search_batch_device", "bcts_search_batch_graph",
    "bcts_submit", "bcts_progress", "bcts_poll", "bcts_serve_config", "bcts_request_bytes",
    "bcts_debug_expand", "bcts_debug_qnet", "bcts_set_timing", "bcts_get_timing",
    "bcts_set_tuning", "bcts_get_tuning", "bcts_autotune",
    "bcts_set_mlp", "bcts_mlp_search", "bcts_mlp_search_device", "bcts_set_beam",
    "bcts_debug_qnet_siblings", "bcts_search_batch_device_noalloc", "bcts_serve_stats",
    "bcts_debug_fail_launches", "bcts_debug_expand_batch", "bcts_graph_create", "bcts_graph_launch",
    "bcts_graph_destroy",
)
TUNE_FUSED, TUNE_FUSED_ROUND, TUNE_FUSED_CHUNK, TUNE_LAYER_CHUNK, TUNE_CORR_FP32, TUNE_MLP_CROSSOVER = 0, 1, 2, 3, 4, 5
TUNE_FP8_K128 = 6
TUNE_CONV1_GROUPS = 7
TUNE_MLP_HOST = 8
TUNE_FC2_FOLDED = 9


class EnvParamsC(ctypes.Structure):
    _fields_ = [("delta", (c_int32 * 2) * MAX_A), ("vel", (c_int32 * 2) * 7)]


class CorrectionC(ctypes.Structure):
    _fields_ = [("enabled", c_int32), ("scale", c_float), ("mode", c_int32)]


class BctsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_P = c_void_p
_create = _sig("bcts_create", c_int32, c_int32, c_size_t, POINTER(c_void_p))
_destroy = _sig("bcts_destroy", None, _P)
_last_error = _sig("bcts_last_error", c_char_p, _P)
_reset = _sig("bcts_reset", c_int32, _P)
_set_env = _sig("bcts_set_env", c_int32, _P, POINTER(EnvParamsC))
_set_qnet = _sig("bcts_set_qnet", c_int32, _P, _P, c_size_t)
_set_precision = _sig("bcts_set_precision", c_int32, _P, c_int32)
_calibrate_fp8 = _sig("bcts_calibrate_fp8", c_int32, _P, c_int32, _P)
_get_fp8_scales = _sig("bcts_get_fp8_scales", c_int32, _P, _P)
_set_fp8_scales = _sig("bcts_set_fp8_scales", c_int32, _P, _P)
_search = _sig("bcts_search", c_int32, _P, c_int32, _P, _P, c_int32, c_int32, c_float, CorrectionC, _P, _P)
_search_batch = _sig("bcts_search_batch", c_int32, _P, c_int32, _P, _P, _P, _P, c_float, CorrectionC, _P, _P)
_search_batch_device = _sig("bcts_search_batch_device", c_int32, _P, c_int32, _P, _P, _P, _P, c_float,
                            CorrectionC, _P, _P, _P)
_search_batch_device_noalloc = _sig("bcts_search_batch_device_noalloc", c_int32, _P, c_int32, _P, _P, _P, _P,
                                    c_float, CorrectionC, _P, _P, _P)
_search_batch_graph = _sig("bcts_search_batch_graph", c_int32, _P, c_int32, _P, _P, _P, _P, c_float,
                           CorrectionC, _P, _P, c_int32, _P)
_submit = _sig("bcts_submit", c_int32, _P, _P, _P, c_int32, c_int32, c_float, CorrectionC, POINTER(c_uint64))
_progress = _sig("bcts_progress", c_int32, _P, POINTER(c_int32))
_poll = _sig("bcts_poll", c_int32, _P, c_uint64, POINTER(c_int32), _P, POINTER(c_double))
_serve_config = _sig("bcts_serve_config", c_int32, _P, c_int32, c_int32)
_serve_stats = _sig("bcts_serve_stats", c_int32, _P, _P)
_graph_create = _sig("bcts_graph_create", c_int32, _P, c_int32, _P, _P, _P, _P, c_float, CorrectionC, _P, _P, _P,
                     POINTER(c_void_p))
_graph_launch = _sig("bcts_graph_launch", c_int32, _P, c_int32, _P)
_graph_destroy = _sig("bcts_graph_destroy", None, _P)
_debug_expand_batch = _sig("bcts_debug_expand_batch", c_int32, _P, c_int32, _P, _P, _P, _P, c_float, _P, _P, _P, _P,
                           _P, _P, _P, _P)
_debug_fail_launches = _sig("bcts_debug_fail_launches", c_int32, _P, c_int32)
_request_bytes = _sig("bcts_request_bytes", c_size_t, c_int32, c_int32)
_debug_expand = _sig("bcts_debug_expand", c_int32, _P, _P, _P, c_int32, c_int32, _P, _P, _P)
_debug_qnet = _sig("bcts_debug_qnet", c_int32, _P, c_int32, _P, c_int32, _P)
_debug_qnet_siblings = _sig("bcts_debug_qnet_siblings", c_int32, _P, c_int32, _P, c_int32, c_int32, _P)
_set_timing = _sig("bcts_set_timing", c_int32, _P, c_int32)
_get_timing = _sig("bcts_get_timing", c_int32, _P, _P)
_set_tuning = _sig("bcts_set_tuning", c_int32, _P, c_int32, ctypes.c_int64)
_get_tuning = _sig("bcts_get_tuning", c_int32, _P, c_int32, POINTER(ctypes.c_int64))
_autotune = _sig("bcts_autotune", c_int32, _P, c_int32, _P, _P, _P, _P, c_float, CorrectionC, _P, _P, c_int32, _P,
                 POINTER(ctypes.c_int64))

_set_mlp = _sig("bcts_set_mlp", c_int32, _P, c_int32, _P, c_size_t)
_set_beam = _sig("bcts_set_beam", c_int32, _P, c_int32)
_mlp_search = _sig("bcts_mlp_search", c_int32, _P, c_int32, _P, c_int32, c_float, CorrectionC, _P, _P)
_mlp_search_device = _sig("bcts_mlp_search_device", c_int32, _P, c_int32, _P, c_int32, c_float, CorrectionC, _P, _P,
                          _P)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(c_void_p)


def _arr(a, dtype, shape=None):
    a = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def correction(enabled: bool = True, scale: float = 1.0, mode: int = CORR_EQ6) -> CorrectionC:
    return CorrectionC(int(bool(enabled)), float(scale), int(mode))


def _check(ctx, st: int):
    if st != OK:
        raise BctsError(st, bcts_last_error(ctx))


# ---- one function per C entry point ----------------------------------------
def bcts_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = c_void_p()
    st = _create(device, hbm_budget_bytes, byref(h))
    if st != OK:
        raise BctsError(st, f"bcts_create(device={device}) failed")
    return h


def bcts_destroy(ctx):
    _destroy(ctx)


def bcts_last_error(ctx) -> str:
    return _last_error(ctx).decode()


def bcts_reset(ctx):
    _check(ctx, _reset(ctx))


def bcts_set_env(ctx, delta, vel):
    e = EnvParamsC()
    d = _arr(delta, np.int32, (MAX_A, 2))
    v = _arr(vel, np.int32, (7, 2))
    for a in range(MAX_A):
        e.delta[a][0], e.delta[a][1] = int(d[a, 0]), int(d[a, 1])
    for i in range(7):
        e.vel[i][0], e.vel[i][1] = int(v[i, 0]), int(v[i, 1])
    _check(ctx, _set_env(ctx, byref(e)))


def bcts_set_qnet(ctx, blob):
    b = _arr(blob, np.float32)
    _check(ctx, _set_qnet(ctx, _ptr(b), b.size))


def bcts_set_precision(ctx, prec: int):
    _check(ctx, _set_precision(ctx, prec))


def bcts_calibrate_fp8(ctx, stacks):
    s = _arr(stacks, np.uint8)
    _check(ctx, _calibrate_fp8(ctx, s.shape[0], _ptr(s)))


def bcts_get_fp8_scales(ctx) -> np.ndarray:
    out = np.zeros(5, np.float32)
    _check(ctx, _get_fp8_scales(ctx, _ptr(out)))
    return out


def bcts_set_fp8_scales(ctx, scales):
    s = _arr(scales, np.float32, (5,))
    _check(ctx, _set_fp8_scales(ctx, _ptr(s)))


def bcts_search(ctx, pos, stacks, depth: int, A: int, gamma: float, corr: CorrectionC):
    p = _arr(pos, np.int32)
    s = _arr(stacks, np.uint8)
    n = p.shape[0]
    act = np.zeros(n, np.int32)
    q = np.zeros((n, A), np.float32)
    _check(ctx, _search(ctx, n, _ptr(p), _ptr(s), depth, A, gamma, corr, _ptr(act), _ptr(q)))
    return act, q


def bcts_search_batch(ctx, pos, stacks, depth, A, gamma: float, corr: CorrectionC):
    p = _arr(pos, np.int32)
    s = _arr(stacks, np.uint8)
    d = _arr(depth, np.int32)
    a = _arr(A, np.int32)
    n = p.shape[0]
    act = np.zeros(n, np.int32)
    q = np.zeros((n, MAX_A), np.float32)
    _check(ctx, _search_batch(ctx, n, _ptr(p), _ptr(s), _ptr(d), _ptr(a), gamma, corr, _ptr(act), _ptr(q)))
    return act, q


def _dev(t, dtype, min_numel: int = 0):
    assert t.is_cuda and t.is_contiguous() and t.dtype == dtype, (t.device, t.dtype)
    if t.numel() < min_numel:
        raise ValueError(f"device buffer holds {t.numel()} elements, the call writes {min_numel}")
    return c_void_p(t.data_ptr())


def bcts_search_batch_device(ctx, pos_t, stacks_t, depth, A, gamma, corr, act_t, q_t, stream=None):
    n = pos_t.shape[0]
    d = _arr(depth, np.int32)
    a = _arr(A, np.int32)
    s = c_void_p(stream.cuda_stream) if stream is not None else c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(ctx, _search_batch_device(ctx, pos_t.shape[0], _dev(pos_t, torch.int32), _dev(stacks_t, torch.uint8),
                                     _ptr(d), _ptr(a), gamma, corr, _dev(act_t, torch.int32, n),
                                     _dev(q_t, torch.float32, n * MAX_A), s))


def bcts_search_batch_device_noalloc(ctx, pos_t, stacks_t, depth, A, gamma, corr, act_t, q_t, stream=None):
    n = pos_t.shape[0]
    d = _arr(depth, np.int32)
    a = _arr(A, np.int32)
    s = c_void_p(stream.cuda_stream) if stream is not None else c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(ctx, _search_batch_device_noalloc(ctx, n, _dev(pos_t, torch.int32), _dev(stacks_t, torch.uint8),
                                             _ptr(d), _ptr(a), gamma, corr, _dev(act_t, torch.int32, n),
                                             _dev(q_t, torch.float32, n * MAX_A), s))


def bcts_search_batch_graph(ctx, pos_t, stacks_t, depth, A, gamma, corr, act_t, q_t, replays=1, stream=None):
    n = pos_t.shape[0]
    d = _arr(depth, np.int32)
    a = _arr(A, np.int32)
    s = c_void_p(stream.cuda_stream) if stream is not None else c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(ctx, _search_batch_graph(ctx, pos_t.shape[0], _dev(pos_t, torch.int32), _dev(stacks_t, torch.uint8),
                                    _ptr(d), _ptr(a), gamma, corr, _dev(act_t, torch.int32, n),
                                    _dev(q_t, torch.float32, n * MAX_A), replays, s))


class Graph:
    """A captured search (bcts_graph_create); launch() replays it."""

    def __init__(self, ctx, pos_t, stacks_t, depth, A, gamma, corr, act_t, q_t, stream=None):
        n = pos_t.shape[0]
        d = _arr(depth, np.int32)
        a = _arr(A, np.int32)
        s = c_void_p(stream.cuda_stream) if stream is not None else c_void_p(torch.cuda.current_stream().cuda_stream)
        h = c_void_p()
        _check(ctx, _graph_create(ctx, n, _dev(pos_t, torch.int32), _dev(stacks_t, torch.uint8), _ptr(d), _ptr(a),
                                  gamma, corr, _dev(act_t, torch.int32, n), _dev(q_t, torch.float32, n * MAX_A), s,
                                  byref(h)))
        self.ctx, self.h = ctx, h
        self._keep = (pos_t, stacks_t, act_t, q_t)      # the buffers the graph reads and writes

    def launch(self, replays: int = 1, stream=None):
        s = c_void_p(stream.cuda_stream) if stream is not None else c_void_p(torch.cuda.current_stream().cuda_stream)
        _check(self.ctx, _graph_launch(self.h, replays, s))

    def close(self):
        if self.h:
            _graph_destroy(self.h)
            self.h = None


def bcts_graph_create(ctx, pos_t, stacks_t, depth, A, gamma, corr, act_t, q_t, stream=None) -> Graph:
    return Graph(ctx, pos_t, stacks_t, depth, A, gamma, corr, act_t, q_t, stream)


def bcts_submit(ctx, pos, stack, depth: int, A: int, gamma: float, corr: CorrectionC) -> int:
    p = _arr(pos, np.int32)
    s = _arr(stack, np.uint8)
    t = c_uint64()
    _check(ctx, _submit(ctx, _ptr(p), _ptr(s), depth, A, gamma, corr, byref(t)))
    return t.value


def bcts_progress(ctx) -> int:
    n = c_int32()
    _check(ctx, _progress(ctx, byref(n)))
    return n.value


def bcts_poll(ctx, ticket: int, A: int):
    """(action, q[A], t_done) when finished, None while busy."""
    act = c_int32()
    q = np.zeros(A, np.float32)
    t = c_double()
    st = _poll(ctx, ticket, byref(act), _ptr(q), byref(t))
    if st == E_BUSY:
        return None
    _check(ctx, st)
    return act.value, q, t.value


def bcts_serve_config(ctx, max_batch: int, max_inflight: int):
    _check(ctx, _serve_config(ctx, max_batch, max_inflight))


def bcts_serve_stats(ctx) -> dict:
    out = np.zeros(8, dtype=np.int64)
    _check(ctx, _serve_stats(ctx, _ptr(out)))
    keys = ("queued", "admitted", "cohorts", "staging", "steps_in_flight", "pool_in_use", "pool_capacity",
            "cohorts_done")
    return dict(zip(keys, (int(v) for v in out)))


def bcts_debug_fail_launches(ctx, count: int):
    _check(ctx, _debug_fail_launches(ctx, count))


def bcts_request_bytes(depth: int, A: int) -> int:
    return int(_request_bytes(depth, A))


def bcts_set_beam(ctx, beam: int):
    _check(ctx, _set_beam(ctx, beam))


def bcts_set_mlp(ctx, A: int, blob):
    b = _arr(blob, np.float32)
    _check(ctx, _set_mlp(ctx, A, _ptr(b), b.size))


def bcts_mlp_search(ctx, states, depth: int, A: int, gamma: float, corr: CorrectionC):
    """(actions int32 [n], q float32 [n][A]) for host states [n][100]; A is
    the model's action count (sizes the output)."""
    st = _arr(states, np.float32)
    n = st.shape[0]
    act = np.zeros(n, np.int32)
    q = np.zeros((n, A), np.float32)
    _check(ctx, _mlp_search(ctx, n, _ptr(st), depth, gamma, corr, _ptr(act), _ptr(q)))
    return act, q


def bcts_mlp_search_device(ctx, states_t, depth: int, gamma: float, corr: CorrectionC, act_t, q_t, stream=None):
    """q_t: float32 [n][A] with A the model's action count (its last dimension)."""
    s = c_void_p(stream.cuda_stream) if stream is not None else c_void_p(torch.cuda.current_stream().cuda_stream)
    n = states_t.shape[0]
    _check(ctx, _mlp_search_device(ctx, n, _dev(states_t, torch.float32, n * 100), depth, gamma, corr,
                                   _dev(act_t, torch.int32, n), _dev(q_t, torch.float32, n * q_t.shape[-1]), s))


def bcts_debug_expand(ctx, pos, stack, depth: int, A: int):
    """Per level k = 1..depth: (positions int32 [A^k][8][2], frames uint8
    [A^k][84][84], rewards int32 [A^k])."""
    p = _arr(pos, np.int32)
    s = _arr(stack, np.uint8)
    total = sum(A ** k for k in range(1, depth + 1))
    op = np.zeros((total, 8, 2), np.int32)
    of = np.zeros((total, 84, 84), np.uint8)
    orw = np.zeros(total, np.int32)
    _check(ctx, _debug_expand(ctx, _ptr(p), _ptr(s), depth, A, _ptr(op), _ptr(of), _ptr(orw)))
    out, at = [], 0
    for k in range(1, depth + 1):
        nk = A ** k
        out.append((op[at:at + nk], of[at:at + nk], orw[at:at + nk]))
        at += nk
    return out


def bcts_debug_expand_batch(ctx, pos, stacks, depth, A, gamma: float):
    """(levels, root_levels): levels[k] = (pos [N][8][2], frames [N][84][84],
    rewards [N], returns [N], keep [K]) for k = 1..max depth; root_levels
    [n][7][3] = (first node, node count, first keep entry or -1) per root
    and level."""
    n = len(depth)
    p = _arr(pos, np.int32, (n, 8, 2))
    s = _arr(stacks, np.uint8, (n, 4, 84, 84))
    d = _arr(depth, np.int32)
    a = _arr(A, np.int32)
    ln = np.zeros(7, np.int64)
    ke = np.zeros(7, np.int64)
    rl = np.zeros((n, 7, 3), np.int64)
    _check(ctx, _debug_expand_batch(ctx, n, _ptr(p), _ptr(s), _ptr(d), _ptr(a), gamma, _ptr(ln), _ptr(ke),
                                    _ptr(rl), None, None, None, None, None))
    tot, ktot = int(ln.sum()), int(ke.sum())
    op = np.zeros((tot, 8, 2), np.int32)
    of = np.zeros((tot, 84, 84), np.uint8)
    orw = np.zeros(tot, np.int32)
    ort = np.zeros(tot, np.float32)
    ok = np.zeros(max(ktot, 1), np.int32)
    _check(ctx, _debug_expand_batch(ctx, n, _ptr(p), _ptr(s), _ptr(d), _ptr(a), gamma, _ptr(ln), _ptr(ke),
                                    _ptr(rl), _ptr(op), _ptr(of), _ptr(orw), _ptr(ort), _ptr(ok)))
    levels, at, kat = {}, 0, 0
    for k in range(1, 7):
        nk, kk = int(ln[k]), int(ke[k])
        if nk == 0:
            continue
        levels[k] = (op[at:at + nk], of[at:at + nk], orw[at:at + nk], ort[at:at + nk], ok[kat:kat + kk])
        at += nk
        kat += kk
    return levels, rl


def bcts_debug_qnet(ctx, stacks, A: int) -> np.ndarray:
    s = _arr(stacks, np.uint8)
    q = np.zeros((s.shape[0], A), np.float32)
    _check(ctx, _debug_qnet(ctx, s.shape[0], _ptr(s), A, _ptr(q)))
    return q


def bcts_debug_qnet_siblings(ctx, stacks, A: int, group: int) -> np.ndarray:
    s = _arr(stacks, np.uint8)
    q = np.zeros((s.shape[0], A), np.float32)
    _check(ctx, _debug_qnet_siblings(ctx, s.shape[0], _ptr(s), A, group, _ptr(q)))
    return q


def bcts_set_timing(ctx, enabled: bool):
    _check(ctx, _set_timing(ctx, int(bool(enabled))))


def bcts_get_timing(ctx) -> np.ndarray:
    out = np.zeros(24, np.float64)
    _check(ctx, _get_timing(ctx, _ptr(out)))
    return out


def bcts_set_tuning(ctx, key: int, value: int):
    _check(ctx, _set_tuning(ctx, key, int(value)))


def bcts_get_tuning(ctx, key: int) -> int:
    v = ctypes.c_int64()
    _check(ctx, _get_tuning(ctx, key, byref(v)))
    return v.value


def bcts_autotune(ctx, pos_t, stacks_t, depth, A, gamma, corr, act_t, q_t, reps=2, stream=None):
    """Returns {fused, round, chunk, us_per_search, fp8_k128} and keeps it on ctx."""
    d = _arr(depth, np.int32)
    a = _arr(A, np.int32)
    s = c_void_p(stream.cuda_stream) if stream is not None else c_void_p(torch.cuda.current_stream().cuda_stream)
    out = (ctypes.c_int64 * 5)()
    n = pos_t.shape[0]
    _check(ctx, _autotune(ctx, n, _dev(pos_t, torch.int32), _dev(stacks_t, torch.uint8), _ptr(d),
                          _ptr(a), gamma, corr, _dev(act_t, torch.int32, n), _dev(q_t, torch.float32, n * MAX_A),
                          reps, s, out))
    return {"fused": int(out[0]), "round": int(out[1]), "chunk": int(out[2]), "us_per_search": int(out[3]),
            "fp8_k128": int(out[4])}


# ---- convenience object ----------------------------------------------------
class Context:
    """Owns one bcts_ctx; methods forward to the functions above."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.h = bcts_create(device, hbm_budget_bytes)

    def close(self):
        if self.h:
            bcts_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __getattr__(self, name):
        fn = globals().get("bcts_" + name)
        if fn is None:
            raise AttributeError(name)
        return lambda *a, **k: fn(self.h, *a, **k)

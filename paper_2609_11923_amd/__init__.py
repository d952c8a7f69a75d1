"""Python binding of the MI355X compiled-CFR library (``include/cfr.h``).

Argument marshalling only: every step of an iteration runs in the HIP kernels
of ``libcfr.so``.  The library must have been built (``python -m
paper_2609_11923_amd.build`` or ``__graft_entry__.build()``); importing the
functions raises if it is missing.  There is no CPU fallback.

The C entry points are exposed under their own names (``cfr_compile``,
``cfr_iterate`` ...).  ``Solver`` wraps a handle with numpy/torch-friendly
helpers; torch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcfr.so")

CFR_OK, CFR_EINVAL, CFR_ENOMEM, CFR_EDEVICE, CFR_EGRAPH, CFR_ESTATE, CFR_EUNSUPPORTED = range(7)
CFR_RULE_CFR_PLUS, CFR_RULE_CFR, CFR_RULE_DCFR, CFR_RULE_PCFR_PLUS = 0, 1, 2, 3
CFR_AVG_LINEAR, CFR_AVG_UNIFORM = 0, 1
CFR_ORDER_SIMULTANEOUS, CFR_ORDER_ALTERNATING = 0, 1
CFR_LAYOUT_BFS, CFR_LAYOUT_PUBLIC = 0, 1
CFR_STRATEGY_CURRENT, CFR_STRATEGY_AVERAGE = 0, 1
CFR_PRECISION_FP32, CFR_PRECISION_FP64 = 0, 1
CFR_SCHEDULE_LEVEL, CFR_SCHEDULE_PERSISTENT, CFR_SCHEDULE_LDS = 0, 1, 2
CFR_FEATURES, CFR_MLP_OUT = 128, 4
CFR_MLP_PARAMS, CFR_MLP_GRADS, CFR_MLP_ADAM_M, CFR_MLP_ADAM_V = 0, 1, 2, 3

_STATUS = {0: "CFR_OK", 1: "CFR_EINVAL", 2: "CFR_ENOMEM", 3: "CFR_EDEVICE", 4: "CFR_EGRAPH", 5: "CFR_ESTATE",
           6: "CFR_EUNSUPPORTED"}

_P = ctypes.c_void_p


class cfr_game_desc(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_int64), ("root", ctypes.c_int64), ("node_type", _P), ("child_begin", _P),
                ("num_children", _P), ("children", _P), ("chance_prob", _P), ("infoset_key", _P), ("payoff", _P),
                ("public_key", _P), ("pot", ctypes.c_double), ("root_hand1", _P), ("root_hand2", _P),
                ("num_hands1", ctypes.c_int32), ("num_hands2", ctypes.c_int32)]


class cfr_options(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int), ("averaging", ctypes.c_int), ("order", ctypes.c_int),
                ("iters_per_graph", ctypes.c_int), ("layout", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("device", ctypes.c_int), ("test_fail_capture", ctypes.c_int), ("precision", ctypes.c_int),
                ("persistent", ctypes.c_int), ("wg_nodes", ctypes.c_int), ("lifecycle", ctypes.c_int),
                ("affine", ctypes.c_int), ("keep_layout", ctypes.c_int), ("group_sets", ctypes.c_int)]


class cfr_tune_result(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("wg_nodes", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("ms_per_iteration", ctypes.c_double), ("failed", ctypes.c_int32)]


class cfr_counts_t(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int64), ("edges", ctypes.c_int64), ("terminals", ctypes.c_int64),
                ("decision_nodes", ctypes.c_int64), ("infosets", ctypes.c_int64), ("slots", ctypes.c_int64),
                ("max_depth", ctypes.c_int32), ("blocks", ctypes.c_int32), ("max_actions", ctypes.c_int32),
                ("br_supported", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("kernels_per_iteration", ctypes.c_int64), ("pot", ctypes.c_double),
                ("child_addressing", ctypes.c_int32), ("node_order_groups", ctypes.c_int32),
                ("node_order_members", ctypes.c_int64), ("group_sets", ctypes.c_int32),
                ("update_groups", ctypes.c_int32)]


class cfr_layout(ctypes.Structure):
    _fields_ = [("counts", cfr_counts_t)] + [(n, _P) for n in (
        "depth_off", "parent", "child_off", "in_slot", "node_infoset", "node_type", "tmpl", "slot_off", "mem_off",
        "mem_node", "iset_player", "iset_key")]


class cfr_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches_per_iteration", ctypes.c_int64),
                ("bytes_per_iteration", ctypes.c_double), ("method_bytes_per_iteration", ctypes.c_double),
                ("ms_per_iteration", ctypes.c_double)]


class cfr_mlp_desc(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int32), ("hidden", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("max_rows", ctypes.c_int32), ("device", ctypes.c_int32), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class CfrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

# exported symbols of include/cfr.h (the ABI tests check the library exports each one)
EXPORTS = ["cfr_default_options", "cfr_layout_host", "cfr_layout_free", "cfr_compile", "cfr_compile_batch",
           "cfr_batch_size", "cfr_batch_exploitability", "cfr_autotune", "cfr_set_schedule", "cfr_set_active",
           "cfr_iterate",
           "cfr_iterations", "cfr_strategy", "cfr_exploitability", "cfr_reset", "cfr_get_state", "cfr_set_regrets",
           "cfr_counts", "cfr_profile", "cfr_debug_rebind", "cfr_destroy", "cfr_last_error",
           "cfr_mlp_default_desc", "cfr_mlp_create", "cfr_mlp_num_params", "cfr_mlp_set_params", "cfr_mlp_get",
           "cfr_mlp_forward", "cfr_mlp_backward", "cfr_mlp_adam", "cfr_mlp_train_step", "cfr_mlp_destroy",
           "cfr_num_infosets", "cfr_features", "cfr_regret_unit", "cfr_warm_start", "cfr_set_payoffs",
           "cfr_set_root_chance", "cfr_set_root_ranges", "cfr_set_state", "cfr_get_prediction", "cfr_get_layout",
           "cfr_persistent_plan_host", "cfr_mlp_forward_noalloc", "cfr_get_game_state"]


def load():
    """Load libcfr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_11923_amd.build` "
                          f"(there is no CPU fallback)")
    # torch ships its own HIP runtime under the same soname; load it first (when installed) so that
    # one runtime serves the process and torch streams/memory stay usable next to this library
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    S = ctypes.c_int
    sig = {
        "cfr_default_options": (None, [ctypes.POINTER(cfr_options)]),
        "cfr_layout_host": (S, [ctypes.POINTER(cfr_game_desc), ctypes.POINTER(cfr_layout)]),
        "cfr_layout_free": (None, [ctypes.POINTER(cfr_layout)]),
        "cfr_compile": (S, [ctypes.POINTER(cfr_game_desc), ctypes.POINTER(cfr_options), ctypes.POINTER(_P)]),
        "cfr_compile_batch": (S, [ctypes.POINTER(cfr_game_desc), ctypes.c_int32, ctypes.POINTER(cfr_options),
                                  ctypes.POINTER(_P)]),
        "cfr_batch_size": (S, [_P, ctypes.POINTER(ctypes.c_int32), _P]),
        "cfr_set_active": (S, [_P, _P, ctypes.c_int32, _P]),
        "cfr_batch_exploitability": (S, [_P, _P, _P, _P, _P, _P, ctypes.c_int32]),
        "cfr_autotune": (S, [_P, ctypes.c_int64, _P, ctypes.c_char_p, ctypes.POINTER(cfr_tune_result)]),
        "cfr_set_schedule": (S, [_P, ctypes.c_int32, ctypes.c_int32]),
        "cfr_iterate": (S, [_P, ctypes.c_int64, _P]),
        "cfr_iterations": (S, [_P, ctypes.POINTER(ctypes.c_int64)]),
        "cfr_strategy": (S, [_P, ctypes.c_int, _P, ctypes.c_int64, ctypes.c_int, _P]),
        "cfr_exploitability": (S, [_P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "cfr_reset": (S, [_P]),
        "cfr_get_state": (S, [_P, _P, _P, ctypes.c_int64, _P]),
        "cfr_set_regrets": (S, [_P, _P, ctypes.c_int64, ctypes.c_int, _P]),
        "cfr_counts": (S, [_P, ctypes.POINTER(cfr_counts_t)]),
        "cfr_profile": (S, [_P, ctypes.c_int64, _P, ctypes.POINTER(cfr_kernel_stat), ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int32)]),
        "cfr_debug_rebind": (S, [_P, ctypes.c_int, ctypes.c_int64]),
        "cfr_destroy": (None, [_P]),
        "cfr_last_error": (ctypes.c_char_p, []),
        "cfr_mlp_default_desc": (None, [ctypes.POINTER(cfr_mlp_desc)]),
        "cfr_mlp_create": (S, [ctypes.POINTER(cfr_mlp_desc), ctypes.POINTER(_P)]),
        "cfr_mlp_num_params": (S, [_P, ctypes.POINTER(ctypes.c_int64)]),
        "cfr_mlp_set_params": (S, [_P, _P, ctypes.c_int64]),
        "cfr_mlp_get": (S, [_P, ctypes.c_int, _P, ctypes.c_int64]),
        "cfr_mlp_forward": (S, [_P, _P, ctypes.c_int64, _P, _P]),
        "cfr_mlp_forward_noalloc": (S, [_P, _P, ctypes.c_int64, _P, _P]),
        "cfr_mlp_backward": (S, [_P, _P, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.POINTER(ctypes.c_double), _P]),
        "cfr_mlp_adam": (S, [_P, ctypes.c_float, _P]),
        "cfr_mlp_train_step": (S, [_P, _P, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_float,
                                   ctypes.POINTER(ctypes.c_double), _P]),
        "cfr_mlp_destroy": (None, [_P]),
        "cfr_num_infosets": (S, [_P, ctypes.POINTER(ctypes.c_int64)]),
        "cfr_features": (S, [_P, _P, _P, _P, ctypes.c_int32, _P, ctypes.c_int64, _P]),
        "cfr_regret_unit": (S, [_P, _P, ctypes.c_int64, _P]),
        "cfr_set_payoffs": (S, [_P, ctypes.c_int32, _P, ctypes.c_int64, _P]),
        "cfr_set_root_chance": (S, [_P, ctypes.c_int32, _P, ctypes.c_int64, _P]),
        "cfr_set_root_ranges": (S, [_P, ctypes.c_int32, _P, ctypes.c_int64, _P, ctypes.c_int64, _P]),
        "cfr_set_state": (S, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int64, _P]),
        "cfr_get_prediction": (S, [_P, _P, ctypes.c_int64, _P]),
        "cfr_get_game_state": (S, [_P, ctypes.c_int32, _P, _P, _P, ctypes.c_int64, _P]),
        "cfr_get_layout": (S, [_P, ctypes.c_int32, ctypes.POINTER(cfr_layout)]),
        "cfr_persistent_plan_host": (S, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P,
                                         ctypes.POINTER(ctypes.c_int32)]),
        "cfr_warm_start": (S, [_P, _P, _P, ctypes.c_int64, ctypes.c_float, ctypes.c_int32, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != CFR_OK:
        raise CfrError(status, load().cfr_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


class GameDesc:
    """cfr_game_desc built from any object with the gamegen.Game array attributes; keeps the arrays alive."""

    def __init__(self, game, with_public_key: bool = True):
        self.arrays = dict(
            node_type=np.ascontiguousarray(game.type, np.int8),
            child_begin=np.ascontiguousarray(game.child_begin, np.int64),
            num_children=np.ascontiguousarray(game.n_children, np.int32),
            children=np.ascontiguousarray(game.children, np.int64),
            chance_prob=np.ascontiguousarray(game.prob, np.float64),
            infoset_key=np.ascontiguousarray(game.key, np.int64),
            payoff=np.ascontiguousarray(game.payoff, np.float64),
        )
        pk = getattr(game, "pub", None)
        if with_public_key and pk is not None:
            self.arrays["public_key"] = np.ascontiguousarray(pk, np.int64)
        d = cfr_game_desc()
        d.num_nodes = len(self.arrays["node_type"])
        d.root = int(getattr(game, "root", 0))
        # a joint deal of the two private hands at the root (subgames): the hands of each root child
        meta = getattr(game, "meta", None) or {}
        if "pair_h1" in meta and "hands1" in meta and "hands2" in meta:
            h1 = np.ascontiguousarray(meta["pair_h1"], np.int32)
            if len(h1) == int(self.arrays["num_children"][d.root]):
                self.arrays["root_hand1"] = h1
                self.arrays["root_hand2"] = np.ascontiguousarray(meta["pair_h2"], np.int32)
                d.num_hands1, d.num_hands2 = len(meta["hands1"]), len(meta["hands2"])
        for k, v in self.arrays.items():
            setattr(d, k, _ptr(v))
        d.pot = float(getattr(game, "pot", 1.0))
        self.desc = d


def cfr_default_options() -> cfr_options:
    o = cfr_options()
    load().cfr_default_options(ctypes.byref(o))
    return o


def cfr_layout_host(game) -> dict:
    """Host-only compile; returns the canonical arrays as numpy copies."""
    gd = game if isinstance(game, GameDesc) else GameDesc(game)
    lay = cfr_layout()
    _check(load().cfr_layout_host(ctypes.byref(gd.desc), ctypes.byref(lay)))
    return _layout_dict(lay)


def cfr_get_layout(h, game: int = 0) -> dict:
    """Canonical arrays of one game of a handle compiled with keep_layout."""
    lay = cfr_layout()
    _check(load().cfr_get_layout(h, int(game), ctypes.byref(lay)))
    return _layout_dict(lay)


def _layout_dict(lay) -> dict:
    try:
        c = lay.counts
        N, I, A, Nd = c.nodes, c.infosets, c.slots, c.decision_nodes

        def arr(ptr, n, dt):
            if n == 0:
                return np.zeros(0, dt)
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(np.ctypeslib.as_ctypes_type(dt))),
                                         shape=(n,)).copy()

        out = dict(
            depth_off=arr(lay.depth_off, c.max_depth + 2, np.int32), parent=arr(lay.parent, N, np.int32),
            child_off=arr(lay.child_off, N + 1, np.int32), in_slot=arr(lay.in_slot, N, np.int32),
            node_infoset=arr(lay.node_infoset, N, np.int32), node_type=arr(lay.node_type, N, np.int8),
            tmpl=arr(lay.tmpl, N, np.float32), slot_off=arr(lay.slot_off, I + 1, np.int32),
            mem_off=arr(lay.mem_off, I + 1, np.int32), mem_node=arr(lay.mem_node, Nd, np.int32),
            iset_player=arr(lay.iset_player, I, np.int8), iset_key=arr(lay.iset_key, I, np.int64),
        )
        out["counts"] = {f: getattr(c, f) for f, _ in cfr_counts_t._fields_}
        return out
    finally:
        load().cfr_layout_free(ctypes.byref(lay))


def cfr_compile(game, options: cfr_options | None = None):
    gd = game if isinstance(game, GameDesc) else GameDesc(game)
    h = _P()
    _check(load().cfr_compile(ctypes.byref(gd.desc), ctypes.byref(options) if options is not None else None,
                              ctypes.byref(h)))
    return h


def cfr_compile_batch(games, options: cfr_options | None = None):
    gds = [g if isinstance(g, GameDesc) else GameDesc(g) for g in games]
    arr = (cfr_game_desc * len(gds))(*[gd.desc for gd in gds])
    h = _P()
    _check(load().cfr_compile_batch(arr, len(gds), ctypes.byref(options) if options is not None else None,
                                    ctypes.byref(h)))
    return h


def cfr_batch_size(h):
    n = ctypes.c_int32()
    _check(load().cfr_batch_size(h, ctypes.byref(n), None))
    base = np.zeros(n.value + 1, np.int64)
    _check(load().cfr_batch_size(h, ctypes.byref(n), _ptr(base)))
    return n.value, base


def cfr_batch_exploitability(h, n: int, stream=None):
    out = [np.zeros(n) for _ in range(4)]
    _check(load().cfr_batch_exploitability(h, stream, *[_ptr(a) for a in out], n))
    return tuple(out)


def cfr_autotune(h, iters: int, stream=None, cache_path: str | None = None) -> dict:
    r = cfr_tune_result()
    _check(load().cfr_autotune(h, int(iters), stream, cache_path.encode() if cache_path else None, ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in cfr_tune_result._fields_}


def cfr_persistent_plan_host(nodes, wg_nodes: int, max_w: int) -> dict:
    """The persistent schedule's work plan for games of the given node counts (host only)."""
    nv = np.ascontiguousarray(nodes, np.int64)
    n = len(nv)
    W = np.zeros(max(n, 1), np.int32)
    q = np.zeros(max(n, 1), np.int32)
    q_off = np.zeros(9, np.int32)
    used = ctypes.c_int32()
    _check(load().cfr_persistent_plan_host(_ptr(nv), n, int(wg_nodes), int(max_w), _ptr(W), _ptr(q), _ptr(q_off),
                                           ctypes.byref(used)))
    return dict(W=W[:n], queue=q[:n], q_off=q_off, wg_nodes=used.value)


def cfr_set_schedule(h, persistent: int, wg_nodes: int = 0):
    _check(load().cfr_set_schedule(h, int(persistent), int(wg_nodes)))


def cfr_set_active(h, active, stream=None):
    """Retire (0) or bring back (1) the games of a batch; active has one entry per game."""
    a = np.ascontiguousarray(np.asarray(active, dtype=np.uint8))
    _check(load().cfr_set_active(h, a.ctypes.data_as(_P), int(a.size), stream))


def cfr_iterate(h, n: int, stream=None):
    _check(load().cfr_iterate(h, int(n), stream))


def cfr_iterations(h) -> int:
    t = ctypes.c_int64()
    _check(load().cfr_iterations(h, ctypes.byref(t)))
    return t.value


def cfr_strategy(h, which: int, dst_ptr, length: int, dst_on_device: bool, stream=None):
    _check(load().cfr_strategy(h, int(which), dst_ptr, int(length), int(dst_on_device), stream))


def cfr_exploitability(h, stream=None):
    e, b1, b2, v = (ctypes.c_double() for _ in range(4))
    _check(load().cfr_exploitability(h, stream, ctypes.byref(e), ctypes.byref(b1), ctypes.byref(b2),
                                     ctypes.byref(v)))
    return e.value, b1.value, b2.value, v.value


def cfr_reset(h):
    _check(load().cfr_reset(h))


def cfr_get_state(h, length: int, stream=None):
    R = np.zeros(max(length, 1), np.float64)
    S = np.zeros(max(length, 1), np.float64)
    _check(load().cfr_get_state(h, _ptr(R), _ptr(S), int(length), stream))
    return R[:length], S[:length]


def cfr_set_regrets(h, src_ptr, length: int, src_on_device: bool, stream=None):
    _check(load().cfr_set_regrets(h, src_ptr, int(length), int(src_on_device), stream))


def cfr_set_state(h, length: int, t: int, regrets=None, strategy_sum=None, prediction=None, stream=None):
    arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (regrets, strategy_sum, prediction)]
    _check(load().cfr_set_state(h, *[_ptr(a) for a in arrs], int(length), int(t), stream))


def cfr_get_prediction(h, length: int, stream=None):
    p = np.zeros(max(length, 1), np.float64)
    _check(load().cfr_get_prediction(h, _ptr(p), int(length), stream))
    return p[:length]


def cfr_get_game_state(h, game: int, length: int, prediction: bool = False, stream=None):
    """(regrets, strategy sums[, prediction]) of one game of a batch, FP64, that game's canonical order."""
    r, s = np.zeros(max(length, 1), np.float64), np.zeros(max(length, 1), np.float64)
    p = np.zeros(max(length, 1), np.float64) if prediction else None
    _check(load().cfr_get_game_state(h, int(game), _ptr(r), _ptr(s), _ptr(p) if p is not None else None,
                                     int(length), stream))
    return (r[:length], s[:length]) + ((p[:length],) if p is not None else ())


def cfr_counts(h) -> dict:
    c = cfr_counts_t()
    _check(load().cfr_counts(h, ctypes.byref(c)))
    return {f: getattr(c, f) for f, _ in cfr_counts_t._fields_}


def cfr_profile(h, n: int, stream=None) -> list[dict]:
    arr = (cfr_kernel_stat * 16)()
    k = ctypes.c_int32()
    _check(load().cfr_profile(h, int(n), stream, arr, 16, ctypes.byref(k)))
    return [dict(name=arr[i].name.decode(), launches_per_iteration=arr[i].launches_per_iteration,
                 bytes_per_iteration=arr[i].bytes_per_iteration,
                 method_bytes_per_iteration=arr[i].method_bytes_per_iteration, ms_per_iteration=arr[i].ms_per_iteration)
            for i in range(k.value)]


def cfr_debug_rebind(h, which: int, delta: int):
    _check(load().cfr_debug_rebind(h, int(which), int(delta)))


def cfr_destroy(h):
    if h:
        load().cfr_destroy(h)


def _dptr(t):
    """Device pointer of a torch tensor (or an int address); None stays NULL."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


def _stream_arg(stream):
    if stream is None:
        return None
    if isinstance(stream, ctypes.c_void_p):
        return stream
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def cfr_mlp_default_desc() -> cfr_mlp_desc:
    d = cfr_mlp_desc()
    load().cfr_mlp_default_desc(ctypes.byref(d))
    return d


def cfr_num_infosets(h) -> int:
    n = ctypes.c_int64()
    _check(load().cfr_num_infosets(h, ctypes.byref(n)))
    return n.value


def cfr_features(h, bucket, history, scalars, x, rows: int, probe_iters: int = 0, stream=None):
    _check(load().cfr_features(h, _dptr(bucket), _dptr(history), _dptr(scalars), int(probe_iters), _dptr(x),
                               int(rows), _stream_arg(stream)))


def cfr_regret_unit(h, unit, rows: int, stream=None):
    _check(load().cfr_regret_unit(h, _dptr(unit), int(rows), _stream_arg(stream)))


def cfr_warm_start(h, mlp, x, rows: int, scale: float, add: bool = False, stream=None):
    _check(load().cfr_warm_start(h, mlp, _dptr(x), int(rows), float(scale), int(add), _stream_arg(stream)))


class Mlp:
    """The warm-start network (cfr_mlp).  Device arrays are torch tensors (or raw addresses)."""

    def __init__(self, in_dim=CFR_FEATURES, hidden=256, n_hidden=3, max_rows=4096, device=0, beta1=0.9,
                 beta2=0.999, eps=1e-8):
        d = cfr_mlp_default_desc()
        d.in_dim, d.hidden, d.n_hidden, d.max_rows, d.device = in_dim, hidden, n_hidden, max_rows, device
        d.beta1, d.beta2, d.eps = beta1, beta2, eps
        self.desc = d
        self.h = _P()
        _check(load().cfr_mlp_create(ctypes.byref(d), ctypes.byref(self.h)))
        n = ctypes.c_int64()
        _check(load().cfr_mlp_num_params(self.h, ctypes.byref(n)))
        self.P = n.value

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, np.float32)
        _check(load().cfr_mlp_set_params(self.h, _ptr(a), a.size))

    def get(self, which=CFR_MLP_PARAMS) -> np.ndarray:
        out = np.zeros(self.P, np.float32)
        _check(load().cfr_mlp_get(self.h, int(which), _ptr(out), self.P))
        return out

    def forward(self, x, rows: int, z, stream=None):
        _check(load().cfr_mlp_forward(self.h, _dptr(x), int(rows), _dptr(z), _stream_arg(stream)))

    def forward_noalloc(self, x, rows: int, z, stream=None):
        """cfr_mlp_forward without device allocation (activations in the library's static scratch; rows <= 8192)."""
        _check(load().cfr_mlp_forward_noalloc(self.h, _dptr(x), int(rows), _dptr(z), _stream_arg(stream)))

    def backward(self, x, target, weight, nact, rows: int, idx=None, n_data: int = 0, want_loss=True, stream=None):
        loss = ctypes.c_double()
        _check(load().cfr_mlp_backward(self.h, _dptr(x), _dptr(target), _dptr(weight), _dptr(nact), _dptr(idx),
                                       int(n_data), int(rows), ctypes.byref(loss) if want_loss else None,
                                       _stream_arg(stream)))
        return loss.value if want_loss else None

    def adam(self, lr: float, stream=None):
        _check(load().cfr_mlp_adam(self.h, float(lr), _stream_arg(stream)))

    def train_step(self, x, target, weight, nact, rows: int, lr: float, idx=None, n_data: int = 0, want_loss=False,
                   stream=None):
        loss = ctypes.c_double()
        _check(load().cfr_mlp_train_step(self.h, _dptr(x), _dptr(target), _dptr(weight), _dptr(nact), _dptr(idx),
                                         int(n_data), int(rows), float(lr),
                                         ctypes.byref(loss) if want_loss else None, _stream_arg(stream)))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "h", None):
            load().cfr_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Owns one compiled game.  ``stream`` may be a torch.cuda.Stream, a raw hipStream_t int, or None."""

    def __init__(self, game, rule=CFR_RULE_CFR_PLUS, averaging=CFR_AVG_LINEAR, order=CFR_ORDER_SIMULTANEOUS,
                 iters_per_graph=1, layout=CFR_LAYOUT_PUBLIC, use_graph=True, device=0, test_fail_capture=False,
                 precision=CFR_PRECISION_FP32, persistent=False, wg_nodes=0, lifecycle=False, affine=True,
                 keep_layout=False, group_sets=0):
        o = cfr_default_options()
        o.rule, o.averaging, o.order = rule, averaging, order
        o.iters_per_graph, o.layout, o.use_graph = iters_per_graph, layout, int(use_graph)
        o.device, o.test_fail_capture = device, int(test_fail_capture)
        o.precision = precision
        o.persistent, o.wg_nodes = int(persistent), int(wg_nodes)
        o.lifecycle = int(lifecycle)
        o.affine = int(affine)
        o.keep_layout = int(keep_layout)
        o.group_sets = int(group_sets)
        self.options = o
        if isinstance(game, (list, tuple)):
            self.h = cfr_compile_batch(game, o)
        else:
            self.h = cfr_compile(game, o)
        self.counts = cfr_counts(self.h)
        self.A = int(self.counts["slots"])
        self.n_games, self.slot_base = cfr_batch_size(self.h)

    @staticmethod
    def _stream(stream):
        if stream is None:
            return None
        if hasattr(stream, "cuda_stream"):
            return ctypes.c_void_p(stream.cuda_stream)
        return ctypes.c_void_p(int(stream))

    def iterate(self, n: int, stream=None):
        cfr_iterate(self.h, n, self._stream(stream))

    @property
    def iterations(self) -> int:
        return cfr_iterations(self.h)

    def strategy(self, average: bool = False, stream=None) -> np.ndarray:
        out = np.zeros(max(self.A, 1), np.float32)
        cfr_strategy(self.h, CFR_STRATEGY_AVERAGE if average else CFR_STRATEGY_CURRENT, _ptr(out), self.A, False,
                     self._stream(stream))
        return out[: self.A]

    def strategy_into(self, tensor, average: bool = False, stream=None):
        """Write into a device tensor (float32, slot count elements)."""
        cfr_strategy(self.h, CFR_STRATEGY_AVERAGE if average else CFR_STRATEGY_CURRENT,
                     ctypes.c_void_p(tensor.data_ptr()), self.A, True, self._stream(stream))

    def state(self, stream=None):
        return cfr_get_state(self.h, self.A, self._stream(stream))

    def set_state(self, regrets=None, strategy_sum=None, t: int = 0, prediction=None, stream=None):
        """Resume from host arrays (canonical order); the next iteration is t + 1."""
        sizes = {len(a) for a in (regrets, strategy_sum, prediction) if a is not None}
        if len(sizes) > 1:
            raise ValueError("regrets, strategy sums and prediction must have the same length")
        cfr_set_state(self.h, sizes.pop() if sizes else self.A, t, regrets, strategy_sum, prediction,
                      self._stream(stream))

    def prediction(self, stream=None) -> np.ndarray:
        return cfr_get_prediction(self.h, self.A, self._stream(stream))

    def game_state(self, game: int, prediction: bool = False, stream=None):
        """(regrets, strategy sums[, prediction]) of game `game` of the batch, in its canonical order."""
        n = int(self.slot_base[game + 1] - self.slot_base[game]) if 0 <= game < self.n_games else 0
        return cfr_get_game_state(self.h, game, n, prediction, self._stream(stream))

    def layout(self, game: int = 0) -> dict:
        return cfr_get_layout(self.h, game)

    def set_root_ranges(self, r1, r2, game: int = 0, stream=None):
        """New root ranges of game `game` (a subgame's joint deal): the library recomputes its root chance."""
        a = np.ascontiguousarray(r1, np.float64)
        b = np.ascontiguousarray(r2, np.float64)
        _check(load().cfr_set_root_ranges(self.h, int(game), _ptr(a), a.size, _ptr(b), b.size, self._stream(stream)))

    def set_regrets(self, r0, stream=None):
        if hasattr(r0, "data_ptr"):
            cfr_set_regrets(self.h, ctypes.c_void_p(r0.data_ptr()), self.A, True, self._stream(stream))
        else:
            a = np.ascontiguousarray(r0, np.float32)
            cfr_set_regrets(self.h, _ptr(a), self.A, False, self._stream(stream))

    def profile(self, n: int, stream=None) -> list[dict]:
        return cfr_profile(self.h, n, self._stream(stream))

    def exploitability(self, stream=None):
        return cfr_exploitability(self.h, self._stream(stream))

    def autotune(self, iters: int, stream=None, cache_path=None) -> dict:
        return cfr_autotune(self.h, iters, self._stream(stream), cache_path)

    def set_schedule(self, persistent: int, wg_nodes: int = 0):
        cfr_set_schedule(self.h, persistent, wg_nodes)

    def set_active(self, active, stream=None):
        """Retire games of the batch (0) or bring them back (1): retired games keep their state while
        the others iterate."""
        cfr_set_active(self.h, active, self._stream(stream))

    def batch_exploitability(self, stream=None):
        """(expl, br1, br2, value) arrays with one entry per game."""
        return cfr_batch_exploitability(self.h, self.n_games, self._stream(stream))

    def reset(self):
        cfr_reset(self.h)

    @property
    def n_infosets(self) -> int:
        return cfr_num_infosets(self.h)

    def features(self, bucket, history, scalars, x, probe_iters: int = 0, stream=None):
        """Feature rows of every information set into the device tensor x (bf16 [I, 128]); resets,
        then runs probe_iters iterations (their strategies fill columns 120-127)."""
        cfr_features(self.h, bucket, history, scalars, x, self.n_infosets, probe_iters, self._stream(stream))

    def set_payoffs(self, payoff, game: int = 0, stream=None):
        """Rewrite game `game`'s terminal payoffs (array over its description's nodes) in place."""
        a = np.ascontiguousarray(payoff, np.float64)
        _check(load().cfr_set_payoffs(self.h, int(game), _ptr(a), a.size, self._stream(stream)))

    def set_root_chance(self, prob, game: int = 0, stream=None):
        """Rewrite game `game`'s root chance probabilities (root children in description order)."""
        a = np.ascontiguousarray(prob, np.float64)
        _check(load().cfr_set_root_chance(self.h, int(game), _ptr(a), a.size, self._stream(stream)))

    def regret_unit(self, unit, stream=None):
        """m(I) of every set into the device float32 tensor unit [I] (after features())."""
        cfr_regret_unit(self.h, unit, self.n_infosets, self._stream(stream))

    def warm_start(self, mlp: "Mlp", x, scale: float, add: bool = False, stream=None):
        cfr_warm_start(self.h, mlp.h, x, self.n_infosets, scale, add, self._stream(stream))

    def close(self):
        if getattr(self, "h", None):
            cfr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

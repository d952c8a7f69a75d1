"""CPU oracle for CFR (TEST INFRASTRUCTURE ONLY).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product path (the GPU library
and its Python binding) never imports, links or runs anything here, and this
package never imports the product.

``Oracle`` wraps ``oracle.c``: a plain single-threaded FP64 CFR by per-history
recursion with chance on the edges, an exact recursive best response, and the
canonical compiled arrays of a game written out from their definitions.  The
sequence-form LP (``oracle.lp``) and the brute-force enumerators
(``oracle.brute``) pin it from outside.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = {False: os.path.join(_HERE, "liboracle.so"), True: os.path.join(_HERE, "liboracle_f32state.so")}


def build_lib(force: bool = False, f32_state: bool = False) -> str:
    """Compile liboracle.so in place (plain C99, gcc -O2, single-threaded).  f32_state builds the
    FP32-state control variant (strategy sums stay FP64)."""
    src = os.path.join(_HERE, "oracle.c")
    so = _SO[f32_state]
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        tmp = so + ".tmp"
        extra = ["-DORACLE_STATE_FLOAT"] if f32_state else []
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall"] + extra +
                              ["-o", tmp, src, "-lm"])
        os.replace(tmp, so)
    return so


_libs = {}
_P = ctypes.c_void_p


def _load(f32_state: bool = False):
    if f32_state not in _libs:
        lib = ctypes.CDLL(build_lib(f32_state=f32_state))
        lib.or_create.restype = _P
        lib.or_create.argtypes = [ctypes.c_int64, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P, ctypes.c_char_p,
                                  ctypes.c_int]
        lib.or_destroy.argtypes = [_P]
        lib.or_counts.argtypes = [_P, _P]
        lib.or_layout.argtypes = [_P] + [_P] * 12
        lib.or_set_options.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.or_set_rule.argtypes = [_P, ctypes.c_int]
        lib.or_set_reverse.argtypes = [_P, ctypes.c_int]
        lib.or_reset.argtypes = [_P]
        lib.or_iterate.argtypes = [_P, ctypes.c_int64]
        lib.or_iterate.restype = ctypes.c_double
        lib.or_iterations.argtypes = [_P]
        lib.or_iterations.restype = ctypes.c_int64
        lib.or_get.argtypes = [_P, _P, _P, _P, _P]
        lib.or_set_state.argtypes = [_P, _P, _P, ctypes.c_int64]
        lib.or_get_pred.argtypes = [_P, _P]
        lib.or_set_pred.argtypes = [_P, _P]
        lib.or_best_response.argtypes = [_P, ctypes.c_int, _P, _P]
        lib.or_best_response.restype = ctypes.c_double
        lib.or_profile_value.argtypes = [_P, _P]
        lib.or_profile_value.restype = ctypes.c_double
        lib.or_exploitability.argtypes = [_P, _P, _P, _P]
        lib.or_exploitability.restype = ctypes.c_double
        lib.or_node_values.argtypes = [_P, _P, _P, _P]
        _libs[f32_state] = lib
    return _libs[f32_state]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


RULES = {"cfr": 0, "cfr+": 1, "dcfr": 2, "pcfr+": 3}


class Oracle:
    """FP64 CFR oracle over one explicit game (a ``gamegen.Game``-like object).
    f32_state=True selects the FP32-state control build; reverse=True sums children in reverse order
    (a control: another correct rounding pattern).  rule (optional) overrides plus:
    "cfr", "cfr+", "dcfr" or "pcfr+" (see oracle.c for their definitions)."""

    def __init__(self, game, plus: bool = True, linear: bool = True, alternating: bool = False,
                 f32_state: bool = False, rule: str | None = None, reverse: bool = False):
        self._lib = lib = _load(f32_state)
        self._keep = [np.ascontiguousarray(game.type, np.int8), np.ascontiguousarray(game.child_begin, np.int64),
                      np.ascontiguousarray(game.n_children, np.int32), np.ascontiguousarray(game.children, np.int64),
                      np.ascontiguousarray(game.prob, np.float64), np.ascontiguousarray(game.key, np.int64),
                      np.ascontiguousarray(game.payoff, np.float64)]
        err = ctypes.create_string_buffer(256)
        t, cb, nc, ch, pr, ky, pay = self._keep
        self._h = lib.or_create(len(t), int(game.root), _ptr(t), _ptr(cb), _ptr(nc), _ptr(ch), _ptr(pr), _ptr(ky),
                                _ptr(pay), err, 256)
        self._keep = None
        if not self._h:
            raise ValueError("oracle: " + err.value.decode())
        self.pot = float(getattr(game, "pot", 1.0))
        c = np.zeros(8, np.int64)
        lib.or_counts(self._h, _ptr(c))
        self.N, self.E, self.Z, self.Ndec, self.I, self.A, self.max_depth, self.D = [int(x) for x in c]
        self.set_options(plus, linear, alternating)
        if rule is not None:
            self._lib.or_set_rule(self._h, RULES[rule])
        if reverse:
            self._lib.or_set_reverse(self._h, 1)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_destroy(h)
            self._h = None

    def set_options(self, plus=True, linear=True, alternating=False):
        self._lib.or_set_options(self._h, int(plus), int(linear), int(alternating))

    def layout(self) -> dict:
        """Canonical compiled arrays (breadth-first numbering; see oracle.c)."""
        N, I, A = self.N, self.I, self.A
        d = dict(
            depth_off=np.zeros(self.max_depth + 2, np.int32), parent=np.zeros(N, np.int32),
            child_off=np.zeros(N + 1, np.int32), in_slot=np.zeros(N, np.int32),
            node_infoset=np.zeros(N, np.int32), node_type=np.zeros(N, np.int8), tmpl=np.zeros(N, np.float32),
            slot_off=np.zeros(I + 1, np.int32), mem_off=np.zeros(I + 1, np.int32),
            mem_node=np.zeros(max(self.Ndec, 1), np.int32), iset_player=np.zeros(max(I, 1), np.int8),
            iset_key=np.zeros(max(I, 1), np.int64),
        )
        self._lib.or_layout(self._h, *[_ptr(d[k]) for k in ("depth_off", "parent", "child_off", "in_slot",
                                                          "node_infoset", "node_type", "tmpl", "slot_off",
                                                          "mem_off", "mem_node", "iset_player", "iset_key")])
        d["mem_node"] = d["mem_node"][: self.Ndec]
        d["iset_player"] = d["iset_player"][:I]
        d["iset_key"] = d["iset_key"][:I]
        return d

    def reset(self):
        self._lib.or_reset(self._h)

    def iterate(self, T: int) -> float:
        return float(self._lib.or_iterate(self._h, int(T)))

    @property
    def t(self) -> int:
        return int(self._lib.or_iterations(self._h))

    def state(self):
        """(R, sbar, sigma_current_next, sigma_avg) in canonical slot order (float64)."""
        A = max(self.A, 1)
        R, S, sc, sa = (np.zeros(A) for _ in range(4))
        self._lib.or_get(self._h, _ptr(R), _ptr(S), _ptr(sc), _ptr(sa))
        return R[: self.A], S[: self.A], sc[: self.A], sa[: self.A]

    def set_state(self, R=None, sbar=None, t=0, pred=None):
        R = None if R is None else np.ascontiguousarray(R, np.float64)
        sbar = None if sbar is None else np.ascontiguousarray(sbar, np.float64)
        self._lib.or_set_state(self._h, _ptr(R), _ptr(sbar), int(t))
        if pred is not None:
            p = np.ascontiguousarray(pred, np.float64)
            self._lib.or_set_pred(self._h, _ptr(p))

    def prediction(self) -> np.ndarray:
        """PCFR+ prediction (the latest instantaneous regret; zero for the other rules), canonical order."""
        p = np.zeros(max(self.A, 1))
        self._lib.or_get_pred(self._h, _ptr(p))
        return p[: self.A]

    def best_response(self, player: int, profile) -> tuple[float, np.ndarray]:
        prof = np.ascontiguousarray(profile, np.float64)
        ast = np.zeros(max(self.I, 1), np.int32)
        v = self._lib.or_best_response(self._h, int(player), _ptr(prof), _ptr(ast))
        return float(v), ast[: self.I]

    def profile_value(self, profile) -> float:
        prof = np.ascontiguousarray(profile, np.float64)
        return float(self._lib.or_profile_value(self._h, _ptr(prof)))

    def exploitability(self):
        """(expl, BR_1, BR_2, value of the average profile), expl = (BR_1 + BR_2) / 2 in payoff units."""
        b1, b2, v = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        e = self._lib.or_exploitability(self._h, ctypes.byref(b1), ctypes.byref(b2), ctypes.byref(v))
        return float(e), b1.value, b2.value, v.value

    def node_values(self, profile):
        """(textbook, chance-weighted) per-node values of a profile, canonical node order."""
        prof = np.ascontiguousarray(profile, np.float64)
        vt, vf = np.zeros(self.N), np.zeros(self.N)
        self._lib.or_node_values(self._h, _ptr(prof), _ptr(vt), _ptr(vf))
        return vt, vf

    def uniform_profile(self) -> np.ndarray:
        lay = self.layout()
        so = lay["slot_off"]
        prof = np.zeros(self.A)
        for i in range(self.I):
            prof[so[i]:so[i + 1]] = 1.0 / (so[i + 1] - so[i])
        return prof

"""ctypes front end of the FP64 CPU reference in ``pdhg_oracle.c``.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU leg of the benchmark).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "pdhg_oracle.c"
_LIB = _HERE / "liboracle.so"

STATUS = {"OPTIMAL": 0, "ITER_LIMIT": 1, "NUMERICAL": 2, "PUSH_DONE": 3, "PUSH_SKIPPED": 5}


def build_oracle(force: bool = True) -> Path:
    """Compile the oracle with gcc (OpenMP for the row-parallel products)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", str(tmp), str(_SRC), "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrParams(C.Structure):
    _fields_ = [
        ("eps_rel", C.c_double), ("eps_abs", C.c_double), ("max_iter", C.c_int64),
        ("check_every", C.c_int32), ("ruiz_iters", C.c_int32),
        ("restart_suff", C.c_double), ("restart_nec", C.c_double), ("restart_art", C.c_double),
        ("pw_smooth", C.c_double), ("pc_alpha", C.c_double),
        ("power_iters", C.c_int32), ("halpern", C.c_int32),
        ("eta_safety", C.c_double), ("reflect_gamma", C.c_double), ("power_tol", C.c_double),
        ("push_min_iters", C.c_int32), ("pad_", C.c_int32),
        ("push_obj_scale", C.c_double), ("push_max_iter", C.c_int64),
        ("push_gate", C.c_int32), ("record_history", C.c_int32), ("push_gate_rows", C.c_double), ("push_gate_min", C.c_int64),
    ]


class OrKKT(C.Structure):
    _fields_ = [
        ("rp2", C.c_double), ("rd2", C.c_double), ("rpinf", C.c_double), ("rdinf", C.c_double),
        ("pobj", C.c_double), ("dobj", C.c_double), ("gap", C.c_double),
        ("rel_p", C.c_double), ("rel_d", C.c_double), ("rel_gap", C.c_double),
        ("p_off", C.c_int64), ("d_zero", C.c_int64), ("candidates", C.c_int64),
        ("est_primal", C.c_int64), ("est_dual", C.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class OrResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("pad_", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
        ("rel_p", C.c_double), ("rel_d", C.c_double), ("rel_gap", C.c_double),
        ("pobj", C.c_double), ("dobj", C.c_double),
    ]


class OrPushResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("pad_", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
        ("n_fix_lower", C.c_int64), ("n_fix_upper", C.c_int64), ("n_rows_to_eq", C.c_int64),
        ("rel_p_push", C.c_double), ("before", OrKKT), ("after", OrKKT),
        ("n_learned_fix", C.c_int64), ("n_learned_undo", C.c_int64),
    ]


class OrDualPushResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("pad_", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
        ("n_cols_free", C.c_int64), ("n_rows_fixed", C.c_int64),
        ("rel_d_push", C.c_double), ("before", OrKKT), ("after", OrKKT),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build_oracle(force=False)
        lib = C.CDLL(str(_LIB))
        P = C.POINTER
        dp = P(C.c_double)
        lib.or_create.restype = C.c_void_p
        lib.or_create.argtypes = [C.c_int32, C.c_int32, C.c_int64, P(C.c_int64), P(C.c_int32), dp, dp, dp,
                                  dp, dp, C.c_char_p, P(OrParams)]
        lib.or_destroy.argtypes = [C.c_void_p]
        lib.or_default_params.argtypes = [P(OrParams)]
        lib.or_iterate.argtypes = [C.c_void_p, C.c_int64, P(OrResult)]
        lib.or_solve.argtypes = [C.c_void_p, P(OrResult)]
        lib.or_corner_push.argtypes = [C.c_void_p, C.c_uint64, P(OrPushResult)]
        lib.or_corner_push_learned.argtypes = [C.c_void_p, P(C.c_float), C.c_double, C.c_uint64, P(OrPushResult)]
        lib.or_features.argtypes = [C.c_void_p, C.c_uint64, dp, dp]
        lib.or_set_threads.argtypes = [C.c_int]
        lib.or_kkt_weighted.restype = C.c_double
        lib.or_kkt_weighted.argtypes = [C.c_double] * 4
        lib.or_restart_decision.restype = C.c_int
        lib.or_restart_decision.argtypes = [P(OrParams), C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int64]
        lib.or_weight_update.restype = C.c_double
        lib.or_weight_update.argtypes = [P(OrParams), C.c_double, C.c_double, C.c_double]
        lib.or_dual_push.argtypes = [C.c_void_p, C.c_uint64, P(OrDualPushResult)]
        lib.or_get_rhs_scaled.argtypes = [C.c_void_p, dp]
        lib.or_kkt_report.argtypes = [C.c_void_p, dp, dp, P(OrKKT)]
        lib.or_get_iterate.argtypes = [C.c_void_p, dp, dp]
        lib.or_get_iterate_scaled.argtypes = [C.c_void_p, dp, dp]
        lib.or_get_solution.argtypes = [C.c_void_p, dp, dp, dp]
        lib.or_get_scaling.argtypes = [C.c_void_p, dp, dp, dp]
        lib.or_get_model_scaled.argtypes = [C.c_void_p, dp, dp, dp, C.c_char_p]
        lib.or_get_nnz.restype = C.c_int64
        lib.or_get_nnz.argtypes = [C.c_void_p]
        lib.or_get_ahat.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32), dp]
        lib.or_splitmix64.restype = C.c_uint64
        lib.or_splitmix64.argtypes = [C.c_uint64]
        lib.or_push_uniform.restype = C.c_double
        lib.or_push_uniform.argtypes = [C.c_uint64, C.c_int64]
        for f in ("or_params_size", "or_kkt_size", "or_push_result_size", "or_dual_push_result_size",
                  "or_num_threads"):
            getattr(lib, f).restype = C.c_int
        assert lib.or_params_size() == C.sizeof(OrParams)
        assert lib.or_kkt_size() == C.sizeof(OrKKT)
        assert lib.or_push_result_size() == C.sizeof(OrPushResult)
        assert lib.or_dual_push_result_size() == C.sizeof(OrDualPushResult)
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def splitmix64(x: int) -> int:
    return int(_load().or_splitmix64(C.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def num_threads() -> int:
    return int(_load().or_num_threads())


def push_uniform(seed: int, j: int) -> float:
    return float(_load().or_push_uniform(C.c_uint64(seed), C.c_int64(j)))


def set_threads(k: int) -> None:
    """Threads of the oracle's row-parallel products from now on."""
    _load().or_set_threads(int(k))


def kkt_weighted(omega: float, p2: float, d2: float, gap2: float) -> float:
    """The weighted KKT measure the restart rule compares."""
    return float(_load().or_kkt_weighted(omega, p2, d2, gap2))


def restart_decision(kc: float, ka: float, kprev: float, k: int, t: int, **params) -> bool:
    """The restart rule of a check, as the oracle's loop applies it."""
    p = default_params(**params)
    return bool(_load().or_restart_decision(C.byref(p), kc, ka, kprev, int(k), int(t)))


def weight_update(omega: float, dx: float, dy: float, **params) -> float:
    """The primal weight after a restart whose anchors moved by dx and dy."""
    p = default_params(**params)
    return float(_load().or_weight_update(C.byref(p), omega, dx, dy))


def default_params(**kw) -> OrParams:
    p = OrParams()
    _load().or_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class OracleSolver:
    """One LP held by the CPU reference (scaled internally; all I/O unscaled)."""

    def __init__(self, lp, **params):
        self.lib = _load()
        self.lp = lp
        self.m, self.n = lp.m, lp.n
        self.params = default_params(**params)
        self._keep = [np.ascontiguousarray(lp.row_ptr, dtype=np.int64), np.ascontiguousarray(lp.col, dtype=np.int32),
                      np.ascontiguousarray(lp.val, dtype=np.float64), np.ascontiguousarray(lp.b, dtype=np.float64),
                      np.ascontiguousarray(lp.c, dtype=np.float64), np.ascontiguousarray(lp.l, dtype=np.float64),
                      np.ascontiguousarray(lp.u, dtype=np.float64)]
        rp, ci, va, b, c, l, u = self._keep
        sense = bytes(np.asarray(lp.sense, dtype=np.uint8))
        self.h = self.lib.or_create(lp.m, lp.n, int(rp[-1]) if rp.size else 0,
                                    rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                    ci.ctypes.data_as(C.POINTER(C.c_int32)), _dp(va), _dp(b), _dp(c), _dp(l), _dp(u),
                                    sense, C.byref(self.params))
        if not self.h:
            raise ValueError("oracle rejected the LP (invalid input)")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.or_destroy(h)
            self.h = None

    def iterate(self, iters: int) -> OrResult:
        r = OrResult()
        self.lib.or_iterate(self.h, int(iters), C.byref(r))
        return r

    def solve(self) -> OrResult:
        r = OrResult()
        self.lib.or_solve(self.h, C.byref(r))
        return r

    def corner_push(self, seed: int) -> OrPushResult:
        r = OrPushResult()
        st = self.lib.or_corner_push(self.h, C.c_uint64(seed), C.byref(r))
        if st < 0:
            raise RuntimeError("corner push needs a prior solve")
        return r

    def corner_push_learned(self, logits, theta: float, seed: int) -> OrPushResult:
        """Corner push with the learned warm start from per-column logits
        (float32, one per column)."""
        lg = np.ascontiguousarray(logits, dtype=np.float32)
        if lg.shape != (self.n,):
            raise ValueError("one logit per column")
        r = OrPushResult()
        st = self.lib.or_corner_push_learned(self.h, lg.ctypes.data_as(C.POINTER(C.c_float)), float(theta),
                                             C.c_uint64(seed), C.byref(r))
        if st == -1:
            raise ValueError("theta must lie in (0, 1)")
        if st < 0:
            raise RuntimeError("corner push needs a prior solve")
        return r

    def features(self, seed: int, with_scale: bool = False):
        """The 16 learned-warm-start features of every column (n x 16); with
        with_scale, also each feature's normalising scale (16)."""
        out = np.zeros((self.n, 16))
        sc = np.zeros(16)
        if self.lib.or_features(self.h, C.c_uint64(seed), _dp(out), _dp(sc)) != 0:
            raise RuntimeError("features need a solve and no push yet")
        return (out, sc) if with_scale else out

    def dual_push(self, seed: int) -> OrDualPushResult:
        """Dual corner push; afterwards solution() gives (x, yhat, zhat)."""
        r = OrDualPushResult()
        st = self.lib.or_dual_push(self.h, C.c_uint64(seed), C.byref(r))
        if st < 0:
            raise RuntimeError("dual push needs a prior solve (and runs once)")
        return r

    def kkt(self, x=None, y=None) -> OrKKT:
        k = OrKKT()
        xa = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        ya = None if y is None else np.ascontiguousarray(y, dtype=np.float64)
        self.lib.or_kkt_report(self.h, None if xa is None else _dp(xa), None if ya is None else _dp(ya), C.byref(k))
        return k

    def iterate_state(self, scaled: bool = False):
        x, y = np.zeros(self.n), np.zeros(self.m)
        f = self.lib.or_get_iterate_scaled if scaled else self.lib.or_get_iterate
        f(self.h, _dp(x), _dp(y))
        return x, y

    def solution(self):
        x, y, z = np.zeros(self.n), np.zeros(self.m), np.zeros(self.n)
        self.lib.or_get_solution(self.h, _dp(x), _dp(y), _dp(z))
        return x, y, z

    def scaling(self):
        dr, dc, o5 = np.zeros(self.m), np.zeros(self.n), np.zeros(5)
        self.lib.or_get_scaling(self.h, _dp(dr), _dp(dc), _dp(o5))
        return {"dr": dr, "dc": dc, "eta": o5[0], "omega": o5[1], "sigma_est": o5[2], "t": int(o5[3]),
                "power_steps": int(o5[4])}

    def model_scaled(self):
        lh, uh, ch = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        sense = C.create_string_buffer(self.m + 1)
        self.lib.or_get_model_scaled(self.h, _dp(lh), _dp(uh), _dp(ch), sense)
        return lh, uh, ch, sense.raw[: self.m]

    def rhs_scaled(self):
        bh = np.zeros(self.m)
        self.lib.or_get_rhs_scaled(self.h, _dp(bh))
        return bh

    def ahat(self):
        nnz = int(self.lib.or_get_nnz(self.h))
        rp = np.zeros(self.m + 1, dtype=np.int64)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros(max(nnz, 1))
        self.lib.or_get_ahat(self.h, rp.ctypes.data_as(C.POINTER(C.c_int64)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
                             _dp(v))
        return rp, ci[:nnz], v[:nnz]

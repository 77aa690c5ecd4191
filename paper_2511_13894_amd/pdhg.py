"""Python binding of libpdhg.so (ctypes; argument marshalling only).

Every entry point of include/pdhg.h is reachable under the same name; all
arithmetic runs in the library's HIP kernels.  The binding refuses to fall
back to anything else: if the library is missing it raises.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path
from typing import Optional

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libpdhg.so"

STATUS = {0: "OPTIMAL", 1: "ITER_LIMIT", 2: "NUMERICAL", 3: "PUSH_DONE", 4: "TIME_LIMIT", 5: "PUSH_SKIPPED"}
PDHG_OPTIMAL, PDHG_ITER_LIMIT, PDHG_NUMERICAL, PDHG_PUSH_DONE, PDHG_TIME_LIMIT, PDHG_PUSH_SKIPPED = range(6)
PDHG_FP64, PDHG_FP32_MIXED = 0, 1
ERRORS = {-1: "INVALID_ARG", -2: "STATE", -3: "OOM", -4: "HIP"}


class PdhgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("eps_rel", C.c_double), ("eps_abs", C.c_double), ("max_iter", C.c_int64),
        ("check_every", C.c_int32), ("ruiz_iters", C.c_int32),
        ("restart_suff", C.c_double), ("restart_nec", C.c_double), ("restart_art", C.c_double),
        ("pw_smooth", C.c_double), ("pc_alpha", C.c_double),
        ("power_iters", C.c_int32), ("halpern", C.c_int32),
        ("eta_safety", C.c_double), ("reflect_gamma", C.c_double), ("power_tol", C.c_double),
        ("push_min_iters", C.c_int32), ("precision", C.c_int32),
        ("push_obj_scale", C.c_double), ("push_max_iter", C.c_int64), ("time_limit", C.c_double),
        ("stream", C.c_void_p), ("verbosity", C.c_int32), ("lanes_at", C.c_int32), ("lanes_a", C.c_int32),
        ("use_graph", C.c_int32), ("timing", C.c_int32), ("autotune", C.c_int32), ("record_history", C.c_int32),
        ("push_compact", C.c_int32), ("push_gate", C.c_int32), ("push_gate_rows", C.c_double),
        ("push_gate_min", C.c_int64),
    ]


class Result(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("pad_", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
        ("rel_p", C.c_double), ("rel_d", C.c_double), ("rel_gap", C.c_double),
        ("pobj", C.c_double), ("dobj", C.c_double), ("seconds", C.c_double),
    ]


class KKTReport(C.Structure):
    _fields_ = [
        ("rp2", C.c_double), ("rd2", C.c_double), ("rpinf", C.c_double), ("rdinf", C.c_double),
        ("pobj", C.c_double), ("dobj", C.c_double), ("gap", C.c_double),
        ("rel_p", C.c_double), ("rel_d", C.c_double), ("rel_gap", C.c_double),
        ("p_off", C.c_int64), ("d_zero", C.c_int64), ("candidates", C.c_int64),
        ("est_primal", C.c_int64), ("est_dual", C.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PushResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("pad_", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
        ("n_fix_lower", C.c_int64), ("n_fix_upper", C.c_int64), ("n_rows_to_eq", C.c_int64),
        ("rel_p_push", C.c_double), ("seconds", C.c_double), ("before", KKTReport), ("after", KKTReport),
        ("n_learned_fix", C.c_int64), ("n_learned_undo", C.c_int64),
    ]


class DualPushResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("pad_", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
        ("n_cols_free", C.c_int64), ("n_rows_fixed", C.c_int64),
        ("rel_d_push", C.c_double), ("seconds", C.c_double), ("before", KKTReport), ("after", KKTReport),
    ]


class Timing(C.Structure):
    _fields_ = [
        ("primal_ms", C.c_double), ("dual_ms", C.c_double), ("samples", C.c_int64),
        ("bytes_primal", C.c_int64), ("bytes_dual", C.c_int64), ("lanes_at", C.c_int32), ("lanes_a", C.c_int32),
    ]


class LpDesc(C.Structure):
    _fields_ = [
        ("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64),
        ("row_ptr", C.POINTER(C.c_int64)), ("col_idx", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double)),
        ("b", C.POINTER(C.c_double)), ("c", C.POINTER(C.c_double)), ("l", C.POINTER(C.c_double)),
        ("u", C.POINTER(C.c_double)), ("sense", C.c_char_p),
    ]


class BatchReport(C.Structure):
    _fields_ = [
        ("count", C.c_int32), ("lanes_at", C.c_int32), ("lanes_a", C.c_int32), ("pad_", C.c_int32),
        ("solve_seconds", C.c_double), ("push_seconds", C.c_double),
        ("solve_lockstep_iters", C.c_int64), ("push_lockstep_iters", C.c_int64),
        ("primal_ms", C.c_double), ("dual_ms", C.c_double), ("samples", C.c_int64),
        ("bytes_primal", C.c_int64), ("bytes_dual", C.c_int64),
        ("total_m", C.c_int64), ("total_n", C.c_int64), ("total_nnz", C.c_int64),
    ]


class TrainParams(C.Structure):
    _fields_ = [
        ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
        ("beta2", C.c_double), ("eps", C.c_double), ("pos_weight", C.c_double), ("seed", C.c_uint64),
    ]


class TrainReport(C.Structure):
    _fields_ = [
        ("loss_first", C.c_double), ("loss_last", C.c_double), ("seconds", C.c_double), ("steps", C.c_int64),
        ("samples_per_s", C.c_double), ("pos_weight", C.c_double),
    ]


MLP_NPARAMS = 5313
MLP_FEATURES = 16

EXPORTS = ["pdhg_default_params", "pdhg_create", "pdhg_solve", "pdhg_iterate", "pdhg_corner_push", "pdhg_kkt",
           "pdhg_get_solution", "pdhg_get_iterate", "pdhg_get_scaling", "pdhg_destroy", "pdhg_last_error",
           "pdhg_struct_size", "pdhg_get_timing", "pdhg_copy_probe", "pdhg_batch_create", "pdhg_batch_solve",
           "pdhg_batch_corner_push", "pdhg_batch_get_solution", "pdhg_batch_get_report", "pdhg_batch_destroy",
           "pdhg_mlp_create", "pdhg_mlp_destroy", "pdhg_mlp_set_params", "pdhg_mlp_get_params", "pdhg_mlp_forward",
           "pdhg_mlp_gradient", "pdhg_default_train_params", "pdhg_mlp_train", "pdhg_features",
           "pdhg_batch_features", "pdhg_batch_corner_push_learned",
           "pdhg_corner_push_learned", "pdhg_get_solution_device", "pdhg_set_start", "pdhg_state_size",
           "pdhg_get_state", "pdhg_set_state", "pdhg_get_solve_solution", "pdhg_batch_get_solve_solution",
           "pdhg_dual_push", "pdhg_batch_dual_push", "pdhg_corner_push_logits", "pdhg_batch_corner_push_logits",
           "pdhg_create_device", "pdhg_mlp_forward_noalloc", "pdhg_batch_create_device"]

_lib = None


def load(path: Optional[Path] = None):
    """Load libpdhg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"{p} is not built; run __graft_entry__.build() (hipcc for gfx950) first")
    lib = C.CDLL(str(p))
    P = C.POINTER
    dp = P(C.c_double)
    lib.pdhg_default_params.argtypes = [P(Params)]
    lib.pdhg_default_params.restype = None
    lib.pdhg_create.argtypes = [C.c_int32, C.c_int32, C.c_int64, P(C.c_int64), P(C.c_int32), dp, dp, dp, dp, dp,
                                C.c_char_p, P(Params), P(C.c_void_p)]
    vp = C.c_void_p
    lib.pdhg_create_device.argtypes = [C.c_int32, C.c_int32, C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, P(Params),
                                       P(C.c_void_p)]
    lib.pdhg_solve.argtypes = [C.c_void_p, P(Result)]
    lib.pdhg_iterate.argtypes = [C.c_void_p, C.c_int64, P(Result)]
    lib.pdhg_corner_push.argtypes = [C.c_void_p, C.c_uint64, P(PushResult)]
    lib.pdhg_dual_push.argtypes = [C.c_void_p, C.c_uint64, P(DualPushResult)]
    lib.pdhg_batch_dual_push.argtypes = [C.c_void_p, P(C.c_uint64), P(DualPushResult)]
    lib.pdhg_kkt.argtypes = [C.c_void_p, dp, dp, P(KKTReport)]
    lib.pdhg_get_solution.argtypes = [C.c_void_p, dp, dp, dp]
    lib.pdhg_get_solve_solution.argtypes = [C.c_void_p, dp, dp, dp]
    lib.pdhg_get_iterate.argtypes = [C.c_void_p, dp, dp]
    lib.pdhg_get_scaling.argtypes = [C.c_void_p, dp, dp, dp]
    lib.pdhg_get_timing.argtypes = [C.c_void_p, P(Timing)]
    lib.pdhg_copy_probe.argtypes = [C.c_int64, C.c_int32, dp]
    lib.pdhg_destroy.argtypes = [C.c_void_p]
    lib.pdhg_destroy.restype = None
    lib.pdhg_batch_create.argtypes = [C.c_int32, P(LpDesc), P(Params), P(C.c_void_p)]
    lib.pdhg_batch_create_device.argtypes = [C.c_int32, P(LpDesc), P(Params), P(C.c_void_p)]
    lib.pdhg_batch_solve.argtypes = [C.c_void_p, P(Result)]
    lib.pdhg_batch_corner_push.argtypes = [C.c_void_p, P(C.c_uint64), P(PushResult)]
    lib.pdhg_batch_get_solution.argtypes = [C.c_void_p, C.c_int32, dp, dp, dp]
    lib.pdhg_batch_get_solve_solution.argtypes = [C.c_void_p, C.c_int32, dp, dp, dp]
    lib.pdhg_batch_get_report.argtypes = [C.c_void_p, P(BatchReport)]
    lib.pdhg_batch_destroy.argtypes = [C.c_void_p]
    lib.pdhg_batch_destroy.restype = None
    fp = P(C.c_float)
    lib.pdhg_mlp_create.argtypes = [C.c_uint64, P(C.c_void_p)]
    lib.pdhg_mlp_destroy.argtypes = [C.c_void_p]
    lib.pdhg_mlp_destroy.restype = None
    lib.pdhg_mlp_set_params.argtypes = [C.c_void_p, fp]
    lib.pdhg_mlp_get_params.argtypes = [C.c_void_p, fp]
    lib.pdhg_mlp_forward.argtypes = [C.c_void_p, fp, C.c_int64, fp]
    lib.pdhg_mlp_forward_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    lib.pdhg_mlp_forward_noalloc.restype = C.c_int
    lib.pdhg_mlp_gradient.argtypes = [C.c_void_p, fp, fp, C.c_int64, C.c_double, fp, P(C.c_double)]
    lib.pdhg_default_train_params.argtypes = [P(TrainParams)]
    lib.pdhg_default_train_params.restype = None
    lib.pdhg_mlp_train.argtypes = [C.c_void_p, fp, fp, C.c_int64, P(TrainParams), P(TrainReport)]
    lib.pdhg_features.argtypes = [C.c_void_p, C.c_uint64, fp]
    lib.pdhg_corner_push_learned.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_uint64, P(PushResult)]
    lib.pdhg_batch_features.argtypes = [C.c_void_p, P(C.c_uint64), fp]
    lib.pdhg_get_solution_device.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.pdhg_set_start.argtypes = [C.c_void_p, dp, dp]
    lib.pdhg_state_size.argtypes = [C.c_void_p, P(C.c_int64)]
    lib.pdhg_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
    lib.pdhg_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
    lib.pdhg_batch_corner_push_learned.argtypes = [C.c_void_p, C.c_void_p, C.c_double, P(C.c_uint64), P(PushResult)]
    lib.pdhg_corner_push_logits.argtypes = [C.c_void_p, fp, C.c_double, C.c_uint64, P(PushResult)]
    lib.pdhg_batch_corner_push_logits.argtypes = [C.c_void_p, fp, C.c_double, P(C.c_uint64), P(PushResult)]
    lib.pdhg_last_error.restype = C.c_char_p
    lib.pdhg_struct_size.restype = C.c_int32
    lib.pdhg_struct_size.argtypes = [C.c_int32]
    for fn in ("pdhg_create", "pdhg_solve", "pdhg_iterate", "pdhg_corner_push", "pdhg_dual_push",
               "pdhg_batch_dual_push", "pdhg_kkt",
               "pdhg_get_solution",
               "pdhg_get_iterate", "pdhg_get_scaling", "pdhg_get_timing", "pdhg_copy_probe", "pdhg_batch_create",
               "pdhg_batch_solve", "pdhg_batch_corner_push", "pdhg_batch_get_solution", "pdhg_batch_get_report",
               "pdhg_mlp_create", "pdhg_mlp_set_params", "pdhg_mlp_get_params", "pdhg_mlp_forward",
               "pdhg_mlp_gradient", "pdhg_mlp_train", "pdhg_features", "pdhg_corner_push_learned",
               "pdhg_batch_features", "pdhg_batch_corner_push_learned", "pdhg_get_solution_device",
               "pdhg_set_start", "pdhg_state_size", "pdhg_get_state", "pdhg_set_state", "pdhg_get_solve_solution",
               "pdhg_batch_get_solve_solution", "pdhg_corner_push_logits", "pdhg_batch_corner_push_logits",
               "pdhg_create_device"):
        getattr(lib, fn).restype = C.c_int
    sizes = [C.sizeof(Params), C.sizeof(Result), C.sizeof(KKTReport), C.sizeof(PushResult), C.sizeof(Timing),
             C.sizeof(LpDesc), C.sizeof(BatchReport), C.sizeof(DualPushResult)]
    for which, want in enumerate(sizes):
        got = lib.pdhg_struct_size(which)
        if got != want:
            raise RuntimeError(f"struct {which} size mismatch: library {got}, binding {want}")
    if path is None:
        _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def default_params(**kw) -> Params:
    p = Params()
    load().pdhg_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": PDHG_FP64, "fp32": PDHG_FP32_MIXED, "fp32_mixed": PDHG_FP32_MIXED}[v]
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def copy_probe(nbytes: int, reps: int = 20) -> float:
    """Achieved GB/s of a plain device copy of nbytes (read + write counted)."""
    _refuse_second_runtime()
    g = C.c_double()
    rc = load().pdhg_copy_probe(int(nbytes), int(reps), C.byref(g))
    if rc != 0:
        raise PdhgError(rc, load().pdhg_last_error().decode())
    return g.value


def _refuse_second_runtime():
    """libpdhg.so runs on the system ROCm HIP runtime.  torch wheels bundle a
    second copy of the HIP/HSA runtime; once torch has initialised it, the
    device is not visible to another runtime in the same process."""
    import sys

    t = sys.modules.get("torch")
    if t is not None:
        try:
            if t.cuda.is_initialized():
                raise RuntimeError("torch has initialised its bundled HIP runtime in this process; "
                                   "libpdhg.so needs the GPU through the system ROCm runtime "
                                   "(use a process without torch GPU calls)")
        except AttributeError:
            pass


_hip = None


def _hip_runtime():
    """The HIP runtime the library links (device memory for DeviceLP)."""
    global _hip
    if _hip is None:
        load()
        h = C.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        h.hipFree.argtypes = [C.c_void_p]
        h.hipDeviceSynchronize.argtypes = []
        for f in ("hipMalloc", "hipMemcpy", "hipFree", "hipDeviceSynchronize"):
            getattr(h, f).restype = C.c_int
        _hip = h
    return _hip


class DeviceLP:
    """An LP's arrays copied once into device memory (the inputs of
    pdhg_create_device): rows must be sorted with unique columns."""

    FIELDS = (("row_ptr", np.int64), ("col", np.int32), ("val", np.float64), ("b", np.float64),
              ("c", np.float64), ("l", np.float64), ("u", np.float64), ("sense", np.uint8))

    def __init__(self, lp):
        _refuse_second_runtime()
        hip = _hip_runtime()
        self.m, self.n, self.nnz = int(lp.m), int(lp.n), int(lp.nnz)
        self.ptr = {}
        for name, dt in self.FIELDS:
            a = np.ascontiguousarray(getattr(lp, name), dtype=dt)
            p = C.c_void_p()
            if hip.hipMalloc(C.byref(p), max(a.nbytes, 8)) != 0:
                self.free()
                raise PdhgError(-3, f"hipMalloc of {name} failed")
            self.ptr[name] = p
            if a.nbytes and hip.hipMemcpy(p, a.ctypes.data_as(C.c_void_p), a.nbytes, 1) != 0:
                self.free()
                raise PdhgError(-4, f"copy of {name} to the device failed")

    def free(self):
        for p in self.ptr.values():
            _hip_runtime().hipFree(p)
        self.ptr = {}

    def __del__(self):
        if getattr(self, "ptr", None):
            self.free()


class Solver:
    """One LP on the GPU (pdhg_create ... pdhg_destroy); a DeviceLP goes
    through pdhg_create_device."""

    def __init__(self, lp, stream=None, **params):
        _refuse_second_runtime()
        self.lib = load()
        self.m, self.n = int(lp.m), int(lp.n)
        self.params = default_params(**params)
        self.params.stream = stream.value if isinstance(stream, C.c_void_p) else stream
        if isinstance(lp, DeviceLP):
            d = lp.ptr
            h = C.c_void_p()
            rc = self.lib.pdhg_create_device(self.m, self.n, lp.nnz, d["row_ptr"], d["col"], d["val"], d["b"], d["c"],
                                             d["l"], d["u"], d["sense"], C.byref(self.params), C.byref(h))
            self._check(rc)
            self.h = h
            return
        rp = np.ascontiguousarray(lp.row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(lp.col, dtype=np.int32)
        va = np.ascontiguousarray(lp.val, dtype=np.float64)
        b = np.ascontiguousarray(lp.b, dtype=np.float64)
        c = np.ascontiguousarray(lp.c, dtype=np.float64)
        l = np.ascontiguousarray(lp.l, dtype=np.float64)
        u = np.ascontiguousarray(lp.u, dtype=np.float64)
        sense = bytes(np.asarray(lp.sense, dtype=np.uint8))
        h = C.c_void_p()
        rc = self.lib.pdhg_create(self.m, self.n, int(rp[-1]) if rp.size else 0,
                                  rp.ctypes.data_as(C.POINTER(C.c_int64)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
                                  _dp(va), _dp(b), _dp(c), _dp(l), _dp(u), sense, C.byref(self.params), C.byref(h))
        self._check(rc)
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise PdhgError(rc, self.lib.pdhg_last_error().decode())

    def __del__(self):
        self.destroy()

    def destroy(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.pdhg_destroy(h)
        self.h = None

    def solve(self) -> Result:
        r = Result()
        self._check(self.lib.pdhg_solve(self.h, C.byref(r)))
        return r

    def iterate(self, iters: int) -> Result:
        r = Result()
        self._check(self.lib.pdhg_iterate(self.h, int(iters), C.byref(r)))
        return r

    def corner_push(self, seed: int) -> PushResult:
        r = PushResult()
        self._check(self.lib.pdhg_corner_push(self.h, C.c_uint64(seed), C.byref(r)))
        return r

    def dual_push(self, seed: int) -> DualPushResult:
        """Dual corner push; afterwards get_solution() gives (x, yhat, zhat)."""
        r = DualPushResult()
        self._check(self.lib.pdhg_dual_push(self.h, C.c_uint64(seed), C.byref(r)))
        return r

    def kkt(self, x=None, y=None) -> KKTReport:
        k = KKTReport()
        xa = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        ya = None if y is None else np.ascontiguousarray(y, dtype=np.float64)
        self._check(self.lib.pdhg_kkt(self.h, None if xa is None else _dp(xa), None if ya is None else _dp(ya),
                                      C.byref(k)))
        return k

    def get_solution(self):
        x, y, z = np.zeros(self.n), np.zeros(self.m), np.zeros(self.n)
        self._check(self.lib.pdhg_get_solution(self.h, _dp(x), _dp(y), _dp(z)))
        return x, y, z

    def get_solve_solution(self):
        """The solve's own (x, y, z), also after a push."""
        x, y, z = np.zeros(self.n), np.zeros(self.m), np.zeros(self.n)
        self._check(self.lib.pdhg_get_solve_solution(self.h, _dp(x), _dp(y), _dp(z)))
        return x, y, z

    def get_iterate(self):
        x, y = np.zeros(self.n), np.zeros(self.m)
        self._check(self.lib.pdhg_get_iterate(self.h, _dp(x), _dp(y)))
        return x, y

    def features(self, seed: int = 0):
        f = np.zeros((self.n, 16), dtype=np.float32)
        self._check(self.lib.pdhg_features(self.h, C.c_uint64(seed), f.ctypes.data_as(C.POINTER(C.c_float))))
        return f

    def corner_push_learned(self, net, theta: float, seed: int) -> PushResult:
        r = PushResult()
        self._check(self.lib.pdhg_corner_push_learned(self.h, net.h, float(theta), C.c_uint64(seed), C.byref(r)))
        return r

    def corner_push_logits(self, logits, theta: float, seed: int) -> PushResult:
        """Learned warm start from caller logits (one float32 per column)."""
        lg = np.ascontiguousarray(logits, dtype=np.float32)
        if lg.shape != (self.n,):
            raise ValueError("one logit per column")
        r = PushResult()
        self._check(self.lib.pdhg_corner_push_logits(self.h, lg.ctypes.data_as(C.POINTER(C.c_float)), float(theta),
                                                     C.c_uint64(seed), C.byref(r)))
        return r

    def set_start(self, x, y):
        xa = np.ascontiguousarray(x, dtype=np.float64)
        ya = np.ascontiguousarray(y, dtype=np.float64)
        self._check(self.lib.pdhg_set_start(self.h, _dp(xa), _dp(ya)))

    def get_state(self) -> bytes:
        nb = C.c_int64()
        self._check(self.lib.pdhg_state_size(self.h, C.byref(nb)))
        buf = C.create_string_buffer(nb.value)
        self._check(self.lib.pdhg_get_state(self.h, buf, nb.value))
        return buf.raw

    def set_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        self._check(self.lib.pdhg_set_state(self.h, buf, len(state)))

    def get_timing(self) -> Timing:
        t = Timing()
        self._check(self.lib.pdhg_get_timing(self.h, C.byref(t)))
        return t

    def get_scaling(self):
        dr, dc, s5 = np.zeros(self.m), np.zeros(self.n), np.zeros(5)
        self._check(self.lib.pdhg_get_scaling(self.h, _dp(dr), _dp(dc), _dp(s5)))
        return {"dr": dr, "dc": dc, "eta": s5[0], "omega": s5[1], "sigma_est": s5[2], "t": int(s5[3]),
                "power_steps": int(s5[4])}


class DeviceBatch:
    """Many LPs' arrays copied once into device memory (the inputs of
    pdhg_batch_create_device): rows must be sorted with unique columns."""

    def __init__(self, lps):
        self.lps = list(lps)
        self.dev = [DeviceLP(lp) for lp in self.lps]


class Batch:
    """Many LPs solved and corner-pushed together (pdhg_batch_*); a
    DeviceBatch goes through pdhg_batch_create_device."""

    def __init__(self, lps, **params):
        _refuse_second_runtime()
        self.lib = load()
        device = isinstance(lps, DeviceBatch)
        self.lps = list(lps.lps) if device else list(lps)
        self.count = len(self.lps)
        self.params = default_params(**params)
        self.params.stream = None
        descs = (LpDesc * self.count)()
        self._keep = []
        if device:
            for d, dl in zip(descs, lps.dev):
                q = dl.ptr
                d.m, d.n, d.nnz = dl.m, dl.n, dl.nnz
                d.row_ptr = C.cast(q["row_ptr"], C.POINTER(C.c_int64))
                d.col_idx = C.cast(q["col"], C.POINTER(C.c_int32))
                d.val, d.b, d.c, d.l, d.u = (C.cast(q[k], C.POINTER(C.c_double)) for k in ("val", "b", "c", "l", "u"))
                d.sense = C.cast(q["sense"], C.c_char_p)
            self._keep.append(lps)
            h = C.c_void_p()
            rc = self.lib.pdhg_batch_create_device(self.count, descs, C.byref(self.params), C.byref(h))
            if rc != 0:
                raise PdhgError(rc, self.lib.pdhg_last_error().decode())
            self.h = h
            return
        for d, lp in zip(descs, self.lps):
            arrs = [np.ascontiguousarray(lp.row_ptr, dtype=np.int64), np.ascontiguousarray(lp.col, dtype=np.int32),
                    np.ascontiguousarray(lp.val, dtype=np.float64), np.ascontiguousarray(lp.b, dtype=np.float64),
                    np.ascontiguousarray(lp.c, dtype=np.float64), np.ascontiguousarray(lp.l, dtype=np.float64),
                    np.ascontiguousarray(lp.u, dtype=np.float64)]
            sense = bytes(np.asarray(lp.sense, dtype=np.uint8))
            self._keep += arrs + [sense]
            rp, ci, va, b, c, l, u = arrs
            d.m, d.n, d.nnz = int(lp.m), int(lp.n), int(rp[-1])
            d.row_ptr = rp.ctypes.data_as(C.POINTER(C.c_int64))
            d.col_idx = ci.ctypes.data_as(C.POINTER(C.c_int32))
            d.val, d.b, d.c, d.l, d.u = _dp(va), _dp(b), _dp(c), _dp(l), _dp(u)
            d.sense = sense
        h = C.c_void_p()
        rc = self.lib.pdhg_batch_create(self.count, descs, C.byref(self.params), C.byref(h))
        if rc != 0:
            raise PdhgError(rc, self.lib.pdhg_last_error().decode())
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise PdhgError(rc, self.lib.pdhg_last_error().decode())

    def __del__(self):
        self.destroy()

    def destroy(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.pdhg_batch_destroy(h)
        self.h = None

    def solve(self):
        r = (Result * self.count)()
        self._check(self.lib.pdhg_batch_solve(self.h, r))
        return list(r)

    def corner_push(self, seeds):
        sd = (C.c_uint64 * self.count)(*[int(v) for v in seeds])
        r = (PushResult * self.count)()
        self._check(self.lib.pdhg_batch_corner_push(self.h, sd, r))
        return list(r)

    def dual_push(self, seeds):
        """Dual corner push of every LP; afterwards get_solution(i) gives (x, yhat, zhat)."""
        sd = (C.c_uint64 * self.count)(*[int(v) for v in seeds])
        r = (DualPushResult * self.count)()
        self._check(self.lib.pdhg_batch_dual_push(self.h, sd, r))
        return list(r)

    def corner_push_learned(self, net, theta: float, seeds):
        sd = (C.c_uint64 * self.count)(*[int(v) for v in seeds])
        r = (PushResult * self.count)()
        self._check(self.lib.pdhg_batch_corner_push_learned(self.h, net.h, float(theta), sd, r))
        return list(r)

    def corner_push_logits(self, logits, theta: float, seeds):
        """Learned warm start of every LP from caller logits (the LPs' columns in batch order)."""
        lg = np.ascontiguousarray(logits, dtype=np.float32)
        if lg.shape != (sum(lp.n for lp in self.lps),):
            raise ValueError("one logit per column of the batch")
        sd = (C.c_uint64 * self.count)(*[int(v) for v in seeds])
        r = (PushResult * self.count)()
        self._check(self.lib.pdhg_batch_corner_push_logits(self.h, lg.ctypes.data_as(C.POINTER(C.c_float)),
                                                           float(theta), sd, r))
        return list(r)

    def features(self, seeds):
        """Per-LP feature arrays (n_i x 16) of the solved batch."""
        sd = (C.c_uint64 * self.count)(*[int(v) for v in seeds])
        n = sum(int(lp.n) for lp in self.lps)
        f = np.zeros((n, 16), dtype=np.float32)
        self._check(self.lib.pdhg_batch_features(self.h, sd, f.ctypes.data_as(C.POINTER(C.c_float))))
        out, k = [], 0
        for lp in self.lps:
            out.append(f[k:k + lp.n])
            k += lp.n
        return out

    def get_solution(self, i):
        lp = self.lps[i]
        x, y, z = np.zeros(lp.n), np.zeros(lp.m), np.zeros(lp.n)
        self._check(self.lib.pdhg_batch_get_solution(self.h, int(i), _dp(x), _dp(y), _dp(z)))
        return x, y, z

    def get_solve_solution(self, i):
        """LP i's solve answer (x, y, z), also after the push."""
        lp = self.lps[i]
        x, y, z = np.zeros(lp.n), np.zeros(lp.m), np.zeros(lp.n)
        self._check(self.lib.pdhg_batch_get_solve_solution(self.h, int(i), _dp(x), _dp(y), _dp(z)))
        return x, y, z

    def report(self) -> BatchReport:
        r = BatchReport()
        self._check(self.lib.pdhg_batch_get_report(self.h, C.byref(r)))
        return r


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Mlp:
    """The per-variable fix predictor on the GPU (pdhg_mlp_*)."""

    def __init__(self, seed: int = 1):
        _refuse_second_runtime()
        self.lib = load()
        h = C.c_void_p()
        rc = self.lib.pdhg_mlp_create(C.c_uint64(seed), C.byref(h))
        if rc != 0:
            raise PdhgError(rc, self.lib.pdhg_last_error().decode())
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise PdhgError(rc, self.lib.pdhg_last_error().decode())

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.pdhg_mlp_destroy(h)
        self.h = None

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == MLP_NPARAMS
        self._check(self.lib.pdhg_mlp_set_params(self.h, _fp(a)))

    def get_params(self):
        a = np.zeros(MLP_NPARAMS, dtype=np.float32)
        self._check(self.lib.pdhg_mlp_get_params(self.h, _fp(a)))
        return a

    def forward_noalloc(self, features_dev, n: int, logits_dev, stream=None):
        """pdhg_mlp_forward_noalloc on device pointers (enqueued, not waited for)."""
        self._check(self.lib.pdhg_mlp_forward_noalloc(self.h, features_dev, int(n), logits_dev, stream))

    def forward(self, features):
        f = np.ascontiguousarray(features, dtype=np.float32).reshape(-1, MLP_FEATURES)
        out = np.zeros(f.shape[0], dtype=np.float32)
        self._check(self.lib.pdhg_mlp_forward(self.h, _fp(f), f.shape[0], _fp(out)))
        return out

    def gradient(self, features, labels, pos_weight):
        f = np.ascontiguousarray(features, dtype=np.float32).reshape(-1, MLP_FEATURES)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        g = np.zeros(MLP_NPARAMS, dtype=np.float32)
        loss = C.c_double()
        self._check(self.lib.pdhg_mlp_gradient(self.h, _fp(f), _fp(y), f.shape[0], float(pos_weight), _fp(g),
                                               C.byref(loss)))
        return g, loss.value

    def train(self, features, labels, **kw):
        t = TrainParams()
        self.lib.pdhg_default_train_params(C.byref(t))
        for k, v in kw.items():
            setattr(t, k, v)
        f = np.ascontiguousarray(features, dtype=np.float32).reshape(-1, MLP_FEATURES)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        r = TrainReport()
        self._check(self.lib.pdhg_mlp_train(self.h, _fp(f), _fp(y), f.shape[0], C.byref(t), C.byref(r)))
        return r

"""ctypes binding of libusbs.so (include/usbs.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: if the shared library is missing or the GPU is absent, the calls
raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libusbs.so")

USBS_OK = 0
USBS_NOT_CONVERGED = 1
USBS_E_INVALID, USBS_E_NOMEM, USBS_E_DEVICE, USBS_E_NUMERIC, USBS_E_STATE = -1, -2, -3, -4, -5
ERRORS = {-1: "USBS_E_INVALID", -2: "USBS_E_NOMEM", -3: "USBS_E_DEVICE", -4: "USBS_E_NUMERIC",
          -5: "USBS_E_STATE"}
PREC = {"f64": 0, "f32": 1, "bf16": 2}
UNITS = {"scaled": 0, "original": 1}

# every symbol that include/usbs.h declares
EXPORTS = [
    "usbs_default_params", "usbs_create", "usbs_solve", "usbs_warm_start", "usbs_free", "usbs_last_error",
    "usbs_op_apply", "usbs_op_eigs", "usbs_op_lowrank_A", "usbs_op_sketch_update", "usbs_op_qp_data",
    "usbs_op_ipm", "usbs_op_nystrom", "usbs_step_iterate", "usbs_get_scaling", "usbs_profile",
    "usbs_footprint_bytes", "usbs_server_create", "usbs_server_submit", "usbs_server_wait",
    "usbs_server_get_stats", "usbs_server_last_error", "usbs_server_free", "usbs_round_maxcut",
    "usbs_get_tuning", "usbs_solve_packed", "usbs_packed_profile", "usbs_get_primal",
    "usbs_get_dual", "usbs_sketch_update_noalloc", "usbs_get_test_matrix",
]
PACK_PHASES = ["spmm", "tn", "nn", "ritz", "ipm", "constraints", "small", "shift", "all"]
PROF = {"spmm": 0, "reorth": 1, "ritz": 2, "ipm": 3, "update": 4}


class UsbsProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
        ("m", ctypes.c_int64), ("n_triplets", ctypes.c_int64), ("a_row", ctypes.c_void_p),
        ("a_i", ctypes.c_void_p), ("a_j", ctypes.c_void_p), ("a_v", ctypes.c_void_p), ("b", ctypes.c_void_p),
        ("is_ineq", ctypes.c_void_p), ("trace", ctypes.c_double), ("psi", ctypes.c_void_p),
    ]


class UsbsParams(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double), ("rho", ctypes.c_double), ("beta", ctypes.c_double),
        ("k_c", ctypes.c_int32), ("k_p", ctypes.c_int32), ("r", ctypes.c_int32),
        ("eps_gap", ctypes.c_double), ("eps_infeas", ctypes.c_double), ("units", ctypes.c_int32),
        ("max_iters", ctypes.c_int32), ("time_limit", ctypes.c_double), ("lanczos_steps", ctypes.c_int32),
        ("lanczos_max_restarts", ctypes.c_int32), ("lanczos_tol", ctypes.c_double),
        ("lanczos_tol_final", ctypes.c_double),
        ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64), ("stream", ctypes.c_void_p),
        ("verbose", ctypes.c_int32), ("autotune", ctypes.c_int32), ("lanczos_tol_rest", ctypes.c_double),
        ("psi_seed", ctypes.c_uint64), ("psi_from_seed", ctypes.c_int32),
    ]


class UsbsResult(ctypes.Structure):
    _fields_ = [
        ("primal_obj", ctypes.c_double), ("dual_bound", ctypes.c_double),
        ("primal_obj_scaled", ctypes.c_double), ("f_scaled", ctypes.c_double),
        ("rel_gap", ctypes.c_double), ("rel_infeas", ctypes.c_double), ("lambda_max", ctypes.c_double),
        ("sketch_primal_obj", ctypes.c_double), ("sketch_rel_infeas", ctypes.c_double),
        ("rel_gap_scaled", ctypes.c_double), ("rel_infeas_scaled", ctypes.c_double),
        ("rel_gap_original", ctypes.c_double), ("rel_infeas_original", ctypes.c_double),
        ("seconds", ctypes.c_double), ("lanczos_matvecs", ctypes.c_int64), ("iters", ctypes.c_int32),
        ("descents", ctypes.c_int32), ("ipm_iters", ctypes.c_int32), ("status", ctypes.c_int32),
        ("lanczos_unconverged", ctypes.c_int32), ("stall_recoveries", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class UsbsServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64), ("params", UsbsParams),
                ("mode", ctypes.c_int32), ("iters_per_launch", ctypes.c_int32), ("packed_max_n", ctypes.c_int64),
                ("large_slots", ctypes.c_int32)]


SERVE = {"streams": 0, "packed": 1}


class UsbsServedResult(ctypes.Structure):
    _fields_ = [
        ("base", UsbsResult), ("grown", UsbsResult),
        ("status_base", ctypes.c_int32), ("status_grown", ctypes.c_int32), ("has_grown", ctypes.c_int32),
        ("slot", ctypes.c_int32), ("footprint_bytes", ctypes.c_int64),
        ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_base_done", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class UsbsServerStats(ctypes.Structure):
    _fields_ = [
        ("queued", ctypes.c_int64), ("running", ctypes.c_int64), ("peak_running", ctypes.c_int64),
        ("completed", ctypes.c_int64), ("budget_bytes", ctypes.c_int64), ("used_bytes", ctypes.c_int64),
        ("peak_used_bytes", ctypes.c_int64), ("seconds", ctypes.c_double),
    ]


_LIB = None


def load_library(path: str | None = None):
    """Load libusbs.so (raises FileNotFoundError if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} not built: run __graft_entry__.build() or paper_2312_11801_amd/build.py")
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "usbs_default_params": (ctypes.c_int, [ctypes.POINTER(UsbsParams)]),
        "usbs_create": (ctypes.c_int, [ctypes.POINTER(UsbsProblem), ctypes.POINTER(UsbsParams),
                                       ctypes.POINTER(vp)]),
        "usbs_solve": (ctypes.c_int, [vp, ctypes.POINTER(UsbsResult), vp, vp, vp]),
        "usbs_warm_start": (ctypes.c_int, [vp, ctypes.POINTER(UsbsProblem)]),
        "usbs_free": (None, [vp]),
        "usbs_last_error": (ctypes.c_char_p, [vp]),
        "usbs_op_apply": (ctypes.c_int, [vp, vp, vp, i32, vp, i32, i32]),
        "usbs_op_eigs": (ctypes.c_int, [vp, vp, i32, vp, vp, vp, vp, vp]),
        "usbs_op_lowrank_A": (ctypes.c_int, [vp, vp, i32, vp, vp]),
        "usbs_op_sketch_update": (ctypes.c_int, [vp, dbl, vp, i32, vp, vp]),
        "usbs_op_qp_data": (ctypes.c_int, [vp, vp, i32, vp, vp, vp, dbl, dbl, vp, vp, vp, vp, vp]),
        "usbs_op_ipm": (ctypes.c_int, [vp, i32, vp, vp, dbl, vp, dbl, vp, vp, vp]),
        "usbs_op_nystrom": (ctypes.c_int, [vp, vp, vp, vp]),
        "usbs_step_iterate": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp]),
        "usbs_get_scaling": (ctypes.c_int, [vp, vp, vp]),
        "usbs_profile": (ctypes.c_int, [vp, i32, i32, vp, vp]),
        "usbs_footprint_bytes": (ctypes.c_int64, [ctypes.POINTER(UsbsProblem), ctypes.POINTER(UsbsParams)]),
        "usbs_server_create": (ctypes.c_int, [ctypes.POINTER(UsbsServerConfig), ctypes.POINTER(vp)]),
        "usbs_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(UsbsProblem), ctypes.POINTER(UsbsProblem),
                                              ctypes.POINTER(i64)]),
        "usbs_server_wait": (ctypes.c_int, [vp, i64, ctypes.POINTER(UsbsServedResult)]),
        "usbs_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(UsbsServerStats)]),
        "usbs_server_last_error": (ctypes.c_char_p, [vp]),
        "usbs_server_free": (None, [vp]),
        "usbs_round_maxcut": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "usbs_get_tuning": (ctypes.c_int, [vp, vp]),
        "usbs_solve_packed": (ctypes.c_int, [vp, i32, i32, vp, ctypes.POINTER(UsbsResult), vp]),
        "usbs_packed_profile": (ctypes.c_int, [vp, i32, vp]),
        "usbs_get_primal": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "usbs_get_dual": (ctypes.c_int, [vp, vp]),
        "usbs_get_test_matrix": (ctypes.c_int, [vp, vp]),
        "usbs_sketch_update_noalloc": (ctypes.c_int, [i64, i32, i32, dbl, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


class UsbsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(a) -> int | None:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


@dataclass
class Params:
    alpha: float = 2.0
    rho: float = 0.01
    beta: float = 0.25
    k_c: int = 10
    k_p: int = 1
    r: int = 10
    eps_gap: float = 1e-3
    eps_infeas: float = 1e-3
    units: str = "scaled"
    max_iters: int = 1000
    time_limit: float = 0.0
    lanczos_steps: int = 8
    lanczos_max_restarts: int = 10
    lanczos_tol: float = 1e-4
    lanczos_tol_final: float = 1e-9
    precision: str = "f64"
    seed: int = 0
    verbose: int = 0
    autotune: int = 1
    lanczos_tol_rest: float = 0.0
    psi_seed: int = 0
    psi_from_seed: bool = False

    def to_c(self, stream: int | None) -> UsbsParams:
        p = UsbsParams()
        load_library().usbs_default_params(ctypes.byref(p))
        for f in ("alpha", "rho", "beta", "k_c", "k_p", "r", "eps_gap", "eps_infeas", "max_iters", "time_limit",
                  "lanczos_steps", "lanczos_max_restarts", "lanczos_tol", "lanczos_tol_final", "seed", "verbose",
                  "autotune", "lanczos_tol_rest", "psi_seed"):
            setattr(p, f, getattr(self, f))
        p.psi_from_seed = int(bool(self.psi_from_seed))
        p.units = UNITS[self.units]
        p.precision = PREC[self.precision]
        p.stream = stream
        return p


class _ProblemArrays:
    """Holds contiguous host copies so that the pointers stay valid during the call."""

    def __init__(self, prob, psi):
        self.rowptr = np.ascontiguousarray(prob.rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(prob.col, dtype=np.int32)
        self.val = np.ascontiguousarray(prob.val, dtype=np.float64)
        self.a_row = np.ascontiguousarray(prob.a_row, dtype=np.int32)
        self.a_i = np.ascontiguousarray(prob.a_i, dtype=np.int32)
        self.a_j = np.ascontiguousarray(prob.a_j, dtype=np.int32)
        self.a_v = np.ascontiguousarray(prob.a_v, dtype=np.float64)
        self.b = np.ascontiguousarray(prob.b, dtype=np.float64)
        self.ineq = np.ascontiguousarray(prob.is_ineq, dtype=np.uint8)
        self.psi = None if psi is None else np.ascontiguousarray(psi, dtype=np.float32)
        self.c = UsbsProblem(
            n=prob.n, rowptr=self.rowptr.ctypes.data, col=self.col.ctypes.data, val=self.val.ctypes.data,
            m=prob.m, n_triplets=self.a_row.size, a_row=self.a_row.ctypes.data, a_i=self.a_i.ctypes.data,
            a_j=self.a_j.ctypes.data, a_v=self.a_v.ctypes.data, b=self.b.ctypes.data,
            is_ineq=self.ineq.ctypes.data, trace=float(prob.trace),
            psi=None if self.psi is None else self.psi.ctypes.data)


def current_stream() -> int | None:
    import torch
    return torch.cuda.current_stream().cuda_stream


class Solver:
    """One USBS instance on the current GPU (usbs_create ... usbs_free)."""

    def __init__(self, prob, params: Params | None = None, psi=None, stream: int | None = None):
        self.lib = load_library()
        self.params = params or Params()
        self.n, self.m = prob.n, prob.m
        self.r = self.params.r if (psi is not None or self.params.psi_from_seed) else 0
        arrs = _ProblemArrays(prob, psi)
        self._cp = self.params.to_c(stream)
        h = ctypes.c_void_p()
        rc = self.lib.usbs_create(ctypes.byref(arrs.c), ctypes.byref(self._cp), ctypes.byref(h))
        self.h = h
        if rc != USBS_OK:
            msg = self.lib.usbs_last_error(h).decode()
            self.lib.usbs_free(h)
            self.h = None
            raise UsbsError(rc, msg)

    def _check(self, rc: int, allow_nc: bool = False) -> int:
        if rc == USBS_OK or (allow_nc and rc == USBS_NOT_CONVERGED):
            return rc
        raise UsbsError(rc, self.lib.usbs_last_error(self.h).decode())

    def solve(self, want_y: bool = True, want_factors: bool = True) -> dict:
        res = UsbsResult()
        y = np.zeros(self.m) if want_y else None
        U = np.zeros((self.n, self.r)) if (want_factors and self.r) else None
        lam = np.zeros(self.r) if (want_factors and self.r) else None
        rc = self.lib.usbs_solve(self.h, ctypes.byref(res), _ptr(y), _ptr(U), _ptr(lam))
        self._check(rc, allow_nc=True)
        out = res.as_dict()
        out.update({"y": y, "U": U, "lam": lam, "converged": rc == USBS_OK})
        return out

    def warm_start(self, grown, psi=None) -> None:
        arrs = _ProblemArrays(grown, psi)
        self._check(self.lib.usbs_warm_start(self.h, ctypes.byref(arrs.c)))
        self.n, self.m = grown.n, grown.m

    def test_matrix(self) -> np.ndarray:
        """The handle's test matrix Psi (n x r, float32)."""
        psi = np.zeros((self.n, self.r), dtype=np.float32)
        self._check(self.lib.usbs_get_test_matrix(self.h, _ptr(psi)))
        return psi

    def round_maxcut(self) -> dict:
        """Best of the r cuts sign(U[:, c]) of the current sketch (App. E.1)."""
        x = np.zeros(self.n, dtype=np.int8)
        cut = ctypes.c_double()
        colm = ctypes.c_int32()
        cuts = np.zeros(max(self.r, 1))
        self._check(self.lib.usbs_round_maxcut(self.h, _ptr(x), ctypes.byref(cut), ctypes.byref(colm), _ptr(cuts)))
        return {"cut": cut.value, "x": x, "column": colm.value, "cuts": cuts[:self.r]}

    def tuning(self) -> dict:
        t = np.zeros(5, dtype=np.int32)
        self._check(self.lib.usbs_get_tuning(self.h, _ptr(t)))
        return dict(zip(("spmm8", "spmm16", "nn_cap", "red_cap", "red_unr"), t.tolist()))

    def scaling(self) -> tuple[float, float]:
        s, t = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.usbs_get_scaling(self.h, ctypes.byref(s), ctypes.byref(t)))
        return s.value, t.value

    # ---- step-level entry points (device tensors) ----
    def op_apply(self, y_dev, X_dev, Y_dev) -> None:
        nb = X_dev.shape[1]
        self._check(self.lib.usbs_op_apply(self.h, _ptr(y_dev), _ptr(X_dev), X_dev.stride(0), _ptr(Y_dev),
                                           Y_dev.stride(0), nb))

    def op_eigs(self, y_dev, k: int, start_dev=None, U_dev=None):
        w = np.zeros(k)
        res = np.zeros(k)
        cyc = ctypes.c_int32()
        self._check(self.lib.usbs_op_eigs(self.h, _ptr(y_dev), k, _ptr(start_dev), _ptr(w), _ptr(U_dev),
                                          _ptr(res), ctypes.byref(cyc)))
        return w, res, cyc.value

    def op_lowrank_A(self, W_dev, lam, out_dev) -> None:
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        self._check(self.lib.usbs_op_lowrank_A(self.h, _ptr(W_dev), W_dev.shape[1], _ptr(lam), _ptr(out_dev)))

    def op_sketch_update(self, g: float, W_dev, lam, P_dev) -> None:
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        self._check(self.lib.usbs_op_sketch_update(self.h, float(g), _ptr(W_dev), W_dev.shape[1], _ptr(lam),
                                                   _ptr(P_dev)))

    def op_qp_data(self, V_dev, y_dev, w_dev, zbar_dev, tau: float, cbar: float) -> dict:
        k = V_dev.shape[1]
        d = k * (k + 1) // 2
        Q11, q12, h1 = np.zeros((d, d)), np.zeros(d), np.zeros(d)
        q22, h2 = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.usbs_op_qp_data(self.h, _ptr(V_dev), k, _ptr(y_dev), _ptr(w_dev), _ptr(zbar_dev),
                                             float(tau), float(cbar), _ptr(Q11), _ptr(q12), ctypes.byref(q22),
                                             _ptr(h1), ctypes.byref(h2)))
        return {"Q11": Q11, "q12": q12, "q22": q22.value, "h1": h1, "h2": h2.value}

    def op_ipm(self, k: int, Q11, q12, q22, h1, h2):
        S = np.zeros((k, k))
        eta = ctypes.c_double()
        it = ctypes.c_int32()
        Q11 = np.ascontiguousarray(Q11, dtype=np.float64)
        q12 = np.ascontiguousarray(q12, dtype=np.float64)
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        self._check(self.lib.usbs_op_ipm(self.h, k, _ptr(Q11), _ptr(q12), float(q22), _ptr(h1), float(h2),
                                         _ptr(S), ctypes.byref(eta), ctypes.byref(it)))
        return S, eta.value, it.value

    def op_nystrom(self, P_dev, U_dev):
        lam = np.zeros(P_dev.shape[1])
        self._check(self.lib.usbs_op_nystrom(self.h, _ptr(P_dev), _ptr(U_dev), _ptr(lam)))
        return lam

    def step_iterate(self, t: int, k: int, light: bool = False):
        """t iterations of Alg. 1; returns the scalars and (unless light) y, V, zbar, P."""
        keys = ["f", "tau", "cbar", "primal", "rel_gap", "rel_infeas", "lambda1", "descents"]
        scal = np.zeros(8)
        if light:
            self._check(self.lib.usbs_step_iterate(self.h, t, None, None, None, None, _ptr(scal)))
            return dict(zip(keys, scal))
        y = np.zeros(self.m)
        V = np.zeros((self.n, 16))
        zbar = np.zeros(self.m)
        P = np.zeros((self.n, max(self.r, 1)))
        self._check(self.lib.usbs_step_iterate(self.h, t, _ptr(y), _ptr(V), _ptr(zbar),
                                               _ptr(P) if self.r else None, _ptr(scal)))
        return {"y": y, "V": V[:, :k], "zbar": zbar, "P": P[:, :self.r], **dict(zip(keys, scal))}

    def primal(self) -> dict:
        """X_{t+1} of the last iteration (scaled units): A X_{t+1}, <C_s, X_{t+1}>, the
        bundle V_t, the QP solution (S, eta) and g = alpha eta / tau_t."""
        k = self.params.k_c + self.params.k_p
        ax = np.zeros(self.m)
        V = np.zeros((self.n, k))
        S = np.zeros((k, k))
        cx, eta, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.usbs_get_primal(self.h, _ptr(ax), ctypes.byref(cx), _ptr(V), _ptr(S),
                                             ctypes.byref(eta), ctypes.byref(g)))
        return {"AX": ax, "cX": cx.value, "V": V, "S": S, "eta": eta.value, "g": g.value}

    def profile(self, category: str | None, reset: bool = True):
        """Return (ms, launches) timed so far for the current category and start timing
        `category` (None stops timing)."""
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        cat = -1 if category is None else PROF[category]
        self._check(self.lib.usbs_profile(self.h, cat, int(reset), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def packed_profile(self, reset: bool = False) -> dict:
        """Device milliseconds of this handle's packed launches per phase."""
        ms = np.zeros(len(PACK_PHASES))
        self._check(self.lib.usbs_packed_profile(self.h, int(reset), _ptr(ms)))
        return dict(zip(PACK_PHASES, ms.tolist()))

    def free(self) -> None:
        if self.h is not None:
            self.lib.usbs_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def solve_packed(solvers: list, iters_per_launch: int = 8, stream: int | None = None) -> list:
    """Solve several instances together in packed launches (usbs_solve_packed): one
    workgroup per instance, up to iters_per_launch iterations per launch.  Returns one
    result dict per solver (as Solver.solve, with y in original units)."""
    lib = load_library()
    cnt = len(solvers)
    hs = (ctypes.c_void_p * cnt)(*[s.h.value for s in solvers])
    res = (UsbsResult * cnt)()
    st = np.zeros(cnt, dtype=np.int32)
    rc = lib.usbs_solve_packed(hs, cnt, int(iters_per_launch), stream, res, _ptr(st))
    if rc < 0:
        raise UsbsError(rc, lib.usbs_last_error(solvers[0].h).decode())
    outs = []
    for q, s in enumerate(solvers):
        d = res[q].as_dict()
        y = np.zeros(s.m)
        s._check(lib.usbs_get_dual(s.h, _ptr(y)))
        d.update({"y": y, "converged": int(st[q]) == USBS_OK, "status_code": int(st[q])})
        outs.append(d)
    return outs


def sketch_update_noalloc(g: float, W_dev, lam, psi_dev, P_dev, stream: int | None = None) -> None:
    """usbs_sketch_update_noalloc: P <- g P + W diag(lam) (W^T Psi) on device tensors,
    without a handle and without device allocation (enqueued on `stream`)."""
    lib = load_library()
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    n, q = W_dev.shape
    r = P_dev.shape[1]
    rc = lib.usbs_sketch_update_noalloc(int(n), int(q), int(r), float(g), _ptr(W_dev), _ptr(lam), _ptr(psi_dev),
                                        _ptr(P_dev), stream)
    if rc != USBS_OK:
        raise UsbsError(rc, lib.usbs_last_error(None).decode())


def footprint_bytes(prob, params: Params | None = None, psi=None) -> int:
    """Device bytes usbs_create would allocate at most for this problem."""
    lib = load_library()
    arrs = _ProblemArrays(prob, psi)
    cp = (params or Params()).to_c(None)
    return int(lib.usbs_footprint_bytes(ctypes.byref(arrs.c), ctypes.byref(cp)))


class Server:
    """Request loop with continuous batching on the current GPU (usbs_server_*).

    submit() queues an instance (and optionally its grown version, warm-started from the
    first solve's resident state); wait() returns the results and the request's times
    (seconds since the server started): submit, admit, base solve done, done."""

    def __init__(self, slots: int = 4, params: Params | None = None, hbm_budget_bytes: int = 0,
                 mode: str = "streams", iters_per_launch: int = 8, packed_max_n: int = 0, large_slots: int = -1):
        self.lib = load_library()
        self.params = params or Params()
        cfg = UsbsServerConfig(slots=slots, hbm_budget_bytes=hbm_budget_bytes, params=self.params.to_c(None),
                               mode=SERVE[mode], iters_per_launch=iters_per_launch, packed_max_n=packed_max_n,
                               large_slots=large_slots)
        h = ctypes.c_void_p()
        rc = self.lib.usbs_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != 0:
            raise UsbsError(rc, "usbs_server_create failed")
        self.h = h

    def submit(self, prob, psi=None, grown=None, psi_grown=None) -> int:
        a = _ProblemArrays(prob, psi)
        g = None if grown is None else _ProblemArrays(grown, psi_grown)
        rid = ctypes.c_int64()
        rc = self.lib.usbs_server_submit(self.h, ctypes.byref(a.c), None if g is None else ctypes.byref(g.c),
                                         ctypes.byref(rid))
        if rc != 0:
            raise UsbsError(rc, self.lib.usbs_server_last_error(self.h).decode())
        return rid.value

    def wait(self, rid: int) -> dict:
        out = UsbsServedResult()
        rc = self.lib.usbs_server_wait(self.h, rid, ctypes.byref(out))
        if rc < 0:
            raise UsbsError(rc, self.lib.usbs_server_last_error(self.h).decode())
        d = {k: getattr(out, k) for k, _ in UsbsServedResult._fields_ if k not in ("base", "grown")}
        d["base"] = out.base.as_dict()
        d["grown"] = out.grown.as_dict() if out.has_grown else None
        return d

    def stats(self) -> dict:
        st = UsbsServerStats()
        self.lib.usbs_server_get_stats(self.h, ctypes.byref(st))
        return {k: getattr(st, k) for k, _ in UsbsServerStats._fields_}

    def close(self) -> None:
        if self.h is not None:
            self.lib.usbs_server_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

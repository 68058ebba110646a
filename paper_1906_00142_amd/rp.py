"""ctypes binding of librpfit with the C ABI's entry-point names.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device arrays are torch tensors on the context's device; host arrays
are NumPy.  The library must have been built in-tree
(``python -m paper_1906_00142_amd.build``); importing the binding works
without it, but every call raises ``RuntimeError`` when it is missing -- there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpfit.so")

RP_OK, RP_EINVAL, RP_ESHAPE, RP_EHIP, RP_ENOMEM, RP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RP_FIT_OK, RP_FIT_RANK_DEFICIENT, RP_FIT_UNDERDETERMINED = 0, 1, 2
RP_FIT_NONFINITE_INPUT, RP_FIT_Q_NONPOSITIVE, RP_FIT_NOT_CONVERGED = 3, 4, 5
RP_FP64, RP_MIXED_FP32, RP_MIXED_BF16, RP_AUTO = 0, 1, 2, 3
RP_TEMPLATE_SINGLE, RP_TEMPLATE_MWPCWP, RP_TEMPLATE_OCCUPANCY = 0, 1, 2
RP_SELECT_MIN, RP_SELECT_MAX = 1, -1
RP_NUM_METRICS, RP_HW_COUNT = 16, 17
RP_LOSS_FWD, RP_LOSS_BWD = 0, 1
RP_GRAM_AUTO, RP_GRAM_MFMA, RP_GRAM_MOMENTS = 0, 1, 2

PRECISIONS = {"fp64": RP_FP64, "fp32": RP_MIXED_FP32, "bf16": RP_MIXED_BF16, "auto": RP_AUTO}
RP_TUNE_COLS = 9
TUNE_COLUMNS = ["nvars", "deg_num", "deg_den", "precision", "gram_algo",
                "us_fp64_moments", "us_fp64_mfma", "us_fp32", "us_bf16"]

EXPORTS = (
    "rp_last_error", "rp_monomials", "rp_monomials_box", "rp_num_coefs", "rp_candidates_2d", "rp_create",
    "rp_destroy", "rp_plan_create", "rp_plan_destroy", "rp_plan_offsets",
    "rp_assemble_design", "rp_gram", "rp_gram_jacobian", "rp_fit_rational", "rp_refine_rational",
    "rp_loss_grad",
    "rp_program_create", "rp_program_destroy", "rp_eval_program_argmin", "rp_eval_program_select",
    "rp_plan_tune", "rp_plan_tuning", "rp_plan_set_tuning", "rp_fit_graph_create",
    "rp_graph_launch", "rp_graph_destroy",
    "rp_program_source", "rp_program_specialize", "rp_spec_source", "rp_eval_spec_select",
    "rp_spec_destroy", "rp_fit_uniform_static", "rp_split_create", "rp_split_destroy",
    "rp_split_fit",
)


class RpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librpfit error {code}: {msg}")
        self.code = code


class FitOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_refine", C.c_int32), ("tol", C.c_double),
                ("check_q", C.c_int32), ("gram_algo", C.c_int32)]


class RefineOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("rtol", C.c_double), ("gram_algo", C.c_int32)]


class ProgramDesc(C.Structure):
    _fields_ = [("template_id", C.c_int32), ("num_programs", C.c_int32),
                ("num_metrics", C.c_int32), ("nvars", C.c_int32),
                ("deg_num", C.c_void_p), ("deg_den", C.c_void_p), ("coef_off", C.c_void_p),
                ("coef", C.c_void_p), ("hw", C.c_void_p), ("scale", C.c_void_p)]


_lock = threading.Lock()
_lib = None


def lib():
    """The loaded library; raises RuntimeError if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_1906_00142_amd.build` (no CPU fallback exists)")
            L = C.CDLL(LIB_PATH)
            vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
            L.rp_last_error.restype = C.c_char_p
            L.rp_monomials.argtypes = [C.c_int, C.c_int, vp, vp]
            L.rp_monomials_box.argtypes = [C.c_int, vp, vp, vp]
            L.rp_num_coefs.argtypes = [C.c_int, C.c_int, C.c_int, vp]
            L.rp_candidates_2d.argtypes = [C.c_int, C.c_int, vp, vp]
            L.rp_create.argtypes = [vp, C.c_int]
            L.rp_destroy.argtypes = [vp]
            L.rp_plan_create.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
            L.rp_plan_destroy.argtypes = [vp]
            L.rp_plan_offsets.argtypes = [vp, vp, vp, vp]
            L.rp_gram.argtypes = [vp, vp, i64, vp, C.c_int, C.c_int, vp, vp]
            L.rp_gram_jacobian.argtypes = [vp, vp, i64, vp, vp, C.c_int, vp, vp]
            L.rp_assemble_design.argtypes = [vp, vp, i64, vp, C.c_int, vp, vp, vp]
            L.rp_fit_rational.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
            L.rp_split_create.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp]
            L.rp_split_destroy.argtypes = [vp]
            L.rp_split_fit.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
            L.rp_fit_uniform_static.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, i64, vp,
                                                vp, vp, vp, vp, vp]
            L.rp_refine_rational.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
            L.rp_loss_grad.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, C.c_int, vp]
            L.rp_program_create.argtypes = [vp, vp, vp]
            L.rp_program_destroy.argtypes = [vp]
            L.rp_eval_program_argmin.argtypes = [vp, vp, C.c_int, vp, C.c_int, C.c_int, C.c_int,
                                                 vp, vp, vp, vp, vp]
            L.rp_program_source.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
            L.rp_program_specialize.argtypes = [vp, vp]
            L.rp_spec_source.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
            L.rp_eval_spec_select.argtypes = [vp, C.c_int, vp, C.c_int, vp, C.c_int, C.c_int,
                                              vp, vp, vp, vp, vp]
            L.rp_spec_destroy.argtypes = [vp]
            L.rp_eval_program_select.argtypes = [vp, C.c_int, vp, C.c_int, vp, C.c_int, vp, C.c_int,
                                                 C.c_int, C.c_int, vp, vp, vp, vp, vp]
            L.rp_plan_tune.argtypes = [vp, vp, i64, vp, vp]
            L.rp_plan_tuning.argtypes = [vp, vp, vp]
            L.rp_plan_set_tuning.argtypes = [vp, vp, C.c_int]
            L.rp_fit_graph_create.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
            L.rp_graph_launch.argtypes = [vp, vp]
            L.rp_graph_destroy.argtypes = [vp]
            _lib = L
    return _lib


def _check(rc):
    if rc != RP_OK:
        raise RpError(rc, lib().rp_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, dtype=None, name="tensor"):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# host tables
# ---------------------------------------------------------------------------

def rp_monomials_box(maxdeg) -> np.ndarray:
    """Exponents of the per-variable degree box (rp_monomials_box)."""
    md = np.ascontiguousarray(maxdeg, dtype=np.int32)
    cnt = C.c_int(0)
    _check(lib().rp_monomials_box(len(md), _np_ptr(md), None, C.byref(cnt)))
    out = np.zeros((cnt.value, len(md)), dtype=np.uint8)
    _check(lib().rp_monomials_box(len(md), _np_ptr(md), _np_ptr(out), C.byref(cnt)))
    return out


def rp_monomials(nvars: int, degree: int) -> np.ndarray:
    cnt = C.c_int(0)
    _check(lib().rp_monomials(nvars, degree, None, C.byref(cnt)))
    out = np.zeros((cnt.value, nvars), dtype=np.uint8)
    _check(lib().rp_monomials(nvars, degree, _np_ptr(out), C.byref(cnt)))
    return out


def rp_num_coefs(nvars: int, deg_num: int, deg_den: int) -> int:
    cnt = C.c_int(0)
    _check(lib().rp_num_coefs(nvars, deg_num, deg_den, C.byref(cnt)))
    return cnt.value


def rp_candidates_2d(max_prod: int = 1024, multiple: int = 64) -> np.ndarray:
    cnt = C.c_int(0)
    _check(lib().rp_candidates_2d(max_prod, multiple, None, C.byref(cnt)))
    out = np.zeros((cnt.value, 2), dtype=np.int32)
    _check(lib().rp_candidates_2d(max_prod, multiple, _np_ptr(out), C.byref(cnt)))
    return out


# ---------------------------------------------------------------------------
# context and plans
# ---------------------------------------------------------------------------

class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().rp_create(C.byref(h), device))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().rp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """rp_plan_create over host metadata of an uneven batch."""

    def __init__(self, ctx: Context, sample_off, nvars, deg_num, deg_den):
        self.ctx = ctx
        self.sample_off = np.ascontiguousarray(sample_off, dtype=np.int64)
        self.nvars = np.ascontiguousarray(nvars, dtype=np.int32)
        self.deg_num = np.ascontiguousarray(deg_num, dtype=np.int32)
        self.deg_den = np.ascontiguousarray(deg_den, dtype=np.int32)
        self.num_fits = len(self.nvars)
        h = C.c_void_p()
        _check(lib().rp_plan_create(ctx.handle, self.num_fits, _np_ptr(self.sample_off),
                                    _np_ptr(self.nvars), _np_ptr(self.deg_num),
                                    _np_ptr(self.deg_den), C.byref(h)))
        self.handle = h
        self.coef_off = np.zeros(self.num_fits + 1, dtype=np.int64)
        self.a_off = np.zeros(self.num_fits + 1, dtype=np.int64)
        self.gram_off = np.zeros(self.num_fits + 1, dtype=np.int64)
        _check(lib().rp_plan_offsets(h, _np_ptr(self.coef_off), _np_ptr(self.a_off),
                                     _np_ptr(self.gram_off)))

    @classmethod
    def for_batch(cls, ctx, batch):
        return cls(ctx, batch.sample_off, batch.nvars, batch.deg_num, batch.deg_den)

    @property
    def num_coefs(self) -> int:
        return int(self.coef_off[-1])

    def close(self):
        if self.handle:
            lib().rp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rp_assemble_design(plan: Plan, x, ld_x: int, y, precision: int, A, rhs, stream=None):
    import torch
    et = {RP_FP64: torch.float64, RP_MIXED_FP32: torch.float32, RP_MIXED_BF16: torch.bfloat16}[precision]
    _check(lib().rp_assemble_design(plan.handle, _dev_ptr(x, torch.float64, "x"), ld_x,
                                    _dev_ptr(y, torch.float64, "y"), precision,
                                    _dev_ptr(A, et, "A"), _dev_ptr(rhs, et, "rhs"),
                                    _stream_ptr(stream)))


def rp_gram(plan: Plan, x, ld_x: int, y, precision: int, gram, gram_algo: int = RP_GRAM_AUTO,
            stream=None):
    import torch
    _check(lib().rp_gram(plan.handle, _dev_ptr(x, torch.float64, "x"), ld_x,
                         _dev_ptr(y, torch.float64, "y"), precision, gram_algo,
                         _dev_ptr(gram, torch.float64, "gram"), _stream_ptr(stream)))


def rp_gram_jacobian(plan: Plan, x, ld_x: int, y, coef, gram, gram_algo: int = RP_GRAM_AUTO,
                     stream=None):
    import torch
    _check(lib().rp_gram_jacobian(plan.handle, _dev_ptr(x, torch.float64, "x"), ld_x,
                                  _dev_ptr(y, torch.float64, "y"),
                                  _dev_ptr(coef, torch.float64, "coef"), gram_algo,
                                  _dev_ptr(gram, torch.float64, "gram"), _stream_ptr(stream)))


def rp_fit_rational(plan: Plan, x, ld_x: int, y, coef, status, resid=None, iters=None,
                    precision: int = RP_FP64, max_refine: int = -1, tol: float = -1.0,
                    check_q: bool = True, gram_algo: int = RP_GRAM_AUTO, stream=None):
    import torch
    o = FitOpts(precision, max_refine, tol, 1 if check_q else 0, gram_algo)
    _check(lib().rp_fit_rational(plan.handle, _dev_ptr(x, torch.float64, "x"), ld_x,
                                 _dev_ptr(y, torch.float64, "y"), C.byref(o),
                                 _dev_ptr(coef, torch.float64, "coef"),
                                 _dev_ptr(status, torch.int32, "status"),
                                 _dev_ptr(resid, torch.float64, "resid"),
                                 _dev_ptr(iters, torch.int32, "iters"), _stream_ptr(stream)))


def rp_fit_uniform_static(ctx: "Context", num_fits: int, num_samples: int, nvars: int,
                          degree: int, x, ld_x: int, y, coef, status, resid, iters=None,
                          stream=None):
    """The FP64 fit of a uniform batch with no plan and no allocation (its
    scratch lives in the library's per-device array)."""
    import torch
    _check(lib().rp_fit_uniform_static(ctx.handle, num_fits, num_samples, nvars, degree,
                                       _dev_ptr(x, torch.float64, "x"), ld_x,
                                       _dev_ptr(y, torch.float64, "y"),
                                       _dev_ptr(coef, torch.float64, "coef"),
                                       _dev_ptr(status, torch.int32, "status"),
                                       _dev_ptr(resid, torch.float64, "resid"),
                                       _dev_ptr(iters, torch.int32, "iters"), _stream_ptr(stream)))


class Split:
    """rp_split_create / rp_split_fit: decision nodes fitted from the samples."""

    def __init__(self, ctx: "Context", num_nodes: int, num_samples: int, nvars: int, degree: int,
                 split_var: int, n_min: int):
        h = C.c_void_p()
        _check(lib().rp_split_create(ctx.handle, num_nodes, num_samples, nvars, degree, split_var,
                                     n_min, C.byref(h)))
        self.handle = h
        self.num_nodes, self.num_samples = num_nodes, num_samples
        self.num_coefs = rp_num_coefs(nvars, degree, degree)

    def fit(self, x, ld_x: int, y, stream=None):
        """Returns device tensors (k, theta, coef_l, coef_r, status_l, status_r, obj)."""
        import torch
        dev = x.device
        F, nc = self.num_nodes, self.num_coefs
        k = torch.empty(F, dtype=torch.int64, device=dev)
        theta = torch.empty(F, dtype=torch.float64, device=dev)
        cl = torch.empty(F * nc, dtype=torch.float64, device=dev)
        cr = torch.empty(F * nc, dtype=torch.float64, device=dev)
        sl = torch.empty(F, dtype=torch.int32, device=dev)
        sr = torch.empty(F, dtype=torch.int32, device=dev)
        obj = torch.empty(F, dtype=torch.float64, device=dev)
        _check(lib().rp_split_fit(self.handle, _dev_ptr(x, torch.float64, "x"), ld_x,
                                  _dev_ptr(y, torch.float64, "y"), _dev_ptr(k, torch.int64, "k"),
                                  _dev_ptr(theta, torch.float64, "theta"),
                                  _dev_ptr(cl, torch.float64, "coef_l"),
                                  _dev_ptr(cr, torch.float64, "coef_r"),
                                  _dev_ptr(sl, torch.int32, "status_l"),
                                  _dev_ptr(sr, torch.int32, "status_r"),
                                  _dev_ptr(obj, torch.float64, "obj"), _stream_ptr(stream)))
        return k, theta, cl, cr, sl, sr, obj

    def close(self):
        if self.handle:
            lib().rp_split_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rp_refine_rational(plan: Plan, x, ld_x: int, y, coef, status, loss, max_iter: int = 20,
                       rtol: float = 1e-14, gram_algo: int = RP_GRAM_AUTO, stream=None):
    import torch
    o = RefineOpts(max_iter, rtol, gram_algo)
    _check(lib().rp_refine_rational(plan.handle, _dev_ptr(x, torch.float64, "x"), ld_x,
                                    _dev_ptr(y, torch.float64, "y"), C.byref(o),
                                    _dev_ptr(coef, torch.float64, "coef"),
                                    _dev_ptr(status, torch.int32, "status"),
                                    _dev_ptr(loss, torch.float64, "loss"), _stream_ptr(stream)))


def rp_loss_grad(plan: Plan, x, ld_x: int, y, coef, loss, dloss=None, dcoef=None,
                 mode: int = RP_LOSS_FWD, stream=None):
    import torch
    _check(lib().rp_loss_grad(plan.handle, _dev_ptr(x, torch.float64, "x"), ld_x,
                              _dev_ptr(y, torch.float64, "y"),
                              _dev_ptr(coef, torch.float32, "coef"),
                              _dev_ptr(loss, torch.float32, "loss"),
                              _dev_ptr(dloss, torch.float32, "dloss"),
                              _dev_ptr(dcoef, torch.float32, "dcoef"), mode, _stream_ptr(stream)))


def rp_plan_tune(plan: Plan, x, ld_x: int, y, stream=None):
    import torch
    _check(lib().rp_plan_tune(plan.handle, _dev_ptr(x, torch.float64, "x"), ld_x,
                              _dev_ptr(y, torch.float64, "y"), _stream_ptr(stream)))


def rp_plan_tuning(plan: Plan):
    """Rows of TUNE_COLUMNS, one per shape bucket: the shape, the chosen form
    of RP_AUTO and FP64 Gram formation, and the measured microseconds of the
    four candidate forms (-1: not measured)."""
    cnt = C.c_int(0)
    _check(lib().rp_plan_tuning(plan.handle, None, C.byref(cnt)))
    t = np.zeros((cnt.value, RP_TUNE_COLS), dtype=np.int32)
    _check(lib().rp_plan_tuning(plan.handle, _np_ptr(t), C.byref(cnt)))
    return t


def rp_plan_set_tuning(plan: Plan, table):
    t = np.ascontiguousarray(table, dtype=np.int32).reshape(-1, RP_TUNE_COLS)
    _check(lib().rp_plan_set_tuning(plan.handle, _np_ptr(t), len(t)))


def save_tuning(plan: Plan, path: str):
    """Persist the plan's tuning table as JSON."""
    import json
    rows = rp_plan_tuning(plan).tolist()
    with open(path, "w") as fh:
        json.dump({"columns": TUNE_COLUMNS, "rows": rows}, fh, indent=1)


def load_tuning(plan: Plan, path: str):
    import json
    with open(path) as fh:
        d = json.load(fh)
    if d.get("columns") != TUNE_COLUMNS:
        raise ValueError(f"{path}: tuning table columns {d.get('columns')} != {TUNE_COLUMNS}")
    rp_plan_set_tuning(plan, np.array(d["rows"], dtype=np.int32).reshape(-1, RP_TUNE_COLS))


class FitGraph:
    """rp_fit_graph_create / rp_graph_launch: the whole fit as one graph launch."""

    def __init__(self, dbatch, coef, status, resid=None, iters=None, precision: int = RP_FP64,
                 max_refine: int = -1, tol: float = -1.0, check_q: bool = True,
                 gram_algo: int = RP_GRAM_AUTO):
        import torch
        o = FitOpts(precision, max_refine, tol, 1 if check_q else 0, gram_algo)
        self._keep = (dbatch, coef, status, resid, iters)
        h = C.c_void_p()
        _check(lib().rp_fit_graph_create(dbatch.plan.handle, _dev_ptr(dbatch.x, torch.float64, "x"),
                                         dbatch.ld_x, _dev_ptr(dbatch.y, torch.float64, "y"),
                                         C.byref(o), _dev_ptr(coef, torch.float64, "coef"),
                                         _dev_ptr(status, torch.int32, "status"),
                                         _dev_ptr(resid, torch.float64, "resid"),
                                         _dev_ptr(iters, torch.int32, "iters"), C.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib().rp_graph_launch(self.handle, _stream_ptr(stream)))

    def close(self):
        if self.handle:
            lib().rp_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# rational programs
# ---------------------------------------------------------------------------

class Program:
    """rp_program_create; keeps references to the device coefficient/hw tensors."""

    def __init__(self, ctx: Context, template_id: int, nvars: int, deg_num, deg_den, coef_off,
                 coef, scale, hw=None, num_programs: int = 1):
        import torch
        self.ctx = ctx
        self.deg_num = np.ascontiguousarray(deg_num, dtype=np.int32)
        self.deg_den = np.ascontiguousarray(deg_den, dtype=np.int32)
        self.coef_off = np.ascontiguousarray(coef_off, dtype=np.int64)
        self.scale = np.ascontiguousarray(scale, dtype=np.float64)
        self.coef = coef
        self.hw = hw
        self.nvars = int(nvars)
        d = ProgramDesc(template_id, num_programs, len(self.deg_num) // max(num_programs, 1), nvars,
                        _np_ptr(self.deg_num).value, _np_ptr(self.deg_den).value,
                        _np_ptr(self.coef_off).value,
                        _dev_ptr(coef, torch.float64, "coef").value,
                        None if hw is None else _dev_ptr(hw, torch.float64, "hw").value,
                        _np_ptr(self.scale).value)
        h = C.c_void_p()
        _check(lib().rp_program_create(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h
        self.num_programs = num_programs

    def close(self):
        if self.handle:
            lib().rp_program_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rp_eval_program_argmin(prog: Program, n_grid, cand, argmin, best, second, values=None,
                           precision: int = RP_FP64, stream=None):
    import torch
    num_cand, cand_dim = (cand.shape[0], cand.shape[1]) if cand.dim() == 2 else (cand.shape[0], 1)
    _check(lib().rp_eval_program_argmin(prog.handle, _dev_ptr(n_grid, torch.float64, "n_grid"),
                                        n_grid.numel(), _dev_ptr(cand, torch.int32, "cand"),
                                        num_cand, cand_dim, precision,
                                        _dev_ptr(argmin, torch.int32, "argmin"),
                                        _dev_ptr(best, torch.float64, "best"),
                                        _dev_ptr(second, torch.float64, "second"),
                                        _dev_ptr(values, torch.float64, "values"),
                                        _stream_ptr(stream)))


def rp_eval_program_select(prog: Program, n_grid, cand, choice, best, second, sense: int = RP_SELECT_MIN,
                           tie_prog: Program | None = None, tie_sense: int = RP_SELECT_MAX,
                           values=None, precision: int = RP_FP64, stream=None):
    import torch
    num_cand, cand_dim = (cand.shape[0], cand.shape[1]) if cand.dim() == 2 else (cand.shape[0], 1)
    _check(lib().rp_eval_program_select(prog.handle, sense, None if tie_prog is None else tie_prog.handle,
                                        tie_sense, _dev_ptr(n_grid, torch.float64, "n_grid"),
                                        n_grid.numel(), _dev_ptr(cand, torch.int32, "cand"),
                                        num_cand, cand_dim, precision,
                                        _dev_ptr(choice, torch.int32, "choice"),
                                        _dev_ptr(best, torch.float64, "best"),
                                        _dev_ptr(second, torch.float64, "second"),
                                        _dev_ptr(values, torch.float64, "values"),
                                        _stream_ptr(stream)))


# ---------------------------------------------------------------------------
# conveniences over the entry points
# ---------------------------------------------------------------------------

class DeviceBatch:
    """A FitBatch's samples resident on the device, with its plan."""

    def __init__(self, ctx: Context, batch, device=None):
        import torch
        dev = torch.device("cuda", ctx.device) if device is None else device
        self.batch = batch
        self.plan = Plan.for_batch(ctx, batch)
        self.x = torch.from_numpy(np.ascontiguousarray(batch.x)).to(dev)
        self.y = torch.from_numpy(np.ascontiguousarray(batch.y)).to(dev)
        self.ld_x = int(batch.x.shape[1])
        self.device = dev
        self.num_fits = batch.num_fits

    def alloc_fit_outputs(self):
        import torch
        coef = torch.zeros(self.plan.num_coefs, dtype=torch.float64, device=self.device)
        status = torch.full((self.num_fits,), -1, dtype=torch.int32, device=self.device)
        resid = torch.zeros(self.num_fits, dtype=torch.float64, device=self.device)
        iters = torch.zeros(self.num_fits, dtype=torch.int32, device=self.device)
        return coef, status, resid, iters

    def fit(self, precision=RP_FP64, max_refine=-1, tol=-1.0, check_q=True, out=None,
            gram_algo=RP_GRAM_AUTO, stream=None):
        coef, status, resid, iters = self.alloc_fit_outputs() if out is None else out
        rp_fit_rational(self.plan, self.x, self.ld_x, self.y, coef, status, resid, iters,
                        precision=precision, max_refine=max_refine, tol=tol, check_q=check_q,
                        gram_algo=gram_algo, stream=stream)
        return coef, status, resid, iters


def rational_loss_function():
    """torch.autograd.Function over rp_loss_grad: loss[f] = sum (N/Q - y)^2."""
    import torch

    class RationalLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, coef, dbatch):
            loss = torch.empty(dbatch.num_fits, dtype=torch.float32, device=coef.device)
            rp_loss_grad(dbatch.plan, dbatch.x, dbatch.ld_x, dbatch.y, coef.contiguous(), loss,
                         mode=RP_LOSS_FWD)
            ctx.save_for_backward(coef)
            ctx.dbatch = dbatch
            return loss

        @staticmethod
        def backward(ctx, dloss):
            (coef,) = ctx.saved_tensors
            db = ctx.dbatch
            loss = torch.empty(db.num_fits, dtype=torch.float32, device=coef.device)
            dcoef = torch.empty_like(coef)
            rp_loss_grad(db.plan, db.x, db.ld_x, db.y, coef.contiguous(), loss,
                         dloss.contiguous().to(torch.float32), dcoef, mode=RP_LOSS_BWD)
            return dcoef, None

    return RationalLoss


def planted_coefs(pl) -> np.ndarray:
    """A workload's planted function as a coefficient vector in the library's
    monomial order (matched by exponent tuple)."""
    num, den = pl.coef_by_tuple()
    En = rp_monomials(pl.nvars, pl.deg_num)
    Ed = rp_monomials(pl.nvars, pl.deg_den)
    return np.array([num[tuple(int(t) for t in e)] for e in En]
                    + [den[tuple(int(t) for t in e)] for e in Ed[1:]])


def program_source(template_id: int, nvars: int, deg_num, deg_den, coef_off, coef, scale,
                   hw=None, num_programs: int = 1) -> str:
    """rp_program_source: the specialised evaluator's HIP source for programs
    given in host arrays (no device needed)."""
    deg_num = np.ascontiguousarray(deg_num, dtype=np.int32)
    deg_den = np.ascontiguousarray(deg_den, dtype=np.int32)
    coef_off = np.ascontiguousarray(coef_off, dtype=np.int64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    scale = np.ascontiguousarray(scale, dtype=np.float64)
    hw = None if hw is None else np.ascontiguousarray(hw, dtype=np.float64)
    d = ProgramDesc(template_id, num_programs, len(deg_num) // max(num_programs, 1), nvars,
                    _np_ptr(deg_num).value, _np_ptr(deg_den).value, _np_ptr(coef_off).value,
                    _np_ptr(coef).value, None if hw is None else _np_ptr(hw).value,
                    _np_ptr(scale).value)
    n = C.c_size_t(0)
    _check(lib().rp_program_source(C.byref(d), None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib().rp_program_source(C.byref(d), buf, C.byref(n)))
    return buf.value.decode()


class Spec:
    """rp_program_specialize: the run-time compiled evaluator of a Program."""

    def __init__(self, prog: Program):
        h = C.c_void_p()
        _check(lib().rp_program_specialize(prog.handle, C.byref(h)))
        self.handle = h
        self.num_programs = prog.num_programs

    def source(self) -> str:
        n = C.c_size_t(0)
        _check(lib().rp_spec_source(self.handle, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().rp_spec_source(self.handle, buf, C.byref(n)))
        return buf.value.decode()

    def close(self):
        if self.handle:
            lib().rp_spec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rp_eval_spec_select(spec: Spec, n_grid, cand, choice, best, second, sense: int = RP_SELECT_MIN,
                        values=None, stream=None):
    import torch
    num_cand, cand_dim = (cand.shape[0], cand.shape[1]) if cand.dim() == 2 else (cand.shape[0], 1)
    _check(lib().rp_eval_spec_select(spec.handle, sense, _dev_ptr(n_grid, torch.float64, "n_grid"),
                                     n_grid.numel(), _dev_ptr(cand, torch.int32, "cand"), num_cand,
                                     cand_dim, _dev_ptr(choice, torch.int32, "choice"),
                                     _dev_ptr(best, torch.float64, "best"),
                                     _dev_ptr(second, torch.float64, "second"),
                                     _dev_ptr(values, torch.float64, "values"), _stream_ptr(stream)))


def program_from_workload(ctx: Context, pw, device=None):
    """Device program, data sizes and 2-D block-format candidates of a
    ProgramWorkload (16 metrics: the MWP-CWP template; 2 metrics: the
    occupancy template).  Returns (Program, n_grid tensor, candidate tensor)."""
    import torch
    dev = torch.device("cuda", ctx.device) if device is None else device
    coefs = [planted_coefs(m) for m in pw.metrics]
    off = np.zeros(len(coefs) + 1, dtype=np.int64)
    np.cumsum([len(c) for c in coefs], out=off[1:])
    deg = np.array([m.deg_num for m in pw.metrics], dtype=np.int32)
    den = np.array([m.deg_den for m in pw.metrics], dtype=np.int32)
    coef_t = torch.from_numpy(np.concatenate(coefs)).to(dev)
    hw_t = torch.from_numpy(np.ascontiguousarray(pw.hw, dtype=np.float64)).to(dev)
    template = {RP_NUM_METRICS: RP_TEMPLATE_MWPCWP, 2: RP_TEMPLATE_OCCUPANCY}[len(pw.metrics)]
    prog = Program(ctx, template, pw.nvars, deg, den, off, coef_t, pw.scales, hw_t)
    n_t = torch.from_numpy(np.ascontiguousarray(pw.n_grid, dtype=np.float64)).to(dev)
    cand_t = torch.from_numpy(rp_candidates_2d(1024, 64)).to(dev)
    return prog, n_t, cand_t

"""NumPy front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the product library and never imports it.

Every function here marshals arrays into the plain C routines of
``oracle.c``; the arithmetic lives there.  See that file's header for the
passage of the paper each routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

STATUS = {"OK": 0, "RANK_DEFICIENT": 1, "UNDERDETERMINED": 2,
          "NONFINITE_INPUT": 3, "Q_NONPOSITIVE_AT_SAMPLE": 4, "NOT_CONVERGED": 5}
TEMPLATE_SINGLE = 0
TEMPLATE_MWPCWP = 1
TEMPLATE_OCCUPANCY = 2


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC",
                               "-shared", "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            dp = C.POINTER(C.c_double)
            ip = C.POINTER(C.c_int32)
            lp = C.POINTER(C.c_int64)
            up = C.POINTER(C.c_uint8)
            L.or_monomials.argtypes = [C.c_int, C.c_int, up, ip]
            L.or_candidates_2d.argtypes = [C.c_int, C.c_int, ip, ip]
            L.or_monomials_box.argtypes = [C.c_int, ip, up, ip]
            L.or_eval_rational.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_long, C.c_long, dp]
            L.or_lstsq.argtypes = [C.c_int, C.c_int, dp, dp, dp]
            L.or_lstsq_fit.argtypes = [C.c_int, C.c_int, dp, dp, dp]
            L.or_design.argtypes = [C.c_long, C.c_int, C.c_int, C.c_int, dp, C.c_long, dp, dp, dp]
            L.or_fit.argtypes = [C.c_long, C.c_int, C.c_int, C.c_int, dp, C.c_long, dp, dp, ip, ip, dp]
            L.or_fit_batch.argtypes = [C.c_int, lp, ip, ip, ip, dp, C.c_long, dp, lp, dp, ip, dp, C.c_int]
            L.or_loss_grad.argtypes = [C.c_long, C.c_int, C.c_int, C.c_int, dp, C.c_long, dp, dp, dp, dp]
            L.or_refine.argtypes = [C.c_long, C.c_int, C.c_int, C.c_int, dp, C.c_long, dp, dp,
                                    C.c_int, C.c_double, dp, ip]
            L.or_mwpcwp.argtypes = [dp, dp, C.c_double, C.c_double, dp]
            L.or_mwpcwp.restype = C.c_double
            L.or_program_value.argtypes = [C.c_int, C.c_int, C.c_int, ip, ip, lp, dp, dp, dp,
                                           C.c_double, ip, C.c_int]
            L.or_program_value.restype = C.c_double
            L.or_argmin.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, ip, lp, dp, dp, C.c_int,
                                    dp, dp, C.c_int, ip, C.c_int, C.c_int, ip, dp, dp]
            L.or_occupancy.argtypes = [C.c_double, C.c_double, dp, C.c_double, C.c_double]
            L.or_occupancy.restype = C.c_double
            L.or_select.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, ip, lp, dp, dp, C.c_int,
                                    C.c_double, C.c_int, C.c_int, ip, ip, lp, dp, dp, C.c_int,
                                    C.c_double, dp, dp, C.c_int, ip, C.c_int, C.c_int, ip, dp, dp]
            L.or_split_fit.argtypes = [C.c_long, C.c_int, C.c_int, C.c_int, C.c_long, dp, C.c_long,
                                       dp, lp, dp, dp, dp, ip, ip, dp, dp]
            L.or_regret.argtypes = [C.c_double, C.c_double, C.c_double]
            L.or_regret.restype = C.c_double
            _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def monomials(nvars: int, degree: int) -> np.ndarray:
    cnt = C.c_int32(0)
    if lib().or_monomials(nvars, degree, None, C.byref(cnt)) != 0:
        raise ValueError("bad monomial arguments")
    out = np.zeros((cnt.value, nvars), dtype=np.uint8)
    lib().or_monomials(nvars, degree, _p(out, C.c_uint8), C.byref(cnt))
    return out


def monomials_box(maxdeg) -> np.ndarray:
    """Exponents of the per-variable degree box, graded order."""
    md = np.ascontiguousarray(maxdeg, dtype=np.int32)
    cnt = C.c_int32(0)
    if lib().or_monomials_box(len(md), _p(md, C.c_int32), None, C.byref(cnt)) != 0:
        raise ValueError("bad degree box")
    out = np.zeros((cnt.value, len(md)), dtype=np.uint8)
    lib().or_monomials_box(len(md), _p(md, C.c_int32), _p(out, C.c_uint8), C.byref(cnt))
    return out


def num_coefs(nvars: int, dn: int, dq: int) -> int:
    return len(monomials(nvars, dn)) + len(monomials(nvars, dq)) - 1


def candidates_2d(max_prod: int = 1024, multiple: int = 64) -> np.ndarray:
    cnt = C.c_int32(0)
    lib().or_candidates_2d(max_prod, multiple, None, C.byref(cnt))
    out = np.zeros((cnt.value, 2), dtype=np.int32)
    lib().or_candidates_2d(max_prod, multiple, _p(out, C.c_int32), C.byref(cnt))
    return out


def lstsq(A: np.ndarray, b: np.ndarray):
    """Minimum-norm least-squares solution by QR with column pivoting + COD."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Acm = np.asfortranarray(A).ravel(order="F").copy()
    bb = _f64(b).copy()
    x = np.zeros(n)
    r = lib().or_lstsq(m, n, _p(Acm, C.c_double), _p(bb, C.c_double), _p(x, C.c_double))
    return x, int(r)


def lstsq_fit(A: np.ndarray, b: np.ndarray):
    """The linearised fit's least-squares solve with its numerical-rank rule
    (natural-order column distances, or independent samples when
    underdetermined).  Returns (x, rank)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Acm = np.asfortranarray(A).ravel(order="F").copy()
    bb = _f64(b).copy()
    x = np.zeros(n)
    r = lib().or_lstsq_fit(m, n, _p(Acm, C.c_double), _p(bb, C.c_double), _p(x, C.c_double))
    return x, int(r)


TAU_COL = 1e-5                       # column rule of the linearised fit
TAU_ROW = 3.1622776601683794e-07     # sample rule, sqrt(1e-13)


def design(u: np.ndarray, y: np.ndarray, dn: int, dq: int):
    u = _f64(u)
    y = _f64(y)
    v, m = u.shape
    n = num_coefs(v, dn, dq)
    A = np.zeros((m, n))
    rhs = np.zeros(m)
    lib().or_design(m, v, dn, dq, _p(u, C.c_double), m, _p(y, C.c_double),
                    _p(A, C.c_double), _p(rhs, C.c_double))
    return A, rhs


def fit(u: np.ndarray, y: np.ndarray, dn: int, dq: int):
    """Linearised LS fit of one model.  Returns (coef, status, rank, resid)."""
    u = _f64(u)
    y = _f64(y)
    v, m = u.shape
    n = num_coefs(v, dn, dq)
    coef = np.zeros(n)
    st, rk = C.c_int32(0), C.c_int32(0)
    rs = C.c_double(0.0)
    lib().or_fit(m, v, dn, dq, _p(u, C.c_double), m, _p(y, C.c_double), _p(coef, C.c_double),
                 C.byref(st), C.byref(rk), C.byref(rs))
    return coef, st.value, rk.value, rs.value


def coef_offsets(nvars, deg_num, deg_den) -> np.ndarray:
    sizes = [num_coefs(int(v), int(a), int(b)) for v, a, b in zip(nvars, deg_num, deg_den)]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def fit_batch(batch, nthreads: int = 1, fits=None):
    """Fit every fit of a FitBatch (or the subset ``fits``) on nthreads host threads.

    Returns (coef, coef_off, status, resid) over the selected fits."""
    if fits is None:
        off, nv, dn, dq = batch.sample_off, batch.nvars, batch.deg_num, batch.deg_den
        x, y = batch.x, batch.y
    else:
        fits = np.asarray(fits)
        parts_x, parts_y, counts = [], [], []
        for f in fits:
            a, b = int(batch.sample_off[f]), int(batch.sample_off[f + 1])
            parts_x.append(batch.x[:, a:b]); parts_y.append(batch.y[a:b]); counts.append(b - a)
        off = np.zeros(len(fits) + 1, dtype=np.int64)
        np.cumsum(counts, out=off[1:])
        x = np.concatenate(parts_x, axis=1) if parts_x else np.zeros((batch.max_vars, 0))
        y = np.concatenate(parts_y) if parts_y else np.zeros(0)
        nv, dn, dq = batch.nvars[fits], batch.deg_num[fits], batch.deg_den[fits]
    off = np.ascontiguousarray(off, dtype=np.int64)
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    dn = np.ascontiguousarray(dn, dtype=np.int32)
    dq = np.ascontiguousarray(dq, dtype=np.int32)
    x = _f64(x)
    y = _f64(y)
    F = len(nv)
    coff = coef_offsets(nv, dn, dq)
    coef = np.zeros(int(coff[-1]))
    status = np.zeros(F, dtype=np.int32)
    resid = np.zeros(F)
    lib().or_fit_batch(F, _p(off, C.c_int64), _p(nv, C.c_int32), _p(dn, C.c_int32),
                       _p(dq, C.c_int32), _p(x, C.c_double), x.shape[1], _p(y, C.c_double),
                       _p(coff, C.c_int64), _p(coef, C.c_double), _p(status, C.c_int32),
                       _p(resid, C.c_double), int(nthreads))
    return coef, coff, status, resid


def _check_coef(coef, nvars: int, dn: int, dq: int):
    """A coefficient vector must hold exactly the model's unknowns (the C
    routines read num_coefs of them and would silently accept a longer one)."""
    want = num_coefs(nvars, dn, dq)
    if coef.ndim != 1 or coef.shape[0] != want:
        raise ValueError(f"coefficient vector of length {coef.shape} for a model with {want} "
                         f"unknowns (nvars={nvars}, deg_num={dn}, deg_den={dq})")


def eval_rational(nvars: int, dn: int, dq: int, coef, u) -> np.ndarray:
    u = _f64(np.asarray(u).reshape(nvars, -1))
    coef = _f64(coef)
    _check_coef(coef, nvars, dn, dq)
    m = u.shape[1]
    out = np.zeros(m)
    lib().or_eval_rational(nvars, dn, dq, _p(coef, C.c_double), _p(u, C.c_double), m, m,
                           _p(out, C.c_double))
    return out


def loss_grad(u, y, dn: int, dq: int, coef):
    u = _f64(u)
    y = _f64(y)
    coef = _f64(coef)
    v, m = u.shape
    _check_coef(coef, v, dn, dq)
    L = C.c_double(0.0)
    g = np.zeros(len(coef))
    lib().or_loss_grad(m, v, dn, dq, _p(u, C.c_double), m, _p(y, C.c_double),
                       _p(coef, C.c_double), C.byref(L), _p(g, C.c_double))
    return L.value, g


def refine(u, y, dn: int, dq: int, coef0, max_iter: int = 100, rtol: float = 1e-14):
    """Levenberg-Marquardt on sum (N/Q - y)^2.  Returns (coef, loss, iters)."""
    u = _f64(u)
    y = _f64(y)
    coef = _f64(coef0).copy()
    v, m = u.shape
    _check_coef(coef, v, dn, dq)
    L = C.c_double(0.0)
    it = C.c_int32(0)
    lib().or_refine(m, v, dn, dq, _p(u, C.c_double), m, _p(y, C.c_double), _p(coef, C.c_double),
                    max_iter, rtol, C.byref(L), C.byref(it))
    return coef, L.value, it.value


def mwpcwp(g, hw, bx: float, by: float):
    g = _f64(g)
    hw = _f64(hw)
    parts = np.zeros(8)
    e = lib().or_mwpcwp(_p(g, C.c_double), _p(hw, C.c_double), float(bx), float(by),
                        _p(parts, C.c_double))
    return e, parts


class Program:
    """A rational program in plain arrays: L metric models per program."""

    def __init__(self, template_id, nvars, deg_num, deg_den, coef, coef_off,
                 hw=None, hw_stride=0, scale=None, num_programs=1):
        self.template_id = int(template_id)
        self.nvars = int(nvars)
        self.dn = np.ascontiguousarray(deg_num, dtype=np.int32)
        self.dq = np.ascontiguousarray(deg_den, dtype=np.int32)
        self.coef = _f64(coef)
        self.coef_off = np.ascontiguousarray(coef_off, dtype=np.int64)
        self.hw = None if hw is None else _f64(hw)
        self.hw_stride = int(hw_stride)
        self.scale = _f64(scale)
        self.num_programs = int(num_programs)
        self.L = len(self.dn) // self.num_programs

    def value(self, p: int, n: float, cand) -> float:
        c = np.ascontiguousarray(cand, dtype=np.int32)
        L = self.L
        hw = None if self.hw is None else self.hw[p * self.hw_stride:]
        hwp = None if hw is None else _p(np.ascontiguousarray(hw), C.c_double)
        return lib().or_program_value(
            self.template_id, L, self.nvars, _p(self.dn[p * L:], C.c_int32),
            _p(self.dq[p * L:], C.c_int32), _p(np.ascontiguousarray(self.coef_off[p * L:]), C.c_int64),
            _p(self.coef, C.c_double), hwp, _p(self.scale, C.c_double), float(n),
            _p(c, C.c_int32), len(c))


def argmin(prog: Program, n_grid, cand, programs=None):
    """Brute-force argmin per (program, n).  Returns (argmin, best, second)."""
    n_grid = _f64(n_grid)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    if cand.ndim == 1:
        cand = cand.reshape(-1, 1)
    num_cand, cdim = cand.shape
    P = prog.num_programs
    am = np.zeros((P, len(n_grid)), dtype=np.int32)
    best = np.zeros((P, len(n_grid)))
    second = np.zeros((P, len(n_grid)))
    hwp = None if prog.hw is None else _p(prog.hw, C.c_double)
    lib().or_argmin(prog.template_id, P, prog.L, prog.nvars, _p(prog.dn, C.c_int32),
                    _p(prog.dq, C.c_int32), _p(prog.coef_off, C.c_int64),
                    _p(prog.coef, C.c_double), hwp, prog.hw_stride, _p(prog.scale, C.c_double),
                    _p(n_grid, C.c_double), len(n_grid), _p(cand, C.c_int32), num_cand, cdim,
                    _p(am, C.c_int32), _p(best, C.c_double), _p(second, C.c_double))
    return am, best, second


def occupancy(regs: float, lds_bytes: float, hw, bx: float, by: float) -> float:
    """Hardware occupancy W_active / W_max (Example 1, equation (occupancy));
    -inf when the block format cannot run."""
    hw = _f64(hw)
    return lib().or_occupancy(float(regs), float(lds_bytes), _p(hw, C.c_double), float(bx), float(by))


def select(prog: Program, n_grid, cand, sense: int = 1, tie: Program | None = None,
           tie_sense: int = -1):
    """Exhaustive selection per (program, n): the candidate whose value is
    best by sense (+1 smallest, -1 largest); exact ties go to the best value
    of the tie program (same (n, candidate), its own sense), then the lowest
    index.  Returns (choice, best, second)."""
    n_grid = _f64(n_grid)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    if cand.ndim == 1:
        cand = cand.reshape(-1, 1)
    num_cand, cdim = cand.shape
    P = prog.num_programs
    ch = np.zeros((P, len(n_grid)), dtype=np.int32)
    best = np.zeros((P, len(n_grid)))
    second = np.zeros((P, len(n_grid)))
    hwp = None if prog.hw is None else _p(prog.hw, C.c_double)
    if tie is not None:
        assert tie.num_programs == P and tie.nvars == prog.nvars
        t_args = (tie.template_id, tie.L, _p(tie.dn, C.c_int32), _p(tie.dq, C.c_int32),
                  _p(tie.coef_off, C.c_int64), _p(tie.coef, C.c_double),
                  None if tie.hw is None else _p(tie.hw, C.c_double), tie.hw_stride, float(tie_sense))
    else:
        t_args = (0, 0, None, None, None, None, None, 0, 1.0)
    rc = lib().or_select(prog.template_id, P, prog.L, prog.nvars, _p(prog.dn, C.c_int32),
                         _p(prog.dq, C.c_int32), _p(prog.coef_off, C.c_int64),
                         _p(prog.coef, C.c_double), hwp, prog.hw_stride, float(sense), *t_args,
                         _p(prog.scale, C.c_double), _p(n_grid, C.c_double), len(n_grid),
                         _p(cand, C.c_int32), num_cand, cdim, _p(ch, C.c_int32),
                         _p(best, C.c_double), _p(second, C.c_double))
    if rc != 0:
        raise ValueError("or_select: bad arguments")
    return ch, best, second


def regret(crt: float, best_t: float, worst_t: float) -> float:
    return lib().or_regret(float(crt), float(best_t), float(worst_t))


def split_fit(u: np.ndarray, y: np.ndarray, degree: int, split_var: int, n_min: int,
              want_all: bool = False):
    """One decision node fitted from the samples (a threshold on u[split_var]
    with a rational of the given degree on each side).  Returns a dict with
    k (samples on the left in sorted order, -1 if no candidate), theta,
    coef_l, coef_r, status_l, status_r, obj and, if want_all, obj_all[k]."""
    u = _f64(u)
    y = _f64(y)
    v, m = u.shape
    n = num_coefs(v, degree, degree)
    k = C.c_int64(0)
    th, ob = C.c_double(0.0), C.c_double(0.0)
    sl, sr = C.c_int32(0), C.c_int32(0)
    cl, cr = np.zeros(n), np.zeros(n)
    oa = np.zeros(m + 1) if want_all else None
    rc = lib().or_split_fit(m, v, degree, split_var, n_min, _p(u, C.c_double), m,
                            _p(y, C.c_double), C.byref(k), C.byref(th), _p(cl, C.c_double),
                            _p(cr, C.c_double), C.byref(sl), C.byref(sr), C.byref(ob),
                            _p(oa, C.c_double) if want_all else None)
    if rc != 0:
        raise ValueError("bad split-fit arguments")
    out = {"k": int(k.value), "theta": th.value, "coef_l": cl, "coef_r": cr,
           "status_l": sl.value, "status_r": sr.value, "obj": ob.value}
    if want_all:
        out["obj_all"] = oa
    return out

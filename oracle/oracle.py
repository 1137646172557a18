"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It never imports the GPU library, and the GPU library never imports
it.  Inputs come from :mod:`bo_casegen`.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OR_OK, OR_NOT_CONVERGED = 0, 1
OR_ERR_SINGULAR_BLOCK, OR_ERR_SINGULAR_COARSE = -5, -6
F_BJ, F_ILU_NATURAL, F_ILU_RB, F_ILU_TILED = 0, 1, 2, 3
QI_DIAG, QI_BLOCK = 0, 1
SMOOTH_GS, SMOOTH_JACOBI, SMOOTH_L1 = 0, 1, 2
CTRL = {"bhp": 0, "wrat": 1, "lrat": 2}
PREC_FP64, PREC_FP32, PREC_FP32_BF16 = 0, 1, 2
CSMOOTH_JACOBI, CSMOOTH_L1 = 0, 1

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class OrProblem(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("top_depth", C.c_double),
        ("kx", _dp), ("ky", _dp), ("kz", _dp), ("phi0", _dp),
        ("p_ref", C.c_double), ("Bw0", C.c_double), ("cw", C.c_double), ("Bo0", C.c_double),
        ("co", C.c_double), ("Bg0", C.c_double), ("cg", C.c_double), ("Rs0", C.c_double),
        ("crs", C.c_double),
        ("mu_w", C.c_double), ("mu_o", C.c_double), ("mu_g", C.c_double), ("c_r", C.c_double),
        ("rho_wsc", C.c_double), ("rho_osc", C.c_double), ("rho_gsc", C.c_double),
        ("swc", C.c_double), ("sor", C.c_double), ("sorg", C.c_double), ("sgc", C.c_double),
        ("nw", C.c_int), ("no", C.c_int), ("ng", C.c_int),
        ("tcoef", C.c_double), ("rb_ft3", C.c_double), ("grav", C.c_double),
        ("gravity", C.c_int), ("inj_total_mobility", C.c_int),
        ("nwells", C.c_int),
        ("w_i", _ip), ("w_j", _ip), ("w_ktop", _ip), ("w_kbot", _ip), ("w_inj", _ip), ("w_ctrl", _ip),
        ("w_target", _dp), ("w_rw", _dp), ("w_skin", _dp),
        ("dual", C.c_int), ("km", _dp), ("phim", _dp), ("sigma", C.c_double),
    ]


class CprOpts(C.Structure):
    _fields_ = [("fpf", C.c_int), ("ftype", C.c_int), ("tile_x", C.c_int), ("tile_y", C.c_int),
                ("theta", C.c_double), ("coarse_max", C.c_int), ("max_levels", C.c_int),
                ("smoother", C.c_int), ("sweeps", C.c_int), ("use_amg", C.c_int), ("qi_mode", C.c_int),
                ("precision", C.c_int), ("csmoother", C.c_int), ("npr", C.c_int)]


class FgmresOpts(C.Structure):
    _fields_ = [("m", C.c_int), ("maxit", C.c_int), ("rtol", C.c_double), ("orth", C.c_int)]


class FgmresStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("rel_residual", C.c_double), ("est_residual", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b  # type: ignore
        _b.build()
    L = C.CDLL(LIB_PATH)
    P = C.POINTER(OrProblem)
    L.or_relperm.argtypes = [P, C.c_double, C.c_double, _f64p]
    L.or_rows.argtypes = [P, C.POINTER(C.c_int)]
    L.or_transfer.argtypes = [P, C.c_int]
    L.or_transfer.restype = C.c_double
    L.or_transmissibility.argtypes = [P, C.c_int, C.c_int]
    L.or_transmissibility.restype = C.c_double
    L.or_pore_volume.argtypes = [P, C.c_int, C.c_double]
    L.or_pore_volume.restype = C.c_double
    L.or_well_index.argtypes = [P, C.c_int, C.c_double, C.c_double]
    L.or_well_index.restype = C.c_double
    L.or_pattern.argtypes = [P, C.c_void_p, C.c_void_p]
    L.or_assemble.argtypes = [P, _f64p, _f64p, C.c_double, _f64p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.or_flux_residual.argtypes = [P, _f64p, _f64p]
    L.or_bsr_spmv.argtypes = [C.c_int, C.c_int, _i32p, _i32p, _f64p, C.c_double, _f64p, C.c_double, _f64p]
    L.or_bsr_spmv.restype = None
    L.or_dense_solve.argtypes = [C.c_int, _f64p, _f64p]
    L.or_qi_decouple.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, _f64p, _f64p]
    L.or_cpr_setup.argtypes = [C.c_void_p, C.c_int, _i32p, _i32p, _f64p, C.POINTER(CprOpts), C.POINTER(C.c_void_p)]
    L.or_cpr_free.argtypes = [C.c_void_p]
    L.or_cpr_free.restype = None
    for f in ("or_cpr_apply", "or_cpr_restrict", "or_cpr_vcycle", "or_cpr_fstage"):
        getattr(L, f).argtypes = [C.c_void_p, _f64p, _f64p]
    L.or_amg_nlevels.argtypes = [C.c_void_p]
    L.or_amg_level_info.argtypes = [C.c_void_p, C.c_int] + [C.POINTER(C.c_int)] * 4 + [C.POINTER(C.c_double)]
    L.or_amg_level_info.restype = None
    L.or_amg_level_get.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 10
    L.or_amg_level_get.restype = None
    L.or_amg_level_roots.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    L.or_amg_level_roots.restype = None
    L.or_cpr_get.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.or_cpr_get.restype = None
    L.or_fgmres.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_void_p, _f64p, _f64p,
                            C.POINTER(FgmresOpts), C.POINTER(FgmresStats), C.c_void_p]
    L.or_arnoldi.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_void_p, _f64p, C.c_int, C.c_int,
                             _f64p, _f64p, _f64p]
    L.or_amg_only.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_double, C.c_int, C.c_int, C.c_int,
                              C.POINTER(C.c_void_p)]
    L.or_amg_strength.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_double, C.c_void_p]
    L.or_amg_aggregate.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_double, C.c_void_p, C.c_void_p]
    L.or_condense_pattern.argtypes = [C.c_int, C.c_int, _i32p, _i32p, C.c_void_p, C.c_void_p]
    L.or_condense_values.argtypes = [C.c_int, C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p]
    L.or_condense_rhs.argtypes = [C.c_int, C.c_int, _f64p, _f64p, _f64p]
    L.or_condense_rhs.restype = None
    L.or_condense_back.argtypes = [C.c_int, C.c_int, _f64p, _f64p, _f64p, _f64p, _f64p]
    L.or_condense_back.restype = None
    L.or_bf16_round.argtypes = [C.c_float]
    L.or_bf16_round.restype = C.c_float
    _lib = L
    return L


def bf16_round(f: float) -> float:
    """The oracle's FP32 -> BF16 rounding (nearest even) of a float value."""
    return float(lib().or_bf16_round(float(np.float32(f))))


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Problem:
    """Keeps the numpy arrays of a case alive behind an ``OrProblem``."""

    def __init__(self, case):
        f = case.fluid
        self.case = case
        self._keep = []

        def d(a):
            a = np.ascontiguousarray(a, dtype=np.float64)
            self._keep.append(a)
            return _ptr(a, C.c_double)

        def i(a):
            a = np.ascontiguousarray(a, dtype=np.int32)
            self._keep.append(a)
            return _ptr(a, C.c_int32)

        W = case.wells
        s = OrProblem()
        s.nx, s.ny, s.nz = case.nx, case.ny, case.nz
        s.dx, s.dy, s.dz, s.top_depth = case.dx, case.dy, case.dz, case.top_depth
        s.kx, s.ky, s.kz, s.phi0 = d(case.kx), d(case.ky), d(case.kz), d(case.phi0)
        for k in ("p_ref", "Bw0", "cw", "Bo0", "co", "Bg0", "cg", "Rs0", "crs", "mu_w", "mu_o",
                  "mu_g", "c_r", "rho_wsc", "rho_osc", "rho_gsc", "swc", "sor", "sorg", "sgc",
                  "tcoef", "rb_ft3", "grav"):
            setattr(s, k, float(f[k]))
        s.nw, s.no, s.ng = int(f["nw"]), int(f["no"]), int(f["ng"])
        s.gravity = int(case.gravity)
        s.inj_total_mobility = int(case.inj_total_mobility)
        s.nwells = len(W)
        s.w_i = i([w.i for w in W] or [0])
        s.w_j = i([w.j for w in W] or [0])
        s.w_ktop = i([w.k_top for w in W] or [0])
        s.w_kbot = i([w.k_bot for w in W] or [0])
        s.w_inj = i([1 if w.kind == "inj" else 0 for w in W] or [0])
        s.w_ctrl = i([CTRL[w.control] for w in W] or [0])
        s.w_target = d([w.target for w in W] or [0.0])
        s.w_rw = d([w.rw for w in W] or [0.25])
        s.w_skin = d([w.skin for w in W] or [0.0])
        s.dual = int(getattr(case, "dual", False))
        s.km = d(case.km if s.dual else [0.0])
        s.phim = d(case.phim if s.dual else [0.0])
        s.sigma = float(getattr(case, "sigma", 0.0))
        self.s = s
        nc = C.c_int()
        self.rows = lib().or_rows(self.ref, C.byref(nc))
        self.ncell = nc.value

    @property
    def ref(self):
        return C.byref(self.s)


def relperm(prob: Problem, sw: float, sg: float) -> dict:
    out = np.zeros(9)
    lib().or_relperm(prob.ref, sw, sg, out)
    return dict(krw=out[0], krow=out[1], krg=out[2], krog=out[3], kro=out[4],
                dkro_dsw=out[5], dkro_dsg=out[6], dkrw=out[7], dkrg=out[8])


def transmissibility(prob: Problem, a: int, b: int) -> float:
    return lib().or_transmissibility(prob.ref, a, b)


def pore_volume(prob: Problem, g: int, p: float) -> float:
    return lib().or_pore_volume(prob.ref, g, p)


def well_index(prob: Problem, g: int, rw: float = 0.25, skin: float = 0.0) -> float:
    return lib().or_well_index(prob.ref, g, rw, skin)


def pattern(prob: Problem):
    L = lib()
    nnzb = L.or_pattern(prob.ref, None, None)
    n = prob.case.n
    rp = np.zeros(prob.rows + 1, np.int32)
    ci = np.zeros(nnzb, np.int32)
    L.or_pattern(prob.ref, rp.ctypes.data, ci.ctypes.data)
    return rp, ci


def residual(prob: Problem, x_old=None, x_new=None, dt=None) -> np.ndarray:
    c = prob.case
    x_old = np.ascontiguousarray(c.x_old if x_old is None else x_old, dtype=np.float64)
    x_new = np.ascontiguousarray(c.x_new if x_new is None else x_new, dtype=np.float64)
    R = np.zeros(3 * prob.rows)
    st = lib().or_assemble(prob.ref, x_old, x_new, c.dt if dt is None else dt, R, None, None, None)
    if st != OR_OK:
        raise RuntimeError(f"or_assemble failed: {st}")
    return R


def jacobian(prob: Problem, x_old=None, x_new=None, dt=None):
    """Returns (rowptr, colind, val (nnzb,3,3), R)."""
    c = prob.case
    x_old = np.ascontiguousarray(c.x_old if x_old is None else x_old, dtype=np.float64)
    x_new = np.ascontiguousarray(c.x_new if x_new is None else x_new, dtype=np.float64)
    rp, ci = pattern(prob)
    val = np.zeros(9 * len(ci))
    R = np.zeros(3 * prob.rows)
    st = lib().or_assemble(prob.ref, x_old, x_new, c.dt if dt is None else dt, R,
                           rp.ctypes.data, ci.ctypes.data, val.ctypes.data)
    if st != OR_OK:
        raise RuntimeError(f"or_assemble failed: {st}")
    return rp, ci, val.reshape(-1, 3, 3), R


def flux_residual(prob: Problem, x=None) -> np.ndarray:
    c = prob.case
    x = np.ascontiguousarray(c.x_new if x is None else x, dtype=np.float64)
    R = np.zeros(3 * prob.ncell)
    lib().or_flux_residual(prob.ref, x, R)
    return R


def transfer(prob: Problem, g: int) -> float:
    return lib().or_transfer(prob.ref, g)


def bsr_spmv(rp, ci, val, x, alpha=1.0, beta=0.0, y=None, bs=3) -> np.ndarray:
    n = len(rp) - 1
    y = np.zeros(bs * n) if y is None else np.array(y, dtype=np.float64, copy=True)
    lib().or_bsr_spmv(n, bs, rp, ci, np.ascontiguousarray(val, dtype=np.float64).reshape(-1),
                      alpha, np.ascontiguousarray(x, dtype=np.float64), beta, y)
    return y


def dense_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    x = np.array(b, dtype=np.float64, copy=True)
    st = lib().or_dense_solve(A.shape[0], A, x)
    if st != OR_OK:
        raise RuntimeError("singular")
    return x


def qi_decouple(rp, ci, val, mode=1):
    """Returns (c (3N), App (nnzb))."""
    n = len(rp) - 1
    w = np.zeros(3 * n)
    app = np.zeros(len(ci))
    st = lib().or_qi_decouple(n, rp, ci, np.ascontiguousarray(val, dtype=np.float64).reshape(-1), mode, w, app)
    if st != OR_OK:
        raise RuntimeError(f"or_qi_decouple failed: {st}")
    return w, app


def cpr_opts(fpf=0, ftype=F_ILU_TILED, tile=(8, 8), theta=0.08, coarse_max=192, max_levels=12,
             smoother=SMOOTH_GS, sweeps=1, use_amg=1, qi_mode=QI_BLOCK, precision=0,
             csmoother=1, npr=0) -> CprOpts:
    """precision: PREC_FP64, or the emulated mixed forms PREC_FP32 / PREC_FP32_BF16;
    csmoother: CSMOOTH_L1 (default) or CSMOOTH_JACOBI on the coarse levels;
    npr: rows of the pressure system (0: all; the cell rows of a system with
    fixed-rate well rows)."""
    return CprOpts(fpf, ftype, tile[0], tile[1], theta, coarse_max, max_levels, smoother,
                   sweeps, use_amg, qi_mode, precision, csmoother, npr)


class Cpr:
    """Oracle CPR preconditioner handle."""

    def __init__(self, prob: Optional[Problem], rp, ci, val, opts: Optional[CprOpts] = None, **kw):
        self.rp = np.ascontiguousarray(rp, dtype=np.int32)
        self.ci = np.ascontiguousarray(ci, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64).reshape(-1)
        self.n = len(self.rp) - 1
        self.opts = opts if opts is not None else cpr_opts(**kw)
        self.npr = self.opts.npr if 0 < self.opts.npr < self.n else self.n
        h = C.c_void_p()
        st = lib().or_cpr_setup(C.addressof(prob.s) if prob is not None else None, self.n,
                                self.rp, self.ci, self.val, C.byref(self.opts), C.byref(h))
        self.status = st
        if st != OR_OK:
            raise RuntimeError(f"or_cpr_setup failed: {st}")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().or_cpr_free(h)
            self.h = None

    def _call(self, f, v, m):
        out = np.zeros(m)
        st = getattr(lib(), f)(self.h, np.ascontiguousarray(v, dtype=np.float64), out)
        if st != OR_OK:
            raise RuntimeError(f"{f} failed: {st}")
        return out

    def apply(self, v):
        return self._call("or_cpr_apply", v, 3 * self.n)

    def restrict(self, v):
        return self._call("or_cpr_restrict", v, self.npr)

    def vcycle(self, b):
        return self._call("or_cpr_vcycle", b, self.npr)

    def fstage(self, r):
        return self._call("or_cpr_fstage", r, 3 * self.n)

    def weights(self):
        w = np.zeros(3 * self.n)
        lib().or_cpr_get(self.h, w.ctypes.data, None)
        return w

    def pivots(self):
        p = np.zeros(9 * self.n)
        lib().or_cpr_get(self.h, None, p.ctypes.data)
        return p.reshape(-1, 3, 3)

    def nlevels(self) -> int:
        return lib().or_amg_nlevels(self.h)

    def level(self, l: int) -> dict:
        n, nnz, pnnz, nc = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        om = C.c_double()
        lib().or_amg_level_info(self.h, l, C.byref(n), C.byref(nnz), C.byref(pnnz), C.byref(nc), C.byref(om))
        n, nnz, pnnz = n.value, nnz.value, pnnz.value
        rp = np.zeros(n + 1, np.int32); ci = np.zeros(nnz, np.int32); v = np.zeros(nnz)
        agg = np.full(n, -2, np.int32); col = np.zeros(n, np.int32)
        prp = np.zeros(n + 1, np.int32); pci = np.zeros(max(pnnz, 1), np.int32); pv = np.zeros(max(pnnz, 1))
        srp = np.zeros(n + 1, np.int32); sci = np.zeros(max(nnz, 1), np.int32)
        lib().or_amg_level_get(self.h, l, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, agg.ctypes.data,
                               col.ctypes.data, prp.ctypes.data, pci.ctypes.data, pv.ctypes.data,
                               srp.ctypes.data, sci.ctypes.data)
        out = dict(n=n, nnz=nnz, rowptr=rp, colind=ci, val=v, color=col, ncolors=nc.value,
                   omega=om.value, strong_rowptr=srp, strong_colind=sci[:srp[-1]])
        if pnnz > 0:
            root = np.zeros(n, np.uint8)
            lib().or_amg_level_roots(self.h, l, root.ctypes.data)
            out.update(agg=agg, p_rowptr=prp, p_colind=pci[:pnnz], p_val=pv[:pnnz], root=root.astype(bool))
        return out


def fgmres(rp, ci, val, b, pc: Optional[Cpr] = None, x0=None, m=30, maxit=1500, rtol=1e-6,
           orth=1, history=False):
    n = len(rp) - 1
    x = np.zeros(3 * n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    o = FgmresOpts(m, maxit, rtol, orth)
    st = FgmresStats()
    hist = np.zeros(maxit + 1)
    rc = lib().or_fgmres(n, np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32),
                         np.ascontiguousarray(val, np.float64).reshape(-1), pc.h if pc else None,
                         np.ascontiguousarray(b, np.float64), x, C.byref(o), C.byref(st),
                         hist.ctypes.data if history else None)
    info = dict(status=rc, iterations=st.iterations, restarts=st.restarts, converged=bool(st.converged),
                rel_residual=st.rel_residual, est_residual=st.est_residual)
    if history:
        info["history"] = hist[: st.iterations + 1].copy()
    return x, info


def arnoldi(rp, ci, val, b, k, pc: Optional[Cpr] = None, orth=1):
    n = len(rp) - 1
    L = 3 * n
    Z = np.zeros(k * L); V = np.zeros((k + 1) * L); H = np.zeros((k + 1) * k)
    st = lib().or_arnoldi(n, np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32),
                          np.ascontiguousarray(val, np.float64).reshape(-1), pc.h if pc else None,
                          np.ascontiguousarray(b, np.float64), k, orth, Z, V, H)
    if st != OR_OK:
        raise RuntimeError("or_arnoldi failed")
    return Z.reshape(k, L), V.reshape(k + 1, L), H.reshape(k + 1, k)


def bsr_to_dense(rp, ci, val) -> np.ndarray:
    n = len(rp) - 1
    val = np.asarray(val).reshape(-1, 3, 3)
    D = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            j = ci[e]
            D[3 * i:3 * i + 3, 3 * j:3 * j + 3] = val[e]
    return D


class Condensed:
    """Dual-porosity system with every matrix cell eliminated exactly (block
    Gaussian elimination of the matrix unknowns, Section 2.1's fracture-matrix
    pairs), and an oracle CPR of the reduced system (fracture cells, then the
    fixed-rate wells; the single-porosity pattern).  ``cpr_kw`` are the
    reduced system's CPR options (``npr`` 0: every reduced row)."""

    def __init__(self, prob: Problem, rp, ci, val, **cpr_kw):
        case = prob.case
        if not getattr(case, "dual", False):
            raise ValueError("Condensed needs a dual-porosity case")
        L = lib()
        self.N, self.nw = case.n, case.nrate
        self.rp = np.ascontiguousarray(rp, np.int32)
        self.ci = np.ascontiguousarray(ci, np.int32)
        val = np.ascontiguousarray(val, np.float64).reshape(-1)
        nnz = L.or_condense_pattern(self.N, self.nw, self.rp, self.ci, None, None)
        if nnz < 0:
            raise RuntimeError("not a dual-porosity pattern")
        nr = self.N + self.nw
        self.srp = np.zeros(nr + 1, np.int32)
        self.sci = np.zeros(nnz, np.int32)
        L.or_condense_pattern(self.N, self.nw, self.rp, self.ci, self.srp.ctypes.data, self.sci.ctypes.data)
        self.sval = np.zeros(9 * nnz)
        self.minv = np.zeros(9 * self.N)
        self.amf = np.zeros(9 * self.N)
        self.wfm = np.zeros(9 * self.N)
        st = L.or_condense_values(self.N, self.nw, self.rp, self.ci, val, self.sval, self.minv, self.amf, self.wfm)
        if st != OR_OK:
            raise RuntimeError(f"or_condense_values failed: {st}")
        self.sval = self.sval.reshape(-1, 3, 3)
        red = dataclasses.replace(case, dual=False, km=None, phim=None, sigma=0.0)
        self.red_prob = Problem(red)
        assert self.red_prob.rows == nr
        self.cpr = Cpr(self.red_prob, self.srp, self.sci, self.sval, **cpr_kw)

    def reduce(self, b):
        out = np.zeros(3 * (self.N + self.nw))
        lib().or_condense_rhs(self.N, self.nw, np.ascontiguousarray(b, np.float64), self.wfm, out)
        return out

    def back(self, b, xr):
        x = np.zeros(3 * (2 * self.N + self.nw))
        lib().or_condense_back(self.N, self.nw, np.ascontiguousarray(b, np.float64),
                               np.ascontiguousarray(xr, np.float64), self.minv, self.amf, x)
        return x

    def apply(self, v):
        """The preconditioner of the full system: exact elimination around
        the reduced system's CPR, z = back(v, CPR(reduce(v)))."""
        return self.back(v, self.cpr.apply(self.reduce(v)))


def condensed_fgmres(rp, ci, val, b, cond: Condensed, x0=None, m=30, maxit=1500, rtol=1e-6, orth=1,
                     max_passes=4):
    """Solves the full dual-porosity system through its condensed form:
    r = b - A x; FGMRES(m) on S d' = reduce(r) to ||S d' - reduce(r)|| <=
    rtol ||b|| (the full residual after back-substitution equals the reduced
    one up to rounding: matrix rows are satisfied exactly); x += back(r, d');
    repeated while the true full residual exceeds rtol ||b||.  Iterations
    count preconditioner applications on the reduced system."""
    n = len(rp) - 1
    x = np.zeros(3 * n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bnorm = np.linalg.norm(b)
    info = dict(iterations=0, restarts=0, passes=0, converged=False, rel_residual=0.0)
    if bnorm == 0.0:
        x[:] = 0.0
        info["converged"] = True
        return x, info
    for _ in range(max_passes):
        r = b - bsr_spmv(rp, ci, val, x)
        rn = np.linalg.norm(r)
        info["rel_residual"] = rn / bnorm
        if rn <= rtol * bnorm:
            info["converged"] = True
            break
        if info["iterations"] >= maxit:
            break
        br = cond.reduce(r)
        d, inner = fgmres(cond.srp, cond.sci, cond.sval, br, cond.cpr, m=m, maxit=maxit - info["iterations"],
                          rtol=rtol * bnorm / np.linalg.norm(br), orth=orth)
        info["iterations"] += inner["iterations"]
        info["restarts"] += inner["restarts"]
        info["passes"] += 1
        x += cond.back(r, d)
    return x, info


class AmgOnly(Cpr):
    """The oracle's AMG hierarchy of a scalar CSR matrix (l1-Jacobi, no grid);
    level(), nlevels() and vcycle() as for a Cpr handle."""

    def __init__(self, rp, ci, val, theta=0.08, coarse_max=192, max_levels=12, keep_singular=False):
        """keep_singular: keep the hierarchy of an operator whose coarsest
        matrix is singular (``status`` then reports it)."""
        self.rp = np.ascontiguousarray(rp, np.int32)
        self.ci = np.ascontiguousarray(ci, np.int32)
        self.val = np.ascontiguousarray(val, np.float64)
        self.n = self.npr = len(self.rp) - 1
        h = C.c_void_p()
        st = lib().or_amg_only(self.n, self.rp, self.ci, self.val, theta, coarse_max, max_levels,
                               int(keep_singular), C.byref(h))
        self.status = st
        if not h.value:
            raise RuntimeError(f"or_amg_only failed: {st}")
        self.h = h


def amg_strength(rp, ci, val, theta=0.08) -> np.ndarray:
    """Symmetrised strength flag of every entry of a scalar CSR matrix."""
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    sf = np.zeros(max(len(ci), 1), np.uint8)
    lib().or_amg_strength(len(rp) - 1, rp, ci, np.ascontiguousarray(val, np.float64), theta, sf.ctypes.data)
    return sf[:len(ci)].astype(bool)


def amg_aggregate(rp, ci, val, roots, theta=0.08):
    """Aggregates (phase 1 and 2) from the given roots; returns (agg, count)."""
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    n = len(rp) - 1
    root = np.zeros(n, np.uint8)
    root[list(roots)] = 1
    agg = np.zeros(n, np.int32)
    nc = lib().or_amg_aggregate(n, rp, ci, np.ascontiguousarray(val, np.float64), theta, root.ctypes.data,
                                agg.ctypes.data)
    return agg, nc

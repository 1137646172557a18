"""ctypes binding of libbo (argument marshalling only; every step runs in the
HIP kernels behind the C ABI declared in include/bo.h).

Device buffers are torch tensors on a ROCm device; the current torch stream is
passed as the HIP stream.  There is no CPU fallback: if libbo.so is missing or
no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbo.so")

BO_OK, BO_NOT_CONVERGED, BO_NN_FALLBACK = 0, 1, 2
BO_ERR_INVALID_ARG, BO_ERR_HIP, BO_ERR_ALLOC, BO_ERR_NONFINITE = -1, -2, -3, -4
BO_ERR_SINGULAR_BLOCK, BO_ERR_SINGULAR_COARSE, BO_ERR_BREAKDOWN, BO_ERR_UNSUPPORTED = -5, -6, -7, -8
BO_F_BJ, BO_F_ILU_NATURAL, BO_F_ILU_TILED = 0, 1, 3
BO_SMOOTH_GS, BO_SMOOTH_JACOBI, BO_SMOOTH_L1 = 0, 1, 2
BO_QI_DIAG, BO_QI_BLOCK = 0, 1
BO_PREC_FP64, BO_PREC_FP32, BO_PREC_FP32_BF16 = 0, 1, 2
BO_CSMOOTH_JACOBI, BO_CSMOOTH_L1 = 0, 1
BO_CTRL_BHP, BO_CTRL_WRATE, BO_CTRL_LRATE = 0, 1, 2

EXPORTS = [
    "bo_last_error", "bo_version", "bo_jacobian_bsr_size", "bo_jacobian_bsr", "bo_bsr_spmv",
    "bo_cpr_default_opts", "bo_cpr_setup", "bo_cpr_update", "bo_cpr_destroy", "bo_cpr_apply", "bo_cpr_spmv",
    "bo_cpr_restrict", "bo_cpr_vcycle", "bo_cpr_fstage", "bo_cpr_levels", "bo_cpr_level_info",
    "bo_cpr_level_copy", "bo_cpr_copy_weights", "bo_fgmres_default_opts", "bo_fgmres_solve",
    "bo_nn_create", "bo_nn_destroy", "bo_nn_num_params", "bo_nn_set_params", "bo_nn_get_params",
    "bo_nn_forward", "bo_nn_backward", "bo_nn_adam_step", "bo_cpr_attach_nn", "bo_cpr_collect_pairs",
    "bo_jacobian_bsr_noalloc", "bo_jacobian_bsr_noalloc_max_rows", "bo_nn_backward_weighted",
    "bo_cpr_pressure_stencil", "bo_newton_default_opts", "bo_newton_create", "bo_newton_destroy",
    "bo_newton_solve", "bo_newton_run", "bo_bicgstab_solve", "bo_jacobian2_bsr_size", "bo_jacobian2_bsr",
    "bo_bsr2_spmv", "bo_cpr2_setup", "bo_cpr2_update", "bo_fgmres_solve2", "bo_bicgstab_solve2",
    "bo_ras_default_opts", "bo_scalar_spmv", "bo_ras_setup", "bo_scalar_solve", "bo_ras_update",
]


class BoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bo status {status}: {msg}")
        self.status = status


class BoBsr(C.Structure):
    _fields_ = [("nbrows", C.c_int32), ("nnzb", C.c_int32), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("val", C.c_void_p)]


class BoFluid(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("p_ref", "Bw0", "cw", "Bo0", "co", "Bg0", "cg", "Rs0", "crs",
                                          "mu_w", "mu_o", "mu_g", "c_r", "rho_wsc", "rho_osc", "rho_gsc",
                                          "swc", "sor", "sorg", "sgc")] + \
              [("nw", C.c_int32), ("no", C.c_int32), ("ng", C.c_int32),
               ("tcoef", C.c_double), ("rb_ft3", C.c_double), ("grav", C.c_double),
               ("gravity", C.c_int32), ("inj_total_mobility", C.c_int32)]


class BoWell(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("k_top", C.c_int32), ("k_bot", C.c_int32),
                ("injector", C.c_int32), ("control", C.c_int32), ("target", C.c_double),
                ("rw", C.c_double), ("skin", C.c_double)]


class BoProblem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("top_depth", C.c_double),
                ("kx", C.c_void_p), ("ky", C.c_void_p), ("kz", C.c_void_p), ("phi0", C.c_void_p),
                ("fluid", BoFluid), ("nwells", C.c_int32), ("wells", C.POINTER(BoWell)),
                ("dual", C.c_int32), ("km", C.c_void_p), ("phim", C.c_void_p), ("sigma", C.c_double)]


class BoCprOpts(C.Structure):
    _fields_ = [("fpf", C.c_int32), ("ftype", C.c_int32), ("tile_x", C.c_int32), ("tile_y", C.c_int32),
                ("theta", C.c_double), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
                ("smoother", C.c_int32), ("sweeps", C.c_int32), ("use_amg", C.c_int32),
                ("qi_mode", C.c_int32), ("precision", C.c_int32), ("csmoother", C.c_int32),
                ("npr", C.c_int32), ("sell_rows", C.c_int32), ("condense", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class BoAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class BoGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dual", C.c_int32)]


class BoFgmresOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("maxit", C.c_int32), ("rtol", C.c_double), ("orth", C.c_int32),
                ("timing", C.c_int32), ("graph", C.c_int32), ("flexible", C.c_int32)]


class BoRasOpts(C.Structure):
    _fields_ = [("tile_x", C.c_int32), ("tile_y", C.c_int32), ("overlap", C.c_int32)]


class BoSolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("rel_residual", C.c_double), ("est_residual", C.c_double), ("spmv_ms", C.c_double),
                ("spmv_calls", C.c_int32), ("nn_used", C.c_int32)]


BO_FORCING_FIXED, BO_FORCING_EW1, BO_FORCING_EW2, BO_FORCING_EW3 = 0, 1, 2, 3
BO_NEWTON_HIST, BO_RUN_HIST = 64, 256


class BoNewtonOpts(C.Structure):
    _fields_ = [("forcing", C.c_int32), ("theta0", C.c_double), ("theta_fixed", C.c_double), ("gamma", C.c_double),
                ("beta", C.c_double), ("theta_min", C.c_double), ("theta_max", C.c_double), ("rtol", C.c_double),
                ("atol", C.c_double), ("max_newton", C.c_int32), ("ds_max", C.c_double)]


class BoNewtonStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("linear_iterations", C.c_int32), ("converged", C.c_int32),
                ("res0", C.c_double), ("res", C.c_double), ("res_hist", C.c_double * (BO_NEWTON_HIST + 1)),
                ("theta_hist", C.c_double * BO_NEWTON_HIST), ("omega_hist", C.c_double * BO_NEWTON_HIST),
                ("lin_hist", C.c_int32 * BO_NEWTON_HIST)]


class BoRunStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("cuts", C.c_int32), ("newton_iterations", C.c_int32),
                ("linear_iterations", C.c_int32), ("t", C.c_double), ("dt_hist", C.c_double * BO_RUN_HIST),
                ("newton_hist", C.c_int32 * BO_RUN_HIST)]


_lib = None


def lib():
    """Loads libbo.so (built by paper_1606_00556_amd/build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BoError(BO_ERR_HIP, f"{LIB_PATH} is not built: run __graft_entry__.build()")
    # torch owns device memory and streams: load its HIP runtime first so that
    # libbo binds to the same runtime instance (one per process)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    L.bo_last_error.restype = C.c_char_p
    L.bo_version.restype = C.c_char_p
    L.bo_jacobian_bsr_size.argtypes = [C.POINTER(BoProblem), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.bo_jacobian_bsr.argtypes = [C.POINTER(BoProblem), vp, vp, C.c_double, C.POINTER(BoBsr), vp, vp]
    L.bo_jacobian_bsr_noalloc.argtypes = [C.POINTER(BoProblem), vp, vp, C.c_double, C.POINTER(BoBsr), vp, vp]
    L.bo_jacobian_bsr_noalloc_max_rows.argtypes = []
    L.bo_jacobian_bsr_noalloc_max_rows.restype = C.c_int32
    L.bo_bsr_spmv.argtypes = [C.POINTER(BoBsr), C.c_double, vp, C.c_double, vp, vp]
    L.bo_cpr_default_opts.argtypes = [C.POINTER(BoCprOpts)]
    L.bo_cpr_default_opts.restype = None
    L.bo_cpr_setup.argtypes = [C.POINTER(BoBsr), C.POINTER(BoGrid), C.POINTER(BoCprOpts), C.POINTER(BoAllocator),
                               C.POINTER(vp), vp]
    L.bo_cpr_update.argtypes = [vp, C.POINTER(BoBsr), vp]
    L.bo_cpr_destroy.argtypes = [vp]
    L.bo_cpr_destroy.restype = None
    for f in ("bo_cpr_apply", "bo_cpr_restrict", "bo_cpr_vcycle", "bo_cpr_fstage"):
        getattr(L, f).argtypes = [vp, vp, vp, vp]
    L.bo_cpr_spmv.argtypes = [vp, C.c_double, vp, C.c_double, vp, vp]
    L.bo_cpr_levels.argtypes = [vp, C.POINTER(C.c_int32)]
    L.bo_cpr_level_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.bo_cpr_level_copy.argtypes = [vp, C.c_int32] + [vp] * 8
    L.bo_cpr_copy_weights.argtypes = [vp, vp]
    L.bo_fgmres_default_opts.argtypes = [C.POINTER(BoFgmresOpts)]
    L.bo_fgmres_default_opts.restype = None
    L.bo_fgmres_solve.argtypes = [vp, C.POINTER(BoBsr), vp, vp, C.POINTER(BoFgmresOpts), C.POINTER(BoSolveStats), vp]
    L.bo_bicgstab_solve.argtypes = [vp, C.POINTER(BoBsr), vp, vp, C.POINTER(BoFgmresOpts), C.POINTER(BoSolveStats),
                                    vp]
    # 2x2-block (two-phase) entry points; bo_bsr2 has bo_bsr's layout
    L.bo_jacobian2_bsr_size.argtypes = [C.POINTER(BoProblem), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.bo_jacobian2_bsr.argtypes = [C.POINTER(BoProblem), vp, vp, C.c_double, C.POINTER(BoBsr), vp, vp]
    L.bo_bsr2_spmv.argtypes = [C.POINTER(BoBsr), C.c_double, vp, C.c_double, vp, vp]
    L.bo_cpr2_setup.argtypes = [C.POINTER(BoBsr), C.POINTER(BoGrid), C.POINTER(BoCprOpts), C.POINTER(BoAllocator),
                                C.POINTER(vp), vp]
    L.bo_cpr2_update.argtypes = [vp, C.POINTER(BoBsr), vp]
    for f in ("bo_fgmres_solve2", "bo_bicgstab_solve2"):
        getattr(L, f).argtypes = [vp, C.POINTER(BoBsr), vp, vp, C.POINTER(BoFgmresOpts), C.POINTER(BoSolveStats), vp]
    # scalar systems with RAS
    L.bo_ras_default_opts.argtypes = [C.POINTER(BoRasOpts)]
    L.bo_ras_default_opts.restype = None
    L.bo_scalar_spmv.argtypes = [C.POINTER(BoGrid), vp, C.c_double, vp, C.c_double, vp, vp]
    L.bo_ras_setup.argtypes = [C.POINTER(BoGrid), vp, C.POINTER(BoRasOpts), C.POINTER(BoAllocator),
                               C.POINTER(vp), vp]
    L.bo_scalar_solve.argtypes = [vp, vp, vp, vp, C.POINTER(BoFgmresOpts), C.POINTER(BoSolveStats), vp]
    L.bo_ras_update.argtypes = [vp, vp, vp]
    L.bo_nn_create.argtypes = [C.POINTER(vp)]
    L.bo_nn_destroy.argtypes = [vp]
    L.bo_nn_destroy.restype = None
    L.bo_nn_num_params.argtypes = []
    L.bo_nn_num_params.restype = C.c_int32
    L.bo_nn_set_params.argtypes = [vp, vp, vp]
    L.bo_nn_get_params.argtypes = [vp, vp, vp, vp]
    L.bo_nn_forward.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp]
    L.bo_nn_backward.argtypes = [vp, vp, C.POINTER(C.c_double), vp]
    L.bo_nn_adam_step.argtypes = [vp, C.c_float, vp]
    L.bo_nn_backward_weighted.argtypes = [vp, vp, vp, C.POINTER(C.c_double), vp]
    L.bo_cpr_pressure_stencil.argtypes = [vp, vp, vp]
    L.bo_cpr_attach_nn.argtypes = [vp, vp, vp, vp]
    L.bo_cpr_collect_pairs.argtypes = [vp, vp, C.c_int32, C.c_double, vp, vp, C.POINTER(C.c_int32), vp]
    L.bo_newton_default_opts.argtypes = [C.POINTER(BoNewtonOpts)]
    L.bo_newton_default_opts.restype = None
    L.bo_newton_create.argtypes = [C.POINTER(BoProblem), C.POINTER(BoGrid), C.POINTER(BoCprOpts), C.POINTER(vp), vp]
    L.bo_newton_destroy.argtypes = [vp]
    L.bo_newton_destroy.restype = None
    L.bo_newton_solve.argtypes = [vp, vp, vp, C.c_double, C.POINTER(BoNewtonOpts), C.POINTER(BoFgmresOpts),
                                  C.POINTER(BoNewtonStats), vp]
    L.bo_newton_run.argtypes = [vp, vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                                C.POINTER(BoNewtonOpts), C.POINTER(BoFgmresOpts), C.POINTER(BoRunStats), vp]
    for f in EXPORTS:
        if f not in ("bo_last_error", "bo_version", "bo_cpr_default_opts", "bo_cpr_destroy",
                     "bo_fgmres_default_opts", "bo_nn_destroy", "bo_nn_num_params",
                     "bo_jacobian_bsr_noalloc_max_rows", "bo_newton_default_opts", "bo_newton_destroy"):
            getattr(L, f).restype = st
    _lib = L
    return L


def _check(status: int, allowed=(BO_OK,)) -> int:
    if status not in allowed:
        raise BoError(status, lib().bo_last_error().decode())
    return status


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr())


# ---- problem marshalling --------------------------------------------------------
@dataclass
class DeviceProblem:
    """A bo_problem whose fields live in device tensors (kept alive here)."""
    s: BoProblem
    tensors: tuple
    wells: object

    @property
    def ref(self):
        return C.byref(self.s)


def problem_from_case(case, device="cuda") -> DeviceProblem:
    import torch
    f = case.fluid
    fl = BoFluid(*[float(f[k]) for k in ("p_ref", "Bw0", "cw", "Bo0", "co", "Bg0", "cg", "Rs0", "crs",
                                         "mu_w", "mu_o", "mu_g", "c_r", "rho_wsc", "rho_osc", "rho_gsc",
                                         "swc", "sor", "sorg", "sgc")],
                 int(f["nw"]), int(f["no"]), int(f["ng"]), float(f["tcoef"]), float(f["rb_ft3"]),
                 float(f["grav"]), int(case.gravity), int(case.inj_total_mobility))
    dual = bool(getattr(case, "dual", False))
    fields = [case.kx, case.ky, case.kz, case.phi0] + ([case.km, case.phim] if dual else [])
    t = tuple(torch.as_tensor(a, dtype=torch.float64).to(device).contiguous() for a in fields)
    W = (BoWell * max(len(case.wells), 1))()
    for q, w in enumerate(case.wells):
        ctrl = {"bhp": BO_CTRL_BHP, "wrat": BO_CTRL_WRATE, "lrat": BO_CTRL_LRATE}[w.control]
        W[q] = BoWell(w.i, w.j, w.k_top, w.k_bot, 1 if w.kind == "inj" else 0, ctrl, w.target, w.rw, w.skin)
    s = BoProblem(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.top_depth,
                  _ptr(t[0]), _ptr(t[1]), _ptr(t[2]), _ptr(t[3]), fl, len(case.wells),
                  C.cast(W, C.POINTER(BoWell)), int(dual), _ptr(t[4]) if dual else None,
                  _ptr(t[5]) if dual else None, float(getattr(case, "sigma", 0.0)))
    return DeviceProblem(s, t, W)


@dataclass
class DeviceBsr:
    """A bo_bsr over device tensors."""
    rowptr: object
    colind: object
    val: object

    @property
    def s(self) -> BoBsr:
        return BoBsr(self.rowptr.numel() - 1, self.colind.numel(), _ptr(self.rowptr), _ptr(self.colind),
                     _ptr(self.val))


# ---- entry points (same names as the C ABI) -----------------------------------------
def bo_version() -> str:
    return lib().bo_version().decode()


def bo_jacobian_bsr_size(p: DeviceProblem):
    n, nnzb = C.c_int32(), C.c_int32()
    _check(lib().bo_jacobian_bsr_size(p.ref, C.byref(n), C.byref(nnzb)))
    return n.value, nnzb.value


def bo_jacobian_bsr(p: DeviceProblem, x_old, x_new, dt: float, J: Optional[DeviceBsr] = None, b=None,
                    stream=None):
    """Assembles J and b = -R.  Allocates J and b when they are not given."""
    import torch
    n, nnzb = bo_jacobian_bsr_size(p)
    dev = x_new.device
    if J is None:
        J = DeviceBsr(torch.empty(n + 1, dtype=torch.int32, device=dev),
                      torch.empty(nnzb, dtype=torch.int32, device=dev),
                      torch.empty(9 * nnzb, dtype=torch.float64, device=dev))
    if b is None:
        b = torch.empty(3 * n, dtype=torch.float64, device=dev)
    s = J.s
    _check(lib().bo_jacobian_bsr(p.ref, _ptr(x_old), _ptr(x_new), float(dt), C.byref(s), _ptr(b),
                                 _stream(stream)))
    return J, b


def bo_jacobian_bsr_noalloc(p: DeviceProblem, x_old, x_new, dt: float, J: DeviceBsr, b, stream=None):
    """bo_jacobian_bsr without any allocation in the library; J and b are
    the caller's (sizes from bo_jacobian_bsr_size)."""
    s = J.s
    _check(lib().bo_jacobian_bsr_noalloc(p.ref, _ptr(x_old), _ptr(x_new), float(dt), C.byref(s), _ptr(b),
                                         _stream(stream)))
    return J, b


def bo_jacobian_bsr_noalloc_max_rows() -> int:
    return int(lib().bo_jacobian_bsr_noalloc_max_rows())


def bo_bsr_spmv(A: DeviceBsr, alpha: float, x, beta: float, y, stream=None):
    s = A.s
    _check(lib().bo_bsr_spmv(C.byref(s), alpha, _ptr(x), beta, _ptr(y), _stream(stream)))
    return y


def bo_cpr_default_opts(**overrides) -> BoCprOpts:
    o = BoCprOpts()
    lib().bo_cpr_default_opts(C.byref(o))
    for k, v in overrides.items():
        if k == "tile":
            o.tile_x, o.tile_y = v
        else:
            setattr(o, k, v)
    return o


def bo_fgmres_default_opts(**overrides) -> BoFgmresOpts:
    o = BoFgmresOpts()
    lib().bo_fgmres_default_opts(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


class Cpr:
    """Owns a bo_cpr handle (bo_cpr_destroy on close / garbage collection).
    bs: block size (3 black oil, 2 two-phase)."""

    def __init__(self, h: int, n: int, bs: int = 3):
        self.h = C.c_void_p(h)
        self.n = n
        self.bs = bs
        self.A = None
        self.allocator = None

    def close(self):
        if self.h:
            lib().bo_cpr_destroy(self.h)
            self.h = None
        self.allocator = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bo_cpr_setup(A: DeviceBsr, grid, opts: Optional[BoCprOpts] = None, stream=None, allocator=None) -> Cpr:
    """grid: (nx, ny, nz) or (nx, ny, nz, dual), or None for the general form
    (see include/bo.h).  allocator: None (the library's hipMalloc) or a pair
    of callables (alloc(nbytes, stream) -> device address, free(address,
    stream)) that supply the handle's device memory for its whole life."""
    o = opts if opts is not None else bo_cpr_default_opts()
    g = BoGrid(*grid) if grid is not None else None
    al = None
    if allocator is not None:
        fa, ff = allocator
        al = BoAllocator(ALLOC_FN(lambda nbytes, ctx, st: fa(int(nbytes), st)),
                         FREE_FN(lambda ptr, ctx, st: ff(ptr, st)), None)
    h = C.c_void_p()
    s = A.s
    _check(lib().bo_cpr_setup(C.byref(s), C.byref(g) if g is not None else None, C.byref(o),
                              C.byref(al) if al is not None else None, C.byref(h), _stream(stream)))
    pc = Cpr(h.value, s.nbrows)
    pc.A = A   # the matrix of the last setup or update (bo_fgmres_solve takes it)
    pc.allocator = al   # the callbacks live as long as the handle
    return pc


def bo_cpr_update(pc: Cpr, A: DeviceBsr, stream=None) -> Cpr:
    s = A.s
    _check(lib().bo_cpr_update(pc.h, C.byref(s), _stream(stream)))
    pc.A = A
    return pc


def bo_cpr_destroy(pc: Cpr):
    pc.close()


def bo_cpr_apply(pc: Cpr, v, z, stream=None):
    _check(lib().bo_cpr_apply(pc.h, _ptr(v), _ptr(z), _stream(stream)))
    return z


def bo_cpr_spmv(pc: Cpr, alpha: float, x, beta: float, y, stream=None):
    _check(lib().bo_cpr_spmv(pc.h, alpha, _ptr(x), beta, _ptr(y), _stream(stream)))
    return y


def bo_cpr_restrict(pc: Cpr, v, rp, stream=None):
    _check(lib().bo_cpr_restrict(pc.h, _ptr(v), _ptr(rp), _stream(stream)))
    return rp


def bo_cpr_vcycle(pc: Cpr, b, x, stream=None):
    _check(lib().bo_cpr_vcycle(pc.h, _ptr(b), _ptr(x), _stream(stream)))
    return x


def bo_cpr_fstage(pc: Cpr, r, x, stream=None):
    _check(lib().bo_cpr_fstage(pc.h, _ptr(r), _ptr(x), _stream(stream)))
    return x


def bo_cpr_levels(pc: Cpr) -> int:
    n = C.c_int32()
    _check(lib().bo_cpr_levels(pc.h, C.byref(n)))
    return n.value


def bo_cpr_level_info(pc: Cpr, l: int) -> dict:
    n, nnz, pnnz, om = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().bo_cpr_level_info(pc.h, l, C.byref(n), C.byref(nnz), C.byref(pnnz), C.byref(om)))
    return dict(n=n.value, nnz=nnz.value, pnnz=pnnz.value, omega=om.value)


def bo_cpr_level_copy(pc: Cpr, l: int) -> dict:
    """Host copies (numpy) of level l."""
    import numpy as np
    info = bo_cpr_level_info(pc, l)
    n, nnz, pnnz = info["n"], info["nnz"], info["pnnz"]
    rp = np.zeros(n + 1, np.int32); ci = np.zeros(max(nnz, 1), np.int32); v = np.zeros(max(nnz, 1))
    agg = np.zeros(max(n, 1), np.int32); root = np.zeros(max(n, 1), np.uint8)
    prp = np.zeros(n + 1, np.int32); pci = np.zeros(max(pnnz, 1), np.int32); pv = np.zeros(max(pnnz, 1))
    _check(lib().bo_cpr_level_copy(pc.h, l, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, agg.ctypes.data,
                                   root.ctypes.data, prp.ctypes.data, pci.ctypes.data, pv.ctypes.data))
    out = dict(info, rowptr=rp, colind=ci[:nnz], val=v[:nnz])
    if pnnz > 0:
        out.update(agg=agg, root=root.astype(bool), p_rowptr=prp, p_colind=pci[:pnnz], p_val=pv[:pnnz])
    return out


def bo_cpr_copy_weights(pc: Cpr):
    import numpy as np
    c = np.zeros(pc.bs * pc.n)
    _check(lib().bo_cpr_copy_weights(pc.h, c.ctypes.data))
    return c


def bo_fgmres_solve(pc: Cpr, A: DeviceBsr, b, x, opts: Optional[BoFgmresOpts] = None, stream=None) -> dict:
    """A: the matrix of pc's last setup or update (the true residual is
    computed from it)."""
    o = opts if opts is not None else bo_fgmres_default_opts()
    st = BoSolveStats()
    s = A.s
    rc = lib().bo_fgmres_solve(pc.h, C.byref(s), _ptr(b), _ptr(x), C.byref(o), C.byref(st), _stream(stream))
    _check(rc, allowed=(BO_OK, BO_NOT_CONVERGED, BO_NN_FALLBACK))
    return dict(status=rc, iterations=st.iterations, restarts=st.restarts, converged=bool(st.converged),
                rel_residual=st.rel_residual, est_residual=st.est_residual, spmv_ms=st.spmv_ms,
                spmv_calls=st.spmv_calls, nn_used=st.nn_used)


def bo_bicgstab_solve(pc: Cpr, A: DeviceBsr, b, x, opts: Optional[BoFgmresOpts] = None, stream=None,
                      allowed=(BO_OK, BO_NOT_CONVERGED)) -> dict:
    """BiCGSTAB with pc (maxit and rtol of opts); A as for bo_fgmres_solve."""
    o = opts if opts is not None else bo_fgmres_default_opts()
    st = BoSolveStats()
    rc = lib().bo_bicgstab_solve(pc.h, C.byref(A.s), _ptr(b), _ptr(x), C.byref(o), C.byref(st), _stream(stream))
    _check(rc, allowed=allowed)
    return dict(status=rc, iterations=st.iterations, restarts=st.restarts, converged=bool(st.converged),
                rel_residual=st.rel_residual, est_residual=st.est_residual)


# ---- learned pressure-stage correction ---------------------------------------

NN_CHANNELS = (2, 16, 16, 16, 1)


def nn_flatten(params) -> np.ndarray:
    """[(W[27, c_in, c_out], b[c_out]) per layer] -> the flat FP32 parameter
    vector of the library (per layer W then b)."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).reshape(-1), np.asarray(b, np.float32)])
                           for W, b in params]).astype(np.float32)


def nn_unflatten(flat: np.ndarray):
    out, off = [], 0
    for l in range(4):
        ci, co = NN_CHANNELS[l], NN_CHANNELS[l + 1]
        W = flat[off:off + 27 * ci * co].reshape(27, ci, co)
        off += 27 * ci * co
        out.append((W, flat[off:off + co]))
        off += co
    return out


class Nn:
    """Owns a bo_nn handle."""

    def __init__(self, params=None):
        h = C.c_void_p()
        _check(lib().bo_nn_create(C.byref(h)))
        self.h = h
        if params is not None:
            self.set_params(params)

    def close(self):
        if self.h:
            lib().bo_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, stream=None):
        flat = params if isinstance(params, np.ndarray) else nn_flatten(params)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == lib().bo_nn_num_params()
        _check(lib().bo_nn_set_params(self.h, flat.ctypes.data, _stream(stream)))

    def get(self, stream=None):
        n = lib().bo_nn_num_params()
        p = np.empty(n, np.float32)
        g = np.empty(n, np.float32)
        _check(lib().bo_nn_get_params(self.h, p.ctypes.data, g.ctypes.data, _stream(stream)))
        return p, g

    def forward(self, x, out, stream=None):
        """x: [nb, nz, ny, nx, 2] float32 device tensor; out: [nb, nz, ny, nx]."""
        nb, nz, ny, nx, c = x.shape
        assert c == 2 and x.is_contiguous() and out.is_contiguous() and out.numel() == nb * nz * ny * nx
        _check(lib().bo_nn_forward(self.h, _ptr(x), _ptr(out), nb, nz, ny, nx, _stream(stream)))
        return out

    def backward(self, target, stream=None) -> float:
        assert target.is_contiguous()
        loss = C.c_double()
        _check(lib().bo_nn_backward(self.h, _ptr(target), C.byref(loss), _stream(stream)))
        return loss.value

    def backward_weighted(self, coef, target, stream=None) -> float:
        """coef: [7, nb, nz, ny, nx] float32 stencil; target: [nb, nz, ny, nx]."""
        assert coef.is_contiguous() and target.is_contiguous() and coef.numel() == 7 * target.numel()
        loss = C.c_double()
        _check(lib().bo_nn_backward_weighted(self.h, _ptr(coef), _ptr(target), C.byref(loss), _stream(stream)))
        return loss.value

    def adam_step(self, lr: float = 1e-3, stream=None):
        _check(lib().bo_nn_adam_step(self.h, C.c_float(lr), _stream(stream)))


def bo_cpr_attach_nn(pc: "Cpr", nn: Optional[Nn], logk=None, stream=None):
    _check(lib().bo_cpr_attach_nn(pc.h, nn.h if nn is not None else None,
                                  _ptr(logk) if logk is not None else None, _stream(stream)))


def bo_cpr_pressure_stencil(pc: "Cpr", stream=None):
    """The level-0 pressure matrix as a [7, N] float32 device tensor."""
    import torch
    coef = torch.empty((7, pc.n), dtype=torch.float32, device="cuda")
    _check(lib().bo_cpr_pressure_stencil(pc.h, _ptr(coef), _stream(stream)))
    return coef


def bo_cpr_collect_pairs(pc: "Cpr", b, ncalls: int = 4, rtol_inner: float = 1e-10, stream=None):
    """Returns (rp, e, got): [ncalls, N] float32 device tensors and the number
    of recorded pairs."""
    import torch
    n = pc.n
    rp = torch.zeros((ncalls, n), dtype=torch.float32, device=b.device)
    e = torch.zeros((ncalls, n), dtype=torch.float32, device=b.device)
    got = C.c_int32()
    _check(lib().bo_cpr_collect_pairs(pc.h, _ptr(b), ncalls, rtol_inner, _ptr(rp), _ptr(e), C.byref(got),
                                      _stream(stream)))
    return rp, e, got.value


# ---- inexact Newton and time steps ---------------------------------------------
def bo_newton_default_opts(**overrides) -> BoNewtonOpts:
    o = BoNewtonOpts()
    lib().bo_newton_default_opts(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


class Newton:
    """Owns a bo_newton handle for a DeviceProblem (kept alive here)."""

    def __init__(self, p: DeviceProblem, grid, copts: Optional[BoCprOpts] = None, stream=None):
        self.p = p
        g = BoGrid(*grid)
        o = copts if copts is not None else bo_cpr_default_opts()
        h = C.c_void_p()
        _check(lib().bo_newton_create(p.ref, C.byref(g), C.byref(o), C.byref(h), _stream(stream)))
        self.h = h

    def close(self):
        if self.h:
            lib().bo_newton_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bo_newton_solve(h: Newton, x_old, x, dt: float, opts: Optional[BoNewtonOpts] = None,
                    fopts: Optional[BoFgmresOpts] = None, stream=None) -> dict:
    o = opts if opts is not None else bo_newton_default_opts()
    fo = fopts if fopts is not None else bo_fgmres_default_opts()
    st = BoNewtonStats()
    rc = lib().bo_newton_solve(h.h, _ptr(x_old), _ptr(x), float(dt), C.byref(o), C.byref(fo), C.byref(st),
                               _stream(stream))
    _check(rc, allowed=(BO_OK, BO_NOT_CONVERGED))
    k = st.iterations
    return dict(status=rc, converged=bool(st.converged), iterations=k, linear_iterations=st.linear_iterations,
                res0=st.res0, res=st.res, res_hist=list(st.res_hist[:k + 1]), theta=list(st.theta_hist[:k]),
                omega=list(st.omega_hist[:k]), linear=list(st.lin_hist[:k]))


def bo_newton_run(h: Newton, x, t_end: float, dt0: float, dt_max: float, dt_min: float = 1e-4,
                  growth: float = 1.5, easy: int = 5, opts: Optional[BoNewtonOpts] = None,
                  fopts: Optional[BoFgmresOpts] = None, stream=None) -> dict:
    o = opts if opts is not None else bo_newton_default_opts()
    fo = fopts if fopts is not None else bo_fgmres_default_opts()
    rs = BoRunStats()
    _check(lib().bo_newton_run(h.h, _ptr(x), float(t_end), float(dt0), float(dt_max), float(dt_min), float(growth),
                               int(easy), C.byref(o), C.byref(fo), C.byref(rs), _stream(stream)))
    n = min(rs.steps, BO_RUN_HIST)
    return dict(steps=rs.steps, cuts=rs.cuts, newton_iterations=rs.newton_iterations,
                linear_iterations=rs.linear_iterations, t=rs.t, dt=list(rs.dt_hist[:n]), newton=list(rs.newton_hist[:n]))


# ---- two-phase oil-water model: 2x2 blocks ----------------------------------------
@dataclass
class DeviceBsr2(DeviceBsr):
    """A bo_bsr2 (2x2 blocks, val 4*nnzb) over device tensors."""


def bo_jacobian2_bsr_size(p: DeviceProblem):
    n, nnzb = C.c_int32(), C.c_int32()
    _check(lib().bo_jacobian2_bsr_size(p.ref, C.byref(n), C.byref(nnzb)))
    return n.value, nnzb.value


def bo_jacobian2_bsr(p: DeviceProblem, x_old, x_new, dt: float, J: Optional[DeviceBsr2] = None, b=None,
                     stream=None):
    """Two-phase J (2x2 blocks) and b = -R for states of 2N doubles (Po, Sw).
    Allocates J and b when they are not given."""
    import torch
    n, nnzb = bo_jacobian2_bsr_size(p)
    dev = x_new.device
    if J is None:
        J = DeviceBsr2(torch.empty(n + 1, dtype=torch.int32, device=dev),
                       torch.empty(nnzb, dtype=torch.int32, device=dev),
                       torch.empty(4 * nnzb, dtype=torch.float64, device=dev))
    if b is None:
        b = torch.empty(2 * n, dtype=torch.float64, device=dev)
    s = J.s
    _check(lib().bo_jacobian2_bsr(p.ref, _ptr(x_old), _ptr(x_new), float(dt), C.byref(s), _ptr(b),
                                  _stream(stream)))
    return J, b


def bo_bsr2_spmv(A: DeviceBsr2, alpha: float, x, beta: float, y, stream=None):
    s = A.s
    _check(lib().bo_bsr2_spmv(C.byref(s), alpha, _ptr(x), beta, _ptr(y), _stream(stream)))
    return y


def bo_cpr2_setup(A: DeviceBsr2, grid, opts: Optional[BoCprOpts] = None, stream=None) -> Cpr:
    """CPR of a 2x2-block matrix on the grid (nx, ny, nz)."""
    o = opts if opts is not None else bo_cpr_default_opts()
    g = BoGrid(*grid)
    h = C.c_void_p()
    s = A.s
    _check(lib().bo_cpr2_setup(C.byref(s), C.byref(g), C.byref(o), None, C.byref(h), _stream(stream)))
    pc = Cpr(h.value, s.nbrows, bs=2)
    pc.A = A
    return pc


def bo_cpr2_update(pc: Cpr, A: DeviceBsr2, stream=None) -> Cpr:
    s = A.s
    _check(lib().bo_cpr2_update(pc.h, C.byref(s), _stream(stream)))
    pc.A = A
    return pc


def _solve2(fn, pc: Cpr, A: DeviceBsr2, b, x, opts, stream):
    o = opts if opts is not None else bo_fgmres_default_opts()
    st = BoSolveStats()
    rc = getattr(lib(), fn)(pc.h, C.byref(A.s), _ptr(b), _ptr(x), C.byref(o), C.byref(st), _stream(stream))
    _check(rc, allowed=(BO_OK, BO_NOT_CONVERGED))
    return dict(status=rc, iterations=st.iterations, restarts=st.restarts, converged=bool(st.converged),
                rel_residual=st.rel_residual, est_residual=st.est_residual, spmv_ms=st.spmv_ms,
                spmv_calls=st.spmv_calls)


def bo_fgmres_solve2(pc: Cpr, A: DeviceBsr2, b, x, opts: Optional[BoFgmresOpts] = None, stream=None) -> dict:
    return _solve2("bo_fgmres_solve2", pc, A, b, x, opts, stream)


def bo_bicgstab_solve2(pc: Cpr, A: DeviceBsr2, b, x, opts: Optional[BoFgmresOpts] = None, stream=None) -> dict:
    return _solve2("bo_bicgstab_solve2", pc, A, b, x, opts, stream)


# ---- scalar pressure systems: GMRES with RAS ------------------------------------
def bo_ras_default_opts(**overrides) -> BoRasOpts:
    o = BoRasOpts()
    lib().bo_ras_default_opts(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def bo_scalar_spmv(grid, coef, alpha: float, x, beta: float, y, stream=None):
    g = BoGrid(*grid)
    _check(lib().bo_scalar_spmv(C.byref(g), _ptr(coef), alpha, _ptr(x), beta, _ptr(y), _stream(stream)))
    return y


def bo_ras_setup(grid, coef, opts: Optional[BoRasOpts] = None, stream=None) -> Cpr:
    """RAS-ILU(0) handle of the scalar system coef (7N device doubles) on grid."""
    o = opts if opts is not None else bo_ras_default_opts()
    g = BoGrid(*grid)
    h = C.c_void_p()
    _check(lib().bo_ras_setup(C.byref(g), _ptr(coef), C.byref(o), None, C.byref(h), _stream(stream)))
    pc = Cpr(h.value, grid[0] * grid[1] * grid[2], bs=1)
    pc.A = coef
    return pc


def bo_ras_update(pc: Cpr, coef, stream=None) -> Cpr:
    _check(lib().bo_ras_update(pc.h, _ptr(coef), _stream(stream)))
    pc.A = coef
    return pc


def bo_scalar_solve(pc: Cpr, coef, b, x, opts: Optional[BoFgmresOpts] = None, stream=None) -> dict:
    o = opts if opts is not None else bo_fgmres_default_opts(flexible=0)
    st = BoSolveStats()
    rc = lib().bo_scalar_solve(pc.h, _ptr(coef), _ptr(b), _ptr(x), C.byref(o), C.byref(st), _stream(stream))
    _check(rc, allowed=(BO_OK, BO_NOT_CONVERGED))
    return dict(status=rc, iterations=st.iterations, restarts=st.restarts, converged=bool(st.converged),
                rel_residual=st.rel_residual, est_residual=st.est_residual, spmv_ms=st.spmv_ms,
                spmv_calls=st.spmv_calls)

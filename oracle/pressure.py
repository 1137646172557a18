"""Oracle (test infrastructure only): the scalar pressure-system solve of the
paper's linear-solver run (Section 4.2: GMRES(30) with the restricted
additive Schwarz preconditioner, a fixed 90 iterations, on one pressure
system), in plain numpy around the C RAS of or_ras.c.

GMRES(m) is Saad's restarted GMRES with right preconditioning (no
flexibility: the preconditioner is one fixed linear operator): from x0,
r0 = b - A x0, v_1 = r0 / |r0|; step j: w = A M^{-1} v_j, modified
Gram-Schmidt against v_1..v_j (h_ij), h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j},
Givens rotations on the Hessenberg columns; after k steps (m, the iteration
cap, or the tolerance) x = x0 + M^{-1} (V_k y_k) with y_k the least-squares
solution, and the cycle restarts from the true residual.  Iterations count
Arnoldi steps.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import oracle as _O


def _lib():
    L = _O.lib()
    if not getattr(L, "_ras_ready", False):
        L.or_ras_setup.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                   C.POINTER(C.c_void_p)]
        L.or_ras_apply.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_ras_free.argtypes = [C.c_void_p]
        L.or_ras_free.restype = None
        L.or_ras_tiles.argtypes = [C.c_void_p]
        L.or_ras_tile_nnz.argtypes = [C.c_void_p, C.c_int]
        L.or_ras_tile.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 5
        L._ras_ready = True
    return L


def spmv(nx, ny, nz, coef, x):
    """y = A x for the slot coefficients coef (7, N)."""
    x = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx)
    c = np.asarray(coef).reshape(7, nz, ny, nx)
    y = c[3] * x
    y[1:, :, :] += c[0, 1:, :, :] * x[:-1, :, :]
    y[:, 1:, :] += c[1, :, 1:, :] * x[:, :-1, :]
    y[:, :, 1:] += c[2, :, :, 1:] * x[:, :, :-1]
    y[:, :, :-1] += c[4, :, :, :-1] * x[:, :, 1:]
    y[:, :-1, :] += c[5, :, :-1, :] * x[:, 1:, :]
    y[:-1, :, :] += c[6, :-1, :, :] * x[1:, :, :]
    return y.reshape(-1)


class Ras:
    """RAS with ILU(0) subdomain solves (tiles of tx x ty columns, overlap)."""

    def __init__(self, nx, ny, nz, coef, tile=(8, 8), overlap=1):
        L = _lib()
        self.coef = np.ascontiguousarray(coef, dtype=np.float64)
        self.n = nx * ny * nz
        h = C.c_void_p()
        st = L.or_ras_setup(nx, ny, nz, self.coef.ctypes.data, tile[0], tile[1], overlap, C.byref(h))
        if st != 0:
            raise RuntimeError(f"or_ras_setup failed: {st}")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            _lib().or_ras_free(h)
            self.h = None

    def apply(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.n)
        _lib().or_ras_apply(self.h, r.ctypes.data, z.ctypes.data)
        return z

    def tiles(self) -> int:
        return _lib().or_ras_tiles(self.h)

    def tile(self, t):
        """(cells, own, rowptr, colind, lu) of tile t's local system."""
        L = _lib()
        nnz = L.or_ras_tile_nnz(self.h, t)
        n = L.or_ras_tile(self.h, t, None, None, None, None, None)
        cell = np.zeros(n, np.int32)
        own = np.zeros(n, np.uint8)
        rp = np.zeros(n + 1, np.int32)
        ci = np.zeros(nnz, np.int32)
        lu = np.zeros(nnz)
        L.or_ras_tile(self.h, t, cell.ctypes.data, own.ctypes.data, rp.ctypes.data, ci.ctypes.data, lu.ctypes.data)
        return cell, own.astype(bool), rp, ci, lu


def gmres(matvec, prec, b, x0=None, m=30, maxit=90, rtol=0.0):
    """Restarted right-preconditioned GMRES(m).  rtol 0: exactly maxit steps
    (unless a breakdown).  Returns (x, info) with iterations, restarts,
    rel_residual (true, at exit) and est (the estimate after each step)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bn = float(np.linalg.norm(b))
    info = dict(iterations=0, restarts=0, converged=False, rel_residual=0.0, est=[])
    if bn == 0.0:
        x[:] = 0.0
        info["converged"] = True
        return x, info
    tol = rtol * bn
    its = 0
    while True:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        info["rel_residual"] = beta / bn
        if beta <= tol and rtol > 0.0:
            info["converged"] = True
            break
        if its >= maxit or beta == 0.0:
            break
        if its > 0:
            info["restarts"] += 1
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            w = matvec(prec(V[j]))
            its += 1
            for i in range(j + 1):
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            V.append(w / hn if hn > 0.0 else w)
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            info["est"].append(abs(g[j + 1]) / bn)
            if (rtol > 0.0 and abs(g[j + 1]) <= tol) or its >= maxit or hn == 0.0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        u = np.zeros_like(b)
        for i in range(k):
            u += y[i] * V[i]
        x = x + prec(u)
    info["iterations"] = its
    return x, info


def solve(case, tile=(8, 8), overlap=1, m=30, maxit=90, rtol=0.0):
    """GMRES(m) + RAS-ILU(0) on a bo_casegen.PressureCase."""
    A = lambda v: spmv(case.nx, case.ny, case.nz, case.coef, v)
    ras = Ras(case.nx, case.ny, case.nz, case.coef, tile, overlap)
    return gmres(A, ras.apply, case.b, m=m, maxit=maxit, rtol=rtol)

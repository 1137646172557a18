"""Oracle (test infrastructure only): right-preconditioned BiCGSTAB, one of
the Krylov solvers Section 3.3 lists and the one Section 4.2's scaling runs
use.  The paper gives no listing; this is van der Vorst's method (SIAM J.
Sci. Stat. Comput. 13, 1992) with the preconditioner applied on the right,
in plain numpy:

  r = b - A x, rhat = r, rho = alpha = omega = 1, p = v = 0
  each step:  rho' = <rhat, r>,  beta = (rho' / rho) (alpha / omega)
              p = r + beta (p - omega v),  phat = M^{-1} p,  v = A phat
              alpha = rho' / <rhat, v>,  s = r - alpha v
              (||s|| small, or maxit reached: x += alpha phat, stop)
              shat = M^{-1} s,  t = A shat,  omega = <t, s> / <t, t>
              x += alpha phat + omega shat,  r = s - omega t

Readings where the method leaves a choice (the GPU solver takes the same):
  - iterations count preconditioner applications (two per step), so that
    maxit compares with FGMRES's; an odd cap ends on the half step's
    iterate x + alpha phat;
  - when the recurrence residual meets rtol ||b|| the true residual b - A x
    is formed, and the recurrences restart from it while it does not;
  - a zero <rhat, r>, <rhat, v>, <t, t> or omega (breakdown) restarts from
    the true residual once; a second breakdown ends with status BREAKDOWN.
"""
from __future__ import annotations

from typing import Callable

import numpy as np

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


def bicgstab(matvec: Callable, prec: Callable, b, x0=None, maxit=1500, rtol=1e-6, true_matvec=None):
    """Solves A x = b.  matvec(v) -> A v (the recurrences), prec(v) -> M^{-1}
    v, true_matvec (default matvec) for the true residual.  Returns (x, info)
    with info: status, iterations, restarts, converged, rel_residual (true),
    est_residual (recurrence)."""
    b = np.asarray(b, dtype=np.float64)
    tmv = true_matvec or matvec
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    info = dict(status=NOT_CONVERGED, iterations=0, restarts=0, converged=False, rel_residual=0.0,
                est_residual=0.0)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        x[:] = 0.0
        info.update(status=OK, converged=True)
        return x, info
    tol = rtol * bnorm
    its, restarts_left = 0, 1
    r = b - tmv(x)
    rn = float(np.linalg.norm(r))
    while True:
        info["rel_residual"] = rn / bnorm
        if rn <= tol:
            info.update(status=OK, converged=True)
            break
        if its >= maxit:
            break
        rhat = r.copy()
        p = np.zeros_like(b)
        v = np.zeros_like(b)
        rho = alpha = omega = 1.0
        breakdown = False
        while its < maxit:
            rho1 = float(rhat @ r)
            if rho1 == 0.0 or not np.isfinite(rho1):
                breakdown = True
                break
            beta = (rho1 / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            phat = prec(p)
            its += 1
            v = matvec(phat)
            rv = float(rhat @ v)
            if rv == 0.0 or not np.isfinite(rv):
                breakdown = True
                break
            alpha = rho1 / rv
            s = r - alpha * v
            sn = float(np.linalg.norm(s))
            if sn <= tol or its >= maxit:
                # converged at the half step, or the cap reached there
                x = x + alpha * phat
                info["est_residual"] = sn / bnorm
                break
            shat = prec(s)
            its += 1
            t = matvec(shat)
            tt = float(t @ t)
            if not (tt > 0.0) or not np.isfinite(tt):
                x = x + alpha * phat
                breakdown = True
                break
            omega = float(t @ s) / tt
            x = x + alpha * phat + omega * shat
            r = s - omega * t
            rr = float(np.linalg.norm(r))
            info["est_residual"] = rr / bnorm
            rho = rho1
            if rr <= tol:
                break
            if omega == 0.0:
                breakdown = True
                break
        r = b - tmv(x)
        rn = float(np.linalg.norm(r))
        if breakdown:
            if rn <= tol:
                continue
            if restarts_left <= 0:
                info.update(status=BREAKDOWN, rel_residual=rn / bnorm)
                break
            restarts_left -= 1
        if its < maxit and rn > tol:
            info["restarts"] += 1
    info["iterations"] = its
    return x, info


def bicgstab_bsr(O, rp, ci, val, b, pc=None, x0=None, maxit=1500, rtol=1e-6):
    """BiCGSTAB on a 3x3 BSR system with an oracle Cpr handle (or none: M = I)."""
    mv = lambda v: O.bsr_spmv(rp, ci, val, v)
    prec = pc.apply if pc is not None else (lambda v: np.array(v, copy=True))
    return bicgstab(mv, prec, b, x0=x0, maxit=maxit, rtol=rtol)


def condensed_bicgstab(O, rp, ci, val, b, cond, x0=None, maxit=1500, rtol=1e-6, max_passes=4):
    """The full dual-porosity system through its condensed form, as the
    oracle's condensed FGMRES: r = b - A x, BiCGSTAB on S d' = reduce(r) to
    rtol ||b|| / ||reduce(r)||, x += back(r, d'), while the full residual
    exceeds rtol ||b||."""
    n = len(rp) - 1
    x = np.zeros(3 * n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.linalg.norm(b))
    info = dict(status=NOT_CONVERGED, iterations=0, restarts=0, passes=0, converged=False, rel_residual=0.0)
    if bnorm == 0.0:
        x[:] = 0.0
        info.update(status=OK, converged=True)
        return x, info
    for _ in range(max_passes):
        r = b - O.bsr_spmv(rp, ci, val, x)
        rn = float(np.linalg.norm(r))
        info["rel_residual"] = rn / bnorm
        if rn <= rtol * bnorm:
            info.update(status=OK, converged=True)
            break
        if info["iterations"] >= maxit:
            break
        br = cond.reduce(r)
        d, inner = bicgstab_bsr(O, cond.srp, cond.sci, cond.sval, br, cond.cpr, maxit=maxit - info["iterations"],
                                rtol=rtol * bnorm / float(np.linalg.norm(br)))
        info["iterations"] += inner["iterations"]
        info["restarts"] += inner["restarts"]
        info["passes"] += 1
        if inner["status"] == BREAKDOWN:
            info["status"] = BREAKDOWN
            break
        x += cond.back(r, d)
    return x, info

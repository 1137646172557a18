"""Oracle (test infrastructure only): the inexact Newton method of Section
3.1 (Algorithm "inexact Newton") with the three forcing-term choices of its
equation for theta_l, and a time step built on it.

For a residual b(x) = -R(x) (the right-hand side the Jacobian assembly
returns, so that J dx = b is the Newton system), iteration l solves
J dx = b(x^l) to ||b(x^l) - J dx|| <= theta_l ||b(x^l)|| and sets
x^{l+1} = x^l + omega dx, until ||b(x^l)|| falls below the stopping value.

Forcing terms, with r^{l-1} = b(x^{l-1}) - J_{l-1} omega dx the linear
model's residual of the step taken:
  choice 1: theta_l = ||b(x^l) - r^{l-1}|| / ||b(x^{l-1})||
  choice 2: theta_l = | ||b(x^l)|| - ||r^{l-1}|| | / ||b(x^{l-1})||
  choice 3: theta_l = gamma (||b(x^l)|| / ||b(x^{l-1})||)^beta
and a fixed theta (the standard Newton method with a tight tolerance).

Readings where the paper is silent (each also applied by the GPU loop):
  - theta_0 (no previous iterate) is the fixed value theta0 (1e-2, the
    paper's example of an inexact tolerance);
  - every theta is clipped to [theta_min, theta_max] = [1e-8, 0.1] (a
    larger ceiling let the dual-porosity test systems stall);
  - choice 2 takes the absolute value (the printed difference can be
    negative);
  - saturation chopping: omega = min(1, ds_max / max |dS|) over the
    saturation unknowns of the cell rows (ds_max = 0.2); pressures and
    well unknowns are not limited;
  - stopping: ||b(x^l)|| <= max(atol, rtol ||b(x^0)||) (2-norm, as printed,
    with the relative form added), at most max_newton iterations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np

FIXED, EW1, EW2, EW3 = 0, 1, 2, 3


@dataclass
class NewtonOpts:
    forcing: int = EW1
    theta0: float = 1e-2
    theta_fixed: float = 1e-7
    gamma: float = 0.9
    beta: float = 2.0
    theta_min: float = 1e-8
    theta_max: float = 0.1
    rtol: float = 1e-6
    atol: float = 0.0
    max_newton: int = 20
    ds_max: float = 0.2


@dataclass
class NewtonLog:
    converged: bool = False
    res: List[float] = field(default_factory=list)       # ||b(x^l)||, l = 0, 1, ...
    theta: List[float] = field(default_factory=list)     # theta_l of each linear solve
    linear_its: List[int] = field(default_factory=list)
    omega: List[float] = field(default_factory=list)


def forcing(o: NewtonOpts, l: int, bnorm: float, bnorm_prev: float, diff_norm: float, rnorm_prev: float) -> float:
    """theta_l from the norms of the current and previous residual, of
    b(x^l) - r^{l-1} (diff_norm) and of r^{l-1} (rnorm_prev)."""
    if o.forcing == FIXED:
        t = o.theta_fixed
    elif l == 0:
        t = o.theta0
    elif o.forcing == EW1:
        t = diff_norm / bnorm_prev
    elif o.forcing == EW2:
        t = abs(bnorm - rnorm_prev) / bnorm_prev
    else:
        t = o.gamma * (bnorm / bnorm_prev) ** o.beta
    return min(max(t, o.theta_min), o.theta_max)


def chop(o: NewtonOpts, dx: np.ndarray, ncell: int) -> float:
    """Step length omega limiting the largest saturation change to ds_max."""
    ds = np.abs(dx[:3 * ncell].reshape(-1, 3)[:, 1:]).max() if ncell > 0 else 0.0
    return 1.0 if ds <= o.ds_max else o.ds_max / ds


def newton(b_of: Callable, jac_of: Callable, solve: Callable, x0: np.ndarray, o: NewtonOpts, ncell: int,
           matvec: Callable):
    """Generic inexact Newton loop.  b_of(x) -> b; jac_of(x) -> J (any
    object); solve(J, b, rtol) -> (dx, linear iterations); matvec(J, v) -> J v.
    Returns (x, NewtonLog)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    log = NewtonLog()
    b = b_of(x)
    bn = float(np.linalg.norm(b))
    log.res.append(bn)
    stop = max(o.atol, o.rtol * bn)
    r_prev = None
    bn_prev = None
    for l in range(o.max_newton + 1):
        if bn <= stop:
            log.converged = True
            break
        if l == o.max_newton:
            break
        diff = float(np.linalg.norm(b - r_prev)) if r_prev is not None else 0.0
        rn = float(np.linalg.norm(r_prev)) if r_prev is not None else 0.0
        theta = forcing(o, l, bn, bn_prev if bn_prev is not None else bn, diff, rn)
        J = jac_of(x)
        dx, its = solve(J, b, theta)
        w = chop(o, dx, ncell)
        step = w * dx
        r_prev = b - matvec(J, step)
        bn_prev = bn
        x = x + step
        log.theta.append(theta)
        log.linear_its.append(its)
        log.omega.append(w)
        b = b_of(x)
        bn = float(np.linalg.norm(b))
        log.res.append(bn)
    return x, log


def newton_time_step(O, prob, x_old, x0, dt, o: NewtonOpts, cpr_kw=None, m=30, maxit=1500):
    """One time step of the black-oil model: inexact Newton on R(x; x_old, dt)
    = 0 from x0, each Newton system solved by CPR-FGMRES (the oracle's) to
    theta_l.  Returns (x, NewtonLog)."""
    cpr_kw = cpr_kw or {}

    def b_of(x):
        return -O.residual(prob, x_old=x_old, x_new=x, dt=dt)

    def jac_of(x):
        rp, ci, val, _ = O.jacobian(prob, x_old=x_old, x_new=x, dt=dt)
        return rp, ci, val

    def solve(J, b, rtol):
        rp, ci, val = J
        pc = O.Cpr(prob, rp, ci, val, **cpr_kw)
        dx, info = O.fgmres(rp, ci, val, b, pc, m=m, maxit=maxit, rtol=rtol)
        return dx, info["iterations"]

    def matvec(J, v):
        rp, ci, val = J
        return O.bsr_spmv(rp, ci, val, v)

    return newton(b_of, jac_of, solve, x0, o, prob.ncell, matvec)


@dataclass
class RunLog:
    steps: List[float] = field(default_factory=list)        # accepted time step sizes
    cuts: int = 0
    newton: List[int] = field(default_factory=list)         # Newton iterations of each accepted step
    linear: int = 0


def run(O, prob, x0, t_end, dt0, dt_max, o: NewtonOpts, cpr_kw=None, growth=1.5, easy=5, dt_min=1e-4,
        max_cuts=8):
    """Time steps from x0 over [0, t_end]: each step is an inexact Newton
    solve from the previous state; a step whose Newton loop does not converge
    is repeated with half the step; after a step that needed at most `easy`
    Newton iterations the next step grows by `growth` (capped at dt_max and
    at the remaining time).  Returns (x, RunLog)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    t, dt, log = 0.0, dt0, RunLog()
    while t < t_end * (1.0 - 1e-12):
        dt = min(dt, t_end - t)
        xn, nl = newton_time_step(O, prob, x, x, dt, o, cpr_kw)
        log.linear += sum(nl.linear_its)
        if not nl.converged:
            log.cuts += 1
            dt *= 0.5
            if dt < dt_min or log.cuts > max_cuts:
                raise RuntimeError(f"time step cut below {dt_min} days")
            continue
        x = xn
        t += dt
        log.steps.append(dt)
        log.newton.append(len(nl.theta))
        if len(nl.theta) <= easy:
            dt = min(dt * growth, dt_max)
    return x, log

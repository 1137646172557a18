"""Pins of the oracle's inexact Newton loop (Section 3.1) and time stepping
(CPU only): on an affine residual each forcing choice has a closed form
(choices 1 and 2 measure the nonlinearity, which is zero there; choice 3
follows theta_l = gamma theta_{l-1}^beta when the linear solver meets each
tolerance exactly); exact Newton on the black-oil residual converges
quadratically (which also checks the analytic Jacobian against the
residual along the whole path); chopping bounds the saturation change; the
time-step loop halves a failed step."""
import numpy as np
import pytest

import bo_casegen as cg
from oracle import newton as NW


def affine_problem(n=40, seed=3):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4.0 + 0.3 * rng.standard_normal((n, n))
    c = rng.standard_normal(n)
    return A, c


def run_affine(forcing):
    A, c = affine_problem()
    o = NW.NewtonOpts(forcing=forcing, theta_min=1e-12, theta_max=0.9, rtol=1e-10, max_newton=30)

    def solve(J, b, theta):
        # meets the tolerance with equality: r = b - A dx = theta b
        return (1.0 - theta) * np.linalg.solve(J, b), 1

    x, log = NW.newton(lambda x: c - A @ x, lambda x: A, solve, np.zeros(len(c)), o, 0, lambda J, v: J @ v)
    return x, log, o


def test_affine_forcing_closed_forms():
    for f in (NW.EW1, NW.EW2):
        x, log, o = run_affine(f)
        # b(x^l) = r^{l-1} exactly on an affine residual: theta_l = 0 -> theta_min
        assert log.theta[0] == o.theta0
        assert all(t == o.theta_min for t in log.theta[1:])
        assert log.converged and len(log.theta) == 2
    x, log, o = run_affine(NW.EW3)
    # ||b(x^l)|| = theta_{l-1} ||b(x^{l-1})||, so theta_l = gamma theta_{l-1}^beta
    assert log.theta[0] == o.theta0
    for l in range(1, len(log.theta)):
        assert log.theta[l] == pytest.approx(max(o.gamma * log.theta[l - 1] ** o.beta, o.theta_min), rel=1e-8)
    for l in range(len(log.theta)):
        assert log.res[l + 1] == pytest.approx(log.theta[l] * log.res[l], rel=1e-8)
    x, log, o = run_affine(NW.FIXED)
    assert all(t == o.theta_fixed for t in log.theta)
    A, c = affine_problem()
    assert np.linalg.norm(A @ x - c) <= 1e-10 * np.linalg.norm(c)


def test_exact_newton_converges_quadratically_on_the_black_oil_residual(oracle_lib):
    O = oracle_lib
    c = cg.tiny_case(8, 6, 4, seed=3, step=0.02, dt=3.0)
    P = O.Problem(c)
    o = NW.NewtonOpts(forcing=NW.FIXED, theta_fixed=1e-12, rtol=1e-13, max_newton=15)
    x, log = NW.newton_time_step(O, P, c.x_old, c.x_new, c.dt, o, cpr_kw=dict(coarse_max=40))
    assert log.converged
    r = np.array(log.res)
    # convergence order log(r_{l+1}/r_l) / log(r_l/r_{l-1}) of full steps
    # above rounding (1e-12 of the first residual): 2 for exact Newton
    q = [np.log(r[l + 1] / r[l]) / np.log(r[l] / r[l - 1]) for l in range(1, len(r) - 1)
         if r[l + 1] > 1e-12 * r[0] and all(w == 1.0 for w in log.omega[l - 1:l + 1])]
    assert len(q) >= 2 and q[-1] >= 1.9, (q, r)


def test_chopping_bounds_the_saturation_change():
    o = NW.NewtonOpts(ds_max=0.2)
    dx = np.zeros(3 * 5 + 3)
    dx[3 * 2 + 1] = 0.5
    dx[3 * 4 + 2] = -0.3
    dx[3 * 5] = 1e4          # a well row's pressure: not limited
    dx[0] = 300.0            # pressures: not limited
    w = NW.chop(o, dx, ncell=5)
    assert w == pytest.approx(0.4, rel=1e-15)
    assert np.abs(w * dx[:15].reshape(5, 3)[:, 1:]).max() <= 0.2 + 1e-15
    assert NW.chop(o, 0.1 * dx, ncell=5) == 1.0


def test_inexact_newton_time_steps(oracle_lib):
    """Ten days in growing steps with each forcing choice: every step
    converges, the steps add up to the interval, and the last state solves
    its own time step."""
    O = oracle_lib
    c = cg.tiny_case(8, 6, 4, seed=3, step=0.0, dt=1.0)
    P = O.Problem(c)
    for f in (NW.EW1, NW.EW2, NW.EW3):
        x, log = NW.run(O, P, c.x_old, 10.0, 1.0, 5.0, NW.NewtonOpts(forcing=f), cpr_kw=dict(coarse_max=40))
        assert sum(log.steps) == pytest.approx(10.0, rel=1e-12)
        assert log.cuts == 0 and len(log.steps) >= 3 and max(log.steps) <= 5.0
        # the step rule: grow by 1.5 after an easy step (<= 5 Newton
        # iterations), keep otherwise; the last step takes what remains
        for k in range(1, len(log.steps) - 1):
            grow = 1.5 if log.newton[k - 1] <= 5 else 1.0
            assert log.steps[k] == pytest.approx(min(log.steps[k - 1] * grow, 5.0), rel=1e-14)


def test_failed_step_is_halved(oracle_lib):
    """A Newton loop limited to one iteration cannot reach the tolerance in a
    long step: the step is halved until one iteration suffices, or the loop
    gives up below the smallest step."""
    O = oracle_lib
    c = cg.tiny_case(8, 6, 4, seed=3, step=0.0, dt=1.0)
    P = O.Problem(c)
    with pytest.raises(RuntimeError):
        NW.run(O, P, c.x_old, 4.0, 4.0, 4.0, NW.NewtonOpts(max_newton=1), cpr_kw=dict(coarse_max=40),
               dt_min=0.01, max_cuts=4)
    x, log = NW.run(O, P, c.x_old, 2.0, 2.0, 2.0, NW.NewtonOpts(max_newton=8), cpr_kw=dict(coarse_max=40))
    assert sum(log.steps) == pytest.approx(2.0)

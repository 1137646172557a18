"""GPU inexact Newton (Section 3.1) and time steps against the oracle's loop
on the same systems: per Newton iterate the forcing term theta_l, the linear
iterations (within max(1, 10 %)), the step length and the residual norm
||b(x^l)|| (1e-6 relative: the iterates agree to the linear solves'
rounding), for each forcing choice, on a single-porosity case and a
dual-porosity case with fixed-rate wells (condensed form); the time-step loop
takes the oracle's steps."""
import math

import numpy as np
import pytest

import bo_casegen as cg
from oracle import newton as NW
from tests.gpu_util import rel_err_parts, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1606_00556_amd import bo
    bo.lib()
    return bo


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def single():
    return cg.tiny_case(12, 10, 5, seed=3, step=0.02, dt=3.0)


def dual():
    return cg.make_dual_case(12, 10, 4, seed=5, wells=[cg.Well(1, 1, 0, 3, "inj", "wrat", 500.0),
                                                        cg.Well(10, 8, 0, 3, "prod", "lrat", 400.0)])


def setups(B, O, case):
    """Matching CPR options of the GPU driver and of the oracle's loop."""
    if case.dual:
        grid = (case.nx, case.ny, case.nz, 1)
        copts = B.bo_cpr_default_opts(condense=1, fpf=1, smoother=B.BO_SMOOTH_L1, coarse_max=40)
        return grid, copts, "condensed"
    return (case.nx, case.ny, case.nz), B.bo_cpr_default_opts(coarse_max=40), dict(coarse_max=40)


def oracle_step(O, case, x_old, x0, dt, o, how):
    P = O.Problem(case)
    if how != "condensed":
        return NW.newton_time_step(O, P, x_old, x0, dt, o, cpr_kw=how)

    def b_of(x):
        return -O.residual(P, x_old=x_old, x_new=x, dt=dt)

    def jac_of(x):
        return O.jacobian(P, x_old=x_old, x_new=x, dt=dt)[:3]

    def solve(J, b, rtol):
        rp, ci, val = J
        cond = O.Condensed(P, rp, ci, val, ftype=O.F_ILU_TILED, smoother=O.SMOOTH_L1, fpf=1, coarse_max=40)
        dx, info = O.condensed_fgmres(rp, ci, val, b, cond, rtol=rtol)
        return dx, info["iterations"]

    return NW.newton(b_of, jac_of, solve, x0, o, P.ncell, lambda J, v: O.bsr_spmv(*J, v))


@pytest.mark.parametrize("forcing", [NW.FIXED, NW.EW1, NW.EW2, NW.EW3])
@pytest.mark.parametrize("name", ["single", "dual"])
def test_newton_iterates_match_oracle(B, O, name, forcing):
    case = single() if name == "single" else dual()
    grid, copts, how = setups(B, O, case)
    o = NW.NewtonOpts(forcing=forcing)
    xo, olog = oracle_step(O, case, case.x_old, case.x_new, case.dt, o, how)
    p = B.problem_from_case(case)
    h = B.Newton(p, grid, copts)
    x = to_dev(case.x_new.copy())
    info = B.bo_newton_solve(h, to_dev(case.x_old), x, case.dt, B.bo_newton_default_opts(forcing=forcing))
    print(f"{name} forcing {forcing}: gpu {info['iterations']} Newton / {info['linear']} linear, "
          f"oracle {len(olog.theta)} / {olog.linear_its}")
    assert info["converged"] and olog.converged
    assert info["iterations"] == len(olog.theta)
    assert np.allclose(info["theta"], olog.theta, rtol=1e-6, atol=0.0)
    assert np.allclose(info["omega"], olog.omega, rtol=1e-9, atol=0.0)
    for a, b in zip(info["linear"], olog.linear_its):
        assert abs(a - b) <= max(1, math.ceil(0.1 * b))
    assert np.allclose(info["res_hist"], olog.res, rtol=1e-6, atol=1e-9 * olog.res[0])
    assert rel_err_parts(to_host(x), xo) <= 1e-8


def test_time_steps_match_oracle(B, O):
    case = cg.tiny_case(8, 6, 4, seed=3, step=0.0, dt=1.0)
    P = O.Problem(case)
    xo, olog = NW.run(O, P, case.x_old, 10.0, 1.0, 5.0, NW.NewtonOpts(), cpr_kw=dict(coarse_max=40))
    h = B.Newton(B.problem_from_case(case), (case.nx, case.ny, case.nz), B.bo_cpr_default_opts(coarse_max=40))
    x = to_dev(case.x_old.copy())
    rs = B.bo_newton_run(h, x, 10.0, 1.0, 5.0)
    assert rs["steps"] == len(olog.steps) and rs["cuts"] == olog.cuts == 0
    assert np.allclose(rs["dt"], olog.steps, rtol=1e-14)
    assert rs["newton"] == olog.newton
    assert rel_err_parts(to_host(x), xo) <= 1e-8

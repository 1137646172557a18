"""Pins of the oracle's BiCGSTAB (Section 3.3's Krylov solvers) to what the
mathematics fixes, independently of its own code:

  - an exact preconditioner (M^{-1} = A^{-1}) solves in one application;
  - with M = I and A diagonalisable with k distinct eigenvalues, the BiCG
    factor of the residual polynomial vanishes after k steps (finite
    termination, at most 2k applications): a wrong beta, alpha or omega
    loses it;
  - its iterates after a fixed number of steps equal scipy's independent
    BiCGSTAB with the same right preconditioner;
  - a system on which <rhat, A r> = 0 breaks the recurrences down, twice;
  - on the black-oil systems with the oracle CPR: the true residual at the
    tolerance, and the condensed dual-porosity form solves the full system.
"""
import numpy as np
import pytest
from scipy.sparse.linalg import LinearOperator
from scipy.sparse.linalg import bicgstab as scipy_bicgstab

import bo_casegen as cg
from oracle import krylov as K


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def _random_system(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + n ** 0.5 * 2.0 * np.eye(n)
    return A, rng.standard_normal(n)


def test_exact_preconditioner_one_application():
    A, b = _random_system(30, 1)
    x, info = K.bicgstab(lambda v: A @ v, lambda v: np.linalg.solve(A, v), b, rtol=1e-12)
    assert info["converged"] and info["iterations"] == 1
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_finite_termination_k_distinct_eigenvalues(k):
    n = 60
    rng = np.random.default_rng(10 + k)
    S = rng.standard_normal((n, n)) + 4.0 * np.eye(n)
    lam = np.repeat(np.linspace(1.0, 4.0, k), n // k + 1)[:n]
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    b = rng.standard_normal(n)
    x, info = K.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-9, maxit=2 * k)
    assert info["converged"], info
    assert info["iterations"] <= 2 * k
    assert np.linalg.norm(b - A @ x) <= 1e-9 * np.linalg.norm(b)
    # one step fewer cannot reach it (the minimal polynomial has degree k)
    _, short = K.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-9, maxit=2 * (k - 1))
    assert not short["converged"]


@pytest.mark.parametrize("steps", [1, 2, 3, 5])
def test_iterates_equal_scipy(steps):
    """Right preconditioning by the inverse of A's 3x3 diagonal blocks (a
    fixed linear operator): after `steps` BiCGSTAB steps (2 steps of
    applications each) the iterate equals scipy's."""
    n = 45
    A, b = _random_system(n, 3)
    A[np.abs(A) < 0.8] = 0.0
    A += 6.0 * np.eye(n)
    Dinv = np.zeros_like(A)
    for i in range(0, n, 3):
        Dinv[i:i + 3, i:i + 3] = np.linalg.inv(A[i:i + 3, i:i + 3])
    x, info = K.bicgstab(lambda v: A @ v, lambda v: Dinv @ v, b, rtol=1e-300, maxit=2 * steps)
    assert info["iterations"] == 2 * steps and not info["converged"]
    M = LinearOperator((n, n), matvec=lambda v: Dinv @ v)
    xs, flag = scipy_bicgstab(A, b, rtol=1e-300, atol=0.0, maxiter=steps, M=M)
    assert flag == steps
    assert np.allclose(x, xs, rtol=1e-11, atol=1e-13 * np.abs(xs).max())


def test_breakdown_twice_is_reported():
    # <rhat, A rhat> = 0 at the first step, and again after the restart
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    b = np.array([1.0, 0.0])
    x, info = K.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-10)
    assert info["status"] == K.BREAKDOWN and not info["converged"]
    assert info["iterations"] == 2 and info["restarts"] == 1


def test_zero_rhs_and_zero_maxit():
    A, b = _random_system(9, 4)
    x, info = K.bicgstab(lambda v: A @ v, lambda v: v, np.zeros(9), x0=np.ones(9))
    assert info["converged"] and info["iterations"] == 0 and not x.any()
    x, info = K.bicgstab(lambda v: A @ v, lambda v: v, b, x0=np.ones(9), maxit=0)
    assert info["status"] == K.NOT_CONVERGED and info["iterations"] == 0 and np.array_equal(x, np.ones(9))
    assert info["rel_residual"] == pytest.approx(np.linalg.norm(b - A @ np.ones(9)) / np.linalg.norm(b))


@pytest.mark.parametrize("make", [lambda: cg.make_case(0), lambda: cg.tiny_case(7, 5, 3, seed=21, step=0.02)])
def test_cpr_bicgstab_solves_black_oil(O, make):
    case = make()
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    b = -R
    x, info = K.bicgstab_bsr(O, rp, ci, val, b, O.Cpr(P, rp, ci, val))
    assert info["converged"] and info["iterations"] > 0
    A = O.bsr_to_dense(rp, ci, val)
    true_rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert true_rel <= 1e-6
    assert info["rel_residual"] == pytest.approx(true_rel, rel=1e-8)
    # the solution of the dense system, to the conditioning times 1e-6
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.cond(A) * np.linalg.norm(xd)


def test_condensed_bicgstab_solves_full_dual_system(O):
    case = cg.make_dual_case(12, 10, 6, seed=5, wells=[cg.Well(1, 1, 0, 5, "inj", "wrat", 900.0),
                                                        cg.Well(10, 8, 0, 5, "prod", "lrat", 800.0),
                                                        cg.Well(6, 2, 1, 4, "prod", "bhp", 2500.0)])
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    b = -R
    cond = O.Condensed(P, rp, ci, val, ftype=O.F_ILU_TILED, smoother=O.SMOOTH_L1, fpf=1, coarse_max=40)
    x, info = K.condensed_bicgstab(O, rp, ci, val, b, cond)
    assert info["converged"] and info["passes"] >= 1
    A = O.bsr_to_dense(rp, ci, val)
    assert np.linalg.norm(b - A @ x) <= 1e-6 * np.linalg.norm(b)

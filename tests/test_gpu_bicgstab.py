"""GPU parity of bo_bicgstab_solve (BiCGSTAB, Section 3.3's Krylov solvers)
against the oracle's BiCGSTAB with the oracle's CPR on the same systems:

  - iterate by iterate: after a fixed number of preconditioner applications
    (no convergence) the GPU iterate equals the oracle's per unknown to 1e-8
    and its true residual to 1e-6 relative (the CPR applications agree to
    1e-10; a few steps amplify that);
  - solves: a true FP64 residual <= 1e-6 (recomputed with the oracle's SpMV)
    and the oracle's iteration count within max(2, 10 %) (two applications
    per step);
  - the condensed dual-porosity form, a zero right-hand side, maxit 0, and
    the refusal of a non-linear (network) preconditioner."""
import math

import numpy as np
import pytest

import bo_casegen as cg
from oracle import krylov as K
from tests.gpu_util import device_bsr, ragged_case, rel_err_parts, setup_both, to_dev, to_host

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


def _gpu_solve(B, gpc, b, n3, **fo):
    import torch
    x = torch.zeros(n3, dtype=torch.float64, device="cuda")
    info = B.bo_bicgstab_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(**fo))
    return to_host(x), info


def test_bicgstab_iterates_match_oracle(B, O):
    case = ragged_case(seed=45)
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    for k in (1, 2, 4, 6, 9):
        xo, oi = K.bicgstab_bsr(O, rp, ci, val, b, opc, maxit=k, rtol=1e-14)
        xg, gi = _gpu_solve(B, gpc, b, 3 * case.n, maxit=k, rtol=1e-14)
        assert gi["iterations"] == oi["iterations"] == k and not gi["converged"]
        assert gi["status"] == B.BO_NOT_CONVERGED
        assert rel_err_parts(xg, xo) <= 1e-8, k
        rel = np.linalg.norm(b - O.bsr_spmv(rp, ci, val, xg)) / np.linalg.norm(b)
        assert rel == pytest.approx(oi["rel_residual"], rel=1e-6), (k, rel, oi["rel_residual"])
        assert gi["rel_residual"] == pytest.approx(rel, rel=1e-8)


@pytest.mark.parametrize("name", ["ragged", "cfg0", "iid_nograv"])
def test_bicgstab_solves_like_oracle(B, O, name):
    case = {"ragged": lambda: ragged_case(), "cfg0": lambda: cg.make_case(0),
            "iid_nograv": lambda: cg.tiny_case(6, 5, 4, seed=8, noise_kind="iid", gravity=False, step=0.02)}[name]()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    xo, oi = K.bicgstab_bsr(O, rp, ci, val, b, opc)
    xg, gi = _gpu_solve(B, gpc, b, 3 * case.n)
    true_rel = np.linalg.norm(b - O.bsr_spmv(rp, ci, val, xg)) / np.linalg.norm(b)
    print(f"{name}: BiCGSTAB applications gpu {gi['iterations']} oracle {oi['iterations']}, true rel {true_rel:.2e}")
    assert gi["converged"] and gi["status"] == B.BO_OK and true_rel <= 1e-6
    assert gi["rel_residual"] == pytest.approx(true_rel, rel=1e-6, abs=1e-12)
    io = oi["iterations"]
    assert abs(gi["iterations"] - io) <= max(2, math.ceil(0.1 * io))


def test_bicgstab_condensed_dual(B, O):
    import torch
    nx, ny, nz = 19, 13, 5
    wells = [cg.Well(0, 0, 0, nz - 1, "inj", "wrat", 900.0), cg.Well(nx - 1, ny - 1, 0, nz - 1, "prod", "lrat", 700.0),
             cg.Well(nx // 2, ny // 2, 1, nz - 2, "prod", "bhp", 2500.0)]
    case = cg.make_dual_case(nx, ny, nz, seed=17, wells=wells)
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    b = -R
    cond = O.Condensed(P, rp, ci, val, ftype=O.F_ILU_TILED, smoother=O.SMOOTH_L1, fpf=1, coarse_max=40)
    gpc = B.bo_cpr_setup(device_bsr(B, rp, ci, val), (nx, ny, nz, 1),
                         B.bo_cpr_default_opts(condense=1, fpf=1, smoother=B.BO_SMOOTH_L1, coarse_max=40))
    xo, oi = K.condensed_bicgstab(O, rp, ci, val, b, cond)
    xg, gi = _gpu_solve(B, gpc, b, 3 * P.rows)
    true_rel = np.linalg.norm(b - O.bsr_spmv(rp, ci, val, xg)) / np.linalg.norm(b)
    print(f"condensed: BiCGSTAB applications gpu {gi['iterations']} oracle {oi['iterations']}, true rel {true_rel:.2e}")
    assert oi["converged"] and gi["converged"] and gi["status"] == B.BO_OK and true_rel <= 1e-6
    io = oi["iterations"]
    assert abs(gi["iterations"] - io) <= max(2, math.ceil(0.1 * io))
    # a fixed number of applications on the reduced system: the oracle's iterate
    xo, oi = K.condensed_bicgstab(O, rp, ci, val, b, cond, maxit=4, rtol=1e-14)
    xg, gi = _gpu_solve(B, gpc, b, 3 * P.rows, maxit=4, rtol=1e-14)
    assert gi["iterations"] == oi["iterations"] == 4
    assert rel_err_parts(xg, xo) <= 1e-8


def test_bicgstab_edge_cases(B, O):
    import torch
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    n3 = 3 * case.n
    # zero right-hand side: x = 0 without an application
    x = torch.ones(n3, dtype=torch.float64, device="cuda")
    info = B.bo_bicgstab_solve(gpc, gpc.A, torch.zeros_like(x), x)
    assert info["converged"] and info["iterations"] == 0 and not to_host(x).any()
    # maxit 0: the initial guess and its true residual
    x0 = np.random.default_rng(3).standard_normal(n3)
    x = to_dev(x0)
    info = B.bo_bicgstab_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(maxit=0))
    assert info["status"] == B.BO_NOT_CONVERGED and info["iterations"] == 0
    assert np.array_equal(to_host(x), x0)
    ref = np.linalg.norm(b - O.bsr_spmv(rp, ci, val, x0)) / np.linalg.norm(b)
    assert info["rel_residual"] == pytest.approx(ref, rel=1e-10)
    # a network attached: the preconditioner is not linear, refused
    nn = B.Nn(cg.cnn_init(23))
    B.bo_cpr_attach_nn(gpc, nn, to_dev(np.log(case.kx)))
    with pytest.raises(B.BoError):
        B.bo_bicgstab_solve(gpc, gpc.A, to_dev(b), torch.zeros(n3, dtype=torch.float64, device="cuda"))
    B.bo_cpr_attach_nn(gpc, None)
    xg, gi = _gpu_solve(B, gpc, b, n3)
    assert gi["converged"]

"""GPU parity of the mixed-precision forms against the oracle's emulation of
the same forms (FP32 hierarchy and factors, or BF16-stored factors; FP64
decoupling, residuals and sums).

Tolerances: stages within 1e-5 relative of the emulation in the FP32 form and
2^-7 in the BF16 form (both sides round the same FP64 values the same way;
the coarse-level sums and the coarsest inverse differ in summation order);
solves reach the true FP64 residual of 1e-6 with an iteration count within
max(1, ceil(0.1 * oracle)) of the emulated oracle's."""
import math

import numpy as np
import pytest

import bo_casegen as cg
from tests.gpu_util import rel_err_parts, ragged_case, rel_err, run_stage, setup_both, solve_both

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 2.0**-7}


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


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["ragged", "cfg0"])
def test_mixed_stages_match_emulation(B, O, prec, name):
    case = ragged_case() if name == "ragged" else cg.make_case(0)
    _, _, _, _, b, opc, gpc = setup_both(B, O, case, coarse_max=40, precision=prec)
    n = case.n
    rng = np.random.default_rng(11)
    rp = rng.standard_normal(n)
    v = rng.standard_normal(3 * n)
    tol = TOL[prec]
    assert rel_err(run_stage(B, gpc, B.bo_cpr_vcycle, rp, n), opc.vcycle(rp)) <= 1e-5
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_fstage, v, 3 * n), opc.fstage(v)) <= tol
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * n), opc.apply(v)) <= tol
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, b, 3 * n), opc.apply(b)) <= tol


@pytest.mark.parametrize("kw", [dict(fpf=1), dict(ftype="bj"), dict(smoother="jacobi", sweeps=2),
                                dict(tile=(5, 3)), dict(use_amg=0), dict(csmoother="jacobi")])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_variants_match_emulation(B, O, prec, kw):
    case = ragged_case(seed=31)
    _, _, _, _, b, opc, gpc = setup_both(B, O, case, coarse_max=40, precision=prec, **kw)
    v = np.random.default_rng(12).standard_normal(3 * case.n)
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * case.n), opc.apply(v)) <= TOL[prec]


def test_fp32_stage_is_not_fp64(B, O):
    """The FP32 form really runs in FP32: its V-cycle differs from the FP64
    oracle's by more than FP64 rounding and by less than FP32 allows."""
    case = ragged_case()
    _, _, _, _, _, opc64, _ = setup_both(B, O, case, coarse_max=40)
    _, _, _, _, _, _, gpc = setup_both(B, O, case, coarse_max=40, precision="fp32")
    rp = np.random.default_rng(13).standard_normal(case.n)
    e = rel_err(run_stage(B, gpc, B.bo_cpr_vcycle, rp, case.n), opc64.vcycle(rp))
    assert 1e-12 < e <= 1e-5, e


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["ragged", "cfg0"])
def test_mixed_fgmres_reaches_fp64_residual(B, O, prec, name):
    case = ragged_case() if name == "ragged" else cg.make_case(0)
    oinfo, ginfo, true_rel, xg, xo = solve_both(B, O, case, precision=prec)
    assert ginfo["converged"] and true_rel <= 1e-6
    io = oinfo["iterations"]
    assert abs(ginfo["iterations"] - io) <= max(1, math.ceil(0.1 * io))
    # error against the FP64 oracle's solution, for the record
    print(f"{name} {prec}: its {ginfo['iterations']} (oracle {io}), |x - x_oracle|/|x_oracle| = "
          f"{rel_err(xg, xo):.2e}")


def test_mixed_update_equals_fresh_setup(B, O):
    import torch
    from tests.gpu_util import device_bsr, oracle_system
    c1, c2 = ragged_case(seed=51), ragged_case(seed=52)
    _, rp1, ci1, val1, _ = oracle_system(O, c1)
    _, rp2, ci2, val2, _ = oracle_system(O, c2)
    grid = (c1.nx, c1.ny, c1.nz)
    opts = B.bo_cpr_default_opts(precision=B.BO_PREC_FP32_BF16)
    pc = B.bo_cpr_setup(device_bsr(B, rp1, ci1, val1), grid, opts)
    B.bo_cpr_update(pc, device_bsr(B, rp2, ci2, val2))
    fresh = B.bo_cpr_setup(device_bsr(B, rp2, ci2, val2), grid, opts)
    v = np.random.default_rng(14).standard_normal(3 * c1.n)
    a = run_stage(B, pc, B.bo_cpr_apply, v, 3 * c1.n)
    f = run_stage(B, fresh, B.bo_cpr_apply, v, 3 * c1.n)
    assert np.array_equal(a, f)

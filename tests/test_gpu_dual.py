"""GPU parity for dual porosity and fixed-rate wells: the Jacobian (fracture,
matrix and well rows) against the oracle, and the general form of CPR (BSR
operator, pressure system over the cell rows, l1-Jacobi level-0 smoother,
block-Jacobi F stage) stage by stage and through FGMRES, in FP64 and the
mixed form.  Tolerances as for the grid form: Jacobian 1e-12 per block,
stages 1e-10 (FP64) or 1e-5 (FP32 form against its emulation), solves to the
true residual 1e-6 with iterations within max(1, ceil(0.1 * oracle))."""
import math

import numpy as np
import pytest

import bo_casegen as cg
from tests.gpu_util import device_bsr, rel_err, rel_err_parts, run_stage, to_dev, to_host

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


def dual_case(nx=19, ny=13, nz=5, seed=7):
    wells = [cg.Well(0, 0, 0, nz - 1, "inj", "wrat", 900.0), cg.Well(nx - 1, ny - 1, 0, nz - 1, "prod", "lrat", 700.0),
             cg.Well(nx // 2, ny // 2, 1, nz - 2, "prod", "bhp", 2500.0),
             cg.Well(nx - 1, 0, 0, nz - 1, "inj", "bhp", 3500.0)]
    return cg.make_dual_case(nx, ny, nz, seed=seed, wells=wells)


def single_rate_case():
    wells = [cg.Well(0, 0, 0, 5, "inj", "wrat", 800.0), cg.Well(18, 12, 0, 5, "prod", "lrat", 600.0)]
    return cg.tiny_case(19, 13, 6, seed=21, step=0.01, wells=wells)


CASES = {"dual": dual_case, "single_rate": single_rate_case}
CASES_BUILT = {}


def gpu_jacobian(B, case):
    p = B.problem_from_case(case)
    J, b = B.bo_jacobian_bsr(p, to_dev(case.x_old), to_dev(case.x_new), case.dt)
    return to_host(J.rowptr), to_host(J.colind), to_host(J.val).reshape(-1, 3, 3), to_host(b)


@pytest.mark.parametrize("name", list(CASES))
def test_jacobian_matches_oracle(B, O, name):
    case = CASES[name]()
    if not case.dual:
        extra = np.array([3200.0, 0.0, 0.0, 2800.0, 0.0, 0.0])
        import dataclasses
        case = dataclasses.replace(case, x_old=np.concatenate([case.x_old, extra]),
                                   x_new=np.concatenate([case.x_new, extra]))
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    grp, gci, gval, gb = gpu_jacobian(B, case)
    assert np.array_equal(grp, rp) and np.array_equal(gci, ci)
    scale = np.abs(val).max()
    for e in range(len(ci)):
        d = np.abs(gval[e] - val[e]).max()
        assert d <= 1e-12 * max(np.abs(val[e]).max(), 1e-300 * scale), (e, d)
    assert rel_err(gb, -R) <= 1e-12
    CASES_BUILT[name] = (case, P, rp, ci, val, -R)


def system(O, name):
    if name not in CASES_BUILT:
        case = CASES[name]()
        if not case.dual:
            import dataclasses
            extra = np.array([3200.0, 0.0, 0.0, 2800.0, 0.0, 0.0])
            case = dataclasses.replace(case, x_old=np.concatenate([case.x_old, extra]),
                                       x_new=np.concatenate([case.x_new, extra]))
        P = O.Problem(case)
        rp, ci, val, R = O.jacobian(P)
        CASES_BUILT[name] = (case, P, rp, ci, val, -R)
    return CASES_BUILT[name]


def both(B, O, name, precision="fp64", **kw):
    case, P, rp, ci, val, b = system(O, name)
    op = dict(fp64=O.PREC_FP64, fp32=O.PREC_FP32, bf16=O.PREC_FP32_BF16)[precision]
    bp = dict(fp64=B.BO_PREC_FP64, fp32=B.BO_PREC_FP32, bf16=B.BO_PREC_FP32_BF16)[precision]
    opc = O.Cpr(P, rp, ci, val, ftype=O.F_BJ, smoother=O.SMOOTH_L1, npr=P.ncell, coarse_max=40,
                precision=op, **kw)
    opts = B.bo_cpr_default_opts(ftype=B.BO_F_BJ, smoother=B.BO_SMOOTH_L1, npr=P.ncell, coarse_max=40,
                                 precision=bp, **kw)
    gpc = B.bo_cpr_setup(device_bsr(B, rp, ci, val), None, opts)
    return case, P, rp, ci, val, b, opc, gpc


@pytest.mark.parametrize("name", list(CASES))
def test_general_cpr_stages_match_oracle(B, O, name):
    case, P, rp, ci, val, b, opc, gpc = both(B, O, name)
    rows, npr = P.rows, P.ncell
    rng = np.random.default_rng(3)
    v = rng.standard_normal(3 * rows)
    assert rel_err(run_stage(B, gpc, B.bo_cpr_restrict, v, npr), opc.restrict(v)) <= 1e-14
    r = rng.standard_normal(npr)
    assert rel_err(run_stage(B, gpc, B.bo_cpr_vcycle, r, npr), opc.vcycle(r)) <= 1e-10
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_fstage, v, 3 * rows), opc.fstage(v)) <= 1e-10
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * rows), opc.apply(v)) <= 1e-10
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, b, 3 * rows), opc.apply(b)) <= 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_general_form_sliced_coarse_matrices(B, O, name):
    """The general form with every CSR level (level 0 included), P and R also
    kept sliced (sell_rows = 1): the cycle and CPR still match the oracle."""
    case, P, rp, ci, val, b = system(O, name)
    opc = O.Cpr(P, rp, ci, val, ftype=O.F_BJ, smoother=O.SMOOTH_L1, npr=P.ncell, coarse_max=40)
    opts = B.bo_cpr_default_opts(ftype=B.BO_F_BJ, smoother=B.BO_SMOOTH_L1, npr=P.ncell, coarse_max=40,
                                 sell_rows=1)
    gpc = B.bo_cpr_setup(device_bsr(B, rp, ci, val), None, opts)
    rng = np.random.default_rng(6)
    r = rng.standard_normal(P.ncell)
    assert rel_err(run_stage(B, gpc, B.bo_cpr_vcycle, r, P.ncell), opc.vcycle(r)) <= 1e-10
    v = rng.standard_normal(3 * P.rows)
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * P.rows), opc.apply(v)) <= 1e-10


@pytest.mark.parametrize("kw", [dict(fpf=1), dict(smoother=1, sweeps=2), dict(csmoother=0)])
def test_general_cpr_variants(B, O, kw):
    okw = dict(kw)
    c, P, rp, ci, val, b = system(O, "dual")
    smoother = kw.get("smoother", 2)
    opc = O.Cpr(P, rp, ci, val, ftype=O.F_BJ, npr=P.ncell, coarse_max=40,
                **{k: v for k, v in dict(okw, smoother=smoother).items()})
    opts = B.bo_cpr_default_opts(ftype=B.BO_F_BJ, npr=P.ncell, coarse_max=40,
                                 **{k: v for k, v in dict(okw, smoother=smoother).items()})
    gpc = B.bo_cpr_setup(device_bsr(B, rp, ci, val), None, opts)
    v = np.random.default_rng(4).standard_normal(3 * P.rows)
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * P.rows), opc.apply(v)) <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_general_mixed_matches_emulation(B, O, prec):
    case, P, rp, ci, val, b, opc, gpc = both(B, O, "dual", precision=prec)
    v = np.random.default_rng(5).standard_normal(3 * P.rows)
    tol = 1e-5 if prec == "fp32" else 2.0**-7
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * P.rows), opc.apply(v)) <= tol


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_general_fgmres(B, O, name, prec):
    import torch
    case, P, rp, ci, val, b, opc, gpc = both(B, O, name, precision=prec)
    xo, oinfo = O.fgmres(rp, ci, val, b, opc)
    x = torch.zeros(3 * P.rows, dtype=torch.float64, device="cuda")
    info = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x)
    r = b - O.bsr_spmv(rp, ci, val, to_host(x))
    assert info["converged"] and np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)
    io = oinfo["iterations"]
    assert abs(info["iterations"] - io) <= max(1, math.ceil(0.1 * io))
    print(f"{name} {prec}: its {info['iterations']} (oracle {io})")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("kw", [dict(), dict(fpf=1), dict(wells_in_pressure=True, fpf=1)])
def test_extended_grid_form_tiled_ilu(B, O, name, kw):
    """The extended grid form: tiled block ILU(0) over fracture tiles, then the
    tiles' matrix cells, then the well rows as a class of their own."""
    import torch
    kw = dict(kw)
    wp = kw.pop("wells_in_pressure", False)
    case, P, rp, ci, val, b = system(O, name)
    npr = P.rows if wp else P.ncell
    opc = O.Cpr(P, rp, ci, val, ftype=O.F_ILU_TILED, smoother=O.SMOOTH_L1, npr=npr, coarse_max=40, **kw)
    opts = B.bo_cpr_default_opts(ftype=B.BO_F_ILU_TILED, smoother=B.BO_SMOOTH_L1, npr=npr, coarse_max=40, **kw)
    gpc = B.bo_cpr_setup(device_bsr(B, rp, ci, val), (case.nx, case.ny, case.nz, int(case.dual)), opts)
    rows = P.rows
    v = np.random.default_rng(6).standard_normal(3 * rows)
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_fstage, v, 3 * rows), opc.fstage(v)) <= 1e-10
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * rows), opc.apply(v)) <= 1e-10
    xo, oinfo = O.fgmres(rp, ci, val, b, opc)
    x = torch.zeros(3 * rows, dtype=torch.float64, device="cuda")
    info = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x)
    r = b - O.bsr_spmv(rp, ci, val, to_host(x))
    assert info["converged"] and np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)
    io = oinfo["iterations"]
    assert abs(info["iterations"] - io) <= max(1, math.ceil(0.1 * io))
    print(f"{name} tiled {kw} wells-in-pressure={wp}: its {info['iterations']} (oracle {io})")


def test_general_form_rejects_grid_only_options(B, O):
    case, P, rp, ci, val, b = system(O, "dual")
    A = device_bsr(B, rp, ci, val)
    with pytest.raises(B.BoError):
        B.bo_cpr_setup(A, None, B.bo_cpr_default_opts(npr=P.ncell))        # tiled ILU needs the grid
    with pytest.raises(B.BoError):
        B.bo_cpr_setup(A, None, B.bo_cpr_default_opts(ftype=B.BO_F_BJ, npr=P.ncell))  # RB-GS needs the grid
    grid = (case.nx, case.ny, case.nz, 1)
    with pytest.raises(B.BoError):   # the extended form's tiled ILU is FP64 only
        B.bo_cpr_setup(A, grid, B.bo_cpr_default_opts(smoother=B.BO_SMOOTH_L1, npr=P.ncell,
                                                      precision=B.BO_PREC_FP32))


def test_jacobian_deep_well_rows(B, O):
    """Wells through 600 layers: the well kernel takes 64 layers per sweep of
    its lanes (ten sweeps), and the fixed-rate well's row sums stay in layer
    order, so the Jacobian matches the oracle as it does for short wells."""
    import dataclasses
    case = cg.tiny_case(3, 3, 600, seed=19, step=0.01,
                        wells=[cg.Well(1, 1, 0, 599, "prod", "lrat", 500.0),
                               cg.Well(0, 0, 0, 599, "inj", "bhp", 3500.0)])
    case = dataclasses.replace(case, x_old=np.concatenate([case.x_old, [2800.0, 0.0, 0.0]]),
                               x_new=np.concatenate([case.x_new, [2800.0, 0.0, 0.0]]))
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    grp, gci, gval, gb = gpu_jacobian(B, case)
    assert np.array_equal(grp, rp) and np.array_equal(gci, ci)
    scale = np.abs(val).max()
    for e in range(len(ci)):
        d = np.abs(gval[e] - val[e]).max()
        assert d <= 1e-12 * max(np.abs(val[e]).max(), 1e-300 * scale), (e, d)
    assert rel_err(gb, -R) <= 1e-12


def test_long_well_row_hierarchy_matches_oracle(B, O):
    """A fixed-rate well through 600 layers makes a pressure row of 601
    entries: its prolongator row takes the global-memory path; the hierarchy
    must still equal the oracle's."""
    import dataclasses
    case = cg.tiny_case(3, 3, 600, seed=9, step=0.01,
                        wells=[cg.Well(1, 1, 0, 599, "prod", "lrat", 500.0),
                               cg.Well(0, 0, 0, 599, "inj", "bhp", 3500.0)])
    case = dataclasses.replace(case, x_old=np.concatenate([case.x_old, [2800.0, 0.0, 0.0]]),
                               x_new=np.concatenate([case.x_new, [2800.0, 0.0, 0.0]]))
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    assert rp[-1] - rp[-2] == 601
    opc = O.Cpr(P, rp, ci, val, ftype=O.F_BJ, smoother=O.SMOOTH_L1, npr=P.rows, coarse_max=40)
    opts = B.bo_cpr_default_opts(ftype=B.BO_F_BJ, smoother=B.BO_SMOOTH_L1, npr=P.rows, coarse_max=40)
    gpc = B.bo_cpr_setup(device_bsr(B, rp, ci, val), None, opts)
    nl = opc.nlevels()
    assert B.bo_cpr_levels(gpc) == nl and nl >= 2
    for l in range(nl - 1):
        ol, gl = opc.level(l), B.bo_cpr_level_copy(gpc, l)
        assert np.array_equal(gl["agg"], ol["agg"])
        assert np.array_equal(gl["p_rowptr"], ol["p_rowptr"]) and np.array_equal(gl["p_colind"], ol["p_colind"])
        assert rel_err(gl["p_val"], ol["p_val"]) <= 1e-12
    v = np.random.default_rng(9).standard_normal(3 * P.rows)
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * P.rows), opc.apply(v)) <= 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_general_handle_spmv_on_sliced_copy(B, O, name):
    """The general form's own SpMV reads a sliced copy of A (64-row slices of
    rows with 2 to 8 blocks, a ragged last slice): with integer data it gives
    the BSR product bit for bit, with real data and alpha, beta it matches
    the BSR kernel to 1e-12."""
    import torch
    case, P, rp, ci, val, b = system(O, name)
    n = len(rp) - 1
    assert n % 64 != 0 and len(set(np.diff(rp))) > 2
    rng = np.random.default_rng(11)
    vi = rng.integers(-1024, 1025, size=val.shape).astype(np.float64)
    x = rng.integers(-1024, 1025, size=3 * n).astype(np.float64)
    opts = B.bo_cpr_default_opts(use_amg=0, ftype=B.BO_F_BJ, npr=P.ncell)
    pc = B.bo_cpr_setup(device_bsr(B, rp, ci, vi), None, opts)
    y = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    B.bo_cpr_spmv(pc, 1.0, to_dev(x), 0.0, y)
    assert np.array_equal(to_host(y), O.bsr_spmv(rp, ci, vi, x))
    pc = B.bo_cpr_setup(device_bsr(B, rp, ci, val), None, opts)
    xr = rng.standard_normal(3 * n)
    y0 = rng.standard_normal(3 * n)
    y = to_dev(y0.copy())
    B.bo_cpr_spmv(pc, -0.75, to_dev(xr), 1.5, y)
    ref = O.bsr_spmv(rp, ci, val, xr, alpha=-0.75, beta=1.5, y=y0)
    assert rel_err(to_host(y), ref) <= 1e-12

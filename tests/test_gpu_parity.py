"""GPU parity: every stage of the HIP path, called through the C ABI, against
the FP64 oracle on the same seeded inputs.

Tolerances: Jacobian and SpMV 1e-12 relative (integer-valued SpMV bit-exact);
preconditioner stages 1e-10 relative; aggregates, roots and patterns
integer-equal; solves must reach a true FP64 residual <= 1e-6 with an
iteration count within max(1, ceil(0.1 * oracle)) of the oracle's."""
import math

import numpy as np
import pytest

import bo_casegen as cg
from tests.gpu_util import (device_bsr, matching_opts, oracle_system, ragged_case, rel_err, rel_err_parts, run_stage,
                            setup_both, solve_both, to_dev, to_host)

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


def gpu_jacobian(B, case):
    import torch
    p = B.problem_from_case(case)
    xo = to_dev(case.x_old)
    xn = to_dev(case.x_new)
    J, b = B.bo_jacobian_bsr(p, xo, xn, case.dt)
    torch.cuda.synchronize()
    return to_host(J.rowptr), to_host(J.colind), to_host(J.val).reshape(-1, 3, 3), to_host(b)


CASES = {
    "ragged": lambda: ragged_case(),
    "cfg0": lambda: cg.make_case(0),
    "line": lambda: cg.tiny_case(9, 1, 1, seed=3, step=0.01,
                                 wells=[cg.Well(0, 0, 0, 0, "inj", "bhp", 3500.0)]),
    "iid_nograv": lambda: cg.tiny_case(6, 5, 4, seed=8, noise_kind="iid", gravity=False, step=0.02),
}


@pytest.mark.parametrize("name", list(CASES))
def test_jacobian_matches_oracle(B, O, name):
    case = CASES[name]()
    _, rp, ci, val, b = oracle_system(O, case)
    grp, gci, gval, gb = gpu_jacobian(B, case)
    assert np.array_equal(grp, rp) and np.array_equal(gci, ci)
    scale = np.abs(val).max()
    # per block relative to the block's own size (wells enter through libm
    # functions, elsewhere the operation order is the oracle's)
    for e in range(len(ci)):
        d = np.abs(gval[e] - val[e]).max()
        assert d <= 1e-12 * max(np.abs(val[e]).max(), 1e-300 * scale), (e, d)
    assert rel_err(gb, b) <= 1e-12


def test_jacobian_is_bitwise_without_wells(B, O):
    case = cg.tiny_case(11, 7, 5, seed=13, noise_kind="iid", step=0.02, wells=[])
    _, rp, ci, val, b = oracle_system(O, case)
    _, _, gval, gb = gpu_jacobian(B, case)
    assert np.array_equal(gval.reshape(-1), val.reshape(-1))
    assert np.array_equal(gb, b)


def test_bsr_spmv_integer_exact(B, O):
    import torch
    case = ragged_case()
    rp, ci = O.pattern(O.Problem(case))
    rng = np.random.default_rng(5)
    val = rng.integers(-1024, 1025, size=(len(ci), 3, 3)).astype(np.float64)
    x = rng.integers(-1024, 1025, size=3 * case.n).astype(np.float64)
    ref = O.bsr_spmv(rp, ci, val, x)
    A = device_bsr(B, rp, ci, val)
    y = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
    B.bo_bsr_spmv(A, 1.0, to_dev(x), 0.0, y)
    assert np.array_equal(to_host(y), ref)
    # the solver's own copy of A (slot layout) must give the same bits
    pc = B.bo_cpr_setup(A, (case.nx, case.ny, case.nz), B.bo_cpr_default_opts(use_amg=0, ftype=B.BO_F_BJ))
    y2 = torch.zeros_like(y)
    B.bo_cpr_spmv(pc, 1.0, to_dev(x), 0.0, y2)
    assert np.array_equal(to_host(y2), ref)


def test_spmv_axpby_random(B, O):
    import torch
    case = ragged_case()
    _, rp, ci, val, _ = oracle_system(O, case)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(3 * case.n)
    y0 = rng.standard_normal(3 * case.n)
    ref = O.bsr_spmv(rp, ci, val, x, alpha=-0.75, beta=1.5, y=y0)
    A = device_bsr(B, rp, ci, val)
    pc = B.bo_cpr_setup(A, (case.nx, case.ny, case.nz), B.bo_cpr_default_opts(use_amg=0, ftype=B.BO_F_BJ))
    y = to_dev(y0.copy())
    # element-wise, each entry against the size of its own terms (sum of
    # |alpha a_ij x_j| and |beta y_i|): no cancellation hides an error
    mag = 0.75 * O.bsr_spmv(rp, ci, np.abs(val), np.abs(x)) + 1.5 * np.abs(y0)
    B.bo_cpr_spmv(pc, -0.75, to_dev(x), 1.5, y)
    assert np.all(np.abs(to_host(y) - ref) <= 1e-14 * mag)
    y = to_dev(y0.copy())
    B.bo_bsr_spmv(A, -0.75, to_dev(x), 1.5, y)
    assert np.all(np.abs(to_host(y) - ref) <= 1e-14 * mag)


def test_decoupling_weights_bitwise(B, O):
    case = cg.make_case(0)
    _, _, _, _, _, opc, gpc = setup_both(B, O, case)
    assert np.array_equal(B.bo_cpr_copy_weights(gpc), opc.weights())


@pytest.mark.parametrize("name", ["ragged", "cfg0"])
def test_amg_hierarchy_matches_oracle(B, O, name):
    case = CASES[name]()
    _, _, _, _, _, opc, gpc = setup_both(B, O, case, coarse_max=40)
    nl = opc.nlevels()
    assert B.bo_cpr_levels(gpc) == nl and nl >= 2
    for l in range(nl):
        ol, gl = opc.level(l), B.bo_cpr_level_copy(gpc, l)
        assert gl["n"] == ol["n"] and gl["nnz"] == ol["nnz"]
        assert np.array_equal(gl["rowptr"], ol["rowptr"]) and np.array_equal(gl["colind"], ol["colind"])
        assert rel_err(gl["val"], ol["val"]) <= 1e-12
        if l < nl - 1:
            assert np.array_equal(gl["agg"], ol["agg"])
            assert np.array_equal(gl["root"], ol["root"])
            assert np.array_equal(gl["p_rowptr"], ol["p_rowptr"])
            assert np.array_equal(gl["p_colind"], ol["p_colind"])
            assert rel_err(gl["p_val"], ol["p_val"]) <= 1e-12
            assert gl["omega"] == pytest.approx(ol["omega"], rel=1e-14)


@pytest.mark.parametrize("name", ["ragged", "cfg0", "line"])
def test_stages_match_oracle(B, O, name):
    case = CASES[name]()
    _, _, _, _, b, opc, gpc = setup_both(B, O, case, coarse_max=40)
    n = case.n
    rng = np.random.default_rng(7)
    v = rng.standard_normal(3 * n)
    assert rel_err(run_stage(B, gpc, B.bo_cpr_restrict, v, n), opc.restrict(v)) <= 1e-14
    rp = rng.standard_normal(n)
    assert rel_err(run_stage(B, gpc, B.bo_cpr_vcycle, rp, n), opc.vcycle(rp)) <= 1e-10
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_fstage, v, 3 * n), opc.fstage(v)) <= 1e-10
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * n), opc.apply(v)) <= 1e-10
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, b, 3 * n), opc.apply(b)) <= 1e-10


@pytest.mark.parametrize("kw", [dict(fpf=1), dict(ftype="bj"), dict(smoother="jacobi", sweeps=2),
                                dict(tile=(4, 4)), dict(tile=(5, 3)), dict(qi="diag"), dict(use_amg=0),
                                dict(csmoother="jacobi"), dict(csmoother="jacobi", sweeps=2)])
def test_cpr_variants_match_oracle(B, O, kw):
    case = ragged_case(seed=31)
    _, _, _, _, b, opc, gpc = setup_both(B, O, case, coarse_max=40, **kw)
    v = np.random.default_rng(8).standard_normal(3 * case.n)
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * case.n), opc.apply(v)) <= 1e-10


@pytest.mark.parametrize("dims", [(9, 7, 5), (8, 7, 5), (7, 6, 5), (5, 5, 5)])
def test_gauss_seidel_colour_pairs(B, O, dims):
    """The level-0 red-black sweeps read a colour-split copy of the pressure
    arrays, pairing cells 2h and 2h+1: grids with odd and even nx, ny and an
    odd cell count (an unpaired last cell) give the oracle's cycle."""
    nx, ny, nz = dims
    case = cg.tiny_case(nx, ny, nz, seed=51, step=0.01)
    _, _, _, _, b, opc, gpc = setup_both(B, O, case, coarse_max=40)
    n = case.n
    r = np.random.default_rng(12).standard_normal(n)
    assert rel_err(run_stage(B, gpc, B.bo_cpr_vcycle, r, n), opc.vcycle(r)) <= 1e-10
    v = np.random.default_rng(13).standard_normal(3 * n)
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * n), opc.apply(v)) <= 1e-10


@pytest.mark.parametrize("kw", [dict(), dict(precision="fp32"), dict(csmoother="jacobi", sweeps=2)])
def test_sliced_coarse_matrices_match_oracle(B, O, kw):
    """With sell_rows = 1 every coarse level operator, P and R is also kept
    sliced (SELL-64, one thread per row, entry-order sums), the form the cycle
    takes on levels of 2^20 rows and more: the V-cycle and the CPR
    application still match the oracle (FP32: its emulation)."""
    case = ragged_case(seed=71)
    _, _, _, _, b, opc, gpc = setup_both(B, O, case, coarse_max=40, sell_rows=1, **kw)
    tol = 1e-5 if kw.get("precision") == "fp32" else 1e-10
    n = case.n
    r = np.random.default_rng(14).standard_normal(n)
    assert rel_err(run_stage(B, gpc, B.bo_cpr_vcycle, r, n), opc.vcycle(r)) <= tol
    v = np.random.default_rng(15).standard_normal(3 * n)
    assert rel_err_parts(run_stage(B, gpc, B.bo_cpr_apply, v, 3 * n), opc.apply(v)) <= tol


def test_ilu_unit_responses_match_oracle(B, O):
    """The tiled block-ILU(0) factors seen through F applied to unit vectors
    (the first cell of a tile and a cell in a tile's interior): element-wise
    within 1e-13 of each entry's scale (the GPU forms the pivots in the
    diagonal form of ILU(0), the oracle in the IKJ form: same values, other
    rounding order)."""
    case = ragged_case(seed=41)
    _, _, _, _, _, opc, gpc = setup_both(B, O, case)
    for cell, comp in ((0, 0), (0, 2), (3 + case.nx * (4 + case.ny * 2), 1)):
        v = np.zeros(3 * case.n)
        v[3 * cell + comp] = 1.0
        x = run_stage(B, gpc, B.bo_cpr_fstage, v, 3 * case.n)
        ref = opc.fstage(v)
        assert np.all(np.abs(x - ref) <= 1e-13 * np.abs(ref).max())
        assert rel_err_parts(x, ref) <= 1e-12


@pytest.mark.parametrize("name", ["ragged", "cfg0"])
def test_fgmres_converges_like_oracle(B, O, name):
    case = CASES[name]()
    oinfo, ginfo, true_rel, xg, xo = solve_both(B, O, case)
    assert ginfo["converged"] and ginfo["status"] == B.BO_OK
    assert true_rel <= 1e-6
    assert ginfo["rel_residual"] == pytest.approx(true_rel, rel=1e-6, abs=1e-12)
    io = oinfo["iterations"]
    assert abs(ginfo["iterations"] - io) <= max(1, math.ceil(0.1 * io))


@pytest.mark.parametrize("orth", [1, 2])
@pytest.mark.parametrize("name", ["ragged", "cfg0"])
def test_fgmres_gram_schmidt_forms(B, O, name, orth):
    """CGS2 (orth 1) and CGS2 with each vector's second projection delayed one
    step (orth 2, the default) build the same Krylov basis up to rounding: the
    oracle's (CGS2) iteration count within 10 % and the true residual at the
    tolerance."""
    case = CASES[name]()
    oinfo, ginfo, true_rel, xg, xo = solve_both(B, O, case, fopts=B.bo_fgmres_default_opts(orth=orth))
    assert ginfo["converged"] and ginfo["status"] == B.BO_OK
    assert true_rel <= 1e-6
    assert ginfo["rel_residual"] == pytest.approx(true_rel, rel=1e-6, abs=1e-12)
    io = oinfo["iterations"]
    assert abs(ginfo["iterations"] - io) <= max(1, math.ceil(0.1 * io))


def test_delayed_request_falls_back_to_cgs2_exactly(B, O):
    """With m > 31 the delayed form (orth 2, the default request) is not
    available and the solver runs CGS2: the Hessenberg columns must then sum
    both projections, so the run equals an explicit orth = 1 run bit for
    bit."""
    import torch
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    xs, infos = [], []
    for orth in (2, 1):
        x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
        infos.append(B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(m=40, orth=orth)))
        xs.append(to_host(x))
    assert infos[0]["converged"] and infos[0]["iterations"] == infos[1]["iterations"]
    assert infos[0]["est_residual"] == infos[1]["est_residual"]
    assert np.array_equal(xs[0], xs[1])
    r = b - O.bsr_spmv(rp, ci, val, xs[0])
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)


@pytest.mark.parametrize("orth", [0, 1, 2])
def test_gmres_minimal_residual_after_k_steps(B, O, orth):
    """After k steps without restart, flexible GMRES with a fixed (linear)
    preconditioner returns the minimal residual over x0 + span(Z_k): a
    property of the Krylov space, not of the Gram-Schmidt form.  Each GPU form
    (MGS, CGS2, CGS2 with the second projection delayed one step) must reach
    the oracle's true residual after k steps; a wrong Hessenberg column or a
    lost basis vector leaves a larger one."""
    import torch
    case = ragged_case(seed=43)
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    for k in (1, 2, 3, 5, 8, 10):
        _, oi = O.fgmres(rp, ci, val, b, opc, maxit=k, rtol=1e-15)
        # (steps whose residual is still far above rounding: near 1e-15 the
        # minimal residual is no longer determined by the space alone)
        assert oi["rel_residual"] > 1e-11
        x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
        gi = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(orth=orth, maxit=k, rtol=1e-15))
        assert gi["iterations"] == oi["iterations"] == k
        r = b - O.bsr_spmv(rp, ci, val, to_host(x))
        rel = np.linalg.norm(r) / np.linalg.norm(b)
        assert rel == pytest.approx(oi["rel_residual"], rel=1e-6), (k, rel, oi["rel_residual"])


def test_fgmres_delayed_small_restart(B, O):
    """The delayed form across restarts (m = 3, m = 1) and when the iteration
    limit ends a cycle early."""
    import torch
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    for m in (3, 1):
        x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
        info = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(m=m, orth=2))
        assert info["converged"] and info["restarts"] >= 1
        r = b - O.bsr_spmv(rp, ci, val, to_host(x))
        assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)
    x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
    info = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(orth=2, maxit=2, rtol=1e-12))
    assert info["status"] == B.BO_NOT_CONVERGED and info["iterations"] == 2


def test_fgmres_mgs_option(B, O):
    import torch
    case = cg.make_case(0)
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
    info = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(orth=0))
    assert info["converged"]
    r = b - O.bsr_spmv(rp, ci, val, to_host(x))
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)


def test_fgmres_deterministic(B, O):
    import torch
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    xs = []
    for _ in range(2):
        x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
        B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x)
        xs.append(to_host(x))
    assert np.array_equal(xs[0], xs[1])


def test_fgmres_timing_option_keeps_result(B, O):
    """Timing records events around the SpMVs only: same iterates, one timed
    SpMV per iteration, a positive total."""
    import torch
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    xs, infos = [], []
    for t in (0, 1):
        x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
        infos.append(B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(timing=t)))
        xs.append(to_host(x))
    assert np.array_equal(xs[0], xs[1])
    assert infos[0]["spmv_calls"] == 0 and infos[0]["spmv_ms"] == 0.0
    assert infos[1]["spmv_calls"] == infos[1]["iterations"] and infos[1]["spmv_ms"] > 0.0


@pytest.mark.parametrize("kw", [dict(), dict(fpf=1), dict(smoother="jacobi", sweeps=2), dict(precision="fp32")])
def test_graph_replay_matches_eager(B, O, kw):
    """The preconditioner replayed as a HIP graph gives the eager result bit
    for bit, over many replays with eager work in between and after an update
    (which captures again)."""
    import torch
    c1, c2 = ragged_case(seed=61), ragged_case(seed=62)
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, c1, **kw)
    _, rp2, ci2, val2, b2 = oracle_system(O, c2)
    for rhs, update in ((b, None), (b, None), (b2, (rp2, ci2, val2)), (b2, None)):
        if update is not None:
            B.bo_cpr_update(gpc, device_bsr(B, *update))
        xs = []
        for g in (0, 1):
            x = torch.zeros(3 * c1.n, dtype=torch.float64, device="cuda")
            info = B.bo_fgmres_solve(gpc, gpc.A, to_dev(rhs), x, B.bo_fgmres_default_opts(graph=g))
            assert info["converged"]
            xs.append((to_host(x), info["iterations"]))
        assert xs[0][1] == xs[1][1] and np.array_equal(xs[0][0], xs[1][0])


def test_fgmres_small_restart_and_maxit(B, O):
    import torch
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
    info = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(m=3))
    assert info["converged"] and info["restarts"] >= 1
    x.zero_()
    info = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(maxit=2, rtol=1e-12))
    assert info["status"] == B.BO_NOT_CONVERGED and info["iterations"] == 2


def test_zero_rhs_gives_zero(B, O):
    import torch
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    x = torch.ones(3 * case.n, dtype=torch.float64, device="cuda")
    info = B.bo_fgmres_solve(gpc, gpc.A, torch.zeros_like(x), x)
    assert info["converged"] and float(x.abs().max()) == 0.0


def test_nonfinite_inputs_are_rejected(B, O):
    import torch
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    bad = b.copy()
    bad[5] = np.nan
    x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BoError) as e:
        B.bo_fgmres_solve(gpc, gpc.A, to_dev(bad), x)
    assert e.value.status == B.BO_ERR_NONFINITE
    v2 = val.copy()
    v2[3, 1, 1] = np.inf
    with pytest.raises(B.BoError) as e:
        B.bo_cpr_setup(device_bsr(B, rp, ci, v2), (case.nx, case.ny, case.nz))
    assert e.value.status == B.BO_ERR_NONFINITE


def test_singular_block_is_reported(B, O):
    case = ragged_case()
    P, rp, ci, val, b = oracle_system(O, case)
    v2 = val.copy()
    d = [e for e in range(rp[4], rp[5]) if ci[e] == 4][0]
    v2[d] = 0.0
    for ft in (B.BO_F_BJ,):
        with pytest.raises(B.BoError) as e:
            B.bo_cpr_setup(device_bsr(B, rp, ci, v2), (case.nx, case.ny, case.nz),
                           B.bo_cpr_default_opts(ftype=ft, use_amg=0))
        assert e.value.status == B.BO_ERR_SINGULAR_BLOCK


def test_pattern_mismatch_is_rejected(B, O):
    case = ragged_case()
    P, rp, ci, val, b = oracle_system(O, case)
    with pytest.raises(B.BoError) as e:
        B.bo_cpr_setup(device_bsr(B, rp, ci, val), (case.nx + 1, case.ny, case.nz))
    assert e.value.status == B.BO_ERR_INVALID_ARG


def test_update_equals_fresh_setup(B, O):
    """bo_cpr_update on a new Jacobian gives bit-identical results to a fresh
    bo_cpr_setup of that Jacobian (the setup is deterministic)."""
    import torch
    c1 = ragged_case(seed=51)
    c2 = ragged_case(seed=52)
    _, rp1, ci1, val1, b1 = oracle_system(O, c1)
    _, rp2, ci2, val2, b2 = oracle_system(O, c2)
    grid = (c1.nx, c1.ny, c1.nz)
    pc = B.bo_cpr_setup(device_bsr(B, rp1, ci1, val1), grid)
    B.bo_cpr_update(pc, device_bsr(B, rp2, ci2, val2))
    fresh = B.bo_cpr_setup(device_bsr(B, rp2, ci2, val2), grid)
    v = np.random.default_rng(9).standard_normal(3 * c2.n)
    a = run_stage(B, pc, B.bo_cpr_apply, v, 3 * c2.n)
    f = run_stage(B, fresh, B.bo_cpr_apply, v, 3 * c2.n)
    assert np.array_equal(a, f)
    x1 = torch.zeros(3 * c2.n, dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(x1)
    i1 = B.bo_fgmres_solve(pc, pc.A, to_dev(b2), x1)
    i2 = B.bo_fgmres_solve(fresh, fresh.A, to_dev(b2), x2)
    assert i1["iterations"] == i2["iterations"] and np.array_equal(to_host(x1), to_host(x2))


def test_failed_update_leaves_handle_unusable(B, O):
    import torch
    c1 = ragged_case(seed=53)
    _, rp, ci, val, b = oracle_system(O, c1)
    pc = B.bo_cpr_setup(device_bsr(B, rp, ci, val), (c1.nx, c1.ny, c1.nz))
    bad = val.copy()
    bad[7, 0, 0] = np.nan
    with pytest.raises(B.BoError):
        B.bo_cpr_update(pc, device_bsr(B, rp, ci, bad))
    x = torch.zeros(3 * c1.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BoError):
        B.bo_fgmres_solve(pc, pc.A, to_dev(b), x)
    B.bo_cpr_update(pc, device_bsr(B, rp, ci, val))
    assert B.bo_fgmres_solve(pc, pc.A, to_dev(b), x)["converged"]


def _singular_pair_system():
    """Two cells on a 2x1x1 grid with blocks [[I, -I], [-I, I]]: singular,
    range {(y, -y)}; its decoupled pressure block is [[1, -1], [-1, 1]]."""
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    I = np.eye(3)
    val = np.stack([I, -I, -I, I])
    return rp, ci, val


def test_singular_coarse_is_reported(B, O):
    """A singular coarsest pressure matrix: the hand-built pair, and the
    incompressible Jacobian without wells (a pure-Neumann pressure block,
    singular to rounding), fail the setup with BO_ERR_SINGULAR_COARSE, as
    the oracle's setup does."""
    from tests.test_oracle_solver import incompressible_no_well_case
    rp, ci, val = _singular_pair_system()
    with pytest.raises(B.BoError) as e:
        B.bo_cpr_setup(device_bsr(B, rp, ci, val), (2, 1, 1))
    assert e.value.status == B.BO_ERR_SINGULAR_COARSE
    c = incompressible_no_well_case()
    P, rp, ci, val, b = oracle_system(O, c)
    for cm in (192, 40, 10):
        with pytest.raises(B.BoError) as e:
            B.bo_cpr_setup(device_bsr(B, rp, ci, val), (c.nx, c.ny, c.nz), B.bo_cpr_default_opts(coarse_max=cm))
        assert e.value.status == B.BO_ERR_SINGULAR_COARSE, cm


@pytest.mark.parametrize("orth", [0, 1, 2])
def test_arnoldi_breakdown_is_reported(B, O, orth):
    """The singular pair with an inconsistent right-hand side (u, u) and an
    exact block-Jacobi F stage (1x1 tiles, no pressure stage): z_1 = v_1 lies
    in the null space, A z_1 = 0, the Hessenberg column is zero and the
    least-squares problem singular: BO_ERR_BREAKDOWN, x left at the initial
    guess."""
    import torch
    rp, ci, val = _singular_pair_system()
    A = device_bsr(B, rp, ci, val)
    pc = B.bo_cpr_setup(A, (2, 1, 1), B.bo_cpr_default_opts(use_amg=0, tile=(1, 1)))
    b = to_dev(np.array([1.0, 2.0, 3.0, 1.0, 2.0, 3.0]))
    x = torch.zeros(6, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BoError) as e:
        B.bo_fgmres_solve(pc, A, b, x, B.bo_fgmres_default_opts(orth=orth))
    assert e.value.status == B.BO_ERR_BREAKDOWN
    assert float(x.abs().max()) == 0.0
    # a consistent right-hand side (y, -y) converges in one step (happy breakdown)
    b2 = to_dev(np.array([1.0, 2.0, 3.0, -1.0, -2.0, -3.0]))
    info = B.bo_fgmres_solve(pc, A, b2, x, B.bo_fgmres_default_opts(orth=orth))
    assert info["converged"] and info["iterations"] == 1


def test_caller_allocator_serves_the_handle(B, O):
    """bo_cpr_setup with a caller allocator (here torch's caching allocator):
    every device buffer of the handle -- hierarchy, factors, operator copies,
    the Krylov basis allocated by the first solve, the condensed form's
    reduced system and inner handle -- comes from it and goes back to it
    by bo_cpr_destroy; results equal those of a handle on hipMalloc bit for
    bit."""
    import torch
    live = {}

    def alloc(nbytes, stream):
        t = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr, stream):
        live.pop(ptr)

    from tests.test_gpu_condensed import rate_case
    for case, grid, opts in ((ragged_case(), None, None),
                             (rate_case(), "dual", dict(condense=1, fpf=1, smoother=B.BO_SMOOTH_L1))):
        P, rp, ci, val, b = oracle_system(O, case)
        A = device_bsr(B, rp, ci, val)
        g = (case.nx, case.ny, case.nz, 1) if grid == "dual" else (case.nx, case.ny, case.nz)
        o = B.bo_cpr_default_opts(**(opts or {}))
        ref = B.bo_cpr_setup(A, g, o)
        pc = B.bo_cpr_setup(A, g, o, allocator=(alloc, free))
        assert len(live) > 0
        n_setup = len(live)
        xs = []
        for h in (ref, pc):
            x = torch.zeros(3 * P.rows, dtype=torch.float64, device="cuda")
            info = B.bo_fgmres_solve(h, A, to_dev(b), x)
            assert info["converged"]
            xs.append(to_host(x))
        assert np.array_equal(xs[0], xs[1])
        assert len(live) > n_setup          # the Krylov basis came from the caller too
        B.bo_cpr_update(pc, A)
        pc.close()
        assert len(live) == 0

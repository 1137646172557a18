"""GPU parity of the two-phase oil-water path (Section 2.2's model, 2x2-block
Jacobians, CPR of Section 3.2) against the two-phase oracle (the black-oil
oracle without the gas phase, its CPR through the 3x3 embedding):

  - Jacobian: pattern bit for bit, each block to 1e-12 of its own size, the
    right-hand side to 1e-12;
  - SpMV (ABI BSR and the handle's slot layout): integer data bit for bit,
    the Jacobian to 1e-12;
  - CPR: weights to 1e-15, hierarchy sizes equal, restriction 1e-14,
    V-cycle, F stage and the whole application per unknown (Po, Sw) to 1e-10
    for block Jacobi and tiled ILU(0), PF and FPF;
  - solves (FGMRES and BiCGSTAB): a true FP64 residual <= 1e-6 recomputed
    with the oracle's SpMV, the oracle's iteration count within 10 %;
  - the 200x200x50 (2M-cell) two-phase system at full size: Jacobian,
    preconditioner application and solve;
  - the options the path does not take are refused."""
import math

import numpy as np
import pytest

import bo_casegen as cg
from oracle import krylov as K
from oracle import twophase as T
from tests.gpu_util import matching_opts, rel_err, rel_err_parts, to_dev, to_host

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


def ragged2(seed=21):
    return cg.two_phase(cg.tiny_case(19, 13, 6, seed=seed, step=0.01,
                                     wells=[cg.Well(0, 0, 0, 5, "inj", "bhp", 3500.0),
                                            cg.Well(18, 12, 0, 5, "prod", "bhp", 2500.0),
                                            cg.Well(9, 6, 1, 4, "prod", "bhp", 2600.0)]))


CASES = {
    "ragged": lambda: ragged2(),
    "cfg0": lambda: cg.two_phase(cg.make_case(0)),
    "iid_nograv": lambda: cg.two_phase(cg.tiny_case(6, 5, 4, seed=8, noise_kind="iid", gravity=False, step=0.02)),
    "line": lambda: cg.two_phase(cg.tiny_case(9, 1, 1, seed=3, step=0.01,
                                              wells=[cg.Well(0, 0, 0, 0, "inj", "bhp", 3500.0)])),
}


def gpu_system(B, case):
    import torch
    p = B.problem_from_case(case)
    J, b = B.bo_jacobian2_bsr(p, to_dev(cg.state2(case.x_old)), to_dev(cg.state2(case.x_new)), case.dt)
    torch.cuda.synchronize()
    return J, b


def oracle_system(O, case):
    P = T.problem(O, case)
    rp, ci, val, R = T.jacobian(O, P)
    return P, rp, ci, val, -R


def device_bsr2(B, rp, ci, val):
    return B.DeviceBsr2(to_dev(np.asarray(rp, np.int32)), to_dev(np.asarray(ci, np.int32)),
                        to_dev(np.ascontiguousarray(val, np.float64).reshape(-1)))


def setup_both2(B, O, case, **kw):
    P, rp, ci, val, b = oracle_system(O, case)
    oo, bo_ = matching_opts(O, B, **kw)
    opc = T.Cpr2(O, P, rp, ci, val, opts=oo)
    gpc = B.bo_cpr2_setup(device_bsr2(B, rp, ci, val), (case.nx, case.ny, case.nz), bo_)
    return P, rp, ci, val, b, opc, gpc


def run(B, gpc, fn, v, m):
    import torch
    out = torch.zeros(m, dtype=torch.float64, device="cuda")
    fn(gpc, to_dev(v), out)
    return to_host(out)


@pytest.mark.parametrize("name", list(CASES))
def test_jacobian2_matches_oracle(B, O, name):
    case = CASES[name]()
    _, rp, ci, val, b = oracle_system(O, case)
    J, gb = gpu_system(B, case)
    assert np.array_equal(to_host(J.rowptr), rp) and np.array_equal(to_host(J.colind), ci)
    gval = to_host(J.val).reshape(-1, 2, 2)
    d = np.abs(gval - val).reshape(len(ci), 4).max(axis=1)
    size = np.maximum(np.abs(val).reshape(len(ci), 4).max(axis=1), 1e-300 * np.abs(val).max())
    assert np.all(d <= 1e-12 * size), int(np.argmax(d / size))
    assert rel_err(to_host(gb), b) <= 1e-12


def test_spmv2_integer_exact(B, O):
    import torch
    case = ragged2()
    P, rp, ci, val, b = oracle_system(O, case)
    n = case.n
    rng = np.random.default_rng(5)
    ival = rng.integers(-512, 513, size=(len(ci), 2, 2)).astype(np.float64)
    diag = ci == np.repeat(np.arange(n), np.diff(rp))
    for c in range(2):
        ival[diag, c, c] = 8192.0 + rng.integers(0, 512, size=int(diag.sum()))
    ix = rng.integers(-512, 513, size=2 * n).astype(np.float64)
    ref = T.spmv(O, rp, ci, ival, ix)
    A = device_bsr2(B, rp, ci, ival)
    y = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    B.bo_bsr2_spmv(A, 1.0, to_dev(ix), 0.0, y)
    assert np.array_equal(to_host(y), ref)
    pc = B.bo_cpr2_setup(A, (case.nx, case.ny, case.nz), B.bo_cpr_default_opts(use_amg=0, ftype=B.BO_F_BJ))
    y.zero_()
    B.bo_cpr_spmv(pc, 1.0, to_dev(ix), 0.0, y)
    assert np.array_equal(to_host(y), ref)
    # the Jacobian, y = 0.5 A x - 2 y0
    x = rng.standard_normal(2 * n)
    y0 = rng.standard_normal(2 * n)
    ref = 0.5 * T.spmv(O, rp, ci, val, x) - 2.0 * y0
    pc = B.bo_cpr2_setup(device_bsr2(B, rp, ci, val), (case.nx, case.ny, case.nz),
                         B.bo_cpr_default_opts(use_amg=0, ftype=B.BO_F_BJ))
    y = to_dev(y0)
    B.bo_cpr_spmv(pc, 0.5, to_dev(x), -2.0, y)
    assert rel_err_parts(to_host(y), ref, parts=2) <= 1e-12
    y = to_dev(y0)
    B.bo_bsr2_spmv(pc.A, 0.5, to_dev(x), -2.0, y)
    assert rel_err_parts(to_host(y), ref, parts=2) <= 1e-12


VARIANTS = [
    dict(),
    dict(fpf=1),
    dict(ftype="bj"),
    dict(tile=(3, 2)),
    dict(smoother="jacobi"),
    dict(tile=(8, 4), fpf=1),
]


@pytest.mark.parametrize("kw", VARIANTS, ids=lambda k: "-".join(f"{a}={b}" for a, b in k.items()) or "default")
@pytest.mark.parametrize("name", ["ragged", "cfg0"])
def test_cpr2_stages_match_oracle(B, O, name, kw):
    case = CASES[name]()
    P, rp, ci, val, b, opc, gpc = setup_both2(B, O, case, **kw)
    n = case.n
    assert np.abs(B.bo_cpr_copy_weights(gpc) - opc.weights()).max() <= 1e-15
    nl = opc.nlevels()
    assert B.bo_cpr_levels(gpc) == nl
    for l in range(nl):
        assert B.bo_cpr_level_info(gpc, l)["n"] == opc.level(l)["n"]
    rng = np.random.default_rng(13)
    v = rng.standard_normal(2 * n)
    assert rel_err(run(B, gpc, B.bo_cpr_restrict, v, n), opc.restrict(v)) <= 1e-14
    r = rng.standard_normal(n)
    assert rel_err(run(B, gpc, B.bo_cpr_vcycle, r, n), opc.vcycle(r)) <= 1e-10
    assert rel_err_parts(run(B, gpc, B.bo_cpr_fstage, v, 2 * n), opc.fstage(v), parts=2) <= 1e-10
    for vec in (v, b):
        assert rel_err_parts(run(B, gpc, B.bo_cpr_apply, vec, 2 * n), opc.apply(vec), parts=2) <= 1e-10


def _oracle_bicgstab(O, rp, ci, val, b, opc, **kw):
    return K.bicgstab(lambda x: T.spmv(O, rp, ci, val, x), opc.apply, b, **kw)


@pytest.mark.parametrize("solver", ["fgmres", "bicgstab"])
@pytest.mark.parametrize("name", ["ragged", "cfg0", "iid_nograv"])
def test_solves2_like_oracle(B, O, name, solver):
    import torch
    case = CASES[name]()
    P, rp, ci, val, b, opc, gpc = setup_both2(B, O, case)
    if solver == "fgmres":
        xo, oi = T.fgmres(O, rp, ci, val, b, opc)
        fn = B.bo_fgmres_solve2
    else:
        xo, oi = _oracle_bicgstab(O, rp, ci, val, b, opc)
        fn = B.bo_bicgstab_solve2
    x = torch.zeros(2 * case.n, dtype=torch.float64, device="cuda")
    gi = fn(gpc, gpc.A, to_dev(b), x)
    xg = to_host(x)
    true_rel = np.linalg.norm(b - T.spmv(O, rp, ci, val, xg)) / np.linalg.norm(b)
    io = oi["iterations"]
    print(f"{name} {solver}: iterations gpu {gi['iterations']} oracle {io}, true rel {true_rel:.2e}")
    assert gi["converged"] and gi["status"] == B.BO_OK and true_rel <= 1e-6
    assert gi["rel_residual"] == pytest.approx(true_rel, rel=1e-6, abs=1e-12)
    assert abs(gi["iterations"] - io) <= max(1 if solver == "fgmres" else 2, math.ceil(0.1 * io))


def test_fgmres2_iterates_match_oracle(B, O):
    """A fixed number of FGMRES steps (no restart): the minimal residual over
    the same Krylov space, so the true residuals agree."""
    import torch
    case = ragged2(seed=43)
    P, rp, ci, val, b, opc, gpc = setup_both2(B, O, case)
    for k in (1, 3, 6):
        _, oi = T.fgmres(O, rp, ci, val, b, opc, maxit=k, rtol=1e-15)
        x = torch.zeros(2 * case.n, dtype=torch.float64, device="cuda")
        gi = B.bo_fgmres_solve2(gpc, gpc.A, to_dev(b), x, B.bo_fgmres_default_opts(maxit=k, rtol=1e-15))
        assert gi["iterations"] == oi["iterations"] == k
        rel = np.linalg.norm(b - T.spmv(O, rp, ci, val, to_host(x))) / np.linalg.norm(b)
        assert rel == pytest.approx(oi["rel_residual"], rel=1e-6)


def test_update2_equals_fresh_setup(B, O):
    import torch
    c1 = cg.two_phase(cg.tiny_case(12, 9, 4, seed=31, step=0.02))
    c2 = cg.two_phase(cg.tiny_case(12, 9, 4, seed=32, step=0.03))
    _, rp, ci, v1, b1 = oracle_system(O, c1)
    _, rp2, ci2, v2, b2 = oracle_system(O, c2)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)
    A1, A2 = device_bsr2(B, rp, ci, v1), device_bsr2(B, rp, ci, v2)
    pc = B.bo_cpr2_setup(A1, (12, 9, 4))
    B.bo_cpr2_update(pc, A2)
    fresh = B.bo_cpr2_setup(A2, (12, 9, 4))
    v = np.random.default_rng(2).standard_normal(2 * c1.n)
    assert np.array_equal(run(B, pc, B.bo_cpr_apply, v, 2 * c1.n), run(B, fresh, B.bo_cpr_apply, v, 2 * c1.n))


def test_two_phase_refusals(B, O):
    import torch
    case = ragged2()
    P, rp, ci, val, b = oracle_system(O, case)
    A = device_bsr2(B, rp, ci, val)
    g = (case.nx, case.ny, case.nz)
    for kw in (dict(precision=B.BO_PREC_FP32), dict(condense=1), dict(smoother=B.BO_SMOOTH_L1)):
        with pytest.raises(B.BoError):
            B.bo_cpr2_setup(A, g, B.bo_cpr_default_opts(**kw))
    with pytest.raises(B.BoError):
        B.bo_cpr2_setup(A, (case.nx, case.ny, case.nz + 1))
    pc = B.bo_cpr2_setup(A, g)
    x = torch.zeros(2 * case.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BoError):  # the 3x3 solver entry points refuse a 2x2 handle
        B.bo_fgmres_solve(pc, pc.A, to_dev(b), x)
    with pytest.raises(B.BoError):
        B.bo_cpr_attach_nn(pc, B.Nn(cg.cnn_init(3)), to_dev(np.log(case.kx)))
    # fixed-rate wells and dual porosity are not part of the two-phase model here
    rate = cg.tiny_case(6, 5, 3, seed=4, wells=[cg.Well(0, 0, 0, 2, "inj", "wrat", 500.0)])
    with pytest.raises(B.BoError):
        B.bo_jacobian2_bsr(B.problem_from_case(rate), to_dev(cg.state2(rate.x_old)), to_dev(cg.state2(rate.x_new)),
                           rate.dt)


_BIG = {}


def big(O):
    if not _BIG:
        case = cg.two_phase(cg.make_case(2, 1))
        P, rp, ci, val, b = oracle_system(O, case)
        _BIG.update(case=case, P=P, rp=rp, ci=ci, val=val, b=b)
    return _BIG


def test_fullsize2_jacobian_and_apply(B, O):
    """The 200x200x50 two-phase system: Jacobian in full, and the default
    CPR's application per unknown against the oracle's."""
    d = big(O)
    case, rp, ci, val, b = d["case"], d["rp"], d["ci"], d["val"], d["b"]
    J, gb = gpu_system(B, case)
    assert np.array_equal(to_host(J.rowptr), rp) and np.array_equal(to_host(J.colind), ci)
    gval = to_host(J.val).reshape(-1, 2, 2)
    dd = np.abs(gval - val).reshape(len(ci), 4).max(axis=1)
    size = np.maximum(np.abs(val).reshape(len(ci), 4).max(axis=1), 1e-300 * np.abs(val).max())
    assert np.all(dd <= 1e-12 * size)
    assert rel_err(to_host(gb), b) <= 1e-12
    opc = T.Cpr2(O, d["P"], rp, ci, val)
    gpc = B.bo_cpr2_setup(J, (case.nx, case.ny, case.nz))
    assert B.bo_cpr_levels(gpc) == opc.nlevels()
    v = np.random.default_rng(9).standard_normal(2 * case.n)
    assert rel_err_parts(run(B, gpc, B.bo_cpr_apply, v, 2 * case.n), opc.apply(v), parts=2) <= 1e-10
    d["opc"] = opc


def test_fullsize2_solve(B, O):
    import torch
    d = big(O)
    case, rp, ci, val, b = d["case"], d["rp"], d["ci"], d["val"], d["b"]
    opc = d.get("opc") or T.Cpr2(O, d["P"], rp, ci, val)
    gpc = B.bo_cpr2_setup(device_bsr2(B, rp, ci, val), (case.nx, case.ny, case.nz))
    x = torch.zeros(2 * case.n, dtype=torch.float64, device="cuda")
    gi = B.bo_fgmres_solve2(gpc, gpc.A, to_dev(b), x)
    true_rel = np.linalg.norm(b - T.spmv(O, rp, ci, val, to_host(x))) / np.linalg.norm(b)
    xo, oi = T.fgmres(O, rp, ci, val, b, opc)
    io = oi["iterations"]
    print(f"2M cells two-phase: iterations gpu {gi['iterations']} oracle {io}, true rel {true_rel:.2e}")
    assert gi["converged"] and true_rel <= 1e-6
    assert abs(gi["iterations"] - io) <= max(1, math.ceil(0.1 * io))

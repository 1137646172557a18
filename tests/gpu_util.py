"""Helpers shared by the GPU parity tests: run the same seeded case through the
oracle (CPU, FP64) and through the HIP library (via its C ABI binding)."""
import numpy as np

import bo_casegen as cg


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.to(torch_dev())


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_system(O, case):
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    return P, rp, ci, val, -R


def device_bsr(B, rp, ci, val):
    import torch
    return B.DeviceBsr(to_dev(rp.astype(np.int32)), to_dev(ci.astype(np.int32)),
                       to_dev(np.asarray(val, dtype=np.float64).reshape(-1)))


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def rel_err_parts(a, b, parts=3):
    """The largest of the per-unknown relative errors: the Po, Sw and Sg
    entries of interleaved 3-vectors compared separately (their scales differ
    by orders of magnitude, so one norm over the whole vector would let the
    small ones drift)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    worst = 0.0
    for q in range(parts):
        bq = b[q::parts]
        den = np.linalg.norm(bq)
        num = np.linalg.norm(a[q::parts] - bq)
        if den == 0.0:
            if num != 0.0:
                return np.inf
            continue
        worst = max(worst, num / den)
    return worst


def matching_opts(O, B, ftype="tiled", fpf=0, tile=(8, 8), coarse_max=256, smoother="gs", sweeps=1,
                  use_amg=1, qi="block", theta=0.08, precision="fp64", csmoother="l1", sell_rows=0):
    """The same CPR configuration for the oracle and the library (sell_rows:
    the library's storage choice for large coarse matrices, not a change of
    the method; coarse_max 256, above the default 192, keeps the coarsest
    levels of the small workloads above the register Gauss-Jordan's 192 rows,
    so the global-memory elimination stays under test)."""
    oft = dict(tiled=O.F_ILU_TILED, bj=O.F_BJ)[ftype]
    bft = dict(tiled=B.BO_F_ILU_TILED, bj=B.BO_F_BJ)[ftype]
    osm = dict(gs=O.SMOOTH_GS, jacobi=O.SMOOTH_JACOBI)[smoother]
    bsm = dict(gs=B.BO_SMOOTH_GS, jacobi=B.BO_SMOOTH_JACOBI)[smoother]
    oqi = dict(block=O.QI_BLOCK, diag=O.QI_DIAG)[qi]
    bqi = dict(block=B.BO_QI_BLOCK, diag=B.BO_QI_DIAG)[qi]
    opr = dict(fp64=O.PREC_FP64, fp32=O.PREC_FP32, bf16=O.PREC_FP32_BF16)[precision]
    bpr = dict(fp64=B.BO_PREC_FP64, fp32=B.BO_PREC_FP32, bf16=B.BO_PREC_FP32_BF16)[precision]
    ocs = dict(jacobi=O.CSMOOTH_JACOBI, l1=O.CSMOOTH_L1)[csmoother]
    bcs = dict(jacobi=B.BO_CSMOOTH_JACOBI, l1=B.BO_CSMOOTH_L1)[csmoother]
    oo = O.cpr_opts(fpf=fpf, ftype=oft, tile=tile, theta=theta, coarse_max=coarse_max, smoother=osm,
                    sweeps=sweeps, use_amg=use_amg, qi_mode=oqi, precision=opr, csmoother=ocs)
    bo = B.bo_cpr_default_opts(fpf=fpf, ftype=bft, tile=tile, theta=theta, coarse_max=coarse_max,
                               smoother=bsm, sweeps=sweeps, use_amg=use_amg, qi_mode=bqi, precision=bpr,
                               csmoother=bcs, sell_rows=sell_rows)
    return oo, bo


def setup_both(B, O, case, **kw):
    """The oracle's and the library's CPR for the same case and options."""
    P, rp, ci, val, b = oracle_system(O, case)
    oo, bo_ = matching_opts(O, B, **kw)
    opc = O.Cpr(P, rp, ci, val, oo)
    A = device_bsr(B, rp, ci, val)
    gpc = B.bo_cpr_setup(A, (case.nx, case.ny, case.nz), bo_)
    return P, rp, ci, val, b, opc, gpc


def run_stage(B, gpc, fn, v, m):
    """Calls one stage entry point (fn(handle, in, out)) on a host vector."""
    import torch
    out = torch.zeros(m, dtype=torch.float64, device="cuda")
    fn(gpc, to_dev(v), out)
    return to_host(out)


def solve_both(B, O, case, fopts=None, **kw):
    """FGMRES with the oracle and with the library (fopts: its solver options,
    default: the library's); the GPU solution's true residual is measured with
    the oracle's SpMV."""
    import torch
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case, **kw)
    xo, oinfo = O.fgmres(rp, ci, val, b, opc)
    x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
    ginfo = B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x, fopts) if fopts is not None else B.bo_fgmres_solve(
        gpc, gpc.A, to_dev(b), x)
    xg = to_host(x)
    r = b - O.bsr_spmv(rp, ci, val, xg)
    return oinfo, ginfo, np.linalg.norm(r) / np.linalg.norm(b), xg, xo


def ragged_case(seed=21):
    """Spans several 8x8 tiles with ragged edges in x and y."""
    return cg.tiny_case(19, 13, 6, seed=seed, step=0.01,
                        wells=[cg.Well(0, 0, 0, 5, "inj", "bhp", 3500.0),
                               cg.Well(18, 12, 0, 5, "prod", "bhp", 2500.0),
                               cg.Well(9, 6, 1, 4, "prod", "bhp", 2600.0)])

"""Pins of the oracle's mixed-precision emulation (CPU only).

The mixed forms store the AMG hierarchy and the F stage's factors rounded to
FP32 (or the factors to BF16) and run those stages in float arithmetic, while
the decoupling, the residuals and the final sums stay FP64.  Nothing prints
what such a form must return, so the pins are: the BF16 rounding against
torch's own FP32 -> BF16 conversion, closeness of every FP32 stage to its FP64
counterpart within what the rounding allows (a dropped term, a wrong sign or a
wrong ordering in the float code would show as an O(1) difference), a float32
brute force of the block-Jacobi form, and solves reaching the true FP64
residual of 1e-6."""
import numpy as np
import pytest

import bo_casegen as cg


def system(O, case):
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    return P, rp, ci, val, -R


def ragged():
    return cg.tiny_case(19, 13, 6, seed=21, step=0.01,
                        wells=[cg.Well(0, 0, 0, 5, "inj", "bhp", 3500.0),
                               cg.Well(18, 12, 0, 5, "prod", "bhp", 2500.0)])


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_bf16_round_matches_torch(oracle_lib):
    import torch
    O = oracle_lib
    rng = np.random.default_rng(3)
    vals = (rng.standard_normal(4000) * np.exp2(rng.integers(-40, 40, 4000))).astype(np.float32)
    # exact ties: 1 + 2^-8 (to 1), 1 + 3 * 2^-8 (to 1 + 2^-6), and negatives
    ties = np.array([1 + 2**-8, 1 + 3 * 2**-8, -(1 + 2**-8), 3 * 2**-20 * (1 + 2**-8)], dtype=np.float32)
    vals = np.concatenate([vals, ties, np.float32([0.0, -0.0])])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    ours = np.array([O.bf16_round(v) for v in vals], dtype=np.float32)
    assert np.array_equal(ours, ref)
    assert O.bf16_round(1 + 2**-8) == 1.0 and O.bf16_round(1 + 3 * 2**-8) == 1 + 2**-6


@pytest.mark.parametrize("ftype", ["tiled", "natural", "rb", "bj"])
def test_fp32_fstage_close_to_fp64(oracle_lib, ftype):
    O = oracle_lib
    ft = dict(tiled=O.F_ILU_TILED, natural=O.F_ILU_NATURAL, rb=O.F_ILU_RB, bj=O.F_BJ)[ftype]
    case = ragged()
    P, rp, ci, val, b = system(O, case)
    r = np.random.default_rng(4).standard_normal(3 * case.n)
    x64 = O.Cpr(P, rp, ci, val, ftype=ft).fstage(r)
    x32 = O.Cpr(P, rp, ci, val, ftype=ft, precision=O.PREC_FP32).fstage(r)
    xbf = O.Cpr(P, rp, ci, val, ftype=ft, precision=O.PREC_FP32_BF16).fstage(r)
    e32, ebf = rel(x32, x64), rel(xbf, x64)
    assert 0.0 < e32 <= 1e-5, e32
    # BF16 factors carry 8 significant bits: error of order 2^-9 per entry
    assert e32 < ebf <= 2.0**-5, ebf


def test_fp32_fstage_diagonal_form_equals_ikj_in_float(oracle_lib):
    """In the FP32 form the F stage is the diagonal ILU(0) form; on a grid
    whose ILU is exact (one line of cells), F(A x) must return x to float
    accuracy times the conditioning of the 3x3 blocks (pressure and saturation
    columns differ by about four orders of magnitude), which a wrong term in
    either sweep would break by O(1)."""
    O = oracle_lib
    case = cg.tiny_case(9, 1, 1, seed=3, step=0.01, wells=[cg.Well(0, 0, 0, 0, "inj", "bhp", 3500.0)])
    P, rp, ci, val, b = system(O, case)
    x = np.random.default_rng(6).standard_normal(3 * case.n)
    y = O.bsr_spmv(rp, ci, val, x)
    assert rel(O.Cpr(P, rp, ci, val, ftype=O.F_ILU_NATURAL).fstage(y), x) <= 1e-10
    pc = O.Cpr(P, rp, ci, val, ftype=O.F_ILU_NATURAL, precision=O.PREC_FP32)
    assert rel(pc.fstage(y), x) <= 1e-3


def test_fp32_vcycle_close_to_fp64(oracle_lib):
    O = oracle_lib
    case = ragged()
    P, rp, ci, val, b = system(O, case)
    bp = np.random.default_rng(7).standard_normal(case.n)
    for sm in (O.SMOOTH_GS, O.SMOOTH_JACOBI):
        v64 = O.Cpr(P, rp, ci, val, smoother=sm, coarse_max=40).vcycle(bp)
        v32 = O.Cpr(P, rp, ci, val, smoother=sm, coarse_max=40, precision=O.PREC_FP32).vcycle(bp)
        e = rel(v32, v64)
        assert 0.0 < e <= 1e-5, (sm, e)


def test_fp32_block_jacobi_brute_force(oracle_lib):
    """F-only CPR with block Jacobi in FP32: z_i = float(A_ii^{-1}) float(v_i)
    in float arithmetic, returned exactly; recomputed here with numpy float32."""
    O = oracle_lib
    case = cg.tiny_case(5, 4, 3, seed=9, step=0.01)
    P, rp, ci, val, b = system(O, case)
    v = np.random.default_rng(8).standard_normal(3 * case.n)
    z = O.Cpr(P, rp, ci, val, ftype=O.F_BJ, use_amg=0, precision=O.PREC_FP32).apply(v)
    ref = np.empty(3 * case.n)
    for i in range(case.n):
        e = [k for k in range(rp[i], rp[i + 1]) if ci[k] == i][0]
        inv = np.linalg.inv(val[e]).astype(np.float32)
        vi = v[3 * i:3 * i + 3].astype(np.float32)
        for q in range(3):
            acc = inv[q, 0] * vi[0]
            acc = np.float32(acc + inv[q, 1] * vi[1])
            acc = np.float32(acc + inv[q, 2] * vi[2])
            ref[3 * i + q] = float(acc)
    # the pivot inverses may differ in the last FP64 bit before rounding
    assert rel(z, ref) <= 1e-6


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("fpf", [0, 1])
def test_mixed_solve_reaches_fp64_residual(oracle_lib, prec, fpf):
    O = oracle_lib
    p = dict(fp32=O.PREC_FP32, bf16=O.PREC_FP32_BF16)[prec]
    case = ragged()
    P, rp, ci, val, b = system(O, case)
    x64, i64 = O.fgmres(rp, ci, val, b, O.Cpr(P, rp, ci, val, fpf=fpf))
    x, info = O.fgmres(rp, ci, val, b, O.Cpr(P, rp, ci, val, fpf=fpf, precision=p))
    r = b - O.bsr_spmv(rp, ci, val, x)
    assert info["converged"] and np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)
    assert abs(info["iterations"] - i64["iterations"]) <= 2

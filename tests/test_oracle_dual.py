"""Pins of the oracle's dual-porosity model and fixed-rate wells (CPU only):
the pattern, the transfer coefficient's closed form, the Jacobian against
central finite differences in every column, conservation of the fluxes and
transfers, the rate constraint's p_h derivative in closed form, and the
single-porosity limit of a vanishing transfer."""
import dataclasses

import numpy as np
import pytest

import bo_casegen as cg

WELLS = [cg.Well(0, 0, 0, 3, "inj", "wrat", 500.0), cg.Well(5, 4, 0, 3, "prod", "lrat", 400.0),
         cg.Well(2, 2, 1, 2, "prod", "bhp", 2500.0)]


def case(**kw):
    return cg.make_dual_case(6, 5, 4, seed=3, wells=WELLS, **kw)


def test_pattern(oracle_lib):
    O = oracle_lib
    c = case()
    P = O.Problem(c)
    rp, ci = O.pattern(P)
    n = c.n
    assert P.rows == 2 * n + 2 and len(rp) == P.rows + 1
    for r in range(P.rows):
        cols = ci[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cols) > 0)
        if n <= r < 2 * n:
            assert list(cols) == [r - n, r]
        elif r < n:
            assert n + r in cols
    # well rows: perforated fracture cells then the row itself
    w0 = 2 * n
    assert list(ci[rp[w0]:rp[w0 + 1]]) == [0 + 6 * (0 + 5 * k) for k in range(4)] + [w0]


def test_transfer_closed_form(oracle_lib):
    O = oracle_lib
    c = case()
    P = O.Problem(c)
    sigma = 4.0 * 3 / 100.0
    assert c.sigma == pytest.approx(sigma, rel=1e-15)
    for g in (0, 17, 119):
        assert O.transfer(P, g) == pytest.approx(0.001127 * sigma * c.km[g] * 50 * 50 * 10, rel=1e-14)


def test_jacobian_matches_finite_differences(oracle_lib):
    O = oracle_lib
    c = case()
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    A = O.bsr_to_dense(rp, ci, val)
    x = c.x_new
    worst = 0.0
    for j in range(len(x)):
        if j >= 3 * 2 * c.n and j % 3 != 0:
            continue  # dummy unknowns of the well rows: identity, checked below
        h = 1e-6 * max(abs(x[j]), 1.0) if j % 3 == 0 else 1e-7
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (O.residual(P, x_new=xp) - O.residual(P, x_new=xm)) / (2 * h)
        scale = max(np.abs(A[:, j]).max(), 1e-300)
        worst = max(worst, np.abs(fd - A[:, j]).max() / scale)
    assert worst <= 1e-6, worst
    for w in range(2):
        r = 2 * c.n + w
        blk = val[[e for e in range(rp[r], rp[r + 1]) if ci[e] == r][0]]
        assert blk[1, 1] == 1.0 and blk[2, 2] == 1.0 and not blk[1:, 0].any()


def test_fluxes_and_transfers_conserve_mass(oracle_lib):
    O = oracle_lib
    c = case()
    P = O.Problem(c)
    F = O.flux_residual(P)
    assert len(F) == 3 * 2 * c.n
    for comp in range(3):
        tot = F[comp::3].sum()
        assert abs(tot) <= 1e-12 * np.abs(F[comp::3]).sum()
    # the transfer alone: matrix rows are minus their fracture's transfer part
    c0 = dataclasses.replace(c, km=np.zeros(c.n))
    F0 = O.flux_residual(O.Problem(c0))
    assert not F0[3 * c.n:].any()
    assert np.allclose((F - F0)[:3 * c.n], -F[3 * c.n:], rtol=1e-12, atol=1e-12 * np.abs(F).max())


def test_rate_constraint_bhp_derivative(oracle_lib):
    """d(rate residual)/d p_h = sum over perforations of WI lambda b, with the
    injector's total mobility and b_w, the producer's oil + water."""
    O = oracle_lib
    c = case()
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    f = c.fluid
    for w, r in ((0, 2 * c.n), (1, 2 * c.n + 1)):
        W = WELLS[w]
        blk = val[[e for e in range(rp[r], rp[r + 1]) if ci[e] == r][0]]
        ref = 0.0
        for k in range(W.k_top, W.k_bot + 1):
            g = W.i + c.nx * (W.j + c.ny * k)
            p, sw, sg = c.x_new[3 * g:3 * g + 3]
            kr = O.relperm(P, sw, sg)
            bw = 1.0 / (f["Bw0"] * (1 - f["cw"] * (p - f["p_ref"])))
            bo = 1.0 / (f["Bo0"] * (1 - f["co"] * (p - f["p_ref"])))
            wi = O.well_index(P, g)
            if W.kind == "inj":
                lt = kr["krw"] / f["mu_w"] + kr["kro"] / f["mu_o"] + kr["krg"] / f["mu_g"]
                ref += wi * lt * bw
            else:
                ref -= wi * (kr["kro"] / f["mu_o"] * bo + kr["krw"] / f["mu_w"] * bw)
        assert blk[0, 0] == pytest.approx(ref, rel=1e-12)


def test_vanishing_transfer_reduces_to_single_porosity(oracle_lib):
    O = oracle_lib
    wells = [cg.Well(0, 0, 0, 3, "inj", "bhp", 3500.0), cg.Well(5, 4, 0, 3, "prod", "bhp", 2500.0)]
    c = cg.make_dual_case(6, 5, 4, seed=3, wells=wells)
    c = dataclasses.replace(c, km=np.zeros(c.n))
    rp, ci, val, R = O.jacobian(O.Problem(c))
    n = c.n
    s = dataclasses.replace(c, dual=False, km=None, phim=None, sigma=0.0,
                            x_old=c.x_old[:3 * n], x_new=c.x_new[:3 * n])
    rp1, ci1, val1, R1 = O.jacobian(O.Problem(s))
    assert np.array_equal(R[:3 * n], R1)
    for r in range(n):
        cols = [e for e in range(rp[r], rp[r + 1]) if ci[e] < n]
        assert np.array_equal(ci[cols], ci1[rp1[r]:rp1[r + 1]])
        assert np.array_equal(val[cols], val1[rp1[r]:rp1[r + 1]])


@pytest.mark.parametrize("ftype", ["bj", "natural", "tiled"])
def test_cpr_on_dual_system_matches_dense_solve(oracle_lib, ftype):
    """CPR with the pressure system over the cell rows only (the well rows stay
    out of A_pp) and an l1-Jacobi level-0 smoother (the dual graph has no grid
    colouring): FGMRES reaches the exact solution of a tiny system."""
    O = oracle_lib
    c = cg.make_dual_case(4, 3, 3, seed=5, wells=[cg.Well(0, 0, 0, 2, "inj", "wrat", 300.0),
                                                   cg.Well(3, 2, 0, 2, "prod", "lrat", 250.0)])
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    b = -R
    ft = dict(bj=O.F_BJ, natural=O.F_ILU_NATURAL, tiled=O.F_ILU_TILED)[ftype]
    pc = O.Cpr(P, rp, ci, val, ftype=ft, smoother=O.SMOOTH_L1, npr=P.ncell, coarse_max=10, tile=(2, 2))
    assert pc.nlevels() >= 2 and pc.npr == 2 * c.n
    x, info = O.fgmres(rp, ci, val, b, pc, rtol=1e-12)
    A = O.bsr_to_dense(rp, ci, val)
    xs = O.dense_solve(A, b)
    cond = np.linalg.cond(A)
    assert info["converged"]
    assert np.linalg.norm(x - xs) <= cond * 1e-12 * np.linalg.norm(xs)
    # the well rows are outside A_pp: restricting a vector that is zero on the
    # cell rows gives zero
    v = np.zeros(3 * P.rows)
    v[3 * 2 * c.n:] = 1.0
    assert not pc.restrict(v).any()


def test_tiled_ilu_with_one_tile_equals_natural_order(oracle_lib):
    """One tile covering the grid orders the dual system as the natural order
    does (fracture cells, then matrix cells); without well rows nothing is
    dropped, so both F stages agree to rounding."""
    O = oracle_lib
    c = cg.make_dual_case(5, 4, 3, seed=5, wells=[cg.Well(0, 0, 0, 2, "inj", "bhp", 3500.0)])
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    t = O.Cpr(P, rp, ci, val, ftype=O.F_ILU_TILED, tile=(8, 8), use_amg=0)
    nat = O.Cpr(P, rp, ci, val, ftype=O.F_ILU_NATURAL, use_amg=0)
    v = np.random.default_rng(3).standard_normal(3 * P.rows)
    a, b = t.fstage(v), nat.fstage(v)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
    # with a fixed-rate well the tiled form drops the well's couplings
    c2 = cg.make_dual_case(5, 4, 3, seed=5, wells=[cg.Well(0, 0, 0, 2, "inj", "wrat", 300.0)])
    P2 = O.Problem(c2)
    rp2, ci2, val2, _ = O.jacobian(P2)
    v2 = np.random.default_rng(4).standard_normal(3 * P2.rows)
    a2 = O.Cpr(P2, rp2, ci2, val2, ftype=O.F_ILU_TILED, tile=(8, 8), use_amg=0).fstage(v2)
    b2 = O.Cpr(P2, rp2, ci2, val2, ftype=O.F_ILU_NATURAL, use_amg=0).fstage(v2)
    assert np.linalg.norm(a2 - b2) > 1e-8 * np.linalg.norm(b2)


# ---- exact elimination of the matrix cells ----------------------------------------
def _dense_schur(O, c, rp, ci, val):
    """The plain definition: S = D_KK - D_KM D_MM^-1 D_MK on the dense matrix,
    K = fracture and well unknowns, M = matrix unknowns (numpy's LU solve)."""
    D = O.bsr_to_dense(rp, ci, val)
    n = c.n
    mu = np.arange(3 * n, 6 * n)
    ku = np.concatenate([np.arange(3 * n), np.arange(6 * n, D.shape[0])])
    return D, ku, mu, D[np.ix_(ku, ku)] - D[np.ix_(ku, mu)] @ np.linalg.solve(D[np.ix_(mu, mu)], D[np.ix_(mu, ku)])


def test_condensed_operator_is_the_schur_complement(oracle_lib):
    O = oracle_lib
    c = case()
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    cond = O.Condensed(P, rp, ci, val, ftype=O.F_BJ, smoother=O.SMOOTH_L1)
    D, ku, mu, S = _dense_schur(O, c, rp, ci, val)
    Sc = O.bsr_to_dense(cond.srp, cond.sci, cond.sval)
    assert np.linalg.norm(Sc - S) <= 1e-12 * np.linalg.norm(S)
    # the reduced pattern is the single-porosity one of the same grid and wells
    rrp, rci = O.pattern(cond.red_prob)
    assert np.array_equal(rrp, cond.srp) and np.array_equal(rci, cond.sci)
    # right-hand side and back-substitution against the dense elimination
    b = -R
    br = cond.reduce(b)
    ref = b[ku] - D[np.ix_(ku, mu)] @ np.linalg.solve(D[np.ix_(mu, mu)], b[mu])
    assert np.linalg.norm(br - ref) <= 1e-12 * np.linalg.norm(ref)
    xk = np.linalg.solve(S, br)
    x = cond.back(b, xk)
    xd = np.linalg.solve(D, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert np.linalg.norm(b - D @ x) <= 1e-10 * np.linalg.norm(b)


def test_condensed_cpr_fgmres_solves_the_full_system(oracle_lib):
    O = oracle_lib
    c = cg.make_dual_case(12, 10, 6, seed=5, wells=[cg.Well(1, 1, 0, 5, "inj", "wrat", 900.0),
                                                     cg.Well(10, 8, 0, 5, "prod", "lrat", 800.0),
                                                     cg.Well(6, 2, 1, 4, "prod", "bhp", 2500.0)])
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    b = -R
    cond = O.Condensed(P, rp, ci, val, ftype=O.F_ILU_TILED, smoother=O.SMOOTH_L1, fpf=1, coarse_max=40)
    x, info = O.condensed_fgmres(rp, ci, val, b, cond)
    assert info["converged"] and info["passes"] == 1
    r = b - O.bsr_spmv(rp, ci, val, x)
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)
    xd = O.dense_solve(O.bsr_to_dense(rp, ci, val), b)
    assert np.linalg.norm(x - xd) <= 1e-3 * np.linalg.norm(xd)
    # the preconditioner of the full system: an exact solve of the matrix rows
    # for any input (its output satisfies every matrix-cell equation)
    v = np.random.default_rng(4).standard_normal(len(b))
    z = cond.apply(v)
    Az = O.bsr_spmv(rp, ci, val, z)
    n = c.n
    assert np.linalg.norm((Az - v)[3 * n:6 * n]) <= 1e-12 * np.linalg.norm(v[3 * n:6 * n])

"""Pins of the oracle's scalar pressure-system solve (GMRES(30) with RAS and
ILU(0) subdomain solves, the paper's linear-solver run) to what the
definitions fix:

  - the slot SpMV against the matrix assembled entry by entry;
  - each subdomain's factors: unit-lower L and upper U on the subdomain's
    pattern with (L U)_ij = a_ij on that pattern (the definition of ILU(0));
    on the 7-point graph only the diagonal differs from A (no fill, no
    triangles);
  - RAS on a line of cells (tridiagonal subdomain matrices, where ILU(0) is
    the exact LU) against the dense formula sum_t R~_t^T A_t^{-1} R_t;
  - RAS in 3-D: each tile's own cells take the local ILU solve of the
    extended tile, and with one tile and no overlap it is global ILU(0);
  - GMRES: after k steps from x0 = 0 its residual is the minimum over the
    preconditioned Krylov space (least squares on an explicit basis), an
    exact preconditioner solves in one step, a restart continues from the
    true residual, and with rtol 0 it runs exactly maxit steps.
"""
import numpy as np
import pytest

import bo_casegen as cg
from oracle import pressure as PR


def dense(case):
    n, nx, ny, nz = case.n, case.nx, case.ny, case.nz
    A = np.zeros((n, n))
    off = [-nx * ny, -nx, -1, 0, 1, nx, nx * ny]
    for g in range(n):
        i, j, k = g % nx, (g // nx) % ny, g // (nx * ny)
        ok = [k > 0, j > 0, i > 0, True, i < nx - 1, j < ny - 1, k < nz - 1]
        for s in range(7):
            if ok[s]:
                A[g, g + off[s]] = case.coef[s, g]
    return A


def test_spmv_against_dense():
    c = cg.pressure_case(7, 5, 4, seed=3)
    x = np.random.default_rng(1).standard_normal(c.n)
    assert np.allclose(PR.spmv(c.nx, c.ny, c.nz, c.coef, x), dense(c) @ x, rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("tile,overlap", [((3, 2), 0), ((3, 2), 1), ((4, 4), 2)])
def test_subdomain_factors_are_ilu0(tile, overlap):
    c = cg.pressure_case(9, 7, 3, seed=4)
    A = dense(c)
    ras = PR.Ras(c.nx, c.ny, c.nz, c.coef, tile, overlap)
    owned = np.zeros(c.n, int)
    for t in range(ras.tiles()):
        cell, own, rp, ci, lu = ras.tile(t)
        owned[cell[own]] += 1
        n = len(cell)
        Al = A[np.ix_(cell, cell)]
        L, U = np.eye(n), np.zeros((n, n))
        pat = np.zeros((n, n), bool)
        for i in range(n):
            for e in range(rp[i], rp[i + 1]):
                j = ci[e]
                pat[i, j] = True
                if j < i:
                    L[i, j] = lu[e]
                else:
                    U[i, j] = lu[e]
        assert np.array_equal(pat, Al != 0.0)
        M = L @ U
        assert np.abs(M - Al)[pat].max() <= 1e-12 * np.abs(Al).max()
        # only the diagonal of U differs from A's (no fill on the 7-point graph)
        off = pat & ~np.eye(n, dtype=bool) & np.triu(np.ones((n, n), bool))
        assert np.array_equal(U[off], Al[off])
    assert np.all(owned == 1)   # the tiles' own cells partition the grid


@pytest.mark.parametrize("overlap", [0, 1, 3])
def test_ras_line_against_dense_formula(overlap):
    c = cg.pressure_case(23, 1, 1, seed=6)
    A = dense(c)
    ras = PR.Ras(c.nx, c.ny, c.nz, c.coef, (5, 1), overlap)
    r = np.random.default_rng(2).standard_normal(c.n)
    z = np.zeros(c.n)
    for t in range((c.nx + 4) // 5):
        i0, i1 = 5 * t, min(5 * t + 5, c.nx)
        e0, e1 = max(i0 - overlap, 0), min(i1 + overlap, c.nx)
        loc = np.arange(e0, e1)
        zl = np.linalg.solve(A[np.ix_(loc, loc)], r[loc])
        z[i0:i1] = zl[i0 - e0:i1 - e0]
    assert np.allclose(ras.apply(r), z, rtol=1e-12, atol=1e-14 * np.abs(z).max())


def test_ras_3d_tiles_and_global_ilu():
    c = cg.pressure_case(8, 6, 4, seed=8)
    A = dense(c)
    r = np.random.default_rng(3).standard_normal(c.n)
    ras = PR.Ras(c.nx, c.ny, c.nz, c.coef, (3, 4), 1)
    z = ras.apply(r)
    for t in range(ras.tiles()):
        cell, own, rp, ci, lu = ras.tile(t)
        n = len(cell)
        L, U = np.eye(n), np.zeros((n, n))
        for i in range(n):
            for e in range(rp[i], rp[i + 1]):
                (L if ci[e] < i else U)[i, ci[e]] = lu[e]
        zl = np.linalg.solve(U, np.linalg.solve(L, r[cell]))
        assert np.allclose(z[cell[own]], zl[own], rtol=1e-12, atol=1e-14 * np.abs(zl).max())
    # one tile, no overlap: global ILU(0) of A, whose product matches A on its pattern
    one = PR.Ras(c.nx, c.ny, c.nz, c.coef, (c.nx, c.ny), 0)
    cell, own, rp, ci, lu = one.tile(0)
    assert np.array_equal(cell, np.arange(c.n)) and own.all()
    L, U = np.eye(c.n), np.zeros((c.n, c.n))
    for i in range(c.n):
        for e in range(rp[i], rp[i + 1]):
            (L if ci[e] < i else U)[i, ci[e]] = lu[e]
    assert np.abs(L @ U - A)[A != 0].max() <= 1e-12 * np.abs(A).max()
    assert np.allclose(one.apply(r), np.linalg.solve(L @ U, r), rtol=1e-10)


def test_gmres_minimal_residual_over_krylov_space():
    c = cg.pressure_case(8, 6, 4, seed=9)
    A = dense(c)
    ras = PR.Ras(c.nx, c.ny, c.nz, c.coef, (4, 3), 1)
    Mi = np.stack([ras.apply(e) for e in np.eye(c.n)], axis=1)   # M^{-1} as a matrix
    b = c.b
    for k in (1, 2, 4, 7):
        x, info = PR.gmres(lambda v: A @ v, ras.apply, b, m=30, maxit=k)
        assert info["iterations"] == k
        # explicit basis of span{M^{-1} (A M^{-1})^i b}, orthonormalised for stability
        K = [b]
        for _ in range(k - 1):
            K.append(A @ (Mi @ K[-1]))
        Q, _ = np.linalg.qr(np.stack(K, axis=1))
        Z = Mi @ Q
        y, *_ = np.linalg.lstsq(A @ Z, b, rcond=None)
        best = np.linalg.norm(b - A @ (Z @ y))
        got = np.linalg.norm(b - A @ x)
        assert got == pytest.approx(best, rel=1e-8), k


def test_gmres_exact_preconditioner_restart_and_fixed_count():
    c = cg.pressure_case(6, 5, 3, seed=10)
    A = dense(c)
    b = c.b
    x, info = PR.gmres(lambda v: A @ v, lambda v: np.linalg.solve(A, v), b, maxit=5, rtol=1e-12)
    assert info["converged"] and info["iterations"] == 1
    ras = PR.Ras(c.nx, c.ny, c.nz, c.coef, (3, 3), 1)
    mv = lambda v: A @ v
    # GMRES(4) for 8 steps = GMRES(4) for 4 steps, then again from its iterate
    x8, i8 = PR.gmres(mv, ras.apply, b, m=4, maxit=8)
    x4, _ = PR.gmres(mv, ras.apply, b, m=4, maxit=4)
    x44, _ = PR.gmres(mv, ras.apply, b, x0=x4, m=4, maxit=4)
    assert i8["iterations"] == 8 and i8["restarts"] == 1
    assert np.allclose(x8, x44, rtol=1e-12, atol=1e-12 * np.abs(x8).max())
    # rtol 0: a fixed count of steps, 90 as in the paper's run
    x, info = PR.solve(c, tile=(3, 3), overlap=1, m=30, maxit=90)
    assert info["iterations"] == 90 and info["restarts"] == 2
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)

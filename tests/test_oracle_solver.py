"""Pins of the oracle's linear algebra (CPU only): SpMV against dense products,
dense LU against LAPACK, the ILU(0) defining property, AMG invariants, the
Arnoldi relation, finite termination and exactness special cases."""
import numpy as np
import pytest

import bo_casegen as cg


def small_system(O, nx=4, ny=4, nz=3, seed=5, **kw):
    c = cg.tiny_case(nx, ny, nz, seed=seed, **kw)
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    return c, P, rp, ci, val, -R


def test_spmv_integer_exact(oracle_lib):
    O = oracle_lib
    c = cg.tiny_case(5, 4, 3)
    rp, ci = O.pattern(O.Problem(c))
    rng = np.random.default_rng(1)
    val = rng.integers(-1024, 1025, size=(len(ci), 3, 3)).astype(np.float64)
    x = rng.integers(-1024, 1025, size=3 * c.n).astype(np.float64)
    y = O.bsr_spmv(rp, ci, val, x)
    A = O.bsr_to_dense(rp, ci, val)
    assert np.array_equal(y, A @ x)


def test_spmv_axpby(oracle_lib):
    O = oracle_lib
    c = cg.tiny_case(5, 4, 3)
    rp, ci = O.pattern(O.Problem(c))
    rng = np.random.default_rng(2)
    val = rng.standard_normal((len(ci), 3, 3))
    x = rng.standard_normal(3 * c.n)
    y0 = rng.standard_normal(3 * c.n)
    y = O.bsr_spmv(rp, ci, val, x, alpha=-0.5, beta=2.0, y=y0)
    A = O.bsr_to_dense(rp, ci, val)
    ref = -0.5 * (A @ x) + 2.0 * y0
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)


def test_dense_solve_matches_lapack(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(3)
    for n in (1, 5, 40):
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        b = rng.standard_normal(n)
        x = O.dense_solve(A, b)
        assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-12 * np.linalg.norm(x)


def dense_M_of_fstage(pc, n3):
    Minv = np.zeros((n3, n3))
    for j in range(n3):
        e = np.zeros(n3); e[j] = 1.0
        Minv[:, j] = pc.fstage(e)
    return np.linalg.inv(Minv)


@pytest.mark.parametrize("ftype", ["natural", "rb", "tiled"])
def test_ilu0_defining_property(oracle_lib, ftype):
    """ILU(0): the product L U equals A on the block pattern (within tiles for
    the tiled form, where couplings between tiles are dropped)."""
    O = oracle_lib
    ft = dict(natural=O.F_ILU_NATURAL, rb=O.F_ILU_RB, tiled=O.F_ILU_TILED)[ftype]
    c, P, rp, ci, val, b = small_system(O, 4, 3, 2)
    pc = O.Cpr(P, rp, ci, val, ftype=ft, tile=(2, 2), use_amg=0)
    M = dense_M_of_fstage(pc, 3 * c.n)
    A = O.bsr_to_dense(rp, ci, val)
    nx, ny = c.nx, c.ny
    tile = lambda g: ((g % nx) // 2, ((g // nx) % ny) // 2)
    scale = np.abs(A).max()
    for i in range(c.n):
        for e in range(rp[i], rp[i + 1]):
            j = ci[e]
            blk = M[3 * i:3 * i + 3, 3 * j:3 * j + 3]
            if ftype == "tiled" and tile(i) != tile(j):
                assert np.abs(blk).max() <= 1e-9 * scale
            else:
                assert np.abs(blk - val[e]).max() <= 1e-9 * scale


def test_ilu0_defining_property_with_well_rows(oracle_lib):
    """Natural order on a grid followed by two fixed-rate well rows: L U
    equals A on the whole block pattern, the cell-well and well-cell blocks
    included.  Each well perforates a whole column, so eliminating a
    perforation updates the block of the perforation below it towards the
    well, and the well row is eliminated against every perforation in turn; a
    dropped or misplaced one of these updates breaks the equality there."""
    import dataclasses
    O = oracle_lib
    c = cg.tiny_case(4, 3, 3, seed=5, wells=[cg.Well(0, 0, 0, 2, "inj", "wrat", 800.0),
                                             cg.Well(3, 2, 0, 2, "prod", "lrat", 600.0)])
    extra = np.tile(np.array([3000.0, 0.0, 0.0]), c.nrate)
    c = dataclasses.replace(c, x_old=np.concatenate([c.x_old, extra]), x_new=np.concatenate([c.x_new, extra]))
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    n = P.rows
    assert n == c.n + 2 and any((ci[rp[i]:rp[i + 1]] >= c.n).any() for i in range(c.n))
    pc = O.Cpr(P, rp, ci, val, ftype=O.F_ILU_NATURAL, use_amg=0)
    M = dense_M_of_fstage(pc, 3 * n)
    scale = np.abs(val).max()
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            j = ci[e]
            assert np.abs(M[3 * i:3 * i + 3, 3 * j:3 * j + 3] - val[e]).max() <= 1e-9 * scale, (i, j)


def test_ilu0_exact_on_a_line(oracle_lib):
    """On an nx x 1 x 1 grid the block pattern is tridiagonal, ILU(0) has no
    dropped fill and is the exact LU: F alone and CPR-PF both solve in one
    FGMRES iteration."""
    O = oracle_lib
    c, P, rp, ci, val, b = small_system(O, 12, 1, 1, wells=[cg.Well(0, 0, 0, 0, "inj", "bhp", 3500.0),
                                                          cg.Well(11, 0, 0, 0, "prod", "bhp", 2500.0)])
    for use_amg in (0, 1):
        pc = O.Cpr(P, rp, ci, val, ftype=O.F_ILU_NATURAL, use_amg=use_amg)
        x, info = O.fgmres(rp, ci, val, b, pc, rtol=1e-10)
        assert info["converged"] and info["iterations"] == 1


def bfs_dist(srp, sci, src, n, cap=3):
    dist = {src: 0}
    frontier = [src]
    for d in range(1, cap + 1):
        nxt = []
        for u in frontier:
            for v in sci[srp[u]:srp[u + 1]]:
                if v not in dist:
                    dist[v] = d
                    nxt.append(v)
        frontier = nxt
    return dist


def test_amg_aggregation_invariants(oracle_lib):
    O = oracle_lib
    c = cg.make_case(0)
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    pc = O.Cpr(P, rp, ci, val, coarse_max=50)
    assert pc.nlevels() >= 2
    for l in range(pc.nlevels() - 1):
        L = pc.level(l)
        n, agg, srp, sci = L["n"], L["agg"], L["strong_rowptr"], L["strong_colind"]
        # strength graph symmetric
        S = set()
        for i in range(n):
            for j in sci[srp[i]:srp[i + 1]]:
                S.add((i, int(j)))
        assert all((j, i) in S for (i, j) in S)
        iso = np.array([srp[i + 1] == srp[i] for i in range(n)])
        assert np.all(agg[iso] == -1) and np.all(agg[~iso] >= 0)
        nc = L_next = pc.level(l + 1)["n"]
        assert set(agg[~iso]) == set(range(nc))
        # roots: smallest-index member of each aggregate that is adjacent to all
        # phase-1 members; check the MIS-2 property via the aggregate structure:
        # every aggregate's nodes are within distance 2 of each other's root.
        P_ = np.zeros((n, nc))
        for i in range(n):
            for e in range(L["p_rowptr"][i], L["p_rowptr"][i + 1]):
                P_[i, L["p_colind"][e]] = L["p_val"][e]
        A = np.zeros((n, n))
        for i in range(n):
            for e in range(L["rowptr"][i], L["rowptr"][i + 1]):
                A[i, L["colind"][e]] = L["val"][e]
        Ln = pc.level(l + 1)
        Ac = np.zeros((nc, nc))
        for i in range(nc):
            for e in range(Ln["rowptr"][i], Ln["rowptr"][i + 1]):
                Ac[i, Ln["colind"][e]] = Ln["val"][e]
        ref = P_.T @ A @ P_
        assert np.abs(Ac - ref).max() <= 1e-12 * np.abs(ref).max()


def test_mis2_independence_and_maximality(oracle_lib):
    """Roots (MIS-2 members) are pairwise more than distance 2 apart in the
    strength graph; every aggregated node lies within distance 2 of the root of
    its own aggregate; aggregates are numbered by root index."""
    O = oracle_lib
    c = cg.make_case(0)
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    pc = O.Cpr(P, rp, ci, val, coarse_max=50)
    L = pc.level(0)
    n, agg, srp, sci, root = L["n"], L["agg"], L["strong_rowptr"], L["strong_colind"], L["root"]
    roots = np.nonzero(root)[0]
    assert np.array_equal(agg[roots], np.arange(len(roots)))
    rootset = set(roots.tolist())
    for r in roots:
        d = bfs_dist(srp, sci, r, n, cap=2)
        assert not (set(d) - {r}) & rootset
        for v, dv in d.items():
            if dv == 1:
                assert agg[v] == agg[r]          # phase 1: neighbours join their root
    covered = {}
    for r in roots:
        for v in bfs_dist(srp, sci, r, n, cap=2):
            covered.setdefault(v, set()).add(agg[r])
    for v in np.nonzero(agg >= 0)[0]:
        assert agg[v] in covered[v]


def test_single_level_amg_is_exact(oracle_lib):
    O = oracle_lib
    c, P, rp, ci, val, b = small_system(O, 5, 4, 3)
    pc = O.Cpr(P, rp, ci, val, coarse_max=1000)
    assert pc.nlevels() == 1
    _, app = O.qi_decouple(rp, ci, val)
    n = c.n
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = app[rp[i]:rp[i + 1]]
    rhs = np.random.default_rng(0).standard_normal(n)
    x = pc.vcycle(rhs)
    assert np.linalg.norm(A @ x - rhs) <= 1e-12 * np.linalg.norm(rhs)


def test_arnoldi_relation(oracle_lib):
    """A Z_k = V_{k+1} Hbar_k (flexible Arnoldi) with a CPR preconditioner."""
    O = oracle_lib
    c, P, rp, ci, val, b = small_system(O, 5, 4, 3)
    pc = O.Cpr(P, rp, ci, val)
    A = O.bsr_to_dense(rp, ci, val)
    for orth in (0, 1):
        k = 8
        Z, V, H = O.arnoldi(rp, ci, val, b, k, pc, orth=orth)
        lhs = A @ Z.T
        rhs = V.T @ H
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(A, 2) * np.linalg.norm(Z)
        if orth == 1:
            # classical Gram-Schmidt with one re-orthogonalisation keeps V
            # orthonormal to working precision ("twice is enough"); modified
            # Gram-Schmidt loses orthogonality in proportion to the condition
            # of A Z and is not held to this bound.
            assert np.linalg.norm(V @ V.T - np.eye(k + 1)) <= 1e-13


def test_gmres_finite_termination(oracle_lib):
    """Without restart and preconditioner, GMRES on n unknowns terminates in at
    most n steps (here n = 48)."""
    O = oracle_lib
    c, P, rp, ci, val, b = small_system(O, 4, 2, 2)
    n3 = 3 * c.n
    x, info = O.fgmres(rp, ci, val, b, None, m=n3, maxit=n3, rtol=1e-9)
    assert info["converged"] and info["iterations"] <= n3


@pytest.mark.parametrize("ftype", ["bj", "natural", "rb", "tiled"])
@pytest.mark.parametrize("fpf", [0, 1])
def test_cpr_fgmres_matches_dense_solution(oracle_lib, ftype, fpf):
    O = oracle_lib
    ft = dict(bj=O.F_BJ, natural=O.F_ILU_NATURAL, rb=O.F_ILU_RB, tiled=O.F_ILU_TILED)[ftype]
    c, P, rp, ci, val, b = small_system(O, 4, 4, 3)
    A = O.bsr_to_dense(rp, ci, val)
    xs = O.dense_solve(A, b)
    pc = O.Cpr(P, rp, ci, val, ftype=ft, fpf=fpf, tile=(2, 2), coarse_max=10)
    x, info = O.fgmres(rp, ci, val, b, pc, rtol=1e-6)
    assert info["converged"]
    r = b - A @ x
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b) * (1 + 1e-12)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(x - xs) <= kappa * 1e-6 * np.linalg.norm(xs)


def test_workload0_converges(oracle_lib):
    O = oracle_lib
    c = cg.make_case(0)
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    pc = O.Cpr(P, rp, ci, val)
    x, info = O.fgmres(rp, ci, val, -R, pc)
    assert info["converged"] and info["rel_residual"] <= 1e-6
    assert info["iterations"] <= 30


def _scipy_vcycle(O, pc, b, csmoother, sweeps=1):
    """The V(s,s) cycle recomposed with scipy from the oracle's own hierarchy:
    level 0 red-black Gauss-Seidel (red then black down, black then red up),
    coarser levels l1-Jacobi or damped Jacobi, coarsest level dense solve."""
    import scipy.sparse as sp
    nl = pc.nlevels()
    As, Ps = [], []
    for l in range(nl):
        L = pc.level(l)
        As.append(sp.csr_matrix((L["val"], L["colind"], L["rowptr"]), shape=(L["n"], L["n"])))
        if l < nl - 1:
            Ps.append(sp.csr_matrix((L["p_val"], L["p_colind"], L["p_rowptr"]),
                                    shape=(L["n"], pc.level(l + 1)["n"])))
    color = pc.level(0)["color"]

    def gs(A, b, x, order):
        A = A.tocsr()
        for c in order:
            for i in np.where(color == c)[0]:
                lo, hi = A.indptr[i], A.indptr[i + 1]
                cols, vals = A.indices[lo:hi], A.data[lo:hi]
                d = vals[cols == i][0]
                s = b[i] - sum(v * x[j] for j, v in zip(cols, vals) if j != i)
                x[i] = s / d
        return x

    def jac(A, b, x):
        if csmoother == O.CSMOOTH_L1:
            return x + (b - A @ x) / np.asarray(abs(A).sum(axis=1)).ravel()
        return x + (2.0 / 3.0) * (b - A @ x) / A.diagonal()

    def vc(l, b):
        A = As[l]
        if l == nl - 1:
            return np.linalg.solve(A.toarray(), b)
        x = np.zeros_like(b)
        for _ in range(sweeps):
            x = gs(A, b, x, (0, 1)) if l == 0 else jac(A, b, x)
        x = x + Ps[l] @ vc(l + 1, Ps[l].T @ (b - A @ x))
        for _ in range(sweeps):
            x = gs(A, b, x, (1, 0)) if l == 0 else jac(A, b, x)
        return x
    return vc(0, b)


@pytest.mark.parametrize("csm", ["l1", "jacobi"])
def test_vcycle_equals_scipy_recomposition(oracle_lib, csm):
    O = oracle_lib
    cs = dict(l1=O.CSMOOTH_L1, jacobi=O.CSMOOTH_JACOBI)[csm]
    c, P, rp, ci, val, b = small_system(O, 10, 9, 4, seed=12)
    pc = O.Cpr(P, rp, ci, val, coarse_max=12, csmoother=cs)
    assert pc.nlevels() >= 3
    bp = np.random.default_rng(3).standard_normal(c.n)
    ref = _scipy_vcycle(O, pc, bp, cs)
    assert np.linalg.norm(pc.vcycle(bp) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_l1_smoother_keeps_high_contrast_cycle_convergent(oracle_lib):
    """Log-normal permeability with sigma = 2: Galerkin products of the
    decoupled pressure matrix lose diagonal dominance on coarse levels; with
    damped Jacobi there the V-cycle diverges, with l1-Jacobi it contracts."""
    import scipy.sparse as sp
    O = oracle_lib
    c = cg.tiny_case(20, 20, 20, seed=4, sigma=2.0, step=0.01, dt=3.0)
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    w, app = O.qi_decouple(rp, ci, val)
    A = sp.csr_matrix((app, ci, rp), shape=(c.n, c.n))
    b = np.random.default_rng(1).standard_normal(c.n)
    out = {}
    for cs in (O.CSMOOTH_JACOBI, O.CSMOOTH_L1):
        pc = O.Cpr(P, rp, ci, val, csmoother=cs, coarse_max=40)
        x = np.zeros(c.n)
        for _ in range(6):
            x = x + pc.vcycle(b - A @ x)
        out[cs] = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert out[O.CSMOOTH_L1] < 0.2 and out[O.CSMOOTH_JACOBI] > 1.0


def incompressible_no_well_case():
    """No wells, rigid rock, constant formation-volume factors and solution
    gas: accumulation has no pressure derivative, so every component's
    pressure block has zero row sums and the decoupled pressure block (and
    every Galerkin product of it) is singular: a pure-Neumann operator."""
    import dataclasses
    c = cg.tiny_case(6, 5, 4, seed=8, wells=[], step=0.0)
    fl = dict(c.fluid)
    fl.update(c_r=0.0, cw=0.0, co=0.0, cg=0.0, crs=0.0)
    return dataclasses.replace(c, fluid=fl)


def test_singular_pressure_block_is_reported(oracle_lib):
    O = oracle_lib
    import scipy.sparse as sp
    c = incompressible_no_well_case()
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    w, app = O.qi_decouple(rp, ci, val)
    A = sp.csr_matrix((app, ci, rp), shape=(c.n, c.n))
    assert np.abs(A @ np.ones(c.n)).max() <= 1e-13 * np.abs(app).max()
    for cm in (192, 40, 10):
        with pytest.raises(RuntimeError) as e:
            O.Cpr(P, rp, ci, val, coarse_max=cm)
        assert str(O.OR_ERR_SINGULAR_COARSE) in str(e.value)
    # the same grid with its wells and compressibilities sets up (the bound is
    # far from the workloads' coarsest pivots)
    P2 = O.Problem(cg.tiny_case(6, 5, 4, seed=8, step=0.0))
    O.Cpr(P2, *O.jacobian(P2)[:3])

"""Pins of the two-phase oracle (Section 2.2's oil-water model and the CPR of
its 2x2-block Jacobians) to what the model and the mathematics fix:

  - the accumulation of one cell and the Darcy flux between two cells in
    closed form from the model's equations (oil row first, then water; Corey
    curves; linear formation volume factors; harmonic-mean transmissibility;
    upstream mobility);
  - the Jacobian against central differences of the residual;
  - the gas phase's data does not enter the two-phase system;
  - the quasi-IMPES weights remove the saturation entry of each diagonal
    block;
  - the F stage's block ILU(0) reproduces A on the kept block pattern (the
    defining property of ILU(0)) and its output solves the factored system;
  - the CPR-preconditioned FGMRES solves the 2x2 system.
"""
import dataclasses
import math

import numpy as np
import pytest

import bo_casegen as cg
from oracle import twophase as T


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def _case(nx, ny, nz, wells=(), gravity=True, seed=5, step=0.02):
    c = cg.tiny_case(nx, ny, nz, seed=seed, step=step, wells=list(wells), gravity=gravity)
    return cg.two_phase(c)


def _fvf_b(B0, c, pref, p):
    return 1.0 / (B0 * (1.0 - c * (p - pref)))


def _corey(s, lo, span, n):
    return min(max((s - lo) / span, 0.0), 1.0) ** n


def test_accumulation_closed_form(O):
    c = _case(1, 1, 1)
    f = c.fluid
    P = T.problem(O, c)
    R = T.residual(O, P)
    acc = c.dx * c.dy * c.dz / (f["rb_ft3"] * c.dt)

    def masses(x):
        p, sw = x[0], x[1]
        phi = c.phi0[0] * (1.0 + f["c_r"] * (p - f["p_ref"]))
        bo = _fvf_b(f["Bo0"], f["co"], f["p_ref"], p)
        bw = _fvf_b(f["Bw0"], f["cw"], f["p_ref"], p)
        return np.array([phi * (1.0 - sw) * bo, phi * sw * bw])

    ref = acc * (masses(c.x_new) - masses(c.x_old))
    assert np.allclose(R, ref, rtol=1e-13, atol=0.0)


def test_flux_closed_form(O):
    # two cells side by side, no gravity, no accumulation change, p0 > p1
    c = _case(2, 1, 1, gravity=False, step=0.0)
    x = c.x_old.copy()
    x[0], x[3] = 3200.0, 2900.0
    x[1], x[4] = 0.45, 0.3
    c = dataclasses.replace(c, x_old=x, x_new=x.copy())
    f = c.fluid
    P = T.problem(O, c)
    R = T.residual(O, P)
    k0, k1 = c.kx[0], c.kx[1]
    Tr = f["tcoef"] * c.dy * c.dz / (c.dx / (2 * k0) + c.dx / (2 * k1))
    span = 1.0 - f["swc"] - f["sor"]
    sw_up = x[1]   # cell 0 is upstream for both phases
    p_up = x[0]
    lo = _corey(1.0 - sw_up, f["sor"], span, f["no"]) / f["mu_o"]
    lw = _corey(sw_up, f["swc"], span, f["nw"]) / f["mu_w"]
    bo = _fvf_b(f["Bo0"], f["co"], f["p_ref"], p_up)
    bw = _fvf_b(f["Bw0"], f["cw"], f["p_ref"], p_up)
    dp = x[0] - x[3]
    Fo, Fw = Tr * lo * bo * dp, Tr * lw * bw * dp
    assert np.allclose(R, [Fo, Fw, -Fo, -Fw], rtol=1e-12, atol=0.0)


def test_jacobian_central_differences(O):
    wells = [cg.Well(0, 0, 0, 2, "inj", "bhp", 3500.0), cg.Well(4, 3, 1, 2, "prod", "bhp", 2500.0)]
    c = _case(5, 4, 3, wells=wells)
    P = T.problem(O, c)
    rp, ci, val, R = T.jacobian(O, P)
    J = O.bsr_to_dense(rp, ci, np.pad(val, ((0, 0), (0, 1), (0, 1))))
    J = J.reshape(c.n, 3, c.n, 3)[:, :2, :, :2].reshape(2 * c.n, 2 * c.n)
    xo2, xn2 = cg.state2(c.x_old), cg.state2(c.x_new)
    rng = np.random.default_rng(3)
    for col in rng.choice(2 * c.n, size=16, replace=False):
        h = 1e-3 if col % 2 == 0 else 1e-6
        xp, xm = xn2.copy(), xn2.copy()
        xp[col] += h
        xm[col] -= h
        fd = (T.residual(O, P, xo2, xp) - T.residual(O, P, xo2, xm)) / (2 * h)
        scale = max(np.abs(J[:, col]).max(), 1e-30)
        assert np.abs(fd - J[:, col]).max() <= 1e-5 * scale, col


def test_gas_data_does_not_enter(O):
    c = _case(4, 3, 2, wells=[cg.Well(0, 0, 0, 1, "inj", "bhp", 3400.0), cg.Well(3, 2, 0, 1, "prod", "bhp", 2600.0)])
    P = T.problem(O, c)
    rp, ci, v1, R1 = T.jacobian(O, P)
    fl = dict(c.fluid, Bg0=0.5, cg=1e-4, mu_g=0.05, rho_gsc=0.08, ng=3)
    P2 = T.problem(O, dataclasses.replace(c, fluid=fl))
    _, _, v2, R2 = T.jacobian(O, P2)
    assert np.allclose(v1, v2, rtol=1e-14, atol=1e-14 * np.abs(v1).max())
    assert np.allclose(R1, R2, rtol=1e-14, atol=1e-14 * np.abs(R1).max())


def test_quasi_impes_weights(O):
    c = cg.two_phase(cg.make_case(0))
    P = T.problem(O, c)
    rp, ci, val, R = T.jacobian(O, P)
    pc = T.Cpr2(O, P, rp, ci, val)
    w = pc.weights().reshape(-1, 2)
    assert not pc.weights3().reshape(-1, 3)[:, 2].any()
    rows = np.repeat(np.arange(c.n), np.diff(rp))
    D = val[ci == rows]
    assert np.all(np.abs(w[:, 0]) == 1.0)
    cD = np.einsum("ni,nij->nj", w, D)
    assert np.all(np.abs(cD[:, 1]) <= 1e-15 * np.abs(D).reshape(c.n, -1).max(axis=1))
    assert np.all(cD[:, 0] > 0.0)


@pytest.mark.parametrize("tile", [(3, 2), (8, 8)])
def test_fstage_is_ilu0_of_the_tiles(O, tile):
    c = _case(7, 5, 3, wells=[cg.Well(0, 0, 0, 2, "inj", "bhp", 3500.0), cg.Well(6, 4, 0, 2, "prod", "bhp", 2500.0)])
    P = T.problem(O, c)
    rp, ci, val, R = T.jacobian(O, P)
    pc = T.Cpr2(O, P, rp, ci, val, tile=tile)
    n = c.n
    tid = lambda g: (g % c.nx) // tile[0] + ((c.nx + tile[0] - 1) // tile[0]) * ((g // c.nx) % c.ny // tile[1])
    A = np.zeros((n, n, 2, 2))
    keep = np.zeros((n, n), bool)
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            j = ci[e]
            if tid(i) == tid(j):
                A[i, j] = val[e]
                keep[i, j] = True
    Einv = pc.pivots()[:, :2, :2]
    assert np.all(pc.pivots()[:, 2, 2] == 1.0)
    E = np.linalg.inv(Einv)
    L = np.zeros_like(A)
    U = np.zeros_like(A)
    order = sorted(range(n), key=lambda g: (tid(g), g))
    rank = np.empty(n, int)
    rank[order] = np.arange(n)
    for i in range(n):
        for j in range(n):
            if keep[i, j] and rank[j] < rank[i]:
                L[i, j] = A[i, j]
            elif keep[i, j] and rank[j] > rank[i]:
                U[i, j] = A[i, j]
    dense = lambda B: B.transpose(0, 2, 1, 3).reshape(2 * n, 2 * n)
    Ed = np.zeros_like(A)
    Edi = np.zeros_like(A)
    for i in range(n):
        Ed[i, i] = E[i]
        Edi[i, i] = Einv[i]
    M = (dense(Ed) + dense(L)) @ dense(Edi) @ (dense(Ed) + dense(U))
    Ad = dense(A)
    mask = np.kron(keep, np.ones((2, 2), bool))
    # ILU(0): the product equals A on every kept block
    assert np.abs(M - Ad)[mask].max() <= 1e-12 * np.abs(Ad).max()
    r = np.random.default_rng(7).standard_normal(2 * n)
    z = pc.fstage(r)
    assert np.linalg.norm(M @ z - r) <= 1e-12 * np.linalg.norm(r) * np.linalg.cond(M)
    assert not pc.c3.fstage(T.embed_vec(r))[2::3].any()


@pytest.mark.parametrize("fpf", [0, 1])
def test_fgmres_solves_two_phase_system(O, fpf):
    c = cg.two_phase(cg.make_case(0))
    P = T.problem(O, c)
    rp, ci, val, R = T.jacobian(O, P)
    b = -R
    pc = T.Cpr2(O, P, rp, ci, val, fpf=fpf)
    x, info = T.fgmres(O, rp, ci, val, b, pc)
    assert info["converged"]
    assert np.linalg.norm(b - T.spmv(O, rp, ci, val, x)) <= 1e-6 * np.linalg.norm(b)
    A = O.bsr_to_dense(rp, ci, np.pad(val, ((0, 0), (0, 1), (0, 1))))
    A = A.reshape(c.n, 3, c.n, 3)[:, :2, :, :2].reshape(2 * c.n, 2 * c.n)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.cond(A) * np.linalg.norm(xd)

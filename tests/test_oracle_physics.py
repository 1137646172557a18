"""Pins of the oracle's physics (CPU only): closed forms, finite differences,
conservation and sign structure.  None of these re-types the oracle's formulas:
each compares it with something the model fixes independently."""
import os

import numpy as np
import pytest

import bo_casegen as cg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")


def golden():
    vals = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()
        vals[k] = float(v)
    return vals


def uniform_case(nx=3, ny=3, nz=3, k=100.0, phi=0.2, **kw):
    c = cg.tiny_case(nx, ny, nz, **kw)
    n = c.n
    c.kx = np.full(n, k); c.ky = np.full(n, k); c.kz = np.full(n, 0.1 * k)
    c.phi0 = np.full(n, phi)
    return c


def test_relperm_closed_form(oracle_lib):
    O = oracle_lib
    g = golden()
    P = O.Problem(uniform_case())
    kr = O.relperm(P, 0.25, 0.05)
    for key in ("krw", "krow", "krg", "krog", "kro"):
        assert kr[key] == pytest.approx(g[key], rel=1e-14, abs=1e-16)


def test_stone2_reduces_to_two_phase(oracle_lib):
    """With no gas, Stone II gives back the oil-water curve (Section 2.1)."""
    O = oracle_lib
    P = O.Problem(uniform_case())
    for sw in np.linspace(0.2, 0.8, 13):
        kr = O.relperm(P, sw, 0.0)
        assert kr["kro"] == pytest.approx(kr["krow"], rel=1e-14, abs=1e-16)
        assert kr["krg"] == 0.0


def test_relperm_derivatives_fd(oracle_lib):
    O = oracle_lib
    P = O.Problem(uniform_case())
    for sw, sg in [(0.3, 0.1), (0.45, 0.05), (0.25, 0.2)]:
        h = 1e-7
        kr = O.relperm(P, sw, sg)
        d_w = (O.relperm(P, sw + h, sg)["kro"] - O.relperm(P, sw - h, sg)["kro"]) / (2 * h)
        d_g = (O.relperm(P, sw, sg + h)["kro"] - O.relperm(P, sw, sg - h)["kro"]) / (2 * h)
        assert kr["dkro_dsw"] == pytest.approx(d_w, rel=1e-6)
        assert kr["dkro_dsg"] == pytest.approx(d_g, rel=1e-6)


def test_geometry_closed_forms(oracle_lib):
    O = oracle_lib
    g = golden()
    c = uniform_case()
    P = O.Problem(c)
    assert O.transmissibility(P, 0, 1) == pytest.approx(g["Tx"], rel=1e-14)
    assert O.transmissibility(P, 0, 3) == pytest.approx(g["Tx"], rel=1e-14)
    assert O.transmissibility(P, 0, 9) == pytest.approx(g["Tz"], rel=1e-14)
    assert O.well_index(P, 0) == pytest.approx(g["WI"], rel=1e-12)
    assert O.pore_volume(P, 0, 3000.0) == pytest.approx(g["Vp"], rel=1e-14)


def test_transmissibility_series_resistance(oracle_lib):
    """The harmonic face transmissibility is two half-cell conductances in series."""
    O = oracle_lib
    c = uniform_case(nx=2, ny=1, nz=1)
    c.kx = np.array([3.0, 700.0]); c.ky = c.kx.copy(); c.kz = 0.1 * c.kx
    P = O.Problem(c)
    half = [0.001127 * c.dy * c.dz * k / (c.dx / 2) for k in c.kx]
    assert O.transmissibility(P, 0, 1) == pytest.approx(1.0 / (1.0 / half[0] + 1.0 / half[1]), rel=1e-14)
    assert O.transmissibility(P, 1, 0) == O.transmissibility(P, 0, 1)


def fd_jacobian_check(O, case, cells, tol):
    P = O.Problem(case)
    rp, ci, val, R = O.jacobian(P)
    x = case.x_new
    worst = 0.0
    for g in cells:
        for q in range(3):
            h = 1e-6 * x[3 * g] if q == 0 else 1e-7
            xp = x.copy(); xp[3 * g + q] += h
            xm = x.copy(); xm[3 * g + q] -= h
            d = (O.residual(P, x_new=xp) - O.residual(P, x_new=xm)) / (2 * h)
            col = np.zeros_like(d)
            for i in range(case.n):
                for e in range(rp[i], rp[i + 1]):
                    if ci[e] == g:
                        col[3 * i:3 * i + 3] = val[e][:, q]
            # per-block comparison on the rows that hold this column
            for i in np.unique(np.nonzero(col)[0] // 3):
                a, b = col[3 * i:3 * i + 3], d[3 * i:3 * i + 3]
                err = np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300)
                worst = max(worst, err)
    assert worst <= tol, worst


@pytest.mark.parametrize("gravity", [True, False])
def test_jacobian_matches_finite_differences(oracle_lib, gravity):
    c = cg.tiny_case(5, 4, 3, seed=11, noise=0.05, noise_kind="iid", step=0.02, gravity=gravity)
    fd_jacobian_check(oracle_lib, c, cells=range(0, c.n, 7), tol=1e-6)


def test_jacobian_fd_workload0(oracle_lib):
    c = cg.make_case(0)
    fd_jacobian_check(oracle_lib, c, cells=[0, 17, 399, 411, 1999], tol=1e-6)


def test_flux_conservation(oracle_lib):
    """No-flow boundary (Section 2.1): fluxes only move mass between cells, so
    each component's flux residual sums to zero over the grid."""
    O = oracle_lib
    c = cg.tiny_case(6, 5, 4, seed=3, noise_kind="iid")
    P = O.Problem(c)
    R = O.flux_residual(P)
    for q in range(3):
        s = np.abs(R[q::3]).sum()
        assert abs(R[q::3].sum()) <= 1e-12 * s


def test_flux_jacobian_column_sums_vanish(oracle_lib):
    """d/dx_j of sum_i flux_i = 0: the block column sums of the flux Jacobian are
    zero.  The accumulation part scales with 1/dt, so J_flux = 2 J(2dt) - J(dt)."""
    O = oracle_lib
    c = cg.tiny_case(5, 4, 3, seed=5, noise_kind="iid", wells=[])
    P = O.Problem(c)
    rp, ci, v1, _ = O.jacobian(P, dt=1.0)
    _, _, v2, _ = O.jacobian(P, dt=2.0)
    vf = 2 * v2 - v1
    n = c.n
    colsum = np.zeros((n, 3, 3))
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            colsum[ci[e]] += vf[e]
    scale = np.abs(vf).max()
    assert np.abs(colsum).max() <= 1e-10 * scale


def test_zero_flux_uniform_pressure(oracle_lib):
    O = oracle_lib
    c = cg.tiny_case(4, 4, 3, seed=9, gravity=False)
    x = c.x_new.copy()
    x[0::3] = 3111.0
    R = O.flux_residual(O.Problem(c), x)
    assert np.abs(R).max() == 0.0


def test_zero_flux_horizontal_with_gravity(oracle_lib):
    """One layer: gravity does not act across horizontal faces."""
    O = oracle_lib
    c = cg.tiny_case(5, 4, 1, seed=9, gravity=True)
    x = c.x_new.copy()
    x[0::3] = 2950.0
    R = O.flux_residual(O.Problem(c), x)
    assert np.abs(R).max() == 0.0


def test_accumulation_only_when_states_equal(oracle_lib):
    """x_new == x_old, no wells, uniform pressure, no gravity: R == 0."""
    O = oracle_lib
    c = cg.tiny_case(4, 3, 3, seed=2, gravity=False, wells=[])
    c.x_new[0::3] = 3000.0
    c.x_old = c.x_new.copy()
    R = O.residual(O.Problem(c))
    assert np.abs(R).max() == 0.0


def test_pressure_blocks_are_m_matrices_in_accumulation_regime(oracle_lib):
    """Without the gravity-density term the pressure column of each component
    is a Z-matrix (upstream fluxes fall with the neighbour's pressure); with a
    small pressure spread the accumulation makes it strictly diagonally
    dominant, and so is the decoupled pressure block."""
    O = oracle_lib
    c = cg.tiny_case(6, 5, 4, seed=4, noise=0.001, noise_kind="iid", gravity=False, wells=[])
    P = O.Problem(c)
    rp, ci, val, _ = O.jacobian(P)
    n = c.n
    for alpha in range(3):
        for i in range(n):
            off = [val[e][alpha, 0] for e in range(rp[i], rp[i + 1]) if ci[e] != i]
            d = [val[e][alpha, 0] for e in range(rp[i], rp[i + 1]) if ci[e] == i][0]
            assert max(off) <= 0.0
            assert d > -sum(off)
    cw, app = O.qi_decouple(rp, ci, val)
    for i in range(n):
        off = [app[e] for e in range(rp[i], rp[i + 1]) if ci[e] != i]
        d = [app[e] for e in range(rp[i], rp[i + 1]) if ci[e] == i][0]
        assert max(off) <= 0.0 and d > -sum(off)


def test_quasi_impes_decouples_diagonal_block(oracle_lib):
    """Block quasi-IMPES (Section 3.2): the decoupled pressure row has zero
    saturation coefficients on the cell's own block."""
    O = oracle_lib
    c = cg.make_case(0)
    P = O.Problem(c)
    rp, ci, val, _ = O.jacobian(P)
    cw, app = O.qi_decouple(rp, ci, val, mode=O.QI_BLOCK)
    cw = cw.reshape(-1, 3)
    for i in range(c.n):
        e = [e for e in range(rp[i], rp[i + 1]) if ci[e] == i][0]
        B = val[e]
        s = cw[i] @ B[:, 1:3]
        scale = np.abs(cw[i][:, None] * B[:, 1:3]).sum(axis=0)
        assert np.all(np.abs(s) <= 1e-13 * scale)
        assert abs(cw[i][0]) == 1.0
        assert cw[i] @ B[:, 0] > 0.0


def test_decoupled_system_has_same_solution(oracle_lib):
    O = oracle_lib
    c = cg.tiny_case(3, 3, 2, seed=8)
    P = O.Problem(c)
    rp, ci, val, R = O.jacobian(P)
    A = O.bsr_to_dense(rp, ci, val)
    b = -R
    cw, _ = O.qi_decouple(rp, ci, val)
    n = c.n
    D = np.eye(3 * n)
    for i in range(n):
        D[3 * i, 3 * i:3 * i + 3] = cw[3 * i:3 * i + 3]
    x1 = np.linalg.solve(A, b)
    x2 = np.linalg.solve(D @ A, D @ b)
    assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x1)


def test_pattern_is_seven_point(oracle_lib):
    O = oracle_lib
    c = cg.tiny_case(4, 3, 2)
    rp, ci = O.pattern(O.Problem(c))
    n = c.n
    # 7-point: N + 2 * (internal faces)
    faces = (c.nx - 1) * c.ny * c.nz + c.nx * (c.ny - 1) * c.nz + c.nx * c.ny * (c.nz - 1)
    assert rp[-1] == n + 2 * faces
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols

"""GPU parity of the scalar pressure-system solve (restricted additive Schwarz
with ILU(0) subdomain solves, standard right-preconditioned GMRES(30), the
paper's linear-solver run) against the oracle:

  - the scalar SpMV: integer data bit for bit, real data to 1e-14;
  - RAS: whole vectors bit for bit (the GPU takes the oracle's operations in
    the oracle's order) for several tile shapes and overlaps on ragged grids;
  - GMRES (flexible 0) after a fixed number of steps (1, 5, one cycle, a
    restart, 90 as in the paper's run): the iterate to 1e-8 and the true
    residual to 1e-6 of the oracle's (CGS2 against the oracle's modified
    Gram-Schmidt: the same Krylov space, other rounding);
  - flexible and standard GMRES with a fixed preconditioner give the same
    iterate, for RAS and for the black-oil CPR;
  - the paper's per-process share (125x125x47 cells, 3e9 / 4096 unknowns)
    in full, and sampled tiles of a larger grid against the oracle's solve
    of the same extended tile."""
import numpy as np
import pytest

import bo_casegen as cg
from oracle import pressure as PR
from tests.gpu_util import rel_err, setup_both, to_dev, to_host, ragged_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1606_00556_amd import bo
    bo.lib()
    return bo


def grid_of(c):
    return (c.nx, c.ny, c.nz)


def test_scalar_spmv(B):
    import torch
    c = cg.pressure_case(23, 17, 7, seed=11)
    rng = np.random.default_rng(1)
    icoef = np.where(c.coef != 0.0, rng.integers(-512, 513, size=c.coef.shape), 0).astype(np.float64)
    ix = rng.integers(-512, 513, size=c.n).astype(np.float64)
    y = torch.zeros(c.n, dtype=torch.float64, device="cuda")
    B.bo_scalar_spmv(grid_of(c), to_dev(icoef.reshape(-1)), 1.0, to_dev(ix), 0.0, y)
    assert np.array_equal(to_host(y), PR.spmv(c.nx, c.ny, c.nz, icoef, ix))
    x = rng.standard_normal(c.n)
    y0 = rng.standard_normal(c.n)
    y = to_dev(y0)
    B.bo_scalar_spmv(grid_of(c), to_dev(c.coef.reshape(-1)), 0.5, to_dev(x), -2.0, y)
    assert rel_err(to_host(y), 0.5 * PR.spmv(c.nx, c.ny, c.nz, c.coef, x) - 2.0 * y0) <= 1e-14


@pytest.mark.parametrize("tile,overlap", [((6, 6), 1), ((8, 8), 0), ((3, 4), 2), ((2, 2), 3), ((5, 1), 1)])
def test_ras_apply_matches_oracle(B, tile, overlap):
    import torch
    c = cg.pressure_case(23, 17, 7, seed=12)
    coef = to_dev(c.coef.reshape(-1))
    pc = B.bo_ras_setup(grid_of(c), coef, B.bo_ras_default_opts(tile_x=tile[0], tile_y=tile[1], overlap=overlap))
    ras = PR.Ras(c.nx, c.ny, c.nz, c.coef, tile, overlap)
    for seed in (2, 3):
        r = np.random.default_rng(seed).standard_normal(c.n)
        z = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        B.bo_cpr_apply(pc, to_dev(r), z)
        # the oracle's operations in the oracle's order: the same bits
        assert np.array_equal(to_host(z), ras.apply(r))


def test_ras_setup_refusals(B):
    c = cg.pressure_case(9, 7, 3, seed=13)
    coef = to_dev(c.coef.reshape(-1))
    with pytest.raises(B.BoError):
        B.bo_ras_setup(grid_of(c), coef, B.bo_ras_default_opts(tile_x=8, tile_y=8, overlap=1))  # 100 lanes
    bad = c.coef.copy()
    bad[3, 5] = np.nan
    with pytest.raises(B.BoError):
        B.bo_ras_setup(grid_of(c), to_dev(bad.reshape(-1)))


@pytest.mark.parametrize("k", [1, 5, 30, 45, 90])
def test_gmres_steps_match_oracle(B, k):
    import torch
    c = cg.pressure_case(23, 17, 7, seed=14)
    coef = to_dev(c.coef.reshape(-1))
    pc = B.bo_ras_setup(grid_of(c), coef)
    xo, oi = PR.solve(c, tile=(6, 6), overlap=1, m=30, maxit=k)
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
    gi = B.bo_scalar_solve(pc, coef, to_dev(c.b), x, B.bo_fgmres_default_opts(flexible=0, maxit=k, rtol=1e-300))
    assert gi["iterations"] == oi["iterations"] == k
    assert gi["restarts"] == oi["restarts"] == (k - 1) // 30
    xg = to_host(x)
    assert rel_err(xg, xo) <= 1e-8
    rel = np.linalg.norm(c.b - PR.spmv(c.nx, c.ny, c.nz, c.coef, xg)) / np.linalg.norm(c.b)
    assert rel == pytest.approx(oi["rel_residual"], rel=1e-6)
    assert gi["rel_residual"] == pytest.approx(rel, rel=1e-8)


def test_flexible_and_standard_agree(B):
    """With a fixed linear preconditioner flexible GMRES and the standard
    form build the same iterate: RAS on the scalar system, and the black-oil
    CPR through bo_fgmres_solve."""
    import torch
    c = cg.pressure_case(19, 13, 6, seed=15)
    coef = to_dev(c.coef.reshape(-1))
    pc = B.bo_ras_setup(grid_of(c), coef)
    xs = []
    for flex in (0, 1):
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        B.bo_scalar_solve(pc, coef, to_dev(c.b), x, B.bo_fgmres_default_opts(flexible=flex, maxit=40, rtol=1e-300))
        xs.append(to_host(x))
    assert rel_err(xs[0], xs[1]) <= 1e-9
    from oracle import oracle as O
    O.lib()
    case = ragged_case()
    P, rp, ci, val, b, opc, gpc = setup_both(B, O, case)
    # flexible with CGS2 against the standard form with CGS2 and with the
    # delayed re-orthogonalisation (whose update goes through S y)
    infos, xs = [], []
    for flex, orth in ((1, 1), (0, 1), (0, 2)):
        x = torch.zeros(3 * case.n, dtype=torch.float64, device="cuda")
        infos.append(B.bo_fgmres_solve(gpc, gpc.A, to_dev(b), x,
                                       B.bo_fgmres_default_opts(flexible=flex, orth=orth)))
        xs.append(to_host(x))
    assert all(i["converged"] and i["iterations"] == infos[0]["iterations"] for i in infos)
    assert rel_err(xs[1], xs[0]) <= 1e-6 and rel_err(xs[2], xs[0]) <= 1e-6


def test_paper_share_full_solve(B):
    """3e9 / 4096 unknowns (125x125x47 = 734,375 cells), the per-process
    share of the paper's largest run: 90 fixed iterations of GMRES(30) with
    RAS, the iterate and the true residual against the oracle's."""
    import torch
    c = cg.pressure_case(125, 125, 47)
    coef = to_dev(c.coef.reshape(-1))
    pc = B.bo_ras_setup(grid_of(c), coef)
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
    gi = B.bo_scalar_solve(pc, coef, to_dev(c.b), x, B.bo_fgmres_default_opts(flexible=0, maxit=90, rtol=1e-300))
    xo, oi = PR.solve(c, tile=(6, 6), overlap=1, m=30, maxit=90)
    xg = to_host(x)
    rel = np.linalg.norm(c.b - PR.spmv(c.nx, c.ny, c.nz, c.coef, xg)) / np.linalg.norm(c.b)
    print(f"share: residual after 90 its gpu {rel:.3e} oracle {oi['rel_residual']:.3e}, |x - x_o|/|x_o| "
          f"{rel_err(xg, xo):.2e}")
    assert gi["iterations"] == 90 and gi["restarts"] == 2
    assert rel == pytest.approx(oi["rel_residual"], rel=1e-5)
    assert rel_err(xg, xo) <= 1e-7


def test_large_grid_sampled_tiles(B):
    """A 400x300x60 grid (7.2M cells): the RAS application on sampled tiles
    against the oracle's RAS of the extended tile alone (its solve depends on
    r inside the extended tile only)."""
    import torch
    c = cg.pressure_case(400, 300, 60, seed=16)
    coef = to_dev(c.coef.reshape(-1))
    pc = B.bo_ras_setup(grid_of(c), coef)
    r = np.random.default_rng(4).standard_normal(c.n)
    z = torch.zeros(c.n, dtype=torch.float64, device="cuda")
    B.bo_cpr_apply(pc, to_dev(r), z)
    zg = to_host(z).reshape(c.nz, c.ny, c.nx)
    R = r.reshape(c.nz, c.ny, c.nx)
    Cf = c.coef.reshape(7, c.nz, c.ny, c.nx)
    tx = ty = 6
    rng = np.random.default_rng(5)
    ntx, nty = (c.nx + tx - 1) // tx, (c.ny + ty - 1) // ty
    for _ in range(12):
        ti, tj = int(rng.integers(ntx)), int(rng.integers(nty))
        i0, j0 = ti * tx, tj * ty
        i1, j1 = min(i0 + tx, c.nx), min(j0 + ty, c.ny)
        e0, e1, f0, f1 = max(i0 - 1, 0), min(i1 + 1, c.nx), max(j0 - 1, 0), min(j1 + 1, c.ny)
        sub = Cf[:, :, f0:f1, e0:e1].copy()
        # couplings leaving the extended tile are not part of its matrix
        sub[2, :, :, 0] = 0.0
        sub[4, :, :, -1] = 0.0
        sub[1, :, 0, :] = 0.0
        sub[5, :, -1, :] = 0.0
        wx, wy = e1 - e0, f1 - f0
        one = PR.Ras(wx, wy, c.nz, sub.reshape(7, -1), (wx, wy), 0)
        zl = one.apply(R[:, f0:f1, e0:e1].reshape(-1)).reshape(c.nz, wy, wx)
        ref = zl[:, j0 - f0:j1 - f0, i0 - e0:i1 - e0]
        got = zg[:, j0:j1, i0:i1]
        assert rel_err(got.reshape(-1), ref.reshape(-1)) <= 1e-13, (ti, tj)


def test_ras_update_equals_fresh_setup(B):
    import torch
    c1 = cg.pressure_case(23, 17, 7, seed=17)
    c2 = cg.pressure_case(23, 17, 7, seed=18)
    pc = B.bo_ras_setup(grid_of(c1), to_dev(c1.coef.reshape(-1)))
    coef2 = to_dev(c2.coef.reshape(-1))
    B.bo_ras_update(pc, coef2)
    fresh = B.bo_ras_setup(grid_of(c2), coef2)
    r = to_dev(np.random.default_rng(6).standard_normal(c1.n))
    z1 = torch.zeros(c1.n, dtype=torch.float64, device="cuda")
    z2 = torch.zeros_like(z1)
    B.bo_cpr_apply(pc, r, z1)
    B.bo_cpr_apply(fresh, r, z2)
    assert torch.equal(z1, z2)

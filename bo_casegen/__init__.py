"""Seeded synthetic inputs for the black-oil Jacobian solve.

This module produces *input data only*: grids, rock fields, reservoir states,
well descriptions and fluid constants.  It contains none of the method's
arithmetic (no properties, fluxes, Jacobians or solvers); both the FP64 CPU
oracle and the HIP library consume what it produces, each through its own code.

Randomness is counter based so that any cell's value can be regenerated on its
own: u = (splitmix64(seed ^ (field_id << 48) ^ cell) >> 11 + 1/2) * 2^-53.
SplitMix64 is Steele, Lea and Flood's public-domain mixer; normals come from
the Box-Muller transform of two such uniforms.

Workloads (the paper's SPE10 / CMG data are not available, so these stand in
for them; the shapes follow the black-oil model of Section 2.1 with the
7-point finite-difference discretisation of Section 3):

The base state is 3000 psi, Sw 0.25, Sg 0.05, each with +-5% relative noise
that is spatially correlated (seeded lattice every 8x8x4 cells, trilinear in
between), so that neighbouring cells differ by at most a few per cent of the
noise amplitude, as in a Newton iterate of a real run.

* ``cfg 0``  20x20x5, log-normal k (ln 100 mD, sigma 1), injector and producer
  in opposite corners, one Jacobian at the first Newton iterate.
* ``cfg 1``  100x100x50, sinuous 1000 mD channels in a 10 mD log-normal
  background, five-spot wells, a 10-system synthetic step sequence.
* ``cfg 2``  200x200x50, log-normal k with sigma 2 and five 0.01 mD barrier
  layers, five-spot wells, the same 10-system sequence.
* ``tiny``   any small grid for pins and parity cases.
* ``two_phase(case)``  the oil-water version of any single-porosity case with
  fixed-BHP wells (Section 2.2): the same grid, rock, wells and oil / water
  state, no gas (S_g = 0) and dead oil (R_s = 0).
* ``pressure_case(nx, ny, nz)``  one scalar pressure system on a grid (the
  paper's pure linear-solver run solves such a system): a 7-point
  diagonally dominant M-matrix with log-normal face coefficients.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional

import numpy as np

__all__ = ["Well", "Case", "FLUID", "uniform", "normal", "make_case",
           "tiny_case", "base_seed", "N_SYSTEMS", "two_phase", "state2", "PressureCase", "pressure_case"]

N_SYSTEMS = 10

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, field_id: int, idx) -> np.ndarray:
    """Counter-based U(0,1) (never exactly 0 or 1) for element ``idx`` of field ``field_id``."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = np.uint64(seed) ^ (np.uint64(field_id) << np.uint64(48))
    z = _splitmix64(key ^ idx)
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def normal(seed: int, field_id: int, idx) -> np.ndarray:
    """Standard normal by Box-Muller from fields ``field_id`` and ``field_id + 1``."""
    u1 = uniform(seed, field_id, idx)
    u2 = uniform(seed, field_id + 1, idx)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# Fluid and rock constants (field units).  The paper leaves these to the input
# deck; the values are the ones every workload here uses.
FLUID = dict(
    p_ref=3000.0,                   # psi
    Bw0=1.01, cw=3.0e-6,            # B_w = Bw0 (1 - cw (p - p_ref))       rb/STB
    Bo0=1.25, co=1.0e-5,            # B_o                                  rb/STB
    Bg0=0.95, cg=3.0e-4,            # B_g                                  rb/Mscf
    Rs0=0.6, crs=2.0e-4,            # R_s = Rs0 (1 + crs (p - p_ref))      Mscf/STB
    mu_w=0.5, mu_o=2.0, mu_g=0.02,  # cP
    c_r=4.0e-6,                     # rock compressibility 1/psi
    rho_wsc=62.4, rho_osc=53.0, rho_gsc=0.0458,  # lbm/ft3, lbm/ft3, lbm/scf
    swc=0.2, sor=0.2, sorg=0.2, sgc=0.0,
    nw=2, no=2, ng=2,               # Corey exponents (integers)
    tcoef=0.001127,                 # Darcy constant, field units
    rb_ft3=5.615,                   # ft3 per reservoir barrel
    grav=1.0 / 144.0,               # psi per (lbm/ft3 * ft)
)


@dataclasses.dataclass
class Well:
    """A vertical well through cells (i, j, k_top..k_bot) (0-based)."""
    i: int
    j: int
    k_top: int
    k_bot: int
    kind: str            # "inj" (water injector) or "prod"
    control: str         # "bhp", or "wrat"/"orat"/"lrat" fixed rates
    target: float        # BHP in psi, or rate in STB/day
    rw: float = 0.25     # wellbore radius, ft
    skin: float = 0.0


@dataclasses.dataclass
class Case:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    top_depth: float
    kx: np.ndarray        # (N,) mD, cell g = i + nx*(j + ny*k)
    ky: np.ndarray
    kz: np.ndarray
    phi0: np.ndarray      # porosity at p_ref
    x_old: np.ndarray     # (3N,) interleaved (Po, Sw, Sg) per cell
    x_new: np.ndarray
    dt: float             # days
    wells: List[Well]
    fluid: dict
    gravity: bool = True
    inj_total_mobility: bool = True
    # dual porosity: matrix permeability (isotropic, for the transfer term) and
    # porosity per location; x_old / x_new then hold N fracture cells, N matrix
    # cells and one (p_h, 0, 0) triple per fixed-rate well
    dual: bool = False
    km: Optional[np.ndarray] = None
    phim: Optional[np.ndarray] = None
    sigma: float = 0.0
    # two-phase oil-water case (see two_phase): x_old / x_new keep the
    # three-slot layout with S_g = 0
    two_phase: bool = False

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nrate(self) -> int:
        return sum(1 for w in self.wells if w.control != "bhp")

    @property
    def rows(self) -> int:
        """Block rows of the system: cells (N or 2N) then fixed-rate wells."""
        return self.n * (2 if self.dual else 1) + self.nrate


def base_seed(cfg: int) -> int:
    return 1606000 + 100 * cfg


# field ids
_F_K, _F_PHI, _F_P, _F_SW, _F_SG, _F_CH = 1, 3, 4, 5, 6, 16


def _cell_ijk(nx, ny, nz):
    g = np.arange(nx * ny * nz, dtype=np.int64)
    return g % nx, (g // nx) % ny, g // (nx * ny)


NOISE_LATTICE = (8, 8, 4)


def smooth_noise(seed, field_id, nx, ny, nz, lattice=NOISE_LATTICE) -> np.ndarray:
    """Spatially correlated noise in [-1, 1]: i.i.d. U(-1,1) values on a coarse
    lattice with spacing ``lattice`` cells, trilinearly interpolated to cell
    centres (the weight of each of the 8 lattice corners is the product of
    its x, y and z weights, taken in that order)."""
    Lx, Ly, Lz = lattice
    mx, my, mz = nx // Lx + 2, ny // Ly + 2, nz // Lz + 2
    lat = (2.0 * uniform(seed, field_id, np.arange(mx * my * mz, dtype=np.uint64)) - 1.0).reshape(mz, my, mx)
    fx = (np.arange(nx, dtype=np.int64) + 0.5) / Lx
    fy = (np.arange(ny, dtype=np.int64) + 0.5) / Ly
    fz = (np.arange(nz, dtype=np.int64) + 0.5) / Lz
    ix, iy, iz = np.floor(fx).astype(np.int64), np.floor(fy).astype(np.int64), np.floor(fz).astype(np.int64)
    tx, ty, tz = fx - ix, fy - iy, fz - iz
    out = np.zeros((nz, ny, nx))
    for a in (0, 1):
        wx = tx if a else 1.0 - tx
        for b in (0, 1):
            wxy = wx[None, :] * (ty if b else 1.0 - ty)[:, None]
            for c in (0, 1):
                w = wxy[None, :, :] * (tz if c else 1.0 - tz)[:, None, None]
                out += w * lat[np.ix_(iz + c, iy + b, ix + a)]
    return out.reshape(-1)


def _noisy_state(seed, nx, ny, nz, p=3000.0, sw=0.25, sg=0.05, rel=0.05, noise="smooth"):
    """Base state with relative noise of amplitude ``rel``.  ``smooth``: the
    correlated field above (a physically plausible Newton state); ``iid``:
    independent per cell."""
    n = nx * ny * nz
    x = np.empty(3 * n)
    for q, (val, fid) in enumerate(((p, _F_P), (sw, _F_SW), (sg, _F_SG))):
        if noise == "iid":
            u = 2.0 * uniform(seed, fid, np.arange(n, dtype=np.uint64)) - 1.0
        else:
            u = smooth_noise(seed, fid, nx, ny, nz)
        x[q::3] = val * (1.0 + rel * u)
    return x


def _porosity(seed, n, lo=0.15, hi=0.25):
    return lo + (hi - lo) * uniform(seed, _F_PHI, np.arange(n, dtype=np.uint64))


def _lognormal(seed, n, mean_ln, sigma):
    return np.exp(mean_ln + sigma * normal(seed, _F_K, np.arange(n, dtype=np.uint64)))


def _channels(seed, nx, ny, nz, kbg, nchan=12, kch=1000.0):
    """Sinuous high-permeability channels: centreline y = y0 + a sin(2 pi x / lam + ph)."""
    k = kbg.copy()
    i, j, kk = _cell_ijk(nx, ny, nz)
    for c in range(nchan):
        u = uniform(seed, _F_CH + c, np.arange(8, dtype=np.uint64))
        y0 = u[0] * ny
        a = 5.0 + 10.0 * u[1]
        lam = 30.0 + 50.0 * u[2]
        ph = 2.0 * np.pi * u[3]
        width = 3.0 + 3.0 * u[4]
        thick = min(3 + int(6.0 * u[5]), 8, nz)
        k0 = int((nz - thick + 1) * u[6])
        yc = y0 + a * np.sin(2.0 * np.pi * (i + 0.5) / lam + ph)
        inside = (np.abs(j + 0.5 - yc) <= 0.5 * width) & (kk >= k0) & (kk < k0 + thick)
        k[inside] = kch
    return k


def _five_spot(nx, ny, nz, p_inj=3500.0, p_prod=2500.0):
    wells = [Well(i, j, 0, nz - 1, "inj", "bhp", p_inj)
             for (i, j) in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1))]
    wells.append(Well(nx // 2, ny // 2, 0, nz - 1, "prod", "bhp", p_prod))
    return wells


def _sequence_state(base, nx, ny, nz, dx, dy, wells, t):
    """Smooth synthetic state at time t (days): pressure rises near injectors and
    falls near the producer, a water front grows from the injectors."""
    if t == 0.0:
        return base.copy()
    # every quantity below depends on the column (i, j) only: computed on the
    # nx x ny columns and repeated over the layers
    i = np.arange(nx, dtype=np.int64)[None, :]
    j = np.arange(ny, dtype=np.int64)[:, None]
    xc, yc = (i + 0.5) * dx, (j + 0.5) * dy
    L = 0.2 * nx * dx
    inj = [w for w in wells if w.kind == "inj"]
    prod = [w for w in wells if w.kind == "prod"]
    d_inj = [np.hypot(xc - (w.i + 0.5) * dx, yc - (w.j + 0.5) * dy) for w in inj]
    d_prod = [np.hypot(xc - (w.i + 0.5) * dx, yc - (w.j + 0.5) * dy) for w in prod]
    layers = lambda a: np.broadcast_to(a, (nz, ny, nx)).reshape(-1)
    shape = layers(sum(np.exp(-d / L) for d in d_inj) - sum(np.exp(-d / L) for d in d_prod))
    x = base.copy()
    x[0::3] = base[0::3] + 300.0 * (1.0 - math.exp(-t / 10.0)) * shape
    dmin = layers(np.min(np.stack(d_inj), axis=0))
    R = 0.3 * nx * dx * math.sqrt(t / 30.0)
    sw0 = base[1::3]
    x[1::3] = sw0 + (0.75 - sw0) * 0.5 * (1.0 - np.tanh((dmin - R) / (3.0 * dx)))
    return x


def make_case(cfg: int, system: int = 1, noise: str = "smooth", field: int = 0) -> Case:
    """The synthetic Jacobian-producing state of workload ``cfg`` (0, 1 or 2).

    For cfg 0 the Jacobian is taken at the first Newton iterate
    (x_new == x_old, dt = 1 day).  For cfg 1 and 2, ``system`` k = 1..10 takes
    x_old = state(3(k-1) days) and x_new = state(3k days) with dt = 3 days.
    ``noise``: "smooth" (the correlated state noise) or "iid" (independent
    per cell; the case name then ends in "/iid").  cfg 3 is the learned
    stage's training set: the 200x200x50 recipe of cfg 2 on the fields of
    seeds 1606300 + ``field`` (cfg 2's own systems are its test set).
    """
    dx, dy, dz, top = 50.0, 50.0, 10.0, 8000.0
    if cfg == 0:
        nx, ny, nz = 20, 20, 5
        seed = base_seed(0)
        n = nx * ny * nz
        kx = _lognormal(seed, n, math.log(100.0), 1.0)
        wells = [Well(0, 0, 0, nz - 1, "inj", "bhp", 3500.0),
                 Well(nx - 1, ny - 1, 0, nz - 1, "prod", "bhp", 2500.0)]
        x = _noisy_state(seed, nx, ny, nz, noise=noise)
        return Case("cfg0" + ("/iid" if noise == "iid" else ""), nx, ny, nz, dx, dy, dz, top, kx, kx.copy(), 0.1 * kx,
                    _porosity(seed, n), x, x.copy(), 1.0, wells, dict(FLUID))
    if cfg in (1, 2, 3):
        if not 1 <= system <= N_SYSTEMS:
            raise ValueError("system must be in 1..10")
        seed = base_seed(cfg) + (field if cfg == 3 else 0)
        if cfg == 1:
            nx, ny, nz = 100, 100, 50
            n = nx * ny * nz
            kx = _channels(seed, nx, ny, nz, _lognormal(seed, n, math.log(10.0), 1.0))
            kz = 0.1 * kx
        else:
            nx, ny, nz = 200, 200, 50
            n = nx * ny * nz
            kx = _lognormal(seed, n, math.log(100.0), 2.0)
            kz = 0.1 * kx
            layer = np.arange(n) // (nx * ny)
            bar = np.isin(layer, (8, 17, 26, 35, 44))
            kx[bar] = 0.01
            kz[bar] = 0.01
        wells = _five_spot(nx, ny, nz)
        base = _noisy_state(seed, nx, ny, nz, noise=noise)
        x_old = _sequence_state(base, nx, ny, nz, dx, dy, wells, 3.0 * (system - 1))
        x_new = _sequence_state(base, nx, ny, nz, dx, dy, wells, 3.0 * system)
        name = f"cfg{cfg}.{system}" if cfg != 3 else f"cfg3/f{field}.{system}"
        return Case(name + ("/iid" if noise == "iid" else ""), nx, ny, nz, dx, dy, dz, top, kx,
                    kx.copy(), kz,
                    _porosity(seed, n), x_old, x_new, 3.0, wells, dict(FLUID))
    raise ValueError(f"unknown workload {cfg}")


def tiny_case(nx: int, ny: int, nz: int, seed: int = 7, *, sigma: float = 1.0,
              noise: float = 0.05, noise_kind: str = "smooth", wells: Optional[List[Well]] = None,
              dt: float = 1.0, step: float = 0.0, gravity: bool = True,
              kz_ratio: float = 0.1) -> Case:
    """A small seeded case.  ``step`` > 0 perturbs x_new away from x_old
    (relative, uniform) so that accumulation terms are active."""
    n = nx * ny * nz
    kx = _lognormal(seed, n, math.log(100.0), sigma)
    if wells is None:
        wells = [Well(0, 0, 0, nz - 1, "inj", "bhp", 3500.0),
                 Well(nx - 1, ny - 1, 0, nz - 1, "prod", "bhp", 2500.0)]
    x_old = _noisy_state(seed, nx, ny, nz, rel=noise, noise=noise_kind)
    x_new = x_old.copy()
    if step > 0.0:
        x_new = x_old * (1.0 + step * (2.0 * uniform(seed + 1, 30, np.arange(3 * n, dtype=np.uint64)) - 1.0))
    return Case(f"tiny{nx}x{ny}x{nz}", nx, ny, nz, 50.0, 50.0, 10.0, 8000.0, kx, kx.copy(),
                kz_ratio * kx, _porosity(seed, n), x_old, x_new, dt, wells, dict(FLUID),
                gravity=gravity)


def two_phase(case: Case) -> Case:
    """The oil-water version of a single-porosity case with fixed-BHP wells:
    S_g = 0 in both states (S_w kept), no dissolved gas (R_s = 0)."""
    if case.dual or any(w.control != "bhp" for w in case.wells):
        raise ValueError("two_phase needs a single-porosity case with fixed-BHP wells")
    fl = dict(case.fluid)
    fl["Rs0"] = 0.0
    fl["crs"] = 0.0
    xo, xn = case.x_old.copy(), case.x_new.copy()
    xo[2::3] = 0.0
    xn[2::3] = 0.0
    return dataclasses.replace(case, name=case.name + "/2p", x_old=xo, x_new=xn, fluid=fl, two_phase=True)


def state2(x: np.ndarray) -> np.ndarray:
    """(Po, Sw) per cell from a three-slot state."""
    return np.ascontiguousarray(np.asarray(x).reshape(-1, 3)[:, :2].reshape(-1))


@dataclasses.dataclass
class PressureCase:
    """A scalar system on an nx x ny x nz grid: coef[s, g] is the coefficient
    of row g on its neighbour through slot s (-z, -y, -x, diagonal, +x, +y,
    +z; 0 where the neighbour lies outside the grid), b the right-hand side."""
    name: str
    nx: int
    ny: int
    nz: int
    coef: np.ndarray   # (7, N)
    b: np.ndarray      # (N,)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


_F_PK, _F_PACC, _F_PP = 50, 51, 52


def pressure_case(nx: int, ny: int, nz: int, seed: int = 1606700, sigma: float = 1.5, acc: float = 1e-3,
                  well_index: float = 10.0, name: Optional[str] = None) -> PressureCase:
    """Seeded scalar pressure system.  Each cell draws a log-coefficient
    z_g = sigma N(0, 1); the face between cells a and b couples them by
    t = t_dir exp((z_a + z_b) / 2) with t_x = t_y = 1, t_z = 2.5, giving the
    off-diagonal entries -t; the diagonal is the sum of the cell's face
    coefficients plus an accumulation term acc * U(0.5, 1.5) and, in the
    five-spot columns (four corner injectors at 3500 psi, a central producer
    at 2500 psi), a well term well_index.  b = accumulation * p_old + well
    term * bhp with p_old = 3000 (1 + 0.05 U(-1, 1)).  Generated one layer
    of cells at a time (large grids)."""
    n = nx * ny * nz
    nxy = nx * ny
    coef = np.zeros((7, n))
    b = np.zeros(n)
    wells = [((0, 0), 3500.0), ((nx - 1, 0), 3500.0), ((0, ny - 1), 3500.0), ((nx - 1, ny - 1), 3500.0),
             ((nx // 2, ny // 2), 2500.0)]
    wcol = np.zeros(nxy)
    wbhp = np.zeros(nxy)
    for (i, j), p in wells:
        wcol[i + nx * j] = well_index
        wbhp[i + nx * j] = p
    ii = np.arange(nxy) % nx
    jj = np.arange(nxy) // nx

    def logc(k):
        return sigma * normal(seed, _F_PK, np.arange(k * nxy, (k + 1) * nxy, dtype=np.uint64))

    z_prev, z_cur = None, logc(0)
    for k in range(nz):
        z_next = logc(k + 1) if k + 1 < nz else None
        g0 = k * nxy
        diag = np.zeros(nxy)
        # x faces (slot 2: -x, slot 4: +x), y faces (1: -y, 5: +y), z faces (0: -z, 6: +z)
        tx = np.exp(0.5 * (z_cur[:-1] + z_cur[1:]))
        tx[(ii[:-1] == nx - 1)] = 0.0                  # no face across a row end
        cm = np.zeros(nxy); cm[1:] = -tx
        cp = np.zeros(nxy); cp[:-1] = -tx
        coef[2, g0:g0 + nxy] = cm
        coef[4, g0:g0 + nxy] = cp
        ty = np.exp(0.5 * (z_cur[:-nx] + z_cur[nx:])) if ny > 1 else np.zeros(0)
        cm = np.zeros(nxy); cm[nx:] = -ty
        cp = np.zeros(nxy); cp[:-nx] = -ty
        coef[1, g0:g0 + nxy] = cm
        coef[5, g0:g0 + nxy] = cp
        if z_prev is not None:
            coef[0, g0:g0 + nxy] = -2.5 * np.exp(0.5 * (z_prev + z_cur))
        if z_next is not None:
            coef[6, g0:g0 + nxy] = -2.5 * np.exp(0.5 * (z_cur + z_next))
        a = acc * (0.5 + uniform(seed, _F_PACC, np.arange(g0, g0 + nxy, dtype=np.uint64)))
        p_old = 3000.0 * (1.0 + 0.05 * (2.0 * uniform(seed, _F_PP, np.arange(g0, g0 + nxy, dtype=np.uint64)) - 1.0))
        off = coef[[0, 1, 2, 4, 5, 6], g0:g0 + nxy]
        coef[3, g0:g0 + nxy] = -off.sum(axis=0) + a + wcol
        b[g0:g0 + nxy] = a * p_old + wcol * wbhp
        z_prev, z_cur = z_cur, z_next
    del ii, jj
    return PressureCase(name or f"pressure{nx}x{ny}x{nz}", nx, ny, nz, coef, b)


# ---- learned pressure-stage correction: seeded initial weights ---------------
_F_CNN = 40


def cnn_init(seed: int = 1606300, channels=(2, 16, 16, 16, 1), last_scale: float = 0.1):
    """He-normal initial weights W[t, c_in, c_out] (27 taps) and zero biases
    per layer, float32, from the counter-based generator; the last layer is
    scaled by ``last_scale`` so that an untrained correction starts small."""
    params = []
    for l in range(len(channels) - 1):
        ci, co = channels[l], channels[l + 1]
        idx = np.arange(27 * ci * co, dtype=np.uint64)
        w = normal(seed, _F_CNN + l, idx).reshape(27, ci, co) * math.sqrt(2.0 / (27 * ci))
        if l == len(channels) - 2:
            w = w * last_scale
        params.append((w.astype(np.float32), np.zeros(co, dtype=np.float32)))
    return params


# ---- dual porosity with fixed-rate wells -----------------------------------------
_F_KM, _F_PHIM, _F_WJIT, _F_WCTRL, _F_MSTATE = 50, 51, 52, 53, 54
SHAPE_L = 10.0        # fracture spacing (ft) in each direction
PHI_F = 0.01          # fracture porosity


def kazemi_sigma(lx=SHAPE_L, ly=SHAPE_L, lz=SHAPE_L) -> float:
    """Shape factor sigma = 4 (1/Lx^2 + 1/Ly^2 + 1/Lz^2) (ft^-2)."""
    return 4.0 * (1.0 / lx ** 2 + 1.0 / ly ** 2 + 1.0 / lz ** 2)


def _dual_state(seed, nx, ny, nz, xf_old, xf_new, wells, lag=None):
    """Matrix cells lag the fractures by one step, with their own correlated
    noise; fixed-rate wells start from the target BHP of their kind."""
    n = nx * ny * nz
    if lag is None:
        lag = _matrix_lag(seed, nx, ny, nz)
    xm_new = xf_old.copy()
    xm_new[0::3] *= lag
    xm_old = xm_new.copy()
    xm_old[0::3] = xm_new[0::3] - 0.5 * (xf_new[0::3] - xf_old[0::3])
    wl = []
    for w in wells:
        if w.control != "bhp":
            wl += [3200.0 if w.kind == "inj" else 2800.0, 0.0, 0.0]
    wv = np.array(wl, dtype=np.float64)
    return (np.concatenate([xf_old, xm_old, wv]), np.concatenate([xf_new, xm_new, wv]))


def line_drive_wells(seed, nx, ny, nz, lines, cols, jitter, rate=2000.0):
    """Wells on lines j = lines[q] (injector and producer lines alternating),
    columns i = cols[r], jittered by up to +-jitter cells; each well's control
    (fixed BHP or fixed rate) by a seeded coin flip."""
    wells = []
    idx = 0
    for q, j0 in enumerate(lines):
        kind = "inj" if q % 2 == 0 else "prod"
        for i0 in cols:
            u = uniform(seed, _F_WJIT, np.array([2 * idx, 2 * idx + 1], dtype=np.uint64))
            i = int(min(max(i0 + round((2 * u[0] - 1) * jitter), 0), nx - 1))
            j = int(min(max(j0 + round((2 * u[1] - 1) * jitter), 0), ny - 1))
            flip = uniform(seed, _F_WCTRL, np.array([idx], dtype=np.uint64))[0] < 0.5
            if flip:
                wells.append(Well(i, j, 0, nz - 1, kind, "wrat" if kind == "inj" else "lrat", rate))
            else:
                wells.append(Well(i, j, 0, nz - 1, kind, "bhp", 3500.0 if kind == "inj" else 2500.0))
            idx += 1
    return wells


def _matrix_lag(seed, nx, ny, nz):
    return 1.0 + 0.02 * (smooth_noise(seed, _F_MSTATE, nx, ny, nz) - 0.5)


@functools.lru_cache(maxsize=1)
def _dual_fields(nx, ny, nz, seed, kf_mean, km_mean, sigma_ln):
    """The parts of a dual-porosity case that do not depend on the system of
    the step sequence (kept for the next system of the same field; callers
    must not modify the arrays)."""
    n = nx * ny * nz
    kx = _lognormal(seed, n, math.log(kf_mean), sigma_ln)
    km = np.exp(math.log(km_mean) + sigma_ln * normal(seed, _F_KM, np.arange(n, dtype=np.uint64)))
    phim = 0.15 + 0.10 * uniform(seed, _F_PHIM, np.arange(n, dtype=np.uint64))
    base = _noisy_state(seed, nx, ny, nz)
    lag = _matrix_lag(seed, nx, ny, nz)
    return kx, km, phim, base, lag


def make_dual_case(nx: int, ny: int, nz: int, seed: int, system: int = 1, wells=None,
                   kf_mean: float = 500.0, km_mean: float = 1.0, sigma_ln: float = 1.0, name=None) -> Case:
    """Dual-porosity case: fractures log-normal around kf_mean (kz = 0.1 kx),
    matrix log-normal around km_mean, phi_f = 0.01, phi_m = U[0.15, 0.25],
    the step sequence of the other workloads applied to the fractures."""
    dx, dy, dz, top = 50.0, 50.0, 10.0, 8000.0
    n = nx * ny * nz
    kx, km, phim, base, lag = _dual_fields(nx, ny, nz, seed, float(kf_mean), float(km_mean), float(sigma_ln))
    kx, km, phim = kx.copy(), km.copy(), phim.copy()
    if wells is None:
        wells = _five_spot(nx, ny, nz)
    xf_old = _sequence_state(base, nx, ny, nz, dx, dy, wells, 3.0 * (system - 1))
    xf_new = _sequence_state(base, nx, ny, nz, dx, dy, wells, 3.0 * system)
    x_old, x_new = _dual_state(seed, nx, ny, nz, xf_old, xf_new, wells, lag)
    return Case(name or f"dual{nx}x{ny}x{nz}.{system}", nx, ny, nz, dx, dy, dz, top, kx, kx.copy(), 0.1 * kx,
                np.full(n, PHI_F), x_old, x_new, 3.0, wells, dict(FLUID), dual=True, km=km, phim=phim,
                sigma=kazemi_sigma())


def make_cfg4(system: int = 1, scale: int = 1) -> Case:
    """The dual-porosity workload: 400x400x100 locations (32M cells), 20 wells
    on 4 lines x 5 columns with seeded jitter and controls.  ``scale`` > 1
    divides nx, ny by it and nz by half of it (a smaller twin for parity)."""
    nx, ny, nz = 400 // scale, 400 // scale, max(100 // max(scale // 2, 1), 4)
    def f(v):
        return int(round(v / scale)) if scale > 1 else v
    lines = [f(v) for v in (50, 150, 250, 350)]
    cols = [f(v) for v in (40, 120, 200, 280, 360)]
    wells = line_drive_wells(base_seed(4), nx, ny, nz, lines, cols, max(10 // scale, 1))
    return make_dual_case(nx, ny, nz, base_seed(4), system, wells, name=f"cfg4/{scale}.{system}")

"""Oracle (test infrastructure only): the two-phase oil-water model of
Section 2.2 and the CPR of its 2x2-block Jacobians.

The paper presents the two-phase model as the black-oil model with the gas
phase ignored: oil and water mass balances, S_o + S_w = 1, unknowns (p_o,
S_w).  This oracle takes exactly that reading.  Its residual and Jacobian
are the black-oil oracle's at S_g = 0 with no dissolved gas (R_s = 0, dead
oil), restricted to the oil and water rows (0, 1) and the (p_o, S_w)
columns (0, 1).  At S_g = 0 the gas mobility is zero and the Stone II oil
relative permeability equals the oil-water Corey curve (the gas-oil curve
is 1 there), up to rounding, so nothing of the gas phase enters these rows.

The CPR of a 2x2-block matrix is the black-oil oracle CPR applied to the
matrix embedded in 3x3 blocks with a decoupled third unknown: zero
couplings, a unit diagonal entry and a zero right-hand side.  Each stage
then acts on the first two components as the 2x2 form does and leaves the
third at zero: the quasi-IMPES weights get a zero third component (the
saturation-saturation block is diag(d_11, 1)), the decoupled pressure
block is the 2x2 system's, and block ILU(0) and block Jacobi keep the
diag(2x2, 1) structure of every block they form.
"""
from __future__ import annotations

import numpy as np


def problem(O, case):
    """The black-oil oracle problem of a two-phase case (bo_casegen.two_phase)."""
    if not getattr(case, "two_phase", False):
        raise ValueError("not a two-phase case")
    return O.Problem(case)


def _expand(x2):
    x2 = np.asarray(x2, dtype=np.float64).reshape(-1, 2)
    x3 = np.zeros((x2.shape[0], 3))
    x3[:, :2] = x2
    return x3.reshape(-1)


def residual(O, P, x_old2=None, x_new2=None, dt=None):
    """R (2N) of the two-phase model: oil and water rows at S_g = 0."""
    c = P.case
    xo = c.x_old if x_old2 is None else _expand(x_old2)
    xn = c.x_new if x_new2 is None else _expand(x_new2)
    R = O.residual(P, x_old=xo, x_new=xn, dt=dt)
    return restrict_vec(R)


def jacobian(O, P, x_old2=None, x_new2=None, dt=None):
    """(rowptr, colind, val (nnzb, 2, 2), R (2N))."""
    c = P.case
    xo = c.x_old if x_old2 is None else _expand(x_old2)
    xn = c.x_new if x_new2 is None else _expand(x_new2)
    rp, ci, val, R = O.jacobian(P, x_old=xo, x_new=xn, dt=dt)
    return rp, ci, np.ascontiguousarray(val[:, :2, :2]), restrict_vec(R)


def embed_blocks(rp, ci, val2):
    """3x3 blocks diag(B, 1) on the diagonal and [[B, 0], [0, 0]] elsewhere."""
    val2 = np.asarray(val2, dtype=np.float64).reshape(-1, 2, 2)
    v3 = np.zeros((len(val2), 3, 3))
    v3[:, :2, :2] = val2
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    v3[np.asarray(ci) == rows, 2, 2] = 1.0
    return v3


def embed_vec(v2):
    return _expand(v2)


def restrict_vec(v3):
    return np.ascontiguousarray(np.asarray(v3).reshape(-1, 3)[:, :2].reshape(-1))


def spmv(O, rp, ci, val2, x):
    return O.bsr_spmv(rp, ci, np.asarray(val2).reshape(-1), x, bs=2)


class Cpr2:
    """The oracle CPR of a 2x2-block system through the embedding; stages on
    2N-vectors (weights: 2N, pressure vectors: N)."""

    def __init__(self, O, P, rp, ci, val2, **kw):
        self.n = len(rp) - 1
        self.c3 = O.Cpr(P, rp, ci, embed_blocks(rp, ci, val2), **kw)

    def apply(self, v2):
        return restrict_vec(self.c3.apply(embed_vec(v2)))

    def fstage(self, r2):
        return restrict_vec(self.c3.fstage(embed_vec(r2)))

    def restrict(self, v2):
        return self.c3.restrict(embed_vec(v2))

    def vcycle(self, b):
        return self.c3.vcycle(b)

    def weights(self):
        return restrict_vec(self.c3.weights())

    def weights3(self):
        return self.c3.weights()

    def pivots(self):
        return self.c3.pivots()

    def nlevels(self):
        return self.c3.nlevels()

    def level(self, l):
        return self.c3.level(l)


def fgmres(O, rp, ci, val2, b2, pc: Cpr2, **kw):
    """The oracle FGMRES on the embedded system; (x (2N), info)."""
    x3, info = O.fgmres(rp, ci, embed_blocks(rp, ci, val2).reshape(-1), embed_vec(b2), pc.c3, **kw)
    return restrict_vec(x3), info

"""Pins of the oracle's aggregation-AMG setup rules on hand-built matrices
(CPU only), each chosen so that a plausible mistake fails it:

- strength: |a_ij| >= theta sqrt(|a_ii a_jj|) in either direction (the
  geometric mean of the two diagonals, absolute values, symmetrised), with
  couplings just above and just below the threshold;
- aggregation from given roots: phase 1 (every strong neighbour of a root
  joins it) and phase 2 (a remaining node joins the phase-1 aggregate of its
  strongest strong neighbour, the smaller aggregate id on a tie; weak
  neighbours and other phase-2 nodes never count; isolated nodes stay out);
- the smoothed prolongator on Neumann operators (zero row sums): with weak
  entries lumped into the filtered diagonal, P 1 = 1 exactly and the Galerkin
  product keeps the constant null space; omega = (4/3) / rho with rho the
  Gershgorin bound of D_F^-1 A_F, which is exactly 2 for these Laplacians
  (so omega = 2/3: a diagonal without the lumped weak entries gives another
  value)."""
import numpy as np
import scipy.sparse as sp


def csr(dense):
    A = sp.csr_matrix(np.asarray(dense, dtype=np.float64))
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


def flags(O, dense, theta=0.08):
    rp, ci, v = csr(dense)
    sf = O.amg_strength(rp, ci, v, theta)
    out = set()
    for i in range(len(rp) - 1):
        for e in range(rp[i], rp[i + 1]):
            if sf[e]:
                out.add((i, int(ci[e])))
    return out


def test_strength_threshold_is_the_geometric_mean_of_the_diagonals(oracle_lib):
    O = oracle_lib
    # (0,1): theta sqrt(4 * 1) = 0.16 < 0.161 -> strong; (1,2): theta sqrt(1 * 9)
    # = 0.24 > 0.239 -> weak (an arithmetic mean, a max or theta |a_ii| alone
    # would decide at least one of them the other way)
    M1 = [[4.0, -0.161, 0.0], [-0.161, 1.0, -0.239], [0.0, -0.239, 9.0]]
    assert flags(O, M1) == {(0, 1), (1, 0)}
    # one direction strong is enough (symmetrised): |a_01| = 0.1 < 0.16 but
    # |a_10| = 0.3 >= 0.16
    M2 = [[1.0, -0.1], [-0.3, 4.0]]
    assert flags(O, M2) == {(0, 1), (1, 0)}
    # absolute values: a positive coupling is as strong as a negative one
    M3 = [[1.0, 0.2], [0.2, 1.0]]
    assert flags(O, M3) == {(0, 1), (1, 0)}
    # negative diagonals: |a_ii a_jj|
    M4 = [[-4.0, 0.161], [0.161, -1.0]]
    assert flags(O, M4) == {(0, 1), (1, 0)}
    # theta 0: every stored off-diagonal coupling is strong, the diagonal never
    assert flags(O, M1, theta=0.0) == {(0, 1), (1, 0), (1, 2), (2, 1)}


def test_aggregation_phases_on_a_hand_built_graph(oracle_lib):
    O = oracle_lib
    n = 12
    D = np.eye(n)
    edges = {(0, 1): 0.5, (0, 2): 0.5, (0, 9): 0.5,          # root 0: phase 1 takes 1, 2, 9
             (6, 5): 0.5, (6, 4): 0.5,                       # root 6: phase 1 takes 5, 4
             (3, 2): 0.3, (3, 4): 0.5,                       # 3: strongest is 4 -> aggregate 1
             (7, 5): 0.4, (7, 9): 0.4,                       # 7: tie, 5 (agg 1) seen first -> aggregate 0
             (10, 4): 0.1, (10, 1): 0.05,                    # 10: 0.05 is weak -> aggregate 1
             (11, 3): 0.9, (11, 2): 0.2}                     # 11: 3 is a phase-2 node -> aggregate 0
    for (i, j), w in edges.items():
        D[i, j] = D[j, i] = -w
    rp, ci, v = csr(D)
    agg, nc = O.amg_aggregate(rp, ci, v, roots=[0, 6])
    assert nc == 2
    assert list(agg) == [0, 0, 0, 1, 1, 1, 1, 0, -1, 0, 1, 0]
    # aggregate ids follow the roots' order
    agg2, _ = O.amg_aggregate(rp, ci, v, roots=[6, 0])
    assert list(agg2) == list(agg)


def neumann_laplacian(nx, ny, nz, wz=1.0):
    """7-point graph Laplacian with unit x/y couplings and z couplings wz:
    zero row sums (no Dirichlet rows)."""
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    for axis, w in ((2, 1.0), (1, 1.0), (0, wz)):
        a = np.take(idx, range(idx.shape[axis] - 1), axis=axis).ravel()
        b = np.take(idx, range(1, idx.shape[axis]), axis=axis).ravel()
        rows += [a, b]; cols += [b, a]; vals += [np.full(a.size, -w)] * 2
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A = A + sp.diags(-np.asarray(A.sum(axis=1)).ravel())
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


def level_csr(L, key="p"):
    if key == "p":
        return sp.csr_matrix((L["p_val"], L["p_colind"], L["p_rowptr"]),
                             shape=(L["n"], int(L["p_colind"].max()) + 1))
    return sp.csr_matrix((L["val"], L["colind"], L["rowptr"]), shape=(L["n"], L["n"]))


def test_prolongator_keeps_constants_and_omega_is_two_thirds(oracle_lib):
    O = oracle_lib
    # isotropic, and with weak z couplings (2^-10 < theta sqrt(a_ii a_jj)),
    # which the filtered matrix lumps into its diagonal
    for wz in (1.0, 2.0 ** -10):
        A = neumann_laplacian(9, 7, 6, wz)
        h = O.AmgOnly(A.indptr, A.indices, A.data, coarse_max=20, keep_singular=True)
        # the Galerkin products keep the null space down to the coarsest
        # matrix, which the setup reports singular
        assert h.status == O.OR_ERR_SINGULAR_COARSE
        assert h.nlevels() >= 3
        for l in range(h.nlevels() - 1):
            L = h.level(l)
            assert (L["agg"] >= 0).all()            # every node aggregated (no isolated node)
            P = level_csr(L)
            one_f = P @ np.ones(P.shape[1])
            assert np.abs(one_f - 1.0).max() <= 1e-14, (wz, l)
            Al = level_csr(L, "a")
            if l == 0:
                assert L["omega"] == 2.0 / 3.0, (wz, L["omega"])
            # the next level is the Galerkin product and keeps the null space
            Ac = level_csr(h.level(l + 1), "a")
            ref = (P.T @ Al @ P).toarray()
            assert np.abs(Ac.toarray() - ref).max() <= 1e-13 * np.abs(ref).max()
            assert np.abs(Ac @ np.ones(Ac.shape[0])).max() <= 1e-12 * np.abs(ref).max()

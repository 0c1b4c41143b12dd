"""Oracle: transfer operators between nested uniform levels.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 3: prolongation I^l (coarse -> fine), restriction R^l = (I^l)^T, and a
projection P^l for iterates.  Readings: I is the nested Q1 interpolation
(fine node 2i -> coarse i with weight 1, fine node 2i+1 -> coarse i and i+1
with weight 1/2, tensor product over directions, the same for every
component); P is injection (fine node 2i -> coarse node i), so that P I = Id.
The coarse feasible set uses the monotone box restriction of the fine
correction box (Sec. 3.2 defers its construction to Kornhuber's monotone
multigrid): lo_H[j] = max_{i : I_ij > 0} lo[i], hi_H[j] = min_{i : I_ij > 0} hi[i].
"""
import numpy as np
import scipy.sparse as sp


def interp_1d(n_coarse_cells):
    """1D interpolation matrix, shape (2 Nc + 1, Nc + 1)."""
    nf, ncn = 2 * n_coarse_cells + 1, n_coarse_cells + 1
    rows, cols, vals = [], [], []
    for i in range(nf):
        if i % 2 == 0:
            rows.append(i); cols.append(i // 2); vals.append(1.0)
        else:
            rows += [i, i]; cols += [(i - 1) // 2, (i + 1) // 2]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, ncn))


def prolongation(d, n_coarse_cells, nc):
    """I acting on interleaved dof vectors (nc components per node)."""
    I1 = interp_1d(n_coarse_cells)
    In = I1
    for _ in range(d - 1):
        In = sp.kron(I1, In)          # slower index outside: x fastest
    I = sp.kron(In, sp.identity(nc)).tocsr()
    I.sum_duplicates()
    I.sort_indices()
    return I


def restriction(d, n_coarse_cells, nc):
    R = prolongation(d, n_coarse_cells, nc).T.tocsr()
    R.sort_indices()
    return R


def injection(d, n_coarse_cells, nc):
    """P: coarse node (i, j, k) takes the fine node (2i, 2j, 2k)."""
    ncn = n_coarse_cells + 1
    nfn = 2 * n_coarse_cells + 1
    idx = np.arange(ncn ** d)
    fine = np.zeros_like(idx)
    stride_c, stride_f = 1, 1
    rem = idx.copy()
    for _ in range(d):
        fine += 2 * (rem % ncn) * stride_f
        rem //= ncn
        stride_f *= nfn
    rows = (idx[:, None] * nc + np.arange(nc)[None, :]).reshape(-1)
    cols = (fine[:, None] * nc + np.arange(nc)[None, :]).reshape(-1)
    return sp.csr_matrix((np.ones(rows.shape[0]), (rows, cols)),
                         shape=(ncn ** d * nc, nfn ** d * nc))


def box_restrict(I, lo, hi):
    """Monotone restriction of a per-dof box through the support of I."""
    Ic = I.tocoo()
    sel = Ic.data > 0.0
    rows, cols = Ic.row[sel], Ic.col[sel]
    loH = np.full(I.shape[1], -np.inf)
    hiH = np.full(I.shape[1], np.inf)
    np.maximum.at(loH, cols, lo[rows])
    np.minimum.at(hiH, cols, hi[rows])
    return loH, hiH

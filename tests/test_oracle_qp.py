"""Pins for the oracle's box-QP solvers (PGS, MPRGP): on small convex
problems both must reach the solution that scipy's bounded least-squares
(BVLS) finds for the same QP, and satisfy the KKT conditions."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import lsq_linear

from oracle import fem, qp

RNG = np.random.default_rng(7)


def _problem(d, N, seed):
    rng = np.random.default_rng(seed)
    g = fem.Grid(d, N)
    mat = fem.material_from_E_nu(1.0, 0.3, 1e-3, 2.0 / N)
    x = rng.standard_normal(g.n_dofs) * 1e-4
    x.reshape(-1, d + 1)[:, d] = rng.uniform(0.0, 0.3, g.n_nodes)
    p = np.full(g.n_nodes, 1e-5)
    dirm = g.default_dirichlet()
    H = fem.hessian(g, x, p, mat, dirm)
    gv = rng.standard_normal(g.n_dofs) * 1e-3
    gv[dirm] = 0.0
    delta = 5e-3
    lo = np.full(g.n_dofs, -delta)
    hi = np.full(g.n_dofs, delta)
    ci = np.arange(g.n_nodes) * (d + 1) + d
    lo[ci] = np.maximum(-x[ci] * 0.5, -delta)   # some c bounds active
    lo[dirm] = hi[dirm] = 0.0
    return g, H, gv, lo, hi, dirm


def _reference(H, gv, lo, hi, free):
    Hf = H.toarray()[np.ix_(free, free)]
    Lc = sla.cholesky(Hf, lower=False)          # Hf = Lc^T Lc
    b = -sla.solve_triangular(Lc, gv[free], trans="T")
    res = lsq_linear(Lc, b, bounds=(lo[free], hi[free]), method="bvls", tol=1e-15)
    s = np.zeros(gv.shape[0])
    s[free] = res.x
    return s


def _kkt(H, gv, lo, hi, s, free):
    r = (gv + H @ s)[free]
    sf, lf, hf = s[free], lo[free], hi[free]
    inner = (sf > lf) & (sf < hf)
    worst = np.abs(r[inner]).max() if inner.any() else 0.0
    worst = max(worst, np.abs(np.minimum(r[sf <= lf], 0)).max() if (sf <= lf).any() else 0)
    worst = max(worst, np.abs(np.maximum(r[sf >= hf], 0)).max() if (sf >= hf).any() else 0)
    return worst


@pytest.mark.parametrize("d,N,seed", [(2, 4, 0), (3, 2, 1), (3, 3, 2)])
def test_pgs_converges_to_box_qp_solution(d, N, seed):
    g, H, gv, lo, hi, dirm = _problem(d, N, seed)
    free = ~dirm
    blocks = qp.colour_blocks(g.node_colour(), g.nc, 2 ** d)
    s = qp.pgs(H, gv, lo, hi, np.zeros(g.n_dofs), blocks, 3000, free)
    ref = _reference(H, gv, lo, hi, free)
    assert np.all(s >= lo) and np.all(s <= hi)
    assert np.abs(s - ref).max() <= 1e-9 * max(np.abs(ref).max(), 1e-30)
    assert _kkt(H, gv, lo, hi, s, free) <= 1e-12 * np.abs(gv).max()


@pytest.mark.parametrize("d,N,seed", [(2, 4, 3), (3, 2, 4), (3, 3, 5)])
def test_mprgp_solves_box_qp(d, N, seed):
    g, H, gv, lo, hi, dirm = _problem(d, N, seed)
    free = ~dirm
    s, its, status = qp.mprgp(H, gv, lo, hi, rtol=1e-12, max_it=5000)
    assert status == "converged"
    ref = _reference(H, gv, lo, hi, free)
    assert np.all(s >= lo) and np.all(s <= hi)
    assert np.abs(s - ref).max() <= 1e-8 * max(np.abs(ref).max(), 1e-30)


def test_pgs_single_sweep_is_sequential_gauss_seidel():
    """One symmetric sweep by colour blocks equals a plain dof-by-dof loop in
    the same order (the blocks are only a vectorisation)."""
    g, H, gv, lo, hi, dirm = _problem(2, 3, 9)
    free = ~dirm
    blocks = qp.colour_blocks(g.node_colour(), g.nc, 4)
    s = qp.pgs(H, gv, lo, hi, np.zeros(g.n_dofs), blocks, 1, free)
    Hd = H.toarray()
    order = [int(j) for J in blocks for j in J]
    t = np.zeros(g.n_dofs)
    fwd = order
    bwd = [int(j) for J in reversed(blocks) for j in J]
    for seq in (fwd, bwd):
        for j in seq:
            if not free[j]:
                continue
            r = gv[j] + Hd[j] @ t
            t[j] = min(max(t[j] - r / Hd[j, j], lo[j]), hi[j])
    assert np.allclose(s, t, rtol=1e-14, atol=1e-20)


def test_pgs_nonpositive_curvature_moves_to_better_bound():
    from scipy.sparse import csr_matrix
    H = csr_matrix(np.array([[-1.0, 0.0], [0.0, 0.0]]))
    gv = np.array([0.5, -0.25])
    lo, hi = np.array([-1.0, -2.0]), np.array([2.0, 1.0])
    s = qp.pgs(H, gv, lo, hi, np.zeros(2), [np.array([0]), np.array([1])], 1)
    # dof 0: m(t) = 0.5 t - 0.5 t^2: m(-1) = -1, m(2) = -1 -> tie -> lo
    # dof 1: m(t) = -0.25 t: best at hi = 1
    assert s[0] == -1.0 and s[1] == 1.0


def test_mprgp_negative_curvature_falls_back_to_separable_minimiser():
    """On a separable QP with indefinite diagonal H the first CG direction
    has p^T H p < 0: MPRGP must report it, and the PGS fallback must land on
    the closed-form box minimiser (per coordinate: clamp(-g/h) where h > 0,
    else the bound with the lower value g t + h t^2 / 2)."""
    from scipy.sparse import diags
    h = np.array([2.0, -1.0, 0.5, -3.0, 1.0, 0.0])
    gv = np.array([0.1, 1.0, -0.2, -2.0, 0.3, 0.4])
    lo = np.array([-1.0, -1.0, -0.1, -1.0, -2.0, -0.5])
    hi = np.array([1.0, 1.0, 0.3, 1.0, 2.0, 0.25])
    H = diags(h).tocsr()
    want = np.empty(h.size)
    for i in range(h.size):
        if h[i] > 0:
            want[i] = min(max(-gv[i] / h[i], lo[i]), hi[i])
        else:
            m = lambda t: gv[i] * t + 0.5 * h[i] * t * t  # noqa: E731
            want[i] = hi[i] if m(hi[i]) < m(lo[i]) else lo[i]
    blocks = [np.array([i]) for i in range(h.size)]
    s, its, status = qp.mprgp(H, gv, lo, hi, rtol=1e-12, max_it=100,
                              fallback=lambda s0: qp.pgs(H, gv, lo, hi, s0, blocks, 1))
    assert status == "negative_curvature" and its == 1
    assert np.allclose(s, want, rtol=0, atol=1e-15)
    assert qp.model_value(H, gv, s) < 0.0

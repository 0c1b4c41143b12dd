"""GPU vs oracle: projected Gauss-Seidel, transfers (bitwise), Galerkin
coarse operators, MPRGP (convex, and its negative-curvature fallback),
reductions."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, qp, transfer
from _util import material, rand_state, field_rel_err, ctx_for, dev, host

pytestmark = pytest.mark.gpu


def _box(g, x, delta, rng):
    d = g.d
    lo = np.full(g.n_dofs, -delta)
    hi = np.full(g.n_dofs, delta)
    ci = np.arange(g.n_nodes) * (d + 1) + d
    lo[ci] = np.maximum(-x[ci] * rng.uniform(0, 1, g.n_nodes), -delta)
    hi[ci] = np.minimum(1.0 - x[ci], delta)
    dirm = g.default_dirichlet()
    lo[dirm] = hi[dirm] = 0.0
    return lo, hi


@pytest.mark.parametrize("d,N,sweeps,split", [(2, 7, 1, 1), (2, 16, 1, 1), (3, 4, 1, 1), (3, 17, 1, 1),
                                               (2, 7, 3, 1), (2, 16, 3, 1), (3, 4, 3, 1), (3, 17, 3, 1),
                                               (2, 16, 3, 2), (3, 4, 3, 2), (3, 17, 3, 2)])
def test_pgs_matches_oracle(d, N, sweeps, split):
    """split 2: the spectral split's assembled stencil (principal axes and
    divided differences per quadrature point)."""
    print(f"case d={d} N={N} sweeps={sweeps} split={split}", flush=True)
    g, x, p = rand_state(d, N, seed=N + sweeps, u_scale=1e-4, c_max=0.6)
    mat = material(N, split)
    rng = np.random.default_rng(N)
    gv = rng.standard_normal(g.n_dofs) * 1e-4
    gv[g.default_dirichlet()] = 0.0
    lo, hi = _box(g, x, 2e-3, rng)
    H = fem.hessian(g, x, p, mat)
    blocks = qp.colour_blocks(g.node_colour(), g.nc, 2 ** d)
    so = qp.pgs(H, gv, lo, hi, np.zeros(g.n_dofs), blocks, sweeps, ~g.default_dirichlet())
    ctx = ctx_for(d, N, 1, mat)
    s = dev(np.zeros(g.n_dofs))
    ctx.smooth(1, dev(x), dev(p), dev(gv), dev(lo), dev(hi), s, sweeps)
    sh = host(s)
    assert np.all(sh >= lo) and np.all(sh <= hi)
    assert field_rel_err(sh, so, d) <= 1e-11


@pytest.mark.parametrize("d,Nc", [(2, 4), (2, 9), (3, 2), (3, 5)])
def test_transfers_bitwise(d, Nc):
    nc = d + 1
    rng = np.random.default_rng(Nc)
    I = transfer.prolongation(d, Nc, nc)
    R = transfer.restriction(d, Nc, nc)
    P = transfer.injection(d, Nc, nc)
    xc = rng.standard_normal(I.shape[1])
    xf = rng.standard_normal(I.shape[0])
    mat = material(2 * Nc)
    ctx = ctx_for(d, 2 * Nc, 2, mat)
    assert np.array_equal(host(ctx.prolong(1, dev(xc))), I @ xc)
    assert np.array_equal(host(ctx.restrict(2, dev(xf), 0)), R @ xf)
    assert np.array_equal(host(ctx.restrict(2, dev(xf), 1)), P @ xf)
    lo, hi = -np.abs(xf), np.abs(rng.standard_normal(xf.shape))
    loH, hiH = transfer.box_restrict(I, lo, hi)
    assert np.array_equal(host(ctx.restrict(2, dev(lo), 2)), loH)
    assert np.array_equal(host(ctx.restrict(2, dev(hi), 3)), hiH)


def _masked_galerkin(d, Nc, Hf):
    I = transfer.prolongation(d, Nc, d + 1)
    R = transfer.restriction(d, Nc, d + 1)
    gc = fem.Grid(d, Nc)
    Dc = sp.diags((~gc.default_dirichlet()).astype(float))
    return (Dc @ (R @ Hf @ I) @ Dc).tocsr(), gc


@pytest.mark.parametrize("d,N,L", [(2, 16, 3), (2, 14, 2), (3, 8, 3), (3, 12, 2), (3, 16, 4)])
def test_coarse_hessvec_is_dense_rap(d, N, L):
    """The load step's coarse Hessians (finest stencil coarsened direction by
    direction) equal D_c (I^T H I) D_c formed densely, level after level."""
    print(f"case d={d} N={N} L={L}", flush=True)
    g, x, p = rand_state(d, N, seed=5 * N + L)
    mat = material(N)
    ctx = ctx_for(d, N, L, mat)
    H = fem.hessian(g, x, p, mat)
    rng = np.random.default_rng(N)
    Hl, Nl = H, N
    for level in range(L - 1, 0, -1):
        Hl, gl = _masked_galerkin(d, Nl // 2, Hl)
        Nl //= 2
        v = rng.standard_normal(gl.n_dofs)
        ref = Hl @ v
        got = host(ctx.coarse_hessvec(level, dev(x), dev(p), dev(v)))
        assert field_rel_err(got, ref, d) <= 1e-12, (level, field_rel_err(got, ref, d))
        got32 = host(ctx.coarse_hessvec(level, dev(x), dev(p), dev(v), fp32_stencil=True))
        assert field_rel_err(got32, ref, d) <= 1e-5


def _masked_element_matrices(g, x, p, mat):
    """The level's own Hessian as element matrices (the oracle's), rows and
    columns of the default Dirichlet dofs zeroed: the input format of
    rmtr_mprgp."""
    dofs, Ke = fem.element_matrices(g, x, p, mat)
    free = (~g.default_dirichlet())[dofs].astype(float)
    return Ke * free[:, :, None] * free[:, None, :]


@pytest.mark.parametrize("d,N", [(2, 8), (3, 4), (3, 8)])
def test_mprgp_matches_oracle_on_convex_qp(d, N):
    print(f"case d={d} N={N}", flush=True)
    g, x, p = rand_state(d, N, seed=3 * N, u_scale=1e-5, p_scale=1e-6, c_max=0.3)
    mat = material(N)
    ctx = ctx_for(d, N, 1, mat)
    H = fem.hessian(g, x, p, mat)
    K = _masked_element_matrices(g, x, p, mat)
    rng = np.random.default_rng(2)
    gv = rng.standard_normal(g.n_dofs) * 1e-4
    gv[g.default_dirichlet()] = 0.0
    lo, hi = _box(g, x, 1e-3, rng)
    so, its_o, st_o = qp.mprgp(H, gv, lo, hi, rtol=1e-12, max_it=3000)
    s, its, st = ctx.mprgp(1, dev(K.reshape(-1)), dev(gv), dev(lo), dev(hi), max_it=3000, rtol=1e-12)
    assert st_o == "converged" and st == 0
    sh = host(s)
    assert np.all(sh >= lo) and np.all(sh <= hi)
    assert np.abs(sh - so).max() <= 1e-8 * np.abs(so).max()


@pytest.mark.parametrize("d,N", [(2, 4), (3, 2)])
def test_mprgp_negative_curvature_pgs_fallback(d, N):
    """Separable QP with an indefinite diagonal (Sec. 3.2.1, reading 16): the
    first MPRGP direction has p^T A p < 0, so the GPU must report status 2
    after one iteration and its PGS fallback must land on the closed-form box
    minimiser: clamp(-g/h) where h > 0, otherwise the bound with the lower
    value of g t + h t^2 / 2 (ties: lo), exactly as the oracle's fallback."""
    from scipy.sparse import diags
    print(f"case d={d} N={N}", flush=True)
    g = fem.Grid(d, N)
    mat = material(N)
    rng = np.random.default_rng(40 + d)
    dirm = g.default_dirichlet()
    h = rng.uniform(0.5, 2.0, g.n_dofs)
    neg = rng.uniform(0, 1, g.n_dofs) < 0.4
    h[neg] = -rng.uniform(0.5, 2.0, neg.sum())
    h[rng.uniform(0, 1, g.n_dofs) < 0.1] = 0.0
    h[dirm] = 1.0
    gv = rng.uniform(-1.0, 1.0, g.n_dofs) * np.where(h <= 0.0, 10.0, 0.1)
    lo = -rng.uniform(0.2, 1.0, g.n_dofs)
    hi = rng.uniform(0.2, 1.0, g.n_dofs)
    gv[dirm] = 0.0
    lo[dirm] = hi[dirm] = 0.0
    free = ~dirm
    assert np.sum(h[free] * gv[free] ** 2) < 0.0          # the first CG direction is g
    want = np.zeros(g.n_dofs)
    for i in np.nonzero(free)[0]:
        if h[i] > 0:
            want[i] = min(max(-gv[i] / h[i], lo[i]), hi[i])
        else:
            m = lambda t: gv[i] * t + 0.5 * h[i] * t * t  # noqa: E731
            want[i] = hi[i] if m(hi[i]) < m(lo[i]) else lo[i]
    # element matrices: each node's diagonal split evenly over the elements
    # around it (1, 2, 4 or 8 of them: exact in binary)
    ijk = g.node_ijk()
    count = np.prod(np.where((ijk == 0) | (ijk == N), 1, 2), axis=1)
    hs = (h.reshape(-1, d + 1) / count[:, None]).reshape(-1)
    dofs = g.elem_dofs()
    K = np.zeros((g.n_elems, dofs.shape[1], dofs.shape[1]))
    K[:, np.arange(dofs.shape[1]), np.arange(dofs.shape[1])] = hs[dofs]
    K *= free[dofs][:, :, None] * free[dofs][:, None, :]
    H = diags(np.where(free, h, 0.0)).tocsr()
    blocks = qp.colour_blocks(g.node_colour(), g.nc, 2 ** d)
    so, its_o, st_o = qp.mprgp(H, gv, lo, hi, rtol=1e-12, max_it=100,
                               fallback=lambda s0: qp.pgs(H, gv, lo, hi, s0, blocks, 50, free))
    assert st_o == "negative_curvature" and its_o == 1
    assert np.allclose(so, want, rtol=1e-14, atol=0)
    ctx = ctx_for(d, N, 1, mat)
    s, its, st = ctx.mprgp(1, dev(K.reshape(-1)), dev(gv), dev(lo), dev(hi), max_it=100, rtol=1e-12,
                           fallback_sweeps=50)
    assert st == 2 and its == 1
    assert np.allclose(host(s), want, rtol=1e-14, atol=0)


def test_dot_and_chi():
    d, N = 3, 9
    g, x, p = rand_state(d, N, seed=1)
    mat = material(N)
    ctx = ctx_for(d, N, 1, mat)
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(g.n_dofs), rng.standard_normal(g.n_dofs)
    assert float(host(ctx.dot(dev(a), dev(b)))[0]) == pytest.approx(float(a @ b), rel=1e-13)
    gr = fem.gradient(g, x, p, mat)
    cl = x[d::d + 1] * rng.uniform(0, 1, g.n_nodes)
    chi = float(host(ctx.chi(1, dev(x), dev(gr), dev(cl)))[0])
    assert chi == pytest.approx(fem.chi(g, x, gr, cl), rel=1e-13)


@pytest.mark.parametrize("d,N,split", [(2, 16, 1), (3, 17, 1), (3, 17, 2)])
def test_pgs_fp32_mixed(d, N, split):
    """FP32 stencil and sweeps (mixed form) vs the FP64 oracle: 3 sweeps of
    single-precision Gauss-Seidel agree to 1e-4 relative; bounds exact."""
    import torch
    g, x, p = rand_state(d, N, seed=77 + N, u_scale=1e-4, c_max=0.6)
    mat = material(N, split)
    rng = np.random.default_rng(N + 1)
    gv = rng.standard_normal(g.n_dofs) * 1e-4
    gv[g.default_dirichlet()] = 0.0
    lo, hi = _box(g, x, 2e-3, rng)
    lo32 = lo.astype(np.float32).astype(np.float64)
    hi32 = hi.astype(np.float32).astype(np.float64)
    H = fem.hessian(g, x, p, mat)
    blocks = qp.colour_blocks(g.node_colour(), g.nc, 2 ** d)
    so = qp.pgs(H, gv, lo32, hi32, np.zeros(g.n_dofs), blocks, 3, ~g.default_dirichlet())
    ctx = ctx_for(d, N, 1, mat)
    s = torch.zeros(g.n_dofs, dtype=torch.float32, device="cuda")
    ctx.smooth(1, dev(x), dev(p), dev(gv, torch.float32), dev(lo, torch.float32), dev(hi, torch.float32), s, 3)
    sh = host(s).astype(np.float64)
    assert np.all(sh >= lo32) and np.all(sh <= hi32)
    assert field_rel_err(sh, so, d) <= 1e-4

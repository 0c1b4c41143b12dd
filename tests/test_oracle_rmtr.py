"""Pins for the oracle's RMTR: level-objective consistency (by finite
differences), the patch test, the one-level special case (plain TR), the
decrease/feasibility invariants, the AT2 1D profile and Sneddon's opening."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fem, fields, qp, rmtr, transfer

RNG = np.random.default_rng(11)


def _setup(d, N, L, p0=1e-3, seed=0):
    rng = np.random.default_rng(seed)
    g = fem.Grid(d, N)
    mat = fem.material_from_E_nu(1.0, 0.3, 1e-3, 2.0 / N)
    c0 = np.zeros(g.n_nodes)
    ijk = g.node_ijk()
    mid = N // 2
    band = (np.abs(ijk[:, 1] - mid) <= 1) & (ijk[:, 0] >= N // 4) & (ijk[:, 0] <= 3 * N // 4)
    if d == 3:
        band &= (ijk[:, 2] >= N // 4) & (ijk[:, 2] <= 3 * N // 4)
    c0[band] = 1.0
    p = np.full(g.n_nodes, p0)
    x = np.zeros(g.n_dofs)
    x[d::d + 1] = c0
    return g, mat, c0, p, x


@pytest.mark.parametrize("d,N,L", [(2, 8, 2), (3, 4, 2)])
@pytest.mark.parametrize("model", ["energy", "zero", "fine"])
def test_level_objective_first_and_second_order_consistency(d, N, L, model):
    g, mat, c0, p, x = _setup(d, N, L)
    x = x + RNG.standard_normal(x.shape) * 1e-3
    x[g.default_dirichlet()] = 0.0
    x[d::d + 1] = np.clip(x[d::d + 1], c0, 1.0)
    s = rmtr.RMTR(d, N, L, mat, p, rmtr.Params(coarse_model=model))
    fine = s.levels[L]
    fine.Lb = np.full(g.n_dofs, -np.inf); fine.Ub = np.full(g.n_dofs, np.inf)
    fine.x0 = x.copy()
    fine.Hmod = fem.hessian(g, x, p, mat)
    s.setup_coarse(L, x, 0.5)
    c = s.levels[L - 1]
    # first order: grad h^{l-1}(x0) = R grad f(x)
    gc = s.h_grad(c, c.x0)
    Rg = s.R[L - 1] @ fem.gradient(g, x, p, mat)
    Rg[c.dirichlet] = 0.0
    assert np.allclose(gc, Rg, rtol=0, atol=1e-13 * np.abs(Rg).max())
    # second order, by central differences of the coarse gradient
    v = RNG.standard_normal(c.x0.shape)
    v[c.dirichlet] = 0.0
    eta = 1e-6
    fd = (s.h_grad(c, c.x0 + eta * v) - s.h_grad(c, c.x0 - eta * v)) / (2 * eta)
    RHIv = s.R[L - 1] @ (fine.Hmod @ (s.I[L - 1] @ v))
    RHIv[c.dirichlet] = 0.0
    assert np.abs(fd - RHIv).max() <= 1e-7 * np.abs(RHIv).max()
    # h_diff is the integral of h_grad (central differences of h along v)
    w = RNG.standard_normal(c.x0.shape) * 1e-3
    w[c.dirichlet] = 0.0
    xa = c.x0 + w
    dh = (s.h_diff(c, xa, eta * v) - s.h_diff(c, xa, -eta * v)) / (2 * eta)
    assert dh == pytest.approx(float(s.h_grad(c, xa) @ v), rel=1e-6)


@pytest.mark.parametrize("d,N,L", [(2, 8, 3), (3, 4, 2)])
def test_patch_test_affine_dirichlet_frozen_c(d, N, L):
    """c frozen (all c dofs fixed), affine Dirichlet data, uniform p: the
    problem is quadratic in u and its minimiser is the affine field."""
    g = fem.Grid(d, N)
    mat = fem.material_from_E_nu(1.0, 0.3, 1e-3, 2.0 / N)
    A = np.eye(d) * 1e-3 + RNG.standard_normal((d, d)) * 2e-4
    X = g.node_coords()
    xa = np.zeros(g.n_dofs)
    xa.reshape(-1, d + 1)[:, :d] = X @ A.T
    xa.reshape(-1, d + 1)[:, d] = 0.25
    dirm = g.default_dirichlet()
    dirm.reshape(-1, d + 1)[:, d] = True
    x = xa.copy()
    x[~dirm] = 0.0
    p = np.full(g.n_nodes, 1e-3)
    prm = rmtr.Params(rtol=1e-12, max_vcycles=300)
    solver = rmtr.RMTR(d, N, L, mat, p, prm, dirichlet=dirm)
    c_low = np.full(g.n_nodes, 0.25)
    xs, st = solver.solve_loadstep(x, c_low)
    assert st.chi <= 1e-12 * st.chi0
    assert np.abs(xs - xa).max() <= 1e-10 * np.abs(xa).max()


def test_one_level_is_plain_trust_region():
    d, N = 2, 6
    g, mat, c0, p, x = _setup(d, N, 1, p0=5e-3)
    prm = rmtr.Params(max_vcycles=4)
    solver = rmtr.RMTR(d, N, 1, mat, p, prm)
    xs, st = solver.solve_loadstep(x.copy(), c0)
    # independent plain TR loop: Hessian frozen per outer cycle, MPRGP QPs
    dirm = g.default_dirichlet()
    free = ~dirm
    blocks = qp.colour_blocks(g.node_colour(), g.nc, 4)
    Lb = np.full(g.n_dofs, -np.inf); Ub = np.full(g.n_dofs, np.inf)
    Lb[d::d + 1] = c0; Ub[d::d + 1] = 1.0
    y = x.copy()
    delta = prm.delta0
    fref = abs(fem.energy(g, y, p, mat)) / np.sqrt(g.n_elems)
    for cyc in range(4):
        H = fem.hessian(g, y, p, mat)
        for it in range(prm.coarse_tr_its):
            gr = fem.gradient(g, y, p, mat)
            lo = np.maximum(Lb - y, -delta); hi = np.minimum(Ub - y, delta)
            lo[dirm] = hi[dirm] = 0.0
            fb = lambda s0: qp.pgs(H, gr, lo, hi, s0.copy(), blocks, prm.fallback_sweeps, free)
            s, _, _ = qp.mprgp(H, gr, lo, hi, None, prm.coarse_qp_rtol, prm.coarse_qp_its, fallback=fb)
            if not np.any(s != 0):
                continue
            pred = -(gr @ s + 0.5 * s @ (H @ s))
            ared = -fem.energy_diff(g, y, s, p, mat)
            tol = 1e-14 * fref
            if abs(pred) <= tol:
                rho = 1.0 if ared >= -tol else -np.inf
            elif pred <= 0:
                rho = -np.inf
            else:
                rho = ared / pred
            if rho > prm.eta1:
                y = y + s
            if rho < prm.eta1:
                delta *= prm.gamma1
            elif rho > prm.eta2:
                delta = min(prm.gamma2 * delta, prm.delta_max)
    assert np.array_equal(xs, y)


@pytest.mark.parametrize("d,N,L", [(2, 16, 3), (3, 4, 2)])
def test_rmtr_invariants(d, N, L):
    g, mat, c0, p, x = _setup(d, N, L, p0=2e-3)
    prm = rmtr.Params(max_vcycles=60)
    solver = rmtr.RMTR(d, N, L, mat, p, prm)
    f_prev = fem.energy(g, x, p, mat)
    energies = [f_prev]
    orig = solver.vcycle

    def tracked(l, xx, delta):
        out = orig(l, xx, delta)
        if l == L:
            energies.append(fem.energy(g, out[0], p, mat))
        return out

    solver.vcycle = tracked
    xs, st = solver.solve_loadstep(x.copy(), c0)
    assert st.chi <= prm.rtol * st.chi0
    assert np.all(np.diff(energies) <= 1e-15 * max(1.0, abs(energies[0])))
    c = xs[d::d + 1]
    assert np.all(c >= c0) and np.all(c <= 1.0)
    assert np.all(xs[g.default_dirichlet()] == 0.0)


def thomas(a, b, c, r):
    n = len(b)
    cp, dp = np.zeros(n), np.zeros(n)
    cp[0], dp[0] = c[0] / b[0], r[0] / b[0]
    for i in range(1, n):
        m = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / m if i < n - 1 else 0.0
        dp[i] = (r[i] - a[i] * dp[i - 1]) / m
    x = np.zeros(n)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def at2_profile_1d(N, ls):
    """Discrete 1D AT2 profile with c(1/2) = 1: Q1 mass and stiffness
    (int c^2 exact, int c'^2 exact), solved by the Thomas algorithm."""
    h = 1.0 / N
    n = N + 1
    a, b, c = np.zeros(n), np.zeros(n), np.zeros(n)
    for e in range(N):
        Me = h / 6 * np.array([[2, 1], [1, 2]]) / ls
        Ke = ls / h * np.array([[1, -1], [-1, 1]])
        Ae = Me + Ke
        i = e
        b[i] += Ae[0, 0]; c[i] += Ae[0, 1]
        a[i + 1] += Ae[1, 0]; b[i + 1] += Ae[1, 1]
    r = np.zeros(n)
    m = N // 2
    a[m], c[m], b[m], r[m] = 0.0, 0.0, 1.0, 1.0
    # eliminate the fixed value from the neighbouring rows
    r[m - 1] -= c[m - 1] * 1.0; c[m - 1] = 0.0
    r[m + 1] -= a[m + 1] * 1.0; a[m + 1] = 0.0
    return thomas(a, b, c, r)


def test_at2_profile_matches_1d_reaction_diffusion():
    """u = 0 (all displacements fixed), p = 0, c = 1 imposed on the line
    x = 1/2: the phase field solves the 1D Q1 problem along x."""
    d, N, L = 2, 32, 3
    g = fem.Grid(d, N)
    ls = 2.0 / N
    mat = fem.material_from_E_nu(1.0, 0.3, 1e-3, ls)
    dirm = np.zeros(g.n_dofs, bool)
    dirm.reshape(-1, 3)[:, :2] = True
    c_low = np.zeros(g.n_nodes)
    c_low[g.node_ijk()[:, 0] == N // 2] = 1.0
    x = np.zeros(g.n_dofs)
    x[2::3] = c_low
    prm = rmtr.Params(rtol=1e-12, max_vcycles=300)
    solver = rmtr.RMTR(d, N, L, mat, np.zeros(g.n_nodes), prm, dirichlet=dirm)
    xs, st = solver.solve_loadstep(x, c_low)
    c = xs[2::3].reshape(N + 1, N + 1)
    prof = at2_profile_1d(N, ls)
    for j in range(N + 1):
        assert np.abs(c[j] - prof).max() <= 1e-10


def test_at2_profile_continuum_limit():
    """With l resolved by several cells the discrete profile approaches
    exp(-|x - 1/2| / l) (Sec. 2: AT2 model)."""
    N, ls = 256, 0.04
    prof = at2_profile_1d(N, ls)
    xs = np.arange(N + 1) / N
    exact = np.exp(-np.abs(xs - 0.5) / ls)
    assert np.abs(prof - exact).max() < 5e-3


@pytest.mark.slow
def test_sneddon_opening_c1():
    """C1 (64^2, one pressurised crack): the crack opens (positive jump of
    u_y across y = 1/2), symmetric in x, with a magnitude near Sneddon's
    4 p a / E' = 3.64e-4 at the centre (loose: the crack band is 3 nodes wide
    and the domain is finite)."""
    wl = W.WORKLOADS["c1_2d_64"]
    g = fem.Grid(2, 64)
    c0, p = fields.initial_fields(g, wl.fractures(), p_uniform=wl.p)
    mat = fem.material_from_E_nu(wl.E, wl.nu, wl.Gc, wl.ls, wl.k)
    x = np.zeros(g.n_dofs)
    x[2::3] = c0
    solver = rmtr.RMTR(2, 64, 3, mat, p)
    xs, st = solver.solve_loadstep(x, c0)
    assert st.chi <= 1e-8 * st.chi0
    uy = xs[1::3].reshape(65, 65)
    off = 8                                        # 4 l = 8 h
    cod = uy[32 + off, :] - uy[32 - off, :]
    Ep = wl.E / (1 - wl.nu ** 2)
    sned = 4 * wl.p * 0.1 / Ep
    assert cod[32] > 0.0
    assert 0.5 * sned < cod[32] < 2.0 * sned
    assert np.allclose(cod, cod[::-1], rtol=1e-6, atol=1e-12)
    assert cod[32] > cod[26] > cod[20]


def _sneddon_error(N, L):
    """The oracle's C1-type load step on N^2 cells (crack half-length
    a = 0.1, p = 1e-3, l_s = 2h): the phase-field crack opening
    w(x) = -int u_y dc/dy dy against Sneddon's 4 p a / E' sqrt(1 - x^2/a^2),
    largest error over |x - 1/2| <= 0.8 a relative to the centre value."""
    g = fem.Grid(2, N)
    c0, p = fields.initial_fields(g, W.fractures.c1_crack(N, 1e-3), p_uniform=1e-3)
    mat = fem.material_from_E_nu(1.0, 0.3, 1e-3, 2.0 / N)
    x = np.zeros(g.n_dofs)
    x[2::3] = c0
    xs, st = rmtr.RMTR(2, N, L, mat, p).solve_loadstep(x, c0)
    assert st.chi <= 1e-8 * st.chi0
    uy = xs[1::3].reshape(N + 1, N + 1)
    c = xs[2::3].reshape(N + 1, N + 1)
    xc = np.arange(N + 1) / N
    a, Ep = 0.1, 1.0 / (1 - 0.3 ** 2)
    sned = 4 * 1e-3 * a / Ep * np.sqrt(np.clip(1 - ((xc - 0.5) / a) ** 2, 0, None))
    w = -np.trapezoid(uy * np.gradient(c, 1.0 / N, axis=0), dx=1.0 / N, axis=0)
    inside = np.abs(xc - 0.5) <= 0.8 * a
    return np.abs(w - sned)[inside].max() / sned.max()


@pytest.mark.slow
def test_sneddon_opening_converges_under_refinement():
    """Sneddon's opening under refinement (the crack fixed, l_s = 2h -> 0):
    the phase-field opening's error falls from 32^2 to 64^2 cells (0.134 ->
    0.100; 0.087 at 128^2, and on the GPU 0.073 at 256^2)."""
    e32, e64 = _sneddon_error(32, 2), _sneddon_error(64, 3)
    assert e64 < e32 < 0.2


@pytest.mark.parametrize("d,N,L", [(2, 8, 3), (3, 4, 2)])
@pytest.mark.parametrize("model", ["energy", "fine"])
def test_first_order_coarse_model(d, N, L, model):
    """First-order variant: grad h^{l-1}(x0) = R grad f(x) still holds, but
    the coarse Hessian is grad^2 f~ at x0 (by central differences of the
    coarse functional's own gradient), not R H I; for the "fine" model
    f~(x) = f(I x), whose gradient is I^T grad f(I x) (central differences
    of its energy differences).  The central differences use a step small
    enough that no Gauss point crosses the kink of the split (the energy is
    piecewise quadratic in u, so the differences are exact up to rounding
    away from it)."""
    rng = np.random.default_rng(100 * d + N + L)
    g, mat, c0, p, x = _setup(d, N, L)
    x = x + rng.standard_normal(x.shape) * 1e-3
    x[g.default_dirichlet()] = 0.0
    x[d::d + 1] = np.clip(x[d::d + 1], c0, 1.0)
    s = rmtr.RMTR(d, N, L, mat, p, rmtr.Params(coarse_model=model, first_order=True))
    fine = s.levels[L]
    fine.Lb = np.full(g.n_dofs, -np.inf); fine.Ub = np.full(g.n_dofs, np.inf)
    fine.x0 = x.copy()
    fine.Hmod = fem.hessian(g, x, p, mat)
    s.setup_coarse(L, x, 0.5)
    c = s.levels[L - 1]
    Rg = s.R[L - 1] @ fem.gradient(g, x, p, mat)
    Rg[c.dirichlet] = 0.0
    assert np.allclose(s.h_grad(c, c.x0), Rg, rtol=0, atol=1e-13 * np.abs(Rg).max())
    v = rng.standard_normal(c.x0.shape)
    v[c.dirichlet] = 0.0
    eta = 1e-8
    fd = (s.h_grad(c, c.x0 + eta * v) - s.h_grad(c, c.x0 - eta * v)) / (2 * eta)
    fdf = (s.ft_grad(c, c.x0 + eta * v) - s.ft_grad(c, c.x0 - eta * v)) / (2 * eta)
    assert np.abs(fd - fdf).max() <= 1e-7 * np.abs(fdf).max()
    assert np.abs(c.Hmod @ v - fdf).max() <= 1e-6 * np.abs(fdf).max()
    RHIv = s.R[L - 1] @ (fine.Hmod @ (s.I[L - 1] @ v))
    RHIv[c.dirichlet] = 0.0
    assert np.abs(fd - RHIv).max() > 1e-3 * np.abs(RHIv).max()   # not the Galerkin product
    # grad f~ is the derivative of f~ (energy differences along w)
    w = rng.standard_normal(c.x0.shape) * 1e-3
    w[c.dirichlet] = 0.0
    xa = c.x0 + w
    dfd = (s.ft_diff(c, xa, eta * v) - s.ft_diff(c, xa, -eta * v)) / (2 * eta)
    assert dfd == pytest.approx(float(s.ft_grad(c, xa) @ v), rel=1e-6)


@pytest.mark.parametrize("model,first", [("fine", False), ("energy", True), ("fine", True), ("zero", False)])
def test_coarse_model_variants_converge(model, first):
    """Every coarse-model variant keeps RMTR's guarantees: the energy never
    rises at the end of a V-cycle, the iterates stay feasible and chi reaches
    1e-8 chi0."""
    d, N, L = 2, 16, 3
    g, mat, c0, p, x = _setup(d, N, L, p0=2e-3)
    solver = rmtr.RMTR(d, N, L, mat, p, rmtr.Params(coarse_model=model, first_order=first, max_vcycles=150))
    xs, st = solver.solve_loadstep(x.copy(), c0)
    assert st.chi <= 1e-8 * st.chi0
    c = xs[d::d + 1]
    assert np.all(c >= c0) and np.all(c <= 1.0)
    assert np.all(xs[g.default_dirichlet()] == 0.0)
    assert st.energy <= fem.energy(g, x, p, mat)


def test_first_order_needs_a_coarse_functional():
    g, mat, c0, p, x = _setup(2, 8, 2)
    with pytest.raises(ValueError):
        rmtr.RMTR(2, 8, 2, mat, p, rmtr.Params(coarse_model="zero", first_order=True))

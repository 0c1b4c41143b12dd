"""Pins for the oracle's discrete functional, gradient and Hessian.

Each check uses something other than the oracle's own formulas: an
independently assembled Voigt-notation Q1 stiffness, the paper's unsplit
density psi_e, the divergence theorem, rigid motions, closed-form integrals of
affine fields, finite differences, and symmetry.
"""
import itertools

import numpy as np
import pytest

from oracle import fem

RNG = np.random.default_rng(12345)


def _mat(split=True, N=4):
    return fem.material_from_E_nu(1.0, 0.3, 1e-3, 2.0 / N, 1e-6, split)


def voigt_stiffness(d, N, lam, mu):
    """Q1 elasticity stiffness for the displacement dofs only (d per node),
    written independently: reference cell [-1, 1]^d, Voigt strains, textbook
    isotropic D, 2-point Gauss from numpy's Legendre routine."""
    h = 1.0 / N
    pts, wts = np.polynomial.legendre.leggauss(2)
    nloc = 2 ** d
    corners = [tuple(2 * ((a >> i) & 1) - 1 for i in range(d)) for a in range(nloc)]
    if d == 3:
        D = np.zeros((6, 6))
        D[:3, :3] = lam
        D[[0, 1, 2], [0, 1, 2]] = lam + 2 * mu
        D[[3, 4, 5], [3, 4, 5]] = mu
    else:
        D = np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, mu]])
    Ke = np.zeros((d * nloc, d * nloc))
    for gq in itertools.product(range(2), repeat=d):
        xi = [pts[i] for i in gq]
        wq = np.prod([wts[i] for i in gq]) * (h / 2) ** d
        dN = np.zeros((nloc, d))
        for a, cr in enumerate(corners):
            for j in range(d):
                v = cr[j] / 2 ** d
                for i in range(d):
                    if i != j:
                        v *= 1 + cr[i] * xi[i]
                dN[a, j] = v * (2.0 / h)
        if d == 3:
            Bm = np.zeros((6, 3 * nloc))
            for a in range(nloc):
                x, y, z = dN[a]
                Bm[:, 3 * a:3 * a + 3] = [[x, 0, 0], [0, y, 0], [0, 0, z],
                                          [0, z, y], [z, 0, x], [y, x, 0]]
        else:
            Bm = np.zeros((3, 2 * nloc))
            for a in range(nloc):
                x, y = dN[a]
                Bm[:, 2 * a:2 * a + 2] = [[x, 0], [0, y], [y, x]]
        Ke += wq * Bm.T @ D @ Bm
    g = fem.Grid(d, N)
    en = g.elem_nodes()
    Kg = np.zeros((d * g.n_nodes, d * g.n_nodes))
    for e in range(en.shape[0]):
        dofs = (en[e][:, None] * d + np.arange(d)[None, :]).reshape(-1)
        Kg[np.ix_(dofs, dofs)] += Ke
    return Kg


@pytest.mark.parametrize("d,N", [(2, 4), (3, 2)])
@pytest.mark.parametrize("split", [True, False])
def test_intact_elasticity_matches_voigt_stiffness(d, N, split):
    g = fem.Grid(d, N)
    mat = _mat(split, N)
    x = np.zeros(g.n_dofs)
    ui = np.arange(g.n_dofs).reshape(-1, d + 1)[:, :d].reshape(-1)
    u = RNG.standard_normal(ui.size)
    x[ui] = u
    p = np.zeros(g.n_nodes)
    K = voigt_stiffness(d, N, mat.lam, mat.mu)
    nodir = np.zeros(g.n_dofs, bool)
    assert fem.energy(g, x, p, mat) == pytest.approx(0.5 * u @ K @ u, rel=1e-13)
    gr = fem.gradient(g, x, p, mat, nodir)
    assert np.allclose(gr[ui], K @ u, rtol=0, atol=1e-13 * np.abs(K @ u).max())
    H = fem.hessian(g, x, p, mat, nodir).toarray()
    assert np.allclose(H[np.ix_(ui, ui)], K, rtol=0, atol=1e-13 * np.abs(K).max())


def psi_e(eps, lam, mu):
    """The paper's strain energy density (Sec. 2)."""
    return 0.5 * lam * np.trace(eps) ** 2 + mu * np.sum(eps * eps)


@pytest.mark.parametrize("d", [2, 3])
def test_affine_state_closed_form(d):
    """Affine u, uniform c, uniform p: f = |Omega| (split density + AT2 + p work).
    For tr eps > 0 the split degrades all of psi_e; for pure compression only
    the deviatoric part (zero here) is degraded and the bulk part K/2 t^2 stays."""
    N = 3
    g = fem.Grid(d, N)
    X = g.node_coords()
    cbar, pval = 0.3, 0.02
    for kind in ("tension", "compression"):
        mat = _mat(True, N)
        if kind == "tension":
            A = RNG.standard_normal((d, d)) * 0.1 + 0.5 * np.eye(d)
        else:
            A = -0.2 * np.eye(d)
        x = np.zeros(g.n_dofs)
        x.reshape(-1, d + 1)[:, :d] = X @ A.T
        x.reshape(-1, d + 1)[:, d] = cbar
        p = np.full(g.n_nodes, pval)
        eps = 0.5 * (A + A.T)
        t = np.trace(eps)
        gdeg = (1 - mat.k) * (1 - cbar) ** 2 + mat.k
        if kind == "tension":
            assert t > 0
            el = gdeg * psi_e(eps, mat.lam, mat.mu)
        else:
            # psi_e = psi+ + psi- always; for t < 0 only psi+ = psi_e - K/2 t^2
            # is degraded (in 3D hydrostatic compression psi_e = K/2 t^2)
            Kb = mat.lam + 2 * mat.mu / 3
            el = gdeg * (psi_e(eps, mat.lam, mat.mu) - 0.5 * Kb * t * t) + 0.5 * Kb * t * t
            if d == 3:
                assert psi_e(eps, mat.lam, mat.mu) == pytest.approx(0.5 * Kb * t * t, rel=1e-14)
        expect = el + 0.5 * mat.Gc * cbar ** 2 / mat.ls + (1 - cbar) ** 2 * pval * t
        assert fem.energy(g, x, p, mat) == pytest.approx(expect, rel=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_rigid_motion_zero_energy_and_gradient(d):
    g = fem.Grid(d, 3)
    mat = _mat(True, 3)
    X = g.node_coords()
    Wm = RNG.standard_normal((d, d))
    Wm = Wm - Wm.T
    u0 = RNG.standard_normal(d)
    x = np.zeros(g.n_dofs)
    x.reshape(-1, d + 1)[:, :d] = u0 + X @ Wm.T
    p = np.full(g.n_nodes, 0.05)
    assert abs(fem.energy(g, x, p, mat)) < 1e-14
    # uniform p only loads the boundary (int dN_a/dx_i = 0 for interior a)
    gr = fem.gradient(g, x, p, mat, g.default_dirichlet())
    assert np.abs(gr).max() < 1e-14
    gr0 = fem.gradient(g, x, 0.0 * p, mat, np.zeros(g.n_dofs, bool))
    assert np.abs(gr0).max() < 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_uniform_pressure_work_vanishes_with_clamped_boundary(d):
    """Divergence theorem: with u = 0 on the boundary, c = 0 and uniform p,
    the pressure work integrates to zero, so f does not depend on p."""
    N = 4
    g = fem.Grid(d, N)
    mat = _mat(True, N)
    x = RNG.standard_normal(g.n_dofs) * 0.1
    x.reshape(-1, d + 1)[:, d] = 0.0
    x[g.default_dirichlet()] = 0.0
    f0 = fem.energy(g, x, np.zeros(g.n_nodes), mat)
    f1 = fem.energy(g, x, np.full(g.n_nodes, 0.37), mat)
    assert f1 == pytest.approx(f0, rel=1e-13, abs=1e-16)
    # and so does the pressure term's gradient on the free displacement dofs
    dirm = g.default_dirichlet()
    g0 = fem.gradient(g, x, np.zeros(g.n_nodes), mat, dirm)
    g1 = fem.gradient(g, x, np.full(g.n_nodes, 0.37), mat, dirm)
    ui = np.arange(g.n_dofs).reshape(-1, d + 1)[:, :d].reshape(-1)
    assert np.allclose(g1[ui], g0[ui], atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_at2_energy_of_affine_phase_field(d):
    """u = 0, c = a + b.x: f = Gc/2 (int c^2 / l + l |b|^2), int over the unit
    cell of (a + b.x)^2 = (a + sum b/2)^2 + sum b^2 / 12."""
    N = 3
    g = fem.Grid(d, N)
    mat = _mat(True, N)
    a, b = 0.2, RNG.uniform(-0.3, 0.3, d)
    x = np.zeros(g.n_dofs)
    x.reshape(-1, d + 1)[:, d] = a + g.node_coords() @ b
    p = np.full(g.n_nodes, 0.1)
    ic2 = (a + b.sum() / 2) ** 2 + np.sum(b * b) / 12
    expect = 0.5 * mat.Gc * (ic2 / mat.ls + mat.ls * np.sum(b * b))
    assert fem.energy(g, x, p, mat) == pytest.approx(expect, rel=1e-13)


def _random_state(g, scale=0.1):
    d = g.d
    x = RNG.standard_normal(g.n_dofs) * scale
    x.reshape(-1, d + 1)[:, d] = RNG.uniform(0.0, 1.0, g.n_nodes)
    p = RNG.uniform(0.5, 1.5, g.n_nodes) * 0.05
    return x, p


@pytest.mark.parametrize("d,N", [(2, 2), (2, 3), (3, 2)])
@pytest.mark.parametrize("split", [True, False])
def test_gradient_finite_differences(d, N, split):
    g = fem.Grid(d, N)
    mat = _mat(split, N)
    x, p = _random_state(g)
    nodir = np.zeros(g.n_dofs, bool)
    gr = fem.gradient(g, x, p, mat, nodir)
    eta = 1e-6
    fd = np.zeros_like(x)
    for i in range(g.n_dofs):
        e = np.zeros_like(x)
        e[i] = eta
        fd[i] = (fem.energy(g, x + e, p, mat) - fem.energy(g, x - e, p, mat)) / (2 * eta)
    assert np.abs(fd - gr).max() <= 1e-8 * np.abs(gr).max()


@pytest.mark.parametrize("d,N", [(2, 3), (3, 2)])
@pytest.mark.parametrize("split", [True, False])
def test_hessian_finite_differences_and_symmetry(d, N, split):
    g = fem.Grid(d, N)
    mat = _mat(split, N)
    x, p = _random_state(g)
    nodir = np.zeros(g.n_dofs, bool)
    H = fem.hessian(g, x, p, mat, nodir)
    eta = 1e-6
    for _ in range(3):
        v = RNG.standard_normal(g.n_dofs)
        fd = (fem.gradient(g, x + eta * v, p, mat, nodir)
              - fem.gradient(g, x - eta * v, p, mat, nodir)) / (2 * eta)
        hv = H @ v
        assert np.abs(fd - hv).max() <= 1e-7 * np.abs(hv).max()
    Hd = H.toarray()
    assert np.abs(Hd - Hd.T).max() <= 1e-14 * np.abs(Hd).max()


def test_dirichlet_rows_and_columns_removed():
    g = fem.Grid(2, 3)
    mat = _mat(True, 3)
    x, p = _random_state(g)
    dirm = g.default_dirichlet()
    gr = fem.gradient(g, x, p, mat, dirm)
    assert np.all(gr[dirm] == 0.0)
    H = fem.hessian(g, x, p, mat, dirm).toarray()
    assert np.all(H[dirm, :] == 0.0) and np.all(H[:, dirm] == 0.0)
    Hfull = fem.hessian(g, x, p, mat, np.zeros(g.n_dofs, bool)).toarray()
    free = ~dirm
    assert np.array_equal(H[np.ix_(free, free)], Hfull[np.ix_(free, free)])


def test_local_rows_match_global():
    g = fem.Grid(3, 3)
    mat = _mat(True, 3)
    x, p = _random_state(g)
    v = RNG.standard_normal(g.n_dofs)
    nodes = np.array([0, 5, 21, 63])
    want, gr, hv = fem.local_rows(g, x, p, mat, nodes, v)
    G = fem.gradient(g, x, p, mat)
    HV = fem.hessvec(g, x, p, mat, np.where(g.default_dirichlet(), 0.0, v))
    assert np.allclose(gr, G[want], rtol=1e-13, atol=1e-17)
    assert np.allclose(hv, HV[want], rtol=1e-13, atol=1e-17)


@pytest.mark.parametrize("d,N", [(2, 3), (3, 2)])
def test_energy_difference_is_a_difference_and_matches_taylor(d, N):
    """The per-element energy difference f(x + s) - f(x) equals the difference
    of the two totals up to rounding, and, on the unsplit (smooth) density,
    differs from the FD-pinned second-order model g^T s + 1/2 s^T H s by a
    third-order term: halving the step divides the gap by about 8."""
    g = fem.Grid(d, N)
    mat = _mat(False, N)
    rng = np.random.default_rng(2024 + d)
    x = rng.standard_normal(g.n_dofs) * 0.1
    x.reshape(-1, d + 1)[:, d] = rng.uniform(0.0, 1.0, g.n_nodes)
    p = rng.uniform(0.5, 1.5, g.n_nodes) * 0.05
    nodir = np.zeros(g.n_dofs, bool)
    gr = fem.gradient(g, x, p, mat, nodir)
    H = fem.hessian(g, x, p, mat, nodir)
    v = rng.standard_normal(g.n_dofs)
    f0 = fem.energy(g, x, p, mat)
    gaps = []
    for eps in (2e-3, 1e-3):
        s = eps * v
        de = fem.energy_diff(g, x, s, p, mat)
        assert abs(de - (fem.energy(g, x + s, p, mat) - f0)) <= 1e-13 * abs(f0)
        gaps.append(abs(de - (gr @ s + 0.5 * s @ (H @ s))))
    assert gaps[1] > 0 and 7.0 <= gaps[0] / gaps[1] <= 9.0


@pytest.mark.parametrize("d,N", [(2, 5), (3, 3)])
def test_neumann_load_divergence_theorem(d, N):
    """The pressure work of an intact body (c = 0, so g_p = 1) with no
    Dirichlet set equals the boundary term b . u of every face (divergence
    theorem, exact under the Gauss rules for Q1 fields), so f(x) - b . x
    carries no pressure load where the material is intact; and a uniform
    traction on one face integrates to traction x face area."""
    rng = np.random.default_rng(4 + d)
    g = fem.Grid(d, N)
    mat = fem.material_from_E_nu(1.0, 0.3, 1e-3, 2.0 / N)
    x = rng.standard_normal(g.n_dofs) * 1e-2
    x[d::d + 1] = 0.0
    p = rng.uniform(0.5, 1.5, g.n_nodes) * 1e-3
    work = fem.energy(g, x, p, mat) - fem.energy(g, x, np.zeros(g.n_nodes), mat)
    b = fem.neumann_load(g, range(2 * d), np.zeros((2 * d, d)), p)
    assert work == pytest.approx(float(b @ x), rel=1e-12)
    # uniform traction on the face x = 1 (face 1), no pressure
    tb = np.zeros((2 * d, d))
    tb[1] = rng.standard_normal(d)
    b1 = fem.neumann_load(g, [1], tb, np.zeros(g.n_nodes)).reshape(-1, d + 1)
    assert np.allclose(b1[:, :d].sum(axis=0), tb[1], rtol=1e-13, atol=0)
    nodes, nrm = fem.face_nodes(g, 1)
    assert np.all(b1[np.setdiff1d(np.arange(g.n_nodes), nodes)] == 0.0)
    assert np.all(b1[:, d] == 0.0)
    # uniform pressure on face y = 0 (face 2): sum = p0 n area
    b2 = fem.neumann_load(g, [2], np.zeros((2 * d, d)), np.full(g.n_nodes, 2e-3)).reshape(-1, d + 1)
    want = np.zeros(d)
    want[1] = -2e-3
    assert np.allclose(b2[:, :d].sum(axis=0), want, rtol=1e-13, atol=1e-18)

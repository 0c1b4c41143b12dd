"""Pins for the oracle's spectral (principal-strain) split.

The checks use what the definition fixes without the oracle's formulas:
closed forms on diagonal and pure-shear strains, psi+ + psi- = psi_e, the
invariance of both parts under rotations, the reduction to the unsplit
density when every principal strain has one sign, the derivative of
eps+ taken by central differences of (eps + sqrt(eps^2)) / 2
(also on repeated principal strains), and finite differences of the
pointwise and assembled energy, gradient and Hessian.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import fem

SPEC = fem.SPLIT_SPECTRAL


def _mat(split=SPEC, N=4, nu=0.3):
    return fem.material_from_E_nu(1.0, nu, 1e-3, 2.0 / N, 1e-6, split)


def _z_of(G, c, dc, u=None):
    d = G.shape[-1]
    z = np.zeros(fem.zdim(d))
    if u is not None:
        z[:d] = u
    z[d:d + d * d] = G.reshape(-1)
    z[d + d * d] = c
    z[d + d * d + 1:] = dc
    return z


def _elastic(z, mat, d, c):
    """The elastic part g psi+ + psi- of W at one point: W minus the crack
    and pressure terms, which here are zero (p = 0) apart from the AT2 term
    removed by hand."""
    W = fem.density(z[None], np.zeros(1), np.zeros((1, d)), mat, d)[0]
    dc = z[d + d * d + 1:]
    return W - 0.5 * mat.Gc * (c * c / mat.ls + mat.ls * np.sum(dc * dc))


def _psi_parts(eps, mat, d):
    """(psi+, psi-) read off W at c = 0 (g = 1) and c = 1 (g = k)."""
    G = eps.copy()
    z0 = _z_of(G, 0.0, np.zeros(d))
    z1 = _z_of(G, 1.0, np.zeros(d))
    W0 = _elastic(z0, mat, d, 0.0)  # psi+ + psi-
    W1 = _elastic(z1, mat, d, 1.0)  # k psi+ + psi-
    psip = (W0 - W1) / (1.0 - mat.k)
    return psip, W0 - psip


def test_diagonal_strain_closed_form():
    mat = _mat()
    a, b, c = 0.03, -0.05, 0.011
    psip, psim = _psi_parts(np.diag([a, b, c]), mat, 3)
    t = a + b + c
    want_p = 0.5 * mat.lam * max(t, 0) ** 2 + mat.mu * (a * a + c * c)
    want_m = 0.5 * mat.lam * min(t, 0) ** 2 + mat.mu * b * b
    assert psip == pytest.approx(want_p, rel=1e-12)
    assert psim == pytest.approx(want_m, rel=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_pure_shear_splits_evenly(d):
    """eps = gamma (e1 e2^T + e2 e1^T): principal strains +gamma, -gamma
    (and 0), t = 0, so psi+ = psi- = mu gamma^2."""
    mat = _mat()
    gam = 0.02
    eps = np.zeros((d, d))
    eps[0, 1] = eps[1, 0] = gam
    psip, psim = _psi_parts(eps, mat, d)
    assert psip == pytest.approx(mat.mu * gam * gam, rel=1e-12)
    assert psim == pytest.approx(mat.mu * gam * gam, rel=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_parts_sum_to_psi_e_and_are_rotation_invariant(d):
    rng = np.random.default_rng(71)
    mat = _mat()
    for _ in range(20):
        A = rng.standard_normal((d, d)) * 0.1
        eps = 0.5 * (A + A.T)
        psip, psim = _psi_parts(eps, mat, d)
        psie = 0.5 * mat.lam * np.trace(eps) ** 2 + mat.mu * np.sum(eps * eps)
        assert psip + psim == pytest.approx(psie, rel=1e-12)
        # both are sums of squares (up to the rounding of reading them off W)
        assert min(psip, psim) >= -1e-13 * psie
        R, _ = np.linalg.qr(rng.standard_normal((d, d)))
        rp, rm = _psi_parts(R @ eps @ R.T, mat, d)
        assert rp == pytest.approx(psip, rel=1e-11, abs=1e-18)
        assert rm == pytest.approx(psim, rel=1e-11, abs=1e-18)


@pytest.mark.parametrize("d", [2, 3])
def test_one_signed_strains_reduce_to_the_unsplit_density(d):
    """All principal strains positive: the whole psi_e is degraded (W equals
    the unsplit W); all negative: nothing is degraded."""
    rng = np.random.default_rng(72)
    spec, uns = _mat(), _mat(split=fem.SPLIT_NONE)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    for sign in (1.0, -1.0):
        ev = sign * rng.uniform(0.01, 0.05, d)
        eps = Q @ np.diag(ev) @ Q.T
        c = 0.4
        # G = eps plus a skew part: the strain sym G stays eps
        Wsk = rng.standard_normal((d, d)) * 0.03
        z = _z_of(eps + (Wsk - Wsk.T), c, rng.standard_normal(d) * 0.1)
        pq, dpq = np.array([0.02]), rng.standard_normal((1, d)) * 0.01
        Ws = fem.density(z[None], pq, dpq, spec, d)[0]
        if sign > 0:
            assert Ws == pytest.approx(fem.density(z[None], pq, dpq, uns, d)[0], rel=1e-12)
        else:
            psie = 0.5 * spec.lam * np.trace(eps) ** 2 + spec.mu * np.sum(eps * eps)
            gdeg = (1 - spec.k) * (1 - c) ** 2 + spec.k
            assert Ws == pytest.approx(fem.density(z[None], pq, dpq, uns, d)[0] + (1 - gdeg) * psie, rel=1e-12)


def _eps_plus(eps):
    """eps+ = (eps + |eps|) / 2 with |eps| the matrix square root of eps^2
    (scipy's Schur-based sqrtm): no eigendecomposition involved."""
    return 0.5 * (eps + np.real(scipy.linalg.sqrtm(eps @ eps)))


def _theta_apply(eps, E):
    ev, Q = fem.principal_strains(eps)
    th = fem.spectral_theta(ev)
    return Q @ (th * (Q.T @ E @ Q)) @ Q.T


@pytest.mark.parametrize("d", [2, 3])
def test_derivative_of_eps_plus_matches_central_differences(d):
    rng = np.random.default_rng(73)
    for case in range(12):
        Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
        if case < 4:
            ev = rng.uniform(-0.05, 0.05, d)
        elif case < 8:
            # a repeated positive pair and one negative (3D), or a repeated pair (2D)
            a = rng.uniform(0.01, 0.05)
            ev = np.array([a, a, -a]) if d == 3 else np.array([a, a])
        else:
            a = rng.uniform(0.01, 0.05)
            ev = np.array([-a, -a, a]) if d == 3 else np.array([-a, -a])
        eps = Q @ np.diag(ev) @ Q.T
        B = rng.standard_normal((d, d))
        E = 0.5 * (B + B.T)
        eta = 1e-7
        fd = (_eps_plus(eps + eta * E) - _eps_plus(eps - eta * E)) / (2 * eta)
        got = _theta_apply(eps, E)
        assert np.abs(got - fd).max() <= 1e-6 * max(np.abs(fd).max(), 1.0)


@pytest.mark.parametrize("d", [2, 3])
def test_pointwise_gradient_and_hessian_match_differences(d):
    rng = np.random.default_rng(74)
    mat = _mat()
    m = fem.zdim(d)
    done = 0
    while done < 10:
        z = rng.standard_normal(m) * 0.05
        z[d + d * d] = rng.uniform(0.1, 0.9)
        G = z[d:d + d * d].reshape(d, d)
        ev = np.linalg.eigvalsh(0.5 * (G + G.T))
        if np.abs(ev).min() < 5e-3 or abs(np.trace(G)) < 5e-3:
            continue  # away from the kinks
        pq = np.array([0.03])
        dpq = rng.standard_normal((1, d)) * 0.01
        gr = fem.density_grad(z[None], pq, dpq, mat, d)[0]
        H = fem.density_hess(z[None], pq, dpq, mat, d)[0]
        eta = 1e-6
        for i in range(m):
            e = np.zeros(m)
            e[i] = eta
            fd = (fem.density((z + e)[None], pq, dpq, mat, d)[0]
                  - fem.density((z - e)[None], pq, dpq, mat, d)[0]) / (2 * eta)
            assert fd == pytest.approx(gr[i], rel=1e-6, abs=1e-9)
            fdg = (fem.density_grad((z + e)[None], pq, dpq, mat, d)[0]
                   - fem.density_grad((z - e)[None], pq, dpq, mat, d)[0]) / (2 * eta)
            assert np.abs(fdg - H[:, i]).max() <= 1e-6 * max(np.abs(H).max(), 1.0)
        assert np.abs(H - H.T).max() <= 1e-14 * np.abs(H).max()
        done += 1


def _random_state(g, rng, scale=0.1):
    d = g.d
    x = rng.standard_normal(g.n_dofs) * scale
    x.reshape(-1, d + 1)[:, d] = rng.uniform(0.0, 1.0, g.n_nodes)
    p = rng.uniform(0.5, 1.5, g.n_nodes) * 0.05
    return x, p


@pytest.mark.parametrize("d,N", [(2, 3), (3, 2)])
def test_assembled_gradient_and_hessian_finite_differences(d, N):
    rng = np.random.default_rng(75)
    g = fem.Grid(d, N)
    mat = _mat(N=N)
    x, p = _random_state(g, rng)
    nodir = np.zeros(g.n_dofs, bool)
    gr = fem.gradient(g, x, p, mat, nodir)
    eta = 1e-6
    fd = np.zeros_like(x)
    for i in range(g.n_dofs):
        e = np.zeros_like(x)
        e[i] = eta
        fd[i] = (fem.energy(g, x + e, p, mat) - fem.energy(g, x - e, p, mat)) / (2 * eta)
    assert np.abs(fd - gr).max() <= 1e-8 * np.abs(gr).max()
    H = fem.hessian(g, x, p, mat, nodir)
    for _ in range(3):
        v = rng.standard_normal(g.n_dofs)
        fdh = (fem.gradient(g, x + eta * v, p, mat, nodir) - fem.gradient(g, x - eta * v, p, mat, nodir)) / (2 * eta)
        hv = H @ v
        assert np.abs(fdh - hv).max() <= 1e-7 * np.abs(hv).max()
    Hd = H.toarray()
    assert np.abs(Hd - Hd.T).max() <= 1e-14 * np.abs(Hd).max()


def test_spectral_and_voldev_agree_on_hydrostatic_states():
    """eps = a I (3D): principal strains all a, so the spectral parts are
    lambda/2 <3a>^2 + 3 mu <a>^2 = K/2 <t>^2 with t = 3a, the volumetric-
    deviatoric parts (e = 0): the two splits give the same W."""
    mat_s, mat_v = _mat(), _mat(split=fem.SPLIT_VOLDEV)
    for a in (0.02, -0.02):
        z = _z_of(a * np.eye(3), 0.3, np.array([0.1, -0.2, 0.05]), u=np.array([0.01, 0.0, -0.02]))
        pq, dpq = np.array([0.01]), np.array([[0.003, -0.001, 0.002]])
        assert fem.density(z[None], pq, dpq, mat_s, 3)[0] == pytest.approx(
            fem.density(z[None], pq, dpq, mat_v, 3)[0], rel=1e-13)

"""Oracle: the discrete phase-field fracture functional on a uniform Q1 grid.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What is computed (paper Sec. 2, eq. (pressurized) and (min_problem_pf); the
strain split, the residual stiffness k and the sign of the pressure work are
the readings listed in the design notes):

  f(x) = sum_e sum_q w_q W(z_q),   w_q = h^d / 2^d,  2^d Gauss points
  W    = g(c) psi+(eps) + psi-(eps) + Gc/2 (c^2/l + l |grad c|^2) + gp(c) pi
  g    = (1-k)(1-c)^2 + k,    gp = (1-c)^2,   pi = div(p u) = p tr(eps) + grad p . u
  psi+ = K/2 <t>+^2 + mu e:e,  psi- = K/2 <t>-^2,   t = tr eps,  e = eps - t/3 I3,
  K    = lambda + 2 mu / 3   (volumetric-deviatoric split; in 2D plane strain).

With split=False (0) the paper's unsplit density is used: psi+ = psi_e =
lambda/2 t^2 + mu eps:eps, psi- = 0 (Sec. 2, first paragraph).  split=2 is
the spectral split on the principal strains eps_a (the principal strains the
implementation section names among its precomputed quantities; Miehe, Hofacker
and Welschinger's form):
  psi+- = lambda/2 <t>+-^2 + mu sum_a <eps_a>+-^2,
  sigma+- = lambda <t>+- I + 2 mu eps+-,   eps+- = sum_a <eps_a>+- n_a n_a^T.

z_q collects, at one quadrature point, the values that W depends on:
  z = (u_0..u_{d-1}, G_00, G_01, .., G_{d-1,d-1}, c, dc_0..dc_{d-1}),
G_ij = du_i/dx_j.  z_q = B_q x_e with a constant matrix B_q (uniform grid), so

  grad f = sum_e sum_q w B_q^T W_z(z_q),   Hess f = sum_e sum_q w B_q^T W_zz(z_q) B_q.

Layout: node n = i + (N+1)(j + (N+1)k), dof = (d+1) n + comp, comp order
(u_x, u_y[, u_z], c).  Dirichlet dofs are removed from the problem (Sec. 2.2,
V_u^t): the gradient has zero rows there and the Hessian zero rows and columns.
"""
import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


SPLIT_NONE, SPLIT_VOLDEV, SPLIT_SPECTRAL = 0, 1, 2


@dataclass
class Material:
    lam: float
    mu: float
    Gc: float
    ls: float
    k: float = 1e-6
    split: int = SPLIT_VOLDEV  # True / False read as 1 / 0

    @property
    def K(self):
        return self.lam + 2.0 * self.mu / 3.0


def material_from_E_nu(E, nu, Gc, ls, k=1e-6, split=True):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return Material(lam, mu, Gc, ls, k, split)


# ---------------------------------------------------------------- grid ----

class Grid:
    """Uniform grid of N^d cells on the unit square/cube."""

    def __init__(self, d, N):
        assert d in (2, 3)
        self.d, self.N = d, N
        self.h = 1.0 / N
        self.nside = N + 1
        self.n_nodes = self.nside ** d
        self.nc = d + 1
        self.n_dofs = self.nc * self.n_nodes
        self.n_elems = N ** d

    def node_ijk(self):
        """Integer coordinates of every node, shape (n_nodes, d), x fastest."""
        idx = np.arange(self.n_nodes)
        out = []
        for _ in range(self.d):
            out.append(idx % self.nside)
            idx = idx // self.nside
        return np.stack(out, axis=1)

    def node_coords(self):
        """x_i = i / N, one correctly rounded division per coordinate."""
        return self.node_ijk().astype(np.float64) / float(self.N)

    def elem_ijk(self):
        idx = np.arange(self.n_elems)
        out = []
        for _ in range(self.d):
            out.append(idx % self.N)
            idx = idx // self.N
        return np.stack(out, axis=1)

    def elem_nodes(self, elems=None):
        """Global node of local node a = ax + 2 ay + 4 az, shape (nE, 2^d)."""
        e = self.elem_ijk() if elems is None else self.elem_ijk()[elems]
        nloc = 1 << self.d
        out = np.zeros((e.shape[0], nloc), dtype=np.int64)
        for a in range(nloc):
            n = np.zeros(e.shape[0], dtype=np.int64)
            stride = 1
            for i in range(self.d):
                n += (e[:, i] + ((a >> i) & 1)) * stride
                stride *= self.nside
            out[:, a] = n
        return out

    def elem_dofs(self, elems=None):
        nodes = self.elem_nodes(elems)
        nc = self.nc
        return (nodes[:, :, None] * nc + np.arange(nc)[None, None, :]).reshape(nodes.shape[0], -1)

    def node_colour(self):
        """2^d-colouring: colour = i%2 + 2 (j%2) + 4 (k%2)."""
        ijk = self.node_ijk()
        col = np.zeros(self.n_nodes, dtype=np.int64)
        for i in range(self.d):
            col += (ijk[:, i] % 2) << i
        return col

    def boundary_nodes(self):
        ijk = self.node_ijk()
        return np.any((ijk == 0) | (ijk == self.N), axis=1)

    def default_dirichlet(self):
        """Dirichlet mask per dof: every displacement component on the boundary."""
        m = np.zeros((self.n_nodes, self.nc), dtype=bool)
        m[self.boundary_nodes(), : self.d] = True
        return m.reshape(-1)


# ------------------------------------------------------ reference data ----

def gauss_points_01():
    """Two-point Gauss-Legendre rule on [0, 1]."""
    r = 1.0 / math.sqrt(3.0)
    return np.array([0.5 * (1.0 - r), 0.5 * (1.0 + r)])


def zdim(d):
    return d + d * d + 1 + d


def reference_B(d, h):
    """B[q] maps the element dofs (node-major, (d+1) per node) to z_q.

    Shape functions N_a(xi) = prod_i phi_{a_i}(xi_i), phi_0 = 1 - s,
    phi_1 = s; derivatives (1/h) phi'_{a_j}(xi_j) prod_{i != j} phi_{a_i}(xi_i).
    Returns (B, w, Nq, dNq) with B of shape (2^d, m, (d+1) 2^d).
    """
    gp = gauss_points_01()
    nq = nloc = 1 << d
    nc = d + 1
    Nq = np.zeros((nq, nloc))
    dNq = np.zeros((nq, nloc, d))
    for q in range(nq):
        xi = [gp[(q >> i) & 1] for i in range(d)]
        for a in range(nloc):
            ai = [(a >> i) & 1 for i in range(d)]
            phi = [xi[i] if ai[i] else 1.0 - xi[i] for i in range(d)]
            dphi = [1.0 if ai[i] else -1.0 for i in range(d)]
            Nq[q, a] = np.prod(phi)
            for j in range(d):
                v = dphi[j] / h
                for i in range(d):
                    if i != j:
                        v *= phi[i]
                dNq[q, a, j] = v
    m = zdim(d)
    B = np.zeros((nq, m, nc * nloc))
    for q in range(nq):
        for a in range(nloc):
            for i in range(d):
                B[q, i, nc * a + i] = Nq[q, a]                       # u_i
                for j in range(d):
                    B[q, d + d * i + j, nc * a + i] = dNq[q, a, j]    # G_ij
            B[q, d + d * d, nc * a + d] = Nq[q, a]                  # c
            for j in range(d):
                B[q, d + d * d + 1 + j, nc * a + d] = dNq[q, a, j]  # dc_j
    w = h ** d / nq
    return B, w, Nq, dNq


# --------------------------------------------------- pointwise density ----

def _unpack(z, d):
    u = z[..., :d]
    G = z[..., d:d + d * d].reshape(z.shape[:-1] + (d, d))
    c = z[..., d + d * d]
    dc = z[..., d + d * d + 1:]
    return u, G, c, dc


def principal_strains(eps):
    """Eigenvalues (ascending) and unit eigenvectors (columns) of the
    symmetric strain at every point (LAPACK's symmetric eigensolver)."""
    return np.linalg.eigh(eps)


def spectral_theta(ev):
    """theta_ab of the derivative of eps+ = sum_a <eps_a>+ n_a n_a^T:
    dEps+ = sum_ab theta_ab (n_a^T dEps n_b) n_a n_b^T with theta_aa =
    H(eps_a) and, for eps_a != eps_b, the divided difference
    (<eps_a>+ - <eps_b>+) / (eps_a - eps_b) (its limit H(eps_a) when equal).
    H(0) = 0, the compressive side, as for the other splits' indicators."""
    pos = np.maximum(ev, 0.0)
    Hs = (ev > 0.0).astype(np.float64)
    la, lb = ev[..., :, None], ev[..., None, :]
    diff = la - lb
    same = diff == 0.0
    num = pos[..., :, None] - pos[..., None, :]
    th = np.where(same, np.broadcast_to(Hs[..., :, None], diff.shape), num / np.where(same, 1.0, diff))
    return th


def density(z, pq, dpq, mat, d):
    """W(z) at quadrature points; pq = p, dpq = grad p at the same points."""
    u, G, c, dc = _unpack(z, d)
    eps = 0.5 * (G + np.swapaxes(G, -1, -2))
    t = np.trace(eps, axis1=-2, axis2=-1)
    epsq = np.sum(eps * eps, axis=(-2, -1))
    if int(mat.split) == SPLIT_SPECTRAL:
        ev, _ = principal_strains(eps)
        psip = 0.5 * mat.lam * np.maximum(t, 0.0) ** 2 + mat.mu * np.sum(np.maximum(ev, 0.0) ** 2, axis=-1)
        psim = 0.5 * mat.lam * np.minimum(t, 0.0) ** 2 + mat.mu * np.sum(np.minimum(ev, 0.0) ** 2, axis=-1)
    elif mat.split:
        K = mat.K
        psip = 0.5 * K * np.maximum(t, 0.0) ** 2 + mat.mu * (epsq - t * t / 3.0)
        psim = 0.5 * K * np.minimum(t, 0.0) ** 2
    else:
        psip = 0.5 * mat.lam * t * t + mat.mu * epsq
        psim = 0.0 * t
    g = (1.0 - mat.k) * (1.0 - c) ** 2 + mat.k
    gp = (1.0 - c) ** 2
    pi = pq * t + np.sum(dpq * u, axis=-1)
    crack = 0.5 * mat.Gc * (c * c / mat.ls + mat.ls * np.sum(dc * dc, axis=-1))
    return g * psip + psim + crack + gp * pi


def _stress_parts(G, mat, d):
    """psi+, sigma+ (d x d), sigma- (d x d), t and the split indicator."""
    eps = 0.5 * (G + np.swapaxes(G, -1, -2))
    t = np.trace(eps, axis1=-2, axis2=-1)
    epsq = np.sum(eps * eps, axis=(-2, -1))
    I = np.eye(d)
    if int(mat.split) == SPLIT_SPECTRAL:
        tp, tm = np.maximum(t, 0.0), np.minimum(t, 0.0)
        ev, Q = principal_strains(eps)
        evp = np.maximum(ev, 0.0)
        epsp = np.einsum('...ia,...a,...ja->...ij', Q, evp, Q)
        psip = 0.5 * mat.lam * tp * tp + mat.mu * np.sum(evp * evp, axis=-1)
        sigp = (mat.lam * tp)[..., None, None] * I + 2.0 * mat.mu * epsp
        sigm = (mat.lam * tm)[..., None, None] * I + 2.0 * mat.mu * (eps - epsp)
    elif mat.split:
        K = mat.K
        tp, tm = np.maximum(t, 0.0), np.minimum(t, 0.0)
        e = eps - (t / 3.0)[..., None, None] * I
        psip = 0.5 * K * tp * tp + mat.mu * (epsq - t * t / 3.0)
        sigp = (K * tp)[..., None, None] * I + 2.0 * mat.mu * e
        sigm = (K * tm)[..., None, None] * I
    else:
        psip = 0.5 * mat.lam * t * t + mat.mu * epsq
        sigp = (mat.lam * t)[..., None, None] * I + 2.0 * mat.mu * eps
        sigm = 0.0 * sigp
    return psip, sigp, sigm, t


def density_grad(z, pq, dpq, mat, d):
    """dW/dz, first variation (derivatives of the density above)."""
    u, G, c, dc = _unpack(z, d)
    psip, sigp, sigm, t = _stress_parts(G, mat, d)
    g = (1.0 - mat.k) * (1.0 - c) ** 2 + mat.k
    dg = -2.0 * (1.0 - mat.k) * (1.0 - c)
    gp = (1.0 - c) ** 2
    dgp = -2.0 * (1.0 - c)
    pi = pq * t + np.sum(dpq * u, axis=-1)
    out = np.zeros(z.shape)
    out[..., :d] = gp[..., None] * dpq
    S = g[..., None, None] * sigp + sigm + (gp * pq)[..., None, None] * np.eye(d)
    out[..., d:d + d * d] = S.reshape(z.shape[:-1] + (d * d,))
    out[..., d + d * d] = dg * psip + mat.Gc * c / mat.ls + dgp * pi
    out[..., d + d * d + 1:] = mat.Gc * mat.ls * dc
    return out


def density_hess(z, pq, dpq, mat, d):
    """d2W/dz2 (m x m per point), second variation; at t = 0 the split
    indicator takes the compressive branch (H+ = [t > 0])."""
    u, G, c, dc = _unpack(z, d)
    psip, sigp, sigm, t = _stress_parts(G, mat, d)
    g = (1.0 - mat.k) * (1.0 - c) ** 2 + mat.k
    dg = -2.0 * (1.0 - mat.k) * (1.0 - c)
    d2g = 2.0 * (1.0 - mat.k)
    dgp = -2.0 * (1.0 - c)
    d2gp = 2.0
    pi = pq * t + np.sum(dpq * u, axis=-1)
    m = zdim(d)
    Hm = np.zeros(z.shape[:-1] + (m, m))
    iG = lambda i, j: d + d * i + j
    ic = d + d * d
    # uu block: only through G.  dW/dG_ij = S_ij(eps); S depends on eps = sym G.
    Pp = None
    if int(mat.split) == SPLIT_SPECTRAL:
        # lambda (g H+ + H-) tr dEps tr DEps + 2 mu (g dEps+ + dEps-) : DEps,
        # dEps- = dEps - dEps+: the shear part is 2 mu dEps : DEps plus
        # 2 mu (g - 1) dEps+ : DEps, dEps+ = P+ dEps with
        # P+_ijkl = sum_ab theta_ab sym(n_a n_b^T)_ij sym(n_a n_b^T)_kl
        Hp = (t > 0.0).astype(np.float64)
        vol = mat.lam * (g * Hp + (1.0 - Hp))
        shear = mat.mu + 0.0 * g
        ev, Q = principal_strains(0.5 * (G + np.swapaxes(G, -1, -2)))
        th = spectral_theta(ev)
        M = 0.5 * (np.einsum('...ia,...jb->...abij', Q, Q) + np.einsum('...ja,...ib->...abij', Q, Q))
        Pp = np.einsum('...ab,...abij,...abkl->...ijkl', th, M, M)
        Pp = 2.0 * mat.mu * (g - 1.0)[..., None, None, None, None] * Pp
    elif mat.split:
        K = mat.K
        Hp = (t > 0.0).astype(np.float64)
        vol = g * K * Hp + K * (1.0 - Hp) - g * 2.0 * mat.mu / 3.0
        shear = g * mat.mu
    else:
        vol = g * mat.lam
        shear = g * mat.mu
    for i in range(d):
        for j in range(d):
            for kk in range(d):
                for l in range(d):
                    v = 0.0
                    if i == j and kk == l:
                        v = v + vol
                    if i == kk and j == l:
                        v = v + shear
                    if i == l and j == kk:
                        v = v + shear
                    if Pp is not None:
                        v = v + Pp[..., i, j, kk, l]
                    if not np.isscalar(v) or v != 0.0:
                        Hm[..., iG(i, j), iG(kk, l)] = v
    # uc coupling
    for i in range(d):
        for j in range(d):
            v = dg * sigp[..., i, j] + (dgp * pq if i == j else 0.0 * pq)
            Hm[..., iG(i, j), ic] = v
            Hm[..., ic, iG(i, j)] = v
        Hm[..., i, ic] = dgp * dpq[..., i]
        Hm[..., ic, i] = dgp * dpq[..., i]
    # cc
    Hm[..., ic, ic] = d2g * psip + mat.Gc / mat.ls + d2gp * pi
    for j in range(d):
        Hm[..., ic + 1 + j, ic + 1 + j] = mat.Gc * mat.ls
    return Hm


# ------------------------------------------------------ element loops ----

def _quad_data(grid, x, p, elems):
    B, w, Nq, dNq = reference_B(grid.d, grid.h)
    dofs = grid.elem_dofs(elems)
    nodes = grid.elem_nodes(elems)
    Xe = x[dofs]                                   # (nE, ndof_e)
    Pe = p[nodes]                                  # (nE, 2^d)
    z = np.einsum("qmk,ek->eqm", B, Xe)
    pq = np.einsum("qa,ea->eq", Nq, Pe)
    dpq = np.einsum("qaj,ea->eqj", dNq, Pe)
    return B, w, dofs, z, pq, dpq


def _chunks(grid, elems, size=65536):
    allel = np.arange(grid.n_elems) if elems is None else np.asarray(elems)
    for s in range(0, allel.shape[0], size):
        yield allel[s:s + size]


def element_energies(grid, x, p, mat, elems=None):
    """Energy of each element, sum_q w W(z_q)."""
    out = []
    for ch in _chunks(grid, elems):
        B, w, dofs, z, pq, dpq = _quad_data(grid, x, p, ch)
        out.append(w * density(z, pq, dpq, mat, grid.d).sum(axis=1))
    return np.concatenate(out) if out else np.zeros(0)


def energy(grid, x, p, mat, elems=None):
    """f(x) = sum of element energies."""
    return float(np.sum(element_energies(grid, x, p, mat, elems)))


def energy_diff(grid, x, s, p, mat, elems=None):
    """f(x + s) - f(x), summed as per-element differences."""
    return float(np.sum(element_energies(grid, x + s, p, mat, elems)
                        - element_energies(grid, x, p, mat, elems)))


def gradient(grid, x, p, mat, dirichlet=None, elems=None):
    """grad f with Dirichlet rows zeroed."""
    gvec = np.zeros(grid.n_dofs)
    for ch in _chunks(grid, elems):
        B, w, dofs, z, pq, dpq = _quad_data(grid, x, p, ch)
        Wz = density_grad(z, pq, dpq, mat, grid.d)
        ge = w * np.einsum("qmk,eqm->ek", B, Wz)
        np.add.at(gvec, dofs.reshape(-1), ge.reshape(-1))
    if dirichlet is None:
        dirichlet = grid.default_dirichlet()
    gvec[dirichlet] = 0.0
    return gvec


def element_matrices(grid, x, p, mat, elems=None):
    """K_e = sum_q w B_q^T W_zz B_q for the selected elements, as two matrix
    products: W_zz B_q per point, then B^T (all points stacked) times it."""
    B, w, dofs, z, pq, dpq = _quad_data(grid, x, p, elems)
    Wzz = density_hess(z, pq, dpq, mat, grid.d)
    WB = np.matmul(Wzz, B[None])                      # (e, q, m, k): W_zz B_q
    ne, nq, m, nk = WB.shape
    Ke = w * np.matmul(B.reshape(nq * m, nk).T[None], WB.reshape(ne, nq * m, nk))
    return dofs, Ke


def hessian(grid, x, p, mat, dirichlet=None, elems=None):
    """Assembled Hessian (CSR) with Dirichlet rows and columns zeroed."""
    rows, cols, vals = [], [], []
    for ch in _chunks(grid, elems, 16384):
        dofs, Ke = element_matrices(grid, x, p, mat, ch)
        nd = dofs.shape[1]
        rows.append(np.repeat(dofs, nd, axis=1).reshape(-1))
        cols.append(np.tile(dofs, (1, nd)).reshape(-1))
        vals.append(Ke.reshape(-1))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(grid.n_dofs, grid.n_dofs)).tocsr()
    H.sum_duplicates()
    if dirichlet is None:
        dirichlet = grid.default_dirichlet()
    D = sp.diags((~dirichlet).astype(np.float64))
    H = (D @ H @ D).tocsr()
    H.sort_indices()
    return H


def hessvec(grid, x, p, mat, v, dirichlet=None):
    """Hess f(x) v on the free dofs."""
    return hessian(grid, x, p, mat, dirichlet) @ v


def local_rows(grid, x, p, mat, nodes, v=None, dirichlet=None):
    """Gradient rows and (optionally) Hv rows for a few nodes only, from the
    elements around them; used to check single entries on very large grids."""
    nodes = np.asarray(nodes)
    ijk = grid.node_ijk()[nodes]
    elems = set()
    for n in range(nodes.shape[0]):
        for a in range(1 << grid.d):
            e = ijk[n] - np.array([(a >> i) & 1 for i in range(grid.d)])
            if np.all(e >= 0) and np.all(e < grid.N):
                eid = 0
                stride = 1
                for i in range(grid.d):
                    eid += int(e[i]) * stride
                    stride *= grid.N
                elems.add(eid)
    elems = np.array(sorted(elems), dtype=np.int64)
    if dirichlet is None:
        dirichlet = grid.default_dirichlet()
    B, w, dofs, z, pq, dpq = _quad_data(grid, x, p, elems)
    Wz = density_grad(z, pq, dpq, mat, grid.d)
    ge = w * np.einsum("qmk,eqm->ek", B, Wz)
    want = (nodes[:, None] * grid.nc + np.arange(grid.nc)[None, :]).reshape(-1)
    pos = {int(dof): r for r, dof in enumerate(want)}
    g_rows = np.zeros(want.shape[0])
    hv_rows = np.zeros(want.shape[0]) if v is not None else None
    if v is not None:
        Wzz = density_hess(z, pq, dpq, mat, grid.d)
        vv = np.where(dirichlet, 0.0, v)
        ze = np.einsum("qmk,ek->eqm", B, vv[dofs])
        he = w * np.einsum("qmk,eqmn,eqn->ek", B, Wzz, ze)
    for e in range(dofs.shape[0]):
        for kk in range(dofs.shape[1]):
            r = pos.get(int(dofs[e, kk]))
            if r is not None:
                g_rows[r] += ge[e, kk]
                if v is not None:
                    hv_rows[r] += he[e, kk]
    mask = dirichlet[want]
    g_rows[mask] = 0.0
    if v is not None:
        hv_rows[mask] = 0.0
    return want, g_rows, hv_rows


def face_nodes(grid, face):
    """Nodes of boundary face `face` = 2 axis + side (side 0: coordinate 0,
    side 1: coordinate 1) and the face's outward unit normal."""
    axis, side = divmod(face, 2)
    ijk = grid.node_ijk()
    n = np.zeros(grid.d)
    n[axis] = 1.0 if side else -1.0
    return np.nonzero(ijk[:, axis] == side * grid.N)[0], n


def neumann_load(grid, faces, traction, p):
    """External load vector of the Neumann terms of eq. (pressurized) on the
    boundary faces listed in `faces` (the part Gamma_N of the boundary where
    the displacement is free):

        b[(d+1) a + i] = int_{Gamma_N} (tbar_i + p n_i) N_a ds,

    so that the functional is f(x) - b . x.  tbar: traction per face
    (shape (2d, d), constant on a face); p: nodal pressure (Q1 on the face).
    Reading: with the pressure work written as + int g_p div(p u) (the sign
    that opens a pressurised crack), the boundary term of the divergence
    theorem enters as - int_{Gamma_N} p n . u, next to - int tbar . u.
    Face cells are integrated with the (d-1)-dimensional 2-point Gauss rule,
    exact for the bilinear integrand."""
    d, N, h = grid.d, grid.N, grid.h
    b = np.zeros(grid.n_dofs)
    gp = gauss_points_01()
    ijk = grid.node_ijk()
    index = {tuple(c): k for k, c in enumerate(ijk)}
    for face in faces:
        axis, side = divmod(face, 2)
        tan = [i for i in range(d) if i != axis]
        nvec = np.zeros(d)
        nvec[axis] = 1.0 if side else -1.0
        tb = np.asarray(traction[face], dtype=np.float64)
        # face cells: lower corner over the tangential directions
        for cell in np.ndindex(*([N] * (d - 1))):
            corners = []
            for a in range(1 << (d - 1)):
                c = [0] * d
                c[axis] = side * N
                for t, ti in enumerate(tan):
                    c[ti] = cell[t] + ((a >> t) & 1)
                corners.append(index[tuple(c)])
            for q in range(1 << (d - 1)):
                xi = [gp[(q >> t) & 1] for t in range(d - 1)]
                Na = np.array([np.prod([xi[t] if (a >> t) & 1 else 1.0 - xi[t] for t in range(d - 1)])
                               for a in range(1 << (d - 1))])
                wq = h ** (d - 1) / (1 << (d - 1))
                pq = float(Na @ p[corners])
                load = tb + pq * nvec
                for a, node in enumerate(corners):
                    b[(d + 1) * node:(d + 1) * node + d] += wq * Na[a] * load
    return b


def diag_blocks(H, grid):
    """(d+1) x (d+1) diagonal block of every node, from an assembled Hessian."""
    nc = grid.nc
    out = np.zeros((grid.n_nodes, nc, nc))
    Hc = H.tocsr()
    for i in range(nc):
        for j in range(nc):
            rows = np.arange(grid.n_nodes) * nc + i
            cols = np.arange(grid.n_nodes) * nc + j
            out[:, i, j] = np.asarray(Hc[rows, cols]).reshape(-1)
    return out


def chi(grid, x, gvec, c_lower, dirichlet=None):
    """Stopping measure || P_F(x - grad f) - x ||_2 over free dofs, with F the
    feasible set c_lower <= c <= 1 (displacements unbounded)."""
    if dirichlet is None:
        dirichlet = grid.default_dirichlet()
    nc = grid.nc
    r = -gvec.copy()
    ci = np.arange(grid.n_nodes) * nc + grid.d
    xc = x[ci]
    r[ci] = np.clip(xc - gvec[ci], c_lower, 1.0) - xc
    r[dirichlet] = 0.0
    return float(np.sqrt(np.sum(r * r)))

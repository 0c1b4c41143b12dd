"""Oracle: trust-region steps and the RMTR V-cycle with Hessian lagging.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Sec. 3 of the paper: Algorithm 1 (V-cycle), Algorithm 2
(Nonlinear_solve: TR iterations), Algorithm 3 (Convergence_control),
eq. (rho_tr) and (rho_ml) for the ratios, eq. (second_order_consistency) and
(delta_terms) for the level objectives, and Sec. 4.2.1 for lagging: one
Hessian per level per V-cycle, taken at the level's initial iterate; the
coarse Hessians are Galerkin products R H I of the lagged finer one, reused
in post-smoothing.

Readings where the paper is silent (listed in the design notes):
  * h^l(x) = f~^l(x) + <dg, x - x0> + 1/2 <x - x0, dH (x - x0)>, with f~^l the
    same discrete functional on the level-l grid (p injected, l_s unchanged),
    or f~^l = 0 ("zero" coarse model), or f~^l(x) = f(I_{l->L} x), the finest
    functional of the prolongated coarse iterate ("fine" coarse model);
  * a caller's Dirichlet set on the finest level is injected to the
    coarse levels (fine node (2i, 2j, 2k) -> coarse node (i, j, k)); the
    default set (every boundary displacement) is its own injection;
  * first-order variant (ablation): dH = 0, so the coarse model is
    f~^l(x) + <dg, x - x0> and its Hessian, lagged like every other, is the
    level's own grad^2 f~^l(x0) instead of the Galerkin product (needs a
    coarse functional: not with the "zero" model);
  * coarse feasible set: x0 + box_restrict(fine correction box);
  * ratio guards: pred <= 0 with s != 0 -> rho = -inf; s = 0 -> skip;
    |pred| <= tol -> rho = 1 if ared >= -tol else -inf, with the round-off
    level tol = 1e-14 |f_ref| / sqrt(n_elements of the level), f_ref the
    energy at the start of the load step; non-finite -> -inf;
  * Alg. 3 literally: accept iff rho > eta1; radius gamma1 D if rho < eta1,
    unchanged on [eta1, eta2], min(gamma2 D, D_max) if rho > eta2 (option:
    gamma1 min(D, |s|_inf) after a rejection, the usual step-based update);
  * Alg. 2 runs exactly i_max iterations.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import fem, qp, transfer


@dataclass
class Params:
    eta1: float = 0.1
    eta2: float = 0.75
    gamma1: float = 0.5
    gamma2: float = 2.0
    delta0: float = 1.0
    delta_max: float = 10.0
    mu1: int = 1
    mu2: int = 1
    pgs_sweeps: int = 3
    coarse_tr_its: int = 5
    coarse_qp_its: int = 500
    coarse_qp_rtol: float = 1e-10
    fallback_sweeps: int = 50
    max_vcycles: int = 200
    rtol: float = 1e-8
    coarse_model: str = "energy"      # or "zero", or "fine" (f o I)
    first_order: bool = False         # coarse models without the dH term
    guard: float = 1e-14
    shrink_to_step: bool = False      # rejected: gamma1 min(delta, |s|_inf)


@dataclass
class Stats:
    vcycles: int = 0
    tr_accepted: int = 0
    tr_rejected: int = 0
    chi0: float = 0.0
    chi: float = 0.0
    energy: float = 0.0
    history: list = field(default_factory=list)


class Level:
    def __init__(self, d, N, mat, p, dirichlet=None):
        self.grid = fem.Grid(d, N)
        self.mat = mat
        self.p = p
        self.dirichlet = self.grid.default_dirichlet() if dirichlet is None else dirichlet
        self.free = ~self.dirichlet
        self.blocks = qp.colour_blocks(self.grid.node_colour(), self.grid.nc, 1 << d)
        # set per V-cycle
        self.x0 = None
        self.Hmod = None
        self.Hf0 = None
        self.dg = None
        self.Lb = None
        self.Ub = None
        self.finest = False


class RMTR:
    """RMTR on the hierarchy N_l = N_L / 2^(L-l), l = 1 (coarsest) .. L."""

    def __init__(self, d, n_cells, n_levels, mat, p_fine, params=None, dirichlet=None, f_ext=None):
        """f_ext: external load vector of the finest level (the Neumann terms,
        fem.neumann_load); the finest functional is then f(x) - f_ext . x."""
        self.prm = params or Params()
        self.f_ext = f_ext
        self.L = n_levels
        self.d = d
        Ns = [n_cells >> (n_levels - l) for l in range(1, n_levels + 1)]
        assert Ns[0] << (n_levels - 1) == n_cells
        self.levels = {}
        p = p_fine
        self.I, self.R, self.P = {}, {}, {}
        mask = dirichlet
        for l in range(n_levels, 0, -1):
            lev = Level(d, Ns[l - 1], mat, p, mask)
            self.levels[l] = lev
            if l > 1:
                Nc = Ns[l - 2]
                self.I[l - 1] = transfer.prolongation(d, Nc, d + 1)
                self.R[l - 1] = transfer.restriction(d, Nc, d + 1)
                self.P[l - 1] = transfer.injection(d, Nc, d + 1)
                nodeP = transfer.injection(d, Nc, 1)
                p = nodeP @ p
                # a caller's Dirichlet set reaches the coarse levels by
                # injection (the coarse dof is fixed where the fine dof it
                # coincides with is); otherwise every level has the default
                # set
                if dirichlet is not None:
                    mask = (self.P[l - 1] @ lev.dirichlet.astype(np.float64)) > 0.5
        self.levels[n_levels].finest = True
        # composite prolongations I_{l -> L} for the "fine" coarse model
        self.IL = {n_levels: None}
        for l in range(n_levels - 1, 0, -1):
            nxt = self.IL[l + 1]
            self.IL[l] = self.I[l] if nxt is None else (nxt @ self.I[l]).tocsr()
        if self.prm.coarse_model not in ("energy", "zero", "fine"):
            raise ValueError(f"unknown coarse model {self.prm.coarse_model!r}")
        if self.prm.first_order and self.prm.coarse_model == "zero":
            raise ValueError("the first-order coarse model needs a coarse functional")
        self.stats = Stats()
        self.f_ref = 1.0

    # ---------------------------------------------------------- level h
    def _ftilde_active(self, lev):
        return lev.finest or self.prm.coarse_model != "zero"

    def _fine(self):
        return self.levels[self.L]

    # ------------------------------------------------- finest functional
    def fine_energy(self, x):
        f = self._fine()
        e = fem.energy(f.grid, x, f.p, f.mat)
        return e if self.f_ext is None else e - float(self.f_ext @ x)

    def fine_energy_diff(self, x, s):
        f = self._fine()
        e = fem.energy_diff(f.grid, x, s, f.p, f.mat)
        return e if self.f_ext is None else e - float(self.f_ext @ s)

    def fine_gradient(self, x):
        f = self._fine()
        g = fem.gradient(f.grid, x, f.p, f.mat, f.dirichlet)
        if self.f_ext is not None:
            g = g - self.f_ext
            g[f.dirichlet] = 0.0
        return g

    def ft_grad(self, lev, x):
        """grad f~ of a coarse level (Dirichlet rows zeroed)."""
        if self.prm.coarse_model == "fine":
            IL = self.IL[self._level_index(lev)]
            g = IL.T @ self.fine_gradient(IL @ x)
            g[lev.dirichlet] = 0.0
            return g
        return fem.gradient(lev.grid, x, lev.p, lev.mat, lev.dirichlet)

    def ft_hessian(self, lev, x):
        """grad^2 f~ of a coarse level at x (Dirichlet rows and columns zeroed)."""
        if self.prm.coarse_model == "fine":
            f = self._fine()
            IL = self.IL[self._level_index(lev)]
            H = IL.T @ fem.hessian(f.grid, IL @ x, f.p, f.mat, f.dirichlet) @ IL
            D = sp.diags(lev.free.astype(np.float64))
            return (D @ H @ D).tocsr()
        return fem.hessian(lev.grid, x, lev.p, lev.mat, lev.dirichlet)

    def ft_diff(self, lev, x, s):
        """f~(x + s) - f~(x) of any level."""
        if lev.finest:
            return self.fine_energy_diff(x, s)
        if self.prm.coarse_model == "fine":
            IL = self.IL[self._level_index(lev)]
            return self.fine_energy_diff(IL @ x, IL @ s)
        return fem.energy_diff(lev.grid, x, s, lev.p, lev.mat)

    def _level_index(self, lev):
        for l, v in self.levels.items():
            if v is lev:
                return l
        raise KeyError("level not in this hierarchy")

    def h_grad(self, lev, x):
        if lev.finest:
            return self.fine_gradient(x)
        g = lev.dg + lev.Hmod @ (x - lev.x0)
        if self._ftilde_active(lev):
            g = g + self.ft_grad(lev, x) - lev.Hf0 @ (x - lev.x0)
        g[lev.dirichlet] = 0.0
        return g

    def h_diff(self, lev, x, s):
        """h(x + s) - h(x)."""
        out = 0.0
        if self._ftilde_active(lev):
            out += self.ft_diff(lev, x, s)
        if not lev.finest:
            dx = x - lev.x0
            dHdx = lev.Hmod @ dx
            dHs = lev.Hmod @ s
            if self._ftilde_active(lev):
                dHdx = dHdx - lev.Hf0 @ dx
                dHs = dHs - lev.Hf0 @ s
            out += float(lev.dg @ s) + float(s @ dHdx) + 0.5 * float(s @ dHs)
        return out

    # ------------------------------------------------------------ boxes
    def step_box(self, lev, x, delta):
        lo = np.maximum(lev.Lb - x, -delta)
        hi = np.minimum(lev.Ub - x, delta)
        lo[lev.dirichlet] = 0.0
        hi[lev.dirichlet] = 0.0
        return lo, hi

    # ------------------------------------------------------------ ratio
    def ratio(self, ared, pred, lev):
        # round-off level of a sum of per-element energy differences: about
        # eps |f| / sqrt(number of elements) (independent element errors)
        tol = self.prm.guard * abs(self.f_ref) / np.sqrt(lev.grid.n_elems)
        if not np.isfinite(ared) or not np.isfinite(pred):
            return -np.inf
        if abs(pred) <= tol:
            return 1.0 if ared >= -tol else -np.inf
        if pred <= 0.0:
            return -np.inf
        return ared / pred

    def control(self, rho, delta, s):
        """Algorithm 3: returns (accept, new radius).  Variant: with
        shrink_to_step the radius after a rejection is gamma1 times the
        smaller of delta and the rejected step's infinity norm."""
        prm = self.prm
        accept = rho > prm.eta1
        if rho < prm.eta1:
            base = min(delta, float(np.max(np.abs(s)))) if prm.shrink_to_step else delta
            delta = prm.gamma1 * base
        elif rho > prm.eta2:
            delta = min(prm.gamma2 * delta, prm.delta_max)
        return accept, delta

    # ---------------------------------------------------------- TR step
    def solve_qp(self, lev, g, lo, hi, coarsest):
        H = lev.Hmod
        if coarsest:
            fb = lambda s0: qp.pgs(H, g, lo, hi, s0.copy(), lev.blocks,
                                   self.prm.fallback_sweeps, lev.free)
            s, _, _ = qp.mprgp(H, g, lo, hi, None, self.prm.coarse_qp_rtol,
                               self.prm.coarse_qp_its, fallback=fb)
            return s
        s = np.zeros_like(g)
        return qp.pgs(H, g, lo, hi, s, lev.blocks, self.prm.pgs_sweeps, lev.free)

    def tr_step(self, lev, x, delta, coarsest=False):
        g = self.h_grad(lev, x)
        lo, hi = self.step_box(lev, x, delta)
        s = self.solve_qp(lev, g, lo, hi, coarsest)
        if not np.any(s != 0.0):
            return x, delta
        pred = -(float(g @ s) + 0.5 * float(s @ (lev.Hmod @ s)))
        ared = -self.h_diff(lev, x, s)
        rho = self.ratio(ared, pred, lev)
        accept, delta = self.control(rho, delta, s)
        if accept:
            self.stats.tr_accepted += 1
            return x + s, delta
        self.stats.tr_rejected += 1
        return x, delta

    def nonlinear_solve(self, lev, x, delta, its, coarsest=False):
        """Algorithm 2 with exactly `its` iterations."""
        for _ in range(its):
            x, delta = self.tr_step(lev, x, delta, coarsest)
        return x, delta

    # ----------------------------------------------------------- V-cycle
    def setup_coarse(self, l, x, delta):
        """Build level l-1 from level l at the pre-smoothed iterate x."""
        lev, c = self.levels[l], self.levels[l - 1]
        I, R, P = self.I[l - 1], self.R[l - 1], self.P[l - 1]
        c.x0 = P @ x
        lo, hi = self.step_box(lev, x, delta)
        loH, hiH = transfer.box_restrict(I, lo, hi)
        c.Lb = c.x0 + loH
        c.Ub = c.x0 + hiH
        g = self.h_grad(lev, x)
        if self.prm.coarse_model != "zero":
            c.Hf0 = self.ft_hessian(c, c.x0)
            c.dg = R @ g - self.ft_grad(c, c.x0)
        else:
            c.Hf0 = None
            c.dg = R @ g
        if self.prm.first_order:
            # dH = 0: the coarse model's Hessian is grad^2 f~ at x0
            c.Hmod = c.Hf0.copy()
        else:
            # Galerkin product restricted to the coarse free dofs (the coarse
            # problem, like the fine one, has no displacement dofs on the
            # boundary)
            Dc = sp.diags(c.free.astype(np.float64))
            c.Hmod = (Dc @ (R @ lev.Hmod @ I) @ Dc).tocsr()
        c.Hmod.sort_indices()
        c.dg[c.dirichlet] = 0.0

    def vcycle(self, l, x, delta):
        lev = self.levels[l]
        if l == 1:
            return self.nonlinear_solve(lev, x, delta, self.prm.coarse_tr_its, coarsest=True)
        x, delta = self.nonlinear_solve(lev, x, delta, self.prm.mu1)
        self.setup_coarse(l, x, delta)
        c = self.levels[l - 1]
        xs, _ = self.vcycle(l - 1, c.x0.copy(), delta)
        sc = xs - c.x0
        if np.any(sc != 0.0):
            s = self.I[l - 1] @ sc
            ared = -self.h_diff(lev, x, s)
            pred = -self.h_diff(c, c.x0, sc)
            rho = self.ratio(ared, pred, lev)
            accept, delta = self.control(rho, delta, s)
            if accept:
                x = x + s
        x, delta = self.nonlinear_solve(lev, x, delta, self.prm.mu2)
        return x, delta

    # -------------------------------------------------------- load step
    def solve_loadstep(self, x, c_lower):
        """Minimise f over c_lower <= c <= 1 from x; returns (x, stats)."""
        prm = self.prm
        fine = self.levels[self.L]
        nc = self.d + 1
        n = fine.grid.n_dofs
        fine.Lb = np.full(n, -np.inf)
        fine.Ub = np.full(n, np.inf)
        fine.Lb[self.d::nc] = c_lower
        fine.Ub[self.d::nc] = 1.0
        self.stats = Stats()
        delta = prm.delta0
        g = self.fine_gradient(x)
        chi0 = fem.chi(fine.grid, x, g, c_lower, fine.dirichlet)
        self.f_ref = self.fine_energy(x)
        self.stats.chi0 = self.stats.chi = chi0
        if chi0 == 0.0:
            return x, self.stats
        for v in range(prm.max_vcycles):
            fine.x0 = x.copy()
            fine.Hmod = fem.hessian(fine.grid, x, fine.p, fine.mat, fine.dirichlet)
            x, delta = self.vcycle(self.L, x, delta)
            g = self.fine_gradient(x)
            chi = fem.chi(fine.grid, x, g, c_lower, fine.dirichlet)
            self.stats.vcycles = v + 1
            self.stats.chi = chi
            self.stats.history.append((chi, delta))
            if chi <= prm.rtol * chi0:
                break
        self.stats.energy = self.fine_energy(x)
        return x, self.stats

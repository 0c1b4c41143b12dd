"""Workload sizes and parameters (synthetic stand-ins for the paper's
fracture-network runs).  Sizes count cells per side on the finest level."""
from dataclasses import dataclass, field

from .fractures import disc_table, rect_network_table, c1_crack


def hierarchy_nodes_per_side(coarse_nodes, n_levels):
    """Nodes per side on the finest of n_levels uniform refinements of a
    grid with coarse_nodes nodes per side: each refinement maps n -> 2n - 1."""
    n = coarse_nodes
    for _ in range(n_levels - 1):
        n = 2 * n - 1
    return n


def level_cells(n_cells_fine, n_levels):
    """Cells per side on levels 1 (coarsest) .. L (finest)."""
    assert n_cells_fine % (1 << (n_levels - 1)) == 0
    return [n_cells_fine >> (n_levels - l) for l in range(1, n_levels + 1)]


@dataclass
class Workload:
    name: str
    dim: int
    n_cells: int
    n_levels: int
    E: float = 1.0
    nu: float = 0.3
    Gc: float = 1e-3
    k: float = 1e-6
    p: float = 1e-3
    seed: int = 0
    n_frac: int = 0
    extra: dict = field(default_factory=dict)
    # solver settings that differ from the defaults (rmtr_params fields)
    solver: dict = field(default_factory=dict)

    @property
    def h(self):
        return 1.0 / self.n_cells

    @property
    def ls(self):
        return 2.0 * self.h

    @property
    def lam(self):
        return self.E * self.nu / ((1.0 + self.nu) * (1.0 - 2.0 * self.nu))

    @property
    def mu(self):
        return self.E / (2.0 * (1.0 + self.nu))

    @property
    def n_nodes(self):
        return (self.n_cells + 1) ** self.dim

    @property
    def n_dofs(self):
        return (self.dim + 1) * self.n_nodes

    def fractures(self):
        if self.dim == 2:
            if self.n_frac == 0:
                return c1_crack(self.n_cells, self.p)
            e = self.extra
            return rect_network_table(self.n_frac, self.seed, e["angle_deg"], e["l_min"], e["l_max"],
                                      e["exponent"], self.h, self.p)
        e = self.extra
        return disc_table(self.n_frac, self.seed, e["centre_lo"], e["centre_hi"],
                          e["r_lo"], e["r_hi"], log_radius=e.get("log_radius", False),
                          p_lo=e.get("p_lo"), p_hi=e.get("p_hi"), p_const=self.p)


WORKLOADS = {
    # 2D, 64x64 cells, one straight crack, uniform p, 3 levels.
    "c1_2d_64": Workload("c1_2d_64", 2, 64, 3),
    # 2D stochastic network (Sec. 5.2): 2048^2 cells (12.6 M dofs, near the
    # paper's 13.6 M), 1000 line fractures of width 2h, hypocentres uniform,
    # orientation U[-80, 80] degrees, lengths from n(l) ~ l^-2 on
    # [0.01, 0.2]; p uniform; 8 levels (coarsest 16^2).
    "f2_2d_2048": Workload("f2_2d_2048", 2, 2048, 8, seed=6, n_frac=1000,
                           extra=dict(angle_deg=80.0, l_min=0.01, l_max=0.2, exponent=2.0)),
    # 3D, 128^3 cells, 10 discs, radii U[0.03, 0.08], centres U[0.2, 0.8]^3.
    "c2_3d_128": Workload("c2_3d_128", 3, 128, 4, seed=2, n_frac=10,
                          extra=dict(centre_lo=0.2, centre_hi=0.8, r_lo=0.03, r_hi=0.08)),
    # 3D, 256^3 cells, 100 discs, radii log-U[0.01, 0.06], centres U[0.1, 0.9]^3.
    # Smoothing: 2 pre- and 2 post-smoothing TR steps of 6 PGS sweeps, and
    # the radius of a rejected step measured from the step taken.
    "c3_3d_256": Workload("c3_3d_256", 3, 256, 5, seed=3, n_frac=100,
                          extra=dict(centre_lo=0.1, centre_hi=0.9, r_lo=0.01, r_hi=0.06,
                                     log_radius=True),
                          solver=dict(mu1=2, mu2=2, pgs_sweeps=6, shrink_to_step=1)),
    # 3D, 384^3 cells, 1000 discs, radii log-U[0.005, 0.04], p_f U[5e-4, 2e-3].
    "c4_3d_384": Workload("c4_3d_384", 3, 384, 5, seed=4, n_frac=1000,
                          extra=dict(centre_lo=0.1, centre_hi=0.9, r_lo=0.005, r_hi=0.04,
                                     log_radius=True, p_lo=5e-4, p_hi=2e-3),
                          solver=dict(mu1=2, mu2=2, pgs_sweeps=6, shrink_to_step=1)),
}

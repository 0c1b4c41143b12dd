"""Oracle: initial phase field c0 and the nodal pressure field.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Nodal inclusion (Sec. 5, first paragraph; Sec. 5.2 for the networks): a node
whose position lies inside a fracture's volumetric description gets c = 1,
every other node c = 0.
  3D: a penny-shaped disc thickened by h (distance from the node to the disc
      at most h);
  2D: a rectangle of the fracture's length and width 2h ("smooth rectangle").
The pressure is a given nodal field (Sec. 2): either uniform, or per fracture,
p_node = max{ p_f : dist(node, disc_f) <= band }, else 0.

All arithmetic is written so that a second implementation can reproduce it
bit for bit: coordinates i/N by one division, dot products summed in index
order without fused multiply-add, and a correctly rounded square root.
"""
import numpy as np

from .fem import Grid


def disc_distance_sq(X, disc):
    """Squared distance from points X (n, 3) to a disc (centre, normal, radius)."""
    cx, cy, cz, nx, ny, nz, r = disc[:7]
    dx = X[:, 0] - cx
    dy = X[:, 1] - cy
    dz = X[:, 2] - cz
    dn = (dx * nx + dy * ny) + dz * nz
    qx = dx - dn * nx
    qy = dy - dn * ny
    qz = dz - dn * nz
    rho2 = (qx * qx + qy * qy) + qz * qz
    out = dn * dn
    outside = rho2 > r * r
    rho = np.sqrt(rho2[outside])
    out = out.copy()
    out[outside] = dn[outside] * dn[outside] + (rho - r) * (rho - r)
    return out


def rect_inside(X, rect):
    """Points X (n, 2) inside the rectangle |d.t| <= a, |d.n| <= w, n = (-t_y, t_x)."""
    cx, cy, tx, ty, a, w = rect[:6]
    dx = X[:, 0] - cx
    dy = X[:, 1] - cy
    dt = dx * tx + dy * ty
    dnn = dx * (-ty) + dy * tx
    return (np.abs(dt) <= a) & (np.abs(dnn) <= w)


def initial_fields(grid: Grid, table, p_uniform=None, p_band=None):
    """Return (c0, p) as float64 nodal arrays.

    p_uniform given: p = p_uniform at every node.  Otherwise (3D only) the
    per-fracture pressure p_f of the table's last column is spread to nodes
    within distance p_band of its disc, taking the maximum over fractures.
    """
    X = grid.node_coords()
    c0 = np.zeros(grid.n_nodes)
    p = np.zeros(grid.n_nodes)
    h = grid.h
    for f in range(table.shape[0]):
        if grid.d == 3:
            d2 = disc_distance_sq(X, table[f])
            c0[d2 <= h * h] = 1.0
            if p_uniform is None:
                sel = d2 <= p_band * p_band
                p[sel] = np.maximum(p[sel], table[f, 7])
        else:
            c0[rect_inside(X, table[f])] = 1.0
            if p_uniform is None:
                raise ValueError("2D pressure field must be uniform")
    if p_uniform is not None:
        p[:] = p_uniform
    return c0, p

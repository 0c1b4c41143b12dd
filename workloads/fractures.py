"""Synthetic fracture networks: tables of parametric fractures.

3D fractures are penny-shaped discs (centre, unit normal, radius, pressure);
2D fractures are thin rectangles (centre, unit tangent, half-length,
half-width, pressure), the volumetric "smooth rectangle" representation of a
line fracture of width 2h.  Tables are float64 arrays, one row per fracture,
generated on the host only, so the oracle and the GPU path read the same
numbers.  Draw order per disc: centre x, y, z; radius; normal (z = 2u-1,
phi = 2*pi*u); then, optionally, the pressure.
"""
import math
import numpy as np

from .splitmix import SplitMix64

DISC_COLS = ("cx", "cy", "cz", "nx", "ny", "nz", "radius", "pressure")
RECT_COLS = ("cx", "cy", "tx", "ty", "half_length", "half_width", "pressure")


def disc_table(n, seed, centre_lo, centre_hi, r_lo, r_hi, log_radius=False,
               p_lo=None, p_hi=None, p_const=0.0):
    """n random discs.  Radii uniform (or log-uniform) in [r_lo, r_hi];
    normals uniform on the unit sphere; pressure uniform in [p_lo, p_hi]
    when given, else p_const."""
    rng = SplitMix64(seed)
    tab = np.zeros((n, len(DISC_COLS)), dtype=np.float64)
    for f in range(n):
        cx = rng.uniform_in(centre_lo, centre_hi)
        cy = rng.uniform_in(centre_lo, centre_hi)
        cz = rng.uniform_in(centre_lo, centre_hi)
        u = rng.uniform()
        if log_radius:
            r = r_lo * (r_hi / r_lo) ** u
        else:
            r = r_lo + (r_hi - r_lo) * u
        z = 2.0 * rng.uniform() - 1.0
        phi = 2.0 * math.pi * rng.uniform()
        s = math.sqrt(max(0.0, 1.0 - z * z))
        nx, ny, nz = s * math.cos(phi), s * math.sin(phi), z
        if p_lo is not None:
            p = rng.uniform_in(p_lo, p_hi)
        else:
            p = p_const
        tab[f] = (cx, cy, cz, nx, ny, nz, r, p)
    return tab


def rect_table(rows):
    """2D fracture table from explicit rows (cx, cy, angle, half_length,
    half_width, pressure); angle in radians from the x axis."""
    tab = np.zeros((len(rows), len(RECT_COLS)), dtype=np.float64)
    for f, (cx, cy, ang, a, w, p) in enumerate(rows):
        if ang == 0.0:
            tx, ty = 1.0, 0.0
        else:
            tx, ty = math.cos(ang), math.sin(ang)
        tab[f] = (cx, cy, tx, ty, a, w, p)
    return tab


def rect_network_table(n, seed, angle_deg, l_min, l_max, exponent, half_width, p_const=0.0):
    """n random line fractures as thin rectangles (the 2D stochastic network
    of the paper's geoscience application, Sec. 5.2): hypocentres uniform over
    the unit square, orientation uniform in [-angle_deg, angle_deg] degrees
    from the x axis, length from the scale-invariant power law
    n(l) ~ l^-exponent on [l_min, l_max] (inverse-CDF draw), width 2 half_width.
    Draw order per fracture: centre x, y; angle; length."""
    rng = SplitMix64(seed)
    tab = np.zeros((n, len(RECT_COLS)), dtype=np.float64)
    a1 = 1.0 - exponent
    lo_p, hi_p = l_min ** a1, l_max ** a1
    for f in range(n):
        cx = rng.uniform()
        cy = rng.uniform()
        ang = math.radians(-angle_deg + 2.0 * angle_deg * rng.uniform())
        u = rng.uniform()
        length = (lo_p + u * (hi_p - lo_p)) ** (1.0 / a1)
        tab[f] = (cx, cy, math.cos(ang), math.sin(ang), 0.5 * length, half_width, p_const)
    return tab


def c1_crack(n_cells, p=1e-3):
    """The straight 2D crack along y = 0.5 for x in [0.4, 0.6], of width 2h."""
    h = 1.0 / n_cells
    return rect_table([(0.5, 0.5, 0.0, 0.1, h, p)])

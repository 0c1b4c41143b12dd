"""Pins for the grid, hierarchy, colouring and initial fields of the oracle."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import fem, fields

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_dof_counts.txt")


def _rows():
    with open(GOLD) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                parts = line.split()
                yield int(parts[0]), parts[1], int(parts[2]), int(parts[3])


@pytest.mark.parametrize("dim,coarse,levels,dofs", list(_rows()))
def test_paper_dof_counts(dim, coarse, levels, dofs):
    """Uniform refinement n -> 2n - 1 per level and d+1 dofs per node
    reproduce every problem size the paper prints."""
    sides = [int(s) for s in coarse.split("x")]
    if len(sides) == 1:
        sides = sides * dim
    fine = [W.hierarchy_nodes_per_side(s, levels) for s in sides]
    n = 1
    for f in fine:
        n *= f
    assert (dim + 1) * n == dofs
    # the weak-scaling remark: 8 N - 7 nodes per side after 4 levels
    if levels == 4:
        assert all(f == 8 * s - 7 for f, s in zip(fine, sides))


def test_grid_counts_and_elements():
    for d, N in [(2, 4), (3, 3)]:
        g = fem.Grid(d, N)
        en = g.elem_nodes()
        assert en.shape == (N ** d, 2 ** d)
        # every interior node belongs to exactly 2^d elements
        counts = np.bincount(en.reshape(-1), minlength=g.n_nodes)
        interior = ~g.boundary_nodes()
        assert np.all(counts[interior] == 2 ** d)
        # element 0's nodes are the corners of the first cell
        ijk = g.node_ijk()[en[0]]
        assert np.array_equal(ijk.max(axis=0), np.ones(d, dtype=int))


def test_colour_classes_are_independent():
    """No two nodes of one colour share an element (the PGS ordering relies on it)."""
    for d, N in [(2, 5), (3, 4)]:
        g = fem.Grid(d, N)
        col = g.node_colour()
        en = g.elem_nodes()
        c = col[en]
        for e in range(en.shape[0]):
            assert len(set(c[e].tolist())) == 2 ** d


def test_c1_crack_nodes():
    """C1 crack: x in [0.4, 0.6], |y - 0.5| <= h, on the 64 x 64 grid."""
    wl = W.WORKLOADS["c1_2d_64"]
    g = fem.Grid(2, 64)
    c0, p = fields.initial_fields(g, wl.fractures(), p_uniform=wl.p)
    ijk = g.node_ijk()[c0 == 1.0]
    assert c0.sum() == 39
    assert set(ijk[:, 0].tolist()) == set(range(26, 39))
    assert set(ijk[:, 1].tolist()) == {31, 32, 33}
    assert np.all(p == wl.p)


def test_disc_distance_against_sampling():
    """Closed-form point-to-disc distance vs brute force over points of the disc."""
    rng = np.random.default_rng(1)
    for trial in range(5):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        disc = np.array([0.5, 0.4, 0.6, n[0], n[1], n[2], 0.2, 0.0])
        # orthonormal in-plane basis
        a = np.cross(n, [1.0, 0.0, 0.0] if abs(n[0]) < 0.9 else [0.0, 1.0, 0.0])
        a /= np.linalg.norm(a)
        b = np.cross(n, a)
        r = np.sqrt(rng.uniform(0, 1, 20000)) * 0.2
        th = rng.uniform(0, 2 * np.pi, 20000)
        pts = disc[:3] + (r * np.cos(th))[:, None] * a + (r * np.sin(th))[:, None] * b
        rim = disc[:3] + 0.2 * (np.cos(th)[:, None] * a + np.sin(th)[:, None] * b)
        pts = np.concatenate([pts, rim])
        X = rng.uniform(0, 1, (50, 3))
        d2 = fields.disc_distance_sq(X, disc)
        brute = np.min(np.sum((X[:, None, :] - pts[None, :, :]) ** 2, axis=2), axis=1)
        assert np.all(np.sqrt(d2) <= np.sqrt(brute) + 1e-12)
        assert np.allclose(np.sqrt(d2), np.sqrt(brute), atol=5e-3)


def test_disc_distance_special_points():
    disc = np.array([0.5, 0.5, 0.5, 0.0, 0.0, 1.0, 0.1, 0.0])
    X = np.array([[0.5, 0.5, 0.7],      # on the axis: |dz|
                  [0.75, 0.5, 0.5],     # in plane, outside: rho - r
                  [0.55, 0.5, 0.5],     # in the disc: 0
                  [0.8, 0.5, 0.9]])     # off-plane, outside rim
    d2 = fields.disc_distance_sq(X, disc)
    assert np.allclose(d2, [0.04, 0.15 ** 2, 0.0, 0.2 ** 2 + 0.4 ** 2], atol=1e-15)


def test_c2_fracture_table_and_inclusion():
    wl = W.WORKLOADS["c2_3d_128"]
    tab = wl.fractures()
    assert tab.shape == (10, 8)
    assert np.all((tab[:, :3] >= 0.2) & (tab[:, :3] <= 0.8))
    assert np.all((tab[:, 6] >= 0.03) & (tab[:, 6] <= 0.08))
    assert np.allclose(np.linalg.norm(tab[:, 3:6], axis=1), 1.0)
    # a small grid: crack volume ~ sum of 2 h pi r^2 (discs thickened by h)
    g = fem.Grid(3, 32)
    c0, _ = fields.initial_fields(g, tab, p_uniform=1e-3)
    vol = c0.sum() * g.h ** 3
    est = np.sum(2 * g.h * np.pi * tab[:, 6] ** 2)
    assert 0.3 * est < vol < 3.0 * est


def test_2d_network_statistics():
    """The 2D stochastic network of the geoscience application (Sec. 5.2):
    hypocentres uniform in the unit square, orientations uniform in
    [-80, 80] degrees, lengths from the power law n(l) ~ l^-2 on [0.01, 0.2],
    whose CDF is F(l) = (1/l_min - 1/l) / (1/l_min - 1/l_max); width 2h."""
    wl = W.WORKLOADS["f2_2d_2048"]
    tab = wl.fractures()
    assert tab.shape == (1000, 7)
    cx, cy, tx, ty, a, w = (tab[:, i] for i in range(6))
    assert np.all((cx >= 0) & (cx < 1) & (cy >= 0) & (cy < 1))
    assert np.allclose(tx * tx + ty * ty, 1.0, atol=1e-15)
    ang = np.degrees(np.arctan2(ty, tx))
    assert np.all(np.abs(ang) <= 80.0)
    length = 2.0 * a
    assert np.all((length >= 0.01) & (length <= 0.2))
    assert np.all(w == 1.0 / 2048)
    F = lambda l: (100.0 - 1.0 / l) / (100.0 - 5.0)  # noqa: E731
    for q in (0.012, 0.02, 0.05, 0.1):
        assert abs(np.mean(length <= q) - F(q)) < 0.05, q
    for q in (-40.0, 0.0, 40.0):
        assert abs(np.mean(ang <= q) - (q + 80.0) / 160.0) < 0.05
    assert abs(np.mean(cx <= 0.5) - 0.5) < 0.05
    # the same seed gives the same table; inclusion marks the rectangles
    assert np.array_equal(tab, wl.fractures())
    g = fem.Grid(2, 128)
    c0, p = fields.initial_fields(g, W.rect_network_table(30, 16, 80.0, 0.05, 0.3, 2.0, 1.0 / 128, 1e-3),
                                  p_uniform=1e-3)
    assert 500 < c0.sum() < 2000 and np.all(p == 1e-3)

"""The 2D stochastic fracture network of the geoscience application
(Sec. 5.2): 1000 line fractures of width 2h on a 2048^2 grid (12.6 M dofs,
8 levels), uniform p.  The initial phase field is checked bit for bit at
sampled nodes against the oracle's inclusion test; a load step, capped at a
fixed number of V-cycles (this workload does not reach 1e-8: see the design
notes on steps that cross the tension/compression kink in broken elements),
must lower the energy, stay feasible and leave an iterate whose gradient
rows at sampled nodes the oracle reproduces.  On a small network (128^2,
30 fractures) the first V-cycles match the oracle's RMTR iterate for
iterate."""
import numpy as np
import pytest

import workloads as W
from oracle import fem, fields, rmtr
from _util import material, ctx_for, dev, host

pytestmark = pytest.mark.gpu


def _ctx(wl):
    import paper_2007_12908_amd as P
    ctx = P.Context(2, wl.n_cells, wl.n_levels, wl.lam, wl.mu, wl.Gc, wl.ls, wl.k)
    c0, p = ctx.init_fields(wl.n_levels, wl.fractures(), band=wl.h, p_mode=0, p_value=wl.p)
    return ctx, c0, p


def _sample(N, c0, rng):
    crack = np.flatnonzero(c0 == 1.0)
    return np.unique(np.concatenate([rng.integers(0, (N + 1) ** 2, 20000),
                                     rng.choice(crack, min(5000, crack.size), replace=False)]))


def test_f2_network_fields_and_capped_loadstep():
    import torch
    import paper_2007_12908_amd as P
    wl = W.WORKLOADS["f2_2d_2048"]
    N, L = wl.n_cells, wl.n_levels
    print("case f2_2d_2048 fields", flush=True)
    ctx, c0d, pd = _ctx(wl)
    c0 = host(c0d)
    rng = np.random.default_rng(5)
    nodes = _sample(N, c0, rng)
    g = fem.Grid(2, N)
    X = g.node_coords()[nodes]
    want = np.zeros(nodes.size)
    for row in wl.fractures():
        want[fields.rect_inside(X, row)] = 1.0
    assert np.array_equal(c0[nodes], want)
    assert c0.sum() > 1e5 and np.all(host(pd) == wl.p)
    print("case f2_2d_2048 capped load step", flush=True)
    x = torch.zeros(3 * (N + 1) ** 2, dtype=torch.float64, device="cuda")
    x.view(-1, 3)[:, 2] = c0d
    E0 = float(host(ctx.energy(L, x, pd))[0])
    st = ctx.solve_loadstep(x, pd, c0d, P.default_params(max_vcycles=60))
    print({k: st[k] for k in ("code", "vcycles", "chi0", "chi", "energy", "seconds")}, flush=True)
    assert st["vcycles"] == 60 or st["code"] == 0
    assert st["energy"] < E0 and st["chi"] < 0.1 * st["chi0"]
    xs = host(x)
    c = xs[2::3]
    assert np.all(c >= c0) and np.all(c <= 1.0)
    bnd = g.boundary_nodes()
    assert np.all(xs.reshape(-1, 3)[bnd, :2] == 0.0)
    G = host(ctx.gradient(L, x, pd))
    rows = rng.choice(nodes, 3000, replace=False)
    mat = fem.material_from_E_nu(wl.E, wl.nu, wl.Gc, wl.ls, wl.k)
    want_rows, go, _ = fem.local_rows(g, xs, host(pd), mat, rows)
    assert np.abs(G[want_rows] - go).max() <= 1e-12 * np.abs(go).max()


def test_small_network_vcycles_match_oracle():
    import paper_2007_12908_amd as P
    N, L = 128, 4
    tab = W.rect_network_table(30, 16, 80.0, 0.05, 0.3, 2.0, 1.0 / N, 1e-3)
    g = fem.Grid(2, N)
    c0, p = fields.initial_fields(g, tab, p_uniform=1e-3)
    mat = material(N)
    x = np.zeros(g.n_dofs)
    x[2::3] = c0
    ctx = ctx_for(2, N, L, mat)
    c0g, pg = ctx.init_fields(L, tab, band=1.0 / N, p_mode=0, p_value=1e-3)
    assert np.array_equal(host(c0g), c0)
    xd = dev(x.copy())
    st = ctx.solve_loadstep(xd, dev(p), dev(c0), P.default_params(max_vcycles=6), history=True)
    solver = rmtr.RMTR(2, N, L, mat, p, rmtr.Params(max_vcycles=6))
    xo, so = solver.solve_loadstep(x.copy(), c0)
    xg = host(xd)
    assert st["vcycles"] == so.vcycles == 6
    assert st["tr_accepted"] == so.tr_accepted and st["tr_rejected"] == so.tr_rejected
    assert st["energy"] == pytest.approx(so.energy, rel=1e-10)
    assert np.abs(xg - xo).max() <= 1e-6 * np.abs(xo).max()
    assert np.allclose(st["chi_history"], [h[0] for h in so.history], rtol=1e-6, atol=0)

"""GPU vs oracle at the benchmark's full size: the c2_3d_128 workload
(128^3 cells, 8,586,756 dofs, 10 penny fractures), in the launch
configuration the benchmark times.

The oracle evaluates what it can at this size: the initial fields and the
energy on the whole grid, gradient and Hv rows at sampled nodes (tile and
chunk edges, the boundary and random interior nodes, each from the elements
around it), and chi of the load step's final iterate (certifying the
solution).  Tolerances as in the small parity tests."""
import numpy as np
import pytest

import workloads as W
from oracle import fem, fields
from _util import field_rel_err, dev, host

pytestmark = pytest.mark.gpu

WL = W.WORKLOADS["c2_3d_128"]
N = WL.n_cells


def _setup():
    import paper_2007_12908_amd as P
    ctx = P.Context(3, N, WL.n_levels, WL.lam, WL.mu, WL.Gc, WL.ls, WL.k)
    c0, p = ctx.init_fields(WL.n_levels, WL.fractures(), band=WL.h, p_mode=0, p_value=WL.p)
    return ctx, c0, p


def _state(c0):
    """The benchmark's state: u ~ N(0, 1e-4) (seed 1234), zero on the
    boundary, c = c0."""
    g = fem.Grid(3, N)
    rng = np.random.default_rng(1234)
    x = np.zeros(g.n_dofs)
    x.reshape(-1, 4)[:, :3] = rng.standard_normal((g.n_nodes, 3)) * 1e-4
    x.reshape(-1, 4)[:, 3] = c0
    x[g.default_dirichlet()] = 0.0
    v = rng.standard_normal(g.n_dofs)
    return g, x, v


def _sample_nodes(g, rng, n_random=1500):
    # tile edges of both tilings (15-node overlapping tiles and 16-element
    # tiles), chunk edges, the boundary
    s = [0, 1, 14, 15, 16, 17, 29, 30, 31, 32, 33, 47, 48, 63, 64, 65, 96, 112, N - 1, N]
    ijk = np.array([(i, j, k) for i in s for j in s[::2] for k in s[::3]])
    nodes = ijk[:, 0] + (N + 1) * (ijk[:, 1] + (N + 1) * ijk[:, 2])
    return np.unique(np.concatenate([nodes, rng.choice(g.n_nodes, n_random, replace=False)]))


def test_fields_energy_and_sampled_rows_fullsize():
    import torch
    print("case c2_3d_128 fields/energy/rows", flush=True)
    ctx, c0d, pd = _setup()
    g = fem.Grid(3, N)
    c0o, po = fields.initial_fields(g, WL.fractures(), p_uniform=WL.p)
    c0 = host(c0d)
    assert np.array_equal(c0, c0o) and np.array_equal(host(pd), po)
    g, x, v = _state(c0)
    xd, vd = dev(x), dev(v)
    E = float(host(ctx.energy(WL.n_levels, xd, pd))[0])
    Eo = fem.energy(g, x, po, _mat())
    assert E == pytest.approx(Eo, rel=1e-12)
    G = host(ctx.gradient(WL.n_levels, xd, pd))
    HV = host(ctx.hessvec(WL.n_levels, xd, pd, vd))
    HV32 = host(ctx.hessvec(WL.n_levels, xd.float(), pd.float(), vd.float())).astype(np.float64)
    rng = np.random.default_rng(5)
    nodes = _sample_nodes(g, rng)
    want, go, hvo = fem.local_rows(g, x, po, _mat(), nodes, v=v)
    assert field_rel_err(G[want], go, 3) <= 1e-12
    assert field_rel_err(HV[want], hvo, 3) <= 1e-12
    # FP32 Hv: oracle on the FP32-rounded inputs
    r32 = lambda a: a.astype(np.float32).astype(np.float64)
    _, _, hvo32 = fem.local_rows(g, r32(x), r32(po), _mat(), nodes, v=r32(v))
    assert field_rel_err(HV32[want], hvo32, 3) <= 2e-5
    del torch


def _mat():
    return fem.material_from_E_nu(WL.E, WL.nu, WL.Gc, WL.ls, WL.k)


@pytest.mark.parametrize("precision", [0, 1])
def test_loadstep_fullsize_certified_by_oracle(precision):
    """One load step of the benchmark (plain FP64 and mixed): the final
    iterate's chi, recomputed from the oracle's FP64 gradient, is within
    1e-8 of chi at the start, and the bounds hold exactly."""
    import torch
    import paper_2007_12908_amd as P
    print(f"case c2_3d_128 load step precision={precision}", flush=True)
    ctx, c0d, pd = _setup()
    x = torch.zeros(4 * (N + 1) ** 3, dtype=torch.float64, device="cuda")
    x.view(-1, 4)[:, 3] = c0d
    st = ctx.solve_loadstep(x, pd, c0d, P.default_params(precision=precision))
    print({k: st[k] for k in ("code", "vcycles", "chi0", "chi", "seconds")}, flush=True)
    assert st["code"] == 0
    g = fem.Grid(3, N)
    xs, c0, p = host(x), host(c0d), host(pd)
    x0 = np.zeros_like(xs)
    x0[3::4] = c0
    mat = _mat()
    chi0 = fem.chi(g, x0, fem.gradient(g, x0, p, mat), c0)
    chi = fem.chi(g, xs, fem.gradient(g, xs, p, mat), c0)
    assert chi <= 1e-8 * chi0 * (1 + 1e-6), (chi / chi0)
    c = xs[3::4]
    assert np.all(c >= c0) and np.all(c <= 1.0)
    assert np.all(xs[g.default_dirichlet()] == 0.0)

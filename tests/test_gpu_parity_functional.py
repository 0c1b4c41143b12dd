"""GPU vs oracle: initial fields, energy, energy difference, gradient, Hv,
diagonal blocks (FP64 and the FP32 mixed-precision form).

Every split is covered: unsplit, volumetric-deviatoric and spectral (the
principal strains from Jacobi rotations on the GPU, LAPACK in the oracle).

Tolerances: FP64 results within 1e-12 relative, element by element and
scaled per field (the displacement block and the phase-field block
separately); the FP32 Hv within
2e-5 relative (single-precision arithmetic over sums of ~10^2 terms whose
magnitudes differ by up to the stiffness contrast g(c) ~ 1e-6 .. 1)."""
import numpy as np
import pytest

import workloads as W
from oracle import fem, fields
from _util import material, rand_state, field_rel_err, ctx_for, dev, host

pytestmark = pytest.mark.gpu

# sizes: tiny, odd (ragged tiles), and several 15-node tiles with a ragged tail
CASES = [(2, 6), (2, 13), (3, 3), (3, 5), (3, 20), (3, 33)]


@pytest.mark.parametrize("d,N", CASES)
@pytest.mark.parametrize("split", [True, False, fem.SPLIT_SPECTRAL])
def test_energy_gradient_hessvec_fp64(d, N, split):
    print(f"case d={d} N={N} split={split}", flush=True)
    g, x, p = rand_state(d, N, seed=100 * d + N)
    mat = material(N, split)
    ctx = ctx_for(d, N, 1, mat)
    xd, pd = dev(x), dev(p)
    E = float(host(ctx.energy(1, xd, pd))[0])
    Eo = fem.energy(g, x, p, mat)
    assert E == pytest.approx(Eo, rel=1e-12)
    G = host(ctx.gradient(1, xd, pd))
    Go = fem.gradient(g, x, p, mat)
    assert field_rel_err(G, Go, d) <= 1e-12
    rng = np.random.default_rng(N)
    v = rng.standard_normal(g.n_dofs)
    HV = host(ctx.hessvec(1, xd, pd, dev(v)))
    H = fem.hessian(g, x, p, mat)
    HVo = H @ np.where(g.default_dirichlet(), 0.0, v)
    assert field_rel_err(HV, HVo, d) <= 1e-12
    s = rng.standard_normal(g.n_dofs) * 1e-3
    dE = float(host(ctx.energy_diff(1, xd, dev(s), pd))[0])
    dEo = fem.energy_diff(g, x, s, p, mat)
    assert dE == pytest.approx(dEo, rel=1e-11, abs=1e-15 * abs(Eo))
    # FP32 step (the mixed form's smoother output): the kernel widens it, so
    # the difference is the FP64 one of the rounded step
    s32 = s.astype(np.float32)
    dE32 = float(host(ctx.energy_diff(1, xd, dev(s32), pd))[0])
    dEo32 = fem.energy_diff(g, x, s32.astype(np.float64), p, mat)
    assert dE32 == pytest.approx(dEo32, rel=1e-11, abs=1e-15 * abs(Eo))
    D = host(ctx.diag_blocks(1, xd, pd)).reshape(-1, d + 1, d + 1)
    Do = fem.diag_blocks(H, g)
    assert np.abs(D - Do).max() <= 1e-12 * np.abs(Do).max()


@pytest.mark.parametrize("N,split,masked", [(48, True, False), (52, False, True)])
def test_large_level_tiles(N, split, masked):
    """Levels of several tiles per side: the energy, gradient and Hv tile
    the elements in 16 x 16 columns (48 is three whole tiles per side, so
    the last border line is the domain's face; 52 leaves a ragged last
    tile), and the gradient and Hv add the tile-border nodes and segment
    seams in their second kernel (at 48, 441 workgroups take one node layer
    each, so every layer above the first is a seam; at 52 some ranges
    cross a column).  Element-by-element parity over the whole grid, with
    the default and a random Dirichlet mask."""
    print(f"case N={N} split={split} masked={masked}", flush=True)
    import torch
    d = 3
    g, x, p = rand_state(d, N, seed=900 + N)
    mat = material(N, split)
    ctx = ctx_for(d, N, 1, mat)
    rng = np.random.default_rng(N)
    dirm, md = None, None
    if masked:
        mask_nodes = rng.integers(0, 1 << (d + 1), g.n_nodes).astype(np.uint8)
        dirm = np.zeros((g.n_nodes, d + 1), bool)
        for k in range(d + 1):
            dirm[:, k] = (mask_nodes >> k) & 1
        dirm = dirm.reshape(-1)
        md = torch.from_numpy(mask_nodes).cuda()
    xd, pd = dev(x), dev(p)
    E = float(host(ctx.energy(1, xd, pd))[0])
    assert E == pytest.approx(fem.energy(g, x, p, mat), rel=1e-12)
    G = host(ctx.gradient(1, xd, pd, md))
    assert field_rel_err(G, fem.gradient(g, x, p, mat, dirm), d) <= 1e-12
    v = rng.standard_normal(g.n_dofs)
    HV = host(ctx.hessvec(1, xd, pd, dev(v), md))
    dmask = g.default_dirichlet() if dirm is None else dirm
    HVo = fem.hessian(g, x, p, mat, dirm) @ np.where(dmask, 0.0, v)
    assert field_rel_err(HV, HVo, d) <= 1e-12


@pytest.mark.parametrize("d,N", [(2, 13), (3, 5), (3, 33)])
def test_custom_dirichlet_mask(d, N):
    g, x, p = rand_state(d, N, seed=7 + N)
    mat = material(N)
    rng = np.random.default_rng(3)
    mask_nodes = rng.integers(0, 1 << (d + 1), g.n_nodes).astype(np.uint8)
    dirm = np.zeros((g.n_nodes, d + 1), bool)
    for k in range(d + 1):
        dirm[:, k] = (mask_nodes >> k) & 1
    dirm = dirm.reshape(-1)
    ctx = ctx_for(d, N, 1, mat)
    import torch
    md = torch.from_numpy(mask_nodes).cuda()
    G = host(ctx.gradient(1, dev(x), dev(p), md))
    Go = fem.gradient(g, x, p, mat, dirm)
    assert field_rel_err(G, Go, d) <= 1e-12
    v = rng.standard_normal(g.n_dofs)
    HV = host(ctx.hessvec(1, dev(x), dev(p), dev(v), md))
    HVo = fem.hessian(g, x, p, mat, dirm) @ np.where(dirm, 0.0, v)
    assert field_rel_err(HV, HVo, d) <= 1e-12


@pytest.mark.parametrize("d,N", [(2, 13), (3, 5), (3, 33)])
@pytest.mark.parametrize("split", [fem.SPLIT_VOLDEV, fem.SPLIT_SPECTRAL])
def test_hessvec_fp32_mixed(d, N, split):
    import torch
    g, x, p = rand_state(d, N, seed=11 * N)
    mat = material(N, split)
    ctx = ctx_for(d, N, 1, mat)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(g.n_dofs)
    HV = host(ctx.hessvec(1, dev(x, torch.float32), dev(p, torch.float32), dev(v, torch.float32)))
    # oracle on the FP32-rounded inputs, in FP64
    x32 = x.astype(np.float32).astype(np.float64)
    p32 = p.astype(np.float32).astype(np.float64)
    v32 = v.astype(np.float32).astype(np.float64)
    HVo = fem.hessian(g, x32, p32, mat) @ np.where(g.default_dirichlet(), 0.0, v32)
    assert field_rel_err(HV, HVo, d) <= 2e-5


def test_init_fields_bitwise_2d():
    wl = W.WORKLOADS["c1_2d_64"]
    g = fem.Grid(2, 64)
    c0o, po = fields.initial_fields(g, wl.fractures(), p_uniform=wl.p)
    ctx = ctx_for(2, 64, 3, material(64))
    c0, p = ctx.init_fields(3, wl.fractures(), band=g.h, p_mode=0, p_value=wl.p)
    assert np.array_equal(host(c0), c0o) and np.array_equal(host(p), po)
    assert host(c0).sum() == 39


@pytest.mark.parametrize("name,N", [("c2_3d_128", 128), ("c3_3d_256", 64)])
def test_init_fields_bitwise_3d(name, N):
    wl = W.WORKLOADS[name]
    g = fem.Grid(3, N)
    tab = wl.fractures()
    c0o, _ = fields.initial_fields(g, tab, p_uniform=wl.p)
    ctx = ctx_for(3, N, 1, material(N))
    c0, p = ctx.init_fields(1, tab, band=g.h, p_mode=0, p_value=wl.p)
    assert np.array_equal(host(c0), c0o)
    assert c0o.sum() > 0


def test_init_fields_per_fracture_pressure_bitwise():
    """C4-style pressure: max p_f of the discs within 4 l_s (= 8 h) of a node."""
    wl = W.WORKLOADS["c4_3d_384"]
    N = 48
    g = fem.Grid(3, N)
    tab = wl.fractures()[:200]
    band = 8.0 * g.h
    c0o, po = fields.initial_fields(g, tab, p_uniform=None, p_band=band)
    ctx = ctx_for(3, N, 1, material(N))
    c0, p = ctx.init_fields(1, tab, band=g.h, p_mode=1, p_band=band)
    assert np.array_equal(host(c0), c0o) and np.array_equal(host(p), po)
    assert (po > 0).sum() > 0


@pytest.mark.parametrize("d,N,c_fill,p_scale", [(3, 1, None, 1e-3), (2, 1, None, 1e-3), (3, 2, 1.0, 1e-3),
                                                (3, 4, 1.0, 0.0), (2, 3, 0.0, 0.0), (3, 17, 1.0, 1e-3)])
def test_degenerate_cases(d, N, c_fill, p_scale):
    """A single element (every node on the boundary), a fully broken field
    (c = 1: g(c) = k and no pressure work), an intact field and zero
    pressure."""
    print(f"case d={d} N={N} c={c_fill} p={p_scale}", flush=True)
    g, x, p = rand_state(d, N, seed=31 * N + d, p_scale=max(p_scale, 1e-30))
    if p_scale == 0.0:
        p[:] = 0.0
    if c_fill is not None:
        x.reshape(-1, d + 1)[:, d] = c_fill
    mat = material(N)
    ctx = ctx_for(d, N, 1, mat)
    xd, pd = dev(x), dev(p)
    E = float(host(ctx.energy(1, xd, pd))[0])
    assert E == pytest.approx(fem.energy(g, x, p, mat), rel=1e-12)
    Go = fem.gradient(g, x, p, mat)
    assert field_rel_err(host(ctx.gradient(1, xd, pd)), Go, d) <= 1e-12
    v = np.random.default_rng(N).standard_normal(g.n_dofs)
    HVo = fem.hessian(g, x, p, mat) @ np.where(g.default_dirichlet(), 0.0, v)
    assert field_rel_err(host(ctx.hessvec(1, xd, pd, dev(v))), HVo, d) <= 1e-12

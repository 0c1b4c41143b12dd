"""The C-ABI library loads on any host and exports every entry point that
include/rmtr.h declares (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmtr.h")
LIB = os.path.join(ROOT, "paper_2007_12908_amd", "librmtr.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rmtr_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary_calls():
    names = declared()
    for n in ["rmtr_energy", "rmtr_gradient", "rmtr_hessvec", "rmtr_smooth", "rmtr_restrict",
              "rmtr_prolong", "rmtr_solve_loadstep"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("librmtr.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_2007_12908_amd import binding
    assert sorted(binding.EXPORTS) == declared()


def test_create_validates_model_without_gpu():
    from paper_2007_12908_amd import binding
    lib = binding.load()
    h = ctypes.c_void_p()
    bad = binding.Model(3, 10, 3, 1, 1.0, 1.0, 1e-3, 0.1, 1e-6)     # 10 % 4 != 0
    assert lib.rmtr_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    good = binding.Model(3, 16, 3, 1, 1.0, 1.0, 1e-3, 0.1, 1e-6)
    assert lib.rmtr_create(ctypes.byref(good), ctypes.byref(h)) == 0
    assert lib.rmtr_level_nodes(h, 1) == 5 ** 3 and lib.rmtr_level_nodes(h, 3) == 17 ** 3
    assert lib.rmtr_level_nodes(h, 4) == -1
    lib.rmtr_destroy(h)
    # split: 0 unsplit, 1 volumetric-deviatoric, 2 spectral; nothing else
    for split, want in ((0, 0), (2, 0), (3, -1), (-1, -1)):
        m = binding.Model(2, 8, 2, split, 1.0, 1.0, 1e-3, 0.1, 1e-6)
        assert lib.rmtr_create(ctypes.byref(m), ctypes.byref(h)) == want
        if want == 0:
            lib.rmtr_destroy(h)
    p = binding.default_params()
    assert (p.eta1, p.eta2, p.gamma1, p.gamma2, p.pgs_sweeps, p.mu1, p.mu2) == (0.1, 0.75, 0.5, 2.0, 3, 1, 1)
    assert p.use_learned == 0 and not p.nn


def test_nn_sizes_without_gpu():
    """Parameter counts of the 8-32-32-32-32-32-4 network of 3x3x3 layers."""
    from oracle import cnn
    from paper_2007_12908_amd import binding
    lib = binding.load()
    nw = sum(27 * a * b for a, b in zip(cnn.CHANNELS[:-1], cnn.CHANNELS[1:]))
    nb = sum(cnn.CHANNELS[1:])
    assert lib.rmtr_nn_size(0, 1, 1, 1) == nw == binding.NN_WEIGHTS
    assert lib.rmtr_nn_size(1, 1, 1, 1) == nb == binding.NN_BIASES
    assert nw + nb == 121124
    assert lib.rmtr_nn_size(2, 3, 4, 5) == 60 * sum(cnn.CHANNELS)
    assert lib.rmtr_nn_size(2, 0, 4, 5) == -1 and lib.rmtr_nn_size(7, 1, 1, 1) == -1


def test_host_arrays_are_refused_without_a_fallback():
    """The product path has no CPU fallback: host tensors are refused before
    the library is called (no GPU call is made)."""
    import torch
    from paper_2007_12908_amd import binding
    assert binding._ptr(None) is None
    with pytest.raises(ValueError, match="device tensors"):
        binding._ptr(torch.zeros(4, dtype=torch.float64))
    ctx = binding.Context(3, 4, 2, 1.0, 1.0, 1e-3, 0.5)
    x = torch.zeros(4 * 5 ** 3, dtype=torch.float64)
    p = torch.zeros(5 ** 3, dtype=torch.float64)
    out = torch.zeros(1, dtype=torch.float64)
    for call in (lambda: ctx.energy(2, x, p, out=out), lambda: ctx.gradient(2, x, p, out=torch.zeros_like(x)),
                 lambda: ctx.hessvec(2, x, p, x, out=torch.zeros_like(x))):
        with pytest.raises(ValueError, match="device tensors"):
            call()


def test_binding_checks_dtype_and_size_before_any_call():
    """A wrongly typed or sized array is refused by the binding (ValueError)
    before the library sees a pointer; the checks come before the device
    check, so they run here on host tensors."""
    import torch
    from paper_2007_12908_amd import binding
    ctx = binding.Context(3, 4, 2, 1.0, 1.0, 1e-3, 0.5)
    n, nn = 4 * 5 ** 3, 5 ** 3
    x = torch.zeros(n, dtype=torch.float64)
    p = torch.zeros(nn, dtype=torch.float64)
    cases = [
        (lambda: ctx.energy(2, x.float(), p), "dtype"),                       # float32 read as double
        (lambda: ctx.energy(2, x[:-4], p), "elements"),                      # short x
        (lambda: ctx.energy(1, x, p), "elements"),                           # x of the wrong level
        (lambda: ctx.gradient(2, x, p, dirichlet=torch.zeros(nn, dtype=torch.int32)), "dtype"),
        (lambda: ctx.gradient(2, x, p, dirichlet=torch.zeros(nn - 1, dtype=torch.uint8)), "elements"),
        (lambda: ctx.hessvec(2, x, p, x.float()), "dtype"),                  # mixed FP64/FP32 operands
        (lambda: ctx.hessvec(2, x.float(), p, x.float()), "dtype"),          # p must follow x_lin
        (lambda: ctx.dot(x, x[:-1]), "elements"),
        (lambda: ctx.chi(2, x, x, p[:-1]), "elements"),
        (lambda: ctx.smooth(2, x, p, x.float(), x, x, x, 3), "dtype"),
        (lambda: ctx.restrict(2, x[:-1]), "elements"),
        (lambda: ctx.prolong(1, x), "elements"),
        (lambda: ctx.solve_loadstep(x, p, p.float()), "dtype"),
        (lambda: ctx.nn_target(2, x, x, torch.zeros(11)), "elements"),
    ]
    for call, what in cases:
        with pytest.raises(ValueError, match=what):
            call()
    with pytest.raises(ValueError, match="level"):
        ctx.level_nodes(3)


def test_workspace_sizes_without_gpu():
    """rmtr_workspace_bytes is host arithmetic over the buffers a load step
    allocates: the FP32 finest stencil of the mixed form makes it smaller,
    the learned proposal adds its 76 floats per finest node (and dalloc's
    256-byte slack and rounding)."""
    from paper_2007_12908_amd import binding
    ctx = binding.Context(3, 32, 3, 1.0, 1.0, 1e-3, 0.5)
    common = ctx.workspace_bytes()
    fp64 = ctx.workspace_bytes(binding.default_params())
    mixed = ctx.workspace_bytes(binding.default_params(precision=1))
    learned = ctx.workspace_bytes(binding.default_params(precision=1, use_learned=1))
    assert 0 < common < mixed < fp64
    nodes = 33 ** 3
    assert learned - mixed == (nodes * 76 * 4 + 256 + 255) // 256 * 256
    # a finer grid needs more, roughly 8x per refinement
    ctx2 = binding.Context(3, 64, 4, 1.0, 1.0, 1e-3, 0.5)
    assert 6 * fp64 < ctx2.workspace_bytes(binding.default_params()) < 10 * fp64


def test_bind_workspace_and_gs_mode_argument_checks_without_gpu():
    """Host-side refusals: a misaligned or empty workspace, a second bind,
    and the hybrid Gauss-Seidel order that is not built; none of them
    reaches the GPU."""
    from paper_2007_12908_amd import binding
    lib = binding.load()
    m = binding.Model(3, 8, 2, 1, 1.0, 1.0, 1e-3, 0.25, 1e-6)
    h = ctypes.c_void_p()
    assert lib.rmtr_create(ctypes.byref(m), ctypes.byref(h)) == 0
    fake = 1 << 20                                  # never dereferenced
    assert lib.rmtr_bind_workspace(h, fake + 8, 4096) == binding.RMTR_E_ARG
    assert lib.rmtr_bind_workspace(h, None, 4096) == binding.RMTR_E_ARG
    assert lib.rmtr_bind_workspace(h, fake, 0) == binding.RMTR_E_ARG
    assert lib.rmtr_bind_workspace(h, fake, 4096) == binding.RMTR_OK
    assert lib.rmtr_workspace_used(h) == 0
    assert lib.rmtr_bind_workspace(h, fake, 4096) == binding.RMTR_E_ARG
    assert b"once" in lib.rmtr_last_error(h)
    prm = binding.default_params(gs_mode=1)
    st = binding.Stats()
    r = lib.rmtr_solve_loadstep(h, fake, fake, None, None, ctypes.byref(prm), fake, ctypes.byref(st), None, None)
    assert r == binding.RMTR_E_ARG and b"gs_mode" in lib.rmtr_last_error(h)
    lib.rmtr_destroy(h)

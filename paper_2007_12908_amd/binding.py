"""Thin ctypes binding of librmtr (include/rmtr.h).

Argument marshalling only: torch tensors are passed as device pointers with
torch's current HIP stream; every computation runs in the library's kernels.
Importing this module loads the in-tree librmtr.so and raises if it is
missing: there is no CPU fallback.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmtr.so")

RMTR_OK = 0
RMTR_NOT_CONVERGED = 1
RMTR_E_ARG = -1
RMTR_E_WORKSPACE = -3
RMTR_FP64 = 0
RMTR_FP32 = 1
SPLIT_NONE, SPLIT_VOLDEV, SPLIT_SPECTRAL = 0, 1, 2  # rmtr_model.split
R_DUAL, R_INJECT, R_BOX_LO, R_BOX_HI = 0, 1, 2, 3

EXPORTS = [
    "rmtr_default_params", "rmtr_create", "rmtr_destroy", "rmtr_last_error", "rmtr_level_nodes",
    "rmtr_init_fields", "rmtr_energy", "rmtr_energy_diff", "rmtr_gradient", "rmtr_hessvec",
    "rmtr_diag_blocks", "rmtr_smooth", "rmtr_restrict", "rmtr_prolong", "rmtr_coarse_hessvec", "rmtr_mprgp", "rmtr_dot", "rmtr_chi", "rmtr_solve_loadstep",
    "rmtr_step_box", "rmtr_nn_size", "rmtr_nn_forward", "rmtr_nn_backward", "rmtr_nn_mse", "rmtr_nn_adam_step",
    "rmtr_nn_to_bf16", "rmtr_nn_features", "rmtr_nn_propose", "rmtr_element_flops",
    "rmtr_workspace_bytes", "rmtr_bind_workspace", "rmtr_workspace_used", "rmtr_energy_noalloc",
    "rmtr_nn_channel_rms", "rmtr_nn_target", "rmtr_nn_fit_scales", "rmtr_neumann_load",
]

NN_WEIGHTS = 120960
NN_BIASES = 164
NN_CHANNELS = (8, 32, 32, 32, 32, 32, 4)


class Net(ctypes.Structure):
    """rmtr_nn: device pointers of a trained proposal network."""
    _fields_ = [("w", ctypes.c_void_p), ("bias", ctypes.c_void_p), ("scales", ctypes.c_void_p)]


class Model(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_cells", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("split", ctypes.c_int32), ("lam", ctypes.c_double), ("mu", ctypes.c_double),
                ("Gc", ctypes.c_double), ("ls", ctypes.c_double), ("k", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("eta1", ctypes.c_double), ("eta2", ctypes.c_double), ("gamma1", ctypes.c_double),
                ("gamma2", ctypes.c_double), ("delta0", ctypes.c_double), ("delta_max", ctypes.c_double),
                ("rtol", ctypes.c_double), ("coarse_qp_rtol", ctypes.c_double), ("guard", ctypes.c_double),
                ("mu1", ctypes.c_int32), ("mu2", ctypes.c_int32), ("pgs_sweeps", ctypes.c_int32),
                ("coarse_tr_its", ctypes.c_int32), ("coarse_qp_its", ctypes.c_int32),
                ("fallback_sweeps", ctypes.c_int32), ("max_vcycles", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("coarse_model", ctypes.c_int32),
                ("use_learned", ctypes.c_int32), ("nn", ctypes.POINTER(Net)),
                ("nn_patience", ctypes.c_int32), ("shrink_to_step", ctypes.c_int32),
                ("gs_mode", ctypes.c_int32), ("first_order", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("vcycles", ctypes.c_int32), ("tr_accepted", ctypes.c_int32),
                ("tr_rejected", ctypes.c_int32), ("status", ctypes.c_int32),
                ("chi0", ctypes.c_double), ("chi", ctypes.c_double), ("energy", ctypes.c_double),
                ("seconds", ctypes.c_double), ("nn_proposed", ctypes.c_int32),
                ("nn_accepted", ctypes.c_int32), ("delta", ctypes.c_double)]


_lib = None


def load():
    """Load librmtr.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: run paper_2007_12908_amd.build first")
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "rmtr_default_params": (None, [ctypes.POINTER(Params)]),
            "rmtr_create": (I32, [ctypes.POINTER(Model), ctypes.POINTER(P)]),
            "rmtr_destroy": (None, [P]),
            "rmtr_last_error": (ctypes.c_char_p, [P]),
            "rmtr_level_nodes": (I64, [P, I32]),
            "rmtr_init_fields": (I32, [P, I32, P, I32, D, I32, D, D, P, P, P]),
            "rmtr_energy": (I32, [P, I32, P, P, P, P]),
            "rmtr_energy_diff": (I32, [P, I32, P, P, I32, P, P, P]),
            "rmtr_gradient": (I32, [P, I32, P, P, P, P, P]),
            "rmtr_hessvec": (I32, [P, I32, P, P, P, P, P, I32, P]),
            "rmtr_diag_blocks": (I32, [P, I32, P, P, P, P, I32, P]),
            "rmtr_smooth": (I32, [P, I32, P, P, P, P, P, P, P, I32, I32, P]),
            "rmtr_restrict": (I32, [P, I32, I32, P, P, I32, P]),
            "rmtr_prolong": (I32, [P, I32, P, P, I32, P]),
            "rmtr_coarse_hessvec": (I32, [P, I32, P, P, P, P, P, I32, P]),
            "rmtr_mprgp": (I32, [P, I32, P, P, P, P, P, I32, D, I32, ctypes.POINTER(I32),
                                 ctypes.POINTER(I32), P]),
            "rmtr_dot": (I32, [P, I64, P, P, P, P]),
            "rmtr_chi": (I32, [P, I32, P, P, P, P, P, P]),
            "rmtr_solve_loadstep": (I32, [P, P, P, P, P, ctypes.POINTER(Params), P, ctypes.POINTER(Stats),
                                          P, P]),
            "rmtr_neumann_load": (I32, [P, I32, I32, P, P, P, P]),
            "rmtr_element_flops": (I64, [I32, I32]),
            "rmtr_step_box": (I32, [P, I32, P, P, D, P, P, P, P]),
            "rmtr_nn_size": (I64, [I32, I32, I32, I32]),
            "rmtr_nn_forward": (I32, [P, P, P, P, I32, I32, I32, P]),
            "rmtr_nn_backward": (I32, [P, P, P, P, P, P, I32, I32, I32, P]),
            "rmtr_nn_mse": (I32, [P, P, P, P, P, P, I32, I32, I32, P]),
            "rmtr_nn_adam_step": (I32, [P, I64, I64, ctypes.c_float, I32, P, P, P, P, P, P]),
            "rmtr_nn_to_bf16": (I32, [P, I64, P, P, P]),
            "rmtr_nn_features": (I32, [P, I32, P, P, P, P, P]),
            "rmtr_nn_propose": (I32, [P, I32, ctypes.POINTER(Net), P, P, P, P, P, P]),
            "rmtr_workspace_bytes": (ctypes.c_size_t, [P, ctypes.POINTER(Params)]),
            "rmtr_bind_workspace": (I32, [P, P, ctypes.c_size_t]),
            "rmtr_workspace_used": (ctypes.c_size_t, [P]),
            "rmtr_energy_noalloc": (I32, [P, I32, P, P, P, P]),
            "rmtr_nn_channel_rms": (I32, [P, I32, P, P, P]),
            "rmtr_nn_target": (I32, [P, I32, P, P, P, P, P]),
            "rmtr_nn_fit_scales": (I32, [P, I32, I32, P, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def default_params(**over):
    p = Params()
    load().rmtr_default_params(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def element_flops(dim, kind):
    """Algorithmic flops of one element for an operator kind (see rmtr.h)."""
    return int(load().rmtr_element_flops(dim, kind))


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("librmtr arrays must be device tensors")
    if not t.is_contiguous():
        raise ValueError("librmtr arrays must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


F64, F32, U8, BF16 = (torch.float64,), (torch.float32,), (torch.uint8,), (torch.int16, torch.uint16)
REAL = (torch.float64, torch.float32)


class _DevPtr(ctypes.c_void_p):
    """A device pointer argument that still knows its tensor, so that the
    device and layout checks run after every array of a call has passed its
    dtype and size checks, and before the library is called."""


def _arr(t, name, dtypes, numel=None, min_numel=None, optional=False):
    """Pointer of t after checking what the kernels will assume about it:
    dtype and element count here, device and layout just before the call.
    A wrong array raises ValueError before the library sees it."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name}: array required")
    if t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {' or '.join(str(d) for d in dtypes)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected at least {min_numel}")
    d = _DevPtr(t.data_ptr())
    d.tensor = t
    return d


class _CurrentStream:
    """Stands for torch's current stream in an argument list; replaced by the
    stream handle only after the array checks (so a refused call never
    touches the GPU)."""


def _stream():
    return _CurrentStream()


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prec(t):
    return RMTR_FP32 if t.dtype == torch.float32 else RMTR_FP64


class Context:
    """One hierarchy (rmtr_create) and the calls of include/rmtr.h on it.

    Every method checks the dtype and element count of each array against
    what the call's kernels assume for the level (raising ValueError before
    the library is called), then passes device pointers and torch's current
    stream."""

    def __init__(self, dim, n_cells, n_levels, lam, mu, Gc, ls, k=1e-6, split=True):
        """split: 0 / False unsplit, 1 / True volumetric-deviatoric,
        2 spectral (SPLIT_* constants)."""
        self.lib = load()
        self.model = Model(dim, n_cells, n_levels, int(split), lam, mu, Gc, ls, k)
        h = ctypes.c_void_p()
        st = self._fn("rmtr_create")(ctypes.byref(self.model), ctypes.byref(h))
        if st != RMTR_OK:
            raise ValueError(f"rmtr_create failed ({st})")
        self.h = h
        self.dim, self.L = dim, n_levels
        self.nc = dim + 1
        self.workspace = None

    def close(self):
        if self.h:
            self._fn("rmtr_destroy")(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fn(self, name):
        """The library function `name`, preceded by the device and layout
        checks of its array arguments."""
        fn = getattr(self.lib, name)

        def call(*args):
            for a in args:
                if isinstance(a, _DevPtr):
                    _ptr(a.tensor)
            return fn(*[_stream_handle() if isinstance(a, _CurrentStream) else a for a in args])
        return call

    def _check(self, st, name):
        if st < 0:
            msg = self._fn("rmtr_last_error")(self.h)
            raise RuntimeError(f"{name} failed ({st}): {msg.decode() if msg else ''}")
        return st

    def level_nodes(self, level):
        n = int(self._fn("rmtr_level_nodes")(self.h, level))
        if n < 0:
            raise ValueError(f"level {level} outside 1..{self.L}")
        return n

    def level_dofs(self, level):
        return self.level_nodes(level) * self.nc

    def level_cells(self, level):
        return self.model.n_cells >> (self.L - level)

    # -- caller-owned workspace
    def workspace_bytes(self, params=None):
        return int(self._fn("rmtr_workspace_bytes")(self.h, None if params is None else ctypes.byref(params)))

    def bind_workspace(self, buf):
        """Bind a uint8 device tensor as the context's only device memory (it
        is kept referenced by the context)."""
        self._check(self._fn("rmtr_bind_workspace")(self.h, _arr(buf, "workspace", U8), buf.numel()),
                    "rmtr_bind_workspace")
        self.workspace = buf

    def workspace_used(self):
        return int(self._fn("rmtr_workspace_used")(self.h))

    # -- fields
    def init_fields(self, level, table, band, p_mode=0, p_value=0.0, p_band=0.0):
        import numpy as np
        tab = np.ascontiguousarray(table, dtype=np.float64)
        if tab.ndim != 2 or tab.shape[1] != (8 if self.dim == 3 else 7):
            raise ValueError(f"fracture table: shape {tab.shape}, expected (n, {8 if self.dim == 3 else 7})")
        n = self.level_nodes(level)
        c0 = torch.empty(n, dtype=torch.float64, device="cuda")
        p = torch.empty(n, dtype=torch.float64, device="cuda")
        self._check(self._fn("rmtr_init_fields")(self.h, level, tab.ctypes.data_as(ctypes.c_void_p), tab.shape[0],
                                              band, p_mode, p_value, p_band, _ptr(c0), _ptr(p), _stream()),
                    "rmtr_init_fields")
        return c0, p

    # -- functional
    def _xp(self, level, x, p, dtypes=F64):
        n, nn = self.level_dofs(level), self.level_nodes(level)
        return _arr(x, "x", dtypes, n), _arr(p, "p", (x.dtype,) if x is not None else dtypes, nn)

    def energy(self, level, x, p, out=None):
        out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else out
        px, pp = self._xp(level, x, p)
        self._check(self._fn("rmtr_energy")(self.h, level, px, pp, _arr(out, "out", F64, min_numel=1), _stream()),
                    "rmtr_energy")
        return out

    def energy_noalloc(self, level, x, p, out):
        """rmtr_energy with no allocation at all: `out` must be given."""
        px, pp = self._xp(level, x, p)
        self._check(self._fn("rmtr_energy_noalloc")(self.h, level, px, pp, _arr(out, "out", F64, min_numel=1),
                                                 _stream()), "rmtr_energy_noalloc")
        return out

    def energy_diff(self, level, x, s, p, out=None):
        out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else out
        px, pp = self._xp(level, x, p)
        ps = _arr(s, "s", REAL, self.level_dofs(level))
        self._check(self._fn("rmtr_energy_diff")(self.h, level, px, ps, _prec(s), pp,
                                              _arr(out, "out", F64, min_numel=1), _stream()), "rmtr_energy_diff")
        return out

    def _dir(self, level, dirichlet):
        return _arr(dirichlet, "dirichlet", U8, self.level_nodes(level), optional=True)

    def gradient(self, level, x, p, dirichlet=None, out=None):
        out = torch.empty_like(x) if out is None else out
        px, pp = self._xp(level, x, p)
        self._check(self._fn("rmtr_gradient")(self.h, level, px, pp, self._dir(level, dirichlet),
                                           _arr(out, "g", F64, self.level_dofs(level)), _stream()),
                    "rmtr_gradient")
        return out

    def hessvec(self, level, x_lin, p, v, dirichlet=None, out=None):
        """FP64, or FP32 when x_lin, p, v and out are all float32."""
        out = torch.empty_like(v) if out is None else out
        px, pp = self._xp(level, x_lin, p, REAL)
        n = self.level_dofs(level)
        pv = _arr(v, "v", (x_lin.dtype,), n)
        po = _arr(out, "Hv", (x_lin.dtype,), n)
        self._check(self._fn("rmtr_hessvec")(self.h, level, px, pp, self._dir(level, dirichlet), pv, po,
                                          _prec(x_lin), _stream()), "rmtr_hessvec")
        return out

    def diag_blocks(self, level, x_lin, p, dirichlet=None):
        nc = self.nc
        px, pp = self._xp(level, x_lin, p, REAL)
        D = torch.empty(self.level_nodes(level) * nc * nc, dtype=x_lin.dtype, device=x_lin.device)
        self._check(self._fn("rmtr_diag_blocks")(self.h, level, px, pp, self._dir(level, dirichlet), _ptr(D),
                                              _prec(x_lin), _stream()), "rmtr_diag_blocks")
        return D

    def smooth(self, level, x_lin, p, g, lo, hi, s, n_sweeps, dirichlet=None):
        """Symmetric PGS; x_lin and p are FP64, g/lo/hi/s FP64 or FP32."""
        px, pp = self._xp(level, x_lin, p)
        n = self.level_dofs(level)
        ps = _arr(s, "s", REAL, n)
        dt = (s.dtype,)
        self._check(self._fn("rmtr_smooth")(self.h, level, px, pp, self._dir(level, dirichlet), _arr(g, "g", dt, n),
                                         _arr(lo, "lo", dt, n), _arr(hi, "hi", dt, n), ps, n_sweeps, _prec(s),
                                         _stream()), "rmtr_smooth")
        return s

    # -- transfers
    def restrict(self, fine_level, fine, mode=R_DUAL):
        if not 2 <= fine_level <= self.L:
            raise ValueError(f"fine level {fine_level} outside 2..{self.L}")
        pf = _arr(fine, "fine", REAL, self.level_dofs(fine_level))
        out = torch.empty(self.level_dofs(fine_level - 1), dtype=fine.dtype, device=fine.device)
        self._check(self._fn("rmtr_restrict")(self.h, fine_level, mode, pf, _ptr(out), _prec(fine), _stream()),
                    "rmtr_restrict")
        return out

    def prolong(self, coarse_level, coarse):
        if not 1 <= coarse_level < self.L:
            raise ValueError(f"coarse level {coarse_level} outside 1..{self.L - 1}")
        pc = _arr(coarse, "coarse", REAL, self.level_dofs(coarse_level))
        out = torch.empty(self.level_dofs(coarse_level + 1), dtype=coarse.dtype, device=coarse.device)
        self._check(self._fn("rmtr_prolong")(self.h, coarse_level, pc, _ptr(out), _prec(coarse), _stream()),
                    "rmtr_prolong")
        return out

    def coarse_hessvec(self, level, x_lin, p, v, dirichlet=None, fp32_stencil=False):
        """Galerkin coarse Hessian of `level` (built from the finest stencil at
        x_lin, FP64 or FP32 storage) applied to the FP64 vector v."""
        if not 1 <= level < self.L:
            raise ValueError(f"level {level} outside 1..{self.L - 1}")
        px, pp = self._xp(self.L, x_lin, p)
        pv = _arr(v, "v", F64, self.level_dofs(level))
        out = torch.empty_like(v)
        self._check(self._fn("rmtr_coarse_hessvec")(self.h, level, px, pp, self._dir(self.L, dirichlet), pv,
                                                 _ptr(out), RMTR_FP32 if fp32_stencil else RMTR_FP64, _stream()),
                    "rmtr_coarse_hessvec")
        return out

    def mprgp(self, level, K, g, lo, hi, max_it=500, rtol=1e-10, fallback_sweeps=50):
        """MPRGP on the QP with element matrices K (one dense ((d+1) 2^d)^2
        row-major block per element of `level`)."""
        n = self.level_dofs(level)
        nd = (1 << self.dim) * self.nc
        pK = _arr(K, "K", F64, self.level_cells(level) ** self.dim * nd * nd)
        s = torch.empty_like(g)
        its, status = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._fn("rmtr_mprgp")(self.h, level, pK, _arr(g, "g", F64, n), _arr(lo, "lo", F64, n),
                                        _arr(hi, "hi", F64, n), _ptr(s), max_it, rtol, fallback_sweeps,
                                        ctypes.byref(its), ctypes.byref(status), _stream()), "rmtr_mprgp")
        return s, its.value, status.value

    # -- reductions
    def dot(self, a, b):
        out = torch.empty(1, dtype=torch.float64, device=a.device)
        pa = _arr(a, "a", F64)
        pb = _arr(b, "b", F64, a.numel())
        self._check(self._fn("rmtr_dot")(self.h, a.numel(), pa, pb, _ptr(out), _stream()), "rmtr_dot")
        return out

    def chi(self, level, x, g, c_lower, dirichlet=None):
        out = torch.empty(1, dtype=torch.float64, device=x.device)
        n, nn = self.level_dofs(level), self.level_nodes(level)
        self._check(self._fn("rmtr_chi")(self.h, level, _arr(x, "x", F64, n), _arr(g, "g", F64, n),
                                      _arr(c_lower, "c_lower", F64, nn), self._dir(level, dirichlet), _ptr(out),
                                      _stream()), "rmtr_chi")
        return out

    def step_box(self, level, x, c_lower, delta, dirichlet=None):
        n, nn = self.level_dofs(level), self.level_nodes(level)
        px = _arr(x, "x", F64, n)
        pc = _arr(c_lower, "c_lower", F64, nn)
        lo, hi = torch.empty_like(x), torch.empty_like(x)
        self._check(self._fn("rmtr_step_box")(self.h, level, px, pc, delta, self._dir(level, dirichlet), _ptr(lo),
                                           _ptr(hi), _stream()), "rmtr_step_box")
        return lo, hi

    # -- learned proposal network
    def nn_size(self, what, nx, ny, nz):
        return int(self._fn("rmtr_nn_size")(what, nx, ny, nz))

    def nn_forward(self, w, bias, act, box):
        nx, ny, nz = box
        self._check(self._fn("rmtr_nn_forward")(self.h, _arr(w, "w", BF16, NN_WEIGHTS), _arr(bias, "bias", F32, NN_BIASES),
                                             _arr(act, "act", F32, min_numel=self.nn_size(2, nx, ny, nz)), nx, ny,
                                             nz, _stream()), "rmtr_nn_forward")
        return act

    def nn_backward(self, w, act, dout, grad, work, box):
        nx, ny, nz = box
        nvox = nx * ny * nz
        self._check(self._fn("rmtr_nn_backward")(self.h, _arr(w, "w", BF16, NN_WEIGHTS),
                                              _arr(act, "act", F32, min_numel=self.nn_size(2, nx, ny, nz)),
                                              _arr(dout, "dout", F32, 4 * nvox),
                                              _arr(grad, "grad", F32, NN_WEIGHTS + NN_BIASES),
                                              _arr(work, "work", F32, min_numel=self.nn_size(3, nx, ny, nz)), nx,
                                              ny, nz, _stream()), "rmtr_nn_backward")
        return grad

    def nn_mse(self, out, target, window, dout, loss, box):
        nx, ny, nz = box
        nvox = nx * ny * nz
        win = (ctypes.c_int32 * 6)(*[int(v) for v in window])
        self._check(self._fn("rmtr_nn_mse")(self.h, _arr(out, "out", F32, 4 * nvox), _arr(target, "target", F32, 4 * nvox),
                                         win, _arr(dout, "dout", F32, 4 * nvox), _arr(loss, "loss", F64, min_numel=1),
                                         nx, ny, nz, _stream()), "rmtr_nn_mse")
        return loss

    def nn_adam_step(self, lr, t, grad, master, m, v, w_bf16=None, n_bf16=0):
        n = master.numel()
        if w_bf16 is not None and w_bf16.numel() < n_bf16:
            raise ValueError(f"w_bf16: {w_bf16.numel()} elements, fewer than n_bf16 = {n_bf16}")
        self._check(self._fn("rmtr_nn_adam_step")(self.h, n, n_bf16, lr, t, _arr(grad, "grad", F32, n),
                                               _arr(master, "master", F32), _arr(m, "m", F32, n), _arr(v, "v", F32, n),
                                               _arr(w_bf16, "w_bf16", BF16, optional=n_bf16 == 0), _stream()),
                    "rmtr_nn_adam_step")

    def nn_to_bf16(self, master, w_bf16):
        self._check(self._fn("rmtr_nn_to_bf16")(self.h, w_bf16.numel(), _arr(master, "master", F32, min_numel=w_bf16.numel()),
                                             _arr(w_bf16, "w_bf16", BF16), _stream()), "rmtr_nn_to_bf16")
        return w_bf16

    def nn_features(self, level, x, g, scales, out=None):
        n = self.level_dofs(level)
        out = torch.empty(self.level_nodes(level) * 8, dtype=torch.float32, device=x.device) if out is None else out
        self._check(self._fn("rmtr_nn_features")(self.h, level, _arr(x, "x", F64, n), _arr(g, "g", F64, n),
                                              _arr(scales, "scales", F32, 12),
                                              _arr(out, "in8", F32, 8 * self.level_nodes(level)), _stream()),
                    "rmtr_nn_features")
        return out

    def nn_channel_rms(self, level, v, out=None):
        out = torch.empty(4, dtype=torch.float64, device=v.device) if out is None else out
        self._check(self._fn("rmtr_nn_channel_rms")(self.h, level, _arr(v, "v", F64, self.level_dofs(level)),
                                                 _arr(out, "rms", F64, min_numel=4), _stream()),
                    "rmtr_nn_channel_rms")
        return out

    def nn_target(self, level, g, s, scales, out=None):
        n = self.level_dofs(level)
        out = torch.empty(n, dtype=torch.float32, device=g.device) if out is None else out
        self._check(self._fn("rmtr_nn_target")(self.h, level, _arr(g, "g", F64, n), _arr(s, "s", F64, n),
                                            _arr(scales, "scales", F32, 12), _arr(out, "t", F32, n), _stream()),
                    "rmtr_nn_target")
        return out

    def nn_fit_scales(self, level, samples, scales):
        """scales (12 FP32) from harvested (x, g, s) triples of `level`."""
        n = self.level_dofs(level)
        ns = len(samples)
        arrs = [(_arr(x, "x", F64, n), _arr(g, "g", F64, n), _arr(s, "s", F64, n)) for x, g, s in samples]
        X = (ctypes.c_void_p * ns)(*[a[0].value for a in arrs])
        G = (ctypes.c_void_p * ns)(*[a[1].value for a in arrs])
        S = (ctypes.c_void_p * ns)(*[a[2].value for a in arrs])
        self._check(self._fn("rmtr_nn_fit_scales")(self.h, level, ns, X, G, S, _arr(scales, "scales", F32, 12),
                                                _stream()), "rmtr_nn_fit_scales")
        return scales

    def nn_propose(self, level, net, x, g, lo, hi, out=None):
        n = self.level_dofs(level)
        out = torch.empty_like(x) if out is None else out
        self._check(self._fn("rmtr_nn_propose")(self.h, level, ctypes.byref(net), _arr(x, "x", F64, n),
                                             _arr(g, "g", F64, n), _arr(lo, "lo", F64, n), _arr(hi, "hi", F64, n),
                                             _arr(out, "s", F64, n), _stream()), "rmtr_nn_propose")
        return out

    # -- load step
    def neumann_load(self, level, faces, traction, p):
        """External load of the Neumann terms on the listed faces (face =
        2 axis + side); traction: (2d, d) array of constant face tractions."""
        import numpy as np
        mask = 0
        for f in faces:
            mask |= 1 << int(f)
        tr = np.ascontiguousarray(traction, dtype=np.float64)
        if tr.shape != (2 * self.dim, self.dim):
            raise ValueError(f"traction: shape {tr.shape}, expected {(2 * self.dim, self.dim)}")
        b = torch.empty(self.level_dofs(level), dtype=torch.float64, device=p.device)
        self._check(self._fn("rmtr_neumann_load")(self.h, level, mask, tr.ctypes.data_as(ctypes.c_void_p),
                                                  _arr(p, "p", F64, self.level_nodes(level)), _ptr(b), _stream()),
                    "rmtr_neumann_load")
        return b

    def solve_loadstep(self, x, p, c_lower, params=None, dirichlet=None, history=False, f_ext=None):
        import numpy as np
        prm = params if params is not None else default_params()
        L = self.L
        px = _arr(x, "x", F64, self.level_dofs(L))
        pp = _arr(p, "p", F64, self.level_nodes(L))
        pc = _arr(c_lower, "c_lower", F64, self.level_nodes(L))
        pf = _arr(f_ext, "f_ext", F64, self.level_dofs(L), optional=True)
        st = Stats()
        hist = np.zeros(max(prm.max_vcycles, 1), dtype=np.float64)
        code = self._check(self._fn("rmtr_solve_loadstep")(self.h, pp, pc, self._dir(L, dirichlet), pf,
                                                        ctypes.byref(prm), px, ctypes.byref(st),
                                                        hist.ctypes.data_as(ctypes.c_void_p), _stream()),
                           "rmtr_solve_loadstep")
        out = {k: getattr(st, k) for k, _ in Stats._fields_}
        out["code"] = code
        if history:
            out["chi_history"] = hist[: st.vcycles].copy()
        return out

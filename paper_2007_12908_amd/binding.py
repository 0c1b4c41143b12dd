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
RMTR_FP64 = 0
RMTR_FP32 = 1
R_DUAL, R_INJECT, R_BOX_LO, R_BOX_HI = 0, 1, 2, 3

EXPORTS = [
    "rmtr_default_params", "rmtr_create", "rmtr_destroy", "rmtr_last_error", "rmtr_level_nodes",
    "rmtr_init_fields", "rmtr_energy", "rmtr_energy_diff", "rmtr_gradient", "rmtr_hessvec",
    "rmtr_diag_blocks", "rmtr_smooth", "rmtr_restrict", "rmtr_prolong", "rmtr_galerkin", "rmtr_coarse_hessvec",
    "rmtr_em_hessvec", "rmtr_em_smooth", "rmtr_mprgp", "rmtr_dot", "rmtr_chi", "rmtr_solve_loadstep",
    "rmtr_step_box", "rmtr_nn_size", "rmtr_nn_forward", "rmtr_nn_backward", "rmtr_nn_mse", "rmtr_nn_adam_step",
    "rmtr_nn_to_bf16", "rmtr_nn_features", "rmtr_nn_propose", "rmtr_element_flops",
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
                ("nn_patience", ctypes.c_int32), ("shrink_to_step", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("vcycles", ctypes.c_int32), ("tr_accepted", ctypes.c_int32),
                ("tr_rejected", ctypes.c_int32), ("status", ctypes.c_int32),
                ("chi0", ctypes.c_double), ("chi", ctypes.c_double), ("energy", ctypes.c_double),
                ("seconds", ctypes.c_double), ("nn_proposed", ctypes.c_int32),
                ("nn_accepted", ctypes.c_int32)]


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
            "rmtr_galerkin": (I32, [P, I32, P, P, P, P, P, P]),
            "rmtr_coarse_hessvec": (I32, [P, I32, P, P, P, P, P, I32, P]),
            "rmtr_em_hessvec": (I32, [P, I32, P, P, P, P]),
            "rmtr_em_smooth": (I32, [P, I32, P, P, P, P, P, I32, P]),
            "rmtr_mprgp": (I32, [P, I32, P, P, P, P, P, I32, D, I32, ctypes.POINTER(I32),
                                 ctypes.POINTER(I32), P]),
            "rmtr_dot": (I32, [P, I64, P, P, P, P]),
            "rmtr_chi": (I32, [P, I32, P, P, P, P, P, P]),
            "rmtr_solve_loadstep": (I32, [P, P, P, P, ctypes.POINTER(Params), P, ctypes.POINTER(Stats),
                                          P, P]),
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


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prec(t):
    return RMTR_FP32 if t.dtype == torch.float32 else RMTR_FP64


class Context:
    """One hierarchy (rmtr_create) and the calls of include/rmtr.h on it."""

    def __init__(self, dim, n_cells, n_levels, lam, mu, Gc, ls, k=1e-6, split=True):
        self.lib = load()
        self.model = Model(dim, n_cells, n_levels, 1 if split else 0, lam, mu, Gc, ls, k)
        h = ctypes.c_void_p()
        st = self.lib.rmtr_create(ctypes.byref(self.model), ctypes.byref(h))
        if st != RMTR_OK:
            raise ValueError(f"rmtr_create failed ({st})")
        self.h = h
        self.dim, self.L = dim, n_levels

    def close(self):
        if self.h:
            self.lib.rmtr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, name):
        if st < 0:
            msg = self.lib.rmtr_last_error(self.h)
            raise RuntimeError(f"{name} failed ({st}): {msg.decode() if msg else ''}")
        return st

    def level_nodes(self, level):
        return int(self.lib.rmtr_level_nodes(self.h, level))

    def level_cells(self, level):
        return self.model.n_cells >> (self.L - level)

    # -- fields
    def init_fields(self, level, table, band, p_mode=0, p_value=0.0, p_band=0.0):
        import numpy as np
        tab = np.ascontiguousarray(table, dtype=np.float64)
        n = self.level_nodes(level)
        c0 = torch.empty(n, dtype=torch.float64, device="cuda")
        p = torch.empty(n, dtype=torch.float64, device="cuda")
        self._check(self.lib.rmtr_init_fields(self.h, level, tab.ctypes.data_as(ctypes.c_void_p), tab.shape[0],
                                              band, p_mode, p_value, p_band, _ptr(c0), _ptr(p), _stream()),
                    "rmtr_init_fields")
        return c0, p

    # -- functional
    def energy(self, level, x, p, out=None):
        out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else out
        self._check(self.lib.rmtr_energy(self.h, level, _ptr(x), _ptr(p), _ptr(out), _stream()), "rmtr_energy")
        return out

    def energy_diff(self, level, x, s, p, out=None):
        out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else out
        self._check(self.lib.rmtr_energy_diff(self.h, level, _ptr(x), _ptr(s), _prec(s), _ptr(p), _ptr(out),
                                              _stream()), "rmtr_energy_diff")
        return out

    def gradient(self, level, x, p, dirichlet=None, out=None):
        out = torch.empty_like(x) if out is None else out
        self._check(self.lib.rmtr_gradient(self.h, level, _ptr(x), _ptr(p), _ptr(dirichlet), _ptr(out),
                                           _stream()), "rmtr_gradient")
        return out

    def hessvec(self, level, x_lin, p, v, dirichlet=None, out=None):
        out = torch.empty_like(v) if out is None else out
        self._check(self.lib.rmtr_hessvec(self.h, level, _ptr(x_lin), _ptr(p), _ptr(dirichlet), _ptr(v),
                                          _ptr(out), _prec(v), _stream()), "rmtr_hessvec")
        return out

    def diag_blocks(self, level, x_lin, p, dirichlet=None):
        nc = self.dim + 1
        D = torch.empty(self.level_nodes(level) * nc * nc, dtype=x_lin.dtype, device=x_lin.device)
        self._check(self.lib.rmtr_diag_blocks(self.h, level, _ptr(x_lin), _ptr(p), _ptr(dirichlet), _ptr(D),
                                              _prec(x_lin), _stream()), "rmtr_diag_blocks")
        return D

    def smooth(self, level, x_lin, p, g, lo, hi, s, n_sweeps, dirichlet=None):
        """Symmetric PGS; x_lin and p are FP64, g/lo/hi/s FP64 or FP32."""
        self._check(self.lib.rmtr_smooth(self.h, level, _ptr(x_lin), _ptr(p), _ptr(dirichlet), _ptr(g),
                                         _ptr(lo), _ptr(hi), _ptr(s), n_sweeps, _prec(s), _stream()),
                    "rmtr_smooth")
        return s

    # -- transfers
    def restrict(self, fine_level, fine, mode=R_DUAL):
        nc = self.dim + 1
        out = torch.empty(self.level_nodes(fine_level - 1) * nc, dtype=fine.dtype, device=fine.device)
        self._check(self.lib.rmtr_restrict(self.h, fine_level, mode, _ptr(fine), _ptr(out), _prec(fine),
                                           _stream()), "rmtr_restrict")
        return out

    def prolong(self, coarse_level, coarse):
        nc = self.dim + 1
        out = torch.empty(self.level_nodes(coarse_level + 1) * nc, dtype=coarse.dtype, device=coarse.device)
        self._check(self.lib.rmtr_prolong(self.h, coarse_level, _ptr(coarse), _ptr(out), _prec(coarse),
                                          _stream()), "rmtr_prolong")
        return out

    # -- Galerkin element matrices
    def galerkin(self, coarse_level, x_lin=None, p=None, dirichlet=None, K_fine=None):
        nd = (1 << self.dim) * (self.dim + 1)
        ne = self.level_cells(coarse_level) ** self.dim
        K = torch.empty(ne * nd * nd, dtype=torch.float64, device="cuda")
        self._check(self.lib.rmtr_galerkin(self.h, coarse_level, _ptr(x_lin), _ptr(p), _ptr(dirichlet),
                                           _ptr(K_fine), _ptr(K), _stream()), "rmtr_galerkin")
        return K

    def coarse_hessvec(self, level, x_lin, p, v, dirichlet=None, fp32_stencil=False):
        """Galerkin coarse Hessian of `level` (built from the finest stencil at
        x_lin, FP64 or FP32 storage) applied to the FP64 vector v."""
        out = torch.empty_like(v)
        self._check(self.lib.rmtr_coarse_hessvec(self.h, level, _ptr(x_lin), _ptr(p), _ptr(dirichlet), _ptr(v),
                                                 _ptr(out), RMTR_FP32 if fp32_stencil else RMTR_FP64, _stream()),
                    "rmtr_coarse_hessvec")
        return out

    def em_hessvec(self, level, K, v):
        out = torch.empty_like(v)
        self._check(self.lib.rmtr_em_hessvec(self.h, level, _ptr(K), _ptr(v), _ptr(out), _stream()),
                    "rmtr_em_hessvec")
        return out

    def em_smooth(self, level, K, g, lo, hi, s, n_sweeps):
        self._check(self.lib.rmtr_em_smooth(self.h, level, _ptr(K), _ptr(g), _ptr(lo), _ptr(hi), _ptr(s), n_sweeps,
                                            _stream()), "rmtr_em_smooth")
        return s

    def mprgp(self, level, K, g, lo, hi, max_it=500, rtol=1e-10, fallback_sweeps=50):
        s = torch.empty_like(g)
        its, status = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.rmtr_mprgp(self.h, level, _ptr(K), _ptr(g), _ptr(lo), _ptr(hi), _ptr(s), max_it, rtol,
                                        fallback_sweeps, ctypes.byref(its), ctypes.byref(status), _stream()),
                    "rmtr_mprgp")
        return s, its.value, status.value

    # -- reductions
    def dot(self, a, b):
        out = torch.empty(1, dtype=torch.float64, device=a.device)
        self._check(self.lib.rmtr_dot(self.h, a.numel(), _ptr(a), _ptr(b), _ptr(out), _stream()), "rmtr_dot")
        return out

    def chi(self, level, x, g, c_lower, dirichlet=None):
        out = torch.empty(1, dtype=torch.float64, device=x.device)
        self._check(self.lib.rmtr_chi(self.h, level, _ptr(x), _ptr(g), _ptr(c_lower), _ptr(dirichlet), _ptr(out),
                                      _stream()), "rmtr_chi")
        return out

    def step_box(self, level, x, c_lower, delta, dirichlet=None):
        lo, hi = torch.empty_like(x), torch.empty_like(x)
        self._check(self.lib.rmtr_step_box(self.h, level, _ptr(x), _ptr(c_lower), delta, _ptr(dirichlet), _ptr(lo),
                                           _ptr(hi), _stream()), "rmtr_step_box")
        return lo, hi

    # -- learned proposal network
    def nn_size(self, what, nx, ny, nz):
        return int(self.lib.rmtr_nn_size(what, nx, ny, nz))

    def nn_forward(self, w, bias, act, box):
        nx, ny, nz = box
        self._check(self.lib.rmtr_nn_forward(self.h, _ptr(w), _ptr(bias), _ptr(act), nx, ny, nz, _stream()),
                    "rmtr_nn_forward")
        return act

    def nn_backward(self, w, act, dout, grad, work, box):
        nx, ny, nz = box
        self._check(self.lib.rmtr_nn_backward(self.h, _ptr(w), _ptr(act), _ptr(dout), _ptr(grad), _ptr(work), nx,
                                              ny, nz, _stream()), "rmtr_nn_backward")
        return grad

    def nn_mse(self, out, target, window, dout, loss, box):
        nx, ny, nz = box
        win = (ctypes.c_int32 * 6)(*[int(v) for v in window])
        self._check(self.lib.rmtr_nn_mse(self.h, _ptr(out), _ptr(target), win, _ptr(dout), _ptr(loss), nx, ny, nz,
                                         _stream()), "rmtr_nn_mse")
        return loss

    def nn_adam_step(self, lr, t, grad, master, m, v, w_bf16=None, n_bf16=0):
        self._check(self.lib.rmtr_nn_adam_step(self.h, master.numel(), n_bf16, lr, t, _ptr(grad), _ptr(master),
                                               _ptr(m), _ptr(v), _ptr(w_bf16), _stream()), "rmtr_nn_adam_step")

    def nn_to_bf16(self, master, w_bf16):
        self._check(self.lib.rmtr_nn_to_bf16(self.h, w_bf16.numel(), _ptr(master), _ptr(w_bf16), _stream()),
                    "rmtr_nn_to_bf16")
        return w_bf16

    def nn_features(self, level, x, g, scales, out=None):
        out = torch.empty(self.level_nodes(level) * 8, dtype=torch.float32, device=x.device) if out is None else out
        self._check(self.lib.rmtr_nn_features(self.h, level, _ptr(x), _ptr(g), _ptr(scales), _ptr(out), _stream()),
                    "rmtr_nn_features")
        return out

    def nn_propose(self, level, net, x, g, lo, hi, out=None):
        out = torch.empty_like(x) if out is None else out
        self._check(self.lib.rmtr_nn_propose(self.h, level, ctypes.byref(net), _ptr(x), _ptr(g), _ptr(lo), _ptr(hi),
                                             _ptr(out), _stream()), "rmtr_nn_propose")
        return out

    # -- load step
    def solve_loadstep(self, x, p, c_lower, params=None, dirichlet=None, history=False):
        import numpy as np
        prm = params if params is not None else default_params()
        st = Stats()
        hist = np.zeros(max(prm.max_vcycles, 1), dtype=np.float64)
        code = self._check(self.lib.rmtr_solve_loadstep(self.h, _ptr(p), _ptr(c_lower), _ptr(dirichlet),
                                                        ctypes.byref(prm), _ptr(x), ctypes.byref(st),
                                                        hist.ctypes.data_as(ctypes.c_void_p), _stream()),
                           "rmtr_solve_loadstep")
        out = {k: getattr(st, k) for k, _ in Stats._fields_}
        out["code"] = code
        if history:
            out["chi_history"] = hist[: st.vcycles].copy()
        return out

// C-ABI of librmtr and the host-side RMTR driver.
//
// The driver follows the paper's Algorithms 1-3 (V-cycle, Nonlinear_solve,
// Convergence_control) with the Hessian lagging of Sec. 4.2.1: one Hessian
// per level and V-cycle, taken at the level's initial iterate (matrix-free on
// the finest level, Galerkin element matrices below), reused for the
// pre-smoothing, the coarse Galerkin product and the post-smoothing.  Every
// vector operation runs in the HIP kernels; the host only makes the scalar
// trust-region decisions, reading the few device scalars each needs.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rmtr.h"
#include "rmtr_kernels.h"

using namespace rmtr;

namespace {

struct Level {
  int N = 0;
  int64_t nodes = 0, n = 0, nelem = 0;
  double h = 0;
  // device buffers, allocated on first use
  double *x0 = nullptr, *xs = nullptr, *Lb = nullptr, *Ub = nullptr, *dg = nullptr, *g = nullptr;
  double *lo = nullptr, *hi = nullptr, *s = nullptr, *sc = nullptr, *hs = nullptr;
  double *t1 = nullptr, *t2 = nullptr, *t3 = nullptr, *t4 = nullptr;
  double *p = nullptr, *K = nullptr, *D = nullptr;
  float *xlf = nullptr, *pf = nullptr, *Df = nullptr, *gf = nullptr, *lof = nullptr, *hif = nullptr, *sf = nullptr;
  double* S = nullptr;      // lagged Hessian as a block stencil (FP64)
  float* Sf = nullptr;      // the same in FP32 (finest level, mixed precision)
  double* coef = nullptr;   // per-element second-variation coefficients (finest level)
  size_t coef_cap = 0;      // doubles held by coef (FP32 coefficients take half)
  double* Sop = nullptr;    // stencil scratch of rmtr_smooth / rmtr_coarse_hessvec
  float* Sopf = nullptr;
  double* coefop = nullptr;
  // prolongation / restriction chains of the coarse model f~ = f o I
  double *ca = nullptr, *cb = nullptr, *cc = nullptr;
  // Dirichlet bits of a coarse level when the finest level has its own
  // set (injected from the level above)
  uint8_t* mask = nullptr;
  bool solver_ready = false;
};

}  // namespace

struct rmtr_ctx {
  rmtr_model model{};
  MatP<double> mat{};
  int L = 0;
  std::vector<Level> lv;  // index 1..L
  double* partials = nullptr;
  double* ring = nullptr;  // ring partials of the 3D element kernels (finest level's size)
  double* scal = nullptr;  // device scalars
  int* flag = nullptr;     // device int flag
  double* hs = nullptr;    // pinned host scalars
  int* hflag = nullptr;    // pinned host flag
  double* table = nullptr;
  size_t table_cap = 0;
  double* mprgp_work = nullptr;
  double* box_tmp = nullptr;    // bounds scratch of rmtr_step_box
  size_t box_cap = 0;
  float* nn_buf = nullptr;      // inference tensors of the proposal network
  size_t nn_cap = 0;
  double* rap_work = nullptr;   // intermediate stencils of the Galerkin coarsening
  size_t rap_cap = 0;
  double* op_st = nullptr;      // stencil scratch of rmtr_mprgp
  size_t op_cap = 0;
  double* op_work = nullptr;    // iteration vectors of rmtr_mprgp
  size_t op_work_cap = 0;
  double* fit_buf = nullptr;    // per-sample RMS values of rmtr_nn_fit_scales
  size_t fit_cap = 0;
  std::vector<void*> allocs;
  // caller-bound workspace (rmtr_bind_workspace): every device buffer is
  // carved from it in order and nothing is allocated
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_used = 0;
  std::string err;
};

namespace {

constexpr int kScal = 64;

rmtr_status fail(rmtr_ctx* c, rmtr_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

// A shortfall of a bound workspace surfaces as hipErrorOutOfMemory from
// dalloc and is reported as RMTR_E_WORKSPACE.
#define HIPCHK(ctx, expr)                                                                        \
  do {                                                                                           \
    hipError_t e__ = (expr);                                                                     \
    if (e__ != hipSuccess) {                                                                     \
      if (e__ == hipErrorOutOfMemory && (ctx)->ws)                                               \
        return fail(ctx, RMTR_E_WORKSPACE, std::string(#expr) + ": bound workspace too small");  \
      return fail(ctx, RMTR_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e__));         \
    }                                                                                            \
  } while (0)

// Bytes one buffer of `bytes` takes: 256 bytes of slack past the end (vector
// loads of a last partial chunk stay inside the allocation), rounded up to
// the 256-byte alignment every buffer starts at.
size_t buf_bytes(size_t bytes) { return (bytes + 256 + 255) & ~size_t(255); }

template <typename T>
hipError_t dalloc(rmtr_ctx* c, T** p, size_t count) {
  const size_t bytes = buf_bytes(count * sizeof(T));
  if (c->ws) {
    if (c->ws_used + bytes > c->ws_bytes) return hipErrorOutOfMemory;
    *p = reinterpret_cast<T*>(c->ws + c->ws_used);
    c->ws_used += bytes;
    return hipSuccess;
  }
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return e;
  c->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return hipSuccess;
}

bool valid_level(const rmtr_ctx* c, int l) { return c && l >= 1 && l <= c->L; }

ElemArgs eargs(const rmtr_ctx* c, int l, const uint8_t* dir) {
  ElemArgs a;
  a.dim = c->model.dim;
  a.N = c->lv[l].N;
  a.h = c->lv[l].h;
  a.m = c->mat;
  a.dir = dir;
  a.ring = c->ring;
  return a;
}

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

// 3D levels run the FP64 gradient and Hv on non-overlapping tiles, except
// with the spectral split
bool uses_ring(const rmtr_ctx* c) { return c->model.dim == 3 && c->mat.split != kSplitSpectral; }

rmtr_status ensure_common(rmtr_ctx* c) {
  if (c->partials) return RMTR_OK;
  HIPCHK(c, dalloc(c, &c->partials, kMaxPartials));
  if (uses_ring(c)) HIPCHK(c, dalloc(c, &c->ring, ring_values(c->lv[c->L].N)));
  HIPCHK(c, dalloc(c, &c->scal, kScal));
  HIPCHK(c, dalloc(c, &c->flag, 4));
  void* h = nullptr;
  // coherent: MPRGP's final reductions are written into it by a kernel
  HIPCHK(c, hipHostMalloc(&h, kScal * sizeof(double) + 64, hipHostMallocCoherent));
  c->hs = static_cast<double*>(h);
  c->hflag = reinterpret_cast<int*>(c->hs + kScal);
  return RMTR_OK;
}

int ndof_elem(int dim) { return (1 << dim) * (dim + 1); }

rmtr_status ensure_solver_level(rmtr_ctx* c, int l, bool mixed, bool fine_model) {
  Level& v = c->lv[l];
  if (fine_model && l >= 2 && !v.ca) {
    HIPCHK(c, dalloc(c, &v.ca, size_t(v.n)));
    HIPCHK(c, dalloc(c, &v.cb, size_t(v.n)));
    if (l == c->L) HIPCHK(c, dalloc(c, &v.cc, size_t(v.n)));
  }
  if (!v.solver_ready) {
    const size_t n = size_t(v.n);
    double** vecs[] = {&v.x0, &v.xs, &v.Lb, &v.Ub, &v.dg, &v.g, &v.lo, &v.hi, &v.s, &v.sc, &v.hs,
                       &v.t1, &v.t2, &v.t3, &v.t4};
    for (double** b : vecs) HIPCHK(c, dalloc(c, b, n));
    HIPCHK(c, dalloc(c, &v.p, size_t(v.nodes)));
    if (l < c->L) HIPCHK(c, dalloc(c, &v.mask, size_t(v.nodes)));
    v.solver_ready = true;
  }
  // stencil of the lagged Hessian: FP32 on the finest level in mixed mode
  const bool want_f32 = mixed && l == c->L && c->L > 1;
  if (want_f32 && !v.Sf) HIPCHK(c, dalloc(c, &v.Sf, stencil_values(c->model.dim, v.N)));
  if (!want_f32 && !v.S) HIPCHK(c, dalloc(c, &v.S, stencil_values(c->model.dim, v.N)));
  if (mixed && l == c->L && !v.xlf) {
    const size_t n = size_t(v.n);
    float** fv[] = {&v.xlf, &v.gf, &v.lof, &v.hif, &v.sf};
    for (float** b : fv) HIPCHK(c, dalloc(c, b, n));
    HIPCHK(c, dalloc(c, &v.pf, size_t(v.nodes)));
  }
  return RMTR_OK;
}

// Device bytes of the buffers above: the common scalars and reduction
// partials, and (with a load step) everything rmtr_solve_loadstep allocates
// for its hierarchy, in the same sizes and rounding as dalloc.
size_t common_bytes(const rmtr_ctx* c) {
  return buf_bytes(kMaxPartials * sizeof(double)) +
         (uses_ring(c) ? buf_bytes(ring_values(c->lv[c->L].N) * sizeof(double)) : 0) +
         buf_bytes(kScal * sizeof(double)) + buf_bytes(4 * sizeof(int));
}

size_t loadstep_bytes(const rmtr_ctx* c, bool mixed, bool learned, bool fine_model) {
  const int d = c->model.dim, L = c->L;
  size_t b = common_bytes(c);
  for (int l = 1; l <= L; ++l) {
    const Level& v = c->lv[l];
    if (fine_model && l >= 2) b += (l == L ? 3 : 2) * buf_bytes(size_t(v.n) * sizeof(double));
    b += 15 * buf_bytes(size_t(v.n) * sizeof(double)) + buf_bytes(size_t(v.nodes) * sizeof(double));
    if (l < L) b += buf_bytes(size_t(v.nodes));
    const bool f32 = mixed && l == L && L > 1;
    b += buf_bytes(stencil_values(d, v.N) * (f32 ? sizeof(float) : sizeof(double)));
    if (mixed && l == L) b += 5 * buf_bytes(size_t(v.n) * sizeof(float)) + buf_bytes(size_t(v.nodes) * sizeof(float));
  }
  b += buf_bytes(mprgp_work_doubles(d, c->lv[1].N) * sizeof(double));
  const bool fine32 = mixed && L > 1;
  if (L > 1) b += buf_bytes(st_rap_work_doubles(d, c->lv[L].N, fine32 ? 1 : 0) * sizeof(double));
  const size_t cv = coef_values(d, c->lv[L].N, c->mat.split);
  b += buf_bytes((fine32 ? (cv + 1) / 2 : cv) * sizeof(double));
  if (learned) b += buf_bytes(size_t(c->lv[L].nodes) * (8 + 32 + 32 + 4) * sizeof(float));
  return b;
}

// grows a context-owned buffer, freeing the previous one
template <typename T>
hipError_t grow(rmtr_ctx* c, T** buf, size_t* cap, size_t count) {
  if (*cap >= count) return hipSuccess;
  if (*buf) {
    // a buffer carved from a bound workspace stays where it is (its space is
    // not reused); an allocated one is freed
    if (!c->ws) {
      for (auto& a : c->allocs)
        if (a == *buf) a = nullptr;
      hipError_t e = hipFree(*buf);
      if (e != hipSuccess) return e;
    }
    *buf = nullptr;
    *cap = 0;
  }
  hipError_t e = dalloc(c, buf, count);
  if (e == hipSuccess) *cap = count;
  return e;
}

// learned proposal on a 3D level: features, ping-pong forward pass, output
// scaled and projected onto [lo, hi]
rmtr_status nn_propose(rmtr_ctx* c, int l, const rmtr_nn& net, const double* x, const double* g, const double* lo,
                       const double* hi, double* s, hipStream_t st) {
  Level& v = c->lv[l];
  const int64_t nvox = v.nodes;
  HIPCHK(c, grow(c, &c->nn_buf, &c->nn_cap, size_t(nvox) * (8 + 32 + 32 + 4)));
  float* in = c->nn_buf;
  float* A = in + nvox * 8;
  float* B = A + nvox * 32;
  float* out = B + nvox * 32;
  float* const layer[7] = {in, A, B, A, B, A, out};
  double* rms = c->scal + 40;
  HIPCHK(c, nn_grad_rms(nvox, g, c->partials, rms, st));
  HIPCHK(c, nn_features(nvox, x, g, net.scales, rms, in, st));
  HIPCHK(c, nn_forward(net.w, net.bias, layer, v.N + 1, v.N + 1, v.N + 1, st));
  HIPCHK(c, nn_proposal(v.n, out, net.scales, rms, lo, hi, s, st));
  return RMTR_OK;
}

// ------------------------------------------------------------ the solver
struct Run {
  rmtr_ctx* c;
  rmtr_params prm;
  hipStream_t st;
  const uint8_t* fdir;
  const double* fext;      // external load of the finest level (may be null)
  bool mixed;
  bool energy_model;       // coarse levels carry f~ (coarse_model 0 or 2)
  bool fine_model;         // f~^l = f o I_{l->L} (coarse_model 2)
  bool first_order;        // coarse models without dH
  double f_ref = 1.0;
  int accepted = 0, rejected = 0;
  int nn_proposed = 0, nn_accepted = 0, nn_misses = 0;
  rmtr_status status = RMTR_OK;
  bool trace = false;  // per-step log on stderr (RMTR_VERBOSE=2)

  // Dirichlet bits of level l: the caller's on the finest level and, when
  // it gave one, their injection on the coarse levels; else the default set
  const uint8_t* dir(int l) const { return l == c->L ? fdir : (fdir ? c->lv[l].mask : nullptr); }
  int dim() const { return c->model.dim; }

  rmtr_status fetch(int k, bool with_flag) {
    HIPCHK(c, hipMemcpyAsync(c->hs, c->scal, k * sizeof(double), hipMemcpyDeviceToHost, st));
    if (with_flag) HIPCHK(c, hipMemcpyAsync(c->hflag, c->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return RMTR_OK;
  }

  bool ftilde(int l) const { return l == c->L || energy_model; }

  // ---- the finest functional f(x) - f_ext . x
  // out = grad of the finest functional at x (Dirichlet rows zero)
  rmtr_status fine_grad(const double* x, double* out) {
    Level& f = c->lv[c->L];
    HIPCHK(c, launch_gradient(eargs(c, c->L, fdir), x, f.p, out, st));
    if (fext) {
      HIPCHK(c, launch_add_scaled(f.n, out, 1.0, fext, -1.0, nullptr, out, st));
      HIPCHK(c, launch_zero_masked(dim(), f.N, out, fdir, st));
    }
    return RMTR_OK;
  }
  // out (device scalar) = f(x + s) - f(x) on the finest level; tmp: one
  // more device scalar
  rmtr_status fine_diff(const double* x, const double* s, double* out, double* tmp) {
    Level& f = c->lv[c->L];
    HIPCHK(c, launch_energy(eargs(c, c->L, fdir), x, s, 0, f.p, c->partials, out, st));
    if (fext) {
      HIPCHK(c, launch_dot(f.n, fext, s, c->partials, tmp, st));
      HIPCHK(c, launch_add_scaled(1, out, 1.0, tmp, -1.0, nullptr, out, st));
    }
    return RMTR_OK;
  }

  // ---- the coarse functional f~^l of a level l < L
  // x of level l prolongated to the finest level, through the chain buf
  rmtr_status to_finest(int l, const double* x, double* Level::*buf) {
    const double* src = x;
    for (int k = l; k < c->L; ++k) {
      double* dst = c->lv[k + 1].*buf;
      HIPCHK(c, launch_prolong(dim(), c->lv[k].N, src, dst, 0, st));
      src = dst;
    }
    return RMTR_OK;
  }
  // a finest-level vector restricted (R = I^T) to level l into out, through
  // the ca chain of the levels in between
  rmtr_status from_finest(int l, const double* fine, double* out) {
    const double* src = fine;
    for (int k = c->L - 1; k >= l; --k) {
      double* dst = k == l ? out : c->lv[k].ca;
      HIPCHK(c, launch_restrict(dim(), c->lv[k].N, RMTR_R_DUAL, src, dst, 0, st));
      src = dst;
    }
    return RMTR_OK;
  }
  // out = grad f~^l(x)
  rmtr_status ft_grad(int l, const double* x, double* out) {
    Level& v = c->lv[l];
    if (!fine_model) {
      HIPCHK(c, launch_gradient(eargs(c, l, dir(l)), x, v.p, out, st));
      return RMTR_OK;
    }
    Level& f = c->lv[c->L];
    rmtr_status r;
    if ((r = to_finest(l, x, &Level::ca)) != RMTR_OK) return r;
    if ((r = fine_grad(f.ca, f.cc)) != RMTR_OK) return r;
    if ((r = from_finest(l, f.cc, out)) != RMTR_OK) return r;
    HIPCHK(c, launch_zero_masked(dim(), v.N, out, dir(l), st));
    return RMTR_OK;
  }
  // out = grad^2 f~^l(x0^l) w
  rmtr_status ft_hv(int l, const double* w, double* out) {
    Level& v = c->lv[l];
    if (!fine_model) {
      HIPCHK(c, launch_hessvec(eargs(c, l, dir(l)), v.x0, v.p, w, out, 0, st));
      return RMTR_OK;
    }
    Level& f = c->lv[c->L];
    rmtr_status r;
    if ((r = to_finest(l, v.x0, &Level::ca)) != RMTR_OK) return r;
    if ((r = to_finest(l, w, &Level::cb)) != RMTR_OK) return r;
    HIPCHK(c, launch_hessvec(eargs(c, c->L, fdir), f.ca, f.p, f.cb, f.cc, 0, st));
    if ((r = from_finest(l, f.cc, out)) != RMTR_OK) return r;
    HIPCHK(c, launch_zero_masked(dim(), v.N, out, dir(l), st));
    return RMTR_OK;
  }
  // f~^l(x + s) - f~^l(x) into the device scalar out
  rmtr_status ft_diff(int l, const double* x, const double* s, double* out) {
    Level& v = c->lv[l];
    if (l == c->L) return fine_diff(x, s, out, c->scal + 63);
    if (!fine_model) {
      HIPCHK(c, launch_energy(eargs(c, l, dir(l)), x, s, 0, v.p, c->partials, out, st));
      return RMTR_OK;
    }
    Level& f = c->lv[c->L];
    rmtr_status r;
    if ((r = to_finest(l, x, &Level::ca)) != RMTR_OK) return r;
    if ((r = to_finest(l, s, &Level::cb)) != RMTR_OK) return r;
    return fine_diff(f.ca, f.cb, out, c->scal + 63);
  }

  // out = grad h^l(x)
  rmtr_status h_grad(int l, const double* x, double* out) {
    Level& v = c->lv[l];
    if (l == c->L) return fine_grad(x, out);
    rmtr_status r;
    if (first_order) {
      // h = f~ + <dg, x - x0>: its Hessian is the lagged grad^2 f~ itself
      if ((r = ft_grad(l, x, v.t3)) != RMTR_OK) return r;
      HIPCHK(c, launch_add_scaled(v.n, v.dg, 1.0, v.t3, 1.0, nullptr, out, st));
      HIPCHK(c, launch_zero_masked(dim(), v.N, out, dir(l), st));
      return RMTR_OK;
    }
    HIPCHK(c, launch_add_scaled(v.n, x, 1.0, v.x0, -1.0, nullptr, v.t1, st));
    HIPCHK(c, launch_st_matvec(dim(), v.N, v.S, v.t1, v.t2, 0, st));
    HIPCHK(c, launch_add_scaled(v.n, v.dg, 1.0, v.t2, 1.0, nullptr, out, st));
    if (energy_model) {
      if ((r = ft_grad(l, x, v.t3)) != RMTR_OK) return r;
      if ((r = ft_hv(l, v.t1, v.t4)) != RMTR_OK) return r;
      HIPCHK(c, launch_add_scaled(v.n, v.t3, 1.0, v.t4, -1.0, out, out, st));
    }
    HIPCHK(c, launch_zero_masked(dim(), v.N, out, dir(l), st));
    return RMTR_OK;
  }

  // enqueue the pieces of h^l(x + s) - h^l(x) into scal[base .. base+3];
  // returns via combine_diff after a fetch.  Reuse of work already done:
  //   kind 1 (after h_grad(l, x) on this level): t1 = x - x0, t2 = S t1 and,
  //          with the energy model, t4 = H~ t1 are valid;
  //   kind 2: x is the level's x0 (t1 = 0);
  //   Ss (may be null): S s, already computed.
  rmtr_status h_diff_enqueue(int l, const double* x, const double* s, int base, int kind = 0,
                             const double* Ss = nullptr) {
    Level& v = c->lv[l];
    double* sc = c->scal + base;
    rmtr_status r;
    if (ftilde(l)) {
      if ((r = ft_diff(l, x, s, sc)) != RMTR_OK) return r;
    } else {
      HIPCHK(c, launch_fill(1, 0.0, sc, st));
    }
    if (l == c->L) return RMTR_OK;
    HIPCHK(c, launch_dot(v.n, v.dg, s, c->partials, sc + 1, st));
    if (first_order) {
      // no dH terms
      HIPCHK(c, launch_fill(2, 0.0, sc + 2, st));
      return RMTR_OK;
    }
    // t2 = (S - H~) (x - x0)
    if (kind == 2) {
      HIPCHK(c, launch_fill(1, 0.0, sc + 2, st));
    } else {
      if (kind == 0) {
        HIPCHK(c, launch_add_scaled(v.n, x, 1.0, v.x0, -1.0, nullptr, v.t1, st));
        HIPCHK(c, launch_st_matvec(dim(), v.N, v.S, v.t1, v.t2, 0, st));
        if (energy_model && (r = ft_hv(l, v.t1, v.t4)) != RMTR_OK) return r;
      }
      if (energy_model) HIPCHK(c, launch_add_scaled(v.n, v.t4, -1.0, nullptr, 0.0, v.t2, v.t2, st));
      HIPCHK(c, launch_dot(v.n, s, v.t2, c->partials, sc + 2, st));
    }
    // t3 = (S - H~) s
    const double* Sv = Ss;
    if (!Sv) {
      HIPCHK(c, launch_st_matvec(dim(), v.N, v.S, s, v.t3, 0, st));
      Sv = v.t3;
    }
    if (energy_model) {
      if ((r = ft_hv(l, s, v.t4)) != RMTR_OK) return r;
      HIPCHK(c, launch_add_scaled(v.n, v.t4, -1.0, nullptr, 0.0, Sv, v.t3, st));
      Sv = v.t3;
    }
    HIPCHK(c, launch_dot(v.n, s, Sv, c->partials, sc + 3, st));
    return RMTR_OK;
  }

  double h_diff_combine(int l, int base) const {
    const double* h = c->hs + base;
    if (l == c->L) return h[0];
    return h[0] + ((h[1] + h[2]) + 0.5 * h[3]);
  }

  // TR ratio with a round-off guard: below the resolution of a sum of
  // per-element energy differences, about eps |f| / sqrt(n_elements), a
  // step the model predicts to be a decrease is accepted unless it is
  // measurably uphill.
  double ratio(double ared, double pred, int l) const {
    const double tol = prm.guard * fabs(f_ref) / sqrt(double(c->lv[l].nelem));
    if (!isfinite(ared) || !isfinite(pred)) return -INFINITY;
    if (fabs(pred) <= tol) return ared >= -tol ? 1.0 : -INFINITY;
    if (pred <= 0.0) return -INFINITY;
    return ared / pred;
  }

  // Alg. 3; with shrink_to_step a rejected step's radius is measured from
  // the step taken, gamma1 min(delta, |s|_inf)
  bool control(double rho, double& delta, double snorm) const {
    const bool accept = rho > prm.eta1;
    if (rho < prm.eta1)
      delta = prm.gamma1 * (prm.shrink_to_step ? fmin(delta, snorm) : delta);
    else if (rho > prm.eta2)
      delta = fmin(prm.gamma2 * delta, prm.delta_max);
    return accept;
  }

  // QP of one TR step on level l into v.s
  rmtr_status solve_qp(int l, bool coarsest) {
    Level& v = c->lv[l];
    if (coarsest) {
      MprgpResult res;
      HIPCHK(c, run_mprgp(dim(), v.N, v.S, dir(l), v.g, v.lo, v.hi, v.s, prm.coarse_qp_its, prm.coarse_qp_rtol,
                          prm.fallback_sweeps, c->mprgp_work, c->hs + 48, &res, st));
      return RMTR_OK;
    }
    if (l == c->L && mixed) {
      // mixed precision: FP32 sweeps on the FP32 stencil, step clamped back
      // into the FP64 box
      HIPCHK(c, launch_convert(v.n, v.g, 0, v.gf, 1, st));
      HIPCHK(c, launch_convert(v.n, v.lo, 0, v.lof, 1, st));
      HIPCHK(c, launch_convert(v.n, v.hi, 0, v.hif, 1, st));
      HIPCHK(c, hipMemsetAsync(v.sf, 0, size_t(v.n) * sizeof(float), st));
      HIPCHK(c, launch_st_pgs(dim(), v.N, v.Sf, fdir, v.gf, v.lof, v.hif, v.sf, prm.pgs_sweeps, 1, st));
      HIPCHK(c, launch_convert(v.n, v.sf, 1, v.s, 0, st));
      HIPCHK(c, launch_clamp(v.n, v.lo, v.hi, v.s, st));
      return RMTR_OK;
    }
    HIPCHK(c, launch_fill(v.n, 0.0, v.s, st));
    HIPCHK(c, launch_st_pgs(dim(), v.N, v.S, dir(l), v.g, v.lo, v.hi, v.s, prm.pgs_sweeps, 0, st));
    return RMTR_OK;
  }

  // Algorithm 2 body: one TR iteration on level l
  rmtr_status tr_step(int l, double* x, double& delta, bool coarsest) {
    Level& v = c->lv[l];
    rmtr_status r;
    if ((r = h_grad(l, x, v.g)) != RMTR_OK) return r;
    HIPCHK(c, launch_step_box(dim(), v.N, x, v.Lb, v.Ub, delta, dir(l), v.lo, v.hi, st));
    if ((r = solve_qp(l, coarsest)) != RMTR_OK) return r;
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), st));
    HIPCHK(c, launch_any_nonzero(v.n, v.s, c->flag, st));
    // model Hessian times s: lagged matrix-free on the finest level (FP64)
    if (l == c->L && !(c->L == 1)) {
      HIPCHK(c, launch_hessvec(eargs(c, l, fdir), v.x0, v.p, v.s, v.hs, 0, st));
    } else {
      HIPCHK(c, launch_st_matvec(dim(), v.N, v.S, v.s, v.hs, 0, st));
    }
    HIPCHK(c, launch_dot(v.n, v.g, v.s, c->partials, c->scal + 4, st));
    HIPCHK(c, launch_dot(v.n, v.s, v.hs, c->partials, c->scal + 5, st));
    if (prm.shrink_to_step) HIPCHK(c, launch_amax(v.n, v.s, c->partials, c->scal + 6, st));
    // on levels below the finest h_grad left t1, t2 (t4) for this x and
    // v.hs = S s
    if ((r = h_diff_enqueue(l, x, v.s, 0, l < c->L ? 1 : 0, l < c->L ? v.hs : nullptr)) != RMTR_OK) return r;
    if ((r = fetch(7, true)) != RMTR_OK) return r;
    if (*c->hflag == 0) {
      if (trace) fprintf(stderr, "rmtr:   tr l=%d s=0\n", l);
      return RMTR_OK;
    }
    const double pred = -(c->hs[4] + 0.5 * c->hs[5]);
    const double ared = -h_diff_combine(l, 0);
    const double rho = ratio(ared, pred, l);
    const double d0 = delta;
    const bool acc = control(rho, delta, c->hs[6]);
    if (trace)
      fprintf(stderr, "rmtr:   tr l=%d pred %.3e ared %.3e rho %.3e delta %.2e %s\n", l, pred, ared, rho, d0,
              acc ? "acc" : "rej");
    if (acc) {
      ++accepted;
      HIPCHK(c, launch_axpy(v.n, 1.0, v.s, x, st));
    } else {
      ++rejected;
    }
    return RMTR_OK;
  }

  // learned proposal on the finest level, judged like a TR step on the
  // lagged model.  The box-projected proposal s is a direction: the step is
  // beta s with beta in (0, 1] the model minimiser along it (s must be a
  // descent direction).  It is a candidate if beta >= 1/2 (the proposal's
  // length is within a factor two of the best along it), the ratio test
  // accepts it and its predicted decrease is at least that of the Cauchy
  // step (d = P(-t g) with t = g^T g / g^T H g, projected onto the step box,
  // then the exact model minimiser alpha d, alpha in [0, 1]).  A candidate
  // replaces the smoother step only if it lowers the energy at least as much
  // as the smoother step from the same state does (or that step would be
  // rejected); the smoother step is computed for the comparison and then
  // discarded.  A rejection leaves x and delta unchanged.
  rmtr_status nn_step(double* x, double delta, bool& taken) {
    taken = false;
    const int L = c->L;
    Level& v = c->lv[L];
    rmtr_status r;
    if ((r = h_grad(L, x, v.g)) != RMTR_OK) return r;
    HIPCHK(c, launch_step_box(dim(), v.N, x, v.Lb, v.Ub, delta, fdir, v.lo, v.hi, st));
    // Cauchy step s_c = P(-t g), t = g^T g / g^T H g (or the box edge)
    HIPCHK(c, launch_hessvec(eargs(c, L, fdir), v.x0, v.p, v.g, v.t1, 0, st));
    HIPCHK(c, launch_dot(v.n, v.g, v.g, c->partials, c->scal + 6, st));
    HIPCHK(c, launch_dot(v.n, v.g, v.t1, c->partials, c->scal + 7, st));
    if ((r = fetch(8, false)) != RMTR_OK) return r;
    const double gg = c->hs[6], gHg = c->hs[7];
    if (!(gg > 0.0) || !isfinite(gg) || !isfinite(gHg)) return RMTR_OK;
    const double t = gHg > 0.0 ? gg / gHg : 1e300;
    HIPCHK(c, launch_add_scaled(v.n, v.g, -t, nullptr, 0.0, nullptr, v.t2, st));
    HIPCHK(c, launch_clamp(v.n, v.lo, v.hi, v.t2, st));
    HIPCHK(c, launch_hessvec(eargs(c, L, fdir), v.x0, v.p, v.t2, v.t3, 0, st));
    HIPCHK(c, launch_dot(v.n, v.g, v.t2, c->partials, c->scal + 6, st));
    HIPCHK(c, launch_dot(v.n, v.t2, v.t3, c->partials, c->scal + 7, st));
    // the proposal
    if ((r = nn_propose(c, L, *prm.nn, x, v.g, v.lo, v.hi, v.s, st)) != RMTR_OK) return r;
    ++nn_proposed;
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), st));
    HIPCHK(c, launch_any_nonzero(v.n, v.s, c->flag, st));
    HIPCHK(c, launch_hessvec(eargs(c, L, fdir), v.x0, v.p, v.s, v.hs, 0, st));
    HIPCHK(c, launch_dot(v.n, v.g, v.s, c->partials, c->scal + 4, st));
    HIPCHK(c, launch_dot(v.n, v.s, v.hs, c->partials, c->scal + 5, st));
    if ((r = fetch(8, true)) != RMTR_OK) return r;
    if (*c->hflag == 0) return RMTR_OK;
    // the proposal is used as a direction: the model minimiser along it
    // within the box (beta in (0, 1]); no descent direction, no step
    const double gs = c->hs[4], sHs = c->hs[5];
    const double gd = c->hs[6], dHd = c->hs[7];
    if (!(gs < 0.0) || !isfinite(sHs)) {
      if (trace) fprintf(stderr, "rmtr:   nn l=%d not a descent direction\n", L);
      return RMTR_OK;
    }
    double beta = 1.0;
    if (sHs > 0.0 && -gs < sHs) beta = -gs / sHs;
    if (beta < 1.0) HIPCHK(c, launch_add_scaled(v.n, v.s, beta, nullptr, 0.0, nullptr, v.s, st));
    const double pred = -(beta * gs + 0.5 * beta * beta * sHs);
    if ((r = h_diff_enqueue(L, x, v.s, 0)) != RMTR_OK) return r;
    if ((r = fetch(1, false)) != RMTR_OK) return r;
    // Cauchy reference: exact model minimiser along the projected direction
    // d = s_c, within the box (alpha in [0, 1] keeps alpha d feasible)
    double alpha = 1.0;
    if (dHd > 0.0 && -gd < dHd) alpha = -gd / dHd;
    const double pred_c = -(alpha * gd + 0.5 * alpha * alpha * dHd);
    const double ared = -h_diff_combine(L, 0);
    const double rho = ratio(ared, pred, L);
    taken = rho > prm.eta1 && pred >= pred_c && beta >= 0.5;
    double ared_s = 0.0, rho_s = 0.0;
    bool smoother_ok = false;
    if (taken) {
      // the smoother step from the same state (as the TR step would compute
      // it), its energy decrease and ratio; the proposal waits in t2
      HIPCHK(c, hipMemcpyAsync(v.t2, v.s, size_t(v.n) * sizeof(double), hipMemcpyDeviceToDevice, st));
      if ((r = solve_qp(L, false)) != RMTR_OK) return r;
      HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), st));
      HIPCHK(c, launch_any_nonzero(v.n, v.s, c->flag, st));
      HIPCHK(c, launch_hessvec(eargs(c, L, fdir), v.x0, v.p, v.s, v.hs, 0, st));
      HIPCHK(c, launch_dot(v.n, v.g, v.s, c->partials, c->scal + 4, st));
      HIPCHK(c, launch_dot(v.n, v.s, v.hs, c->partials, c->scal + 5, st));
      if ((r = h_diff_enqueue(L, x, v.s, 0)) != RMTR_OK) return r;
      if ((r = fetch(6, true)) != RMTR_OK) return r;
      if (*c->hflag) {
        const double pred_s = -(c->hs[4] + 0.5 * c->hs[5]);
        ared_s = -h_diff_combine(L, 0);
        rho_s = ratio(ared_s, pred_s, L);
        smoother_ok = rho_s > prm.eta1;
      }
      taken = !smoother_ok || ared >= ared_s;
    }
    if (trace)
      fprintf(stderr, "rmtr:   nn l=%d beta %.3e pred %.3e cauchy %.3e ared %.3e rho %.3e smoother ared %.3e rho %.3e %s\n",
              L, beta, pred, pred_c, ared, rho, ared_s, rho_s, taken ? "acc" : "rej");
    if (taken) {
      ++nn_accepted;
      HIPCHK(c, launch_axpy(v.n, 1.0, v.t2, x, st));
    }
    return RMTR_OK;
  }

  rmtr_status nonlinear_solve(int l, double* x, double& delta, int its, bool coarsest) {
    for (int i = 0; i < its; ++i) {
      rmtr_status r = tr_step(l, x, delta, coarsest);
      if (r != RMTR_OK) return r;
    }
    return RMTR_OK;
  }

  rmtr_status setup_coarse(int l, const double* x, double delta) {
    Level& f = c->lv[l];
    Level& cc = c->lv[l - 1];
    const int d = dim();
    HIPCHK(c, launch_restrict(d, cc.N, RMTR_R_INJECT, x, cc.x0, 0, st));
    HIPCHK(c, launch_step_box(d, f.N, x, f.Lb, f.Ub, delta, dir(l), f.lo, f.hi, st));
    HIPCHK(c, launch_restrict(d, cc.N, RMTR_R_BOX_LO, f.lo, cc.lo, 0, st));
    HIPCHK(c, launch_restrict(d, cc.N, RMTR_R_BOX_HI, f.hi, cc.hi, 0, st));
    HIPCHK(c, launch_add_scaled(cc.n, cc.x0, 1.0, cc.lo, 1.0, nullptr, cc.Lb, st));
    HIPCHK(c, launch_add_scaled(cc.n, cc.x0, 1.0, cc.hi, 1.0, nullptr, cc.Ub, st));
    rmtr_status r = h_grad(l, x, f.g);
    if (r != RMTR_OK) return r;
    if (first_order) {
      // the coarse level's own Hessian at x0 (rediscretised, lagged); the
      // finest level's coefficient buffer is free once its stencil is built
      // and holds the coarse level's coefficients
      HIPCHK(c, launch_st_assemble(eargs(c, l - 1, dir(l - 1)), cc.x0, cc.p, c->lv[c->L].coef, cc.S, 0, st));
    } else {
      // lagged coarse Hessian R H I (default coarse Dirichlet set) from the
      // level's stencil
      const bool f32 = l == c->L && mixed;
      HIPCHK(c, launch_st_rap(d, f.N, f32 ? static_cast<const void*>(f.Sf) : static_cast<const void*>(f.S),
                              f32 ? 1 : 0, cc.S, dir(l - 1), c->rap_work, st));
    }
    HIPCHK(c, launch_restrict(d, cc.N, RMTR_R_DUAL, f.g, cc.dg, 0, st));
    if (energy_model) {
      if ((r = ft_grad(l - 1, cc.x0, cc.t3)) != RMTR_OK) return r;
      HIPCHK(c, launch_add_scaled(cc.n, cc.t3, -1.0, nullptr, 0.0, cc.dg, cc.dg, st));
    }
    HIPCHK(c, launch_zero_masked(d, cc.N, cc.dg, dir(l - 1), st));
    return RMTR_OK;
  }

  rmtr_status vcycle(int l, double* x, double& delta) {
    rmtr_status r;
    if (l == 1) return nonlinear_solve(1, x, delta, prm.coarse_tr_its, true);
    int pre = prm.mu1;
    if (l == c->L && prm.use_learned && pre > 0 && (prm.nn_patience <= 0 || nn_misses < prm.nn_patience)) {
      bool taken = false;
      if ((r = nn_step(x, delta, taken)) != RMTR_OK) return r;
      nn_misses = taken ? 0 : nn_misses + 1;
      if (taken) --pre;
    }
    if ((r = nonlinear_solve(l, x, delta, pre, false)) != RMTR_OK) return r;
    if ((r = setup_coarse(l, x, delta)) != RMTR_OK) return r;
    Level& f = c->lv[l];
    Level& cc = c->lv[l - 1];
    HIPCHK(c, hipMemcpyAsync(cc.xs, cc.x0, cc.n * sizeof(double), hipMemcpyDeviceToDevice, st));
    double dc = delta;
    if ((r = vcycle(l - 1, cc.xs, dc)) != RMTR_OK) return r;
    HIPCHK(c, launch_add_scaled(cc.n, cc.xs, 1.0, cc.x0, -1.0, nullptr, cc.sc, st));
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), st));
    HIPCHK(c, launch_any_nonzero(cc.n, cc.sc, c->flag, st));
    HIPCHK(c, launch_prolong(dim(), cc.N, cc.sc, f.s, 0, st));
    // setup_coarse's h_grad(l, x) left t1, t2 (t4) of level l for this x
    if ((r = h_diff_enqueue(l, x, f.s, 0, 1)) != RMTR_OK) return r;
    if ((r = h_diff_enqueue(l - 1, cc.x0, cc.sc, 8, 2)) != RMTR_OK) return r;
    if (prm.shrink_to_step) HIPCHK(c, launch_amax(f.n, f.s, c->partials, c->scal + 12, st));
    if ((r = fetch(13, true)) != RMTR_OK) return r;
    if (*c->hflag) {
      const double ared = -h_diff_combine(l, 0);
      const double pred = -h_diff_combine(l - 1, 8);
      const double rho = ratio(ared, pred, l);
      const double d0 = delta;
      const bool acc = control(rho, delta, c->hs[12]);
      if (trace)
        fprintf(stderr, "rmtr:   cc l=%d pred %.3e ared %.3e rho %.3e delta %.2e %s\n", l, pred, ared, rho, d0,
                acc ? "acc" : "rej");
      if (acc) HIPCHK(c, launch_axpy(f.n, 1.0, f.s, x, st));
    } else if (trace) {
      fprintf(stderr, "rmtr:   cc l=%d s=0\n", l);
    }
    return nonlinear_solve(l, x, delta, prm.mu2, false);
  }
};

// ------------------------------------------------ arithmetic of one element
// A scalar that counts the floating-point additions, subtractions,
// multiplications and divisions done on data; operations among constants
// (material parameters, h, literals) are folded by the compiler and are not
// counted.  Instantiating the element operators with it gives their exact
// algorithmic flop count per element.
struct Cnt {
  double v = 0.0;
  bool k = true;  // constant
  static int64_t ops;
  Cnt() = default;
  Cnt(double x) : v(x), k(true) {}
  static Cnt var(double x) {
    Cnt c(x);
    c.k = false;
    return c;
  }
  static Cnt bin(const Cnt& a, const Cnt& b, double r) {
    Cnt c(r);
    c.k = a.k && b.k;
    if (!c.k) ++ops;
    return c;
  }
  friend Cnt operator+(const Cnt& a, const Cnt& b) { return bin(a, b, a.v + b.v); }
  friend Cnt operator-(const Cnt& a, const Cnt& b) { return bin(a, b, a.v - b.v); }
  friend Cnt operator*(const Cnt& a, const Cnt& b) { return bin(a, b, a.v * b.v); }
  friend Cnt operator/(const Cnt& a, const Cnt& b) { return bin(a, b, a.v / b.v); }
  Cnt operator-() const {
    Cnt c = *this;
    c.v = -v;
    return c;
  }
  Cnt& operator+=(const Cnt& b) { return *this = *this + b; }
  Cnt& operator-=(const Cnt& b) { return *this = *this - b; }
  Cnt& operator*=(const Cnt& b) { return *this = *this * b; }
  friend bool operator>(const Cnt& a, const Cnt& b) { return a.v > b.v; }
  friend bool operator<(const Cnt& a, const Cnt& b) { return a.v < b.v; }
  friend bool operator==(const Cnt& a, const Cnt& b) { return a.v == b.v; }
  friend bool operator!=(const Cnt& a, const Cnt& b) { return a.v != b.v; }
  friend Cnt sqrt(const Cnt& a) { return bin(a, a, std::sqrt(a.v)); }
};
int64_t Cnt::ops = 0;

template <int DIM>
MatP<Cnt> cnt_mat() {
  MatP<Cnt> m;
  m.lam = 0.57;
  m.mu = 0.38;
  m.K = m.lam.v + 2.0 * m.mu.v / 3.0;
  m.Gc = 1e-3;
  m.ls = 0.1;
  m.k = 1e-6;
  m.split = 1;
  set_derived(m);
  return m;
}

template <int DIM>
int64_t count_kind(int kind) {
  constexpr int NL = 1 << DIM, NC = DIM + 1;
  const MatP<Cnt> m = cnt_mat<DIM>();
  const Cnt invh(20.0), w(1e-4);
  Cnt X[NL][NC], V[NL][NC], P[NL];
  for (int a = 0; a < NL; ++a) {
    P[a] = Cnt::var(1e-3 * (1 + a));
    for (int k = 0; k < NC; ++k) {
      X[a][k] = Cnt::var(k == DIM ? 0.1 * a : 1e-3 * (a + k));
      V[a][k] = Cnt::var(0.3 * (a - k));
    }
  }
  Cnt::ops = 0;
  if (kind == 4 || (DIM == 2 && (kind == 2 || kind == 3))) {
    // node-centric visit of one element for one node (PGS pass, 2D kernels)
    Cnt r[NC];
    node_contrib<DIM, Cnt>(kind == 2 ? 0 : 1, m, invh, w, X, V, P, 0, r);
    return Cnt::ops;
  }
  Cnt pq[NL], dpq[NL][DIM];
  elem_pq<DIM, Cnt>(P, invh, pq, dpq);
  Zq<DIM, Cnt> z[NL];
  if (kind == 0 || kind == 1) {
    elem_z<DIM, Cnt>(X, invh, z);
    Cnt e = 0.0;
    e.k = false;
    for (int q = 0; q < NL; ++q) e += density<DIM, Cnt>(m, z[q], pq[q], dpq[q]);
    if (kind == 1) {
      for (int a = 0; a < NL; ++a)
        for (int k = 0; k < NC; ++k) X[a][k] += V[a][k];
      elem_z<DIM, Cnt>(X, invh, z);
      Cnt e1 = 0.0;
      e1.k = false;
      for (int q = 0; q < NL; ++q) e1 += density<DIM, Cnt>(m, z[q], pq[q], dpq[q]);
      e = e1 - e;
    }
    e = w * e;
    return Cnt::ops;
  }
  if constexpr (DIM == 3) {
    Cnt r[8][4];
    if (kind == 2) ElemOp3<0, Cnt>::eval(m, invh, w, X, V, P, r);
    if (kind == 3) ElemOp3<1, Cnt>::eval(m, invh, w, X, V, P, r);
    return Cnt::ops;
  }
  return -1;
}

// The quarter-wise evaluation of the 3D FP64 kernels (energy, gradient, Hv;
// volumetric-deviatoric form), as k_energy_q3 / k_elem_q3 run it.
int64_t count_quarter(int kind) {
  const MatP<Cnt> m = cnt_mat<3>();
  const ElemScale<Cnt> sc = elem_scale<Cnt>(Cnt(20.0), Cnt(1e-4));
  const SymConst<Cnt> kc = sym_const<Cnt>(m, sc);
  const Cnt cdc = sc.a2 * m.Gc_l, a2Gcl2 = Cnt(0.5) * sc.a2 * m.Gc_l;
  Cnt X[8][4], V[8][4], P[8];
  for (int a = 0; a < 8; ++a) {
    P[a] = Cnt::var(1e-3 * (1 + a));
    for (int k = 0; k < 4; ++k) {
      X[a][k] = Cnt::var(k == 3 ? 0.1 * a : 1e-3 * (a + k));
      V[a][k] = Cnt::var(0.3 * (a - k));
    }
  }
  Cnt::ops = 0;
  Cnt e = 0.0;
  e.k = false;
  Cnt r[4][8];
  for (int qq = 0; qq < 4; ++qq) {
    const Cnt xy = gauss_xi<Cnt>(qq & 1), xz = gauss_xi<Cnt>(qq >> 1);
    QPoint<Cnt> zq[2];
    for (int k = 0; k < 5; ++k) {
      Cnt f[8];
      for (int a = 0; a < 8; ++a) f[a] = k < 4 ? X[a][k] : P[a];
      if (k == 3 && kind == 3) {
        Cnt val[2];
        qtr_forward_val<Cnt>(f, xz, xy, val);
        zq[0].c = val[0];
        zq[1].c = val[1];
        continue;
      }
      Cnt val[2], dx, dy[2], dz[2];
      qtr_forward<Cnt>(f, xz, xy, val, dx, dy, dz);
      for (int qx = 0; qx < 2; ++qx) {
        Cnt* d = k < 3 ? zq[qx].G[k] : k == 3 ? zq[qx].dc : zq[qx].dp;
        if (k < 3) zq[qx].u[k] = val[qx];
        if (k == 3) zq[qx].c = val[qx];
        if (k == 4) zq[qx].p = val[qx];
        d[0] = dx;
        d[1] = dy[qx];
        d[2] = dz[qx];
      }
    }
    if (kind == 0) {
      for (int qx = 0; qx < 2; ++qx) e += energy_point_sym<Cnt, true>(kc, a2Gcl2, zq[qx]);
      continue;
    }
    Zq<3, Cnt> o[2];
    if (kind == 2) {
      for (int qx = 0; qx < 2; ++qx) grad_point_sym<Cnt, true>(kc, cdc, zq[qx], o[qx]);
    } else {
      HessSym<Cnt> hc[2];
      for (int qx = 0; qx < 2; ++qx) hess_sym_coef<Cnt, true>(kc, zq[qx], hc[qx]);
      Zq<3, Cnt> zv[2];
      for (int k = 0; k < 4; ++k) {
        Cnt f[8];
        for (int a = 0; a < 8; ++a) f[a] = V[a][k];
        Cnt val[2], dx, dy[2], dz[2];
        qtr_forward<Cnt>(f, xz, xy, val, dx, dy, dz);
        for (int qx = 0; qx < 2; ++qx) {
          Cnt* d = k < 3 ? zv[qx].G[k] : zv[qx].dc;
          if (k < 3) zv[qx].u[k] = val[qx]; else zv[qx].c = val[qx];
          d[0] = dx;
          d[1] = dy[qx];
          d[2] = dz[qx];
        }
      }
      for (int qx = 0; qx < 2; ++qx) hess_sym_apply<Cnt>(hc[qx], cdc, zv[qx], o[qx]);
    }
    for (int k = 0; k < 4; ++k) {
      Cnt cv[2], cx[2], cy[2], cz[2];
      for (int qx = 0; qx < 2; ++qx) {
        cv[qx] = k < 3 ? o[qx].u[k] : o[qx].c;
        cx[qx] = k < 3 ? o[qx].G[k][0] : o[qx].dc[0];
        cy[qx] = k < 3 ? o[qx].G[k][1] : o[qx].dc[1];
        cz[qx] = k < 3 ? o[qx].G[k][2] : o[qx].dc[2];
      }
      if (qq == 0)
        for (int a = 0; a < 8; ++a) r[k][a] = Cnt(0.0);
      qtr_backward<Cnt>(cv, cx, cy, cz, xz, xy, r[k]);
    }
  }
  return Cnt::ops;
}

}  // namespace

// ----------------------------------------- fixed scratch of the no-alloc call
// Partial sums of rmtr_energy_noalloc, one per workgroup of the energy kernel,
// live in this fixed device array instead of allocated memory.  Each GPU the
// library runs on holds its own copy until the process ends; every call on
// that GPU shares it and it keeps the last call's values (each call writes
// every partial it reads, so nothing has to start at zero).
constexpr int kNoAllocPartials = kMaxPartials;
__device__ __align__(256) double scratch[kNoAllocPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current (the array's name is only a host-side
// stand-in and must never reach a kernel).
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double*>(q);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}
}  // namespace

// ================================================================== C-ABI
extern "C" {

int64_t rmtr_element_flops(int32_t dim, int32_t kind) {
  if (kind < 0 || kind > 4) return -1;
  if (dim == 3 && (kind == 0 || kind == 2 || kind == 3)) return count_quarter(kind);
  if (dim == 3) return count_kind<3>(kind);
  if (dim == 2) return count_kind<2>(kind);
  return -1;
}

void rmtr_default_params(rmtr_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->eta1 = 0.1;
  p->eta2 = 0.75;
  p->gamma1 = 0.5;
  p->gamma2 = 2.0;
  p->delta0 = 1.0;
  p->delta_max = 10.0;
  p->rtol = 1e-8;
  p->coarse_qp_rtol = 1e-10;
  p->guard = 1e-14;
  p->mu1 = 1;
  p->mu2 = 1;
  p->pgs_sweeps = 3;
  p->coarse_tr_its = 5;
  p->coarse_qp_its = 500;
  p->fallback_sweeps = 50;
  p->max_vcycles = 200;
  p->precision = RMTR_FP64;
  p->coarse_model = 0;
  p->nn_patience = 3;
  p->shrink_to_step = 0;
  p->gs_mode = 0;
  p->first_order = 0;
}

rmtr_status rmtr_create(const rmtr_model* m, rmtr_ctx** out) {
  if (!m || !out) return RMTR_E_ARG;
  *out = nullptr;
  if (m->dim != 2 && m->dim != 3) return RMTR_E_ARG;
  if (m->n_levels < 1 || m->n_levels > 12 || m->n_cells < 1) return RMTR_E_ARG;
  if (m->n_cells % (1 << (m->n_levels - 1)) != 0) return RMTR_E_ARG;
  if (!(m->mu > 0.0) || !(m->lambda + 2.0 * m->mu / 3.0 > 0.0) || !(m->Gc > 0.0) || !(m->ls > 0.0) ||
      !(m->k >= 0.0 && m->k < 1.0))
    return RMTR_E_ARG;
  if (m->split < kSplitNone || m->split > kSplitSpectral) return RMTR_E_ARG;
  rmtr_ctx* c = new rmtr_ctx();
  c->model = *m;
  c->mat.lam = m->lambda;
  c->mat.mu = m->mu;
  c->mat.K = m->lambda + 2.0 * m->mu / 3.0;
  c->mat.Gc = m->Gc;
  c->mat.ls = m->ls;
  c->mat.k = m->k;
  c->mat.split = m->split;
  set_derived(c->mat);
  c->L = m->n_levels;
  c->lv.resize(c->L + 1);
  for (int l = 1; l <= c->L; ++l) {
    Level& v = c->lv[l];
    v.N = m->n_cells >> (c->L - l);
    v.h = 1.0 / double(v.N);
    v.nodes = 1;
    v.nelem = 1;
    for (int i = 0; i < m->dim; ++i) {
      v.nodes *= (v.N + 1);
      v.nelem *= v.N;
    }
    v.n = v.nodes * (m->dim + 1);
  }
  *out = c;
  return RMTR_OK;
}

void rmtr_destroy(rmtr_ctx* c) {
  if (!c) return;
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->hs) (void)hipHostFree(c->hs);
  delete c;
}

const char* rmtr_last_error(const rmtr_ctx* c) { return c ? c->err.c_str() : "null context"; }

int64_t rmtr_level_nodes(const rmtr_ctx* c, int32_t level) {
  if (!valid_level(c, level)) return -1;
  return c->lv[level].nodes;
}

rmtr_status rmtr_init_fields(rmtr_ctx* c, int32_t level, const double* table, int32_t n_frac, double band,
                             int32_t p_mode, double p_value, double p_band, double* c0, double* p, void* stream) {
  if (!valid_level(c, level) || !c0 || n_frac < 0 || (n_frac > 0 && !table))
    return fail(c, RMTR_E_ARG, "rmtr_init_fields: bad arguments");
  if (p_mode == 1 && c->model.dim != 3) return fail(c, RMTR_E_ARG, "rmtr_init_fields: per-fracture p needs 3D");
  const int cols = c->model.dim == 3 ? 8 : 7;
  const size_t need = size_t(n_frac) * cols + 1;
  HIPCHK(c, grow(c, &c->table, &c->table_cap, need));
  if (n_frac > 0)
    HIPCHK(c, hipMemcpyAsync(c->table, table, size_t(n_frac) * cols * sizeof(double), hipMemcpyHostToDevice, S(stream)));
  HIPCHK(c, launch_init_fields(c->model.dim, c->lv[level].N, c->table, n_frac, band, p_mode, p_value, p_band, c0, p,
                               S(stream)));
  // the host table must stay readable until the copy is done
  HIPCHK(c, hipStreamSynchronize(S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_energy(rmtr_ctx* c, int32_t level, const double* x, const double* p, double* out, void* stream) {
  if (!valid_level(c, level) || !x || !p || !out) return fail(c, RMTR_E_ARG, "rmtr_energy: bad arguments");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, launch_energy(eargs(c, level, nullptr), x, nullptr, 0, p, c->partials, out, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_energy_noalloc(rmtr_ctx* c, int32_t level, const double* x, const double* p, double* out,
                                void* stream) {
  if (!valid_level(c, level) || !x || !p || !out) return fail(c, RMTR_E_ARG, "rmtr_energy_noalloc: bad arguments");
  const ElemArgs a = eargs(c, level, nullptr);
  const int need = energy_partials(a);
  if (need > kNoAllocPartials)
    return fail(c, RMTR_E_ARG, "rmtr_energy_noalloc: level needs " + std::to_string(need) +
                                   " partial sums, the fixed scratch holds " + std::to_string(kNoAllocPartials));
  double* ptr = nullptr;
  HIPCHK(c, scratch_address(&ptr));
  HIPCHK(c, launch_energy(a, x, nullptr, 0, p, ptr, out, S(stream)));
  return RMTR_OK;
}

size_t rmtr_workspace_bytes(const rmtr_ctx* c, const rmtr_params* prm) {
  if (!c) return 0;
  if (!prm) return common_bytes(c);
  return loadstep_bytes(c, prm->precision == RMTR_FP32, prm->use_learned != 0, prm->coarse_model == 2);
}

rmtr_status rmtr_bind_workspace(rmtr_ctx* c, void* dev, size_t bytes) {
  if (!c) return RMTR_E_ARG;
  if (!dev || bytes == 0 || (reinterpret_cast<uintptr_t>(dev) & 255u) != 0)
    return fail(c, RMTR_E_ARG, "rmtr_bind_workspace: needs a non-empty, 256-byte aligned device buffer");
  if (c->ws || c->partials || !c->allocs.empty())
    return fail(c, RMTR_E_ARG, "rmtr_bind_workspace: bind once, before the context's first device call");
  c->ws = static_cast<char*>(dev);
  c->ws_bytes = bytes;
  c->ws_used = 0;
  return RMTR_OK;
}

size_t rmtr_workspace_used(const rmtr_ctx* c) { return c ? c->ws_used : 0; }

rmtr_status rmtr_energy_diff(rmtr_ctx* c, int32_t level, const double* x, const void* s, int32_t s_precision,
                             const double* p, double* out, void* stream) {
  if (!valid_level(c, level) || !x || !s || !p || !out) return fail(c, RMTR_E_ARG, "rmtr_energy_diff: bad arguments");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, launch_energy(eargs(c, level, nullptr), x, s, s_precision == RMTR_FP32, p, c->partials, out, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_gradient(rmtr_ctx* c, int32_t level, const double* x, const double* p, const uint8_t* dir,
                          double* g, void* stream) {
  if (!valid_level(c, level) || !x || !p || !g) return fail(c, RMTR_E_ARG, "rmtr_gradient: bad arguments");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, launch_gradient(eargs(c, level, dir), x, p, g, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_hessvec(rmtr_ctx* c, int32_t level, const void* xl, const void* p, const uint8_t* dir,
                         const void* v, void* hv, int32_t precision, void* stream) {
  if (!valid_level(c, level) || !xl || !p || !v || !hv) return fail(c, RMTR_E_ARG, "rmtr_hessvec: bad arguments");
  if (v == hv) return fail(c, RMTR_E_ARG, "rmtr_hessvec: v and Hv must not alias");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, launch_hessvec(eargs(c, level, dir), xl, p, v, hv, precision == RMTR_FP32, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_diag_blocks(rmtr_ctx* c, int32_t level, const void* xl, const void* p, const uint8_t* dir, void* D,
                             int32_t precision, void* stream) {
  if (!valid_level(c, level) || !xl || !p || !D) return fail(c, RMTR_E_ARG, "rmtr_diag_blocks: bad arguments");
  HIPCHK(c, launch_diag_blocks(eargs(c, level, dir), xl, p, D, precision == RMTR_FP32, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_smooth(rmtr_ctx* c, int32_t level, const double* xl, const double* p, const uint8_t* dir,
                        const void* g, const void* lo, const void* hi, void* s, int32_t n_sweeps, int32_t precision,
                        void* stream) {
  if (!valid_level(c, level) || !xl || !p || !g || !lo || !hi || !s || n_sweeps < 0)
    return fail(c, RMTR_E_ARG, "rmtr_smooth: bad arguments");
  const bool f32 = precision == RMTR_FP32;
  Level& v = c->lv[level];
  if (!v.coefop) HIPCHK(c, dalloc(c, &v.coefop, coef_values(c->model.dim, v.N, c->mat.split)));
  void* Sm = nullptr;
  if (f32) {
    if (!v.Sopf) HIPCHK(c, dalloc(c, &v.Sopf, stencil_values(c->model.dim, v.N)));
    Sm = v.Sopf;
  } else {
    if (!v.Sop) HIPCHK(c, dalloc(c, &v.Sop, stencil_values(c->model.dim, v.N)));
    Sm = v.Sop;
  }
  HIPCHK(c, launch_st_assemble(eargs(c, level, dir), xl, p, v.coefop, Sm, f32, S(stream)));
  HIPCHK(c, launch_st_pgs(c->model.dim, v.N, Sm, dir, g, lo, hi, s, n_sweeps, f32, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_restrict(rmtr_ctx* c, int32_t fine_level, int32_t mode, const void* fine, void* coarse,
                          int32_t precision, void* stream) {
  if (!valid_level(c, fine_level) || fine_level < 2 || mode < 0 || mode > 3 || !fine || !coarse)
    return fail(c, RMTR_E_ARG, "rmtr_restrict: bad arguments");
  HIPCHK(c, launch_restrict(c->model.dim, c->lv[fine_level - 1].N, mode, fine, coarse, precision == RMTR_FP32,
                            S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_prolong(rmtr_ctx* c, int32_t coarse_level, const void* coarse, void* fine, int32_t precision,
                         void* stream) {
  if (!valid_level(c, coarse_level) || coarse_level >= c->L || !coarse || !fine)
    return fail(c, RMTR_E_ARG, "rmtr_prolong: bad arguments");
  HIPCHK(c, launch_prolong(c->model.dim, c->lv[coarse_level].N, coarse, fine, precision == RMTR_FP32, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_coarse_hessvec(rmtr_ctx* c, int32_t level, const double* xl, const double* p, const uint8_t* dir,
                                const double* v, double* hv, int32_t precision, void* stream) {
  if (!valid_level(c, level) || level >= c->L || !xl || !p || !v || !hv || v == hv)
    return fail(c, RMTR_E_ARG, "rmtr_coarse_hessvec: bad arguments");
  const bool f32 = precision == RMTR_FP32;
  const int L = c->L, d = c->model.dim;
  Level& f = c->lv[L];
  if (!f.coefop) HIPCHK(c, dalloc(c, &f.coefop, coef_values(d, f.N, c->mat.split)));
  void* Sm = nullptr;
  if (f32) {
    if (!f.Sopf) HIPCHK(c, dalloc(c, &f.Sopf, stencil_values(d, f.N)));
    Sm = f.Sopf;
  } else {
    if (!f.Sop) HIPCHK(c, dalloc(c, &f.Sop, stencil_values(d, f.N)));
    Sm = f.Sop;
  }
  HIPCHK(c, launch_st_assemble(eargs(c, L, dir), xl, p, f.coefop, Sm, f32, S(stream)));
  HIPCHK(c, grow(c, &c->rap_work, &c->rap_cap, st_rap_work_doubles(d, f.N, f32 ? 1 : 0)));
  const void* src = Sm;
  int src32 = f32 ? 1 : 0;
  for (int l = L - 1; l >= level; --l) {
    Level& cl = c->lv[l];
    if (!cl.Sop) HIPCHK(c, dalloc(c, &cl.Sop, stencil_values(d, cl.N)));
    HIPCHK(c, launch_st_rap(d, c->lv[l + 1].N, src, src32, cl.Sop, nullptr, c->rap_work, S(stream)));
    src = cl.Sop;
    src32 = 0;
  }
  HIPCHK(c, launch_st_matvec(d, c->lv[level].N, c->lv[level].Sop, v, hv, 0, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_mprgp(rmtr_ctx* c, int32_t level, const double* K, const double* g, const double* lo, const double* hi,
                       double* s, int32_t max_it, double rtol, int32_t fallback_sweeps, int32_t* iterations,
                       int32_t* status, void* stream) {
  if (!valid_level(c, level) || !K || !g || !lo || !hi || !s || max_it < 0)
    return fail(c, RMTR_E_ARG, "rmtr_mprgp: bad arguments");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, grow(c, &c->op_work, &c->op_work_cap, mprgp_work_doubles(c->model.dim, c->lv[level].N)));
  HIPCHK(c, grow(c, &c->op_st, &c->op_cap, stencil_values(c->model.dim, c->lv[level].N)));
  HIPCHK(c, launch_em_to_st(c->model.dim, c->lv[level].N, K, c->op_st, 0, S(stream)));
  MprgpResult res;
  HIPCHK(c, run_mprgp(c->model.dim, c->lv[level].N, c->op_st, nullptr, g, lo, hi, s, max_it, rtol, fallback_sweeps,
                      c->op_work, c->hs + 48, &res, S(stream)));
  HIPCHK(c, hipStreamSynchronize(S(stream)));
  if (iterations) *iterations = res.iterations;
  if (status) *status = res.status;
  return RMTR_OK;
}

rmtr_status rmtr_dot(rmtr_ctx* c, int64_t n, const double* a, const double* b, double* out, void* stream) {
  if (!c || n < 0 || !a || !b || !out) return fail(c, RMTR_E_ARG, "rmtr_dot: bad arguments");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, launch_dot(n, a, b, c->partials, out, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_chi(rmtr_ctx* c, int32_t level, const double* x, const double* g, const double* cl,
                     const uint8_t* dir, double* out, void* stream) {
  if (!valid_level(c, level) || !x || !g || !cl || !out) return fail(c, RMTR_E_ARG, "rmtr_chi: bad arguments");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, launch_chi(c->model.dim, c->lv[level].N, x, g, cl, dir, c->partials, c->scal + 60, S(stream)));
  // chi = sqrt(sum of squares), on the device
  HIPCHK(c, hipMemcpyAsync(c->hs + 60, c->scal + 60, sizeof(double), hipMemcpyDeviceToHost, S(stream)));
  HIPCHK(c, hipStreamSynchronize(S(stream)));
  const double v = sqrt(c->hs[60]);
  HIPCHK(c, hipMemcpyAsync(out, &v, sizeof(double), hipMemcpyHostToDevice, S(stream)));
  HIPCHK(c, hipStreamSynchronize(S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_solve_loadstep(rmtr_ctx* c, const double* p, const double* c_lower, const uint8_t* dir,
                                const double* f_ext, const rmtr_params* prm, double* x, rmtr_stats* stats,
                                double* chi_history, void* stream) {
  if (!c || !p || !c_lower || !prm || !x) return fail(c, RMTR_E_ARG, "rmtr_solve_loadstep: bad arguments");
  if (prm->mu1 < 0 || prm->mu2 < 0 || prm->pgs_sweeps < 0 || prm->max_vcycles < 0 || !(prm->eta1 > 0.0) ||
      prm->eta1 > prm->eta2 || !(prm->gamma1 > 0.0) || prm->gamma1 > 1.0 || prm->gamma2 < 1.0 ||
      !(prm->delta0 > 0.0))
    return fail(c, RMTR_E_ARG, "rmtr_solve_loadstep: invalid parameters");
  if (prm->gs_mode != 0)
    return fail(c, RMTR_E_ARG, "rmtr_solve_loadstep: only gs_mode 0 (global node colours) is built");
  if (prm->coarse_model < 0 || prm->coarse_model > 2)
    return fail(c, RMTR_E_ARG, "rmtr_solve_loadstep: coarse_model must be 0, 1 or 2");
  if (prm->first_order && prm->coarse_model != 0)
    return fail(c, RMTR_E_ARG, "rmtr_solve_loadstep: first_order needs coarse_model 0 (the level's own functional)");
  if (prm->use_learned &&
      (c->model.dim != 3 || c->L < 2 || !prm->nn || !prm->nn->w || !prm->nn->bias || !prm->nn->scales))
    return fail(c, RMTR_E_ARG, "rmtr_solve_loadstep: the learned proposal needs 3D, L >= 2 and a network");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = S(stream);
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  const bool mixed = prm->precision == RMTR_FP32;
  for (int l = 1; l <= c->L; ++l)
    if ((r = ensure_solver_level(c, l, mixed, prm->coarse_model == 2)) != RMTR_OK) return r;
  if (!c->mprgp_work) HIPCHK(c, dalloc(c, &c->mprgp_work, mprgp_work_doubles(c->model.dim, c->lv[1].N)));
  // the finest level's stencil and its coefficients are FP32 in the mixed
  // form (with more than one level): half the memory
  const bool fine32 = mixed && c->L > 1;
  if (c->L > 1)
    HIPCHK(c, grow(c, &c->rap_work, &c->rap_cap, st_rap_work_doubles(c->model.dim, c->lv[c->L].N, fine32 ? 1 : 0)));
  {
    const size_t cv = coef_values(c->model.dim, c->lv[c->L].N, c->mat.split);
    HIPCHK(c, grow(c, &c->lv[c->L].coef, &c->lv[c->L].coef_cap, fine32 ? (cv + 1) / 2 : cv));
  }
  Run run{c, *prm, st, dir, f_ext, mixed, prm->coarse_model != 1, prm->coarse_model == 2, prm->first_order != 0};
  const int L = c->L, d = c->model.dim;
  Level& f = c->lv[L];
  // pressure on every level: fine copy, then injection
  HIPCHK(c, hipMemcpyAsync(f.p, p, f.nodes * sizeof(double), hipMemcpyDeviceToDevice, st));
  for (int l = L - 1; l >= 1; --l) HIPCHK(c, launch_inject_scalar(d, c->lv[l].N, c->lv[l + 1].p, c->lv[l].p, st));
  if (mixed) HIPCHK(c, launch_convert(f.nodes, f.p, 0, f.pf, 1, st));
  HIPCHK(c, launch_fine_bounds(d, f.N, c_lower, f.Lb, f.Ub, st));
  if (dir)
    for (int l = L - 1; l >= 1; --l)
      HIPCHK(c, launch_inject_mask(d, c->lv[l].N, l + 1 == L ? dir : c->lv[l + 1].mask, c->lv[l].mask, st));
  double delta = prm->delta0;
  if ((r = run.fine_grad(x, f.g)) != RMTR_OK) return r;
  HIPCHK(c, launch_chi(d, f.N, x, f.g, c_lower, dir, c->partials, c->scal, st));
  HIPCHK(c, launch_energy(eargs(c, L, dir), x, nullptr, 0, f.p, c->partials, c->scal + 1, st));
  if (f_ext)
    HIPCHK(c, launch_dot(f.n, f_ext, x, c->partials, c->scal + 2, st));
  else
    HIPCHK(c, launch_fill(1, 0.0, c->scal + 2, st));
  if ((r = run.fetch(3, false)) != RMTR_OK) return r;
  const double chi0 = sqrt(c->hs[0]);
  run.f_ref = c->hs[1] - c->hs[2];
  rmtr_stats out{};
  out.chi0 = out.chi = chi0;
  int vc = 0;
  const char* vb = getenv("RMTR_VERBOSE");
  const bool verbose = vb && vb[0] && vb[0] != '0';
  run.trace = vb && vb[0] == '2';
  if (verbose) fprintf(stderr, "rmtr: chi0 %.6e f %.6e\n", chi0, run.f_ref);
  if (chi0 > 0.0 && isfinite(chi0)) {
    for (vc = 0; vc < prm->max_vcycles;) {
      // lagged Hessian of this V-cycle: linearisation point x0 = x
      HIPCHK(c, hipMemcpyAsync(f.x0, x, f.n * sizeof(double), hipMemcpyDeviceToDevice, st));
      if (L == 1) {
        HIPCHK(c, launch_st_assemble(eargs(c, 1, dir), f.x0, f.p, f.coef, f.S, 0, st));
      } else if (mixed) {
        HIPCHK(c, launch_st_assemble(eargs(c, L, dir), f.x0, f.p, f.coef, f.Sf, 1, st));
      } else {
        HIPCHK(c, launch_st_assemble(eargs(c, L, dir), f.x0, f.p, f.coef, f.S, 0, st));
      }
      if ((r = run.vcycle(L, x, delta)) != RMTR_OK) return r;
      ++vc;
      if ((r = run.fine_grad(x, f.g)) != RMTR_OK) return r;
      HIPCHK(c, launch_chi(d, f.N, x, f.g, c_lower, dir, c->partials, c->scal, st));
      if ((r = run.fetch(1, false)) != RMTR_OK) return r;
      out.chi = sqrt(c->hs[0]);
      if (chi_history) chi_history[vc - 1] = out.chi;
      if (verbose) {
        fprintf(stderr, "rmtr: vcycle %d chi/chi0 %.3e delta %.3e accepted %d rejected %d nn %d/%d\n", vc,
                out.chi / chi0, delta, run.accepted, run.rejected, run.nn_accepted, run.nn_proposed);
        fflush(stderr);
      }
      if (!isfinite(out.chi)) return fail(c, RMTR_E_NONFINITE, "rmtr_solve_loadstep: non-finite iterate");
      if (out.chi <= prm->rtol * chi0) break;
    }
  }
  HIPCHK(c, launch_energy(eargs(c, L, dir), x, nullptr, 0, f.p, c->partials, c->scal, st));
  if (f_ext)
    HIPCHK(c, launch_dot(f.n, f_ext, x, c->partials, c->scal + 1, st));
  else
    HIPCHK(c, launch_fill(1, 0.0, c->scal + 1, st));
  if ((r = run.fetch(2, false)) != RMTR_OK) return r;
  out.energy = c->hs[0] - c->hs[1];
  out.vcycles = vc;
  out.tr_accepted = run.accepted;
  out.tr_rejected = run.rejected;
  out.nn_proposed = run.nn_proposed;
  out.nn_accepted = run.nn_accepted;
  out.delta = delta;
  out.status = (chi0 == 0.0 || out.chi <= prm->rtol * chi0) ? RMTR_OK : RMTR_NOT_CONVERGED;
  out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = out;
  return out.status;
}


rmtr_status rmtr_step_box(rmtr_ctx* c, int32_t level, const double* x, const double* cl, double delta,
                          const uint8_t* dir, double* lo, double* hi, void* stream) {
  if (!valid_level(c, level) || level != c->L || !x || !cl || !lo || !hi || !(delta >= 0.0))
    return fail(c, RMTR_E_ARG, "rmtr_step_box: bad arguments");
  Level& v = c->lv[level];
  HIPCHK(c, grow(c, &c->box_tmp, &c->box_cap, size_t(2 * v.n)));
  double* Lb = c->box_tmp;
  double* Ub = c->box_tmp + v.n;
  HIPCHK(c, launch_fine_bounds(c->model.dim, v.N, cl, Lb, Ub, S(stream)));
  HIPCHK(c, launch_step_box(c->model.dim, v.N, x, Lb, Ub, delta, dir, lo, hi, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_neumann_load(rmtr_ctx* c, int32_t level, int32_t face_mask, const double* traction,
                              const double* p, double* b, void* stream) {
  if (!valid_level(c, level) || !b || !p || face_mask < 0 || face_mask >= (1 << (2 * c->model.dim)) ||
      (face_mask && !traction))
    return fail(c, RMTR_E_ARG, "rmtr_neumann_load: bad arguments");
  NeumannTraction tr{};
  const int d = c->model.dim;
  for (int f = 0; f < 2 * d; ++f)
    for (int i = 0; i < d; ++i) tr.t[f][i] = traction ? traction[d * f + i] : 0.0;
  HIPCHK(c, launch_neumann_load(d, c->lv[level].N, face_mask, tr, p, b, S(stream)));
  return RMTR_OK;
}

int64_t rmtr_nn_size(int32_t what, int32_t nx, int32_t ny, int32_t nz) {
  if (what == 0) return nn_weight_count();
  if (what == 1) return nn_bias_count();
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  const int64_t nvox = int64_t(nx) * ny * nz;
  if (what == 2) return nn_act_floats(nvox);
  if (what == 3) return int64_t(nn_backward_work_floats(nvox));
  return -1;
}

static bool nn_box_ok(int32_t nx, int32_t ny, int32_t nz) {
  return nx >= 1 && ny >= 1 && nz >= 1 && int64_t(nx) * ny * nz <= (int64_t(1) << 31) / 32;
}

rmtr_status rmtr_nn_forward(rmtr_ctx* c, const uint16_t* w, const float* bias, float* act, int32_t nx, int32_t ny,
                            int32_t nz, void* stream) {
  if (!c || !w || !bias || !act || !nn_box_ok(nx, ny, nz)) return fail(c, RMTR_E_ARG, "rmtr_nn_forward: bad arguments");
  float* layer[7];
  nn_layers(act, int64_t(nx) * ny * nz, layer);
  HIPCHK(c, nn_forward(w, bias, layer, nx, ny, nz, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_backward(rmtr_ctx* c, const uint16_t* w, const float* act, const float* dout, float* grad,
                             float* work, int32_t nx, int32_t ny, int32_t nz, void* stream) {
  if (!c || !w || !act || !dout || !grad || !work || !nn_box_ok(nx, ny, nz))
    return fail(c, RMTR_E_ARG, "rmtr_nn_backward: bad arguments");
  HIPCHK(c, nn_backward(w, act, dout, grad, grad + nn_weight_count(), nx, ny, nz, work, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_mse(rmtr_ctx* c, const float* out, const float* target, const int32_t* win, float* dout,
                        double* loss, int32_t nx, int32_t ny, int32_t nz, void* stream) {
  if (!c || !out || !target || !win || !dout || !loss || !nn_box_ok(nx, ny, nz))
    return fail(c, RMTR_E_ARG, "rmtr_nn_mse: bad arguments");
  const int32_t n3[3] = {nx, ny, nz};
  for (int i = 0; i < 3; ++i)
    if (win[2 * i] < 0 || win[2 * i + 1] > n3[i] || win[2 * i] >= win[2 * i + 1])
      return fail(c, RMTR_E_ARG, "rmtr_nn_mse: empty or out-of-range window");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  const int wi[6] = {win[0], win[1], win[2], win[3], win[4], win[5]};
  HIPCHK(c, nn_mse(out, target, dout, nx, ny, nz, wi, c->partials, loss, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_adam_step(rmtr_ctx* c, int64_t n, int64_t n_bf16, float lr, int32_t t, const float* grad,
                              float* master, float* m, float* v, uint16_t* w_bf16, void* stream) {
  if (!c || n < 0 || n_bf16 < 0 || n_bf16 > n || t < 1 || !grad || !master || !m || !v || (n_bf16 > 0 && !w_bf16))
    return fail(c, RMTR_E_ARG, "rmtr_nn_adam_step: bad arguments");
  HIPCHK(c, nn_adam(n, n_bf16, lr, t, grad, master, m, v, w_bf16, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_to_bf16(rmtr_ctx* c, int64_t n, const float* master, uint16_t* w_bf16, void* stream) {
  if (!c || n < 0 || (n > 0 && (!master || !w_bf16))) return fail(c, RMTR_E_ARG, "rmtr_nn_to_bf16: bad arguments");
  HIPCHK(c, nn_to_bf16(n, master, w_bf16, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_features(rmtr_ctx* c, int32_t level, const double* x, const double* g, const float* scales,
                             float* in8, void* stream) {
  if (!valid_level(c, level) || c->model.dim != 3 || !x || !g || !scales || !in8)
    return fail(c, RMTR_E_ARG, "rmtr_nn_features: bad arguments (3D only)");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  double* rms = c->scal + 40;
  HIPCHK(c, nn_grad_rms(c->lv[level].nodes, g, c->partials, rms, S(stream)));
  HIPCHK(c, nn_features(c->lv[level].nodes, x, g, scales, rms, in8, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_channel_rms(rmtr_ctx* c, int32_t level, const double* v, double* rms, void* stream) {
  if (!valid_level(c, level) || c->model.dim != 3 || !v || !rms)
    return fail(c, RMTR_E_ARG, "rmtr_nn_channel_rms: bad arguments (3D only)");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, nn_grad_rms(c->lv[level].nodes, v, c->partials, rms, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_target(rmtr_ctx* c, int32_t level, const double* g, const double* s, const float* scales,
                           float* t, void* stream) {
  if (!valid_level(c, level) || c->model.dim != 3 || !g || !s || !scales || !t)
    return fail(c, RMTR_E_ARG, "rmtr_nn_target: bad arguments (3D only)");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  double* rms = c->scal + 40;
  HIPCHK(c, nn_grad_rms(c->lv[level].nodes, g, c->partials, rms, S(stream)));
  HIPCHK(c, nn_target(c->lv[level].n, s, scales, rms, t, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_fit_scales(rmtr_ctx* c, int32_t level, int32_t n_samples, const double* const* x,
                               const double* const* g, const double* const* s, float* scales, void* stream) {
  if (!valid_level(c, level) || c->model.dim != 3 || n_samples < 1 || !x || !g || !s || !scales)
    return fail(c, RMTR_E_ARG, "rmtr_nn_fit_scales: bad arguments (3D only)");
  for (int i = 0; i < n_samples; ++i)
    if (!x[i] || !g[i] || !s[i]) return fail(c, RMTR_E_ARG, "rmtr_nn_fit_scales: null sample");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  HIPCHK(c, grow(c, &c->fit_buf, &c->fit_cap, size_t(12) * n_samples));
  const int64_t nn = c->lv[level].nodes;
  for (int i = 0; i < n_samples; ++i) {
    HIPCHK(c, nn_grad_rms(nn, x[i], c->partials, c->fit_buf + 12 * i, S(stream)));
    HIPCHK(c, nn_grad_rms(nn, g[i], c->partials, c->fit_buf + 12 * i + 4, S(stream)));
    HIPCHK(c, nn_grad_rms(nn, s[i], c->partials, c->fit_buf + 12 * i + 8, S(stream)));
  }
  HIPCHK(c, nn_fit_scales(n_samples, c->fit_buf, scales, S(stream)));
  return RMTR_OK;
}

rmtr_status rmtr_nn_propose(rmtr_ctx* c, int32_t level, const rmtr_nn* net, const double* x, const double* g,
                            const double* lo, const double* hi, double* s, void* stream) {
  if (!valid_level(c, level) || c->model.dim != 3 || !net || !net->w || !net->bias || !net->scales || !x || !g ||
      !lo || !hi || !s)
    return fail(c, RMTR_E_ARG, "rmtr_nn_propose: bad arguments (3D only)");
  rmtr_status r = ensure_common(c);
  if (r != RMTR_OK) return r;
  return nn_propose(c, level, *net, x, g, lo, hi, s, S(stream));
}

}  // extern "C"

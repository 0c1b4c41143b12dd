// MPRGP (Dostal's modified proportioning with reduced gradient projection)
// for the coarsest-level trust-region subproblem (Sec. 3.2.1):
//     min 1/2 s^T A s - b^T s,  lo <= s <= hi,   A = coarse Hessian, b = -g.
// The level's element matrices are first assembled into a 3^d-point block
// stencil (stencil_kernels.hip), so every matrix-vector product is a
// row-parallel pass over contiguous rows.  The
// host drives the iteration; every reduction is a fixed-order two-stage tree,
// so the scalars (and the branch taken) do not depend on scheduling.
#include <math.h>

#include "rmtr_kernels.h"

namespace rmtr {
namespace {

constexpr int kB = 256;
constexpr int kNV = 5;  // reduced values per pass: four sums and one min

template <int DIM>
constexpr int n_off() {
  return DIM == 3 ? 27 : 9;
}

int nblocks(int64_t n) {
  int64_t b = (n + kB - 1) / kB;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return int(b);
}

__device__ inline void bred(double (&v)[kNV], double (*sh)[kB], double* out) {
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kNV; ++k) sh[k][t] = v[k];
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int k = 0; k < kNV - 1; ++k) sh[k][t] += sh[k][t + s];
      sh[kNV - 1][t] = fmin(sh[kNV - 1][t], sh[kNV - 1][t + s]);
    }
    __syncthreads();
  }
  if (t == 0)
#pragma unroll
    for (int k = 0; k < kNV; ++k) out[k] = sh[k][0];
}

__device__ inline void vinit(double (&v)[kNV]) {
#pragma unroll
  for (int k = 0; k < kNV - 1; ++k) v[k] = 0.0;
  v[kNV - 1] = INFINITY;
}

__global__ __launch_bounds__(kB) void k_final(const double* __restrict__ partials, int nb, double* __restrict__ out) {
  __shared__ double sh[kNV][kB];
  double v[kNV];
  vinit(v);
  for (int i = threadIdx.x; i < nb; i += kB) {
#pragma unroll
    for (int k = 0; k < kNV - 1; ++k) v[k] += partials[kNV * i + k];
    v[kNV - 1] = fmin(v[kNV - 1], partials[kNV * i + kNV - 1]);
  }
  bred(v, sh, out);
}

__device__ inline bool is_free(double s, double lo, double hi) { return s > lo && s < hi; }

__device__ inline double chop(double s, double g, double lo, double hi) {
  if (!(lo < hi)) return 0.0;
  double r = 0.0;
  if (s <= lo) r += fmin(g, 0.0);
  if (s >= hi) r += fmax(g, 0.0);
  return r;
}

// state sums of (s, gr): ||phi + beta||^2, beta^T beta, phit^T phi, and
// phi^T Ad (when Ad is given); phi and beta are written.
__device__ inline void state_terms(double abar, double si, double gi, double l, double h, double* phi,
                                   double* beta, int64_t i, const double* Ad, double (&v)[kNV]) {
  const double f = is_free(si, l, h) ? gi : 0.0;
  const double b = chop(si, gi, l, h);
  phi[i] = f;
  beta[i] = b;
  const double ft = f > 0.0 ? fmin((si - l) / abar, f) : fmax((si - h) / abar, f);
  v[0] += (f + b) * (f + b);
  v[1] += b * b;
  v[2] += ft * f;
  if (Ad) v[3] += f * Ad[i];
}

__global__ __launch_bounds__(kB) void k_state(int64_t n, double abar, const double* __restrict__ s,
                                              const double* __restrict__ gr, const double* __restrict__ lo,
                                              const double* __restrict__ hi, double* __restrict__ phi,
                                              double* __restrict__ beta, double* __restrict__ partials) {
  __shared__ double sh[kNV][kB];
  double v[kNV];
  vinit(v);
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    state_terms(abar, s[i], gr[i], lo[i], hi[i], phi, beta, i, nullptr, v);
  bred(v, sh, partials + kNV * blockIdx.x);
}

// d^T A d, g^T d (slots 0, 1) and the largest feasible step along -d (min).
__global__ __launch_bounds__(kB) void k_dir(int64_t n, const double* __restrict__ s, const double* __restrict__ gr,
                                            const double* __restrict__ d, const double* __restrict__ Ad,
                                            const double* __restrict__ lo, const double* __restrict__ hi,
                                            double* __restrict__ partials) {
  __shared__ double sh[kNV][kB];
  double v[kNV];
  vinit(v);
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const double di = d[i];
    v[0] += di * Ad[i];
    v[1] += gr[i] * di;
    if (di > 0.0) v[kNV - 1] = fmin(v[kNV - 1], (s[i] - lo[i]) / di);
    if (di < 0.0) v[kNV - 1] = fmin(v[kNV - 1], (s[i] - hi[i]) / di);
  }
  bred(v, sh, partials + kNV * blockIdx.x);
}

// s -= a d (clipped to the box if clip); gr -= a Ad; then the state sums
// of the new point, with phi^T Ad in slot 3.
__global__ __launch_bounds__(kB) void k_step_state(int64_t n, double a, int clip, double abar,
                                                   const double* __restrict__ d, const double* __restrict__ Ad,
                                                   const double* __restrict__ lo, const double* __restrict__ hi,
                                                   double* __restrict__ s, double* __restrict__ gr,
                                                   double* __restrict__ phi, double* __restrict__ beta,
                                                   double* __restrict__ partials) {
  __shared__ double sh[kNV][kB];
  double v[kNV];
  vinit(v);
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    double si = s[i] - a * d[i];
    if (clip) si = fmin(fmax(si, lo[i]), hi[i]);
    const double gi = gr[i] - a * Ad[i];
    s[i] = si;
    gr[i] = gi;
    state_terms(abar, si, gi, lo[i], hi[i], phi, beta, i, Ad, v);
  }
  bred(v, sh, partials + kNV * blockIdx.x);
}

// expansion step: s -= af p, then s = P(s - abar phi(s, gr - af Ap))
__global__ __launch_bounds__(kB) void k_expand(int64_t n, double af, double abar, const double* __restrict__ p,
                                               const double* __restrict__ Ap, const double* __restrict__ lo,
                                               const double* __restrict__ hi, double* __restrict__ s,
                                               const double* __restrict__ gr) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const double si = s[i] - af * p[i];
    const double gi = gr[i] - af * Ap[i];
    const double f = is_free(si, lo[i], hi[i]) ? gi : 0.0;
    s[i] = fmin(fmax(si - abar * f, lo[i]), hi[i]);
  }
}

// gr = A s + g (A s given), then the state sums
__global__ __launch_bounds__(kB) void k_regrad_state(int64_t n, double abar, const double* __restrict__ As,
                                                     const double* __restrict__ g, const double* __restrict__ s,
                                                     const double* __restrict__ lo, const double* __restrict__ hi,
                                                     double* __restrict__ gr, double* __restrict__ phi,
                                                     double* __restrict__ beta, double* __restrict__ partials) {
  __shared__ double sh[kNV][kB];
  double v[kNV];
  vinit(v);
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const double gi = As[i] + g[i];
    gr[i] = gi;
    state_terms(abar, s[i], gi, lo[i], hi[i], phi, beta, i, nullptr, v);
  }
  bred(v, sh, partials + kNV * blockIdx.x);
}

// p = phi - bet p
__global__ __launch_bounds__(kB) void k_pupd(int64_t n, double bet, const double* __restrict__ phi,
                                             double* __restrict__ p) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    p[i] = phi[i] - bet * p[i];
}


}  // namespace

size_t mprgp_work_doubles(int dim, int N) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  const int64_t n = nn * (dim + 1);
  return size_t(5 * n + kNV * 1024 + 2 * kNV + 16);
}

hipError_t run_mprgp(int dim, int N, const double* S, const uint8_t* dir, const double* g, const double* lo,
                     const double* hi, double* s, int max_it, double rtol, int fallback_sweeps, double* work,
                     double* hs, MprgpResult* res, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  const int64_t n = nn * (dim + 1);
  double* gr = work;
  double* phi = gr + n;
  double* beta = phi + n;
  double* p = beta + n;
  double* Ad = p + n;
  double* part = Ad + n;
  const int nb = nblocks(n);
  const dim3 gb(nb), tb(kB);
  hipError_t e;
#define CK(x)                      \
  do {                             \
    e = (x);                       \
    if (e != hipSuccess) return e; \
  } while (0)
  // the final reduction writes straight into the (mapped, coherent) host
  // scalars; the synchronisation makes them visible
#define FETCH()                                                                     \
  do {                                                                              \
    hipLaunchKernelGGL(k_final, dim3(1), tb, 0, st, part, nb, hs);                  \
    CK(hipGetLastError());                                                          \
    CK(hipStreamSynchronize(st));                                                   \
  } while (0)
#define MATVEC(v, out) CK(launch_st_matvec(dim, N, S, v, out, 0, st))
  res->iterations = 0;
  res->status = 1;
  CK(launch_fill(n, 0.0, s, st));
  // ||A|| bound and ||b||
  {
    int nbr = 0;
    CK(launch_st_rowabs(dim, N, S, g, part, &nbr, st));
    hipLaunchKernelGGL(k_final, dim3(1), tb, 0, st, part, nbr, hs);
    CK(hipGetLastError());
    CK(hipStreamSynchronize(st));
  }
  const double normA = -hs[kNV - 1];
  const double bnorm = sqrt(hs[0]);
  if (!(normA > 0.0)) {
    res->status = 0;
    return hipSuccess;
  }
  const double abar = 1.9 / normA;
  const double tol = rtol * fmax(bnorm, 1e-300);
  // s = 0: gr = A s - b = g
  CK(hipMemcpyAsync(gr, g, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_state, gb, tb, 0, st, n, abar, s, gr, lo, hi, phi, beta, part);
  CK(hipGetLastError());
  CK(hipMemcpyAsync(p, phi, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  FETCH();
  int it = 0;
  bool negcurv = false;
  while (it < max_it) {
    const double normr = sqrt(hs[0]), bb = hs[1], pf = hs[2];
    if (normr <= tol) {
      res->status = 0;
      break;
    }
    ++it;
    if (bb <= pf) {
      MATVEC(p, Ad);
      hipLaunchKernelGGL(k_dir, gb, tb, 0, st, n, s, gr, p, Ad, lo, hi, part);
      CK(hipGetLastError());
      FETCH();
      const double pAp = hs[0], gp = hs[1], af = hs[kNV - 1];
      if (!(pAp > 0.0)) {
        negcurv = true;
        break;
      }
      const double acg = gp / pAp;
      if (acg <= af) {
        hipLaunchKernelGGL(k_step_state, gb, tb, 0, st, n, acg, 0, abar, p, Ad, lo, hi, s, gr, phi, beta, part);
        CK(hipGetLastError());
        FETCH();
        const double bet = hs[3] / pAp;
        hipLaunchKernelGGL(k_pupd, gb, tb, 0, st, n, bet, phi, p);
        CK(hipGetLastError());
      } else {
        hipLaunchKernelGGL(k_expand, gb, tb, 0, st, n, af, abar, p, Ad, lo, hi, s, gr);
        CK(hipGetLastError());
        MATVEC(s, Ad);
        hipLaunchKernelGGL(k_regrad_state, gb, tb, 0, st, n, abar, Ad, g, s, lo, hi, gr, phi, beta, part);
        CK(hipGetLastError());
        CK(hipMemcpyAsync(p, phi, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        FETCH();
      }
    } else {
      // proportioning step along the chopped gradient, kept inside the box
      MATVEC(beta, Ad);
      hipLaunchKernelGGL(k_dir, gb, tb, 0, st, n, s, gr, beta, Ad, lo, hi, part);
      CK(hipGetLastError());
      FETCH();
      const double dAd = hs[0], gd = hs[1], af = hs[kNV - 1];
      if (!(dAd > 0.0)) {
        negcurv = true;
        break;
      }
      const double a = fmin(gd / dAd, af);
      // beta is rewritten by the new state: step along a copy in p
      CK(hipMemcpyAsync(p, beta, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(k_step_state, gb, tb, 0, st, n, a, 1, abar, p, Ad, lo, hi, s, gr, phi, beta, part);
      CK(hipGetLastError());
      CK(hipMemcpyAsync(p, phi, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      FETCH();
    }
  }
  res->iterations = it;
  if (negcurv) {
    res->status = 2;
    CK(launch_st_pgs(dim, N, S, dir, g, lo, hi, s, fallback_sweeps, 0, st));
  } else if (it >= max_it && res->status != 0) {
    res->status = 1;
  }
  return hipSuccess;
#undef CK
#undef FETCH
#undef MATVEC
}

}  // namespace rmtr

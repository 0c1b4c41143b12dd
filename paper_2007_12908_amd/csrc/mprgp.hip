// MPRGP (Dostal's modified proportioning with reduced gradient projection)
// for the coarsest-level trust-region subproblem (Sec. 3.2.1):
//     min 1/2 s^T A s - b^T s,  lo <= s <= hi,   A = coarse Hessian, b = -g.
// The level's element matrices are first assembled into a 3^d-point block
// stencil (one row of (d+1) x 3^d x (d+1) values per node row), so every
// matrix-vector product is a row-parallel pass over contiguous rows.  The
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

// ---------------------------------------------------------------- stencil
// S[((n NC + al) NO + o) NC + be]: assembled entry between row (n, al) and
// column (n + off(o), be); off(o) = (o%3 - 1, (o/3)%3 - 1, o/9 - 1).
template <int DIM>
__global__ __launch_bounds__(kB) void k_em_to_stencil(int N, const double* __restrict__ K, double* __restrict__ S) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, ND = NL * NC, NO = n_off<DIM>();
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  for (int64_t row = int64_t(blockIdx.x) * kB + threadIdx.x; row < nn * NC; row += int64_t(gridDim.x) * kB) {
    const int64_t n = row / NC;
    const int al = int(row % NC);
    int c[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r % ns);
      r /= ns;
    }
    double* out = S + row * (NO * NC);
    for (int o = 0; o < NO; ++o) {
      int m[DIM];
      bool ok = true;
      int oo = o;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        m[i] = c[i] + oo % 3 - 1;
        oo /= 3;
        ok &= (m[i] >= 0) & (m[i] <= N);
      }
      for (int be = 0; be < NC; ++be) {
        double entry = 0.0;
        if (ok) {
          for (int a = 0; a < NL; ++a) {
            int e[DIM];
            bool eok = true;
            int b = 0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              e[i] = c[i] - ((a >> i) & 1);
              eok &= (e[i] >= 0) & (e[i] < N);
              const int bi = m[i] - e[i];
              eok &= (bi == 0) | (bi == 1);
              b |= (bi & 1) << i;
            }
            if (!eok) continue;
            int64_t eid = 0, st = 1;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              eid += int64_t(e[i]) * st;
              st *= N;
            }
            entry += K[eid * ND * ND + (NC * a + al) * ND + NC * b + be];
          }
        }
        out[o * NC + be] = entry;
      }
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(kB) void k_st_matvec(int N, const double* __restrict__ S, const double* __restrict__ v,
                                                  double* __restrict__ y) {
  constexpr int NC = DIM + 1, NO = n_off<DIM>();
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  for (int64_t row = int64_t(blockIdx.x) * kB + threadIdx.x; row < nn * NC; row += int64_t(gridDim.x) * kB) {
    const int64_t n = row / NC;
    int c[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r % ns);
      r /= ns;
    }
    const double* srow = S + row * (NO * NC);
    double acc = 0.0;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      int64_t m = 0, st = 1;
      bool ok = true;
      int oo = o;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        const int mi = c[i] + oo % 3 - 1;
        oo /= 3;
        ok &= (mi >= 0) & (mi <= N);
        m += int64_t(mi) * st;
        st *= ns;
      }
      if (!ok) continue;
#pragma unroll
      for (int be = 0; be < NC; ++be) acc += srow[o * NC + be] * v[NC * m + be];
    }
    y[row] = acc;
  }
}

// Gershgorin bound of ||A|| (max row sum of |A|, as -min in the last slot)
// and g^T g in slot 0.
template <int DIM>
__global__ __launch_bounds__(kB) void k_rowabs(int64_t nrows, const double* __restrict__ S,
                                               const double* __restrict__ g, double* __restrict__ partials) {
  constexpr int NC = DIM + 1, NO = n_off<DIM>();
  __shared__ double sh[kNV][kB];
  double v[kNV];
  vinit(v);
  for (int64_t row = int64_t(blockIdx.x) * kB + threadIdx.x; row < nrows; row += int64_t(gridDim.x) * kB) {
    const double* srow = S + row * (NO * NC);
    double rs = 0.0;
    for (int j = 0; j < NO * NC; ++j) rs += fabs(srow[j]);
    v[kNV - 1] = fmin(v[kNV - 1], -rs);
    v[0] += g[row] * g[row];
  }
  bred(v, sh, partials + kNV * blockIdx.x);
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

template <int DIM>
int64_t stencil_doubles(int N) {
  int64_t nn = 1;
  for (int i = 0; i < DIM; ++i) nn *= (N + 1);
  return nn * (DIM + 1) * n_off<DIM>() * (DIM + 1);
}

}  // namespace

size_t mprgp_work_doubles(int dim, int N) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  const int64_t n = nn * (dim + 1);
  const int64_t st = dim == 3 ? stencil_doubles<3>(N) : stencil_doubles<2>(N);
  return size_t(5 * n + n * (dim + 1) + st + kNV * 1024 + 2 * kNV + 16);
}

hipError_t run_mprgp(int dim, int N, const double* K, const uint8_t* dir, const double* g, const double* lo,
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
  double* D = Ad + n;  // node diagonal blocks for the fallback sweeps: n * (dim+1) doubles
  double* S = D + n * (dim + 1);
  double* part = S + (dim == 3 ? stencil_doubles<3>(N) : stencil_doubles<2>(N));
  double* red = part + kNV * 1024;
  const int nb = nblocks(n);
  const dim3 gb(nb), tb(kB);
  hipError_t e;
#define CK(x)                      \
  do {                             \
    e = (x);                       \
    if (e != hipSuccess) return e; \
  } while (0)
#define FETCH()                                                                     \
  do {                                                                              \
    hipLaunchKernelGGL(k_final, dim3(1), tb, 0, st, part, nb, red);                 \
    CK(hipGetLastError());                                                          \
    CK(hipMemcpyAsync(hs, red, kNV * sizeof(double), hipMemcpyDeviceToHost, st));   \
    CK(hipStreamSynchronize(st));                                                   \
  } while (0)
#define MATVEC(v, out)                                                                    \
  do {                                                                                    \
    if (dim == 3)                                                                         \
      hipLaunchKernelGGL(k_st_matvec<3>, dim3(nblocks(n)), tb, 0, st, N, S, v, out);     \
    else                                                                                  \
      hipLaunchKernelGGL(k_st_matvec<2>, dim3(nblocks(n)), tb, 0, st, N, S, v, out);     \
    CK(hipGetLastError());                                                                \
  } while (0)
  res->iterations = 0;
  res->status = 1;
  CK(launch_fill(n, 0.0, s, st));
  // assembled stencil, ||A|| bound and ||b||
  {
    int64_t gbk = (n + kB - 1) / kB;
    if (gbk > 262140) gbk = 262140;
    if (dim == 3)
      hipLaunchKernelGGL(k_em_to_stencil<3>, dim3(int(gbk)), tb, 0, st, N, K, S);
    else
      hipLaunchKernelGGL(k_em_to_stencil<2>, dim3(int(gbk)), tb, 0, st, N, K, S);
    CK(hipGetLastError());
  }
  if (dim == 3)
    hipLaunchKernelGGL(k_rowabs<3>, gb, tb, 0, st, n, S, g, part);
  else
    hipLaunchKernelGGL(k_rowabs<2>, gb, tb, 0, st, n, S, g, part);
  CK(hipGetLastError());
  FETCH();
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
    CK(launch_em_diag(dim, N, K, D, 0, st));
    CK(launch_em_pgs(dim, N, K, D, dir, g, lo, hi, s, fallback_sweeps, 0, st));
  } else if (it >= max_it && res->status != 0) {
    res->status = 1;
  }
  return hipSuccess;
#undef CK
#undef FETCH
#undef MATVEC
}

}  // namespace rmtr

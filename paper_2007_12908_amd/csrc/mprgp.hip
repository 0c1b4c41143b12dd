// MPRGP (Dostal's modified proportioning with reduced gradient projection)
// for the coarsest-level trust-region subproblem (Sec. 3.2.1):
//     min 1/2 s^T A s - b^T s,  lo <= s <= hi,   A = coarse Hessian, b = -g.
// The operator is the level's element-matrix Hessian.  The host drives the
// iteration; every reduction is a fixed-order two-stage tree, so the scalars
// (and the branch taken) do not depend on scheduling.
#include <math.h>

#include "rmtr_kernels.h"

namespace rmtr {
namespace {

constexpr int kB = 256;
constexpr int kNV = 4;  // reduced values per pass

int nblocks(int64_t n) {
  int64_t b = (n + kB - 1) / kB;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return int(b);
}

// Block reduction of kNV values: the first three are sums, the last a min.
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

__global__ __launch_bounds__(kB) void k_final(const double* __restrict__ partials, int nb, double* __restrict__ out) {
  __shared__ double sh[kNV][kB];
  double v[kNV] = {0.0, 0.0, 0.0, INFINITY};
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

// phi, beta and the sums ||phi + beta||^2, beta^T beta, phit^T phi.
__global__ __launch_bounds__(kB) void k_state(int64_t n, double abar, const double* __restrict__ s,
                                              const double* __restrict__ gr, const double* __restrict__ lo,
                                              const double* __restrict__ hi, double* __restrict__ phi,
                                              double* __restrict__ beta, double* __restrict__ partials) {
  __shared__ double sh[kNV][kB];
  double v[kNV] = {0.0, 0.0, 0.0, INFINITY};
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const double si = s[i], gi = gr[i], l = lo[i], h = hi[i];
    const double f = is_free(si, l, h) ? gi : 0.0;
    const double b = chop(si, gi, l, h);
    phi[i] = f;
    beta[i] = b;
    const double ft = f > 0.0 ? fmin((si - l) / abar, f) : fmax((si - h) / abar, f);
    v[0] += (f + b) * (f + b);
    v[1] += b * b;
    v[2] += ft * f;
  }
  bred(v, sh, partials + kNV * blockIdx.x);
}

// d^T A d, g^T d, and the largest feasible step along -d.
__global__ __launch_bounds__(kB) void k_dir(int64_t n, const double* __restrict__ s, const double* __restrict__ gr,
                                            const double* __restrict__ d, const double* __restrict__ Ad,
                                            const double* __restrict__ lo, const double* __restrict__ hi,
                                            double* __restrict__ partials) {
  __shared__ double sh[kNV][kB];
  double v[kNV] = {0.0, 0.0, 0.0, INFINITY};
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const double di = d[i];
    v[0] += di * Ad[i];
    v[1] += gr[i] * di;
    if (di > 0.0) v[3] = fmin(v[3], (s[i] - lo[i]) / di);
    if (di < 0.0) v[3] = fmin(v[3], (s[i] - hi[i]) / di);
  }
  bred(v, sh, partials + kNV * blockIdx.x);
}

// s -= a d; gr -= a Ad; optional clip to the box; phi = free gradient;
// partial phi^T Ad.
__global__ __launch_bounds__(kB) void k_step(int64_t n, double a, int clip, const double* __restrict__ d,
                                             const double* __restrict__ Ad, const double* __restrict__ lo,
                                             const double* __restrict__ hi, double* __restrict__ s,
                                             double* __restrict__ gr, double* __restrict__ phi,
                                             double* __restrict__ partials) {
  __shared__ double sh[kNV][kB];
  double v[kNV] = {0.0, 0.0, 0.0, INFINITY};
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    double si = s[i] - a * d[i];
    if (clip) si = fmin(fmax(si, lo[i]), hi[i]);
    const double gi = gr[i] - a * Ad[i];
    s[i] = si;
    gr[i] = gi;
    const double f = is_free(si, lo[i], hi[i]) ? gi : 0.0;
    phi[i] = f;
    v[0] += f * Ad[i];
  }
  bred(v, sh, partials + kNV * blockIdx.x);
}

// expansion: s = clip(s - abar phi)
__global__ __launch_bounds__(kB) void k_expand(int64_t n, double abar, const double* __restrict__ phi,
                                               const double* __restrict__ lo, const double* __restrict__ hi,
                                               double* __restrict__ s) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    s[i] = fmin(fmax(s[i] - abar * phi[i], lo[i]), hi[i]);
}

// gr = A s + g (A s in Ad); phi = free gradient
__global__ __launch_bounds__(kB) void k_regrad(int64_t n, const double* __restrict__ As, const double* __restrict__ g,
                                               const double* __restrict__ s, const double* __restrict__ lo,
                                               const double* __restrict__ hi, double* __restrict__ gr,
                                               double* __restrict__ phi) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const double gi = As[i] + g[i];
    gr[i] = gi;
    phi[i] = is_free(s[i], lo[i], hi[i]) ? gi : 0.0;
  }
}

// p = phi - bet p
__global__ __launch_bounds__(kB) void k_pupd(int64_t n, double bet, const double* __restrict__ phi,
                                             double* __restrict__ p) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    p[i] = phi[i] - bet * p[i];
}

__global__ __launch_bounds__(kB) void k_clip(int64_t n, const double* __restrict__ lo, const double* __restrict__ hi,
                                             double* __restrict__ s) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    s[i] = fmin(fmax(s[i], lo[i]), hi[i]);
}

// Row sums of |A| of the assembled element-matrix operator (Gershgorin bound
// of ||A||), reduced as a max in the last slot; the sums of g^T g in slot 0.
template <int DIM>
__global__ __launch_bounds__(kB) void k_rowabs(int N, const double* __restrict__ K, const double* __restrict__ g,
                                               double* __restrict__ partials) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, ND = NL * NC;
  __shared__ double sh[kNV][kB];
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  double v[kNV] = {0.0, 0.0, 0.0, INFINITY};
  for (int64_t n = int64_t(blockIdx.x) * kB + threadIdx.x; n < nn; n += int64_t(gridDim.x) * kB) {
    int c[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r % ns);
      r /= ns;
    }
    for (int k = 0; k < NC; ++k) {
      double rowsum = 0.0;
      // neighbour nodes m = c + off, off in {-1,0,1}^DIM, and their components
      for (int o = 0; o < (DIM == 3 ? 27 : 9); ++o) {
        int off[DIM], m[DIM];
        bool ok = true;
        int oo = o;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
          off[i] = oo % 3 - 1;
          oo /= 3;
          m[i] = c[i] + off[i];
          ok &= (m[i] >= 0) & (m[i] <= N);
        }
        if (!ok) continue;
        for (int l = 0; l < NC; ++l) {
          double entry = 0.0;
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
            entry += K[eid * ND * ND + (NC * a + k) * ND + NC * b + l];
          }
          rowsum += fabs(entry);
        }
      }
      v[3] = fmin(v[3], -rowsum);
      const double gi = g[NC * n + k];
      v[0] += gi * gi;
    }
  }
  bred(v, sh, partials + kNV * blockIdx.x);
}

}  // namespace

size_t mprgp_work_doubles(int dim, int N) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  const int64_t n = nn * (dim + 1);
  return size_t(5 * n + n * (dim + 1) + kNV * 1024 + 2 * kNV + 16);
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
  double* part = D + n * (dim + 1);
  double* red = part + kNV * 1024;
  const int nb = nblocks(n);
  const int nbn = nblocks(nn);
  hipError_t e;
#define CK(x)                              \
  do {                                     \
    e = (x);                               \
    if (e != hipSuccess) return e;         \
  } while (0)
#define FETCH()                                                                             \
  do {                                                                                      \
    CK(hipMemcpyAsync(hs, red, kNV * sizeof(double), hipMemcpyDeviceToHost, st));         \
    CK(hipStreamSynchronize(st));                                                           \
  } while (0)
  res->iterations = 0;
  res->status = 1;
  // s = 0 start; ||A|| bound and ||b||
  CK(launch_fill(n, 0.0, s, st));
  if (dim == 3)
    hipLaunchKernelGGL(k_rowabs<3>, dim3(nbn), dim3(kB), 0, st, N, K, g, part);
  else
    hipLaunchKernelGGL(k_rowabs<2>, dim3(nbn), dim3(kB), 0, st, N, K, g, part);
  CK(hipGetLastError());
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kB), 0, st, part, nbn, red);
  FETCH();
  const double normA = -hs[3];
  const double bnorm = sqrt(hs[0]);
  if (!(normA > 0.0)) {
    res->status = 0;
    return hipSuccess;
  }
  const double abar = 1.9 / normA;
  const double tol = rtol * fmax(bnorm, 1e-300);
  // gr = A s - b = g (s = 0)
  CK(hipMemcpyAsync(gr, g, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_state, dim3(nb), dim3(kB), 0, st, n, abar, s, gr, lo, hi, phi, beta, part);
  CK(hipGetLastError());
  CK(hipMemcpyAsync(p, phi, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kB), 0, st, part, nb, red);
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
      CK(launch_em_hessvec(dim, N, K, p, Ad, dir, 0, st));
      hipLaunchKernelGGL(k_dir, dim3(nb), dim3(kB), 0, st, n, s, gr, p, Ad, lo, hi, part);
      CK(hipGetLastError());
      hipLaunchKernelGGL(k_final, dim3(1), dim3(kB), 0, st, part, nb, red);
      FETCH();
      const double pAp = hs[0], gp = hs[1], af = hs[3];
      if (!(pAp > 0.0)) {
        negcurv = true;
        break;
      }
      const double acg = gp / pAp;
      if (acg <= af) {
        hipLaunchKernelGGL(k_step, dim3(nb), dim3(kB), 0, st, n, acg, 0, p, Ad, lo, hi, s, gr, phi, part);
        CK(hipGetLastError());
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kB), 0, st, part, nb, red);
        FETCH();
        const double bet = hs[0] / pAp;
        hipLaunchKernelGGL(k_pupd, dim3(nb), dim3(kB), 0, st, n, bet, phi, p);
        CK(hipGetLastError());
      } else {
        hipLaunchKernelGGL(k_step, dim3(nb), dim3(kB), 0, st, n, af, 0, p, Ad, lo, hi, s, gr, phi, part);
        CK(hipGetLastError());
        hipLaunchKernelGGL(k_expand, dim3(nb), dim3(kB), 0, st, n, abar, phi, lo, hi, s);
        CK(hipGetLastError());
        CK(launch_em_hessvec(dim, N, K, s, Ad, dir, 0, st));
        hipLaunchKernelGGL(k_regrad, dim3(nb), dim3(kB), 0, st, n, Ad, g, s, lo, hi, gr, phi);
        CK(hipGetLastError());
        CK(hipMemcpyAsync(p, phi, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      }
    } else {
      // proportioning step along the chopped gradient
      CK(launch_em_hessvec(dim, N, K, beta, Ad, dir, 0, st));
      hipLaunchKernelGGL(k_dir, dim3(nb), dim3(kB), 0, st, n, s, gr, beta, Ad, lo, hi, part);
      CK(hipGetLastError());
      hipLaunchKernelGGL(k_final, dim3(1), dim3(kB), 0, st, part, nb, red);
      FETCH();
      const double dAd = hs[0], gd = hs[1], af = hs[3];
      if (!(dAd > 0.0)) {
        negcurv = true;
        break;
      }
      const double a = fmin(gd / dAd, af);
      hipLaunchKernelGGL(k_step, dim3(nb), dim3(kB), 0, st, n, a, 1, beta, Ad, lo, hi, s, gr, phi, part);
      CK(hipGetLastError());
      CK(hipMemcpyAsync(p, phi, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_state, dim3(nb), dim3(kB), 0, st, n, abar, s, gr, lo, hi, phi, beta, part);
    CK(hipGetLastError());
    // k_state rewrites phi from the same s and gr; p was set from it above
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kB), 0, st, part, nb, red);
    FETCH();
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
}

}  // namespace rmtr

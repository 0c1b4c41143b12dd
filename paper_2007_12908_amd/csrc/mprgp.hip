// MPRGP (Dostal's modified proportioning with reduced gradient projection)
// for the coarsest-level trust-region subproblem (Sec. 3.2.1):
//     min 1/2 s^T A s - b^T s,  lo <= s <= hi,   A = coarse Hessian, b = -g.
// The level's element matrices are first assembled into a 3^d-point block
// stencil (stencil_kernels.hip), so every matrix-vector product is a
// row-parallel pass over contiguous rows.  The
// host drives the iteration and reads two sets of reduced scalars per
// iteration.  The products A d are fused with the row-local work that
// consumes them; each workgroup writes its partial sums, and a
// one-workgroup kernel adds them in a fixed order into host-mapped memory,
// so the scalars (and the branch taken) do not depend on scheduling.
#include <math.h>

#include "rmtr_kernels.h"
#include "stencil_layout.h"

namespace rmtr {
namespace {

constexpr int kB = 256;
constexpr int kMvB = 3 * kChunk;  // fused products: one wavefront per neighbour plane
constexpr int kNV = 5;            // reduced values per pass: four sums and one min
constexpr int kMaxBlocks = 1024;

int nblocks(int64_t n, int per_block) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return int(b);
}

__device__ inline void vinit(double (&v)[kNV]) {
#pragma unroll
  for (int k = 0; k < kNV - 1; ++k) v[k] = 0.0;
  v[kNV - 1] = INFINITY;
}

__device__ inline double vop(int k, double a, double b) { return k == kNV - 1 ? fmin(a, b) : a + b; }

// reduce v over the workgroup (butterfly in each wavefront, then the
// wavefronts in order); the result is valid in thread 0
template <int NW>
__device__ inline void block_reduce(double (&v)[kNV], double (*sh)[kNV]) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < kNV; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] = vop(k, v[k], __shfl_xor(v[k], off));
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < kNV; ++k) sh[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      double r = sh[0][k];
#pragma unroll
      for (int i = 1; i < NW; ++i) r = vop(k, r, sh[i][k]);
      v[k] = r;
    }
}

// workgroup partials of v at partials[kNV blockIdx.x + k]
template <int NW>
__device__ inline void block_partials(double (&v)[kNV], double* __restrict__ partials) {
  __shared__ double sh[NW][kNV];
  block_reduce<NW>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < kNV; ++k) partials[kNV * blockIdx.x + k] = v[k];
}

// fixed-order sum of nb partials into out[0 .. kNV) (host-mapped), then the
// pass's sequence number q into *seq (host-mapped), released at system
// scope after the sums
__global__ __launch_bounds__(kB) void k_final(const double* __restrict__ partials, int nb, double* __restrict__ out,
                                              unsigned long long* seq, unsigned long long q) {
  __shared__ double sh[kB / 64][kNV];
  double v[kNV];
  vinit(v);
  for (int i = threadIdx.x; i < nb; i += kB)
#pragma unroll
    for (int k = 0; k < kNV; ++k) v[k] = vop(k, v[k], partials[kNV * i + k]);
  block_reduce<kB / 64>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kNV; ++k) out[k] = v[k];
    __hip_atomic_store(seq, q, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
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
// phi^T Ad (when Ad is given); phi and beta are written, and phi also to
// pout when given.
__device__ inline void state_terms(double abar, double si, double gi, double l, double h, double* phi, double* beta,
                                   double* pout, int64_t i, const double* Ad, double (&v)[kNV]) {
  const double f = is_free(si, l, h) ? gi : 0.0;
  const double b = chop(si, gi, l, h);
  phi[i] = f;
  beta[i] = b;
  if (pout) pout[i] = f;
  const double ft = f > 0.0 ? fmin((si - l) / abar, f) : fmax((si - h) / abar, f);
  v[0] += (f + b) * (f + b);
  v[1] += b * b;
  v[2] += ft * f;
  if (Ad) v[3] += f * Ad[i];
}

__global__ __launch_bounds__(kB) void k_state(int64_t n, double abar, const double* __restrict__ s,
                                              const double* __restrict__ gr, const double* __restrict__ lo,
                                              const double* __restrict__ hi, double* __restrict__ phi,
                                              double* __restrict__ beta, double* __restrict__ p, double* __restrict__ partials) {
  double v[kNV];
  vinit(v);
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    state_terms(abar, s[i], gr[i], lo[i], hi[i], phi, beta, p, i, nullptr, v);
  block_partials<kB / 64>(v, partials);
}

// Fused product and row-local pass over the rows of A (al-major order, 64
// rows per workgroup, one wavefront per neighbour plane):
//   MODE 0: Ad = A d; d^T A d, g^T d (slots 0, 1) and the largest feasible
//           step along -d (min slot);
//   MODE 1: gr = A d + g (d = s); the state sums of (s, gr), phi also to p.
template <int DIM, int MODE>
__global__ __launch_bounds__(kMvB) void k_mv_fused(Colours cg, const double* __restrict__ S,
                                                   const double* __restrict__ d, double* __restrict__ Ad,
                                                   const double* __restrict__ g, const double* __restrict__ s,
                                                   double* __restrict__ gr, const double* __restrict__ lo,
                                                   const double* __restrict__ hi, double abar,
                                                   double* __restrict__ phi, double* __restrict__ beta,
                                                   double* __restrict__ p, double* __restrict__ partials) {
  constexpr int NC = DIM + 1;
  __shared__ double part[2][kChunk];
  const int64_t nodes = cg.base[1 << DIM], rows = nodes * NC;
  const int lane = threadIdx.x % kChunk, pl = threadIdx.x / kChunk;
  double v[kNV];
  vinit(v);
  for (int64_t r0 = int64_t(blockIdx.x) * kChunk; r0 < rows; r0 += int64_t(gridDim.x) * kChunk) {
    const int64_t it = r0 + lane;
    double acc = 0.0;
    int64_t n = 0;
    int al = 0;
    if (it < rows) {
      al = int(it / nodes);
      acc = st_row_plane<DIM>(cg, S, d, it % nodes, al, pl, n);
    }
    if (pl > 0) part[pl - 1][lane] = acc;
    __syncthreads();
    if (pl == 0 && it < rows) {
      const int64_t i = NC * n + al;
      const double a = (acc + part[0][lane]) + part[1][lane];
      if (MODE == 0) {
        Ad[i] = a;
        const double di = d[i];
        v[0] += di * a;
        v[1] += gr[i] * di;
        if (di > 0.0) v[kNV - 1] = fmin(v[kNV - 1], (s[i] - lo[i]) / di);
        if (di < 0.0) v[kNV - 1] = fmin(v[kNV - 1], (s[i] - hi[i]) / di);
      } else {
        const double gi = a + g[i];
        gr[i] = gi;
        state_terms(abar, s[i], gi, lo[i], hi[i], phi, beta, p, i, nullptr, v);
      }
    }
    __syncthreads();
  }
  block_partials<kMvB / 64>(v, partials);
}

// s -= a d (clipped to the box if clip); gr -= a Ad; then the state sums
// of the new point, with phi^T Ad in slot 3 (phi also to p when given).
// d may be beta: each element is read before it is rewritten.
__global__ __launch_bounds__(kB) void k_step_state(int64_t n, double a, int clip, double abar, const double* d,
                                                   const double* __restrict__ Ad, const double* __restrict__ lo,
                                                   const double* __restrict__ hi, double* __restrict__ s,
                                                   double* __restrict__ gr, double* __restrict__ phi, double* beta,
                                                   double* p, double* __restrict__ partials) {
  double v[kNV];
  vinit(v);
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    double si = s[i] - a * d[i];
    if (clip) si = fmin(fmax(si, lo[i]), hi[i]);
    const double gi = gr[i] - a * Ad[i];
    s[i] = si;
    gr[i] = gi;
    state_terms(abar, si, gi, lo[i], hi[i], phi, beta, p, i, Ad, v);
  }
  block_partials<kB / 64>(v, partials);
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

// p = phi - bet p
__global__ __launch_bounds__(kB) void k_pupd(int64_t n, double bet, const double* __restrict__ phi,
                                             double* __restrict__ p) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    p[i] = phi[i] - bet * p[i];
}

// Wait until k_final has published sequence number q: a bounded busy wait on
// the host-mapped word, which ends sooner than a stream synchronisation for
// these short passes; after the bound the stream is synchronised, so a failed
// launch still reports its error.
hipError_t wait_for(const unsigned long long* seq, unsigned long long q, hipStream_t st) {
  for (int i = 0; i < (1 << 22); ++i)
    if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == q) return hipSuccess;
  return hipStreamSynchronize(st);
}

}  // namespace

size_t mprgp_work_doubles(int dim, int N) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  const int64_t n = nn * (dim + 1);
  return size_t(5 * n + kNV * kMaxBlocks + 2 * kNV + 16);
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
  const Colours cg = colours(dim, N);
  const dim3 ge(nblocks(n, kB)), te(kB);
  const dim3 gm(nblocks(n, kChunk)), tm(kMvB);
  hipError_t e;
#define CK(x)                      \
  do {                             \
    e = (x);                       \
    if (e != hipSuccess) return e; \
  } while (0)
  // the final sum of a pass's nbk partials is written straight into the
  // (mapped, coherent) host memory hs[0 .. kNV), followed by the pass's
  // sequence number in hs[8]
  unsigned long long* seq = reinterpret_cast<unsigned long long*>(hs + 8);
  unsigned long long q = __atomic_load_n(seq, __ATOMIC_ACQUIRE);
#define FETCH(nbk)                                                                  \
  do {                                                                              \
    ++q;                                                                            \
    hipLaunchKernelGGL(k_final, dim3(1), te, 0, st, part, int(nbk), hs, seq, q);    \
    CK(hipGetLastError());                                                          \
    CK(wait_for(seq, q, st));                                                       \
  } while (0)
  res->iterations = 0;
  res->status = 1;
  CK(launch_fill(n, 0.0, s, st));
  // ||A|| bound and ||b||
  {
    int nbr = 0;
    CK(launch_st_rowabs(dim, N, S, g, part, &nbr, st));
    FETCH(nbr);
  }
  const double normA = -hs[kNV - 1];
  const double bnorm = sqrt(hs[0]);
  if (!(normA > 0.0)) {
    res->status = 0;
    return hipSuccess;
  }
  const double abar = 1.9 / normA;
  const double tol = rtol * fmax(bnorm, 1e-300);
  // Ad = A d with the direction sums (mode 0), or gr = A s + g with the
  // state sums and p = phi (mode 1)
  auto fused = [&](int mode, const double* dv) -> hipError_t {
    if (dim == 3) {
      if (mode == 0)
        hipLaunchKernelGGL((k_mv_fused<3, 0>), gm, tm, 0, st, cg, S, dv, Ad, g, s, gr, lo, hi, abar, phi, beta, p,
                           part);
      else
        hipLaunchKernelGGL((k_mv_fused<3, 1>), gm, tm, 0, st, cg, S, dv, Ad, g, s, gr, lo, hi, abar, phi, beta, p,
                           part);
    } else {
      if (mode == 0)
        hipLaunchKernelGGL((k_mv_fused<2, 0>), gm, tm, 0, st, cg, S, dv, Ad, g, s, gr, lo, hi, abar, phi, beta, p,
                           part);
      else
        hipLaunchKernelGGL((k_mv_fused<2, 1>), gm, tm, 0, st, cg, S, dv, Ad, g, s, gr, lo, hi, abar, phi, beta, p,
                           part);
    }
    return hipGetLastError();
  };
  // s = 0: gr = A s - b = g; p = phi
  CK(hipMemcpyAsync(gr, g, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_state, ge, te, 0, st, n, abar, s, gr, lo, hi, phi, beta, p, part);
  CK(hipGetLastError());
  FETCH(ge.x);
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
      CK(fused(0, p));
      FETCH(gm.x);
      const double pAp = hs[0], gp = hs[1], af = hs[kNV - 1];
      if (!(pAp > 0.0)) {
        negcurv = true;
        break;
      }
      const double acg = gp / pAp;
      if (acg <= af) {
        hipLaunchKernelGGL(k_step_state, ge, te, 0, st, n, acg, 0, abar, p, Ad, lo, hi, s, gr, phi, beta,
                           (double*)nullptr, part);
        CK(hipGetLastError());
        FETCH(ge.x);
        const double bet = hs[3] / pAp;
        hipLaunchKernelGGL(k_pupd, ge, te, 0, st, n, bet, phi, p);
        CK(hipGetLastError());
      } else {
        hipLaunchKernelGGL(k_expand, ge, te, 0, st, n, af, abar, p, Ad, lo, hi, s, gr);
        CK(hipGetLastError());
        CK(fused(1, s));
        FETCH(gm.x);
      }
    } else {
      // proportioning step along the chopped gradient, kept inside the box
      CK(fused(0, beta));
      FETCH(gm.x);
      const double dAd = hs[0], gd = hs[1], af = hs[kNV - 1];
      if (!(dAd > 0.0)) {
        negcurv = true;
        break;
      }
      const double a = fmin(gd / dAd, af);
      hipLaunchKernelGGL(k_step_state, ge, te, 0, st, n, a, 1, abar, beta, Ad, lo, hi, s, gr, phi, beta, p, part);
      CK(hipGetLastError());
      FETCH(ge.x);
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
}

}  // namespace rmtr

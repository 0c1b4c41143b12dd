// MPRGP (Dostal's modified proportioning with reduced gradient projection)
// for the coarsest-level trust-region subproblem (Sec. 3.2.1):
//     min 1/2 s^T A s - b^T s,  lo <= s <= hi,   A = coarse Hessian, b = -g.
// The level's element matrices are first assembled into a 3^d-point block
// stencil (stencil_kernels.hip), so every matrix-vector product is a
// row-parallel pass over contiguous rows.  The products A d are fused with
// the row-local work that consumes them; each workgroup writes its partial
// sums, and one-workgroup kernels add them in a fixed order and take the
// iteration's decisions on the device (so the scalars, and the branch taken,
// do not depend on scheduling).  The host enqueues the iterations in
// batches and reads back only whether the iteration has stopped.
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

// Iteration state kept on the device, so the host enqueues iterations in
// batches and reads back only whether the iteration has stopped.  The
// decisions are the host loop's, taken by one-workgroup kernels from the
// fixed-order sums of the passes before them.
struct MpCtl {
  double st[kNV];   // state sums: ||phi + beta||^2, beta^T beta, phit^T phi, phi^T Ad
  double dr[kNV];   // direction sums: d^T A d, g^T d, largest feasible step (min slot)
  double a, pAp, bet, tol;
  int mode;         // direction of this iteration: 0 p (conjugate gradient), 1 beta (proportioning)
  int kind;         // step taken: 1 CG step, 2 expansion, 3 proportioning, 0 none
  int it, status, stop, max_it;
};

__device__ inline void sum_partials(const double* __restrict__ partials, int nb, double (&v)[kNV]) {
  __shared__ double sh[kB / 64][kNV];
  vinit(v);
  for (int i = threadIdx.x; i < nb; i += kB)
#pragma unroll
    for (int k = 0; k < kNV; ++k) v[k] = vop(k, v[k], partials[kNV * i + k]);
  block_reduce<kB / 64>(v, sh);
}

// After a state pass: its sums, the CG coefficient of a CG step, then the
// test at the top of the next iteration (iteration cap, then the projected
// gradient), and the next direction.  When q > 0 the stop flag, iteration
// count and status go to host-mapped memory, followed by sequence word q.
__global__ __launch_bounds__(kB) void k_mp_state(MpCtl* ctl, const double* __restrict__ partials, int nb_step,
                                                 int nb_mv, double* hs, unsigned long long* seq,
                                                 unsigned long long q) {
  const bool run = !ctl->stop;
  double v[kNV];
  if (run) sum_partials(partials, ctl->kind == 2 ? nb_mv : nb_step, v);
  if (threadIdx.x == 0) {
    if (run) {
#pragma unroll
      for (int k = 0; k < kNV; ++k) ctl->st[k] = v[k];
      if (ctl->kind == 1) ctl->bet = v[3] / ctl->pAp;
      if (ctl->it >= ctl->max_it) {
        ctl->status = 1;
        ctl->stop = 1;
      } else if (sqrt(v[0]) <= ctl->tol) {
        ctl->status = 0;
        ctl->stop = 1;
      } else {
        ++ctl->it;
        ctl->mode = v[1] <= v[2] ? 0 : 1;
      }
    }
    if (q) {
      hs[0] = double(ctl->stop);
      hs[1] = double(ctl->it);
      hs[2] = double(ctl->status);
      __hip_atomic_store(seq, q, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// After the product along the direction: the step length and kind, or the
// stop on non-positive curvature.
__global__ __launch_bounds__(kB) void k_mp_dir(MpCtl* ctl, const double* __restrict__ partials, int nb) {
  if (ctl->stop) return;
  double v[kNV];
  sum_partials(partials, nb, v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kNV; ++k) ctl->dr[k] = v[k];
    const double dAd = v[0], gd = v[1], af = v[kNV - 1];
    if (!(dAd > 0.0)) {
      ctl->status = 2;
      ctl->stop = 1;
      ctl->kind = 0;
    } else if (ctl->mode == 0) {
      const double acg = gd / dAd;
      ctl->pAp = dAd;
      if (acg <= af) {
        ctl->kind = 1;
        ctl->a = acg;
      } else {
        ctl->kind = 2;
        ctl->a = af;
      }
    } else {
      ctl->kind = 3;
      ctl->a = fmin(gd / dAd, af);
    }
  }
}

__global__ void k_mp_init(MpCtl* ctl, double tol, int max_it) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kNV; ++k) ctl->st[k] = ctl->dr[k] = 0.0;
    ctl->a = ctl->pAp = ctl->bet = 0.0;
    ctl->tol = tol;
    ctl->mode = ctl->kind = ctl->it = ctl->stop = 0;
    ctl->status = 1;
    ctl->max_it = max_it;
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
//   With a control block (ctl != nullptr) the pass runs only while the
//   iteration has not stopped: MODE 0 along p or beta as ctl->mode says,
//   MODE 1 only after an expansion step.
template <int DIM, int MODE>
__global__ __launch_bounds__(kMvB) void k_mv_fused(Colours cg, const double* __restrict__ S,
                                                   const double* d, double* __restrict__ Ad,
                                                   const double* __restrict__ g, const double* __restrict__ s,
                                                   double* __restrict__ gr, const double* __restrict__ lo,
                                                   const double* __restrict__ hi, double abar,
                                                   double* phi, double* beta,
                                                   double* p, double* __restrict__ partials,
                                                   const MpCtl* ctl) {
  if (ctl) {
    if (ctl->stop || (MODE == 1 && ctl->kind != 2)) return;
    if (MODE == 0) d = ctl->mode == 0 ? p : beta;
  }
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

// The step of a device-driven iteration as ctl->kind says: CG step along p
// (state sums with phi^T Ad), proportioning step along beta clipped to the
// box (state sums, p = phi), or the expansion step (no sums; the next pass
// recomputes the state).
__global__ __launch_bounds__(kB) void k_mp_step(const MpCtl* ctl, int64_t n, double abar, const double* __restrict__ Ad,
                                                const double* __restrict__ lo, const double* __restrict__ hi,
                                                double* __restrict__ s, double* __restrict__ gr,
                                                double* __restrict__ phi, double* beta, double* p,
                                                double* __restrict__ partials) {
  if (ctl->stop) return;
  const int kind = ctl->kind;
  const double a = ctl->a;
  if (kind == 2) {
    for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
      const double si = s[i] - a * p[i];
      const double gi = gr[i] - a * Ad[i];
      const double f = is_free(si, lo[i], hi[i]) ? gi : 0.0;
      s[i] = fmin(fmax(si - abar * f, lo[i]), hi[i]);
    }
    return;
  }
  if (kind != 1 && kind != 3) return;
  const double* d = kind == 1 ? p : beta;
  double* pout = kind == 3 ? p : nullptr;
  const bool clip = kind == 3;
  double v[kNV];
  vinit(v);
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    double si = s[i] - a * d[i];
    if (clip) si = fmin(fmax(si, lo[i]), hi[i]);
    const double gi = gr[i] - a * Ad[i];
    s[i] = si;
    gr[i] = gi;
    state_terms(abar, si, gi, lo[i], hi[i], phi, beta, pout, i, Ad, v);
  }
  block_partials<kB / 64>(v, partials);
}

// p = phi - bet p after a CG step of a device-driven iteration
__global__ __launch_bounds__(kB) void k_mp_pupd(const MpCtl* ctl, int64_t n, const double* __restrict__ phi,
                                                double* __restrict__ p) {
  if (ctl->stop || ctl->kind != 1) return;
  const double bet = ctl->bet;
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
  return size_t(5 * n + kNV * kMaxBlocks + 2 * kNV + 16 + (sizeof(MpCtl) + 7) / 8);
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
  // state sums and p = phi (mode 1); with ctl, as the device-side state says
  auto fused = [&](int mode, const double* dv, const MpCtl* ctl) -> hipError_t {
    if (dim == 3) {
      if (mode == 0)
        hipLaunchKernelGGL((k_mv_fused<3, 0>), gm, tm, 0, st, cg, S, dv, Ad, g, s, gr, lo, hi, abar, phi, beta, p,
                           part, ctl);
      else
        hipLaunchKernelGGL((k_mv_fused<3, 1>), gm, tm, 0, st, cg, S, dv, Ad, g, s, gr, lo, hi, abar, phi, beta, p,
                           part, ctl);
    } else {
      if (mode == 0)
        hipLaunchKernelGGL((k_mv_fused<2, 0>), gm, tm, 0, st, cg, S, dv, Ad, g, s, gr, lo, hi, abar, phi, beta, p,
                           part, ctl);
      else
        hipLaunchKernelGGL((k_mv_fused<2, 1>), gm, tm, 0, st, cg, S, dv, Ad, g, s, gr, lo, hi, abar, phi, beta, p,
                           part, ctl);
    }
    return hipGetLastError();
  };
  // s = 0: gr = A s - b = g; p = phi
  CK(hipMemcpyAsync(gr, g, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_state, ge, te, 0, st, n, abar, s, gr, lo, hi, phi, beta, p, part);
  CK(hipGetLastError());
  // The iterations run on the device: per iteration the product along the
  // direction, the step decision, the step, the product after an expansion,
  // the state decision and the CG update of p, each pass skipping itself
  // when the iteration has stopped or its step is not the one taken.  The
  // host enqueues them in batches and reads back, after each batch, whether
  // the iteration stopped.
  MpCtl* ctl = reinterpret_cast<MpCtl*>(part + kNV * kMaxBlocks);
  hipLaunchKernelGGL(k_mp_init, dim3(1), dim3(64), 0, st, ctl, tol, max_it);
  CK(hipGetLastError());
  hipLaunchKernelGGL(k_mp_state, dim3(1), te, 0, st, ctl, part, int(ge.x), int(gm.x), hs, seq, 0ull);
  CK(hipGetLastError());
  constexpr int kBatch = 10;
  for (;;) {
    for (int b = 0; b < kBatch; ++b) {
      CK(fused(0, p, ctl));
      hipLaunchKernelGGL(k_mp_dir, dim3(1), te, 0, st, ctl, part, int(gm.x));
      hipLaunchKernelGGL(k_mp_step, ge, te, 0, st, ctl, n, abar, Ad, lo, hi, s, gr, phi, beta, p, part);
      CK(hipGetLastError());
      CK(fused(1, s, ctl));
      const unsigned long long qb = b == kBatch - 1 ? ++q : 0ull;
      hipLaunchKernelGGL(k_mp_state, dim3(1), te, 0, st, ctl, part, int(ge.x), int(gm.x), hs, seq, qb);
      hipLaunchKernelGGL(k_mp_pupd, ge, te, 0, st, ctl, n, phi, p);
      CK(hipGetLastError());
    }
    CK(wait_for(seq, q, st));
    if (hs[0] != 0.0) break;
  }
  const int it = int(hs[1]);
  res->status = int(hs[2]);
  const bool negcurv = res->status == 2;
  res->iterations = it;
  if (negcurv) CK(launch_st_pgs(dim, N, S, dir, g, lo, hi, s, fallback_sweeps, 0, st));
  return hipSuccess;
#undef CK
#undef FETCH
}

}  // namespace rmtr

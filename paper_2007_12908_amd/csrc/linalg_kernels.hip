// Vector kernels of the RMTR loop: deterministic dot products (fixed-order
// two-stage tree), the stopping measure chi, trust-region boxes, copies and
// conversions.
#include "rmtr_kernels.h"

namespace rmtr {
namespace {

constexpr int kB = 256;

int nblocks(int64_t n) {
  int64_t b = (n + kB - 1) / kB;
  if (b < 1) b = 1;
  if (b > kMaxPartials) b = kMaxPartials;
  return int(b);
}

int gridn(int64_t n) {
  int64_t b = (n + kB - 1) / kB;
  if (b < 1) b = 1;
  if (b > 262140) b = 262140;
  return int(b);
}

__device__ inline double bsum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(kB) void k_dot(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                            double* __restrict__ partials) {
  __shared__ double sh[kB];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) acc += a[i] * b[i];
  double t = bsum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// max |a_i|: per-block maxima, then one block takes the maximum of those
__global__ __launch_bounds__(kB) void k_amax(int64_t n, const double* __restrict__ a, double* __restrict__ partials) {
  __shared__ double sh[kB];
  double m = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) m = fmax(m, fabs(a[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kB) void k_amax_final(const double* __restrict__ partials, int n, double* __restrict__ out) {
  __shared__ double sh[kB];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) m = fmax(m, partials[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// chi^2 = || P_F(x - g) - x ||^2 over free dofs; F: c_lower <= c <= 1.
template <int DIM>
__global__ __launch_bounds__(kB) void k_chi(int N, const double* __restrict__ x, const double* __restrict__ g,
                                            const double* __restrict__ cl, const uint8_t* __restrict__ dir,
                                            double* __restrict__ partials) {
  __shared__ double sh[kB];
  constexpr int NC = DIM + 1;
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  double acc = 0.0;
  for (int64_t n = int64_t(blockIdx.x) * kB + threadIdx.x; n < nn; n += int64_t(gridDim.x) * kB) {
    int c[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r % ns);
      r /= ns;
    }
    const uint8_t mk = dir ? dir[n] : default_mask<DIM>(c, N);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (mk & (1u << k)) continue;
      double v;
      if (k < DIM) {
        v = -g[NC * n + k];
      } else {
        const double xc = x[NC * n + k];
        double t = xc - g[NC * n + k];
        t = t < cl[n] ? cl[n] : t;
        t = t > 1.0 ? 1.0 : t;
        v = t - xc;
      }
      acc += v * v;
    }
  }
  double t = bsum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kB) void k_axpy(int64_t n, double alpha, const double* __restrict__ x,
                                             double* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) y[i] += alpha * x[i];
}

// out = alpha a + beta b + c   (b or c may be null)
__global__ __launch_bounds__(kB) void k_add_scaled(int64_t n, const double* __restrict__ a, double alpha,
                                                   const double* __restrict__ b, double beta,
                                                   const double* __restrict__ c, double* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    double v = alpha * a[i];
    if (b) v += beta * b[i];
    if (c) v += c[i];
    out[i] = v;
  }
}

// lo = max(Lb - x, -delta), hi = min(Ub - x, delta); Dirichlet dofs 0.
template <int DIM>
__global__ __launch_bounds__(kB) void k_step_box(int N, const double* __restrict__ x, const double* __restrict__ Lb,
                                                 const double* __restrict__ Ub, double delta,
                                                 const uint8_t* __restrict__ dir, double* __restrict__ lo,
                                                 double* __restrict__ hi) {
  constexpr int NC = DIM + 1;
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  for (int64_t n = int64_t(blockIdx.x) * kB + threadIdx.x; n < nn; n += int64_t(gridDim.x) * kB) {
    int c[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r % ns);
      r /= ns;
    }
    const uint8_t mk = dir ? dir[n] : default_mask<DIM>(c, N);
    // a node's components are read and written together (3D: 32 bytes)
    double xv[NC], lv[NC], uv[NC], lo_v[NC], hi_v[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      xv[k] = x[NC * n + k];
      lv[k] = Lb[NC * n + k];
      uv[k] = Ub[NC * n + k];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const bool fixed = mk & (1u << k);
      lo_v[k] = fixed ? 0.0 : fmax(lv[k] - xv[k], -delta);
      hi_v[k] = fixed ? 0.0 : fmin(uv[k] - xv[k], delta);
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      lo[NC * n + k] = lo_v[k];
      hi[NC * n + k] = hi_v[k];
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(kB) void k_fine_bounds(int N, const double* __restrict__ cl, double* __restrict__ Lb,
                                                    double* __restrict__ Ub) {
  constexpr int NC = DIM + 1;
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  for (int64_t n = int64_t(blockIdx.x) * kB + threadIdx.x; n < nn; n += int64_t(gridDim.x) * kB) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      Lb[NC * n + k] = -INFINITY;
      Ub[NC * n + k] = INFINITY;
    }
    Lb[NC * n + DIM] = cl[n];
    Ub[NC * n + DIM] = 1.0;
  }
}

template <typename A, typename B>
__global__ __launch_bounds__(kB) void k_convert(int64_t n, const A* __restrict__ a, B* __restrict__ b) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) b[i] = B(a[i]);
}

template <int DIM>
__global__ __launch_bounds__(kB) void k_zero_masked(int N, double* __restrict__ v, const uint8_t* __restrict__ dir) {
  constexpr int NC = DIM + 1;
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  for (int64_t n = int64_t(blockIdx.x) * kB + threadIdx.x; n < nn; n += int64_t(gridDim.x) * kB) {
    int c[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r % ns);
      r /= ns;
    }
    const uint8_t mk = dir ? dir[n] : default_mask<DIM>(c, N);
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (mk & (1u << k)) v[NC * n + k] = 0.0;
  }
}

__global__ __launch_bounds__(kB) void k_fill(int64_t n, double v, double* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) out[i] = v;
}

__global__ __launch_bounds__(kB) void k_any_nonzero(int64_t n, const double* __restrict__ v, int* __restrict__ flag) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    if (v[i] != 0.0) *flag = 1;
}

__global__ __launch_bounds__(kB) void k_clamp(int64_t n, const double* __restrict__ lo, const double* __restrict__ hi,
                                              double* __restrict__ s) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB)
    s[i] = fmin(fmax(s[i], lo[i]), hi[i]);
}

// coarse scalar nodal field = fine values at nodes (2i, 2j, 2k)
template <int DIM, typename T>
__global__ __launch_bounds__(kB) void k_inject_scalar(int Nc, const T* __restrict__ f, T* __restrict__ c) {
  const int64_t nsc = Nc + 1, nsf = 2 * Nc + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= nsc;
  for (int64_t n = int64_t(blockIdx.x) * kB + threadIdx.x; n < nn; n += int64_t(gridDim.x) * kB) {
    int64_t r = n, m = 0, s = 1;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      m += 2 * (r % nsc) * s;
      r /= nsc;
      s *= nsf;
    }
    c[n] = f[m];
  }
}

}  // namespace

hipError_t launch_clamp(int64_t n, const double* lo, const double* hi, double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_clamp, dim3(gridn(n)), dim3(kB), 0, st, n, lo, hi, s);
  return hipGetLastError();
}

hipError_t launch_inject_scalar(int dim, int Nc, const double* fine, double* coarse, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (Nc + 1);
  if (dim == 3)
    hipLaunchKernelGGL((k_inject_scalar<3, double>), dim3(gridn(nn)), dim3(kB), 0, st, Nc, fine, coarse);
  else
    hipLaunchKernelGGL((k_inject_scalar<2, double>), dim3(gridn(nn)), dim3(kB), 0, st, Nc, fine, coarse);
  return hipGetLastError();
}

hipError_t launch_inject_mask(int dim, int Nc, const uint8_t* fine, uint8_t* coarse, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (Nc + 1);
  if (dim == 3)
    hipLaunchKernelGGL((k_inject_scalar<3, uint8_t>), dim3(gridn(nn)), dim3(kB), 0, st, Nc, fine, coarse);
  else
    hipLaunchKernelGGL((k_inject_scalar<2, uint8_t>), dim3(gridn(nn)), dim3(kB), 0, st, Nc, fine, coarse);
  return hipGetLastError();
}

hipError_t launch_dot(int64_t n, const double* a, const double* b, double* partials, double* out, hipStream_t st) {
  int nb = nblocks(n);
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kB), 0, st, n, a, b, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_partials(partials, nb, out, st);
}

hipError_t launch_amax(int64_t n, const double* a, double* partials, double* out, hipStream_t st) {
  int nb = nblocks(n);
  hipLaunchKernelGGL(k_amax, dim3(nb), dim3(kB), 0, st, n, a, partials);
  hipLaunchKernelGGL(k_amax_final, dim3(1), dim3(kB), 0, st, partials, nb, out);
  return hipGetLastError();
}

hipError_t launch_chi(int dim, int N, const double* x, const double* g, const double* c_lower, const uint8_t* dir,
                      double* partials, double* out, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  int nb = nblocks(nn);
  if (dim == 3)
    hipLaunchKernelGGL(k_chi<3>, dim3(nb), dim3(kB), 0, st, N, x, g, c_lower, dir, partials);
  else
    hipLaunchKernelGGL(k_chi<2>, dim3(nb), dim3(kB), 0, st, N, x, g, c_lower, dir, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_partials(partials, nb, out, st);
}

hipError_t launch_axpy(int64_t n, double alpha, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(gridn(n)), dim3(kB), 0, st, n, alpha, x, y);
  return hipGetLastError();
}

hipError_t launch_add_scaled(int64_t n, const double* a, double alpha, const double* b, double beta, const double* c,
                             double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_add_scaled, dim3(gridn(n)), dim3(kB), 0, st, n, a, alpha, b, beta, c, out);
  return hipGetLastError();
}

hipError_t launch_step_box(int dim, int N, const double* x, const double* Lb, const double* Ub, double delta,
                           const uint8_t* dir, double* lo, double* hi, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  if (dim == 3)
    hipLaunchKernelGGL(k_step_box<3>, dim3(gridn(nn)), dim3(kB), 0, st, N, x, Lb, Ub, delta, dir, lo, hi);
  else
    hipLaunchKernelGGL(k_step_box<2>, dim3(gridn(nn)), dim3(kB), 0, st, N, x, Lb, Ub, delta, dir, lo, hi);
  return hipGetLastError();
}

hipError_t launch_fine_bounds(int dim, int N, const double* c_lower, double* Lb, double* Ub, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  if (dim == 3)
    hipLaunchKernelGGL(k_fine_bounds<3>, dim3(gridn(nn)), dim3(kB), 0, st, N, c_lower, Lb, Ub);
  else
    hipLaunchKernelGGL(k_fine_bounds<2>, dim3(gridn(nn)), dim3(kB), 0, st, N, c_lower, Lb, Ub);
  return hipGetLastError();
}

hipError_t launch_convert(int64_t n, const void* src, int src_fp32, void* dst, int dst_fp32, hipStream_t st) {
  dim3 g(gridn(n));
  if (src_fp32 && dst_fp32)
    hipLaunchKernelGGL((k_convert<float, float>), g, dim3(kB), 0, st, n, (const float*)src, (float*)dst);
  else if (src_fp32)
    hipLaunchKernelGGL((k_convert<float, double>), g, dim3(kB), 0, st, n, (const float*)src, (double*)dst);
  else if (dst_fp32)
    hipLaunchKernelGGL((k_convert<double, float>), g, dim3(kB), 0, st, n, (const double*)src, (float*)dst);
  else
    hipLaunchKernelGGL((k_convert<double, double>), g, dim3(kB), 0, st, n, (const double*)src, (double*)dst);
  return hipGetLastError();
}

hipError_t launch_zero_masked(int dim, int N, double* v, const uint8_t* dir, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  if (dim == 3)
    hipLaunchKernelGGL(k_zero_masked<3>, dim3(gridn(nn)), dim3(kB), 0, st, N, v, dir);
  else
    hipLaunchKernelGGL(k_zero_masked<2>, dim3(gridn(nn)), dim3(kB), 0, st, N, v, dir);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(gridn(n)), dim3(kB), 0, st, n, v, out);
  return hipGetLastError();
}

hipError_t launch_any_nonzero(int64_t n, const double* v, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_any_nonzero, dim3(gridn(n)), dim3(kB), 0, st, n, v, flag);
  return hipGetLastError();
}

}  // namespace rmtr

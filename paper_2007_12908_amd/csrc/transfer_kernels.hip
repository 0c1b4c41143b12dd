// Level transfers (Sec. 3): prolongation I (nested Q1 interpolation),
// restriction R = I^T, injection P, and the monotone box restriction
// (max / min over the support of a coarse basis function).  Every sum runs
// over its terms in ascending node order and every weight is a power of two,
// so the results are reproducible bit for bit.
#include "rmtr_kernels.h"

namespace rmtr {
namespace {

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_prolong(int Nc, const T* __restrict__ xc, T* __restrict__ xf) {
  constexpr int NC = DIM + 1;
  const int Nf = 2 * Nc;
  const int64_t nsf = Nf + 1, nsc = Nc + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= nsf;
  for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < nn; n += int64_t(gridDim.x) * blockDim.x) {
    int f[DIM], lo[DIM], cnt[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      f[i] = int(r % nsf);
      r /= nsf;
      lo[i] = f[i] >> 1;
      cnt[i] = (f[i] & 1) ? 2 : 1;
    }
    T acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = T(0);
    // ascending coarse index: slowest direction outermost
    if constexpr (DIM == 3) {
      for (int bz = 0; bz < cnt[2]; ++bz)
        for (int by = 0; by < cnt[1]; ++by)
          for (int bx = 0; bx < cnt[0]; ++bx) {
            const T wgt = T((cnt[0] == 2 ? 0.5 : 1.0) * (cnt[1] == 2 ? 0.5 : 1.0) * (cnt[2] == 2 ? 0.5 : 1.0));
            const int64_t m = (lo[0] + bx) + nsc * ((lo[1] + by) + nsc * (lo[2] + bz));
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[k] += wgt * xc[NC * m + k];
          }
    } else {
      for (int by = 0; by < cnt[1]; ++by)
        for (int bx = 0; bx < cnt[0]; ++bx) {
          const T wgt = T((cnt[0] == 2 ? 0.5 : 1.0) * (cnt[1] == 2 ? 0.5 : 1.0));
          const int64_t m = (lo[0] + bx) + nsc * (lo[1] + by);
#pragma unroll
          for (int k = 0; k < NC; ++k) acc[k] += wgt * xc[NC * m + k];
        }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) xf[NC * n + k] = acc[k];
  }
}

// MODE 0: R = I^T (weighted sum), 1: injection, 2: max, 3: min.
template <int DIM, int MODE, typename T>
__global__ __launch_bounds__(256) void k_restrict(int Nc, const T* __restrict__ xf, T* __restrict__ xc) {
  constexpr int NC = DIM + 1;
  const int Nf = 2 * Nc;
  const int64_t nsf = Nf + 1, nsc = Nc + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= nsc;
  for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < nn; n += int64_t(gridDim.x) * blockDim.x) {
    int c[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r % nsc);
      r /= nsc;
    }
    if (MODE == 1) {
      int64_t m = 0, s = 1;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        m += int64_t(2 * c[i]) * s;
        s *= nsf;
      }
#pragma unroll
      for (int k = 0; k < NC; ++k) xc[NC * n + k] = xf[NC * m + k];
      continue;
    }
    int lo[DIM], hi[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      lo[i] = max(2 * c[i] - 1, 0);
      hi[i] = min(2 * c[i] + 1, Nf);
    }
    T acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = MODE == 0 ? T(0) : (MODE == 2 ? T(-INFINITY) : T(INFINITY));
    const int zlo = DIM == 3 ? lo[2] : 0, zhi = DIM == 3 ? hi[2] : 0;
    for (int fz = zlo; fz <= zhi; ++fz)
      for (int fy = lo[1]; fy <= hi[1]; ++fy)
        for (int fx = lo[0]; fx <= hi[0]; ++fx) {
          const int64_t m = fx + nsf * (fy + nsf * int64_t(fz));
          if (MODE == 0) {
            T wgt = T((fx == 2 * c[0] ? 1.0 : 0.5) * (fy == 2 * c[1] ? 1.0 : 0.5) *
                      (DIM == 3 ? (fz == 2 * c[DIM == 3 ? 2 : 0] ? 1.0 : 0.5) : 1.0));
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[k] += wgt * xf[NC * m + k];
          } else if (MODE == 2) {
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[k] = fmax(acc[k], xf[NC * m + k]);
          } else {
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[k] = fmin(acc[k], xf[NC * m + k]);
          }
        }
#pragma unroll
    for (int k = 0; k < NC; ++k) xc[NC * n + k] = acc[k];
  }
}

int gridn(int64_t work) {
  int64_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  if (b > 262140) b = 262140;
  return int(b);
}

template <int DIM, typename T>
hipError_t restrict_t(int Nc, int mode, const T* xf, T* xc, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < DIM; ++i) nn *= (Nc + 1);
  dim3 g(gridn(nn));
  switch (mode) {
    case 0: hipLaunchKernelGGL((k_restrict<DIM, 0, T>), g, dim3(256), 0, st, Nc, xf, xc); break;
    case 1: hipLaunchKernelGGL((k_restrict<DIM, 1, T>), g, dim3(256), 0, st, Nc, xf, xc); break;
    case 2: hipLaunchKernelGGL((k_restrict<DIM, 2, T>), g, dim3(256), 0, st, Nc, xf, xc); break;
    case 3: hipLaunchKernelGGL((k_restrict<DIM, 3, T>), g, dim3(256), 0, st, Nc, xf, xc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_prolong(int dim, int Nc, const void* xc, void* xf, int fp32, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (2 * Nc + 1);
  dim3 g(gridn(nn));
  if (dim == 3) {
    if (fp32)
      hipLaunchKernelGGL((k_prolong<3, float>), g, dim3(256), 0, st, Nc, (const float*)xc, (float*)xf);
    else
      hipLaunchKernelGGL((k_prolong<3, double>), g, dim3(256), 0, st, Nc, (const double*)xc, (double*)xf);
  } else {
    if (fp32)
      hipLaunchKernelGGL((k_prolong<2, float>), g, dim3(256), 0, st, Nc, (const float*)xc, (float*)xf);
    else
      hipLaunchKernelGGL((k_prolong<2, double>), g, dim3(256), 0, st, Nc, (const double*)xc, (double*)xf);
  }
  return hipGetLastError();
}

hipError_t launch_restrict(int dim, int Nc, int mode, const void* xf, void* xc, int fp32, hipStream_t st) {
  if (dim == 3)
    return fp32 ? restrict_t<3, float>(Nc, mode, (const float*)xf, (float*)xc, st)
                : restrict_t<3, double>(Nc, mode, (const double*)xf, (double*)xc, st);
  return fp32 ? restrict_t<2, float>(Nc, mode, (const float*)xf, (float*)xc, st)
              : restrict_t<2, double>(Nc, mode, (const double*)xf, (double*)xc, st);
}

}  // namespace rmtr

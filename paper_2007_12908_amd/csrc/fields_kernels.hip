// Nodal inclusion initialisation of the phase field (Sec. 5, first
// paragraph): c0 = 1 at nodes inside a fracture's volumetric description,
// else 0; and the nodal pressure field (uniform, or the largest pressure of
// the fractures within a band around the node).  Written without fused
// multiply-add and with correctly rounded division and square root so that
// any IEEE implementation of the same formulas gives the same bits.
#pragma clang fp contract(off)
#include "rmtr_kernels.h"

namespace rmtr {
namespace {

// 3D table row: cx cy cz nx ny nz radius pressure
__device__ inline double disc_dist2(double X, double Y, double Z, const double* t) {
  const double dx = X - t[0], dy = Y - t[1], dz = Z - t[2];
  const double dn = (dx * t[3] + dy * t[4]) + dz * t[5];
  const double qx = dx - dn * t[3], qy = dy - dn * t[4], qz = dz - dn * t[5];
  const double rho2 = (qx * qx + qy * qy) + qz * qz;
  const double r = t[6];
  if (rho2 > r * r) {
    const double e = __dsqrt_rn(rho2) - r;
    return dn * dn + e * e;
  }
  return dn * dn;
}

// 2D table row: cx cy tx ty half_length half_width pressure
__device__ inline bool rect_in(double X, double Y, const double* t) {
  const double dx = X - t[0], dy = Y - t[1];
  const double dt = dx * t[2] + dy * t[3];
  const double dn = dx * (-t[3]) + dy * t[2];
  return fabs(dt) <= t[4] && fabs(dn) <= t[5];
}

template <int DIM>
__global__ __launch_bounds__(256) void k_init(int N, const double* __restrict__ tab, int nf, double band, int p_mode,
                                              double p_value, double p_band, double* __restrict__ c0,
                                              double* __restrict__ p) {
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  const double dN = double(N);
  for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < nn; n += int64_t(gridDim.x) * blockDim.x) {
    int64_t r = n;
    double X[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      X[i] = double(r % ns) / dN;
      r /= ns;
    }
    double c = 0.0, pv = 0.0;
    for (int f = 0; f < nf; ++f) {
      if (DIM == 3) {
        const double* t = tab + 8 * f;
        const double d2 = disc_dist2(X[0], X[1], X[2], t);
        if (d2 <= band * band) c = 1.0;
        if (p_mode == 1 && d2 <= p_band * p_band) pv = fmax(pv, t[7]);
      } else {
        const double* t = tab + 7 * f;
        if (rect_in(X[0], X[1], t)) c = 1.0;
      }
    }
    c0[n] = c;
    if (p) p[n] = p_mode == 0 ? p_value : pv;
  }
}

}  // namespace

hipError_t launch_init_fields(int dim, int N, const double* table, int n_frac, double band, int p_mode,
                              double p_value, double p_band, double* c0, double* p, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  int64_t b = (nn + 255) / 256;
  if (b > 262140) b = 262140;
  if (dim == 3)
    hipLaunchKernelGGL(k_init<3>, dim3(int(b)), dim3(256), 0, st, N, table, n_frac, band, p_mode, p_value, p_band, c0,
                       p);
  else
    hipLaunchKernelGGL(k_init<2>, dim3(int(b)), dim3(256), 0, st, N, table, n_frac, band, p_mode, p_value, p_band, c0,
                       p);
  return hipGetLastError();
}

}  // namespace rmtr

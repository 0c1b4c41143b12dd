// External load vector of the Neumann terms of eq. (pressurized): on the
// boundary faces where the displacement is free (Gamma_N),
//   b[(d+1) n + i] = int_{Gamma_N} (tbar_i + p n_i) N_n ds,
// so that the functional is f(x) - b . x.  The traction tbar is constant on
// a face; p is the nodal (Q1) pressure; face cells are integrated with the
// (d-1)-dimensional 2-point Gauss rule (exact for the bilinear integrand).
#include "rmtr_kernels.h"

namespace rmtr {
namespace {

// Thread per node: every selected face through the node, every face cell of
// that face around it.
template <int DIM>
__global__ __launch_bounds__(256) void k_neumann(int N, double h, int face_mask, NeumannTraction tr,
                                                 const double* __restrict__ p, double* __restrict__ b) {
  constexpr int NC = DIM + 1, NT = DIM - 1, NQ = 1 << NT;
  const int64_t ns = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= ns;
  const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  const double wq = (DIM == 3 ? h * h : h) / double(NQ);
  for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < nn; n += int64_t(gridDim.x) * blockDim.x) {
    int c[DIM];
    int64_t r = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r % ns);
      r /= ns;
    }
    double acc[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) acc[i] = 0.0;
#pragma unroll
    for (int f = 0; f < 2 * DIM; ++f) {
      const int axis = f >> 1, side = f & 1;
      if (!((face_mask >> f) & 1) || c[axis] != side * N) continue;
      int tan[NT > 0 ? NT : 1];
      int t = 0;
#pragma unroll
      for (int i = 0; i < DIM; ++i)
        if (i != axis) tan[t++] = i;
      const double nrm = side ? 1.0 : -1.0;
      // face cells touching the node: lower corner c[tan] - o, o in {0, 1}^NT
#pragma unroll
      for (int cell = 0; cell < NQ; ++cell) {
        int lo[NT > 0 ? NT : 1];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          lo[k] = c[tan[k]] - ((cell >> k) & 1);
          ok &= lo[k] >= 0 && lo[k] < N;
        }
        if (!ok) continue;
        // the node is local corner `me` of the face cell
        int me = 0;
#pragma unroll
        for (int k = 0; k < NT; ++k) me |= (c[tan[k]] - lo[k]) << k;
        double pc[NQ];
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          int cc[DIM];
#pragma unroll
          for (int i = 0; i < DIM; ++i) cc[i] = c[i];
#pragma unroll
          for (int k = 0; k < NT; ++k) cc[tan[k]] = lo[k] + ((a >> k) & 1);
          int64_t id = 0, s = 1;
#pragma unroll
          for (int i = 0; i < DIM; ++i) {
            id += int64_t(cc[i]) * s;
            s *= ns;
          }
          pc[a] = p[id];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          double Na[NQ];
#pragma unroll
          for (int a = 0; a < NQ; ++a) {
            double v = 1.0;
#pragma unroll
            for (int k = 0; k < NT; ++k) {
              const double xi = gp[(q >> k) & 1];
              v *= ((a >> k) & 1) ? xi : 1.0 - xi;
            }
            Na[a] = v;
          }
          double pq = 0.0;
#pragma unroll
          for (int a = 0; a < NQ; ++a) pq += Na[a] * pc[a];
          const double wn = wq * Na[me];
#pragma unroll
          for (int i = 0; i < DIM; ++i) acc[i] += wn * (tr.t[f][i] + (i == axis ? pq * nrm : 0.0));
        }
      }
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) b[NC * n + i] = acc[i];
    b[NC * n + DIM] = 0.0;
  }
}

}  // namespace

hipError_t launch_neumann_load(int dim, int N, int face_mask, const NeumannTraction& tr, const double* p, double* b,
                               hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  int64_t g = (nn + 255) / 256;
  if (g > 262140) g = 262140;
  const double h = 1.0 / double(N);
  if (dim == 3)
    hipLaunchKernelGGL(k_neumann<3>, dim3(int(g)), dim3(256), 0, st, N, h, face_mask, tr, p, b);
  else
    hipLaunchKernelGGL(k_neumann<2>, dim3(int(g)), dim3(256), 0, st, N, h, face_mask, tr, p, b);
  return hipGetLastError();
}

}  // namespace rmtr

// Coarse-level Hessians stored as element matrices, and the operators that
// use them.
//
// Galerkin products (eq. (delta_terms), R grad^2 h I) on nested Q1 grids
// are assembled element by element: the interpolation restricted to a coarse
// element E maps E's nodes onto the nodes of each of its 2^d children, with
// the constant weights P_c[a][b] = prod_i phi_{b_i}((c_i + a_i) / 2).  Hence
//   R H I = sum_E Q_E^T ( sum_c P_c^T K_{e_c} P_c ) Q_E,
// so every level keeps one dense (d+1) 2^d square matrix per element.  The
// finest level's K_e are never stored: the coarse matrices of level L-1 are
// built directly from the lagged matrix-free Hessian.  Dirichlet rows and
// columns are zero on every level.
#include "rmtr_kernels.h"

namespace rmtr {

namespace {

template <int DIM>
__device__ inline double child_weight(int c, int a, int b) {
  double v = 1.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    const double t = 0.5 * double(((c >> i) & 1) + ((a >> i) & 1));
    v *= ((b >> i) & 1) ? t : 1.0 - t;
  }
  return v;
}

template <int DIM>
__device__ inline uint8_t mask_at(const uint8_t* dir, const int (&ijk)[DIM], int N) {
  int64_t n = 0, s = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    n += int64_t(ijk[i]) * s;
    s *= (N + 1);
  }
  return dir ? dir[n] : default_mask<DIM>(ijk, N);
}

// ---------------------------------------------------- from matrix-free H
// Threads of a 64-wide block: ND = (DIM+1) 2^DIM threads per coarse element,
// thread j owns column j = (DIM+1) b' + beta of K_E.
// same_level != 0: no coarsening (one child, the element itself, identity
// weights): the element matrices of the level's own Hessian.
template <int DIM>
__global__ __launch_bounds__(64) void k_galerkin_matfree(int Nf, double h, MatP<double> m, int same_level,
                                                         const uint8_t* __restrict__ dirf,
                                                         const uint8_t* __restrict__ dirc,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ p, double* __restrict__ Kc) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, ND = NL * NC, EPB = 64 / ND;
  __shared__ double sX[EPB][NL][NC];
  __shared__ double sP[EPB][NL];
  __shared__ uint8_t sM[EPB][NL];
  __shared__ HessCoef<DIM, double> sH[EPB][NL];
  const int Nc = same_level ? Nf : Nf / 2;
  const int nchild = same_level ? 1 : NL;
  int64_t nce = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nce *= Nc;
  const int slot = threadIdx.x / ND;
  const int col = threadIdx.x % ND;
  const int64_t E = int64_t(blockIdx.x) * EPB + slot;
  const bool active = slot < EPB && E < nce;
  int Ec[DIM] = {};
  if (active) {
    int64_t r = E;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      Ec[i] = int(r % Nc);
      r /= Nc;
    }
  }
  const double invh = 1.0 / h;
  double w = 1.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) w *= 0.5 * h;
  const int bcol = col / NC, beta = col % NC;
  double acc[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) acc[i] = 0.0;
  for (int c = 0; c < nchild; ++c) {
    // child element's lower corner (fine indices)
    int e[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) e[i] = same_level ? Ec[i] : 2 * Ec[i] + ((c >> i) & 1);
    if (active && col < NL) {
      int nd[DIM];
#pragma unroll
      for (int i = 0; i < DIM; ++i) nd[i] = e[i] + ((col >> i) & 1);
      int64_t n = 0, s = 1;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        n += int64_t(nd[i]) * s;
        s *= (Nf + 1);
      }
#pragma unroll
      for (int k = 0; k < NC; ++k) sX[slot][col][k] = x[NC * n + k];
      sP[slot][col] = p[n];
      sM[slot][col] = dirf ? dirf[n] : default_mask<DIM>(nd, Nf);
    }
    __syncthreads();
    if (active && col < NL) {
      const int q = col;
      double X[NL][NC], P[NL];
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        P[a] = sP[slot][a];
#pragma unroll
        for (int k = 0; k < NC; ++k) X[a][k] = sX[slot][a][k];
      }
      Zq<DIM, double> z;
      double pq, dpq[DIM];
      interp_scalar_q<DIM, double>(q, P, invh, pq, dpq);
      interp_q<DIM, double>(q, X, invh, z);
      hess_coef<DIM, double>(m, z, pq, dpq, sH[slot][q]);
    }
    __syncthreads();
    if (active) {
      // fine element vector: P_c[:, bcol] in component beta (Dirichlet zeroed)
      double ve[NL];
#pragma unroll
      for (int a = 0; a < NL; ++a)
        ve[a] = (sM[slot][a] & (1u << beta)) ? 0.0
                : same_level                 ? (a == bcol ? 1.0 : 0.0)
                                             : child_weight<DIM>(c, a, bcol);
      double r[NL][NC];
#pragma unroll
      for (int a = 0; a < NL; ++a)
#pragma unroll
        for (int k = 0; k < NC; ++k) r[a][k] = 0.0;
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        Zq<DIM, double> z, o;
        zero<DIM, double>(z);
#pragma unroll
        for (int a = 0; a < NL; ++a) {
          const double n = refN<DIM>(q, a) * ve[a];
          if (beta < DIM) {
            z.u[beta] += n;
#pragma unroll
            for (int j = 0; j < DIM; ++j) z.G[beta][j] += refdN<DIM>(q, a, j) * invh * ve[a];
          } else {
            z.c += n;
#pragma unroll
            for (int j = 0; j < DIM; ++j) z.dc[j] += refdN<DIM>(q, a, j) * invh * ve[a];
          }
        }
        const HessCoef<DIM, double> hc = sH[slot][q];
        hess_apply<DIM, double>(m, hc, z, o);
#pragma unroll
        for (int a = 0; a < NL; ++a) project_q_node<DIM, double>(q, a, invh, w, o, r[a]);
      }
      // mask fine Dirichlet rows, then acc[(b, alpha)] += sum_a P_c[a][b] r[a][alpha]
#pragma unroll
      for (int a = 0; a < NL; ++a)
#pragma unroll
        for (int k = 0; k < NC; ++k)
          if (sM[slot][a] & (1u << k)) r[a][k] = 0.0;
#pragma unroll
      for (int b = 0; b < NL; ++b)
#pragma unroll
        for (int a = 0; a < NL; ++a) {
          const double wc = same_level ? (a == b ? 1.0 : 0.0) : child_weight<DIM>(c, a, b);
#pragma unroll
          for (int k = 0; k < NC; ++k) acc[NC * b + k] += wc * r[a][k];
        }
    }
    __syncthreads();
  }
  if (!active) return;
  // coarse Dirichlet rows / column
  uint8_t mc[NL];
#pragma unroll
  for (int b = 0; b < NL; ++b) {
    int nd[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) nd[i] = Ec[i] + ((b >> i) & 1);
    mc[b] = mask_at<DIM>(dirc, nd, Nc);
  }
  const bool colmask = (mc[bcol] >> beta) & 1u;
  double* K = Kc + E * (ND * ND);
#pragma unroll
  for (int row = 0; row < ND; ++row) {
    const bool rm = (mc[row / NC] >> (row % NC)) & 1u;
    K[row * ND + col] = (rm || colmask) ? 0.0 : acc[row];
  }
}

// ------------------------------- from matrix-free H, fine-quadrature form
// Because the coarse Q1 space is nested in the fine one, R H I restricted to
// a coarse element E is E's element matrix integrated with the 2^d x 2^d
// fine quadrature points of its children, using the second-variation
// coefficients of the fine level at those points:
//   K_E[(b,al),(b',be)] = sum_k w_f z_k(b,al)^T d2W_k z_k(b',be),
// where z_k(b, al) is coarse basis function b in component al evaluated
// (value and gradient) at fine point k.  Those values are constants
// (pn[k][b], pd[k][b][j], unit fine cell) passed in `tab`.  Valid when no
// fine Dirichlet dof feeds a free coarse dof, which holds for the default
// Dirichlet set (a fine boundary node interpolates only from coarse
// boundary nodes).
template <int DIM, int NE>
__global__ __launch_bounds__(256) void k_galerkin_fineq(int Nf, double h, MatP<double> m,
                                                        const double* __restrict__ tab,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ p, double* __restrict__ Kc) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, ND = NL * NC, NK = NL * NL;
  constexpr int NCOEF = 3 + DIM * DIM + DIM;  // vol, shear, Ccc, S, Pc
  __shared__ double sT[NK][NL][DIM + 1];      // pd[k][b][0..DIM-1], pn[k][b]
  __shared__ double sC[NE][NK][NCOEF];
  const int Nc = Nf / 2;
  int64_t nce = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nce *= Nc;
  const int tid = threadIdx.x;
  for (int i = tid; i < NK * NL * (DIM + 1); i += 256) (&sT[0][0][0])[i] = tab[i];
  const double invh = 1.0 / h;
  // phase 1: coefficients at every fine point of NE coarse elements
  for (int t = tid; t < NE * NK; t += 256) {
    const int el = t / NK, k = t % NK, c = k / NL, q = k % NL;
    const int64_t E = int64_t(blockIdx.x) * NE + el;
    if (E >= nce) continue;
    int e[DIM];
    int64_t r = E;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      e[i] = 2 * int(r % Nc) + ((c >> i) & 1);
      r /= Nc;
    }
    double X[NL][NC], P[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      int64_t n = 0, s = 1;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        n += int64_t(e[i] + ((a >> i) & 1)) * s;
        s *= (Nf + 1);
      }
#pragma unroll
      for (int kk = 0; kk < NC; ++kk) X[a][kk] = x[NC * n + kk];
      P[a] = p[n];
    }
    Zq<DIM, double> z;
    double pq, dpq[DIM];
    interp_scalar_q<DIM, double>(q, P, invh, pq, dpq);
    interp_q<DIM, double>(q, X, invh, z);
    HessCoef<DIM, double> hc;
    hess_coef<DIM, double>(m, z, pq, dpq, hc);
    double* o = sC[el][k];
    o[0] = hc.vol;
    o[1] = hc.shear;
    o[2] = hc.Ccc;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      o[3 + DIM * DIM + i] = hc.Pc[i];
#pragma unroll
      for (int j = 0; j < DIM; ++j) o[3 + DIM * i + j] = hc.S[i][j];
    }
  }
  __syncthreads();
  // phase 2: every entry of the NE coarse element matrices
  double w = 1.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) w *= 0.5 * h;
  const double s2 = w * invh * invh, s1 = w * invh, s0 = w;
  const double gcl = m.Gc * m.ls;
  for (int ent = tid; ent < ND * ND; ent += 256) {
    const int row = ent / ND, col = ent % ND;
    const int b = row / NC, al = row % NC, bp = col / NC, be = col % NC;
    double acc[NE];
#pragma unroll
    for (int el = 0; el < NE; ++el) acc[el] = 0.0;
    for (int k = 0; k < NK; ++k) {
      const double* tb = sT[k][b];
      const double* tp = sT[k][bp];
      if (al < DIM && be < DIM) {
        double dd = 0.0;
#pragma unroll
        for (int j = 0; j < DIM; ++j) dd += tb[j] * tp[j];
        const double tv = s2 * tb[al] * tp[be];
        const double ts = s2 * ((al == be ? dd : 0.0) + tb[be] * tp[al]);
#pragma unroll
        for (int el = 0; el < NE; ++el) acc[el] += sC[el][k][0] * tv + sC[el][k][1] * ts;
      } else if (al < DIM) {
        const double nn = s0 * tb[DIM] * tp[DIM];
#pragma unroll
        for (int el = 0; el < NE; ++el) {
          double v = sC[el][k][3 + DIM * DIM + al] * nn;
#pragma unroll
          for (int j = 0; j < DIM; ++j) v += sC[el][k][3 + DIM * al + j] * s1 * tb[j] * tp[DIM];
          acc[el] += v;
        }
      } else if (be < DIM) {
        const double nn = s0 * tb[DIM] * tp[DIM];
#pragma unroll
        for (int el = 0; el < NE; ++el) {
          double v = sC[el][k][3 + DIM * DIM + be] * nn;
#pragma unroll
          for (int j = 0; j < DIM; ++j) v += sC[el][k][3 + DIM * be + j] * s1 * tp[j] * tb[DIM];
          acc[el] += v;
        }
      } else {
        double dd = 0.0;
#pragma unroll
        for (int j = 0; j < DIM; ++j) dd += tb[j] * tp[j];
        const double nn = s0 * tb[DIM] * tp[DIM];
#pragma unroll
        for (int el = 0; el < NE; ++el) acc[el] += sC[el][k][2] * nn + gcl * s2 * dd;
      }
    }
#pragma unroll
    for (int el = 0; el < NE; ++el) {
      const int64_t E = int64_t(blockIdx.x) * NE + el;
      if (E >= nce) continue;
      int Ec[DIM];
      int64_t r = E;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        Ec[i] = int(r % Nc);
        r /= Nc;
      }
      int nb[DIM], nbp[DIM];
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        nb[i] = Ec[i] + ((b >> i) & 1);
        nbp[i] = Ec[i] + ((bp >> i) & 1);
      }
      const bool mk = ((default_mask<DIM>(nb, Nc) >> al) & 1u) || ((default_mask<DIM>(nbp, Nc) >> be) & 1u);
      Kc[E * (ND * ND) + ent] = mk ? 0.0 : acc[el];
    }
  }
}

// ------------------------------------------------- from element matrices
template <int DIM>
__global__ __launch_bounds__(64) void k_galerkin_em(int Nc, const double* __restrict__ Kf,
                                                    const uint8_t* __restrict__ dirc, double* __restrict__ Kc) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, ND = NL * NC, EPB = 64 / ND;
  const int Nf = 2 * Nc;
  int64_t nce = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nce *= Nc;
  const int slot = threadIdx.x / ND;
  const int col = threadIdx.x % ND;
  const int64_t E = int64_t(blockIdx.x) * EPB + slot;
  if (slot >= EPB || E >= nce) return;
  int Ec[DIM];
  {
    int64_t r = E;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      Ec[i] = int(r % Nc);
      r /= Nc;
    }
  }
  const int bcol = col / NC, beta = col % NC;
  double acc[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) acc[i] = 0.0;
  for (int c = 0; c < NL; ++c) {
    int64_t ef = 0, s = 1;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      ef += int64_t(2 * Ec[i] + ((c >> i) & 1)) * s;
      s *= Nf;
    }
    const double* K = Kf + ef * (ND * ND);
    double ve[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) ve[a] = child_weight<DIM>(c, a, bcol);
    double r[ND];
#pragma unroll
    for (int row = 0; row < ND; ++row) {
      double t = 0.0;
#pragma unroll
      for (int a = 0; a < NL; ++a) t += K[row * ND + NC * a + beta] * ve[a];
      r[row] = t;
    }
#pragma unroll
    for (int b = 0; b < NL; ++b)
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        const double wc = child_weight<DIM>(c, a, b);
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[NC * b + k] += wc * r[NC * a + k];
      }
  }
  uint8_t mc[NL];
#pragma unroll
  for (int b = 0; b < NL; ++b) {
    int nd[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) nd[i] = Ec[i] + ((b >> i) & 1);
    mc[b] = mask_at<DIM>(dirc, nd, Nc);
  }
  const bool colmask = (mc[bcol] >> beta) & 1u;
  double* K = Kc + E * (ND * ND);
#pragma unroll
  for (int row = 0; row < ND; ++row) {
    const bool rm = (mc[row / NC] >> (row % NC)) & 1u;
    K[row * ND + col] = (rm || colmask) ? 0.0 : acc[row];
  }
}

// --------------------------------------------------- element-matrix ops
// y_n = sum over the elements E around node n of rows(n) of K_E v_E.
template <int DIM, typename T>
__device__ inline void em_rows(int N, const T* __restrict__ K, const T* __restrict__ v, const int (&c)[DIM],
                               T (&r)[DIM + 1]) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, ND = NL * NC;
  const int64_t nside = N + 1;
#pragma unroll
  for (int k = 0; k < NC; ++k) r[k] = T(0);
  for (int a = 0; a < NL; ++a) {
    int e[DIM];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      e[i] = c[i] - ((a >> i) & 1);
      ok &= (e[i] >= 0) & (e[i] < N);
    }
    if (!ok) continue;
    int64_t eid = 0, s = 1;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      eid += int64_t(e[i]) * s;
      s *= N;
    }
    const T* Ke = K + eid * (ND * ND);
    T ve[ND];
#pragma unroll
    for (int b = 0; b < NL; ++b) {
      int64_t n = 0, st = 1;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        n += int64_t(e[i] + ((b >> i) & 1)) * st;
        st *= nside;
      }
#pragma unroll
      for (int k = 0; k < NC; ++k) ve[NC * b + k] = v[NC * n + k];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T* row = Ke + (NC * a + k) * ND;
      T t = T(0);
#pragma unroll
      for (int j = 0; j < ND; ++j) t += row[j] * ve[j];
      r[k] += t;
    }
  }
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_em_hessvec(int N, const T* __restrict__ K, const T* __restrict__ v,
                                                    T* __restrict__ y) {
  constexpr int NC = DIM + 1;
  const int64_t nside = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= nside;
  for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < nn; n += int64_t(gridDim.x) * blockDim.x) {
    int c[DIM];
    int64_t r_ = n;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = int(r_ % nside);
      r_ /= nside;
    }
    T r[NC];
    em_rows<DIM, T>(N, K, v, c, r);
#pragma unroll
    for (int k = 0; k < NC; ++k) y[NC * n + k] = r[k];
  }
}

int gridn(int64_t work, int block) {
  int64_t b = (work + block - 1) / block;
  if (b < 1) b = 1;
  if (b > 262140) b = 262140;
  return int(b);
}

}  // namespace

void galerkin_fineq_table(int dim, std::vector<double>& out) {
  const int NL = 1 << dim;
  out.assign(size_t(NL) * NL * NL * (dim + 1), 0.0);
  for (int c = 0; c < NL; ++c)
    for (int q = 0; q < NL; ++q)
      for (int b = 0; b < NL; ++b) {
        double* o = &out[((size_t(c) * NL + q) * NL + b) * (dim + 1)];
        for (int a = 0; a < NL; ++a) {
          double wgt = 1.0;
          for (int i = 0; i < dim; ++i) {
            const double t = 0.5 * double(((c >> i) & 1) + ((a >> i) & 1));
            wgt *= ((b >> i) & 1) ? t : 1.0 - t;
          }
          if (wgt == 0.0) continue;
          for (int j = 0; j < dim; ++j)
            o[j] += wgt * (dim == 3 ? refdN<3>(q, a, j) : refdN<2>(q, a, j));
          o[dim] += wgt * (dim == 3 ? refN<3>(q, a) : refN<2>(q, a));
        }
      }
}

hipError_t launch_galerkin_from_matfree(const ElemArgs& fine, const double* xl, const double* p, double* Kc,
                                        int same_level, const uint8_t* dirc, const double* fineq_tab,
                                        hipStream_t st) {
  const int Nc = same_level ? fine.N : fine.N / 2;
  int64_t nce = 1;
  for (int i = 0; i < fine.dim; ++i) nce *= Nc;
  if (!same_level && fine.dir == nullptr && dirc == nullptr && fineq_tab != nullptr) {
    if (fine.dim == 3) {
      constexpr int NE = 4;
      hipLaunchKernelGGL((k_galerkin_fineq<3, NE>), dim3(int((nce + NE - 1) / NE)), dim3(256), 0, st, fine.N,
                         fine.h, fine.m, fineq_tab, xl, p, Kc);
    } else {
      constexpr int NE = 16;
      hipLaunchKernelGGL((k_galerkin_fineq<2, NE>), dim3(int((nce + NE - 1) / NE)), dim3(256), 0, st, fine.N,
                         fine.h, fine.m, fineq_tab, xl, p, Kc);
    }
    return hipGetLastError();
  }
  if (fine.dim == 3) {
    const int epb = 64 / 32;
    hipLaunchKernelGGL(k_galerkin_matfree<3>, dim3(int((nce + epb - 1) / epb)), dim3(64), 0, st, fine.N, fine.h,
                       fine.m, same_level, fine.dir, dirc, xl, p, Kc);
  } else {
    const int epb = 64 / 12;
    hipLaunchKernelGGL(k_galerkin_matfree<2>, dim3(int((nce + epb - 1) / epb)), dim3(64), 0, st, fine.N, fine.h,
                       fine.m, same_level, fine.dir, dirc, xl, p, Kc);
  }
  return hipGetLastError();
}

hipError_t launch_galerkin_from_em(int dim, int Nc, const double* Kf, double* Kc, const uint8_t* dirc,
                                   hipStream_t st) {
  int64_t nce = 1;
  for (int i = 0; i < dim; ++i) nce *= Nc;
  if (dim == 3)
    hipLaunchKernelGGL(k_galerkin_em<3>, dim3(int((nce + 1) / 2)), dim3(64), 0, st, Nc, Kf, dirc, Kc);
  else
    hipLaunchKernelGGL(k_galerkin_em<2>, dim3(int((nce + 4) / 5)), dim3(64), 0, st, Nc, Kf, dirc, Kc);
  return hipGetLastError();
}

hipError_t launch_em_hessvec(int dim, int N, const void* K, const void* v, void* hv, const uint8_t* dir, int fp32,
                             hipStream_t st) {
  (void)dir;  // rows and columns of Dirichlet dofs are already zero in K
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  dim3 g(gridn(nn, 256));
  if (dim == 3) {
    if (fp32)
      hipLaunchKernelGGL((k_em_hessvec<3, float>), g, dim3(256), 0, st, N, (const float*)K, (const float*)v,
                         (float*)hv);
    else
      hipLaunchKernelGGL((k_em_hessvec<3, double>), g, dim3(256), 0, st, N, (const double*)K, (const double*)v,
                         (double*)hv);
  } else {
    if (fp32)
      hipLaunchKernelGGL((k_em_hessvec<2, float>), g, dim3(256), 0, st, N, (const float*)K, (const float*)v,
                         (float*)hv);
    else
      hipLaunchKernelGGL((k_em_hessvec<2, double>), g, dim3(256), 0, st, N, (const double*)K, (const double*)v,
                         (double*)hv);
  }
  return hipGetLastError();
}

}  // namespace rmtr

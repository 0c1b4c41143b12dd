// Device-side building blocks of the phase-field fracture functional on a
// uniform Q1 grid: reference-element data, the pointwise density and its first
// and second variations, and sum-factorised interpolation for hexahedra.
//
// The discrete functional is the one of the paper's Sec. 2, eq. (pressurized)
// with the AT2 choice w(c) = c^2, c_w = 2, integrated with 2^d Gauss points:
//   W = g(c) psi+ + psi- + Gc/2 (c^2/l + l |grad c|^2) + gp(c) div(p u)
//   g = (1-k)(1-c)^2 + k,  gp = (1-c)^2,  div(p u) = p tr(eps) + grad p . u
//   psi+ = K/2 <t>+^2 + mu e:e,  psi- = K/2 <t>-^2  (t = tr eps, e its deviator
//   in 3D, K = lambda + 2 mu / 3; 2D is plane strain), the unsplit
//   psi+ = lambda/2 t^2 + mu eps:eps, psi- = 0, or the spectral split on the
//   principal strains eps_a: psi+- = lambda/2 <t>+-^2 + mu sum_a <eps_a>+-^2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Element-level building blocks are callable from host code as well, so the
// library can count their arithmetic by instantiating them with a counting
// scalar type (rmtr_element_flops).
#define RMTR_FN __host__ __device__ inline

namespace rmtr {

// Two-point Gauss rule on [0, 1]: xi = (1 -+ 1/sqrt(3)) / 2.
#define RMTR_GA 0.78867513459481288225457439025098  // 1 - xi_0 = xi_1
#define RMTR_GB 0.21132486540518711774542560974902  // xi_0 = 1 - xi_1

// MatP::split
constexpr int kSplitNone = 0, kSplitVolDev = 1, kSplitSpectral = 2;
// Which split code a function carries (template argument SK): kAnySplit
// decides from MatP::split at run time, kNoSpectral carries the unsplit and
// volumetric-deviatoric forms only, kSplitSpectral the spectral form only.
// The 3D element kernels are instantiated per family, so the spectral
// branch costs the other forms no registers.
constexpr int kAnySplit = -1, kNoSpectral = -2;

template <int SK>
RMTR_FN bool spectral_split(int split) {
  return SK == kSplitSpectral || (SK == kAnySplit && split == kSplitSpectral);
}

template <typename T>
struct MatP {
  T lam, mu, K, Gc, ls, k;
  int split;
  // derived once on the host (set_derived), so no kernel divides
  T third, mu23, Gc_ls, Gc_l;  // 1/3, 2 mu / 3, Gc / l, Gc l
};

template <typename T>
RMTR_FN void set_derived(MatP<T>& m) {
  m.third = T(1) / T(3);
  m.mu23 = T(2) * m.mu / T(3);
  m.Gc_ls = m.Gc / m.ls;
  m.Gc_l = m.Gc * m.ls;
}

// One level of the hierarchy: N cells per side, (N+1)^DIM nodes.
template <typename T>
struct LevelP {
  int N;
  int64_t nside;   // N + 1
  T h, invh, w;    // w = h^DIM / 2^DIM (quadrature weight)
};

// phi_b at Gauss point q along one direction: phi_0 = 1 - xi, phi_1 = xi.
__host__ __device__ constexpr double shape1(int b, int q) {
  return b ? (q ? RMTR_GA : RMTR_GB) : (q ? RMTR_GB : RMTR_GA);
}

template <int DIM>
__host__ __device__ constexpr double refN(int q, int a) {
  double v = 1.0;
  for (int i = 0; i < DIM; ++i) v *= shape1((a >> i) & 1, (q >> i) & 1);
  return v;
}

// derivative along j on the unit cell (multiply by 1/h)
template <int DIM>
__host__ __device__ constexpr double refdN(int q, int a, int j) {
  double v = ((a >> j) & 1) ? 1.0 : -1.0;
  for (int i = 0; i < DIM; ++i)
    if (i != j) v *= shape1((a >> i) & 1, (q >> i) & 1);
  return v;
}

// ------------------------------------------------------------------------
// Quantities at one quadrature point: u, G = grad u (G[i][j] = du_i/dx_j),
// c, grad c.
template <int DIM, typename T>
struct Zq {
  T u[DIM];
  T G[DIM][DIM];
  T c;
  T dc[DIM];
};

template <int DIM, typename T>
RMTR_FN void zero(Zq<DIM, T>& z) {
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    z.u[i] = T(0);
    z.dc[i] = T(0);
#pragma unroll
    for (int j = 0; j < DIM; ++j) z.G[i][j] = T(0);
  }
  z.c = T(0);
}

// ------------------------------------------------------------------------
// Principal strains.  Symmetric eigendecomposition of a DIM x DIM matrix by
// the cyclic Jacobi method (Golub and Van Loan, Matrix Computations,
// Sec. 8.5): sweeps over the pairs (p, q) = (0,1), (0,2), (1,2), each
// zeroing A[p][q] by a plane rotation J from the symmetric 2 x 2 Schur step
//   tau = (A_qq - A_pp) / (2 A_pq),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2),  s = t c,   A <- J^T A J,  Q <- Q J.
// One rotation diagonalises a 2 x 2 matrix exactly; the 3 x 3 iteration
// converges quadratically and a fixed number of sweeps reaches rounding
// level.  With eigenvectors (VEC) it stops earlier once the off-diagonal
// part is below rounding against the diagonal (usually after two or three
// sweeps): there each rotation also turns Q.  On return ev holds the
// eigenvalues and, when VEC, the columns of Q the eigenvectors.
template <int DIM, typename T, bool VEC>
RMTR_FN void sym_eig(T (&A)[DIM][DIM], T (&ev)[DIM], T (&Q)[DIM][DIM]) {
  if (VEC) {
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) Q[i][j] = T(i == j ? 1 : 0);
  }
  constexpr int kSweeps = DIM == 2 ? 1 : (sizeof(T) >= 8 ? 5 : 4);
  constexpr int kPairs = DIM == 2 ? 1 : 3;
  const T eps = sizeof(T) >= 8 ? T(1.1102230246251565e-16) : T(5.9604645e-8);  // unit roundoff
#pragma unroll
  for (int sw = 0; sw < kSweeps; ++sw) {
    if (DIM == 3 && VEC && sw > 0) {
      const T off = (A[0][1] < T(0) ? -A[0][1] : A[0][1]) + (A[0][2] < T(0) ? -A[0][2] : A[0][2]) +
                    (A[1][2] < T(0) ? -A[1][2] : A[1][2]);
      const T dg = (A[0][0] < T(0) ? -A[0][0] : A[0][0]) + (A[1][1] < T(0) ? -A[1][1] : A[1][1]) +
                   (A[2][2] < T(0) ? -A[2][2] : A[2][2]);
      if (!(off > eps * dg)) break;
    }
#pragma unroll
    for (int pr = 0; pr < kPairs; ++pr) {
      const int p = pr == 2 ? 1 : 0, q = pr == 0 ? 1 : 2;
      const T apq = A[p][q];
      if (apq != T(0)) {
        const T tau = (A[q][q] - A[p][p]) / (T(2) * apq);
        const T at = tau < T(0) ? -tau : tau;
        // sqrt(1 + tau^2) without overflow for large |tau|
        const T ia = T(1) / at;
        const T r = at > T(1) ? at * sqrt(T(1) + ia * ia) : sqrt(T(1) + at * at);
        T t = T(1) / (at + r);
        if (tau < T(0)) t = -t;
        const T c = T(1) / sqrt(T(1) + t * t), sn = t * c;
        A[p][p] -= t * apq;
        A[q][q] += t * apq;
        A[p][q] = A[q][p] = T(0);
        if (DIM == 3) {
          const int o = 3 - p - q;
          const T aop = A[o][p], aoq = A[o][q];
          A[o][p] = A[p][o] = c * aop - sn * aoq;
          A[o][q] = A[q][o] = sn * aop + c * aoq;
        }
        if (VEC) {
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            const T qp = Q[k][p], qq = Q[k][q];
            Q[k][p] = c * qp - sn * qq;
            Q[k][q] = sn * qp + c * qq;
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < DIM; ++i) ev[i] = A[i][i];
}

// f theta_ab: the derivative of eps+ = sum_a <eps_a>+ n_a n_a^T along a
// symmetric direction E is sum_ab theta_ab (n_a^T E n_b) n_a n_b^T with
// theta_aa = H(eps_a) and, for eps_a != eps_b, the divided difference
// (<eps_a>+ - <eps_b>+) / (eps_a - eps_b) (H(eps_a) when they are equal);
// H(0) = 0 (the compressive side, as for the volumetric indicator).
template <int DIM, typename T>
RMTR_FN void spectral_theta(const T (&ev)[DIM], T f, T (&th)[DIM][DIM]) {
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      const T pa = ev[a] > T(0) ? ev[a] : T(0), pb = ev[b] > T(0) ? ev[b] : T(0);
      const T df = ev[a] - ev[b];
      th[a][b] = (a == b || df == T(0)) ? (ev[a] > T(0) ? f : T(0)) : f * (pa - pb) / df;
    }
}

// out += Q (th o (Q^T E Q)) Q^T with E = sym(G) (o: entrywise product).
template <int DIM, typename T>
RMTR_FN void spectral_apply(const T (&Q)[DIM][DIM], const T (&th)[DIM][DIM], const T (&G)[DIM][DIM],
                            T (&out)[DIM][DIM]) {
  T E[DIM][DIM], B[DIM][DIM], C[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) E[i][j] = T(0.5) * (G[i][j] + G[j][i]);
  // B = E Q, C = Q^T B (scaled by th)
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      T v = T(0);
#pragma unroll
      for (int j = 0; j < DIM; ++j) v += E[i][j] * Q[j][b];
      B[i][b] = v;
    }
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      T v = T(0);
#pragma unroll
      for (int i = 0; i < DIM; ++i) v += Q[i][a] * B[i][b];
      C[a][b] = th[a][b] * v;
    }
  // out += Q C Q^T
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      T v = T(0);
#pragma unroll
      for (int a = 0; a < DIM; ++a) v += Q[i][a] * C[a][b];
      B[i][b] = v;
    }
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      T v = T(0);
#pragma unroll
      for (int b = 0; b < DIM; ++b) v += B[i][b] * Q[j][b];
      out[i][j] += v;
    }
}

// Spectral parts from the strain e (symmetric): psi+, psi-, sigma+ and
// sigma- (both full tensors); with VEC also the principal strains and axes.
template <int DIM, typename T, bool VEC>
RMTR_FN void spectral_parts(const MatP<T>& m, const T (&e)[DIM][DIM], T t, T& psip, T& psim, T (&sigp)[DIM][DIM],
                            T (&sigm)[DIM][DIM], T (&ev)[DIM], T (&Q)[DIM][DIM]) {
  T A[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) A[i][j] = e[i][j];
  sym_eig<DIM, T, true>(A, ev, Q);
  const T tp = t > T(0) ? t : T(0);
  const T tm = t > T(0) ? T(0) : t;
  T sp = T(0), sm = T(0), evp[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    evp[a] = ev[a] > T(0) ? ev[a] : T(0);
    const T en = ev[a] - evp[a];
    sp += evp[a] * evp[a];
    sm += en * en;
  }
  psip = T(0.5) * m.lam * tp * tp + m.mu * sp;
  psim = T(0.5) * m.lam * tm * tm + m.mu * sm;
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      T ep = T(0);
#pragma unroll
      for (int a = 0; a < DIM; ++a) ep += Q[i][a] * evp[a] * Q[j][a];
      sigp[i][j] = T(2) * m.mu * ep + (i == j ? m.lam * tp : T(0));
      sigm[i][j] = T(2) * m.mu * (e[i][j] - ep) + (i == j ? m.lam * tm : T(0));
    }
}

// Spectral psi+ and psi- only (eigenvalues without axes).
template <int DIM, typename T>
RMTR_FN void spectral_energy(const MatP<T>& m, const T (&e)[DIM][DIM], T t, T& psip, T& psim) {
  T A[DIM][DIM], ev[DIM], Q[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) A[i][j] = e[i][j];
  sym_eig<DIM, T, false>(A, ev, Q);
  const T tp = t > T(0) ? t : T(0);
  const T tm = t > T(0) ? T(0) : t;
  T sp = T(0), sm = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T pa = ev[a] > T(0) ? ev[a] : T(0);
    const T na = ev[a] - pa;
    sp += pa * pa;
    sm += na * na;
  }
  psip = T(0.5) * m.lam * tp * tp + m.mu * sp;
  psim = T(0.5) * m.lam * tm * tm + m.mu * sm;
}

// Strain energy split: psi+, psi-, sigma+ and sigma- (symmetric DIM x DIM),
// t = tr eps; for the spectral split also the principal strains and axes.
template <int DIM, typename T>
struct Split {
  T t, psip, psim, sigp[DIM][DIM], sigm[DIM][DIM];
  T ev[DIM], Q[DIM][DIM];
};

template <int DIM, typename T, int SK = kAnySplit>
RMTR_FN void split_parts(const MatP<T>& m, const T (&G)[DIM][DIM], Split<DIM, T>& s) {
  T t = T(0), epsq = T(0);
#pragma unroll
  for (int i = 0; i < DIM; ++i) t += G[i][i];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      T e = T(0.5) * (G[i][j] + G[j][i]);
      epsq += e * e;
    }
  s.t = t;
  if (spectral_split<SK>(m.split)) {
    T e[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) e[i][j] = T(0.5) * (G[i][j] + G[j][i]);
    spectral_parts<DIM, T, true>(m, e, t, s.psip, s.psim, s.sigp, s.sigm, s.ev, s.Q);
  } else if (m.split) {
    T tp = t > T(0) ? t : T(0);
    T tm = t > T(0) ? T(0) : t;
    s.psip = T(0.5) * m.K * tp * tp + m.mu * (epsq - t * t * m.third);
    s.psim = T(0.5) * m.K * tm * tm;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        T e = T(0.5) * (G[i][j] + G[j][i]);
        s.sigp[i][j] = T(2) * m.mu * e + (i == j ? (m.K * tp - m.mu23 * t) : T(0));
        s.sigm[i][j] = i == j ? m.K * tm : T(0);
      }
  } else {
    s.psip = T(0.5) * m.lam * t * t + m.mu * epsq;
    s.psim = T(0);
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        T e = T(0.5) * (G[i][j] + G[j][i]);
        s.sigp[i][j] = T(2) * m.mu * e + (i == j ? m.lam * t : T(0));
        s.sigm[i][j] = T(0);
      }
  }
}

// psi+ and psi- alone (the energy needs no stresses or axes).
template <int DIM, typename T, int SK = kAnySplit>
RMTR_FN void split_energy(const MatP<T>& m, const T (&G)[DIM][DIM], T& psip, T& psim, T& t) {
  t = T(0);
  T epsq = T(0), e[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) t += G[i][i];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      e[i][j] = T(0.5) * (G[i][j] + G[j][i]);
      epsq += e[i][j] * e[i][j];
    }
  if (spectral_split<SK>(m.split)) {
    spectral_energy<DIM, T>(m, e, t, psip, psim);
  } else if (m.split) {
    const T tp = t > T(0) ? t : T(0);
    const T tm = t > T(0) ? T(0) : t;
    psip = T(0.5) * m.K * tp * tp + m.mu * (epsq - t * t * m.third);
    psim = T(0.5) * m.K * tm * tm;
  } else {
    psip = T(0.5) * m.lam * t * t + m.mu * epsq;
    psim = T(0);
  }
}

// W at a quadrature point.
template <int DIM, typename T, int SK = kAnySplit>
RMTR_FN T density(const MatP<T>& m, const Zq<DIM, T>& z, T p, const T (&dp)[DIM]) {
  struct {
    T t, psip, psim;
  } s;
  split_energy<DIM, T, SK>(m, z.G, s.psip, s.psim, s.t);
  T omc = T(1) - z.c;
  T g = (T(1) - m.k) * omc * omc + m.k;
  T gp = omc * omc;
  T pi = p * s.t;
  T dcq = T(0);
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    pi += dp[i] * z.u[i];
    dcq += z.dc[i] * z.dc[i];
  }
  T crack = T(0.5) * (m.Gc_ls * z.c * z.c + m.Gc_l * dcq);
  return g * s.psip + s.psim + crack + gp * pi;
}

// dW/dz (first variation), written into out.
template <int DIM, typename T, int SK = kAnySplit>
RMTR_FN void density_grad(const MatP<T>& m, const Zq<DIM, T>& z, T p, const T (&dp)[DIM],
                                    Zq<DIM, T>& out) {
  Split<DIM, T> s;
  split_parts<DIM, T, SK>(m, z.G, s);
  T omc = T(1) - z.c;
  T g = (T(1) - m.k) * omc * omc + m.k;
  T dg = T(-2) * (T(1) - m.k) * omc;
  T gp = omc * omc;
  T dgp = T(-2) * omc;
  T pi = p * s.t;
#pragma unroll
  for (int i = 0; i < DIM; ++i) pi += dp[i] * z.u[i];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    out.u[i] = gp * dp[i];
    out.dc[i] = m.Gc_l * z.dc[i];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
      out.G[i][j] = g * s.sigp[i][j] + s.sigm[i][j] + (i == j ? gp * p : T(0));
  }
  out.c = dg * s.psip + m.Gc_ls * z.c + dgp * pi;
}

// Coefficients of the second variation at a linearisation point.
//   uu: vol tr(dG) tr(DG) + shear (dG:DG + dG:DG^T)
//       [+ sum_ab th_ab (Q^T sym dG Q)_ab (Q^T sym DG Q)_ab, spectral split:
//        th = 2 mu (g - 1) theta, Q the principal axes]
//   uc: S : dG Dc + Pc . du Dc (and symmetric)
//   cc: Ccc dc Dc + Gc l grad dc . grad Dc
template <int DIM, typename T>
struct HessCoef {
  T vol, shear, Ccc;
  T S[DIM][DIM];
  T Pc[DIM];
  T Q[DIM][DIM], th[DIM][DIM];  // spectral split only
};

template <int DIM, typename T, int SK = kAnySplit>
RMTR_FN void hess_coef(const MatP<T>& m, const Zq<DIM, T>& z, T p, const T (&dp)[DIM],
                                 HessCoef<DIM, T>& hc) {
  Split<DIM, T> s;
  split_parts<DIM, T, SK>(m, z.G, s);
  T omc = T(1) - z.c;
  T g = (T(1) - m.k) * omc * omc + m.k;
  T dg = T(-2) * (T(1) - m.k) * omc;
  T d2g = T(2) * (T(1) - m.k);
  T dgp = T(-2) * omc;
  T pi = p * s.t;
#pragma unroll
  for (int i = 0; i < DIM; ++i) pi += dp[i] * z.u[i];
  if (spectral_split<SK>(m.split)) {
    // lambda (g H+ + H-) tr tr + 2 mu dEps:DEps + 2 mu (g - 1) dEps+:DEps
    T Hp = s.t > T(0) ? T(1) : T(0);
    hc.vol = m.lam * (g * Hp + (T(1) - Hp));
    hc.shear = m.mu;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) hc.Q[i][j] = s.Q[i][j];
    spectral_theta<DIM, T>(s.ev, T(2) * m.mu * (g - T(1)), hc.th);
  } else if (m.split) {
    T Hp = s.t > T(0) ? T(1) : T(0);
    hc.vol = g * m.K * Hp + m.K * (T(1) - Hp) - g * m.mu23;
    hc.shear = g * m.mu;
  } else {
    hc.vol = g * m.lam;
    hc.shear = g * m.mu;
  }
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    hc.Pc[i] = dgp * dp[i];
#pragma unroll
    for (int j = 0; j < DIM; ++j) hc.S[i][j] = dg * s.sigp[i][j] + (i == j ? dgp * p : T(0));
  }
  hc.Ccc = d2g * s.psip + m.Gc_ls + T(2) * pi;
}

// Second variation applied to a direction v (z-vector of v at the point).
template <int DIM, typename T, int SK = kAnySplit>
RMTR_FN void hess_apply(const MatP<T>& m, const HessCoef<DIM, T>& hc, const Zq<DIM, T>& v,
                                  Zq<DIM, T>& out) {
  T tv = T(0);
#pragma unroll
  for (int i = 0; i < DIM; ++i) tv += v.G[i][i];
  T oc = hc.Ccc * v.c;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    out.u[i] = hc.Pc[i] * v.c;
    out.dc[i] = m.Gc_l * v.dc[i];
    oc += hc.Pc[i] * v.u[i];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      out.G[i][j] = hc.shear * (v.G[i][j] + v.G[j][i]) + hc.S[i][j] * v.c + (i == j ? hc.vol * tv : T(0));
      oc += hc.S[i][j] * v.G[i][j];
    }
  }
  out.c = oc;
  if (spectral_split<SK>(m.split)) spectral_apply<DIM, T>(hc.Q, hc.th, v.G, out.G);
}

// ------------------------------------------------------------------------
// Plain (not factorised) interpolation for any DIM: z_q = B_q x_e.
template <int DIM, typename T>
RMTR_FN void interp_q(int q, const T (&X)[1 << DIM][DIM + 1], T invh, Zq<DIM, T>& z) {
  zero<DIM, T>(z);
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a) {
    const T n = T(refN<DIM>(q, a));
#pragma unroll
    for (int i = 0; i < DIM; ++i) z.u[i] += n * X[a][i];
    z.c += n * X[a][DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const T dn = T(refdN<DIM>(q, a, j)) * invh;
#pragma unroll
      for (int i = 0; i < DIM; ++i) z.G[i][j] += dn * X[a][i];
      z.dc[j] += dn * X[a][DIM];
    }
  }
}

template <int DIM, typename T>
RMTR_FN void interp_scalar_q(int q, const T (&P)[1 << DIM], T invh, T& p, T (&dp)[DIM]) {
  p = T(0);
#pragma unroll
  for (int j = 0; j < DIM; ++j) dp[j] = T(0);
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a) {
    p += T(refN<DIM>(q, a)) * P[a];
#pragma unroll
    for (int j = 0; j < DIM; ++j) dp[j] += T(refdN<DIM>(q, a, j)) * invh * P[a];
  }
}

// r_a += w B_{q,a}^T out  for one local node a (all components).
template <int DIM, typename T>
RMTR_FN void project_q_node(int q, int a, T invh, T w, const Zq<DIM, T>& o, T (&r)[DIM + 1]) {
  const T n = T(refN<DIM>(q, a));
  T dn[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) dn[j] = T(refdN<DIM>(q, a, j)) * invh;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    T acc = n * o.u[i];
#pragma unroll
    for (int j = 0; j < DIM; ++j) acc += dn[j] * o.G[i][j];
    r[i] += w * acc;
  }
  T acc = n * o.c;
#pragma unroll
  for (int j = 0; j < DIM; ++j) acc += dn[j] * o.dc[j];
  r[DIM] += w * acc;
}

// ------------------------------------------------------------------------
// Sum-factorised Q1 interpolation on a hexahedron with the 2-point rule.
// f[a], a = ax + 2 ay + 4 az  ->  value and gradient (unit cell) at the 8
// points q = qx + 2 qy + 4 qz.
template <typename T>
RMTR_FN void sf_forward3(const T (&f)[8], T (&val)[8], T (&dx)[8], T (&dy)[8], T (&dz)[8]) {
  const T A0 = T(RMTR_GA), B0 = T(RMTR_GB);  // phi_0(q0), phi_1(q0)
  // stage x: fx[qx][ay][az], gx[ay][az]
  T fx[2][2][2], gx[2][2];
#pragma unroll
  for (int ay = 0; ay < 2; ++ay)
#pragma unroll
    for (int az = 0; az < 2; ++az) {
      T f0 = f[0 + 2 * ay + 4 * az], f1 = f[1 + 2 * ay + 4 * az];
      fx[0][ay][az] = A0 * f0 + B0 * f1;
      fx[1][ay][az] = B0 * f0 + A0 * f1;
      gx[ay][az] = f1 - f0;
    }
  // stage y
  T fxy[2][2][2], gxy[2][2], gyx[2][2];
#pragma unroll
  for (int az = 0; az < 2; ++az) {
#pragma unroll
    for (int qx = 0; qx < 2; ++qx) {
      fxy[qx][0][az] = A0 * fx[qx][0][az] + B0 * fx[qx][1][az];
      fxy[qx][1][az] = B0 * fx[qx][0][az] + A0 * fx[qx][1][az];
      gyx[qx][az] = fx[qx][1][az] - fx[qx][0][az];
    }
    gxy[0][az] = A0 * gx[0][az] + B0 * gx[1][az];
    gxy[1][az] = B0 * gx[0][az] + A0 * gx[1][az];
  }
  // stage z
#pragma unroll
  for (int qy = 0; qy < 2; ++qy)
#pragma unroll
    for (int qx = 0; qx < 2; ++qx) {
      const int q0 = qx + 2 * qy, q1 = q0 + 4;
      val[q0] = A0 * fxy[qx][qy][0] + B0 * fxy[qx][qy][1];
      val[q1] = B0 * fxy[qx][qy][0] + A0 * fxy[qx][qy][1];
      T d = fxy[qx][qy][1] - fxy[qx][qy][0];
      dz[q0] = d;
      dz[q1] = d;
      T gx0 = A0 * gxy[qy][0] + B0 * gxy[qy][1];
      T gx1 = B0 * gxy[qy][0] + A0 * gxy[qy][1];
      dx[q0] = gx0;
      dx[q1] = gx1;
      T gy0 = A0 * gyx[qx][0] + B0 * gyx[qx][1];
      T gy1 = B0 * gyx[qx][0] + A0 * gyx[qx][1];
      dy[q0] = gy0;
      dy[q1] = gy1;
    }
}

// Transpose of sf_forward3: r[a] += sum_q N_qa cv[q] + dN_qa . (cx, cy, cz)[q]
// (unit-cell derivatives; scale cx..cz by 1/h beforehand).
template <typename T>
RMTR_FN void sf_backward3(const T (&cv)[8], const T (&cx)[8], const T (&cy)[8], const T (&cz)[8],
                                    T (&r)[8]) {
  const T A0 = T(RMTR_GA), B0 = T(RMTR_GB);
  T Fxy[2][2][2], Gxy[2][2], Gyx[2][2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int az = 0; az < 2; ++az) {
      Gxy[q][az] = T(0);
      Gyx[q][az] = T(0);
    }
#pragma unroll
  for (int qy = 0; qy < 2; ++qy)
#pragma unroll
    for (int qx = 0; qx < 2; ++qx) {
      const int q0 = qx + 2 * qy, q1 = q0 + 4;
      T zz = cz[q0] + cz[q1];
      Fxy[qx][qy][0] = A0 * cv[q0] + B0 * cv[q1] - zz;
      Fxy[qx][qy][1] = B0 * cv[q0] + A0 * cv[q1] + zz;
      Gxy[qy][0] += A0 * cx[q0] + B0 * cx[q1];
      Gxy[qy][1] += B0 * cx[q0] + A0 * cx[q1];
      Gyx[qx][0] += A0 * cy[q0] + B0 * cy[q1];
      Gyx[qx][1] += B0 * cy[q0] + A0 * cy[q1];
    }
  T Fx[2][2][2], Gx[2][2];
#pragma unroll
  for (int az = 0; az < 2; ++az) {
#pragma unroll
    for (int qx = 0; qx < 2; ++qx) {
      Fx[qx][0][az] = A0 * Fxy[qx][0][az] + B0 * Fxy[qx][1][az] - Gyx[qx][az];
      Fx[qx][1][az] = B0 * Fxy[qx][0][az] + A0 * Fxy[qx][1][az] + Gyx[qx][az];
    }
    Gx[0][az] = A0 * Gxy[0][az] + B0 * Gxy[1][az];
    Gx[1][az] = B0 * Gxy[0][az] + A0 * Gxy[1][az];
  }
#pragma unroll
  for (int ay = 0; ay < 2; ++ay)
#pragma unroll
    for (int az = 0; az < 2; ++az) {
      r[0 + 2 * ay + 4 * az] += A0 * Fx[0][ay][az] + B0 * Fx[1][ay][az] - Gx[ay][az];
      r[1 + 2 * ay + 4 * az] += B0 * Fx[0][ay][az] + A0 * Fx[1][ay][az] + Gx[ay][az];
    }
}

// z-vectors at all 2^DIM points (3D: sum-factorised; 2D: plain).
template <int DIM, typename T>
RMTR_FN void elem_z(const T (&X)[1 << DIM][DIM + 1], T invh, Zq<DIM, T> (&z)[1 << DIM]) {
  if constexpr (DIM == 3) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      T f[8], val[8], dx[8], dy[8], dz[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) f[a] = X[a][k];
      sf_forward3<T>(f, val, dx, dy, dz);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (k < 3) {
          z[q].u[k] = val[q];
          z[q].G[k][0] = dx[q] * invh;
          z[q].G[k][1] = dy[q] * invh;
          z[q].G[k][2] = dz[q] * invh;
        } else {
          z[q].c = val[q];
          z[q].dc[0] = dx[q] * invh;
          z[q].dc[1] = dy[q] * invh;
          z[q].dc[2] = dz[q] * invh;
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < (1 << DIM); ++q) interp_q<DIM, T>(q, X, invh, z[q]);
  }
}

template <int DIM, typename T>
RMTR_FN void elem_pq(const T (&P)[1 << DIM], T invh, T (&pq)[1 << DIM], T (&dpq)[1 << DIM][DIM]) {
  if constexpr (DIM == 3) {
    T dx[8], dy[8], dz[8];
    sf_forward3<T>(P, pq, dx, dy, dz);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      dpq[q][0] = dx[q] * invh;
      dpq[q][1] = dy[q] * invh;
      dpq[q][2] = dz[q] * invh;
    }
  } else {
#pragma unroll
    for (int q = 0; q < (1 << DIM); ++q) interp_scalar_q<DIM, T>(q, P, invh, pq[q], dpq[q]);
  }
}

// r[a][k] = sum_q w B_{q,a}^T o_q for all nodes of the element.
template <int DIM, typename T>
RMTR_FN void elem_project(const Zq<DIM, T> (&o)[1 << DIM], T invh, T w, T (&r)[1 << DIM][DIM + 1]) {
  if constexpr (DIM == 3) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      T cv[8], cx[8], cy[8], cz[8], rr[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (k < 3) {
          cv[q] = w * o[q].u[k];
          cx[q] = w * invh * o[q].G[k][0];
          cy[q] = w * invh * o[q].G[k][1];
          cz[q] = w * invh * o[q].G[k][2];
        } else {
          cv[q] = w * o[q].c;
          cx[q] = w * invh * o[q].dc[0];
          cy[q] = w * invh * o[q].dc[1];
          cz[q] = w * invh * o[q].dc[2];
        }
        rr[q] = T(0);
      }
      sf_backward3<T>(cv, cx, cy, cz, rr);
#pragma unroll
      for (int a = 0; a < 8; ++a) r[a][k] = rr[a];
    }
  } else {
#pragma unroll
    for (int a = 0; a < (1 << DIM); ++a)
#pragma unroll
      for (int k = 0; k <= DIM; ++k) r[a][k] = T(0);
#pragma unroll
    for (int q = 0; q < (1 << DIM); ++q)
#pragma unroll
      for (int a = 0; a < (1 << DIM); ++a) project_q_node<DIM, T>(q, a, invh, w, o[q], r[a]);
  }
}

// ------------------------------------------------ per-element operators
// 3D element operators on unit-cell derivatives.  With G' = h grad (the
// derivative on the unit cell) the element's rows are
//   r = sum_q B'_q^T o_q,
// where o_q already carries the quadrature weight w and the 1/h of the
// test-function derivatives: o.u and o.c are scaled by w, o.G and o.dc by
// w / h.  The pointwise coefficients absorb these factors (a1 = w / h,
// a2 = w / h^2), so the interpolations and the projection need no scaling.
template <typename T>
struct ElemScale {
  T w, a1, a2;
};

template <typename T>
RMTR_FN ElemScale<T> elem_scale(T invh, T w) {
  ElemScale<T> e;
  e.w = w;
  e.a1 = w * invh;
  e.a2 = e.a1 * invh;
  return e;
}

// Split parts on unit-cell strains: psi' = h^2 psi, sig' = h sig, t' = h t
// (every split is positively homogeneous of degree 2 in the strain).
template <typename T>
RMTR_FN void split_unit(const MatP<T>& m, const T (&G)[3][3], T& t, T& psip, T (&sigp)[3][3], T& sigm) {
  t = G[0][0] + G[1][1] + G[2][2];
  T e[3][3], epsq = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      e[i][j] = T(0.5) * (G[i][j] + G[j][i]);
      epsq += e[i][j] * e[i][j];
    }
  T diag;
  if (m.split) {
    const T tp = t > T(0) ? t : T(0);
    const T tm = t > T(0) ? T(0) : t;
    psip = T(0.5) * m.K * tp * tp + m.mu * (epsq - t * t * m.third);
    diag = m.K * tp - m.mu23 * t;
    sigm = m.K * tm;
  } else {
    psip = T(0.5) * m.lam * t * t + m.mu * epsq;
    diag = m.lam * t;
    sigm = T(0);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) sigp[i][j] = T(2) * m.mu * e[i][j] + (i == j ? diag : T(0));
}

// Scaled first variation at one point: z holds unit-cell derivatives of
// u and c, dp the unit-cell gradient of p.
template <typename T, int SK = kNoSpectral>
RMTR_FN void density_grad_unit(const MatP<T>& m, const ElemScale<T>& sc, const Zq<3, T>& z, T p,
                               const T (&dp)[3], Zq<3, T>& o) {
  if constexpr (SK == kSplitSpectral) {
    // sigma- is a full tensor here
    const T t = z.G[0][0] + z.G[1][1] + z.G[2][2];
    T e[3][3], psip, psim, sigp[3][3], sigm[3][3], ev[3], Q[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) e[i][j] = T(0.5) * (z.G[i][j] + z.G[j][i]);
    spectral_parts<3, T, true>(m, e, t, psip, psim, sigp, sigm, ev, Q);
    const T omc = T(1) - z.c;
    const T g = (T(1) - m.k) * omc * omc + m.k;
    const T dg = T(-2) * (T(1) - m.k) * omc;
    const T gp = omc * omc;
    const T dgp = T(-2) * omc;
    T pi = p * t;
#pragma unroll
    for (int i = 0; i < 3; ++i) pi += dp[i] * z.u[i];
    const T dia = sc.a1 * gp * p;
    const T cdc = sc.a2 * m.Gc_l;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      o.u[i] = sc.a1 * gp * dp[i];
      o.dc[i] = cdc * z.dc[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) o.G[i][j] = sc.a2 * (g * sigp[i][j] + sigm[i][j]) + (i == j ? dia : T(0));
    }
    o.c = sc.a2 * dg * psip + sc.w * m.Gc_ls * z.c + sc.a1 * dgp * pi;
    return;
  }
  T t, psip, sigp[3][3], sigm;
  split_unit<T>(m, z.G, t, psip, sigp, sigm);
  const T omc = T(1) - z.c;
  const T g = (T(1) - m.k) * omc * omc + m.k;
  const T dg = T(-2) * (T(1) - m.k) * omc;
  const T gp = omc * omc;
  const T dgp = T(-2) * omc;
  T pi = p * t;
#pragma unroll
  for (int i = 0; i < 3; ++i) pi += dp[i] * z.u[i];
  const T a2g = sc.a2 * g;
  const T dia = sc.a2 * sigm + sc.a1 * gp * p;
  const T a1gp = sc.a1 * gp;
  const T cdc = sc.a2 * m.Gc_l;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o.u[i] = a1gp * dp[i];
    o.dc[i] = cdc * z.dc[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) o.G[i][j] = a2g * sigp[i][j] + (i == j ? dia : T(0));
  }
  o.c = sc.a2 * dg * psip + sc.w * m.Gc_ls * z.c + sc.a1 * dgp * pi;
}

// Scaled second-variation coefficients at the linearisation point.
template <typename T, int SK = kNoSpectral>
RMTR_FN void hess_coef_unit(const MatP<T>& m, const ElemScale<T>& sc, const Zq<3, T>& z, T p, const T (&dp)[3],
                            HessCoef<3, T>& hc) {
  T t, psip, sigp[3][3], sigm;
  T ev[3];
  if constexpr (SK == kSplitSpectral) {
    t = z.G[0][0] + z.G[1][1] + z.G[2][2];
    T e[3][3], psim, sgm[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) e[i][j] = T(0.5) * (z.G[i][j] + z.G[j][i]);
    spectral_parts<3, T, true>(m, e, t, psip, psim, sigp, sgm, ev, hc.Q);
    sigm = T(0);
  } else {
    split_unit<T>(m, z.G, t, psip, sigp, sigm);
  }
  const T omc = T(1) - z.c;
  const T g = (T(1) - m.k) * omc * omc + m.k;
  const T dg = T(-2) * (T(1) - m.k) * omc;
  const T d2g = T(2) * (T(1) - m.k);
  const T dgp = T(-2) * omc;
  T pi = p * t;
#pragma unroll
  for (int i = 0; i < 3; ++i) pi += dp[i] * z.u[i];
  if constexpr (SK == kSplitSpectral) {
    const T Hp = t > T(0) ? T(1) : T(0);
    hc.vol = sc.a2 * m.lam * (g * Hp + (T(1) - Hp));
    hc.shear = sc.a2 * m.mu;
    spectral_theta<3, T>(ev, sc.a2 * T(2) * m.mu * (g - T(1)), hc.th);
  } else {
    if (m.split) {
      const T Hp = t > T(0) ? T(1) : T(0);
      hc.vol = sc.a2 * (g * m.K * Hp + m.K * (T(1) - Hp) - g * m.mu23);
    } else {
      hc.vol = sc.a2 * g * m.lam;
    }
    hc.shear = sc.a2 * g * m.mu;
  }
  const T a2dg = sc.a2 * dg;
  const T a1dgp = sc.a1 * dgp;
  const T dia = a1dgp * p;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    hc.Pc[i] = a1dgp * dp[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) hc.S[i][j] = a2dg * sigp[i][j] + (i == j ? dia : T(0));
  }
  hc.Ccc = sc.a2 * d2g * psip + sc.w * m.Gc_ls + T(2) * sc.a1 * pi;
}

// Scaled second variation applied to v (unit-cell derivatives); cdc = a2 Gc l.
template <typename T, int SK = kNoSpectral>
RMTR_FN void hess_apply_unit(const HessCoef<3, T>& hc, T cdc, const Zq<3, T>& v, Zq<3, T>& o) {
  const T tv = v.G[0][0] + v.G[1][1] + v.G[2][2];
  T oc = hc.Ccc * v.c;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o.u[i] = hc.Pc[i] * v.c;
    o.dc[i] = cdc * v.dc[i];
    oc += hc.Pc[i] * v.u[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      o.G[i][j] = hc.shear * (v.G[i][j] + v.G[j][i]) + hc.S[i][j] * v.c + (i == j ? hc.vol * tv : T(0));
      oc += hc.S[i][j] * v.G[i][j];
    }
  }
  o.c = oc;
  if constexpr (SK == kSplitSpectral) spectral_apply<3, T>(hc.Q, hc.th, v.G, o.G);
}

// Values and unit-cell derivatives at the 8 points.
template <typename T>
RMTR_FN void elem_z_unit(const T (&X)[8][4], Zq<3, T> (&z)[8]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T f[8], val[8], dx[8], dy[8], dz[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) f[a] = X[a][k];
    sf_forward3<T>(f, val, dx, dy, dz);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (k < 3) {
        z[q].u[k] = val[q];
        z[q].G[k][0] = dx[q];
        z[q].G[k][1] = dy[q];
        z[q].G[k][2] = dz[q];
      } else {
        z[q].c = val[q];
        z[q].dc[0] = dx[q];
        z[q].dc[1] = dy[q];
        z[q].dc[2] = dz[q];
      }
    }
  }
}

template <typename T>
RMTR_FN void elem_project_unit(const Zq<3, T> (&o)[8], T (&r)[8][4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T cv[8], cx[8], cy[8], cz[8], rr[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (k < 3) {
        cv[q] = o[q].u[k];
        cx[q] = o[q].G[k][0];
        cy[q] = o[q].G[k][1];
        cz[q] = o[q].G[k][2];
      } else {
        cv[q] = o[q].c;
        cx[q] = o[q].dc[0];
        cy[q] = o[q].dc[1];
        cz[q] = o[q].dc[2];
      }
      rr[q] = T(0);
    }
    sf_backward3<T>(cv, cx, cy, cz, rr);
#pragma unroll
    for (int a = 0; a < 8; ++a) r[a][k] = rr[a];
  }
}

// MODE 0: gradient of f at X.  MODE 1: Hessian at X applied to V.  SK:
// kNoSpectral or kSplitSpectral (the split family the code carries).
template <int MODE, typename T, int SK = kNoSpectral>
struct ElemOp3 {
  // computes r[8][4] for one element
  __host__ __device__ static inline void eval(const MatP<T>& m, T invh, T w, const T (&X)[8][4], const T (&V)[8][4],
                                     const T (&P)[8], T (&r)[8][4]) {
    const ElemScale<T> sc = elem_scale<T>(invh, w);
    T pq[8], dpx[8], dpy[8], dpz[8];
    sf_forward3<T>(P, pq, dpx, dpy, dpz);
    Zq<3, T> o[8];
    {
      Zq<3, T> z[8];
      elem_z_unit<T>(X, z);
      if (MODE == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const T dp[3] = {dpx[q], dpy[q], dpz[q]};
          density_grad_unit<T, SK>(m, sc, z[q], pq[q], dp, o[q]);
        }
      } else if (SK == kSplitSpectral) {
        // the spectral coefficients carry the principal axes: form each
        // point's coefficients and apply them at once rather than keeping
        // all eight
        elem_z_unit<T>(V, o);
        const T cdc = sc.a2 * m.Gc_l;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const T dp[3] = {dpx[q], dpy[q], dpz[q]};
          HessCoef<3, T> hc;
          hess_coef_unit<T, SK>(m, sc, z[q], pq[q], dp, hc);
          Zq<3, T> vq = o[q];
          hess_apply_unit<T, SK>(hc, cdc, vq, o[q]);
        }
      } else {
        HessCoef<3, T> hc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const T dp[3] = {dpx[q], dpy[q], dpz[q]};
          hess_coef_unit<T>(m, sc, z[q], pq[q], dp, hc[q]);
        }
        elem_z_unit<T>(V, z);
        const T cdc = sc.a2 * m.Gc_l;
#pragma unroll
        for (int q = 0; q < 8; ++q) hess_apply_unit<T>(hc[q], cdc, z[q], o[q]);
      }
    }
    elem_project_unit<T>(o, r);
  }
};

// ------------------------------------------------------------------------
// Quarter-wise 3D element operators.  The 8 Gauss points of an element are
// taken two at a time: a quarter fixes the point's y and z coordinates
// (qy, qz) and holds the two points qx = 0, 1.  A quarter's values and
// unit-cell derivatives come from the element's 8 nodal values by one
// interpolation stage per direction (z, then y, then x), each written as
// f0 + xi (f1 - f0) so that the difference f1 - f0 is also the derivative
// along that direction; the adjoint runs the stages backwards.  Working on
// two points at a time keeps the per-element state small (the operator
// coefficients of two points, not eight), at the price of repeating the
// first two stages once per quarter.

// Gauss coordinate of point index q in one direction: xi_0 = 1 - xi_1.
template <typename T>
RMTR_FN T gauss_xi(int q) {
  return q ? T(RMTR_GA) : T(RMTR_GB);
}

// Values and unit-cell derivatives of one nodal field at the quarter's two
// points.  f[a], a = ax + 2 ay + 4 az; xz, xy the quarter's z and y Gauss
// coordinates.  dx is the same at both points.
template <typename T>
RMTR_FN void qtr_forward(const T (&f)[8], T xz, T xy, T (&val)[2], T& dx, T (&dy)[2], T (&dz)[2]) {
  T vz[2][2], gz[2][2];
#pragma unroll
  for (int ay = 0; ay < 2; ++ay)
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
      const T f0 = f[ax + 2 * ay], f1 = f[ax + 2 * ay + 4];
      gz[ax][ay] = f1 - f0;
      vz[ax][ay] = f0 + xz * gz[ax][ay];
    }
  T vy[2], gy[2], gzy[2];
#pragma unroll
  for (int ax = 0; ax < 2; ++ax) {
    gy[ax] = vz[ax][1] - vz[ax][0];
    vy[ax] = vz[ax][0] + xy * gy[ax];
    gzy[ax] = gz[ax][0] + xy * (gz[ax][1] - gz[ax][0]);
  }
  dx = vy[1] - vy[0];
  const T ddy = gy[1] - gy[0], ddz = gzy[1] - gzy[0];
#pragma unroll
  for (int qx = 0; qx < 2; ++qx) {
    const T xx = gauss_xi<T>(qx);
    val[qx] = vy[0] + xx * dx;
    dy[qx] = gy[0] + xx * ddy;
    dz[qx] = gzy[0] + xx * ddz;
  }
}

// Values only (a field whose gradient the operator does not need).
template <typename T>
RMTR_FN void qtr_forward_val(const T (&f)[8], T xz, T xy, T (&val)[2]) {
  T vy[2];
#pragma unroll
  for (int ax = 0; ax < 2; ++ax) {
    const T v0 = f[ax] + xz * (f[ax + 4] - f[ax]);
    const T v1 = f[ax + 2] + xz * (f[ax + 6] - f[ax + 2]);
    vy[ax] = v0 + xy * (v1 - v0);
  }
  const T dx = vy[1] - vy[0];
#pragma unroll
  for (int qx = 0; qx < 2; ++qx) val[qx] = vy[0] + gauss_xi<T>(qx) * dx;
}

// Transpose of qtr_forward: r[a] += sum over the two points of
// N_a cv + dN_a/dx cx + dN_a/dy cy + dN_a/dz cz (unit-cell derivatives).
template <typename T>
RMTR_FN void qtr_backward(const T (&cv)[2], const T (&cx)[2], const T (&cy)[2], const T (&cz)[2], T xz, T xy,
                          T (&r)[8]) {
  const T A = T(RMTR_GA), B = T(RMTR_GB);
  // x stage: the two points' weights back onto the x-nodes of the quarter
  const T sx = cx[0] + cx[1];
  T avy[2], agy[2], agz[2];
  avy[0] = A * cv[0] + B * cv[1] - sx;
  avy[1] = B * cv[0] + A * cv[1] + sx;
  agy[0] = A * cy[0] + B * cy[1];
  agy[1] = B * cy[0] + A * cy[1];
  agz[0] = A * cz[0] + B * cz[1];
  agz[1] = B * cz[0] + A * cz[1];
  // y stage, then z stage into the nodes
  const T wy0 = T(1) - xy, wz0 = T(1) - xz;
#pragma unroll
  for (int ax = 0; ax < 2; ++ax) {
    const T av0 = wy0 * avy[ax] - agy[ax], av1 = xy * avy[ax] + agy[ax];
    const T ag0 = wy0 * agz[ax], ag1 = xy * agz[ax];
    r[ax] += wz0 * av0 - ag0;
    r[ax + 4] += xz * av0 + ag0;
    r[ax + 2] += wz0 * av1 - ag1;
    r[ax + 6] += xz * av1 + ag1;
  }
}

// X-side quantities of one point that the operators need (unit cell):
// u, the symmetric strain parts, c, dc (gradient only), p, grad p.
template <typename T>
struct QPoint {
  T u[3];
  T G[3][3];
  T c;
  T dc[3];
  T p;
  T dp[3];
};

// Unit-cell split parts at one point, symmetric form: t = tr G', psip = h^2
// psi+, the diagonal and off-diagonal of sigma+' = h sigma+ (sig_ij for
// i < j in the order xy, xz, yz), sigm' the diagonal of sigma-' (h sigma-).
template <typename T>
RMTR_FN void split_sym_unit(const MatP<T>& m, const T (&G)[3][3], T& t, T& psip, T (&sd)[3], T (&so)[3], T& sigm) {
  t = G[0][0] + G[1][1] + G[2][2];
  const T e01 = T(0.5) * (G[0][1] + G[1][0]);
  const T e02 = T(0.5) * (G[0][2] + G[2][0]);
  const T e12 = T(0.5) * (G[1][2] + G[2][1]);
  const T epsq = G[0][0] * G[0][0] + G[1][1] * G[1][1] + G[2][2] * G[2][2] +
                 T(2) * (e01 * e01 + e02 * e02 + e12 * e12);
  T diag;
  if (m.split) {
    const T tp = t > T(0) ? t : T(0);
    const T tm = t > T(0) ? T(0) : t;
    psip = T(0.5) * m.K * tp * tp + m.mu * (epsq - t * t * m.third);
    diag = m.K * tp - m.mu23 * t;
    sigm = m.K * tm;
  } else {
    psip = T(0.5) * m.lam * t * t + m.mu * epsq;
    diag = m.lam * t;
    sigm = T(0);
  }
  const T mu2 = T(2) * m.mu;
#pragma unroll
  for (int i = 0; i < 3; ++i) sd[i] = mu2 * G[i][i] + diag;
  so[0] = mu2 * e01;
  so[1] = mu2 * e02;
  so[2] = mu2 * e12;
}

// Scaled second-variation coefficients at a point (unsplit or
// volumetric-deviatoric split) in symmetric form: S = Sd on the diagonal and
// So off it (xy, xz, yz).
template <typename T>
struct HessSym {
  T vol, shear, Ccc;
  T Sd[3], So[3], Pc[3];
};

// Products of the material constants and the element scale factors that
// the pointwise coefficients use, formed once per kernel (uniform).
template <typename T>
struct SymConst {
  int split;
  T k, omk;           // k, 1 - k
  T hK, mu3, K, mu23;  // K / 2, mu / 3, K, 2 mu / 3 (split); lambda / 2, 0, lambda, 0 (unsplit)
  T mu, mu2;          // mu, 2 mu
  T a2K, a2Kmu, a2mu23, a2mu;   // a2 K, a2 (K - 2 mu / 3), a2 2 mu / 3, a2 mu (unsplit: a2 lambda for K)
  T m2a2omk, m2a1;    // -2 a2 (1 - k), -2 a1: a2 g' / (1 - c), a1 gp' / (1 - c)
  T a2d2g, a1x2, wGcl;  // a2 g'', 2 a1, w Gc / l
  T a1, a2;
};

template <typename T>
RMTR_FN SymConst<T> sym_const(const MatP<T>& m, const ElemScale<T>& sc) {
  SymConst<T> c;
  c.split = m.split;
  c.k = m.k;
  c.omk = T(1) - m.k;
  c.mu = m.mu;
  c.mu2 = T(2) * m.mu;
  if (m.split) {
    c.hK = T(0.5) * m.K;
    c.mu3 = m.mu * m.third;
    c.K = m.K;
    c.mu23 = m.mu23;
  } else {
    c.hK = T(0.5) * m.lam;
    c.mu3 = T(0);
    c.K = m.lam;
    c.mu23 = T(0);
  }
  c.a2K = sc.a2 * c.K;
  c.a2mu23 = sc.a2 * c.mu23;
  c.a2Kmu = c.a2K - c.a2mu23;
  c.a2mu = sc.a2 * m.mu;
  c.m2a2omk = T(-2) * sc.a2 * c.omk;
  c.m2a1 = T(-2) * sc.a1;
  c.a2d2g = T(2) * sc.a2 * c.omk;
  c.a1x2 = T(2) * sc.a1;
  c.wGcl = sc.w * m.Gc_ls;
  c.a1 = sc.a1;
  c.a2 = sc.a2;
  return c;
}

// VD: the volumetric-deviatoric split (else the unsplit form), fixed at
// compile time so the kernels carry one form's arithmetic only.
template <typename T, bool VD>
RMTR_FN void hess_sym_coef(const SymConst<T>& k, const QPoint<T>& z, HessSym<T>& hc) {
  const T t = z.G[0][0] + z.G[1][1] + z.G[2][2];
  const T s01 = z.G[0][1] + z.G[1][0], s02 = z.G[0][2] + z.G[2][0], s12 = z.G[1][2] + z.G[2][1];
  // |eps|^2 = sum G_ii^2 + (s01^2 + s02^2 + s12^2) / 2
  const T epsq = z.G[0][0] * z.G[0][0] + z.G[1][1] * z.G[1][1] + z.G[2][2] * z.G[2][2] +
                 T(0.5) * (s01 * s01 + s02 * s02 + s12 * s12);
  // split: psi+ = K/2 <t>+^2 + mu (|eps|^2 - t^2 / 3), diag(sigma+) - 2 mu eps = K <t>+ - 2 mu t / 3;
  // unsplit: lambda/2 t^2 + mu |eps|^2 and lambda t (tp = t, mu3 = mu23 = 0)
  const T tp = VD ? (t > T(0) ? t : T(0)) : t;
  const T psip = VD ? k.hK * tp * tp + k.mu * epsq - k.mu3 * t * t : k.hK * t * t + k.mu * epsq;
  const T diag = VD ? k.K * tp - k.mu23 * t : k.K * t;
  const T omc = T(1) - z.c;
  const T g = k.omk * (omc * omc) + k.k;
  const T pi = z.p * t + z.dp[0] * z.u[0] + z.dp[1] * z.u[1] + z.dp[2] * z.u[2];
  // vol = a2 (g K H+ + K H- - g 2 mu / 3) (split), a2 g lambda (unsplit)
  hc.vol = VD ? (t > T(0) ? g * k.a2Kmu : k.a2K - g * k.a2mu23) : g * k.a2K;
  hc.shear = k.a2mu * g;
  const T a2dg = k.m2a2omk * omc;
  const T a1dgp = k.m2a1 * omc;
  const T dd = a2dg * diag + a1dgp * z.p;
  const T a2dg2mu = a2dg * k.mu2, a2dgmu = a2dg * k.mu;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    hc.Sd[i] = a2dg2mu * z.G[i][i] + dd;
    hc.Pc[i] = a1dgp * z.dp[i];
  }
  hc.So[0] = a2dgmu * s01;
  hc.So[1] = a2dgmu * s02;
  hc.So[2] = a2dgmu * s12;
  hc.Ccc = k.a2d2g * psip + (k.a1x2 * pi + k.wGcl);
}

// The coefficients applied to the direction v (unit-cell quantities); o is
// symmetric in G, so o.G[i][j] and o.G[j][i] are written from one value.
template <typename T>
RMTR_FN void hess_sym_apply(const HessSym<T>& hc, T cdc, const Zq<3, T>& v, Zq<3, T>& o) {
  const T tv = v.G[0][0] + v.G[1][1] + v.G[2][2];
  const T s01 = v.G[0][1] + v.G[1][0], s02 = v.G[0][2] + v.G[2][0], s12 = v.G[1][2] + v.G[2][1];
  const T vt = hc.vol * tv, sh2 = T(2) * hc.shear;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o.u[i] = hc.Pc[i] * v.c;
    o.dc[i] = cdc * v.dc[i];
    o.G[i][i] = sh2 * v.G[i][i] + hc.Sd[i] * v.c + vt;
  }
  o.G[0][1] = o.G[1][0] = hc.shear * s01 + hc.So[0] * v.c;
  o.G[0][2] = o.G[2][0] = hc.shear * s02 + hc.So[1] * v.c;
  o.G[1][2] = o.G[2][1] = hc.shear * s12 + hc.So[2] * v.c;
  o.c = hc.Ccc * v.c + hc.Pc[0] * v.u[0] + hc.Pc[1] * v.u[1] + hc.Pc[2] * v.u[2] + hc.Sd[0] * v.G[0][0] +
        hc.Sd[1] * v.G[1][1] + hc.Sd[2] * v.G[2][2] + hc.So[0] * s01 + hc.So[1] * s02 + hc.So[2] * s12;
}

// Scaled energy density at a point (unsplit or volumetric-deviatoric),
// w W from the unit-cell quantities: the strain energies are h^2 times the
// true ones and the pressure work h times, so
//   w W = a2 (g psi+' + psi-' + Gc l/2 |dc'|^2) + w Gc/(2 l) c^2 + a1 gp pi'.
template <typename T, bool VD>
RMTR_FN T energy_point_sym(const SymConst<T>& k, T a2Gcl2, const QPoint<T>& z) {
  const T t = z.G[0][0] + z.G[1][1] + z.G[2][2];
  const T s01 = z.G[0][1] + z.G[1][0], s02 = z.G[0][2] + z.G[2][0], s12 = z.G[1][2] + z.G[2][1];
  const T epsq = z.G[0][0] * z.G[0][0] + z.G[1][1] * z.G[1][1] + z.G[2][2] * z.G[2][2] +
                 T(0.5) * (s01 * s01 + s02 * s02 + s12 * s12);
  const T tp = VD ? (t > T(0) ? t : T(0)) : t;
  const T tm = VD ? (t > T(0) ? T(0) : t) : T(0);
  const T psip = VD ? k.hK * tp * tp + k.mu * epsq - k.mu3 * t * t : k.hK * t * t + k.mu * epsq;
  const T psim = VD ? k.hK * tm * tm : T(0);
  const T omc = T(1) - z.c;
  const T gp = omc * omc;
  const T g = k.omk * gp + k.k;
  const T pi = z.p * t + z.dp[0] * z.u[0] + z.dp[1] * z.u[1] + z.dp[2] * z.u[2];
  const T dcq = z.dc[0] * z.dc[0] + z.dc[1] * z.dc[1] + z.dc[2] * z.dc[2];
  return k.a2 * (g * psip + psim) + a2Gcl2 * dcq + T(0.5) * k.wGcl * z.c * z.c + k.a1 * gp * pi;
}

// Scaled first variation at a point (unsplit or volumetric-deviatoric),
// symmetric in G.
template <typename T, bool VD>
RMTR_FN void grad_point_sym(const SymConst<T>& k, T cdc, const QPoint<T>& z, Zq<3, T>& o) {
  const T t = z.G[0][0] + z.G[1][1] + z.G[2][2];
  const T s01 = z.G[0][1] + z.G[1][0], s02 = z.G[0][2] + z.G[2][0], s12 = z.G[1][2] + z.G[2][1];
  const T epsq = z.G[0][0] * z.G[0][0] + z.G[1][1] * z.G[1][1] + z.G[2][2] * z.G[2][2] +
                 T(0.5) * (s01 * s01 + s02 * s02 + s12 * s12);
  const T tp = VD ? (t > T(0) ? t : T(0)) : t;
  const T tm = VD ? (t > T(0) ? T(0) : t) : T(0);
  const T psip = VD ? k.hK * tp * tp + k.mu * epsq - k.mu3 * t * t : k.hK * t * t + k.mu * epsq;
  const T diag = VD ? k.K * tp - k.mu23 * t : k.K * t;
  const T sigm = VD ? k.K * tm : T(0);
  const T omc = T(1) - z.c;
  const T gp = omc * omc;
  const T g = k.omk * gp + k.k;
  const T pi = z.p * t + z.dp[0] * z.u[0] + z.dp[1] * z.u[1] + z.dp[2] * z.u[2];
  const T a2g = k.a2 * g;
  const T a1gp = k.a1 * gp;
  const T dia = a2g * diag + (k.a2 * sigm + a1gp * z.p);
  const T a2g2mu = a2g * k.mu2, a2gmu = a2g * k.mu;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o.u[i] = a1gp * z.dp[i];
    o.dc[i] = cdc * z.dc[i];
    o.G[i][i] = a2g2mu * z.G[i][i] + dia;
  }
  o.G[0][1] = o.G[1][0] = a2gmu * s01;
  o.G[0][2] = o.G[2][0] = a2gmu * s02;
  o.G[1][2] = o.G[2][1] = a2gmu * s12;
  o.c = (k.m2a2omk * omc) * psip + k.wGcl * z.c + (k.m2a1 * omc) * pi;
}

// Contribution of one element to the rows of its local node aloc:
// MODE 0 gradient of f at X, MODE 1 Hessian at X applied to V.
template <int DIM, typename T, int SK = kAnySplit>
RMTR_FN void node_contrib(int MODE, const MatP<T>& m, T invh, T w, const T (&X)[1 << DIM][DIM + 1],
                                    const T (&V)[1 << DIM][DIM + 1], const T (&P)[1 << DIM], int aloc,
                                    T (&r)[DIM + 1]) {
#pragma unroll
  for (int q = 0; q < (1 << DIM); ++q) {
    Zq<DIM, T> z, o;
    T pq, dpq[DIM];
    interp_scalar_q<DIM, T>(q, P, invh, pq, dpq);
    interp_q<DIM, T>(q, X, invh, z);
    if (MODE == 0) {
      density_grad<DIM, T, SK>(m, z, pq, dpq, o);
    } else {
      HessCoef<DIM, T> hc;
      hess_coef<DIM, T, SK>(m, z, pq, dpq, hc);
      interp_q<DIM, T>(q, V, invh, z);
      hess_apply<DIM, T, SK>(m, hc, z, o);
    }
    project_q_node<DIM, T>(q, aloc, invh, w, o, r);
  }
}


// Default Dirichlet set: every displacement component on the boundary.
template <int DIM>
RMTR_FN uint8_t default_mask(const int (&ijk)[DIM], int N) {
  bool b = false;
#pragma unroll
  for (int i = 0; i < DIM; ++i) b |= (ijk[i] == 0) | (ijk[i] == N);
  return b ? uint8_t((1u << DIM) - 1u) : uint8_t(0);
}

}  // namespace rmtr

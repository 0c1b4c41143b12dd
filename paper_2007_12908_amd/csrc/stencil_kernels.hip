// Assembled block stencils of the lagged Hessian, and the smoother and
// matrix-vector product that run on them.
//
// Sec. 4.2.1 takes one Hessian per level and V-cycle and reuses it for every
// smoothing step; Sec. 4.2.2 stores the diagonal blocks apart for the
// Gauss-Seidel sweeps.  Here each level's lagged Hessian is assembled once
// per V-cycle into a 3^d-point block stencil: for every node, (d+1) rows of
// 3^d x (d+1) values,
//   row (n, al), entry (o, be) = H[(n, al), (n + off(o), be)],
//   off(o) = (o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1),
// with rows and columns of Dirichlet dofs zero.  Storage is colour-major so
// that the threads of a Gauss-Seidel colour pass read consecutive addresses:
// nodes are grouped by colour (i%2 + 2 (j%2) + 4 (k%2)); node t of colour c
// (t = lexicographic index among the colour's nodes) keeps value k of its
// row block (k = (al 3^d + o)(d+1) + be) at
//   S[base[c] * RB + k * cnt[c] + t],   RB = (d+1) 3^d (d+1).
#include "rmtr_kernels.h"

namespace rmtr {
namespace {

constexpr int kB = 256;

template <int DIM>
constexpr int n_off() {
  return DIM == 3 ? 27 : 9;
}

template <int DIM>
constexpr int n_coef() {
  return 3 + DIM * DIM + DIM;  // vol, shear, Ccc, S (DIM x DIM), Pc (DIM)
}

template <int DIM>
constexpr int row_block() {
  return (DIM + 1) * n_off<DIM>() * (DIM + 1);
}

int gridn(int64_t work) {
  int64_t b = (work + kB - 1) / kB;
  if (b < 1) b = 1;
  if (b > 262140) b = 262140;
  return int(b);
}

// Colour geometry of one level.
struct Colours {
  int N;
  int64_t cnt[8];   // nodes per colour
  int64_t base[9];  // prefix sums of cnt
  int len[8][3];    // nodes per direction within a colour
};

Colours colours(int dim, int N) {
  Colours g{};
  g.N = N;
  g.base[0] = 0;
  for (int c = 0; c < (1 << dim); ++c) {
    int64_t n = 1;
    for (int i = 0; i < dim; ++i) {
      g.len[c][i] = (N - ((c >> i) & 1)) / 2 + 1;
      n *= g.len[c][i];
    }
    g.cnt[c] = n;
    g.base[c + 1] = g.base[c] + n;
  }
  return g;
}

// thread index -> (colour, index within colour, node coordinates, node id)
template <int DIM>
__device__ inline int locate(const Colours& g, int64_t id, int64_t& t, int (&c)[DIM], int64_t& n) {
  int col = 0;
#pragma unroll
  for (int k = 1; k < (1 << DIM); ++k)
    if (id >= g.base[k]) col = k;
  t = id - g.base[col];
  int64_t r = t, s = 1;
  n = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    c[i] = 2 * int(r % g.len[col][i]) + ((col >> i) & 1);
    r /= g.len[col][i];
    n += int64_t(c[i]) * s;
    s *= (g.N + 1);
  }
  return col;
}

// Second-variation coefficients at the 2^DIM quadrature points of every
// element, stored structure-of-arrays: C[(q n_coef + k) ne + e].
template <int DIM>
__global__ __launch_bounds__(kB) void k_coef(int N, double h, MatP<double> m, const double* __restrict__ x,
                                             const double* __restrict__ p, double* __restrict__ C) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, NK = n_coef<DIM>();
  int64_t ne = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) ne *= N;
  const int64_t ns = N + 1;
  const double invh = 1.0 / h;
  for (int64_t e = int64_t(blockIdx.x) * kB + threadIdx.x; e < ne; e += int64_t(gridDim.x) * kB) {
    int ec[DIM];
    int64_t r = e;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      ec[i] = int(r % N);
      r /= N;
    }
    double X[NL][NC], P[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      int64_t n = 0, s = 1;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        n += int64_t(ec[i] + ((a >> i) & 1)) * s;
        s *= ns;
      }
#pragma unroll
      for (int k = 0; k < NC; ++k) X[a][k] = x[NC * n + k];
      P[a] = p[n];
    }
    double pq[NL], dpq[NL][DIM];
    elem_pq<DIM, double>(P, invh, pq, dpq);
    Zq<DIM, double> z[NL];
    elem_z<DIM, double>(X, invh, z);
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      HessCoef<DIM, double> hc;
      hess_coef<DIM, double>(m, z[q], pq[q], dpq[q], hc);
      double* o = C + int64_t(q * NK) * ne + e;
      o[0 * ne] = hc.vol;
      o[1 * ne] = hc.shear;
      o[2 * ne] = hc.Ccc;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        o[int64_t(3 + DIM * DIM + i) * ne] = hc.Pc[i];
#pragma unroll
        for (int j = 0; j < DIM; ++j) o[int64_t(3 + DIM * i + j) * ne] = hc.S[i][j];
      }
    }
  }
}

// Element contributions of one parity class of elements (class bits =
// e_i % 2): elements of one class share no node, so each pass adds its
// contributions with plain read-modify-write, and the 2^d passes sum every
// entry in the same order.  A thread owns one element and one (local node a,
// component al) row block: the 2^d x (d+1) entries towards the element's
// local nodes b,
//   sum_q w B_{q,a,al}^T d2W_q B_{q,b,be}.
// Lanes take consecutive elements of the class, whose nodes a are
// consecutive nodes of one colour, so the stencil updates are coalesced.
// Blocks are laid out so that the 2^d (d+1) row planes of an element chunk
// run on the same XCD (block b: xcd = b % 8) and share its L2 for the
// coefficients.
template <int DIM, typename TO>
__global__ __launch_bounds__(kB) void k_st_elem(Colours g, double h, double gcl, int cls, int64_t ncls,
                                                int64_t nchunks, const double* __restrict__ C,
                                                const uint8_t* __restrict__ dir, TO* __restrict__ S) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, NK = n_coef<DIM>(), NO = n_off<DIM>(), RB = row_block<DIM>();
  constexpr int NPL = NL * NC;  // row planes (a, al)
  const int N = g.N;
  int64_t ne = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) ne *= N;
  const int64_t bid = blockIdx.x;
  const int xcd = int(bid % 8);
  const int64_t j = bid / 8;
  const int plane = int(j % NPL);
  const int64_t chunk = (j / NPL) * 8 + xcd;
  if (chunk >= nchunks) return;
  const int64_t k = chunk * kB + threadIdx.x;  // element index within the class
  if (k >= ncls) return;
  const int a = plane / NC, al = plane % NC;
  // element coordinates: e_i = 2 t_i + bit_i(cls)
  int e[DIM];
  {
    int64_t r = k;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const int bit = (cls >> i) & 1;
      const int len = (N - bit + 1) / 2;
      e[i] = 2 * int(r % len) + bit;
      r /= len;
    }
  }
  int64_t eid = 0, st = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    eid += int64_t(e[i]) * st;
    st *= N;
  }
  const double invh = 1.0 / h;
  double w = 1.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) w *= 0.5 * h;
  double acc[NL][NC];
#pragma unroll
  for (int b = 0; b < NL; ++b)
#pragma unroll
    for (int be = 0; be < NC; ++be) acc[b][be] = 0.0;
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const double* cf = C + int64_t(q * NK) * ne + eid;
    const double vol = cf[0], shear = cf[ne], ccc = cf[2 * ne];
    double Sr[DIM][DIM], Pc[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      Pc[i] = cf[int64_t(3 + DIM * DIM + i) * ne];
#pragma unroll
      for (int jj = 0; jj < DIM; ++jj) Sr[i][jj] = cf[int64_t(3 + DIM * i + jj) * ne];
    }
    // shape data of local node a (runtime a: select from the unrolled table)
    double Na = 0.0, dNa[DIM];
#pragma unroll
    for (int jj = 0; jj < DIM; ++jj) dNa[jj] = 0.0;
#pragma unroll
    for (int aa = 0; aa < NL; ++aa)
      if (aa == a) {
        Na = refN<DIM>(q, aa);
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) dNa[jj] = refdN<DIM>(q, aa, jj) * invh;
      }
    double dNal = 0.0, Sal[DIM], Pcal = 0.0;
#pragma unroll
    for (int jj = 0; jj < DIM; ++jj) Sal[jj] = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
      if (i == al) {
        dNal = dNa[i];
        Pcal = Pc[i];
#pragma unroll
        for (int jj = 0; jj < DIM; ++jj) Sal[jj] = Sr[i][jj];
      }
    double SdNa = 0.0;  // sum_j S[al][j] dNa[j]
#pragma unroll
    for (int jj = 0; jj < DIM; ++jj) SdNa += Sal[jj] * dNa[jj];
#pragma unroll
    for (int b = 0; b < NL; ++b) {
      const double Nb = refN<DIM>(q, b);
      double dNb[DIM];
      double dd = 0.0;
#pragma unroll
      for (int jj = 0; jj < DIM; ++jj) {
        dNb[jj] = refdN<DIM>(q, b, jj) * invh;
        dd += dNa[jj] * dNb[jj];
      }
      if (al < DIM) {
        double dNbal = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i)
          if (i == al) dNbal = dNb[i];
#pragma unroll
        for (int be = 0; be < DIM; ++be)
          acc[b][be] += w * (vol * dNal * dNb[be] + shear * ((al == be ? dd : 0.0) + dNa[be] * dNbal));
        acc[b][DIM] += w * (SdNa * Nb + Pcal * Na * Nb);
      } else {
#pragma unroll
        for (int be = 0; be < DIM; ++be) {
          double cu = Pc[be] * Na * Nb;
#pragma unroll
          for (int jj = 0; jj < DIM; ++jj) cu += Sr[be][jj] * dNb[jj] * Na;
          acc[b][be] += w * cu;
        }
        acc[b][DIM] += w * (ccc * Na * Nb + gcl * dd);
      }
    }
  }
  // node a of this element: colour and index within the colour
  int c[DIM];
  int col = 0;
  int64_t t = 0, n = 0, mul = 1, sn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    c[i] = e[i] + ((a >> i) & 1);
    col |= (c[i] & 1) << i;
  }
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    t += int64_t(c[i] >> 1) * mul;
    mul *= g.len[col][i];
    n += int64_t(c[i]) * sn;
    sn *= (N + 1);
  }
  const uint8_t mrow = dir ? dir[n] : default_mask<DIM>(c, N);
  if ((mrow >> al) & 1u) return;
  const int64_t cnt = g.cnt[col];
  TO* out = S + g.base[col] * RB + t;
#pragma unroll
  for (int b = 0; b < NL; ++b) {
    int m[DIM], o = 0, om = 1;
    int64_t mid = 0, s2 = 1;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      m[i] = e[i] + ((b >> i) & 1);
      o += (((b >> i) & 1) - ((a >> i) & 1) + 1) * om;
      om *= 3;
      mid += int64_t(m[i]) * s2;
      s2 *= (N + 1);
    }
    const uint8_t mcol = dir ? dir[mid] : default_mask<DIM>(m, N);
#pragma unroll
    for (int be = 0; be < NC; ++be) {
      if ((mcol >> be) & 1u) continue;
      TO* dst = out + int64_t((al * NO + o) * NC + be) * cnt;
      *dst = TO(double(*dst) + acc[b][be]);
    }
  }
}

__global__ __launch_bounds__(kB) void k_zero_d(int64_t n, double* __restrict__ a) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) a[i] = 0.0;
}

__global__ __launch_bounds__(kB) void k_zero_f(int64_t n, float* __restrict__ a) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) a[i] = 0.0f;
}

// Element matrices -> stencil: thread per (node, row al).
template <int DIM, typename TO>
__global__ __launch_bounds__(kB) void k_em_to_st(Colours g, const double* __restrict__ K, TO* __restrict__ S) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, ND = NL * NC, NO = n_off<DIM>(), RB = row_block<DIM>();
  const int N = g.N;
  const int64_t nodes = g.base[1 << DIM];
  for (int64_t it = int64_t(blockIdx.x) * kB + threadIdx.x; it < nodes * NC; it += int64_t(gridDim.x) * kB) {
    const int64_t id = it % nodes;
    const int al = int(it / nodes);
    int64_t t, n;
    int c[DIM];
    const int col = locate<DIM>(g, id, t, c, n);
    double acc[NO][NC];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int be = 0; be < NC; ++be) acc[o][be] = 0.0;
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      int e[DIM];
      bool ok = true;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        e[i] = c[i] - ((a >> i) & 1);
        ok &= (e[i] >= 0) & (e[i] < N);
      }
      if (!ok) continue;
      int64_t eid = 0, st = 1;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        eid += int64_t(e[i]) * st;
        st *= N;
      }
      const double* Ke = K + eid * ND * ND + (NC * a + al) * ND;
#pragma unroll
      for (int b = 0; b < NL; ++b) {
        int o = 0, mul = 1;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
          o += (((b >> i) & 1) - ((a >> i) & 1) + 1) * mul;
          mul *= 3;
        }
#pragma unroll
        for (int be = 0; be < NC; ++be) acc[o][be] += Ke[NC * b + be];
      }
    }
    const int64_t cnt = g.cnt[col];
    TO* out = S + g.base[col] * RB + t;
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int be = 0; be < NC; ++be) out[int64_t((al * NO + o) * NC + be) * cnt] = TO(acc[o][be]);
  }
}

// y = H v: thread per row (node, al); the rows of one component al form
// consecutive work items, so lanes read consecutive stencil values.
template <int DIM, typename T>
__global__ __launch_bounds__(kB) void k_st_mv(Colours g, const T* __restrict__ S, const T* __restrict__ v,
                                              T* __restrict__ y) {
  constexpr int NC = DIM + 1, NO = n_off<DIM>(), RB = row_block<DIM>();
  const int N = g.N;
  const int64_t nodes = g.base[1 << DIM];
  const int64_t ns = N + 1;
  for (int64_t it = int64_t(blockIdx.x) * kB + threadIdx.x; it < nodes * NC; it += int64_t(gridDim.x) * kB) {
    const int64_t id = it % nodes;
    const int al = int(it / nodes);
    int64_t t, n;
    int c[DIM];
    const int col = locate<DIM>(g, id, t, c, n);
    const int64_t cnt = g.cnt[col];
    const T* Sn = S + g.base[col] * RB + int64_t(al * NO * NC) * cnt + t;
    T acc = T(0);
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
      for (int be = 0; be < NC; ++be) acc += Sn[int64_t(o * NC + be) * cnt] * v[NC * m + be];
    }
    y[NC * n + al] = acc;
  }
}

// Gershgorin bound: row sums of |H| (max as -min in the last slot) and g^T g.
template <int DIM>
__global__ __launch_bounds__(kB) void k_st_rowabs(Colours g, const double* __restrict__ S,
                                                  const double* __restrict__ gv, double* __restrict__ partials) {
  constexpr int NC = DIM + 1, NO = n_off<DIM>(), RB = row_block<DIM>();
  __shared__ double sh[2][kB];
  const int64_t nodes = g.base[1 << DIM];
  double mn = INFINITY, gg = 0.0;
  for (int64_t id = int64_t(blockIdx.x) * kB + threadIdx.x; id < nodes; id += int64_t(gridDim.x) * kB) {
    int64_t t, n;
    int c[DIM];
    const int col = locate<DIM>(g, id, t, c, n);
    const int64_t cnt = g.cnt[col];
    const double* Sn = S + g.base[col] * RB + t;
    for (int al = 0; al < NC; ++al) {
      double rs = 0.0;
      for (int j = 0; j < NO * NC; ++j) rs += fabs(Sn[int64_t(al * NO * NC + j) * cnt]);
      mn = fmin(mn, -rs);
      gg += gv[NC * n + al] * gv[NC * n + al];
    }
  }
  const int tid = threadIdx.x;
  sh[0][tid] = gg;
  sh[1][tid] = mn;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sh[0][tid] += sh[0][tid + s];
      sh[1][tid] = fmin(sh[1][tid], sh[1][tid + s]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    partials[5 * blockIdx.x + 0] = sh[0][0];
    partials[5 * blockIdx.x + 1] = 0.0;
    partials[5 * blockIdx.x + 2] = 0.0;
    partials[5 * blockIdx.x + 3] = 0.0;
    partials[5 * blockIdx.x + 4] = sh[1][0];
  }
}

template <typename T>
__device__ inline T pgs_update_st(T s, T r, T d, T lo, T hi) {
  if (d > T(1e-300)) {
    T u = s - r / d;
    u = u < lo ? lo : u;
    u = u > hi ? hi : u;
    return u;
  }
  const T tl = lo - s, th = hi - s;
  const T ml = r * tl + T(0.5) * d * tl * tl;
  const T mh = r * th + T(0.5) * d * th * th;
  return mh < ml ? hi : lo;
}

// One colour pass of projected Gauss-Seidel: a thread per node of colour
// `col`; the components are updated in order (backward: reverse) with the
// node's diagonal block (offset (3^d - 1) / 2).
template <int DIM, typename T>
__global__ __launch_bounds__(kB) void k_st_pgs(Colours g, int col, int backward, const T* __restrict__ S,
                                               const uint8_t* __restrict__ dir, const T* __restrict__ gv,
                                               const T* __restrict__ lo, const T* __restrict__ hi,
                                               T* __restrict__ s) {
  constexpr int NC = DIM + 1, NO = n_off<DIM>(), CEN = (NO - 1) / 2, RB = row_block<DIM>();
  const int N = g.N;
  const int64_t ns = N + 1;
  const int64_t cnt = g.cnt[col];
  for (int64_t t = int64_t(blockIdx.x) * kB + threadIdx.x; t < cnt; t += int64_t(gridDim.x) * kB) {
    int c[DIM];
    int64_t r_ = t, n = 0, st = 1;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      c[i] = 2 * int(r_ % g.len[col][i]) + ((col >> i) & 1);
      r_ /= g.len[col][i];
      n += int64_t(c[i]) * st;
      st *= ns;
    }
    const uint8_t mk = dir ? dir[n] : default_mask<DIM>(c, N);
    if (mk == uint8_t((1u << NC) - 1u)) continue;
    const T* Sn = S + g.base[col] * RB + t;
    T r[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) r[k] = gv[NC * n + k];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      int64_t m = 0, s2 = 1;
      bool ok = true;
      int oo = o;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        const int mi = c[i] + oo % 3 - 1;
        oo /= 3;
        ok &= (mi >= 0) & (mi <= N);
        m += int64_t(mi) * s2;
        s2 *= ns;
      }
      if (!ok) continue;
      T sv[NC];
#pragma unroll
      for (int be = 0; be < NC; ++be) sv[be] = s[NC * m + be];
#pragma unroll
      for (int al = 0; al < NC; ++al)
#pragma unroll
        for (int be = 0; be < NC; ++be) r[al] += Sn[int64_t((al * NO + o) * NC + be) * cnt] * sv[be];
    }
    T sn[NC], s0[NC], D[NC][NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      s0[k] = s[NC * n + k];
      sn[k] = s0[k];
#pragma unroll
      for (int l = 0; l < NC; ++l) D[k][l] = Sn[int64_t((k * NO + CEN) * NC + l) * cnt];
    }
#pragma unroll
    for (int kk = 0; kk < NC; ++kk) {
      const int k = backward ? NC - 1 - kk : kk;
      if (mk & (1u << k)) continue;
      T rk = r[k];
#pragma unroll
      for (int l = 0; l < NC; ++l) rk += D[k][l] * (sn[l] - s0[l]);
      sn[k] = pgs_update_st<T>(sn[k], rk, D[k][k], lo[NC * n + k], hi[NC * n + k]);
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) s[NC * n + k] = sn[k];
  }
}

}  // namespace

size_t stencil_values(int dim, int N) {
  int64_t nn = 1;
  for (int i = 0; i < dim; ++i) nn *= (N + 1);
  return size_t(nn) * (dim + 1) * (dim == 3 ? 27 : 9) * (dim + 1);
}

size_t coef_values(int dim, int N) {
  int64_t ne = 1;
  for (int i = 0; i < dim; ++i) ne *= N;
  return size_t(ne) * (1 << dim) * (3 + dim * dim + dim);
}

template <int DIM, typename TO>
static hipError_t st_assemble_t(const ElemArgs& a, const double* xl, const double* p, double* coef, TO* S,
                                hipStream_t st) {
  constexpr int NL = 1 << DIM, NC = DIM + 1;
  int64_t ne = 1;
  for (int i = 0; i < DIM; ++i) ne *= a.N;
  const Colours g = colours(DIM, a.N);
  const double gcl = a.m.Gc * a.m.ls;
  const int64_t nval = int64_t(stencil_values(DIM, a.N));
  if (sizeof(TO) == 8)
    hipLaunchKernelGGL(k_zero_d, dim3(gridn(nval)), dim3(kB), 0, st, nval, (double*)S);
  else
    hipLaunchKernelGGL(k_zero_f, dim3(gridn(nval)), dim3(kB), 0, st, nval, (float*)S);
  hipLaunchKernelGGL(k_coef<DIM>, dim3(gridn(ne)), dim3(kB), 0, st, a.N, a.h, a.m, xl, p, coef);
  for (int cls = 0; cls < NL; ++cls) {
    int64_t ncls = 1;
    for (int i = 0; i < DIM; ++i) ncls *= (a.N - ((cls >> i) & 1) + 1) / 2;
    if (ncls == 0) continue;
    const int64_t nchunks = (ncls + kB - 1) / kB;
    const int64_t nblk = ((nchunks + 7) / 8) * 8 * (NL * NC);
    hipLaunchKernelGGL((k_st_elem<DIM, TO>), dim3(unsigned(nblk)), dim3(kB), 0, st, g, a.h, gcl, cls, ncls, nchunks,
                       coef, a.dir, S);
  }
  return hipGetLastError();
}

hipError_t launch_st_assemble(const ElemArgs& a, const double* xl, const double* p, double* coef, void* S,
                              int fp32, hipStream_t st) {
  if (a.dim == 3)
    return fp32 ? st_assemble_t<3, float>(a, xl, p, coef, (float*)S, st)
                : st_assemble_t<3, double>(a, xl, p, coef, (double*)S, st);
  return fp32 ? st_assemble_t<2, float>(a, xl, p, coef, (float*)S, st)
              : st_assemble_t<2, double>(a, xl, p, coef, (double*)S, st);
}

hipError_t launch_em_to_st(int dim, int N, const double* K, void* S, int fp32, hipStream_t st) {
  const Colours g = colours(dim, N);
  const dim3 gd(gridn(g.base[1 << dim] * (dim + 1)));
  if (dim == 3) {
    if (fp32)
      hipLaunchKernelGGL((k_em_to_st<3, float>), gd, dim3(kB), 0, st, g, K, (float*)S);
    else
      hipLaunchKernelGGL((k_em_to_st<3, double>), gd, dim3(kB), 0, st, g, K, (double*)S);
  } else {
    if (fp32)
      hipLaunchKernelGGL((k_em_to_st<2, float>), gd, dim3(kB), 0, st, g, K, (float*)S);
    else
      hipLaunchKernelGGL((k_em_to_st<2, double>), gd, dim3(kB), 0, st, g, K, (double*)S);
  }
  return hipGetLastError();
}

hipError_t launch_st_matvec(int dim, int N, const void* S, const void* v, void* y, int fp32, hipStream_t st) {
  const Colours g = colours(dim, N);
  const dim3 gd(gridn(g.base[1 << dim] * (dim + 1)));
  if (dim == 3) {
    if (fp32)
      hipLaunchKernelGGL((k_st_mv<3, float>), gd, dim3(kB), 0, st, g, (const float*)S, (const float*)v, (float*)y);
    else
      hipLaunchKernelGGL((k_st_mv<3, double>), gd, dim3(kB), 0, st, g, (const double*)S, (const double*)v,
                         (double*)y);
  } else {
    if (fp32)
      hipLaunchKernelGGL((k_st_mv<2, float>), gd, dim3(kB), 0, st, g, (const float*)S, (const float*)v, (float*)y);
    else
      hipLaunchKernelGGL((k_st_mv<2, double>), gd, dim3(kB), 0, st, g, (const double*)S, (const double*)v,
                         (double*)y);
  }
  return hipGetLastError();
}

hipError_t launch_st_rowabs(int dim, int N, const double* S, const double* gv, double* partials, int* nblocks_out,
                            hipStream_t st) {
  const Colours g = colours(dim, N);
  int nb = gridn(g.base[1 << dim]);
  if (nb > 1024) nb = 1024;
  *nblocks_out = nb;
  if (dim == 3)
    hipLaunchKernelGGL(k_st_rowabs<3>, dim3(nb), dim3(kB), 0, st, g, S, gv, partials);
  else
    hipLaunchKernelGGL(k_st_rowabs<2>, dim3(nb), dim3(kB), 0, st, g, S, gv, partials);
  return hipGetLastError();
}

template <int DIM, typename T>
static hipError_t st_sweeps(int N, const T* S, const uint8_t* dir, const T* gv, const T* lo, const T* hi, T* s,
                            int n_sweeps, hipStream_t st) {
  constexpr int NCOL = 1 << DIM;
  const Colours g = colours(DIM, N);
  for (int it = 0; it < n_sweeps; ++it)
    for (int bw = 0; bw < 2; ++bw)
      for (int cc = 0; cc < NCOL; ++cc) {
        const int col = bw ? NCOL - 1 - cc : cc;
        hipLaunchKernelGGL((k_st_pgs<DIM, T>), dim3(gridn(g.cnt[col])), dim3(kB), 0, st, g, col, bw, S, dir, gv, lo,
                           hi, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

hipError_t launch_st_pgs(int dim, int N, const void* S, const uint8_t* dir, const void* g, const void* lo,
                         const void* hi, void* s, int n_sweeps, int fp32, hipStream_t st) {
  if (dim == 3) {
    if (fp32)
      return st_sweeps<3, float>(N, (const float*)S, dir, (const float*)g, (const float*)lo, (const float*)hi,
                                 (float*)s, n_sweeps, st);
    return st_sweeps<3, double>(N, (const double*)S, dir, (const double*)g, (const double*)lo, (const double*)hi,
                                (double*)s, n_sweeps, st);
  }
  if (fp32)
    return st_sweeps<2, float>(N, (const float*)S, dir, (const float*)g, (const float*)lo, (const float*)hi,
                               (float*)s, n_sweeps, st);
  return st_sweeps<2, double>(N, (const double*)S, dir, (const double*)g, (const double*)lo, (const double*)hi,
                              (double*)s, n_sweeps, st);
}

}  // namespace rmtr

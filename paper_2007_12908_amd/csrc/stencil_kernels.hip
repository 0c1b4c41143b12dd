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
// with rows and columns of Dirichlet dofs zero.  Storage is colour-major and
// chunked so that a wavefront of a Gauss-Seidel colour pass streams one
// contiguous block: nodes are grouped by colour (i%2 + 2 (j%2) + 4 (k%2)),
// each colour padded to a multiple of 64 nodes (pbase[c] = padded start);
// node t of colour c (t = lexicographic index among the colour's nodes)
// keeps value k of its row block (k = (al 3^d + o)(d+1) + be) at
//   S[(pbase[c] + 64 (t / 64)) RB + 64 k + t % 64],   RB = (d+1) 3^d (d+1).
#include "rmtr_kernels.h"
#include "stencil_layout.h"

namespace rmtr {
namespace {

constexpr int kB = 256;

// Coefficients per quadrature point: vol, shear, Ccc, S (DIM x DIM), Pc
// (DIM); the spectral split adds its principal axes Q and th (DIM x DIM each).
template <int DIM, bool SPEC>
constexpr int n_coef() {
  return 3 + DIM * DIM + DIM + (SPEC ? 2 * DIM * DIM : 0);
}

int gridn(int64_t work) {
  int64_t b = (work + kB - 1) / kB;
  if (b < 1) b = 1;
  if (b > 262140) b = 262140;
  return int(b);
}

// Second-variation coefficients at the 2^DIM quadrature points of every
// element, element-major: C[(e 2^DIM + q) n_coef + k].
template <int DIM, typename TC, bool SPEC>
__global__ __launch_bounds__(kB) void k_coef(int N, double h, MatP<double> m, const double* __restrict__ x,
                                             const double* __restrict__ p, TC* __restrict__ C) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, NK = n_coef<DIM, SPEC>(), NK0 = n_coef<DIM, false>();
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
      hess_coef<DIM, double, SPEC ? kSplitSpectral : kNoSpectral>(m, z[q], pq[q], dpq[q], hc);
      TC* o = C + (e * NL + q) * NK;
      if constexpr (SPEC) {
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            o[NK0 + DIM * i + j] = TC(hc.Q[i][j]);
            o[NK0 + DIM * DIM + DIM * i + j] = TC(hc.th[i][j]);
          }
      }
      o[0] = TC(hc.vol);
      o[1] = TC(hc.shear);
      o[2] = TC(hc.Ccc);
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        o[3 + DIM * DIM + i] = TC(hc.Pc[i]);
#pragma unroll
        for (int j = 0; j < DIM; ++j) o[3 + DIM * i + j] = TC(hc.S[i][j]);
      }
    }
  }
}

// Node-centric assembly: a thread owns one row (n, al) and, in 3D, one
// z-plane of its neighbour blocks (dz = pz - 1, 9 blocks); 2D has one plane
// of 9 blocks.  It sums, over the elements around n and their quadrature
// points,
//   w B_{q,a,al}^T d2W_q B_{q,b,be}     (n = local node a, neighbour = b),
// and writes each stencil value once (zero on Dirichlet rows and columns
// and towards missing neighbours), so no zeroing pass or read-modify-write
// is needed.  Work items run al fastest: the four rows of a node share the
// element coefficients they load, and consecutive nodes of a colour give
// coalesced stores.  The lagged Hessian is symmetric: in 3D only the 14
// blocks towards n itself and its upper neighbours (dz = 1; dz = 0 with
// dy = 1, or dy = 0 and dx = 1) are summed, and each of the 13 off-diagonal
// ones is stored twice, in n's row and, transposed, in the row of the
// neighbour m = n + off(o) towards n (offset 26 - o).
// Basis values and unit-cell gradients of the Q1 element at its Gauss
// points, [q][a][0] = N_a(q), [q][a][1 + j] = dN_a/dxi_j(q), as a constant
// table: the point index of the assembly's loop is uniform, so its entries
// come in through scalar loads instead of vector arithmetic.
template <int DIM, typename T>
struct RefTab {
  T v[1 << DIM][1 << DIM][DIM + 1];
};
template <int DIM, typename T>
constexpr RefTab<DIM, T> make_ref_tab() {
  RefTab<DIM, T> t{};
  for (int q = 0; q < (1 << DIM); ++q)
    for (int a = 0; a < (1 << DIM); ++a) {
      t.v[q][a][0] = T(refN<DIM>(q, a));
      for (int j = 0; j < DIM; ++j) t.v[q][a][1 + j] = T(refdN<DIM>(q, a, j));
    }
  return t;
}
template <int DIM, typename T>
__constant__ RefTab<DIM, T> kRefTab = make_ref_tab<DIM, T>();

template <int DIM, typename TO, bool SPEC>
__device__ inline void st_node_item(const Colours& g, double h, double gcl_d, const TO* __restrict__ C,
                                    const uint8_t* __restrict__ dir, TO* __restrict__ S, int al, int64_t id,
                                    int pz) {
  constexpr int NL = 1 << DIM, NC = DIM + 1, NK = n_coef<DIM, SPEC>(), NK0 = n_coef<DIM, false>(),
                NO = n_off<DIM>(), RB = row_block<DIM>();
  constexpr int NP = DIM == 3 ? 3 : 1, OPP = NO / NP;
  const int N = g.N;
  const int64_t ns = N + 1;
  using T = TO;  // arithmetic in the stencil's precision
  const T invh = T(1.0 / h);
  const T gcl = T(gcl_d);
  double wd = 1.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) wd *= 0.5 * h;
  const T w = T(wd);
  {
    int64_t t, n;
    int c[DIM];
    const int col = locate<DIM>(g, id, t, c, n);
    const uint8_t mrow = dir ? dir[n] : default_mask<DIM>(c, N);
    const bool row_fixed = (mrow >> al) & 1u;
    T acc[OPP][NC];
#pragma unroll
    for (int o = 0; o < OPP; ++o)
#pragma unroll
      for (int be = 0; be < NC; ++be) acc[o][be] = T(0);
    if (!row_fixed) {
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        // element e = c - bits(a); n is its local node a
        const int az = DIM == 3 ? (a >> 2) & 1 : 0;
        if (DIM == 3 && ((pz == 0 && az == 0) || (pz == 2 && az == 1))) continue;
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
        const T* cfe = C + eid * (NL * NK);
#pragma unroll 1
        for (int q = 0; q < NL; ++q) {
          const T* cf = cfe + q * NK;
          const T vol = cf[0], shear = cf[1], ccc = cf[2];
          T Sr[DIM][DIM], Pc[DIM];
#pragma unroll
          for (int i = 0; i < DIM; ++i) {
            Pc[i] = cf[3 + DIM * DIM + i];
#pragma unroll
            for (int jj = 0; jj < DIM; ++jj) Sr[i][jj] = cf[3 + DIM * i + jj];
          }
          const T Na = kRefTab<DIM, T>.v[q][a][0];
          T dNa[DIM];
#pragma unroll
          for (int jj = 0; jj < DIM; ++jj) dNa[jj] = kRefTab<DIM, T>.v[q][a][1 + jj] * invh;
          T dNal = T(0), Sal[DIM], Pcal = T(0);
#pragma unroll
          for (int jj = 0; jj < DIM; ++jj) Sal[jj] = T(0);
#pragma unroll
          for (int i = 0; i < DIM; ++i)
            if (i == al) {
              dNal = dNa[i];
              Pcal = Pc[i];
#pragma unroll
              for (int jj = 0; jj < DIM; ++jj) Sal[jj] = Sr[i][jj];
            }
          T SdNa = T(0);
#pragma unroll
          for (int jj = 0; jj < DIM; ++jj) SdNa += Sal[jj] * dNa[jj];
          // spectral split: the test function's projected strain
          // A_cd = (Q^T sym(e_al dNa^T) Q)_cd, weighted by th (Tha = th o A);
          // the entry towards (b, be) is then Q[be][:] . (Tha Q^T dNb)
          T Qs[DIM][DIM], Tha[DIM][DIM];
          if constexpr (SPEC) {
            T ya[DIM], Qal[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
              for (int jj = 0; jj < DIM; ++jj) Qs[i][jj] = cf[NK0 + DIM * i + jj];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
              T v = T(0);
#pragma unroll
              for (int jj = 0; jj < DIM; ++jj) v += dNa[jj] * Qs[jj][c];
              ya[c] = v;
              Qal[c] = T(0);
#pragma unroll
              for (int i = 0; i < DIM; ++i)
                if (i == al) Qal[c] = Qs[i][c];
            }
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
              for (int d2 = 0; d2 < DIM; ++d2)
                Tha[c][d2] = cf[NK0 + DIM * DIM + DIM * c + d2] * T(0.5) * (Qal[c] * ya[d2] + ya[c] * Qal[d2]);
          }
#pragma unroll
          for (int b = 0; b < NL; ++b) {
            const int bz = DIM == 3 ? (b >> 2) & 1 : 0;
            if (DIM == 3 && bz - az + 1 != pz) continue;
            // in-plane offset of node b relative to node a
            int o = 0, om = 1;
#pragma unroll
            for (int i = 0; i < (DIM == 3 ? 2 : DIM); ++i) {
              o += (((b >> i) & 1) - ((a >> i) & 1) + 1) * om;
              om *= 3;
            }
            // 3D: blocks towards lower neighbours are the transposes of
            // blocks the neighbour computes and stores for this node too
            if (DIM == 3 && pz == 1 && o < 4) continue;
            const T Nb = kRefTab<DIM, T>.v[q][b][0];
            T dNb[DIM];
            T dd = T(0);
#pragma unroll
            for (int jj = 0; jj < DIM; ++jj) {
              dNb[jj] = kRefTab<DIM, T>.v[q][b][1 + jj] * invh;
              dd += dNa[jj] * dNb[jj];
            }
            if (al < DIM) {
              T dNbal = T(0);
#pragma unroll
              for (int i = 0; i < DIM; ++i)
                if (i == al) dNbal = dNb[i];
#pragma unroll
              for (int be = 0; be < DIM; ++be)
                acc[o][be] += w * (vol * dNal * dNb[be] + shear * ((al == be ? dd : T(0)) + dNa[be] * dNbal));
              if constexpr (SPEC) {
                T yb[DIM], zb[DIM];
#pragma unroll
                for (int d2 = 0; d2 < DIM; ++d2) {
                  T v = T(0);
#pragma unroll
                  for (int jj = 0; jj < DIM; ++jj) v += dNb[jj] * Qs[jj][d2];
                  yb[d2] = v;
                }
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                  T v = T(0);
#pragma unroll
                  for (int d2 = 0; d2 < DIM; ++d2) v += Tha[c][d2] * yb[d2];
                  zb[c] = v;
                }
#pragma unroll
                for (int be = 0; be < DIM; ++be) {
                  T v = T(0);
#pragma unroll
                  for (int c = 0; c < DIM; ++c) v += Qs[be][c] * zb[c];
                  acc[o][be] += w * v;
                }
              }
              acc[o][DIM] += w * (SdNa * Nb + Pcal * Na * Nb);
            } else {
#pragma unroll
              for (int be = 0; be < DIM; ++be) {
                T cu = Pc[be] * Na * Nb;
#pragma unroll
                for (int jj = 0; jj < DIM; ++jj) cu += Sr[be][jj] * dNb[jj] * Na;
                acc[o][be] += w * cu;
              }
              acc[o][DIM] += w * (ccc * Na * Nb + gcl * dd);
            }
          }
        }
      }
    }
    TO* out = S + st_row<DIM>(g, col, t);
#pragma unroll
    for (int o = 0; o < OPP; ++o) {
      if (DIM == 3 && pz == 1 && o < 4) continue;
      const int of = o + OPP * pz;
      int m[DIM];
      bool inside = true;
      int64_t mid = 0, s2 = 1;
      int oo = of;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        m[i] = c[i] + oo % 3 - 1;
        oo /= 3;
        inside &= (m[i] >= 0) & (m[i] <= N);
        mid += int64_t(m[i]) * s2;
        s2 *= ns;
      }
      const uint8_t mcol = inside ? (dir ? dir[mid] : default_mask<DIM>(m, N)) : uint8_t(0xff);
      // 3D: the value is also entry (be, 26 - of, al) of neighbour m's row
      // block, a lower block that m's own work items skip
      TO* tr = nullptr;
      if (DIM == 3 && of > NO / 2 && inside) {
        const int cm = (m[0] & 1) + 2 * (m[1] & 1) + 4 * (m[2 % DIM] & 1);
        const int64_t tm = int64_t(m[0] >> 1) + int64_t(g.len[cm][0]) *
                                                    (int64_t(m[1] >> 1) + int64_t(g.len[cm][1]) * (m[2 % DIM] >> 1));
        tr = S + st_row<DIM>(g, cm, tm) + int64_t((NO - 1 - of) * NC + al) * kChunk;
      }
#pragma unroll
      for (int be = 0; be < NC; ++be) {
        const T v = (row_fixed || ((mcol >> be) & 1u)) ? T(0) : acc[o][be];
        out[((al * NO + of) * NC + be) * kChunk] = TO(v);
        if (tr) tr[int64_t(be * NO * NC) * kChunk] = TO(v);
      }
    }
    // 3D: blocks towards missing lower neighbours get no transposed value;
    // the plane-1 item writes them as zero
    if (DIM == 3 && pz == 1) {
#pragma unroll
      for (int k = 0; k < NO / 2; ++k) {
        const int d0 = c[0] + k % 3 - 1, d1 = c[1] + (k / 3) % 3 - 1, d2 = c[2 % DIM] + k / 9 - 1;
        if (d0 >= 0 && d0 <= N && d1 >= 0 && d1 <= N && d2 >= 0 && d2 <= N) continue;
#pragma unroll
        for (int be = 0; be < NC; ++be) out[((al * NO + k) * NC + be) * kChunk] = TO(0);
      }
    }
  }
}

// Work order.  2D: (al, node, plane) with al fastest over the colour-major
// node order.  3D: a workgroup takes one 64-node chunk of one colour and
// one plane (64 nodes x 4 rows); the workgroups that land on one XCD
// (b % 8) take chunks x, x + 8, ... and, for each, all 8 colours and 3
// planes in turn, so the element coefficients around a chunk are fetched
// into that XCD's L2 once and reused by the 24 workgroups that need them.
constexpr bool kBlockedOrder = true;

template <int DIM, typename TO, bool SPEC>
__global__ __launch_bounds__(kB) void k_st_node(Colours g, double h, double gcl, const TO* __restrict__ C,
                                                const uint8_t* __restrict__ dir, TO* __restrict__ S) {
  constexpr int NC = DIM + 1, NP = DIM == 3 ? 3 : 1;
  const int64_t nodes = g.base[1 << DIM];
  if constexpr (DIM == 3 && kBlockedOrder) {
    int64_t J = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) J = max(J, (g.cnt[c] + kChunk - 1) / kChunk);
    const int64_t nblk = 8 * 24 * ((J + 7) / 8);
    const int al = int(threadIdx.x) & 3;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
      const int x = int(b & 7);
      const int64_t k = b >> 3;
      const int inner = int(k % 24);
      const int col = inner & 7, pz = inner >> 3;
      const int64_t t = (x + 8 * (k / 24)) * kChunk + (threadIdx.x >> 2);
      // plane dz = -1 holds transposes of blocks computed elsewhere only
      if (pz > 0 && t < g.cnt[col]) st_node_item<DIM, TO, SPEC>(g, h, gcl, C, dir, S, al, g.base[col] + t, pz);
    }
  } else {
    const int64_t work = nodes * NC * NP;
    for (int64_t it = int64_t(blockIdx.x) * kB + threadIdx.x; it < work; it += int64_t(gridDim.x) * kB) {
      const int al = int(it % NC);
      const int64_t r1 = it / NC;
      st_node_item<DIM, TO, SPEC>(g, h, gcl, C, dir, S, al, r1 % nodes, int(r1 / nodes));
    }
  }
}

// ---------------------------------------------------------------- RAP
// Galerkin coarsening R S I of a block stencil (eq. (delta_terms)) for the
// nested trilinear (bilinear) prolongation, done one direction at a time:
// I = I_x (x) I_y (x) I_z, so R S I = R_z R_y R_x S I_x I_y I_z, and each
// factor maps a 3-point stencil direction to a 3-point one.  One pass
// coarsens direction D: output node C takes the fine rows a_D = 2 C_D + da
// (weight 1 for da = 0, 1/2 for da = +-1); an entry towards offset o_D in
// {-1, 0, 1} reaches the fine node b_D = a_D + o_D, whose coarse parents are
// J_D = C_D + e/2 (e = da + o_D even, weight 1) or C_D + (e -+ 1)/2 (odd,
// weight 1/2 each).  Components are not mixed (the prolongation is scalar).
// Intermediate stencils are node-major structure-of-arrays,
// T[k nn + node] with k = (al 3^d + o)(d+1) + be; the finest input and the
// coarse output use the colour-major layout above.  The last pass zeroes the
// rows and columns of the coarse Dirichlet dofs.
struct Box3 {
  int n[3];  // nodes per direction (n[2] = 1 in 2D)
};

template <int DIM>
__device__ inline int64_t colour_index(const Colours& g, const int (&a)[DIM], int64_t k) {
  constexpr int RB = row_block<DIM>();
  int col = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) col |= (a[i] & 1) << i;
  int64_t t = 0, mul = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    t += int64_t(a[i] >> 1) * mul;
    mul *= g.len[col][i];
  }
  return (g.pbase[col] + (t & ~int64_t(kChunk - 1))) * RB + k * kChunk + (t & (kChunk - 1));
}

template <int DIM>
__device__ inline int64_t box_index(const Box3& b, const int (&a)[DIM]) {
  int64_t id = 0, mul = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    id += int64_t(a[i]) * mul;
    mul *= b.n[i];
  }
  return id;
}

template <int DIM, int D, typename TI, typename TO, int IN_COL, int OUT_COL>
__global__ __launch_bounds__(kB) void k_st_rap1(Colours gin, Box3 bin, Colours gout, Box3 bout,
                                                const TI* __restrict__ Sin, TO* __restrict__ Sout,
                                                const uint8_t* __restrict__ dirc) {
  constexpr int NC = DIM + 1, NO = n_off<DIM>(), NOTH = NO / 3;
  int64_t nin = 1, nout = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    nin *= bin.n[i];
    nout *= bout.n[i];
  }
  const int64_t work = nout * NC * NOTH;
  for (int64_t it = int64_t(blockIdx.x) * kB + threadIdx.x; it < work; it += int64_t(gridDim.x) * kB) {
    const int64_t node = it % nout;
    const int64_t r1 = it / nout;
    const int al = int(r1 % NC);
    const int oth = int(r1 / NC);
    int C[DIM];
    {
      int64_t r = node;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        C[i] = int(r % bout.n[i]);
        r /= bout.n[i];
      }
    }
    // offset digits of the other directions (in order of increasing index)
    int od[DIM];
    {
      int r = oth;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        if (i == D) continue;
        od[i] = r % 3;
        r /= 3;
      }
    }
    double acc[3][NC];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int be = 0; be < NC; ++be) acc[j][be] = 0.0;
#pragma unroll
    for (int da = -1; da <= 1; ++da) {
      int a[DIM];
#pragma unroll
      for (int i = 0; i < DIM; ++i) a[i] = C[i];
      a[D] = 2 * C[D] + da;
      if (a[D] < 0 || a[D] >= bin.n[D]) continue;
      const double wa = da == 0 ? 1.0 : 0.5;
#pragma unroll
      for (int oD = 0; oD < 3; ++oD) {
        int o = 0, om = 1;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
          o += (i == D ? oD : od[i]) * om;
          om *= 3;
        }
        const int e = da + oD - 1;  // b_D - 2 C_D, in -2 .. 2
        double v[NC];
#pragma unroll
        for (int be = 0; be < NC; ++be) {
          const int64_t k = int64_t((al * NO + o) * NC + be);
          v[be] = IN_COL ? double(Sin[colour_index<DIM>(gin, a, k)]) : double(Sin[k * nin + box_index<DIM>(bin, a)]);
        }
        if ((e & 1) == 0) {
          const int J = e / 2 + 1;
#pragma unroll
          for (int be = 0; be < NC; ++be) acc[J][be] += wa * v[be];
        } else {
          const int J0 = (e - 1) / 2 + 1, J1 = (e + 1) / 2 + 1;
#pragma unroll
          for (int be = 0; be < NC; ++be) {
            acc[J0][be] += 0.5 * wa * v[be];
            acc[J1][be] += 0.5 * wa * v[be];
          }
        }
      }
    }
    bool row_fixed = false;
    if (OUT_COL) {
      const uint8_t mrow = dirc ? dirc[box_index<DIM>(bout, C)] : default_mask<DIM>(C, bout.n[0] - 1);
      row_fixed = (mrow >> al) & 1u;
    }
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      int o = 0, om = 1;
      int m[DIM];
      bool inside = true;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        const int di = i == D ? J : od[i];
        o += di * om;
        om *= 3;
        m[i] = C[i] + di - 1;
        inside &= (m[i] >= 0) & (m[i] < bout.n[i]);
      }
      uint8_t mcol = 0;
      if (OUT_COL && inside) mcol = dirc ? dirc[box_index<DIM>(bout, m)] : default_mask<DIM>(m, bout.n[0] - 1);
#pragma unroll
      for (int be = 0; be < NC; ++be) {
        const int64_t k = int64_t((al * NO + o) * NC + be);
        double val = acc[J][be];
        if (OUT_COL) {
          if (row_fixed || !inside || ((mcol >> be) & 1u)) val = 0.0;
          Sout[colour_index<DIM>(gout, C, k)] = TO(val);
        } else {
          Sout[k * nout + node] = TO(val);
        }
      }
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
    TO* out = S + st_row<DIM>(g, col, t);
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int be = 0; be < NC; ++be) out[((al * NO + o) * NC + be) * kChunk] = TO(acc[o][be]);
  }
}

// y = H v: a workgroup takes 64 consecutive rows of the al-major work order
// (so lanes read consecutive stencil values) and gives each of the three
// neighbour planes of the rows to one wavefront; the plane sums are added
// in LDS in a fixed order.
constexpr int kMvB = 3 * kChunk;

template <int DIM, typename T>
__global__ __launch_bounds__(kMvB) void k_st_mv(Colours g, const T* __restrict__ S, const T* __restrict__ v,
                                                T* __restrict__ y) {
  constexpr int NC = DIM + 1;
  __shared__ T part[2][kChunk];
  const int64_t nodes = g.base[1 << DIM], rows = nodes * NC;
  const int lane = threadIdx.x % kChunk, pl = threadIdx.x / kChunk;
  for (int64_t r0 = int64_t(blockIdx.x) * kChunk; r0 < rows; r0 += int64_t(gridDim.x) * kChunk) {
    const int64_t it = r0 + lane;
    T acc = T(0);
    int64_t n = 0;
    int al = 0;
    if (it < rows) {
      al = int(it / nodes);
      acc = st_row_plane<DIM>(g, S, v, it % nodes, al, pl, n);
    }
    if (pl > 0) part[pl - 1][lane] = acc;
    __syncthreads();
    if (pl == 0 && it < rows) y[NC * n + al] = (acc + part[0][lane]) + part[1][lane];
    __syncthreads();
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
    const double* Sn = S + st_row<DIM>(g, col, t);
    for (int al = 0; al < NC; ++al) {
      double rs = 0.0;
      for (int j = 0; j < NO * NC; ++j) rs += fabs(Sn[(al * NO * NC + j) * kChunk]);
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
// node's diagonal block (offset (3^d - 1) / 2).  MODE 0: forward, 1:
// backward, 2: forward then backward, 3: backward then forward.  The last
// two are two passes over the same colour in a row, where a symmetric sweep
// turns (the forward half ends on the colour the backward half starts
// with, and a backward half ends on the colour the next sweep starts
// with): the neighbours do not change in between, so the second component
// sweep continues from the same neighbour sum and the row is read once.
template <int DIM, typename T, int MODE>
__global__ __launch_bounds__(kB) void k_st_pgs(Colours g, int col, const T* __restrict__ S,
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
    const T* Sn = S + st_row<DIM>(g, col, t);
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
        for (int be = 0; be < NC; ++be) r[al] += Sn[((al * NO + o) * NC + be) * kChunk] * sv[be];
    }
    T sn[NC], s0[NC], D[NC][NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      s0[k] = s[NC * n + k];
      sn[k] = s0[k];
#pragma unroll
      for (int l = 0; l < NC; ++l) D[k][l] = Sn[((k * NO + CEN) * NC + l) * kChunk];
    }
#pragma unroll
    for (int pass = 0; pass < (MODE >= 2 ? 2 : 1); ++pass) {
      const bool backward = (MODE == 1 || MODE == 3) != (pass == 1);
#pragma unroll
      for (int kk = 0; kk < NC; ++kk) {
        const int k = backward ? NC - 1 - kk : kk;
        if (mk & (1u << k)) continue;
        T rk = r[k];
#pragma unroll
        for (int l = 0; l < NC; ++l) rk += D[k][l] * (sn[l] - s0[l]);
        sn[k] = pgs_update_st<T>(sn[k], rk, D[k][k], lo[NC * n + k], hi[NC * n + k]);
      }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) s[NC * n + k] = sn[k];
  }
}

}  // namespace

size_t stencil_values(int dim, int N) {
  const Colours g = colours(dim, N);
  return size_t(g.pbase[1 << dim]) * (dim + 1) * (dim == 3 ? 27 : 9) * (dim + 1);
}

size_t coef_values(int dim, int N, int split) {
  int64_t ne = 1;
  for (int i = 0; i < dim; ++i) ne *= N;
  return size_t(ne) * (1 << dim) * (3 + dim * dim + dim + (split == kSplitSpectral ? 2 * dim * dim : 0));
}

template <int DIM, typename TO>
static hipError_t st_assemble_t(const ElemArgs& a, const double* xl, const double* p, double* coef, TO* S,
                                hipStream_t st) {
  constexpr int NL = 1 << DIM, NC = DIM + 1;
  int64_t ne = 1;
  for (int i = 0; i < DIM; ++i) ne *= a.N;
  const Colours g = colours(DIM, a.N);
  const double gcl = a.m.Gc * a.m.ls;
  // coefficients in the stencil's precision (the FP32 stencil of the mixed
  // form is assembled from FP32 coefficients in FP32 arithmetic)
  TO* cf = reinterpret_cast<TO*>(coef);
  constexpr int NP = DIM == 3 ? 3 : 1;
  const int64_t work = g.base[NL] * NC * NP;
  if (a.m.split == kSplitSpectral) {
    hipLaunchKernelGGL((k_coef<DIM, TO, true>), dim3(gridn(ne)), dim3(kB), 0, st, a.N, a.h, a.m, xl, p, cf);
    hipLaunchKernelGGL((k_st_node<DIM, TO, true>), dim3(gridn(work)), dim3(kB), 0, st, g, a.h, gcl, cf, a.dir, S);
  } else {
    hipLaunchKernelGGL((k_coef<DIM, TO, false>), dim3(gridn(ne)), dim3(kB), 0, st, a.N, a.h, a.m, xl, p, cf);
    hipLaunchKernelGGL((k_st_node<DIM, TO, false>), dim3(gridn(work)), dim3(kB), 0, st, g, a.h, gcl, cf, a.dir, S);
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
  int64_t nb = (g.base[1 << dim] * (dim + 1) + kChunk - 1) / kChunk;
  if (nb > 262140) nb = 262140;
  const dim3 gd(static_cast<uint32_t>(nb)), tb(kMvB);
  if (dim == 3) {
    if (fp32)
      hipLaunchKernelGGL((k_st_mv<3, float>), gd, tb, 0, st, g, (const float*)S, (const float*)v, (float*)y);
    else
      hipLaunchKernelGGL((k_st_mv<3, double>), gd, tb, 0, st, g, (const double*)S, (const double*)v,
                         (double*)y);
  } else {
    if (fp32)
      hipLaunchKernelGGL((k_st_mv<2, float>), gd, tb, 0, st, g, (const float*)S, (const float*)v, (float*)y);
    else
      hipLaunchKernelGGL((k_st_mv<2, double>), gd, tb, 0, st, g, (const double*)S, (const double*)v,
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
  // the colour passes of the sweeps in order: colours 0 .. NCOL-1 forward,
  // then NCOL-1 .. 0 backward, per sweep; two passes in a row over the same
  // colour run as one launch (MODE 2 or 3)
  const int np = 2 * NCOL * n_sweeps;
  for (int i = 0; i < np;) {
    const int half = (i / NCOL) & 1, cc = i % NCOL;
    const int col = half ? NCOL - 1 - cc : cc;
    const bool twice = i + 1 < np && cc == NCOL - 1;  // the next pass is over the same colour
    const int mode = twice ? 2 + half : half;
    const dim3 gd(gridn(g.cnt[col])), tb(kB);
    switch (mode) {
      case 0: hipLaunchKernelGGL((k_st_pgs<DIM, T, 0>), gd, tb, 0, st, g, col, S, dir, gv, lo, hi, s); break;
      case 1: hipLaunchKernelGGL((k_st_pgs<DIM, T, 1>), gd, tb, 0, st, g, col, S, dir, gv, lo, hi, s); break;
      case 2: hipLaunchKernelGGL((k_st_pgs<DIM, T, 2>), gd, tb, 0, st, g, col, S, dir, gv, lo, hi, s); break;
      default: hipLaunchKernelGGL((k_st_pgs<DIM, T, 3>), gd, tb, 0, st, g, col, S, dir, gv, lo, hi, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    i += twice ? 2 : 1;
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

size_t st_rap_work_doubles(int dim, int Nf, int fp32) {
  const int Nc = Nf / 2;
  const size_t rb = size_t(dim == 3 ? row_block<3>() : row_block<2>());
  size_t a = 1, b = 1;
  for (int i = 0; i < dim; ++i) {
    a *= size_t(i == 0 ? Nc + 1 : Nf + 1);
    b *= size_t(i <= 1 ? Nc + 1 : Nf + 1);
  }
  const size_t vals = (a + (dim == 3 ? b : 0)) * rb;
  return fp32 ? (vals + 1) / 2 : vals;
}

// intermediates in the fine stencil's precision (FP32 from an FP32 fine
// stencil: half the work memory; the sums are FP64 in every pass)
template <int DIM, typename TI>
static hipError_t st_rap_t(int Nf, const TI* Sf, double* Sc, const uint8_t* dirc, double* work, hipStream_t st) {
  const int Nc = Nf / 2;
  const Colours gf = colours(DIM, Nf), gc = colours(DIM, Nc);
  Box3 b0{{Nf + 1, Nf + 1, DIM == 3 ? Nf + 1 : 1}};
  Box3 b1{{Nc + 1, Nf + 1, DIM == 3 ? Nf + 1 : 1}};
  Box3 b2{{Nc + 1, Nc + 1, DIM == 3 ? Nf + 1 : 1}};
  Box3 b3{{Nc + 1, Nc + 1, DIM == 3 ? Nc + 1 : 1}};
  constexpr int NC = DIM + 1, NOTH = n_off<DIM>() / 3;
  auto grid = [&](const Box3& b) {
    int64_t n = int64_t(b.n[0]) * b.n[1] * b.n[2];
    return dim3(gridn(n * NC * NOTH));
  };
  TI* T1 = reinterpret_cast<TI*>(work);
  if constexpr (DIM == 3) {
    TI* T2 = T1 + int64_t(b1.n[0]) * b1.n[1] * b1.n[2] * row_block<DIM>();
    hipLaunchKernelGGL((k_st_rap1<DIM, 0, TI, TI, 1, 0>), grid(b1), dim3(kB), 0, st, gf, b0, gc, b1, Sf, T1, dirc);
    hipLaunchKernelGGL((k_st_rap1<DIM, 1, TI, TI, 0, 0>), grid(b2), dim3(kB), 0, st, gf, b1, gc, b2, T1, T2, dirc);
    hipLaunchKernelGGL((k_st_rap1<DIM, 2, TI, double, 0, 1>), grid(b3), dim3(kB), 0, st, gf, b2, gc, b3, T2, Sc,
                       dirc);
  } else {
    hipLaunchKernelGGL((k_st_rap1<DIM, 0, TI, TI, 1, 0>), grid(b1), dim3(kB), 0, st, gf, b0, gc, b1, Sf, T1, dirc);
    hipLaunchKernelGGL((k_st_rap1<DIM, 1, TI, double, 0, 1>), grid(b3), dim3(kB), 0, st, gf, b1, gc, b3, T1, Sc,
                       dirc);
  }
  return hipGetLastError();
}

hipError_t launch_st_rap(int dim, int Nf, const void* Sf, int fp32, double* Sc, const uint8_t* dirc, double* work,
                         hipStream_t st) {
  if (dim == 3)
    return fp32 ? st_rap_t<3, float>(Nf, (const float*)Sf, Sc, dirc, work, st)
                : st_rap_t<3, double>(Nf, (const double*)Sf, Sc, dirc, work, st);
  return fp32 ? st_rap_t<2, float>(Nf, (const float*)Sf, Sc, dirc, work, st)
              : st_rap_t<2, double>(Nf, (const double*)Sf, Sc, dirc, work, st);
}

}  // namespace rmtr

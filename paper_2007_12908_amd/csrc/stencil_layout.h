// Storage of the assembled block stencils of the lagged Hessian (Sec. 4.2.1):
// for every node, (d+1) rows of 3^d x (d+1) values,
//   row (n, al), entry (o, be) = H[(n, al), (n + off(o), be)],
//   off(o) = (o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1),
// colour-major and chunked: nodes are grouped by colour
// (i%2 + 2 (j%2) + 4 (k%2)), each colour padded to a multiple of 64 nodes
// (pbase[c] = padded start); node t of colour c keeps value
// k = (al 3^d + o)(d+1) + be of its row block at
//   S[(pbase[c] + 64 (t / 64)) RB + 64 k + t % 64],   RB = (d+1) 3^d (d+1).
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace rmtr {
namespace {

template <int DIM>
constexpr int n_off() {
  return DIM == 3 ? 27 : 9;
}

template <int DIM>
constexpr int row_block() {
  return (DIM + 1) * n_off<DIM>() * (DIM + 1);
}

// Colour geometry of one level.
constexpr int kChunk = 64;  // nodes per stencil chunk (one wavefront)

struct Colours {
  int N;
  int64_t cnt[8];    // nodes per colour
  int64_t base[9];   // prefix sums of cnt
  int64_t pbase[9];  // prefix sums of cnt rounded up to kChunk
  int len[8][3];     // nodes per direction within a colour
};

inline Colours colours(int dim, int N) {
  Colours g{};
  g.N = N;
  g.base[0] = 0;
  g.pbase[0] = 0;
  for (int c = 0; c < (1 << dim); ++c) {
    int64_t n = 1;
    for (int i = 0; i < dim; ++i) {
      g.len[c][i] = (N - ((c >> i) & 1)) / 2 + 1;
      n *= g.len[c][i];
    }
    g.cnt[c] = n;
    g.base[c + 1] = g.base[c] + n;
    g.pbase[c + 1] = g.pbase[c] + (n + kChunk - 1) / kChunk * kChunk;
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

// start of the row block of node t of colour col; value k sits at + kChunk k
template <int DIM>
__device__ inline int64_t st_row(const Colours& g, int col, int64_t t) {
  return (g.pbase[col] + (t & ~int64_t(kChunk - 1))) * row_block<DIM>() + (t & (kChunk - 1));
}

// Part of row (node id of the al-major work order, component al) of H v:
// the 3^(d-1) neighbour blocks whose last coordinate is offset by pl - 1.
// The three planes of a row go to three wavefronts so that a small level
// still spreads over the chip; n returns the node.
template <int DIM, typename T>
__device__ inline T st_row_plane(const Colours& g, const T* __restrict__ S, const T* __restrict__ v, int64_t id,
                                 int al, int pl, int64_t& n) {
  constexpr int NC = DIM + 1, NO = n_off<DIM>(), NQ = NO / 3;
  int64_t t;
  int c[DIM];
  const int col = locate<DIM>(g, id, t, c, n);
  const int N = g.N;
  const int64_t ns = N + 1;
  const int ml = c[DIM - 1] + pl - 1;
  T acc = T(0);
  if (ml < 0 || ml > N) return acc;
  const T* Sp = S + st_row<DIM>(g, col, t) + int64_t((al * NO + pl * NQ) * NC) * kChunk;
  const int64_t mb = int64_t(ml) * (DIM == 3 ? ns * ns : ns);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int m0 = c[0] + q % 3 - 1;
    bool ok = m0 >= 0 && m0 <= N;
    int64_t m = mb + m0;
    if (DIM == 3) {
      const int m1 = c[1] + q / 3 - 1;
      ok = ok && m1 >= 0 && m1 <= N;
      m += int64_t(m1) * ns;
    }
    if (!ok) continue;
#pragma unroll
    for (int be = 0; be < NC; ++be) acc += Sp[(q * NC + be) * kChunk] * v[NC * m + be];
  }
  return acc;
}

}  // namespace
}  // namespace rmtr

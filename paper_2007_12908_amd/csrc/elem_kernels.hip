// Matrix-free element kernels on the Q1 grid: energy, energy difference,
// gradient, Hessian-vector product and node diagonal blocks.  FP64 throughout, with FP32 variants of the
// Hessian-based operators for the mixed-precision form.
#include <algorithm>
#include <type_traits>

#include "rmtr_kernels.h"

namespace rmtr {

namespace {

constexpr int kBlock = 256;

template <int DIM>
__device__ inline void node_ijk(int64_t n, int64_t nside, int (&ijk)[DIM]) {
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    ijk[i] = int(n % nside);
    n /= nside;
  }
}

template <int DIM>
__device__ inline int64_t node_id(const int (&ijk)[DIM], int64_t nside) {
  int64_t n = 0, s = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    n += int64_t(ijk[i]) * s;
    s *= nside;
  }
  return n;
}

template <int DIM>
__device__ inline uint8_t node_mask(const uint8_t* dir, int64_t n, const int (&ijk)[DIM], int N) {
  return dir ? dir[n] : default_mask<DIM>(ijk, N);
}

template <typename T>
__device__ inline MatP<T> cast_mat(const MatP<double>& m) {
  MatP<T> r;
  r.lam = T(m.lam);
  r.mu = T(m.mu);
  r.K = T(m.K);
  r.Gc = T(m.Gc);
  r.ls = T(m.ls);
  r.k = T(m.k);
  r.split = m.split;
  r.third = T(m.third);
  r.mu23 = T(m.mu23);
  r.Gc_ls = T(m.Gc_ls);
  r.Gc_l = T(m.Gc_l);
  return r;
}

// Block sum of one double per thread; thread 0 gets the result.
__device__ inline double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

// Load the 2^DIM nodes of element with lower corner e (node-major layout).
template <int DIM, typename TS, typename T>
__device__ inline void load_elem(const TS* x, const int (&e)[DIM], int64_t nside, T (&X)[1 << DIM][DIM + 1]) {
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a) {
    int c[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) c[i] = e[i] + ((a >> i) & 1);
    const int64_t n = node_id<DIM>(c, nside);
#pragma unroll
    for (int k = 0; k <= DIM; ++k) X[a][k] = T(x[(DIM + 1) * n + k]);
  }
}

template <int DIM, typename TS, typename T>
__device__ inline void load_elem_scalar(const TS* p, const int (&e)[DIM], int64_t nside, T (&P)[1 << DIM]) {
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a) {
    int c[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) c[i] = e[i] + ((a >> i) & 1);
    P[a] = T(p[node_id<DIM>(c, nside)]);
  }
}

// Zero the Dirichlet components of an element's nodal values.
template <int DIM, typename T>
__device__ inline void mask_elem(const uint8_t* dir, const int (&e)[DIM], int N, T (&X)[1 << DIM][DIM + 1]) {
  const int64_t nside = N + 1;
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a) {
    int c[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) c[i] = e[i] + ((a >> i) & 1);
    const uint8_t mk = node_mask<DIM>(dir, node_id<DIM>(c, nside), c, N);
#pragma unroll
    for (int k = 0; k <= DIM; ++k)
      if (mk & (1u << k)) X[a][k] = T(0);
  }
}

// ------------------------------------------------------------------ energy
// One thread per element; per-block partial sums in a fixed order.
template <int DIM, typename TS, int SK>
__global__ __launch_bounds__(kBlock) void k_energy(int N, double h, MatP<double> m, const double* __restrict__ x,
                                                   const TS* __restrict__ s, const double* __restrict__ p,
                                                   double* __restrict__ partials) {
  __shared__ double sh[kBlock];
  const int64_t ne = int64_t(N) * N * (DIM == 3 ? N : 1);
  const int64_t nside = N + 1;
  const double invh = 1.0 / h;
  double w = 1.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) w *= 0.5 * h;
  double acc = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < ne; e += int64_t(gridDim.x) * blockDim.x) {
    int ec[DIM];
    int64_t r = e;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      ec[i] = int(r % N);
      r /= N;
    }
    double X[1 << DIM][DIM + 1], P[1 << DIM];
    load_elem<DIM, double, double>(x, ec, nside, X);
    load_elem_scalar<DIM, double, double>(p, ec, nside, P);
    double pq[1 << DIM], dpq[1 << DIM][DIM];
    elem_pq<DIM, double>(P, invh, pq, dpq);
    Zq<DIM, double> z[1 << DIM];
    elem_z<DIM, double>(X, invh, z);
    double we = 0.0;
    if (s == nullptr) {
#pragma unroll
      for (int q = 0; q < (1 << DIM); ++q) we += density<DIM, double, SK>(m, z[q], pq[q], dpq[q]);
    } else {
      double W0 = 0.0;
#pragma unroll
      for (int q = 0; q < (1 << DIM); ++q) W0 += density<DIM, double, SK>(m, z[q], pq[q], dpq[q]);
      double S[1 << DIM][DIM + 1];
      load_elem<DIM, TS, double>(s, ec, nside, S);
#pragma unroll
      for (int a = 0; a < (1 << DIM); ++a)
#pragma unroll
        for (int k = 0; k <= DIM; ++k) X[a][k] += S[a][k];
      elem_z<DIM, double>(X, invh, z);
      double W1 = 0.0;
#pragma unroll
      for (int q = 0; q < (1 << DIM); ++q) W1 += density<DIM, double, SK>(m, z[q], pq[q], dpq[q]);
      we = W1 - W0;
    }
    acc += w * we;
  }
  double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_reduce_partials(const double* __restrict__ partials, int n,
                                                            double* __restrict__ out) {
  __shared__ double sh[kBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
  double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = tot;
}

// 3D element-centric kernel: a 16 x 16 tile of element columns marches up
// in z; each element's 8 nodal contributions are exchanged through LDS and
// summed by the thread that owns the node, so no atomics are needed and the
// sum order is fixed.  Tiles overlap by one element column so that each
// tile owns the 15 x 15 nodes whose four in-plane elements it computes.
constexpr int kTile = 16;
constexpr int kOwn = kTile - 1;

// One column segment: the tile (bx, by) writes its owned nodes of node
// layers [z0, z1); it computes element layers z0 - 1 .. z1 - 1 (those that
// touch them).  The tile's node layers are staged in LDS: each
// node layer of the tile (17 x 17 nodes: x, v and p) is copied from memory
// into LDS by the asynchronous global-to-LDS loads, one layer ahead of the
// element layer that needs it, so the loads of the next layer overlap the
// arithmetic of the current one; each element then reads its eight nodes
// from LDS instead of from memory (a node is fetched once per tile, not once
// per element around it).
constexpr int kTN = kTile + 1;         // nodes per tile side
constexpr int kTNodes = kTN * kTN;     // nodes per tile layer

#define RMTR_LDS(ptr) ((void __attribute__((address_space(3)))*)(ptr))

template <typename T>
struct LayerLds {
  T x[3][kTNodes][4];
  T v[3][kTNodes][4];
  T p[3][kTNodes];
};

// The pieces one thread copies for every node layer of a tile: 16-byte
// pieces of x (and v) and 4-byte pieces of p.  Per round r the thread's piece
// is c = 256 r + tid; its node's in-plane offset (nodes outside the grid are
// clamped: only inactive elements see them) and the piece's byte offset
// within the node are the same for every layer, so they are formed once per
// column segment.
template <typename T>
struct DmaPlan {
  static constexpr int kCpn = 4 * int(sizeof(T)) / 16;  // 16-byte pieces per node (x or v)
  static constexpr int kPpn = int(sizeof(T)) / 4;       // 4-byte pieces per node (p)
  static constexpr int kRx = (kTNodes * kCpn + 255) / 256;
  static constexpr int kRp = (kTNodes * kPpn + 255) / 256;
  int xoff[kRx];  // byte offset of the piece in x (within a node layer), -1: none
  int poff[kRp];
};

template <typename T>
__device__ inline DmaPlan<T> dma_plan(int N, int bx, int by) {
  DmaPlan<T> d;
  const int tid = threadIdx.x;
  const int ns = N + 1;
  auto plane = [&](int node) {
    const int ix = node % kTN, iy = node / kTN;
    const int gx = min(max(bx * kOwn - 1 + ix, 0), N);
    const int gy = min(max(by * kOwn - 1 + iy, 0), N);
    return gx + ns * gy;
  };
#pragma unroll
  for (int r = 0; r < DmaPlan<T>::kRx; ++r) {
    const int c = r * 256 + tid;
    d.xoff[r] = c < kTNodes * DmaPlan<T>::kCpn
                    ? plane(c / DmaPlan<T>::kCpn) * 4 * int(sizeof(T)) + 16 * (c % DmaPlan<T>::kCpn)
                    : -1;
  }
#pragma unroll
  for (int r = 0; r < DmaPlan<T>::kRp; ++r) {
    const int c = r * 256 + tid;
    d.poff[r] = c < kTNodes * DmaPlan<T>::kPpn
                    ? plane(c / DmaPlan<T>::kPpn) * int(sizeof(T)) + 4 * (c % DmaPlan<T>::kPpn)
                    : -1;
  }
  return d;
}

// Copy node layer z of the tile into LDS slot `slot`.
template <int MODE, typename T>
__device__ inline void dma_layer(int N, const DmaPlan<T>& d, int z, int slot, const T* __restrict__ x,
                                 const T* __restrict__ p, const T* __restrict__ v, LayerLds<T>& L) {
  // the global-to-LDS copy exists in device code only (the host pass of a
  // template instantiated from several kernels would otherwise reject it)
#if defined(__HIP_DEVICE_COMPILE__)
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int64_t ns = N + 1;
  const int64_t zl = ns * ns * int64_t(z);
  const char* xz = reinterpret_cast<const char*>(x + 4 * zl);
  const char* vz = reinterpret_cast<const char*>(v + 4 * zl);
  const char* pz = reinterpret_cast<const char*>(p + zl);
#pragma unroll
  for (int r = 0; r < DmaPlan<T>::kRx; ++r) {
    if (d.xoff[r] >= 0) {
      char* xb = reinterpret_cast<char*>(&L.x[slot][0][0]) + (r * 256 + wave * 64) * 16;
      __builtin_amdgcn_global_load_lds(xz + d.xoff[r], RMTR_LDS(xb), 16, 0, 0);
      if (MODE == 1) {
        char* vb = reinterpret_cast<char*>(&L.v[slot][0][0]) + (r * 256 + wave * 64) * 16;
        __builtin_amdgcn_global_load_lds(vz + d.xoff[r], RMTR_LDS(vb), 16, 0, 0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < DmaPlan<T>::kRp; ++r) {
    if (d.poff[r] >= 0) {
      char* pb = reinterpret_cast<char*>(&L.p[slot][0]) + (r * 256 + wave * 64) * 4;
      __builtin_amdgcn_global_load_lds(pz + d.poff[r], RMTR_LDS(pb), 4, 0, 0);
    }
  }
#endif
}

template <int MODE, typename T, int SK>
__device__ inline void elem_segment3_lds(int N, const MatP<T>& m, T invh, T w, int bx, int by, int z0, int z1,
                                         const uint8_t* __restrict__ dir, const T* __restrict__ x,
                                         const T* __restrict__ p, const T* __restrict__ v, T* __restrict__ out,
                                         T (*lo_sh)[4][4], T (*hi_sh)[4][4], LayerLds<T>& L) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int ex = bx * kOwn - 1 + tx;
  const int ey = by * kOwn - 1 + ty;
  const int ox = ex + 1, oy = ey + 1;
  const bool ecol = ex >= 0 && ex < N && ey >= 0 && ey < N;
  const bool owner = tx < kOwn && ty < kOwn && ox <= N && oy <= N;
  const int64_t nside = N + 1;
  const int zs = max(z0 - 1, 0), ze = min(z1 - 1, N - 1);
  // node layers sit in a ring of three LDS slots: layer z in slot (z - zs) % 3
  const DmaPlan<T> dp = dma_plan<T>(N, bx, by);
  if (zs <= ze) {
    dma_layer<MODE, T>(N, dp, zs, 0, x, p, v, L);
    dma_layer<MODE, T>(N, dp, zs + 1, 1, x, p, v, L);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  T acc[4] = {T(0), T(0), T(0), T(0)};
  int sb = 0;
  for (int ez = zs; ez <= ze; ++ez) {
    const int st = sb == 2 ? 0 : sb + 1, sn = st == 2 ? 0 : st + 1;
    T X[8][4], V[8][4], P[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int node = (ty + ((a >> 1) & 1)) * kTN + tx + (a & 1);
      const int sl = (a >> 2) ? st : sb;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        X[a][k] = L.x[sl][node][k];
        V[a][k] = MODE == 1 ? L.v[sl][node][k] : T(0);
      }
      P[a] = L.p[sl][node];
    }
    const int ec[3] = {ex, ey, ez};
    if (MODE == 1 && ecol) mask_elem<3, T>(dir, ec, N, V);
    // node layer ez + 2 goes to the slot that held layer ez - 1 (last read
    // before the previous iteration's closing barrier); it is issued after
    // this element's reads (and its Dirichlet bits), so none of them waits
    // for it
    if (ez + 2 <= N && ez + 1 <= ze) dma_layer<MODE, T>(N, dp, ez + 2, sn, x, p, v, L);
    T r[8][4];
    if (ecol) {
      ElemOp3<MODE, T, SK>::eval(m, invh, w, X, V, P, r);
    } else {
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int k = 0; k < 4; ++k) r[a][k] = T(0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        lo_sh[tid][a][k] = r[a][k];
        hi_sh[tid][a][k] = r[a + 4][k];
      }
    __syncthreads();
    if (owner) {
      if (ez >= z0) {
        const int nz = ez;
        const int64_t n = int64_t(ox) + nside * (int64_t(oy) + nside * nz);
        const int c[3] = {ox, oy, nz};
        const uint8_t mk = node_mask<3>(dir, n, c, N);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          T s = acc[k] + lo_sh[tid][3][k] + lo_sh[tid + 1][2][k] + lo_sh[tid + 16][1][k] + lo_sh[tid + 17][0][k];
          out[4 * n + k] = (mk & (1u << k)) ? T(0) : s;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        acc[k] = hi_sh[tid][3][k] + hi_sh[tid + 1][2][k] + hi_sh[tid + 16][1][k] + hi_sh[tid + 17][0][k];
    }
    // layer ez + 2 is in LDS, slot sb is read and the exchange buffers are
    // free again
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    sb = st;
  }
  if (owner && ze + 1 < z1) {
    const int nz = ze + 1;
    const int64_t n = int64_t(ox) + nside * (int64_t(oy) + nside * nz);
    const int c[3] = {ox, oy, nz};
    const uint8_t mk = node_mask<3>(dir, n, c, N);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[4 * n + k] = (mk & (1u << k)) ? T(0) : acc[k];
  }
}

// 3D energy (and FP64 energy difference) on the same tiles: each tile
// column counts the elements it owns (tile-local column tx >= 1, the column
// tx = 0 belonging to the tile before it) and the element layers of its
// segment of node layers, so every element is counted exactly once; node
// layers are staged in LDS as for the scatter kernels (x in the x slots, the
// step s in the v slots).  Each workgroup writes one partial sum (threads in
// element order, then a fixed tree), so the result is deterministic.
template <bool DIFF, int SK>
__device__ inline double energy3_lds(int N, double h, const MatP<double>& m, int tiles, const double* __restrict__ x,
                                     const double* __restrict__ s, const double* __restrict__ p,
                                     LayerLds<double>& L) {
  constexpr int MODE = DIFF ? 1 : 0;  // stage the step in the v slots
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const double invh = 1.0 / h;
  const double w = h * h * h / 8.0;
  const int64_t nz = N + 1;
  const int64_t work = int64_t(tiles) * tiles * nz;
  const int64_t u1 = work * (blockIdx.x + 1) / gridDim.x;
  double acc = 0.0;
  for (int64_t u = work * blockIdx.x / gridDim.x; u < u1;) {
    const int64_t col = u / nz;
    const int z0 = int(u - col * nz);
    const int z1 = int(min(nz, int64_t(z0) + (u1 - u)));
    const int bx = int(col % tiles), by = int(col / tiles);
    const int ex = bx * kOwn - 1 + tx, ey = by * kOwn - 1 + ty;
    const bool mine = tx >= 1 && ty >= 1 && ex < N && ey < N;
    const int zs = z0, ze = min(z1, N) - 1;
    if (zs <= ze) {
      const DmaPlan<double> dp = dma_plan<double>(N, bx, by);
      dma_layer<MODE, double>(N, dp, zs, 0, x, p, s, L);
      dma_layer<MODE, double>(N, dp, zs + 1, 1, x, p, s, L);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      int sb = 0;
      for (int ez = zs; ez <= ze; ++ez) {
        const int st = sb == 2 ? 0 : sb + 1, sn = st == 2 ? 0 : st + 1;
        double X[8][4], S[8][4], P[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int node = (ty + ((a >> 1) & 1)) * kTN + tx + (a & 1);
          const int sl = (a >> 2) ? st : sb;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            X[a][k] = L.x[sl][node][k];
            S[a][k] = DIFF ? L.v[sl][node][k] : 0.0;
          }
          P[a] = L.p[sl][node];
        }
        if (ez + 2 <= N && ez + 1 <= ze) dma_layer<MODE, double>(N, dp, ez + 2, sn, x, p, s, L);
        if (mine) {
          double pq[8], dpq[8][3];
          elem_pq<3, double>(P, invh, pq, dpq);
          Zq<3, double> z[8];
          elem_z<3, double>(X, invh, z);
          double we = 0.0;
#pragma unroll
          for (int q = 0; q < 8; ++q) we += density<3, double, SK>(m, z[q], pq[q], dpq[q]);
          if (DIFF) {
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
              for (int k = 0; k < 4; ++k) X[a][k] += S[a][k];
            elem_z<3, double>(X, invh, z);
            double w1 = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) w1 += density<3, double, SK>(m, z[q], pq[q], dpq[q]);
            we = w1 - we;
          }
          acc += w * we;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        sb = st;
      }
    }
    u += z1 - z0;
  }
  return acc;
}

// The energy alone fits two workgroups per compute unit (<= 256 registers,
// two LDS rings); the difference keeps both states and runs one.
template <int SK>
__global__ __launch_bounds__(256, 2) void k_energy3_lds(int N, double h, MatP<double> m, int tiles,
                                                        const double* __restrict__ x, const double* __restrict__ p,
                                                        double* __restrict__ partials) {
  __shared__ LayerLds<double> L;
  __shared__ double sh[256];
  const double tot = block_sum(energy3_lds<false, SK>(N, h, m, tiles, x, x, p, L), sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <int SK>
__global__ __launch_bounds__(256) void k_energy_diff3_lds(int N, double h, MatP<double> m, int tiles,
                                                          const double* __restrict__ x, const double* __restrict__ s,
                                                          const double* __restrict__ p, double* __restrict__ partials) {
  __shared__ LayerLds<double> L;
  __shared__ double sh[256];
  const double tot = block_sum(energy3_lds<true, SK>(N, h, m, tiles, x, s, p, L), sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// The work is the tiles x (N + 1) node layers, ordered column by column,
// and split into gridDim.x equal contiguous ranges, one per workgroup: the
// grid is sized to the workgroups the chip holds at once, so every compute
// unit gets the same number of layers (a range that starts inside a column
// recomputes one element layer).
template <int MODE, typename T, int SK>
__device__ inline void elem_scatter3(int N, T h, const MatP<double>& md, int tiles,
                                     const uint8_t* __restrict__ dir, const T* __restrict__ x,
                                     const T* __restrict__ p, const T* __restrict__ v, T* __restrict__ out) {
  __shared__ T lo_sh[256][4][4];
  __shared__ T hi_sh[256][4][4];
  __shared__ LayerLds<T> lds;
  const MatP<T> m = cast_mat<T>(md);
  const T invh = T(1) / h;
  const T w = h * h * h / T(8);
  const int64_t nz = N + 1;
  const int64_t work = int64_t(tiles) * tiles * nz;
  const int64_t u1 = work * (blockIdx.x + 1) / gridDim.x;
  for (int64_t u = work * blockIdx.x / gridDim.x; u < u1;) {
    const int64_t col = u / nz;
    const int z0 = int(u - col * nz);
    const int z1 = int(min(nz, int64_t(z0) + (u1 - u)));
    elem_segment3_lds<MODE, T, SK>(N, m, invh, w, int(col % tiles), int(col / tiles), z0, z1, dir, x, p, v, out, lo_sh,
                               hi_sh, lds);
    u += z1 - z0;
  }
}

// FP64: one wavefront per SIMD (the element state does not fit in less than
// the full register file); FP32: two, which the smaller state allows (the
// spectral split's FP32 variant, with the principal axes, runs one).
template <int MODE, typename T, int SK>
__global__ __launch_bounds__(256) void k_elem_scatter3(int N, T h, MatP<double> md, int tiles,
                                                       const uint8_t* __restrict__ dir,
                                                       const T* __restrict__ x, const T* __restrict__ p,
                                                       const T* __restrict__ v, T* __restrict__ out) {
  elem_scatter3<MODE, T, SK>(N, h, md, tiles, dir, x, p, v, out);
}

template <int MODE>
__global__ __launch_bounds__(256, 2) void k_elem_scatter3_f32(int N, float h, MatP<double> md, int tiles,
                                                              const uint8_t* __restrict__ dir,
                                                              const float* __restrict__ x,
                                                              const float* __restrict__ p,
                                                              const float* __restrict__ v, float* __restrict__ out) {
  elem_scatter3<MODE, float, kNoSpectral>(N, h, md, tiles, dir, x, p, v, out);
}

// Node-centric kernels (any DIM): a thread per node sums the contributions
// of the 2^DIM elements around it.  Used in 2D and for per-node quantities.
template <int DIM, int MODE, typename T, int SK>
__global__ __launch_bounds__(kBlock) void k_node_gather(int N, T h, MatP<double> md, const uint8_t* __restrict__ dir,
                                                        const T* __restrict__ x, const T* __restrict__ p,
                                                        const T* __restrict__ v, T* __restrict__ out) {
  const MatP<T> m = cast_mat<T>(md);
  const int64_t nside = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= nside;
  const T invh = T(1) / h;
  T w = T(1);
#pragma unroll
  for (int i = 0; i < DIM; ++i) w *= T(0.5) * h;
  for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < nn; n += int64_t(gridDim.x) * blockDim.x) {
    int c[DIM];
    node_ijk<DIM>(n, nside, c);
    T r[DIM + 1];
#pragma unroll
    for (int k = 0; k <= DIM; ++k) r[k] = T(0);
#pragma unroll
    for (int a = 0; a < (1 << DIM); ++a) {
      // element whose local node a is this node
      int e[DIM];
      bool ok = true;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        e[i] = c[i] - ((a >> i) & 1);
        ok &= (e[i] >= 0) & (e[i] < N);
      }
      if (!ok) continue;
      T X[1 << DIM][DIM + 1], V[1 << DIM][DIM + 1], P[1 << DIM];
      load_elem<DIM, T, T>(x, e, nside, X);
      load_elem_scalar<DIM, T, T>(p, e, nside, P);
      if (MODE == 1) {
        load_elem<DIM, T, T>(v, e, nside, V);
        mask_elem<DIM, T>(dir, e, N, V);
      }
      node_contrib<DIM, T, SK>(MODE, m, invh, w, X, V, P, a, r);
    }
    const uint8_t mk = node_mask<DIM>(dir, n, c, N);
#pragma unroll
    for (int k = 0; k <= DIM; ++k) out[(DIM + 1) * n + k] = (mk & (1u << k)) ? T(0) : r[k];
  }
}

// Node diagonal blocks D[n][k][l] (full (DIM+1)^2 block, Dirichlet rows and
// columns zero).
template <int DIM, typename T, int SK>
__global__ __launch_bounds__(kBlock) void k_diag_blocks(int N, T h, MatP<double> md, const uint8_t* __restrict__ dir,
                                                        const T* __restrict__ x, const T* __restrict__ p,
                                                        T* __restrict__ D) {
  constexpr int NC = DIM + 1;
  const MatP<T> m = cast_mat<T>(md);
  const int64_t nside = N + 1;
  int64_t nn = 1;
#pragma unroll
  for (int i = 0; i < DIM; ++i) nn *= nside;
  const T invh = T(1) / h;
  T w = T(1);
#pragma unroll
  for (int i = 0; i < DIM; ++i) w *= T(0.5) * h;
  for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < nn; n += int64_t(gridDim.x) * blockDim.x) {
    int c[DIM];
    node_ijk<DIM>(n, nside, c);
    T blk[NC][NC];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int l = 0; l < NC; ++l) blk[k][l] = T(0);
    for (int a = 0; a < (1 << DIM); ++a) {
      int e[DIM];
      bool ok = true;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        e[i] = c[i] - ((a >> i) & 1);
        ok &= (e[i] >= 0) & (e[i] < N);
      }
      if (!ok) continue;
      T X[1 << DIM][DIM + 1], P[1 << DIM];
      load_elem<DIM, T, T>(x, e, nside, X);
      load_elem_scalar<DIM, T, T>(p, e, nside, P);
#pragma unroll
      for (int q = 0; q < (1 << DIM); ++q) {
        Zq<DIM, T> z;
        T pq, dpq[DIM];
        interp_scalar_q<DIM, T>(q, P, invh, pq, dpq);
        interp_q<DIM, T>(q, X, invh, z);
        HessCoef<DIM, T> hc;
        hess_coef<DIM, T, SK>(m, z, pq, dpq, hc);
        const T nq = T(refN<DIM>(q, a));
        T dn[DIM];
#pragma unroll
        for (int j = 0; j < DIM; ++j) dn[j] = T(refdN<DIM>(q, a, j)) * invh;
#pragma unroll
        for (int l = 0; l < NC; ++l) {
          // z-vector of the unit dof (a, l)
          Zq<DIM, T> u, o;
          zero<DIM, T>(u);
          if (l < DIM) {
            u.u[l] = nq;
#pragma unroll
            for (int j = 0; j < DIM; ++j) u.G[l][j] = dn[j];
          } else {
            u.c = nq;
#pragma unroll
            for (int j = 0; j < DIM; ++j) u.dc[j] = dn[j];
          }
          hess_apply<DIM, T, SK>(m, hc, u, o);
          T col[NC];
#pragma unroll
          for (int k = 0; k < NC; ++k) col[k] = T(0);
          project_q_node<DIM, T>(q, a, invh, w, o, col);
#pragma unroll
          for (int k = 0; k < NC; ++k) blk[k][l] += col[k];
        }
      }
    }
    const uint8_t mk = node_mask<DIM>(dir, n, c, N);
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int l = 0; l < NC; ++l)
        D[(int64_t(NC) * NC) * n + NC * k + l] = ((mk >> k) & 1u) || ((mk >> l) & 1u) ? T(0) : blk[k][l];
  }
}

// Calls f with the split family of m as a compile-time constant
// (std::integral_constant): kernels are instantiated once per family.
template <typename F>
void with_split(const MatP<double>& m, F&& f) {
  if (m.split == kSplitSpectral)
    f(std::integral_constant<int, kSplitSpectral>());
  else
    f(std::integral_constant<int, kNoSpectral>());
}

// Compute units of the current device, read once per device.
int compute_units() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

int grid_for(int64_t work) {
  int64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 65535 * 4) b = 65535 * 4;
  return int(b);
}

}  // namespace

// ----------------------------------------------------------------- launch
hipError_t launch_reduce_partials(const double* partials, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, partials, n, out);
  return hipGetLastError();
}

// Workgroups of the tiled 3D energy: as many as fit on the chip at once
// (two per compute unit for the energy, one for the difference), fewer on
// coarse levels with fewer tile layers.
int64_t energy3_groups(int N, bool diff) {
  const int tiles = (N + 1 + kOwn - 1) / kOwn;
  const int64_t work = int64_t(tiles) * tiles * (N + 1);
  return std::max<int64_t>(1, std::min<int64_t>(int64_t(compute_units()) * (diff ? 1 : 2), work));
}

int energy_partials(const ElemArgs& a) {
  if (a.dim == 3) return int(std::min<int64_t>(energy3_groups(a.N, false), kMaxPartials));
  const int64_t ne = int64_t(a.N) * a.N;
  int64_t nb = (ne + kBlock - 1) / kBlock;
  if (nb > kMaxPartials) nb = kMaxPartials;
  if (nb < 1) nb = 1;
  return int(nb);
}

hipError_t launch_energy(const ElemArgs& a, const double* x, const void* s, int s_fp32, const double* p,
                         double* partials, double* out, hipStream_t st) {
  int nb = energy_partials(a);
  if (a.dim == 3 && !s_fp32) {
    const int tiles = (a.N + 1 + kOwn - 1) / kOwn;
    const bool spec = a.m.split == kSplitSpectral;
    if (s) {
      nb = int(std::min<int64_t>(energy3_groups(a.N, true), kMaxPartials));
      if (spec)
        hipLaunchKernelGGL(k_energy_diff3_lds<kSplitSpectral>, dim3(nb), dim3(256), 0, st, a.N, a.h, a.m, tiles, x,
                           (const double*)s, p, partials);
      else
        hipLaunchKernelGGL(k_energy_diff3_lds<kNoSpectral>, dim3(nb), dim3(256), 0, st, a.N, a.h, a.m, tiles, x,
                           (const double*)s, p, partials);
    } else if (spec) {
      hipLaunchKernelGGL(k_energy3_lds<kSplitSpectral>, dim3(nb), dim3(256), 0, st, a.N, a.h, a.m, tiles, x, p,
                         partials);
    } else {
      hipLaunchKernelGGL(k_energy3_lds<kNoSpectral>, dim3(nb), dim3(256), 0, st, a.N, a.h, a.m, tiles, x, p, partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partials, nb, out, st);
  }
  if (a.dim == 3) {
    // FP32 step: one thread per element
    const int64_t ne = int64_t(a.N) * a.N * a.N;
    nb = int(std::max<int64_t>(1, std::min<int64_t>((ne + kBlock - 1) / kBlock, kMaxPartials)));
  }
  with_split(a.m, [&](auto sk) {
    constexpr int SK = decltype(sk)::value;
    if (a.dim == 3) {
      if (s_fp32)
        hipLaunchKernelGGL((k_energy<3, float, SK>), dim3(nb), dim3(kBlock), 0, st, a.N, a.h, a.m, x, (const float*)s,
                           p, partials);
      else
        hipLaunchKernelGGL((k_energy<3, double, SK>), dim3(nb), dim3(kBlock), 0, st, a.N, a.h, a.m, x,
                           (const double*)s, p, partials);
    } else {
      if (s_fp32)
        hipLaunchKernelGGL((k_energy<2, float, SK>), dim3(nb), dim3(kBlock), 0, st, a.N, a.h, a.m, x, (const float*)s,
                           p, partials);
      else
        hipLaunchKernelGGL((k_energy<2, double, SK>), dim3(nb), dim3(kBlock), 0, st, a.N, a.h, a.m, x,
                           (const double*)s, p, partials);
    }
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_partials(partials, nb, out, st);
}

template <int MODE, typename T>
static hipError_t launch_scatter(const ElemArgs& a, const T* x, const T* p, const T* v, T* out, hipStream_t st) {
  if (a.dim == 3) {
    const int tiles = (a.N + 1 + kOwn - 1) / kOwn;
    // one workgroup per compute unit (FP64), two (FP32); a coarse level with
    // fewer node layers than that gets one layer per workgroup (latency, not
    // the recomputed element layer, bounds it there)
    const int64_t work = int64_t(tiles) * tiles * (a.N + 1);
    const bool spec = a.m.split == kSplitSpectral;
    int64_t nb = int64_t(compute_units()) * (sizeof(T) == 4 && !spec ? 2 : 1);
    nb = std::max<int64_t>(1, std::min(nb, work));
    if (spec)
      hipLaunchKernelGGL((k_elem_scatter3<MODE, T, kSplitSpectral>), dim3(unsigned(nb)), dim3(256), 0, st, a.N,
                         T(a.h), a.m, tiles, a.dir, x, p, v, out);
    else if constexpr (sizeof(T) == 4)
      hipLaunchKernelGGL((k_elem_scatter3_f32<MODE>), dim3(unsigned(nb)), dim3(256), 0, st, a.N, T(a.h), a.m, tiles,
                         a.dir, x, p, v, out);
    else
      hipLaunchKernelGGL((k_elem_scatter3<MODE, T, kNoSpectral>), dim3(unsigned(nb)), dim3(256), 0, st, a.N, T(a.h),
                         a.m, tiles, a.dir, x, p, v, out);
  } else {
    int64_t nn = int64_t(a.N + 1) * (a.N + 1);
    with_split(a.m, [&](auto sk) {
      hipLaunchKernelGGL((k_node_gather<2, MODE, T, decltype(sk)::value>), dim3(grid_for(nn)), dim3(kBlock), 0, st,
                         a.N, T(a.h), a.m, a.dir, x, p, v, out);
    });
  }
  return hipGetLastError();
}

hipError_t launch_gradient(const ElemArgs& a, const double* x, const double* p, double* g, hipStream_t st) {
  return launch_scatter<0, double>(a, x, p, nullptr, g, st);
}

hipError_t launch_hessvec(const ElemArgs& a, const void* xl, const void* p, const void* v, void* hv, int fp32,
                          hipStream_t st) {
  if (fp32)
    return launch_scatter<1, float>(a, (const float*)xl, (const float*)p, (const float*)v, (float*)hv, st);
  return launch_scatter<1, double>(a, (const double*)xl, (const double*)p, (const double*)v, (double*)hv, st);
}

hipError_t launch_diag_blocks(const ElemArgs& a, const void* xl, const void* p, void* D, int fp32, hipStream_t st) {
  int64_t nn = 1;
  for (int i = 0; i < a.dim; ++i) nn *= (a.N + 1);
  dim3 grid(grid_for(nn));
  with_split(a.m, [&](auto sk) {
    constexpr int SK = decltype(sk)::value;
    if (a.dim == 3) {
      if (fp32)
        hipLaunchKernelGGL((k_diag_blocks<3, float, SK>), grid, dim3(kBlock), 0, st, a.N, float(a.h), a.m, a.dir,
                           (const float*)xl, (const float*)p, (float*)D);
      else
        hipLaunchKernelGGL((k_diag_blocks<3, double, SK>), grid, dim3(kBlock), 0, st, a.N, a.h, a.m, a.dir,
                           (const double*)xl, (const double*)p, (double*)D);
    } else {
      if (fp32)
        hipLaunchKernelGGL((k_diag_blocks<2, float, SK>), grid, dim3(kBlock), 0, st, a.N, float(a.h), a.m, a.dir,
                           (const float*)xl, (const float*)p, (float*)D);
      else
        hipLaunchKernelGGL((k_diag_blocks<2, double, SK>), grid, dim3(kBlock), 0, st, a.N, a.h, a.m, a.dir,
                           (const double*)xl, (const double*)p, (double*)D);
    }
  });
  return hipGetLastError();
}

}  // namespace rmtr

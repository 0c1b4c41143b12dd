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

// 3D element-centric kernels: a 16 x 16 tile of element columns marches up
// in z; each element's 8 nodal contributions are exchanged through LDS (or
// registers) and summed by the thread that owns the node, so no atomics
// are needed and the sum order is fixed.  Two tilings: tiles that overlap
// by one element column and row, so that each tile owns the 15 x 15 nodes
// whose four in-plane elements it computes (the all-points kernels of the
// FP32 Hv and the spectral split), and non-overlapping tiles whose border
// nodes are summed by a second kernel (the FP64 gradient and Hv, below);
// the energy kernels count each element once on non-overlapping tiles.
constexpr int kTile = 16;
constexpr int kOwn = kTile - 1;

// One column segment: the tile (bx, by) writes its owned nodes of node
// layers [z0, z1); on overlapping tiles it computes element layers
// z0 - 1 .. z1 - 1 (those that touch them).  The tile's node layers are
// staged in LDS: each
// node layer of the tile (17 x 17 nodes: x, v and p) is copied from memory
// into LDS by the asynchronous global-to-LDS loads, one layer ahead of the
// element layer that needs it, so the loads of the next layer overlap the
// arithmetic of the current one; each element then reads its eight nodes
// from LDS instead of from memory (a node is fetched once per tile, not once
// per element around it).
constexpr int kTN = kTile + 1;         // nodes per tile side
constexpr int kTNodes = kTN * kTN;     // nodes per tile layer

// The FP64 gradient and Hv tile the elements without overlap instead
// (16 x 16 element columns from (16 bx, 16 by)): the nodes on a tile's border
// (local x or y index 0 or 16) are touched by the elements of the tiles next
// to it too.  A tile writes its partial sums of those 64 nodes per node
// layer to a ring buffer, ring[(tile column, z)][slot][component], and a
// second kernel adds the partials of the one to four tiles around each
// border node in a fixed order (no atomics).
constexpr int kRing = 4 * kTile;

// A workgroup's column segment [z0, z1) evaluates only its own element
// layers, so its first node layer misses the share of the element layer
// below; the segment under it, which ends there, writes that share (all
// 17 x 17 tile nodes) to the workgroup's seam slot, and the border kernel
// adds it.  Doubles per slot, and the most slots (workgroups) a launch uses.
constexpr int kSeam = kTNodes * 4;
constexpr int kMaxSeams = 2048;

// slot of border node (ix, iy): bottom row 0..16, top row 17..33, left
// column (iy = 1..15) 34..48, right column 49..63
__host__ __device__ constexpr int ring_slot(int ix, int iy) {
  return iy == 0 ? ix : iy == kTile ? kTN + ix : ix == 0 ? 2 * kTN + iy - 1 : 2 * kTN + kOwn + iy - 1;
}

// LDS of the border nodes outside the lanes' own (tx + 1, ty + 1): element
// column 0's shares of the left column (its y-combine), and the z carries
// of the bottom row, the left column and the corner
template <typename T>
struct EdgeLds {
  T col[2][4][kTN];
  T cr[4][kTile];
  T cc[4][kTile];
  T c0[4];
};

// Workgroups are dispatched to the eight XCDs in turn (workgroup b to XCD
// b mod 8).  Numbering them XCD by XCD instead (a bijection of [0, g)) gives
// each XCD a contiguous range of the column-major (tile column, layer) work:
// tiles next to each other in x then run on one XCD, at the same layers at
// about the same time, and the node lines their halos share are read into
// that XCD's L2 once.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block() {
  const int64_t b = blockIdx.x, g = gridDim.x, x = b % kXcds;
  return x * (g / kXcds) + min(x, g % kXcds) + b / kXcds;
}

// Last word of a raw buffer resource (32-bit data, no swizzle) on gfx950.
constexpr int kRsrcWord3 = 0x00020000;

#define RMTR_LDS(ptr) ((void __attribute__((address_space(3)))*)(ptr))

// Node layers in LDS component-major (one array of the tile's 17 x 17
// nodes per component), so that the lanes of a wavefront, which take
// neighbouring nodes, read neighbouring words.
template <typename T>
struct LayerLds {
  T x[3][4][kTNodes];
  T v[3][4][kTNodes];
  T p[3][kTNodes];
};

// The 4-byte pieces one thread copies for every node layer of a tile.  Per
// round r the thread's piece is c = 256 r + tid of one component array (node
// c / W, word c % W of the value, W = sizeof(T) / 4); the piece's offset in a
// node layer of x (and v) and of p is the same for every layer and, up to
// the component, for every component, so it is formed once per column
// segment (nodes outside the grid are clamped: only inactive elements see
// them).
template <typename T>
struct DmaPlan {
  static constexpr int kW = int(sizeof(T)) / 4;                 // words per value
  static constexpr int kR = (kTNodes * kW + 255) / 256;         // rounds per component array
  int xoff[kR];  // byte offset of the piece in x (component 0), -1: none
  int poff[kR];  // byte offset of the piece in p
};

// (gx0, gy0): the grid node of the tile's first LDS node
template <typename T>
__device__ inline DmaPlan<T> dma_plan(int N, int gx0, int gy0) {
  DmaPlan<T> d;
  const int tid = threadIdx.x;
  const int ns = N + 1;
#pragma unroll
  for (int r = 0; r < DmaPlan<T>::kR; ++r) {
    const int c = r * 256 + tid;
    if (c < kTNodes * DmaPlan<T>::kW) {
      const int node = c / DmaPlan<T>::kW, word = c % DmaPlan<T>::kW;
      const int ix = node % kTN, iy = node / kTN;
      const int gx = min(max(gx0 + ix, 0), N);
      const int gy = min(max(gy0 + iy, 0), N);
      const int pl = gx + ns * gy;
      d.xoff[r] = pl * 4 * int(sizeof(T)) + 4 * word;
      d.poff[r] = pl * int(sizeof(T)) + 4 * word;
    } else {
      d.xoff[r] = -1;
      d.poff[r] = -1;
    }
  }
  return d;
}

// Copy node layer z of the tile into LDS slot `slot` (x, v when MODE == 1,
// and p), transposing the node-major vectors into component arrays.
template <int MODE, typename T, class LDS>
__device__ inline void dma_layer(int N, const DmaPlan<T>& d, int z, int slot, const T* __restrict__ x,
                                 const T* __restrict__ p, const T* __restrict__ v, LDS& L) {
  // the global-to-LDS copy exists in device code only (the host pass of a
  // template instantiated from several kernels would otherwise reject it)
#if defined(__HIP_DEVICE_COMPILE__)
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int64_t ns = N + 1;
  const int64_t zl = ns * ns * int64_t(z);
  // buffer resources over node layer z of x, v and p (uniform base, byte
  // size of the layer): the copies then need one unsigned 32-bit offset per
  // lane and no 64-bit address
  const int xbytes = int(4 * ns * ns * int64_t(sizeof(T))), pbytes = int(ns * ns * int64_t(sizeof(T)));
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void*)(x + 4 * zl), (short)0, xbytes, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc((void*)(v + 4 * zl), (short)0, xbytes, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void*)(p + zl), (short)0, pbytes, kRsrcWord3);
#pragma unroll
  for (int r = 0; r < DmaPlan<T>::kR; ++r) {
    if (d.xoff[r] >= 0) {
      const int lb = (r * 256 + wave * 64) * 4;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, RMTR_LDS(reinterpret_cast<char*>(&L.x[slot][k][0]) + lb), 4,
                                                 d.xoff[r], k * int(sizeof(T)), 0, 0);
        if constexpr (MODE == 1)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rv, RMTR_LDS(reinterpret_cast<char*>(&L.v[slot][k][0]) + lb), 4,
                                                   d.xoff[r], k * int(sizeof(T)), 0, 0);
      }
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rp, RMTR_LDS(reinterpret_cast<char*>(&L.p[slot][0]) + lb), 4,
                                               d.poff[r], 0, 0, 0);
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
  const DmaPlan<T> dp = dma_plan<T>(N, bx * kOwn - 1, by * kOwn - 1);
  if (zs <= ze) {
    dma_layer<MODE, T, LayerLds<T>>(N, dp, zs, 0, x, p, v, L);
    dma_layer<MODE, T, LayerLds<T>>(N, dp, zs + 1, 1, x, p, v, L);
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
        X[a][k] = L.x[sl][k][node];
        V[a][k] = MODE == 1 ? L.v[sl][k][node] : T(0);
      }
      P[a] = L.p[sl][node];
    }
    const int ec[3] = {ex, ey, ez};
    if (MODE == 1 && ecol) mask_elem<3, T>(dir, ec, N, V);
    // node layer ez + 2 goes to the slot that held layer ez - 1 (last read
    // before the previous iteration's closing barrier); it is issued after
    // this element's reads (and its Dirichlet bits), so none of them waits
    // for it
    if (ez + 2 <= N && ez + 1 <= ze) dma_layer<MODE, T, LayerLds<T>>(N, dp, ez + 2, sn, x, p, v, L);
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

// 3D energy (and FP64 energy difference) on non-overlapping tiles: tile
// (bx, by) holds the 16 x 16 element columns from (16 bx, 16 by) (its LDS
// nodes from the same corner) and counts the element layers of its segment
// of node layers, so every element is counted exactly once; node layers are
// staged in LDS as for the scatter kernels (x in the x slots, the step s in
// the v slots).  Each workgroup writes one partial sum (threads in
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
  const int64_t lb = xcd_block();
  const int64_t u1 = work * (lb + 1) / gridDim.x;
  double acc = 0.0;
  for (int64_t u = work * lb / gridDim.x; u < u1;) {
    const int64_t col = u / nz;
    const int z0 = int(u - col * nz);
    const int z1 = int(min(nz, int64_t(z0) + (u1 - u)));
    const int bx = int(col % tiles), by = int(col / tiles);
    const int ex = bx * kTile + tx, ey = by * kTile + ty;
    const bool mine = ex < N && ey < N;
    const int zs = z0, ze = min(z1, N) - 1;
    if (zs <= ze) {
      const DmaPlan<double> dp = dma_plan<double>(N, bx * kTile, by * kTile);
      dma_layer<MODE, double, LayerLds<double>>(N, dp, zs, 0, x, p, s, L);
      dma_layer<MODE, double, LayerLds<double>>(N, dp, zs + 1, 1, x, p, s, L);
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
            X[a][k] = L.x[sl][k][node];
            S[a][k] = DIFF ? L.v[sl][k][node] : 0.0;
          }
          P[a] = L.p[sl][node];
        }
        if (ez + 2 <= N && ez + 1 <= ze) dma_layer<MODE, double, LayerLds<double>>(N, dp, ez + 2, sn, x, p, s, L);
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

// Node layers of x and p only (the energy's ring).
template <typename T>
struct LayerLdsXP {
  T x[3][4][kTNodes];
  T p[3][kTNodes];
};

// Energy, unsplit and volumetric-deviatoric forms: the quarter-wise
// evaluation of the element kernels (two Gauss points at a time from the
// nodal values in LDS), which keeps the state small enough for four
// workgroups per compute unit.  The tiles do not overlap here: tile
// (bx, by) holds the 16 x 16 element columns from (16 bx, 16 by) (its LDS
// nodes from the same corner), and every element of the grid belongs to
// exactly one tile column and, through the node-layer ranges, one element
// layer; partial sums per workgroup in a fixed order, as energy3_lds.
// `tiles`: element tiles per side, ceil(N / 16).
template <bool VD>
__device__ inline double energy3_q(int N, const SymConst<double>& kc, double a2Gcl2, int tiles,
                                   const double* __restrict__ x, const double* __restrict__ p, LayerLdsXP<double>& L) {
  using T = double;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t nz = N + 1;
  const int64_t work = int64_t(tiles) * tiles * nz;
  const int64_t lb = xcd_block();
  const int64_t u1 = work * (lb + 1) / gridDim.x;
  int nd[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) nd[a] = (ty + ((a >> 1) & 1)) * kTN + tx + (a & 1);
  double acc = 0.0;
  for (int64_t u = work * lb / gridDim.x; u < u1;) {
    const int64_t col = u / nz;
    const int z0 = int(u - col * nz);
    const int z1 = int(min(nz, int64_t(z0) + (u1 - u)));
    const int bx = int(col % tiles), by = int(col / tiles);
    const int ex = bx * kTile + tx, ey = by * kTile + ty;
    const bool mine = ex < N && ey < N;
    const int zs = z0, ze = min(z1, N) - 1;
    if (zs <= ze) {
      const DmaPlan<T> dp = dma_plan<T>(N, bx * kTile, by * kTile);
      dma_layer<0, T, LayerLdsXP<T>>(N, dp, zs, 0, x, p, x, L);
      dma_layer<0, T, LayerLdsXP<T>>(N, dp, zs + 1, 1, x, p, x, L);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      int sb = 0;
      for (int ez = zs; ez <= ze; ++ez) {
        const int st = sb == 2 ? 0 : sb + 1, sn = st == 2 ? 0 : st + 1;
        if (ez + 2 <= N && ez + 1 <= ze) dma_layer<0, T, LayerLdsXP<T>>(N, dp, ez + 2, sn, x, p, x, L);
        if (mine) {
#pragma nounroll
          for (int qq = 0; qq < 4; ++qq) {
            // re-read the nodal values in every quarter (see elem_segment3_q)
            __asm__ __volatile__("" ::: "memory");
            const T xy = gauss_xi<T>(qq & 1), xz = gauss_xi<T>(qq >> 1);
            QPoint<T> zq[2];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
              T f[8];
#pragma unroll
              for (int a = 0; a < 8; ++a) f[a] = k < 4 ? L.x[(a >> 2) ? st : sb][k][nd[a]] : L.p[(a >> 2) ? st : sb][nd[a]];
              T val[2], dx, dy[2], dz[2];
              qtr_forward<T>(f, xz, xy, val, dx, dy, dz);
#pragma unroll
              for (int qx = 0; qx < 2; ++qx) {
                if (k < 3) {
                  zq[qx].u[k] = val[qx];
                  zq[qx].G[k][0] = dx;
                  zq[qx].G[k][1] = dy[qx];
                  zq[qx].G[k][2] = dz[qx];
                } else if (k == 3) {
                  zq[qx].c = val[qx];
                  zq[qx].dc[0] = dx;
                  zq[qx].dc[1] = dy[qx];
                  zq[qx].dc[2] = dz[qx];
                } else {
                  zq[qx].p = val[qx];
                  zq[qx].dp[0] = dx;
                  zq[qx].dp[1] = dy[qx];
                  zq[qx].dp[2] = dz[qx];
                }
              }
            }
            acc += energy_point_sym<T, VD>(kc, a2Gcl2, zq[0]) + energy_point_sym<T, VD>(kc, a2Gcl2, zq[1]);
          }
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

// kc from sym_const on the host; a2Gcl2 = a2 Gc l / 2
template <bool VD>
__global__ __launch_bounds__(256, 4) void k_energy_q3(int N, SymConst<double> kc, double a2Gcl2, int tiles,
                                                      const double* __restrict__ x, const double* __restrict__ p,
                                                      double* __restrict__ partials) {
  __shared__ LayerLdsXP<double> L;
  __shared__ double sh[256];
  const double tot = block_sum(energy3_q<VD>(N, kc, a2Gcl2, tiles, x, p, L), sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
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
// and split into gridDim.x equal contiguous ranges, one per workgroup in its
// XCD-major numbering (xcd_block): the grid is sized to the workgroups the
// chip holds at once, so every compute unit gets the same number of layers
// (a range that starts inside a column recomputes one element layer).
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
  const int64_t lb = xcd_block();
  const int64_t u1 = work * (lb + 1) / gridDim.x;
  for (int64_t u = work * lb / gridDim.x; u < u1;) {
    const int64_t col = u / nz;
    const int z0 = int(u - col * nz);
    const int z1 = int(min(nz, int64_t(z0) + (u1 - u)));
    elem_segment3_lds<MODE, T, SK>(N, m, invh, w, int(col % tiles), int(col / tiles), z0, z1, dir, x, p, v, out, lo_sh,
                               hi_sh, lds);
    u += z1 - z0;
  }
}

// All eight points of an element at once: the FP32 Hv (two wavefronts per
// SIMD) and the spectral split (one).
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

// ------------------------------------------------- quarter-wise element kernels
// Gradient and Hessian action (unsplit and volumetric-deviatoric forms) on
// the same tiles and LDS ring as elem_segment3_lds, with a per-element state
// small enough for two workgroups per compute unit in FP64 (four in FP32):
// the element's nodal values are read from the LDS ring once per quarter of
// its Gauss points (qtr_forward) instead of being held for all eight, and
// the element's nodal results are combined with the neighbours' in two
// steps: along x between adjacent lanes of a 16-lane row (DPP row shift),
// then along y through a small LDS buffer.

// Value of v held by lane + 1 of the same 16-lane row (row_shl:1); the last
// lane of a row gets 0.
__device__ inline float row_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, true));
}
__device__ inline double row_next(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x101, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x101, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

template <int MODE, typename T, bool VD, bool EDGE>
__device__ inline void elem_segment3_q(int N, const MatP<T>& m, const ElemScale<T>& sc, const SymConst<T>& kc, int bx,
                                       int by, int tiles, int z0, int z1,
                                       const uint8_t* __restrict__ dir, const T* __restrict__ x,
                                       const T* __restrict__ p, const T* __restrict__ v, T* __restrict__ out,
                                       T* __restrict__ edge, T* __restrict__ seam, T (*ysh)[4][256], EdgeLds<T>& R,
                                       LayerLds<T>& L) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  // EDGE: the tile's elements start at (16 bx, 16 by); otherwise one column
  // and row earlier (overlapping tiles)
  const int gx0 = EDGE ? bx * kTile : bx * kOwn - 1, gy0 = EDGE ? by * kTile : by * kOwn - 1;
  const int ex = gx0 + tx;
  const int ey = gy0 + ty;
  const int ox = ex + 1, oy = ey + 1;
  const bool ecol = ex >= 0 && ex < N && ey >= 0 && ey < N;
  const bool owner = (EDGE || (tx < kOwn && ty < kOwn)) && ox <= N && oy <= N;
  const int64_t nside = N + 1;
  const T cdc = sc.a2 * m.Gc_l;
  // EDGE: only the segment's own element layers; its first node layer is
  // left without the share of the element layer below, which the segment
  // under it leaves in its seam slot.  Otherwise that element layer is
  // recomputed here.
  const int zs = EDGE ? z0 : max(z0 - 1, 0), ze = min(z1 - 1, N - 1);
  const DmaPlan<T> dp = dma_plan<T>(N, gx0, gy0);
  // tile-local node (ix, iy) of node layer z: a border node's sum goes to
  // the ring partials, any other node's (every element around it is in the
  // tile) to the output, Dirichlet components zero
  const int64_t ring0 = (int64_t(by) * tiles + bx) * nside;
  auto emit = [&](int ix, int iy, int z, const T (&s)[4]) {
    if (EDGE && (ix == 0 || iy == 0 || ix == kTile || iy == kTile)) {
      T* e = edge + ((ring0 + z) * kRing + ring_slot(ix, iy)) * 4;
#pragma unroll
      for (int k = 0; k < 4; ++k) e[k] = s[k];
    } else {
      const int c[3] = {gx0 + ix, gy0 + iy, z};
      const int64_t n = int64_t(c[0]) + nside * (int64_t(c[1]) + nside * z);
      const uint8_t mk = node_mask<3>(dir, n, c, N);
#pragma unroll
      for (int k = 0; k < 4; ++k) out[4 * n + k] = (mk & (1u << k)) ? T(0) : s[k];
    }
  };
  if (EDGE) {
    // z carries of the border nodes this lane holds besides its own node
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (ty == 0) R.cr[k][tx] = T(0);
      if (tx == 0) R.cc[k][ty] = T(0);
      if (tid == 0) R.c0[k] = T(0);
      if (tid < 2) R.col[tid][k][kTile] = T(0);
    }
  }
  if (zs <= ze) {
    dma_layer<MODE, T, LayerLds<T>>(N, dp, zs, 0, x, p, v, L);
    dma_layer<MODE, T, LayerLds<T>>(N, dp, zs + 1, 1, x, p, v, L);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  T acc[4] = {T(0), T(0), T(0), T(0)};
  int sb = 0;
  for (int ez = zs; ez <= ze; ++ez) {
    const int st = sb == 2 ? 0 : sb + 1, sn = st == 2 ? 0 : st + 1;
    // node layer ez + 2 goes to the slot that held layer ez - 1, free since
    // the previous iteration's closing barrier
    if (ez + 2 <= N && ez + 1 <= ze) dma_layer<MODE, T, LayerLds<T>>(N, dp, ez + 2, sn, x, p, v, L);
    T r[4][8];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int a = 0; a < 8; ++a) r[k][a] = T(0);
    if (ecol) {
      // Dirichlet bits of the direction's 8 nodes (4 per node)
      uint32_t vm = 0;
      if (MODE == 1) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int c[3] = {ex + (a & 1), ey + ((a >> 1) & 1), ez + (a >> 2)};
          const int64_t n = int64_t(c[0]) + nside * (int64_t(c[1]) + nside * c[2]);
          vm |= uint32_t(node_mask<3>(dir, n, c, N)) << (4 * a);
        }
      }
      int nd[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) nd[a] = (ty + ((a >> 1) & 1)) * kTN + tx + (a & 1);
#pragma nounroll
      for (int qq = 0; qq < 4; ++qq) {
        // the nodal values are re-read from LDS in every quarter: keep the
        // compiler from hoisting the reads out of the loop (which would hold
        // all of them in registers)
        __asm__ __volatile__("" ::: "memory");
        const T xy = gauss_xi<T>(qq & 1), xz = gauss_xi<T>(qq >> 1);
        QPoint<T> zq[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          T f[8];
#pragma unroll
          for (int a = 0; a < 8; ++a) f[a] = L.x[(a >> 2) ? st : sb][k][nd[a]];
          if (k < 3 || MODE == 0) {
            T val[2], dx, dy[2], dz[2];
            qtr_forward<T>(f, xz, xy, val, dx, dy, dz);
#pragma unroll
            for (int qx = 0; qx < 2; ++qx) {
              if (k < 3) {
                zq[qx].u[k] = val[qx];
                zq[qx].G[k][0] = dx;
                zq[qx].G[k][1] = dy[qx];
                zq[qx].G[k][2] = dz[qx];
              } else {
                zq[qx].c = val[qx];
                zq[qx].dc[0] = dx;
                zq[qx].dc[1] = dy[qx];
                zq[qx].dc[2] = dz[qx];
              }
            }
          } else {
            T val[2];
            qtr_forward_val<T>(f, xz, xy, val);
            zq[0].c = val[0];
            zq[1].c = val[1];
          }
        }
        {
          T f[8];
#pragma unroll
          for (int a = 0; a < 8; ++a) f[a] = L.p[(a >> 2) ? st : sb][nd[a]];
          T val[2], dx, dy[2], dz[2];
          qtr_forward<T>(f, xz, xy, val, dx, dy, dz);
#pragma unroll
          for (int qx = 0; qx < 2; ++qx) {
            zq[qx].p = val[qx];
            zq[qx].dp[0] = dx;
            zq[qx].dp[1] = dy[qx];
            zq[qx].dp[2] = dz[qx];
          }
        }
        Zq<3, T> o[2];
        if (MODE == 0) {
#pragma unroll
          for (int qx = 0; qx < 2; ++qx) grad_point_sym<T, VD>(kc, cdc, zq[qx], o[qx]);
        } else {
          HessSym<T> hc[2];
#pragma unroll
          for (int qx = 0; qx < 2; ++qx) hess_sym_coef<T, VD>(kc, zq[qx], hc[qx]);
          Zq<3, T> zv[2];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            T f[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) f[a] = L.v[(a >> 2) ? st : sb][k][nd[a]];
            if (vm) {
#pragma unroll
              for (int a = 0; a < 8; ++a)
                if ((vm >> (4 * a + k)) & 1u) f[a] = T(0);
            }
            T val[2], dx, dy[2], dz[2];
            qtr_forward<T>(f, xz, xy, val, dx, dy, dz);
#pragma unroll
            for (int qx = 0; qx < 2; ++qx) {
              if (k < 3) {
                zv[qx].u[k] = val[qx];
                zv[qx].G[k][0] = dx;
                zv[qx].G[k][1] = dy[qx];
                zv[qx].G[k][2] = dz[qx];
              } else {
                zv[qx].c = val[qx];
                zv[qx].dc[0] = dx;
                zv[qx].dc[1] = dy[qx];
                zv[qx].dc[2] = dz[qx];
              }
            }
          }
#pragma unroll
          for (int qx = 0; qx < 2; ++qx) hess_sym_apply<T>(hc[qx], cdc, zv[qx], o[qx]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          T cv[2], cx[2], cy[2], cz[2];
#pragma unroll
          for (int qx = 0; qx < 2; ++qx) {
            cv[qx] = k < 3 ? o[qx].u[k] : o[qx].c;
            cx[qx] = k < 3 ? o[qx].G[k][0] : o[qx].dc[0];
            cy[qx] = k < 3 ? o[qx].G[k][1] : o[qx].dc[1];
            cz[qx] = k < 3 ? o[qx].G[k][2] : o[qx].dc[2];
          }
          qtr_backward<T>(cv, cx, cy, cz, xz, xy, r[k]);
        }
      }
    }
    // combine: along x from the next lane of the row (every lane takes part)
    // (the lane's indices are formed again here, opaque to the compiler, so
    // that the addresses below are not held in registers through the
    // quarter loop)
    int tidr = tid;
    __asm__ __volatile__("" : "+v"(tidr));
    const int txr = tidr & 15, tyr = tidr >> 4;
    T cs[2][2][4];  // [ay][az][k]: this and the next element's share of node (tx + 1, ty + ay, ez + az)
#pragma unroll
    for (int ay = 0; ay < 2; ++ay)
#pragma unroll
      for (int az = 0; az < 2; ++az)
#pragma unroll
        for (int k = 0; k < 4; ++k) cs[ay][az][k] = r[k][1 + 2 * ay + 4 * az] + row_next(r[k][2 * ay + 4 * az]);
    // along y through LDS
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ysh[az][k][tidr] = cs[0][az][k];
        // EDGE: column 0's shares of the left border nodes (0, ty)
        if (EDGE && txr == 0) R.col[az][k][tyr] = r[k][4 * az];
      }
    __syncthreads();
    if (owner) {
      // the last element row's nodes (EDGE) have no row above in the tile
      T up[2][4];
#pragma unroll
      for (int az = 0; az < 2; ++az)
#pragma unroll
        for (int k = 0; k < 4; ++k) up[az][k] = (!EDGE || tyr < kOwn) ? ysh[az][k][(tidr + 16) & 255] : T(0);
      if (ez >= z0) {
        T s[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] = acc[k] + cs[1][0][k] + up[0][k];
        emit(txr + 1, tyr + 1, ez, s);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] = cs[1][1][k] + up[1][k];
    }
    if (EDGE) {
      // border nodes outside the lanes' own: the bottom row (tx + 1, 0), the
      // left column (0, ty + 1) and the corner (0, 0)
      if (tyr == 0 && ox <= N) {
        if (ez >= z0) {
          T s[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) s[k] = R.cr[k][txr] + cs[0][0][k];
          emit(txr + 1, 0, ez, s);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) R.cr[k][txr] = cs[0][1][k];
      }
      if (txr == 0 && oy <= N) {
        if (ez >= z0) {
          T s[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) s[k] = R.cc[k][tyr] + r[k][2] + R.col[0][k][tyr + 1];
          emit(0, tyr + 1, ez, s);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) R.cc[k][tyr] = r[k][6] + R.col[1][k][tyr + 1];
      }
      if (tidr == 0) {
        if (ez >= z0) {
          T s[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) s[k] = R.c0[k] + r[k][0];
          emit(0, 0, ez, s);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) R.c0[k] = r[k][4];
      }
    }
    // layer ez + 2 is in LDS, slot sb and the y buffer are free again
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    sb = st;
  }
  // node layer ze + 1 from the carries: the top layer N, or (EDGE, a
  // segment that ends below the top) the next segment's first layer, whose
  // share from this segment goes to the seam slot (tile-local node-major,
  // four components)
  const bool top = ze + 1 < z1;
  if (top || (EDGE && z1 <= N)) {
    const int nz = ze + 1;
    auto put = [&](int ix, int iy, const T (&s)[4]) {
      if (top) {
        emit(ix, iy, nz, s);
      } else {
        T* q = seam + (iy * kTN + ix) * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = s[k];
      }
    };
    if (owner) put(tx + 1, ty + 1, acc);
    if (EDGE) {
      T s[4];
      if (ty == 0 && ox <= N) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] = R.cr[k][tx];
        put(tx + 1, 0, s);
      }
      if (tx == 0 && oy <= N) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] = R.cc[k][ty];
        put(0, ty + 1, s);
      }
      if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] = R.c0[k];
        put(0, 0, s);
      }
    }
  }
}

// FP64, two workgroups per compute unit (at most 256 registers, 77 KB of
// LDS each).
// The pointwise constants kc are formed on the host (sym_const), so they
// reach the kernel as scalar arguments and take no vector registers.
template <int MODE, bool VD, bool EDGE>
__global__ __launch_bounds__(256, 2) void k_elem_q3(int N, double h, MatP<double> md, SymConst<double> kc, int tiles,
                                                    const uint8_t* __restrict__ dir, const double* __restrict__ x,
                                                    const double* __restrict__ p, const double* __restrict__ v,
                                                    double* __restrict__ out, double* __restrict__ edge,
                                                    double* __restrict__ seam) {
  using T = double;
  __shared__ T ysh[2][4][256];
  __shared__ EdgeLds<T> rl;
  __shared__ LayerLds<T> lds;
  const MatP<T> m = md;
  const ElemScale<T> sc = elem_scale<T>(T(1) / h, h * h * h / T(8));
  const int64_t nz = N + 1;
  const int64_t work = int64_t(tiles) * tiles * nz;
  // the seam slot and the work range belong to the logical index
  const int64_t lb = xcd_block();
  const int64_t u1 = work * (lb + 1) / gridDim.x;
  for (int64_t u = work * lb / gridDim.x; u < u1;) {
    const int64_t col = u / nz;
    const int z0 = int(u - col * nz);
    const int z1 = int(min(nz, int64_t(z0) + (u1 - u)));
    elem_segment3_q<MODE, T, VD, EDGE>(N, m, sc, kc, int(col % tiles), int(col / tiles), tiles, z0, z1, dir, x, p, v,
                                       out, edge, EDGE ? seam + lb * kSeam : nullptr, ysh, rl, lds);
    u += z1 - z0;
  }
}

// Border nodes and seams of the non-overlapping tiles.  Threads
// [0, border): a thread per border node and layer adds the ring partials of
// the tiles that hold the node (tile rows, then columns, ascending), each
// with the seam share below it when the node layer starts a segment, and
// writes the sum, Dirichlet components zero.  The border nodes of a layer
// are those on the lines x = 16 i (every y), then those on the lines
// y = 16 j off them.  Threads [border, border + (g - 1) 225): the interior
// nodes of the first node layer of each segment that starts above the
// bottom (workgroup b >= 1 of the g the element kernel ran, in its logical
// numbering, xcd_block), which get the seam share of workgroup b - 1 added.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ring_sum(int N, int tiles, int g, const uint8_t* __restrict__ dir,
                                                     const T* __restrict__ ring, const T* __restrict__ seam,
                                                     T* __restrict__ out) {
  const int nside = N + 1;
  const int nvl = N / kTile + 1;
  const int per_v = nvl * nside;
  const int nh = nside - nvl;
  const int per_layer = per_v + nvl * nh;
  const int64_t border = int64_t(per_layer) * nside;
  const int64_t total = border + int64_t(g - 1) * kOwn * kOwn;
  const int64_t work = int64_t(tiles) * tiles * nside;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    int gx, gy, z;
    const T* sl0 = nullptr;  // seam slot of an interior node
    if (t < border) {
      z = int(t / per_layer);
      int r = int(t - int64_t(z) * per_layer);
      if (r < per_v) {
        gx = kTile * (r / nside);
        gy = r % nside;
      } else {
        r -= per_v;
        gy = kTile * (r / nh);
        const int q = r % nh;
        gx = kTile * (q / kOwn) + q % kOwn + 1;
      }
    } else {
      const int64_t t2 = t - border;
      const int64_t b = 1 + t2 / (kOwn * kOwn);
      const int j = int(t2 % (kOwn * kOwn));
      const int64_t u0 = work * b / g;
      const int64_t col = u0 / nside;
      z = int(u0 - col * nside);
      gx = kTile * int(col % tiles) + 1 + j % kOwn;
      gy = kTile * int(col / tiles) + 1 + j / kOwn;
      if (z == 0 || gx > N || gy > N) continue;
      sl0 = seam + (b - 1) * kSeam + ((gy % kTile) * kTN + gx % kTile) * 4;
    }
    const int c[3] = {gx, gy, z};
    const int64_t n = int64_t(gx) + int64_t(nside) * (int64_t(gy) + int64_t(nside) * z);
    const uint8_t mk = node_mask<3>(dir, n, c, N);
    T s[4];
    if (sl0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] = out[4 * n + k] + sl0[k];
    } else {
      const int bx0 = (gx % kTile == 0 && gx > 0) ? gx / kTile - 1 : gx / kTile, bx1 = min(gx / kTile, tiles - 1);
      const int by0 = (gy % kTile == 0 && gy > 0) ? gy / kTile - 1 : gy / kTile, by1 = min(gy / kTile, tiles - 1);
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] = T(0);
      for (int by = by0; by <= by1; ++by)
        for (int bx = bx0; bx <= bx1; ++bx) {
          const int ix = gx - kTile * bx, iy = gy - kTile * by;
          const int64_t u = (int64_t(by) * tiles + bx) * nside + z;
          const T* e = ring + u * (4 * kRing) + 4 * ring_slot(ix, iy);
#pragma unroll
          for (int k = 0; k < 4; ++k) s[k] += e[k];
          // the workgroup whose range starts at this node layer, if any
          const int64_t b = (u * g + work - 1) / work;
          if (z > 0 && b >= 1 && b < g && work * b / g == u) {
            const T* q = seam + (b - 1) * kSeam + (iy * kTN + ix) * 4;
#pragma unroll
            for (int k = 0; k < 4; ++k) s[k] += q[k];
          }
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out[4 * n + k] = (mk & (1u << k)) ? T(0) : s[k];
  }
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

// doubles of the ring partials proper (the seam slots follow them)
size_t ring_part(int N) {
  const size_t et = size_t((N + kTile - 1) / kTile);
  return et * et * size_t(N + 1) * 4 * kRing;
}

}  // namespace

size_t ring_values(int N) {
  const size_t et = size_t((N + kTile - 1) / kTile);
  const size_t slots = std::min(et * et * size_t(N + 1), size_t(kMaxSeams));
  return ring_part(N) + slots * kSeam;
}

// ----------------------------------------------------------------- launch
hipError_t launch_reduce_partials(const double* partials, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, partials, n, out);
  return hipGetLastError();
}

// Workgroups of the tiled 3D energy: as many as fit on the chip at once
// (four per compute unit for the quarter-wise energy, two for the spectral
// split's, one for the difference), fewer on coarse levels with fewer tile
// layers.
int64_t energy3_groups(int N, bool diff, bool spec) {
  // the energy kernels tile the elements without overlap (16 x 16 element
  // columns)
  const int tiles = (N + kTile - 1) / kTile;
  const int64_t work = int64_t(tiles) * tiles * (N + 1);
  return std::max<int64_t>(1, std::min<int64_t>(int64_t(compute_units()) * (diff ? 1 : spec ? 2 : 4), work));
}

int energy_partials(const ElemArgs& a) {
  if (a.dim == 3)
    return int(std::min<int64_t>(energy3_groups(a.N, false, a.m.split == kSplitSpectral), kMaxPartials));
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
    const int tiles = (a.N + kTile - 1) / kTile;
    const bool spec = a.m.split == kSplitSpectral;
    if (s) {
      nb = int(std::min<int64_t>(energy3_groups(a.N, true, spec), kMaxPartials));
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
      const ElemScale<double> sc = elem_scale<double>(1.0 / a.h, a.h * a.h * a.h / 8.0);
      hipLaunchKernelGGL((a.m.split ? k_energy_q3<true> : k_energy_q3<false>), dim3(nb), dim3(256), 0, st, a.N,
                         sym_const<double>(a.m, sc), 0.5 * sc.a2 * a.m.Gc_l, tiles, x, p, partials);
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
    // overlapping tiles (the all-points kernels, and the quarter-wise one
    // without a ring buffer); a coarse level with fewer tile layers than the
    // grid gets one layer per workgroup (latency bounds it there)
    const int tiles = (a.N + 1 + kOwn - 1) / kOwn;
    const int64_t work = int64_t(tiles) * tiles * (a.N + 1);
    const bool spec = a.m.split == kSplitSpectral;
    // FP64 (unsplit, volumetric-deviatoric): the quarter-wise kernel, two
    // workgroups per compute unit; FP32: all eight points per element, two
    // workgroups (fewer instructions, and FP32 state fits); spectral split:
    // one workgroup
    int64_t nb = int64_t(compute_units()) * (spec ? 1 : 2);
    nb = std::max<int64_t>(1, std::min(nb, work));
    if (spec)
      hipLaunchKernelGGL((k_elem_scatter3<MODE, T, kSplitSpectral>), dim3(unsigned(nb)), dim3(256), 0, st, a.N,
                         T(a.h), a.m, tiles, a.dir, x, p, v, out);
    else if constexpr (sizeof(T) == 4)
      hipLaunchKernelGGL((k_elem_scatter3_f32<MODE>), dim3(unsigned(nb)), dim3(256), 0, st, a.N, T(a.h), a.m, tiles,
                         a.dir, x, p, v, out);
    else {
      const SymConst<double> kc = sym_const<double>(a.m, elem_scale<double>(1.0 / a.h, a.h * a.h * a.h / 8.0));
      if (a.ring) {
        // non-overlapping tiles, then the border nodes' sums
        const int et = (a.N + kTile - 1) / kTile;
        const int64_t ework = int64_t(et) * et * (a.N + 1);
        const int enb = int(std::max<int64_t>(
            1, std::min<int64_t>({int64_t(compute_units()) * 2, ework, int64_t(kMaxSeams)})));
        double* seam = a.ring + ring_part(a.N);
        hipLaunchKernelGGL((a.m.split ? k_elem_q3<MODE, true, true> : k_elem_q3<MODE, false, true>),
                           dim3(unsigned(enb)), dim3(256), 0, st, a.N, T(a.h), a.m, kc, et, a.dir, x, p, v, out,
                           a.ring, seam);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int nvl = a.N / kTile + 1;
        const int64_t border = (int64_t(nvl) * (a.N + 1) + int64_t(nvl) * (a.N + 1 - nvl)) * (a.N + 1);
        hipLaunchKernelGGL(k_ring_sum<double>, dim3(grid_for(border + int64_t(enb - 1) * kOwn * kOwn)),
                           dim3(kBlock), 0, st, a.N, et, enb, a.dir, (const double*)a.ring, (const double*)seam,
                           out);
      } else {
        hipLaunchKernelGGL((a.m.split ? k_elem_q3<MODE, true, false> : k_elem_q3<MODE, false, false>),
                           dim3(unsigned(nb)), dim3(256), 0, st, a.N, T(a.h), a.m, kc, tiles, a.dir, x, p, v, out,
                           (double*)nullptr, (double*)nullptr);
      }
    }
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

// The learned fine-level proposal: a 3D convolutional network (six 3x3x3
// layers, channels 8 -> 32 -> 32 -> 32 -> 32 -> 32 -> 4, ReLU after the
// first five, zero padding), with BF16 weights and BF16 matrix-core
// products summed in FP32, and the kernels that train it (backward passes,
// MSE loss, Adam).
//
// Tensors are channels-last FP32 on a box of nx x ny x nz voxels (voxel
// v = x + nx (y + ny z)), the layout of the node-major grid vectors.  Layer
// weights are [27][Cin][Cout] with offset k = (dx+1) + 3 (dy+1) + 9 (dz+1):
//   y[v][co] = b[co] + sum_k sum_ci W[k][ci][co] x[v + off(k)][ci].
#include <algorithm>

#include "rmtr_kernels.h"

namespace rmtr {
namespace {

constexpr int kB = 256;

// round-to-nearest-even FP32 -> BF16 (NaN stays a quiet NaN), one hardware
// conversion on gfx950 (checked against the bit-level definition over all
// 2^32 inputs)
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

struct Box {
  int nx, ny, nz;
};

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// 3x3x3 convolution on the matrix cores with the input staged in LDS, for
// the forward pass and for the data gradient:
//   out[v][o] = (bias[o]) + sum_k sum_i Wl[k][i][o] in[v + SIGN off(k)][i]
// (forward: Wl = W, SIGN +1; data gradient: Wl[k][i][o] = W[k][o][i],
// SIGN -1).  With MASK_OUT the result is zeroed where mask <= 0: the data
// gradient of layer l is stored already multiplied by the ReLU derivative
// of layer l - 1's output (mask = that output), which is how both passes
// of layer l - 1 consume it.  A workgroup computes a tile of 32 x 4 x 2 output voxels: wavefront w
// the two x-rows (y0 + w, z0) and (y0 + w, z0 + 1), each a 32-voxel x
// 32-output MFMA tile (v_mfma_f32_32x32x16_bf16, reduction over offsets x
// input channels in chunks of 16).  The tile's input with its one-voxel halo
// (34 x 6 x 4 voxels) is converted to BF16 once into LDS, so each input
// value is read from memory about 3.2 times instead of 27; the weights sit
// in LDS for the whole kernel.  Voxel and weight rows are padded by eight
// BF16 values so the 16-byte operand reads of a wavefront hit distinct
// banks.  Lane l holds A[l % 32][8 (l / 32) + t] and B[8 (l / 32) + t]
// [l % 32] (t = 0..7); accumulator r of lane l is
// C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
template <int NI, int NO, int SIGN, int TRANS, int BIAS, int RELU_OUT, int MASK_OUT>
__global__ __launch_bounds__(256) void k_conv_tile(Box b, const float* __restrict__ in,
                                                   const float* __restrict__ mask, const uint16_t* __restrict__ W,
                                                   const float* __restrict__ bias, float* __restrict__ out) {
  constexpr int NIP = NI < 16 ? 16 : NI;  // input channels padded to the MFMA chunk
  static_assert(NI % 4 == 0 && NIP % 16 == 0 && NO <= 32, "channel counts");
  constexpr int SP = NIP + 8, WP = NIP + 8;  // padded voxel and weight rows (BF16 values)
  constexpr int SX = 34, SY = 6, SZ = 4, NG = NIP / 4;
  __shared__ __align__(16) uint16_t sW[27 * 32 * WP];
  __shared__ __align__(16) uint16_t sIn[SZ * SY * SX * SP];
  for (int e = threadIdx.x; e < 27 * 32 * NIP; e += 256) {
    const int k = e / (32 * NIP), o = (e / NIP) % 32, i = e % NIP;
    uint16_t wv = 0;
    if (o < NO && i < NI) wv = TRANS ? W[(k * NO + o) * NI + i] : W[(k * NI + i) * NO + o];
    sW[(k * 32 + o) * WP + i] = wv;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;
  const int xt = (b.nx + 31) / 32, yt = (b.ny + 3) / 4, zt = (b.nz + 1) / 2;
  const int64_t ntiles = int64_t(xt) * yt * zt;
  // the tile's input (with halo) is loaded into registers one tile ahead, so
  // the loads of tile T + gridDim.x are in flight while tile T is computed
  constexpr int NST = SZ * SY * SX * NG, NIT = (NST + 255) / 256;
  float4 buf[NIT];
  auto load_tile = [&](int64_t T) {
    const int x0 = 32 * int(T % xt);
    const int y0 = 4 * int((T / xt) % yt);
    const int z0 = 2 * int(T / (int64_t(xt) * yt));
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
      const int e = int(threadIdx.x) + 256 * j;
      const int g = e % NG, vs = e / NG;
      const int sx = vs % SX, sy = (vs / SX) % SY, sz = vs / (SX * SY);
      const int X = x0 - 1 + sx, Y = y0 - 1 + sy, Z = z0 - 1 + sz;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NST && 4 * g < NI && X >= 0 && X < b.nx && Y >= 0 && Y < b.ny && Z >= 0 && Z < b.nz) {
        const int64_t off = ((int64_t(Z) * b.ny + Y) * b.nx + X) * NI + 4 * g;
        a = *reinterpret_cast<const float4*>(in + off);
      }
      buf[j] = a;
    }
  };
  if (int64_t(blockIdx.x) < ntiles) load_tile(blockIdx.x);
  for (int64_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
    const int x0 = 32 * int(T % xt);
    const int y0 = 4 * int((T / xt) % yt);
    const int z0 = 2 * int(T / (int64_t(xt) * yt));
    __syncthreads();  // the previous tile's reads of sIn are done (and sW is staged)
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
      const int e = int(threadIdx.x) + 256 * j;
      if (e < NST) {
        const int g = e % NG, vs = e / NG;
        bf16x4 q;
        q[0] = short(f2bf(buf[j].x));
        q[1] = short(f2bf(buf[j].y));
        q[2] = short(f2bf(buf[j].z));
        q[3] = short(f2bf(buf[j].w));
        *reinterpret_cast<bf16x4*>(sIn + vs * SP + 4 * g) = q;
      }
    }
    __syncthreads();
    if (T + gridDim.x < ntiles) load_tile(T + gridDim.x);
    f32x16 acc0, acc1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      acc0[r] = 0.0f;
      acc1[r] = 0.0f;
    }
    for (int k = 0; k < 27; ++k) {
      const int dx = SIGN * (k % 3 - 1), dy = SIGN * ((k / 3) % 3 - 1), dz = SIGN * (k / 9 - 1);
      const uint16_t* wk = sW + (k * 32 + li) * WP + 8 * lk;
      const uint16_t* a0 = sIn + (((1 + dz) * SY + (wave + 1 + dy)) * SX + (li + 1 + dx)) * SP + 8 * lk;
      const uint16_t* a1 = a0 + SY * SX * SP;
#pragma unroll
      for (int ic = 0; ic < NIP / 16; ++ic) {
        const bf16x8 bw = *reinterpret_cast<const bf16x8*>(wk + 16 * ic);
        const bf16x8 v0 = *reinterpret_cast<const bf16x8*>(a0 + 16 * ic);
        const bf16x8 v1 = *reinterpret_cast<const bf16x8*>(a1 + 16 * ic);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v0, bw, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v1, bw, acc1, 0, 0, 0);
      }
    }
    const int o = li, y = y0 + wave;
    if (o < NO && y < b.ny) {
      const float bo = BIAS ? bias[o] : 0.0f;
#pragma unroll
      for (int zr = 0; zr < 2; ++zr) {
        const int z = z0 + zr;
        if (z >= b.nz) continue;
        const int64_t base = ((int64_t(z) * b.ny + y) * b.nx + x0) * NO + o;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 8 * (r / 4) + 4 * lk + (r % 4);
          if (x0 + i < b.nx) {
            float val = (zr ? acc1[r] : acc0[r]) + bo;
            if (RELU_OUT) val = fmaxf(val, 0.0f);
            if (MASK_OUT && !(mask[base + int64_t(i) * NO] > 0.0f)) val = 0.0f;
            out[base + int64_t(i) * NO] = val;
          }
        }
      }
    }
  }
}

// Register-blocked variant of the same convolution, used for the forward
// pass (2.28 ms against 2.47 ms for k_conv_tile at 129^3; the data
// gradient keeps k_conv_tile, 6.36 ms against 6.69 ms for the backward pass
// with this kernel): a workgroup computes
// 32 x 4 x 4 output voxels, wavefront w the four x-rows (y0 .. y0 + 3,
// z0 + w).  For one input shift (dx, dz) and one 16-channel chunk the
// wavefront reads the six input rows y0 - 1 .. y0 + 4 once and the three
// weight blocks of dy = -1, 0, 1, and issues the twelve products row r x
// offset dy (input row r + 1 + dy): 0.75 operand reads per matrix-core
// product instead of 1.5.  The tile's input with its halo (34 x 6 x 6
// voxels) is converted to BF16 into LDS once per tile (loaded into registers
// one tile ahead); the weights stay in LDS.  Rows are padded by four BF16
// values (72 bytes between voxels) so that input and weights fit the
// compute unit's LDS together.  Operand and accumulator layouts as in
// k_conv_tile.
template <int NI, int NO, int SIGN, int TRANS, int BIAS, int RELU_OUT, int MASK_OUT>
__global__ __launch_bounds__(256) void k_conv_blk(Box b, const float* __restrict__ in,
                                                  const float* __restrict__ mask, const uint16_t* __restrict__ W,
                                                  const float* __restrict__ bias, float* __restrict__ out) {
  constexpr int NIP = NI < 16 ? 16 : NI;
  static_assert(NI % 4 == 0 && NIP % 16 == 0 && NO <= 32, "channel counts");
  constexpr int SP = NIP + 4, WP = NIP + 4;
  constexpr int SX = 34, SY = 6, SZ = 6, NG = NIP / 4;
  __shared__ __align__(16) uint16_t sW[27 * 32 * WP];
  __shared__ __align__(16) uint16_t sIn[SZ * SY * SX * SP];
  for (int e = threadIdx.x; e < 27 * 32 * NIP; e += 256) {
    const int k = e / (32 * NIP), o = (e / NIP) % 32, i = e % NIP;
    uint16_t wv = 0;
    if (o < NO && i < NI) wv = TRANS ? W[(k * NO + o) * NI + i] : W[(k * NI + i) * NO + o];
    sW[(k * 32 + o) * WP + i] = wv;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;
  const int xt = (b.nx + 31) / 32, yt = (b.ny + 3) / 4, zt = (b.nz + 3) / 4;
  const int64_t ntiles = int64_t(xt) * yt * zt;
  constexpr int NST = SZ * SY * SX * NG, NIT = (NST + 255) / 256;
  float4 buf[NIT];
  auto load_tile = [&](int64_t T) {
    const int x0 = 32 * int(T % xt);
    const int y0 = 4 * int((T / xt) % yt);
    const int z0 = 4 * int(T / (int64_t(xt) * yt));
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
      const int e = int(threadIdx.x) + 256 * j;
      const int g = e % NG, vs = e / NG;
      const int sx = vs % SX, sy = (vs / SX) % SY, sz = vs / (SX * SY);
      const int X = x0 - 1 + sx, Y = y0 - 1 + sy, Z = z0 - 1 + sz;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NST && 4 * g < NI && X >= 0 && X < b.nx && Y >= 0 && Y < b.ny && Z >= 0 && Z < b.nz) {
        const int64_t off = ((int64_t(Z) * b.ny + Y) * b.nx + X) * NI + 4 * g;
        a = *reinterpret_cast<const float4*>(in + off);
      }
      buf[j] = a;
    }
  };
  if (int64_t(blockIdx.x) < ntiles) load_tile(blockIdx.x);
  for (int64_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
    const int x0 = 32 * int(T % xt);
    const int y0 = 4 * int((T / xt) % yt);
    const int z0 = 4 * int(T / (int64_t(xt) * yt));
    __syncthreads();  // the previous tile's reads of sIn are done (and sW is staged)
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
      const int e = int(threadIdx.x) + 256 * j;
      if (e < NST) {
        const int g = e % NG, vs = e / NG;
        bf16x4 q;
        q[0] = short(f2bf(buf[j].x));
        q[1] = short(f2bf(buf[j].y));
        q[2] = short(f2bf(buf[j].z));
        q[3] = short(f2bf(buf[j].w));
        *reinterpret_cast<bf16x4*>(sIn + vs * SP + 4 * g) = q;
      }
    }
    __syncthreads();
    if (T + gridDim.x < ntiles) load_tile(T + gridDim.x);
    f32x16 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[r][i] = 0.0f;
    for (int dzi = 0; dzi < 3; ++dzi) {
      const int zs = wave + dzi;  // LDS z of the input rows: output z + (dzi - 1)
#pragma unroll
      for (int dxi = 0; dxi < 3; ++dxi) {
#pragma unroll
        for (int ic = 0; ic < NIP / 16; ++ic) {
          bf16x8 a[6];
#pragma unroll
          for (int j = 0; j < 6; ++j)
            a[j] = *reinterpret_cast<const bf16x8*>(sIn + ((zs * SY + j) * SX + li + dxi) * SP + 16 * ic + 8 * lk);
#pragma unroll
          for (int dyi = 0; dyi < 3; ++dyi) {
            // the input shift (dxi - 1, dyi - 1, dzi - 1) is offset k of
            // the forward weights, or the mirrored offset for the data
            // gradient
            const int k = SIGN > 0 ? dxi + 3 * dyi + 9 * dzi : (2 - dxi) + 3 * (2 - dyi) + 9 * (2 - dzi);
            const bf16x8 bw = *reinterpret_cast<const bf16x8*>(sW + (k * 32 + li) * WP + 16 * ic + 8 * lk);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[r + dyi], bw, acc[r], 0, 0, 0);
          }
        }
      }
    }
    const int o = li, z = z0 + wave;
    if (o < NO && z < b.nz) {
      const float bo = BIAS ? bias[o] : 0.0f;
#pragma unroll
      for (int yr = 0; yr < 4; ++yr) {
        const int y = y0 + yr;
        if (y >= b.ny) continue;
        const int64_t base = ((int64_t(z) * b.ny + y) * b.nx + x0) * NO + o;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 8 * (r / 4) + 4 * lk + (r % 4);
          if (x0 + i < b.nx) {
            float val = acc[yr][r] + bo;
            if (RELU_OUT) val = fmaxf(val, 0.0f);
            if (MASK_OUT && !(mask[base + int64_t(i) * NO] > 0.0f)) val = 0.0f;
            out[base + int64_t(i) * NO] = val;
          }
        }
      }
    }
  }
}

// Weight and bias gradient on the matrix cores with LDS tiles: for each
// offset k,
//   dW[k][ci][co] = sum_v X[v + off(k)][ci] dYm[v][co],   db[co] = sum_v dYm[v][co]
// (dYm = the output gradient times the layer's ReLU derivative, as the data
// gradient of the next layer stores it) is a 32 x 32 GEMM reduced over
// voxels, 16 per v_mfma_f32_32x32x16_bf16.  A workgroup takes tiles of
// 32 x 4 x 2 voxels (as k_conv_tile); per tile it stores in LDS, as BF16,
// the tile's dYm transposed ([row][co][x]) and the input with its halo
// transposed ([z][y][ci][x], x 16-byte aligned), so a lane's eight
// voxel-consecutive operand values are one aligned 16-byte read.  Nine
// wavefronts, one per (dy, dz); each keeps the three offsets dx = -1, 0, 1
// and builds their operands from one aligned read and its two neighbours
// (byte alignment of register pairs).  Every workgroup writes one partial
// row (27 CIN COUT + COUT values); the bias sums are FP32 over the unrounded
// dYm, per thread and then across threads in a fixed order.
// Position of x-entry xq (0..47, six blocks of eight) in the LDS row of
// input channel ci: the blocks of a row are rotated by ci / 8, which spreads
// the transposing stores of a wavefront (eight 4-channel groups) over all
// bank groups; a block stays 16-byte aligned for the operand reads.
__device__ inline int xslot(int ci, int xq) { return ((((xq >> 3) + (ci >> 3)) % 6) << 3) | (xq & 7); }

template <int CIN, int COUT>
__global__ __launch_bounds__(576) void k_conv_bwd_w_tile(Box b, const float* __restrict__ X,
                                                         const float* __restrict__ dY,
                                                         float* __restrict__ partial) {
  static_assert(CIN % 4 == 0 && COUT % 4 == 0 && CIN <= 32 && COUT <= 32, "channel counts");
  constexpr int NT = 576, NE = CIN * COUT;
  constexpr int SX = 34, SY = 6, SZ = 4, XW = 48, DW = 40;
  constexpr int NGI = CIN / 4, NGO = COUT / 4;
  static_assert(NT % NGO == 0, "fixed channel group per thread");
  __shared__ __align__(16) uint16_t sX[SZ * SY * 32 * XW];  // [z][y][ci][x + 7]
  __shared__ __align__(16) uint16_t sD[8 * 32 * DW];        // [row][co][x]
  __shared__ float sB[NT][4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lk = lane >> 5;
  // channel rows beyond CIN / COUT stay zero
  for (int e = tid; e < SZ * SY * 32 * XW; e += NT) sX[e] = 0;
  for (int e = tid; e < 8 * 32 * DW; e += NT) sD[e] = 0;
  f32x16 acc[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.0f;
  float bacc[4] = {0.f, 0.f, 0.f, 0.f};
  const int dyw = wave % 3 - 1, dzw = wave / 3 - 1;
  const int xt = (b.nx + 31) / 32, yt = (b.ny + 3) / 4, zt = (b.nz + 1) / 2;
  const int64_t ntiles = int64_t(xt) * yt * zt;
  for (int64_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
    const int x0 = 32 * int(T % xt);
    const int y0 = 4 * int((T / xt) % yt);
    const int z0 = 2 * int(T / (int64_t(xt) * yt));
    __syncthreads();  // the previous tile's operand reads are done
    // output gradient of the tile's 256 voxels, transposed
    for (int e = tid; e < 256 * NGO; e += NT) {
      const int g = e % NGO, vt = e / NGO;
      const int xx = vt & 31, r = vt >> 5;  // r = zr * 4 + yw
      const int x = x0 + xx, y = y0 + (r & 3), z = z0 + (r >> 2);
      float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
      if (x < b.nx && y < b.ny && z < b.nz) {
        const int64_t off = ((int64_t(z) * b.ny + y) * b.nx + x) * COUT + 4 * g;
        d = *reinterpret_cast<const float4*>(dY + off);
      }
      bacc[0] += d.x;
      bacc[1] += d.y;
      bacc[2] += d.z;
      bacc[3] += d.w;
      uint16_t* dst = sD + (r * 32 + 4 * g) * DW + xx;
      dst[0] = f2bf(d.x);
      dst[DW] = f2bf(d.y);
      dst[2 * DW] = f2bf(d.z);
      dst[3 * DW] = f2bf(d.w);
    }
    // the layer input with its halo, transposed
    for (int e = tid; e < SZ * SY * SX * NGI; e += NT) {
      const int g = e % NGI, vs = e / NGI;
      const int sx = vs % SX, sy = (vs / SX) % SY, sz = vs / (SX * SY);
      const int x = x0 - 1 + sx, y = y0 - 1 + sy, z = z0 - 1 + sz;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
      if (x >= 0 && x < b.nx && y >= 0 && y < b.ny && z >= 0 && z < b.nz)
        a = *reinterpret_cast<const float4*>(X + ((int64_t(z) * b.ny + y) * b.nx + x) * CIN + 4 * g);
      uint16_t* dst = sX + ((sz * SY + sy) * 32 + 4 * g) * XW + xslot(4 * g, sx + 7);
      dst[0] = f2bf(a.x);
      dst[XW] = f2bf(a.y);
      dst[2 * XW] = f2bf(a.z);
      dst[3 * XW] = f2bf(a.w);
    }
    __syncthreads();
#pragma unroll 1
    for (int r = 0; r < 8; ++r) {
      const int yw = r & 3, zr = r >> 2;
      const uint16_t* xrow = sX + (((zr + 1 + dzw) * SY + (yw + 1 + dyw)) * 32 + li) * XW;
      const uint16_t* drow = sD + (r * 32 + li) * DW;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int xp = 8 + 16 * c + 8 * lk;  // first of the lane's eight voxels (dx = 0)
        const bf16x8 bd = *reinterpret_cast<const bf16x8*>(drow + 16 * c + 8 * lk);
        const uint4 m = *reinterpret_cast<const uint4*>(xrow + xslot(li, xp));
        const uint32_t lft = *reinterpret_cast<const uint32_t*>(xrow + xslot(li, xp - 2));
        const uint32_t rgt = *reinterpret_cast<const uint32_t*>(xrow + xslot(li, xp + 8));
        // dx = -1: elements xp - 1 .. xp + 6;  dx = +1: xp + 1 .. xp + 8
        const uint32_t n0 = __builtin_amdgcn_alignbyte(m.x, lft, 2);
        const uint32_t n1 = __builtin_amdgcn_alignbyte(m.y, m.x, 2);
        const uint32_t n2 = __builtin_amdgcn_alignbyte(m.z, m.y, 2);
        const uint32_t n3 = __builtin_amdgcn_alignbyte(m.w, m.z, 2);
        const uint32_t p3 = __builtin_amdgcn_alignbyte(rgt, m.w, 2);
        const uint4 am = make_uint4(n0, n1, n2, n3);
        const uint4 ap = make_uint4(n1, n2, n3, p3);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8*>(&am), bd, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8*>(&m), bd, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8*>(&ap), bd, acc[2], 0, 0, 0);
      }
    }
  }
  float* outp = partial + int64_t(blockIdx.x) * (27 * NE + COUT);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int k = j + 3 * (dyw + 1) + 9 * (dzw + 1);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ci = 8 * (r / 4) + 4 * lk + (r % 4), co = li;
      if (ci < CIN && co < COUT) outp[k * NE + ci * COUT + co] = acc[j][r];
    }
  }
  // bias: thread t holds channel group t % NGO; sum over the threads of a
  // group in thread order
#pragma unroll
  for (int q = 0; q < 4; ++q) sB[tid][q] = bacc[q];
  __syncthreads();
  if (tid < COUT) {
    const int g = tid / 4, q = tid % 4;
    float sum = 0.0f;
    for (int t = g; t < NT; t += NGO) sum += sB[t][q];
    outp[27 * NE + tid] = sum;
  }
}

// second stage: fixed-order sum of the partial rows.  A workgroup takes
// kSumCols consecutive entries; its kSumGroups thread groups sum the rows
// i = g, g + kSumGroups, ... (in increasing order) of each entry, and the
// group sums are added in group order.
constexpr int kSumCols = 32, kSumGroups = kB / kSumCols;

__global__ __launch_bounds__(kB) void k_sum_partials(const float* __restrict__ partial, int nblk, int64_t len,
                                                     float* __restrict__ dw, float* __restrict__ db, int64_t nw) {
  __shared__ float sh[kSumGroups][kSumCols];
  const int c = int(threadIdx.x) % kSumCols, grp = int(threadIdx.x) / kSumCols;
  for (int64_t e0 = int64_t(blockIdx.x) * kSumCols; e0 < len; e0 += int64_t(gridDim.x) * kSumCols) {
    const int64_t e = e0 + c;
    float s = 0.0f;
    if (e < len)
      for (int i = grp; i < nblk; i += kSumGroups) s += partial[int64_t(i) * len + e];
    sh[grp][c] = s;
    __syncthreads();
    if (grp == 0 && e < len) {
      float t = sh[0][c];
#pragma unroll
      for (int k = 1; k < kSumGroups; ++k) t += sh[k][c];
      if (e < nw)
        dw[e] = t;
      else
        db[e - nw] = t;
    }
    __syncthreads();
  }
}

// MSE over the window [w0, w1) per direction and all channels:
// dout = 2 (out - target) / count inside, 0 outside; partial sums of squares.
__global__ __launch_bounds__(kB) void k_mse(Box b, int C, int wx0, int wx1, int wy0, int wy1, int wz0, int wz1,
                                            float inv_count, double inv_count_d, const float* __restrict__ out,
                                            const float* __restrict__ target, float* __restrict__ dout,
                                            double* __restrict__ partials) {
  __shared__ double sh[kB];
  const int64_t n = int64_t(b.nx) * b.ny * b.nz * C;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const int64_t v = i / C;
    const int x = int(v % b.nx), y = int((v / b.nx) % b.ny), z = int(v / (int64_t(b.nx) * b.ny));
    const bool in = x >= wx0 && x < wx1 && y >= wy0 && y < wy1 && z >= wz0 && z < wz1;
    const float d = in ? out[i] - target[i] : 0.0f;
    dout[i] = 2.0f * d * inv_count;
    acc += double(d) * double(d);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0] * inv_count_d;
}

// Adam with bias correction on FP32 master weights; the BF16 copy follows.
__global__ __launch_bounds__(kB) void k_adam(int64_t n, int64_t n_bf16, float lr, float b1, float b2, float eps, float c1, float c2,
                                             const float* __restrict__ g, float* __restrict__ p,
                                             float* __restrict__ m, float* __restrict__ v,
                                             uint16_t* __restrict__ pbf) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pbf && i < n_bf16) pbf[i] = f2bf(pi);
  }
}

__global__ __launch_bounds__(kB) void k_to_bf16(int64_t n, const float* __restrict__ a, uint16_t* __restrict__ b) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) b[i] = f2bf(a[i]);
}

// Per-component root mean square of a nodal 4-vector field, first stage
// (sums of squares per block, 4 values per block).
__global__ __launch_bounds__(kB) void k_sumsq4(int64_t nn, const double* __restrict__ g, double* __restrict__ part) {
  __shared__ double sh[4][kB];
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t n = int64_t(blockIdx.x) * kB + threadIdx.x; n < nn; n += int64_t(gridDim.x) * kB)
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] += g[4 * n + k] * g[4 * n + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int st = kB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st)
#pragma unroll
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// second stage: rms[k] = sqrt(sum / nn), fixed order
__global__ void k_rms4(int nblk, int64_t nn, const double* __restrict__ part, double* __restrict__ rms) {
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += part[4 * i + threadIdx.x];
    rms[threadIdx.x] = sqrt(s / double(nn));
  }
}

// Network input from the grid state: channels (u, c) of x times sc[0..3],
// then g / rms(g) times sc[4..7] (rms per component; 0 where rms = 0), so the
// network sees gradients of unit size at every stage of a solve.
__global__ __launch_bounds__(kB) void k_features(int64_t nn, const double* __restrict__ x,
                                                 const double* __restrict__ g, const float* __restrict__ sc,
                                                 const double* __restrict__ rms, float* __restrict__ feat) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < nn * 8; i += int64_t(gridDim.x) * kB) {
    const int64_t n = i / 8;
    const int k = int(i % 8);
    if (k < 4) {
      feat[i] = float(x[4 * n + k]) * sc[k];
    } else {
      const double r = rms[k - 4];
      feat[i] = r > 0.0 ? float(g[4 * n + k - 4] / r) * sc[k] : 0.0f;
    }
  }
}

// Proposal: s = out * sc[8 + k] * rms(g)_k, projected onto [lo, hi].
__global__ __launch_bounds__(kB) void k_proposal(int64_t n, const float* __restrict__ out,
                                                 const float* __restrict__ sc, const double* __restrict__ rms,
                                                 const double* __restrict__ lo, const double* __restrict__ hi,
                                                 double* __restrict__ s) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const double v = double(out[i]) * double(sc[8 + i % 4]) * rms[i % 4];
    s[i] = fmin(fmax(isfinite(v) ? v : 0.0, lo[i]), hi[i]);
  }
}

// Training target: t = s_k / (sc[8 + k] rms(g)_k), 0 where that vanishes
// (the inverse of the output scaling of k_proposal).
__global__ __launch_bounds__(kB) void k_target(int64_t n, const double* __restrict__ s,
                                               const float* __restrict__ sc, const double* __restrict__ rms,
                                               float* __restrict__ t) {
  for (int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kB) {
    const double den = double(sc[8 + i % 4]) * rms[i % 4];
    t[i] = den > 0.0 ? float(s[i] / den) : 0.0f;
  }
}

// Normalisation constants from the per-sample RMS values r[12 i + j]
// (j < 4: state x, 4..7: gradient g, 8..11: step s) of ns samples, in sample
// order: sc[k] = 1 / mean_i rms(x_k), sc[4 + k] = 1 (g is divided by its own
// RMS at run time), sc[8 + k] = mean_i rms(s_k) / rms(g_k) (samples with
// rms(g_k) = 0 count as 0); a constant that comes out 0 becomes 1.
__global__ void k_fit_scales(int ns, const double* __restrict__ r, float* __restrict__ sc) {
  const int k = threadIdx.x;
  if (k >= 4) return;
  double xs = 0.0, ratio = 0.0;
  for (int i = 0; i < ns; ++i) {
    xs += r[12 * i + k];
    const double rg = r[12 * i + 4 + k];
    ratio += rg > 0.0 ? r[12 * i + 8 + k] / rg : 0.0;
  }
  xs /= double(ns);
  ratio /= double(ns);
  sc[k] = xs > 0.0 ? float(1.0 / xs) : 1.0f;
  sc[4 + k] = 1.0f;
  sc[8 + k] = ratio > 0.0 ? float(ratio) : 1.0f;
}

int gridn(int64_t work) {
  int64_t b = (work + kB - 1) / kB;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return int(b);
}

// Tiled-kernel grids: persistent workgroups (each stages the layer's weights
// once, or writes one partial row), at most cap
int conv_tile_grid(const Box& b, int cap = 512) {
  const int64_t tiles = int64_t((b.nx + 31) / 32) * ((b.ny + 3) / 4) * ((b.nz + 1) / 2);
  return int(std::max<int64_t>(1, std::min<int64_t>(tiles, cap)));
}

// k_conv_blk: one workgroup per compute unit (150 KB of LDS)
int conv_blk_grid(const Box& b) {
  const int64_t tiles = int64_t((b.nx + 31) / 32) * ((b.ny + 3) / 4) * ((b.nz + 3) / 4);
  return int(std::max<int64_t>(1, std::min<int64_t>(tiles, 256)));
}

}  // namespace

// ------------------------------------------------------------- launchers
static const int kCh[7] = {8, 32, 32, 32, 32, 32, 4};

int64_t nn_weight_count() {
  int64_t n = 0;
  for (int l = 0; l < 6; ++l) n += int64_t(27) * kCh[l] * kCh[l + 1];
  return n;
}
int64_t nn_bias_count() {
  int64_t n = 0;
  for (int l = 0; l < 6; ++l) n += kCh[l + 1];
  return n;
}
int64_t nn_act_floats(int64_t nvox) {
  int64_t n = 0;
  for (int l = 0; l < 7; ++l) n += nvox * kCh[l];
  return n;
}

static int64_t w_off(int l) {
  int64_t n = 0;
  for (int i = 0; i < l; ++i) n += int64_t(27) * kCh[i] * kCh[i + 1];
  return n;
}
static int64_t b_off(int l) {
  int64_t n = 0;
  for (int i = 0; i < l; ++i) n += kCh[i + 1];
  return n;
}
static int64_t a_off(int l, int64_t nvox) {
  int64_t n = 0;
  for (int i = 0; i < l; ++i) n += nvox * kCh[i];
  return n;
}

// layer[0] = the 8-channel input (filled by the caller), layer[l+1] = the
// output of layer l; layer[6] = the 4-channel result.  Buffers may be shared
// between layers that are not adjacent (ping-pong inference).
hipError_t nn_forward(const uint16_t* w, const float* bias, float* const layer[7], int nx, int ny, int nz,
                      hipStream_t st) {
  const Box b{nx, ny, nz};
  const int64_t nvox = int64_t(nx) * ny * nz;
  for (int l = 0; l < 6; ++l) {
    const float* X = layer[l];
    float* Y = layer[l + 1];
    const uint16_t* W = w + w_off(l);
    const float* bb = bias + b_off(l);
    const dim3 grid(conv_blk_grid(b));
    if (l == 0)
      hipLaunchKernelGGL((k_conv_blk<8, 32, 1, 0, 1, 1, 0>), grid, dim3(256), 0, st, b, X, nullptr, W, bb, Y);
    else if (l < 5)
      hipLaunchKernelGGL((k_conv_blk<32, 32, 1, 0, 1, 1, 0>), grid, dim3(256), 0, st, b, X, nullptr, W, bb, Y);
    else
      hipLaunchKernelGGL((k_conv_blk<32, 4, 1, 0, 1, 0, 0>), grid, dim3(256), 0, st, b, X, nullptr, W, bb, Y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void nn_layers(float* act, int64_t nvox, float* layer[7]) {
  for (int l = 0; l < 7; ++l) layer[l] = act + a_off(l, nvox);
}

size_t nn_backward_work_floats(int64_t nvox) {
  // two gradient buffers of 32 channels + partial rows of the largest layer
  const int64_t nblk = 512;
  return size_t(2 * nvox * 32 + nblk * (27 * 32 * 32 + 32) + 64);
}

// dout: gradient w.r.t. act[6]; writes dw (all weights, FP32) and db.
hipError_t nn_backward(const uint16_t* w, const float* act, const float* dout, float* dw, float* db, int nx, int ny,
                       int nz, float* work, hipStream_t st) {
  const Box b{nx, ny, nz};
  const int64_t nvox = int64_t(nx) * ny * nz;
  float* gA = work;
  float* gB = work + nvox * 32;
  float* part = work + 2 * nvox * 32;
  // one partial row per weight-gradient workgroup: 256 workgroups (one per
  // compute unit, as their LDS allows) keep the fixed-order sum short
  const int nblk = conv_tile_grid(b, 256);
  const float* dY = dout;
  for (int l = 5; l >= 0; --l) {
    const int cin = kCh[l], cout = kCh[l + 1];
    const float* X = act + a_off(l, nvox);
    const uint16_t* W = w + w_off(l);
    const int64_t len = int64_t(27) * cin * cout + cout;
    // weights (dY arrives multiplied by the ReLU derivative already, see
    // the data gradient below; layer 5 has no ReLU on its output)
    if (l == 5)
      hipLaunchKernelGGL((k_conv_bwd_w_tile<32, 4>), dim3(nblk), dim3(576), 0, st, b, X, dY, part);
    else if (l > 0)
      hipLaunchKernelGGL((k_conv_bwd_w_tile<32, 32>), dim3(nblk), dim3(576), 0, st, b, X, dY, part);
    else
      hipLaunchKernelGGL((k_conv_bwd_w_tile<8, 32>), dim3(nblk), dim3(576), 0, st, b, X, dY, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(unsigned((len + kSumCols - 1) / kSumCols)), dim3(kB), 0, st, part, nblk,
                       len, dw + w_off(l), db + b_off(l), int64_t(27) * cin * cout);
    if (l == 0) break;
    float* dX = (l % 2) ? gA : gB;
    // data gradient: input dY (cout channels), output cin channels,
    // transposed weights, mirrored offsets; stored multiplied by the ReLU
    // derivative of layer l - 1 (its output X > 0)
    if (l == 5)
      hipLaunchKernelGGL((k_conv_tile<4, 32, -1, 1, 0, 0, 1>), dim3(conv_tile_grid(b)), dim3(256), 0, st, b, dY,
                         X, W, nullptr, dX);
    else
      hipLaunchKernelGGL((k_conv_tile<32, 32, -1, 1, 0, 0, 1>), dim3(conv_tile_grid(b)), dim3(256), 0, st, b, dY,
                         X, W, nullptr, dX);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dY = dX;
  }
  return hipGetLastError();
}

hipError_t nn_mse(const float* out, const float* target, float* dout, int nx, int ny, int nz, const int* window,
                  double* partials, double* loss_dev, hipStream_t st) {
  const Box b{nx, ny, nz};
  const int64_t cnt = int64_t(window[1] - window[0]) * (window[3] - window[2]) * (window[5] - window[4]) * 4;
  int nblk = gridn(int64_t(nx) * ny * nz * 4);
  if (nblk > kMaxPartials) nblk = kMaxPartials;
  hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(kB), 0, st, b, 4, window[0], window[1], window[2], window[3], window[4],
                     window[5], cnt > 0 ? float(1.0 / double(cnt)) : 0.0f, cnt > 0 ? 1.0 / double(cnt) : 0.0, out,
                     target, dout, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_reduce_partials(partials, nblk, loss_dev, st);
  return e;
}

hipError_t nn_adam(int64_t n, int64_t n_bf16, float lr, int t, const float* g, float* p, float* m, float* v,
                   uint16_t* pbf, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = float(1.0 - pow(0.9, double(t))), c2 = float(1.0 - pow(0.999, double(t)));
  hipLaunchKernelGGL(k_adam, dim3(gridn(n)), dim3(kB), 0, st, n, n_bf16, lr, b1, b2, 1e-8f, c1, c2, g, p, m, v,
                     pbf);
  return hipGetLastError();
}

hipError_t nn_to_bf16(int64_t n, const float* a, uint16_t* b, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(gridn(n)), dim3(kB), 0, st, n, a, b);
  return hipGetLastError();
}

hipError_t nn_grad_rms(int64_t nn, const double* g, double* partials, double* rms, hipStream_t st) {
  int nblk = gridn(nn);
  if (nblk > kMaxPartials / 4) nblk = kMaxPartials / 4;
  hipLaunchKernelGGL(k_sumsq4, dim3(nblk), dim3(kB), 0, st, nn, g, partials);
  hipLaunchKernelGGL(k_rms4, dim3(1), dim3(64), 0, st, nblk, nn, partials, rms);
  return hipGetLastError();
}

hipError_t nn_features(int64_t nn, const double* x, const double* g, const float* scales, const double* rms,
                       float* feat, hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3(gridn(nn * 8)), dim3(kB), 0, st, nn, x, g, scales, rms, feat);
  return hipGetLastError();
}

hipError_t nn_proposal(int64_t n, const float* out, const float* scales, const double* rms, const double* lo,
                       const double* hi, double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_proposal, dim3(gridn(n)), dim3(kB), 0, st, n, out, scales, rms, lo, hi, s);
  return hipGetLastError();
}

hipError_t nn_target(int64_t n, const double* s, const float* scales, const double* rms, float* t, hipStream_t st) {
  hipLaunchKernelGGL(k_target, dim3(gridn(n)), dim3(kB), 0, st, n, s, scales, rms, t);
  return hipGetLastError();
}

hipError_t nn_fit_scales(int ns, const double* rms_samples, float* scales, hipStream_t st) {
  hipLaunchKernelGGL(k_fit_scales, dim3(1), dim3(64), 0, st, ns, rms_samples, scales);
  return hipGetLastError();
}

}  // namespace rmtr

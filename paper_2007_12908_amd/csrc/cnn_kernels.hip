// The learned fine-level proposal: a 3D convolutional network (six 3x3x3
// layers, channels 8 -> 32 -> 32 -> 32 -> 32 -> 32 -> 4, ReLU after the
// first five, zero padding), with BF16 weights and FP32 arithmetic, and the
// kernels that train it (backward passes, MSE loss, Adam).
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

__device__ inline float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// round-to-nearest-even FP32 -> BF16
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

struct Box {
  int nx, ny, nz;
};

__device__ inline bool nb(const Box& b, int x, int y, int z, int k, int64_t& u, int sign) {
  const int dx = (k % 3 - 1) * sign, dy = ((k / 3) % 3 - 1) * sign, dz = (k / 9 - 1) * sign;
  const int X = x + dx, Y = y + dy, Z = z + dz;
  if (X < 0 || X >= b.nx || Y < 0 || Y >= b.ny || Z < 0 || Z >= b.nz) return false;
  u = int64_t(X) + int64_t(b.nx) * (Y + int64_t(b.ny) * Z);
  return true;
}

// Direct 3x3x3 convolution, used for the forward pass and for the data
// gradient:
//   out[v][o] = (bias[o]) + sum_k sum_i Wl[k][i][o] m(in)[v + SIGN off(k)][i]
// Forward: Wl = W (SIGN +1).  Data gradient: Wl[k][i][o] = W[k][o][i]
// (transposed while staging, SIGN -1) and m(in) = in masked by the ReLU of
// the layer's output (mask > 0).  Weights of the layer sit in LDS as BF16.
// A thread computes V consecutive voxels of one x-row for CG consecutive
// outputs: each LDS weight read (CG values) feeds V CG FMAs and each input
// load (4 channels of a voxel) feeds 4 CG FMAs.  The waves of a block
// share the voxels and split the outputs, so weight reads are broadcasts.
template <int NI, int NO, int SIGN, int TRANS, int BIAS, int RELU_OUT, int MASK_IN>
__global__ __launch_bounds__(kB) void k_conv(Box b, const float* __restrict__ in, const float* __restrict__ mask,
                                             const uint16_t* __restrict__ W, const float* __restrict__ bias,
                                             float* __restrict__ out) {
  constexpr int V = 4;
  constexpr int CG = NO < 8 ? NO : 8, NG = NO / CG, VGB = kB / NG;
  static_assert(NI % 4 == 0 && NO % CG == 0, "channel counts");
  __shared__ __align__(16) uint16_t sW[27 * NI * NO];
  for (int e = threadIdx.x; e < 27 * NI * NO; e += kB) {
    if (TRANS) {
      // sW[k][i][o] = W[k][o][i] with W of shape [27][NO][NI]
      const int k = e / (NI * NO), r = e % (NI * NO), i = r / NO, o = r % NO;
      sW[e] = W[(k * NO + o) * NI + i];
    } else {
      sW[e] = W[e];
    }
  }
  __syncthreads();
  const int gpr = (b.nx + V - 1) / V;
  const int64_t ngroups = int64_t(gpr) * b.ny * b.nz;
  const int gq = threadIdx.x / VGB, lv = threadIdx.x % VGB;
  for (int64_t G = int64_t(blockIdx.x) * VGB + lv; G < ngroups; G += int64_t(gridDim.x) * VGB) {
    const int x0 = V * int(G % gpr);
    const int64_t r = G / gpr;
    const int y = int(r % b.ny), z = int(r / b.ny);
    float acc[V][CG];
#pragma unroll
    for (int j = 0; j < V; ++j)
#pragma unroll
      for (int o = 0; o < CG; ++o) acc[j][o] = BIAS ? bias[gq * CG + o] : 0.0f;
    for (int k = 0; k < 27; ++k) {
      const int dx = SIGN * (k % 3 - 1), dy = SIGN * ((k / 3) % 3 - 1), dz = SIGN * (k / 9 - 1);
      const int Y = y + dy, Z = z + dz;
      if (Y < 0 || Y >= b.ny || Z < 0 || Z >= b.nz) continue;
      const int64_t row = (int64_t(Z) * b.ny + Y) * b.nx;
      bool ok[V];
      int64_t ub[V];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int X = x0 + j + dx;
        ok[j] = (x0 + j < b.nx) && X >= 0 && X < b.nx;
        ub[j] = (row + (ok[j] ? X : 0)) * NI;
      }
      const uint16_t* wk = sW + k * NI * NO + gq * CG;
      for (int i = 0; i < NI; i += 4) {
        float xin[V][4];
#pragma unroll
        for (int j = 0; j < V; ++j) {
          float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
          if (ok[j]) {
            a = *reinterpret_cast<const float4*>(in + ub[j] + i);
            if (MASK_IN) {
              const float4 mk = *reinterpret_cast<const float4*>(mask + ub[j] + i);
              a.x = mk.x > 0.0f ? a.x : 0.0f;
              a.y = mk.y > 0.0f ? a.y : 0.0f;
              a.z = mk.z > 0.0f ? a.z : 0.0f;
              a.w = mk.w > 0.0f ? a.w : 0.0f;
            }
          }
          xin[j][0] = a.x;
          xin[j][1] = a.y;
          xin[j][2] = a.z;
          xin[j][3] = a.w;
        }
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          float w[CG];
          const uint16_t* wp = wk + (i + ii) * NO;
          if (CG == 8) {
            const uint4 q = *reinterpret_cast<const uint4*>(wp);
            const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              w[2 * h] = __uint_as_float(qq[h] << 16);
              w[2 * h + 1] = __uint_as_float(qq[h] & 0xffff0000u);
            }
          } else {
#pragma unroll
            for (int o = 0; o < CG; ++o) w[o] = bf2f(wp[o]);
          }
#pragma unroll
          for (int j = 0; j < V; ++j)
#pragma unroll
            for (int o = 0; o < CG; ++o) acc[j][o] += xin[j][ii] * w[o];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (x0 + j >= b.nx) continue;
      float* op = out + ((int64_t(z) * b.ny + y) * b.nx + x0 + j) * NO + gq * CG;
#pragma unroll
      for (int o = 0; o < CG; ++o) op[o] = RELU_OUT ? fmaxf(acc[j][o], 0.0f) : acc[j][o];
    }
  }
}

// Forward convolution as an implicit GEMM on the matrix cores
// (v_mfma_f32_32x32x8_bf16, FP32 accumulation): a wavefront computes a tile
// of 32 x-consecutive voxels of one row by 32 output channels; the reduction
// runs over the 27 offsets times the input channels in chunks of 8.  The
// A operand is the layer input (FP32 in memory) rounded to BF16 on load,
// the B operand the layer's BF16 weights, staged in LDS as [k][o][i] so a
// lane reads its four consecutive input channels with one 8-byte load.
// Lane l holds A[l % 32][4 (l / 32) + t] and B[4 (l / 32) + t][l % 32]
// (t = 0..3); accumulator r of lane l is C[8 (r / 4) + 4 (l / 32) + r % 4]
// [l % 32].  Products of BF16 values are exact in FP32, so the result is
// the FP32 sum of the exact products.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <int NI, int NO, int RELU_OUT>
__global__ __launch_bounds__(256) void k_conv_mfma(Box b, const float* __restrict__ in,
                                                   const uint16_t* __restrict__ W, const float* __restrict__ bias,
                                                   float* __restrict__ out) {
  static_assert(NI % 8 == 0 && NO <= 32, "input channels in chunks of 8, at most 32 outputs");
  constexpr int NIP = NI, NOP = 32;
  __shared__ __align__(16) uint16_t sW[27 * NOP * NIP];
  for (int e = threadIdx.x; e < 27 * NOP * NIP; e += 256) {
    const int k = e / (NOP * NIP), o = (e / NIP) % NOP, i = e % NIP;
    sW[e] = o < NO ? W[(k * NI + i) * NO + o] : uint16_t(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;  // A row / B column, K half
  const int xtiles = (b.nx + 31) / 32;
  const int64_t ntiles = int64_t(xtiles) * b.ny * b.nz;
  for (int64_t T = int64_t(blockIdx.x) * 4 + wave; T < ntiles; T += int64_t(gridDim.x) * 4) {
    const int x0 = 32 * int(T % xtiles);
    const int64_t row = T / xtiles;
    const int y = int(row % b.ny), z = int(row / b.ny);
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int k = 0; k < 27; ++k) {
      const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
      const int Y = y + dy, Z = z + dz;
      if (Y < 0 || Y >= b.ny || Z < 0 || Z >= b.nz) continue;  // uniform over the wavefront
      const int X = x0 + li + dx;
      const bool ok = x0 + li < b.nx && X >= 0 && X < b.nx;
      const float* src = in + ((int64_t(Z) * b.ny + Y) * b.nx + (ok ? X : 0)) * NI + 4 * lk;
      const uint16_t* wk = sW + (k * NOP + li) * NIP + 4 * lk;
#pragma unroll
      for (int ic = 0; ic < NI / 8; ++ic) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ok) v = *reinterpret_cast<const float4*>(src + 8 * ic);
        bf16x4 a;
        a[0] = short(f2bf(v.x));
        a[1] = short(f2bf(v.y));
        a[2] = short(f2bf(v.z));
        a[3] = short(f2bf(v.w));
        const bf16x4 bw = *reinterpret_cast<const bf16x4*>(wk + 8 * ic);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bw, acc, 0, 0, 0);
      }
    }
    const int o = li;
    if (o < NO) {
      const float bo = bias[o];
      float* dst = out + ((int64_t(z) * b.ny + y) * b.nx + x0) * NO + o;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r / 4) + 4 * lk + (r % 4);
        if (x0 + i < b.nx) {
          const float val = acc[r] + bo;
          dst[int64_t(i) * NO] = RELU_OUT ? fmaxf(val, 0.0f) : val;
        }
      }
    }
  }
}

// Weight and bias gradient, first stage: each block sums over its voxel range
//   dW[k][ci][co] += X[v + off(k)][ci] dYm[v][co],  db[co] += dYm[v][co]
// into its own partial row (27 CIN COUT + COUT values).  Per tile of TV
// voxels, dYm is staged in LDS once and the shifted inputs once per offset;
// a thread owns an RI x RO block of the (ci, co) plane for all 27 offsets.
template <int CIN, int COUT, int RELU>
__global__ __launch_bounds__(kB) void k_conv_bwd_w(Box b, const float* __restrict__ X, const float* __restrict__ dY,
                                                   const float* __restrict__ Yact, int64_t vox_per_block,
                                                   float* __restrict__ partial) {
  constexpr int TV = 64, NE = CIN * COUT;
  constexpr int RI = NE >= 4 * kB ? 2 : 1, RO = RI;
  constexpr int TI = CIN / RI, TO = COUT / RO;
  static_assert(TI * TO <= kB && (TV * CIN) % kB == 0, "tiling");
  constexpr int XPT = TV * CIN / kB;
  __shared__ __align__(16) float sD[TV][COUT];
  __shared__ __align__(16) float sX[TV][CIN];
  const int64_t nvox = int64_t(b.nx) * b.ny * b.nz;
  const int64_t v0 = int64_t(blockIdx.x) * vox_per_block;
  const int64_t v1 = min(v0 + vox_per_block, nvox);
  const int tid = threadIdx.x;
  const bool owner = tid < TI * TO;
  const int ci0 = RI * (tid / TO), co0 = RO * (tid % TO);
  float acc[27][RI][RO];
#pragma unroll
  for (int k = 0; k < 27; ++k)
#pragma unroll
    for (int a = 0; a < RI; ++a)
#pragma unroll
      for (int c = 0; c < RO; ++c) acc[k][a][c] = 0.0f;
  float accb = 0.0f;
  for (int64_t vt = v0; vt < v1; vt += TV) {
    // coordinates of this thread's gather elements
    int gx[XPT], gy[XPT], gz[XPT];
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const int64_t v = vt + (tid + kB * j) / CIN;
      if (v < v1) {
        gx[j] = int(v % b.nx);
        gy[j] = int((v / b.nx) % b.ny);
        gz[j] = int(v / (int64_t(b.nx) * b.ny));
      } else {
        gx[j] = -4;  // outside for every offset
        gy[j] = 0;
        gz[j] = 0;
      }
    }
    __syncthreads();
    for (int e = tid; e < TV * COUT; e += kB) {
      const int64_t v = vt + e / COUT;
      float d = 0.0f;
      if (v < v1) {
        d = dY[v * COUT + e % COUT];
        if (RELU && !(Yact[v * COUT + e % COUT] > 0.0f)) d = 0.0f;
      }
      sD[e / COUT][e % COUT] = d;
    }
    __syncthreads();
    if (tid < COUT)
      for (int t = 0; t < TV; ++t) accb += sD[t][tid];
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
      if (k > 0) __syncthreads();
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        const int e = tid + kB * j;
        const int xx = gx[j] + dx, yy = gy[j] + dy, zz = gz[j] + dz;
        float xv = 0.0f;
        if (xx >= 0 && xx < b.nx && yy >= 0 && yy < b.ny && zz >= 0 && zz < b.nz)
          xv = X[((int64_t(zz) * b.ny + yy) * b.nx + xx) * CIN + e % CIN];
        sX[e / CIN][e % CIN] = xv;
      }
      __syncthreads();
      if (owner) {
        for (int t = 0; t < TV; ++t) {
          float xa[RI], da[RO];
#pragma unroll
          for (int a = 0; a < RI; ++a) xa[a] = sX[t][ci0 + a];
#pragma unroll
          for (int c = 0; c < RO; ++c) da[c] = sD[t][co0 + c];
#pragma unroll
          for (int a = 0; a < RI; ++a)
#pragma unroll
            for (int c = 0; c < RO; ++c) acc[k][a][c] += xa[a] * da[c];
        }
      }
    }
  }
  float* outp = partial + int64_t(blockIdx.x) * (27 * NE + COUT);
  if (owner) {
#pragma unroll
    for (int k = 0; k < 27; ++k)
#pragma unroll
      for (int a = 0; a < RI; ++a)
#pragma unroll
        for (int c = 0; c < RO; ++c) outp[k * NE + (ci0 + a) * COUT + co0 + c] = acc[k][a][c];
  }
  if (tid < COUT) outp[27 * NE + tid] = accb;
}

// Weight gradient on the matrix cores: for each offset k,
//   dW[k][ci][co] = sum_v X[v + off(k)][ci] dYm[v][co]
// is a 32 x 32 GEMM whose reduction runs over voxels, 8 per MFMA: lane l
// feeds A[ci = l % 32][voxel 4 (l / 32) + t] and B[voxel 4 (l / 32) + t]
// [co = l % 32], both rounded to BF16; the four wavefronts of a block split
// the 27 offsets (7, 7, 7, 6) and share the voxel chunks; partial rows per
// block as in k_conv_bwd_w (bias partials summed in FP32 by wavefront 0).
template <int CIN, int COUT, int RELU>
__global__ __launch_bounds__(256) void k_conv_bwd_w_mfma(Box b, const float* __restrict__ X,
                                                         const float* __restrict__ dY,
                                                         const float* __restrict__ Yact, int64_t vox_per_block,
                                                         float* __restrict__ partial) {
  static_assert(CIN <= 32 && COUT <= 32, "one 32 x 32 tile per offset");
  constexpr int NE = CIN * COUT, KW = 7;
  const int64_t nvox = int64_t(b.nx) * b.ny * b.nz;
  const int64_t v0 = int64_t(blockIdx.x) * vox_per_block;
  const int64_t v1 = min(v0 + vox_per_block, nvox);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;
  f32x16 acc[KW];
#pragma unroll
  for (int j = 0; j < KW; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.0f;
  float accb = 0.0f;
  for (int64_t vt = v0; vt < v1; vt += 8) {
    int cx[4], cy[4], cz[4];
    bool vok[4];
    bf16x4 bb;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t v = vt + 4 * lk + t;
      vok[t] = v < v1;
      const int64_t vv = vok[t] ? v : v0;
      // 32-bit division (boxes hold fewer than 2^31 voxels)
      const uint32_t u = uint32_t(vv), nx = uint32_t(b.nx), nxy = uint32_t(b.nx) * uint32_t(b.ny);
      cz[t] = int(u / nxy);
      const uint32_t rxy = u - uint32_t(cz[t]) * nxy;
      cy[t] = int(rxy / nx);
      cx[t] = int(rxy - uint32_t(cy[t]) * nx);
      float d = 0.0f;
      if (vok[t] && li < COUT) {
        d = dY[vv * COUT + li];
        if (RELU && !(Yact[vv * COUT + li] > 0.0f)) d = 0.0f;
      }
      accb += d;
      bb[t] = short(f2bf(d));
    }
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      const int k = wave + 4 * j;
      if (k >= 27) break;
      const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
      bf16x4 a;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int xx = cx[t] + dx, yy = cy[t] + dy, zz = cz[t] + dz;
        float xv = 0.0f;
        if (vok[t] && li < CIN && xx >= 0 && xx < b.nx && yy >= 0 && yy < b.ny && zz >= 0 && zz < b.nz)
          xv = X[((int64_t(zz) * b.ny + yy) * b.nx + xx) * CIN + li];
        a[t] = short(f2bf(xv));
      }
      acc[j] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bb, acc[j], 0, 0, 0);
    }
  }
  float* outp = partial + int64_t(blockIdx.x) * (27 * NE + COUT);
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    const int k = wave + 4 * j;
    if (k >= 27) break;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ci = 8 * (r / 4) + 4 * lk + (r % 4), co = li;
      if (ci < CIN && co < COUT) outp[k * NE + ci * COUT + co] = acc[j][r];
    }
  }
  // bias partial: lanes l and l + 32 hold the two voxel halves of channel l
  const float other = __shfl_xor(accb, 32);
  if (wave == 0 && lk == 0 && li < COUT) outp[27 * NE + li] = accb + other;
}

// second stage: fixed-order sum of the partial rows
__global__ __launch_bounds__(kB) void k_sum_partials(const float* __restrict__ partial, int nblk, int64_t len,
                                                     float* __restrict__ dw, float* __restrict__ db, int64_t nw) {
  for (int64_t e = int64_t(blockIdx.x) * kB + threadIdx.x; e < len; e += int64_t(gridDim.x) * kB) {
    float s = 0.0f;
    for (int i = 0; i < nblk; ++i) s += partial[int64_t(i) * len + e];
    if (e < nw)
      dw[e] = s;
    else
      db[e - nw] = s;
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

int gridn(int64_t work) {
  int64_t b = (work + kB - 1) / kB;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return int(b);
}

// convolution grids: persistent blocks (each stages the layer's weights in
// LDS once), about four per compute unit
int convgrid(int64_t work) {
  const int g = gridn(work);
  return g < 1024 ? g : 1024;
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
    const int64_t tiles = int64_t((nx + 31) / 32) * ny * nz;
    const dim3 grid(unsigned(std::min<int64_t>((tiles + 3) / 4, 2048)));
    if (l == 0)
      hipLaunchKernelGGL((k_conv_mfma<8, 32, 1>), grid, dim3(256), 0, st, b, X, W, bb, Y);
    else if (l < 5)
      hipLaunchKernelGGL((k_conv_mfma<32, 32, 1>), grid, dim3(256), 0, st, b, X, W, bb, Y);
    else
      hipLaunchKernelGGL((k_conv_mfma<32, 4, 0>), grid, dim3(256), 0, st, b, X, W, bb, Y);
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
  int nblk = 512;
  if (nvox < 512 * 64) nblk = int((nvox + 63) / 64);
  const int64_t vpb = (nvox + nblk - 1) / nblk;
  const float* dY = dout;
  for (int l = 5; l >= 0; --l) {
    const int cin = kCh[l], cout = kCh[l + 1];
    const float* X = act + a_off(l, nvox);
    const float* Yact = act + a_off(l + 1, nvox);
    const uint16_t* W = w + w_off(l);
    const int64_t len = int64_t(27) * cin * cout + cout;
    // weights: layer 5 has no ReLU on its output
    if (l == 5)
      hipLaunchKernelGGL((k_conv_bwd_w_mfma<32, 4, 0>), dim3(nblk), dim3(256), 0, st, b, X, dY, Yact, vpb, part);
    else if (l > 0)
      hipLaunchKernelGGL((k_conv_bwd_w_mfma<32, 32, 1>), dim3(nblk), dim3(256), 0, st, b, X, dY, Yact, vpb, part);
    else
      hipLaunchKernelGGL((k_conv_bwd_w_mfma<8, 32, 1>), dim3(nblk), dim3(256), 0, st, b, X, dY, Yact, vpb, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(gridn(len)), dim3(kB), 0, st, part, nblk, len, dw + w_off(l),
                       db + b_off(l), int64_t(27) * cin * cout);
    if (l == 0) break;
    float* dX = (l % 2) ? gA : gB;
    // data gradient: inputs dY (cout channels, masked by the layer's ReLU),
    // outputs cin channels, transposed weights, mirrored offsets
    const int64_t groups = int64_t((nx + 3) / 4) * ny * nz;
    if (l == 5)
      hipLaunchKernelGGL((k_conv<4, 32, -1, 1, 0, 0, 0>), dim3(convgrid(groups * 4)), dim3(kB), 0, st, b, dY,
                         nullptr, W, nullptr, dX);
    else
      hipLaunchKernelGGL((k_conv<32, 32, -1, 1, 0, 0, 1>), dim3(convgrid(groups * 4)), dim3(kB), 0, st, b, dY, Yact,
                         W, nullptr, dX);
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

}  // namespace rmtr

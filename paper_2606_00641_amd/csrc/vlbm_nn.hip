// Learned coarse-grid correction (include/vlbm_nn.h): BF16 MFMA convolution
// kernels (forward, data gradient, weight gradient), loss, Adam, restriction, the
// FP64 gate and the corrected coarse step.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (gfx950): one
// workgroup (8 wavefronts, two tile rows each) computes a 16 x 16 tile of output positions for every
// output channel; the 18 x 18 input halo (periodic) is staged in LDS in
// channels-last order so that one lane's A fragment (8 consecutive input channels
// of one tap, or 8 taps' worth for 8-channel inputs) is a single 16-byte LDS read.
// B fragments (weights) are packed once per weight update in the exact lane order
// of the instruction and held in registers for the whole tile.
//
// MFMA 16x16x32 operand layout (verified on the device): lane l holds
// A[i = l % 16][k = 8 (l / 16) + e] and B[k = 8 (l / 16) + e][j = l % 16] for
// e = 0..7; the result D[i = 4 (l / 16) + r][j = l % 16] for r = 0..3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "vlbm.h"
#include "vlbm_ctx.h"
#include "vlbm_device.h"
#include "vlbm_kernels.h"
#include "vlbm_nn.h"

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef unsigned short bf16_t;

constexpr int TILE = 16;
constexpr int HALO = TILE + 2;
constexpr int kThreads = 256;
// Convolution workgroups: eight wavefronts, two tile rows each (measured against four
// rows per wavefront: 13 % faster on a 256^2 lattice, 10 % on 384 x 192 x 192 in 3D;
// one row per wavefront was slower again).
constexpr int kConvRows = 2;
constexpr int kConvThreads = 64 * (TILE / kConvRows);
constexpr int kMaxLayers = 8;
constexpr int kGateThreads = 256;

// Sum of a double over the 64 lanes of a wavefront, in every lane.  The four levels
// inside each row of 16 lanes use DPP row rotations (by 8, 4, 2, 1; VALU only, every
// lane of a row ends with the row's sum), the two levels across rows lane shuffles.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0x128>(v);  // row_ror:8
  v += dpp_f64<0x124>(v);  // row_ror:4
  v += dpp_f64<0x122>(v);  // row_ror:2
  v += dpp_f64<0x121>(v);  // row_ror:1
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

enum { MODE_HIDDEN = 0, MODE_LAST = 1, MODE_BWD = 2 };

__host__ __device__ inline int ksteps(int cin) { return (9 * cin + 31) / 32; }
__host__ __device__ inline int ntiles(int cout) { return (cout + 15) / 16; }

__device__ __forceinline__ bf16_t f2bf(float f) {
  const unsigned u = __float_as_uint(f);
  return (bf16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // nearest even (finite)
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float((unsigned)b << 16); }

// exact GELU and its derivative (standard normal CDF via erf)
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// ---------------------------------------------------------------------------
// weight packing into B-fragment order
// ---------------------------------------------------------------------------
// Forward (flip = 0): B[k][n] = W[n][c][tap] with k = tap * CIN + c over this conv's
// input channels CIN and outputs n < COUT.
// Data gradient (flip = 1) of a layer with weights W[o][c][tap] (o < CO, c < CI): a
// convolution of dZ (CI' = CO input channels) producing CO' = CI outputs with
// B[k = tap' * CO + o][n = c] = W[o][c][ntap - 1 - tap'] (taps mirrored: offset -> -offset).
// ntap = 9 (3x3) or 27 (3x3x3, tap = 9 kz + 3 ky + kx): the 27 taps are packed as three
// z-slabs of the 3x3 layout, slab kz at offset kz * ksteps * ntiles * 512.
__global__ void k_pack(const float* __restrict__ W, int CI, int CO, int flip, int ntap, bf16_t* __restrict__ out) {
  const int cin = flip ? CO : CI;    // input channels of the packed convolution
  const int cout = flip ? CI : CO;   // its output channels
  const int KS = ksteps(cin), NT = ntiles(cout);
  const int per_slab = KS * NT * 64 * 8;
  const int total = (ntap / 9) * per_slab;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= total) return;
  const int slab = q / per_slab, qs = q % per_slab;
  const int e = qs & 7, lane = (qs >> 3) & 63, st = qs >> 9;
  const int t = st % NT, s = st / NT;
  const int k = 32 * s + 8 * (lane >> 4) + e;
  const int n = 16 * t + (lane & 15);
  const int tap2 = k / cin, c = k % cin;
  float v = 0.0f;
  if (tap2 < 9 && n < cout) {
    const int tap = 9 * slab + tap2;
    if (!flip)
      v = W[((size_t)n * CI + c) * ntap + tap];
    else
      v = W[((size_t)c * CI + n) * ntap + (ntap - 1 - tap)];  // W[o = c][c_in = n][mirrored tap]
  }
  out[q] = f2bf(v);
}

// ---------------------------------------------------------------------------
// convolution (forward, and data gradient with the mirrored packed weights)
// ---------------------------------------------------------------------------
// act: BF16 channels-last [S][H][W][CIN] over S = B * D slices (D = 1: a batch of 2D
// lattices; D > 1: B 3D lattices of D slices each, periodic in z).  NZT = 1 for the
// 3x3 kernel, 3 for the 3x3x3 kernel (the halos of slices z-1, z, z+1 are staged
// and the packed weights of each z-slab are loaded in turn).  Output, by MODE:
//  HIDDEN: z = conv + bias; out_act (BF16 NHWC COUT) = GELU(z); out_z (FP32 NHWC, optional) = z
//  LAST:   out_z (FP32 channel-major [COUT][B][H][W]) = (conv + bias) * oscale + oshift
//  BWD:    out_act (BF16 NHWC COUT) = conv * GELU'(zprev), zprev FP32 NHWC COUT
template <int CIN, int COUT, int MODE, int NZT>
__global__ __launch_bounds__(kConvThreads) void k_conv(const bf16_t* __restrict__ act, const bf16_t* __restrict__ wpack,
                                                   const float* __restrict__ bias, int D, int H, int W,
                                                   bf16_t* __restrict__ out_act, float* __restrict__ out_z,
                                                   const float* __restrict__ zprev,
                                                   const float* __restrict__ oscale,
                                                   const float* __restrict__ oshift) {
  constexpr int KS = (9 * CIN + 31) / 32;
  constexpr int NT = (COUT + 15) / 16;
  constexpr int CH = CIN / 8;
  constexpr int MR = kConvRows;     // rows of the 16 x 16 tile per wavefront
  constexpr int NTH = kConvThreads;
  // The input halo, and after the products the FP32 results of the tile (HIDDEN and
  // BWD), share one LDS buffer.  Result rows are padded by 4 floats so that the four
  // lane groups of a store land in distinct banks.
  constexpr int OS = COUT + 4;
  // Halo positions are stored unpadded, 2 CIN bytes apart.  (Padding the 32-channel
  // positions to 40 channels, meant to spread the A-fragment reads over the banks,
  // was measured with SQ_LDS_BANK_CONFLICT to raise the conflict cycles by a third
  // and left the time unchanged.)
  constexpr int PS = CIN;
  constexpr int kTileBytes = NZT * HALO * HALO * PS * 2;
  constexpr int kOutBytes = MODE == MODE_LAST ? 0 : TILE * TILE * OS * 4;
  __shared__ __attribute__((aligned(16))) unsigned char lds[kTileBytes > kOutBytes ? kTileBytes : kOutBytes];
  bf16_t* tile = reinterpret_cast<bf16_t*>(lds);
  const int sl = blockIdx.z, ty0 = blockIdx.y * TILE, tx0 = blockIdx.x * TILE;
  const int zl = sl % D, zbase = sl - zl;  // slice within its lattice, first slice of the lattice
  for (int q = threadIdx.x; q < NZT * HALO * HALO * CH; q += NTH) {
    const int zs = q / (HALO * HALO * CH), r = q % (HALO * HALO * CH);
    const int pix = r / CH, ch = r % CH;
    const int hy = pix / HALO, hx = pix % HALO;
    int gz = zl + zs - NZT / 2;
    int gy = ty0 - 1 + hy;
    int gx = tx0 - 1 + hx;
    gz = gz < 0 ? gz + D : (gz >= D ? gz - D : gz);
    gy = gy < 0 ? gy + H : (gy >= H ? gy - H : gy);
    gx = gx < 0 ? gx + W : (gx >= W ? gx - W : gx);
    const uint4 v =
        *reinterpret_cast<const uint4*>(act + (((size_t)(zbase + gz) * H + gy) * W + gx) * CIN + ch * 8);
    *reinterpret_cast<uint4*>(tile + (zs * HALO * HALO + pix) * PS + ch * 8) = v;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  bf16x8 bw[KS][NT];
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int t = 0; t < NT; ++t)
      bw[s][t] = *reinterpret_cast<const bf16x8*>(wpack + ((size_t)(s * NT + t) * 64 + lane) * 8);
  __syncthreads();

  f32x4 acc[MR][NT];
#pragma unroll
  for (int m = 0; m < MR; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  const int px = lane & 15, g = lane >> 4;
#pragma unroll 1
  for (int zs = 0; zs < NZT; ++zs) {
    if (zs > 0) {  // weights of the next z-slab
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          bw[s][t] = *reinterpret_cast<const bf16x8*>(wpack + ((size_t)((zs * KS + s) * NT + t) * 64 + lane) * 8);
    }
    const bf16_t* tz = tile + zs * HALO * HALO * PS;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int py = MR * wv + m;
        bf16x8 a;
        if constexpr (CIN == 32) {
          const int dy = s / 3, dx = s % 3;
          a = *reinterpret_cast<const bf16x8*>(tz + ((py + dy) * HALO + px + dx) * PS + 8 * g);
        } else {
          const int tap = 4 * s + g;  // 8 input channels: 4 taps per K step
          if (tap < 9) {
            const int dy = tap / 3, dx = tap % 3;
            a = *reinterpret_cast<const bf16x8*>(tz + ((py + dy) * HALO + px + dx) * PS);
          } else {
            a = bf16x8{};  // zero padding of K
          }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][t], acc[m][t], 0, 0, 0);
      }
    }
  }

  if constexpr (MODE == MODE_LAST) {
    // channel-major output: a lane's four results are four consecutive x of one channel
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int y = ty0 + MR * wv + m;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int co = 16 * t + (lane & 15);
        if (co >= COUT) continue;
        const float b = bias[co], sc = oscale[co], sh = oshift[co];
        float4 o;
        o.x = (acc[m][t][0] + b) * sc + sh;
        o.y = (acc[m][t][1] + b) * sc + sh;
        o.z = (acc[m][t][2] + b) * sc + sh;
        o.w = (acc[m][t][3] + b) * sc + sh;
        *reinterpret_cast<float4*>(out_z + (((size_t)co * gridDim.z + sl) * H + y) * W + tx0 + 4 * g) = o;
      }
    }
  } else {
    // channels-last outputs: stage the tile's results [position][channel] in LDS, then
    // every thread finishes four consecutive channels of a position with 16-byte loads
    // and stores
    float* ob = reinterpret_cast<float*>(lds);
    __syncthreads();  // every wavefront is done with the halo
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int co = 16 * t + (lane & 15);
        if (co >= COUT) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) ob[((MR * wv + m) * TILE + 4 * g + r) * OS + co] = acc[m][t][r];
      }
    __syncthreads();
    constexpr int C4 = COUT / 4;
    for (int q = threadIdx.x; q < TILE * TILE * C4; q += NTH) {
      const int pos = q / C4, c0 = 4 * (q % C4);
      const int y = ty0 + pos / TILE, x = tx0 + pos % TILE;
      const size_t nhwc = (((size_t)sl * H + y) * W + x) * COUT + c0;
      const float4 v = *reinterpret_cast<const float4*>(ob + pos * OS + c0);
      float a[4];
      if constexpr (MODE == MODE_HIDDEN) {
        const float4 b = *reinterpret_cast<const float4*>(bias + c0);
        const float4 z = make_float4(v.x + b.x, v.y + b.y, v.z + b.z, v.w + b.w);
        a[0] = gelu(z.x), a[1] = gelu(z.y), a[2] = gelu(z.z), a[3] = gelu(z.w);
        if (out_z) *reinterpret_cast<float4*>(out_z + nhwc) = z;
      } else {
        const float4 zp = *reinterpret_cast<const float4*>(zprev + nhwc);
        a[0] = v.x * gelu_grad(zp.x), a[1] = v.y * gelu_grad(zp.y);
        a[2] = v.z * gelu_grad(zp.z), a[3] = v.w * gelu_grad(zp.w);
      }
      uint2 packed;
      packed.x = (unsigned)f2bf(a[0]) | ((unsigned)f2bf(a[1]) << 16);
      packed.y = (unsigned)f2bf(a[2]) | ((unsigned)f2bf(a[3]) << 16);
      *reinterpret_cast<uint2*>(out_act + nhwc) = packed;
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[o][c][tap] = sum_{b,p} dZ[b,p,o] act[b, p + off(tap), c];
// db[o] = sum dZ.  GEMM with M = o, N = (tap, c), K = positions; each workgroup
// accumulates over a fixed set of tiles and writes one partial (reduced later in a
// fixed order, so the result is deterministic).  Positions run over S slices of
// D-slice lattices (as k_conv); blockIdx.y selects the z-slab of a 3x3x3 kernel
// (gridDim.y = 3; taps 9 kz + 3 ky + kx, columns of the partial tap * CIN + c over
// all 27 taps) or is 0 for the 3x3 kernel (gridDim.y = 1).
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(kThreads) void k_conv_bw(const bf16_t* __restrict__ act, const bf16_t* __restrict__ dz,
                                                      int S, int D, int H, int W, float* __restrict__ part_w,
                                                      float* __restrict__ part_b) {
  constexpr int NJ = 9 * CIN;  // columns of this z-slab
  constexpr int NTJ = (NJ + 15) / 16;
  constexpr int MT = (COUT + 15) / 16;
  constexpr int NTW = (NTJ + 3) / 4;  // N tiles per wavefront
  // LDS rows padded against bank conflicts: a channel's halo (324 elements) to 326, an
  // odd number of dwords, so that the 16 channels a lane group reads fall in distinct
  // banks; a row of dZ (256 positions, 512 bytes: every lane of a group in one bank) by
  // 8 elements, 33 16-byte groups.
  constexpr int AS = HALO * HALO + 2;
  constexpr int DZS = TILE * TILE + 8;
  __shared__ __attribute__((aligned(16))) bf16_t aT[CIN * AS];
  __shared__ __attribute__((aligned(16))) bf16_t dzT[MT * 16 * DZS];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4;
  f32x4 acc[MT][NTW];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int u = 0; u < NTW; ++u) acc[mt][u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  float db = 0.0f;
  const int slab = blockIdx.y, nslab = gridDim.y;
  const int tiles_x = W / TILE, tiles_y = H / TILE;
  const int ntile = S * tiles_x * tiles_y;
  for (int tid = blockIdx.x; tid < ntile; tid += gridDim.x) {
    const int sl = tid / (tiles_x * tiles_y);
    const int rem = tid % (tiles_x * tiles_y);
    const int ty0 = (rem / tiles_x) * TILE, tx0 = (rem % tiles_x) * TILE;
    const int zl = sl % D;
    int gz = zl + slab - nslab / 2;
    gz = gz < 0 ? gz + D : (gz >= D ? gz - D : gz);
    const int asl = sl - zl + gz;  // input slice of this z-slab
    __syncthreads();  // previous tile fully consumed
    for (int q = threadIdx.x; q < HALO * HALO * (CIN / 8); q += kThreads) {
      const int pix = q / (CIN / 8), ch = q % (CIN / 8);
      const int hy = pix / HALO, hx = pix % HALO;
      int gy = ty0 - 1 + hy;
      int gx = tx0 - 1 + hx;
      gy = gy < 0 ? gy + H : (gy >= H ? gy - H : gy);
      gx = gx < 0 ? gx + W : (gx >= W ? gx - W : gx);
      const uint4 v = *reinterpret_cast<const uint4*>(act + (((size_t)asl * H + gy) * W + gx) * CIN + ch * 8);
      const bf16_t* e = reinterpret_cast<const bf16_t*>(&v);
#pragma unroll
      for (int j = 0; j < 8; ++j) aT[(ch * 8 + j) * AS + hy * HALO + hx] = e[j];
    }
    for (int q = threadIdx.x; q < MT * 16 * TILE * TILE; q += kThreads) {
      const int o = q / (TILE * TILE), p = q % (TILE * TILE);
      const int y = ty0 + p / TILE, x = tx0 + p % TILE;
      dzT[o * DZS + p] = o < COUT ? dz[(((size_t)sl * H + y) * W + x) * COUT + o] : (bf16_t)0;
    }
    __syncthreads();
    if (slab == 0 && (int)threadIdx.x < COUT) {
      float sacc = 0.0f;
      for (int p = 0; p < TILE * TILE; ++p) sacc += bf2f(dzT[threadIdx.x * DZS + p]);
      db += sacc;
    }
#pragma unroll
    for (int s = 0; s < (TILE * TILE) / 32; ++s) {
      bf16x8 afr[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        afr[mt] = *reinterpret_cast<const bf16x8*>(dzT + (16 * mt + (lane & 15)) * DZS + 32 * s + 8 * g);
      const int pos0 = 32 * s + 8 * g;  // 8 consecutive positions of one tile row
      const int py = pos0 / TILE, px0 = pos0 % TILE;
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        const int nt = wv + 4 * u;
        if (nt >= NTJ) continue;
        const int j = 16 * nt + (lane & 15);
        bf16x8 bfr = bf16x8{};
        if (j < NJ) {
          const int tap = j / CIN, c = j % CIN;
          const int dy = tap / 3, dx = tap % 3;
          const bf16_t* src = aT + c * AS + (py + dy) * HALO + px0 + dx;  // 8 positions, unaligned
#pragma unroll
          for (int e = 0; e < 8; ++e) bfr[e] = __builtin_bit_cast(__bf16, src[e]);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[mt], bfr, acc[mt][u], 0, 0, 0);
      }
    }
  }
  // partial results of this workgroup
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int u = 0; u < NTW; ++u) {
      const int nt = wv + 4 * u;
      if (nt >= NTJ) continue;
      const int j = 16 * nt + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * mt + 4 * g + r;
        if (o < COUT && j < NJ)
          part_w[((size_t)blockIdx.x * COUT + o) * (nslab * NJ) + slab * NJ + j] = acc[mt][u][r];
      }
    }
  if (slab == 0 && (int)threadIdx.x < COUT) part_b[(size_t)blockIdx.x * COUT + threadIdx.x] = db;
}

// Sum the partials in block order into the master-layout gradient:
// grad_W[o][c][tap] = sum_blk part_w[blk][o][tap * CIN + c]; grad_b[o] = sum part_b
// (ntap = 9 or 27 taps).
__global__ void k_reduce_grads(const float* __restrict__ part_w, const float* __restrict__ part_b, int nblk,
                               int CIN, int COUT, int ntap, float* __restrict__ gW, float* __restrict__ gb) {
  const int NJ = ntap * CIN;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < COUT * NJ) {
    const int o = q / NJ, rem = q % NJ;  // rem = c * ntap + tap in master order
    const int c = rem / ntap, tap = rem % ntap;
    const int j = tap * CIN + c;
    float s = 0.0f;
    for (int blk = 0; blk < nblk; ++blk) s += part_w[((size_t)blk * COUT + o) * NJ + j];
    gW[q] = s;
  } else if (q < COUT * NJ + COUT) {
    const int o = q - COUT * NJ;
    float s = 0.0f;
    for (int blk = 0; blk < nblk; ++blk) s += part_b[(size_t)blk * COUT + o];
    gb[o] = s;
  }
}

// raw moments X (FP32 channel-major [C][B][H][W]) -> standardised BF16 NHWC (C = 8)
__global__ void k_prep(const float* __restrict__ X, int B, int C, int H, int W, const float* __restrict__ mean,
                       const float* __restrict__ istd, bf16_t* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // = b * HW + p
  const size_t BHW = (size_t)B * H * W;
  if (q >= BHW) return;
  for (int c = 0; c < C; ++c) out[q * C + c] = f2bf((X[(size_t)c * BHW + q] - mean[c]) * istd[c]);
}

// MSE on standardised outputs: y (FP32 [C][B][H][W]), target T raw -> (T - mean) * istd.
// dZ = 2 (y - t) / n as BF16 NHWC; per-block FP64 partial sums of (y - t)^2.
__global__ __launch_bounds__(kThreads) void k_loss(const float* __restrict__ y, const float* __restrict__ T, int B,
                                                   int C, int H, int W, const float* __restrict__ mean,
                                                   const float* __restrict__ istd, bf16_t* __restrict__ dz,
                                                   double* __restrict__ partial) {
  __shared__ double sh[kThreads / 64];
  const size_t HW = (size_t)H * W;
  const size_t n = (size_t)B * C * HW;
  const double inv_n = 1.0 / (double)n;
  double acc = 0.0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const size_t BHW = (size_t)B * HW;
    const size_t c = q / BHW, bp = q % BHW;  // bp = b * HW + p
    const float t = (T[q] - mean[c]) * istd[c];
    const float d = y[q] - t;
    acc += (double)d * (double)d;
    dz[bp * C + c] = f2bf((float)(2.0 * inv_n) * d);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += sh[w];
    partial[blockIdx.x] = s * inv_n;
  }
}

__global__ void k_sum_partials(const double* __restrict__ partial, int n, double* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += partial[j];
    out[0] = s;
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.0f - b1) * gq;
  const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// block mean of a moment field (FP64 accumulation), minus an optional field
__global__ void k_restrict(const float* __restrict__ Qf, int K, int nx, int ny, int nz, int r, int rz,
                           const float* __restrict__ minus, float* __restrict__ Qc) {
  const int cx = nx / r, cy = ny / r, cz = nz / rz;
  const size_t nc = (size_t)cx * cy * cz;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc * K) return;
  const int k = (int)(q / nc);
  const size_t c = q % nc;
  const int x = (int)(c % cx), y = (int)((c / cx) % cy), z = (int)(c / ((size_t)cx * cy));
  double s = 0.0;
  for (int dz = 0; dz < rz; ++dz)
    for (int dy = 0; dy < r; ++dy)
      for (int dx = 0; dx < r; ++dx)
        s += Qf[(size_t)k * nx * ny * nz + ((size_t)(z * rz + dz) * ny + (y * r + dy)) * nx + (x * r + dx)];
  double v = s / (double)(r * r * rz);
  if (minus) v -= (double)minus[q];
  Qc[q] = (float)v;
}

// ---------------------------------------------------------------------------
// corrected coarse stepping (2D, 8 variables)
// ---------------------------------------------------------------------------

// Cells x - e_i (periodic) for i = 0..2D (rest, +x, -x, +y, -y[, +z, -z]) of cell c.
// D = 2: the grid is a batch of independent 2D lattices along z; D = 3: one 3D lattice.
template <int D>
__device__ inline void upwind_cells(const vlbm::Grid& g, size_t c, size_t* up) {
  const size_t nxy = (size_t)g.nx * g.ny;
  const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / nxy);
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
  const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y + 1 == g.ny ? 0 : y + 1;
  const size_t sl = (size_t)z * nxy;
  up[0] = c;
  up[1] = sl + (size_t)y * g.nx + xm;
  up[2] = sl + (size_t)y * g.nx + xp;
  up[3] = sl + (size_t)ym * g.nx + x;
  up[4] = sl + (size_t)yp * g.nx + x;
  if constexpr (D == 3) {
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z + 1 == g.nz ? 0 : z + 1;
    const size_t r = (size_t)y * g.nx + x;
    up[5] = (size_t)zm * nxy + r;
    up[6] = (size_t)zp * nxy + r;
  }
}

// add w_i dQ_k to every population at the given parity; ctl NULL: dQ_k = dq[k][c];
// else only if ctl[0], with dQ_k = dq[k][c] - mean[b][k] of control block ctl (the
// layout launch_sweep_inj describes).  FP16/BF16 deviations are decoded, incremented in
// FP32 and encoded again
template <int ST, int D>
__global__ void k_inject(const vlbm::Grid g, const vlbm::Codec cd, int parity, const float* __restrict__ dq,
                         const int* __restrict__ ctl, double wi_d) {
  using S = vlbm::Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  constexpr int K = 8, NQ = 2 * D + 1;
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N || (ctl && !ctl[0])) return;
  size_t up[NQ];
  upwind_cells<D>(g, c, up);
  const int* mean = ctl ? ctl + 1 + 8 * vlbm::inj_lattice(D, (int)(c / ((size_t)g.nx * g.ny))) : nullptr;
  T* F = static_cast<T*>(g.f);
  // same weights, in the same type, as the injecting sweep
  const R wi = (R)wi_d;
  const R w0 = vlbm::rest_weight<R, D>(wi);
  for (int k = 0; k < K; ++k) {
    const R d = (R)(mean ? dq[(size_t)k * N + c] - __int_as_float(mean[k]) : dq[(size_t)k * N + c]);
    if (d == R(0)) continue;  // nothing to add: the stored values stay as they are
    for (int i = 0; i < NQ; ++i) {
      const int slot = parity == 0 ? i : vlbm::opposite(i);
      const size_t dst = parity == 0 ? c : up[i];
      T& v = F[(size_t)(k * NQ + slot) * g.stride + dst];
      v = S::enc(S::dec(v, cd, k * NQ + i) + (i == 0 ? w0 : wi) * d, cd, k * NQ + i);
    }
  }
}

struct GateBounds {
  double corr[8];
  double divb_rel, divb_abs;
};

// Gate statistics of the network's raw correction.  The fine run, its restriction and
// the coarse VLBM all keep each lattice's totals of rho, rho u, E and B (up to the Powell
// source), so the correction they define has zero total; projecting the prediction onto
// that (each lattice's mean removed, channel by channel) keeps a small bias of the
// network from accumulating in the totals over many steps.  The projection is not
// applied here: k_gate_final forms the means from these sums and the injection
// subtracts them, and since a constant has no central difference and
// sum (r - m)^2 = sum r^2 - 2 m sum r + n m^2, the gate's statistics of the projected
// correction follow from those of the raw one.
// Every workgroup works inside one lattice (blockIdx.y) and accumulates over its cells
// the FP64 partials: [0..7] sum r_k^2, [8..15] sum r_k, [16] sum divc(X)^2,
// [17] sum divc(X + r)^2, [18] non-finite count, [19] sum |B(X)|^2 (the D components
// the divergence sees), [20] (gm1 > 0) count of cells X + r leaves with rho <= 0 or a
// negative pressure (gm1 = gamma - 1; meaningful where the correction is not
// projected, so that X + r is the corrected state); r = raw, the network's output.
// D = 2: nz lattices of nx x ny (divergence of the in-plane field); D = 3: one
// nx x ny x nz lattice.
constexpr int kGateNP = 21;

template <int D>
__global__ __launch_bounds__(kGateThreads) void k_gate_partials(const float* __restrict__ X, const float* __restrict__ raw,
                                                                int nx, int ny, int nz, double gm1,
                                                                double* __restrict__ partial) {
  constexpr int NP = kGateNP;
  __shared__ double sh[kGateThreads / 64][NP];
  const int nb = gridDim.y, b = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[NP];
  for (int j = 0; j < NP; ++j) acc[j] = 0.0;
  // 32-bit cell arithmetic: a corrected context has at most 2^28 cells
  const unsigned nxy = (unsigned)nx * (unsigned)ny, N32 = nxy * (unsigned)nz, ncl = N32 / (unsigned)nb;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < ncl; i += gridDim.x * blockDim.x) {
    const unsigned c = (unsigned)b * ncl + i;
    const unsigned z = c / nxy, r = c - z * nxy, y = r / (unsigned)nx, x = r - y * (unsigned)nx;
    const unsigned sl = z * nxy;  // z-slice
    const unsigned xp = sl + y * nx + (x + 1 == (unsigned)nx ? 0 : x + 1), xm = sl + y * nx + (x == 0 ? nx - 1 : x - 1);
    const unsigned yp = sl + (y + 1 == (unsigned)ny ? 0 : y + 1) * nx + x, ym = sl + (y == 0 ? ny - 1 : y - 1) * nx + x;
    for (int k = 0; k < 8; ++k) {
      const double d = raw[k * N32 + c];
      acc[k] += d * d;
      acc[8 + k] += d;
      if (!(d - d == 0.0)) acc[18] += 1.0;
    }
    const float* Bx = X + 5 * N32;
    const float* By = X + 6 * N32;
    const float* rBx = raw + 5 * N32;
    const float* rBy = raw + 6 * N32;
    double dv = 0.5 * ((double)Bx[xp] - Bx[xm]) + 0.5 * ((double)By[yp] - By[ym]);
    double ddv = 0.5 * ((double)rBx[xp] - rBx[xm]) + 0.5 * ((double)rBy[yp] - rBy[ym]);
    double b2 = (double)Bx[c] * Bx[c] + (double)By[c] * By[c];
    if constexpr (D == 3) {
      const unsigned zp = (z + 1 == (unsigned)nz ? 0 : z + 1) * nxy + r, zm = (z == 0 ? nz - 1 : z - 1) * nxy + r;
      const float* Bz = X + 7 * N32;
      const float* rBz = raw + 7 * N32;
      dv += 0.5 * ((double)Bz[zp] - Bz[zm]);
      ddv += 0.5 * ((double)rBz[zp] - rBz[zm]);
      b2 += (double)Bz[c] * Bz[c];
    }
    const double dv2 = dv + ddv;
    acc[16] += dv * dv;
    acc[17] += dv2 * dv2;
    acc[19] += b2;
    if (gm1 > 0.0) {
      double q[8];
      for (int k = 0; k < 8; ++k) q[k] = (double)X[k * N32 + c] + (double)raw[k * N32 + c];
      const double kin = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
      const double mag = 0.5 * (q[5] * q[5] + q[6] * q[6] + q[7] * q[7]);
      if (!(q[0] > 0.0) || !(gm1 * (q[4] - kin - mag) >= 0.0)) acc[20] += 1.0;
    }
  }
  for (int j = 0; j < NP; ++j) {
    acc[j] = wave_sum(acc[j]);
    if (lane == 0) sh[wv][j] = acc[j];
  }
  __syncthreads();
  if ((int)threadIdx.x < NP) {
    double sum = 0.0;
    for (int w = 0; w < kGateThreads / 64; ++w) sum += sh[w][threadIdx.x];
    // sum-major, [kGateNP][all workgroups]: the decision kernel reads each sum's
    // workgroup values with whole-line loads
    partial[(size_t)threadIdx.x * gridDim.x * gridDim.y + (size_t)b * gridDim.x + blockIdx.x] = sum;
  }
}

// The decision and the projection's means, one workgroup.  partial: kGateNP sums x (nb
// lattices x gbpl workgroups), sum-major (k_gate_partials); ncl cells per lattice.
// With project: mean m[b][k] = (float)(sum over lattice b of r_k / ncl), written to the
// control block ctl (layout of launch_sweep_inj) -- for one lattice from the batch-wide
// sums; for a batch the (lattice, channel) pairs are taken by groups of G threads (a
// power of two, fixed by nb), each thread summing the lattice's workgroup sums w = r,
// r + G, ... in that order, a lane-shuffle tree over the group; without it the means
// stay 0.  The correction passes when it is finite, every
// ||dQ_k||_2 <= gb->corr[k] (||dQ_k||^2 = sum r_k^2 + sum over lattices of
// (ncl m^2 - 2 m sum r_k)), ||divc(X + dQ)||_2 <= (1 + gb->divb_rel) ||divc(X)||_2 +
// gb->divb_abs ||B(X)||_2 and no cell is left unphysical (partial [20]): ctl[0] = 1, else
// ctl[0] = 0 and *fallbacks += 1.  Batch-wide
// sums: thread t takes workgroups t, t + 256, ... in that order, wave_sum per
// wavefront, thread 0 adds the four wavefronts in order.  (A separate launch: deciding
// in the last workgroup of the partials kernel needs a device-scope release fence in
// every workgroup, which on this chip writes back L2; measured at 2D 256^2 and 3D 64^3,
// that one kernel took longer than the two.)
constexpr int kFinalThreads = 256;
__global__ __launch_bounds__(kFinalThreads) void k_gate_final(const double* __restrict__ partial, int nb, int gbpl,
                                                              double ncl, int project,
                                                              const GateBounds* __restrict__ gb,
                                                              int* __restrict__ ctl,
                                                              long long* __restrict__ fallbacks) {
  constexpr int NP = kGateNP, NR = NP + 8;  // the sums, then the projection's terms
  __shared__ double sh[kFinalThreads / 64][NR];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nblk = nb * gbpl;
  double t[NR];
  for (int j = 0; j < NR; ++j) t[j] = 0.0;
#pragma unroll 4
  for (int w = (int)threadIdx.x; w < nblk; w += kFinalThreads)
    for (int j = 0; j < NP; ++j) t[j] += partial[(size_t)j * nblk + w];
  // per-lattice sums of a batch (one lattice: the batch-wide sums serve, below)
  if (project && nb > 1) {
    const int P = 8 * nb;
    int G = 1;
    while (G < 32 && 2 * G * P <= kFinalThreads) G *= 2;
    const int per = kFinalThreads / G, g = (int)threadIdx.x / G, r = (int)threadIdx.x % G;
    for (int p0 = 0; p0 < P; p0 += per) {  // the same trip count in every thread
      const int p = p0 + g;
      double s1 = 0.0;
      if (p < P) {
        const double* q = partial + (size_t)(8 + (p & 7)) * nblk + (size_t)(p >> 3) * gbpl;
#pragma unroll 8
        for (int w = r; w < gbpl; w += G) s1 += q[w];
      }
      for (int off = G / 2; off > 0; off >>= 1) s1 += __shfl_xor(s1, off);
      if (p < P && r == 0) {
        const float m = (float)(s1 / ncl);
        ctl[1 + p] = __float_as_int(m);
        const double md = m, d = ncl * md * md - 2.0 * md * s1;
#pragma unroll
        for (int k = 0; k < 8; ++k)  // constant indices keep t in registers
          if (k == (p & 7)) t[NP + k] += d;
      }
    }
  }
  const bool batch_terms = project && nb > 1;
#pragma unroll
  for (int j = 0; j < NR; ++j)
    if (j < NP || batch_terms) {
      t[j] = wave_sum(t[j]);
      if (lane == 0) sh[wv][j] = t[j];
    }
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int j = 0; j < NR; ++j)
    if (j < NP || batch_terms) {
      t[j] = sh[0][j];
      for (int w = 1; w < kFinalThreads / 64; ++w) t[j] += sh[w][j];
    }
  if (project && nb == 1)
    for (int k = 0; k < 8; ++k) {
      const float m = (float)(t[8 + k] / ncl);
      ctl[1 + k] = __float_as_int(m);
      const double md = m;
      t[NP + k] = ncl * md * md - 2.0 * md * t[8 + k];
    }
  bool ok = t[18] == 0.0 && t[20] == 0.0;
  for (int k = 0; k < 8; ++k) ok = ok && sqrt(fmax(t[k] + t[NP + k], 0.0)) <= gb->corr[k];
  ok = ok && sqrt(t[17]) <= (1.0 + gb->divb_rel) * sqrt(t[16]) + gb->divb_abs * sqrt(t[19]);
  ctl[0] = ok ? 1 : 0;
  if (!ok) *fallbacks += 1;
}

}  // namespace

// Open-lattice corrected stepping: if the gate accepted (ctl[0]), the correction joins the
// network's next input, X += dQ, and its standardised BF16 form is recomputed.
__global__ __launch_bounds__(256) void k_net_accept(float* __restrict__ X, bf16_t* __restrict__ act,
                                                    const float* __restrict__ dq, const int* __restrict__ ctl,
                                                    const float* __restrict__ mean, const float* __restrict__ istd,
                                                    size_t N) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N || !ctl[0]) return;
  unsigned h[8];
  for (int k = 0; k < 8; ++k) {
    const float x = X[(size_t)k * N + c] + dq[(size_t)k * N + c];
    X[(size_t)k * N + c] = x;
    const unsigned u = __float_as_uint((x - mean[k]) * istd[k]);
    h[k] = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // BF16, nearest even
  }
  *reinterpret_cast<uint4*>(act + c * 8) =
      make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
struct vlbm_nn {
  int dim = 2, ntap = 9, nzt = 1;  // 3x3 (dim 2) or 3x3x3 (dim 3) kernels; nzt = ntap / 9
  int cin = 0, width = 0, layers = 0;
  int ci[kMaxLayers] = {}, co[kMaxLayers] = {};
  size_t woff[kMaxLayers] = {}, boff[kMaxLayers] = {};  // offsets into the flat parameter vector
  size_t nparam = 0;
  hipStream_t stream = nullptr;
  float* d_param = nullptr;  // FP32 master
  float* d_grad = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  bf16_t* d_wf[kMaxLayers] = {};  // packed forward B fragments
  bf16_t* d_wb[kMaxLayers] = {};  // packed data-gradient B fragments (layers >= 1)
  float* d_norm = nullptr;        // in_mean[8], in_istd[8], out_mean[8], out_std[8], ones[8], zeros[8], out_istd[8]
  long long t = 0;
  float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  // activation workspace (grown on demand)
  size_t ws_positions = 0;
  bf16_t* d_act[kMaxLayers + 1] = {};  // layer inputs, BF16 NHWC
  float* d_z[kMaxLayers] = {};         // hidden pre-activations FP32 NHWC
  float* d_y = nullptr;                // last layer output FP32 NCHW
  bf16_t* d_dz[2] = {};                // data-gradient ping-pong, BF16 NHWC
  float* d_part_w = nullptr;
  float* d_part_b = nullptr;
  double* d_part_loss = nullptr;
  double* d_loss = nullptr;
  int bw_blocks = 0;
  long long ws_gen = 0;  // incremented whenever the activation workspace is reallocated
  // corrected stepping: buffers kept from call to call (grown on demand), the stream and
  // event the steps run with, and the instantiated graph of a pair of steps together with
  // what it was captured for (context identity and generation, workspace generation,
  // parity at its start, projection on or off)
  struct Corr {
    size_t n = 0;
    int gblk = 0, nbatch = 0;
    float* X = nullptr;
    float* raw[2] = {nullptr, nullptr};  // the network's output, ping-pong
    int* ctl = nullptr;                  // two control blocks of 1 + 8 nbatch words
    long long* fb = nullptr;
    double* gpart = nullptr;
    GateBounds* gb = nullptr;
    GateBounds gb_host{};
    hipStream_t cs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraphExec_t exec = nullptr;
    long long uid = -1, gen = -1, ws_gen = -1;
    int par = -1, project = -1;
  } corr;
  std::string err;
};

namespace {

thread_local std::string g_nn_err;

vlbm_status nfail(vlbm_nn* nn, vlbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (nn)
    nn->err = buf;
  else
    g_nn_err = buf;
  return s;
}

#define NN_HIP(nn, call)                                                                                   \
  do {                                                                                                     \
    hipError_t e_ = (call);                                                                                \
    if (e_ != hipSuccess)                                                                                  \
      return nfail(nn, e_ == hipErrorOutOfMemory ? VLBM_ERR_OOM : VLBM_ERR_HIP, "%s: %s", #call,           \
                   hipGetErrorString(e_));                                                                 \
  } while (0)

size_t packed_elems(int cin, int cout, int nzt) { return (size_t)nzt * ksteps(cin) * ntiles(cout) * 64 * 8; }

// S slices of D-slice lattices (D = 1 for 2D lattices); nzt = 1 (3x3) or 3 (3x3x3)
hipError_t launch_conv(int cin, int cout, int mode, int nzt, const bf16_t* act, const bf16_t* wpack,
                       const float* bias, int S, int D, int H, int W, bf16_t* out_act, float* out_z,
                       const float* zprev, const float* oscale, const float* oshift, hipStream_t s) {
  const dim3 grd(W / TILE, H / TILE, S), blk(kConvThreads);
#define CONV_CASE(CI, CO, M, Z)                                                                          \
  if (cin == CI && cout == CO && mode == M && nzt == Z) {                                               \
    hipLaunchKernelGGL((k_conv<CI, CO, M, Z>), grd, blk, 0, s, act, wpack, bias, D, H, W, out_act, out_z, \
                       zprev, oscale, oshift);                                                         \
    return hipGetLastError();                                                                          \
  }
#define CONV_CASES(Z)             \
  CONV_CASE(8, 32, MODE_HIDDEN, Z)  \
  CONV_CASE(32, 32, MODE_HIDDEN, Z) \
  CONV_CASE(32, 8, MODE_LAST, Z)    \
  CONV_CASE(8, 8, MODE_LAST, Z)     \
  CONV_CASE(8, 32, MODE_BWD, Z)     \
  CONV_CASE(32, 32, MODE_BWD, Z)
  CONV_CASES(1)
  CONV_CASES(3)
#undef CONV_CASES
#undef CONV_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_conv_bw(int cin, int cout, int nzt, const bf16_t* act, const bf16_t* dz, int S, int D, int H,
                          int W, float* part_w, float* part_b, int nblk, hipStream_t s) {
  const dim3 grd(nblk, nzt), blk(kThreads);
  if (cin == 8 && cout == 32)
    hipLaunchKernelGGL((k_conv_bw<8, 32>), grd, blk, 0, s, act, dz, S, D, H, W, part_w, part_b);
  else if (cin == 32 && cout == 32)
    hipLaunchKernelGGL((k_conv_bw<32, 32>), grd, blk, 0, s, act, dz, S, D, H, W, part_w, part_b);
  else if (cin == 32 && cout == 8)
    hipLaunchKernelGGL((k_conv_bw<32, 8>), grd, blk, 0, s, act, dz, S, D, H, W, part_w, part_b);
  else if (cin == 8 && cout == 8)
    hipLaunchKernelGGL((k_conv_bw<8, 8>), grd, blk, 0, s, act, dz, S, D, H, W, part_w, part_b);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

vlbm_status repack(vlbm_nn* nn) {
  for (int l = 0; l < nn->layers; ++l) {
    const size_t nf = packed_elems(nn->ci[l], nn->co[l], nn->nzt);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, nn->stream,
                       nn->d_param + nn->woff[l], nn->ci[l], nn->co[l], 0, nn->ntap, nn->d_wf[l]);
    NN_HIP(nn, hipGetLastError());
    if (l > 0) {
      const size_t nb = packed_elems(nn->co[l], nn->ci[l], nn->nzt);
      hipLaunchKernelGGL(k_pack, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, nn->stream,
                         nn->d_param + nn->woff[l], nn->ci[l], nn->co[l], 1, nn->ntap, nn->d_wb[l]);
      NN_HIP(nn, hipGetLastError());
    }
  }
  return VLBM_OK;
}

// batch lattices of nz x ny x nx (nz = 1 for a 3x3 network)
vlbm_status check_shape(vlbm_nn* nn, int batch, int nx, int ny, int nz) {
  if (batch < 1 || nx < TILE || ny < TILE || nx % TILE || ny % TILE)
    return nfail(nn, VLBM_ERR_ARG, "batch >= 1 and nx, ny positive multiples of %d required (got %d, %d, %d)",
                 TILE, batch, nx, ny);
  if (nn->dim == 2 && nz != 1) return nfail(nn, VLBM_ERR_ARG, "a 3x3 network takes nz = 1 (got %d)", nz);
  if (nz < 1) return nfail(nn, VLBM_ERR_ARG, "nz >= 1 required (got %d)", nz);
  if ((size_t)batch * nz > 65535) return nfail(nn, VLBM_ERR_ARG, "batch * nz must not exceed 65535");
  if ((size_t)batch * nz * nx * ny > ((size_t)1 << 28))
    return nfail(nn, VLBM_ERR_ARG, "batch * nz * ny * nx too large");
  return VLBM_OK;
}

vlbm_status ensure_workspace(vlbm_nn* nn, size_t positions) {
  if (positions <= nn->ws_positions) return VLBM_OK;
  for (int l = 0; l <= nn->layers; ++l)
    if (nn->d_act[l]) (void)hipFree(nn->d_act[l]), nn->d_act[l] = nullptr;
  for (int l = 0; l < nn->layers; ++l)
    if (nn->d_z[l]) (void)hipFree(nn->d_z[l]), nn->d_z[l] = nullptr;
  if (nn->d_y) (void)hipFree(nn->d_y), nn->d_y = nullptr;
  for (int j = 0; j < 2; ++j)
    if (nn->d_dz[j]) (void)hipFree(nn->d_dz[j]), nn->d_dz[j] = nullptr;
  nn->ws_positions = 0;
  ++nn->ws_gen;
  NN_HIP(nn, hipMalloc(&nn->d_act[0], positions * nn->cin * sizeof(bf16_t)));
  for (int l = 0; l < nn->layers; ++l) {
    NN_HIP(nn, hipMalloc(&nn->d_act[l + 1], positions * nn->co[l] * sizeof(bf16_t)));
    NN_HIP(nn, hipMalloc(&nn->d_z[l], positions * nn->co[l] * sizeof(float)));
  }
  NN_HIP(nn, hipMalloc(&nn->d_y, positions * nn->cin * sizeof(float)));
  for (int j = 0; j < 2; ++j) NN_HIP(nn, hipMalloc(&nn->d_dz[j], positions * nn->width * sizeof(bf16_t)));
  nn->ws_positions = positions;
  return VLBM_OK;
}

// forward pass; mode_train keeps the pre-activations.  Writes nn->d_y (NCHW FP32),
// scaled by oscale/oshift.
// X == NULL: the first layer's input is already in nn->d_act[0].
vlbm_status forward(vlbm_nn* nn, const float* X, int B, int nx, int ny, int nz, bool train, const float* oscale,
                    const float* oshift, float* yout, hipStream_t s) {
  const int S = B * nz;  // slices
  const size_t P = (size_t)S * nx * ny;
  vlbm_status st = ensure_workspace(nn, P);
  if (st != VLBM_OK) return st;
  const float* norm = nn->d_norm;
  if (X) {
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, X, S, nn->cin, ny, nx,
                       norm + 0, norm + 8, nn->d_act[0]);
    NN_HIP(nn, hipGetLastError());
  }
  for (int l = 0; l < nn->layers; ++l) {
    const bool last = l == nn->layers - 1;
    NN_HIP(nn, launch_conv(nn->ci[l], nn->co[l], last ? MODE_LAST : MODE_HIDDEN, nn->nzt, nn->d_act[l],
                           nn->d_wf[l], nn->d_param + nn->boff[l], S, nz, ny, nx,
                           last ? nullptr : nn->d_act[l + 1], last ? yout : (train ? nn->d_z[l] : nullptr),
                           nullptr, oscale, oshift, s));
  }
  return VLBM_OK;
}

// The corrected step's persistent state: its graph (drop_graph), and with all = true
// also its buffers, event and stream.
void corr_release(vlbm_nn* nn, bool all) {
  auto& q = nn->corr;
  if (q.exec) (void)hipGraphExecDestroy(q.exec);
  q.exec = nullptr;
  q.uid = -1;
  if (!all) return;
  void* bufs[] = {q.X, q.raw[0], q.raw[1], q.ctl, q.fb, q.gpart, q.gb};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  q.X = q.raw[0] = q.raw[1] = nullptr;
  q.ctl = nullptr;
  q.fb = nullptr;
  q.gpart = nullptr;
  q.gb = nullptr;
  q.n = 0;
  q.gblk = q.nbatch = 0;
  if (q.ev) (void)hipEventDestroy(q.ev);
  if (q.cs) (void)hipStreamDestroy(q.cs);
  q.ev = nullptr;
  q.cs = nullptr;
}

// Buffers for N cells, gblk gate workgroups and nbatch lattices; the stream and event
// on first use.  Growing the buffers drops the graph (it holds their addresses).
hipError_t corr_reserve(vlbm_nn* nn, size_t N, int gblk, int nbatch) {
  auto& q = nn->corr;
  hipError_t e = hipSuccess;
  if (!q.cs) e = hipStreamCreateWithFlags(&q.cs, hipStreamNonBlocking);
  if (e == hipSuccess && !q.ev) e = hipEventCreateWithFlags(&q.ev, hipEventDisableTiming);
  if (e != hipSuccess || (N <= q.n && gblk <= q.gblk && nbatch <= q.nbatch && q.X)) return e;
  hipStream_t cs = q.cs;
  hipEvent_t ev = q.ev;
  q.cs = nullptr;
  q.ev = nullptr;
  corr_release(nn, true);  // keeps the stream and event (taken out above)
  q.cs = cs;
  q.ev = ev;
  e = hipMalloc(&q.X, 8 * N * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&q.raw[0], 8 * N * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&q.raw[1], 8 * N * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&q.ctl, 2 * (1 + 8 * (size_t)nbatch) * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&q.fb, sizeof(long long));
  if (e == hipSuccess) e = hipMalloc(&q.gpart, (size_t)gblk * kGateNP * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&q.gb, sizeof(GateBounds));
  if (e != hipSuccess) {
    corr_release(nn, true);
    return e;
  }
  q.n = N;
  q.gblk = gblk;
  q.nbatch = nbatch;
  return hipSuccess;
}

}  // namespace

extern "C" {

vlbm_status vlbm_nn_create(int32_t dim, int32_t cin, int32_t width, int32_t layers, void* stream,
                           vlbm_nn** out) {
  if (!out) return nfail(nullptr, VLBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if ((dim != 2 && dim != 3) || cin != 8 || width != 32 || layers < 1 || layers > kMaxLayers)
    return nfail(nullptr, VLBM_ERR_ARG, "supported: dim = 2 or 3, cin = 8, width = 32, 1 <= layers <= %d",
                 kMaxLayers);
  vlbm_nn* nn = new (std::nothrow) vlbm_nn();
  if (!nn) return nfail(nullptr, VLBM_ERR_OOM, "host allocation failed");
  nn->dim = dim;
  nn->ntap = dim == 2 ? 9 : 27;
  nn->nzt = nn->ntap / 9;
  nn->cin = cin;
  nn->width = width;
  nn->layers = layers;
  nn->stream = static_cast<hipStream_t>(stream);
  size_t off = 0;
  for (int l = 0; l < layers; ++l) {
    nn->ci[l] = l == 0 ? cin : width;
    nn->co[l] = l == layers - 1 ? cin : width;
    nn->woff[l] = off;
    off += (size_t)nn->co[l] * nn->ci[l] * nn->ntap;
    nn->boff[l] = off;
    off += nn->co[l];
  }
  nn->nparam = off;
  hipError_t e = hipMalloc(&nn->d_param, off * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&nn->d_grad, off * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&nn->d_m, off * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&nn->d_v, off * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&nn->d_norm, 7 * 8 * sizeof(float));
  for (int l = 0; l < layers && e == hipSuccess; ++l) {
    e = hipMalloc(&nn->d_wf[l], packed_elems(nn->ci[l], nn->co[l], nn->nzt) * sizeof(bf16_t));
    if (e == hipSuccess && l > 0)
      e = hipMalloc(&nn->d_wb[l], packed_elems(nn->co[l], nn->ci[l], nn->nzt) * sizeof(bf16_t));
  }
  nn->bw_blocks = 512;
  if (e == hipSuccess)
    e = hipMalloc(&nn->d_part_w, (size_t)nn->bw_blocks * width * nn->ntap * width * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&nn->d_part_b, (size_t)nn->bw_blocks * width * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&nn->d_part_loss, 1024 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&nn->d_loss, sizeof(double));
  if (e != hipSuccess) {
    vlbm_nn_destroy(nn);
    return nfail(nullptr, VLBM_ERR_OOM, "device allocation failed: %s", hipGetErrorString(e));
  }
  std::vector<float> zero(off, 0.0f);
  e = hipMemcpy(nn->d_param, zero.data(), off * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(nn->d_m, zero.data(), off * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(nn->d_v, zero.data(), off * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(nn->d_grad, zero.data(), off * sizeof(float), hipMemcpyHostToDevice);
  float norm[56];
  for (int c = 0; c < 8; ++c) {
    norm[c] = 0.0f;       // in_mean
    norm[8 + c] = 1.0f;   // in_istd
    norm[16 + c] = 0.0f;  // out_mean
    norm[24 + c] = 1.0f;  // out_std
    norm[32 + c] = 1.0f;  // ones
    norm[40 + c] = 0.0f;  // zeros
    norm[48 + c] = 1.0f;  // out_istd
  }
  if (e == hipSuccess) e = hipMemcpy(nn->d_norm, norm, sizeof norm, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    vlbm_nn_destroy(nn);
    return nfail(nullptr, VLBM_ERR_HIP, "initialisation: %s", hipGetErrorString(e));
  }
  if (repack(nn) != VLBM_OK || hipStreamSynchronize(nn->stream) != hipSuccess) {
    const std::string msg = nn->err;
    vlbm_nn_destroy(nn);
    return nfail(nullptr, VLBM_ERR_HIP, "weight packing: %s", msg.c_str());
  }
  *out = nn;
  return VLBM_OK;
}

void vlbm_nn_destroy(vlbm_nn* nn) {
  if (!nn) return;
  float* fl[] = {nn->d_param, nn->d_grad, nn->d_m, nn->d_v, nn->d_norm, nn->d_y, nn->d_part_w, nn->d_part_b};
  for (float* p : fl)
    if (p) (void)hipFree(p);
  for (int l = 0; l < kMaxLayers; ++l) {
    if (nn->d_wf[l]) (void)hipFree(nn->d_wf[l]);
    if (nn->d_wb[l]) (void)hipFree(nn->d_wb[l]);
    if (nn->d_z[l]) (void)hipFree(nn->d_z[l]);
  }
  for (int l = 0; l <= kMaxLayers; ++l)
    if (nn->d_act[l]) (void)hipFree(nn->d_act[l]);
  for (int j = 0; j < 2; ++j)
    if (nn->d_dz[j]) (void)hipFree(nn->d_dz[j]);
  if (nn->d_part_loss) (void)hipFree(nn->d_part_loss);
  if (nn->d_loss) (void)hipFree(nn->d_loss);
  corr_release(nn, true);
  delete nn;
}

const char* vlbm_nn_last_error(const vlbm_nn* nn) { return nn ? nn->err.c_str() : g_nn_err.c_str(); }

vlbm_status vlbm_nn_num_params(const vlbm_nn* nn, size_t* n) {
  if (!nn || !n) return VLBM_ERR_ARG;
  *n = nn->nparam;
  return VLBM_OK;
}

vlbm_status vlbm_nn_set_weights(vlbm_nn* nn, const float* w, size_t n) {
  if (!nn) return VLBM_ERR_ARG;
  if (!w || n != nn->nparam) return nfail(nn, VLBM_ERR_ARG, "need %zu weights", nn->nparam);
  for (size_t j = 0; j < n; ++j)
    if (!std::isfinite(w[j])) return nfail(nn, VLBM_ERR_ARG, "weight %zu not finite", j);
  NN_HIP(nn, hipMemcpyAsync(nn->d_param, w, n * sizeof(float), hipMemcpyHostToDevice, nn->stream));
  NN_HIP(nn, hipMemsetAsync(nn->d_m, 0, n * sizeof(float), nn->stream));
  NN_HIP(nn, hipMemsetAsync(nn->d_v, 0, n * sizeof(float), nn->stream));
  nn->t = 0;
  vlbm_status st = repack(nn);
  if (st != VLBM_OK) return st;
  NN_HIP(nn, hipStreamSynchronize(nn->stream));
  return VLBM_OK;
}

vlbm_status vlbm_nn_get_weights(const vlbm_nn* nn_c, float* w, size_t n) {
  vlbm_nn* nn = const_cast<vlbm_nn*>(nn_c);
  if (!nn) return VLBM_ERR_ARG;
  if (!w || n != nn->nparam) return nfail(nn, VLBM_ERR_ARG, "need %zu weights", nn->nparam);
  NN_HIP(nn, hipMemcpyAsync(w, nn->d_param, n * sizeof(float), hipMemcpyDeviceToHost, nn->stream));
  NN_HIP(nn, hipStreamSynchronize(nn->stream));
  return VLBM_OK;
}

vlbm_status vlbm_nn_set_norm(vlbm_nn* nn, const double* in_mean, const double* in_std, const double* out_mean,
                             const double* out_std) {
  if (!nn) return VLBM_ERR_ARG;
  if (!in_mean || !in_std || !out_mean || !out_std) return nfail(nn, VLBM_ERR_ARG, "NULL normalisation array");
  float norm[56];
  for (int c = 0; c < 8; ++c) {
    if (!(in_std[c] > 0.0) || !(out_std[c] > 0.0) || !std::isfinite(in_mean[c]) || !std::isfinite(out_mean[c]))
      return nfail(nn, VLBM_ERR_ARG, "channel %d: std must be > 0 and means finite", c);
    norm[c] = (float)in_mean[c];
    norm[8 + c] = (float)(1.0 / in_std[c]);
    norm[16 + c] = (float)out_mean[c];
    norm[24 + c] = (float)out_std[c];
    norm[32 + c] = 1.0f;
    norm[40 + c] = 0.0f;
    norm[48 + c] = (float)(1.0 / out_std[c]);
  }
  NN_HIP(nn, hipMemcpyAsync(nn->d_norm, norm, sizeof norm, hipMemcpyHostToDevice, nn->stream));
  NN_HIP(nn, hipStreamSynchronize(nn->stream));
  return VLBM_OK;
}

vlbm_status vlbm_nn_forward(vlbm_nn* nn, const float* X, float* dQ, int32_t batch, int32_t nx, int32_t ny,
                            int32_t nz) {
  if (!nn) return VLBM_ERR_ARG;
  if (!X || !dQ) return nfail(nn, VLBM_ERR_ARG, "NULL array");
  if (reinterpret_cast<uintptr_t>(dQ) % 16) return nfail(nn, VLBM_ERR_ARG, "dQ must be 16-byte aligned");
  vlbm_status st = check_shape(nn, batch, nx, ny, nz);
  if (st != VLBM_OK) return st;
  // dQ = out_mean + out_std * y
  return forward(nn, X, batch, nx, ny, nz, false, nn->d_norm + 24, nn->d_norm + 16, dQ, nn->stream);
}

vlbm_status vlbm_nn_loss_grad(vlbm_nn* nn, const float* X, const float* T, int32_t B, int32_t nx, int32_t ny,
                              int32_t nz, double* loss, float* grad) {
  if (!nn) return VLBM_ERR_ARG;
  if (!X || !T) return nfail(nn, VLBM_ERR_ARG, "NULL array");
  vlbm_status st = check_shape(nn, B, nx, ny, nz);
  if (st != VLBM_OK) return st;
  const int S = B * nz;  // slices
  // forward in standardised units (scale 1, shift 0), output into the workspace
  st = ensure_workspace(nn, (size_t)S * nx * ny);
  if (st != VLBM_OK) return st;
  st = forward(nn, X, B, nx, ny, nz, true, nn->d_norm + 32, nn->d_norm + 40, nn->d_y, nn->stream);
  if (st != VLBM_OK) return st;
  const int L = nn->layers;
  const int lblocks = 1024;
  hipLaunchKernelGGL(k_loss, dim3(lblocks), dim3(kThreads), 0, nn->stream, nn->d_y, T, S, nn->cin, ny, nx,
                     nn->d_norm + 16, nn->d_norm + 48, nn->d_dz[0], nn->d_part_loss);
  NN_HIP(nn, hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, nn->stream, nn->d_part_loss, lblocks, nn->d_loss);
  NN_HIP(nn, hipGetLastError());
  // backward: dZ of layer l lives in d_dz[cur]
  int cur = 0;
  const int ntile = S * (nx / TILE) * (ny / TILE);
  const int nblk = ntile < nn->bw_blocks ? ntile : nn->bw_blocks;
  for (int l = L - 1; l >= 0; --l) {
    NN_HIP(nn, launch_conv_bw(nn->ci[l], nn->co[l], nn->nzt, nn->d_act[l], nn->d_dz[cur], S, nz, ny, nx,
                              nn->d_part_w, nn->d_part_b, nblk, nn->stream));
    const int nred = nn->co[l] * nn->ci[l] * nn->ntap + nn->co[l];
    hipLaunchKernelGGL(k_reduce_grads, dim3((nred + 255) / 256), dim3(256), 0, nn->stream, nn->d_part_w,
                       nn->d_part_b, nblk, nn->ci[l], nn->co[l], nn->ntap, nn->d_grad + nn->woff[l],
                       nn->d_grad + nn->boff[l]);
    NN_HIP(nn, hipGetLastError());
    if (l > 0) {
      // dA_{l-1} = conv(dZ_l, mirrored W_l); dZ_{l-1} = dA_{l-1} * GELU'(z_{l-1})
      NN_HIP(nn, launch_conv(nn->co[l], nn->ci[l], MODE_BWD, nn->nzt, nn->d_dz[cur], nn->d_wb[l], nullptr, S, nz,
                             ny, nx, nn->d_dz[1 - cur], nullptr, nn->d_z[l - 1], nullptr, nullptr, nn->stream));
      cur = 1 - cur;
    }
  }
  if (loss) NN_HIP(nn, hipMemcpyAsync(loss, nn->d_loss, sizeof(double), hipMemcpyDeviceToHost, nn->stream));
  if (grad)
    NN_HIP(nn, hipMemcpyAsync(grad, nn->d_grad, nn->nparam * sizeof(float), hipMemcpyDeviceToHost, nn->stream));
  if (loss || grad) NN_HIP(nn, hipStreamSynchronize(nn->stream));
  return VLBM_OK;
}

vlbm_status vlbm_nn_adam_config(vlbm_nn* nn, float beta1, float beta2, float eps) {
  if (!nn) return VLBM_ERR_ARG;
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return nfail(nn, VLBM_ERR_ARG, "betas in [0, 1), eps > 0 required");
  nn->b1 = beta1;
  nn->b2 = beta2;
  nn->eps = eps;
  return VLBM_OK;
}

vlbm_status vlbm_nn_adam_step(vlbm_nn* nn, float lr) {
  if (!nn) return VLBM_ERR_ARG;
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return nfail(nn, VLBM_ERR_ARG, "lr must be >= 0");
  nn->t += 1;
  const float c1 = (float)(1.0 - std::pow((double)nn->b1, (double)nn->t));
  const float c2 = (float)(1.0 - std::pow((double)nn->b2, (double)nn->t));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((nn->nparam + 255) / 256)), dim3(256), 0, nn->stream, nn->d_param,
                     nn->d_grad, nn->d_m, nn->d_v, nn->nparam, lr, nn->b1, nn->b2, nn->eps, c1, c2);
  NN_HIP(nn, hipGetLastError());
  return repack(nn);
}

vlbm_status vlbm_nn_train_step(vlbm_nn* nn, const float* X, const float* T, int32_t batch, int32_t nx, int32_t ny,
                               int32_t nz, float lr, double* loss) {
  vlbm_status st = vlbm_nn_loss_grad(nn, X, T, batch, nx, ny, nz, loss, nullptr);
  if (st != VLBM_OK) return st;
  return vlbm_nn_adam_step(nn, lr);
}

vlbm_status vlbm_restrict(const float* Qf, int32_t K, int32_t nx, int32_t ny, int32_t nz, int32_t r, int32_t rz,
                          const float* minus, float* Qc, void* stream) {
  if (!Qf || !Qc || K < 1 || r < 1 || rz < 1 || nx < 1 || ny < 1 || nz < 1) return VLBM_ERR_ARG;
  if (nx % r || ny % r || nz % rz) return VLBM_ERR_ARG;
  const size_t n = (size_t)K * (nx / r) * (ny / r) * (nz / rz);
  hipLaunchKernelGGL(k_restrict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     Qf, K, nx, ny, nz, r, rz, minus, Qc);
  return hipGetLastError() == hipSuccess ? VLBM_OK : VLBM_ERR_HIP;
}

namespace {
// a periodic ideal-MHD context (2D batch or 3D lattice, any storage form)
bool correctable(const vlbm_ctx* c) {
  return c->K == 8 && c->p.model == VLBM_IDEAL && !c->has_faces && c->p.body == 0 && c->p.source == 0;
}
// Contexts a correction can be added to: the 8-variable ideal model with the direct
// source, any faces, no body or the homogenized one (every cell is fluid there).
bool injectable(const vlbm_ctx* c) {
  return c->K == 8 && c->p.model == VLBM_IDEAL && c->p.body != 1 && c->p.source == 0;
}

// The launchers below index by storage * 2 + (dimension - 2): the storage codes of
// vlbm.h and of the kernels agree.
void launch_inject(const vlbm_ctx* c, int par, const float* dq, const int* ctl, hipStream_t s) {
  const dim3 cgrid((unsigned)(((size_t)c->N + 255) / 256)), cblk(256);
  switch (c->p.storage * 2 + (c->D - 2)) {
#define INJ_CASE(ST, D)                                                                                   \
  case ST * 2 + (D - 2):                                                                                  \
    hipLaunchKernelGGL((k_inject<ST, D>), cgrid, cblk, 0, s, c->g, c->cd, par, dq, ctl, c->ph.wi);        \
    break;
    INJ_CASE(vlbm::ST_F64, 2) INJ_CASE(vlbm::ST_F64, 3) INJ_CASE(vlbm::ST_F32, 2) INJ_CASE(vlbm::ST_F32, 3)
    INJ_CASE(vlbm::ST_F16, 2) INJ_CASE(vlbm::ST_F16, 3) INJ_CASE(vlbm::ST_BF16, 2) INJ_CASE(vlbm::ST_BF16, 3)
#undef INJ_CASE
    default: break;
  }
}

}  // namespace

vlbm_status vlbm_inject(vlbm_ctx* c, const float* dQ) {
  if (!c || !dQ) return VLBM_ERR_ARG;
  if (!c->initialized) return VLBM_ERR_STATE;
  if (!injectable(c)) return VLBM_ERR_ARG;
  launch_inject(c, (int)(c->step & 1), dQ, nullptr, c->stream);
  return hipGetLastError() == hipSuccess ? VLBM_OK : VLBM_ERR_HIP;
}

vlbm_status vlbm_step_corrected(vlbm_ctx* c, vlbm_nn* nn, int32_t n, const double* bound_corr,
                                double bound_divb_rel, double bound_divb_abs, int32_t project_totals,
                                int64_t* n_fallback) {
  if (!c || !nn) return VLBM_ERR_ARG;
  if (!c->initialized) return VLBM_ERR_STATE;
  if (n < 0 || !bound_corr) return nfail(nn, VLBM_ERR_ARG, "n >= 0 and bound_corr required");
  // periodic lattices: the fused path (the sweep injects); a 3D lattice with faces or
  // the homogenized body: the open path (a separate injection and moments pass)
  const bool open = !correctable(c);
  if ((open && (!injectable(c) || c->D != 3)) || c->N > (1LL << 28) || c->p.collision != 0)
    return nfail(nn, VLBM_ERR_ARG,
                 "corrected stepping needs an ideal-MHD BGK context: periodic (2D or 3D) without a body, or "
                 "3D with static faces and/or the homogenized body");
  if (open && project_totals)
    return nfail(nn, VLBM_ERR_ARG,
                 "the projection onto zero lattice totals needs a periodic lattice without a body: with faces or a "
                 "body the totals change (pass project_totals = 0)");
  if (nn->dim != c->D)
    return nfail(nn, VLBM_ERR_ARG, "a %dD context needs a network of dim %d (got %d)", c->D, c->D, nn->dim);
  // 2D: the context's nz is a batch of lattices; 3D: one lattice of nz slices
  const int nbatch = c->D == 2 ? c->p.nz : 1, nzl = c->D == 2 ? 1 : c->p.nz;
  vlbm_status st = check_shape(nn, nbatch, c->p.nx, c->p.ny, nzl);
  if (st != VLBM_OK) return st;
  GateBounds gb;
  for (int k = 0; k < 8; ++k) {
    if (!(bound_corr[k] >= 0.0)) return nfail(nn, VLBM_ERR_ARG, "bound_corr[%d] must be >= 0", k);
    gb.corr[k] = bound_corr[k];
  }
  if (!(bound_divb_rel >= 0.0) || !(bound_divb_abs >= 0.0))
    return nfail(nn, VLBM_ERR_ARG, "div B bounds must be >= 0");
  gb.divb_rel = bound_divb_rel;
  gb.divb_abs = bound_divb_abs;
  // positivity of the corrected state, where it is X + raw (no projection)
  const double gm1_gate = project_totals ? 0.0 : c->ph.gm1;
  const size_t N = (size_t)c->N;
  hipStream_t s = c->stream;
  const size_t ncl = N / (size_t)nbatch;  // cells per lattice (the projection's unit)
  // gate workgroups per lattice, about 1024 in all
  const int gbpl = (int)std::max<size_t>(
      1, std::min<size_t>((ncl + kGateThreads - 1) / kGateThreads, std::max<size_t>(1, 1024 / (size_t)nbatch)));
  const int gblk = gbpl * nbatch;
  // the network's workspace first: its (re)allocation must not happen under capture
  st = ensure_workspace(nn, N);
  if (st != VLBM_OK) return st;
  hipError_t e = corr_reserve(nn, N, gblk, nbatch);
  if (e != hipSuccess)
    return nfail(nn, e == hipErrorOutOfMemory ? VLBM_ERR_OOM : VLBM_ERR_HIP, "corrected step: %s",
                 hipGetErrorString(e));
  auto& q = nn->corr;
  // the periodic path runs on the handle's own stream, ordered after s; the open path
  // on the context's stream, where its plain step runs
  hipStream_t cs = open ? s : q.cs;
  q.gb_host = gb;  // lives in the handle: the copy below may read it after returning
  if (!open) {
    e = hipEventRecord(q.ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, q.ev, 0);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(q.gb, &q.gb_host, sizeof(GateBounds), hipMemcpyHostToDevice, cs);
  // both control blocks cleared: nothing pending, means 0
  int* ctl[2] = {q.ctl, q.ctl + 1 + 8 * nbatch};
  if (e == hipSuccess) e = hipMemsetAsync(q.ctl, 0, 2 * (1 + 8 * (size_t)nbatch) * sizeof(int), cs);
  if (e == hipSuccess) e = hipMemsetAsync(q.fb, 0, sizeof(long long), cs);
  if (e == hipSuccess && open) {
    // Open lattice (static faces, homogenized body), eager: the body's box changes every
    // step.  X holds the network's input, the moments of the state at a step's start.
    // Per step: the network on X; the plain step (faces, sweep, body); the moments X' of
    // its result; the gate on X' + dQ, the state the correction would make (its norms,
    // div B and positivity); an accepted correction goes into the populations at once,
    // and X := X' + dQ (with its standardised form) is the next step's input.
    const int gb3 = gbpl;
    const vlbm::MomentsOut mo{q.X, nn->d_act[0], nn->d_norm + 0, nn->d_norm + 8};
    const size_t Nc = (size_t)c->N;
    if (n > 0) e = vlbm::launch_net_input(c->L, c->g, c->cd, (int)(c->step & 1), mo);
    for (int32_t j = 0; j < n && st == VLBM_OK && e == hipSuccess; ++j) {
      st = forward(nn, nullptr, 1, c->p.nx, c->p.ny, c->p.nz, false, nn->d_norm + 24, nn->d_norm + 16, q.raw[0],
                   cs);
      if (st != VLBM_OK) break;
      st = vlbm_step_one(c);
      if (st != VLBM_OK) {
        (void)hipStreamSynchronize(cs);
        return nfail(nn, st, "corrected step: %s", c->err.c_str());
      }
      e = vlbm::launch_net_input(c->L, c->g, c->cd, (int)(c->step & 1), mo);
      if (e != hipSuccess) break;
      hipLaunchKernelGGL(k_gate_partials<3>, dim3((unsigned)gb3, 1u), dim3(kGateThreads), 0, cs, q.X, q.raw[0],
                         c->p.nx, c->p.ny, c->p.nz, gm1_gate, q.gpart);
      hipLaunchKernelGGL(k_gate_final, dim3(1), dim3(kFinalThreads), 0, cs, q.gpart, 1, gb3, (double)ncl, 0, q.gb,
                         ctl[0], q.fb);
      launch_inject(c, (int)(c->step & 1), q.raw[0], ctl[0], cs);
      hipLaunchKernelGGL(k_net_accept, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, cs, q.X, nn->d_act[0],
                         q.raw[0], ctl[0], nn->d_norm + 0, nn->d_norm + 8, Nc);
      e = hipGetLastError();
    }
    long long nfb = 0;
    const hipError_t ce = hipMemcpyAsync(&nfb, q.fb, sizeof nfb, hipMemcpyDeviceToHost, cs);
    const hipError_t se = hipStreamSynchronize(cs);
    if (e == hipSuccess) e = ce != hipSuccess ? ce : se;
    if (st != VLBM_OK) return st;
    if (e != hipSuccess)
      return nfail(nn, e == hipErrorOutOfMemory ? VLBM_ERR_OOM : VLBM_ERR_HIP, "corrected step: %s",
                   hipGetErrorString(e));
    if (n_fallback) *n_fallback = nfb;
    return VLBM_OK;
  }
  vlbm::Launch L = c->L;
  L.stream = cs;
  int cur = 0;  // raw[cur], ctl[cur]: the pending correction (not yet in the populations)
  // one corrected step: the sweep injecting the pending correction (it also writes the
  // moments it collides with), the network on those moments, the gate of its
  // correction and its projection's means (pending until the next sweep).  Kernels
  // only, so that it can be captured.
  auto step = [&]() -> vlbm_status {
    const int par = (int)(c->step & 1);
    // the sweep injects the pending correction and writes the moments it collides with
    // (this step's network input, X and its standardised BF16 form); the network's
    // correction for them is injected by the next sweep
    const vlbm::MomentsOut mo{q.X, nn->d_act[0], nn->d_norm + 0, nn->d_norm + 8};
    e = vlbm::launch_sweep_inj(L, c->g, c->ph, c->cd, par, q.raw[cur], ctl[cur], mo);
    if (e != hipSuccess) return VLBM_ERR_HIP;
    vlbm_status fs = forward(nn, nullptr, nbatch, c->p.nx, c->p.ny, nzl, false, nn->d_norm + 24, nn->d_norm + 16,
                             q.raw[1 - cur], cs);
    if (fs != VLBM_OK) return fs;
    // gate statistics, then the decision and (when asked for) the projection's means
    const dim3 ggrid((unsigned)gbpl, (unsigned)nbatch);
    if (c->D == 2)
      hipLaunchKernelGGL(k_gate_partials<2>, ggrid, dim3(kGateThreads), 0, cs, q.X, q.raw[1 - cur], c->p.nx,
                         c->p.ny, c->p.nz, gm1_gate, q.gpart);
    else
      hipLaunchKernelGGL(k_gate_partials<3>, ggrid, dim3(kGateThreads), 0, cs, q.X, q.raw[1 - cur], c->p.nx,
                         c->p.ny, c->p.nz, gm1_gate, q.gpart);
    hipLaunchKernelGGL(k_gate_final, dim3(1), dim3(kFinalThreads), 0, cs, q.gpart, nbatch, gbpl, (double)ncl,
                       project_totals ? 1 : 0, q.gb, ctl[1 - cur], q.fb);
    e = hipGetLastError();
    if (e != hipSuccess) return VLBM_ERR_HIP;
    ++c->step;
    cur = 1 - cur;
    return VLBM_OK;
  };
  int32_t done = 0;
  // two steps eagerly, then pairs of steps replayed from a graph: a pair returns parity
  // and ping-pong slot to where they started, so one captured pair serves every later
  // pair, in this call and in later calls on the same context while nothing it took by
  // value or by address has changed
  for (; done < n && done < 2 && e == hipSuccess; ++done) {
    st = step();
    if (st != VLBM_OK) break;
  }
  const int par0 = (int)(c->step & 1);
  const bool cached = q.exec && q.uid == c->uid && q.gen == c->gen && q.ws_gen == nn->ws_gen &&
                      q.par == par0 && q.project == (project_totals ? 1 : 0);
  if (st == VLBM_OK && e == hipSuccess && !cached && n - done >= 4) {
    corr_release(nn, false);
    const long long step0 = c->step;
    const int cur0 = cur;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const vlbm_status s1 = step();
      const vlbm_status s2 = s1 == VLBM_OK ? step() : s1;
      const hipError_t ce = hipStreamEndCapture(cs, &graph);
      c->step = step0;  // the captured steps have not run
      cur = cur0;
      if (s2 == VLBM_OK && ce == hipSuccess && graph &&
          hipGraphInstantiate(&q.exec, graph, nullptr, nullptr, 0) != hipSuccess)
        q.exec = nullptr;
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();  // a failed capture leaves the eager path below
      e = hipSuccess;
      if (q.exec) {
        q.uid = c->uid;
        q.gen = c->gen;
        q.ws_gen = nn->ws_gen;
        q.par = par0;
        q.project = project_totals ? 1 : 0;
      }
    }
  }
  const bool use_graph = q.exec && q.uid == c->uid && q.gen == c->gen && q.ws_gen == nn->ws_gen &&
                         q.par == par0 && q.project == (project_totals ? 1 : 0);
  if (st == VLBM_OK && e == hipSuccess && use_graph)
    for (; n - done >= 2; done += 2) {
      e = hipGraphLaunch(q.exec, cs);
      if (e != hipSuccess) break;
      c->step += 2;
    }
  for (; st == VLBM_OK && done < n && e == hipSuccess; ++done) st = step();
  if (st == VLBM_OK && e == hipSuccess && n > 0) {
    // the last accepted correction goes into the populations
    launch_inject(c, (int)(c->step & 1), q.raw[cur], ctl[cur], cs);
    e = hipGetLastError();
  }
  long long nfb = 0;
  const hipError_t ce = hipMemcpyAsync(&nfb, q.fb, sizeof nfb, hipMemcpyDeviceToHost, cs);
  const hipError_t se = hipStreamSynchronize(cs);  // also when a step failed: nothing stays in flight
  if (e == hipSuccess) e = ce != hipSuccess ? ce : se;
  if (st != VLBM_OK) return st;
  if (e != hipSuccess)
    return nfail(nn, e == hipErrorOutOfMemory ? VLBM_ERR_OOM : VLBM_ERR_HIP, "corrected step: %s", hipGetErrorString(e));
  if (n_fallback) *n_fallback = nfb;
  return VLBM_OK;
}

}  // extern "C"

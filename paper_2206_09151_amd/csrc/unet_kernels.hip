// gfx950 kernels of the artefact-correction network (a small 3D U-Net; not part of the
// paper's method): 3x3x3 / 1x1x1 convolutions with zero padding, bias and ReLU, their
// input and weight gradients, 2x average pooling, 2x nearest upsampling, the MSE loss
// and Adam.  Activations and gradients are FP32 [C][n][n][n]; weights are the BF16
// rounding (nearest even) of the FP32 master parameters; every sum is FP32 (the loss in
// FP64) in a fixed order, so a training step is bitwise reproducible.
//
// Convolutions work on 8x8x8 output tiles (256 threads, two voxels each, z and z+4).  A
// chunk of input channels is staged into LDS with its one-voxel halo (zero outside the
// volume) and the chunk's weights are staged as FP32 in [ci][tap][co] order, so a
// thread's 16 output channels of one (ci, tap) are four 16-byte LDS reads shared by the
// whole workgroup.  The input gradient is the same correlation with the kernel flipped
// and input / output channels exchanged; the ReLU mask of the layer's output is applied
// to the incoming gradient while it is staged.  The weight gradient reduces over all
// voxels: workgroups own (16 co x 16 ci) channel pairs and a chunk of 8x8x4 tiles, write
// one partial per chunk, and a second kernel sums the partials in chunk order.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "unet_internal.hpp"

namespace unet {

constexpr int TS = 8;    // output tile edge
constexpr int CIC = 4;   // input channels per staged chunk
constexpr int COB = 16;  // output channels per workgroup

__device__ __forceinline__ float bf(const __hip_bfloat16 v) { return __bfloat162float(v); }

// channel c of a two-source input (channels [0, c0) from x0, the rest from x1)
__device__ __forceinline__ const float* chan(const float* x0, int c0, const float* x1, int c, size_t vol) {
  return c < c0 ? x0 + size_t(c) * vol : x1 + size_t(c - c0) * vol;
}

// ------------------------------------------------------------------ forward
// out[co] = act(b[co] + sum_ci sum_t w[co][ci][t] in[ci][r + t - h]) (+ res) for co in
// [co0, co0 + cob), cob = min(COB, cout).
template <int KS>
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ x0, int c0,
                                                  const float* __restrict__ x1, int cin,
                                                  const __hip_bfloat16* __restrict__ w,
                                                  const float* __restrict__ b, float* __restrict__ out, int cout,
                                                  int n, int relu, const float* __restrict__ res) {
  constexpr int H = KS / 2, TH = TS + 2 * H, K3 = KS * KS * KS;
  __shared__ float xs[CIC][TH][TH][TH];
  __shared__ float4 ws[CIC][K3][COB / 4];
  const int t = threadIdx.x;
  const int lx = t % TS, ly = (t / TS) % TS, lz = t / (TS * TS);
  const int nt = (n + TS - 1) / TS;
  const int tile = blockIdx.x;
  const int x0t = (tile % nt) * TS, y0t = ((tile / nt) % nt) * TS, z0t = (tile / (nt * nt)) * TS;
  const int co0 = blockIdx.y * COB;
  const int cob = min(COB, cout - co0);
  const size_t vol = size_t(n) * n * n;
  float acc0[COB], acc1[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc0[c] = acc1[c] = 0.0f;
  for (int ci0 = 0; ci0 < cin; ci0 += CIC) {
    __syncthreads();
    for (int idx = t; idx < CIC * TH * TH * TH; idx += 256) {
      const int c = idx / (TH * TH * TH), r = idx % (TH * TH * TH);
      const int hz = r / (TH * TH), hy = (r / TH) % TH, hx = r % TH;
      const int gz = z0t + hz - H, gy = y0t + hy - H, gx = x0t + hx - H;
      float v = 0.0f;
      if (ci0 + c < cin && unsigned(gz) < unsigned(n) && unsigned(gy) < unsigned(n) && unsigned(gx) < unsigned(n))
        v = chan(x0, c0, x1, ci0 + c, vol)[(size_t(gz) * n + gy) * n + gx];
      xs[c][hz][hy][hx] = v;
    }
    for (int idx = t; idx < CIC * K3 * COB; idx += 256) {
      const int c = idx / (K3 * COB), tp = (idx / COB) % K3, co = idx % COB;
      float v = 0.0f;
      if (ci0 + c < cin && co < cob) v = bf(w[(size_t(co0 + co) * cin + ci0 + c) * K3 + tp]);
      reinterpret_cast<float*>(&ws[c][tp][0])[co] = v;
    }
    __syncthreads();
    const int cn = min(CIC, cin - ci0);
    for (int c = 0; c < cn; ++c) {
#pragma unroll
      for (int tp = 0; tp < K3; ++tp) {
        const int dz = tp / (KS * KS), dy = (tp / KS) % KS, dx = tp % KS;
        const float v0 = xs[c][lz + dz][ly + dy][lx + dx];
        const float v1 = xs[c][lz + 4 + dz][ly + dy][lx + dx];
#pragma unroll
        for (int q = 0; q < COB / 4; ++q) {
          const float4 wv = ws[c][tp][q];
          acc0[4 * q + 0] += wv.x * v0;
          acc0[4 * q + 1] += wv.y * v0;
          acc0[4 * q + 2] += wv.z * v0;
          acc0[4 * q + 3] += wv.w * v0;
          acc1[4 * q + 0] += wv.x * v1;
          acc1[4 * q + 1] += wv.y * v1;
          acc1[4 * q + 2] += wv.z * v1;
          acc1[4 * q + 3] += wv.w * v1;
        }
      }
    }
  }
  const int gx = x0t + lx, gy = y0t + ly;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int gz = z0t + lz + 4 * half;
    if (gx >= n || gy >= n || gz >= n) continue;
    const size_t v = (size_t(gz) * n + gy) * n + gx;
#pragma unroll
    for (int c = 0; c < COB; ++c) {
      if (c < cob) {
        float o = (half ? acc1[c] : acc0[c]) + b[co0 + c];
        if (relu) o = fmaxf(o, 0.0f);
        if (res) o += res[v];
        out[size_t(co0 + c) * vol + v] = o;
      }
    }
  }
}

// ------------------------------------------------------------------ input gradient
// gx[ci] = sum_co sum_t w[co][ci][t] gm[co][r + h - t], gm = g * (y > 0) (no mask when
// y is null); gx channels [0, c0) go to gx0, the rest to gx1.
template <int KS>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const float* __restrict__ g, const float* __restrict__ y,
                                                       int cout, const __hip_bfloat16* __restrict__ w,
                                                       float* __restrict__ gx0, int c0, float* __restrict__ gx1,
                                                       int cin, int n) {
  constexpr int H = KS / 2, TH = TS + 2 * H, K3 = KS * KS * KS;
  __shared__ float gs[CIC][TH][TH][TH];
  __shared__ float4 ws[CIC][K3][COB / 4];
  const int t = threadIdx.x;
  const int lx = t % TS, ly = (t / TS) % TS, lz = t / (TS * TS);
  const int nt = (n + TS - 1) / TS;
  const int tile = blockIdx.x;
  const int x0t = (tile % nt) * TS, y0t = ((tile / nt) % nt) * TS, z0t = (tile / (nt * nt)) * TS;
  const int ci0 = blockIdx.y * COB;                    // this workgroup's input-gradient channels
  const int cib = min(COB, cin - ci0);
  const size_t vol = size_t(n) * n * n;
  float acc0[COB], acc1[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc0[c] = acc1[c] = 0.0f;
  for (int o0 = 0; o0 < cout; o0 += CIC) {
    __syncthreads();
    for (int idx = t; idx < CIC * TH * TH * TH; idx += 256) {
      const int c = idx / (TH * TH * TH), r = idx % (TH * TH * TH);
      const int hz = r / (TH * TH), hy = (r / TH) % TH, hx = r % TH;
      const int gz = z0t + hz - H, gy = y0t + hy - H, gxx = x0t + hx - H;
      float v = 0.0f;
      if (o0 + c < cout && unsigned(gz) < unsigned(n) && unsigned(gy) < unsigned(n) && unsigned(gxx) < unsigned(n)) {
        const size_t a = size_t(o0 + c) * vol + (size_t(gz) * n + gy) * n + gxx;
        v = g[a];
        if (y && !(y[a] > 0.0f)) v = 0.0f;
      }
      gs[c][hz][hy][hx] = v;
    }
    // ws[o][t'][ci] = w[o][ci][K3 - 1 - t'] (flipped taps, input channels along the vector)
    for (int idx = t; idx < CIC * K3 * COB; idx += 256) {
      const int c = idx / (K3 * COB), tp = (idx / COB) % K3, ci = idx % COB;
      float v = 0.0f;
      if (o0 + c < cout && ci < cib) v = bf(w[(size_t(o0 + c) * cin + ci0 + ci) * K3 + (K3 - 1 - tp)]);
      reinterpret_cast<float*>(&ws[c][tp][0])[ci] = v;
    }
    __syncthreads();
    const int cn = min(CIC, cout - o0);
    for (int c = 0; c < cn; ++c) {
#pragma unroll
      for (int tp = 0; tp < K3; ++tp) {
        const int dz = tp / (KS * KS), dy = (tp / KS) % KS, dx = tp % KS;
        const float v0 = gs[c][lz + dz][ly + dy][lx + dx];
        const float v1 = gs[c][lz + 4 + dz][ly + dy][lx + dx];
#pragma unroll
        for (int q = 0; q < COB / 4; ++q) {
          const float4 wv = ws[c][tp][q];
          acc0[4 * q + 0] += wv.x * v0;
          acc0[4 * q + 1] += wv.y * v0;
          acc0[4 * q + 2] += wv.z * v0;
          acc0[4 * q + 3] += wv.w * v0;
          acc1[4 * q + 0] += wv.x * v1;
          acc1[4 * q + 1] += wv.y * v1;
          acc1[4 * q + 2] += wv.z * v1;
          acc1[4 * q + 3] += wv.w * v1;
        }
      }
    }
  }
  const int gx = x0t + lx, gy = y0t + ly;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int gz = z0t + lz + 4 * half;
    if (gx >= n || gy >= n || gz >= n) continue;
    const size_t v = (size_t(gz) * n + gy) * n + gx;
#pragma unroll
    for (int c = 0; c < COB; ++c) {
      if (c < cib) {
        const int ci = ci0 + c;
        float* dst = ci < c0 ? gx0 + size_t(ci) * vol : gx1 + size_t(ci - c0) * vol;
        dst[v] = half ? acc1[c] : acc0[c];
      }
    }
  }
}

// ------------------------------------------------------------------ weight gradient
// Partial sums over a chunk of 8x8x4 tiles:
//   pw[chunk][co][ci][t] = sum_v gm[co][v] in[ci][v + t - h],  pb[chunk][co] = sum_v gm[co][v]
// Workgroup = (chunk, 16x16 channel-pair block); thread = (co, ci) pair, K3 accumulators.
constexpr int WTZ = 4;   // tile depth of the weight-gradient kernel

template <int KS>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float* __restrict__ x0, int c0,
                                                    const float* __restrict__ x1, int cin,
                                                    const float* __restrict__ g, const float* __restrict__ y,
                                                    int cout, int n, int tiles_per_chunk,
                                                    float* __restrict__ pw, float* __restrict__ pb) {
  constexpr int H = KS / 2, TX = TS + 2 * H, TZ = WTZ + 2 * H, K3 = KS * KS * KS;
  constexpr int TV = TS * TS * WTZ;
  constexpr int CP = TZ * TX * TX + 1;   // odd channel pitch: the 16 channels of a wave hit distinct banks
  __shared__ float xs[16 * CP];
  __shared__ float gsm[16][TV];
  const int t = threadIdx.x;
  const int co_l = t / 16, ci_l = t % 16;
  const int nco = (cout + 15) / 16;
  const int co0 = (blockIdx.y % nco) * 16, ci0 = (blockIdx.y / nco) * 16;
  const int co = co0 + co_l, ci = ci0 + ci_l;
  const int ntx = (n + TS - 1) / TS, ntz = (n + WTZ - 1) / WTZ;
  const int ntiles = ntx * ntx * ntz;
  const size_t vol = size_t(n) * n * n;
  float acc[K3];
#pragma unroll
  for (int k = 0; k < K3; ++k) acc[k] = 0.0f;
  float accb = 0.0f;
  const int tile_end = min(ntiles, (int(blockIdx.x) + 1) * tiles_per_chunk);
  for (int tile = blockIdx.x * tiles_per_chunk; tile < tile_end; ++tile) {
    const int x0t = (tile % ntx) * TS, y0t = ((tile / ntx) % ntx) * TS, z0t = (tile / (ntx * ntx)) * WTZ;
    __syncthreads();
    for (int idx = t; idx < 16 * TZ * TX * TX; idx += 256) {
      const int c = idx / (TZ * TX * TX), r = idx % (TZ * TX * TX);
      const int hz = r / (TX * TX), hy = (r / TX) % TX, hx = r % TX;
      const int gz = z0t + hz - H, gy = y0t + hy - H, gx = x0t + hx - H;
      float v = 0.0f;
      if (ci0 + c < cin && unsigned(gz) < unsigned(n) && unsigned(gy) < unsigned(n) && unsigned(gx) < unsigned(n))
        v = chan(x0, c0, x1, ci0 + c, vol)[(size_t(gz) * n + gy) * n + gx];
      xs[c * CP + (hz * TX + hy) * TX + hx] = v;
    }
    for (int idx = t; idx < 16 * TV; idx += 256) {
      const int c = idx / TV, r = idx % TV;
      const int lz = r / (TS * TS), ly = (r / TS) % TS, lx = r % TS;
      const int gz = z0t + lz, gy = y0t + ly, gx = x0t + lx;
      float v = 0.0f;
      if (co0 + c < cout && gz < n && gy < n && gx < n) {
        const size_t a = size_t(co0 + c) * vol + (size_t(gz) * n + gy) * n + gx;
        v = g[a];
        if (y && !(y[a] > 0.0f)) v = 0.0f;
      }
      gsm[c][r] = v;
    }
    __syncthreads();
    for (int r = 0; r < TV; ++r) {
      const int lz = r / (TS * TS), ly = (r / TS) % TS, lx = r % TS;
      const float gv = gsm[co_l][r];
      accb += gv;
#pragma unroll
      for (int k = 0; k < K3; ++k) {
        const int dz = k / (KS * KS), dy = (k / KS) % KS, dx = k % KS;
        acc[k] += gv * xs[ci_l * CP + ((lz + dz) * TX + ly + dy) * TX + lx + dx];
      }
    }
  }
  if (co < cout && ci < cin) {
    float* dst = pw + (size_t(blockIdx.x) * cout * cin + size_t(co) * cin + ci) * K3;
#pragma unroll
    for (int k = 0; k < K3; ++k) dst[k] = acc[k];
  }
  if (ci0 == 0 && ci_l == 0 && co < cout) pb[size_t(blockIdx.x) * cout + co] = accb;
}

// ------------------------------------------------------------------ matrix-core convolutions
// The 3x3x3 convolutions run on the matrix cores as implicit GEMMs with
// v_mfma_f32_16x16x16_bf16 (a 16 x 16 x 16 product per instruction; lane l holds
// A[l%16][4(l/16)..+3], B[4(l/16)..+3][l%16] and D[4(l/16)+i][l%16]).  Weights are BF16
// values already; an FP32 activation or gradient v is split into BF16 hi + lo
// (v = hi + lo + e, |e| <= 2^-18 |v|) and both halves are multiplied, so the products keep
// FP32-level accuracy: two instructions per product in the forward and input-gradient
// passes, three (hi*hi + hi*lo + lo*hi) in the weight gradient, whose operands are both
// FP32.
//
// LDS layouts follow one rule: a 64-bit LDS read is served sixteen lanes at a time, so the
// sixteen lanes of a group (the M or N index of the product) read 128 contiguous bytes;
// staging writes from lanes that walk along x use strides of 2 (mod 32) dwords.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf_bits(float v) {
  const __hip_bfloat16 h = __float2bfloat16(v);
  return *reinterpret_cast<const unsigned short*>(&h);
}
__device__ __forceinline__ float bits_bf(unsigned short u) { return __uint_as_float(unsigned(u) << 16); }

__device__ __forceinline__ void split_bf16(float v, unsigned& hi, unsigned& lo) {
  hi = bf_bits(v);
  lo = bf_bits(v - bits_bf(static_cast<unsigned short>(hi)));
}

// hi / lo halves of four values, packed as four BF16 each
__device__ __forceinline__ void split4(const float* v, uint2& hi, uint2& lo) {
  unsigned h[4], l[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) split_bf16(v[j], h[j], l[j]);
  hi = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
  lo = make_uint2(l[0] | (l[1] << 16), l[2] | (l[3] << 16));
}

__device__ __forceinline__ f32x4 mfma16(const bf16x4 a, const bf16x4 b, const f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 lds4(const unsigned short* p) { return *reinterpret_cast<const bf16x4*>(p); }

// ---- forward and input gradient: output tiles of 16 x 4 x 4 voxels (x, y, z), halo 18 x 6 x 6;
// wave w computes z-plane w, its four 16-voxel blocks being the four x-rows.  These use
// v_mfma_f32_16x16x32_bf16 (lane l holds A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16]) with
// the hi and lo halves of 16 input channels packed into K = 32: A = [hi c0..15, lo c0..15],
// B = [w c0..15, w c0..15], so one instruction forms sum_c (hi + lo) w.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma32(const bf16x8 a, const bf16x8 b, const f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 lds8(const unsigned short* p) { return *reinterpret_cast<const bf16x8*>(p); }

constexpr int FHX = 18, FHY = 6, FHV = 18 * 6 * 6;

__host__ __device__ __forceinline__ int ftiles(int n) { return ((n + 15) / 16) * ((n + 3) / 4) * ((n + 3) / 4); }

__device__ __forceinline__ void ftile_origin(int tile, int n, int& x0t, int& y0t, int& z0t) {
  const int ntx = (n + 15) / 16, nty = (n + 3) / 4;
  x0t = (tile % ntx) * 16;
  y0t = ((tile / ntx) % nty) * 4;
  z0t = (tile / (ntx * nty)) * 4;
}

__device__ __forceinline__ uint4 pack8(const unsigned* h) {
  return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// Stage 16 channels [ch0, ch0 + 16) of a two-source input around the tile into LDS as
// [4 parts][648 halo voxels][8] BF16: part 0 / 1 = hi of channels 0-7 / 8-15, part 2 / 3 =
// lo of the same; with MASK a value is zeroed where mask <= 0.  Work item it = 648 h + hv
// covers channels 8 h .. 8 h + 7 of halo voxel hv.  Loads are unconditional (an
// out-of-range element reads voxel 0 of its channel and is zeroed) and issued in batches.
template <bool MASK>
__device__ __forceinline__ void stage_vox16(unsigned short* xs, const float* x0, int c0, const float* x1, int ch0,
                                            const float* mask, int n, int x0t, int y0t, int z0t, size_t vol) {
  constexpr int ITEMS = 2 * FHV, PER = (ITEMS + 255) / 256, BATCH = MASK ? 2 : 3;
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += BATCH) {
    float v[BATCH][8], mk[BATCH][8];
    bool in[BATCH];
#pragma unroll
    for (int kk = 0; kk < BATCH; ++kk) {
      const int it = threadIdx.x + 256 * (k0 + kk);
      const int h = min(it / FHV, 1), hv = it % FHV;
      const int hz = hv / (FHX * FHY), hy = (hv / FHX) % FHY, hx = hv % FHX;
      const int gz = z0t + hz - 1, gy = y0t + hy - 1, gx = x0t + hx - 1;
      in[kk] = k0 + kk < PER && it < ITEMS && unsigned(gz) < unsigned(n) && unsigned(gy) < unsigned(n) &&
               unsigned(gx) < unsigned(n);
      const size_t off = in[kk] ? (size_t(gz) * n + gy) * n + gx : 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = ch0 + 8 * h + j;
        v[kk][j] = chan(x0, c0, x1, c, vol)[off];
        if (MASK) mk[kk][j] = mask[size_t(c) * vol + off];
      }
    }
#pragma unroll
    for (int kk = 0; kk < BATCH; ++kk) {
      const int it = threadIdx.x + 256 * (k0 + kk);
      unsigned hi[8], lo[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        split_bf16(in[kk] && (!MASK || mk[kk][j] > 0.0f) ? v[kk][j] : 0.0f, hi[j], lo[j]);
      if (k0 + kk < PER && it < ITEMS) {
        const int h = it / FHV, hv = it % FHV;
        reinterpret_cast<uint4*>(xs)[h * FHV + hv] = pack8(hi);
        reinterpret_cast<uint4*>(xs)[(2 + h) * FHV + hv] = pack8(lo);
      }
    }
  }
}

// contiguous copy of `shorts` BF16 values (a multiple of 8) from global memory into LDS, in
// rounds of four unconditional 16-byte loads per thread
__device__ __forceinline__ void copy_weights(unsigned short* dst, const unsigned short* src, int shorts) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  const int n16 = shorts / 8;
  for (int base = 0; base < n16; base += 1024) {
    uint4 r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = s[min(base + int(threadIdx.x) + 256 * j, n16 - 1)];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = base + int(threadIdx.x) + 256 * j;
      if (i < n16) d[i] = r[j];
    }
  }
}

// The 27-tap product of one wave: its z-plane of the tile times NB 16-channel blocks of the
// staged weights ws[tap][2][NB*16][8].  For each (dz, dx) the six halo rows the wave needs
// are read once and serve the three dy taps.
template <int NB>
__device__ __forceinline__ void taps_product(const unsigned short* xs, const unsigned short* ws, int wave, int m,
                                             int kg, f32x4 (&acc)[4][NB]) {
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      bf16x8 a[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) a[r] = lds8(&xs[(kg * FHV + ((wave + dz) * FHY + r) * FHX + m + dx) * 8]);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int tap = (dz * 3 + dy) * 3 + dx;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bf16x8 bw = lds8(&ws[((tap * 2 + (kg & 1)) * (NB * 16) + 16 * nb + m) * 8]);
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) acc[mb][nb] = mfma32(a[mb + dy], bw, acc[mb][nb]);
        }
      }
    }
}

// Write a finished tile through LDS so that global stores are whole 16-byte x-runs: the
// accumulators go to o[c][z][y][x] (channel stride OS floats), then thread groups store
// float4s of each channel's rows.  dst(c) gives channel c's output volume.
constexpr int OS = 260;   // 256 + 4: the float4 writes of eight lanes hit distinct banks

template <int NB, class Dst>
__device__ __forceinline__ void store_tile(const f32x4 (&acc)[4][NB], float* o, int wave, int m, int kg, int n,
                                           int x0t, int y0t, int z0t, Dst dst) {
  __syncthreads();
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      *reinterpret_cast<f32x4*>(&o[(16 * nb + m) * OS + wave * 64 + mb * 16 + 4 * kg]) = acc[mb][nb];
  __syncthreads();
  const size_t vol = size_t(n) * n * n;
  (void)vol;
  for (int f = threadIdx.x; f < NB * 16 * 64; f += 256) {
    const int c = f >> 6, z = (f >> 4) & 3, yy = (f >> 2) & 3, xq = f & 3;
    const int gz = z0t + z, gy = y0t + yy, gx = x0t + 4 * xq;
    if (gz >= n || gy >= n || gx >= n) continue;
    const f32x4 v = *reinterpret_cast<const f32x4*>(&o[c * OS + z * 64 + yy * 16 + 4 * xq]);
    float* d = dst(c) + (size_t(gz) * n + gy) * n + gx;
    if ((n & 3) == 0) {
      *reinterpret_cast<f32x4*>(d) = v;
    } else {
      for (int i = 0; i < 4 && gx + i < n; ++i) d[i] = v[i];
    }
  }
}

// Forward: out[co] = act(b + conv(in)) for cout = 16 NB, cin a multiple of 16; wf holds the
// layer's weights as [cin/16][27][2][cout][8] BF16 (input channel 16 chunk + 8 half + i).
template <int NB>
__global__ __launch_bounds__(256) void k_conv_fwd_mfma(const float* __restrict__ x0, int c0,
                                                       const float* __restrict__ x1, int cin,
                                                       const unsigned short* __restrict__ wf,
                                                       const float* __restrict__ b, float* __restrict__ out, int n,
                                                       int relu) {
  constexpr int XS = 4 * FHV * 8, WS = 27 * NB * 16 * 16;   // shorts
  __shared__ __attribute__((aligned(16))) unsigned short smem[XS + WS];
  unsigned short* xs = smem;
  unsigned short* ws = smem + XS;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  int x0t, y0t, z0t;
  ftile_origin(blockIdx.x, n, x0t, y0t, z0t);
  const size_t vol = size_t(n) * n * n;
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int ci0 = 0; ci0 < cin; ci0 += 16) {
    __syncthreads();
    stage_vox16<false>(xs, x0, c0, x1, ci0, nullptr, n, x0t, y0t, z0t, vol);
    copy_weights(ws, wf + size_t(ci0 / 16) * (27 * NB * 256), 27 * NB * 256);
    __syncthreads();
    taps_product<NB>(xs, ws, wave, m, kg, acc);
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const float bias = b[16 * nb + m];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float o = acc[mb][nb][i] + bias;
        acc[mb][nb][i] = relu ? fmaxf(o, 0.0f) : o;
      }
  }
  store_tile<NB>(acc, reinterpret_cast<float*>(smem), wave, m, kg, n, x0t, y0t, z0t,
                 [=](int c) { return out + size_t(c) * vol; });
}

// Input gradient: gx[ci] = sum_co sum_t w[co][ci][t] gm[co][r + 1 - t], gm = g (y > 0), for
// cin = 16 NBI (channels [0, c0) into gx0, the rest into gx1) and cout a multiple of 16; wd
// holds the weights as [cout/16][27][2][cin][8] BF16 with the taps reversed, so that the
// product is the same cross-correlation as the forward one.
template <int NBI>
__global__ __launch_bounds__(256) void k_conv_bwd_data_mfma(const float* __restrict__ g, const float* __restrict__ y,
                                                            int cout, const unsigned short* __restrict__ wd,
                                                            float* __restrict__ gx0, int c0,
                                                            float* __restrict__ gx1, int n) {
  constexpr int XS = 4 * FHV * 8, WS = 27 * NBI * 16 * 16;   // shorts
  __shared__ __attribute__((aligned(16))) unsigned short smem[XS + WS];
  unsigned short* gs = smem;
  unsigned short* ws = smem + XS;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  int x0t, y0t, z0t;
  ftile_origin(blockIdx.x, n, x0t, y0t, z0t);
  const size_t vol = size_t(n) * n * n;
  f32x4 acc[4][NBI];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NBI; ++nb) acc[mb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int o0 = 0; o0 < cout; o0 += 16) {
    __syncthreads();
    stage_vox16<true>(gs, g, cout, nullptr, o0, y, n, x0t, y0t, z0t, vol);
    copy_weights(ws, wd + size_t(o0 / 16) * (27 * NBI * 256), 27 * NBI * 256);
    __syncthreads();
    taps_product<NBI>(gs, ws, wave, m, kg, acc);
  }
  store_tile<NBI>(acc, reinterpret_cast<float*>(smem), wave, m, kg, n, x0t, y0t, z0t,
                  [=](int c) { return c < c0 ? gx0 + size_t(c) * vol : gx1 + size_t(c - c0) * vol; });
}

// ---- weight gradient: tiles of 8 x 8 x 4 voxels, halo 10 x 10 x 6.  The reduction runs over
// voxels; the input's halo z range is kept as three 4-deep windows (window w holding halo
// z = w .. w + 3), so that a tap (dz, dy, dx) reads aligned groups of four z.  Layouts of the
// single-input-channel kernel (16 x 16 x 16 products, K step = 4 columns x 4 z):
//   A (masked output gradient): [64 columns][16 co][4 z], column stride WA_S shorts;
//   B (layer input): [100 halo columns][3 windows][4].
constexpr int WA_S = 68;            // 64 + 4: staging writes along x are conflict-free
constexpr int WA_PER = 4;           // A items (co, column) per thread: 16 * 64 / 256
constexpr int WB_PER = 7;           // B items (ci, halo column) per thread: ceil(16 * 100 / 256)

__host__ __device__ __forceinline__ int wtiles(int n) { return ((n + 7) / 8) * ((n + 7) / 8) * ((n + 3) / 4); }

__device__ __forceinline__ void wtile_origin(int tile, int n, int& x0t, int& y0t, int& z0t) {
  const int ntx = (n + 7) / 8;
  x0t = (tile % ntx) * 8;
  y0t = ((tile / ntx) % ntx) * 8;
  z0t = (tile / (ntx * ntx)) * 4;
}

struct WTileRegs {
  float g[WA_PER][4], y[WA_PER][4];
  float x[WB_PER][6];
  unsigned va;                 // validity of g (bit 4 k + z)
  unsigned long long vb;       // validity of x (bit 6 k + hz)
};

// Load (into registers) the tile's output-gradient block of channels co0 .. co0 + 15 with
// the layer output y (for the ReLU mask) and its input channels ci0 .. ci0 + nci - 1 (nci =
// 16, or 1 for the single-channel first layer) of x.  Loads are unconditional (out-of-range
// elements read a valid address) and their values are not touched here, so that many stay
// in flight together; validity is kept as bit masks and applied when the tile is stored.
// Addresses are a wave-uniform base plus a 32-bit element offset.
template <bool LOAD_A = true, bool LOAD_B = true>
__device__ __forceinline__ void wtile_load(WTileRegs& r, const float* x, const float* g, const float* y, int co0,
                                           int ci0, int nci, int n, int x0t, int y0t, int z0t, size_t vol) {
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const unsigned nn = unsigned(n) * unsigned(n);
  if (LOAD_A) r.va = 0;
  if (LOAD_B) r.vb = 0;
#pragma unroll
  for (int k = 0; k < (LOAD_A ? WA_PER : 0); ++k) {
    // item it = 256 k + 64 wave + lane: channel co0 + 4 k + wave, column lane
    const size_t cofs = size_t(co0 + 4 * k + wave) * vol;
    const float* gb = g + cofs;
    const float* yb = y + cofs;
    const int gy = y0t + (lane >> 3), gx = x0t + (lane & 7);
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int gz = z0t + z;
      const bool in = gz < n && gy < n && gx < n;
      const unsigned o = in ? unsigned(gz) * nn + unsigned(gy) * unsigned(n) + unsigned(gx) : 0u;
      r.g[k][z] = gb[o];
      r.y[k][z] = yb[o];
      r.va |= unsigned(in) << (4 * k + z);
    }
  }
  const float* xb = x + size_t(ci0) * vol;
#pragma unroll
  for (int k = 0; k < (LOAD_B ? WB_PER : 0); ++k) {
    const int it = threadIdx.x + 256 * k;
    const int c = it / 100, cp = it % 100;
    const int gy = y0t + cp / 10 - 1, gx = x0t + cp % 10 - 1;
    const bool inc = c < nci && unsigned(gy) < unsigned(n) && unsigned(gx) < unsigned(n);
    const unsigned cofs = unsigned(min(c, nci - 1)) * unsigned(vol);
#pragma unroll
    for (int hz = 0; hz < 6; ++hz) {
      const int gz = z0t + hz - 1;
      const bool in = inc && unsigned(gz) < unsigned(n);
      r.x[k][hz] = xb[in ? cofs + unsigned(gz) * nn + unsigned(gy) * unsigned(n) + unsigned(gx) : cofs];
      r.vb |= static_cast<unsigned long long>(in) << (6 * k + hz);
    }
  }
}

__device__ __forceinline__ float wtile_g(const WTileRegs& r, int k, int z) {
  return ((r.va >> (4 * k + z)) & 1u) && r.y[k][z] > 0.0f ? r.g[k][z] : 0.0f;
}
__device__ __forceinline__ float wtile_x(const WTileRegs& r, int k, int hz) {
  return ((r.vb >> (6 * k + hz)) & 1ull) ? r.x[k][hz] : 0.0f;
}

// Split the loaded tile into the LDS layouts (B with CI channels per window and halo-column
// stride BS); adds the masked gradient to bsum (bias).
template <int CI, int BS>
__device__ __forceinline__ void wtile_store(const WTileRegs& r, unsigned short* ah, unsigned short* al,
                                            unsigned short* bh, unsigned short* bl, float (&bsum)[WA_PER]) {
#pragma unroll
  for (int k = 0; k < WA_PER; ++k) {
    const int it = threadIdx.x + 256 * k;
    const int co = it >> 6, col = it & 63;
    float v[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      v[z] = wtile_g(r, k, z);
      bsum[k] += v[z];
    }
    uint2 hi, lo;
    split4(v, hi, lo);
    *reinterpret_cast<uint2*>(&ah[col * WA_S + co * 4]) = hi;
    *reinterpret_cast<uint2*>(&al[col * WA_S + co * 4]) = lo;
  }
#pragma unroll
  for (int k = 0; k < WB_PER; ++k) {
    const int it = threadIdx.x + 256 * k;
    const int c = it / 100, cp = it % 100;
    if (c >= CI) continue;
    unsigned h[6], l[6];
#pragma unroll
    for (int hz = 0; hz < 6; ++hz) split_bf16(wtile_x(r, k, hz), h[hz], l[hz]);
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const int o = cp * BS + (w * CI + c) * 4;
      *reinterpret_cast<uint2*>(&bh[o]) = make_uint2(h[w] | (h[w + 1] << 16), h[w + 2] | (h[w + 3] << 16));
      *reinterpret_cast<uint2*>(&bl[o]) = make_uint2(l[w] | (l[w + 1] << 16), l[w + 2] | (l[w + 3] << 16));
    }
  }
}

// Fixed-order bias sum of the workgroup: thread t holds co = t / 64 + 4 k.
__device__ __forceinline__ void wtile_bias(const float (&bsum)[WA_PER], float* red, float* dst) {
#pragma unroll
  for (int k = 0; k < WA_PER; ++k) red[k * 256 + threadIdx.x] = bsum[k];
  __syncthreads();
  if (threadIdx.x < 16) {
    const int co = threadIdx.x;
    const float* p = red + (co >> 2) * 256 + (co & 3) * 64;
    float s = 0.0f;
    for (int j = 0; j < 64; ++j) s += p[j];
    dst[co] = s;
  }
}

// Layouts of the 16-channel weight-gradient kernel, which uses v_mfma_f32_16x16x32_bf16 with
// K = 32 voxels (one y-row of the tile plane x 4 z; lane group q holds columns 2q, 2q + 1):
//   A (masked output gradient), hi and lo planes: [32 column pairs][16 co][2 columns x 4 z],
//     pair stride PA_S shorts;
//   B (layer input), hi and lo planes: [100 halo columns][16 ci][8 z (the 6 halo z, then 0)],
//     halo-column stride PB_S shorts.  A tap's four z (dz .. dz + 3) are cut from a lane's
//     8-z group with a funnel shift for odd dz, so one read serves the three dz taps.
constexpr int PA_S = 136;           // 128 + 8: staging writes along x are conflict-free
constexpr int PB_S = 136;           // 16 * 8 + 8, likewise

__device__ __forceinline__ bf16x8 zwindow(const uint4 c0, const uint4 c1, int dz) {
  uint4 w;
  if (dz == 0) {
    w = make_uint4(c0.x, c0.y, c1.x, c1.y);
  } else if (dz == 2) {
    w = make_uint4(c0.y, c0.z, c1.y, c1.z);
  } else {
    w = make_uint4(__builtin_amdgcn_alignbit(c0.y, c0.x, 16), __builtin_amdgcn_alignbit(c0.z, c0.y, 16),
                   __builtin_amdgcn_alignbit(c1.y, c1.x, 16), __builtin_amdgcn_alignbit(c1.z, c1.y, 16));
  }
  return *reinterpret_cast<const bf16x8*>(&w);
}

template <bool STORE_A, bool STORE_B>
__device__ __forceinline__ void wtile_store32(const WTileRegs& r, unsigned short* ah, unsigned short* al,
                                              unsigned short* bh, unsigned short* bl, float (&bsum)[WA_PER]) {
#pragma unroll
  for (int k = 0; k < (STORE_A ? WA_PER : 0); ++k) {
    const int it = threadIdx.x + 256 * k;
    const int co = it >> 6, col = it & 63;
    float v[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      v[z] = wtile_g(r, k, z);
      bsum[k] += v[z];
    }
    uint2 hi, lo;
    split4(v, hi, lo);
    const int o = (col >> 1) * PA_S + co * 8 + (col & 1) * 4;
    *reinterpret_cast<uint2*>(&ah[o]) = hi;
    *reinterpret_cast<uint2*>(&al[o]) = lo;
  }
#pragma unroll
  for (int k = 0; k < (STORE_B ? WB_PER : 0); ++k) {
    const int it = threadIdx.x + 256 * k;
    const int c = it / 100, cp = it % 100;
    if (c >= 16) continue;
    unsigned h[6], l[6];
#pragma unroll
    for (int hz = 0; hz < 6; ++hz) split_bf16(wtile_x(r, k, hz), h[hz], l[hz]);
    *reinterpret_cast<uint4*>(&bh[cp * PB_S + c * 8]) =
        make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), 0u);
    *reinterpret_cast<uint4*>(&bl[cp * PB_S + c * 8]) =
        make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), 0u);
  }
}

// Weight-gradient partials of a 16 x 16 (co, ci) block over a chunk of tiles:
// pw[chunk][co][ci][t] = sum_v gm[co][v] in[ci][v + t - 1].  Taps are dealt to the waves by
// their (dy, dx) group g = 3 dy + dx: wave w takes groups w and w + 4 with all three dz, and
// waves 0-2 also take group 8 at dz = w (seven taps each, six for wave 3); every wave runs
// over all rows of the tile, one LDS read of a column's eight z serving the dz taps of a
// group.  Each 32-voxel step takes three products (hi hi, hi lo, lo hi).  Two workgroups
// fit a CU (72 KB of LDS each), so one's tile loads overlap the other's products.  The
// workgroup with ci block 0 also writes the bias partial pb[chunk][co].
__global__ __launch_bounds__(256, 2) void k_conv_bwd_w_mfma(const float* __restrict__ x0, int cin,
                                                            const float* __restrict__ g, const float* __restrict__ y,
                                                            int cout, int n, int tiles_per_chunk,
                                                            float* __restrict__ pw, float* __restrict__ pb) {
  constexpr int AS = 32 * PA_S, BS = 100 * PB_S;   // shorts per plane
  __shared__ __attribute__((aligned(16))) unsigned short smem[2 * AS + 2 * BS];
  unsigned short* ah = smem;
  unsigned short* al = smem + AS;
  unsigned short* bh = smem + 2 * AS;
  unsigned short* bl = smem + 2 * AS + BS;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int m = lane & 15, kg = lane >> 4;
  const int nco = cout / 16;
  const int cb = blockIdx.y % nco, ib = blockIdx.y / nco;
  const int ntiles = wtiles(n);
  const size_t vol = size_t(n) * n * n;
  // B offsets of this wave's groups: (dy * 10 + dx) halo columns
  const int g0 = wave, g1 = wave + 4;
  const int off0 = ((g0 / 3) * 10 + g0 % 3) * PB_S, off1 = ((g1 / 3) * 10 + g1 % 3) * PB_S;
  const int off8 = (2 * 10 + 2) * PB_S;
  f32x4 acc[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  float bsum[WA_PER] = {0.0f, 0.0f, 0.0f, 0.0f};
  const int tile_end = min(ntiles, int(blockIdx.x + 1) * tiles_per_chunk);
  for (int tile = blockIdx.x * tiles_per_chunk; tile < tile_end; ++tile) {
    int x0t, y0t, z0t;
    wtile_origin(tile, n, x0t, y0t, z0t);
    // the gradient block is loaded while other waves may still multiply the previous tile;
    // the input block after it, to bound the registers in flight
    WTileRegs r;
    wtile_load<true, false>(r, x0, g, y, 16 * cb, 16 * ib, 16, n, x0t, y0t, z0t, vol);
    __syncthreads();
    wtile_store32<true, false>(r, ah, al, bh, bl, bsum);
    wtile_load<false, true>(r, x0, g, y, 16 * cb, 16 * ib, 16, n, x0t, y0t, z0t, vol);
    wtile_store32<false, true>(r, ah, al, bh, bl, bsum);
    __syncthreads();
#pragma unroll 2
    for (int row = 0; row < 8; ++row) {
      const bf16x8 a_hi = lds8(&ah[(4 * row + kg) * PA_S + m * 8]);
      const bf16x8 a_lo = lds8(&al[(4 * row + kg) * PA_S + m * 8]);
      const int base = (row * 10 + 2 * kg) * PB_S + m * 8;
#pragma unroll
      for (int gi = 0; gi < 2; ++gi) {
        const int o = base + (gi ? off1 : off0);
        const uint4 h0 = *reinterpret_cast<const uint4*>(&bh[o]);
        const uint4 h1 = *reinterpret_cast<const uint4*>(&bh[o + PB_S]);
        const uint4 l0 = *reinterpret_cast<const uint4*>(&bl[o]);
        const uint4 l1 = *reinterpret_cast<const uint4*>(&bl[o + PB_S]);
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
          const bf16x8 b_hi = zwindow(h0, h1, dz), b_lo = zwindow(l0, l1, dz);
          f32x4& a = acc[3 * gi + dz];
          a = mfma32(a_hi, b_hi, a);
          a = mfma32(a_hi, b_lo, a);
          a = mfma32(a_lo, b_hi, a);
        }
      }
      if (wave < 3) {
        const int o = base + off8;
        const uint4 h0 = *reinterpret_cast<const uint4*>(&bh[o]);
        const uint4 h1 = *reinterpret_cast<const uint4*>(&bh[o + PB_S]);
        const uint4 l0 = *reinterpret_cast<const uint4*>(&bl[o]);
        const uint4 l1 = *reinterpret_cast<const uint4*>(&bl[o + PB_S]);
        const bf16x8 b_hi = zwindow(h0, h1, wave), b_lo = zwindow(l0, l1, wave);
        acc[6] = mfma32(a_hi, b_hi, acc[6]);
        acc[6] = mfma32(a_hi, b_lo, acc[6]);
        acc[6] = mfma32(a_lo, b_hi, acc[6]);
      }
    }
  }
  const int ci = 16 * ib + m;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    if (j == 6 && wave == 3) break;
    const int tap = j < 6 ? (j % 3) * 9 + (j < 3 ? g0 : g1) : wave * 9 + 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = 16 * cb + 4 * kg + i;
      pw[((size_t(blockIdx.x) * cout + co) * cin + ci) * 27 + tap] = acc[j][i];
    }
  }
  if (ib == 0) {
    __syncthreads();
    wtile_bias(bsum, reinterpret_cast<float*>(smem), pb + size_t(blockIdx.x) * cout + 16 * cb);
  }
}

// Single-input-channel variant (the first layer): the 27 taps (padded to 32) form the N
// dimension, B[k][tap] = in[v_k + tap - 1]; wave w takes the K steps st = w, w + 4, ...
// and the four waves' sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_conv_bwd_w_mfma_c1(const float* __restrict__ x, const float* __restrict__ g,
                                                            const float* __restrict__ y, int cout, int n,
                                                            int tiles_per_chunk, float* __restrict__ pw,
                                                            float* __restrict__ pb) {
  constexpr int BS1 = 12;
  __shared__ __attribute__((aligned(16))) unsigned short ah[64 * WA_S];
  __shared__ __attribute__((aligned(16))) unsigned short al[64 * WA_S];
  __shared__ __attribute__((aligned(16))) unsigned short bh[100 * BS1];
  __shared__ __attribute__((aligned(16))) unsigned short bl[100 * BS1];
  __shared__ float red[4 * 2 * 64 * 4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  const int cb = blockIdx.y;
  const int ntiles = wtiles(n);
  const size_t vol = size_t(n) * n * n;
  int toff[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int tap = min(16 * nb + m, 26);
    toff[nb] = (((tap / 3) % 3) * 10 + tap % 3) * BS1 + 4 * (tap / 9);
  }
  f32x4 acc[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
  float bsum[WA_PER] = {0.0f, 0.0f, 0.0f, 0.0f};
  const int tile0 = blockIdx.x * tiles_per_chunk;
  const int tile_end = min(ntiles, tile0 + tiles_per_chunk);
  WTileRegs r;
  if (tile0 < tile_end) {
    int x0t, y0t, z0t;
    wtile_origin(tile0, n, x0t, y0t, z0t);
    wtile_load(r, x, g, y, 16 * cb, 0, 1, n, x0t, y0t, z0t, vol);
  }
  for (int tile = tile0; tile < tile_end; ++tile) {
    __syncthreads();
    wtile_store<1, BS1>(r, ah, al, bh, bl, bsum);
    __syncthreads();
    if (tile + 1 < tile_end) {
      int x0t, y0t, z0t;
      wtile_origin(tile + 1, n, x0t, y0t, z0t);
      wtile_load(r, x, g, y, 16 * cb, 0, 1, n, x0t, y0t, z0t, vol);
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int col = 4 * (wave + 4 * s4) + kg;
      const bf16x4 a_hi = lds4(&ah[col * WA_S + m * 4]);
      const bf16x4 a_lo = lds4(&al[col * WA_S + m * 4]);
      const int base = ((col >> 3) * 10 + (col & 7)) * BS1;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const bf16x4 b_hi = lds4(&bh[base + toff[nb]]);
        const bf16x4 b_lo = lds4(&bl[base + toff[nb]]);
        acc[nb] = mfma16(a_hi, b_hi, acc[nb]);
        acc[nb] = mfma16(a_hi, b_lo, acc[nb]);
        acc[nb] = mfma16(a_lo, b_hi, acc[nb]);
      }
    }
  }
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[((wave * 2 + nb) * 64 + lane) * 4 + i] = acc[nb][i];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int tap = 16 * nb + m;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float s = 0.0f;
        for (int w = 0; w < 4; ++w) s += red[((w * 2 + nb) * 64 + lane) * 4 + i];
        if (tap < 27) pw[(size_t(blockIdx.x) * cout + 16 * cb + 4 * kg + i) * 27 + tap] = s;
      }
    }
  }
  __syncthreads();
  wtile_bias(bsum, reinterpret_cast<float*>(ah), pb + size_t(blockIdx.x) * cout + 16 * cb);
}

// Two-stage fixed-order sum of the chunk partials: stage 1 sums chunks s, s + S, s + 2S, ...
// of element i (weights, then biases) into q[s][i]; stage 2 sums q over s in order.
__global__ void k_reduce_slices(const float* __restrict__ pw, const float* __restrict__ pb, int chunks, int nw,
                                int nb, int slices, float* __restrict__ q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (i >= nw + nb) return;
  float acc = 0.0f;
  if (i < nw)
    for (int k = s; k < chunks; k += slices) acc += pw[size_t(k) * nw + i];
  else
    for (int k = s; k < chunks; k += slices) acc += pb[size_t(k) * nb + (i - nw)];
  q[size_t(s) * (nw + nb) + i] = acc;
}

__global__ void k_sum_slices(const float* __restrict__ q, int nw, int nb, int slices, float* __restrict__ gw,
                             float* __restrict__ gb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw + nb) return;
  float acc = 0.0f;
  for (int s = 0; s < slices; ++s) acc += q[size_t(s) * (nw + nb) + i];
  if (i < nw)
    gw[i] = acc;
  else
    gb[i - nw] = acc;
}

// Weight layouts of a 3x3x3 layer for the matrix-core kernels:
//   wf[cin/16][27][2][cout][8]:  wf[c][t][h][co][i] = w[co][16 c + 8 h + i][t]  (forward)
//   wd[cout/16][27][2][cin][8]:  wd[c][t][h][ci][i] = w[16 c + 8 h + i][ci][26 - t]
//     (input gradient, taps reversed).
__global__ void k_weight_layout(const __hip_bfloat16* __restrict__ w, int cout, int cin,
                                unsigned short* __restrict__ wf, unsigned short* __restrict__ wd) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= cout * cin * 27) return;
  const int tap = idx % 27, ci = (idx / 27) % cin, co = idx / (27 * cin);
  const unsigned short v = reinterpret_cast<const unsigned short*>(w)[idx];
  wf[(((size_t(ci / 16) * 27 + tap) * 2 + (ci % 16) / 8) * cout + co) * 8 + ci % 8] = v;
  wd[(((size_t(co / 16) * 27 + (26 - tap)) * 2 + (co % 16) / 8) * cin + ci) * 8 + co % 8] = v;
}

// ------------------------------------------------------------------ resampling
// One thread per output voxel of channel blockIdx.y (32-bit index arithmetic).
__global__ void k_pool2(const float* __restrict__ x, float* __restrict__ y, int n) {
  const unsigned h = unsigned(n) / 2, hv = h * h * h;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= hv) return;
  const unsigned xx = i % h, yy = (i / h) % h, zz = i / (h * h), un = unsigned(n);
  const float* src = x + size_t(blockIdx.y) * un * un * un + (2 * zz * un + 2 * yy) * un + 2 * xx;
  float s = 0.0f;
  for (unsigned a = 0; a < 2; ++a)
    for (unsigned bq = 0; bq < 2; ++bq)
      for (unsigned cq = 0; cq < 2; ++cq) s += src[(a * un + bq) * un + cq];
  y[size_t(blockIdx.y) * hv + i] = 0.125f * s;
}

// y (n^3) = nearest 2x upsampling of x ((n/2)^3)
__global__ void k_up2(const float* __restrict__ x, float* __restrict__ y, int n) {
  const unsigned un = unsigned(n), h = un / 2, nv = un * un * un;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const unsigned xx = i % un, yy = (i / un) % un, zz = i / (un * un);
  y[size_t(blockIdx.y) * nv + i] = x[size_t(blockIdx.y) * h * h * h + ((zz / 2) * h + yy / 2) * h + xx / 2];
}

// gx ((n/2)^3) = sum of g (n^3) over each 2x2x2 block
__global__ void k_up2_bwd(const float* __restrict__ g, float* __restrict__ gx, int n) {
  const unsigned h = unsigned(n) / 2, hv = h * h * h;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= hv) return;
  const unsigned xx = i % h, yy = (i / h) % h, zz = i / (h * h), un = unsigned(n);
  const float* src = g + size_t(blockIdx.y) * un * un * un + (2 * zz * un + 2 * yy) * un + 2 * xx;
  float s = 0.0f;
  for (unsigned a = 0; a < 2; ++a)
    for (unsigned bq = 0; bq < 2; ++bq)
      for (unsigned cq = 0; cq < 2; ++cq) s += src[(a * un + bq) * un + cq];
  gx[size_t(blockIdx.y) * hv + i] = s;
}

// gx (n^3) = g((n/2)^3)/8 at the coarse voxel + add (n^3)
__global__ void k_pool2_bwd_add(const float* __restrict__ g, const float* __restrict__ add, float* __restrict__ gx,
                                int n) {
  const unsigned un = unsigned(n), h = un / 2, nv = un * un * un;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const unsigned xx = i % un, yy = (i / un) % un, zz = i / (un * un);
  const size_t o = size_t(blockIdx.y) * nv + i;
  gx[o] = 0.125f * g[size_t(blockIdx.y) * h * h * h + ((zz / 2) * h + yy / 2) * h + xx / 2] + add[o];
}

// Four consecutive x per thread (n a multiple of 4): float4 stores.
__global__ void k_up2_v4(const float* __restrict__ x, float* __restrict__ y, int n) {
  const unsigned un = unsigned(n), h = un / 2, q = un / 4, nq = q * un * un;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const unsigned xq = i % q, yy = (i / q) % un, zz = i / (q * un);
  const float* src = x + size_t(blockIdx.y) * h * h * h + ((zz / 2) * h + yy / 2) * h + 2 * xq;
  const float a = src[0], b = src[1];
  reinterpret_cast<float4*>(y + size_t(blockIdx.y) * un * un * un)[i] = make_float4(a, a, b, b);
}

__global__ void k_pool2_bwd_add_v4(const float* __restrict__ g, const float* __restrict__ add, float* __restrict__ gx,
                                   int n) {
  const unsigned un = unsigned(n), h = un / 2, q = un / 4, nq = q * un * un;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const unsigned xq = i % q, yy = (i / q) % un, zz = i / (q * un);
  const float* src = g + size_t(blockIdx.y) * h * h * h + ((zz / 2) * h + yy / 2) * h + 2 * xq;
  const float a = 0.125f * src[0], b = 0.125f * src[1];
  const size_t o = size_t(blockIdx.y) * nq + i;
  const float4 s = reinterpret_cast<const float4*>(add)[o];
  reinterpret_cast<float4*>(gx)[o] = make_float4(a + s.x, a + s.y, b + s.z, b + s.w);
}

// ------------------------------------------------------------------ 1x1 output layer (cout = 1)
// Weight-gradient partials of the 1x1 layer: pw[chunk][ci] = sum_v g[v] x[ci][v] and
// pb[chunk] = sum_v g[v] over the chunk's voxels (thread-strided sums, then a fixed tree).
__global__ __launch_bounds__(256) void k_wgrad1x1(const float* __restrict__ x, int cin, const float* __restrict__ g,
                                                  unsigned nv, unsigned per, float* __restrict__ pw,
                                                  float* __restrict__ pb) {
  __shared__ float red[17][256];
  float acc[17];
#pragma unroll
  for (int c = 0; c < 17; ++c) acc[c] = 0.0f;
  const unsigned v0 = blockIdx.x * per, v1 = min(nv, v0 + per);
  for (unsigned v = v0 + threadIdx.x; v < v1; v += 256) {
    const float gv = g[v];
    acc[16] += gv;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c < cin) acc[c] += gv * x[size_t(c) * nv + v];
  }
#pragma unroll
  for (int c = 0; c < 17; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (int(threadIdx.x) < off)
#pragma unroll
      for (int c = 0; c < 17; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < unsigned(cin)) pw[size_t(blockIdx.x) * cin + threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 0) pb[blockIdx.x] = red[16][0];
}


// y[v] = res[v] + b + sum_ci w[ci] x[ci][v]; one thread per voxel, channels summed in order.
__global__ void k_conv1x1_fwd(const float* __restrict__ x, int cin, const __hip_bfloat16* __restrict__ w,
                              const float* __restrict__ b, const float* __restrict__ res, float* __restrict__ y,
                              unsigned nv) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  float s = b[0];
  for (int c = 0; c < cin; ++c) s += __bfloat162float(w[c]) * x[size_t(c) * nv + v];
  y[v] = res ? res[v] + s : s;
}

// gx[ci][v] = w[ci] g[v]
__global__ void k_conv1x1_bwd_data(const float* __restrict__ g, const __hip_bfloat16* __restrict__ w, int cin,
                                   float* __restrict__ gx, unsigned nv) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const float gv = g[v];
  for (int c = 0; c < cin; ++c) gx[size_t(c) * nv + v] = __bfloat162float(w[c]) * gv;
}

// ------------------------------------------------------------------ loss and optimiser
// gy = 2 (y - t) / V; part[block] = sum over the block's voxels of (y - t)^2 (FP64, fixed tree)
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ tg,
                                             float* __restrict__ gy, double* __restrict__ part, size_t count) {
  __shared__ double red[256];
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  double s = 0.0;
  if (i < count) {
    const float r = y[i] - tg[i];
    gy[i] = 2.0f * r / float(count);
    s = double(r) * double(r);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (int(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// one workgroup: each thread sums a strided subset of the partials in order, then a fixed tree
__global__ __launch_bounds__(256) void k_mse_final(const double* __restrict__ part, int nparts, size_t count,
                                                   double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (int(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / double(count);
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int count, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_round_bf16(const float* __restrict__ th, __hip_bfloat16* __restrict__ w, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) w[i] = __float2bfloat16(th[i]);   // round to nearest even
}

// ------------------------------------------------------------------ launchers
static unsigned blocks(size_t count) { return unsigned((count + 255) / 256); }

bool mfma_layer(int ks, int cin, int cout) {
  return ks == 3 && (cin % 16 == 0 || cin == 1) && cout % 16 == 0 && cout <= 64 && cin <= 96;
}

hipError_t weight_layout(const __hip_bfloat16* w, int cout, int cin, unsigned short* wf, unsigned short* wd,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_weight_layout, dim3(blocks(size_t(cout) * cin * 27)), dim3(256), 0, s, w, cout, cin, wf, wd);
  return hipGetLastError();
}


hipError_t conv_fwd(int ks, const float* x0, int c0, const float* x1, int cin, const __hip_bfloat16* w,
                    const unsigned short* wf, const float* b, float* out, int cout, int n, int relu,
                    const float* res, hipStream_t s) {
  if (wf && mfma_layer(ks, cin, cout) && cin % 16 == 0 && !res) {
    const dim3 grid(unsigned(ftiles(n)));
    switch (cout / 16) {
      case 1: hipLaunchKernelGGL(k_conv_fwd_mfma<1>, grid, dim3(256), 0, s, x0, c0, x1, cin, wf, b, out, n, relu); break;
      case 2: hipLaunchKernelGGL(k_conv_fwd_mfma<2>, grid, dim3(256), 0, s, x0, c0, x1, cin, wf, b, out, n, relu); break;
      case 4: hipLaunchKernelGGL(k_conv_fwd_mfma<4>, grid, dim3(256), 0, s, x0, c0, x1, cin, wf, b, out, n, relu); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (ks == 1 && cout == 1 && !x1 && !relu) {
    const unsigned nv = unsigned(n) * unsigned(n) * unsigned(n);
    hipLaunchKernelGGL(k_conv1x1_fwd, dim3(blocks(nv)), dim3(256), 0, s, x0, cin, w, b, res, out, nv);
    return hipGetLastError();
  }
  const int nt = (n + TS - 1) / TS;
  const dim3 grid(unsigned(nt * nt * nt), unsigned((cout + COB - 1) / COB));
  if (ks == 3)
    hipLaunchKernelGGL(k_conv_fwd<3>, grid, dim3(256), 0, s, x0, c0, x1, cin, w, b, out, cout, n, relu, res);
  else
    hipLaunchKernelGGL(k_conv_fwd<1>, grid, dim3(256), 0, s, x0, c0, x1, cin, w, b, out, cout, n, relu, res);
  return hipGetLastError();
}

hipError_t conv_bwd_data(int ks, const float* g, const float* y, int cout, const __hip_bfloat16* w,
                         const unsigned short* wd, float* gx0, int c0, float* gx1, int cin, int n, hipStream_t s) {
  if (wd && y && mfma_layer(ks, cin, cout) && cin % 16 == 0) {   // the matrix-core kernels take the ReLU mask
    const dim3 grid(unsigned(ftiles(n)));
    switch (cin / 16) {
      case 1: hipLaunchKernelGGL(k_conv_bwd_data_mfma<1>, grid, dim3(256), 0, s, g, y, cout, wd, gx0, c0, gx1, n); break;
      case 2: hipLaunchKernelGGL(k_conv_bwd_data_mfma<2>, grid, dim3(256), 0, s, g, y, cout, wd, gx0, c0, gx1, n); break;
      case 3: hipLaunchKernelGGL(k_conv_bwd_data_mfma<3>, grid, dim3(256), 0, s, g, y, cout, wd, gx0, c0, gx1, n); break;
      case 4: hipLaunchKernelGGL(k_conv_bwd_data_mfma<4>, grid, dim3(256), 0, s, g, y, cout, wd, gx0, c0, gx1, n); break;
      case 6: hipLaunchKernelGGL(k_conv_bwd_data_mfma<6>, grid, dim3(256), 0, s, g, y, cout, wd, gx0, c0, gx1, n); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (ks == 1 && cout == 1 && !y && c0 >= cin) {
    const unsigned nv = unsigned(n) * unsigned(n) * unsigned(n);
    hipLaunchKernelGGL(k_conv1x1_bwd_data, dim3(blocks(nv)), dim3(256), 0, s, g, w, cin, gx0, nv);
    return hipGetLastError();
  }
  const int nt = (n + TS - 1) / TS;
  const dim3 grid(unsigned(nt * nt * nt), unsigned((cin + COB - 1) / COB));
  if (ks == 3)
    hipLaunchKernelGGL(k_conv_bwd_data<3>, grid, dim3(256), 0, s, g, y, cout, w, gx0, c0, gx1, cin, n);
  else
    hipLaunchKernelGGL(k_conv_bwd_data<1>, grid, dim3(256), 0, s, g, y, cout, w, gx0, c0, gx1, cin, n);
  return hipGetLastError();
}

// Chunking of the weight-gradient reduction: about 1024 (2048 for the single-channel kernel)
// workgroups over the (co, ci) block pairs (1024 chunks for a 1x1 layer, 128 for other
// layers of the general kernel), every chunk holding at least one tile.
static void wgrad_split(int ks, int cin, int cout, int n, int& chunks, int& per) {
  int ntiles;
  int target;
  if (mfma_layer(ks, cin, cout)) {
    ntiles = wtiles(n);
    const int pairs = (cout / 16) * (cin == 1 ? 1 : cin / 16);
    const int wgs = cin == 1 ? 2048 : 1024;
    target = (wgs + pairs - 1) / pairs;
  } else {
    const int ntx = (n + TS - 1) / TS, ntz = (n + WTZ - 1) / WTZ;
    ntiles = ntx * ntx * ntz;
    target = ks == 1 ? 1024 : 128;
  }
  chunks = std::max(1, std::min(ntiles, target));
  per = (ntiles + chunks - 1) / chunks;
  chunks = (ntiles + per - 1) / per;
}

static int wgrad_slices(int chunks) { return std::min(chunks, 32); }

void wgrad_workspace(int ks, int cin, int cout, int n, size_t& pw_floats, size_t& pb_floats, size_t& q_floats) {
  int chunks, per;
  wgrad_split(ks, cin, cout, n, chunks, per);
  const size_t nw = size_t(cout) * cin * ks * ks * ks;
  pw_floats = size_t(chunks) * nw;
  pb_floats = size_t(chunks) * cout;
  q_floats = size_t(wgrad_slices(chunks)) * (nw + cout);
}

hipError_t conv_bwd_w(int ks, const float* x0, int c0, const float* x1, int cin, const float* g, const float* y,
                      int cout, int n, float* pw, float* pb, float* q, float* gw, float* gb, hipStream_t s) {
  int chunks, per;
  wgrad_split(ks, cin, cout, n, chunks, per);
  const int nw = cout * cin * ks * ks * ks;
  if (y && !x1 && mfma_layer(ks, cin, cout)) {   // matrix-core kernels: one input tensor, ReLU mask
    if (cin == 1)
      hipLaunchKernelGGL(k_conv_bwd_w_mfma_c1, dim3(unsigned(chunks), unsigned(cout / 16)), dim3(256), 0, s, x0, g, y,
                         cout, n, per, pw, pb);
    else
      hipLaunchKernelGGL(k_conv_bwd_w_mfma, dim3(unsigned(chunks), unsigned((cout / 16) * (cin / 16))), dim3(256), 0,
                         s, x0, cin, g, y, cout, n, per, pw, pb);
  } else if (ks == 1 && cout == 1 && cin <= 16 && !y && !x1) {
    const unsigned nv = unsigned(n) * unsigned(n) * unsigned(n);
    const unsigned vper = (nv + unsigned(chunks) - 1) / unsigned(chunks);
    hipLaunchKernelGGL(k_wgrad1x1, dim3(unsigned(chunks)), dim3(256), 0, s, x0, cin, g, nv, vper, pw, pb);
  } else {
    const int nco = (cout + 15) / 16, nci = (cin + 15) / 16;
    const dim3 grid(unsigned(chunks), unsigned(nco * nci));
    if (ks == 3)
      hipLaunchKernelGGL(k_conv_bwd_w<3>, grid, dim3(256), 0, s, x0, c0, x1, cin, g, y, cout, n, per, pw, pb);
    else
      hipLaunchKernelGGL(k_conv_bwd_w<1>, grid, dim3(256), 0, s, x0, c0, x1, cin, g, y, cout, n, per, pw, pb);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int slices = wgrad_slices(chunks);
  hipLaunchKernelGGL(k_reduce_slices, dim3(blocks(size_t(nw + cout)), unsigned(slices)), dim3(256), 0, s, pw, pb,
                     chunks, nw, cout, slices, q);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_slices, dim3(blocks(size_t(nw + cout))), dim3(256), 0, s, q, nw, cout, slices, gw, gb);
  return hipGetLastError();
}

static dim3 vox_grid(size_t voxels, int c) { return dim3(blocks(voxels), unsigned(c)); }

hipError_t pool2(const float* x, float* y, int c, int n, hipStream_t s) {
  const size_t h = size_t(n / 2);
  hipLaunchKernelGGL(k_pool2, vox_grid(h * h * h, c), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t up2(const float* x, float* y, int c, int n, hipStream_t s) {
  if (n % 4 == 0)
    hipLaunchKernelGGL(k_up2_v4, vox_grid(size_t(n) * n * n / 4, c), dim3(256), 0, s, x, y, n);
  else
    hipLaunchKernelGGL(k_up2, vox_grid(size_t(n) * n * n, c), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t up2_bwd(const float* g, float* gx, int c, int n, hipStream_t s) {
  const size_t h = size_t(n / 2);
  hipLaunchKernelGGL(k_up2_bwd, vox_grid(h * h * h, c), dim3(256), 0, s, g, gx, n);
  return hipGetLastError();
}

hipError_t pool2_bwd_add(const float* g, const float* add, float* gx, int c, int n, hipStream_t s) {
  if (n % 4 == 0)
    hipLaunchKernelGGL(k_pool2_bwd_add_v4, vox_grid(size_t(n) * n * n / 4, c), dim3(256), 0, s, g, add, gx, n);
  else
    hipLaunchKernelGGL(k_pool2_bwd_add, vox_grid(size_t(n) * n * n, c), dim3(256), 0, s, g, add, gx, n);
  return hipGetLastError();
}

hipError_t mse(const float* y, const float* tg, float* gy, double* part, double* loss, size_t count, hipStream_t s) {
  const unsigned nb = blocks(count);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, y, tg, gy, part, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, s, part, int(nb), count, loss);
  return hipGetLastError();
}

hipError_t adam(float* th, const float* g, float* m, float* v, int count, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(blocks(size_t(count))), dim3(256), 0, s, th, g, m, v, count, lr, b1, b2, eps, c1,
                     c2);
  return hipGetLastError();
}

hipError_t round_bf16(const float* th, __hip_bfloat16* w, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_round_bf16, dim3(blocks(size_t(count))), dim3(256), 0, s, th, w, count);
  return hipGetLastError();
}

}  // namespace unet

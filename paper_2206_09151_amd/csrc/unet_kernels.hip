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

// grad[w] = sum over chunks (in order) of pw; grad[b] likewise (layer's slice of the gradient vector).
__global__ void k_reduce_chunks(const float* __restrict__ pw, const float* __restrict__ pb, int chunks, int nw,
                                int nb, float* __restrict__ gw, float* __restrict__ gb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) {
    float s = 0.0f;
    for (int k = 0; k < chunks; ++k) s += pw[size_t(k) * nw + i];
    gw[i] = s;
  } else if (i < nw + nb) {
    const int j = i - nw;
    float s = 0.0f;
    for (int k = 0; k < chunks; ++k) s += pb[size_t(k) * nb + j];
    gb[j] = s;
  }
}

// ------------------------------------------------------------------ matrix-core convolutions
// The 3x3x3 convolutions with 16-multiple channel counts run on the matrix cores as
// implicit GEMMs with v_mfma_f32_16x16x16_bf16 (16 voxels x 16 channels x 16 channels per
// instruction; lane l holds A[l%16][4(l/16)..+3], B[4(l/16)..+3][l%16] and
// D[4(l/16)+i][l%16]).  Weights are BF16 values already; an FP32 activation or gradient
// is split into BF16 hi + lo (v = hi + lo + e, |e| <= 2^-18 |v|) and both halves are
// multiplied, so the result keeps FP32-level accuracy: two instructions per product for
// the forward and input-gradient passes, three (hi*hi + hi*lo + lo*hi) for the weight
// gradient, whose operands are both FP32.  Tiles: 8 x 8 x 4 output voxels per workgroup,
// one z-plane (four 16-voxel blocks) per wave, input channels in chunks of 16 staged in
// LDS as [voxel][channel] with their halo.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MHV = 600;   // halo voxels of an 8 x 8 x 4 tile (10 x 10 x 6)
constexpr int MVS = 20;    // LDS stride of a halo voxel (16 channels + 4 pad shorts: 40 bytes)

__device__ __forceinline__ unsigned short bf_bits(float v) {
  const __hip_bfloat16 h = __float2bfloat16(v);
  return *reinterpret_cast<const unsigned short*>(&h);
}
__device__ __forceinline__ float bits_bf(unsigned short u) { return __uint_as_float(unsigned(u) << 16); }

__device__ __forceinline__ void split_bf16(float v, unsigned short& hi, unsigned short& lo) {
  hi = bf_bits(v);
  lo = bf_bits(v - bits_bf(hi));
}

__device__ __forceinline__ f32x4 mfma16(const bf16x4 a, const bf16x4 b, const f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Stage 16 channels [ch0, ch0 + 16) of a (two-source) input around the tile, split hi / lo;
// with mask (non-null) the value is multiplied by (mask > 0) first.
__device__ __forceinline__ void stage_split(unsigned short* xh, unsigned short* xl, const float* x0, int c0,
                                            const float* x1, int cin, int ch0, const float* mask, int n,
                                            int x0t, int y0t, int z0t, size_t vol) {
  for (int idx = threadIdx.x; idx < 16 * MHV; idx += 256) {
    const int c = idx / MHV, hv = idx % MHV;
    const int hz = hv / 100, hy = (hv / 10) % 10, hx = hv % 10;
    const int gz = z0t + hz - 1, gy = y0t + hy - 1, gx = x0t + hx - 1;
    float v = 0.0f;
    if (ch0 + c < cin && unsigned(gz) < unsigned(n) && unsigned(gy) < unsigned(n) && unsigned(gx) < unsigned(n)) {
      const size_t off = (size_t(gz) * n + gy) * n + gx;
      v = chan(x0, c0, x1, ch0 + c, vol)[off];
      if (mask && !(mask[size_t(ch0 + c) * vol + off] > 0.0f)) v = 0.0f;
    }
    unsigned short hi, lo;
    split_bf16(v, hi, lo);
    xh[hv * MVS + c] = hi;
    xl[hv * MVS + c] = lo;
  }
}

// Forward: out[co] = act(b + conv(in)), cout = 16 NB, cin a multiple of 16.
template <int NB>
__global__ __launch_bounds__(256) void k_conv_fwd_mfma(const float* __restrict__ x0, int c0,
                                                       const float* __restrict__ x1, int cin,
                                                       const __hip_bfloat16* __restrict__ w,
                                                       const float* __restrict__ b, float* __restrict__ out, int n,
                                                       int relu) {
  __shared__ __attribute__((aligned(16))) unsigned short xh[MHV * MVS];
  __shared__ __attribute__((aligned(16))) unsigned short xl[MHV * MVS];
  __shared__ __attribute__((aligned(16))) unsigned short ws[27 * NB * 16 * 16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  const int ntx = (n + 7) / 8;
  const int tile = blockIdx.x;
  const int x0t = (tile % ntx) * 8, y0t = ((tile / ntx) % ntx) * 8, z0t = (tile / (ntx * ntx)) * 4;
  const size_t vol = size_t(n) * n * n;
  const unsigned short* wb = reinterpret_cast<const unsigned short*>(w);
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int ci0 = 0; ci0 < cin; ci0 += 16) {
    __syncthreads();
    stage_split(xh, xl, x0, c0, x1, cin, ci0, nullptr, n, x0t, y0t, z0t, vol);
    for (int idx = t; idx < 27 * NB * 16 * 16; idx += 256) {
      const int c = idx % 16, co = (idx / 16) % (NB * 16), tap = idx / (16 * NB * 16);
      ws[idx] = wb[(size_t(co) * cin + ci0 + c) * 27 + tap];
    }
    __syncthreads();
    for (int tap = 0; tap < 27; ++tap) {
      const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
      bf16x4 ah[4], al[4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const int hv = ((wave + dz) * 10 + (2 * mb + (m >> 3) + dy)) * 10 + (m & 7) + dx;
        ah[mb] = *reinterpret_cast<const bf16x4*>(&xh[hv * MVS + 4 * kg]);
        al[mb] = *reinterpret_cast<const bf16x4*>(&xl[hv * MVS + 4 * kg]);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x4 bw = *reinterpret_cast<const bf16x4*>(&ws[((tap * NB + nb) * 16 + m) * 16 + 4 * kg]);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          acc[mb][nb] = mfma16(ah[mb], bw, acc[mb][nb]);
          acc[mb][nb] = mfma16(al[mb], bw, acc[mb][nb]);
        }
      }
    }
  }
  const int gz = z0t + wave;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int mm = 4 * kg + i;
      const int gy = y0t + 2 * mb + (mm >> 3), gx = x0t + (mm & 7);
      if (gz >= n || gy >= n || gx >= n) continue;
      const size_t v = (size_t(gz) * n + gy) * n + gx;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = 16 * nb + m;
        float o = acc[mb][nb][i] + b[co];
        if (relu) o = fmaxf(o, 0.0f);
        out[size_t(co) * vol + v] = o;
      }
    }
}

// Input gradient: gx[ci] = sum_co sum_t w[co][ci][t] gm[co][r + 1 - t], gm = g (y > 0);
// cin = 16 NBI output channels (split over gx0 / gx1 at c0), cout a multiple of 16.
template <int NBI>
__global__ __launch_bounds__(256) void k_conv_bwd_data_mfma(const float* __restrict__ g, const float* __restrict__ y,
                                                            int cout, const __hip_bfloat16* __restrict__ w,
                                                            float* __restrict__ gx0, int c0,
                                                            float* __restrict__ gx1, int cin, int n) {
  __shared__ __attribute__((aligned(16))) unsigned short gh[MHV * MVS];
  __shared__ __attribute__((aligned(16))) unsigned short gl[MHV * MVS];
  __shared__ __attribute__((aligned(16))) unsigned short ws[27 * NBI * 16 * 16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  const int ntx = (n + 7) / 8;
  const int tile = blockIdx.x;
  const int x0t = (tile % ntx) * 8, y0t = ((tile / ntx) % ntx) * 8, z0t = (tile / (ntx * ntx)) * 4;
  const size_t vol = size_t(n) * n * n;
  const unsigned short* wb = reinterpret_cast<const unsigned short*>(w);
  f32x4 acc[4][NBI];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NBI; ++nb) acc[mb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int o0 = 0; o0 < cout; o0 += 16) {
    __syncthreads();
    stage_split(gh, gl, g, cout, nullptr, cout, o0, y, n, x0t, y0t, z0t, vol);
    // ws[tap'][ci][c] = w[o0 + c][ci][26 - tap'] (flipped taps)
    for (int idx = t; idx < 27 * NBI * 16 * 16; idx += 256) {
      const int c = idx % 16, ci = (idx / 16) % (NBI * 16), tp = idx / (16 * NBI * 16);
      ws[idx] = wb[(size_t(o0 + c) * cin + ci) * 27 + (26 - tp)];
    }
    __syncthreads();
    for (int tap = 0; tap < 27; ++tap) {
      const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
      bf16x4 ah[4], al[4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const int hv = ((wave + dz) * 10 + (2 * mb + (m >> 3) + dy)) * 10 + (m & 7) + dx;
        ah[mb] = *reinterpret_cast<const bf16x4*>(&gh[hv * MVS + 4 * kg]);
        al[mb] = *reinterpret_cast<const bf16x4*>(&gl[hv * MVS + 4 * kg]);
      }
#pragma unroll
      for (int nb = 0; nb < NBI; ++nb) {
        const bf16x4 bw = *reinterpret_cast<const bf16x4*>(&ws[((tap * NBI + nb) * 16 + m) * 16 + 4 * kg]);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          acc[mb][nb] = mfma16(ah[mb], bw, acc[mb][nb]);
          acc[mb][nb] = mfma16(al[mb], bw, acc[mb][nb]);
        }
      }
    }
  }
  const int gz = z0t + wave;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int mm = 4 * kg + i;
      const int gy = y0t + 2 * mb + (mm >> 3), gx = x0t + (mm & 7);
      if (gz >= n || gy >= n || gx >= n) continue;
      const size_t v = (size_t(gz) * n + gy) * n + gx;
#pragma unroll
      for (int nb = 0; nb < NBI; ++nb) {
        const int ci = 16 * nb + m;
        float* dst = ci < c0 ? gx0 + size_t(ci) * vol : gx1 + size_t(ci - c0) * vol;
        dst[v] = acc[mb][nb][i];
      }
    }
}

// Weight gradient partials: pw[chunk][co][ci][t] = sum_v gm[co][v] in[ci][v + t - 1] over a
// chunk of 8x8x4 tiles.  Workgroup = (chunk, 2x2 block of (co, ci) 16-blocks); wave = one
// (co, ci) block with 27 accumulators; a 16-voxel K step is one z-plane half-tile row pair.
__global__ __launch_bounds__(256) void k_conv_bwd_w_mfma(const float* __restrict__ x0, int c0,
                                                         const float* __restrict__ x1, int cin,
                                                         const float* __restrict__ g, const float* __restrict__ y,
                                                         int cout, int n, int tiles_per_chunk,
                                                         float* __restrict__ pw) {
  constexpr int TV = 256;                                // voxels of a tile
  __shared__ __attribute__((aligned(16))) unsigned short ah_s[2][16][TV];
  __shared__ __attribute__((aligned(16))) unsigned short al_s[2][16][TV];
  __shared__ unsigned short bh_s[2][16][MHV];
  __shared__ unsigned short bl_s[2][16][MHV];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  const int ncb = cout / 16, nib = cin / 16;
  const int nqc = (ncb + 1) / 2;
  const int cb0 = 2 * (blockIdx.y % nqc), ib0 = 2 * (blockIdx.y / nqc);
  const int cbl = wave >> 1, ibl = wave & 1;             // this wave's block within the quad
  const bool active = cb0 + cbl < ncb && ib0 + ibl < nib;
  const int ntx = (n + 7) / 8, ntz = (n + 3) / 4;
  const int ntiles = ntx * ntx * ntz;
  const size_t vol = size_t(n) * n * n;
  f32x4 acc[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int tile_end = min(ntiles, (int(blockIdx.x) + 1) * tiles_per_chunk);
  for (int tile = blockIdx.x * tiles_per_chunk; tile < tile_end; ++tile) {
    const int x0t = (tile % ntx) * 8, y0t = ((tile / ntx) % ntx) * 8, z0t = (tile / (ntx * ntx)) * 4;
    __syncthreads();
    // masked output gradient of the quad's two co blocks, split, [block][co][voxel]
    for (int idx = t; idx < 2 * 16 * TV; idx += 256) {
      const int v = idx % TV, c = (idx / TV) % 16, blk = idx / (16 * TV);
      const int co = 16 * (cb0 + blk) + c;
      const int gz = z0t + v / 64, gy = y0t + (v / 8) % 8, gx = x0t + v % 8;
      float val = 0.0f;
      if (co < cout && gz < n && gy < n && gx < n) {
        const size_t a = size_t(co) * vol + (size_t(gz) * n + gy) * n + gx;
        val = g[a];
        if (y && !(y[a] > 0.0f)) val = 0.0f;
      }
      unsigned short hi, lo;
      split_bf16(val, hi, lo);
      ah_s[blk][c][v] = hi;
      al_s[blk][c][v] = lo;
    }
    // input of the quad's two ci blocks with the halo, split, [block][ci][halo voxel]
    for (int idx = t; idx < 2 * 16 * MHV; idx += 256) {
      const int hv = idx % MHV, c = (idx / MHV) % 16, blk = idx / (16 * MHV);
      const int ci = 16 * (ib0 + blk) + c;
      const int hz = hv / 100, hy = (hv / 10) % 10, hx = hv % 10;
      const int gz = z0t + hz - 1, gy = y0t + hy - 1, gx = x0t + hx - 1;
      float val = 0.0f;
      if (ci < cin && unsigned(gz) < unsigned(n) && unsigned(gy) < unsigned(n) && unsigned(gx) < unsigned(n))
        val = chan(x0, c0, x1, ci, vol)[(size_t(gz) * n + gy) * n + gx];
      unsigned short hi, lo;
      split_bf16(val, hi, lo);
      bh_s[blk][c][hv] = hi;
      bl_s[blk][c][hv] = lo;
    }
    __syncthreads();
    if (!active) continue;
    for (int st = 0; st < TV / 16; ++st) {
      // A: rows co (m), k = voxels 16 st + 4 kg .. + 3
      const bf16x4 ahi = *reinterpret_cast<const bf16x4*>(&ah_s[cbl][m][16 * st + 4 * kg]);
      const bf16x4 alo = *reinterpret_cast<const bf16x4*>(&al_s[cbl][m][16 * st + 4 * kg]);
      // the four voxels of this lane's k group: one x-run of 4 in row (z, y)
      const int z = st / 4, yy = 2 * (st % 4) + (kg >> 1), xb = 4 * (kg & 1);
#pragma unroll
      for (int tap = 0; tap < 27; ++tap) {
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
        const int hv = ((z + dz) * 10 + yy + dy) * 10 + xb + dx;
        const unsigned short* ph = &bh_s[ibl][m][hv];
        const unsigned short* pl = &bl_s[ibl][m][hv];
        const bf16x4 bhi = {short(ph[0]), short(ph[1]), short(ph[2]), short(ph[3])};
        const bf16x4 blo = {short(pl[0]), short(pl[1]), short(pl[2]), short(pl[3])};
        acc[tap] = mfma16(ahi, bhi, acc[tap]);
        acc[tap] = mfma16(ahi, blo, acc[tap]);
        acc[tap] = mfma16(alo, bhi, acc[tap]);
      }
    }
  }
  if (!active) return;
  const int ci = 16 * (ib0 + ibl) + m;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int co = 16 * (cb0 + cbl) + 4 * kg + i;
    float* dst = pw + (size_t(blockIdx.x) * cout * cin + size_t(co) * cin + ci) * 27;
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) dst[tap] = acc[tap][i];
  }
}

// Bias-gradient partials pb[chunk][co] = sum over the chunk's tiles of gm[co] (FP32, fixed tree).
__global__ __launch_bounds__(256) void k_bias_partial(const float* __restrict__ g, const float* __restrict__ y,
                                                      int cout, int n, int tiles_per_chunk, float* __restrict__ pb) {
  __shared__ float red[256];
  const int co = blockIdx.y;
  const int ntx = (n + 7) / 8, ntz = (n + 3) / 4;
  const int ntiles = ntx * ntx * ntz;
  const size_t vol = size_t(n) * n * n;
  float s = 0.0f;
  const int tile_end = min(ntiles, (int(blockIdx.x) + 1) * tiles_per_chunk);
  for (int tile = blockIdx.x * tiles_per_chunk; tile < tile_end; ++tile) {
    const int x0t = (tile % ntx) * 8, y0t = ((tile / ntx) % ntx) * 8, z0t = (tile / (ntx * ntx)) * 4;
    const int v = threadIdx.x;
    const int gz = z0t + v / 64, gy = y0t + (v / 8) % 8, gx = x0t + v % 8;
    if (gz < n && gy < n && gx < n) {
      const size_t a = size_t(co) * vol + (size_t(gz) * n + gy) * n + gx;
      if (!y || y[a] > 0.0f) s += g[a];
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (int(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) pb[size_t(blockIdx.x) * cout + co] = red[0];
}

// ------------------------------------------------------------------ resampling
__global__ void k_pool2(const float* __restrict__ x, float* __restrict__ y, int c, int n) {
  const int h = n / 2;
  const size_t total = size_t(c) * h * h * h;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int xx = int(i % h), yy = int((i / h) % h), zz = int((i / (size_t(h) * h)) % h);
  const size_t ch = i / (size_t(h) * h * h);
  const float* src = x + ch * size_t(n) * n * n;
  float s = 0.0f;
  for (int a = 0; a < 2; ++a)
    for (int bq = 0; bq < 2; ++bq)
      for (int cq = 0; cq < 2; ++cq) s += src[(size_t(2 * zz + a) * n + 2 * yy + bq) * n + 2 * xx + cq];
  y[i] = 0.125f * s;
}

// y (n^3, c channels) = nearest 2x upsampling of x ((n/2)^3)
__global__ void k_up2(const float* __restrict__ x, float* __restrict__ y, int c, int n) {
  const int h = n / 2;
  const size_t total = size_t(c) * n * n * n;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int xx = int(i % n), yy = int((i / n) % n), zz = int((i / (size_t(n) * n)) % n);
  const size_t ch = i / (size_t(n) * n * n);
  y[i] = x[ch * size_t(h) * h * h + (size_t(zz / 2) * h + yy / 2) * h + xx / 2];
}

// gx ((n/2)^3) = sum of g (n^3) over each 2x2x2 block
__global__ void k_up2_bwd(const float* __restrict__ g, float* __restrict__ gx, int c, int n) {
  const int h = n / 2;
  const size_t total = size_t(c) * h * h * h;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int xx = int(i % h), yy = int((i / h) % h), zz = int((i / (size_t(h) * h)) % h);
  const size_t ch = i / (size_t(h) * h * h);
  const float* src = g + ch * size_t(n) * n * n;
  float s = 0.0f;
  for (int a = 0; a < 2; ++a)
    for (int bq = 0; bq < 2; ++bq)
      for (int cq = 0; cq < 2; ++cq) s += src[(size_t(2 * zz + a) * n + 2 * yy + bq) * n + 2 * xx + cq];
  gx[i] = s;
}

// gx (n^3) = g((n/2)^3)/8 at the coarse voxel + add (n^3)
__global__ void k_pool2_bwd_add(const float* __restrict__ g, const float* __restrict__ add, float* __restrict__ gx,
                                int c, int n) {
  const int h = n / 2;
  const size_t total = size_t(c) * n * n * n;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int xx = int(i % n), yy = int((i / n) % n), zz = int((i / (size_t(n) * n)) % n);
  const size_t ch = i / (size_t(n) * n * n);
  gx[i] = 0.125f * g[ch * size_t(h) * h * h + (size_t(zz / 2) * h + yy / 2) * h + xx / 2] + add[i];
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

static bool mfma_ok(int ks, int cin, int cout) { return ks == 3 && cin % 16 == 0 && cout % 16 == 0; }

hipError_t conv_fwd(int ks, const float* x0, int c0, const float* x1, int cin, const __hip_bfloat16* w,
                    const float* b, float* out, int cout, int n, int relu, const float* res, hipStream_t s) {
  if (mfma_ok(ks, cin, cout) && !res && (cout == 16 || cout == 32 || cout == 64)) {
    const int ntx = (n + 7) / 8, ntz = (n + 3) / 4;
    const dim3 grid(unsigned(ntx * ntx * ntz));
    if (cout == 16)
      hipLaunchKernelGGL(k_conv_fwd_mfma<1>, grid, dim3(256), 0, s, x0, c0, x1, cin, w, b, out, n, relu);
    else if (cout == 32)
      hipLaunchKernelGGL(k_conv_fwd_mfma<2>, grid, dim3(256), 0, s, x0, c0, x1, cin, w, b, out, n, relu);
    else
      hipLaunchKernelGGL(k_conv_fwd_mfma<4>, grid, dim3(256), 0, s, x0, c0, x1, cin, w, b, out, n, relu);
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

hipError_t conv_bwd_data(int ks, const float* g, const float* y, int cout, const __hip_bfloat16* w, float* gx0,
                         int c0, float* gx1, int cin, int n, hipStream_t s) {
  if (mfma_ok(ks, cin, cout) && cin <= 96) {
    const int ntx = (n + 7) / 8, ntz = (n + 3) / 4;
    const dim3 grid(unsigned(ntx * ntx * ntz));
    switch (cin / 16) {
      case 1: hipLaunchKernelGGL(k_conv_bwd_data_mfma<1>, grid, dim3(256), 0, s, g, y, cout, w, gx0, c0, gx1, cin, n); break;
      case 2: hipLaunchKernelGGL(k_conv_bwd_data_mfma<2>, grid, dim3(256), 0, s, g, y, cout, w, gx0, c0, gx1, cin, n); break;
      case 3: hipLaunchKernelGGL(k_conv_bwd_data_mfma<3>, grid, dim3(256), 0, s, g, y, cout, w, gx0, c0, gx1, cin, n); break;
      case 4: hipLaunchKernelGGL(k_conv_bwd_data_mfma<4>, grid, dim3(256), 0, s, g, y, cout, w, gx0, c0, gx1, cin, n); break;
      case 6: hipLaunchKernelGGL(k_conv_bwd_data_mfma<6>, grid, dim3(256), 0, s, g, y, cout, w, gx0, c0, gx1, cin, n); break;
      default: return hipErrorInvalidValue;
    }
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

int weight_grad_chunks(int n) {
  const int ntx = (n + TS - 1) / TS, ntz = (n + WTZ - 1) / WTZ;
  const int ntiles = ntx * ntx * ntz;
  return ntiles < 128 ? ntiles : 128;
}

hipError_t conv_bwd_w(int ks, const float* x0, int c0, const float* x1, int cin, const float* g, const float* y,
                      int cout, int n, float* pw, float* pb, float* gw, float* gb, hipStream_t s) {
  const int ntx = (n + TS - 1) / TS, ntz = (n + WTZ - 1) / WTZ;
  const int ntiles = ntx * ntx * ntz;
  const int chunks = weight_grad_chunks(n);
  const int per = (ntiles + chunks - 1) / chunks;
  const int nco = (cout + 15) / 16, nci = (cin + 15) / 16;
  if (mfma_ok(ks, cin, cout)) {
    const dim3 gq(unsigned(chunks), unsigned(((nco + 1) / 2) * ((nci + 1) / 2)));
    hipLaunchKernelGGL(k_conv_bwd_w_mfma, gq, dim3(256), 0, s, x0, c0, x1, cin, g, y, cout, n, per, pw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_partial, dim3(unsigned(chunks), unsigned(cout)), dim3(256), 0, s, g, y, cout, n, per,
                       pb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nw = cout * cin * 27;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(blocks(size_t(nw + cout))), dim3(256), 0, s, pw, pb, chunks, nw, cout,
                       gw, gb);
    return hipGetLastError();
  }
  const dim3 grid(unsigned(chunks), unsigned(nco * nci));
  if (ks == 3)
    hipLaunchKernelGGL(k_conv_bwd_w<3>, grid, dim3(256), 0, s, x0, c0, x1, cin, g, y, cout, n, per, pw, pb);
  else
    hipLaunchKernelGGL(k_conv_bwd_w<1>, grid, dim3(256), 0, s, x0, c0, x1, cin, g, y, cout, n, per, pw, pb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nw = cout * cin * ks * ks * ks;
  hipLaunchKernelGGL(k_reduce_chunks, dim3(blocks(size_t(nw + cout))), dim3(256), 0, s, pw, pb, chunks, nw, cout, gw,
                     gb);
  return hipGetLastError();
}

hipError_t pool2(const float* x, float* y, int c, int n, hipStream_t s) {
  const size_t h = size_t(n / 2);
  hipLaunchKernelGGL(k_pool2, dim3(blocks(size_t(c) * h * h * h)), dim3(256), 0, s, x, y, c, n);
  return hipGetLastError();
}

hipError_t up2(const float* x, float* y, int c, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_up2, dim3(blocks(size_t(c) * n * n * n)), dim3(256), 0, s, x, y, c, n);
  return hipGetLastError();
}

hipError_t up2_bwd(const float* g, float* gx, int c, int n, hipStream_t s) {
  const size_t h = size_t(n / 2);
  hipLaunchKernelGGL(k_up2_bwd, dim3(blocks(size_t(c) * h * h * h)), dim3(256), 0, s, g, gx, c, n);
  return hipGetLastError();
}

hipError_t pool2_bwd_add(const float* g, const float* add, float* gx, int c, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_pool2_bwd_add, dim3(blocks(size_t(c) * n * n * n)), dim3(256), 0, s, g, add, gx, c, n);
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

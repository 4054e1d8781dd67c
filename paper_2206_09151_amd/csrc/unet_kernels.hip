// gfx950 kernels of the artefact-correction network (a small 3D U-Net; not part of the
// paper's method): 3x3x3 / 1x1x1 convolutions with zero padding, bias and ReLU, their
// input and weight gradients, 2x average pooling, 2x nearest upsampling, the MSE loss
// and Adam.  Weights are the BF16 rounding (nearest even) of the FP32 master parameters;
// activations and gradients are FP32; every sum runs in a fixed order (the loss in FP64),
// so a training step is bitwise reproducible.
//
// Layout: a volume of C channels is stored channel-last.  Element (v, c) of a view (p, s)
// is p[v * s + c] with v = (z n + y) n + x and s the channel count of the buffer, so a
// voxel's channels are one contiguous run (a 16-channel group is one 64-byte line) and a
// channel concatenation is two views at different channel offsets of one wider buffer.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "unet_internal.hpp"

namespace unet {

// ------------------------------------------------------------------ matrix-core convolutions
// The 3x3x3 convolutions run on the matrix cores as implicit GEMMs.  Weights are BF16
// values already; an FP32 activation or gradient v is split into BF16 hi + lo
// (v = hi + lo + e, |e| <= 2^-18 |v|) and both halves are multiplied, so a product carries at
// most that relative error: two products in the forward and input-gradient passes, three
// (hi hi, hi lo, lo hi) in the weight gradient, whose operands are both FP32.
//
// LDS layouts follow one rule: a 64-bit LDS read is served sixteen lanes at a time, so the
// sixteen lanes of a group (the M or N index of the product) read 128 contiguous bytes.
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

// Stage 16 channels [ch0, ch0 + 16) of the input view (x, sx) around the tile into LDS as
// [4 parts][648 halo voxels][8] BF16: part 0 / 1 = hi of channels 0-7 / 8-15, part 2 / 3 =
// lo of the same; with MASK a value is zeroed where the mask view (mask, sm) is <= 0.  Work
// item it = 648 h + hv covers channels 8 h .. 8 h + 7 of halo voxel hv: two 16-byte loads.
// Loads are unconditional (an out-of-range item reads voxel 0 and is zeroed) and issued in
// batches, so that many are in flight.
template <bool MASK>
__device__ __forceinline__ void stage_vox16(unsigned short* xs, const float* x, int sx, int ch0, const float* mask,
                                            int sm, int n, int x0t, int y0t, int z0t) {
  constexpr int ITEMS = 2 * FHV, PER = (ITEMS + 255) / 256, BATCH = MASK ? 2 : 3;
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += BATCH) {
    float4 v[BATCH][2], mk[BATCH][2];
    bool in[BATCH];
#pragma unroll
    for (int kk = 0; kk < BATCH; ++kk) {
      const int it = threadIdx.x + 256 * (k0 + kk);
      const int h = min(it / FHV, 1), hv = it % FHV;
      const int hz = hv / (FHX * FHY), hy = (hv / FHX) % FHY, hx = hv % FHX;
      const int gz = z0t + hz - 1, gy = y0t + hy - 1, gx = x0t + hx - 1;
      in[kk] = k0 + kk < PER && it < ITEMS && unsigned(gz) < unsigned(n) && unsigned(gy) < unsigned(n) &&
               unsigned(gx) < unsigned(n);
      const size_t vox = in[kk] ? (size_t(gz) * n + gy) * n + gx : 0;
      const float4* src = reinterpret_cast<const float4*>(x + vox * sx + ch0 + 8 * h);
      v[kk][0] = src[0];
      v[kk][1] = src[1];
      if (MASK) {
        const float4* ms = reinterpret_cast<const float4*>(mask + vox * sm + ch0 + 8 * h);
        mk[kk][0] = ms[0];
        mk[kk][1] = ms[1];
      }
    }
#pragma unroll
    for (int kk = 0; kk < BATCH; ++kk) {
      const int it = threadIdx.x + 256 * (k0 + kk);
      const float vals[8] = {v[kk][0].x, v[kk][0].y, v[kk][0].z, v[kk][0].w,
                             v[kk][1].x, v[kk][1].y, v[kk][1].z, v[kk][1].w};
      float mks[8];
      if (MASK) {
        mks[0] = mk[kk][0].x; mks[1] = mk[kk][0].y; mks[2] = mk[kk][0].z; mks[3] = mk[kk][0].w;
        mks[4] = mk[kk][1].x; mks[5] = mk[kk][1].y; mks[6] = mk[kk][1].z; mks[7] = mk[kk][1].w;
      }
      unsigned hi[8], lo[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) split_bf16(in[kk] && (!MASK || mks[j] > 0.0f) ? vals[j] : 0.0f, hi[j], lo[j]);
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

// Write a finished tile (16 x 4 x 4 voxels, NB 16-channel blocks) to the output view
// (out, so): the accumulators go through LDS as o[voxel][channel] (voxel stride C + 4
// floats), then each voxel's C channels leave as 16-byte runs.
template <int NB>
__device__ __forceinline__ void store_tile(const f32x4 (&acc)[4][NB], float* o, int wave, int m, int kg, int n,
                                           int x0t, int y0t, int z0t, float* out, int so) {
  constexpr int C = NB * 16, OSC = C + 4, Q = C / 4;
  __syncthreads();
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) o[((wave * 4 + mb) * 16 + 4 * kg + i) * OSC + 16 * nb + m] = acc[mb][nb][i];
  __syncthreads();
  for (int f = threadIdx.x; f < 256 * Q; f += 256) {
    const int vox = f / Q, q = f % Q;
    const int gz = z0t + (vox >> 6), gy = y0t + ((vox >> 4) & 3), gx = x0t + (vox & 15);
    if (gz >= n || gy >= n || gx >= n) continue;
    const f32x4 v = *reinterpret_cast<const f32x4*>(&o[vox * OSC + 4 * q]);
    *reinterpret_cast<f32x4*>(out + ((size_t(gz) * n + gy) * n + gx) * so + 4 * q) = v;
  }
}

// Forward: out[co] = act(b + conv(in)) for cout = 16 NB, cin a multiple of 16; wf holds the
// layer's weights as [cin/16][27][2][cout][8] BF16 (input channel 16 chunk + 8 half + i).
template <int NB>
__global__ __launch_bounds__(256) void k_conv_fwd_mfma(const float* __restrict__ x, int sx, int cin,
                                                       const unsigned short* __restrict__ wf,
                                                       const float* __restrict__ b, float* __restrict__ out, int so,
                                                       int n, int relu) {
  constexpr int XS = 4 * FHV * 8, WS = 27 * NB * 16 * 16;   // shorts
  __shared__ __attribute__((aligned(16))) unsigned short smem[XS + WS];
  unsigned short* xs = smem;
  unsigned short* ws = smem + XS;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  int x0t, y0t, z0t;
  ftile_origin(blockIdx.x, n, x0t, y0t, z0t);
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int ci0 = 0; ci0 < cin; ci0 += 16) {
    __syncthreads();
    stage_vox16<false>(xs, x, sx, ci0, nullptr, 0, n, x0t, y0t, z0t);
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
  store_tile<NB>(acc, reinterpret_cast<float*>(smem), wave, m, kg, n, x0t, y0t, z0t, out, so);
}

// Input gradient: gx[ci] = sum_co sum_t w[co][ci][t] gm[co][r + 1 - t], gm = g (y > 0), for
// cin = 16 NBI and cout a multiple of 16; wd holds the weights as [cout/16][27][2][cin][8]
// BF16 with the taps reversed, so that the product is the same correlation as the forward.
template <int NBI>
__global__ __launch_bounds__(256) void k_conv_bwd_data_mfma(const float* __restrict__ g, int sg,
                                                            const float* __restrict__ y, int sy, int cout,
                                                            const unsigned short* __restrict__ wd,
                                                            float* __restrict__ gx, int sgx, int n) {
  constexpr int XS = 4 * FHV * 8, WS = 27 * NBI * 16 * 16;   // shorts
  __shared__ __attribute__((aligned(16))) unsigned short smem[XS + WS];
  unsigned short* gs = smem;
  unsigned short* ws = smem + XS;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  int x0t, y0t, z0t;
  ftile_origin(blockIdx.x, n, x0t, y0t, z0t);
  f32x4 acc[4][NBI];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NBI; ++nb) acc[mb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int o0 = 0; o0 < cout; o0 += 16) {
    __syncthreads();
    stage_vox16<true>(gs, g, sg, o0, y, sy, n, x0t, y0t, z0t);
    copy_weights(ws, wd + size_t(o0 / 16) * (27 * NBI * 256), 27 * NBI * 256);
    __syncthreads();
    taps_product<NBI>(gs, ws, wave, m, kg, acc);
  }
  store_tile<NBI>(acc, reinterpret_cast<float*>(smem), wave, m, kg, n, x0t, y0t, z0t, gx, sgx);
}

// ---- weight gradient: tiles of 8 x 8 x 4 voxels, halo 10 x 10 x 6.  The reduction runs over
// voxels; the input's halo z range is kept per column as eight z (the six halo z, then 0),
// so a tap's four z (dz .. dz + 3) are cut from a lane's group with a funnel shift for odd
// dz.  K = 32 voxels per v_mfma_f32_16x16x32_bf16: one y-row of the tile plane x 4 z, lane
// group q holding columns 2q, 2q + 1.  LDS layouts:
//   A (masked output gradient), hi and lo planes: [32 column pairs][16 co][2 columns x 4 z],
//     pair stride PA_S shorts;
//   B (layer input), hi and lo planes: [100 halo columns][CI ci][8 z], column stride PB_S.
constexpr int PA_S = 136;           // 128 + 8: staging writes are conflict-free
constexpr int PB_S = 136;           // 16 * 8 + 8, likewise

__host__ __device__ __forceinline__ int wtiles(int n) { return ((n + 7) / 8) * ((n + 7) / 8) * ((n + 3) / 4); }

__device__ __forceinline__ void wtile_origin(int tile, int n, int& x0t, int& y0t, int& z0t) {
  const int ntx = (n + 7) / 8;
  x0t = (tile % ntx) * 8;
  y0t = ((tile / ntx) % ntx) * 8;
  z0t = (tile / (ntx * ntx)) * 4;
}

// A: thread t owns tile column t / 4 (of 64) and channel quad t % 4: four z of four
// channels of the output gradient and of the layer output (the ReLU mask).  Loads are
// unconditional (an out-of-range voxel reads voxel 0) and their values are not touched
// until the tile is stored, so that many stay in flight; validity is kept as a bit mask.
struct ATile {
  float4 g[4], y[4];
  unsigned valid;
};

__device__ __forceinline__ void atile_load(ATile& r, const float* g, int sg, const float* y, int sy, int co0, int n,
                                           int x0t, int y0t, int z0t) {
  const int col = threadIdx.x >> 2, quad = threadIdx.x & 3;
  const int gy = y0t + (col >> 3), gx = x0t + (col & 7);
  r.valid = 0u;
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    const int gz = z0t + z;
    const bool in = gz < n && gy < n && gx < n;
    const size_t vox = in ? (size_t(gz) * n + gy) * n + gx : 0;
    r.g[z] = *reinterpret_cast<const float4*>(g + vox * sg + co0 + 4 * quad);
    r.y[z] = *reinterpret_cast<const float4*>(y + vox * sy + co0 + 4 * quad);
    r.valid |= unsigned(in) << z;
  }
}

// A into LDS (hi, lo); adds the masked gradient to bsum (bias of channels 4 quad + c).
__device__ __forceinline__ void atile_store(const ATile& r, unsigned short* ah, unsigned short* al,
                                            float (&bsum)[4]) {
  const int col = threadIdx.x >> 2, quad = threadIdx.x & 3;
  float v[4][4];   // [channel][z]
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    const bool in = (r.valid >> z) & 1u;
    const float gz4[4] = {r.g[z].x, r.g[z].y, r.g[z].z, r.g[z].w};
    const float yz4[4] = {r.y[z].x, r.y[z].y, r.y[z].z, r.y[z].w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      v[c][z] = in && yz4[c] > 0.0f ? gz4[c] : 0.0f;
      bsum[c] += v[c][z];
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint2 hi, lo;
    split4(v[c], hi, lo);
    const int o = (col >> 1) * PA_S + (4 * quad + c) * 8 + (col & 1) * 4;
    *reinterpret_cast<uint2*>(&ah[o]) = hi;
    *reinterpret_cast<uint2*>(&al[o]) = lo;
  }
}

// B (16 input channels): items it = t + 256 k (it < 400) own halo column it / 4 and channel
// quad it % 4: six z of four channels.
struct BTile {
  float4 x[2][6];
  unsigned valid;
};

__device__ __forceinline__ void btile_load(BTile& r, const float* x, int sx, int ci0, int n, int x0t, int y0t,
                                           int z0t) {
  r.valid = 0u;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int it = threadIdx.x + 256 * k;
    const int cp = min(it >> 2, 99), quad = it & 3;
    const int gy = y0t + cp / 10 - 1, gx = x0t + cp % 10 - 1;
    const bool inc = it < 400 && unsigned(gy) < unsigned(n) && unsigned(gx) < unsigned(n);
#pragma unroll
    for (int hz = 0; hz < 6; ++hz) {
      const int gz = z0t + hz - 1;
      const bool in = inc && unsigned(gz) < unsigned(n);
      const size_t vox = in ? (size_t(gz) * n + gy) * n + gx : 0;
      r.x[k][hz] = *reinterpret_cast<const float4*>(x + vox * sx + ci0 + 4 * quad);
      r.valid |= unsigned(in) << (6 * k + hz);
    }
  }
}

__device__ __forceinline__ void btile_store(const BTile& r, unsigned short* bh, unsigned short* bl) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int it = threadIdx.x + 256 * k;
    if (it >= 400) continue;
    const int cp = it >> 2, quad = it & 3;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      unsigned h[6], l[6];
#pragma unroll
      for (int hz = 0; hz < 6; ++hz) {
        const float4 q4 = r.x[k][hz];
        const float xv = c == 0 ? q4.x : c == 1 ? q4.y : c == 2 ? q4.z : q4.w;
        split_bf16((r.valid >> (6 * k + hz)) & 1u ? xv : 0.0f, h[hz], l[hz]);
      }
      const int o = cp * PB_S + (4 * quad + c) * 8;
      *reinterpret_cast<uint4*>(&bh[o]) = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), 0u);
      *reinterpret_cast<uint4*>(&bl[o]) = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), 0u);
    }
  }
}

// Fixed-order bias sum of the workgroup: thread t holds channels 4 (t % 4) + c; the 64
// threads of a quad are added in column order.
__device__ __forceinline__ void wtile_bias(const float (&bsum)[4], float* red, float* dst) {
#pragma unroll
  for (int c = 0; c < 4; ++c) red[c * 256 + threadIdx.x] = bsum[c];
  __syncthreads();
  if (threadIdx.x < 16) {
    const int co = threadIdx.x, quad = co >> 2, c = co & 3;
    float s = 0.0f;
    for (int j = 0; j < 64; ++j) s += red[c * 256 + 4 * j + quad];
    dst[co] = s;
  }
}

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

// Weight-gradient partials with the taps dealt by column: a wave takes the nine taps of one
// dx over a band of consecutive voxel rows, stepping through the band's halo rows, so that one
// LDS read of a halo row serves the three dy taps of the voxel rows it borders (a window of
// three A rows stays in registers).  The (dx, rows) bands of the four waves:
//   wave 0: dx 0 rows 0-5;  wave 1: dx 0 rows 6-7, dx 1 rows 0-3;
//   wave 2: dx 1 rows 4-7, dx 2 rows 0-1;  wave 3: dx 2 rows 2-7,
// 54 (tap, row) steps each, at most two dx (18 accumulators) per wave, and 192 LDS reads of
// 16 bytes per lane and tile (416 when each wave takes whole (dy, dx) tap groups, whose
// reads serve only their three dz taps: 4.71 against 4.60 ms per training step at 128^3).
// A tap's two partial sums (its lower rows, its upper rows, each over the chunk's tiles in
// order) are added once at the end, lower first.  Two workgroups per CU (72 KB of LDS
// each), so one's tile loads overlap the other's products; the workgroup with ci block 0
// also writes the bias partial pb[chunk][co].
template <int RLO, int RHI>
__device__ __forceinline__ void wgrad_band(f32x4 (&acc)[9], const unsigned short* ah, const unsigned short* al,
                                           const unsigned short* bh, const unsigned short* bl, int dx, int m,
                                           int kg) {
  bf16x8 wa_hi[3], wa_lo[3];   // A rows r % 3 of the window
#pragma unroll
  for (int hr = RLO; hr <= RHI + 2; ++hr) {
    if (hr <= RHI) {
      wa_hi[hr % 3] = lds8(&ah[(4 * hr + kg) * PA_S + m * 8]);
      wa_lo[hr % 3] = lds8(&al[(4 * hr + kg) * PA_S + m * 8]);
    }
    const int o = (hr * 10 + 2 * kg + dx) * PB_S + m * 8;
    const uint4 h0 = *reinterpret_cast<const uint4*>(&bh[o]);
    const uint4 h1 = *reinterpret_cast<const uint4*>(&bh[o + PB_S]);
    const uint4 l0 = *reinterpret_cast<const uint4*>(&bl[o]);
    const uint4 l1 = *reinterpret_cast<const uint4*>(&bl[o + PB_S]);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int r = hr - dy;
      if (r < RLO || r > RHI) continue;
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        // the three products of one (tap, row) step, in the order hi hi, hi lo, lo hi
        const bf16x8 b_hi = zwindow(h0, h1, dz), b_lo = zwindow(l0, l1, dz);
        f32x4& a = acc[3 * dy + dz];
        a = mfma32(wa_hi[r % 3], b_hi, a);
        a = mfma32(wa_hi[r % 3], b_lo, a);
        a = mfma32(wa_lo[r % 3], b_hi, a);
      }
    }
    // one halo row's reads at a time
    __builtin_amdgcn_sched_barrier(0);
  }
}

__global__ __launch_bounds__(256, 2) void k_conv_bwd_w_mfma_cols(const float* __restrict__ x, int sx, int cin,
                                                                 const float* __restrict__ g, int sg,
                                                                 const float* __restrict__ y, int sy, int cout,
                                                                 int n, int tiles_per_chunk, float* __restrict__ pw,
                                                                 float* __restrict__ pb) {
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
  // acc0: the wave's first band (dx = wave), acc1: its second (dx = wave + 1; waves 1 and 2)
  f32x4 acc0[9], acc1[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    acc0[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    acc1[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  float bsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  const int tile_end = min(ntiles, int(blockIdx.x + 1) * tiles_per_chunk);
  for (int tile = blockIdx.x * tiles_per_chunk; tile < tile_end; ++tile) {
    int x0t, y0t, z0t;
    wtile_origin(tile, n, x0t, y0t, z0t);
    // the gradient block is loaded while other waves may still multiply the previous tile;
    // the input block after it, to bound the registers in flight (loading the next tile's
    // blocks during the products instead spills and is slower)
    ATile ra;
    atile_load(ra, g, sg, y, sy, 16 * cb, n, x0t, y0t, z0t);
    __syncthreads();
    atile_store(ra, ah, al, bsum);
    BTile rb;
    btile_load(rb, x, sx, 16 * ib, n, x0t, y0t, z0t);
    btile_store(rb, bh, bl);
    __syncthreads();
    if (wave == 0) {
      wgrad_band<0, 5>(acc0, ah, al, bh, bl, 0, m, kg);
    } else if (wave == 1) {
      wgrad_band<6, 7>(acc0, ah, al, bh, bl, 0, m, kg);
      wgrad_band<0, 3>(acc1, ah, al, bh, bl, 1, m, kg);
    } else if (wave == 2) {
      wgrad_band<4, 7>(acc0, ah, al, bh, bl, 1, m, kg);
      wgrad_band<0, 1>(acc1, ah, al, bh, bl, 2, m, kg);
    } else {
      wgrad_band<2, 7>(acc0, ah, al, bh, bl, 2, m, kg);
    }
  }
  // partials through LDS as part[dx][lower / upper rows][tap j][lane], then tap sums of dx = wave
  f32x4* part = reinterpret_cast<f32x4*>(smem);
  auto slot = [&](int dx, int upper, int j) { return ((dx * 2 + upper) * 9 + j) * 64 + lane; };
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    if (wave == 0) {
      part[slot(0, 0, j)] = acc0[j];
    } else if (wave == 1) {
      part[slot(0, 1, j)] = acc0[j];
      part[slot(1, 0, j)] = acc1[j];
    } else if (wave == 2) {
      part[slot(1, 1, j)] = acc0[j];
      part[slot(2, 0, j)] = acc1[j];
    } else {
      part[slot(2, 1, j)] = acc0[j];
    }
  }
  __syncthreads();
  if (wave < 3) {
    const int dx = wave, ci = 16 * ib + m;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const f32x4 tot = part[slot(dx, 0, j)] + part[slot(dx, 1, j)];
      const int dy = j / 3, dz = j % 3;
      const int tap = 9 * dz + 3 * dy + dx;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = 16 * cb + 4 * kg + i;
        pw[((size_t(blockIdx.x) * cout + co) * cin + ci) * 27 + tap] = tot[i];
      }
    }
  }
  if (ib == 0) {
    __syncthreads();
    wtile_bias(bsum, reinterpret_cast<float*>(smem), pb + size_t(blockIdx.x) * cout + 16 * cb);
  }
}

// Single-input-channel variant (the first layer): the 27 taps (padded to 32) form the N
// dimension of 16x16x16 products (lane l holds A[l%16][4(l/16)..+3], B[4(l/16)..+3][l%16]),
// B[k][tap] = in[v_k + tap - 1], K step = 4 columns x 4 z; wave w takes the steps
// st = w, w + 4, ... and the four waves' sums are added in a fixed order.  The input is a
// plain volume; its halo sits in LDS as [100 halo columns][3 windows][4 z].
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(const bf16x4 a, const bf16x4 b, const f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x4 lds4(const unsigned short* p) { return *reinterpret_cast<const bf16x4*>(p); }

__global__ __launch_bounds__(256) void k_conv_bwd_w_mfma_c1(const float* __restrict__ x,
                                                            const float* __restrict__ g, int sg,
                                                            const float* __restrict__ y, int sy, int cout, int n,
                                                            int tiles_per_chunk, float* __restrict__ pw,
                                                            float* __restrict__ pb) {
  constexpr int BS1 = 12;
  __shared__ __attribute__((aligned(16))) unsigned short ah[32 * PA_S];
  __shared__ __attribute__((aligned(16))) unsigned short al[32 * PA_S];
  __shared__ __attribute__((aligned(16))) unsigned short bh[100 * BS1];
  __shared__ __attribute__((aligned(16))) unsigned short bl[100 * BS1];
  __shared__ float red[4 * 2 * 64 * 4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kg = lane >> 4;
  const int cb = blockIdx.y;
  const int ntiles = wtiles(n);
  int toff[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int tap = min(16 * nb + m, 26);
    toff[nb] = (((tap / 3) % 3) * 10 + tap % 3) * BS1 + 4 * (tap / 9);
  }
  f32x4 acc[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
  float bsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  const int tile_end = min(ntiles, int(blockIdx.x + 1) * tiles_per_chunk);
  for (int tile = blockIdx.x * tiles_per_chunk; tile < tile_end; ++tile) {
    int x0t, y0t, z0t;
    wtile_origin(tile, n, x0t, y0t, z0t);
    ATile ra;
    atile_load(ra, g, sg, y, sy, 16 * cb, n, x0t, y0t, z0t);
    // the input halo column of threads 0..99: six z (unconditional loads, masked later)
    float xv[6];
    unsigned xvalid = 0u;
    {
      const int cp = min(t, 99);
      const int gy = y0t + cp / 10 - 1, gx = x0t + cp % 10 - 1;
      const bool inc = t < 100 && unsigned(gy) < unsigned(n) && unsigned(gx) < unsigned(n);
#pragma unroll
      for (int hz = 0; hz < 6; ++hz) {
        const int gz = z0t + hz - 1;
        const bool in = inc && unsigned(gz) < unsigned(n);
        xv[hz] = x[in ? (size_t(gz) * n + gy) * n + gx : 0];
        xvalid |= unsigned(in) << hz;
      }
    }
    __syncthreads();
    atile_store(ra, ah, al, bsum);
    if (t < 100) {
      unsigned h[6], l[6];
#pragma unroll
      for (int hz = 0; hz < 6; ++hz) split_bf16((xvalid >> hz) & 1u ? xv[hz] : 0.0f, h[hz], l[hz]);
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        *reinterpret_cast<uint2*>(&bh[t * BS1 + 4 * w]) = make_uint2(h[w] | (h[w + 1] << 16), h[w + 2] | (h[w + 3] << 16));
        *reinterpret_cast<uint2*>(&bl[t * BS1 + 4 * w]) = make_uint2(l[w] | (l[w + 1] << 16), l[w + 2] | (l[w + 3] << 16));
      }
    }
    __syncthreads();
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      // K step st = wave + 4 s4 covers columns 4 st .. 4 st + 3 (one x-half of row st / 2);
      // lane group kg takes column 4 st + kg, whose A values sit in pair (4 st + kg) / 2
      const int st = wave + 4 * s4;
      const int col = 4 * st + kg;
      const bf16x4 a_hi = lds4(&ah[(col >> 1) * PA_S + m * 8 + (col & 1) * 4]);
      const bf16x4 a_lo = lds4(&al[(col >> 1) * PA_S + m * 8 + (col & 1) * 4]);
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

// ------------------------------------------------------------------ first layer (one input channel)
// out[v][co] = act(b[co] + sum_t w[co][t] x[v + t - 1]) for cout = 16: one thread per voxel
// (27 input taps, 16 outputs written as four 16-byte runs).
__global__ __launch_bounds__(256) void k_conv_fwd_c1(const float* __restrict__ x,
                                                     const __hip_bfloat16* __restrict__ w,
                                                     const float* __restrict__ b, float* __restrict__ out, int so,
                                                     int n, int relu) {
  __shared__ float ws[27][16];
  for (int i = threadIdx.x; i < 27 * 16; i += 256) ws[i % 27][i / 27] = __bfloat162float(w[i]);   // w[co][tap]
  __syncthreads();
  const unsigned nn = unsigned(n), nv = nn * nn * nn;
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int ix = int(v % nn), iy = int((v / nn) % nn), iz = int(v / (nn * nn));
  float acc[16];
#pragma unroll
  for (int co = 0; co < 16; ++co) acc[co] = b[co];
#pragma unroll 9
  for (int tap = 0; tap < 27; ++tap) {
    const int gz = iz + tap / 9 - 1, gy = iy + (tap / 3) % 3 - 1, gx = ix + tap % 3 - 1;
    const bool in = unsigned(gz) < nn && unsigned(gy) < nn && unsigned(gx) < nn;
    const float xv = in ? x[(size_t(gz) * n + gy) * n + gx] : 0.0f;
#pragma unroll
    for (int co = 0; co < 16; ++co) acc[co] += ws[tap][co] * xv;
  }
  float4* dst = reinterpret_cast<float4*>(out + size_t(v) * so);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float4 r = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
    if (relu) r = make_float4(fmaxf(r.x, 0.0f), fmaxf(r.y, 0.0f), fmaxf(r.z, 0.0f), fmaxf(r.w, 0.0f));
    dst[q] = r;
  }
}

// ------------------------------------------------------------------ 1x1 output layer (cout = 1)
// y[v] = res[v] + b + sum_ci w[ci] x[v][ci]; channels summed in order (cin a multiple of 4).
__global__ void k_conv1x1_fwd(const float* __restrict__ x, int sx, int cin, const __hip_bfloat16* __restrict__ w,
                              const float* __restrict__ b, const float* __restrict__ res, float* __restrict__ y,
                              unsigned nv) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const float4* xv = reinterpret_cast<const float4*>(x + size_t(v) * sx);
  float s = b[0];
  for (int q = 0; q < cin / 4; ++q) {
    const float4 a = xv[q];
    s += __bfloat162float(w[4 * q]) * a.x;
    s += __bfloat162float(w[4 * q + 1]) * a.y;
    s += __bfloat162float(w[4 * q + 2]) * a.z;
    s += __bfloat162float(w[4 * q + 3]) * a.w;
  }
  y[v] = res ? res[v] + s : s;
}

// gx[v][ci] = w[ci] g[v]
__global__ void k_conv1x1_bwd_data(const float* __restrict__ g, const __hip_bfloat16* __restrict__ w, int cin,
                                   float* __restrict__ gx, int sgx, unsigned nv) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const float gv = g[v];
  float4* dst = reinterpret_cast<float4*>(gx + size_t(v) * sgx);
  for (int q = 0; q < cin / 4; ++q)
    dst[q] = make_float4(__bfloat162float(w[4 * q]) * gv, __bfloat162float(w[4 * q + 1]) * gv,
                         __bfloat162float(w[4 * q + 2]) * gv, __bfloat162float(w[4 * q + 3]) * gv);
}

// Weight-gradient partials of the 1x1 layer: pw[chunk][ci] = sum_v g[v] x[v][ci] and
// pb[chunk] = sum_v g[v] over the chunk's voxels (thread-strided sums, then a fixed tree);
// cin <= 16, a multiple of 4.
__global__ __launch_bounds__(256) void k_wgrad1x1(const float* __restrict__ x, int sx, int cin,
                                                  const float* __restrict__ g, unsigned nv, unsigned per,
                                                  float* __restrict__ pw, float* __restrict__ pb) {
  __shared__ float red[17][256];
  float acc[17];
#pragma unroll
  for (int c = 0; c < 17; ++c) acc[c] = 0.0f;
  const unsigned v0 = blockIdx.x * per, v1 = min(nv, v0 + per);
  for (unsigned v = v0 + threadIdx.x; v < v1; v += 256) {
    const float gv = g[v];
    acc[16] += gv;
    const float4* xv = reinterpret_cast<const float4*>(x + size_t(v) * sx);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (4 * q >= cin) break;
      const float4 a = xv[q];
      acc[4 * q] += gv * a.x;
      acc[4 * q + 1] += gv * a.y;
      acc[4 * q + 2] += gv * a.z;
      acc[4 * q + 3] += gv * a.w;
    }
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

// ------------------------------------------------------------------ resampling
// One thread per (voxel, 4-channel quad) of the output; C a multiple of 4, 32-bit indices.
__device__ __forceinline__ float4 f4add(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ __forceinline__ float4 f4scale(float4 a, float s) { return make_float4(a.x * s, a.y * s, a.z * s, a.w * s); }

// y ((n/2)^3) = 2x2x2 average of x (n^3)
__global__ void k_pool2(const float* __restrict__ x, int sx, float* __restrict__ y, int sy, int c, int n) {
  const unsigned h = unsigned(n) / 2, q = unsigned(c) / 4;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= h * h * h * q) return;
  const unsigned qq = i % q, vc = i / q;
  const unsigned xx = vc % h, yy = (vc / h) % h, zz = vc / (h * h), un = unsigned(n);
  float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (unsigned a = 0; a < 2; ++a)
    for (unsigned bq = 0; bq < 2; ++bq)
      for (unsigned cq = 0; cq < 2; ++cq) {
        const size_t v = (size_t(2 * zz + a) * un + 2 * yy + bq) * un + 2 * xx + cq;
        s = f4add(s, *reinterpret_cast<const float4*>(x + v * sx + 4 * qq));
      }
  *reinterpret_cast<float4*>(y + size_t(vc) * sy + 4 * qq) = f4scale(s, 0.125f);
}

// y (n^3) = nearest 2x upsampling of x ((n/2)^3)
__global__ void k_up2(const float* __restrict__ x, int sx, float* __restrict__ y, int sy, int c, int n) {
  const unsigned un = unsigned(n), h = un / 2, q = unsigned(c) / 4;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= un * un * un * q) return;
  const unsigned qq = i % q, v = i / q;
  const unsigned xx = v % un, yy = (v / un) % un, zz = v / (un * un);
  const size_t vc = (size_t(zz / 2) * h + yy / 2) * h + xx / 2;
  *reinterpret_cast<float4*>(y + size_t(v) * sy + 4 * qq) = *reinterpret_cast<const float4*>(x + vc * sx + 4 * qq);
}

// gx ((n/2)^3) = sum of g (n^3) over each 2x2x2 block
__global__ void k_up2_bwd(const float* __restrict__ g, int sg, float* __restrict__ gx, int sgx, int c, int n) {
  const unsigned h = unsigned(n) / 2, q = unsigned(c) / 4;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= h * h * h * q) return;
  const unsigned qq = i % q, vc = i / q;
  const unsigned xx = vc % h, yy = (vc / h) % h, zz = vc / (h * h), un = unsigned(n);
  float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (unsigned a = 0; a < 2; ++a)
    for (unsigned bq = 0; bq < 2; ++bq)
      for (unsigned cq = 0; cq < 2; ++cq) {
        const size_t v = (size_t(2 * zz + a) * un + 2 * yy + bq) * un + 2 * xx + cq;
        s = f4add(s, *reinterpret_cast<const float4*>(g + v * sg + 4 * qq));
      }
  *reinterpret_cast<float4*>(gx + size_t(vc) * sgx + 4 * qq) = s;
}

// gx (n^3) = g ((n/2)^3) / 8 at the coarse voxel + add (n^3)
__global__ void k_pool2_bwd_add(const float* __restrict__ g, int sg, const float* __restrict__ add, int sa,
                                float* __restrict__ gx, int sgx, int c, int n) {
  const unsigned un = unsigned(n), h = un / 2, q = unsigned(c) / 4;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= un * un * un * q) return;
  const unsigned qq = i % q, v = i / q;
  const unsigned xx = v % un, yy = (v / un) % un, zz = v / (un * un);
  const size_t vc = (size_t(zz / 2) * h + yy / 2) * h + xx / 2;
  const float4 a = f4scale(*reinterpret_cast<const float4*>(g + vc * sg + 4 * qq), 0.125f);
  const float4 b = *reinterpret_cast<const float4*>(add + size_t(v) * sa + 4 * qq);
  *reinterpret_cast<float4*>(gx + size_t(v) * sgx + 4 * qq) = f4add(a, b);
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

hipError_t conv_fwd(int ks, const float* x, int sx, int cin, const __hip_bfloat16* w, const unsigned short* wf,
                    const float* b, float* out, int so, int cout, int n, int relu, const float* res, hipStream_t s) {
  if (ks == 3 && cin == 1 && cout == 16 && !res) {
    hipLaunchKernelGGL(k_conv_fwd_c1, dim3(blocks(size_t(n) * n * n)), dim3(256), 0, s, x, w, b, out, so, n, relu);
    return hipGetLastError();
  }
  if (wf && mfma_layer(ks, cin, cout) && cin % 16 == 0 && !res) {
    const dim3 grid(unsigned(ftiles(n)));
    switch (cout / 16) {
      case 1: hipLaunchKernelGGL(k_conv_fwd_mfma<1>, grid, dim3(256), 0, s, x, sx, cin, wf, b, out, so, n, relu); break;
      case 2: hipLaunchKernelGGL(k_conv_fwd_mfma<2>, grid, dim3(256), 0, s, x, sx, cin, wf, b, out, so, n, relu); break;
      case 4: hipLaunchKernelGGL(k_conv_fwd_mfma<4>, grid, dim3(256), 0, s, x, sx, cin, wf, b, out, so, n, relu); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (ks == 1 && cout == 1 && cin % 4 == 0 && !relu) {
    const unsigned nv = unsigned(n) * unsigned(n) * unsigned(n);
    hipLaunchKernelGGL(k_conv1x1_fwd, dim3(blocks(nv)), dim3(256), 0, s, x, sx, cin, w, b, res, out, nv);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;   // not a layer of this network
}

hipError_t conv_bwd_data(int ks, const float* g, int sg, const float* y, int sy, int cout, const __hip_bfloat16* w,
                         const unsigned short* wd, float* gx, int sgx, int cin, int n, hipStream_t s) {
  if (wd && y && mfma_layer(ks, cin, cout) && cin % 16 == 0) {   // the matrix-core kernels take the ReLU mask
    const dim3 grid(unsigned(ftiles(n)));
    switch (cin / 16) {
      case 1: hipLaunchKernelGGL(k_conv_bwd_data_mfma<1>, grid, dim3(256), 0, s, g, sg, y, sy, cout, wd, gx, sgx, n); break;
      case 2: hipLaunchKernelGGL(k_conv_bwd_data_mfma<2>, grid, dim3(256), 0, s, g, sg, y, sy, cout, wd, gx, sgx, n); break;
      case 3: hipLaunchKernelGGL(k_conv_bwd_data_mfma<3>, grid, dim3(256), 0, s, g, sg, y, sy, cout, wd, gx, sgx, n); break;
      case 4: hipLaunchKernelGGL(k_conv_bwd_data_mfma<4>, grid, dim3(256), 0, s, g, sg, y, sy, cout, wd, gx, sgx, n); break;
      case 6: hipLaunchKernelGGL(k_conv_bwd_data_mfma<6>, grid, dim3(256), 0, s, g, sg, y, sy, cout, wd, gx, sgx, n); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (ks == 1 && cout == 1 && !y && cin % 4 == 0) {
    const unsigned nv = unsigned(n) * unsigned(n) * unsigned(n);
    hipLaunchKernelGGL(k_conv1x1_bwd_data, dim3(blocks(nv)), dim3(256), 0, s, g, w, cin, gx, sgx, nv);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

// Chunking of the weight-gradient reduction: about 1024 (2048 for the single-channel kernel)
// workgroups over the (co, ci) block pairs, every chunk holding at least one tile; 1024
// voxel ranges for the 1x1 layer.
static void wgrad_split(int ks, int cin, int cout, int n, int& chunks, int& per) {
  if (ks == 1) {
    const size_t nv = size_t(n) * n * n;
    chunks = int(std::max<size_t>(1, std::min<size_t>(1024, (nv + 255) / 256)));
    per = int((nv + size_t(chunks) - 1) / size_t(chunks));
    chunks = int((nv + size_t(per) - 1) / size_t(per));
    return;
  }
  const int ntiles = wtiles(n);
  const int pairs = (cout / 16) * (cin == 1 ? 1 : cin / 16);
  const int wgs = cin == 1 ? 2048 : 1024;
  const int target = (wgs + pairs - 1) / pairs;
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

hipError_t conv_bwd_w(int ks, const float* x, int sx, int cin, const float* g, int sg, const float* y, int sy,
                      int cout, int n, float* pw, float* pb, float* q, float* gw, float* gb, hipStream_t s) {
  int chunks, per;
  wgrad_split(ks, cin, cout, n, chunks, per);
  const int nw = cout * cin * ks * ks * ks;
  if (ks == 3 && y && cin == 1 && cout % 16 == 0) {
    hipLaunchKernelGGL(k_conv_bwd_w_mfma_c1, dim3(unsigned(chunks), unsigned(cout / 16)), dim3(256), 0, s, x, g, sg,
                       y, sy, cout, n, per, pw, pb);
  } else if (ks == 3 && y && mfma_layer(ks, cin, cout) && cin % 16 == 0) {
    hipLaunchKernelGGL(k_conv_bwd_w_mfma_cols, dim3(unsigned(chunks), unsigned((cout / 16) * (cin / 16))), dim3(256),
                       0, s, x, sx, cin, g, sg, y, sy, cout, n, per, pw, pb);
  } else if (ks == 1 && cout == 1 && cin <= 16 && cin % 4 == 0 && !y) {
    const unsigned nv = unsigned(n) * unsigned(n) * unsigned(n);
    hipLaunchKernelGGL(k_wgrad1x1, dim3(unsigned(chunks)), dim3(256), 0, s, x, sx, cin, g, nv, unsigned(per), pw, pb);
  } else {
    return hipErrorInvalidValue;
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

hipError_t pool2(const float* x, int sx, float* y, int sy, int c, int n, hipStream_t s) {
  const size_t h = size_t(n / 2);
  hipLaunchKernelGGL(k_pool2, dim3(blocks(h * h * h * (c / 4))), dim3(256), 0, s, x, sx, y, sy, c, n);
  return hipGetLastError();
}

hipError_t up2(const float* x, int sx, float* y, int sy, int c, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_up2, dim3(blocks(size_t(n) * n * n * (c / 4))), dim3(256), 0, s, x, sx, y, sy, c, n);
  return hipGetLastError();
}

hipError_t up2_bwd(const float* g, int sg, float* gx, int sgx, int c, int n, hipStream_t s) {
  const size_t h = size_t(n / 2);
  hipLaunchKernelGGL(k_up2_bwd, dim3(blocks(h * h * h * (c / 4))), dim3(256), 0, s, g, sg, gx, sgx, c, n);
  return hipGetLastError();
}

hipError_t pool2_bwd_add(const float* g, int sg, const float* add, int sa, float* gx, int sgx, int c, int n,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_pool2_bwd_add, dim3(blocks(size_t(n) * n * n * (c / 4))), dim3(256), 0, s, g, sg, add, sa, gx,
                     sgx, c, n);
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

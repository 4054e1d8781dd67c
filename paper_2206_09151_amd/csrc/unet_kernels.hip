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

__global__ void k_mse_final(const double* __restrict__ part, int nparts, size_t count, double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < nparts; ++k) s += part[k];
  loss[0] = s / double(count);
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

hipError_t conv_fwd(int ks, const float* x0, int c0, const float* x1, int cin, const __hip_bfloat16* w,
                    const float* b, float* out, int cout, int n, int relu, const float* res, hipStream_t s) {
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
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, part, int(nb), count, loss);
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

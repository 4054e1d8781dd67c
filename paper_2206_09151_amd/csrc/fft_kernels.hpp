// Spectra and depth-plane kernels of the reconstruction for every supported detector
// size M (all 2,3,5-smooth M in [16, 256]), as templates; each size is instantiated in
// exactly one of the fft_sizes_*.hip translation units, which register a launcher for
// it in the size table of tomo_kernels.hip.
//
//   k_spectra   per view: g = ln(I/I_in) (eq. 4 left side), 2D DFT (F2 of Section 2,
//               kernel exp(-i 2 pi r.q)), multiplied by the plan's filter table so
//               that the Hermitian split needed below is ready:
//                 Q1 = (1+i) F_h G / M^2,   Q2 = -(1+i) F_a G / M^2,
//               F = C W H (eq. 11), F_h / F_a its Hermitian / anti-Hermitian parts.
//   k_planes    per view and plane pair (j, K-1-j): the planes' spectra are
//               Y_j = Herm[F e^{-i phi_j} G], phi_j = pi lambda z'_j q^2 (eq. 3 on the
//               paraboloid of eqs. 8/10).  Since z'_{K-1-j} = -z'_j,
//                 Y_j + i Y_{K-1-j} = cos(phi_j) Q1 + sin(phi_j) Q2,
//               and one complex inverse 2D FFT yields plane j (real part) and plane
//               K-1-j (imaginary part).  Writes the stack [view][row][plane][col].
//   k_spectra_split / k_planes_split: the same as P^2 independent H x H transforms,
//               M = P H: for M > 200, whose M x M block does not fit in one CU's LDS, and
//               for 162, 180 and 200, whose direct transforms would need R1 = 27 to 40
//               values per thread in registers and spill at the 1000-thread workgroup.
//   k_planes_rows: the planes of 160, 192 and 256 as P blocks of whole output rows.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fft.hpp"

namespace tomo {

// ------------------------------------------------------------------ FFT shapes
// M = R1 * R2 with M * R2 <= 1024 threads; R1 values per thread in registers.
template <int M>
struct Shape;
template <> struct Shape<16> : Fft2Shape<16, 4, 4> {};
template <> struct Shape<18> : Fft2Shape<18, 6, 3> {};
template <> struct Shape<20> : Fft2Shape<20, 5, 4> {};
template <> struct Shape<24> : Fft2Shape<24, 6, 4> {};
template <> struct Shape<25> : Fft2Shape<25, 5, 5> {};
template <> struct Shape<27> : Fft2Shape<27, 9, 3> {};
template <> struct Shape<30> : Fft2Shape<30, 6, 5> {};
template <> struct Shape<32> : Fft2Shape<32, 8, 4> {};
template <> struct Shape<36> : Fft2Shape<36, 6, 6> {};
template <> struct Shape<40> : Fft2Shape<40, 10, 4> {};
template <> struct Shape<45> : Fft2Shape<45, 9, 5> {};
template <> struct Shape<48> : Fft2Shape<48, 12, 4> {};
template <> struct Shape<50> : Fft2Shape<50, 10, 5> {};
template <> struct Shape<54> : Fft2Shape<54, 9, 6> {};
template <> struct Shape<60> : Fft2Shape<60, 10, 6> {};
template <> struct Shape<64> : Fft2Shape<64, 16, 4> {};
template <> struct Shape<72> : Fft2Shape<72, 12, 6> {};
template <> struct Shape<75> : Fft2Shape<75, 15, 5> {};
template <> struct Shape<80> : Fft2Shape<80, 20, 4> {};
template <> struct Shape<81> : Fft2Shape<81, 9, 9> {};
template <> struct Shape<90> : Fft2Shape<90, 15, 6> {};
template <> struct Shape<96> : Fft2Shape<96, 24, 4> {};
template <> struct Shape<100> : Fft2Shape<100, 10, 10> {};
template <> struct Shape<108> : Fft2Shape<108, 18, 6> {};
template <> struct Shape<120> : Fft2Shape<120, 24, 5> {};
template <> struct Shape<125> : Fft2Shape<125, 25, 5> {};
template <> struct Shape<128> : Fft2Shape<128, 16, 8> {};
template <> struct Shape<135> : Fft2Shape<135, 27, 5> {};
template <> struct Shape<144> : Fft2Shape<144, 24, 6> {};
template <> struct Shape<150> : Fft2Shape<150, 30, 5> {};
template <> struct Shape<160> : Fft2Shape<160, 40, 4> {};
template <> struct Shape<192> : Fft2Shape<192, 48, 4> {};

// Exchanges through half-size LDS (real, then imaginary parts): in the plane kernels
// where the full block would leave room for only one workgroup per CU (two fit then),
// in the spectra kernel only where the full block would not fit in one CU's LDS.
template <int M>
constexpr bool kSplit = (Shape<M>::LDS_BYTES > 80 * 1024);
template <int M>
constexpr bool kSplitSpectra = (Shape<M>::LDS_BYTES > 160 * 1024);

// ------------------------------------------------------------------ plane storage types
// FP32, BF16 (round to nearest even), FP16 (per-view power-of-two scale).
template <class T>
__device__ __forceinline__ T to_store(float v);
template <>
__device__ __forceinline__ float to_store<float>(float v) { return v; }
template <>
__device__ __forceinline__ __hip_bfloat16 to_store<__hip_bfloat16>(float v) { return __float2bfloat16(v); }
template <>
__device__ __forceinline__ __half to_store<__half>(float v) { return __float2half_rn(v); }

template <class T>
__device__ __forceinline__ float from_store(T v);
template <>
__device__ __forceinline__ float from_store<float>(float v) { return v; }
template <>
__device__ __forceinline__ float from_store<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }
template <>
__device__ __forceinline__ float from_store<__half>(__half v) { return __half2float(v); }

// Filtered spectrum (Q1, Q2) of one coefficient: the filter table entry f times G.
__device__ __forceinline__ float4 filtered(const float4 f, const float2 gg) {
  float4 o;
  o.x = f.x * gg.x - f.y * gg.y;
  o.y = f.x * gg.y + f.y * gg.x;
  o.z = f.z * gg.x - f.w * gg.y;
  o.w = f.z * gg.y + f.w * gg.x;
  return o;
}

// FP16 plane scale: the power of two that puts a view's spectral bound at 2^14.
__device__ __forceinline__ float fp16_scale(float l1) { return l1 > 0.0f ? exp2f(14.0f - ceilf(log2f(l1))) : 1.0f; }

// ------------------------------------------------------------------ K1: spectra
template <int M>
__global__ __launch_bounds__(Shape<M>::T) void k_spectra(const float* __restrict__ images,
                                                         const float4* __restrict__ filt,
                                                         const float2* __restrict__ tw_fwd,
                                                         float4* __restrict__ q, int* __restrict__ status,
                                                         double inv_iin, float* __restrict__ scale) {
  using S = Shape<M>;
  __shared__ float2 lds[kSplitSpectra<M> ? (S::LDS_SPLIT_FLOATS + 1) / 2 : S::LDS_ELEMS];
  __shared__ float red[(S::T + 63) / 64];
  const int t = threadIdx.x;
  const int view = blockIdx.x;
  const int line = t % M, r = t / M;
  const float* img = images + size_t(view) * M * M;
  float2 x[S::XN];
  int bad = 0;
#pragma unroll
  for (int m = 0; m < S::R1; ++m) {
    const float iv = img[(r + S::R2 * m) * M + line];
    const bool ok = (iv > 0.0f) && (iv < INFINITY);
    bad |= !ok;
    // contrast in FP64, rounded once: ln(I/I_in) of an FP32 intensity near I_in
    const double g = ok ? log(double(iv) * inv_iin) : 0.0;
    x[m] = make_float2(float(g), 0.0f);
  }
  if (bad) atomicOr(status, 1);
  if constexpr (kSplitSpectra<M>) fft2_block_split<S, false>(x, reinterpret_cast<float*>(lds), tw_fwd);
  else fft2_block<S, false>(x, lds, tw_fwd);
  const int sg = t % S::R2, ky = t / S::R2;
  const size_t row = (size_t(view) * M + ky) * M;
  float l1 = 0.0f;
#pragma unroll
  for (int e = 0; e < S::E; ++e) {
    if (!S::has_s(sg * S::E + e)) continue;
#pragma unroll
    for (int k2 = 0; k2 < S::R2; ++k2) {
      const int kx = sg * S::E + e + S::R1 * k2;
      const float4 o = filtered(filt[row + kx], x[e * S::R2 + k2]);
      q[row + kx] = o;
      l1 += fabsf(o.x) + fabsf(o.y) + fabsf(o.z) + fabsf(o.w);
    }
  }
  if (scale) {
    // FP16 plane storage: every plane value of this view is bounded by
    // sum_k |cos Q1 + sin Q2| <= sum_k (|Q1| + |Q2|) <= l1; scale by the power of two that
    // puts this bound at 2^14 (exact scaling, values stay below the FP16 maximum).
    // Fixed-order reduction: wave sums, then the wave partials in order.
    for (int off = 32; off > 0; off >>= 1) l1 += __shfl_xor(l1, off, 64);
    if ((t & 63) == 0) red[t >> 6] = l1;
    __syncthreads();
    if (t == 0) {
      float tot = 0.0f;
      for (int w = 0; w < (S::T + 63) / 64; ++w) tot += red[w];
      scale[view] = fp16_scale(tot);
    }
  }
}

// ------------------------------------------------------------------ K3: planes
// Workgroup -> (view, pair) mapping keeps all pairs of one view on one XCD
// (workgroups are dealt to the 8 XCDs round robin), so the view's Q block is
// fetched into one L2 only.
template <int M, class OutT>
__global__ __launch_bounds__(Shape<M>::T) void k_planes(const float4* __restrict__ q,
                                                        const float2* __restrict__ prop,
                                                        const float2* __restrict__ tw_inv,
                                                        OutT* __restrict__ stack, int K, int npairs,
                                                        int nb, const float* __restrict__ scale) {
  using S = Shape<M>;
  __shared__ float2 lds[kSplit<M> ? (S::LDS_SPLIT_FLOATS + 1) / 2 : S::LDS_ELEMS];
  const int wg = blockIdx.x;
  const int xcd = wg & 7, k = wg >> 3;
  int view, p;
  if (nb == 1 || nb == 2 || nb == 4) {
    // fewer views than XCDs: view xcd % nb, its pairs dealt over the 8 / nb XCDs that share it
    view = xcd % nb;
    p = k * (8 / nb) + xcd / nb;
    if (p >= npairs) return;  // whole workgroup leaves together: no barrier is skipped by part of it
  } else {
    view = xcd + 8 * int(unsigned(k) / unsigned(npairs));
    p = int(unsigned(k) % unsigned(npairs));
    if (view >= nb) return;
  }
  const int t = threadIdx.x;
  const int line = t % M;
  int r_;
  if constexpr (M % 64 == 0) r_ = __builtin_amdgcn_readfirstlane(t / M);
  else r_ = t / M;
  const int r = r_;
  const float4* qv = q + size_t(view) * M * M;
  const float2* pr = prop + size_t(p) * M;
  const float2 cx = pr[line];
  float2 x[S::XN];
#pragma unroll
  for (int m = 0; m < S::R1; ++m) {
    const int ky = r + S::R2 * m;
    const float2 cy = pr[ky];
    const float c = cx.x * cy.x - cx.y * cy.y;   // cos(phi_x + phi_y)
    const float sn = cx.y * cy.x + cx.x * cy.y;  // sin(phi_x + phi_y)
    const float4 qq = qv[ky * M + line];
    x[m] = make_float2(c * qq.x + sn * qq.z, c * qq.y + sn * qq.w);
  }
  // FP16 planes: per-view power-of-two scale (other storage types are not scaled), read
  // before the transform so that its latency overlaps the spectrum loads; the empty asm
  // keeps the compiler from sinking the read to the stores, where its wait would also
  // wait for the last exchange's LDS reads
  float sc = 1.0f;
  if constexpr (std::is_same<OutT, __half>::value) {
    sc = scale[view];
    asm volatile("" : "+v"(sc));
  }
  if constexpr (kSplit<M>) fft2_block_split<S, true>(x, reinterpret_cast<float*>(lds), tw_inv);
  else fft2_block<S, true>(x, lds, tw_inv);
  const int sg = t % S::R2, y = t / S::R2;
  const int pa = p, pb = K - 1 - p;
  OutT* rowa = stack + ((size_t(view) * M + y) * K + pa) * M;
  OutT* rowb = stack + ((size_t(view) * M + y) * K + pb) * M;
#pragma unroll
  for (int k2 = 0; k2 < S::R2; ++k2) {
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      if (!S::has_s(sg * S::E + e)) continue;
      const int xc = sg * S::E + e + S::R1 * k2;
      rowa[xc] = to_store<OutT>(x[e * S::R2 + k2].x * sc);
    }
  }
  if (pb != pa) {
#pragma unroll
    for (int k2 = 0; k2 < S::R2; ++k2) {
#pragma unroll
      for (int e = 0; e < S::E; ++e) {
        if (!S::has_s(sg * S::E + e)) continue;
        const int xc = sg * S::E + e + S::R1 * k2;
        rowb[xc] = to_store<OutT>(x[e * S::R2 + k2].y * sc);
      }
    }
  }
}

// ------------------------------------------------------------------ row-split plane kernels
// For M = 160, 192 and 256, whose direct transforms hold 40 / 48 values per thread (160: with
// spills) or whose block does not fit in one CU's LDS (256): a radix-P decimation in
// frequency on the row index only splits the M x M inverse transform into P blocks of
// H x M (H = M / P):
//   X[P k1 + p1][k2] = DFT_{H x M}(n1, n2) { w_M^(p1 n1) sum_{a<P} w_P^(a p1) x[n1 + H a][n2] }
// Workgroup (view, pair, p1) computes the output rows P k1 + p1: the input terms are formed
// P times per coefficient (not P^2 times as in the P x P split), and every workgroup writes
// whole rows.  Measured per view of a single-axis scan: 160 (P = 2, 16 values per thread,
// one workgroup per CU): 14.6 us against 20.6 direct and 17.2 with P = 4; 192 (P = 4,
// 12 values, two workgroups per CU): 15.6 against 19.1 direct and 17.4 with P = 2; 256
// (P = 2, 32 values, one workgroup per CU): 300 us per 8-view launch against 308 with P = 4
// (two workgroups per CU, but twice the input terms) and 357 for the 2 x 2 block split.
template <int M>
struct RowSplit;
template <> struct RowSplit<160> : RectShape<80, 16, 5, 160, 16, 10> {};   // 800 threads
template <> struct RowSplit<192> : RectShape<48, 12, 4, 192, 12, 16> {};   // 768 threads
template <> struct RowSplit<256> : RectShape<128, 32, 4, 256, 32, 8> {};   // 1024 threads

// Block p1's input of a row-split plane kernel: x[m] = w_M^(p1 n1) sum_a w_P^(a p1)
// Y[n1 + H a][n2], n1 = r + R2C m, Y = cos(phi) Q1 + sin(phi) Q2 (phi = phi_x + phi_y);
// P1 a compile-time block index.
template <class S, int M, int P1>
__device__ __forceinline__ void rows_input(const float4* __restrict__ qv, const float2* __restrict__ pr,
                                           const float2* __restrict__ tw, int r, int n2, float2 (&x)[S::XN]) {
  constexpr int P = S::P, H = S::MC;
  const float2 cx = pr[n2];
#pragma unroll
  for (int m = 0; m < S::R1C; ++m) {
    const int n1 = r + S::R2C * m;
    float2 acc = make_float2(0.0f, 0.0f);
    StaticFor<0, P>::run([&](auto ca) {
      constexpr int a = decltype(ca)::value;
      const float2 cy = pr[n1 + H * a];
      const float c = cx.x * cy.x - cx.y * cy.y;   // cos(phi_x + phi_y)
      const float sn = cx.y * cy.x + cx.x * cy.y;  // sin(phi_x + phi_y)
      const float4 qq = qv[(n1 + H * a) * M + n2];
      const float2 z = make_float2(c * qq.x + sn * qq.z, c * qq.y + sn * qq.w);
      if constexpr (a == 0) acc = z;
      else if constexpr (P == 2 || P == 4) acc = cadd(acc, rot<P, a * P1, true>(z));   // exact: 1, +i, -1, -i
      else acc = cadd(acc, cmul(z, tw[H * ((a * P1) % P)]));                              // w_P^(a p1) = w_M^(H a p1)
    });
    if constexpr (P1 == 0) x[m] = acc;
    else x[m] = cmul(acc, tw[(P1 * n1) % M]);
  }
}

template <int M, class OutT>
__global__ __launch_bounds__(RowSplit<M>::T) void k_planes_rows(const float4* __restrict__ q,
                                                                 const float2* __restrict__ prop,
                                                                 const float2* __restrict__ tw,
                                                                 OutT* __restrict__ stack, int K, int npairs,
                                                                 int nb, const float* __restrict__ scale) {
  using S = RowSplit<M>;
  constexpr int P = S::P, H = S::MC;
  static_assert(P == 2 || P == 4, "block coefficients of P = 2 and 4 only");
  __shared__ float lds[S::LDS_FLOATS];
  const int wg = blockIdx.x;
  const int xcd = wg & 7, k = wg >> 3;
  const unsigned per_view = unsigned(npairs) * P;
  int view;
  unsigned rem;
  if (nb == 1 || nb == 2 || nb == 4) {
    // fewer views than XCDs: view xcd % nb, its (pair, block) units dealt over the 8 / nb XCDs
    view = xcd % nb;
    rem = unsigned(k) * unsigned(8 / nb) + unsigned(xcd / nb);
    if (rem >= per_view) return;   // whole workgroup leaves together
  } else {
    view = xcd + 8 * int(unsigned(k) / per_view);
    rem = unsigned(k) % per_view;
    if (view >= nb) return;        // whole workgroup leaves together
  }
  const int p = int(rem / P), p1 = int(rem % P);
  const int t = threadIdx.x;
  const int n2 = t % M;
  int r_;
  if constexpr (M % 64 == 0) r_ = __builtin_amdgcn_readfirstlane(t / M);
  else r_ = t / M;
  const int r = r_;
  const float4* qv = q + size_t(view) * M * M;
  const float2* pr = prop + size_t(p) * M;
  float2 x[S::XN];
  if constexpr (P == 4) {
    // the block's quarter turns as operand swaps: one instantiation per block
    switch (p1) {   // uniform across the workgroup
      case 0: rows_input<S, M, 0>(qv, pr, tw, r, n2, x); break;
      case 1: rows_input<S, M, 1>(qv, pr, tw, r, n2, x); break;
      case 2: rows_input<S, M, 2>(qv, pr, tw, r, n2, x); break;
      default: rows_input<S, M, 3>(qv, pr, tw, r, n2, x); break;
    }
  } else {
    // P = 2: the block's sign is a select (one instantiation keeps the registers low)
    const float2 cx = pr[n2];
#pragma unroll
    for (int m = 0; m < S::R1C; ++m) {
      const int n1 = r + S::R2C * m;
      float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const float2 cy = pr[n1 + H * a];
        const float c = cx.x * cy.x - cx.y * cy.y;   // cos(phi_x + phi_y)
        const float sn = cx.y * cy.x + cx.x * cy.y;  // sin(phi_x + phi_y)
        const float4 qq = qv[(n1 + H * a) * M + n2];
        const float2 z = make_float2(c * qq.x + sn * qq.z, c * qq.y + sn * qq.w);
        if (a == 0) acc = z;
        else acc = p1 ? csub(acc, z) : cadd(acc, z);   // w_2^(a p1) = (-1)^(a p1)
      }
      x[m] = p1 == 0 ? acc : cmul(acc, tw[(p1 * n1) % M]);
    }
  }
  // FP16 planes: per-view power-of-two scale, read before the transform (see k_planes)
  float sc = 1.0f;
  if constexpr (std::is_same<OutT, __half>::value) {
    sc = scale[view];
    asm volatile("" : "+v"(sc));
  }
  fft2_rect_split<S, true>(x, lds, tw);
  const int sg = t % S::R2R, y = t / S::R2R;
  const int row = P * y + p1;
  const int pa = p, pb = K - 1 - p;
  OutT* rowa = stack + ((size_t(view) * M + row) * K + pa) * M;
  OutT* rowb = stack + ((size_t(view) * M + row) * K + pb) * M;
#pragma unroll
  for (int k2 = 0; k2 < S::R2R; ++k2) {
#pragma unroll
    for (int e = 0; e < S::ER; ++e) {
      if (!S::has_r(sg * S::ER + e)) continue;
      rowa[sg * S::ER + e + S::R1R * k2] = to_store<OutT>(x[e * S::R2R + k2].x * sc);
    }
  }
  if (pb != pa) {
#pragma unroll
    for (int k2 = 0; k2 < S::R2R; ++k2) {
#pragma unroll
      for (int e = 0; e < S::ER; ++e) {
        if (!S::has_r(sg * S::ER + e)) continue;
        rowb[sg * S::ER + e + S::R1R * k2] = to_store<OutT>(x[e * S::R2R + k2].y * sc);
      }
    }
  }
}

// ------------------------------------------------------------------ M = P H (162, 180, 200, 216 ... 256; the planes of 256 use the row split)
// An M x M block with M > 200 does not fit in one CU's LDS.  One radix-P decimation in
// frequency on both axes splits it into P^2 independent H x H transforms:
//   X[P k1 + p1][P k2 + p2] = DFT_H(n1,n2) { w_M^(p1 n1 + p2 n2) sum_{a,b<P} w_P^(a p1 + b p2) x[n1 + H a][n2 + H b] }
// with w_M = exp(-+ i 2 pi / M) and w_P = w_M^H.  Each block (p1, p2) is one workgroup
// running the H x H LDS transform; it reads its inputs from all P^2 input blocks and
// writes every P-th output row and column.  The P^2 workgroups of a transform share an XCD.

// w_P^(k) for k < P from the M-point twiddle table; P = 2 needs only a sign.
template <int P>
__device__ __forceinline__ float2 split_coef(const float2* __restrict__ tw, int H, int k) {
  if constexpr (P == 2) return make_float2(k ? -1.0f : 1.0f, 0.0f);
  else return tw[H * k];
}

// g = ln(I/I_in) of an M x M image -> filtered spectra (Q1, Q2) at the block's output
// positions; l1part[view][block] = partial spectral bound for the FP16 scale.
template <int H, int P>
__global__ __launch_bounds__(Shape<H>::T) void k_spectra_split(const float* __restrict__ images,
                                                              const float4* __restrict__ filt,
                                                              const float2* __restrict__ tw_m,
                                                              const float2* __restrict__ tw_h,
                                                              float4* __restrict__ q, int* __restrict__ status,
                                                              double inv_iin, float* __restrict__ l1part) {
  using S = Shape<H>;
  constexpr int M = P * H;
  __shared__ float2 lds[(S::LDS_SPLIT_FLOATS + 1) / 2];
  __shared__ float red[(S::T + 63) / 64];
  const int t = threadIdx.x;
  const int view = int(blockIdx.x / (P * P));
  const unsigned blk = blockIdx.x % (P * P);
  const int p1 = int(blk / P), p2 = int(blk % P);
  const int n2 = t % H;
  int r_;   // uniform across a wave when H is a multiple of the wave size
  if constexpr (H % 64 == 0) r_ = __builtin_amdgcn_readfirstlane(t / H);
  else r_ = t / H;
  const int r = r_;
  const float* img = images + size_t(view) * M * M;
  float2 x[S::XN];
  int bad = 0;
#pragma unroll
  for (int m = 0; m < S::R1; ++m) {
    const int n1 = r + S::R2 * m;
    float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
      for (int b = 0; b < P; ++b) {
        const float iv = img[(n1 + H * a) * M + n2 + H * b];
        const bool ok = (iv > 0.0f) && (iv < INFINITY);
        bad |= !ok;
        const float g = ok ? float(log(double(iv) * inv_iin)) : 0.0f;
        const float2 w = split_coef<P>(tw_m, H, (a * p1 + b * p2) % P);
        acc.x += w.x * g;
        acc.y += w.y * g;
      }
    }
    const int ti = p1 * n1 + p2 * n2;   // < 2M
    x[m] = cmul(acc, tw_m[ti >= M ? ti - M : ti]);
  }
  if (bad) atomicOr(status, 1);
  fft2_block_split<S, false>(x, reinterpret_cast<float*>(lds), tw_h);
  const int sg = t % S::R2, yy = t / S::R2;
  const int ky = P * yy + p1;
  const size_t row = (size_t(view) * M + ky) * M;
  float l1 = 0.0f;
#pragma unroll
  for (int e = 0; e < S::E; ++e) {
    if (!S::has_s(sg * S::E + e)) continue;
#pragma unroll
    for (int k2 = 0; k2 < S::R2; ++k2) {
      const int kx = P * (sg * S::E + e + S::R1 * k2) + p2;
      const float4 o = filtered(filt[row + kx], x[e * S::R2 + k2]);
      q[row + kx] = o;
      l1 += fabsf(o.x) + fabsf(o.y) + fabsf(o.z) + fabsf(o.w);
    }
  }
  if (l1part) {
    for (int off = 32; off > 0; off >>= 1) l1 += __shfl_xor(l1, off, 64);
    if ((t & 63) == 0) red[t >> 6] = l1;
    __syncthreads();
    if (t == 0) {
      float tot = 0.0f;
      for (int w = 0; w < (S::T + 63) / 64; ++w) tot += red[w];
      l1part[blockIdx.x] = tot;
    }
  }
}

// FP16 plane scale of each view from its P^2 block bounds (fixed summation order).
template <int P>
__global__ void k_scale_split(const float* __restrict__ l1part, float* __restrict__ scale, int nb) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nb) return;
  float tot = 0.0f;
  for (int b = 0; b < P * P; ++b) tot += l1part[P * P * v + b];
  scale[v] = fp16_scale(tot);
}

// Input of block (P1, P2) of a 2 x 2 split (M = 2H) at the thread's R1 points: per point
// the four propagated quadrant values (a, b) enter with sign (-1)^(a P1 + b P2).  The block is
// a template argument, so the signs fold into the FMAs; the quadrants come by buffer loads whose
// quadrant offset is a constant scalar operand.
template <int H, int A, int B, bool NEG>
__device__ __forceinline__ void split2_term(const __amdgpu_buffer_rsrc_t& rs, int vo, float2 cx, float2 cy,
                                            float2& acc) {
  constexpr int M = 2 * H;
  float c = cx.x * cy.x - cx.y * cy.y;   // cos(phi_x + phi_y)
  float sn = cx.y * cy.x + cx.x * cy.y;  // sin(phi_x + phi_y)
  if constexpr (NEG) {
    c = -c;
    sn = -sn;
  }
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, (H * A * M + H * B) * int(sizeof(float4)), 0);
  acc.x = fmaf(c, __uint_as_float(v[0]), fmaf(sn, __uint_as_float(v[2]), acc.x));
  acc.y = fmaf(c, __uint_as_float(v[1]), fmaf(sn, __uint_as_float(v[3]), acc.y));
}

template <class S, int H, int P1, int P2>
__device__ __forceinline__ void split2_input(const float4* __restrict__ qv, const float2* __restrict__ pr,
                                             const float2* __restrict__ tw_m, int r, int n2,
                                             float2 (&x)[S::XN]) {
  constexpr int M = 2 * H;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float4*>(qv), short(0),
                                                                      M * M * int(sizeof(float4)), 0x00020000);
  const float2 cx0 = pr[n2], cx1 = pr[n2 + H];
#pragma unroll
  for (int m = 0; m < S::R1; ++m) {
    const int n1 = r + S::R2 * m;
    const int vo = (n1 * M + n2) * int(sizeof(float4));
    const float2 cy0 = pr[n1], cy1 = pr[n1 + H];
    float2 acc = make_float2(0.0f, 0.0f);
    split2_term<H, 0, 0, false>(rs, vo, cx0, cy0, acc);
    split2_term<H, 0, 1, P2 != 0>(rs, vo, cx1, cy0, acc);
    split2_term<H, 1, 0, P1 != 0>(rs, vo, cx0, cy1, acc);
    split2_term<H, 1, 1, (P1 ^ P2) != 0>(rs, vo, cx1, cy1, acc);
    const int ti = P1 * n1 + P2 * n2;   // < 2M
    x[m] = cmul(acc, tw_m[ti >= M ? ti - M : ti]);
    // one point's loads at a time: registers stay few enough for two workgroups per CU,
    // whose other waves hide the load latency
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Plane pairs of M x M spectra: workgroup (view, pair, block).
template <int H, int P, class OutT>
__global__ __launch_bounds__(Shape<H>::T, H == 128 ? 8 : 1) void k_planes_split(const float4* __restrict__ q,
                                                             const float2* __restrict__ prop,
                                                             const float2* __restrict__ tw_m,
                                                             const float2* __restrict__ tw_h,
                                                             OutT* __restrict__ stack, int K, int npairs, int nb,
                                                             const float* __restrict__ scale) {
  using S = Shape<H>;
  constexpr int M = P * H;
  __shared__ float2 lds[(S::LDS_SPLIT_FLOATS + 1) / 2];
  const int wg = blockIdx.x;
  const int xcd = wg & 7, k = wg >> 3;
  // (unsigned: the compiler then needs no sign fix-ups, and keeps the registers it needs low)
  const unsigned per_view = unsigned(npairs) * P * P;
  int view;
  unsigned rem;
  if (nb == 1 || nb == 2 || nb == 4) {
    // fewer views than XCDs: view xcd % nb, its (pair, block) units dealt over the 8 / nb XCDs
    // that share it
    view = xcd % nb;
    rem = unsigned(k) * unsigned(8 / nb) + unsigned(xcd / nb);
    if (rem >= per_view) return;   // whole workgroup leaves together
  } else {
    view = xcd + 8 * int(unsigned(k) / per_view);
    rem = unsigned(k) % per_view;
    if (view >= nb) return;        // whole workgroup leaves together
  }
  const int p = int(rem / (P * P));
  const unsigned blk = rem % (P * P);
  const int p1 = int(blk / P), p2 = int(blk % P);
  const int t = threadIdx.x;
  const int n2 = t % H;
  int r_;   // uniform across a wave when H is a multiple of the wave size
  if constexpr (H % 64 == 0) r_ = __builtin_amdgcn_readfirstlane(t / H);
  else r_ = t / H;
  const int r = r_;
  const float4* qv = q + size_t(view) * M * M;
  const float2* pr = prop + size_t(p) * M;
  float2 x[S::XN];
  if constexpr (P == 2) {
    switch (blk) {   // uniform across the workgroup
      case 0: split2_input<S, H, 0, 0>(qv, pr, tw_m, r, n2, x); break;
      case 1: split2_input<S, H, 0, 1>(qv, pr, tw_m, r, n2, x); break;
      case 2: split2_input<S, H, 1, 0>(qv, pr, tw_m, r, n2, x); break;
      default: split2_input<S, H, 1, 1>(qv, pr, tw_m, r, n2, x); break;
    }
  } else {
    float2 cxs[P];
#pragma unroll
    for (int b = 0; b < P; ++b) cxs[b] = pr[n2 + H * b];
#pragma unroll
    for (int m = 0; m < S::R1; ++m) {
      const int n1 = r + S::R2 * m;
      float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const float2 cy = pr[n1 + H * a];
#pragma unroll
        for (int b = 0; b < P; ++b) {
          const float2 cx = cxs[b];
          const float c = cx.x * cy.x - cx.y * cy.y;   // cos(phi_x + phi_y)
          const float sn = cx.y * cy.x + cx.x * cy.y;  // sin(phi_x + phi_y)
          const float4 qq = qv[(n1 + H * a) * M + n2 + H * b];
          const float2 z = make_float2(c * qq.x + sn * qq.z, c * qq.y + sn * qq.w);
          acc = cadd(acc, cmul(z, split_coef<P>(tw_m, H, (a * p1 + b * p2) % P)));
        }
      }
      const int ti = p1 * n1 + p2 * n2;   // < 2M
      x[m] = cmul(acc, tw_m[ti >= M ? ti - M : ti]);
    }
  }
  // FP16 planes: per-view power-of-two scale, read before the transform (see k_planes)
  float sc = 1.0f;
  if constexpr (std::is_same<OutT, __half>::value) {
    sc = scale[view];
    asm volatile("" : "+v"(sc));
  }
  fft2_block_split<S, true>(x, reinterpret_cast<float*>(lds), tw_h);
  const int sg = t % S::R2, yy = t / S::R2;
  const int y = P * yy + p1;
  const int pa = p, pb = K - 1 - p;
  OutT* rowa = stack + ((size_t(view) * M + y) * K + pa) * M;
  OutT* rowb = stack + ((size_t(view) * M + y) * K + pb) * M;
#pragma unroll
  for (int k2 = 0; k2 < S::R2; ++k2) {
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      if (!S::has_s(sg * S::E + e)) continue;
      const int xc = P * (sg * S::E + e + S::R1 * k2) + p2;
      rowa[xc] = to_store<OutT>(x[e * S::R2 + k2].x * sc);
      if (pb != pa) rowb[xc] = to_store<OutT>(x[e * S::R2 + k2].y * sc);
    }
  }
}

// ------------------------------------------------------------------ launchers
// Arguments of one spectra / planes launch, whatever the size.
struct SpectraLaunch {
  const float* images;
  const float4* filt;
  const float2* tw;        // M-point forward twiddles
  const float2* tw_h;      // H-point forward twiddles (split sizes)
  float4* q;
  int* status;
  double inv_iin;
  float* scale;            // FP16 planes: per-view scale out, else null
  float* l1part;           // split sizes with FP16 planes: [nb][P^2] partial bounds
  int nb;
  hipStream_t s;
};
struct PlanesLaunch {
  int dtype;               // 0 FP32, 1 BF16, 2 FP16
  const float4* q;
  const float2* prop;
  const float2* tw;        // M-point inverse twiddles
  const float2* tw_h;      // H-point inverse twiddles (split sizes)
  void* stack;
  int K, npairs, nb;
  const float* scale;
  hipStream_t s;
};

template <int M>
hipError_t spectra_direct(const SpectraLaunch& a) {
  hipLaunchKernelGGL(k_spectra<M>, dim3(a.nb), dim3(Shape<M>::T), 0, a.s, a.images, a.filt, a.tw, a.q, a.status,
                     a.inv_iin, a.scale);
  return hipGetLastError();
}

template <int M, class OutT>
hipError_t planes_direct_t(const PlanesLaunch& a, const float* scale) {
  // one workgroup per (view, pair), eight XCD columns; the kernel's mapping for nb = 1, 2, 4
  // spreads each view's pairs over 8 / nb XCDs
  const int nb = a.nb, npairs = a.npairs;
  const int reps = (nb == 1 || nb == 2 || nb == 4) ? 8 / nb : 0;
  const int rows = reps ? (npairs + reps - 1) / reps : npairs * ((nb + 7) / 8);
  hipLaunchKernelGGL((k_planes<M, OutT>), dim3(8 * rows), dim3(Shape<M>::T), 0, a.s, a.q, a.prop, a.tw,
                     static_cast<OutT*>(a.stack), a.K, npairs, nb, scale);
  return hipGetLastError();
}

template <int M>
hipError_t planes_direct(const PlanesLaunch& a) {
  switch (a.dtype) {
    case 0: return planes_direct_t<M, float>(a, nullptr);
    case 1: return planes_direct_t<M, __hip_bfloat16>(a, nullptr);
    case 2: return a.scale ? planes_direct_t<M, __half>(a, a.scale) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int M, class OutT>
hipError_t planes_rows_t(const PlanesLaunch& a, const float* scale) {
  // eight XCD columns; for nb = 1, 2, 4 the kernel deals each view's (pair, block) units over
  // 8 / nb XCDs, otherwise one view per XCD
  constexpr int P = RowSplit<M>::P;
  const int per_view = P * a.npairs;
  const int reps = (a.nb == 1 || a.nb == 2 || a.nb == 4) ? 8 / a.nb : 0;
  const int rows = reps ? (per_view + reps - 1) / reps : per_view * ((a.nb + 7) / 8);
  hipLaunchKernelGGL((k_planes_rows<M, OutT>), dim3(8 * rows), dim3(RowSplit<M>::T), 0, a.s, a.q, a.prop, a.tw,
                     static_cast<OutT*>(a.stack), a.K, a.npairs, a.nb, scale);
  return hipGetLastError();
}

template <int M>
hipError_t planes_rows(const PlanesLaunch& a) {
  switch (a.dtype) {
    case 0: return planes_rows_t<M, float>(a, nullptr);
    case 1: return planes_rows_t<M, __hip_bfloat16>(a, nullptr);
    case 2: return a.scale ? planes_rows_t<M, __half>(a, a.scale) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int H, int P>
hipError_t spectra_split(const SpectraLaunch& a) {
  hipLaunchKernelGGL((k_spectra_split<H, P>), dim3(P * P * a.nb), dim3(Shape<H>::T), 0, a.s, a.images, a.filt, a.tw,
                     a.tw_h, a.q, a.status, a.inv_iin, a.scale ? a.l1part : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.scale) return e;
  hipLaunchKernelGGL(k_scale_split<P>, dim3((a.nb + 255) / 256), dim3(256), 0, a.s, a.l1part, a.scale, a.nb);
  return hipGetLastError();
}

template <int H, int P, class OutT>
hipError_t planes_split_t(const PlanesLaunch& a, const float* scale) {
  // eight XCD columns; for nb = 1, 2, 4 the kernel deals each view's (pair, block) units over
  // 8 / nb XCDs, otherwise one view per XCD
  const int per_view = P * P * a.npairs;
  const int reps = (a.nb == 1 || a.nb == 2 || a.nb == 4) ? 8 / a.nb : 0;
  const int rows = reps ? (per_view + reps - 1) / reps : per_view * ((a.nb + 7) / 8);
  hipLaunchKernelGGL((k_planes_split<H, P, OutT>), dim3(8 * rows), dim3(Shape<H>::T), 0, a.s, a.q,
                     a.prop, a.tw, a.tw_h, static_cast<OutT*>(a.stack), a.K, a.npairs, a.nb, scale);
  return hipGetLastError();
}

template <int H, int P>
hipError_t planes_split(const PlanesLaunch& a) {
  switch (a.dtype) {
    case 0: return planes_split_t<H, P, float>(a, nullptr);
    case 1: return planes_split_t<H, P, __hip_bfloat16>(a, nullptr);
    case 2: return a.scale ? planes_split_t<H, P, __half>(a, a.scale) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// A size's launchers, threads per workgroup and block split (P = 1: direct).  The tables
// of these are host data, filled at load time (not constant-initialised, so that the
// device compilation does not take them, and the host launchers they point to, along).
struct FftSize {
  int M, P, threads;
  hipError_t (*spectra)(const SpectraLaunch&);
  hipError_t (*planes)(const PlanesLaunch&);
};

template <int M>
__host__ FftSize direct_size() {
  return FftSize{M, 1, Shape<M>::T, &spectra_direct<M>, &planes_direct<M>};
}
// Direct spectra, row-split planes (the plan's tables are those of a direct size).
template <int M>
__host__ FftSize rows_size() {
  return FftSize{M, 1, Shape<M>::T, &spectra_direct<M>, &planes_rows<M>};
}
// P x P block spectra (H = M / P), row-split planes.
template <int H, int P>
__host__ FftSize split_rows_size() {
  return FftSize{P * H, P, Shape<H>::T, &spectra_split<H, P>, &planes_rows<P * H>};
}
template <int H, int P>
__host__ FftSize split_size() {
  return FftSize{P * H, P, Shape<H>::T, &spectra_split<H, P>, &planes_split<H, P>};
}

}  // namespace tomo

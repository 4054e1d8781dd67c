// gfx950 kernels of the Fourier-space form of the method: eq. 11 (or its swapped
// form, eq. 12) realised by gridding the filtered 2D spectra of all views onto the
// N^3 grid of 3D frequencies (spacing 1/(N dx)), dividing by the regularised
// sampling matrix, the Fourier-space noise filter of Section 3, and one inverse
// 3D FFT.
//
//   k_ffilter    per-variant table multiplied into the image DFT by the spectra
//                kernel: (H_n(q) s(k), 0) for eq. 11 or (s(k), 0) for eq. 12, where
//                s(k) = exp(i pi (M-1)(kx+ky)/M) moves the DFT phase origin to the
//                detector centre (M-1)/2.  FP64, stored FP32.
//   k_fbound     fixed-point unit 2^-e of the accumulator from the per-view spectral
//                bounds: every vertex sum stays below 2^62 in magnitude.
//   k_fclear     zero the accumulator.
//   k_fsplat     every (view, ky, kx) value to the 8 vertices around its paraboloid
//                point p (trilinear weights, text after eq. 11) as 64-bit fixed-point
//                integer atomics: integer addition is order independent, so the sums
//                are bitwise reproducible.  Only +p is splatted; the Hermitian image
//                at -p (the object is real) is folded in by k_fnorm.  For even N the
//                accumulator has one extra index (N/2) per axis, the reflection of the
//                lowest plane.
//   k_fnorm      A(k) = (F(k) + conj F(-k))/2 * S/(S^2 + eps_S); zero |A| below
//                NSR M / sqrt(S); eq. 12 bracket at |k|/(N dx); times
//                C dx^2 / (N dx)^3 and exp(-i 2 pi k.c / N), c = (N-1)/2 (voxel
//                centre origin); written in FFT order.
//   k_fft_axis   inverse 1D FFTs of all lines along one axis of the N^3 grid, staged
//                through LDS, in place; the last pass writes the real part, the volume.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.hpp"
#include "geom.hpp"
#include "tomo_internal.hpp"

namespace tomo {

// ------------------------------------------------------------------ filter table
__global__ void k_ffilter(FilterArgs fa, const ViewGeom* __restrict__ geom, int eq12, float4* __restrict__ filt) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t per = size_t(fa.M) * fa.M;
  if (i >= per * fa.n_views) return;
  const int n = int(i / per);
  const int ky = int((i % per) / fa.M), kx = int(i % fa.M);
  const int M = fa.M;
  // exp(i pi t / M) with t = (M-1)(kx~ + ky~) reduced mod 2M in integers
  long long t = (long long)(M - 1) * (signed_index(kx, M) + signed_index(ky, M)) % (2LL * M);
  if (t < 0) t += 2LL * M;
  double ss, sc;
  sincos(M_PI * double(t) / double(M), &ss, &sc);
  double fr = sc, fi = ss;
  if (!eq12) {
    const double qx = signed_q(kx, M, fa.dx), qy = signed_q(ky, M, fa.dx);
    const double chi = M_PI * fa.lambda * geom[n].R * (qx * qx + qy * qy) - atan(fa.sigma);
    double sn, cs;
    sincos(chi, &sn, &cs);
    const double hr = sn / (sn * sn + fa.epsilon);
    const double hi = fa.ewald ? -cs / (cs * cs + fa.epsilon) : 0.0;
    fr = hr * sc - hi * ss;
    fi = hr * ss + hi * sc;
  }
  filt[i] = make_float4(float(fr), float(fi), 0.0f, 0.0f);
}

// ------------------------------------------------------------------ accumulator scale
// view_scale[v] = 2^14 / (power of two >= the view's sum of |Re| + |Im|), from the spectra kernel.
// A vertex sum is bounded by the sum over all samples of |Re| + |Im| (weights of one
// sample add up to one), so B = sum_v 2^14 / view_scale[v] bounds it; the unit puts B
// at 2^62.  Sequential FP64 sum: fixed order.
__global__ void k_fbound(const float* __restrict__ view_scale, int n, double* __restrict__ fix) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double b = 0.0;
  for (int v = 0; v < n; ++v) b += 16384.0 / double(view_scale[v]);
  const double e = b > 0.0 ? 62.0 - ceil(log2(b)) : 0.0;
  fix[0] = exp2(e);
  fix[1] = exp2(-e);
}

__global__ void k_fclear(ulonglong2* __restrict__ acc, size_t count) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) acc[i] = make_ulonglong2(0ull, 0ull);
}

// ------------------------------------------------------------------ splat
__global__ __launch_bounds__(256) void k_fsplat(FilterArgs fa, const ViewGeom* __restrict__ geom,
                                                const float4* __restrict__ q, const double* __restrict__ fix,
                                                unsigned long long* __restrict__ acc, int P) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t per = size_t(fa.M) * fa.M;
  if (i >= per * fa.n_views) return;
  const int n = int(i / per);
  const int ky = int((i % per) / fa.M), kx = int(i % fa.M);
  const float4 val = q[i];
  const double unit = fix[0];
  const double vr = double(val.x) * unit, vi = double(val.y) * unit;
  double p[3];
  sample_point(fa, geom[n], ky, kx, p);
  const int lo = -(fa.N / 2);
  int i0[3];
  double t[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double f = p[a] - lo;
    const double fl = floor(f);
    i0[a] = int(fl);
    t[a] = f - fl;
  }
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const int jx = i0[0] + cx, jy = i0[1] + cy, jz = i0[2] + cz;
        if (unsigned(jx) >= unsigned(P) || unsigned(jy) >= unsigned(P) || unsigned(jz) >= unsigned(P)) continue;
        const double w = (cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1]) * (cz ? t[2] : 1.0 - t[2]);
        const long long ar = llrint(w * vr), ai = llrint(w * vi);
        unsigned long long* dst = acc + 2 * ((size_t(jz) * P + jy) * P + jx);
        if (ar) atomicAdd(dst, (unsigned long long)ar);
        if (ai) atomicAdd(dst + 1, (unsigned long long)ai);
      }
}

// ------------------------------------------------------------------ normalise
__global__ __launch_bounds__(256) void k_fnorm(FourierNormArgs a, const unsigned long long* __restrict__ acc,
                                               const unsigned long long* __restrict__ smat,
                                               const double* __restrict__ fix, float2* __restrict__ grid) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int N = a.N, P = a.P;
  const size_t n3 = size_t(N) * N * N;
  if (i >= n3) return;
  const int jx = int(i % N), jy = int((i / N) % N), jz = int(i / (size_t(N) * N));
  const int lo = -(N / 2);
  const int kx = jx + lo, ky = jy + lo, kz = jz + lo;
  // index of -k: -k - lo = -j - 2 lo, inside [0, P)
  const int mx = -jx - 2 * lo, my = -jy - 2 * lo, mz = -jz - 2 * lo;
  const ulonglong2 f = reinterpret_cast<const ulonglong2*>(acc)[(size_t(jz) * P + jy) * P + jx];
  const ulonglong2 g = reinterpret_cast<const ulonglong2*>(acc)[(size_t(mz) * P + my) * P + mx];
  const double inv_unit = fix[1];
  double re = 0.5 * (double((long long)f.x) + double((long long)g.x)) * inv_unit;
  double im = 0.5 * (double((long long)f.y) - double((long long)g.y)) * inv_unit;
  const double S = double(smat[i]) / kFix;
  const double ws = S / (S * S + a.eps_s);
  re *= ws;
  im *= ws;
  if (a.nsr_m > 0.0) {
    const bool keep = S > 0.0 && sqrt(re * re + im * im) >= a.nsr_m / sqrt(S);
    if (!keep) re = im = 0.0;
  }
  if (a.eq12) {
    const double kk = double(kx) * kx + double(ky) * ky + double(kz) * kz;
    const double nd = double(N) * a.dx;
    const double chi = M_PI * a.lambda * a.R * kk / (nd * nd) - atan(a.sigma);
    double sn, cs;
    sincos(chi, &sn, &cs);
    const double hr = sn / (sn * sn + a.epsilon);
    const double hi = a.ewald ? -cs / (cs * cs + a.epsilon) : 0.0;
    const double r2 = re * hr - im * hi, i2 = re * hi + im * hr;
    re = r2;
    im = i2;
  }
  // exp(-i pi t / N), t = (N-1)(kx+ky+kz) mod 2N
  long long t = (long long)(N - 1) * (kx + ky + kz) % (2LL * N);
  if (t < 0) t += 2LL * N;
  double ps, pc;
  sincos(M_PI * double(t) / double(N), &ps, &pc);
  const double orr = (re * pc + im * ps) * a.out_scale;
  const double oii = (im * pc - re * ps) * a.out_scale;
  const int fx = (kx + N) % N, fy = (ky + N) % N, fz = (kz + N) % N;
  grid[(size_t(fz) * N + fy) * N + fx] = make_float2(float(orr), float(oii));
}

// ------------------------------------------------------------------ 1D FFT along an axis
// N = R1 * R2 (R2 | R1), L lines per workgroup, R2 threads per line.
template <int N_, int R1_, int R2_, int L_>
struct AxisShape {
  static constexpr int N = N_, R1 = R1_, R2 = R2_, L = L_;
  static constexpr int T = L * R2;
  static constexpr int E = R1 / R2;
  static constexpr int LP = L + 1;   // LDS pitch of one axis position (float2)
  static_assert(R1 * R2 == N && R1 % R2 == 0 && N % L == 0, "axis FFT shape");
};
template <int N>
struct Axis;
template <> struct Axis<16> : AxisShape<16, 4, 4, 16> {};
template <> struct Axis<32> : AxisShape<32, 8, 4, 32> {};
template <> struct Axis<48> : AxisShape<48, 12, 4, 48> {};
template <> struct Axis<64> : AxisShape<64, 16, 4, 64> {};
template <> struct Axis<80> : AxisShape<80, 20, 4, 40> {};
template <> struct Axis<96> : AxisShape<96, 24, 4, 48> {};
template <> struct Axis<128> : AxisShape<128, 16, 8, 32> {};
template <> struct Axis<256> : AxisShape<256, 16, 16, 16> {};

// X[s + R1 k2] = sum_r W_R2^(r k2) W_N^(r s) sum_m W_R1^(m s) x[r + R2 m], W = exp(+i 2 pi / .)
// axis 0: lines along x (L consecutive rows); axis 1: along y; axis 2: along z (L consecutive x).
template <int N>
__global__ __launch_bounds__(Axis<N>::T) void k_fft_axis(float2* __restrict__ data, float* __restrict__ real_out,
                                                        const float2* __restrict__ tw, int axis) {
  using A = Axis<N>;
  __shared__ float2 tile[N * A::LP];
  const int t = threadIdx.x;
  const int b = blockIdx.x;
  size_t base, sj, sl;
  if (axis == 0) {
    base = size_t(b) * A::L * N;
    sj = 1;
    sl = N;
  } else {
    constexpr int per = N / A::L;
    const int outer = b / per, x0 = (b % per) * A::L;
    if (axis == 1) {
      base = size_t(outer) * N * N + x0;
      sj = N;
    } else {
      base = size_t(outer) * N + x0;
      sj = size_t(N) * N;
    }
    sl = 1;
  }
  // coalesced load: the memory-contiguous index runs fastest across the threads
  for (int idx = t; idx < N * A::L; idx += A::T) {
    const int j = axis == 0 ? idx % N : idx / A::L;
    const int l = axis == 0 ? idx / N : idx % A::L;
    tile[j * A::LP + l] = data[base + j * sj + l * sl];
  }
  __syncthreads();
  const int l = t % A::L, r = t / A::L;
  float2 x[A::R1];
#pragma unroll
  for (int m = 0; m < A::R1; ++m) x[m] = tile[(r + A::R2 * m) * A::LP + l];
  Dft<A::R1, true>::run(x);
#pragma unroll
  for (int s = 1; s < A::R1; ++s) x[s] = cmul(x[s], tw[r * s]);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < A::R1; ++s) tile[(s * A::R2 + r) * A::LP + l] = x[s];
  __syncthreads();
  float2 y[A::E][A::R2];
#pragma unroll
  for (int e = 0; e < A::E; ++e) {
    const int s = r * A::E + e;
#pragma unroll
    for (int rr = 0; rr < A::R2; ++rr) y[e][rr] = tile[(s * A::R2 + rr) * A::LP + l];
    Dft<A::R2, true>::run(y[e]);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < A::E; ++e) {
    const int s = r * A::E + e;
#pragma unroll
    for (int k2 = 0; k2 < A::R2; ++k2) tile[(s + A::R1 * k2) * A::LP + l] = y[e][k2];
  }
  __syncthreads();
  for (int idx = t; idx < N * A::L; idx += A::T) {
    const int j = axis == 0 ? idx % N : idx / A::L;
    const int l2 = axis == 0 ? idx / N : idx % A::L;
    const float2 v = tile[j * A::LP + l2];
    const size_t addr = base + j * sj + l2 * sl;
    if (real_out) real_out[addr] = v.x;
    else data[addr] = v;
  }
}

// ------------------------------------------------------------------ launchers
bool fourier_grid_supported(int N) {
  switch (N) {
    case 16: case 32: case 48: case 64: case 80: case 96: case 128: case 256: return true;
    default: return false;
  }
}

hipError_t launch_fourier_filter(const FilterArgs& fa, const ViewGeom* geom, int eq12, float4* filt,
                                 hipStream_t s) {
  const size_t total = size_t(fa.M) * fa.M * fa.n_views;
  hipLaunchKernelGGL(k_ffilter, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, fa, geom, eq12, filt);
  return hipGetLastError();
}

hipError_t launch_fourier_splat(const FilterArgs& fa, const ViewGeom* geom, const float4* q, const float* view_scale,
                                double* fix, unsigned long long* acc, int P, hipStream_t s) {
  hipLaunchKernelGGL(k_fbound, dim3(1), dim3(64), 0, s, view_scale, fa.n_views, fix);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t cells = size_t(P) * P * P;
  hipLaunchKernelGGL(k_fclear, dim3(unsigned((cells + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<ulonglong2*>(acc), cells);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t total = size_t(fa.M) * fa.M * fa.n_views;
  hipLaunchKernelGGL(k_fsplat, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, fa, geom, q, fix, acc, P);
  return hipGetLastError();
}

template <int N>
static hipError_t fft3_impl(float2* grid, float* vol, const float2* tw, hipStream_t s) {
  const dim3 blocks(unsigned(size_t(N) * N / Axis<N>::L));
  for (int axis = 0; axis < 3; ++axis) {
    hipLaunchKernelGGL(k_fft_axis<N>, blocks, dim3(Axis<N>::T), 0, s, grid, axis == 2 ? vol : nullptr, tw, axis);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fourier_inverse(const FourierNormArgs& a, const unsigned long long* acc,
                                  const unsigned long long* smat, const double* fix, float2* grid, const float2* tw,
                                  float* vol, hipStream_t s) {
  const size_t n3 = size_t(a.N) * a.N * a.N;
  hipLaunchKernelGGL(k_fnorm, dim3(unsigned((n3 + 255) / 256)), dim3(256), 0, s, a, acc, smat, fix, grid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (a.N) {
    case 16: return fft3_impl<16>(grid, vol, tw, s);
    case 32: return fft3_impl<32>(grid, vol, tw, s);
    case 48: return fft3_impl<48>(grid, vol, tw, s);
    case 64: return fft3_impl<64>(grid, vol, tw, s);
    case 80: return fft3_impl<80>(grid, vol, tw, s);
    case 96: return fft3_impl<96>(grid, vol, tw, s);
    case 128: return fft3_impl<128>(grid, vol, tw, s);
    case 256: return fft3_impl<256>(grid, vol, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tomo

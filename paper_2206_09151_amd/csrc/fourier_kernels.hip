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
//
// Precomputed gridding operator (plan time): the vertex -> (sample, weight) lists do not
// depend on the images, so the plan stores them as a compressed sparse row matrix over
// the P^3 vertices (k_fop_count, a host prefix sum, k_fop_fill, k_fop_sort: entries of a
// vertex in ascending sample order).  Per call, k_fgather forms F(k) and F(-k) of every
// grid vertex as FP64 sums in that fixed order -- deterministic, no atomics -- and applies
// the k_fnorm steps in the same kernel.
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
// Steps after the Hermitian fold for grid vertex i = (jz, jy, jx): S^-1, NSR threshold,
// eq. 12 bracket, centring phase and constant; stores into the FFT-order grid.
__device__ __forceinline__ void finish_vertex(const FourierNormArgs& a, size_t i, int jx, int jy, int jz, double re,
                                              double im, const unsigned long long* __restrict__ smat,
                                              float2* __restrict__ grid) {
  const int N = a.N;
  const int lo = -(N / 2);
  const int kx = jx + lo, ky = jy + lo, kz = jz + lo;
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

__global__ __launch_bounds__(256) void k_fnorm(FourierNormArgs a, const unsigned long long* __restrict__ acc,
                                               const unsigned long long* __restrict__ smat,
                                               const double* __restrict__ fix, float2* __restrict__ grid) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int N = a.N, P = a.P;
  const size_t n3 = size_t(N) * N * N;
  if (i >= n3) return;
  const int jx = int(i % N), jy = int((i / N) % N), jz = int(i / (size_t(N) * N));
  const int lo = -(N / 2);
  // index of -k: -k - lo = -j - 2 lo, inside [0, P)
  const int mx = -jx - 2 * lo, my = -jy - 2 * lo, mz = -jz - 2 * lo;
  const ulonglong2 f = reinterpret_cast<const ulonglong2*>(acc)[(size_t(jz) * P + jy) * P + jx];
  const ulonglong2 g = reinterpret_cast<const ulonglong2*>(acc)[(size_t(mz) * P + my) * P + mx];
  const double inv_unit = fix[1];
  const double re = 0.5 * (double((long long)f.x) + double((long long)g.x)) * inv_unit;
  const double im = 0.5 * (double((long long)f.y) - double((long long)g.y)) * inv_unit;
  finish_vertex(a, i, jx, jy, jz, re, im, smat, grid);
}

// ------------------------------------------------------------------ gridding operator
// Trilinear taps of sample i (view n, bin (ky, kx)) on the P^3 vertex grid with positive
// weight: calls f(cell, w) in a fixed tap order.
template <class F>
__device__ __forceinline__ void for_each_tap(const FilterArgs& fa, const ViewGeom& g, int ky, int kx, int P, F&& f) {
  double p[3];
  sample_point(fa, g, ky, kx, p);
  const int lo = -(fa.N / 2);
  int i0[3];
  double t[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double fl = floor(p[a] - lo);
    i0[a] = int(fl);
    t[a] = (p[a] - lo) - fl;
  }
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const int jx = i0[0] + cx, jy = i0[1] + cy, jz = i0[2] + cz;
        if (unsigned(jx) >= unsigned(P) || unsigned(jy) >= unsigned(P) || unsigned(jz) >= unsigned(P)) continue;
        const double w = (cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1]) * (cz ? t[2] : 1.0 - t[2]);
        if (w > 0.0) f((size_t(jz) * P + jy) * P + jx, w);
      }
}

__global__ __launch_bounds__(256) void k_fop_count(FilterArgs fa, const ViewGeom* __restrict__ geom, int P,
                                                   unsigned* __restrict__ count) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t per = size_t(fa.M) * fa.M;
  if (i >= per * fa.n_views) return;
  const int n = int(i / per);
  const int ky = int((i % per) / fa.M), kx = int(i % fa.M);
  for_each_tap(fa, geom[n], ky, kx, P, [&](size_t cell, double) { atomicAdd(count + cell, 1u); });
}

__global__ __launch_bounds__(256) void k_fop_fill(FilterArgs fa, const ViewGeom* __restrict__ geom, int P,
                                                  const unsigned* __restrict__ row_ptr, unsigned* __restrict__ cursor,
                                                  int2* __restrict__ ent) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t per = size_t(fa.M) * fa.M;
  if (i >= per * fa.n_views) return;
  const int n = int(i / per);
  const int ky = int((i % per) / fa.M), kx = int(i % fa.M);
  for_each_tap(fa, geom[n], ky, kx, P, [&](size_t cell, double w) {
    const unsigned slot = atomicAdd(cursor + cell, 1u);
    // the counting pass visited the same taps; the guard keeps every store in the vertex's range
    if (row_ptr[cell] + slot < row_ptr[cell + 1])
      ent[size_t(row_ptr[cell]) + slot] = make_int2(int(i), __float_as_int(float(w)));
  });
}

// Entries of every vertex in ascending sample order (insertion sort; lists are short
// except near the origin and the rotation axis).
__global__ __launch_bounds__(256) void k_fop_sort(size_t cells, const unsigned* __restrict__ row_ptr,
                                                  int2* __restrict__ ent) {
  const size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const unsigned b = row_ptr[c], e = row_ptr[c + 1];
  for (unsigned j = b + 1; j < e; ++j) {
    const int2 v = ent[j];
    unsigned k = j;
    while (k > b && ent[k - 1].x > v.x) {
      ent[k] = ent[k - 1];
      --k;
    }
    ent[k] = v;
  }
}

// Sum of w * value over a vertex's entries (FP64, ascending sample order).  Four entries
// are fetched per round so that four spectrum loads are in flight at once.
__device__ __forceinline__ void gather_vertex(size_t cell, const unsigned* __restrict__ row_ptr,
                                              const int2* __restrict__ ent, const float2* __restrict__ q2,
                                              double& re, double& im) {
  re = 0.0;
  im = 0.0;
  const unsigned b = row_ptr[cell], e = row_ptr[cell + 1];
  unsigned j = b;
  for (; j + 4 <= e; j += 4) {
    int2 v[4];
    float2 s[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = ent[j + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] = q2[2 * size_t(v[u].x)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double w = double(__int_as_float(v[u].y));
      re += w * double(s[u].x);
      im += w * double(s[u].y);
    }
  }
  for (; j < e; ++j) {
    const int2 v = ent[j];
    const float2 s = q2[2 * size_t(v.x)];
    const double w = double(__int_as_float(v.y));
    re += w * double(s.x);
    im += w * double(s.y);
  }
}

// Lane-strided partial sum of a vertex's entries (the wave-cooperative path).
__device__ __forceinline__ void gather_strided(unsigned b, unsigned e, int lane, const int2* __restrict__ ent,
                                               const float2* __restrict__ q2, double& re, double& im) {
  for (unsigned j = b + lane; j < e; j += 64) {
    const int2 v = ent[j];
    const float2 s = q2[2 * size_t(v.x)];
    const double w = double(__int_as_float(v.y));
    re += w * double(s.x);
    im += w * double(s.y);
  }
}

// Entries above which a vertex pair is summed by the whole wave (vertices near the
// origin and the rotation axis collect one entry per view).
constexpr unsigned kHeavy = 48;

// One thread per pair (k, -k): the Hermitian fold gives A(-k) = conj A(k), so both
// vertices are finished from the same two sums.  The thread of the pair's lower flat
// index owns it; a vertex whose mirror lies outside the grid (the lowest plane of an
// even N) owns itself.  Pairs with more than kHeavy entries are summed by all 64 lanes
// of the wave (lane-strided partial sums, then a fixed butterfly), one pair after the
// other; the rest sequentially by their owner.  Both orders are fixed: deterministic.
__global__ __launch_bounds__(256) void k_fgather(FourierNormArgs a, const unsigned* __restrict__ row_ptr,
                                                 const int2* __restrict__ ent, const float4* __restrict__ q,
                                                 const unsigned long long* __restrict__ smat,
                                                 float2* __restrict__ grid) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int N = a.N, P = a.P;
  const size_t n3 = size_t(N) * N * N;
  const int jx = int(i % N), jy = int((i / N) % N), jz = int(i / (size_t(N) * N));
  const int lo = -(N / 2);
  const int mx = -jx - 2 * lo, my = -jy - 2 * lo, mz = -jz - 2 * lo;
  const bool mirror_in = mx < N && my < N && mz < N;
  const size_t mi = (size_t(mz) * N + my) * N + mx;
  const bool owner = i < n3 && !(mirror_in && mi < i);
  const float2* q2 = reinterpret_cast<const float2*>(q);
  unsigned bk = 0, ek = 0, bm = 0, em = 0;
  if (owner) {
    const size_t ck = (size_t(jz) * P + jy) * P + jx, cm = (size_t(mz) * P + my) * P + mx;
    bk = row_ptr[ck];
    ek = row_ptr[ck + 1];
    bm = row_ptr[cm];
    em = row_ptr[cm + 1];
  }
  const bool heavy = owner && (ek - bk) + (em - bm) > kHeavy;
  double fr = 0.0, fi = 0.0, gr = 0.0, gi = 0.0;
  if (owner && !heavy) {
    gather_vertex((size_t(jz) * P + jy) * P + jx, row_ptr, ent, q2, fr, fi);
    gather_vertex((size_t(mz) * P + my) * P + mx, row_ptr, ent, q2, gr, gi);
  }
  unsigned long long todo = __ballot(heavy);
  while (todo) {
    const int src = __ffsll(static_cast<long long>(todo)) - 1;
    todo &= todo - 1;
    const unsigned b1 = __shfl(bk, src, 64), e1 = __shfl(ek, src, 64);
    const unsigned b2 = __shfl(bm, src, 64), e2 = __shfl(em, src, 64);
    double pr = 0.0, pi = 0.0, sr = 0.0, si = 0.0;
    gather_strided(b1, e1, lane, ent, q2, pr, pi);
    gather_strided(b2, e2, lane, ent, q2, sr, si);
    for (int off = 32; off > 0; off >>= 1) {
      pr += __shfl_xor(pr, off, 64);
      pi += __shfl_xor(pi, off, 64);
      sr += __shfl_xor(sr, off, 64);
      si += __shfl_xor(si, off, 64);
    }
    if (lane == src) {
      fr = pr;
      fi = pi;
      gr = sr;
      gi = si;
    }
  }
  if (!owner) return;
  const double ar = 0.5 * (fr + gr), ai = 0.5 * (fi - gi);
  finish_vertex(a, i, jx, jy, jz, ar, ai, smat, grid);
  if (mirror_in && mi != i) finish_vertex(a, mi, mx, my, mz, ar, -ai, smat, grid);
}

// ------------------------------------------------------------------ 1D FFT along an axis
// N = R1 * R2 (R1 >= R2; when R2 does not divide R1 the last stage-2 slots of some threads
// are idle), L lines per workgroup (L | N), R2 threads per line.
template <int N_, int R1_, int R2_, int L_>
struct AxisShape {
  static constexpr int N = N_, R1 = R1_, R2 = R2_, L = L_;
  static constexpr int T = L * R2;
  static constexpr int E = (R1 + R2 - 1) / R2;
  static constexpr int LP = L + 1;   // LDS pitch of one axis position (float2)
  static_assert(R1 * R2 == N && R1 >= R2 && N % L == 0 && T <= 1024, "axis FFT shape");
};
template <int N>
struct Axis;
template <> struct Axis<16> : AxisShape<16, 4, 4, 16> {};
template <> struct Axis<18> : AxisShape<18, 6, 3, 18> {};
template <> struct Axis<20> : AxisShape<20, 5, 4, 20> {};
template <> struct Axis<24> : AxisShape<24, 6, 4, 24> {};
template <> struct Axis<25> : AxisShape<25, 5, 5, 25> {};
template <> struct Axis<27> : AxisShape<27, 9, 3, 27> {};
template <> struct Axis<30> : AxisShape<30, 6, 5, 30> {};
template <> struct Axis<32> : AxisShape<32, 8, 4, 32> {};
template <> struct Axis<36> : AxisShape<36, 6, 6, 36> {};
template <> struct Axis<40> : AxisShape<40, 10, 4, 40> {};
template <> struct Axis<45> : AxisShape<45, 9, 5, 45> {};
template <> struct Axis<48> : AxisShape<48, 12, 4, 48> {};
template <> struct Axis<50> : AxisShape<50, 10, 5, 50> {};
template <> struct Axis<54> : AxisShape<54, 9, 6, 54> {};
template <> struct Axis<60> : AxisShape<60, 10, 6, 60> {};
template <> struct Axis<64> : AxisShape<64, 16, 4, 64> {};
template <> struct Axis<72> : AxisShape<72, 12, 6, 36> {};
template <> struct Axis<75> : AxisShape<75, 15, 5, 25> {};
template <> struct Axis<80> : AxisShape<80, 20, 4, 40> {};
template <> struct Axis<81> : AxisShape<81, 9, 9, 27> {};
template <> struct Axis<90> : AxisShape<90, 15, 6, 30> {};
template <> struct Axis<96> : AxisShape<96, 24, 4, 48> {};
template <> struct Axis<100> : AxisShape<100, 10, 10, 25> {};
template <> struct Axis<108> : AxisShape<108, 18, 6, 36> {};
template <> struct Axis<120> : AxisShape<120, 24, 5, 40> {};
template <> struct Axis<125> : AxisShape<125, 25, 5, 25> {};
template <> struct Axis<128> : AxisShape<128, 16, 8, 32> {};
template <> struct Axis<135> : AxisShape<135, 27, 5, 27> {};
template <> struct Axis<144> : AxisShape<144, 24, 6, 36> {};
template <> struct Axis<150> : AxisShape<150, 30, 5, 30> {};
template <> struct Axis<160> : AxisShape<160, 40, 4, 32> {};
template <> struct Axis<162> : AxisShape<162, 27, 6, 27> {};
template <> struct Axis<180> : AxisShape<180, 36, 5, 36> {};
template <> struct Axis<192> : AxisShape<192, 24, 8, 32> {};
template <> struct Axis<200> : AxisShape<200, 40, 5, 40> {};
template <> struct Axis<216> : AxisShape<216, 36, 6, 24> {};
template <> struct Axis<225> : AxisShape<225, 25, 9, 25> {};
template <> struct Axis<240> : AxisShape<240, 24, 10, 16> {};
template <> struct Axis<243> : AxisShape<243, 27, 9, 27> {};
template <> struct Axis<250> : AxisShape<250, 25, 10, 25> {};
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
    if (s >= A::R1) continue;
#pragma unroll
    for (int rr = 0; rr < A::R2; ++rr) y[e][rr] = tile[(s * A::R2 + rr) * A::LP + l];
    Dft<A::R2, true>::run(y[e]);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < A::E; ++e) {
    const int s = r * A::E + e;
    if (s >= A::R1) continue;
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
bool fourier_grid_supported(int N) { return launch_fourier_fft3(N, nullptr, nullptr, nullptr, nullptr) != hipErrorInvalidValue; }

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

hipError_t launch_fourier_op_count(const FilterArgs& fa, const ViewGeom* geom, int P, unsigned* count,
                                  hipStream_t s) {
  const size_t total = size_t(fa.M) * fa.M * fa.n_views;
  hipLaunchKernelGGL(k_fop_count, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, fa, geom, P, count);
  return hipGetLastError();
}

hipError_t launch_fourier_op_fill(const FilterArgs& fa, const ViewGeom* geom, int P, const unsigned* row_ptr,
                                 unsigned* cursor, int2* ent, hipStream_t s) {
  const size_t total = size_t(fa.M) * fa.M * fa.n_views;
  hipLaunchKernelGGL(k_fop_fill, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, fa, geom, P, row_ptr, cursor,
                     ent);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t cells = size_t(P) * P * P;
  hipLaunchKernelGGL(k_fop_sort, dim3(unsigned((cells + 255) / 256)), dim3(256), 0, s, cells, row_ptr, ent);
  return hipGetLastError();
}

template <int N>
static hipError_t fft3_impl(float2* grid, float* vol, const float2* tw, hipStream_t s) {
  if (!grid) return hipSuccess;   // size query: nothing is launched
  const dim3 blocks(unsigned(size_t(N) * N / Axis<N>::L));
  for (int axis = 0; axis < 3; ++axis) {
    hipLaunchKernelGGL(k_fft_axis<N>, blocks, dim3(Axis<N>::T), 0, s, grid, axis == 2 ? vol : nullptr, tw, axis);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fourier_gather(const FourierNormArgs& a, const unsigned* row_ptr, const int2* ent,
                                 const float4* q, const unsigned long long* smat, float2* grid, hipStream_t s) {
  const size_t n3 = size_t(a.N) * a.N * a.N;
  hipLaunchKernelGGL(k_fgather, dim3(unsigned((n3 + 255) / 256)), dim3(256), 0, s, a, row_ptr, ent, q, smat, grid);
  return hipGetLastError();
}

hipError_t launch_fourier_norm(const FourierNormArgs& a, const unsigned long long* acc, const unsigned long long* smat,
                               const double* fix, float2* grid, hipStream_t s) {
  const size_t n3 = size_t(a.N) * a.N * a.N;
  hipLaunchKernelGGL(k_fnorm, dim3(unsigned((n3 + 255) / 256)), dim3(256), 0, s, a, acc, smat, fix, grid);
  return hipGetLastError();
}

// With grid == nullptr only reports whether N is supported (hipSuccess) or not.
hipError_t launch_fourier_fft3(int N, float2* grid, const float2* tw, float* vol, hipStream_t s) {
  switch (N) {
    case 16: return fft3_impl<16>(grid, vol, tw, s);
    case 18: return fft3_impl<18>(grid, vol, tw, s);
    case 20: return fft3_impl<20>(grid, vol, tw, s);
    case 24: return fft3_impl<24>(grid, vol, tw, s);
    case 25: return fft3_impl<25>(grid, vol, tw, s);
    case 27: return fft3_impl<27>(grid, vol, tw, s);
    case 30: return fft3_impl<30>(grid, vol, tw, s);
    case 32: return fft3_impl<32>(grid, vol, tw, s);
    case 36: return fft3_impl<36>(grid, vol, tw, s);
    case 40: return fft3_impl<40>(grid, vol, tw, s);
    case 45: return fft3_impl<45>(grid, vol, tw, s);
    case 48: return fft3_impl<48>(grid, vol, tw, s);
    case 50: return fft3_impl<50>(grid, vol, tw, s);
    case 54: return fft3_impl<54>(grid, vol, tw, s);
    case 60: return fft3_impl<60>(grid, vol, tw, s);
    case 64: return fft3_impl<64>(grid, vol, tw, s);
    case 72: return fft3_impl<72>(grid, vol, tw, s);
    case 75: return fft3_impl<75>(grid, vol, tw, s);
    case 80: return fft3_impl<80>(grid, vol, tw, s);
    case 81: return fft3_impl<81>(grid, vol, tw, s);
    case 90: return fft3_impl<90>(grid, vol, tw, s);
    case 96: return fft3_impl<96>(grid, vol, tw, s);
    case 100: return fft3_impl<100>(grid, vol, tw, s);
    case 108: return fft3_impl<108>(grid, vol, tw, s);
    case 120: return fft3_impl<120>(grid, vol, tw, s);
    case 125: return fft3_impl<125>(grid, vol, tw, s);
    case 128: return fft3_impl<128>(grid, vol, tw, s);
    case 135: return fft3_impl<135>(grid, vol, tw, s);
    case 144: return fft3_impl<144>(grid, vol, tw, s);
    case 150: return fft3_impl<150>(grid, vol, tw, s);
    case 160: return fft3_impl<160>(grid, vol, tw, s);
    case 162: return fft3_impl<162>(grid, vol, tw, s);
    case 180: return fft3_impl<180>(grid, vol, tw, s);
    case 192: return fft3_impl<192>(grid, vol, tw, s);
    case 200: return fft3_impl<200>(grid, vol, tw, s);
    case 216: return fft3_impl<216>(grid, vol, tw, s);
    case 225: return fft3_impl<225>(grid, vol, tw, s);
    case 240: return fft3_impl<240>(grid, vol, tw, s);
    case 243: return fft3_impl<243>(grid, vol, tw, s);
    case 250: return fft3_impl<250>(grid, vol, tw, s);
    case 256: return fft3_impl<256>(grid, vol, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tomo

// Register DFT codelets and an LDS-staged 2D FFT for one workgroup on gfx950.
//
// The 2D transform of an M x M complex block (M = R1 * R2) runs with M * R2 threads.
// Each 1D pass is a two-stage Cooley-Tukey split of the index
//   k = r + R2*m  ->  X[s + R1*k2] = sum_r W_R2^(r k2) W_M^(r s) sum_m W_R1^(m s) x[r + R2 m]
// stage 1: a radix-R1 DFT in registers per (line, r), then the twiddle W_M^(r s);
// stage 2: radix-R2 DFTs over r, after one exchange through LDS.  Between the
// column and the row pass the block is transposed through LDS.  Stage-1 thread
// mapping keeps r uniform across a 64-lane wave (M >= 64), so twiddle loads are
// scalar.  The last stage maps lanes so that consecutive lanes own consecutive
// output columns of one row (coalesced stores).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace tomo {

// ---------------------------------------------------------------- compile-time trig
constexpr double kPi = 3.141592653589793238462643383279502884;

// sin/cos of 2*pi*num/den by Taylor series after folding the angle into [-pi, pi].
constexpr double ce_sin_turn(long num, long den) {
  long n = ((num % den) + den) % den;           // [0, den)
  double x = 2.0 * kPi * double(n) / double(den);
  if (x > kPi) x -= 2.0 * kPi;                  // [-pi, pi]
  double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double ce_cos_turn(long num, long den) { return ce_sin_turn(num * 4 + den, den * 4); }

template <int I, int N>
struct StaticFor {
  template <class F>
  __device__ __forceinline__ static void run(F&& f) {
    if constexpr (I < N) {
      f(std::integral_constant<int, I>{});
      StaticFor<I + 1, N>::run(f);
    }
  }
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (FWD) or +i (INV): the quarter turn of the transform's kernel
template <bool INV>
__device__ __forceinline__ float2 qturn(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// v * exp(sgn * i*2*pi*K/R), sgn = -1 forward, +1 inverse; exact for multiples of a quarter turn.
template <int R, int K, bool INV>
__device__ __forceinline__ float2 rot(float2 v) {
  constexpr int k = ((K % R) + R) % R;
  if constexpr (k == 0) {
    return v;
  } else if constexpr (4 * k == R) {
    return qturn<INV>(v);
  } else if constexpr (2 * k == R) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * k == 3 * R) {
    return qturn<!INV>(v);
  } else {
      constexpr float c = float(ce_cos_turn(k, R));
      constexpr float s = float(INV ? ce_sin_turn(k, R) : -ce_sin_turn(k, R));
      return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// ---------------------------------------------------------------- DFT codelets
// In-place DFT of R registers, natural order in and out.
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
  __device__ __forceinline__ static void run(float2*) {}
};

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    constexpr float h = 0.86602540378443864676f;  // sin(2 pi / 3)
    float2 t1 = cadd(x[1], x[2]);
    float2 t2 = csub(x[1], x[2]);
    float2 m = make_float2(x[0].x - 0.5f * t1.x, x[0].y - 0.5f * t1.y);
    float2 r = qturn<INV>(cscale(t2, h));  // -+ i * sin(2pi/3) * (x1 - x2)
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    float2 c = cadd(x[1], x[3]), d = qturn<INV>(csub(x[1], x[3]));
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, d);
    x[3] = csub(b, d);
  }
};

template <bool INV>
struct Dft<5, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    constexpr float c1 = float(ce_cos_turn(1, 5)), c2 = float(ce_cos_turn(2, 5));
    constexpr float s1 = float(ce_sin_turn(1, 5)), s2 = float(ce_sin_turn(2, 5));
    float2 a1 = cadd(x[1], x[4]), a2 = cadd(x[2], x[3]);
    float2 b1 = csub(x[1], x[4]), b2 = csub(x[2], x[3]);
    float2 m1 = make_float2(x[0].x + c1 * a1.x + c2 * a2.x, x[0].y + c1 * a1.y + c2 * a2.y);
    float2 m2 = make_float2(x[0].x + c2 * a1.x + c1 * a2.x, x[0].y + c2 * a1.y + c1 * a2.y);
    // qturn applies the transform's sign of i
    float2 n1 = qturn<INV>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    float2 n2 = qturn<INV>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    x[0] = make_float2(x[0].x + a1.x + a2.x, x[0].y + a1.y + a2.y);
    x[1] = cadd(m1, n1);
    x[4] = csub(m1, n1);
    x[2] = cadd(m2, n2);
    x[3] = csub(m2, n2);
  }
};

constexpr int first_factor(int r) {
  return (r % 4 == 0 && r != 4) ? 4 : (r % 2 == 0 ? 2 : (r % 3 == 0 ? 3 : (r % 5 == 0 ? 5 : r)));
}

// Composite R = A * B:  n = a + A b,  k = kb + B ka.
template <int R, bool INV>
struct Dft {
  static constexpr int A = first_factor(R);
  static constexpr int B = R / A;
  static_assert(A * B == R && A > 1 && B > 1, "only 2,3,5-smooth radices");
  __device__ __forceinline__ static void run(float2* x) {
    float2 t[R];
    StaticFor<0, A>::run([&](auto ca) {
      constexpr int a = decltype(ca)::value;
      float2 s[B];
#pragma unroll
      for (int b = 0; b < B; ++b) s[b] = x[a + A * b];
      Dft<B, INV>::run(s);
      StaticFor<0, B>::run([&](auto ckb) {
        constexpr int kb = decltype(ckb)::value;
        t[a * B + kb] = rot<R, a * kb, INV>(s[kb]);
      });
    });
#pragma unroll
    for (int kb = 0; kb < B; ++kb) {
      float2 s[A];
#pragma unroll
      for (int a = 0; a < A; ++a) s[a] = t[a * B + kb];
      Dft<A, INV>::run(s);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) x[kb + B * ka] = s[ka];
    }
  }
};

// ---------------------------------------------------------------- 2D FFT in LDS
// Thread mapping (t = threadIdx.x, T = M*R2 threads, E = ceil(R1/R2)):
//   column stage 1: line = t % M (column kx), r = t / M; holds x[m] = Z[r + R2 m][line]
//   row stage 2 output: sg = t % R2, y = t / R2; holds out[e*R2 + k2] =
//       b[y][sg*E + e + R1*k2]     (e < E, k2 < R2), valid where s = sg*E + e < R1
// When R2 does not divide R1 the last stage-2 slots of some threads are idle (has_s).
template <int M_, int R1_, int R2_>
struct Fft2Shape {
  static constexpr int M = M_, R1 = R1_, R2 = R2_;
  static constexpr int T = M * R2;
  static constexpr int E = (R1 + R2 - 1) / R2;  // stage-2 DFTs per thread
  static constexpr bool EXACT = (E * R2 == R1);
  static constexpr int XN = E * R2 > R1 ? E * R2 : R1;   // registers per thread (complex)
  // stage-1 output index s = sg*E + e exists
  __device__ __forceinline__ static bool has_s(int s) { return EXACT || s < R1; }
  static constexpr int TP = M + 1;            // transpose pitch (float2)
  static constexpr int SP = R2 * M + 2;       // exchange pitch per stage-1 output index s
  static constexpr int LDS_ELEMS = (M * TP > R1 * SP) ? M * TP : R1 * SP;
  static constexpr size_t LDS_BYTES = size_t(LDS_ELEMS) * sizeof(float2);
  // component-split variant: each exchange moves the real parts, then the imaginary
  // parts, through a float buffer of half the bytes
  static constexpr int SPF = R2 * M + 4;      // float exchange pitch per s
  static constexpr int LDS_SPLIT_FLOATS = (M * TP > R1 * SPF) ? M * TP : R1 * SPF;
  static_assert(R1 * R2 == M && R1 >= R2, "M = R1*R2 with R1 >= R2");
  static_assert(T <= 1024, "at most 1024 threads");
  static_assert(!EXACT || R1 * (R2 * M + 4) <= LDS_SPLIT_FLOATS, "paired exchange fits the split buffer");
};

// Twiddle table tw[k] = exp(sgn i 2 pi k / M), FP64-rounded; index (r*s) mod M.
template <class S, bool INV>
__device__ __forceinline__ void fft2_block(float2 (&x)[S::XN], float2* __restrict__ lds,
                                           const float2* __restrict__ tw) {
  constexpr int M = S::M, R1 = S::R1, R2 = S::R2, E = S::E, TP = S::TP, SP = S::SP;
  const int t = threadIdx.x;
  const int line = t % M;
  // r is uniform across a wave when M is a multiple of the wave size: say so, so
  // that the twiddle loads below become scalar loads
  int r_;
  if constexpr (M % 64 == 0) r_ = __builtin_amdgcn_readfirstlane(t / M);
  else r_ = t / M;
  const int r = r_;

  // ---- column pass, stage 1 (radix R1 over m), twiddle W_M^(r s)
  Dft<R1, INV>::run(x);
#pragma unroll
  for (int s = 1; s < R1; ++s) x[s] = cmul(x[s], tw[(r * s) % M]);
#pragma unroll
  for (int s = 0; s < R1; ++s) lds[s * SP + r * M + line] = x[s];
  __syncthreads();
  // ---- column pass, stage 2 (radix R2 over r) for s = sg*E + e, sg = t / M
  {
    const int sg = t / M;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = sg * E + e;
      if (!S::has_s(s)) continue;
      float2 y[R2];
#pragma unroll
      for (int rr = 0; rr < R2; ++rr) y[rr] = lds[s * SP + rr * M + line];
      Dft<R2, INV>::run(y);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) x[e * R2 + k2] = y[k2];
    }
    __syncthreads();
    // transpose: element (row Y = s + R1*k2, column = line)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = sg * E + e;
      if (!S::has_s(s)) continue;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) lds[(s + R1 * k2) * TP + line] = x[e * R2 + k2];
    }
  }
  __syncthreads();
  // ---- row pass, stage 1: thread (row = line, r) reads columns r + R2*m
#pragma unroll
  for (int m = 0; m < R1; ++m) x[m] = lds[line * TP + r + R2 * m];
  __syncthreads();
  Dft<R1, INV>::run(x);
#pragma unroll
  for (int s = 1; s < R1; ++s) x[s] = cmul(x[s], tw[(r * s) % M]);
#pragma unroll
  for (int s = 0; s < R1; ++s) lds[s * SP + r * M + line] = x[s];
  __syncthreads();
  // ---- row pass, stage 2: thread (sg = t % R2, y = t / R2)
  {
    const int sg = t % R2;
    const int y = t / R2;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = sg * E + e;
      if (!S::has_s(s)) continue;
      float2 v[R2];
#pragma unroll
      for (int rr = 0; rr < R2; ++rr) v[rr] = lds[s * SP + rr * M + y];
      Dft<R2, INV>::run(v);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) x[e * R2 + k2] = v[k2];
    }
  }
}


// Same transform, thread mapping and results as fft2_block, with every LDS exchange
// done in two rounds -- real parts, then imaginary parts -- through a float buffer
// of half the bytes (Shape::LDS_SPLIT_FLOATS), so two workgroups fit in one CU's
// LDS and overlap each other's barriers.  No extra registers: a component is read
// back into the slots its own values were written from.
template <class S, bool INV>
__device__ __forceinline__ void fft2_block_split(float2 (&x)[S::XN], float* __restrict__ lds,
                                                 const float2* __restrict__ tw) {
  constexpr int M = S::M, R1 = S::R1, R2 = S::R2, E = S::E, TP = S::TP, SPF = S::SPF;
  const int t = threadIdx.x;
  const int line = t % M;
  int r_;
  if constexpr (M % 64 == 0) r_ = __builtin_amdgcn_readfirstlane(t / M);
  else r_ = t / M;
  const int r = r_;
  const int sgc = t / M;

  // ---- column pass, stage 1
  Dft<R1, INV>::run(x);
#pragma unroll
  for (int s = 1; s < R1; ++s) x[s] = cmul(x[s], tw[(r * s) % M]);
  // ---- exchange 1: x[s] of (line, r) -> thread (line, sgc) gets x[e*R2 + rr] = X1[s = sgc*E + e][rr]
  if constexpr (E % 2 == 0 && S::EXACT) {
    // the values of stage-1 outputs s and s+1 side by side (s even): each thread writes and
    // reads 8 bytes at a time, half the LDS instructions for the same bytes
    float2* lds2 = reinterpret_cast<float2*>(lds);
    constexpr int SP2 = R2 * M + 4;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
      for (int s = 0; s < R1; s += 2)
        lds2[(s / 2) * SP2 + r * M + line] = comp ? make_float2(x[s].y, x[s + 1].y) : make_float2(x[s].x, x[s + 1].x);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; e += 2) {
        const int i = (sgc * E + e) / 2;
#pragma unroll
        for (int rr = 0; rr < R2; ++rr) {
          const float2 v = lds2[i * SP2 + rr * M + line];
          if (comp) { x[e * R2 + rr].y = v.x; x[(e + 1) * R2 + rr].y = v.y; }
          else { x[e * R2 + rr].x = v.x; x[(e + 1) * R2 + rr].x = v.y; }
        }
      }
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
      for (int s = 0; s < R1; ++s) lds[s * SPF + r * M + line] = comp ? x[s].y : x[s].x;
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int s = sgc * E + e;
        if (!S::has_s(s)) continue;
#pragma unroll
        for (int rr = 0; rr < R2; ++rr) {
          const float v = lds[s * SPF + rr * M + line];
          if (comp) x[e * R2 + rr].y = v;
          else x[e * R2 + rr].x = v;
        }
      }
      __syncthreads();
    }
  }
  // ---- column pass, stage 2 (radix R2 over rr), in place per e
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (S::has_s(sgc * E + e)) Dft<R2, INV>::run(&x[e * R2]);
  // ---- transpose: (row Y = s + R1*k2, column line) -> thread (row line, r) gets columns r + R2*m
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = sgc * E + e;
      if (!S::has_s(s)) continue;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) lds[(s + R1 * k2) * TP + line] = comp ? x[e * R2 + k2].y : x[e * R2 + k2].x;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < R1; ++m) {
      const float v = lds[line * TP + r + R2 * m];
      if (comp) x[m].y = v;
      else x[m].x = v;
    }
    __syncthreads();
  }
  // ---- row pass, stage 1
  Dft<R1, INV>::run(x);
#pragma unroll
  for (int s = 1; s < R1; ++s) x[s] = cmul(x[s], tw[(r * s) % M]);
  // ---- exchange 3: thread (sg = t % R2, y = t / R2) gets X1[s = sg*E + e][rr] of row y
  const int sg = t % R2, yy = t / R2;
  if constexpr (E % 2 == 0 && S::EXACT) {
    float2* lds2 = reinterpret_cast<float2*>(lds);
    constexpr int SP2 = R2 * M + 4;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
      for (int s = 0; s < R1; s += 2)
        lds2[(s / 2) * SP2 + r * M + line] = comp ? make_float2(x[s].y, x[s + 1].y) : make_float2(x[s].x, x[s + 1].x);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; e += 2) {
        const int i = (sg * E + e) / 2;
#pragma unroll
        for (int rr = 0; rr < R2; ++rr) {
          const float2 v = lds2[i * SP2 + rr * M + yy];
          if (comp) { x[e * R2 + rr].y = v.x; x[(e + 1) * R2 + rr].y = v.y; }
          else { x[e * R2 + rr].x = v.x; x[(e + 1) * R2 + rr].x = v.y; }
        }
      }
      if (comp == 0) __syncthreads();
    }
  } else {
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
      for (int s = 0; s < R1; ++s) lds[s * SPF + r * M + line] = comp ? x[s].y : x[s].x;
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int s = sg * E + e;
        if (!S::has_s(s)) continue;
#pragma unroll
        for (int rr = 0; rr < R2; ++rr) {
          const float v = lds[s * SPF + rr * M + yy];
          if (comp) x[e * R2 + rr].y = v;
          else x[e * R2 + rr].x = v;
        }
      }
      if (comp == 0) __syncthreads();
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (S::has_s(sg * E + e)) Dft<R2, INV>::run(&x[e * R2]);
}

// ---------------------------------------------------------------- rectangular 2D FFT in LDS
// An MC x MR block (MC rows, MR columns): column transforms of length MC = R1C * R2C over
// the MR columns, then row transforms of length MR = R1R * R2R over the MC rows, with one
// thread count T = MR * R2C = MC * R2R.  Same two-stage split per pass and component-split
// exchanges as fft2_block_split.  Twiddles come from the MR-point table: W_MC^k = W_MR^(P k)
// with P = MR / MC.
//   column pass input:  thread (line = t % MR, r = t / MR) holds x[m] = Z[r + R2C m][line]
//   row pass output:    thread (sg = t % R2R, y = t / R2R) holds out[e*R2R + k2] =
//                       b[y][sg*ER + e + R1R*k2]  (valid where sg*ER + e < R1R)
template <int MC_, int R1C_, int R2C_, int MR_, int R1R_, int R2R_>
struct RectShape {
  static constexpr int MC = MC_, R1C = R1C_, R2C = R2C_, MR = MR_, R1R = R1R_, R2R = R2R_;
  static constexpr int P = MR / MC;
  static constexpr int T = MR * R2C;
  static constexpr int EC = (R1C + R2C - 1) / R2C, ER = (R1R + R2R - 1) / R2R;
  static constexpr int max2(int a, int b) { return a > b ? a : b; }
  static constexpr int XN = max2(max2(R1C, EC * R2C), max2(R1R, ER * R2R));
  static constexpr int SPC = R2C * MR + 4;   // exchange pitch per column-pass output s (floats)
  static constexpr int SPR = R2R * MC + 4;   // exchange pitch per row-pass output s
  static constexpr int TP = MR + 1;          // transpose pitch
  static constexpr int LDS_FLOATS = max2(max2(R1C * SPC, MC * TP), R1R * SPR);
  __device__ __forceinline__ static bool has_c(int s) { return s < R1C; }
  __device__ __forceinline__ static bool has_r(int s) { return s < R1R; }
  static_assert(R1C * R2C == MC && R1R * R2R == MR && MR % MC == 0, "factorisations");
  static_assert(T == MC * R2R && T <= 1024, "one thread count for both passes");
};

template <class S, bool INV>
__device__ __forceinline__ void fft2_rect_split(float2 (&x)[S::XN], float* __restrict__ lds,
                                                const float2* __restrict__ tw) {
  constexpr int MC = S::MC, R1C = S::R1C, R2C = S::R2C, EC = S::EC, SPC = S::SPC;
  constexpr int MR = S::MR, R1R = S::R1R, R2R = S::R2R, ER = S::ER, SPR = S::SPR, TP = S::TP, P = S::P;
  const int t = threadIdx.x;
  const int line = t % MR;
  int r_;   // uniform across a wave when MR is a multiple of the wave size
  if constexpr (MR % 64 == 0) r_ = __builtin_amdgcn_readfirstlane(t / MR);
  else r_ = t / MR;
  const int rc = r_;
  // ---- column pass, stage 1 (radix R1C over m), twiddle W_MC^(r s) = W_MR^(P r s)
  Dft<R1C, INV>::run(x);
#pragma unroll
  for (int s = 1; s < R1C; ++s) x[s] = cmul(x[s], tw[(P * rc * s) % MR]);
  // ---- exchange 1: thread (line, sgc = t / MR) gets x[e*R2C + rr] = X1[sgc*EC + e][rr]
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
    for (int s = 0; s < R1C; ++s) lds[s * SPC + rc * MR + line] = comp ? x[s].y : x[s].x;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EC; ++e) {
      const int s = rc * EC + e;
      if (!S::has_c(s)) continue;
#pragma unroll
      for (int rr = 0; rr < R2C; ++rr) {
        const float v = lds[s * SPC + rr * MR + line];
        if (comp) x[e * R2C + rr].y = v;
        else x[e * R2C + rr].x = v;
      }
    }
    __syncthreads();
  }
  // ---- column pass, stage 2 (radix R2C over rr)
#pragma unroll
  for (int e = 0; e < EC; ++e)
    if (S::has_c(rc * EC + e)) Dft<R2C, INV>::run(&x[e * R2C]);
  // ---- transpose: (row Y = s + R1C*k2, column line) -> thread (row = t % MC, r = t / MC)
  // gets columns r + R2R*m of its row
  const int row = t % MC, rr_ = t / MC;
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
    for (int e = 0; e < EC; ++e) {
      const int s = rc * EC + e;
      if (!S::has_c(s)) continue;
#pragma unroll
      for (int k2 = 0; k2 < R2C; ++k2) lds[(s + R1C * k2) * TP + line] = comp ? x[e * R2C + k2].y : x[e * R2C + k2].x;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < R1R; ++m) {
      const float v = lds[row * TP + rr_ + R2R * m];
      if (comp) x[m].y = v;
      else x[m].x = v;
    }
    __syncthreads();
  }
  // ---- row pass, stage 1 (radix R1R), twiddle W_MR^(r s)
  Dft<R1R, INV>::run(x);
#pragma unroll
  for (int s = 1; s < R1R; ++s) x[s] = cmul(x[s], tw[(rr_ * s) % MR]);
  // ---- exchange 3: thread (sg = t % R2R, y = t / R2R) gets X1[sg*ER + e][rr] of row y
  const int sg = t % R2R, yy = t / R2R;
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
    for (int s = 0; s < R1R; ++s) lds[s * SPR + rr_ * MC + row] = comp ? x[s].y : x[s].x;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < ER; ++e) {
      const int s = sg * ER + e;
      if (!S::has_r(s)) continue;
#pragma unroll
      for (int q = 0; q < R2R; ++q) {
        const float v = lds[s * SPR + q * MC + yy];
        if (comp) x[e * R2R + q].y = v;
        else x[e * R2R + q].x = v;
      }
    }
    if (comp == 0) __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < ER; ++e)
    if (S::has_r(sg * ER + e)) Dft<R2R, INV>::run(&x[e * R2R]);
}

}  // namespace tomo

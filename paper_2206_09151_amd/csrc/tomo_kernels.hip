// gfx950 kernels of the reconstruction hot path.
//
//   k_spectra, k_planes (fft_kernels.hpp, instantiated per size in fft_sizes_*.hip):
//               contrast, 2D DFT and the eq. 11 filter; depth propagation (eq. 3) and
//               the inverse 2D FFTs that write the plane stacks.  This file keeps
//               the size table that dispatches them.
//   k_grid_*    trilinear gather of the stacks at every voxel's view-frame position
//               (text after eq. 11), summed over the batch's views in ascending
//               order in registers, then one read-modify-write of V (no atomics).
//   k_filter_table, k_sampling_*: plan-time tables in FP64, stored FP32.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fft_kernels.hpp"
#include "fft_sizes.hpp"
#include "geom.hpp"
#include "tomo_internal.hpp"

namespace tomo {

// ------------------------------------------------------------------ inspection
__global__ void k_spectra_out(const float4* __restrict__ q, float2* __restrict__ out, size_t count,
                              float m2) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float4 v = q[i];
  // F G = M^2 (Q1 - Q2) / (1 + i),  1/(1+i) = (1 - i)/2
  const float a = v.x - v.z, b = v.y - v.w;
  out[i] = make_float2(0.5f * m2 * (a + b), 0.5f * m2 * (b - a));
}

// ------------------------------------------------------------------ K4: gridding
constexpr int GT = 16;  // voxel tile edge (x) x (z or y) per 256-thread workgroup

// Box geometry shared by the LDS-staged gridding kernels: 16-byte chunks of VEC stored
// values, BOXW columns per staged (row, plane), LDS pitch BOXP, AX_BOXH planes per row.
template <class InT>
struct AxisBox;
template <>
struct AxisBox<float> {   // 4 values per 16-byte chunk
  static constexpr int VEC = 4, BOXW = 28, BOXP = 28;
};
template <>
struct AxisBox<__hip_bfloat16> {   // 8 values per chunk
  static constexpr int VEC = 8, BOXW = 32, BOXP = 36;
};
template <>
struct AxisBox<__half> {
  static constexpr int VEC = 8, BOXW = 32, BOXP = 36;
};
constexpr int AX_BOXH = 24;     // planes staged per row

union Chunk16 {
  uint4 u;
  float f[4];
  unsigned short h[8];
};

template <class InT>
__device__ __forceinline__ float chunk_value(const Chunk16& c, int k);
template <>
__device__ __forceinline__ float chunk_value<float>(const Chunk16& c, int k) { return c.f[k]; }
template <>
__device__ __forceinline__ float chunk_value<__hip_bfloat16>(const Chunk16& c, int k) {
  return __uint_as_float(unsigned(c.h[k]) << 16);
}
template <>
__device__ __forceinline__ float chunk_value<__half>(const Chunk16& c, int k) {
  return __half2float(__ushort_as_half(c.h[k]));
}

// Keeps v in a register as an opaque value: the compiler may not hoist what is computed
// from it out of the loop it sits in (for values needed only on rarely taken paths).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Single-axis views (v = y exactly, M - N even): the detector row of voxel row iy is
// iy + (M-N)/2 exactly, so the trilinear weights reduce to bilinear ones in (plane, col),
// shared by the YB voxel rows of a thread.  Per view, the workgroup's 16 x 16 (x, z) tile
// maps into a rotated square of the (plane, col) grid; its bounding box with every tap (at
// most 24 planes x 28 columns; the column start rounded down to a 16-byte boundary) is staged
// in LDS for the YB rows, zero outside the stack, so the bilinear taps are plain LDS reads.
// Only the view's own box is fetched (17 x 20 at 0 degrees, the full 24 x 28 near 45): over a
// half-turn scan that is 17% fewer bytes into LDS than the fixed 24 x 28 box.
//
// The footprints of FP32, BF16 or FP16 planes are fetched straight into LDS in their
// storage type.  The staged box is chunk-linear in 16-byte slots: 7 chunks per (row, plane)
// for FP32; for 16-bit values 4 chunks and a fifth slot that is never fetched, so that a
// (row, plane) spans 20 dwords rather than 16 and planes lp and lp + 2 of the rotated tap
// pattern fall on different LDS banks (at 16 dwords a wave's reads met 3.3 bank cycles per
// half-wave against 1.8 at 20, in a count over the scan's angles).  Wave w's
// i-th load of a view covers slots 256 i + 64 w + lane, and buffer loads with the LDS
// destination write them in place (lane l's 16 bytes land 16 l bytes after the wave's LDS
// base; lanes past the last chunk are switched off and write nothing).  Chunks outside the
// stack get an offset beyond the buffer's range, which the hardware fills with zeros, so no
// masks or register staging are needed.  Two box buffers alternate: view n + 1 is in flight
// while view n is interpolated, and each view takes one barrier.  The 4- and 8-row FP32 kernels
// keep one box instead (fetch, wait, interpolate, two barriers per view): at 4 rows half the
// LDS lets eight workgroups share a CU instead of seven, so a 128^3 volume's 2048 tiles run in
// one round rather than 1.14 (32.3 against 34.5 us per 15-view launch); at 8 rows seven instead
// of three (34.1 against 42.3 us).  The 16-bit 4-row kernel fits eight workgroups with two
// boxes; at 8 rows one box (eight workgroups instead of five) made the 16-bit kernel slower
// (50.8 against 47.2 us per 32-view launch).  A 16-bit tap pair (lc, lc + 1) is the 32-bit
// window at bit 16 (lc & 1) of the two dwords from element 2 (lc >> 1); FP16 values are
// unscaled through the interpolation weights (the per-view scale is a power of two).
template <class InT>
struct DmaBox;
template <>
struct DmaBox<float> {
  static constexpr int VEC = 4, BOXW = 28;
};
template <>
struct DmaBox<__hip_bfloat16> {
  static constexpr int VEC = 8, BOXW = 32;
};
template <>
struct DmaBox<__half> {
  static constexpr int VEC = 8, BOXW = 32;
};
typedef __attribute__((address_space(3))) void lds_void_t;
constexpr unsigned kOutOfRange = 0x80000000u;      // beyond every buffer range: reads as zero

template <int YB, class InT>
__global__ __launch_bounds__(256) void k_grid_axis_dma(const InT* __restrict__ stack,
                                                       const ViewGeom* __restrict__ geom,
                                                       const float* __restrict__ scale,
                                                       float* __restrict__ vol, int N, int M, int K, int nb,
                                                       int accumulate, int flat, double hm, double hk) {
  constexpr int VEC = DmaBox<InT>::VEC, BOXW = DmaBox<InT>::BOXW, QN = BOXW / VEC;
  constexpr int ES = int(sizeof(InT));                  // bytes per stored value
  constexpr int QP = ES == 2 ? QN + 1 : QN;             // 16-byte slots per staged (row, plane)
  constexpr int PITCH = QP * 4;                         // dwords per staged (row, plane)
  constexpr int NE = YB * AX_BOXH * QP;                 // slots per staged view
  constexpr int PER = (NE + 255) / 256;                 // loads per thread per view
  // 16-bit values: one dword of padding, the pair read may touch the dword after a row's last
  constexpr int PAD = ES == 2 ? 4 : 0;
  constexpr bool ONE_BOX = YB >= 4 && ES == 4;
  __shared__ __attribute__((aligned(16))) unsigned box0[NE * 4 + PAD];
  __shared__ __attribute__((aligned(16))) unsigned box1[ONE_BOX ? 4 : NE * 4 + PAD];
  const int ntx = (N + GT - 1) / GT;
  const int tiles = ntx * ntx;
  const int wg = blockIdx.x, xcd = wg & 7, k = wg >> 3;
  const int yblk = xcd + 8 * (k / tiles), tile = k % tiles;
  const int y0 = yblk * YB;
  if (y0 >= N) return;                                  // uniform
  const int tx0 = (tile % ntx) * GT, tz0 = (tile / ntx) * GT;
  const int ix = tx0 + (threadIdx.x % GT);
  const int iz = tz0 + (threadIdx.x / GT);
  const bool live = ix < N && iz < N;
  const double c = 0.5 * (N - 1);
  const double rx = ix - c, rz = iz - c;
  const int rowoff = (M - N) / 2;
  const size_t view_sz = size_t(K) * M * M;
  const int wbase = (threadIdx.x & ~63) * 4;            // this wave's first dword in a box, per load
  const int lane = threadIdx.x & 63;

  // Box origins: lane l of every wave computes the origin of view obase + l (FP64, from
  // the tile corners); per view the workgroup-uniform origin is read out of lane n - obase
  // into scalar registers, so the per-view cost is two lane reads.
  // The box of a view: columns c0 .. c0 + cw - 1 (cw a multiple of VEC) and planes
  // p0 .. p0 + bh - 1, from the tile's corner extremes; the taps of a voxel lie at most one
  // past the floor of its coordinates, and one more column and plane absorb a last-bit
  // difference between the corner and the voxel arithmetic (within the 24 x 28 maximum).
  int obase = -64, lane_c0 = 0, lane_p0 = 0, lane_cw = 0, lane_bh = 0;
  auto origin = [&](int n, int& c0, int& p0, int& cw, int& bh) {
    if (n >= obase + 64) {
      obase = n;
      const int v = n + lane;
      int cc = 0, pp = 0, ww = 0, hh = 0;
      if (v < nb) {
        const int t0 = opaque(tx0), z0 = opaque(tz0);
        const double ax = t0 - c, bx = t0 + GT - 1 - c, az = z0 - c, bz = z0 + GT - 1 - c;
        const ViewGeom& g = geom[v];
        const double cmin = fmin(g.u[0] * ax, g.u[0] * bx) + fmin(g.u[2] * az, g.u[2] * bz) + hm;
        const double cmax = fmax(g.u[0] * ax, g.u[0] * bx) + fmax(g.u[2] * az, g.u[2] * bz) + hm;
        const double pmin = fmin(g.d[0] * ax, g.d[0] * bx) + fmin(g.d[2] * az, g.d[2] * bz) + hk;
        const double pmax = fmax(g.d[0] * ax, g.d[0] * bx) + fmax(g.d[2] * az, g.d[2] * bz) + hk;
        cc = int(floor(cmin)) & ~(VEC - 1);
        pp = flat ? 0 : int(floor(pmin));
        ww = min(BOXW, (int(floor(cmax)) - cc + 3 + VEC - 1) & ~(VEC - 1));
        hh = flat ? 2 : min(AX_BOXH, int(floor(pmax)) - pp + 3);
      }
      lane_c0 = cc;
      lane_p0 = pp;
      lane_cw = ww;
      lane_bh = hh;
    }
    c0 = __builtin_amdgcn_readlane(lane_c0, n - obase);
    p0 = __builtin_amdgcn_readlane(lane_p0, n - obase);
    cw = __builtin_amdgcn_readlane(lane_cw, n - obase);
    bh = __builtin_amdgcn_readlane(lane_bh, n - obase);
  };
  // per chunk slot: byte offset from the box origin (rows all present), and for boxes that
  // cross the stack's edge its (plane, column) position and detector-row term
  // (the host launches this kernel only for M a multiple of VEC and views below 2^31 bytes)
  const bool rows_in = y0 + YB <= N && y0 + rowoff >= 0 && y0 + YB - 1 + rowoff < M;
  unsigned cfo[PER];
  int cq[PER], cpl[PER], crow[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i;
    const int q = e % QP, pl = (e / QP) % AX_BOXH, j = e / (QP * AX_BOXH);
    const int row = y0 + j + rowoff;
    cq[i] = VEC * q;                                    // the spare slot (q = QN) has cq = BOXW >= cw
    cpl[i] = pl;
    crow[i] = (e < NE && y0 + j < N && unsigned(row) < unsigned(M)) ? row * K : -1;
    cfo[i] = rows_in ? unsigned((row * K + pl) * M + VEC * q) * unsigned(ES) : kOutOfRange;
  }
  // slot i exists for every thread below the last load; in the last one only below NE
  auto has = [&](int i) { return NE % 256 == 0 || i < PER - 1 || int(threadIdx.x) + 256 * i < NE; };
  auto load = [&](int n, int c0, int p0, int cw, int bh, unsigned* dst) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<InT*>(stack + size_t(n) * view_sz), short(0), int(view_sz * ES), 0x00020000);
    // slots outside the view's box fetch nothing (their LDS words are never read)
    if (rows_in && p0 >= 0 && p0 + bh <= K && c0 >= 0 && c0 + cw <= M) {
      const int so = (p0 * M + c0) * ES;
#pragma unroll
      for (int i = 0; i < PER; ++i)
        if (has(i) && cpl[i] < bh && cq[i] < cw)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(dst + 1024 * i + wbase), 16,
                                                   int(cfo[i]), so, 0, 0);
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        if (has(i) && cpl[i] < bh && cq[i] < cw) {
          const int pp = p0 + cpl[i], cc = c0 + cq[i];
          const bool ok = crow[i] >= 0 && unsigned(pp) < unsigned(K) && unsigned(cc) < unsigned(M);
          const unsigned off = ok ? unsigned((crow[i] + pp) * M + cc) * unsigned(ES) : kOutOfRange;
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(dst + 1024 * i + wbase), 16, int(off), 0,
                                                   0, 0);
        }
      }
    }
  };

  float acc[YB];
#pragma unroll
  for (int j = 0; j < YB; ++j) acc[j] = 0.0f;
  int oc0 = 0, op0 = 0, oc1 = 0, op1 = 0;              // origins of the views in each buffer
  int ow0 = 0, oh0 = 0, ow1 = 0, oh1 = 0;              // and their box extents
  // view n from buffer b: wait for this wave's loads of it (and for its own reads of the
  // other buffer), barrier (every wave's share has landed; every wave is done with the
  // other buffer), issue view n + 1 into the other buffer, interpolate
  // wait for this wave's loads and LDS reads, then for every wave (a plain barrier: the
  // workgroup fence of __syncthreads is not needed after the wait)
  auto sync = [&]() {
    __builtin_amdgcn_s_waitcnt(7 << 4);                 // vmcnt(0) lgkmcnt(0)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // interpolation of view n from its staged box bx (origin column cb, plane pb)
  auto interp = [&](const unsigned* bx, int cb, int pb, int n) {
    if (live) {
      const ViewGeom& g = geom[n];
      // flat (one plane, K = 1): a zero depth direction gives fp = 0 (hk = 0, origin plane
      // 0), so lp = 0 and tz = 0, and the second plane's taps (zero-filled) get weight 0
      const double d0 = flat ? 0.0 : g.d[0], d2 = flat ? 0.0 : g.d[2];
      const double fc = fmax(g.u[0] * rx + g.u[2] * rz + (hm - cb), 0.0);
      const double fp = fmax(d0 * rx + d2 * rz + (hk - pb), 0.0);
      // fc, fp >= 0: truncation is the floor, fract the remainder (exact in FP64)
      const int lc = int(fc), lp = int(fp);
      float tx = float(__builtin_amdgcn_fract(fc));
      const float tz = float(__builtin_amdgcn_fract(fp));
      float ux = 1.0f - tx;
      if constexpr (std::is_same<InT, __half>::value) {
        const float inv = 1.0f / scale[n];              // exact: the scale is a power of two
        ux *= inv;
        tx *= inv;
      }
      const float w00 = (1.0f - tz) * ux, w01 = (1.0f - tz) * tx;
      const float w10 = tz * ux, w11 = tz * tx;
      const int pofs = int(__umul24(unsigned(lp), unsigned(PITCH)));   // lp < AX_BOXH
#pragma unroll
      for (int j = 0; j < YB; ++j) {
        float a0, a1, b0, b1;                           // taps (lp, lc), (lp, lc+1), (lp+1, lc), (lp+1, lc+1)
        if constexpr (ES == 4) {
          const float* r0 = reinterpret_cast<const float*>(bx) + j * AX_BOXH * PITCH + pofs + lc;
          const float* r1 = r0 + PITCH;
          a0 = r0[0], a1 = r0[1], b0 = r1[0], b1 = r1[1];
        } else {
          const unsigned* r0 = bx + j * AX_BOXH * PITCH + pofs + (lc >> 1);
          const unsigned* r1 = r0 + PITCH;
          const unsigned sh = unsigned(lc & 1) * 16u;
          const unsigned pa = __builtin_amdgcn_alignbit(r0[1], r0[0], sh);
          const unsigned pb2 = __builtin_amdgcn_alignbit(r1[1], r1[0], sh);
          if constexpr (std::is_same<InT, __half>::value) {
            a0 = __half2float(__ushort_as_half((unsigned short)(pa & 0xffffu)));
            a1 = __half2float(__ushort_as_half((unsigned short)(pa >> 16)));
            b0 = __half2float(__ushort_as_half((unsigned short)(pb2 & 0xffffu)));
            b1 = __half2float(__ushort_as_half((unsigned short)(pb2 >> 16)));
          } else {
            a0 = __uint_as_float(pa << 16), a1 = __uint_as_float(pa & 0xffff0000u);
            b0 = __uint_as_float(pb2 << 16), b1 = __uint_as_float(pb2 & 0xffff0000u);
          }
        }
        acc[j] = fmaf(w11, b1, fmaf(w10, b0, fmaf(w01, a1, fmaf(w00, a0, acc[j]))));
      }
    }
  };
  auto step = [&](unsigned* bx, int& cb, int& pb, unsigned* other, int& co, int& po, int& wo, int& ho, int n) {
    if (n >= nb) return;                                // uniform
    sync();
    if (n + 1 < nb) {
      origin(n + 1, co, po, wo, ho);
      load(n + 1, co, po, wo, ho, other);
    }
    interp(bx, cb, pb, n);
  };
  if constexpr (ONE_BOX) {
    // one box: every wave is done with the previous view, fetch, every wave's share has
    // landed, interpolate
    for (int n = 0; n < nb; ++n) {
      if (n > 0) sync();
      origin(n, oc0, op0, ow0, oh0);
      load(n, oc0, op0, ow0, oh0, box0);
      sync();
      interp(box0, oc0, op0, n);
    }
  } else {
    if (nb > 0) {
      origin(0, oc0, op0, ow0, oh0);
      load(0, oc0, op0, ow0, oh0, box0);
    }
    for (int n0 = 0; n0 < nb; n0 += 2) {
      step(box0, oc0, op0, box1, oc1, op1, ow1, oh1, n0);
      step(box1, oc1, op1, box0, oc0, op0, ow0, oh0, n0 + 1);
    }
  }
  if (!live) return;
#pragma unroll
  for (int j = 0; j < YB; ++j) {
    const int iy = y0 + j;
    if (iy < N) {
      float* dst = vol + (size_t(iz) * N + iy) * N + ix;
      *dst = accumulate ? *dst + acc[j] : acc[j];
    }
  }
}

// General view frames with a compact footprint (e.g. single-axis scans with a tilt):
// per view the bounding box of the workgroup's 16 (x) x YB (y) x 16 (z) voxel tile in
// (row, plane, column) coordinates is staged into LDS when it fits in BR x 24 x BOXW;
// the eight trilinear taps are then LDS reads.  Views whose box does not fit (steep
// tilts, directions far from the rotation axis) are gathered from global memory.
constexpr int BX_BR = 12;       // detector rows staged per view

template <int YB, class InT>
__global__ __launch_bounds__(256) void k_grid_box(const InT* __restrict__ stack,
                                                  const ViewGeom* __restrict__ geom,
                                                  const float* __restrict__ scale,
                                                  float* __restrict__ vol, int N, int M, int K,
                                                  int nb, int accumulate, int flat) {
  using B = AxisBox<InT>;
  constexpr int VEC = B::VEC, BOXW = B::BOXW, BOXP = B::BOXP;
  constexpr int BR = BX_BR, BH = AX_BOXH;
  constexpr int QN = BOXW / VEC;
  constexpr int NE = BR * BH * QN;
  constexpr int PER = (NE + 255) / 256;
  __shared__ float box[BR][BH][BOXP];
  const int ntx = (N + GT - 1) / GT;
  const int tiles = ntx * ntx;
  const int wg = blockIdx.x, xcd = wg & 7, k = wg >> 3;
  const int yblk = xcd + 8 * (k / tiles), tile = k % tiles;
  const int y0 = yblk * YB;
  if (y0 >= N) return;                                  // uniform
  const int tx0 = (tile % ntx) * GT, tz0 = (tile / ntx) * GT;
  const int ix = tx0 + (threadIdx.x % GT);
  const int iz = tz0 + (threadIdx.x / GT);
  const bool live = ix < N && iz < N;
  const double c = 0.5 * (N - 1);
  const double rx = ix - c, rz = iz - c;
  const double hm = 0.5 * (M - 1), hk = 0.5 * (K - 1);
  const size_t plane_sz = size_t(K) * M;
  const bool vec = (M % VEC) == 0;
  const double lo[3] = {tx0 - c, y0 - c, tz0 - c};
  const double hi[3] = {tx0 + GT - 1 - c, y0 + YB - 1 - c, tz0 + GT - 1 - c};

  // box of view n: origin (r0, p0, c0) and whether it fits (uniform)
  auto origin = [&](int n, int& r0, int& p0, int& c0) -> bool {
    const ViewGeom& g = geom[n];
    double cmin = hm, cmax = hm, rmin = hm, rmax = hm, pmin = hk, pmax = hk;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cmin += fmin(g.u[a] * lo[a], g.u[a] * hi[a]);
      cmax += fmax(g.u[a] * lo[a], g.u[a] * hi[a]);
      rmin += fmin(g.v[a] * lo[a], g.v[a] * hi[a]);
      rmax += fmax(g.v[a] * lo[a], g.v[a] * hi[a]);
      pmin += fmin(g.d[a] * lo[a], g.d[a] * hi[a]);
      pmax += fmax(g.d[a] * lo[a], g.d[a] * hi[a]);
    }
    c0 = int(floor(cmin)) & ~(VEC - 1);
    r0 = int(floor(rmin));
    p0 = flat ? 0 : int(floor(pmin));
    // taps reach floor(max)+1; keep one slot of slack for rounding
    return vec && (int(floor(cmax)) + 2 - c0 < BOXW) && (int(floor(rmax)) + 2 - r0 < BR) &&
           (flat || int(floor(pmax)) + 2 - p0 < BH);
  };
  auto fetch = [&](int n, int r0, int p0, int c0, uint4 (&v)[PER], unsigned& valid) {
    const InT* vbase = stack + size_t(n) * plane_sz * M;
    valid = 0u;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int q = e % QN, pl = (e / QN) % BH, j = e / (QN * BH);
      const int row = r0 + j, pp = p0 + pl, cc = c0 + VEC * q;
      const bool ok = e < NE && unsigned(row) < unsigned(M) && unsigned(pp) < unsigned(K) && cc >= 0 && cc < M &&
                      vec;
      valid |= ok ? (1u << i) : 0u;
      const int rowc = min(max(row, 0), M - 1), ppc = min(max(pp, 0), K - 1);
      const int ccc = min(max(cc, 0), M - VEC);
      v[i] = *reinterpret_cast<const uint4*>(stack + size_t(n) * plane_sz * M + (size_t(rowc) * K + ppc) * M +
                                             (vec ? ccc : 0));
      (void)vbase;
    }
  };
  auto stage = [&](const uint4 (&v)[PER], unsigned valid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < NE) {
        const int q = e % QN, pl = (e / QN) % BH, j = e / (QN * BH);
        Chunk16 x;
        x.u = (valid >> i) & 1u ? v[i] : make_uint4(0u, 0u, 0u, 0u);
        float* dst = &box[j][pl][VEC * q];
#pragma unroll
        for (int h = 0; h < VEC; h += 4)
          *reinterpret_cast<float4*>(dst + h) = make_float4(chunk_value<InT>(x, h), chunk_value<InT>(x, h + 1),
                                                            chunk_value<InT>(x, h + 2), chunk_value<InT>(x, h + 3));
      }
    }
  };

  float acc[YB];
#pragma unroll
  for (int j = 0; j < YB; ++j) acc[j] = 0.0f;
  uint4 buf[PER];
  unsigned valid = 0u;
  int r0 = 0, p0 = 0, c0 = 0;
  bool fits = false;
  if (nb > 0) {
    fits = origin(0, r0, p0, c0);
    if (fits) fetch(0, r0, p0, c0, buf, valid);
  }
  for (int n = 0; n < nb; ++n) {
    const bool fits_n = fits;
    const int rr0 = r0, pp0 = p0, cc0 = c0;
    __syncthreads();                                    // previous view's LDS reads are done
    if (fits_n) stage(buf, valid);
    __syncthreads();
    if (n + 1 < nb) {                                   // next view's loads overlap this view's math
      fits = origin(n + 1, r0, p0, c0);
      if (fits) fetch(n + 1, r0, p0, c0, buf, valid);
    }
    if (!live) continue;
    const ViewGeom& g = geom[n];
    const float inv = scale ? 1.0f / scale[n] : 1.0f;   // exact: the scale is a power of two
    const double bc = g.u[0] * rx + g.u[2] * rz + hm;
    const double br = g.v[0] * rx + g.v[2] * rz + hm;
    const double bp = g.d[0] * rx + g.d[2] * rz + hk;
    if (fits_n) {
      // box-local coordinates of the thread's first voxel row in FP64, rounded once; the
      // other rows step by (u_y, v_y, d_y) in FP32 (|local| < 32: error ~1e-6 voxel)
      const double ry0 = y0 - c;
      const float lc0 = float(g.u[1] * ry0 + bc - cc0), lr0 = float(g.v[1] * ry0 + br - rr0);
      const float lp0 = flat ? 0.0f : float(g.d[1] * ry0 + bp - pp0);
      const float uy = float(g.u[1]), vy = float(g.v[1]), dy = flat ? 0.0f : float(g.d[1]);
#pragma unroll
      for (int j = 0; j < YB; ++j) {
        // fmax guards against a rounding-level dip below the box origin
        const float fc = fmaxf(fmaf(float(j), uy, lc0), 0.0f);
        const float fr = fmaxf(fmaf(float(j), vy, lr0), 0.0f);
        const float fp = fmaxf(fmaf(float(j), dy, lp0), 0.0f);
        const float fc0 = floorf(fc), fr0 = floorf(fr), fp0 = floorf(fp);
        const float tc = fc - fc0, tr = fr - fr0, tp = fp - fp0;
        const int lc = int(fc0), lr = int(fr0), lp = int(fp0);
        const int lp1 = flat ? lp : lp + 1;
        const float* a0 = &box[lr][lp][lc];
        const float* a1 = &box[lr][lp1][lc];
        const float* b0 = &box[lr + 1][lp][lc];
        const float* b1 = &box[lr + 1][lp1][lc];
        const float wp1 = flat ? 0.0f : tp, wp0 = 1.0f - wp1;
        const float v0 = a0[0] + tc * (a0[1] - a0[0]);
        const float v1 = a1[0] + tc * (a1[1] - a1[0]);
        const float v2 = b0[0] + tc * (b0[1] - b0[0]);
        const float v3 = b1[0] + tc * (b1[1] - b1[0]);
        acc[j] += inv * ((1.0f - tr) * (wp0 * v0 + wp1 * v1) + tr * (wp0 * v2 + wp1 * v3));
      }
    } else {
      const InT* base = stack + size_t(n) * plane_sz * M;
      // one voxel row per iteration (rare path: keep its registers small)
#pragma unroll 1
      for (int j = 0; j < YB; ++j) {
        const double ry = (y0 + j) - c;
        const double fc = g.u[1] * ry + bc, fr = g.v[1] * ry + br, fp = g.d[1] * ry + bp;
        const double fc0 = floor(fc), fr0 = floor(fr), fp0 = floor(fp);
        const float tc = float(fc - fc0), tr = float(fr - fr0), tp = float(fp - fp0);
        const int c0i = int(fc0), r0i = int(fr0), p0i = int(fp0);
        const float wc0 = (unsigned(c0i) < unsigned(M)) ? 1.0f - tc : 0.0f;
        const float wc1 = (unsigned(c0i + 1) < unsigned(M)) ? tc : 0.0f;
        const float wr0 = (unsigned(r0i) < unsigned(M)) ? 1.0f - tr : 0.0f;
        const float wr1 = (unsigned(r0i + 1) < unsigned(M)) ? tr : 0.0f;
        const float wp0 = flat ? 1.0f : (unsigned(p0i) < unsigned(K)) ? 1.0f - tp : 0.0f;
        const float wp1 = flat ? 0.0f : (unsigned(p0i + 1) < unsigned(K)) ? tp : 0.0f;
        const int c0c = min(max(c0i, 0), M - 1), c1c = min(max(c0i + 1, 0), M - 1);
        const int r0c = min(max(r0i, 0), M - 1), r1c = min(max(r0i + 1, 0), M - 1);
        const int p0c = flat ? 0 : min(max(p0i, 0), K - 1), p1c = flat ? 0 : min(max(p0i + 1, 0), K - 1);
        const InT* a0 = base + (size_t(r0c) * K + p0c) * M;
        const InT* a1 = base + (size_t(r0c) * K + p1c) * M;
        const InT* b0 = base + (size_t(r1c) * K + p0c) * M;
        const InT* b1 = base + (size_t(r1c) * K + p1c) * M;
        const float v0 = wc0 * from_store<InT>(a0[c0c]) + wc1 * from_store<InT>(a0[c1c]);
        const float v1 = wc0 * from_store<InT>(a1[c0c]) + wc1 * from_store<InT>(a1[c1c]);
        const float v2 = wc0 * from_store<InT>(b0[c0c]) + wc1 * from_store<InT>(b0[c1c]);
        const float v3 = wc0 * from_store<InT>(b1[c0c]) + wc1 * from_store<InT>(b1[c1c]);
        const float add = inv * (wr0 * (wp0 * v0 + wp1 * v1) + wr1 * (wp0 * v2 + wp1 * v3));
#pragma unroll
        for (int jj = 0; jj < YB; ++jj) acc[jj] += (jj == j) ? add : 0.0f;
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int j = 0; j < YB; ++j) {
    const int iy = y0 + j;
    if (iy < N) {
      float* dst = vol + (size_t(iz) * N + iy) * N + ix;
      *dst = accumulate ? *dst + acc[j] : acc[j];
    }
  }
}

// Near-axis general frames (single-axis scans with a tilt, directions close to the rotation
// axis's normal plane): per view, the bounding box of the workgroup's 16 (x) x YB (y) x 16 (z)
// voxel tile in (row, plane, column) coordinates -- BR = YB + 4 detector rows x 24 planes x
// BOXW columns -- is fetched straight into LDS by buffer loads with the LDS destination, as in
// k_grid_axis_dma: chunk-linear boxes, chunks outside the stack zero-filled by the hardware, two
// boxes alternating so that view n + 1 is in flight while view n is interpolated (trilinear:
// eight LDS taps per voxel row; with ONE_BOX a single box, fetched and then interpolated, two
// barriers per view).  Per view the box origin, its extent and whether the footprint
// fits are computed one view per lane (FP64, from the tile corners) and read out with readlane;
// only the view's own extent is fetched, and a view whose footprint does not fit is gathered
// for that tile straight from global memory.  The 4-row kernel is held to five waves per SIMD
// (five workgroups per CU, which its LDS box allows): 360 against 385 us per 8-view launch at
// 256^3 with FP32 stacks over a tilt-jittered scan (for directions far from the axis, whose
// footprints often take the global gather, the bound costs time: the autotuner sees both); the
// 8-row kernel would spill at that bound.
template <int YB>
constexpr int tilt_waves_per_eu() { return YB == 4 ? 5 : 1; }
template <int YB, class InT, bool ONE_BOX>
__global__ __launch_bounds__(256, tilt_waves_per_eu<YB>()) void k_grid_tilt_dma(const InT* __restrict__ stack,
                                                       const ViewGeom* __restrict__ geom,
                                                       const float* __restrict__ scale,
                                                       float* __restrict__ vol, int N, int M, int K, int nb,
                                                       int accumulate, int flat, double hm, double hk) {
  constexpr int VEC = DmaBox<InT>::VEC, BOXW = DmaBox<InT>::BOXW, QN = BOXW / VEC;
  constexpr int ES = int(sizeof(InT));                  // bytes per stored value
  constexpr int BR = YB + 4, BH = AX_BOXH;              // rows and planes staged per view
  constexpr int QP = ES == 2 ? QN + 1 : QN;             // 16-byte slots per (row, plane): one spare for 16-bit
  constexpr int PITCH = QP * 4;                         // dwords per staged (row, plane)
  constexpr int NE = BR * BH * QP;                      // slots per staged view
  constexpr int PER = (NE + 255) / 256;                 // loads per thread per view
  constexpr int PAD = ES == 2 ? 4 : 0;                  // 16-bit tap pairs may read one dword past a row
  __shared__ __attribute__((aligned(16))) unsigned box0[NE * 4 + PAD];
  __shared__ __attribute__((aligned(16))) unsigned box1[ONE_BOX ? 4 : NE * 4 + PAD];
  const int ntx = (N + GT - 1) / GT;
  const int tiles = ntx * ntx;
  const int wg = blockIdx.x, xcd = wg & 7, k = wg >> 3;
  const int yblk = xcd + 8 * (k / tiles), tile = k % tiles;
  const int y0 = yblk * YB;
  if (y0 >= N) return;                                  // uniform
  const int tx0 = (tile % ntx) * GT, tz0 = (tile / ntx) * GT;
  const int ix = tx0 + (threadIdx.x % GT);
  const int iz = tz0 + (threadIdx.x / GT);
  const bool live = ix < N && iz < N;
  const double c = 0.5 * (N - 1);
  const double rx = ix - c, rz = iz - c, ry0 = y0 - c;
  const size_t view_sz = size_t(K) * M * M;
  const int wbase = (threadIdx.x & ~63) * 4;            // this wave's first dword in a box, per load
  const int lane = threadIdx.x & 63;

  // box origin (column rounded down to a 16-byte chunk), extent and fit of view n, one view per
  // lane; the extent is packed as columns | rows << 10 | planes << 20
  int obase = -64, lane_c0 = 0, lane_r0 = 0, lane_p0 = 0, lane_fit = 0, lane_ext = 0;
  auto origin = [&](int n, int& c0, int& r0, int& p0, int& ext) -> bool {
    if (n >= obase + 64) {
      obase = n;
      const int v = n + lane;
      int cc = 0, rr = 0, pp = 0, ft = 0, ex = 0;
      if (v < nb) {
        const int t0 = opaque(tx0), z0 = opaque(tz0);
        const double lo[3] = {t0 - c, ry0, z0 - c};
        const double hi[3] = {t0 + GT - 1 - c, ry0 + (YB - 1), z0 + GT - 1 - c};
        const ViewGeom& g = geom[v];
        double cmin = hm, cmax = hm, rmin = hm, rmax = hm, pmin = hk, pmax = hk;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          cmin += fmin(g.u[a] * lo[a], g.u[a] * hi[a]);
          cmax += fmax(g.u[a] * lo[a], g.u[a] * hi[a]);
          rmin += fmin(g.v[a] * lo[a], g.v[a] * hi[a]);
          rmax += fmax(g.v[a] * lo[a], g.v[a] * hi[a]);
          pmin += fmin(g.d[a] * lo[a], g.d[a] * hi[a]);
          pmax += fmax(g.d[a] * lo[a], g.d[a] * hi[a]);
        }
        cc = int(floor(cmin)) & ~(VEC - 1);
        rr = int(floor(rmin));
        pp = flat ? 0 : int(floor(pmin));
        // taps reach floor(max) + 1; one slot of slack for the FP32 rounding of the local coordinates
        const int cn = int(floor(cmax)) + 3 - cc, rn = int(floor(rmax)) + 3 - rr;
        const int pn = flat ? 2 : int(floor(pmax)) + 3 - pp;
        ft = cn <= BOXW && rn <= BR && pn <= BH;
        if (ft) ex = ((cn + VEC - 1) & ~(VEC - 1)) | (rn << 10) | (pn << 20);
      }
      lane_c0 = cc;
      lane_r0 = rr;
      lane_p0 = pp;
      lane_fit = ft;
      lane_ext = ex;
    }
    c0 = __builtin_amdgcn_readlane(lane_c0, n - obase);
    r0 = __builtin_amdgcn_readlane(lane_r0, n - obase);
    p0 = __builtin_amdgcn_readlane(lane_p0, n - obase);
    ext = __builtin_amdgcn_readlane(lane_ext, n - obase);
    return __builtin_amdgcn_readlane(lane_fit, n - obase) != 0;
  };
  // per chunk slot: byte offset from the box origin, and its (row, plane, column) in the box
  // (the host launches this kernel only for M a multiple of VEC and views below 2^31 bytes)
  unsigned cfo[PER];
  int cj[PER], cpl[PER], cq[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i;
    const int q = e % QP, pl = (e / QP) % BH, j = e / (QP * BH);
    cq[i] = VEC * q;
    cpl[i] = pl;
    cj[i] = e < NE && q < QN ? j : -1;                  // the spare 16-bit slot is never fetched
    cfo[i] = unsigned((j * K + pl) * M + VEC * q) * unsigned(ES);
  }
  auto has = [&](int i) {
    return (NE % 256 == 0 || i < PER - 1 || int(threadIdx.x) + 256 * i < NE) && (QP == QN || cq[i] < BOXW);
  };
  auto load = [&](int n, int c0, int r0, int p0, int ext, unsigned* dst) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<InT*>(stack + size_t(n) * view_sz), short(0), int(view_sz * ES), 0x00020000);
    // slots outside the view's extent fetch nothing (their LDS words are never read)
    const int cw = ext & 1023, rh = (ext >> 10) & 1023, bh = ext >> 20;
    auto in_ext = [&](int i) { return cq[i] < cw && cj[i] < rh && cpl[i] < bh; };
    if (r0 >= 0 && r0 + rh <= M && p0 >= 0 && p0 + bh <= K && c0 >= 0 && c0 + cw <= M) {
      const int so = ((r0 * K + p0) * M + c0) * ES;
#pragma unroll
      for (int i = 0; i < PER; ++i)
        if (has(i) && in_ext(i))
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(dst + 1024 * i + wbase), 16, int(cfo[i]), so,
                                                   0, 0);
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        if (has(i) && in_ext(i)) {
          const int row = r0 + cj[i], pp = p0 + cpl[i], cc = c0 + cq[i];
          const bool ok = cj[i] >= 0 && unsigned(row) < unsigned(M) && unsigned(pp) < unsigned(K) &&
                          unsigned(cc) < unsigned(M);
          const unsigned off = ok ? unsigned((row * K + pp) * M + cc) * unsigned(ES) : kOutOfRange;
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(dst + 1024 * i + wbase), 16, int(off), 0,
                                                   0, 0);
        }
      }
    }
  };

  float acc[YB];
#pragma unroll
  for (int j = 0; j < YB; ++j) acc[j] = 0.0f;
  int oc0 = 0, or0 = 0, op0 = 0, oc1 = 0, or1 = 0, op1 = 0;   // origins of the views in each buffer
  int oe0 = 0, oe1 = 0;                                       // their extents
  bool of0 = false, of1 = false;                              // their footprints fit
  // wait for this wave's loads and LDS reads, then for every wave
  auto sync = [&]() {
    __builtin_amdgcn_s_waitcnt(7 << 4);                 // vmcnt(0) lgkmcnt(0)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // interpolation of view n from its staged box bx (origin cb, rb, pb; fb: it fits)
  auto interp = [&](const unsigned* bx, int cb, int rb, int pb, bool fb, int n) {
    if (!live) return;
    const ViewGeom& g = geom[n];
    float inv = 1.0f;
    if constexpr (std::is_same<InT, __half>::value) inv = 1.0f / scale[n];   // exact: a power of two
    // flat (one plane): a zero depth direction and hk = 0 put every tap on plane 0 with the
    // second plane's (zero-filled) taps at weight 0
    const double d0 = flat ? 0.0 : g.d[0], d1 = flat ? 0.0 : g.d[1], d2 = flat ? 0.0 : g.d[2];
    if (fb) {
      // box-local coordinates of the first voxel row in FP64, rounded once; the other rows
      // step by (u_y, v_y, d_y) in FP32 (|local| < 32: error ~1e-6 voxel)
      const float lc0 = float(g.u[0] * rx + g.u[1] * ry0 + g.u[2] * rz + (hm - cb));
      const float lr0 = float(g.v[0] * rx + g.v[1] * ry0 + g.v[2] * rz + (hm - rb));
      const float lp0 = float(d0 * rx + d1 * ry0 + d2 * rz + (hk - pb));
      const float uy = float(g.u[1]), vy = float(g.v[1]), dy = float(d1);
#pragma unroll
      for (int j = 0; j < YB; ++j) {
        // fmax guards a rounding-level dip below the box origin; non-negative: truncation floors
        const float fc = fmaxf(fmaf(float(j), uy, lc0), 0.0f);
        const float fr = fmaxf(fmaf(float(j), vy, lr0), 0.0f);
        const float fp = fmaxf(fmaf(float(j), dy, lp0), 0.0f);
        const int lc = int(fc), lr = int(fr), lp = int(fp);
        const float tc = fc - float(lc), tr = fr - float(lr), tp = fp - float(lp);
        const int o = (lr * BH + lp) * PITCH;           // dwords to (row lr, plane lp)
        float t[8];                                     // (row, plane, col) = (lr + a, lp + b, lc + e) at 4a + 2b + e
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
          const int oo = o + (ab >> 1) * BH * PITCH + (ab & 1) * PITCH;
          if constexpr (ES == 4) {
            const float* r0 = reinterpret_cast<const float*>(bx) + oo + lc;
            t[2 * ab] = r0[0];
            t[2 * ab + 1] = r0[1];
          } else {
            const unsigned* r0 = bx + oo + (lc >> 1);
            const unsigned pr = __builtin_amdgcn_alignbit(r0[1], r0[0], unsigned(lc & 1) * 16u);
            if constexpr (std::is_same<InT, __half>::value) {
              t[2 * ab] = __half2float(__ushort_as_half((unsigned short)(pr & 0xffffu)));
              t[2 * ab + 1] = __half2float(__ushort_as_half((unsigned short)(pr >> 16)));
            } else {
              t[2 * ab] = __uint_as_float(pr << 16);
              t[2 * ab + 1] = __uint_as_float(pr & 0xffff0000u);
            }
          }
        }
        const float v00 = fmaf(tc, t[1] - t[0], t[0]), v01 = fmaf(tc, t[3] - t[2], t[2]);
        const float v10 = fmaf(tc, t[5] - t[4], t[4]), v11 = fmaf(tc, t[7] - t[6], t[6]);
        const float w0 = fmaf(tp, v01 - v00, v00), w1 = fmaf(tp, v11 - v10, v10);
        acc[j] = fmaf(inv, fmaf(tr, w1 - w0, w0), acc[j]);
      }
    } else {
      const InT* base = stack + size_t(n) * view_sz;
      // footprint too large for the box: one voxel row per iteration from global memory
#pragma unroll 1
      for (int j = 0; j < YB; ++j) {
        const double ry = ry0 + j;
        const double fc = g.u[0] * rx + g.u[1] * ry + g.u[2] * rz + hm;
        const double fr = g.v[0] * rx + g.v[1] * ry + g.v[2] * rz + hm;
        const double fp = d0 * rx + d1 * ry + d2 * rz + hk;
        const double fc0 = floor(fc), fr0 = floor(fr), fp0 = floor(fp);
        const float tc = float(fc - fc0), tr = float(fr - fr0), tp = float(fp - fp0);
        const int c0i = int(fc0), r0i = int(fr0), p0i = int(fp0);
        const float wc0 = (unsigned(c0i) < unsigned(M)) ? 1.0f - tc : 0.0f;
        const float wc1 = (unsigned(c0i + 1) < unsigned(M)) ? tc : 0.0f;
        const float wr0 = (unsigned(r0i) < unsigned(M)) ? 1.0f - tr : 0.0f;
        const float wr1 = (unsigned(r0i + 1) < unsigned(M)) ? tr : 0.0f;
        const float wp0 = (unsigned(p0i) < unsigned(K)) ? 1.0f - tp : 0.0f;
        const float wp1 = (unsigned(p0i + 1) < unsigned(K)) ? tp : 0.0f;
        const int c0c = min(max(c0i, 0), M - 1), c1c = min(max(c0i + 1, 0), M - 1);
        const int r0c = min(max(r0i, 0), M - 1), r1c = min(max(r0i + 1, 0), M - 1);
        const int p0c = min(max(p0i, 0), K - 1), p1c = min(max(p0i + 1, 0), K - 1);
        const InT* a0 = base + (size_t(r0c) * K + p0c) * M;
        const InT* a1 = base + (size_t(r0c) * K + p1c) * M;
        const InT* b0 = base + (size_t(r1c) * K + p0c) * M;
        const InT* b1 = base + (size_t(r1c) * K + p1c) * M;
        const float v0 = wc0 * from_store<InT>(a0[c0c]) + wc1 * from_store<InT>(a0[c1c]);
        const float v1 = wc0 * from_store<InT>(a1[c0c]) + wc1 * from_store<InT>(a1[c1c]);
        const float v2 = wc0 * from_store<InT>(b0[c0c]) + wc1 * from_store<InT>(b0[c1c]);
        const float v3 = wc0 * from_store<InT>(b1[c0c]) + wc1 * from_store<InT>(b1[c1c]);
        const float add = inv * (wr0 * (wp0 * v0 + wp1 * v1) + wr1 * (wp0 * v2 + wp1 * v3));
#pragma unroll
        for (int jj = 0; jj < YB; ++jj) acc[jj] += (jj == j) ? add : 0.0f;
      }
    }
  };
  // two boxes: view n + 1 is fetched while view n is interpolated, one barrier per view
  auto step = [&](const unsigned* bx, int& cb, int& rb, int& pb, bool& fb, unsigned* other, int& co, int& ro,
                  int& po, int& eo, bool& fo, int n) {
    if (n >= nb) return;                                // uniform
    sync();
    if (n + 1 < nb) {
      fo = origin(n + 1, co, ro, po, eo);
      if (fo) load(n + 1, co, ro, po, eo, other);
    }
    interp(bx, cb, rb, pb, fb, n);
  };
  if constexpr (ONE_BOX) {
    // one box (half the LDS, so more workgroups per CU hide each other's fetches): fetch,
    // wait, interpolate, two barriers per view
    for (int n = 0; n < nb; ++n) {
      if (n > 0) sync();                                // every wave is done with the box
      of0 = origin(n, oc0, or0, op0, oe0);
      if (of0) load(n, oc0, or0, op0, oe0, box0);
      sync();
      interp(box0, oc0, or0, op0, of0, n);
    }
  } else {
    if (nb > 0) {
      of0 = origin(0, oc0, or0, op0, oe0);
      if (of0) load(0, oc0, or0, op0, oe0, box0);
    }
    for (int n0 = 0; n0 < nb; n0 += 2) {
      step(box0, oc0, or0, op0, of0, box1, oc1, or1, op1, oe1, of1, n0);
      step(box1, oc1, or1, op1, of1, box0, oc0, or0, op0, oe0, of0, n0 + 1);
    }
  }
  if (!live) return;
#pragma unroll
  for (int j = 0; j < YB; ++j) {
    const int iy = y0 + j;
    if (iy < N) {
      float* dst = vol + (size_t(iz) * N + iy) * N + ix;
      *dst = accumulate ? *dst + acc[j] : acc[j];
    }
  }
}

// General view frames, cubic tiles: 8 x 8 x 8 voxels, two per thread (iz and iz + 4).
// The voxel centres of a cube of edge 8 span at most 7 (|a_x| + |a_y| + |a_z|) <= 7 sqrt(3)
// < 12.2 along any unit vector a, so with the taps and the floor of the origin a box of
// 16 rows x 16 planes x CW columns (column start rounded down to a 16-byte boundary) holds
// the footprint for every view: no fallback path, whatever the orientation.
template <class InT>
struct CubeBox;
template <>
struct CubeBox<float> {
  static constexpr int VEC = 4, CW = 20, CP = 20;
};
template <>
struct CubeBox<__hip_bfloat16> {
  static constexpr int VEC = 8, CW = 24, CP = 24;
};
template <>
struct CubeBox<__half> {
  static constexpr int VEC = 8, CW = 24, CP = 24;
};
constexpr int CB_E = 8;    // voxel tile edge
constexpr int CB_R = 16;   // rows and planes staged per view

template <class InT>
__global__ __launch_bounds__(256) void k_grid_cube(const InT* __restrict__ stack,
                                                   const ViewGeom* __restrict__ geom,
                                                   const float* __restrict__ scale,
                                                   float* __restrict__ vol, int N, int M, int K,
                                                   int nb, int accumulate, int flat) {
  using B = CubeBox<InT>;
  constexpr int VEC = B::VEC, CW = B::CW, CP = B::CP;
  constexpr int QN = CW / VEC;
  constexpr int NE = CB_R * CB_R * QN;
  constexpr int PER = (NE + 255) / 256;
  __shared__ float box[CB_R][CB_R][CP];
  // tiles of one XCD are consecutive in x, then y, then z (neighbours share stack rows in L2)
  const int ntc = (N + CB_E - 1) / CB_E;
  const int tiles = ntc * ntc * ntc;
  const int per = (tiles + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= tiles) return;                           // uniform
  const int tx0 = (tile % ntc) * CB_E, ty0 = ((tile / ntc) % ntc) * CB_E, tz0 = (tile / (ntc * ntc)) * CB_E;
  const int ix = tx0 + (threadIdx.x % CB_E), iy = ty0 + (threadIdx.x / CB_E) % CB_E;
  const int iz0 = tz0 + int(threadIdx.x) / (CB_E * CB_E);
  const bool live0 = ix < N && iy < N && iz0 < N, live1 = ix < N && iy < N && iz0 + 4 < N;
  const double c = 0.5 * (N - 1);
  const double rx = ix - c, ry = iy - c, rz0 = iz0 - c;
  const double hm = 0.5 * (M - 1), hk = 0.5 * (K - 1);
  const size_t plane_sz = size_t(K) * M;
  const bool vec = (M % VEC) == 0;
  const double lo[3] = {tx0 - c, ty0 - c, tz0 - c};
  const double hi[3] = {tx0 + CB_E - 1 - c, ty0 + CB_E - 1 - c, tz0 + CB_E - 1 - c};

  auto origin = [&](int n, int& r0, int& p0, int& c0) {
    const ViewGeom& g = geom[n];
    double cmin = hm, rmin = hm, pmin = hk;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cmin += fmin(g.u[a] * lo[a], g.u[a] * hi[a]);
      rmin += fmin(g.v[a] * lo[a], g.v[a] * hi[a]);
      pmin += fmin(g.d[a] * lo[a], g.d[a] * hi[a]);
    }
    c0 = int(floor(cmin)) & ~(VEC - 1);
    r0 = int(floor(rmin));
    p0 = flat ? 0 : int(floor(pmin));
  };
  // The view-independent part of every staged chunk (its row, plane and column offsets in
  // the box and its LDS offset), computed once; per view only the box origin moves.
  int cj[PER], cpl[PER], cq[PER], cdst[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i;
    cq[i] = VEC * (e % QN);
    cpl[i] = (e / QN) % CB_R;
    cj[i] = e < NE ? e / (QN * CB_R) : -1;
    cdst[i] = e < NE ? (cj[i] * CB_R + cpl[i]) * CP + cq[i] : -1;
  }
  auto fetch = [&](int n, int r0, int p0, int c0, uint4 (&v)[PER], unsigned& valid) {
    const InT* vbase = stack + size_t(n) * plane_sz * M;
    valid = 0u;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int row = r0 + cj[i], pp = p0 + cpl[i], cc = c0 + cq[i];
      const bool ok = cj[i] >= 0 && unsigned(row) < unsigned(M) && unsigned(pp) < unsigned(K) && cc >= 0 && cc < M;
      valid |= ok ? (1u << i) : 0u;
      const int rowc = min(max(row, 0), M - 1), ppc = min(max(pp, 0), K - 1);
      if (vec) {
        const unsigned off = unsigned(rowc * K + ppc) * unsigned(M) + unsigned(min(max(cc, 0), M - VEC));
        v[i] = *reinterpret_cast<const uint4*>(vbase + off);
      } else {
        const InT* src = vbase + (size_t(rowc) * K + ppc) * M;
        Chunk16 x;
#pragma unroll
        for (int kk = 0; kk < VEC; ++kk) {
          const int ce = min(max(cc + kk, 0), M - 1);
          const bool ek = unsigned(cc + kk) < unsigned(M);
          if constexpr (VEC == 4) x.f[kk] = ek ? from_store<InT>(src[ce]) : 0.0f;
          else x.h[kk] = ek ? reinterpret_cast<const unsigned short*>(src)[ce] : (unsigned short)0;
        }
        v[i] = x.u;
        if (cj[i] >= 0 && unsigned(row) < unsigned(M) && unsigned(pp) < unsigned(K)) valid |= (1u << i);
      }
    }
  };
  auto stage = [&](const uint4 (&v)[PER], unsigned valid) {
    float* boxf = &box[0][0][0];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (cdst[i] >= 0) {
        Chunk16 x;
        x.u = (valid >> i) & 1u ? v[i] : make_uint4(0u, 0u, 0u, 0u);
        float* dst = boxf + cdst[i];
#pragma unroll
        for (int h = 0; h < VEC; h += 4)
          *reinterpret_cast<float4*>(dst + h) = make_float4(chunk_value<InT>(x, h), chunk_value<InT>(x, h + 1),
                                                            chunk_value<InT>(x, h + 2), chunk_value<InT>(x, h + 3));
      }
    }
  };

  float acc0 = 0.0f, acc1 = 0.0f;
  uint4 buf[PER];
  unsigned valid = 0u;
  int r0 = 0, p0 = 0, c0 = 0;
  if (nb > 0) {
    origin(0, r0, p0, c0);
    fetch(0, r0, p0, c0, buf, valid);
  }
  for (int n = 0; n < nb; ++n) {
    const int rr0 = r0, pp0 = p0, cc0 = c0;
    __syncthreads();
    stage(buf, valid);
    __syncthreads();
    if (n + 1 < nb) {
      origin(n + 1, r0, p0, c0);
      fetch(n + 1, r0, p0, c0, buf, valid);
    }
    const ViewGeom& g = geom[n];
    const float inv = scale ? 1.0f / scale[n] : 1.0f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double rz = rz0 + 4 * h;
      // box-local coordinates (FP64, rounded once); fmax guards a rounding-level dip below the origin
      const float fc = float(fmax(g.u[0] * rx + g.u[1] * ry + g.u[2] * rz + hm - cc0, 0.0));
      const float fr = float(fmax(g.v[0] * rx + g.v[1] * ry + g.v[2] * rz + hm - rr0, 0.0));
      const float fp = flat ? 0.0f : float(fmax(g.d[0] * rx + g.d[1] * ry + g.d[2] * rz + hk - pp0, 0.0));
      const float fc0 = floorf(fc), fr0 = floorf(fr), fp0 = floorf(fp);
      const float tc = fc - fc0, tr = fr - fr0, tp = flat ? 0.0f : fp - fp0;
      const int lc = int(fc0), lr = int(fr0), lp = int(fp0);
      const int lp1 = flat ? lp : lp + 1;
      const float* a0 = &box[lr][lp][lc];
      const float* a1 = &box[lr][lp1][lc];
      const float* b0 = &box[lr + 1][lp][lc];
      const float* b1 = &box[lr + 1][lp1][lc];
      const float v0 = a0[0] + tc * (a0[1] - a0[0]);
      const float v1 = a1[0] + tc * (a1[1] - a1[0]);
      const float v2 = b0[0] + tc * (b0[1] - b0[0]);
      const float v3 = b1[0] + tc * (b1[1] - b1[0]);
      const float add = inv * ((1.0f - tr) * ((1.0f - tp) * v0 + tp * v1) + tr * ((1.0f - tp) * v2 + tp * v3));
      if (h == 0) acc0 += add;
      else acc1 += add;
    }
  }
  if (live0) {
    float* dst = vol + (size_t(iz0) * N + iy) * N + ix;
    *dst = accumulate ? *dst + acc0 : acc0;
  }
  if (live1) {
    float* dst = vol + (size_t(iz0 + 4) * N + iy) * N + ix;
    *dst = accumulate ? *dst + acc1 : acc1;
  }
}

// The cube kernel for FP32 stacks with M a multiple of 4: the same tiles, box origins and
// interpolation (bit for bit), with each view's footprint fetched straight into LDS by buffer
// loads (no register staging, no per-chunk clamps: chunks outside the stack get an offset past
// the buffer's range and read as zeros).  Per view only the footprint's own extent of the
// 16 x 16 x 20 box is fetched (over random directions about 2.2 times fewer bytes than the
// whole box), and the box origins and extents of 64 views are computed at once, one view per
// lane.  Each staged row is followed by CD_XS spare 16-byte slots that are never fetched: at a
// row pitch of 344 dwords the tap reads of a wave (an 8 x 8 voxel slice, rotated into the box)
// meet 3.5 bank cycles per pair read in a count over random directions, against 5.3 at 320,
// where taps in different rows fall on one bank.  One box and two barriers per view: a
// second box (view n + 1 in flight while view n is interpolated) halves the workgroups per CU
// and measured slower.
constexpr int CD_QN = 5;                        // fetched 16-byte chunks per (row, plane)
constexpr int CD_XS = 6;                        // spare slots per staged row
constexpr int CD_SR = CB_R * CD_QN + CD_XS;     // slots per staged row
constexpr int CD_NE = CB_R * CD_SR;             // slots per box
constexpr int CD_RP = CD_SR * 4, CD_PP = CD_QN * 4;   // row and plane pitch, dwords

__global__ __launch_bounds__(256) void k_grid_cube_dma(const float* __restrict__ stack,
                                                       const ViewGeom* __restrict__ geom,
                                                       float* __restrict__ vol, int N, int M, int K, int nb,
                                                       int accumulate, int flat) {
  constexpr int PER = (CD_NE + 255) / 256;
  __shared__ __attribute__((aligned(16))) float box[CD_NE * 4];
  const int ntc = (N + CB_E - 1) / CB_E;
  const int tiles = ntc * ntc * ntc;
  const int per = (tiles + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= tiles) return;                           // uniform
  const int tx0 = (tile % ntc) * CB_E, ty0 = ((tile / ntc) % ntc) * CB_E, tz0 = (tile / (ntc * ntc)) * CB_E;
  const int ix = tx0 + (threadIdx.x % CB_E), iy = ty0 + (threadIdx.x / CB_E) % CB_E;
  const int iz0 = tz0 + int(threadIdx.x) / (CB_E * CB_E);
  const bool live0 = ix < N && iy < N && iz0 < N, live1 = ix < N && iy < N && iz0 + 4 < N;
  const double c = 0.5 * (N - 1);
  const double rx = ix - c, ry = iy - c, rz0 = iz0 - c;
  const double hm = 0.5 * (M - 1), hk = 0.5 * (K - 1);
  const size_t view_sz = size_t(K) * M * M;
  const int wbase = (threadIdx.x & ~63) * 4;           // this wave's first dword in the box, per load
  const int lane = threadIdx.x & 63;

  // Box origin as in k_grid_cube and extent of a view, lane l of every wave for view
  // obase + l; per view the workgroup-uniform values are read out of one lane into scalar
  // registers.  Taps lie at most one past the floor of a voxel's coordinates, and one more
  // row, plane and column absorb a last-bit difference between the corner and the voxel
  // arithmetic (at most 16 rows, 16 planes and 20 columns: a tile's footprint spans < 12.2).
  int obase = -64, lane_o = 0, lane_e = 0;
  auto origin = [&](int n, int& r0, int& p0, int& c0, int& rh, int& ph, int& cw) {
    if (n >= obase + 64) {
      obase = n;
      const int v = n + lane;
      int o = 0, ex = 0;
      if (v < nb) {
        const double lo[3] = {opaque(tx0) - c, opaque(ty0) - c, opaque(tz0) - c};
        const double hi[3] = {lo[0] + (CB_E - 1), lo[1] + (CB_E - 1), lo[2] + (CB_E - 1)};
        const ViewGeom& g = geom[v];
        // one detector coordinate at a time (fewer registers live at once)
        auto extremes = [&](const double* w, double h0, int& fmn, int& fmx) {
          double mn = h0, mx = h0;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            mn += fmin(w[a] * lo[a], w[a] * hi[a]);
            mx += fmax(w[a] * lo[a], w[a] * hi[a]);
          }
          fmn = int(floor(mn));
          fmx = int(floor(mx));
          __builtin_amdgcn_sched_barrier(0);
        };
        int cmn, cmx, rmn, rmx, pmn, pmx;
        extremes(g.u, hm, cmn, cmx);
        extremes(g.v, hm, rmn, rmx);
        extremes(g.d, hk, pmn, pmx);
        const int cc = cmn & ~3;
        const int rr = rmn;
        const int pp = flat ? 0 : pmn;
        const int ww = min(4 * CD_QN, (cmx - cc + 3 + 3) & ~3);
        const int hh = min(CB_R, rmx - rr + 3);
        const int dd = flat ? 1 : min(CB_R, pmx - pp + 3);
        // packed in 12-bit fields, offset by 1024 (rows, planes) and 2048 (columns): a tile
        // corner is at most sqrt(3) (N - 1) / 2 < 887 from the volume centre (N <= 1024), so
        // every origin lies in [-890, 1024 + 887) (M <= 256, K <= 2048)
        o = (rr + 1024) | ((pp + 1024) << 12);
        ex = (cc + 2048) | (ww << 12) | (hh << 18) | (dd << 24);
      }
      lane_o = o;
      lane_e = ex;
    }
    const int o = __builtin_amdgcn_readlane(lane_o, n - obase);
    const int ex = __builtin_amdgcn_readlane(lane_e, n - obase);
    r0 = (o & 4095) - 1024;
    p0 = ((o >> 12) & 4095) - 1024;
    c0 = (ex & 4095) - 2048;
    cw = (ex >> 12) & 63;
    rh = (ex >> 18) & 63;
    ph = (ex >> 24) & 63;
  };
  // per slot: row, plane and column in the box (row CB_R, never below a row extent: spare
  // slot or past the box) and the byte offset from the box origin
  // (the host launches this kernel only for M a multiple of 4 and views below 2^31 bytes)
  unsigned cfo[PER];
  int crw[PER], cpl[PER], cq[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i;
    const int row = e / CD_SR, rem = e % CD_SR;
    crw[i] = (e < CD_NE && rem < CB_R * CD_QN) ? row : CB_R;
    cpl[i] = rem / CD_QN;
    cq[i] = 4 * (rem % CD_QN);
    cfo[i] = unsigned((row * K + cpl[i]) * M + cq[i]) * 4u;
  }
  // slots outside the view's extent fetch nothing (their LDS words are never read)
  auto load = [&](int n, int r0, int p0, int c0, int rh, int ph, int cw) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(stack + size_t(n) * view_sz), short(0), int(view_sz * 4), 0x00020000);
    if (r0 >= 0 && r0 + rh <= M && p0 >= 0 && p0 + ph <= K && c0 >= 0 && c0 + cw <= M) {
      const int so = ((r0 * K + p0) * M + c0) * 4;
#pragma unroll
      for (int i = 0; i < PER; ++i)
        if (crw[i] < rh && cpl[i] < ph && cq[i] < cw)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(box + 1024 * i + wbase), 16, int(cfo[i]), so,
                                                   0, 0);
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        if (crw[i] < rh && cpl[i] < ph && cq[i] < cw) {
          // c0 and M are multiples of 4: a chunk is wholly inside or wholly outside the columns
          const int row = r0 + crw[i], pp = p0 + cpl[i], cc = c0 + cq[i];
          const bool ok = unsigned(row) < unsigned(M) && unsigned(pp) < unsigned(K) && unsigned(cc) < unsigned(M);
          const unsigned off = ok ? unsigned((row * K + pp) * M + cc) * 4u : kOutOfRange;
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(box + 1024 * i + wbase), 16, int(off), 0, 0,
                                                   0);
        }
      }
    }
  };
  auto sync = [&]() {
    __builtin_amdgcn_s_waitcnt(7 << 4);                // vmcnt(0) lgkmcnt(0): this wave's loads and reads
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  float acc0 = 0.0f, acc1 = 0.0f;
  for (int n = 0; n < nb; ++n) {
    int rr0, pp0, cc0, rh, ph, cw;
    sync();                                            // every wave is done with the box
    origin(n, rr0, pp0, cc0, rh, ph, cw);
    load(n, rr0, pp0, cc0, rh, ph, cw);
    sync();                                            // every wave's share has landed
    // interpolation as in k_grid_cube
    const ViewGeom& g = geom[n];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double rz = rz0 + 4 * h;
      const float fc = float(fmax(g.u[0] * rx + g.u[1] * ry + g.u[2] * rz + hm - cc0, 0.0));
      const float fr = float(fmax(g.v[0] * rx + g.v[1] * ry + g.v[2] * rz + hm - rr0, 0.0));
      const float fp = flat ? 0.0f : float(fmax(g.d[0] * rx + g.d[1] * ry + g.d[2] * rz + hk - pp0, 0.0));
      const float fc0 = floorf(fc), fr0 = floorf(fr), fp0 = floorf(fp);
      const float tc = fc - fc0, tr = fr - fr0, tp = flat ? 0.0f : fp - fp0;
      const int lc = int(fc0), lr = int(fr0), lp = int(fp0);
      const int lp1 = flat ? lp : lp + 1;
      const float* a0 = box + lr * CD_RP + lp * CD_PP + lc;
      const float* a1 = box + lr * CD_RP + lp1 * CD_PP + lc;
      const float* b0 = a0 + CD_RP;
      const float* b1 = a1 + CD_RP;
      const float v0 = a0[0] + tc * (a0[1] - a0[0]);
      const float v1 = a1[0] + tc * (a1[1] - a1[0]);
      const float v2 = b0[0] + tc * (b0[1] - b0[0]);
      const float v3 = b1[0] + tc * (b1[1] - b1[0]);
      const float add = (1.0f - tr) * ((1.0f - tp) * v0 + tp * v1) + tr * ((1.0f - tp) * v2 + tp * v3);
      if (h == 0) acc0 += add;
      else acc1 += add;
    }
  }
  if (live0) {
    float* dst = vol + (size_t(iz0) * N + iy) * N + ix;
    *dst = accumulate ? *dst + acc0 : acc0;
  }
  if (live1) {
    float* dst = vol + (size_t(iz0 + 4) * N + iy) * N + ix;
    *dst = accumulate ? *dst + acc1 : acc1;
  }
}

// ------------------------------------------------------------------ plan tables (FP64)

__device__ __forceinline__ double2 filter_value(const FilterArgs& fa, const ViewGeom& g,
                                                const double* wv, int ky, int kx, int n) {
  const double qx = signed_q(kx, fa.M, fa.dx), qy = signed_q(ky, fa.M, fa.dx);
  const double q2 = qx * qx + qy * qy;
  double w;
  if (fa.mode == 0) w = g.a * fabs(qx);
  else if (fa.mode == 1) w = 2.0 * sqrt(q2) / double(fa.n_views);
  else w = wv[(size_t(n) * fa.M + ky) * fa.M + kx];
  const double omega = atan(fa.sigma);
  const double cst = fa.lambda / (4.0 * M_PI * sqrt(1.0 + fa.sigma * fa.sigma));
  const double chi = M_PI * fa.lambda * g.R * q2 - omega;
  double sn, cs;
  sincos(chi, &sn, &cs);
  const double hre = sn / (sn * sn + fa.epsilon);
  const double him = fa.ewald ? -cs / (cs * cs + fa.epsilon) : 0.0;
  return make_double2(cst * w * hre, cst * w * him);
}

__global__ void k_filter_table(FilterArgs fa, const ViewGeom* __restrict__ geom,
                               const double* __restrict__ wtab, float4* __restrict__ filt) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t per = size_t(fa.M) * fa.M;
  if (i >= per * fa.n_views) return;
  const int n = int(i / per);
  const int ky = int((i % per) / fa.M), kx = int(i % fa.M);
  const ViewGeom g = geom[n];
  const double2 f = filter_value(fa, g, wtab, ky, kx, n);
  const double2 fm = filter_value(fa, g, wtab, (fa.M - ky) % fa.M, (fa.M - kx) % fa.M, n);
  // F_h = (F(k) + conj F(-k))/2, F_a = (F(k) - conj F(-k))/2
  const double hr = 0.5 * (f.x + fm.x), hi = 0.5 * (f.y - fm.y);
  const double ar = 0.5 * (f.x - fm.x), ai = 0.5 * (f.y + fm.y);
  const double inv = 1.0 / (double(fa.M) * double(fa.M));
  // G1 = (1+i) F_h / M^2,  G2 = -(1+i) F_a / M^2
  float4 o;
  o.x = float((hr - hi) * inv);
  o.y = float((hr + hi) * inv);
  o.z = float(-(ar - ai) * inv);
  o.w = float(-(ar + ai) * inv);
  filt[i] = o;
}

// Sampling matrix in 2^-32 fixed point (integer atomics: order independent).
__global__ void k_sampling_splat(FilterArgs fa, const ViewGeom* __restrict__ geom,
                                 unsigned long long* __restrict__ smat) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t per = size_t(fa.M) * fa.M;
  if (i >= per * fa.n_views) return;
  const int n = int(i / per);
  const int ky = int((i % per) / fa.M), kx = int(i % fa.M);
  double p[3];
  sample_point(fa, geom[n], ky, kx, p);
  const int N = fa.N, lo = -(N / 2);
  for (int sgn = 0; sgn < 2; ++sgn) {
    double f[3];
    int i0[3];
    double t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      f[a] = (sgn ? -p[a] : p[a]) - lo;
      const double fl = floor(f[a]);
      i0[a] = int(fl);
      t[a] = f[a] - fl;
    }
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          const int jx = i0[0] + cx, jy = i0[1] + cy, jz = i0[2] + cz;
          if (unsigned(jx) >= unsigned(N) || unsigned(jy) >= unsigned(N) || unsigned(jz) >= unsigned(N))
            continue;
          const double w = (cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1]) * (cz ? t[2] : 1.0 - t[2]);
          const unsigned long long fx = (unsigned long long)llrint(0.5 * w * kFix);
          atomicAdd(&smat[(size_t(jz) * N + jy) * N + jx], fx);
        }
  }
}

__global__ void k_sampling_weights(FilterArgs fa, const ViewGeom* __restrict__ geom,
                                   const unsigned long long* __restrict__ smat, double* __restrict__ wtab) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t per = size_t(fa.M) * fa.M;
  if (i >= per * fa.n_views) return;
  const int n = int(i / per);
  const int ky = int((i % per) / fa.M), kx = int(i % fa.M);
  double p[3];
  sample_point(fa, geom[n], ky, kx, p);
  const int N = fa.N, lo = -(N / 2), hi = (N + 1) / 2 - 1;
  bool inside = true;
  double t[3];
  int i0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    inside = inside && (p[a] >= lo) && (p[a] <= hi);
    const double f = p[a] - lo;
    const double fl = floor(f);
    i0[a] = int(fl);
    t[a] = f - fl;
  }
  double shat = 0.0;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const int jx = i0[0] + cx, jy = i0[1] + cy, jz = i0[2] + cz;
        if (unsigned(jx) >= unsigned(N) || unsigned(jy) >= unsigned(N) || unsigned(jz) >= unsigned(N))
          continue;
        const double w = (cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1]) * (cz ? t[2] : 1.0 - t[2]);
        shat += w * (double(smat[(size_t(jz) * N + jy) * N + jx]) / kFix);
      }
  const double scale = double(fa.M) * fa.M / (double(N) * N * N * fa.dx);
  wtab[i] = inside ? scale * shat / (shat * shat + fa.eps_sampling) : 0.0;
}

// ------------------------------------------------------------------ launchers
// Size table of the spectra / plane kernels: one group per translation unit.
const FftSize* fft_size(int M) {
  struct Group {
    const FftSize* sizes;
    int count;
  };
  static const Group groups[] = {
      {kFftSizesA, kFftSizesACount}, {kFftSizesB, kFftSizesBCount}, {kFftSizesC, kFftSizesCCount},
      {kFftSizesD, kFftSizesDCount}, {kFftSizesE, kFftSizesECount}, {kFftSizesF, kFftSizesFCount},
      {kFftSizesG, kFftSizesGCount}, {kFftSizesH, kFftSizesHCount}, {kFftSizesI, kFftSizesICount},
      {kFftSizesJ, kFftSizesJCount}};
  for (const Group& g : groups)
    for (int i = 0; i < g.count; ++i)
      if (g.sizes[i].M == M) return &g.sizes[i];
  return nullptr;
}

bool fft_supported(int M) { return fft_size(M) != nullptr; }

int fft_threads(int M) {
  const FftSize* f = fft_size(M);
  return f ? f->threads : 0;
}

int fft_split(int M) {
  const FftSize* f = fft_size(M);
  return f ? f->P : 0;
}

hipError_t launch_spectra(int M, const float* images, const float4* filt, const float2* tw_fwd,
                          float4* q, int* status, double inv_iin, float* scale, int nb, hipStream_t s,
                          const float2* tw_half_fwd, float* l1part) {
  if (nb <= 0) return hipSuccess;
  const FftSize* f = fft_size(M);
  if (!f) return hipErrorInvalidValue;
  return f->spectra(SpectraLaunch{images, filt, tw_fwd, tw_half_fwd, q, status, inv_iin, scale, l1part, nb, s});
}

hipError_t launch_planes(int M, int dtype, const float4* q, const float2* prop, const float2* tw_inv,
                         void* stack, int K, int npairs, int nb, const float* scale, hipStream_t s,
                         const float2* tw_half_inv) {
  if (nb <= 0) return hipSuccess;
  const FftSize* f = fft_size(M);
  if (!f) return hipErrorInvalidValue;
  return f->planes(PlanesLaunch{dtype, q, prop, tw_inv, tw_half_inv, stack, K, npairs, nb, scale, s});
}

template <int kYB, class InT>
static hipError_t grid_impl(bool axis_fast, const void* stack, const ViewGeom* geom, const float* scale,
                            float* vol, int N, int M, int K, int nb, int accumulate, int flat, hipStream_t s) {
  const dim3 grid((N + GT - 1) / GT, (N + GT - 1) / GT, (N + kYB - 1) / kYB);
  const InT* st = static_cast<const InT*>(stack);
  if (axis_fast) {
    // flat grid: (x, z) tiles x row blocks, row blocks padded to a multiple of 8 (one XCD each).
    // Supported sizes (M a multiple of 16, K <= 2 N <= 512) always meet the kernel's conditions.
    if (M % DmaBox<InT>::VEC != 0 || size_t(K) * M * M * sizeof(InT) > size_t(0x7fffffff))
      return hipErrorInvalidValue;
    const int tiles = int(grid.x * grid.y);
    const int yblocks8 = int((grid.z + 7) / 8 * 8);
    hipLaunchKernelGGL((k_grid_axis_dma<kYB, InT>), dim3(unsigned(tiles * yblocks8)), dim3(256), 0, s, st, geom,
                       scale, vol, N, M, K, nb, accumulate, flat, 0.5 * (M - 1), 0.5 * (K - 1));
  } else if constexpr (kYB >= 4) {
    const int tiles = int(grid.x * grid.y);
    const int yblocks8 = int((grid.z + 7) / 8 * 8);
    hipLaunchKernelGGL((k_grid_box<kYB, InT>), dim3(unsigned(tiles * yblocks8)), dim3(256), 0, s, st, geom,
                       scale, vol, N, M, K, nb, accumulate, flat);
  } else {
    return hipErrorInvalidValue;   // 2 rows per thread: single-axis plans only
  }
  return hipGetLastError();
}

template <int YB>
static hipError_t grid_dtype(bool axis_fast, int dtype, const void* stack, const ViewGeom* geom, const float* scale,
                             float* vol, int N, int M, int K, int nb, int accumulate, int flat, hipStream_t s) {
  switch (dtype) {
    case 0: return grid_impl<YB, float>(axis_fast, stack, geom, nullptr, vol, N, M, K, nb, accumulate, flat, s);
    case 1:
      return grid_impl<YB, __hip_bfloat16>(axis_fast, stack, geom, nullptr, vol, N, M, K, nb, accumulate, flat, s);
    case 2: return grid_impl<YB, __half>(axis_fast, stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
    default: return hipErrorInvalidValue;
  }
}

template <class InT>
static hipError_t grid_cube_impl(const void* stack, const ViewGeom* geom, const float* scale, float* vol, int N,
                                 int M, int K, int nb, int accumulate, int flat, hipStream_t s) {
  const int ntc = (N + CB_E - 1) / CB_E;
  const int per = (ntc * ntc * ntc + 7) / 8;
  if constexpr (std::is_same<InT, float>::value) {
    if (M % 4 == 0 && size_t(K) * M * M * sizeof(float) <= size_t(0x7fffffff)) {
      hipLaunchKernelGGL(k_grid_cube_dma, dim3(unsigned(8 * per)), dim3(256), 0, s,
                         static_cast<const float*>(stack), geom, vol, N, M, K, nb, accumulate, flat);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL(k_grid_cube<InT>, dim3(unsigned(8 * per)), dim3(256), 0, s, static_cast<const InT*>(stack),
                     geom, scale, vol, N, M, K, nb, accumulate, flat);
  return hipGetLastError();
}

template <int YB, class InT>
static hipError_t grid_tilt_impl(const void* stack, const ViewGeom* geom, const float* scale, float* vol, int N,
                                 int M, int K, int nb, int accumulate, int flat, hipStream_t s) {
  if (M % DmaBox<InT>::VEC != 0 || size_t(K) * M * M * sizeof(InT) > size_t(0x7fffffff)) return hipErrorInvalidValue;
  const int ntx = (N + GT - 1) / GT;
  const int yblocks8 = ((N + YB - 1) / YB + 7) / 8 * 8;
  // 4 and 8 rows: one box per workgroup, five / four workgroups per CU (at 88 / 118 VGPRs)
  // instead of three / two with two boxes (at 256^3 per 8-view launch, before the five-wave
  // bound on 4 rows: 376 vs 385 us, 363 vs 446 us); 2 rows keep two boxes
  hipLaunchKernelGGL((k_grid_tilt_dma<YB, InT, YB >= 4>), dim3(unsigned(ntx * ntx * yblocks8)), dim3(256), 0, s,
                     static_cast<const InT*>(stack), geom, scale, vol, N, M, K, nb, accumulate, flat, 0.5 * (M - 1),
                     flat ? 0.0 : 0.5 * (K - 1));
  return hipGetLastError();
}

template <int YB>
static hipError_t grid_tilt_dtype(int dtype, const void* stack, const ViewGeom* geom, const float* scale, float* vol,
                                  int N, int M, int K, int nb, int accumulate, int flat, hipStream_t s) {
  switch (dtype) {
    case 0: return grid_tilt_impl<YB, float>(stack, geom, nullptr, vol, N, M, K, nb, accumulate, flat, s);
    case 1: return grid_tilt_impl<YB, __hip_bfloat16>(stack, geom, nullptr, vol, N, M, K, nb, accumulate, flat, s);
    case 2: return grid_tilt_impl<YB, __half>(stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grid(bool axis_fast, int dtype, const void* stack, const ViewGeom* geom, const float* scale,
                       float* vol, int N, int M, int K, int nb, int accumulate, int flat, hipStream_t s, int rows) {
  if (rows == kGridTilt8 && !axis_fast)
    return grid_tilt_dtype<8>(dtype, stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
  if (rows == kGridTilt4 && !axis_fast)
    return grid_tilt_dtype<4>(dtype, stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
  if (rows == kGridTilt2 && !axis_fast)
    return grid_tilt_dtype<2>(dtype, stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
  if (rows == 0 && !axis_fast) {
    switch (dtype) {
      case 0: return grid_cube_impl<float>(stack, geom, nullptr, vol, N, M, K, nb, accumulate, flat, s);
      case 1: return grid_cube_impl<__hip_bfloat16>(stack, geom, nullptr, vol, N, M, K, nb, accumulate, flat, s);
      case 2: return grid_cube_impl<__half>(stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (rows == 4) return grid_dtype<4>(axis_fast, dtype, stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
  if (rows == 2 && axis_fast)
    return grid_dtype<2>(axis_fast, dtype, stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
  if (rows == 8) return grid_dtype<8>(axis_fast, dtype, stack, geom, scale, vol, N, M, K, nb, accumulate, flat, s);
  return hipErrorInvalidValue;
}

hipError_t launch_filter_table(const FilterArgs& fa, const ViewGeom* geom, const double* wtab, float4* filt,
                               hipStream_t s) {
  const size_t total = size_t(fa.M) * fa.M * fa.n_views;
  hipLaunchKernelGGL(k_filter_table, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, fa, geom, wtab,
                     filt);
  return hipGetLastError();
}

hipError_t launch_sampling(const FilterArgs& fa, const ViewGeom* geom, unsigned long long* smat,
                           double* wtab, hipStream_t s) {
  const size_t total = size_t(fa.M) * fa.M * fa.n_views;
  const dim3 grid(unsigned((total + 255) / 256));
  hipLaunchKernelGGL(k_sampling_splat, grid, dim3(256), 0, s, fa, geom, smat);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sampling_weights, grid, dim3(256), 0, s, fa, geom, smat, wtab);
  return hipGetLastError();
}

hipError_t launch_sampling_splat(const FilterArgs& fa, const ViewGeom* geom, unsigned long long* smat,
                                 hipStream_t s) {
  const size_t total = size_t(fa.M) * fa.M * fa.n_views;
  hipLaunchKernelGGL(k_sampling_splat, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, fa, geom, smat);
  return hipGetLastError();
}

hipError_t launch_spectra_out(const float4* q, float2* out, int M, int nb, hipStream_t s) {
  const size_t count = size_t(M) * M * nb;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spectra_out, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, q, out, count,
                     float(double(M) * M));
  return hipGetLastError();
}

}  // namespace tomo

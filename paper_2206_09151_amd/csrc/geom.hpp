// Frequency-grid geometry shared by the plan-time tables and the Fourier-space kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "tomo_internal.hpp"

namespace tomo {

// Signed frequency index of DFT bin k (fftfreq order).
__device__ __forceinline__ int signed_index(int k, int M) { return (k < (M + 1) / 2) ? k : k - M; }

// Spatial frequency of DFT bin k of an M-point transform with sample spacing dx.
__device__ __forceinline__ double signed_q(int k, int M, double dx) {
  return double(signed_index(k, M)) / (double(M) * dx);
}

// Point p = qx u + qy v - ewald (lambda q^2 / 2) d of detector bin (ky, kx) on the view's
// paraboloid (eqs. 8/10), in units of the 3D grid spacing 1/(N dx).
__device__ __forceinline__ void sample_point(const FilterArgs& fa, const ViewGeom& g, int ky, int kx,
                                             double* p) {
  const double qx = signed_q(kx, fa.M, fa.dx), qy = signed_q(ky, fa.M, fa.dx);
  const double qz = -double(fa.ewald) * fa.lambda * (qx * qx + qy * qy) * 0.5;
  const double sc = double(fa.N) * fa.dx;
#pragma unroll
  for (int a = 0; a < 3; ++a) p[a] = (qx * g.u[a] + qy * g.v[a] + qz * g.d[a]) * sc;
}

// Sampling matrix fixed point: 2^-32 units.
constexpr double kFix = 4294967296.0;

}  // namespace tomo

// Internal interface between the C-ABI host code and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tomo {

// Per-view geometry in FP64: detector frame (u, v, d), distance R_n and the
// angular quadrature weight a_n of the axis ramp.
struct ViewGeom {
  double u[3], v[3], d[3];
  double R, a, pad;
};

struct FilterArgs {
  int n_views, M, N;
  double dx, lambda, sigma, epsilon, eps_sampling;
  int ewald, mode;  // mode: 0 axis ramp, 1 isotropic ramp, 2 sampling matrix
};

// Supported detector sizes of the LDS-resident 2D FFT (every 2,3,5-smooth M in [16, 256]),
// threads per workgroup, and the block split P (1: direct; M = P H for M > 200).
bool fft_supported(int M);
int fft_threads(int M);
int fft_split(int M);

// g = ln(I/I_in) -> 2D DFT -> (G1 G, G2 G) for nb views.  filt, q: [nb][M][M] float4.
// scale (FP16 planes only, else NULL): per-view power-of-two plane scale, [nb].
// Split sizes (P > 1) also need the H-point twiddles, H = M / P (tw_half_fwd), and a
// [nb][P^2] scratch for the block bounds (l1part, FP16 only).
hipError_t launch_spectra(int M, const float* images, const float4* filt, const float2* tw_fwd,
                          float4* q, int* status, double inv_iin, float* scale, int nb, hipStream_t s,
                          const float2* tw_half_fwd, float* l1part);
// Plane pairs (p, K-1-p), p < npairs, of nb views -> stack [nb][M][K][M] of dtype
// (0 FP32, 1 BF16, 2 FP16 scaled by scale[view]).
hipError_t launch_planes(int M, int dtype, const float4* q, const float2* prop, const float2* tw_inv,
                         void* stack, int K, int npairs, int nb, const float* scale, hipStream_t s,
                         const float2* tw_half_inv);
// Trilinear gather of nb stacks into V[N][N][N] (accumulate: V += ..., else V = ...).
// flat: one plane without depth axis (no Ewald curvature): bilinear in the detector plane.
// rows: voxel rows per thread (4 or 8) of the row-tiled kernels; for views in general frames
// (single-axis plans keep the row-tiled kernel) 0 selects the cubic-tile kernel and kGridTilt8 /
// kGridTilt4 / kGridTilt2 the near-axis LDS-fetch box kernel with 8 / 4 / 2 voxel rows per thread.
constexpr int kGridTilt8 = -8, kGridTilt4 = -4, kGridTilt2 = -2;
hipError_t launch_grid(bool axis_fast, int dtype, const void* stack, const ViewGeom* geom, const float* scale,
                       float* vol, int N, int M, int K, int nb, int accumulate, int flat, hipStream_t s, int rows);
// Plan-time tables.
hipError_t launch_filter_table(const FilterArgs& fa, const ViewGeom* geom, const double* wtab,
                               float4* filt, hipStream_t s);
hipError_t launch_sampling(const FilterArgs& fa, const ViewGeom* geom, unsigned long long* smat,
                           double* wtab, hipStream_t s);
hipError_t launch_sampling_splat(const FilterArgs& fa, const ViewGeom* geom, unsigned long long* smat,
                                 hipStream_t s);
hipError_t launch_spectra_out(const float4* q, float2* out, int M, int nb, hipStream_t s);

// ---- Fourier-space form (eq. 11 / eq. 12 by 3D gridding)
struct FourierNormArgs {
  int N, P;            // grid edge; accumulator edge (N + 1 for even N)
  int eq12, ewald;
  double eps_s;        // regulariser of S^-1
  double nsr_m;        // NSR * M (0: no threshold)
  double out_scale;    // C dx^2 / (N dx)^3
  double dx, lambda, sigma, epsilon, R;   // eq. 12 bracket
};
bool fourier_grid_supported(int N);
// filt [n][M][M]: (H_n s, 0) (eq. 11) or (s, 0) (eq. 12), s = centring phase of the DFT.
hipError_t launch_fourier_filter(const FilterArgs& fa, const ViewGeom* geom, int eq12, float4* filt,
                                 hipStream_t s);
// Fixed-point unit from view_scale [n] into fix[2], clear acc [P^3][2], splat q [n][M][M] (.xy).
hipError_t launch_fourier_splat(const FilterArgs& fa, const ViewGeom* geom, const float4* q, const float* view_scale,
                                double* fix, unsigned long long* acc, int P, hipStream_t s);
// Hermitian fold + normalisation of the accumulator into grid [N^3] (FFT order).
hipError_t launch_fourier_norm(const FourierNormArgs& a, const unsigned long long* acc, const unsigned long long* smat,
                               const double* fix, float2* grid, hipStream_t s);
// Inverse 3D FFT of grid (tw: [N] exp(+i 2 pi k/N)), real part into vol [N^3].
hipError_t launch_fourier_fft3(int N, float2* grid, const float2* tw, float* vol, hipStream_t s);
// Gridding operator: per-vertex entry counts (count [P^3], zeroed), then the entries
// (sample index, FP32 weight) at row_ptr [P^3 + 1] offsets (cursor [P^3], zeroed), sorted.
hipError_t launch_fourier_op_count(const FilterArgs& fa, const ViewGeom* geom, int P, unsigned* count,
                                  hipStream_t s);
hipError_t launch_fourier_op_fill(const FilterArgs& fa, const ViewGeom* geom, int P, const unsigned* row_ptr,
                                 unsigned* cursor, int2* ent, hipStream_t s);
// Gather through the operator, Hermitian fold and normalisation into grid [N^3] (FFT order).
hipError_t launch_fourier_gather(const FourierNormArgs& a, const unsigned* row_ptr, const int2* ent,
                                 const float4* q, const unsigned long long* smat, float2* grid, hipStream_t s);

}  // namespace tomo

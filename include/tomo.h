/*
 * tomo.h -- C ABI of the MI355X (gfx950) reconstruction library libtomo.so.
 *
 * Method: Gureyev, Brown, Quiney, Allen, "Fast unified reconstruction algorithm
 * for conventional, phase-contrast and diffraction tomography", arXiv:2206.09151.
 * For every view n the library forms the log-contrast g = ln(I_n / I_in)
 * (eq. 4 left side), its 2D DFT, applies the Tikhonov-regularised CTF inverse of
 * eq. (11) with a density weight W_n(q) that replaces 1/n_q (text after eq. 11),
 * back-propagates the result to K depth planes with the Fresnel propagator of
 * eq. (3) (the Ewald paraboloid of eqs. 8/10), keeps the real part, and grids
 * the plane stacks into the voxel volume by trilinear interpolation (eight
 * neighbours, weights summing to one; text after eq. 11), summed over views.
 * With ewald = 0 the bracket's imaginary part and the depth planes are dropped
 * (eq. 13: phase-contrast / conventional CT).
 *
 * Conventions (all calls):
 *   - Volume V: float32 [N][N][N], index [iz][iy][ix] (x fastest).  Voxel
 *     (iz,iy,ix) sits at ((ix,iy,iz) - (N-1)/2) * voxel_size, relative to the
 *     rotation centre.
 *   - Image n: float32 [M][M], index [row][col]; pixel (a,b) sits at
 *     x' = (b-(M-1)/2) dx along u_n, y' = (a-(M-1)/2) dx along v_n.  Images are
 *     flat-field normalised intensities; every value must be finite and > 0.
 *   - View frame: d_n is the unit illumination direction (beam along +d_n);
 *     v_n is the lab y axis projected onto the detector plane (lab x if d_n is
 *     within 1e-6 of +-y) unless vaxes gives it; u_n = v_n x d_n.
 *   - Depth planes z'_j = (j - (K-1)/2) * voxel_size, j = 0..K-1.  dist[n] = R_n
 *     is measured from the plane z' = 0 through the rotation centre.
 *   - Plane stack (tomo_backpropagate output / tomo_grid input): [nb][M][K][M] of the
 *     plan's plane_dtype, index [view][row][plane][col]; with ewald = 0, K = 1.
 *   - Device pointers must be 256-byte aligned device allocations owned by the
 *     caller; they are never freed or retained by the library.
 *   - Streams are hipStream_t passed as void*; NULL means the null stream.
 *     Every call enqueues asynchronously on its stream except where stated.
 *     A plan is used by one stream at a time; apart from the per-GPU workspace of
 *     tomo_backpropagate_noalloc there is no global state.
 *
 * Errors: every call returns tomo_status and never aborts or throws.
 *   TOMO_EINVAL       bad argument (null pointer, non-unit direction, bad range)
 *   TOMO_ENOMEM       device allocation failed or would exceed max_workspace_bytes
 *   TOMO_EDEVICE      a HIP call failed (message in tomo_last_error)
 *   TOMO_EDOMAIN      an image value was <= 0 or not finite (detected on the
 *                     device; reported by the next synchronising call)
 *   TOMO_EUNSUPPORTED size or option not implemented (message says which)
 */
#ifndef TOMO_H
#define TOMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tomo_plan_s* tomo_plan_t;

typedef enum {
  TOMO_OK = 0,
  TOMO_EINVAL = 1,
  TOMO_ENOMEM = 2,
  TOMO_EDEVICE = 3,
  TOMO_EDOMAIN = 4,
  TOMO_EUNSUPPORTED = 5
} tomo_status;

/* Density weight W_n(q) replacing 1/n_q of eq. (11) (text after eq. 11, Section 4):
 *   TOMO_RAMP_AXIS  a_n |q.u_n|: single-axis scan about y (every d_n.y == 0 within
 *                   1e-9); a_n = trapezoid weight of the view's angle folded into
 *                   [0, pi) (pi/n for uniform 180- or 360-degree scans).
 *   TOMO_RAMP_ISO   2|q|/n: directions uniform on the sphere.
 *   TOMO_SAMPLING   M^2/(N^3 dx) * S/(S^2 + eps_sampling) with S the trilinear
 *                   sampling matrix on the N^3 Fourier grid (spacing 1/(N dx)),
 *                   interpolated at the sample; every sample and its point
 *                   reflection add half their weights; zero off the grid. */
typedef enum { TOMO_RAMP_AXIS = 0, TOMO_RAMP_ISO = 1, TOMO_SAMPLING = 2 } tomo_weight_mode;

/* Storage type of the plane stack.  Interpolation and accumulation are FP32 for all
 * three.  TOMO_BF16 rounds each plane value to nearest even; TOMO_F16 first multiplies a
 * view's planes by a power of two chosen from a bound on the view's plane values
 * (2^14 / sum of spectral magnitudes, rounded to a power of two) so that they sit in
 * the FP16 normal range; the plan keeps that per-view scale and tomo_grid divides it
 * out, so FP16 stacks must be gridded by the plan that back-propagated them. */
typedef enum { TOMO_F32 = 0, TOMO_BF16 = 1, TOMO_F16 = 2 } tomo_dtype;

typedef struct {
  int32_t n_vox;          /* N: volume edge in voxels (>= 2) */
  int32_t n_pix;          /* M: image edge in pixels; 0 -> N */
  int32_t n_planes;       /* K: depth planes per view; 0 -> N (ewald = 1); forced to 1 when ewald = 0 */
  int32_t n_angles;       /* n: number of views (>= 1) */
  double voxel_size;      /* dx [m], voxel edge = detector pixel (> 0) */
  double wavelength;      /* lambda [m] (> 0) */
  double sigma;           /* beta/delta of the monomorphous object (finite); omega = atan(sigma) */
  double epsilon;         /* Tikhonov epsilon of eq. (11) (> 0) */
  double eps_sampling;    /* regulariser of S^-1 in TOMO_SAMPLING (>= 0; 0 -> 1e-3) */
  double i_in;            /* flat-field intensity I_in (> 0; 0 -> 1) */
  int32_t ewald;          /* 1: eq. (11) with depth planes; 0: eq. (13), one plane */
  int32_t weight_mode;    /* tomo_weight_mode */
  int32_t plane_dtype;    /* tomo_dtype of the plane stack */
  int32_t angle_batch;    /* views per internal batch of tomo_reconstruct; 0 -> automatic */
  int32_t fourier;        /* workspace of tomo_fourier_reconstruct (needs n_vox among the
                             FFT sizes below): 0 none; 1 the gridding operator, built here (8 bytes
                             per non-zero trilinear weight, at most 64 n M^2 bytes), used as a
                             gather per call; 2 a per-call splat with 64-bit integer atomics
                             (16 (N+1)^3 bytes) */
  int32_t tune;           /* 1: time the gridding variants on a batch of stacks at plan time
                             and keep the fastest: 4 or 8 voxel rows per thread (also 2 for
                             single-axis plans), and for views in general frames also 8x8x8
                             cubic tiles and the near-axis box kernel (footprints of 16 x 8, 4
                             or 2 x 16 voxel tiles fetched straight into LDS); 0: 8 rows;
                             2: cubic tiles for general frames; 3, 4, 5: the near-axis box
                             kernel with 4, 8, 2 rows for general frames (single-axis plans
                             keep 8 rows for 2 to 4 and take 2 rows for 5).  Single-axis plans
                             give identical results either way; for other frames the choice
                             moves only the FP32 rounding */
  size_t max_workspace_bytes; /* 0 -> unlimited; otherwise tomo_plan fails with TOMO_ENOMEM
                                 when plan tables + workspace would exceed it */
} tomo_params;

/* Create a plan: validates parameters, builds the view frames, the density
 * weights, the per-view filter table C W_n H_n (computed in FP64 on the device,
 * stored FP32) and the propagator table, and allocates the workspace.
 *   p      parameters (host; copied)
 *   dirs   host double [n][3], unit illumination directions (|norm - 1| <= 1e-9)
 *   vaxes  host double [n][3] detector row axes, or NULL for the default rule
 *   dist   host double [n], R_n (finite)
 *   stream hipStream_t the plan's set-up work runs on (synchronised before return)
 *   out    receives the plan; untouched on error.
 * Supported: M every 2^a 3^b 5^c in [16, 256] (others: TOMO_EUNSUPPORTED); N in [2, 1024];
 * K in [1, 2N]; with fourier = 1 or 2 also N = 2^a 3^b 5^c in [16, 256].  Single-axis
 * plans whose stack rows are whole 16-byte chunks (M a multiple of 4, or of 8 for 16-bit
 * planes, and M - N even) use the single-axis gridding kernel; the others use the
 * general-frame kernels (the cubic-tile kernel when M is not such a multiple). */
tomo_status tomo_plan(const tomo_params* p, const double* dirs, const double* vaxes,
                      const double* dist, void* stream, tomo_plan_t* out);

/* Back-propagate views [first, first+nb): contrast, 2D DFT, filter (eq. 11),
 * propagation to every depth plane (eq. 3), real part.  Writes the plane stacks
 * d_planes (device, [nb][M][K][M] of plane_dtype, fully overwritten).
 * d_images: device float32 [nb][M][M], the images of those views.  Asynchronous:
 * an invalid image value raises TOMO_EDOMAIN at the next tomo_sync/tomo_reconstruct.
 * Uses the plan's spectrum slots of those views (calls on one plan are serial). */
tomo_status tomo_backpropagate(tomo_plan_t plan, const float* d_images, int32_t first, int32_t nb,
                               void* d_planes, void* stream);

/* tomo_backpropagate for callers that cannot allocate device memory (work recorded under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and the same output, bit for bit, but the filtered spectra of the nb views
 * (16 M^2 bytes per view) live in a static device workspace of
 * TOMO_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on (from the
 * first plan made there until the process ends) instead of the plan's workspace.  The call
 * allocates no device or host memory on success: no hipMalloc, hipFree or allocating
 * library routine (plan timing is not recorded for it).  Arguments and layouts as
 * tomo_backpropagate; the plan (made beforehand) still provides its tables and the FP16
 * per-view scales.
 *   TOMO_EINVAL  bad range or pointer, or nb * 16 M^2 > TOMO_NOALLOC_SCRATCH_BYTES (the
 *                message says so; split the views over several calls)
 *   TOMO_EDEVICE the workspace's device address could not be obtained or a launch failed
 * Every call on one GPU uses that GPU's single workspace: calls that overlap in time on one
 * GPU (on different streams, or from different plans or threads) race and must be
 * serialised by the caller.  A call leaves the spectra of its views in the workspace; each
 * call overwrites what it reads, so nothing needs clearing between calls. */
#define TOMO_NOALLOC_SCRATCH_BYTES (32u << 20)
tomo_status tomo_backpropagate_noalloc(tomo_plan_t plan, const float* d_images, int32_t first, int32_t nb,
                                       void* d_planes, void* stream);

/* Grid plane stacks of views [first, first+nb) into the volume: for every voxel
 * the trilinear value of each view's stack at the voxel's view-frame position
 * (taps outside the stack count as zero) is added to d_volume (device float32
 * [N][N][N], accumulated: V += sum over the nb views, in ascending view order).
 * Deterministic: no atomics. */
tomo_status tomo_grid(tomo_plan_t plan, const void* d_planes, int32_t first, int32_t nb,
                      float* d_volume, void* stream);

/* Whole reconstruction: d_volume (device float32 [N][N][N]) is overwritten with
 * the sum over all n views, processed in internal batches of the plan's batch
 * size.  d_images: device float32 [n][M][M].  Synchronises the stream once at
 * the end to report TOMO_EDOMAIN. */
tomo_status tomo_reconstruct(tomo_plan_t plan, const float* d_images, float* d_volume, void* stream);

/* tomo_reconstruct without the final synchronisation: every kernel of the reconstruction
 * is enqueued on the stream and the call returns at once, so that repeated
 * reconstructions keep the GPU busy without a host round trip per call.  The result is
 * the same as tomo_reconstruct's, bit for bit.  An invalid image value is reported as
 * TOMO_EDOMAIN by the next tomo_sync (or tomo_reconstruct) on the plan; argument errors
 * are returned at once as TOMO_EINVAL. */
tomo_status tomo_reconstruct_async(tomo_plan_t plan, const float* d_images, float* d_volume, void* stream);

/* Synchronise the stream and report any device-detected domain error since the
 * last report (TOMO_EDOMAIN) or TOMO_OK. */
tomo_status tomo_sync(tomo_plan_t plan, void* stream);

/* Filtered spectra of views [first, first+nb) for inspection: d_out (device
 * float32 complex, [nb][M][M][2], index [view][ky][kx][re/im]) receives
 * P_n = C W_n H_n DFT2(ln(I_n/I_in)) as defined by eq. (11) (no 1/M^2 factor). */
tomo_status tomo_filtered_spectra(tomo_plan_t plan, const float* d_images, int32_t first,
                                  int32_t nb, float* d_out, void* stream);

/* Fourier-space form of the method (the paper's own gridding): every view's
 * spectrum DFT2(ln(I_n/I_in)), with its phase origin moved to the detector centre,
 * is multiplied by the bracket H_n of eq. (11) (variant TOMO_EQ11) or left as is
 * (TOMO_EQ12), and spread, with its complex conjugate at the reflected point, over
 * the eight vertices of the N^3 grid of 3D frequencies (spacing 1/(N dx)) around
 * its paraboloid point q_x u_n + q_y v_n - ewald (lambda q^2/2) d_n, half of the
 * trilinear weights each (text after eq. 11).  The grid is divided by the
 * regularised sampling matrix, S/(S^2 + eps_sampling); coefficients whose
 * magnitude (in the images' DFT units) is below nsr * M / sqrt(S) are zeroed
 * (Section 3; nsr = 0 keeps all); TOMO_EQ12 then multiplies by the bracket of
 * eq. (12) at the common R and the 3D frequency |k|/(N dx); the inverse 3D Fourier
 * integral at the voxel centres, times C = lambda / (4 pi sqrt(1 + sigma^2)), is
 * written to d_volume (device float32 [N][N][N], overwritten).
 * With fourier = 1 every vertex sums its contributions in FP64 in ascending sample
 * order (the plan sorted the operator's entries); with fourier = 2 the splat adds 64-bit
 * fixed-point integers (unit from a bound on the sums).  Either way results are
 * bitwise reproducible.  Needs a plan made with fourier = 1 or 2;
 * TOMO_EQ12 needs every dist[n] equal (else TOMO_EINVAL).  weight_mode, n_planes
 * and plane_dtype do not enter.  d_images: device float32 [n][M][M].
 * Synchronises the stream at the end to report TOMO_EDOMAIN. */
typedef enum { TOMO_EQ11 = 11, TOMO_EQ12 = 12 } tomo_fourier_variant;
tomo_status tomo_fourier_reconstruct(tomo_plan_t plan, const float* d_images, int32_t variant,
                                     double nsr, float* d_volume, void* stream);

/* tomo_fourier_reconstruct without the final synchronisation (as tomo_reconstruct_async
 * is to tomo_reconstruct): the kernels are enqueued and the call returns; a domain error
 * is reported by the next tomo_sync; the result is the same bit for bit. */
tomo_status tomo_fourier_reconstruct_async(tomo_plan_t plan, const float* d_images, int32_t variant,
                                           double nsr, float* d_volume, void* stream);

/* Per-kernel timing (tracing).  While enabled, every kernel launch of the plan is
 * bracketed by two HIP events recorded on the launch's stream.  Kinds:
 *   0 = contrast + DFT + filter (spectra), 1 = depth planes (inverse FFTs),
 *   2 = gridding, 3 = Fourier-space gridding (fourier = 1: operator gather with the
 *   normalisation; fourier = 2: bound, clear, splat), 4 = Fourier-space normalisation
 *   (fourier = 2 only) and inverse 3D FFT.
 * tomo_timing_read synchronises on the recorded events, adds their elapsed
 * times to the totals, and returns, per kind, total milliseconds and launch
 * counts since the last reset (reset != 0 clears them afterwards).  total_ms and
 * launches are host arrays of TOMO_TIMING_KINDS entries. */
#define TOMO_TIMING_KINDS 5
tomo_status tomo_timing_enable(tomo_plan_t plan, int32_t enable);
tomo_status tomo_timing_read(tomo_plan_t plan, double* total_ms, int64_t* launches, int32_t reset);

/* Batched uneven jobs: many independent reconstructions (each with its own plan, of any
 * size and geometry) recorded once into one HIP graph and launched with one call.
 * tomo_batch_create records, for job j, every kernel tomo_reconstruct would launch for
 * plans[j] on d_images[j] -> d_volumes[j] (no synchronisation inside); the jobs are dealt
 * to `lanes` parallel branches of the graph (0 -> min(count, 8)), longest job first onto
 * the least loaded branch (work = N^3 n), so kernels of different jobs run concurrently.
 *   plans      host array of count distinct plans (each job needs its own workspace)
 *   d_images   host array of count device pointers, float32 [n_j][M_j][M_j]
 *   d_volumes  host array of count device pointers, float32 [N_j][N_j][N_j] (overwritten)
 * The buffers and plans are bound into the graph: they must stay valid and at the same
 * addresses for every launch, and the plans must not run other work concurrently with a
 * launch.  Plan timing is off while recording (the graph holds no event nodes).
 * tomo_batch_launch enqueues the graph on stream (asynchronous); tomo_batch_sync
 * synchronises stream and reports TOMO_EDOMAIN if any job saw an invalid image value
 * (tomo_batch_error names the first such job).  Errors of tomo_batch_create are reported
 * by tomo_plan_error. */
typedef struct tomo_batch_s* tomo_batch_t;
tomo_status tomo_batch_create(const tomo_plan_t* plans, const float* const* d_images, float* const* d_volumes,
                              int32_t count, int32_t lanes, tomo_batch_t* out);
tomo_status tomo_batch_launch(tomo_batch_t batch, void* stream);
tomo_status tomo_batch_sync(tomo_batch_t batch, void* stream);
const char* tomo_batch_error(tomo_batch_t batch);
tomo_status tomo_batch_destroy(tomo_batch_t batch);

/* Gridding variant of the plan: voxel rows per thread (4 or 8, or 2 for single-axis plans) of the
 * row-tiled kernels, 0 for cubic tiles, -8, -4 or -2 for the near-axis box kernel with 8, 4 or 2
 * rows per thread (see tune). */
int32_t tomo_grid_rows(tomo_plan_t plan);

/* Non-zero entries of the plan's Fourier-space gridding operator (0 unless fourier = 1). */
size_t tomo_fourier_entries(tomo_plan_t plan);

/* Bytes of plan tables + workspace that tomo_plan would allocate for p (0 if p is invalid;
 * with fourier = 1 an upper bound: the operator's exact size is known after planning). */
size_t tomo_workspace_bytes(const tomo_params* p);

/* Views per internal batch of tomo_reconstruct (plane stacks held at once). */
int32_t tomo_batch_capacity(tomo_plan_t plan);

/* Bytes of nb plane stacks in the layout above. */
size_t tomo_stack_bytes(tomo_plan_t plan, int32_t nb);

/* Static description of a status code. */
const char* tomo_status_string(tomo_status s);

/* Message of the last failing call on this plan ("" if none).  Valid until the
 * next call on the plan. */
const char* tomo_last_error(tomo_plan_t plan);

/* Message of the last tomo_plan failure in this thread. */
const char* tomo_plan_error(void);

/* Release the plan's device memory (synchronises its last stream). NULL is OK. */
tomo_status tomo_destroy(tomo_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* TOMO_H */

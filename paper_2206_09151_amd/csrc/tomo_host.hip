// C-ABI host side of libtomo.so: validation, view frames, plan tables, workspace,
// batching and error reporting.  Every compute step runs in the kernels of
// tomo_kernels.hip; the host only prepares geometry constants (frames, angular
// weights, propagator and twiddle tables) in FP64 at plan time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "tomo.h"
#include "tomo_internal.hpp"

using tomo::ViewGeom;

struct tomo_plan_s {
  tomo_params p{};
  int N = 0, M = 0, K = 0, n = 0, npairs = 0, batch = 0;
  int split = 1;                // block split of the detector-size FFT (M = P H for M > 200)
  bool axis_fast = false;
  int grid_rows = 8;            // gridding variant: 8 or 4 voxel rows per thread, 0 cubic tiles (params.tune)
  ViewGeom* d_geom = nullptr;   // [n]
  float4* d_filt = nullptr;     // [n][M][M]
  float2* d_prop = nullptr;     // [npairs][M]
  float2* d_tw_fwd = nullptr;   // [M]
  float2* d_tw_inv = nullptr;   // [M]
  float2* d_tw2_fwd = nullptr;  // [H] twiddles of the block sub-transforms of split sizes (M = P H)
  float2* d_tw2_inv = nullptr;  // [H]
  float* d_l1part = nullptr;    // [n][P^2] block spectral bounds of split sizes (FP16 planes)
  float4* d_q = nullptr;        // [n][M][M]  filtered spectra of every view
  void* d_stack = nullptr;      // [batch][M][K][M] of the plane storage type
  float* d_scale = nullptr;     // [n] FP16 plane scale per view (powers of two)
  int* d_status = nullptr;
  // Fourier-space form (params.fourier = 1: gridding operator, 2: atomic splat)
  int P = 0;                            // vertex-grid edge: N + 1 for even N, N for odd N
  float4* d_ffilt = nullptr;            // [n][M][M] filter of the Fourier-space variant built last
  int ffilt_variant = 0;                // 11, 12, or 0 before the first call
  float* d_fview = nullptr;             // [n] per-view spectral bound (power-of-two scale)
  double* d_ffix = nullptr;             // [2] fixed-point unit and its inverse
  unsigned long long* d_facc = nullptr; // [P][P][P][2] fixed-point accumulator
  unsigned long long* d_fsmat = nullptr;// [N][N][N] sampling matrix, 2^-32 units
  float2* d_fgrid = nullptr;            // [N][N][N] complex grid of the inverse FFT
  float2* d_tw3 = nullptr;              // [N] exp(+i 2 pi k / N)
  unsigned* d_oprow = nullptr;          // [P^3 + 1] gridding operator row offsets
  int2* d_opent = nullptr;              // [entries] (sample index, FP32 weight bits)
  size_t op_entries = 0;
  bool same_R = true;
  double R0 = 0.0;
  void* scratch = nullptr;              // this device's copy of the allocation-free workspace
  std::string err;                      // capacity reserved at plan time (error paths of the
                                        // allocation-free call assign within it)
  // tracing: events around launches while timing is on
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<hipEvent_t> pool;
  std::vector<Rec> recs;
  double tot_ms[TOMO_TIMING_KINDS] = {};
  long long launches[TOMO_TIMING_KINDS] = {};
};

static __device__ __align__(256) unsigned char scratch[TOMO_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_plan_error;

// Workspace of tomo_backpropagate_noalloc: the filtered spectra of the views of one call.
// A file-scope device array (one copy per GPU, kept until the process ends); host code
// reaches it only through the address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(TOMO_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

constexpr double kPi = 3.141592653589793238462643383279502884;

struct Resolved {
  int N, M, K, n, npairs, batch, P;
  size_t table_bytes, work_bytes;
};

size_t dtype_bytes(int dtype) { return dtype == TOMO_F32 ? 4 : 2; }

size_t stack_view_bytes(int M, int K, int dtype) { return size_t(M) * K * M * dtype_bytes(dtype); }

// Resolve defaults and sizes; returns an error message or "" and fills r.
std::string resolve(const tomo_params* p, Resolved* r) {
  if (!p) return "params is NULL";
  if (p->n_vox < 2 || p->n_vox > 1024) return "n_vox must be in [2, 1024]";
  if (p->n_angles < 1) return "n_angles must be >= 1";
  if (!(p->voxel_size > 0) || !std::isfinite(p->voxel_size)) return "voxel_size must be finite and > 0";
  if (!(p->wavelength > 0) || !std::isfinite(p->wavelength)) return "wavelength must be finite and > 0";
  if (!std::isfinite(p->sigma)) return "sigma must be finite";
  if (!(p->epsilon > 0) || !std::isfinite(p->epsilon)) return "epsilon must be finite and > 0";
  if (p->eps_sampling < 0 || !std::isfinite(p->eps_sampling)) return "eps_sampling must be finite and >= 0";
  if (p->i_in < 0 || !std::isfinite(p->i_in)) return "i_in must be finite and >= 0";
  if (p->ewald != 0 && p->ewald != 1) return "ewald must be 0 or 1";
  if (p->weight_mode < 0 || p->weight_mode > 2) return "weight_mode must be 0, 1 or 2";
  if (p->plane_dtype < 0 || p->plane_dtype > 2) return "plane_dtype must be 0, 1 or 2";
  if (p->angle_batch < 0) return "angle_batch must be >= 0";
  if (p->fourier < 0 || p->fourier > 2) return "fourier must be 0, 1 or 2";
  if (p->tune < 0 || p->tune > 5) return "tune must be in [0, 5]";
  r->N = p->n_vox;
  r->M = p->n_pix ? p->n_pix : p->n_vox;
  if (p->n_pix < 0) return "n_pix must be >= 0";
  if (p->n_planes < 0) return "n_planes must be >= 0";
  r->K = p->ewald ? (p->n_planes ? p->n_planes : p->n_vox) : 1;
  if (r->K > 2 * r->N) return "n_planes must be <= 2 * n_vox";
  r->n = p->n_angles;
  r->npairs = (r->K + 1) / 2;
  const size_t sv = stack_view_bytes(r->M, r->K, p->plane_dtype);
  const size_t qv = size_t(r->M) * r->M * sizeof(float4);
  if (p->angle_batch > 0) {
    r->batch = std::min(p->angle_batch, r->n);
  } else {
    // automatic: about 128 MiB of stacks per batch (they stay in the 256 MB last-level
    // cache between the back-propagation and the gridding kernels), a multiple of 8
    // and at least 8 views: the plane kernels put each view on one of the 8 XCDs
    const size_t target = size_t(128) << 20;
    int b = int(std::max<size_t>(8, target / sv));
    b -= b % 8;
    r->batch = std::min(b, r->n);
  }
  r->table_bytes = size_t(r->n) * sizeof(ViewGeom) + size_t(r->n) * qv + size_t(r->npairs) * r->M * 8 +
                   4 * size_t(r->M) * 8 + size_t(r->n) * 4 * 10 + 256;
  r->work_bytes = size_t(r->n) * qv + size_t(r->batch) * sv;
  r->P = r->N + (r->N % 2 == 0 ? 1 : 0);
  if (p->fourier) {
    const size_t n3 = size_t(r->N) * r->N * r->N, p3 = size_t(r->P) * r->P * r->P;
    r->table_bytes += size_t(r->n) * qv + n3 * 8 + size_t(r->N) * 8 + size_t(r->n) * 4 + 16;
    r->work_bytes += n3 * 8;
    if (p->fourier == 2) {
      r->work_bytes += p3 * 16;
    } else {
      // operator: row offsets + at most 8 entries of 8 bytes per sample (the exact count
      // is known after the plan's counting pass)
      r->table_bytes += (p3 + 1) * 4 + size_t(r->n) * r->M * r->M * 8 * 8;
    }
  }
  return "";
}

std::string supported(const tomo_params* p, const Resolved& r) {
  if (!tomo::fft_supported(r.M)) {
    char b[160];
    std::snprintf(b, sizeof b, "n_pix = %d not supported (supported: every M = 2^a 3^b 5^c in [16, 256])", r.M);
    return b;
  }
  if (p->fourier && !tomo::fourier_grid_supported(r.N)) {
    char b[160];
    std::snprintf(b, sizeof b,
                  "fourier = 1 or 2 needs n_vox = 2^a 3^b 5^c in [16, 256] (got %d)", r.N);
    return b;
  }
  return "";
}

// O1-style frames in FP64: v = y projected on the detector plane (x near the poles), u = v x d.
void make_frames(const double* dirs, const double* vaxes, int n, std::vector<ViewGeom>& g) {
  g.resize(n);
  for (int i = 0; i < n; ++i) {
    const double* d = dirs + 3 * i;
    double ref[3];
    if (vaxes) {
      std::memcpy(ref, vaxes + 3 * i, sizeof ref);
    } else {
      // |y x d| = sqrt(d_x^2 + d_z^2)
      const double cr = std::sqrt(d[0] * d[0] + d[2] * d[2]);
      ref[0] = cr < 1e-6 ? 1.0 : 0.0;
      ref[1] = cr < 1e-6 ? 0.0 : 1.0;
      ref[2] = 0.0;
    }
    const double dot = ref[0] * d[0] + ref[1] * d[1] + ref[2] * d[2];
    double v[3] = {ref[0] - dot * d[0], ref[1] - dot * d[1], ref[2] - dot * d[2]};
    const double nv = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (double& x : v) x /= nv;
    ViewGeom& vg = g[i];
    for (int a = 0; a < 3; ++a) {
      vg.d[a] = d[a];
      vg.v[a] = v[a];
    }
    vg.u[0] = v[1] * d[2] - v[2] * d[1];
    vg.u[1] = v[2] * d[0] - v[0] * d[2];
    vg.u[2] = v[0] * d[1] - v[1] * d[0];
    vg.R = 0;
    vg.a = 0;
    vg.pad = 0;
  }
}

// Trapezoid weights of the view angles folded into [0, pi) on a circle of period pi.
void axis_weights(const double* dirs, int n, std::vector<ViewGeom>& g) {
  std::vector<double> phi(n);
  for (int i = 0; i < n; ++i) {
    double a = std::atan2(dirs[3 * i], dirs[3 * i + 2]);
    a = std::fmod(a, kPi);
    if (a < 0) a += kPi;
    if (a >= kPi) a -= kPi;
    phi[i] = a;
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return phi[a] < phi[b]; });
  for (int k = 0; k < n; ++k) {
    const double nxt = (k + 1 < n) ? phi[order[k + 1]] : phi[order[0]] + kPi;
    const double prv = (k > 0) ? phi[order[k - 1]] : phi[order[n - 1]] - kPi;
    g[order[k]].a = 0.5 * (nxt - prv);
  }
}

// Device address of the current device's copy of `scratch`, looked up once per device.
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

template <class T>
hipError_t dev_alloc(T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc(reinterpret_cast<void**>(ptr), count * sizeof(T));
}

hipEvent_t take_event(tomo_plan_s* pl) {
  if (!pl->pool.empty()) {
    hipEvent_t e = pl->pool.back();
    pl->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing only (read after the stream is synchronised): no system-scope fence, which would
  // write back and invalidate caches around every timed launch and slow the launches it times
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Launch wrapper: records an event pair around the launch when timing is on.
template <class F>
hipError_t timed(tomo_plan_s* pl, int kind, hipStream_t s, F&& launch) {
  if (!pl->timing) return launch();
  hipEvent_t a = take_event(pl), b = take_event(pl);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  pl->recs.push_back({kind, a, b});
  return e;
}

void free_plan(tomo_plan_s* pl) {
  for (auto& r : pl->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pl->pool) (void)hipEventDestroy(e);
  pl->recs.clear();
  pl->pool.clear();
  (void)hipFree(pl->d_geom);
  (void)hipFree(pl->d_filt);
  (void)hipFree(pl->d_prop);
  (void)hipFree(pl->d_tw_fwd);
  (void)hipFree(pl->d_tw_inv);
  (void)hipFree(pl->d_tw2_fwd);
  (void)hipFree(pl->d_tw2_inv);
  (void)hipFree(pl->d_l1part);
  (void)hipFree(pl->d_q);
  (void)hipFree(pl->d_stack);
  (void)hipFree(pl->d_scale);
  (void)hipFree(pl->d_status);
  (void)hipFree(pl->d_ffilt);
  (void)hipFree(pl->d_fview);
  (void)hipFree(pl->d_ffix);
  (void)hipFree(pl->d_facc);
  (void)hipFree(pl->d_fsmat);
  (void)hipFree(pl->d_fgrid);
  (void)hipFree(pl->d_tw3);
  (void)hipFree(pl->d_oprow);
  (void)hipFree(pl->d_opent);
}

tomo_status fail(tomo_plan_s* pl, tomo_status st, const std::string& msg) {
  if (pl) pl->err = msg;
  return st;
}

tomo_status dev_fail(tomo_plan_s* pl, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  if (pl) pl->err = m;
  return TOMO_EDEVICE;
}

}  // namespace

extern "C" {

const char* tomo_status_string(tomo_status s) {
  switch (s) {
    case TOMO_OK: return "ok";
    case TOMO_EINVAL: return "invalid argument";
    case TOMO_ENOMEM: return "out of device memory or workspace limit";
    case TOMO_EDEVICE: return "device error";
    case TOMO_EDOMAIN: return "image value <= 0 or not finite";
    case TOMO_EUNSUPPORTED: return "unsupported size or option";
  }
  return "unknown status";
}

const char* tomo_last_error(tomo_plan_t plan) { return plan ? plan->err.c_str() : "plan is NULL"; }

const char* tomo_plan_error(void) { return g_plan_error.c_str(); }

size_t tomo_workspace_bytes(const tomo_params* p) {
  Resolved r{};
  if (!resolve(p, &r).empty()) return 0;
  return r.table_bytes + r.work_bytes;
}

int32_t tomo_batch_capacity(tomo_plan_t plan) { return plan ? plan->batch : 0; }

size_t tomo_fourier_entries(tomo_plan_t plan) { return plan ? plan->op_entries : 0; }

int32_t tomo_grid_rows(tomo_plan_t plan) { return plan ? plan->grid_rows : 0; }

size_t tomo_stack_bytes(tomo_plan_t plan, int32_t nb) {
  if (!plan || nb < 0) return 0;
  return size_t(nb) * stack_view_bytes(plan->M, plan->K, plan->p.plane_dtype);
}

tomo_status tomo_plan(const tomo_params* p, const double* dirs, const double* vaxes, const double* dist,
                      void* stream, tomo_plan_t* out) {
  g_plan_error.clear();
  auto perr = [](tomo_status st, const std::string& m) {
    g_plan_error = m;
    return st;
  };
  if (!out) return perr(TOMO_EINVAL, "out is NULL");
  if (!dirs) return perr(TOMO_EINVAL, "dirs is NULL");
  if (!dist) return perr(TOMO_EINVAL, "dist is NULL");
  Resolved r{};
  std::string m = resolve(p, &r);
  if (!m.empty()) return perr(TOMO_EINVAL, m);
  m = supported(p, r);
  if (!m.empty()) return perr(TOMO_EUNSUPPORTED, m);
  for (int i = 0; i < r.n; ++i) {
    const double* d = dirs + 3 * i;
    const double nn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!std::isfinite(nn) || std::fabs(nn - 1.0) > 1e-9) {
      char b[96];
      std::snprintf(b, sizeof b, "direction %d is not a unit vector (norm %.17g)", i, nn);
      return perr(TOMO_EINVAL, b);
    }
    if (!std::isfinite(dist[i])) return perr(TOMO_EINVAL, "dist must be finite");
    if (p->weight_mode == TOMO_RAMP_AXIS && std::fabs(d[1]) > 1e-9)
      return perr(TOMO_EINVAL, "TOMO_RAMP_AXIS needs every direction perpendicular to the y axis");
    if (vaxes) {
      const double* va = vaxes + 3 * i;
      const double dot = va[0] * d[0] + va[1] * d[1] + va[2] * d[2];
      const double px = va[0] - dot * d[0], py = va[1] - dot * d[1], pz = va[2] - dot * d[2];
      if (!(std::sqrt(px * px + py * py + pz * pz) > 1e-9))
        return perr(TOMO_EINVAL, "vaxes must have a component perpendicular to its direction");
    }
  }
  const size_t total = r.table_bytes + r.work_bytes;
  if (p->max_workspace_bytes && total > p->max_workspace_bytes) {
    char b[128];
    std::snprintf(b, sizeof b, "plan needs %zu bytes > max_workspace_bytes %zu", total, p->max_workspace_bytes);
    return perr(TOMO_ENOMEM, b);
  }

  auto* pl = new tomo_plan_s();
  pl->p = *p;
  pl->N = r.N;
  pl->M = r.M;
  pl->K = r.K;
  pl->n = r.n;
  pl->npairs = r.npairs;
  pl->batch = r.batch;
  pl->P = r.P;
  pl->split = tomo::fft_split(r.M);
  pl->p.n_pix = r.M;
  pl->p.n_planes = r.K;
  if (pl->p.i_in == 0) pl->p.i_in = 1.0;
  if (pl->p.eps_sampling == 0) pl->p.eps_sampling = 1e-3;
  hipStream_t s = static_cast<hipStream_t>(stream);

  std::vector<ViewGeom> geo;
  make_frames(dirs, vaxes, r.n, geo);
  for (int i = 0; i < r.n; ++i) geo[i].R = dist[i];
  pl->R0 = dist[0];
  for (int i = 1; i < r.n; ++i) pl->same_R = pl->same_R && dist[i] == dist[0];
  if (p->weight_mode == TOMO_RAMP_AXIS) axis_weights(dirs, r.n, geo);
  // Single-axis gather path: every v is exactly the y axis and u, d lie in the xz plane,
  // and detector rows line up with voxel rows (M - N even).
  // (the LDS-fetch kernel moves 16-byte chunks: M a multiple of 4 FP32 or 8 16-bit values)
  const int vec = p->plane_dtype == TOMO_F32 ? 4 : 8;
  bool axis = ((r.M - r.N) % 2 == 0) && (r.M % vec == 0);
  for (int i = 0; i < r.n && axis; ++i)
    axis = geo[i].v[0] == 0.0 && geo[i].v[1] == 1.0 && geo[i].v[2] == 0.0 && geo[i].u[1] == 0.0 &&
           geo[i].d[1] == 0.0;
  pl->axis_fast = axis;

  // propagator table: (cos, sin)(pi lambda z'_p q^2), z'_p = (p - (K-1)/2) dx; twiddles
  std::vector<float2> prop(size_t(r.npairs) * r.M), twf(r.M), twi(r.M);
  for (int pp = 0; pp < r.npairs; ++pp) {
    const double z = (pp - 0.5 * (r.K - 1)) * p->voxel_size;
    for (int k = 0; k < r.M; ++k) {
      const int ks = (k < (r.M + 1) / 2) ? k : k - r.M;
      const double q = ks / (double(r.M) * p->voxel_size);
      const double ph = kPi * p->wavelength * z * q * q;
      prop[size_t(pp) * r.M + k] = make_float2(float(std::cos(ph)), float(std::sin(ph)));
    }
  }
  for (int k = 0; k < r.M; ++k) {
    const double a = 2.0 * kPi * k / r.M;
    twf[k] = make_float2(float(std::cos(a)), float(-std::sin(a)));
    twi[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }
  // H-point twiddles of the P^2 block transforms of split sizes (M = P H)
  const int split = tomo::fft_split(r.M);
  const int hpts = split > 1 ? r.M / split : 1;
  std::vector<float2> tw2f(hpts), tw2i(hpts);
  for (int k = 0; k < hpts; ++k) {
    const double a = 2.0 * kPi * k / hpts;
    tw2f[k] = make_float2(float(std::cos(a)), float(-std::sin(a)));
    tw2i[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }

  hipError_t e = hipSuccess;
  const size_t mm = size_t(r.M) * r.M;
  if ((e = dev_alloc(&pl->d_geom, size_t(r.n))) != hipSuccess ||
      (e = dev_alloc(&pl->d_filt, mm * r.n)) != hipSuccess ||
      (e = dev_alloc(&pl->d_prop, prop.size())) != hipSuccess ||
      (e = dev_alloc(&pl->d_tw_fwd, size_t(r.M))) != hipSuccess ||
      (e = dev_alloc(&pl->d_tw_inv, size_t(r.M))) != hipSuccess ||
      (e = dev_alloc(&pl->d_tw2_fwd, size_t(hpts))) != hipSuccess ||
      (e = dev_alloc(&pl->d_tw2_inv, size_t(hpts))) != hipSuccess ||
      (e = dev_alloc(&pl->d_l1part, size_t(split * split) * r.n)) != hipSuccess ||
      (e = dev_alloc(&pl->d_q, mm * r.n)) != hipSuccess ||
      (e = dev_alloc(reinterpret_cast<char**>(&pl->d_stack),
                     size_t(r.batch) * stack_view_bytes(r.M, r.K, p->plane_dtype))) != hipSuccess ||
      (e = dev_alloc(&pl->d_scale, size_t(r.n))) != hipSuccess ||
      (e = dev_alloc(&pl->d_status, size_t(1))) != hipSuccess) {
    free_plan(pl);
    delete pl;
    (void)hipGetLastError();
    return perr(e == hipErrorOutOfMemory ? TOMO_ENOMEM : TOMO_EDEVICE,
                std::string("allocation failed: ") + hipGetErrorString(e));
  }
  double* d_wtab = nullptr;
  unsigned long long* d_smat = nullptr;
  auto cleanup_fail = [&](hipError_t err, const char* where) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(d_wtab);
    (void)hipFree(d_smat);
    free_plan(pl);
    delete pl;
    (void)hipGetLastError();
    return perr(err == hipErrorOutOfMemory ? TOMO_ENOMEM : TOMO_EDEVICE,
                std::string(where) + ": " + hipGetErrorString(err));
  };
  if ((e = hipMemcpyAsync(pl->d_geom, geo.data(), sizeof(ViewGeom) * r.n, hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(pl->d_prop, prop.data(), sizeof(float2) * prop.size(), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(pl->d_tw_fwd, twf.data(), sizeof(float2) * r.M, hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(pl->d_tw_inv, twi.data(), sizeof(float2) * r.M, hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(pl->d_tw2_fwd, tw2f.data(), sizeof(float2) * hpts, hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(pl->d_tw2_inv, tw2i.data(), sizeof(float2) * hpts, hipMemcpyHostToDevice, s)) ||
      (e = hipMemsetAsync(pl->d_status, 0, sizeof(int), s)))
    return cleanup_fail(e, "upload");

  tomo::FilterArgs fa{};
  fa.n_views = r.n;
  fa.M = r.M;
  fa.N = r.N;
  fa.dx = p->voxel_size;
  fa.lambda = p->wavelength;
  fa.sigma = p->sigma;
  fa.epsilon = p->epsilon;
  fa.eps_sampling = pl->p.eps_sampling;
  fa.ewald = p->ewald;
  fa.mode = p->weight_mode;
  if (p->weight_mode == TOMO_SAMPLING) {
    const size_t n3 = size_t(r.N) * r.N * r.N;
    if ((e = dev_alloc(&d_smat, n3)) != hipSuccess || (e = dev_alloc(&d_wtab, mm * r.n)) != hipSuccess)
      return cleanup_fail(e, "sampling-matrix allocation");
    if ((e = hipMemsetAsync(d_smat, 0, n3 * sizeof(unsigned long long), s)) != hipSuccess)
      return cleanup_fail(e, "sampling-matrix clear");
    if ((e = tomo::launch_sampling(fa, pl->d_geom, d_smat, d_wtab, s)) != hipSuccess)
      return cleanup_fail(e, "sampling-matrix kernels");
  }
  if ((e = tomo::launch_filter_table(fa, pl->d_geom, d_wtab, pl->d_filt, s)) != hipSuccess)
    return cleanup_fail(e, "filter-table kernel");
  if (p->fourier) {
    const size_t n3 = size_t(r.N) * r.N * r.N, p3 = size_t(r.P) * r.P * r.P;
    std::vector<float2> tw3(r.N);
    for (int k = 0; k < r.N; ++k) {
      const double a = 2.0 * kPi * k / r.N;
      tw3[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
    }
    if ((e = dev_alloc(&pl->d_ffilt, mm * r.n)) != hipSuccess || (e = dev_alloc(&pl->d_fview, size_t(r.n))) ||
        (e = dev_alloc(&pl->d_ffix, size_t(2))) || (p->fourier == 2 && (e = dev_alloc(&pl->d_facc, 2 * p3))) ||
        (e = dev_alloc(&pl->d_fsmat, n3)) || (e = dev_alloc(&pl->d_fgrid, n3)) ||
        (e = dev_alloc(&pl->d_tw3, size_t(r.N))))
      return cleanup_fail(e, "Fourier-space workspace allocation");
    if ((e = hipMemcpyAsync(pl->d_tw3, tw3.data(), sizeof(float2) * r.N, hipMemcpyHostToDevice, s)) ||
        (e = hipMemsetAsync(pl->d_fsmat, 0, n3 * sizeof(unsigned long long), s)) ||
        (e = tomo::launch_sampling_splat(fa, pl->d_geom, pl->d_fsmat, s)))
      return cleanup_fail(e, "Fourier-space sampling matrix");
    if (p->fourier == 1) {
      // gridding operator: count, prefix sum on the host, fill, sort
      unsigned* d_count = nullptr;
      auto op_fail = [&](hipError_t err, const char* where) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(d_count);
        return cleanup_fail(err, where);
      };
      if ((e = dev_alloc(&d_count, p3)) || (e = dev_alloc(&pl->d_oprow, p3 + 1)))
        return op_fail(e, "gridding-operator allocation");
      if ((e = hipMemsetAsync(d_count, 0, p3 * sizeof(unsigned), s)) ||
          (e = tomo::launch_fourier_op_count(fa, pl->d_geom, r.P, d_count, s)))
        return op_fail(e, "gridding-operator count");
      std::vector<unsigned> cnt(p3), row(p3 + 1);
      if ((e = hipMemcpyAsync(cnt.data(), d_count, p3 * sizeof(unsigned), hipMemcpyDeviceToHost, s)) ||
          (e = hipStreamSynchronize(s)))
        return op_fail(e, "gridding-operator count read");
      unsigned long long acc = 0;
      for (size_t c = 0; c < p3; ++c) {
        row[c] = unsigned(acc);
        acc += cnt[c];
        if (acc > 0xffffffffull) {
          (void)hipFree(d_count);
          free_plan(pl);
          delete pl;
          return perr(TOMO_EUNSUPPORTED, "gridding operator exceeds 2^32 entries; use fourier = 2");
        }
      }
      row[p3] = unsigned(acc);
      pl->op_entries = size_t(acc);
      if ((e = dev_alloc(&pl->d_opent, std::max<size_t>(pl->op_entries, 1))) ||
          (e = hipMemcpyAsync(pl->d_oprow, row.data(), (p3 + 1) * sizeof(unsigned), hipMemcpyHostToDevice, s)) ||
          (e = hipMemsetAsync(d_count, 0, p3 * sizeof(unsigned), s)) ||
          (e = hipMemsetAsync(pl->d_opent, 0, std::max<size_t>(pl->op_entries, 1) * sizeof(int2), s)) ||
          (e = tomo::launch_fourier_op_fill(fa, pl->d_geom, r.P, pl->d_oprow, d_count, pl->d_opent, s)) ||
          (e = hipStreamSynchronize(s)))
        return op_fail(e, "gridding-operator fill");
      (void)hipFree(d_count);
    }
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return cleanup_fail(e, "plan synchronise");
  (void)hipFree(d_wtab);
  (void)hipFree(d_smat);
  d_wtab = nullptr;
  d_smat = nullptr;
  // general frames: the cubic tiles when asked for, and always when stack rows cannot be
  // fetched as 16-byte chunks (the row-tiled box kernel would gather every view from memory)
  if ((p->tune == 2 || r.M % vec != 0) && !pl->axis_fast) pl->grid_rows = 0;
  if (p->tune >= 3 && !pl->axis_fast && r.M % vec == 0)
    pl->grid_rows = p->tune == 3 ? tomo::kGridTilt4 : p->tune == 4 ? tomo::kGridTilt8 : tomo::kGridTilt2;
  if (p->tune == 5 && pl->axis_fast) pl->grid_rows = 2;
  if (p->tune == 1) {
    // time the gridding variants on a full batch of (zero) stacks and keep the fastest; results
    // do not depend on the choice.  Each timed launch follows a plane-kernel launch that writes
    // the batch's stacks, as in a reconstruction, so that the caches hold what they hold then
    // (timed on idle caches, variants that re-read stack rows look faster than they are).  The
    // timed batch takes views spread evenly over the scan: a variant's speed depends on how
    // many footprints fit its box, which changes along the scan
    float* d_vol = nullptr;
    ViewGeom* d_gs = nullptr;
    hipEvent_t ea = nullptr, eb = nullptr;
    auto tune_fail = [&](hipError_t err) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(d_vol);
      (void)hipFree(d_gs);
      if (ea) (void)hipEventDestroy(ea);
      if (eb) (void)hipEventDestroy(eb);
      return cleanup_fail(err, "gridding autotune");
    };
    const size_t n3 = size_t(r.N) * r.N * r.N;
    std::vector<ViewGeom> gs(r.batch);
    for (int i = 0; i < r.batch; ++i) gs[i] = geo[size_t(i) * r.n / r.batch];
    if ((e = dev_alloc(&d_vol, n3)) || (e = dev_alloc(&d_gs, size_t(r.batch))) ||
        (e = hipMemcpyAsync(d_gs, gs.data(), gs.size() * sizeof(ViewGeom), hipMemcpyHostToDevice, s)) ||
        (e = hipEventCreateWithFlags(&ea, hipEventDisableSystemFence)) ||
        (e = hipEventCreateWithFlags(&eb, hipEventDisableSystemFence)) ||
        (e = hipMemsetAsync(pl->d_q, 0, size_t(r.batch) * mm * sizeof(float4), s)) ||
        (e = hipMemsetAsync(d_vol, 0, n3 * sizeof(float), s)) ||
        (e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(pl->d_scale), 0x3f800000u, size_t(r.n), s)))
      return tune_fail(e);
    float best = 0.0f;
    for (int rows : {8, 4, 2, 0, tomo::kGridTilt8, tomo::kGridTilt4, tomo::kGridTilt2}) {
      // the cubic tiles and the near-axis box serve general frames only, 2 rows per thread
      // (twice the workgroups of 4, for small volumes) single-axis plans only; the row-tiled
      // and near-axis kernels need stack rows of whole 16-byte chunks
      if (rows <= 0 && pl->axis_fast) continue;
      if (rows == 2 && !pl->axis_fast) continue;
      if (rows != 0 && r.M % vec != 0) continue;
      float tot = 0.0f;
      for (int rep = 0; rep < 4; ++rep) {
        if ((e = tomo::launch_planes(r.M, p->plane_dtype, pl->d_q, pl->d_prop, pl->d_tw_inv, pl->d_stack, r.K,
                                     r.npairs, r.batch, pl->d_scale, s, pl->d_tw2_inv)) ||
            (e = hipEventRecord(ea, s)) ||
            (e = tomo::launch_grid(pl->axis_fast, p->plane_dtype, pl->d_stack, d_gs, pl->d_scale, d_vol, r.N,
                                   r.M, r.K, r.batch, 1, p->ewald ? 0 : 1, s, rows)) ||
            (e = hipEventRecord(eb, s)) || (e = hipEventSynchronize(eb)))
          return tune_fail(e);
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, ea, eb))) return tune_fail(e);
        if (rep > 0) tot += ms;   // the first launch warms up
      }
      if (rows == 8 || tot < best) {
        best = tot;
        pl->grid_rows = rows;
      }
    }
    (void)hipFree(d_vol);
    (void)hipFree(d_gs);
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
  }
  // address of this device's allocation-free workspace (looked up again by that call if
  // this fails); the error string gets room for that call's messages
  if (scratch_address(&pl->scratch) != hipSuccess) {
    pl->scratch = nullptr;
    (void)hipGetLastError();
  }
  pl->err.reserve(256);
  *out = pl;
  return TOMO_OK;
}

tomo_status tomo_destroy(tomo_plan_t plan) {
  if (!plan) return TOMO_OK;
  (void)hipDeviceSynchronize();
  free_plan(plan);
  delete plan;
  return TOMO_OK;
}

static tomo_status check_range(tomo_plan_t pl, int32_t first, int32_t nb) {
  if (first < 0 || nb < 0 || first > pl->n || nb > pl->n - first)
    return fail(pl, TOMO_EINVAL, "view range [first, first+nb) outside [0, n_angles)");
  return TOMO_OK;
}

// Spectra of views [first, first+nb) into the plan's per-view slots of d_q.
static tomo_status run_spectra(tomo_plan_t pl, const float* d_images, int32_t first, int32_t nb, hipStream_t s) {
  const size_t mm = size_t(pl->M) * pl->M;
  float* scale = pl->p.plane_dtype == TOMO_F16 ? pl->d_scale + first : nullptr;
  hipError_t e = timed(pl, 0, s, [&] {
    return tomo::launch_spectra(pl->M, d_images, pl->d_filt + size_t(first) * mm, pl->d_tw_fwd,
                                pl->d_q + size_t(first) * mm, pl->d_status, 1.0 / pl->p.i_in, scale, nb, s,
                                pl->d_tw2_fwd, pl->d_l1part + size_t(pl->split * pl->split) * first);
  });
  if (e != hipSuccess) return dev_fail(pl, e, "spectra kernel");
  return TOMO_OK;
}

tomo_status tomo_backpropagate(tomo_plan_t pl, const float* d_images, int32_t first, int32_t nb, void* d_planes,
                               void* stream) {
  if (!pl) return TOMO_EINVAL;
  pl->err.clear();
  if (nb == 0) return TOMO_OK;
  if (!d_images || !d_planes) return fail(pl, TOMO_EINVAL, "null device pointer");
  tomo_status st = check_range(pl, first, nb);
  if (st != TOMO_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = run_spectra(pl, d_images, first, nb, s)) != TOMO_OK) return st;
  const size_t mm = size_t(pl->M) * pl->M;
  hipError_t e = timed(pl, 1, s, [&] {
    return tomo::launch_planes(pl->M, pl->p.plane_dtype, pl->d_q + size_t(first) * mm, pl->d_prop, pl->d_tw_inv,
                               d_planes, pl->K, pl->npairs, nb, pl->d_scale + first, s, pl->d_tw2_inv);
  });
  if (e != hipSuccess) return dev_fail(pl, e, "planes kernel");
  return TOMO_OK;
}

// Message into the plan's reserved error string without growing it.
static tomo_status fail_fixed(tomo_plan_t pl, tomo_status st, const char* a, const char* b = nullptr) {
  pl->err.clear();
  const size_t cap = pl->err.capacity();
  for (const char* part : {a, b}) {
    if (!part) continue;
    const size_t room = cap > pl->err.size() ? cap - pl->err.size() : 0;
    pl->err.append(part, std::min(room, std::strlen(part)));
  }
  return st;
}

tomo_status tomo_backpropagate_noalloc(tomo_plan_t pl, const float* d_images, int32_t first, int32_t nb,
                                       void* d_planes, void* stream) {
  if (!pl) return TOMO_EINVAL;
  pl->err.clear();
  if (nb == 0) return TOMO_OK;
  if (!d_images || !d_planes) return fail_fixed(pl, TOMO_EINVAL, "null device pointer");
  if (first < 0 || nb < 0 || first > pl->n || nb > pl->n - first)
    return fail_fixed(pl, TOMO_EINVAL, "view range [first, first+nb) outside [0, n_angles)");
  if (size_t(nb) * pl->M * pl->M * sizeof(float4) > kScratchBytes)
    return fail_fixed(pl, TOMO_EINVAL,
                      "nb views need more than TOMO_NOALLOC_SCRATCH_BYTES (16 M^2 bytes per view); pass fewer views");
  if (!pl->scratch) {
    const hipError_t e = scratch_address(&pl->scratch);
    if (e != hipSuccess) {
      pl->scratch = nullptr;
      return fail_fixed(pl, TOMO_EDEVICE, "workspace address: ", hipGetErrorString(e));
    }
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t mm = size_t(pl->M) * pl->M;
  float4* q = static_cast<float4*>(pl->scratch);
  float* scale = pl->p.plane_dtype == TOMO_F16 ? pl->d_scale + first : nullptr;
  hipError_t e = tomo::launch_spectra(pl->M, d_images, pl->d_filt + size_t(first) * mm, pl->d_tw_fwd, q,
                                      pl->d_status, 1.0 / pl->p.i_in, scale, nb, s, pl->d_tw2_fwd,
                                      pl->d_l1part + size_t(pl->split * pl->split) * first);
  if (e != hipSuccess) return fail_fixed(pl, TOMO_EDEVICE, "spectra kernel: ", hipGetErrorString(e));
  e = tomo::launch_planes(pl->M, pl->p.plane_dtype, q, pl->d_prop, pl->d_tw_inv, d_planes, pl->K, pl->npairs, nb,
                          pl->d_scale + first, s, pl->d_tw2_inv);
  if (e != hipSuccess) return fail_fixed(pl, TOMO_EDEVICE, "planes kernel: ", hipGetErrorString(e));
  return TOMO_OK;
}

tomo_status tomo_grid(tomo_plan_t pl, const void* d_planes, int32_t first, int32_t nb, float* d_volume,
                      void* stream) {
  if (!pl) return TOMO_EINVAL;
  pl->err.clear();
  if (nb == 0) return TOMO_OK;
  if (!d_planes || !d_volume) return fail(pl, TOMO_EINVAL, "null device pointer");
  if (first < 0 || nb < 0 || first > pl->n || nb > pl->n - first)
    return fail(pl, TOMO_EINVAL, "view range [first, first+nb) outside [0, n_angles)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = timed(pl, 2, s, [&] {
    return tomo::launch_grid(pl->axis_fast, pl->p.plane_dtype, d_planes, pl->d_geom + first, pl->d_scale + first,
                             d_volume, pl->N, pl->M, pl->K, nb, 1, pl->p.ewald ? 0 : 1, s,
                             pl->grid_rows);
  });
  if (e != hipSuccess) return dev_fail(pl, e, "grid kernel");
  return TOMO_OK;
}

tomo_status tomo_sync(tomo_plan_t pl, void* stream) {
  if (!pl) return TOMO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(pl, e, "synchronise");
  int flag = 0;
  if ((e = hipMemcpy(&flag, pl->d_status, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return dev_fail(pl, e, "status read");
  if (flag) {
    const int zero = 0;
    if ((e = hipMemcpy(pl->d_status, &zero, sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
      return dev_fail(pl, e, "status reset");
    return fail(pl, TOMO_EDOMAIN, "an image value was <= 0 or not finite");
  }
  return TOMO_OK;
}

// Every kernel of one reconstruction, enqueued on s (no synchronisation).
static tomo_status enqueue_reconstruct(tomo_plan_t pl, const float* d_images, float* d_volume, hipStream_t s) {
  const size_t mm = size_t(pl->M) * pl->M;
  // spectra of all views in one launch (one workgroup per view), then per batch the
  // depth planes and the gridding
  tomo_status st = run_spectra(pl, d_images, 0, pl->n, s);
  if (st != TOMO_OK) return st;
  for (int first = 0; first < pl->n; first += pl->batch) {
    const int nb = std::min(pl->batch, pl->n - first);
    hipError_t e = timed(pl, 1, s, [&] {
      return tomo::launch_planes(pl->M, pl->p.plane_dtype, pl->d_q + size_t(first) * mm, pl->d_prop,
                                 pl->d_tw_inv, pl->d_stack, pl->K, pl->npairs, nb, pl->d_scale + first, s,
                                 pl->d_tw2_inv);
    });
    if (e != hipSuccess) return dev_fail(pl, e, "planes kernel");
    e = timed(pl, 2, s, [&] {
      return tomo::launch_grid(pl->axis_fast, pl->p.plane_dtype, pl->d_stack, pl->d_geom + first,
                               pl->d_scale + first, d_volume, pl->N, pl->M, pl->K, nb, first > 0 ? 1 : 0,
                               pl->p.ewald ? 0 : 1, s, pl->grid_rows);
    });
    if (e != hipSuccess) return dev_fail(pl, e, "grid kernel");
  }
  return TOMO_OK;
}

tomo_status tomo_reconstruct(tomo_plan_t pl, const float* d_images, float* d_volume, void* stream) {
  if (!pl) return TOMO_EINVAL;
  pl->err.clear();
  if (!d_images || !d_volume) return fail(pl, TOMO_EINVAL, "null device pointer");
  tomo_status st = enqueue_reconstruct(pl, d_images, d_volume, static_cast<hipStream_t>(stream));
  if (st != TOMO_OK) return st;
  return tomo_sync(pl, stream);
}

tomo_status tomo_reconstruct_async(tomo_plan_t pl, const float* d_images, float* d_volume, void* stream) {
  if (!pl) return TOMO_EINVAL;
  pl->err.clear();
  if (!d_images || !d_volume) return fail(pl, TOMO_EINVAL, "null device pointer");
  return enqueue_reconstruct(pl, d_images, d_volume, static_cast<hipStream_t>(stream));
}

tomo_status tomo_timing_enable(tomo_plan_t pl, int32_t enable) {
  if (!pl) return TOMO_EINVAL;
  pl->timing = enable != 0;
  return TOMO_OK;
}

tomo_status tomo_timing_read(tomo_plan_t pl, double* total_ms, int64_t* launches, int32_t reset) {
  if (!pl || !total_ms || !launches) return TOMO_EINVAL;
  for (auto& r : pl->recs) {
    float ms = 0;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return dev_fail(pl, e, "timing events");
    pl->tot_ms[r.kind] += ms;
    pl->launches[r.kind] += 1;
    pl->pool.push_back(r.a);
    pl->pool.push_back(r.b);
  }
  pl->recs.clear();
  for (int k = 0; k < TOMO_TIMING_KINDS; ++k) {
    total_ms[k] = pl->tot_ms[k];
    launches[k] = pl->launches[k];
    if (reset) {
      pl->tot_ms[k] = 0;
      pl->launches[k] = 0;
    }
  }
  return TOMO_OK;
}

tomo_status tomo_filtered_spectra(tomo_plan_t pl, const float* d_images, int32_t first, int32_t nb, float* d_out,
                                  void* stream) {
  if (!pl) return TOMO_EINVAL;
  pl->err.clear();
  if (nb == 0) return TOMO_OK;
  if (!d_images || !d_out) return fail(pl, TOMO_EINVAL, "null device pointer");
  tomo_status st = check_range(pl, first, nb);
  if (st != TOMO_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = run_spectra(pl, d_images, first, nb, s)) != TOMO_OK) return st;
  hipError_t e = tomo::launch_spectra_out(pl->d_q + size_t(first) * size_t(pl->M) * pl->M,
                                          reinterpret_cast<float2*>(d_out), pl->M, nb, s);
  if (e != hipSuccess) return dev_fail(pl, e, "spectra output kernel");
  return TOMO_OK;
}

// Every kernel of one Fourier-space reconstruction, enqueued on the stream (no synchronisation).
static tomo_status enqueue_fourier(tomo_plan_t pl, const float* d_images, int32_t variant, double nsr,
                                   float* d_volume, void* stream) {
  if (!pl) return TOMO_EINVAL;
  pl->err.clear();
  if (!d_images || !d_volume) return fail(pl, TOMO_EINVAL, "null device pointer");
  if (!pl->p.fourier) return fail(pl, TOMO_EINVAL, "plan was made with fourier = 0");
  if (variant != TOMO_EQ11 && variant != TOMO_EQ12) return fail(pl, TOMO_EINVAL, "variant must be 11 or 12");
  if (!(nsr >= 0) || !std::isfinite(nsr)) return fail(pl, TOMO_EINVAL, "nsr must be finite and >= 0");
  if (variant == TOMO_EQ12 && !pl->same_R)
    return fail(pl, TOMO_EINVAL, "eq. 12 needs one common distance R for every view");
  hipStream_t s = static_cast<hipStream_t>(stream);
  tomo::FilterArgs fa{};
  fa.n_views = pl->n;
  fa.M = pl->M;
  fa.N = pl->N;
  fa.dx = pl->p.voxel_size;
  fa.lambda = pl->p.wavelength;
  fa.sigma = pl->p.sigma;
  fa.epsilon = pl->p.epsilon;
  fa.eps_sampling = pl->p.eps_sampling;
  fa.ewald = pl->p.ewald;
  fa.mode = pl->p.weight_mode;
  hipError_t e = hipSuccess;
  if (pl->ffilt_variant != variant) {
    if ((e = tomo::launch_fourier_filter(fa, pl->d_geom, variant == TOMO_EQ12, pl->d_ffilt, s)) != hipSuccess)
      return dev_fail(pl, e, "Fourier filter table");
    pl->ffilt_variant = variant;
  }
  e = timed(pl, 0, s, [&] {
    return tomo::launch_spectra(pl->M, d_images, pl->d_ffilt, pl->d_tw_fwd, pl->d_q, pl->d_status,
                                1.0 / pl->p.i_in, pl->d_fview, pl->n, s, pl->d_tw2_fwd, pl->d_l1part);
  });
  if (e != hipSuccess) return dev_fail(pl, e, "spectra kernel");
  tomo::FourierNormArgs na{};
  na.N = pl->N;
  na.P = pl->P;
  na.eq12 = variant == TOMO_EQ12;
  na.ewald = pl->p.ewald;
  na.eps_s = pl->p.eps_sampling;
  na.nsr_m = nsr * pl->M;
  const double cst = pl->p.wavelength / (4.0 * kPi * std::sqrt(1.0 + pl->p.sigma * pl->p.sigma));
  const double nd = pl->N * pl->p.voxel_size;
  na.out_scale = cst * pl->p.voxel_size * pl->p.voxel_size / (nd * nd * nd);
  na.dx = pl->p.voxel_size;
  na.lambda = pl->p.wavelength;
  na.sigma = pl->p.sigma;
  na.epsilon = pl->p.epsilon;
  na.R = pl->R0;
  if (pl->p.fourier == 1) {
    e = timed(pl, 3, s, [&] {
      return tomo::launch_fourier_gather(na, pl->d_oprow, pl->d_opent, pl->d_q, pl->d_fsmat, pl->d_fgrid, s);
    });
    if (e != hipSuccess) return dev_fail(pl, e, "Fourier gridding-operator kernel");
  } else {
    e = timed(pl, 3, s, [&] {
      return tomo::launch_fourier_splat(fa, pl->d_geom, pl->d_q, pl->d_fview, pl->d_ffix, pl->d_facc, pl->P, s);
    });
    if (e != hipSuccess) return dev_fail(pl, e, "Fourier splat kernels");
    e = timed(pl, 4, s, [&] {
      return tomo::launch_fourier_norm(na, pl->d_facc, pl->d_fsmat, pl->d_ffix, pl->d_fgrid, s);
    });
    if (e != hipSuccess) return dev_fail(pl, e, "Fourier normalise kernel");
  }
  e = timed(pl, 4, s, [&] { return tomo::launch_fourier_fft3(pl->N, pl->d_fgrid, pl->d_tw3, d_volume, s); });
  if (e != hipSuccess) return dev_fail(pl, e, "Fourier inverse FFT kernels");
  return TOMO_OK;
}

tomo_status tomo_fourier_reconstruct(tomo_plan_t pl, const float* d_images, int32_t variant, double nsr,
                                     float* d_volume, void* stream) {
  const tomo_status st = enqueue_fourier(pl, d_images, variant, nsr, d_volume, stream);
  if (st != TOMO_OK) return st;
  return tomo_sync(pl, stream);
}

tomo_status tomo_fourier_reconstruct_async(tomo_plan_t pl, const float* d_images, int32_t variant, double nsr,
                                           float* d_volume, void* stream) {
  return enqueue_fourier(pl, d_images, variant, nsr, d_volume, stream);
}

// ---------------------------------------------------------------- batched jobs
struct tomo_batch_s {
  std::vector<tomo_plan_t> plans;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string err;
};

tomo_status tomo_batch_create(const tomo_plan_t* plans, const float* const* d_images, float* const* d_volumes,
                              int32_t count, int32_t lanes, tomo_batch_t* out) {
  g_plan_error.clear();
  auto perr = [](tomo_status st, const std::string& m) {
    g_plan_error = m;
    return st;
  };
  if (!out || !plans || !d_images || !d_volumes) return perr(TOMO_EINVAL, "null argument");
  if (count < 1) return perr(TOMO_EINVAL, "count must be >= 1");
  if (lanes < 0) return perr(TOMO_EINVAL, "lanes must be >= 0");
  for (int j = 0; j < count; ++j) {
    if (!plans[j] || !d_images[j] || !d_volumes[j]) return perr(TOMO_EINVAL, "null plan or buffer in the job list");
    for (int k = 0; k < j; ++k)
      if (plans[k] == plans[j]) return perr(TOMO_EINVAL, "a plan appears twice (jobs need their own workspace)");
  }
  const int L = std::min<int>(count, lanes > 0 ? lanes : 8);
  // longest job first onto the least loaded lane (work = N^3 n voxel-angle updates)
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  auto work = [&](int j) { return double(plans[j]->N) * plans[j]->N * plans[j]->N * plans[j]->n; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  std::vector<double> load(L, 0.0);
  std::vector<std::vector<int>> lane_jobs(L);
  for (int j : order) {
    const int l = int(std::min_element(load.begin(), load.end()) - load.begin());
    load[l] += work(j);
    lane_jobs[l].push_back(j);
  }
  hipStream_t s = nullptr;   // recording stream of the batch's own (the null stream cannot be captured)
  std::vector<hipStream_t> ls(L, nullptr);
  std::vector<hipEvent_t> join(L, nullptr);
  hipEvent_t fork = nullptr;
  std::vector<bool> timing(count);
  auto cleanup = [&]() {
    if (s) (void)hipStreamDestroy(s);
    for (auto& x : ls)
      if (x) (void)hipStreamDestroy(x);
    for (auto& x : join)
      if (x) (void)hipEventDestroy(x);
    if (fork) (void)hipEventDestroy(fork);
    for (int j = 0; j < count; ++j) plans[j]->timing = timing[j];
  };
  for (int j = 0; j < count; ++j) {
    timing[j] = plans[j]->timing;
    plans[j]->timing = false;   // no event nodes in the graph
  }
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    e = hipStreamCreateWithFlags(&ls[l], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join[l], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    cleanup();
    return perr(TOMO_EDEVICE, std::string("batch set-up: ") + hipGetErrorString(e));
  }
  hipGraph_t graph = nullptr;
  if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    cleanup();
    return perr(TOMO_EDEVICE, std::string("begin capture: ") + hipGetErrorString(e));
  }
  tomo_status st = TOMO_OK;
  e = hipEventRecord(fork, s);
  for (int l = 0; l < L && e == hipSuccess && st == TOMO_OK; ++l) {
    e = hipStreamWaitEvent(ls[l], fork, 0);
    for (size_t k = 0; k < lane_jobs[l].size() && e == hipSuccess && st == TOMO_OK; ++k) {
      const int j = lane_jobs[l][k];
      st = enqueue_reconstruct(plans[j], d_images[j], d_volumes[j], ls[l]);
    }
    if (e == hipSuccess && st == TOMO_OK) e = hipEventRecord(join[l], ls[l]);
    if (e == hipSuccess && st == TOMO_OK) e = hipStreamWaitEvent(s, join[l], 0);
  }
  const hipError_t ec = hipStreamEndCapture(s, &graph);
  if (e == hipSuccess) e = ec;
  if (st != TOMO_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    cleanup();
    (void)hipGetLastError();
    return perr(st != TOMO_OK ? st : TOMO_EDEVICE,
                st != TOMO_OK ? std::string("job recording failed") : std::string("capture: ") + hipGetErrorString(e));
  }
  hipGraphExec_t exec = nullptr;
  if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    cleanup();
    return perr(TOMO_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  cleanup();
  auto* b = new tomo_batch_s();
  b->plans.assign(plans, plans + count);
  b->graph = graph;
  b->exec = exec;
  *out = b;
  return TOMO_OK;
}

tomo_status tomo_batch_launch(tomo_batch_t b, void* stream) {
  if (!b) return TOMO_EINVAL;
  b->err.clear();
  hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    b->err = std::string("graph launch: ") + hipGetErrorString(e);
    return TOMO_EDEVICE;
  }
  return TOMO_OK;
}

tomo_status tomo_batch_sync(tomo_batch_t b, void* stream) {
  if (!b) return TOMO_EINVAL;
  b->err.clear();
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    b->err = std::string("synchronise: ") + hipGetErrorString(e);
    return TOMO_EDEVICE;
  }
  int first_bad = -1;
  for (size_t j = 0; j < b->plans.size(); ++j) {
    const tomo_status st = tomo_sync(b->plans[j], nullptr);
    if (st == TOMO_EDOMAIN && first_bad < 0) first_bad = int(j);
    if (st != TOMO_OK && st != TOMO_EDOMAIN) {
      b->err = "job " + std::to_string(j) + ": " + b->plans[j]->err;
      return st;
    }
  }
  if (first_bad >= 0) {
    b->err = "job " + std::to_string(first_bad) + ": an image value was <= 0 or not finite";
    return TOMO_EDOMAIN;
  }
  return TOMO_OK;
}

const char* tomo_batch_error(tomo_batch_t b) { return b ? b->err.c_str() : "batch is NULL"; }

tomo_status tomo_batch_destroy(tomo_batch_t b) {
  if (!b) return TOMO_OK;
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return TOMO_OK;
}

}  // extern "C"

// C-ABI host side of the artefact-correction network: parameter layout, workspace,
// and the order of the forward, backward and optimiser kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "tomo_unet.h"
#include "unet_internal.hpp"

namespace {

struct Layer {
  int cin, cout, ks;
};
// e1a e1b e2a e2b b_a b_b d2a d2b d1a d1b out
const Layer kLayers[] = {{1, 16, 3},  {16, 16, 3}, {16, 32, 3}, {32, 32, 3}, {32, 64, 3}, {64, 64, 3},
                         {96, 32, 3}, {32, 32, 3}, {48, 16, 3}, {16, 16, 3}, {16, 1, 1}};
constexpr int kNL = 11;
enum { E1A, E1B, E2A, E2B, BA, BB, D2A, D2B, D1A, D1B, OUT };

int weights_of(int l) { return kLayers[l].cout * kLayers[l].cin * kLayers[l].ks * kLayers[l].ks * kLayers[l].ks; }

// offsets of each layer's weights (bias follows them)
std::vector<int> offsets() {
  std::vector<int> off(kNL + 1, 0);
  for (int l = 0; l < kNL; ++l) off[l + 1] = off[l] + weights_of(l) + kLayers[l].cout;
  return off;
}

thread_local std::string g_err;

}  // namespace

struct tomo_unet_s {
  int n = 0;
  size_t v1 = 0, v2 = 0, v3 = 0;
  std::vector<int> off;
  float *e1a = nullptr, *c1 = nullptr, *p1 = nullptr, *e2a = nullptr, *c2 = nullptr, *p2 = nullptr;
  float *ba = nullptr, *bb = nullptr, *d2a = nullptr, *d2b = nullptr, *d1a = nullptr, *d1b = nullptr;
  float *y = nullptr, *gy = nullptr;
  float *g_d1b = nullptr, *g_d1a = nullptr, *g_c1 = nullptr, *g_d2b = nullptr, *g_d2a = nullptr, *g_c2 = nullptr;
  float *g_bb = nullptr, *g_ba = nullptr, *g_p2 = nullptr, *g_e2b = nullptr, *g_e2a = nullptr, *g_p1 = nullptr;
  float *g_e1b = nullptr, *g_e1a = nullptr;
  __hip_bfloat16* wbf = nullptr;
  unsigned short *wf = nullptr, *wd = nullptr;   // matrix-core weight layouts (same offsets as wbf)
  float *pw = nullptr, *pb = nullptr, *q = nullptr;
  double* part = nullptr;
  std::vector<void*> allocs;
  std::string err;
};

namespace {

template <class T>
hipError_t grab(tomo_unet_s* u, T** p, size_t count) {
  *p = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) u->allocs.push_back(*p);
  return e;
}

void release(tomo_unet_s* u) {
  for (void* p : u->allocs) (void)hipFree(p);
  u->allocs.clear();
}

tomo_status fail(tomo_unet_s* u, hipError_t e, const char* where) {
  u->err = std::string(where) + ": " + hipGetErrorString(e);
  return TOMO_EDEVICE;
}

const __hip_bfloat16* W(const tomo_unet_s* u, int l) { return u->wbf + u->off[l]; }
bool has_layout(int l) {
  const Layer& L = kLayers[l];
  return unet::mfma_layer(L.ks, L.cin, L.cout) && L.cin % 16 == 0;
}
const unsigned short* WF(const tomo_unet_s* u, int l) { return has_layout(l) ? u->wf + u->off[l] : nullptr; }
const unsigned short* WD(const tomo_unet_s* u, int l) { return has_layout(l) ? u->wd + u->off[l] : nullptr; }
const float* B(const tomo_unet_s* u, const float* th, int l) { return th + u->off[l] + weights_of(l); }

// Activations are channel-last (a voxel's channels contiguous).  The two concatenations are
// buffers of 48 (level 1) and 96 (level 2) channels: the upsampled decoder features fill the
// first 32 / 64 channels, and the encoder writes its output straight into the rest.
hipError_t forward(tomo_unet_s* u, const float* th, const float* x, float* y, hipStream_t s) {
  const int n = u->n, h = n / 2, q = n / 4;
  hipError_t e;
  const int P = u->off[kNL];
  if ((e = unet::round_bf16(th, u->wbf, P, s))) return e;
  for (int l = 0; l < kNL; ++l)
    if (has_layout(l) &&
        (e = unet::weight_layout(W(u, l), kLayers[l].cout, kLayers[l].cin, u->wf + u->off[l], u->wd + u->off[l], s)))
      return e;
  float* e1b = u->c1 + 32;   // channels 32..47 of the level-1 concatenation
  float* e2b = u->c2 + 64;   // channels 64..95 of the level-2 concatenation
  if ((e = unet::conv_fwd(3, x, 1, 1, W(u, E1A), WF(u, E1A), B(u, th, E1A), u->e1a, 16, 16, n, 1, nullptr, s))) return e;
  if ((e = unet::conv_fwd(3, u->e1a, 16, 16, W(u, E1B), WF(u, E1B), B(u, th, E1B), e1b, 48, 16, n, 1, nullptr, s))) return e;
  if ((e = unet::pool2(e1b, 48, u->p1, 16, 16, n, s))) return e;
  if ((e = unet::conv_fwd(3, u->p1, 16, 16, W(u, E2A), WF(u, E2A), B(u, th, E2A), u->e2a, 32, 32, h, 1, nullptr, s))) return e;
  if ((e = unet::conv_fwd(3, u->e2a, 32, 32, W(u, E2B), WF(u, E2B), B(u, th, E2B), e2b, 96, 32, h, 1, nullptr, s))) return e;
  if ((e = unet::pool2(e2b, 96, u->p2, 32, 32, h, s))) return e;
  if ((e = unet::conv_fwd(3, u->p2, 32, 32, W(u, BA), WF(u, BA), B(u, th, BA), u->ba, 64, 64, q, 1, nullptr, s))) return e;
  if ((e = unet::conv_fwd(3, u->ba, 64, 64, W(u, BB), WF(u, BB), B(u, th, BB), u->bb, 64, 64, q, 1, nullptr, s))) return e;
  if ((e = unet::up2(u->bb, 64, u->c2, 96, 64, h, s))) return e;
  if ((e = unet::conv_fwd(3, u->c2, 96, 96, W(u, D2A), WF(u, D2A), B(u, th, D2A), u->d2a, 32, 32, h, 1, nullptr, s))) return e;
  if ((e = unet::conv_fwd(3, u->d2a, 32, 32, W(u, D2B), WF(u, D2B), B(u, th, D2B), u->d2b, 32, 32, h, 1, nullptr, s))) return e;
  if ((e = unet::up2(u->d2b, 32, u->c1, 48, 32, n, s))) return e;
  if ((e = unet::conv_fwd(3, u->c1, 48, 48, W(u, D1A), WF(u, D1A), B(u, th, D1A), u->d1a, 16, 16, n, 1, nullptr, s))) return e;
  if ((e = unet::conv_fwd(3, u->d1a, 16, 16, W(u, D1B), WF(u, D1B), B(u, th, D1B), u->d1b, 16, 16, n, 1, nullptr, s))) return e;
  return unet::conv_fwd(1, u->d1b, 16, 16, W(u, OUT), WF(u, OUT), B(u, th, OUT), y, 1, 1, n, 0, x, s);
}

// weight + bias gradient of layer l into grad, and (optionally) its input gradient; every
// tensor is a view (pointer, channel count of its buffer)
hipError_t layer_back(tomo_unet_s* u, int l, const float* in, int sin, const float* g, int sg, const float* yout,
                      int sy, int n, float* grad, float* gx, int sgx, hipStream_t s) {
  const Layer& L = kLayers[l];
  hipError_t e = unet::conv_bwd_w(L.ks, in, sin, L.cin, g, sg, yout, sy, L.cout, n, u->pw, u->pb, u->q,
                                  grad + u->off[l], grad + u->off[l] + weights_of(l), s);
  if (e != hipSuccess || !gx) return e;
  return unet::conv_bwd_data(L.ks, g, sg, yout, sy, L.cout, W(u, l), WD(u, l), gx, sgx, L.cin, n, s);
}

hipError_t backward(tomo_unet_s* u, const float* x, float* grad, hipStream_t s) {
  const int n = u->n, h = n / 2, q = n / 4;
  float* e1b = u->c1 + 32;
  float* e2b = u->c2 + 64;
  hipError_t e;
  if ((e = layer_back(u, OUT, u->d1b, 16, u->gy, 1, nullptr, 0, n, grad, u->g_d1b, 16, s))) return e;
  if ((e = layer_back(u, D1B, u->d1a, 16, u->g_d1b, 16, u->d1b, 16, n, grad, u->g_d1a, 16, s))) return e;
  if ((e = layer_back(u, D1A, u->c1, 48, u->g_d1a, 16, u->d1a, 16, n, grad, u->g_c1, 48, s))) return e;
  if ((e = unet::up2_bwd(u->g_c1, 48, u->g_d2b, 32, 32, n, s))) return e;
  if ((e = layer_back(u, D2B, u->d2a, 32, u->g_d2b, 32, u->d2b, 32, h, grad, u->g_d2a, 32, s))) return e;
  if ((e = layer_back(u, D2A, u->c2, 96, u->g_d2a, 32, u->d2a, 32, h, grad, u->g_c2, 96, s))) return e;
  if ((e = unet::up2_bwd(u->g_c2, 96, u->g_bb, 64, 64, h, s))) return e;
  if ((e = layer_back(u, BB, u->ba, 64, u->g_bb, 64, u->bb, 64, q, grad, u->g_ba, 64, s))) return e;
  if ((e = layer_back(u, BA, u->p2, 32, u->g_ba, 64, u->ba, 64, q, grad, u->g_p2, 32, s))) return e;
  if ((e = unet::pool2_bwd_add(u->g_p2, 32, u->g_c2 + 64, 96, u->g_e2b, 32, 32, h, s))) return e;
  if ((e = layer_back(u, E2B, u->e2a, 32, u->g_e2b, 32, e2b, 96, h, grad, u->g_e2a, 32, s))) return e;
  if ((e = layer_back(u, E2A, u->p1, 16, u->g_e2a, 32, u->e2a, 32, h, grad, u->g_p1, 16, s))) return e;
  if ((e = unet::pool2_bwd_add(u->g_p1, 16, u->g_c1 + 32, 48, u->g_e1b, 16, 16, n, s))) return e;
  if ((e = layer_back(u, E1B, u->e1a, 16, u->g_e1b, 16, e1b, 48, n, grad, u->g_e1a, 16, s))) return e;
  return layer_back(u, E1A, x, 1, u->g_e1a, 16, u->e1a, 16, n, grad, nullptr, 0, s);
}

}  // namespace

extern "C" {

int32_t tomo_unet_param_count(void) { return offsets()[kNL]; }

tomo_status tomo_unet_create(int32_t n, tomo_unet_t* out) {
  g_err.clear();
  if (!out) {
    g_err = "out is NULL";
    return TOMO_EINVAL;
  }
  if (n < 8 || n > 256 || n % 4 != 0) {
    g_err = "n must be a multiple of 4 in [8, 256]";
    return TOMO_EINVAL;
  }
  auto* u = new tomo_unet_s();
  u->n = n;
  u->v1 = size_t(n) * n * n;
  u->v2 = u->v1 / 8;
  u->v3 = u->v2 / 8;
  u->off = offsets();
  // weight-gradient workspace: the largest any layer needs at its level's edge
  size_t max_pw = 0, max_pb = 0, max_q = 0;
  const int level_n[kNL] = {n, n, n / 2, n / 2, n / 4, n / 4, n / 2, n / 2, n, n, n};
  for (int l = 0; l < kNL; ++l) {
    size_t a, b, c;
    unet::wgrad_workspace(kLayers[l].ks, kLayers[l].cin, kLayers[l].cout, level_n[l], a, b, c);
    max_pw = std::max(max_pw, a);
    max_pb = std::max(max_pb, b);
    max_q = std::max(max_q, c);
  }
  const size_t v1 = u->v1, v2 = u->v2, v3 = u->v3;
  hipError_t e;
  if ((e = grab(u, &u->e1a, 16 * v1)) || (e = grab(u, &u->c1, 48 * v1)) || (e = grab(u, &u->p1, 16 * v2)) ||
      (e = grab(u, &u->e2a, 32 * v2)) || (e = grab(u, &u->c2, 96 * v2)) || (e = grab(u, &u->p2, 32 * v3)) ||
      (e = grab(u, &u->ba, 64 * v3)) || (e = grab(u, &u->bb, 64 * v3)) || (e = grab(u, &u->d2a, 32 * v2)) ||
      (e = grab(u, &u->d2b, 32 * v2)) || (e = grab(u, &u->d1a, 16 * v1)) || (e = grab(u, &u->d1b, 16 * v1)) ||
      (e = grab(u, &u->y, v1)) || (e = grab(u, &u->gy, v1)) || (e = grab(u, &u->g_d1b, 16 * v1)) ||
      (e = grab(u, &u->g_d1a, 16 * v1)) || (e = grab(u, &u->g_c1, 48 * v1)) || (e = grab(u, &u->g_d2b, 32 * v2)) ||
      (e = grab(u, &u->g_d2a, 32 * v2)) || (e = grab(u, &u->g_c2, 96 * v2)) || (e = grab(u, &u->g_bb, 64 * v3)) ||
      (e = grab(u, &u->g_ba, 64 * v3)) || (e = grab(u, &u->g_p2, 32 * v3)) || (e = grab(u, &u->g_e2b, 32 * v2)) ||
      (e = grab(u, &u->g_e2a, 32 * v2)) || (e = grab(u, &u->g_p1, 16 * v2)) || (e = grab(u, &u->g_e1b, 16 * v1)) ||
      (e = grab(u, &u->g_e1a, 16 * v1)) || (e = grab(u, &u->wbf, size_t(u->off[kNL]))) ||
      (e = grab(u, &u->wf, size_t(u->off[kNL]))) || (e = grab(u, &u->wd, size_t(u->off[kNL]))) ||
      (e = grab(u, &u->pw, max_pw)) || (e = grab(u, &u->pb, max_pb)) || (e = grab(u, &u->q, max_q)) ||
      (e = grab(u, &u->part, (v1 + 255) / 256))) {
    release(u);
    delete u;
    (void)hipGetLastError();
    g_err = std::string("allocation failed: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? TOMO_ENOMEM : TOMO_EDEVICE;
  }
  *out = u;
  return TOMO_OK;
}

tomo_status tomo_unet_forward(tomo_unet_t u, const float* d_params, const float* d_x, float* d_y, void* stream) {
  if (!u) return TOMO_EINVAL;
  u->err.clear();
  if (!d_params || !d_x || !d_y) {
    u->err = "null device pointer";
    return TOMO_EINVAL;
  }
  hipError_t e = forward(u, d_params, d_x, d_y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TOMO_OK : fail(u, e, "forward kernels");
}

tomo_status tomo_unet_gradient(tomo_unet_t u, const float* d_params, const float* d_x, const float* d_target,
                               float* d_grad, double* d_loss, void* stream) {
  if (!u) return TOMO_EINVAL;
  u->err.clear();
  if (!d_params || !d_x || !d_target || !d_grad || !d_loss) {
    u->err = "null device pointer";
    return TOMO_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = forward(u, d_params, d_x, u->y, s);
  if (e == hipSuccess) e = unet::mse(u->y, d_target, u->gy, u->part, d_loss, u->v1, s);
  if (e == hipSuccess) e = backward(u, d_x, d_grad, s);
  return e == hipSuccess ? TOMO_OK : fail(u, e, "gradient kernels");
}

tomo_status tomo_unet_adam(tomo_unet_t u, float* d_params, const float* d_grad, float* d_m, float* d_v, int32_t step,
                           float lr, float beta1, float beta2, float eps, void* stream) {
  if (!u) return TOMO_EINVAL;
  u->err.clear();
  if (!d_params || !d_grad || !d_m || !d_v) {
    u->err = "null device pointer";
    return TOMO_EINVAL;
  }
  if (step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0)) {
    u->err = "need step >= 1, lr > 0, 0 <= beta < 1, eps >= 0";
    return TOMO_EINVAL;
  }
  const float c1 = float(1.0 - std::pow(double(beta1), step)), c2 = float(1.0 - std::pow(double(beta2), step));
  hipError_t e = unet::adam(d_params, d_grad, d_m, d_v, u->off[kNL], lr, beta1, beta2, eps, c1, c2,
                            static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TOMO_OK : fail(u, e, "adam kernel");
}

const char* tomo_unet_error(tomo_unet_t u) { return u ? u->err.c_str() : g_err.c_str(); }

tomo_status tomo_unet_destroy(tomo_unet_t u) {
  if (!u) return TOMO_OK;
  (void)hipDeviceSynchronize();
  release(u);
  delete u;
  return TOMO_OK;
}

}  // extern "C"

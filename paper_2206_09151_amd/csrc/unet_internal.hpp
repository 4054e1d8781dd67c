// Internal interface between the network's C-ABI host code and its gfx950 kernels.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cstddef>

namespace unet {

// out[co] = act(b + conv_ks(in)) (+ res), input channels [0, c0) from x0 and [c0, cin) from x1.
hipError_t conv_fwd(int ks, const float* x0, int c0, const float* x1, int cin, const __hip_bfloat16* w,
                    const float* b, float* out, int cout, int n, int relu, const float* res, hipStream_t s);
// Input gradient of a conv layer; g masked by (y > 0) unless y is null; channels [0, c0) into gx0.
hipError_t conv_bwd_data(int ks, const float* g, const float* y, int cout, const __hip_bfloat16* w, float* gx0,
                         int c0, float* gx1, int cin, int n, hipStream_t s);
// Weight and bias gradients (fixed-order chunk partials pw / pb, then their sums into gw / gb).
hipError_t conv_bwd_w(int ks, const float* x0, int c0, const float* x1, int cin, const float* g, const float* y,
                      int cout, int n, float* pw, float* pb, float* gw, float* gb, hipStream_t s);
int weight_grad_chunks(int n);
hipError_t pool2(const float* x, float* y, int c, int n, hipStream_t s);
hipError_t up2(const float* x, float* y, int c, int n, hipStream_t s);
hipError_t up2_bwd(const float* g, float* gx, int c, int n, hipStream_t s);
hipError_t pool2_bwd_add(const float* g, const float* add, float* gx, int c, int n, hipStream_t s);
hipError_t mse(const float* y, const float* tg, float* gy, double* part, double* loss, size_t count, hipStream_t s);
hipError_t adam(float* th, const float* g, float* m, float* v, int count, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s);
hipError_t round_bf16(const float* th, __hip_bfloat16* w, int count, hipStream_t s);

}  // namespace unet

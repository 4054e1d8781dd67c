// Internal interface between the network's C-ABI host code and its gfx950 kernels.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cstddef>

namespace unet {

// Volumes are channel-last: element (v, c) of a view (p, s) is p[v * s + c], v = (z n + y) n + x,
// s the channel count of the underlying buffer (a multiple of 16 for multi-channel views).
//
// Whether a layer runs on the matrix-core kernels (3x3x3, cout in {16, 32, 64}, cin a
// multiple of 16 up to 96, or cin == 1 for the weight gradient).
bool mfma_layer(int ks, int cin, int cout);
// BF16 weight layouts of a matrix-core layer (cin and cout multiples of 16): wf for the
// forward, wd (taps reversed) for the input gradient; each holds cout * cin * 27 values.
hipError_t weight_layout(const __hip_bfloat16* w, int cout, int cin, unsigned short* wf, unsigned short* wd,
                         hipStream_t s);
// out = act(b + conv_ks(x)) (+ res) for the network's layers: 3x3x3 with one input channel
// (the first layer), 3x3x3 on the matrix cores (wf, the forward layout), or the 1x1 output
// layer (cout = 1, res added); hipErrorInvalidValue for anything else.
hipError_t conv_fwd(int ks, const float* x, int sx, int cin, const __hip_bfloat16* w, const unsigned short* wf,
                    const float* b, float* out, int so, int cout, int n, int relu, const float* res, hipStream_t s);
// Input gradient gx of a layer from its output gradient g, masked by (y > 0) for the ReLU
// layers (matrix cores, wd the input-gradient layout) or unmasked for the 1x1 output layer.
hipError_t conv_bwd_data(int ks, const float* g, int sg, const float* y, int sy, int cout, const __hip_bfloat16* w,
                         const unsigned short* wd, float* gx, int sgx, int cin, int n, hipStream_t s);
// Weight and bias gradients: fixed-order chunk partials pw / pb, slice sums q, then gw / gb.
hipError_t conv_bwd_w(int ks, const float* x, int sx, int cin, const float* g, int sg, const float* y, int sy,
                      int cout, int n, float* pw, float* pb, float* q, float* gw, float* gb, hipStream_t s);
// Workspace (floats) conv_bwd_w needs for a layer.
void wgrad_workspace(int ks, int cin, int cout, int n, size_t& pw_floats, size_t& pb_floats, size_t& q_floats);
// Resampling of c channels (a multiple of 4) between views; n is the fine edge.
hipError_t pool2(const float* x, int sx, float* y, int sy, int c, int n, hipStream_t s);
hipError_t up2(const float* x, int sx, float* y, int sy, int c, int n, hipStream_t s);
hipError_t up2_bwd(const float* g, int sg, float* gx, int sgx, int c, int n, hipStream_t s);
hipError_t pool2_bwd_add(const float* g, int sg, const float* add, int sa, float* gx, int sgx, int c, int n,
                         hipStream_t s);
hipError_t mse(const float* y, const float* tg, float* gy, double* part, double* loss, size_t count, hipStream_t s);
hipError_t adam(float* th, const float* g, float* m, float* v, int count, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s);
hipError_t round_bf16(const float* th, __hip_bfloat16* w, int count, hipStream_t s);

}  // namespace unet

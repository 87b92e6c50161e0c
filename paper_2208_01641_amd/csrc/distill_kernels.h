// Host interface to the training kernels of the distilled synthesis network.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace lic {

enum WgradXType { XT_F32 = 0, XT_BF16 = 1, XT_I8 = 2 };     // layer input: float, bf16, int8 symbol + mu
enum WgradGType { GT_NHWC = 0, GT_NCHW3 = 1 };              // output gradient: NHWC, or 3-channel NCHW

// Weight gradient of a transposed convolution with weights [ci][co][k][k],
// stride s, padding p: x is the layer input [n][H][W][ci] (NHWC), g the
// gradient of its output [n][Ho][Wo][co] (NHWC) or [n][3][Ho][Wo] (NCHW).
struct WgradArgs {
    const void* x;
    const float* mu;          // per-channel offsets of int8 inputs
    const float* g;
    float* part;              // workspace: [nchunk][ci][k k co] partial sums
    float* dw;                // result [ci][co][k][k]
    int n, H, W, ci, Ho, Wo, co, k, s, p;
    int chunk;                // input pixels per partial sum (multiple of 16)
    int ncol_tiles;           // ceil(k k co / 64)
};

// Sample indices of one training batch, passed by value in the kernel arguments.
struct SampleList {
    int32_t idx[64];
};
// dst[i] = src[idx[i]] for i < n, each sample `bytes` long (a multiple of 16)
hipError_t launch_gather_samples(const void* src, long bytes, const SampleList& l, int n, void* dst, hipStream_t s);

hipError_t launch_wgrad(const WgradArgs& a, int xt, int gt, hipStream_t s);
// out[o] = sum over pixels of g [P][co] (co divides 256)
hipError_t launch_colsum(const float* g, long P, int co, int chunk, float* part, float* out, hipStream_t s);
// g = 2 (pred - target) / count over [n][3][plane]; loss = mean squared error;
// dbias3[o] = sum of g over channel o
hipError_t launch_mse(const float* pred, const float* target, int n, long plane, int chunks, float* g, float* part_sq,
                      float* part_g, float* loss, float* dbias3, hipStream_t s);
// AdamW step t: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// w = w (1 - lr wd) - lr (m / c1) / (sqrt(v / c2) + eps), c = 1 - b^t
struct AdamCoef {
    float lr, b1, omb1, b2, omb2, eps, decay, c1, c2;
};
hipError_t launch_adamw(float* w, float* m, float* v, const float* g, long n, const AdamCoef& k, hipStream_t s);
hipError_t launch_gather_pack(const float* master, const int32_t* idx, long n, float* out32, void* out16,
                              hipStream_t s);
// Device address and size of the fixed workspace of the allocation-free
// forward pass, on the current device (looked up once per device).
constexpr size_t kDistillScratchBytes = size_t(32) << 20;
hipError_t distill_scratch(void** ptr, size_t* bytes);
// *out = sum of (a - b)^2 over n elements
hipError_t launch_sqdiff(const float* a, const float* b, long n, int chunk, float* part, float* out, hipStream_t s);

}  // namespace lic

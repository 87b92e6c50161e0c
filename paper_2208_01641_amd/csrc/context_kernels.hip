// Element-wise kernels of the context model's two checkerboard passes
// (mean-scale hyperprior with parallel context prediction).
//
// Latents [n][Hy][Wy][C] are split into two sets by the two-pass order:
// anchors ((r + c) even, coded first with parameters from the hyperprior
// alone) and the rest (coded second, with a context of the decoded anchors).
// The checkerboard-major layout [n][part][Hy][Wy/2][C] keeps each set's
// positions contiguous row by row (entry j of row r is column
// 2 j + ((r + part) & 1)), so a row slice of a set is one contiguous range for
// the entropy coder.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "kernels.h"

namespace lic {

namespace {

// One thread per 4 channels of one position of the set.
__global__ void cb_fill_kernel(float* __restrict__ buf, int n, int Hy, int Wy, int ld, int off, int C, int part,
                               float value)
{
    const int c4 = C / 4, Wh = Wy / 2;
    const long total = (long)n * Hy * Wh * c4;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int q = (int)(i % c4);
    long p = i / c4;
    const int j = (int)(p % Wh);
    p /= Wh;
    const int r = (int)(p % Hy);
    const int img = (int)(p / Hy);
    const int c = 2 * j + ((r + part) & 1);
    float4* dst = reinterpret_cast<float4*>(buf + (((long)img * Hy + r) * Wy + c) * ld + off + 4 * q);
    *dst = make_float4(value, value, value, value);
}

// y_hat = sym + mean at the positions of one set: sym and mean in the
// checkerboard-major layout, y_hat on the full grid as float32 and / or bf16.
__global__ void cb_dequant_kernel(const int8_t* __restrict__ sym, const float* __restrict__ mean,
                                  float* __restrict__ out32, __hip_bfloat16* __restrict__ out16, int n, int Hy,
                                  int Wy, int C, int part)
{
    const int c4 = C / 4, Wh = Wy / 2;
    const long total = (long)n * Hy * Wh * c4;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int q = (int)(i % c4);
    long p = i / c4;
    const int j = (int)(p % Wh);
    p /= Wh;
    const int r = (int)(p % Hy);
    const int img = (int)(p / Hy);
    const long src = ((((long)img * 2 + part) * Hy + r) * Wh + j) * C + 4 * q;
    const char4 s = *reinterpret_cast<const char4*>(sym + src);
    const float4 m = *reinterpret_cast<const float4*>(mean + src);
    const float4 v = make_float4((float)s.x + m.x, (float)s.y + m.y, (float)s.z + m.z, (float)s.w + m.w);
    const int c = 2 * j + ((r + part) & 1);
    const long dst = (((long)img * Hy + r) * Wy + c) * C + 4 * q;
    if (out32) *reinterpret_cast<float4*>(out32 + dst) = v;
    if (out16) {
        out16[dst + 0] = __float2bfloat16(v.x);
        out16[dst + 1] = __float2bfloat16(v.y);
        out16[dst + 2] = __float2bfloat16(v.z);
        out16[dst + 3] = __float2bfloat16(v.w);
    }
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ in, __hip_bfloat16* __restrict__ out, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = __float2bfloat16(in[i]);
}

}  // namespace

hipError_t launch_f32_to_bf16(const float* in, void* out, long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, s, in,
                       static_cast<__hip_bfloat16*>(out), n);
    return hipGetLastError();
}

hipError_t launch_cb_fill(float* buf, int n, int Hy, int Wy, int ld, int off, int C, int part, float value,
                          hipStream_t s)
{
    if (C % 4 || off % 4 || ld % 4 || Wy % 2 || (part != 0 && part != 1)) return hipErrorInvalidValue;
    const long total = (long)n * Hy * (Wy / 2) * (C / 4);
    if (total == 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(cb_fill_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, buf, n,
                       Hy, Wy, ld, off, C, part, value);
    return hipGetLastError();
}

hipError_t launch_cb_dequant(const int8_t* sym, const float* mean, float* out32, void* out16, int n, int Hy, int Wy,
                             int C, int part, hipStream_t s)
{
    if (C % 4 || Wy % 2 || (part != 0 && part != 1)) return hipErrorInvalidValue;
    const long total = (long)n * Hy * (Wy / 2) * (C / 4);
    if (total == 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(cb_dequant_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, sym,
                       mean, out32, static_cast<__hip_bfloat16*>(out16), n, Hy, Wy, C, part);
    return hipGetLastError();
}

}  // namespace lic

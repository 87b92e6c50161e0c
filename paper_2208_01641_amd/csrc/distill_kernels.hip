// Training kernels of the distilled synthesis network: weight gradients of
// transposed convolutions on MFMA, bias gradients, the MSE loss with its
// gradient, AdamW, and the gather that refreshes the packed GEMM weights from
// the FP32 master copy.  The forward passes and the input gradients run on the
// implicit-GEMM convolution kernels.  Every reduction is done in a fixed
// order (per-chunk partial sums, then a sequential sum over the chunks), so a
// training step gives the same bits on every run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "distill_kernels.h"

namespace lic {

// Workspace of the allocation-free forward pass: the two hidden activations
// of one call.  Every device that runs that pass holds its own copy of this
// array until the process ends; host code reaches it only through the
// address that hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[kDistillScratchBytes];

hipError_t distill_scratch(void** ptr, size_t* bytes)
{
    constexpr int kMaxDevices = 64;
    static std::mutex m;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(m);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kDistillScratchBytes;
    return hipSuccess;
}

typedef float f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ weight grads
// For a transposed convolution out[s j + u - p] += w[c][o][u] x[j][c], the
// weight gradient is, per tap (u, v), a contraction over the input pixels j:
//   dW[c][o][u][v] = sum_j x[j][c] * g[s j + (u, v) - p][o].
// As one GEMM: rows = input channels c, columns = (tap, o), K = input pixels.
// A block computes a 64 x 64 tile over one chunk of pixels and writes the
// partial sum; wgrad_reduce adds the chunks in order.
//
// Staging: 16 pixels at a time go through LDS (each thread loads 4
// consecutive channels of one pixel for x and 4 consecutive columns for g),
// double-buffered so one barrier per stage suffices.  Each of the 4 waves
// owns a 32 x 32 quarter of the tile: 2 x 2 v_mfma_f32_16x16x4_f32 per
// K-step, A[row = c][k = pixel] and B[k = pixel][col] read from LDS.
constexpr int kWgStride = 80;     // LDS row pitch (floats): conflict-free for the operand reads

template <int XT, int GT>
__global__ void __launch_bounds__(256) wgrad_mfma(WgradArgs a)
{
    __shared__ float xs[2][16][kWgStride];
    __shared__ float gs[2][16][kWgStride];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, kg = lane >> 4;
    const int ctiles = a.ci / 64;
    int b = blockIdx.x;
    const int ct = b % ctiles;
    b /= ctiles;
    const int nt = b % a.ncol_tiles;
    const int chunk = b / a.ncol_tiles;
    const int HW = a.H * a.W;
    const long P = (long)a.n * HW;
    const long p0 = (long)chunk * a.chunk;
    const long p1 = p0 + a.chunk < P ? p0 + a.chunk : P;
    const int ncol = a.k * a.k * a.co;

    // loader: pixel row lr of the stage, 4 consecutive channels / columns at lc
    const int lr = tid >> 4, lc = (tid & 15) * 4;
    const int c0 = ct * 64 + lc;
    const int col0 = nt * 64 + lc;
    f4 xr, gr;
    auto load = [&](long pb) {
        const long p = pb + lr;
        xr = f4{0.0f, 0.0f, 0.0f, 0.0f};
        gr = f4{0.0f, 0.0f, 0.0f, 0.0f};
        if (p >= p1) return;
        if constexpr (XT == XT_F32) {
            xr = *reinterpret_cast<const f4*>(static_cast<const float*>(a.x) + p * a.ci + c0);
        } else if constexpr (XT == XT_BF16) {
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            const bf16x4 h = *reinterpret_cast<const bf16x4*>(static_cast<const __bf16*>(a.x) + p * a.ci + c0);
            for (int i = 0; i < 4; ++i) xr[i] = (float)h[i];
        } else {
            const uint32_t u = *reinterpret_cast<const uint32_t*>(static_cast<const int8_t*>(a.x) + p * a.ci + c0);
            for (int i = 0; i < 4; ++i) xr[i] = (float)(int8_t)(u >> (8 * i)) + a.mu[c0 + i];
        }
        const int img = (int)(p / HW);
        const int r = (int)(p - (long)img * HW);
        const int jy = r / a.W, jx = r - (r / a.W) * a.W;
        if constexpr (GT == GT_NHWC) {
            // co is a multiple of 4: the 4 columns share one tap
            if (col0 < ncol) {
                const int tap = col0 / a.co, o = col0 - tap * a.co;
                const int u = tap / a.k, v = tap - u * a.k;
                const int gy = a.s * jy + u - a.p, gx = a.s * jx + v - a.p;
                if (gy >= 0 && gy < a.Ho && gx >= 0 && gx < a.Wo)
                    gr = *reinterpret_cast<const f4*>(a.g + (((long)img * a.Ho + gy) * a.Wo + gx) * a.co + o);
            }
        } else {
            // 3-channel NCHW gradient: columns (tap, o) one by one
            for (int i = 0; i < 4; ++i) {
                const int col = col0 + i;
                if (col >= ncol) break;
                const int tap = col / 3, o = col - 3 * (col / 3);
                const int u = tap / a.k, v = tap - u * a.k;
                const int gy = a.s * jy + u - a.p, gx = a.s * jx + v - a.p;
                if (gy >= 0 && gy < a.Ho && gx >= 0 && gx < a.Wo)
                    gr[i] = a.g[(((long)img * 3 + o) * a.Ho + gy) * a.Wo + gx];
            }
        }
    };

    const int wm = wave & 1, wn = wave >> 1;
    f4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    int buf = 0;
    load(p0);
    for (long pb = p0; pb < p1; pb += 16) {
        *reinterpret_cast<f4*>(&xs[buf][lr][lc]) = xr;
        *reinterpret_cast<f4*>(&gs[buf][lr][lc]) = gr;
        __syncthreads();
        if (pb + 16 < p1) load(pb + 16);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + kg;
            float A[2], B[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) A[i] = xs[buf][kk][wm * 32 + i * 16 + l16];
#pragma unroll
            for (int j = 0; j < 2; ++j) B[j] = gs[buf][kk][wn * 32 + j * 16 + l16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[i], B[j], acc[i][j], 0, 0, 0);
        }
        buf ^= 1;
    }

    // D[4 kg + e][l16] of each 16 x 16 block
    float* part = a.part + (long)chunk * a.ci * ncol;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = nt * 64 + wn * 32 + j * 16 + l16;
            if (col >= ncol) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = ct * 64 + wm * 32 + i * 16 + kg * 4 + e;
                part[(long)c * ncol + col] = acc[i][j][e];
            }
        }
}

// dW in the layer's own layout [ci][co][k][k] = sum over chunks, in order.
__global__ void wgrad_reduce(const float* __restrict__ part, int nchunk, int ci, int co, int k, float* __restrict__ dw)
{
    const int ncol = k * k * co;
    const long total = (long)ci * ncol;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i / ncol), col = (int)(i - (long)c * ncol);
    float s = 0.0f;
    for (int q = 0; q < nchunk; ++q) s += part[(long)q * total + i];
    const int tap = col / co, o = col - tap * co;
    dw[((long)c * co + o) * k * k + tap] = s;
}

// ------------------------------------------------------------- bias grads
// Per-chunk channel sums of an NHWC gradient [P][co] (256 / co pixel rows per
// block step, combined in LDS in row order), then a sequential sum over chunks.
__global__ void __launch_bounds__(256) colsum_partial(const float* __restrict__ g, long P, int co, int chunk,
                                                      float* __restrict__ part)
{
    __shared__ float red[256];
    const int rows = 256 / co;
    const int r = threadIdx.x / co, o = threadIdx.x - (threadIdx.x / co) * co;
    const long p0 = (long)blockIdx.x * chunk;
    const long p1 = p0 + chunk < P ? p0 + chunk : P;
    float s = 0.0f;
    if (r < rows)
        for (long p = p0 + r; p < p1; p += rows) s += g[p * co + o];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < co) {
        float t = 0.0f;
        for (int q = 0; q < rows; ++q) t += red[q * co + threadIdx.x];
        part[(long)blockIdx.x * co + threadIdx.x] = t;
    }
}

// out[j] = scale * sum_q part[q * stride + j * jstride], q = 0 .. nq - 1 in order
__global__ void sum_chunks(const float* __restrict__ part, int nq, long stride, long jstride, int n, float scale,
                           float* __restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.0f;
    for (int q = 0; q < nq; ++q) s += part[(long)q * stride + (long)j * jstride];
    out[j] = scale * s;
}

// -------------------------------------------------------------------- MSE
// g = 2 (pred - target) / count over NCHW [n][3][H][W]; block (plane, chunk)
// writes its sum of squared errors and its sum of g (the output bias
// gradient), each reduced over the block in a fixed tree order.
__global__ void __launch_bounds__(256) mse_grad(const float* __restrict__ pred, const float* __restrict__ target,
                                                long plane, int chunks, float inv2, float* __restrict__ g,
                                                float* __restrict__ part_sq, float* __restrict__ part_g)
{
    __shared__ float rs[256], rg[256];
    const int pl = blockIdx.x / chunks, ch = blockIdx.x - pl * chunks;
    const long len = (plane + chunks - 1) / chunks;
    const long i0 = ch * len, i1 = i0 + len < plane ? i0 + len : plane;
    const float* pp = pred + (long)pl * plane;
    const float* tp = target + (long)pl * plane;
    float* gp = g + (long)pl * plane;
    float sq = 0.0f, sg = 0.0f;
    for (long i = i0 + threadIdx.x; i < i1; i += 256) {
        const float d = pp[i] - tp[i];
        const float gi = inv2 * d;
        gp[i] = gi;
        sq += d * d;
        sg += gi;
    }
    rs[threadIdx.x] = sq;
    rg[threadIdx.x] = sg;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            rs[threadIdx.x] += rs[threadIdx.x + w];
            rg[threadIdx.x] += rg[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_sq[blockIdx.x] = rs[0];
        part_g[blockIdx.x] = rg[0];
    }
}

// out[o] = sum over b, then chunk, of part[(b * 3 + o) * chunks + chunk]
__global__ void sum_planes3(const float* __restrict__ part, int n, int chunks, float* __restrict__ out)
{
    const int o = threadIdx.x;
    if (o >= 3) return;
    float s = 0.0f;
    for (int b = 0; b < n; ++b)
        for (int q = 0; q < chunks; ++q) s += part[((long)b * 3 + o) * chunks + q];
    out[o] = s;
}

// ------------------------------------------------------------------ AdamW
// Decoupled weight decay, bias-corrected moments (c1 = 1 - b1^t, c2 = 1 - b2^t).
// Coefficients come from the host, computed in double and rounded once.
__global__ void adamw(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                      long n, AdamCoef k)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = k.b1 * m[i] + k.omb1 * gi;
    const float vi = k.b2 * v[i] + k.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] = w[i] * k.decay - k.lr * (mi / k.c1) / (sqrtf(vi / k.c2) + k.eps);
}

// packed[i] = master[idx[i]] (0 where idx < 0), as FP32 and optionally bf16
__global__ void gather_pack(const float* __restrict__ master, const int32_t* __restrict__ idx, long n,
                            float* __restrict__ out32, __bf16* __restrict__ out16)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t j = idx[i];
    const float v = j >= 0 ? master[j] : 0.0f;
    if (out32) out32[i] = v;
    if (out16) out16[i] = (__bf16)v;
}

// batch assembly from a device-resident data set, 16 bytes per thread
__global__ void gather_samples(const uint4* __restrict__ src, long words, SampleList l, uint4* __restrict__ dst)
{
    const int i = blockIdx.y;
    const uint4* s = src + (long)l.idx[i] * words;
    uint4* d = dst + (long)i * words;
    for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (long)gridDim.x * blockDim.x) d[w] = s[w];
}

// sum of squared differences of two NCHW images, per block then in order
__global__ void __launch_bounds__(256) sqdiff_partial(const float* __restrict__ a, const float* __restrict__ b, long n,
                                                      int chunk, float* __restrict__ part)
{
    __shared__ float r[256];
    const long i0 = (long)blockIdx.x * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    float s = 0.0f;
    for (long i = i0 + threadIdx.x; i < i1; i += 256) {
        const float d = a[i] - b[i];
        s += d * d;
    }
    r[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = r[0];
}

// ---------------------------------------------------------------- launchers
hipError_t launch_wgrad(const WgradArgs& a, int xt, int gt, hipStream_t s)
{
    const long P = (long)a.n * a.H * a.W;
    const int nchunk = (int)((P + a.chunk - 1) / a.chunk);
    const long blocks = (long)(a.ci / 64) * a.ncol_tiles * nchunk;
    if (blocks <= 0) return hipSuccess;
    void (*fn)(WgradArgs) = nullptr;
    if (gt == GT_NHWC) fn = xt == XT_F32 ? wgrad_mfma<XT_F32, GT_NHWC> : xt == XT_BF16 ? wgrad_mfma<XT_BF16, GT_NHWC> : wgrad_mfma<XT_I8, GT_NHWC>;
    else fn = xt == XT_F32 ? wgrad_mfma<XT_F32, GT_NCHW3> : xt == XT_BF16 ? wgrad_mfma<XT_BF16, GT_NCHW3> : wgrad_mfma<XT_I8, GT_NCHW3>;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(256), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long total = (long)a.ci * a.k * a.k * a.co;
    hipLaunchKernelGGL(wgrad_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a.part, nchunk, a.ci, a.co,
                       a.k, a.dw);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* g, long P, int co, int chunk, float* part, float* out, hipStream_t s)
{
    const int nq = (int)((P + chunk - 1) / chunk);
    hipLaunchKernelGGL(colsum_partial, dim3(nq), dim3(256), 0, s, g, P, co, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_chunks, dim3((co + 63) / 64), dim3(64), 0, s, part, nq, (long)co, 1L, co, 1.0f, out);
    return hipGetLastError();
}

hipError_t launch_mse(const float* pred, const float* target, int n, long plane, int chunks, float* g, float* part_sq,
                      float* part_g, float* loss, float* dbias3, hipStream_t s)
{
    const double count = (double)n * 3 * plane;
    hipLaunchKernelGGL(mse_grad, dim3(n * 3 * chunks), dim3(256), 0, s, pred, target, plane, chunks,
                       (float)(2.0 / count), g, part_sq, part_g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // loss = sum of all block sums / count
    hipLaunchKernelGGL(sum_chunks, dim3(1), dim3(64), 0, s, part_sq, n * 3 * chunks, 1L, 0L, 1, (float)(1.0 / count),
                       loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // bias gradient of output channel o: the blocks of planes (b, o)
    hipLaunchKernelGGL(sum_planes3, dim3(1), dim3(64), 0, s, part_g, n, chunks, dbias3);
    return hipGetLastError();
}

hipError_t launch_adamw(float* w, float* m, float* v, const float* g, long n, const AdamCoef& k, hipStream_t s)
{
    hipLaunchKernelGGL(adamw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, m, v, g, n, k);
    return hipGetLastError();
}

hipError_t launch_gather_pack(const float* master, const int32_t* idx, long n, float* out32, void* out16,
                              hipStream_t s)
{
    hipLaunchKernelGGL(gather_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, master, idx, n, out32,
                       static_cast<__bf16*>(out16));
    return hipGetLastError();
}

hipError_t launch_gather_samples(const void* src, long bytes, const SampleList& l, int n, void* dst, hipStream_t s)
{
    if (bytes % 16 != 0 || n < 1 || n > 64) return hipErrorInvalidValue;
    const long words = bytes / 16;
    const unsigned bx = (unsigned)std::min<long>(256, (words + 255) / 256);
    hipLaunchKernelGGL(gather_samples, dim3(bx, n), dim3(256), 0, s, static_cast<const uint4*>(src), words, l,
                       static_cast<uint4*>(dst));
    return hipGetLastError();
}

hipError_t launch_sqdiff(const float* a, const float* b, long n, int chunk, float* part, float* out, hipStream_t s)
{
    const int nq = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(sqdiff_partial, dim3(nq), dim3(256), 0, s, a, b, n, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_chunks, dim3(1), dim3(64), 0, s, part, nq, 1L, 0L, 1, 1.0f, out);
    return hipGetLastError();
}

}  // namespace lic

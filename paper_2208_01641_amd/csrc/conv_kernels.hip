// Implicit-GEMM convolution kernels for CDNA4 (gfx950), FP32 on MFMA.
//
// One kernel template covers every layer of the analysis / synthesis and
// hyper transforms (strided 5x5 and 3x3 convolutions, and stride-2 5x5
// transposed convolutions split into sub-pixel phases), with the element-wise
// work of each layer fused into its loader and epilogue:
//   loaders  : float NHWC, |float| NHWC (h_a input), int8 symbols + per-channel
//              offset (dequantisation of y_hat / z_hat), and the 3-channel NCHW
//              image with the 64-multiple zero padding done by bounds checks.
//   epilogues: bias, ReLU, GDN / IGDN (channel-mixing sum as a second MFMA
//              contraction on the registers of the first), quantisation to
//              int8 symbols, scale-table index, and the final clamp + crop.
//
// GEMM view: rows = output channels (MFMA A operand, packed weights), columns
// = output pixels (B operand, gathered activations), K = taps x input
// channels.  v_mfma_f32_16x16x4_f32: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4*(l/16)+i][l%16], i = 0..3.  K is walked in
// chunks of 16 input channels: lane group g = l/16 loads 4 consecutive
// channels 4g..4g+3 of its pixel (one 16-byte load) and k-step e of the chunk
// contracts channel 4g+e.  The D layout then gives each lane 4 consecutive
// output channels of one pixel, which is exactly the B-operand layout the
// GDN contraction over channels needs - no data movement between the two.
#include <hip/hip_runtime.h>

#include "../../include/lic.h"
#include "conv_args.h"
#include "kernels.h"

namespace lic {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16x16x4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Blocks are dispatched round-robin over the 8 XCDs (block L goes to XCD
// L % 8).  Give each XCD a contiguous range of logical tiles so that tiles
// sharing input halos and weights share one L2.
__device__ __forceinline__ int xcd_logical_tile(int L, int T)
{
    const int xcd = L & 7, slot = L >> 3;
    int prefix = 0;
    for (int q = 0; q < xcd; ++q) prefix += (T + 7 - q) >> 3;
    return prefix + slot;
}

// TAG is the layer id: it changes no code but gives every layer its own
// kernel symbol, so profiles attribute time per layer.
template <int TAG, int CIN, int MT, int NT, int WAVES, int LD, int EP>
__global__ void __launch_bounds__(64 * WAVES) conv_igemm_f32(ConvArgs a)
{
    constexpr int KC = CIN / 16;
    static_assert(CIN % 16 == 0, "K chunks of 16");
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int l16 = lane & 15;
    const int kg = lane >> 4;

    int logical = xcd_logical_tile(blockIdx.x, gridDim.x);
    const int cog = logical % a.ncog;
    logical /= a.ncog;
    const int phase = logical % a.nphase;
    const int tile = logical / a.nphase;
    const PhaseDesc* __restrict__ ph = a.ph + phase;
    const int ntaps = ph->ntaps;
    const float* __restrict__ wbase = ph->w;
    const int CoP = a.ncog * MT * 16;
    const int co0 = cog * MT * 16;

    const int HWg = a.Hg * a.Wg;
    const int total = a.n * HWg;
    const int pix0 = (tile * WAVES + wave) * (NT * 16);
    if (pix0 >= total) return;   // no LDS, no barriers: whole idle waves may leave

    int img[NT], gy[NT], gx[NT];
    bool pv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int p = pix0 + t * 16 + l16;
        pv[t] = p < total;
        const int q = pv[t] ? p : 0;
        img[t] = q / HWg;
        const int r = q - img[t] * HWg;
        gy[t] = r / a.Wg;
        gx[t] = r - gy[t] * a.Wg;
    }

    f4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const f4 b = *reinterpret_cast<const f4*>(a.bias + co0 + mt * 16 + kg * 4);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = b;
    }

    auto loadA = [&](int t, int kc, f4 (&A)[MT]) {
        const float* wp = wbase + ((long)t * CoP + co0 + l16) * CIN + kc * 16 + kg * 4;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) A[mt] = *reinterpret_cast<const f4*>(wp + (long)mt * 16 * CIN);
    };

    auto loadB = [&](int t, int kc, f4 (&B)[NT]) {
        if constexpr (LD == LD_RGB) {
            // 5x5 stride-2 taps over 3 channels flattened: k = (5u + v) * 3 + c, zero beyond 75.
            const float* in = static_cast<const float*>(a.in);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                f4 v;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = kc * 16 + kg * 4 + e;
                    const int tap = k / 3, c = k - 3 * (k / 3);
                    const int u = tap / 5, w = tap - 5 * (tap / 5);
                    const int iy = gy[nt] * 2 + u - 2, ix = gx[nt] * 2 + w - 2;
                    const bool ok = pv[nt] && k < 75 && iy >= 0 && iy < a.Hin && ix >= 0 && ix < a.Win;
                    float val = 0.0f;
                    if (ok) val = in[(((long)img[nt] * 3 + c) * a.Hin + iy) * a.Win + ix];
                    v[e] = val;
                }
                B[nt] = v;
            }
        } else {
            const int dy = ph->dy[t], dx = ph->dx[t];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int iy = gy[nt] * a.s_in + dy, ix = gx[nt] * a.s_in + dx;
                const bool ok = pv[nt] && iy >= 0 && iy < a.Hin && ix >= 0 && ix < a.Win;
                const long off = (((long)img[nt] * a.Hin + iy) * a.Win + ix) * CIN + kc * 16 + kg * 4;
                f4 v = {0.0f, 0.0f, 0.0f, 0.0f};
                if constexpr (LD == LD_I8) {
                    if (ok) {
                        const uint32_t u = *reinterpret_cast<const uint32_t*>(static_cast<const int8_t*>(a.in) + off);
                        const f4 mu = *reinterpret_cast<const f4*>(a.mu_in + kc * 16 + kg * 4);
                        v[0] = (float)(int8_t)(u & 0xffu) + mu[0];
                        v[1] = (float)(int8_t)((u >> 8) & 0xffu) + mu[1];
                        v[2] = (float)(int8_t)((u >> 16) & 0xffu) + mu[2];
                        v[3] = (float)(int8_t)(u >> 24) + mu[3];
                    }
                } else {
                    if (ok) v = *reinterpret_cast<const f4*>(static_cast<const float*>(a.in) + off);
                    if constexpr (LD == LD_F32_ABS) {
                        v[0] = fabsf(v[0]); v[1] = fabsf(v[1]); v[2] = fabsf(v[2]); v[3] = fabsf(v[3]);
                    }
                }
                B[nt] = v;
            }
        }
    };

    auto compute = [&](const f4 (&A)[MT], const f4 (&B)[NT]) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma16x16x4(A[mt][e], B[nt][e], acc[mt][nt]);
    };

    // K loop, double-buffered in registers: chunk k+1 is in flight while
    // chunk k feeds the matrix cores.
    const int K = ntaps * KC;
    f4 A0[MT], B0[NT], A1[MT], B1[NT];
    loadA(0, 0, A0);
    loadB(0, 0, B0);
    for (int k = 0; k < K; k += 2) {
        const bool has1 = k + 1 < K;
        if (has1) {
            loadA((k + 1) / KC, (k + 1) % KC, A1);
            loadB((k + 1) / KC, (k + 1) % KC, B1);
        }
        compute(A0, B0);
        if (k + 2 < K) {
            loadA((k + 2) / KC, (k + 2) % KC, A0);
            loadB((k + 2) / KC, (k + 2) % KC, B0);
        }
        if (has1) compute(A1, B1);
    }

    // ------------------------------------------------------------ epilogue
    long obase[NT];
    int oy[NT], ox[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        oy[nt] = gy[nt] * a.s_out + ph->oy;
        ox[nt] = gx[nt] * a.s_out + ph->ox;
        obase[nt] = (((long)img[nt] * a.Hout + oy[nt]) * a.Wout + ox[nt]) * a.Co;
    }

    if constexpr (EP == EP_GDN || EP == EP_IGDN) {
        // n = beta + gamma (x*x): [Co x Co] x [Co x pixels] on MFMA, K chunk
        // kc2 of the contraction is exactly this lane's accumulator row block.
        f4 nacc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const f4 b = *reinterpret_cast<const f4*>(a.beta + mt * 16 + kg * 4);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) nacc[mt][nt] = b;
        }
#pragma unroll
        for (int kc2 = 0; kc2 < MT; ++kc2) {
            f4 G[MT], X[NT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                G[mt] = *reinterpret_cast<const f4*>(a.gamma + (long)(mt * 16 + l16) * a.Co + kc2 * 16 + kg * 4);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) X[nt] = acc[kc2][nt] * acc[kc2][nt];
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) nacc[mt][nt] = mfma16x16x4(G[mt][e], X[nt][e], nacc[mt][nt]);
        }
        float* out = static_cast<float*>(a.out);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                f4 y;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float r = sqrtf(nacc[mt][nt][i]);
                    y[i] = (EP == EP_GDN) ? acc[mt][nt][i] / r : acc[mt][nt][i] * r;
                }
                if (pv[nt]) *reinterpret_cast<f4*>(out + obase[nt] + mt * 16 + kg * 4) = y;
            }
    } else if constexpr (EP == EP_NONE || EP == EP_RELU) {
        float* out = static_cast<float*>(a.out);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = co0 + mt * 16 + kg * 4;
                f4 y = acc[mt][nt];
                if constexpr (EP == EP_RELU) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) y[i] = fmaxf(y[i], 0.0f);
                }
                if (pv[nt] && c < a.Co) *reinterpret_cast<f4*>(out + obase[nt] + c) = y;
            }
    } else if constexpr (EP == EP_QUANT) {
        float* out = static_cast<float*>(a.out);
        int8_t* sym = static_cast<int8_t*>(a.aux);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = co0 + mt * 16 + kg * 4;
                if (!(pv[nt] && c < a.Co)) continue;
                const f4 y = acc[mt][nt];
                const f4 mu = *reinterpret_cast<const f4*>(a.qmu + c);
                uint32_t packed = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float q = rintf(y[i] - mu[i]);
                    q = fminf(fmaxf(q, -64.0f), 64.0f);
                    packed |= ((uint32_t)((int)q) & 0xffu) << (8 * i);
                }
                if (out) *reinterpret_cast<f4*>(out + obase[nt] + c) = y;
                *reinterpret_cast<uint32_t*>(sym + obase[nt] + c) = packed;
            }
    } else if constexpr (EP == EP_INDEX) {
        uint8_t* idxo = static_cast<uint8_t*>(a.out);
        float* vout = static_cast<float*>(a.aux);
        const float* __restrict__ thr = a.thr;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = co0 + mt * 16 + kg * 4;
                if (!(pv[nt] && c < a.Co)) continue;
                const f4 y = acc[mt][nt];
                uint32_t packed = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // exp output: exp(v) > t_k  <=>  v > ln t_k (thr holds ln t_k);
                    // ReLU output: max(v, 0, t_0) against t_k (thr holds t_k).
                    const float s = a.hs_exp ? y[i] : fmaxf(fmaxf(y[i], 0.0f), thr[0]);
                    int lo = 0, hi = 63;            // idx = #{k < 63 : thr[k] < s}
#pragma unroll
                    for (int it = 0; it < 6; ++it) {
                        const int mid = (lo + hi) >> 1;
                        if (lo < hi) {
                            if (thr[mid] < s) lo = mid + 1; else hi = mid;
                        }
                    }
                    packed |= (uint32_t)lo << (8 * i);
                }
                *reinterpret_cast<uint32_t*>(idxo + obase[nt] + c) = packed;
                if (vout) *reinterpret_cast<f4*>(vout + obase[nt] + c) = y;
            }
    } else if constexpr (EP == EP_RGB) {
        // rows r = 3 * (2 py + px) + c of the single m-tile are the four
        // sub-pixel phases of the 3 output channels
        static_assert(MT == 1, "EP_RGB uses one m-tile");
        float* out = static_cast<float*>(a.out);
        float* pre = static_cast<float*>(a.aux);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (!pv[nt]) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = kg * 4 + i;
                if (r >= 12) continue;
                const int q = r / 3, c = r - 3 * (r / 3);
                const int y = gy[nt] * 2 + (q >> 1), x = gx[nt] * 2 + (q & 1);
                const float v = acc[0][nt][i];
                if (pre) pre[(((long)img[nt] * 3 + c) * a.Hout + y) * a.Wout + x] = v;
                if (y < a.Hc && x < a.Wc)
                    out[(((long)img[nt] * 3 + c) * a.Hc + y) * a.Wc + x] = fminf(fmaxf(v, 0.0f), 1.0f);
            }
        }
    }
}

// ---------------------------------------------------------------- registry
struct KernelEntry {
    KernelKey key;
    void (*fn)(ConvArgs);
};

#define LIC_K(TAG, CIN, MT, NT, WV, LD, EP) \
    {{TAG, CIN, MT, NT, WV, LD, EP}, conv_igemm_f32<TAG, CIN, MT, NT, WV, LD, EP>}
// both tile configurations of a non-GDN layer: large (4 m-tiles x 2 n-tiles,
// 4 waves) and small (1 x 1, one wave) for grids too small to fill the chip
#define LIC_K2(TAG, CIN, LD, EP) LIC_K(TAG, CIN, 4, 2, 4, LD, EP), LIC_K(TAG, CIN, 1, 1, 1, LD, EP)

static const KernelEntry kEntries[] = {
    // g_a: GDN layers hold every channel of their pixels in one wave
    LIC_K(LIC_GA0, 80, 8, 2, 4, LD_RGB, EP_GDN), LIC_K(LIC_GA0, 80, 12, 1, 4, LD_RGB, EP_GDN),
    LIC_K(LIC_GA1, 128, 8, 2, 4, LD_F32, EP_GDN), LIC_K(LIC_GA1, 192, 12, 1, 4, LD_F32, EP_GDN),
    LIC_K(LIC_GA2, 128, 8, 2, 4, LD_F32, EP_GDN), LIC_K(LIC_GA2, 192, 12, 1, 4, LD_F32, EP_GDN),
    LIC_K2(LIC_GA3, 128, LD_F32, EP_QUANT), LIC_K2(LIC_GA3, 192, LD_F32, EP_QUANT),
    // h_a
    LIC_K2(LIC_HA0, 192, LD_F32_ABS, EP_RELU), LIC_K2(LIC_HA0, 320, LD_F32_ABS, EP_RELU),
    LIC_K2(LIC_HA1, 128, LD_F32, EP_RELU), LIC_K2(LIC_HA1, 192, LD_F32, EP_RELU),
    LIC_K2(LIC_HA2, 128, LD_F32, EP_QUANT), LIC_K2(LIC_HA2, 192, LD_F32, EP_QUANT),
    // h_s
    LIC_K2(LIC_HS0, 128, LD_I8, EP_RELU), LIC_K2(LIC_HS0, 192, LD_I8, EP_RELU),
    LIC_K2(LIC_HS1, 128, LD_F32, EP_RELU), LIC_K2(LIC_HS1, 192, LD_F32, EP_RELU),
    LIC_K2(LIC_HS2, 128, LD_F32, EP_INDEX), LIC_K2(LIC_HS2, 192, LD_F32, EP_INDEX),
    // g_s
    LIC_K(LIC_GS0, 192, 8, 2, 4, LD_I8, EP_IGDN), LIC_K(LIC_GS0, 320, 12, 1, 4, LD_I8, EP_IGDN),
    LIC_K(LIC_GS1, 128, 8, 2, 4, LD_F32, EP_IGDN), LIC_K(LIC_GS1, 192, 12, 1, 4, LD_F32, EP_IGDN),
    LIC_K(LIC_GS2, 128, 8, 2, 4, LD_F32, EP_IGDN), LIC_K(LIC_GS2, 192, 12, 1, 4, LD_F32, EP_IGDN),
    LIC_K(LIC_GS3, 128, 1, 4, 4, LD_F32, EP_RGB), LIC_K(LIC_GS3, 192, 1, 4, 4, LD_F32, EP_RGB),
};

bool kernel_available(const KernelKey& k)
{
    for (const auto& e : kEntries)
        if (e.key == k) return true;
    return false;
}

hipError_t launch_conv(const KernelKey& k, const ConvArgs& args, int nblocks, hipStream_t stream)
{
    for (const auto& e : kEntries)
        if (e.key == k) {
            hipLaunchKernelGGL(e.fn, dim3(nblocks), dim3(64 * k.waves), 0, stream, args);
            return hipGetLastError();
        }
    return hipErrorInvalidDeviceFunction;
}

}  // namespace lic

// Implicit-GEMM convolution kernels for CDNA4 (gfx950) on MFMA, FP32
// accumulation over four operand forms: FP32 (v_mfma_f32_16x16x4_f32),
// split-FP32 (each FP32 operand as the exact sum of three bf16 parts, the six
// part products of order <= 2 on the bf16 matrix cores), bf16, and OCP e4m3
// with per-row FP32 scales (v_mfma_scale_f32_16x16x128_f8f6f4).
//
// One kernel template covers every layer of the analysis / synthesis and
// hyper transforms (strided 5x5 and 3x3 convolutions, and stride-2 5x5
// transposed convolutions split into sub-pixel phases), with the element-wise
// work of each layer fused into its loader and epilogue:
//   loaders  : float NHWC, |float| NHWC (h_a input), int8 symbols + per-channel
//              offset (dequantisation of y_hat / z_hat), and the 3-channel NCHW
//              image with the 64-multiple zero padding done by bounds checks.
//   epilogues: bias, ReLU, GDN / IGDN or 1DN (channel-mixing sum of x^2, or
//              of |x| for 1DN, as a second MFMA contraction on the registers
//              of the first), quantisation to
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
// The other forms keep that arrangement with 32 channels per chunk (bf16,
// split-FP32) or 128 (tap, channel) pairs (e4m3).
//
// Data movement: the GDN layers of whole frames stage each K chunk's weight
// tile once per block in an LDS ring (from registers, or for split-FP32 with
// two pixel tiles per wave straight from global memory into LDS) and the
// gamma slices of the epilogue likewise; pixels stay in per-wave register
// rings.  The stride-1 output layer stages halo tiles (a block's rows of
// pixels with a one-pixel border) and the weights in LDS per channel slice.
// Small grids split K over the waves of a block with a fixed-order LDS
// reduction.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "../../include/lic.h"
#include "conv_args.h"
#include "kernels.h"

namespace lic {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16x16x4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Operand precision of the convolution GEMM (accumulation is always FP32).
//   DT_F32 : v_mfma_f32_16x16x4_f32, 16-channel K chunks, 4 channels per lane
//   DT_BF16: v_mfma_f32_16x16x32_bf16, 32-channel K chunks, 8 channels per
//            lane (one 16-byte load); activations between layers are stored
//            as bf16, GDN / IGDN and all epilogue arithmetic stay FP32.
template <int DT> struct Prec;
// Frag: weight (A) fragment of one lane and K chunk; BIn: pixel (B) values
// as loaded from NHWC activations; BFrag: B as fed to the matrix cores;
// Elem / WElem: activation / weight element; WMUL: weight elements per
// weight value.
template <> struct Prec<DT_F32> {
    using Frag = f4;
    using Elem = float;
    using WElem = float;
    using BIn = f4;
    using BFrag = f4;
    static constexpr int KCH = 16, KE = 4, WMUL = 1;
};
template <> struct Prec<DT_BF16> {
    using Frag = bf16x8;
    using Elem = __bf16;
    using WElem = __bf16;
    using BIn = bf16x8;
    using BFrag = bf16x8;
    static constexpr int KCH = 32, KE = 8, WMUL = 1;
};
//   DT_F32X: FP32 operands split exactly into three bf16 parts (each rounded
//            to nearest from what the previous parts leave: v = v0 + v1 + v2
//            up to 2^-27 |v|); the products of parts i + j <= 2 run on
//            v_mfma_f32_16x16x32_bf16 (each exact in FP32) with FP32
//            accumulation, so a product carries a relative error near
//            2^-25, the level of FP32 rounding.  Weights are split on the host
//            ([part][8] per 8 channels), activations stay FP32 and are split
//            when a chunk is used.
struct Split3 {
    bf16x8 p[3];
};
struct F32x8 {
    f4 lo, hi;
};
template <> struct Prec<DT_F32X> {
    using Frag = Split3;
    using Elem = float;
    using WElem = __bf16;
    using BIn = F32x8;
    using BFrag = Split3;
    static constexpr int KCH = 32, KE = 8, WMUL = 3;
};
//   DT_FP8 : v_mfma_scale_f32_16x16x128_f8f6f4 on OCP e4m3 operands (unit
//            block scales), K walked over the flattened (tap, channel) axis in
//            chunks of 128: lane group g takes 32 consecutive channels of one
//            tap (channels per tap are a multiple of 32).  Weights carry a
//            per-row FP32 scale and activations are stored as e4m3(q x) with
//            a per-layer q, both undone in the epilogue; the operands come
//            from e4m3 activations only (the image layer and g_s's first and
//            last layers of that form run on bf16 operands).
template <> struct Prec<DT_FP8> {
    using Frag = i32x8;
    using Elem = uint8_t;
    using WElem = uint8_t;
    using BIn = i32x8;
    using BFrag = i32x8;
    static constexpr int KCH = 128, KE = 32, WMUL = 1;
};

// eight FP32 values as G bf16 parts, each rounded to nearest (v_cvt_pk_bf16_f32,
// two values per instruction) from what the previous parts leave, which is
// exact in FP32: v = v0 + ... + v_{G-1} up to the rounding of the last part
template <int G>
__device__ __forceinline__ void split_parts(const float (&v)[8], bf16x8 (&out)[G])
{
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    u32x4 w[G];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f2 r = {v[2 * j], v[2 * j + 1]};
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const b2 h = __builtin_convertvector(r, b2);
            w[g][j] = __builtin_bit_cast(uint32_t, h);
            if (g + 1 < G) r -= __builtin_convertvector(h, f2);
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) out[g] = __builtin_bit_cast(bf16x8, w[g]);
}

// eight FP32 values as three bf16 parts (v = v0 + v1 + v2 up to 2^-27 |v|)
__device__ __forceinline__ Split3 split3(const float (&v)[8])
{
    Split3 s;
    split_parts<3>(v, s.p);
    return s;
}

// e4m3 code of two floats in the low 16 bits, saturated to +-448 first
__device__ __forceinline__ uint32_t e4m3x2(float lo, float hi)
{
    lo = fminf(fmaxf(lo, -448.0f), 448.0f);
    hi = fminf(fmaxf(hi, -448.0f), 448.0f);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(lo, hi, 0, false) & 0xffffu;
}

// unit E8M0 block scale (2^0) of the scaled MFMA
constexpr int kE8M0One = 127;

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
// KSPLIT > 1 (small grids): the WAVES = KSPLIT waves of a block share one
// output tile and take interleaved K chunks; their partial sums are added in
// LDS in the fixed wave order 0, 1, ..., KSPLIT-1, so results do not depend
// on timing, batch size or which stream runs the kernel.
// The split-FP32 kernels and the e4m3 GDN kernels on e4m3 activations are
// built for two blocks (two waves per SIMD, 256 registers):
// without the bound the compiler's split between VGPRs and accumulation
// registers would take more than 256 in total.
template <int TAG, int CIN, int MT, int NT, int WAVES, int KSPLIT, int LD, int EP, int DT>
__global__ void __launch_bounds__(64 * WAVES,
                                  DT == DT_F32X || (DT == DT_FP8 && WAVES == 4 && KSPLIT == 1 && MT <= 12 && LD == LD_F32) ? 2 : 1)
conv_igemm(ConvArgs a)
{
    using Frag = typename Prec<DT>::Frag;
    using Elem = typename Prec<DT>::Elem;
    using WElem = typename Prec<DT>::WElem;
    using BIn = typename Prec<DT>::BIn;
    using BFrag = typename Prec<DT>::BFrag;
    constexpr int KCH = Prec<DT>::KCH, KE = Prec<DT>::KE, WMUL = Prec<DT>::WMUL;
    // int8 symbols stay raw in the prefetch ring (with their offsets) and are
    // converted when the chunk is used, so the conversion never waits on a
    // load that is still in flight
    struct I8Raw {
        uint32_t w[KE / 4];
        float mu[KE];
    };
    // image values likewise stay FP32 in the ring in the bf16 form
    struct RgbRaw {
        float x[KE];
    };
    using BRaw = typename std::conditional<
        LD == LD_I8 && DT != DT_FP8, I8Raw,
        typename std::conditional<LD == LD_RGB && (DT == DT_BF16 || DT == DT_F32X), RgbRaw, BIn>::type>::type;
    constexpr int KC = DT == DT_FP8 ? 1 : CIN / KCH;
    static_assert(DT == DT_FP8 ? CIN % 32 == 0 : CIN % KCH == 0, "whole K chunks");
    static_assert(DT == DT_F32 || DT == DT_F32X || LD != LD_F32_ABS, "|y| loader is FP32 only");
    static_assert(KSPLIT == 1 || KSPLIT == WAVES, "split-K blocks share one tile");
    static_assert(KSPLIT == 1 || EP != EP_RGB, "no split-K for the RGB output layer");
    static_assert(EP != EP_MASK || DT == DT_F32, "gradients are FP32");
    constexpr int PIXW = WAVES / KSPLIT;           // waves with distinct pixel groups
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);     // uniform: scalar registers
    const int l16 = lane & 15;
    const int kg = lane >> 4;

    int logical = xcd_logical_tile(blockIdx.x, gridDim.x);
    const int cog = logical % a.ncog;
    logical /= a.ncog;
    const int phase = logical % a.nphase;
    const int tile = logical / a.nphase;
    const PhaseDesc* __restrict__ ph = a.ph + phase;
    const int ntaps = ph->ntaps;
    // tap table held across the wave: lane t keeps (dy, dx) of tap t, read
    // back with readlane / bpermute (no memory access inside the K loop, so
    // the wait for a chunk's operands never covers the prefetched ones)
    const int tapv = lane < ntaps ? (((int)ph->dy[lane] & 0xffff) | ((int)ph->dx[lane] << 16)) : 0;
    const WElem* __restrict__ wbase = static_cast<const WElem*>(a.w) + ph->woff * WMUL;
    const int CoP = a.ncog * MT * 16;
    const int co0 = cog * MT * 16;

    const int HWg = a.Hg * a.Wg;
    const int total = a.n * HWg;
    const int kslot = wave % KSPLIT;
    const int pix0 = (tile * PIXW + wave / KSPLIT) * (NT * 16);
    // without split-K there is no barrier, so idle waves may leave; with it,
    // every wave of the block has the same pix0 and leaves together
    // (GDN blocks of four unsplit waves keep idle waves: they take part in the
    // barriers of the shared weight and gamma staging)
    constexpr bool kGLds = KSPLIT == 1 && WAVES == 4 && (EP == EP_GDN || EP == EP_IGDN);
    // (e4m3: 8 or 12 row blocks)
    constexpr bool kALdsEarly = kGLds && DT != DT_F32X && LD != LD_RGB && MT % 4 == 0 &&
                                (DT != DT_FP8 || (LD == LD_F32 && (MT == 8 || MT == 12)));
    // the split-FP32 form stages the (three times larger) weight tiles of its
    // GDN layers in LDS: a 2-stage ring filled from one register set (other
    // shapes would load them per wave)
    constexpr bool kALdsX = DT == DT_F32X && kGLds && MT % 4 == 0;
    if (!kGLds && LD != LD_TILE && pix0 >= total) return;
    // one LDS buffer for the staged weight ring of the K loop and, after it,
    // the staged gamma slices of the GDN epilogue
    constexpr int kGP = (DT == DT_F32 || DT == DT_F32X) ? 3 : 2;   // bf16 parts of gamma
    constexpr int kAWords = kALdsEarly ? (DT == DT_FP8 ? 2 * MT * 16 * 36 : 3 * MT * 16 * 20) : kALdsX ? 2 * MT * 16 * 52
                          : LD == LD_TILE ? 2 * ((WAVES + 2) * (NT * 16 + 2) + 9 * MT * 16) * 16 : 0;
    constexpr int kGWords = kGLds ? 2 * kGP * MT * 16 * 16 : 0;
    constexpr int kSmemWords = (kAWords > kGWords ? kAWords : kGWords) > 0 ? (kAWords > kGWords ? kAWords : kGWords) : 4;
    __shared__ __attribute__((aligned(16))) uint32_t smem[kSmemWords];

    int img[NT], gy[NT], gx[NT];
    bool pv[NT];
    // halo-tile loader: the block covers TH grid rows (one per wave) of TW
    // pixels starting at (t_y0, t_x0) of image t_img
    constexpr bool kTile = LD == LD_TILE;
    static_assert(!kTile || (KSPLIT == 1 && (DT == DT_F32 || DT == DT_BF16)), "halo tiles: FP32 / bf16, no split-K");
    constexpr int TW = NT * 16, TH = WAVES;
    int t_img = 0, t_y0 = 0, t_x0 = 0;
    if constexpr (kTile) {
        const int bxn = (a.Wg + TW - 1) / TW, byn = (a.Hg + TH - 1) / TH;
        t_img = tile / (bxn * byn);
        const int rem = tile - t_img * (bxn * byn);
        t_y0 = (rem / bxn) * TH;
        t_x0 = (rem - (rem / bxn) * bxn) * TW;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int y = t_y0 + wave, x = t_x0 + t * 16 + l16;
            pv[t] = t_img < a.n && y < a.Hg && x < a.Wg;
            img[t] = pv[t] ? t_img : 0;
            gy[t] = pv[t] ? y : 0;
            gx[t] = pv[t] ? x : 0;
        }
    } else {
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
    }

    f4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        // (loaded by every wave and selected: a load on one path only would
        // make the K loop's wait counts conservative)
        f4 b = {0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (DT != DT_FP8) {
            const f4 bl = *reinterpret_cast<const f4*>(a.bias + co0 + mt * 16 + kg * 4);
            if (kslot == 0) b = bl;
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = b;
    }

    auto loadA = [&](int t, int kc, Frag (&A)[MT]) __attribute__((always_inline)) {
        const WElem* wp = wbase + (((long)t * CoP + co0 + l16) * CIN + kc * KCH + kg * KE) * WMUL;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) A[mt] = *reinterpret_cast<const Frag*>(wp + (long)mt * 16 * CIN * WMUL);
    };

    auto loadB = [&](int t, int kc, BRaw (&B)[NT]) __attribute__((always_inline)) {
        if constexpr (LD == LD_RGB) {
            // kk x kk taps over 3 NCHW channels flattened, k = (kk u + v) * 3 + c,
            // zero beyond 3 kk^2 (g_a's first layer: kk = 5, stride 2, pad 2)
            const float* in = static_cast<const float*>(a.in);
            const float* zero = static_cast<const float*>(a.zero);
            const int kk = a.kk, kn = 3 * a.kk * a.kk;
            const long plane = (long)a.Hin * a.Win;
            const int k0 = kc * KCH + kg * KE;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                // walk (u, w, ch) from k0 without a division per element;
                // outside the image (or past 3 kk^2) read the zero page
                int tap = k0 / 3, ch = k0 - 3 * (k0 / 3);
                int u = tap / kk, w = tap - kk * (tap / kk);
                const float* base = in + (long)img[nt] * 3 * plane;
                float x[KE];
#pragma unroll
                for (int e = 0; e < KE; ++e) {
                    const int iy = gy[nt] * a.s_in + u - a.pad, ix = gx[nt] * a.s_in + w - a.pad;
                    const bool ok = pv[nt] && k0 + e < kn && iy >= 0 && iy < a.Hin && ix >= 0 && ix < a.Win;
                    x[e] = *(ok ? base + ch * plane + (long)iy * a.Win + ix : zero);
                    if (++ch == 3) {
                        ch = 0;
                        if (++w == kk) {
                            w = 0;
                            ++u;
                        }
                    }
                }
                if constexpr (DT == DT_BF16 || DT == DT_F32X) {
                    RgbRaw r;
#pragma unroll
                    for (int e = 0; e < KE; ++e) r.x[e] = x[e];
                    B[nt] = r;
                } else {
                    Frag v;
#pragma unroll
                    for (int e = 0; e < KE; ++e) v[e] = (Elem)x[e];
                    B[nt] = v;
                }
            }
        } else {
            const int tv = __builtin_amdgcn_readlane(tapv, t);
            const int dy = (int)(short)(tv & 0xffff), dx = tv >> 16;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int iy = gy[nt] * a.s_in + dy, ix = gx[nt] * a.s_in + dx;
                const bool ok = pv[nt] && iy >= 0 && iy < a.Hin && ix >= 0 && ix < a.Win;
                // branch-free: out-of-image lanes read the zero page, so every
                // lane issues its load and nothing waits on it before use
                const long off = (((long)img[nt] * a.Hin + iy) * a.Win + ix) * CIN + kc * KCH + kg * KE;
                if constexpr (LD == LD_I8 && DT != DT_FP8) {
                    // y_hat / z_hat = symbol + per-channel offset; zero outside the image
                    const int8_t* src = ok ? static_cast<const int8_t*>(a.in) + off : static_cast<const int8_t*>(a.zero);
                    const float* mu = ok ? a.mu_in + kc * KCH + kg * KE : static_cast<const float*>(a.zero);
                    I8Raw r;
                    if constexpr (KE == 4) {
                        r.w[0] = *reinterpret_cast<const uint32_t*>(src);
                    } else {
                        const uint2 u = *reinterpret_cast<const uint2*>(src);
                        r.w[0] = u.x;
                        r.w[1] = u.y;
                    }
#pragma unroll
                    for (int e = 0; e < KE; e += 4) *reinterpret_cast<f4*>(&r.mu[e]) = *reinterpret_cast<const f4*>(mu + e);
                    B[nt] = r;
                } else {
                    const Elem* src = ok ? static_cast<const Elem*>(a.in) + off : static_cast<const Elem*>(a.zero);
                    B[nt] = *reinterpret_cast<const BIn*>(src);
                }
            }
        }
    };

    // the B operand of a ring entry: int8 symbols + offsets converted, |y|
    // taken for the h_a input, everything else as loaded
    auto cook = [&](const BRaw& r) __attribute__((always_inline)) -> BFrag {
        if constexpr (DT == DT_F32X) {
            float v[8];
            if constexpr (LD == LD_I8) {
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = (float)(int8_t)(r.w[e / 4] >> (8 * (e % 4))) + r.mu[e];
            } else if constexpr (LD == LD_RGB) {
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = r.x[e];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = LD == LD_F32_ABS ? fabsf(r.lo[e]) : r.lo[e];
                    v[4 + e] = LD == LD_F32_ABS ? fabsf(r.hi[e]) : r.hi[e];
                }
            }
            return split3(v);
        } else if constexpr (LD == LD_I8 && DT != DT_FP8) {
            Frag v;
#pragma unroll
            for (int e = 0; e < KE; ++e) v[e] = (Elem)((float)(int8_t)(r.w[e / 4] >> (8 * (e % 4))) + r.mu[e]);
            return v;
        } else if constexpr (LD == LD_RGB && DT == DT_BF16) {
            Frag v;
#pragma unroll
            for (int e = 0; e < KE; ++e) v[e] = (Elem)r.x[e];
            return v;
        } else if constexpr (LD == LD_F32_ABS) {
            Frag v = r;
#pragma unroll
            for (int e = 0; e < KE; ++e) v[e] = fabsf(v[e]);
            return v;
        } else {
            return r;
        }
    };

    // the six part products of the split-FP32 form, smallest first
    auto mfma_x = [](const Split3& A, const Split3& B, f4 c) __attribute__((always_inline)) -> f4 {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.p[0], B.p[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.p[1], B.p[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.p[2], B.p[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.p[0], B.p[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.p[1], B.p[0], c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.p[0], B.p[0], c, 0, 0, 0);
    };
    auto compute = [&](const Frag (&A)[MT], const BRaw (&Braw)[NT]) __attribute__((always_inline)) {
        BFrag B[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) B[nt] = cook(Braw[nt]);
        if constexpr (DT == DT_F32X) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_x(A[mt], B[nt], acc[mt][nt]);
        } else if constexpr (DT == DT_F32) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma16x16x4(A[mt][e], B[nt][e], acc[mt][nt]);
        } else if constexpr (DT == DT_BF16) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B[nt], acc[mt][nt], 0, 0, 0);
        } else {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                        A[mt], B[nt], acc[mt][nt], 0, 0, 0, kE8M0One, 0, kE8M0One);
        }
    };

    // Addresses of the gathered loaders: each pixel's window origin (tap
    // offset 0) is computed once; a tap adds (dy Win + dx) CIN elements and
    // the bounds test compares the origin row / column with the image, so
    // the K loop has no 64-bit multiplies per tap.
    constexpr long InE = LD == LD_I8 ? 1 : (long)sizeof(Elem);      // bytes per input element
    int oy0[NT], ox0[NT];
    const uint8_t* pbase[NT];
    if constexpr (LD != LD_RGB && LD != LD_TILE) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            oy0[nt] = gy[nt] * a.s_in;
            ox0[nt] = gx[nt] * a.s_in;
            pbase[nt] = static_cast<const uint8_t*>(a.in) +
                        ((((long)img[nt] * a.Hin + oy0[nt]) * a.Win + ox0[nt]) * CIN + (DT == DT_FP8 ? 0 : kg * KE)) * InE;
        }
    }

    // DT_FP8: chunk kc of the flattened (tap, channel) axis; this lane group
    // takes channels c .. c + 31 of tap t (t >= ntaps: past the end, zeros)
    auto loadA8 = [&](int kc, Frag (&A)[MT]) __attribute__((always_inline)) {
        const int f = kc * KCH + kg * KE;
        const int t = f / CIN, c = f - (f / CIN) * CIN;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            // past the last tap: read the zero page (no divergent load)
            const WElem* src = t < ntaps ? wbase + ((long)t * CoP + co0 + mt * 16 + l16) * CIN + c
                                         : static_cast<const WElem*>(a.zero);
            A[mt] = *reinterpret_cast<const Frag*>(src);
        }
    };
    // (e4m3 operands come only from e4m3 activations: the image layer and
    // g_s's first and last layers run on bf16 operands in that form)
    static_assert(DT != DT_FP8 || LD == LD_F32, "e4m3 operands load e4m3 activations only");
    auto loadB8 = [&](int kc, Frag (&B)[NT]) __attribute__((always_inline)) {
      if constexpr (DT == DT_FP8) {
        const int f = kc * KCH + kg * KE;
        const int t = f / CIN, c = f - (f / CIN) * CIN;
        const int tv = __builtin_amdgcn_ds_bpermute(4 * (t < ntaps ? t : 0), tapv);
        const int dy = (int)(short)(tv & 0xffff), dx = tv >> 16;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bool ok = t < ntaps && pv[nt] && (unsigned)(oy0[nt] + dy) < (unsigned)a.Hin &&
                            (unsigned)(ox0[nt] + dx) < (unsigned)a.Win;
            const int off = (dy * a.Win + dx) * CIN + c;              // from the window origin
            const Elem* src = ok ? reinterpret_cast<const Elem*>(pbase[nt]) + off : static_cast<const Elem*>(a.zero);
            B[nt] = *reinterpret_cast<const Frag*>(src);
        }
      }
    };

    // values an e4m3 store clamps to +-448, counted once per wave (rare: the
    // activation scales are calibrated so that it does not happen)
    auto count_sat = [&](const f4& v) __attribute__((always_inline)) {
        if (!a.sat) return;
        const bool s = fabsf(v[0]) > 448.0f || fabsf(v[1]) > 448.0f || fabsf(v[2]) > 448.0f || fabsf(v[3]) > 448.0f;
        const unsigned long long m = __ballot(s);
        if (m && lane == __ffsll((long long)m) - 1) atomicAdd(a.sat, (unsigned long long)__popcll(m));
    };
    // stores 4 consecutive channels of one pixel in the activation storage type
    auto store_act = [&](long idx, const f4& y) __attribute__((always_inline)) {
        if constexpr (DT == DT_F32 || DT == DT_F32X) {
            *reinterpret_cast<f4*>(static_cast<float*>(a.out) + idx) = y;
        } else if ((DT == DT_FP8 && !a.out_bf16) || (DT == DT_BF16 && a.out_e4m3)) {
            const f4 v = a.out_q * y;
            count_sat(v);
            *reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(a.out) + idx) =
                e4m3x2(v[0], v[1]) | (e4m3x2(v[2], v[3]) << 16);
        } else {
            bf16x4 h;
#pragma unroll
            for (int i = 0; i < 4; ++i) h[i] = (__bf16)y[i];
            *reinterpret_cast<bf16x4*>(static_cast<__bf16*>(a.out) + idx) = h;
        }
    };

    // K loop over this wave's chunks k = kslot, kslot + KSPLIT, ..., with a
    // register ring of P chunk buffers: P - 1 chunks are in flight while one
    // feeds the matrix cores (as deep as the register budget allows: small
    // tiles have less MFMA work per chunk to hide the load latency behind).
    constexpr int STAGE = (MT * (int)sizeof(Frag) + NT * (int)sizeof(BRaw)) / 4;   // VGPRs per chunk buffer
    constexpr int BUDGET = WAVES >= 8 ? 64 : 128;                     // VGPRs for the ring
    // (the image loader has only a handful of chunks: keep its ring short)
    constexpr int P = DT == DT_F32X ? 2 : kALdsEarly ? 3
                  : (LD == LD_RGB || BUDGET / STAGE < 2) ? 2 : (BUDGET / STAGE > 4 ? 4 : BUDGET / STAGE);
    const int K = DT == DT_FP8 ? (ntaps * CIN + KCH - 1) / KCH : ntaps * KC;
    const int nk = (K - kslot + KSPLIT - 1) / KSPLIT;
    // Gathered (NHWC) loaders walk this wave's chunks kslot, kslot + KSPLIT,
    // ... with a cursor, channel chunk outer and tap inner: all taps of one
    // 16- (bf16: 32-) channel slice of the input window are consumed while the
    // slice is in cache, so the input is fetched from HBM about once (tap-outer
    // order re-reads the whole window once per tap).  The load calls below
    // come in exactly the cursor's order.
    constexpr bool kCursor = DT != DT_FP8 && LD != LD_RGB;
    int cur_t = kslot % ntaps, cur_kc = kslot / ntaps;
    // one step of the cursor (KSPLIT chunks) as whole channel slices plus
    // taps, so a step needs one compare and no loop: a loop between the
    // loads of the ring and their use makes the compiler's wait counts
    // conservative (it then waits for every chunk in flight but the newest)
    const int adv_kc = KSPLIT / ntaps, adv_t = KSPLIT - adv_kc * ntaps;
    // (the tap offset is the same for every lane: dy, dx come from readlane,
    // so it stays on the scalar unit)
    long toff = 0;                                                   // tap offset in elements
    bool pok[NT];
    auto set_tap = [&](int t) __attribute__((always_inline)) {
        const int tv = __builtin_amdgcn_readlane(tapv, t < ntaps ? t : 0);
        const int dy = (int)(short)(tv & 0xffff), dx = tv >> 16;
        toff = ((long)dy * a.Win + dx) * CIN;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            // (bitwise and: no branch, so the loop stays one block)
            pok[nt] = pv[nt] & ((unsigned)(oy0[nt] + dy) < (unsigned)a.Hin) & ((unsigned)(ox0[nt] + dx) < (unsigned)a.Win);
    };
    if constexpr (kCursor) set_tap(cur_t);
    auto cursor_loadB = [&](BRaw (&B)[NT]) __attribute__((always_inline)) {
      if constexpr (kCursor) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if constexpr (LD == LD_I8) {
                const int8_t* src = pok[nt] ? reinterpret_cast<const int8_t*>(pbase[nt] + toff + cur_kc * KCH)
                                            : static_cast<const int8_t*>(a.zero);
                const float* mu = pok[nt] ? a.mu_in + cur_kc * KCH + kg * KE : static_cast<const float*>(a.zero);
                I8Raw r;
                if constexpr (KE == 4) {
                    r.w[0] = *reinterpret_cast<const uint32_t*>(src);
                } else {
                    const uint2 u = *reinterpret_cast<const uint2*>(src);
                    r.w[0] = u.x;
                    r.w[1] = u.y;
                }
#pragma unroll
                for (int e = 0; e < KE; e += 4) *reinterpret_cast<f4*>(&r.mu[e]) = *reinterpret_cast<const f4*>(mu + e);
                B[nt] = r;
            } else {
                const Elem* src = pok[nt] ? reinterpret_cast<const Elem*>(pbase[nt] + (toff + cur_kc * KCH) * InE)
                                          : static_cast<const Elem*>(a.zero);
                B[nt] = *reinterpret_cast<const BIn*>(src);
            }
        }
        cur_t += adv_t;
        cur_kc += adv_kc;
        if (cur_t >= ntaps) {
            cur_t -= ntaps;
            ++cur_kc;
        }
        set_tap(cur_t);
      }
    };
    auto load_cursor = [&](Frag (&A)[MT], BRaw (&B)[NT]) __attribute__((always_inline)) {
        if constexpr (kCursor) {
            const WElem* wp = wbase + (((long)cur_t * CoP + co0 + l16) * CIN + cur_kc * KCH + kg * KE) * WMUL;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) A[mt] = *reinterpret_cast<const Frag*>(wp + (long)mt * 16 * CIN * WMUL);
            cursor_loadB(B);
        }
    };
    auto load = [&](int kk, Frag (&A)[MT], BRaw (&B)[NT]) __attribute__((always_inline)) {
        if constexpr (DT == DT_FP8) {
            loadA8(kk, A);
            loadB8(kk, B);
        } else if constexpr (kCursor) {
            load_cursor(A, B);
        } else {
            loadA(kk / KC, kk % KC, A);
            loadB(kk / KC, kk % KC, B);
        }
    };
    // Shared weights (GDN layers, one pixel tile per wave, no split-K): the
    // four waves of a block need the same weight rows for every chunk, so the
    // block stages each chunk's weight tile in LDS once (two 16-byte pieces
    // per thread; e4m3: four) instead of every wave fetching it: a 3-stage
    // LDS ring, filled two chunks ahead from registers loaded two chunks
    // before that (e4m3: a 2-stage ring, below), one barrier per chunk.  The
    // pixel operands keep their per-wave ring.
    constexpr bool kALds = kALdsEarly;
    if constexpr (kALds) {
        static_assert(P == 3, "the shared-weight loop is written for a 3-deep ring");
        // a chunk row is 64 bytes (FP32 / bf16) or 128 bytes (e4m3: the
        // flattened (tap, channel) chunk, 32 bytes per lane group), padded by
        // 16 bytes in LDS so the 16 rows of one fragment load hit distinct banks
        constexpr int RB = KCH * (int)sizeof(WElem);
        constexpr int PPR = RB / 16;                        // 16-byte pieces per row
        constexpr int AROW = RB / 4 + 4;                    // LDS row pitch in dwords
        constexpr int ROWS = MT * 16;
        constexpr int NPIECE = ROWS * PPR / 256;            // pieces per thread per chunk
        static_assert(ROWS * PPR % 256 == 0, "whole pieces per thread");
        uint32_t* const As = smem;                          // [stages][ROWS][AROW]
        static_assert((DT == DT_FP8 ? 2 : 3) * ROWS * AROW <= kSmemWords, "weight ring fits the LDS buffer");
        const int tid = threadIdx.x;
        int a_t = 0, a_kc = 0, a_k = 0;
        auto a_gload = [&](u32x4 (&r)[NPIECE]) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < NPIECE; ++i) {
                const int q = tid + i * 256, row = q / PPR, c16 = q - (q / PPR) * PPR;
                const void* src;
                if constexpr (DT == DT_FP8) {
                    // flattened position of the piece; past the last tap: zeros
                    const int f = a_k * KCH + c16 * 16, t = f / CIN, c = f - (f / CIN) * CIN;
                    src = t < ntaps ? static_cast<const void*>(wbase + ((long)t * CoP + co0 + row) * CIN + c) : a.zero;
                } else {
                    src = wbase + ((long)a_t * CoP + co0 + row) * CIN + a_kc * KCH + c16 * (16 / (int)sizeof(WElem));
                }
                r[i] = *reinterpret_cast<const u32x4*>(src);
            }
            ++a_k;
            if (++a_t == ntaps) {
                a_t = 0;
                ++a_kc;
            }
        };
        auto a_store = [&](int stage, const u32x4 (&r)[NPIECE]) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < NPIECE; ++i) {
                const int q = tid + i * 256, row = q / PPR, c16 = q - (q / PPR) * PPR;
                *reinterpret_cast<u32x4*>(&As[(stage * ROWS + row) * AROW + c16 * 4]) = r[i];
            }
        };
        auto a_frag = [&](int stage, Frag (&A)[MT]) __attribute__((always_inline)) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const uint32_t* src = &As[(stage * ROWS + mt * 16 + l16) * AROW + kg * (RB / 16)];
                if constexpr (DT == DT_FP8) {
                    const u32x4 lo = *reinterpret_cast<const u32x4*>(src), hi = *reinterpret_cast<const u32x4*>(src + 4);
                    A[mt] = i32x8{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
                } else {
                    A[mt] = __builtin_bit_cast(Frag, *reinterpret_cast<const u32x4*>(src));
                }
            }
        };
        // pixels of chunk kk (the e4m3 loader takes the flat chunk index)
        auto loadBs = [&](int kk, BRaw (&B)[NT]) __attribute__((always_inline)) {
            if constexpr (DT == DT_FP8) loadB8(kk, B);
            else cursor_loadB(B);
        };
      if constexpr (DT == DT_FP8) {
        // e4m3: a two-stage ring, so that the kernel fits two waves per SIMD
        // (the three-stage ring's register sets, with operands of 32 bytes
        // per lane, need one wave per SIMD).  Chunk c sits in register set
        // c % 2, LDS stage c % 2 and pixel buffer c % 2.  Step k issues the
        // weight loads of chunk k + 2 (into the set of chunk k, stored one
        // step earlier) and the pixel loads of chunk k + 1, multiplies chunk
        // k, and stores chunk k + 1 (loaded at the start of step k - 1) into
        // the stage chunk k - 1 used before the last barrier.
        u32x4 ra[2][NPIECE];
        BRaw Bp[2][NT];
        if (0 < nk) a_gload(ra[0]);
        if (1 < nk) a_gload(ra[1]);
        if (0 < nk) loadBs(0, Bp[0]);
        if (0 < nk) a_store(0, ra[0]);
        __syncthreads();
        auto step = [&](int k, auto jc, bool guard) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;          // k % 2
            if (!guard || k + 2 < nk) a_gload(ra[j]);
            if (!guard || k + 1 < nk) loadBs(k + 1, Bp[1 - j]);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const uint32_t* src = &As[(j * ROWS + mt * 16 + l16) * AROW + kg * (RB / 16)];
                const u32x4 lo = *reinterpret_cast<const u32x4*>(src), hi = *reinterpret_cast<const u32x4*>(src + 4);
                const Frag A = i32x8{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                                     (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                        A, Bp[j][nt], acc[mt][nt], 0, 0, 0, kE8M0One, 0, kE8M0One);
            }
            // (keeps the scheduler from sinking this chunk's products below
            // the barrier, where they would hold two chunks of fragments)
            __builtin_amdgcn_sched_barrier(0);
            if (!guard || k + 1 < nk) a_store(1 - j, ra[1 - j]);
            __syncthreads();
        };
        int k0 = 0;
        using J0 = std::integral_constant<int, 0>;
        using J1 = std::integral_constant<int, 1>;
        for (; k0 + 3 < nk; k0 += 2) {
            step(k0, J0{}, false);
            step(k0 + 1, J1{}, false);
        }
        for (; k0 < nk; k0 += 2) {
            step(k0, J0{}, true);
            if (k0 + 1 < nk) step(k0 + 1, J1{}, true);
        }
      } else {
        BRaw Bb[P][NT];
        u32x4 ra[3][NPIECE];
        // prologue: weights of chunks 0..2 in registers, 0 and 1 in LDS, 3 in flight
        if (0 < nk) a_gload(ra[0]);
        if (1 < nk) a_gload(ra[1]);
        if (2 < nk) a_gload(ra[2]);
#pragma unroll
        for (int j = 0; j < P - 1; ++j)
            if (j < nk) loadBs(j, Bb[j]);
        if (0 < nk) a_store(0, ra[0]);
        if (1 < nk) a_store(1, ra[1]);
        if (3 < nk) a_gload(ra[0]);
        __syncthreads();
        // chunk k: weights in stage k % 3 (register set k % 3), pixels in Bb[k % 3]
        // (j is a compile-time constant so that every ring index is static)
        auto step = [&](int k, auto jc, bool guard) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;
            if (!guard || k + P - 1 < nk) loadBs(k + P - 1, Bb[(j + P - 1) % P]);
            Frag A[MT];
            a_frag(j, A);
            compute(A, Bb[j]);
            if (!guard || k + 2 < nk) a_store((j + 2) % 3, ra[(j + 2) % 3]);
            if (!guard || k + 4 < nk) a_gload(ra[(j + 1) % 3]);
            __syncthreads();
        };
        int k0 = 0;
        using J0 = std::integral_constant<int, 0>;
        using J1 = std::integral_constant<int, 1>;
        using J2 = std::integral_constant<int, 2>;
        for (; k0 + 6 < nk; k0 += 3) {
            step(k0, J0{}, false);
            step(k0 + 1, J1{}, false);
            step(k0 + 2, J2{}, false);
        }
        for (; k0 < nk; k0 += 3) {
            step(k0, J0{}, true);
            if (k0 + 1 < nk) step(k0 + 1, J1{}, true);
            if (k0 + 2 < nk) step(k0 + 2, J2{}, true);
        }
      }
    }
    if constexpr (kALdsX) {
        // Split-FP32 weights: per chunk a row holds 32 channels x 3 parts
        // (192 bytes, twelve 16-byte pieces), padded to 208 bytes in LDS so
        // that the 16 rows read by one 16-byte load land in distinct banks.
        // Chunk k + 1 is loaded into the other stage while chunk k feeds the
        // matrix cores; one barrier per chunk.  With two pixel tiles per wave
        // the tiles go from global memory straight into LDS
        // (global_load_lds_dwordx4: lane L of an instruction fills the 16
        // bytes at base + 16 L), so no registers and no LDS stores stage
        // them.  With one pixel tile the matrix work of a chunk is too short
        // to cover that path's wait, and the chunk is fetched into registers
        // (issued before the pixel prefetch, so waiting for it never waits
        // for those) and stored after the chunk's products.
        constexpr bool kDirect = NT >= 2;
        constexpr int AROW = 52;
        constexpr int ROWS = MT * 16;
        static_assert(2 * ROWS * AROW <= kSmemWords, "weight ring fits the LDS buffer");
        uint32_t* const As = smem;                          // [2][ROWS][AROW]
        int a_t = 0, a_kc = 0;
        auto a_next = [&]() __attribute__((always_inline)) {
            if (++a_t == ntaps) {
                a_t = 0;
                ++a_kc;
            }
        };
        // direct path: a stage is ROWS rows of 13 slots (12 data pieces and
        // the pad slot); the 64-slot instructions go round-robin to the waves
        constexpr int SLOTS = ROWS * 13;
        constexpr int NI = SLOTS / 64;
        constexpr int NIW = kDirect ? (NI + WAVES - 1) / WAVES : 1;   // instructions per wave
        static_assert(SLOTS % 64 == 0 && AROW == 52, "whole 64-slot instructions over 208-byte rows");
        // per-lane element offsets of this wave's slots from the chunk's first
        // row (fixed over the K loop); the pad slot re-reads its row's first
        // piece, which lands in the pad and is never read back
        int soff[NIW];
        if constexpr (kDirect) {
#pragma unroll
            for (int u = 0; u < NIW; ++u) {
                const int q = (u * WAVES + wave) * 64 + lane, row = q / 13, c = q - (q / 13) * 13;
                soff[u] = row * CIN * 3 + (c < 12 ? c * 8 : 0);
            }
        }
        // register path: twelve 16-byte pieces per row, NPIECE per thread
        constexpr int PPR = 12;
        constexpr int NPIECE = kDirect ? 1 : ROWS * PPR / 256;
        static_assert(kDirect || ROWS * PPR % 256 == 0, "whole pieces per thread");
        const int tid = threadIdx.x;
        u32x4 ra[NPIECE];
        // issue the loads of the next chunk (into LDS stage `stage` on the direct path)
        auto a_fetch = [&](int stage) __attribute__((always_inline)) {
            const WElem* cb = wbase + ((long)a_t * CoP + co0) * CIN * 3 + a_kc * KCH * 3;
            if constexpr (kDirect) {
#pragma unroll
                for (int u = 0; u < NIW; ++u) {
                    const int i = u * WAVES + wave;
                    if (NI % WAVES == 0 || i < NI) {
#if defined(__HIP_DEVICE_COMPILE__)   // device builtin: the host pass would drop the kernel stub
                        __builtin_amdgcn_global_load_lds(cb + soff[u], smem + (stage * ROWS * AROW + i * 256), 16, 0, 0);
#endif
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < NPIECE; ++i) {
                    const int q = tid + i * 256, row = q / PPR, c = q - (q / PPR) * PPR;
                    ra[i] = *reinterpret_cast<const u32x4*>(cb + row * CIN * 3 + c * 8);
                }
            }
            (void)cb;
            a_next();
        };
        // make the fetched chunk (if `fetched`) visible to every wave; the
        // LDS side of the direct loads is invisible to the compiler's own
        // waits, so that path waits for every load of this wave first
        auto a_publish = [&](int stage, bool fetched) __attribute__((always_inline)) {
            if constexpr (kDirect) {
                __builtin_amdgcn_s_waitcnt(0);
            } else if (fetched) {
#pragma unroll
                for (int i = 0; i < NPIECE; ++i) {
                    const int q = tid + i * 256, row = q / PPR, c = q - (q / PPR) * PPR;
                    *reinterpret_cast<u32x4*>(&As[(stage * ROWS + row) * AROW + c * 4]) = ra[i];
                }
            }
            __syncthreads();
        };
        BRaw Bb[P][NT];
        // pixels of chunk kk: the gathered loaders walk their cursor, the
        // image loader takes the flat chunk index
        auto loadBk = [&](int kk, BRaw (&B)[NT]) __attribute__((always_inline)) {
            if constexpr (kCursor) cursor_loadB(B);
            else loadB(kk / KC, kk % KC, B);
        };
        // prologue: chunk 0 in LDS, pixels of chunks 0 .. P - 2 in flight
        if (0 < nk) a_fetch(0);
#pragma unroll
        for (int j = 0; j < P - 1; ++j)
            if (j < nk) loadBk(j, Bb[j]);
        a_publish(0, 0 < nk);
        auto step = [&](int k, auto jc, bool guard) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;
            // chunk k + 1 for the other stage (its readers passed the last barrier)
            if (!guard || k + 1 < nk) a_fetch(1 - j);
            if (!guard || k + P - 1 < nk) loadBk(k + P - 1, Bb[(j + P - 1) % P]);
            BFrag B[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) B[nt] = cook(Bb[j][nt]);
            const int base = (j * ROWS + l16) * AROW + kg * 12;          // stage k % 2 = j
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                Split3 A;
#pragma unroll
                for (int g = 0; g < 3; ++g)
                    A.p[g] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&As[base + mt * 16 * AROW + g * 4]));
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_x(A, B[nt], acc[mt][nt]);
            }
            a_publish(1 - j, !guard || k + 1 < nk);
        };
        static_assert(P == 2, "the split-FP32 loop is written for a 2-deep pixel ring");
        int k0 = 0;
        using J0 = std::integral_constant<int, 0>;
        using J1 = std::integral_constant<int, 1>;
        for (; k0 + 2 < nk; k0 += 2) {
            step(k0, J0{}, false);
            step(k0 + 1, J1{}, false);
        }
        for (; k0 < nk; k0 += 2) {
            step(k0, J0{}, true);
            if (k0 + 1 < nk) step(k0 + 1, J1{}, true);
        }
    }
    if constexpr (kTile) {
        // Per channel slice (KCH channels, 64 bytes per pixel) the block
        // stages its (TH + 2) x (TW + 2) halo tile and the slice's weights of
        // up to 9 taps in LDS: every input pixel is fetched once per block
        // instead of once per tap.  The next slice is fetched into registers
        // while the taps of this one run (no global load inside the tap loop),
        // double-buffered, one barrier per slice.  Layout, 16 words a row:
        // [halo pixel (hr, hc)] then [tap][weight row].
        constexpr int HC = TW + 2, HR = TH + 2;
        constexpr int NHALO = HR * HC;                      // staged pixels
        constexpr int NROWS = NHALO + 9 * MT * 16;          // plus weight rows
        constexpr int PIECES = NROWS * 4;                   // 16-byte pieces
        constexpr int SPT = (PIECES + 255) / 256;
        static_assert(WAVES == 4, "one block row per wave, 256 threads");
        static_assert(KCH * (int)sizeof(Elem) == 64, "64-byte channel slices");
        static_assert(2 * NROWS * 16 <= kSmemWords, "tile fits the LDS buffer");
        const int tid = threadIdx.x;
        u32x4 rt[SPT];
        auto t_gload = [&](int kc) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int q = tid + i * 256;
                const int row = q >> 2, c4 = q & 3;
                const void* src = a.zero;
                if (row < NHALO) {
                    const int hr = row / HC, hc = row - (row / HC) * HC;
                    const int y = t_y0 + hr - 1, x = t_x0 + hc - 1;
                    if (t_img < a.n && y >= 0 && y < a.Hin && x >= 0 && x < a.Win)
                        src = static_cast<const Elem*>(a.in) + (((long)t_img * a.Hin + y) * a.Win + x) * CIN + kc * KCH +
                              c4 * (16 / (int)sizeof(Elem));
                } else if (row < NROWS) {
                    const int wr = row - NHALO, t = wr / (MT * 16), r = wr - (wr / (MT * 16)) * (MT * 16);
                    if (t < ntaps)
                        src = wbase + ((long)t * CoP + co0 + r) * CIN + kc * KCH + c4 * (16 / (int)sizeof(WElem));
                }
                if (PIECES % 256 == 0 || q < PIECES) rt[i] = *reinterpret_cast<const u32x4*>(src);
            }
        };
        auto t_store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int q = tid + i * 256;
                if (PIECES % 256 == 0 || q < PIECES) *reinterpret_cast<u32x4*>(&smem[buf * NROWS * 16 + q * 4]) = rt[i];
            }
        };
        t_gload(0);
        t_store(0);
        __syncthreads();
        const int nkc = KC;                                 // channel slices
        for (int kc = 0; kc < nkc; ++kc) {
            if (kc + 1 < nkc) t_gload(kc + 1);
            const uint32_t* T = smem + (kc & 1) * NROWS * 16;
#pragma unroll 1
            for (int t = 0; t < ntaps; ++t) {
                const int tv = __builtin_amdgcn_readlane(tapv, t);
                const int dy = (int)(short)(tv & 0xffff), dx = tv >> 16;
                Frag A[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    A[mt] = __builtin_bit_cast(Frag, *reinterpret_cast<const u32x4*>(
                                                         &T[(NHALO + t * MT * 16 + mt * 16 + l16) * 16 + kg * 4]));
                BRaw B[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    B[nt] = __builtin_bit_cast(BRaw, *reinterpret_cast<const u32x4*>(
                                                         &T[((wave + 1 + dy) * HC + nt * 16 + l16 + 1 + dx) * 16 + kg * 4]));
                compute(A, B);
            }
            if (kc + 1 < nkc) {
                t_store((kc + 1) & 1);                      // its last readers were slice kc - 1
                __syncthreads();
            }
        }
    }
    Frag Ab[(kALds || kALdsX || kTile) ? 1 : P][MT];
    BRaw Bb[(kALds || kALdsX || kTile) ? 1 : P][NT];
    if constexpr (!kALds && !kALdsX && !kTile) {
    // steady state: every step issues its prefetch unconditionally, so the
    // wait before a chunk's MFMAs only covers that chunk's own loads.  The
    // prologue before it is unconditional too: a load that some path skips
    // makes the compiler's wait counts at the loop head count from that path
    // (it then waits for every chunk in flight)
    int k0 = 0;
    if (2 * P - 2 < nk) {
#pragma unroll
        for (int j = 0; j < P - 1; ++j) {
            load(kslot + j * KSPLIT, Ab[j], Bb[j]);
            __builtin_amdgcn_sched_barrier(0);          // chunks issued in order, oldest first
        }
        for (; k0 + 2 * P - 2 < nk; k0 += P) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
                load(kslot + (k0 + j + P - 1) * KSPLIT, Ab[(j + P - 1) % P], Bb[(j + P - 1) % P]);
                compute(Ab[j], Bb[j]);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < P - 1; ++j)
            if (j < nk) load(kslot + j * KSPLIT, Ab[j], Bb[j]);
    }
    for (; k0 < nk; k0 += P) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int k = k0 + j;
            if (k >= nk) break;
            if (k + P - 1 < nk) load(kslot + (k + P - 1) * KSPLIT, Ab[(j + P - 1) % P], Bb[(j + P - 1) % P]);
            compute(Ab[j], Bb[j]);
        }
    }
    }

    if constexpr (KSPLIT > 1) {
        __shared__ f4 red[(KSPLIT > 1 ? KSPLIT - 1 : 1) * MT * NT * 64];
        if (kslot > 0) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) red[(((kslot - 1) * MT + mt) * NT + nt) * 64 + lane] = acc[mt][nt];
        }
        __syncthreads();
        if (kslot > 0) return;
        // one partner wave at a time (keeps the partial sums out of registers)
#pragma unroll 1
        for (int w = 1; w < KSPLIT; ++w)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] += red[(((w - 1) * MT + mt) * NT + nt) * 64 + lane];
    }

    if constexpr (DT == DT_FP8) {
        // undo the operand scales, then add the bias
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const f4 rs = *reinterpret_cast<const f4*>(a.rscale + co0 + mt * 16 + kg * 4);
            const f4 b = *reinterpret_cast<const f4*>(a.bias + co0 + mt * 16 + kg * 4);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = acc[mt][nt] * rs + b;
        }
    }

    // ------------------------------------------------------------ epilogue
    long obase[NT];
    int oy[NT], ox[NT];
    const long ldo = a.co_ld ? a.co_ld : a.Co;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        oy[nt] = gy[nt] * a.s_out + ph->oy;
        ox[nt] = gx[nt] * a.s_out + ph->ox;
        obase[nt] = (((long)img[nt] * a.Hout + oy[nt]) * a.Wout + ox[nt]) * ldo + a.co_off;
    }

    // Byte outputs (symbols, scale indices) often go straight to mapped host
    // memory: stage the wave's tile in LDS and write each pixel's MT x 16
    // channel bytes as whole 16-byte pieces (one 64-byte line for MT = 4)
    // rather than 4-byte pieces spread over the lanes.
    constexpr bool kBytes = EP == EP_QUANT || EP == EP_INDEX;
    // scale-table index of a pre-activation scale y: #{k < 63 : thr[k] < s}
    // with s = y (thr holds ln t_k: exp(y) > t_k <=> y > ln t_k) or s =
    // max(y, 0, t_0) (thr holds t_k).  The table is log-spaced, so (s -
    // thr[0]) / step (ReLU: log2(s / thr[0]) / step) is within a step or two
    // of the count; from there the count is settled by comparisons with the
    // table itself (ts, staged per wave in LDS), so the result is exactly the
    // count whatever the first guess.
    auto scale_count = [&](float y, const float* ts, float t0, float inv) __attribute__((always_inline)) {
        const float s = a.hs_exp ? y : fmaxf(fmaxf(y, 0.0f), t0);
        // (the guess needs no exact division: the comparisons settle it)
        const float u = a.hs_exp ? (s - t0) * inv : (__log2f(s) - __log2f(t0)) * inv;
        int e = (int)ceilf(fminf(fmaxf(u, 0.0f), 63.0f));     // NaN: 0
        while (e < 63 && ts[e] < s) ++e;
        while (e > 0 && !(ts[e - 1] < s)) --e;
        return e;
    };
    __shared__ __attribute__((aligned(16))) uint32_t obytes[kBytes ? PIXW : 1][kBytes ? NT * 16 : 1][kBytes ? MT * 4 : 1];
    auto store_bytes = [&](const uint32_t (&pk)[MT][NT], uint8_t* dst) __attribute__((always_inline)) {
        uint32_t (&w)[kBytes ? NT * 16 : 1][kBytes ? MT * 4 : 1] = obytes[wave / KSPLIT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) w[nt * 16 + l16][mt * 4 + kg] = pk[mt][nt];
        // lanes of one wave read each other's words: LDS completes a wave's
        // accesses in order; the fences keep the compiler from reordering
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        constexpr int PIECES = NT * 16 * MT;                 // 16-byte pieces of the tile
#pragma unroll
        for (int q0 = 0; q0 < PIECES; q0 += 64) {
            const int q = q0 + lane;
            const int p = q / MT, m = q - (q / MT) * MT;
            const int P = pix0 + p;
            if ((PIECES % 64 == 0 || q < PIECES) && P < total && co0 + m * 16 < a.Co) {
                const int im = P / HWg, r = P - (P / HWg) * HWg;
                const int yy = r / a.Wg, xx = r - (r / a.Wg) * a.Wg;
                const long o = (((long)im * a.Hout + yy * a.s_out + ph->oy) * a.Wout + xx * a.s_out + ph->ox) * a.Co;
                *reinterpret_cast<u32x4*>(dst + o + co0 + m * 16) = *reinterpret_cast<const u32x4*>(&w[p][m * 4]);
            }
        }
    };

    if constexpr (EP == EP_GDN || EP == EP_IGDN) {
        // n = beta + gamma (x*x) (1DN: beta + gamma |x|): [Co x Co] x [Co x
        // pixels] on the bf16 matrix cores with FP32 accumulation.  x*x (|x|)
        // and gamma are each split into
        // bf16 parts rounded to nearest (v = v0 + v1 + v2 + e, |e| <= 2^-27 |v|;
        // gamma's parts are precomputed); the products of parts whose orders
        // sum to at most GP - 1 are kept: six for the FP32 form (relative error
        // of n about 2^-25, the level of FP32 rounding), three for the bf16 and
        // e4m3 forms (about 2^-16, far below their bf16 / e4m3 outputs).  Every
        // product of bf16 parts is exact in FP32.  One K chunk of 32 channels
        // is the row-block pair (2p, 2p+1) of the accumulators: slot i of lane
        // group kg holds channel (2p + i/4) 16 + 4 kg + i%4, which is exactly
        // this lane's accumulator element, and gamma's parts are stored in
        // the same channel order.
        static_assert(MT % 2 == 0, "GDN rows come in 32-channel pairs");
        constexpr int GP = kGP;                     // bf16 parts per operand
        const bf16x8* __restrict__ gsp = static_cast<const bf16x8*>(a.gsplit);
        constexpr int NPAIR = MT / 2;
        f4 nacc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const f4 b = *reinterpret_cast<const f4*>(a.beta + mt * 16 + kg * 4);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) nacc[mt][nt] = b;
        }
        // Whole blocks stage gamma one 32-channel slice (all rows, GP parts)
        // at a time in LDS, double-buffered: slice p + 1 is fetched into
        // registers while slice p feeds the matrix cores, so the block reads
        // gamma from L2 once instead of once per wave.  Slice layout: 16-byte
        // chunk (g Co + r) 4 + kg = gamma parts of row r, lane group kg.
        constexpr int SCH = GP * MT * 16 * 4;       // 16-byte chunks per slice
        constexpr int SPT = kGLds ? (SCH + 255) / 256 : 1;
        u32x4* const gbuf = reinterpret_cast<u32x4*>(smem);
        u32x4 gst[SPT];
        auto g_fetch = [&](int p) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int q = threadIdx.x + i * 256;
                if (SCH % 256 == 0 || q < SCH) {
                    const int gr = q >> 2, kq = q & 3;         // gr = g Co + r
                    gst[i] = *reinterpret_cast<const u32x4*>(gsp + ((long)gr * NPAIR + p) * 4 + kq);
                }
            }
        };
        auto g_put = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int q = threadIdx.x + i * 256;
                if (SCH % 256 == 0 || q < SCH) gbuf[buf * SCH + q] = gst[i];
            }
        };
        if constexpr (kGLds) {
            static_assert(2 * SCH * 4 <= kSmemWords, "two gamma slices fit the LDS buffer");
            g_fetch(0);
            __syncthreads();                        // the K loop's last LDS reads are done
            g_put(0);
            __syncthreads();
        }
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) {
            if constexpr (kGLds) {
                if (p + 1 < NPAIR) g_fetch(p + 1);
            }
            bf16x8 S[GP][NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                float r[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float x = acc[2 * p + i / 4][nt][i % 4];
                    r[i] = a.norm1 ? fabsf(x) : x * x;
                }
                bf16x8 parts[GP];
                split_parts<GP>(r, parts);
#pragma unroll
                for (int g = 0; g < GP; ++g) S[g][nt] = parts[g];
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                bf16x8 G[GP];
#pragma unroll
                for (int g = 0; g < GP; ++g) {
                    if constexpr (kGLds)
                        G[g] = __builtin_bit_cast(bf16x8, gbuf[(p & 1) * SCH + (g * MT * 16 + mt * 16 + l16) * 4 + kg]);
                    else
                        G[g] = gsp[((long)(g * a.Co + mt * 16 + l16) * NPAIR + p) * 4 + kg];
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    // smallest products first
                    if constexpr (GP == 3) {
                        nacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(G[0], S[2][nt], nacc[mt][nt], 0, 0, 0);
                        nacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(G[1], S[1][nt], nacc[mt][nt], 0, 0, 0);
                        nacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(G[2], S[0][nt], nacc[mt][nt], 0, 0, 0);
                    }
                    nacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(G[0], S[1][nt], nacc[mt][nt], 0, 0, 0);
                    nacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(G[1], S[0][nt], nacc[mt][nt], 0, 0, 0);
                    nacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(G[0], S[0][nt], nacc[mt][nt], 0, 0, 0);
                }
            }
            if constexpr (kGLds) {
                if (p + 1 < NPAIR) {
                    g_put((p + 1) & 1);             // that buffer's last reader was slice p - 1
                    __syncthreads();
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                f4 y;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // GDN: x times the hardware reciprocal square root, IGDN:
                    // x times the hardware square root (each within about one
                    // ulp; n >= beta > 0; the correctly rounded sqrtf costs a
                    // dozen more instructions per value); 1DN: x times the
                    // hardware reciprocal (about one ulp), inverse x n
                    const float nv = nacc[mt][nt][i];
                    if (EP == EP_GDN)
                        y[i] = acc[mt][nt][i] * (a.norm1 ? __builtin_amdgcn_rcpf(nv) : __builtin_amdgcn_rsqf(nv));
                    else
                        y[i] = acc[mt][nt][i] * (a.norm1 ? nv : __builtin_amdgcn_sqrtf(nv));
                }
                if (pv[nt]) store_act(obase[nt] + mt * 16 + kg * 4, y);
            }
    } else if constexpr (EP == EP_NONE || EP == EP_RELU) {
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
                if (pv[nt] && c < a.Co) store_act(obase[nt] + c, y);
            }
    } else if constexpr (EP == EP_QUANT) {
        float* out = static_cast<float*>(a.out);
        uint32_t pk[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = co0 + mt * 16 + kg * 4;
                const bool ok = pv[nt] && c < a.Co;
                const f4 y = acc[mt][nt];
                const f4 mu = ok ? *reinterpret_cast<const f4*>(a.qmu + c) : f4{0.0f, 0.0f, 0.0f, 0.0f};
                uint32_t packed = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float q = rintf(y[i] - mu[i]);
                    q = fminf(fmaxf(q, -64.0f), 64.0f);
                    packed |= ((uint32_t)((int)q) & 0xffu) << (8 * i);
                }
                pk[mt][nt] = packed;
                if (out && ok) *reinterpret_cast<f4*>(out + obase[nt] + c) = y;
            }
        store_bytes(pk, static_cast<uint8_t*>(a.aux));
    } else if constexpr (EP == EP_INDEX) {
        uint8_t* idxo = static_cast<uint8_t*>(a.out);
        float* vout = static_cast<float*>(a.aux);
        const float* __restrict__ thr = a.thr;
        __shared__ float thr_s[PIXW][64];
        float* const ts = thr_s[wave / KSPLIT];
        ts[lane] = lane < 63 ? thr[lane] : __builtin_inff();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float t0 = thr[0];
        const float inv = a.hs_exp ? 62.0f / (thr[62] - t0) : 62.0f / __log2f(thr[62] / t0);
        int cnt[MT][NT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) cnt[mt][nt][i] = scale_count(acc[mt][nt][i], ts, t0, inv);
        uint32_t pk[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = co0 + mt * 16 + kg * 4;
                uint32_t packed = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) packed |= (uint32_t)cnt[mt][nt][i] << (8 * i);
                pk[mt][nt] = packed;
                if (vout && pv[nt] && c < a.Co) *reinterpret_cast<f4*>(vout + obase[nt] + c) = acc[mt][nt];
            }
        store_bytes(pk, idxo);
    } else if constexpr (EP == EP_MSCALE) {
        // rows 2c, 2c + 1 of the tile are the mean and the pre-activation
        // scale of latent channel c: the f4 of lane group kg holds channels
        // c0, c0 + 1 with c0 = (co0 + 16 mt + 4 kg) / 2
        const int M = a.Co / 2, Wh = a.Wout / 2;
        uint8_t* idxo = static_cast<uint8_t*>(a.out);
        int8_t* symo = static_cast<int8_t*>(a.aux);
        const float* __restrict__ thr = a.thr;
        __shared__ float thr_s[PIXW][64];
        float* const ts = thr_s[wave / KSPLIT];
        ts[lane] = lane < 63 ? thr[lane] : __builtin_inff();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float t0 = thr[0];
        const float inv = a.hs_exp ? 62.0f / (thr[62] - t0) : 62.0f / __log2f(thr[62] / t0);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            // checkerboard-major element of this pixel: entry gx of row oy
            const long cpix = (((long)img[nt] * 2 + a.cb_part) * a.Hout + oy[nt]) * Wh + gx[nt];
            const long fpix = ((long)img[nt] * a.Hout + oy[nt]) * a.Wout + ox[nt];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int c0 = (co0 + mt * 16 + kg * 4) / 2;
                if (!pv[nt] || c0 >= M) continue;
                const f4 v = acc[mt][nt];
                const int e0 = scale_count(v[1], ts, t0, inv), e1 = scale_count(v[3], ts, t0, inv);
                *reinterpret_cast<uint16_t*>(idxo + cpix * M + c0) = (uint16_t)(e0 | (e1 << 8));
                if (a.ysrc) {
                    const float2 y = *reinterpret_cast<const float2*>(a.ysrc + fpix * M + c0);
                    const float q0 = fminf(fmaxf(rintf(y.x - v[0]), -64.0f), 64.0f);
                    const float q1 = fminf(fmaxf(rintf(y.y - v[2]), -64.0f), 64.0f);
                    if (symo)
                        *reinterpret_cast<uint16_t*>(symo + cpix * M + c0) =
                            (uint16_t)(((uint32_t)((int)q0) & 0xffu) | (((uint32_t)((int)q1) & 0xffu) << 8));
                    *reinterpret_cast<float2*>(a.yq + fpix * M + c0) = make_float2(q0 + v[0], q1 + v[2]);
                } else {
                    *reinterpret_cast<float2*>(a.yq + cpix * M + c0) = make_float2(v[0], v[2]);
                }
            }
        }
    } else if constexpr (EP == EP_RGB) {
        // rows r = 3 (S py + px) + c are the S x S sub-pixel phases of the 3
        // output channels of a stride-S transposed convolution (S = s_out)
        float* out = static_cast<float*>(a.out);
        float* pre = static_cast<float*>(a.aux);
        const int S = a.s_out, nrow = 3 * a.s_out * a.s_out;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if (!pv[nt]) continue;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = mt * 16 + kg * 4 + i;
                    if (r >= nrow) continue;
                    const int q = r / 3, c = r - 3 * (r / 3);
                    const int py = q / S, px = q - S * (q / S);
                    const int y = gy[nt] * S + py, x = gx[nt] * S + px;
                    const float v = acc[mt][nt][i];
                    if (pre) pre[(((long)img[nt] * 3 + c) * a.Hout + y) * a.Wout + x] = v;
                    if (out && y < a.Hc && x < a.Wc)
                        out[(((long)img[nt] * 3 + c) * a.Hc + y) * a.Wc + x] = fminf(fmaxf(v, 0.0f), 1.0f);
                }
            }
    } else if constexpr (EP == EP_MASK) {
        // ReLU backward: the gradient passes where the forward activation
        // (aux, same layout as out) was positive
        const float* mask = static_cast<const float*>(a.aux);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = co0 + mt * 16 + kg * 4;
                if (!(pv[nt] && c < a.Co)) continue;
                const f4 m = *reinterpret_cast<const f4*>(mask + obase[nt] + c);
                f4 y = acc[mt][nt];
#pragma unroll
                for (int i = 0; i < 4; ++i) y[i] = m[i] > 0.0f ? y[i] : 0.0f;
                *reinterpret_cast<f4*>(static_cast<float*>(a.out) + obase[nt] + c) = y;
            }
    }
}

// ---------------------------------------------------------------- registry
struct KernelEntry {
    KernelKey key;
    void (*fn)(ConvArgs);
};

#define LIC_KSD(TAG, CIN, MT, NT, WV, KS, LD, EP, DT) \
    {{TAG, CIN, MT, NT, WV, KS, LD, EP, DT}, conv_igemm<TAG, CIN, MT, NT, WV, KS, LD, EP, DT>}
#define LIC_KS(TAG, CIN, MT, NT, WV, KS, LD, EP) LIC_KSD(TAG, CIN, MT, NT, WV, KS, LD, EP, DT_F32)
#define LIC_K(TAG, CIN, MT, NT, WV, LD, EP) LIC_KS(TAG, CIN, MT, NT, WV, 1, LD, EP)
// bf16 operand variants of the analysis / synthesis layers
#define LIC_KB(TAG, CIN, MT, NT, WV, LD, EP) LIC_KSD(TAG, CIN, MT, NT, WV, 1, LD, EP, DT_BF16)
#define LIC_KGB(TAG, CIN, MT, NT, LD, EP) \
    LIC_KSD(TAG, CIN, MT, NT, 4, 1, LD, EP, DT_BF16), LIC_KSD(TAG, CIN, MT, NT, 4, 4, LD, EP, DT_BF16)
#define LIC_K2B(TAG, CIN, LD, EP)                                                                \
    LIC_KSD(TAG, CIN, 4, 2, 4, 1, LD, EP, DT_BF16), LIC_KSD(TAG, CIN, 4, 2, 4, 4, LD, EP, DT_BF16), \
        LIC_KSD(TAG, CIN, 4, 2, 8, 8, LD, EP, DT_BF16), LIC_KSD(TAG, CIN, 1, 1, 8, 8, LD, EP, DT_BF16)
// split-FP32 operands: whole-frame GDN layers of the FP32 form
#define LIC_KX(TAG, CIN, MT, NT, LD, EP) LIC_KSD(TAG, CIN, MT, NT, 4, 1, LD, EP, DT_F32X)
// e4m3 operand variants (precision form): g_a and g_s
#define LIC_KF(TAG, CIN, MT, NT, WV, LD, EP) LIC_KSD(TAG, CIN, MT, NT, WV, 1, LD, EP, DT_FP8)
#define LIC_KGF(TAG, CIN, MT, NT, LD, EP) \
    LIC_KSD(TAG, CIN, MT, NT, 4, 1, LD, EP, DT_FP8), LIC_KSD(TAG, CIN, MT, NT, 4, 4, LD, EP, DT_FP8)
#define LIC_K2F(TAG, CIN, LD, EP)                                                              \
    LIC_KSD(TAG, CIN, 4, 2, 4, 1, LD, EP, DT_FP8), LIC_KSD(TAG, CIN, 4, 2, 4, 4, LD, EP, DT_FP8), \
        LIC_KSD(TAG, CIN, 4, 2, 8, 8, LD, EP, DT_FP8), LIC_KSD(TAG, CIN, 1, 1, 8, 8, LD, EP, DT_FP8)
// the tile configurations of a non-GDN layer: large (4 m-tiles x 2 n-tiles,
// 4 pixel-parallel waves), large with 4-way split-K, and small (1 x 1) with
// 8-way split-K, for grids too small to fill the chip
// GDN / IGDN layers: pixel-parallel, or 4-way split-K with the
// normalisation done by the first wave after the reduction
#define LIC_KG(TAG, CIN, MT, NT, LD, EP) LIC_K(TAG, CIN, MT, NT, 4, LD, EP), LIC_KS(TAG, CIN, MT, NT, 4, 4, LD, EP)
#define LIC_K2(TAG, CIN, LD, EP)                                                               \
    LIC_K(TAG, CIN, 4, 2, 4, LD, EP), LIC_KS(TAG, CIN, 4, 2, 4, 4, LD, EP), LIC_KS(TAG, CIN, 4, 2, 8, 8, LD, EP), \
        LIC_KS(TAG, CIN, 1, 1, 8, 8, LD, EP)

static const KernelEntry kEntries[] = {
    // g_a: GDN layers hold every channel of their pixels in one wave (split-K
    // variants for grids that would leave SIMDs idle)
    LIC_K(LIC_GA0, 96, 8, 2, 4, LD_RGB, EP_GDN), LIC_K(LIC_GA0, 96, 12, 1, 4, LD_RGB, EP_GDN),
    LIC_KG(LIC_GA1, 128, 8, 2, LD_F32, EP_GDN), LIC_KG(LIC_GA1, 192, 12, 1, LD_F32, EP_GDN),
    LIC_KG(LIC_GA2, 128, 8, 2, LD_F32, EP_GDN), LIC_KG(LIC_GA2, 192, 12, 1, LD_F32, EP_GDN),
    LIC_K2(LIC_GA3, 128, LD_F32, EP_QUANT), LIC_K2(LIC_GA3, 192, LD_F32, EP_QUANT),
    // h_a
    LIC_K2(LIC_HA0, 192, LD_F32_ABS, EP_RELU), LIC_K2(LIC_HA0, 320, LD_F32_ABS, EP_RELU),
    LIC_K2(LIC_HA1, 128, LD_F32, EP_RELU), LIC_K2(LIC_HA1, 192, LD_F32, EP_RELU),
    LIC_K2(LIC_HA2, 128, LD_F32, EP_QUANT), LIC_K2(LIC_HA2, 192, LD_F32, EP_QUANT),
    // h_s
    LIC_K2(LIC_HS0, 128, LD_I8, EP_RELU), LIC_K2(LIC_HS0, 192, LD_I8, EP_RELU),
    LIC_K2(LIC_HS1, 128, LD_F32, EP_RELU), LIC_K2(LIC_HS1, 192, LD_F32, EP_RELU),
    LIC_K2(LIC_HS2, 128, LD_F32, EP_INDEX), LIC_K2(LIC_HS2, 192, LD_F32, EP_INDEX),
    // context model (N = 128, M = 192): h_a on y, h_s to psi, the context
    // convolution, the entropy-parameter layers of both passes, g_s from y_hat
    LIC_K2(LIC_HA0, 192, LD_F32, EP_RELU), LIC_K2(LIC_HS2, 128, LD_F32, EP_NONE),
    LIC_K2(LIC_CX, 192, LD_F32, EP_NONE),
    LIC_K2(LIC_EP0A, 768, LD_F32, EP_RELU), LIC_K2(LIC_EP1A, 640, LD_F32, EP_RELU),
    LIC_K2(LIC_EP2A, 512, LD_F32, EP_MSCALE),
    LIC_K2(LIC_EP0N, 768, LD_F32, EP_RELU), LIC_K2(LIC_EP1N, 640, LD_F32, EP_RELU),
    LIC_K2(LIC_EP2N, 512, LD_F32, EP_MSCALE),
    LIC_KG(LIC_GS0, 192, 8, 2, LD_F32, EP_IGDN), LIC_KX(LIC_GS0, 192, 8, 2, LD_F32, EP_IGDN),
    LIC_KX(LIC_GS0, 192, 8, 1, LD_F32, EP_IGDN), LIC_KGB(LIC_GS0, 192, 8, 2, LD_F32, EP_IGDN),
    LIC_KB(LIC_GS0, 192, 8, 1, 4, LD_F32, EP_IGDN),
    // g_s
    LIC_KG(LIC_GS0, 192, 8, 2, LD_I8, EP_IGDN), LIC_KG(LIC_GS0, 320, 12, 1, LD_I8, EP_IGDN),
    LIC_KG(LIC_GS1, 128, 8, 2, LD_F32, EP_IGDN), LIC_KG(LIC_GS1, 192, 12, 1, LD_F32, EP_IGDN),
    LIC_KG(LIC_GS2, 128, 8, 2, LD_F32, EP_IGDN), LIC_KG(LIC_GS2, 192, 12, 1, LD_F32, EP_IGDN),
    LIC_K(LIC_GS3, 128, 1, 4, 4, LD_F32, EP_RGB), LIC_K(LIC_GS3, 192, 1, 4, 4, LD_F32, EP_RGB),
    LIC_K(LIC_GS3, 128, 1, 4, 4, LD_TILE, EP_RGB), LIC_K(LIC_GS3, 192, 1, 4, 4, LD_TILE, EP_RGB),
    LIC_KX(LIC_GA1, 128, 8, 2, LD_F32, EP_GDN), LIC_KX(LIC_GA1, 192, 12, 1, LD_F32, EP_GDN),
    LIC_KX(LIC_GA2, 128, 8, 2, LD_F32, EP_GDN), LIC_KX(LIC_GA2, 192, 12, 1, LD_F32, EP_GDN),
    LIC_KX(LIC_GS0, 192, 8, 2, LD_I8, EP_IGDN), LIC_KX(LIC_GS0, 320, 12, 1, LD_I8, EP_IGDN),
    LIC_KX(LIC_GS1, 128, 8, 2, LD_F32, EP_IGDN), LIC_KX(LIC_GS1, 192, 12, 1, LD_F32, EP_IGDN),
    LIC_KX(LIC_GS2, 128, 8, 2, LD_F32, EP_IGDN), LIC_KX(LIC_GS2, 192, 12, 1, LD_F32, EP_IGDN),
    LIC_KX(LIC_GA0, 96, 8, 2, LD_RGB, EP_GDN), LIC_KX(LIC_GA0, 96, 12, 1, LD_RGB, EP_GDN),
    // (one pixel group per wave: grids between half and one wave per SIMD)
    LIC_KX(LIC_GA1, 128, 8, 1, LD_F32, EP_GDN), LIC_KX(LIC_GA2, 128, 8, 1, LD_F32, EP_GDN),
    LIC_KX(LIC_GS0, 192, 8, 1, LD_I8, EP_IGDN), LIC_KX(LIC_GS1, 128, 8, 1, LD_F32, EP_IGDN),
    LIC_KX(LIC_GS2, 128, 8, 1, LD_F32, EP_IGDN),
    // bf16 operands (precision form): g_a and g_s; h_a / h_s stay FP32
    LIC_KB(LIC_GA0, 96, 8, 2, 4, LD_RGB, EP_GDN), LIC_KB(LIC_GA0, 96, 12, 1, 4, LD_RGB, EP_GDN),
    LIC_KGB(LIC_GA1, 128, 8, 2, LD_F32, EP_GDN), LIC_KGB(LIC_GA1, 192, 12, 1, LD_F32, EP_GDN),
    LIC_KGB(LIC_GA2, 128, 8, 2, LD_F32, EP_GDN), LIC_KGB(LIC_GA2, 192, 12, 1, LD_F32, EP_GDN),
    LIC_K2B(LIC_GA3, 128, LD_F32, EP_QUANT), LIC_K2B(LIC_GA3, 192, LD_F32, EP_QUANT),
    LIC_KGB(LIC_GS0, 192, 8, 2, LD_I8, EP_IGDN), LIC_KGB(LIC_GS0, 320, 12, 1, LD_I8, EP_IGDN),
    LIC_KGB(LIC_GS1, 128, 8, 2, LD_F32, EP_IGDN), LIC_KGB(LIC_GS1, 192, 12, 1, LD_F32, EP_IGDN),
    LIC_KGB(LIC_GS2, 128, 8, 2, LD_F32, EP_IGDN), LIC_KGB(LIC_GS2, 192, 12, 1, LD_F32, EP_IGDN),
    LIC_KB(LIC_GS3, 128, 1, 4, 4, LD_F32, EP_RGB), LIC_KB(LIC_GS3, 192, 1, 4, 4, LD_F32, EP_RGB),
    LIC_KB(LIC_GS3, 128, 1, 4, 4, LD_TILE, EP_RGB), LIC_KB(LIC_GS3, 192, 1, 4, 4, LD_TILE, EP_RGB),
    LIC_KB(LIC_GA1, 128, 8, 1, 4, LD_F32, EP_GDN), LIC_KB(LIC_GA2, 128, 8, 1, 4, LD_F32, EP_GDN),
    LIC_KB(LIC_GS0, 192, 8, 1, 4, LD_I8, EP_IGDN), LIC_KB(LIC_GS1, 128, 8, 1, 4, LD_F32, EP_IGDN),
    LIC_KB(LIC_GS2, 128, 8, 1, 4, LD_F32, EP_IGDN),
    // e4m3 operands (precision form): g_a and g_s
    LIC_KGF(LIC_GA1, 128, 8, 2, LD_F32, EP_GDN), LIC_KGF(LIC_GA1, 192, 12, 1, LD_F32, EP_GDN),
    LIC_KGF(LIC_GA2, 128, 8, 2, LD_F32, EP_GDN), LIC_KGF(LIC_GA2, 192, 12, 1, LD_F32, EP_GDN),
    // one 16-pixel group per wave (grids between half and one wave per SIMD)
    LIC_KF(LIC_GA2, 128, 8, 1, 4, LD_F32, EP_GDN),
    LIC_K2F(LIC_GA3, 128, LD_F32, EP_QUANT), LIC_K2F(LIC_GA3, 192, LD_F32, EP_QUANT),
    // (g_s's first layer runs on bf16 operands in this form: no e4m3 kernel)
    LIC_KGF(LIC_GS1, 128, 8, 2, LD_F32, EP_IGDN), LIC_KGF(LIC_GS1, 192, 12, 1, LD_F32, EP_IGDN),
    LIC_KGF(LIC_GS2, 128, 8, 2, LD_F32, EP_IGDN), LIC_KGF(LIC_GS2, 192, 12, 1, LD_F32, EP_IGDN),
    // distilled synthesis network (64 hidden channels): forward in FP32 or
    // bf16 operands, input gradients (ReLU-masked) in FP32
    LIC_K2(TAG_DT1, 192, LD_I8, EP_RELU), LIC_K2(TAG_DT1, 320, LD_I8, EP_RELU),
    LIC_K2B(TAG_DT1, 192, LD_I8, EP_RELU), LIC_K2B(TAG_DT1, 320, LD_I8, EP_RELU),
    LIC_K2(TAG_DT2, 64, LD_F32, EP_RELU), LIC_K2B(TAG_DT2, 64, LD_F32, EP_RELU),
    LIC_K(TAG_DT3, 64, 3, 4, 4, LD_F32, EP_RGB), LIC_KB(TAG_DT3, 64, 3, 4, 4, LD_F32, EP_RGB),
    LIC_K(TAG_DT3, 64, 3, 4, 4, LD_TILE, EP_RGB), LIC_KB(TAG_DT3, 64, 3, 4, 4, LD_TILE, EP_RGB),
    LIC_K2(TAG_DB2, 64, LD_F32, EP_MASK), LIC_K2(TAG_DB3, 192, LD_RGB, EP_MASK),
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

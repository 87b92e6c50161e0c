// Launch descriptors shared by the host-side planner and the HIP kernels.
#pragma once
#include <stdint.h>

namespace lic {

// Input loaders (what the implicit-GEMM "pixel" operand is read from).
enum Loader : int {
    LD_F32 = 0,      // float NHWC activations
    LD_F32_ABS = 1,  // |float| NHWC (h_a takes |y|)
    LD_I8 = 2,       // int8 NHWC symbols, dequantised as sym + mu[c]
    LD_RGB = 3,      // float NCHW 3-channel tensor, kk x kk taps flattened with the
                     // channels (image ingest with its zero pad; 3-channel gradients)
    LD_TILE = 4,     // float / bf16 NHWC activations of a stride-1 grid whose taps lie
                     // within one pixel: each block stages its tile of rows (one per
                     // wave) with a one-pixel halo, and the weights, in LDS per
                     // channel slice
};

// Epilogues fused after the K loop.
enum Epilogue : int {
    EP_NONE = 0,
    EP_RELU = 1,
    EP_GDN = 2,      // y = x / sqrt(beta + gamma (x*x))   (all channels in one wave)
    EP_IGDN = 3,     // y = x * sqrt(beta + gamma (x*x))
    EP_QUANT = 4,    // out = v (float), aux = clamp(rne(v - mu[c]), -64, 64) int8
    EP_INDEX = 5,    // out = scale-table index uint8, aux = v (float, optional)
    EP_RGB = 6,      // transposed conv to 3 channels, all S x S phases as 3 S^2
                     // GEMM rows: out = clamp(v, 0, 1) cropped NCHW, aux = v NCHW
    EP_MASK = 7,     // out = v where aux (forward activation) > 0, else 0
    EP_MSCALE = 8,   // context model: GEMM rows in pairs (mean, pre-activation scale)
                     // of one latent channel; out = scale-table index uint8, aux =
                     // clamp(rne(y - mean), -64, 64) int8 (with ysrc), both in the
                     // checkerboard-major layout; yq = sym + mean on the full grid
                     // (with ysrc) or the mean, checkerboard-major (without)
};

// Checkerboard-major layout of a latent tensor [n][Hy][Wy][C] split by the
// two-pass order: [n][part][Hy][Wy/2][C], part 0 the anchors ((r + c) even),
// part 1 the rest; entry j of row r is column 2 j + ((r + part) & 1).

// Operand precision of a layer's GEMM.
enum DType : int {
    DT_F32 = 0,
    DT_BF16 = 1,
    DT_FP8 = 2,      // OCP e4m3 operands with per-row FP32 scales (rscale)
    DT_F32X = 3,     // FP32 operands as exact sums of three bf16 parts: the six part
                     // products of order <= 2 on the bf16 matrix cores, FP32
                     // accumulation (weights pre-split in ConvArgs::w; FP32 activations)
};

// One phase of a layer.  A plain convolution has one phase; a stride-2
// transposed convolution is split into the four sub-pixel phases, each a
// stride-1 convolution over the input grid with its own subset of taps.
struct PhaseDesc {
    int32_t ntaps;
    int32_t oy, ox;          // output position = s_out * grid + (oy, ox)
    int32_t pad_;
    int64_t woff;            // element offset of this phase's packed weights
                             // [ntaps][CoP][CIN] from ConvArgs::w
    int8_t dy[32], dx[32];   // tap offsets: input = s_in * grid + (dy, dx)
};

struct ConvArgs {
    const void* in;
    void* out;
    void* aux;
    const PhaseDesc* ph;     // [nphase] (device)
    const void* w;           // packed weights of every phase (float, bf16 or e4m3)
    const void* wx;          // the same as bf16 parts for DT_F32X (or null): per 8 channels
                             // [part 0 x8][part 1 x8][part 2 x8], offsets 3 x those of w
    const void* zero;        // >= 64 zero bytes: the source of out-of-image reads
    const float* bias;       // [CoP]
    const float* mu_in;      // LD_I8 offsets [CIN]
    const void* gsplit;      // GDN gamma [Co][Co] as three bf16 parts, [part][r][p][kg][i] of
                             // shape [3][Co][Co/32][4][8]: part of gamma[r][(2p + i/4) 16 + 4 kg + i%4]
    const float* beta;       // GDN [Co]
    const float* qmu;        // EP_QUANT offsets [Co]
    const float* thr;        // EP_INDEX thresholds [63]
    int n, Hin, Win;         // input tensor (per image)
    int Hg, Wg, s_in;        // GEMM pixel grid (per image)
    int Hout, Wout, s_out;   // output tensor (per image)
    int Co;                  // real output channels
    int nphase, ncog;        // phases, output-channel groups
    int hs_exp;              // EP_INDEX: 1 = thresholds are ln(t_k), else t_k with ReLU
    int norm1;               // EP_GDN / EP_IGDN: 1 = 1DN, n = beta + gamma |x|, y = x / n
                             // (inverse y = x n); 0 = GDN, n = beta + gamma (x*x), y = x / sqrt(n)
    int Hc, Wc;              // EP_RGB crop size
    int kk, pad;             // LD_RGB kernel size and padding
    const float* rscale;     // DT_FP8: per packed row, weight scale x input scale
    float out_q;             // DT_FP8: activations are stored as e4m3(out_q * value)
    int out_e4m3;            // DT_BF16 kernels: store e4m3(out_q * value) instead of bf16
                             // (the e4m3 form's image layer runs on bf16 operands)
    unsigned long long* sat; // e4m3 stores: count of values clamped to +-448 (null: not counted)
    int out_bf16;            // DT_FP8 kernels: store bf16 instead of e4m3 (the e4m3 form's
                             // last GDN layer feeds an output layer on bf16 operands)
    int co_ld, co_off;       // activation stores: channel stride of the output tensor
                             // (0: Co) and first channel written (concatenated tensors)
    const float* ysrc;       // EP_MSCALE: y, NHWC full grid (encoder), or null (decoder)
    float* yq;               // EP_MSCALE: y_hat (encoder) or mean (decoder), see EP_MSCALE
    int cb_part;             // EP_MSCALE: the checkerboard set the phases cover (0, 1)
};

}  // namespace lic

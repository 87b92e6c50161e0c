// Distilled synthesis network: a 3-layer transposed-convolution stand-in for
// g_s, trained on the GPU (forward and input gradients on the implicit-GEMM
// kernels, weight gradients, loss and AdamW on the kernels of
// distill_kernels.hip) and usable in the decoder in place of g_s.
#pragma once
#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "../../include/lic.h"
#include "conv_args.h"
#include "kernels.h"
#include "packing.h"

namespace lic {

struct DistillNet {
    // one packed GEMM layer (forward layer or input-gradient convolution)
    struct Layer {
        ConvShape shape{};
        int co = 0, k = 0, s = 0, p = 0;
        long w_off = 0;                  // element offset of the packed weights in the arenas
        long b_off = -1;                 // element offset of the packed bias in arena32 (-1: none)
        std::vector<PhaseDesc> ph;       // .woff: element offset in the arena
        PhaseDesc* d_ph = nullptr;
    };

    lic_distill_config cfg{};
    std::string err;
    int M = 0, F = 0;
    long off[6] = {};                    // parameter arrays in the master vector
    long nparam = 0;
    hipStream_t stream = nullptr;
    std::vector<void*> allocs;

    float* d_master = nullptr;           // FP32 parameters
    float* d_m = nullptr;
    float* d_v = nullptr;
    float* d_grad = nullptr;
    int32_t* d_pidx = nullptr;           // master index of every packed element (-1: zero)
    float* d_arena32 = nullptr;          // packed FP32 weights of all layers, then biases
    void* d_arena16 = nullptr;           // packed bf16 weights of the forward layers
    long n_arena = 0, n_fwd_w = 0;
    Layer fwd[3], dg2, dg3;
    float* d_zero = nullptr;             // zero offsets and biases

    // activations and gradients for max_batch x max_hy x max_wy
    void* d_h1 = nullptr;
    void* d_h2 = nullptr;
    float* d_pre = nullptr;
    float* d_dout = nullptr;
    float* d_dh2 = nullptr;
    float* d_dh1 = nullptr;
    int8_t* d_sym = nullptr;
    float* d_tgt = nullptr;
    float* d_part = nullptr;             // weight-gradient partial sums
    long part_cap = 0;
    float* d_cpart = nullptr;            // bias-gradient partial sums
    float* d_mpart = nullptr;            // loss partial sums (squared error, gradient)
    float* d_loss = nullptr;
    long t = 0;                          // AdamW steps taken

    ~DistillNet();
    int create(const lic_distill_config& c, const float* params, size_t n);
    // Launches the forward pass on stream s (no wait); pre / x_hat as in lic.h.
    // h1 / h2: the hidden activations (null: the handle's own buffers).
    int forward(const int8_t* sym, const float* mu, int n, int hy, int wy, float* pre, float* x_hat, int H, int W,
                hipStream_t s, void* h1 = nullptr, void* h2 = nullptr);
    // Bytes of the two hidden activations of an n x hy x wy call, the second
    // starting at *h2_off (256-byte aligned).
    size_t hidden_bytes(int n, int hy, int wy, size_t* h2_off) const;
    // Loss and gradients into d_grad (stream, no wait); loss to loss_dev.
    int backward(const int8_t* sym, const float* mu, const float* target, int n, int hy, int wy, float* loss_dev);
    int update();                        // AdamW step and repack
    int repack();                        // packed weights from the master copy
    int check_dims(int n, int hy, int wy);

private:
    void* alloc(size_t bytes);
    int build_layer(Layer& L, int tag, int ld, int ep, int dt, PackKind kind, int ci, int co, int k, int s, int p,
                    bool w_deconv, int kimg, long src_w, long src_b, std::vector<int32_t>& idx,
                    std::vector<int32_t>& bidx);
};

}  // namespace lic

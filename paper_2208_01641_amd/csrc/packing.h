// Weight packing for the implicit-GEMM convolution kernels, as index maps.
//
// Every element of a packed weight matrix names the element of the layer's
// weight array (PyTorch layout) that it holds, or -1 for a structural zero
// (K padding, taps a sub-pixel phase does not use).  The codec fills the
// values once when it loads a model; the distilled synthesis network gathers
// them again on the GPU after every optimizer step.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "conv_args.h"

namespace lic {

enum PackKind {
    PK_IMG = 0,      // 3-channel NCHW input (LD_RGB): K = (kk u + v) * 3 + c, padded to kimg
    PK_CONV = 1,     // strided convolution: one phase, k*k taps of [cop][ci]
    PK_DECONV = 2,   // stride-s transposed convolution: s*s sub-pixel phases
    PK_ROWS = 3,     // stride-s transposed convolution to 3 channels: all s*s
                     // phases as 3 s^2 GEMM rows over one input neighbourhood
};

struct PackMap {
    std::vector<PhaseDesc> ph;         // taps and output offsets; .w unset
    std::vector<size_t> off;           // element offset of each phase in idx
    std::vector<int32_t> idx;          // source element of every packed element
    std::vector<int32_t> bias_idx;     // source bias element of every packed row
    int cin = 0;                       // packed K per tap (kimg for PK_IMG)
    int cop = 0;                       // packed rows (multiple of 16)
};

// ci, co: input and output channels of the layer; k: kernel size; s: stride;
// p: padding; w_deconv: the weight array is [ci][co][k][k] (transposed
// convolution) instead of [co][ci][k][k]; kimg: packed K for PK_IMG.
PackMap pack_map(PackKind kind, int ci, int co, int k, int s, int p, bool w_deconv, int kimg = 0);

}  // namespace lic

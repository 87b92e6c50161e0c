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

// A stride-1 convolution ([co][ci][k][k] weights) evaluated only at one set
// of the checkerboard order of a latent grid: part 0 the anchors ((r + c)
// even), part 1 the rest.  Each set is two stride-2 sub-grids, so the GEMM
// runs over the Hy/2 x Wy/2 grid with two phases: output (2 a + oy, 2 b + ox)
// with (oy, ox) = (0, 0), (1, 1) for the anchors and (0, 1), (1, 0) for the
// rest, input 2 (a, b) + (oy + u - k/2, ox + v - k/2).  k = 1: the one tap;
// k > 1: only the taps (u, v) with u + v - 2 (k/2) odd (the context mask, whose
// taps from a non-anchor all fall on anchors).  pair_rows: packed rows 2 c and
// 2 c + 1 hold output channels c and co/2 + c (mean and scale of latent c).
PackMap pack_map_checkerboard(int ci, int co, int k, int part, bool pair_rows);

}  // namespace lic

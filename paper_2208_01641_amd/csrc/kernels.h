// Host-side interface to the HIP kernels.
#pragma once
#include <hip/hip_runtime_api.h>

#include <string>

#include "conv_args.h"

namespace lic {

// Template configuration of one implicit-GEMM kernel instantiation:
// input channels per tap (K chunking), m-tiles (16 output channels each) and
// n-tiles (16 pixels each) per wave, waves per block, loader and epilogue.
struct KernelKey {
    int tag, cin, mt, nt, waves, ksplit, ld, ep, dt;   // tag = layer id (one kernel symbol per layer)
    bool operator==(const KernelKey& o) const
    {
        return tag == o.tag && cin == o.cin && mt == o.mt && nt == o.nt && waves == o.waves &&
               ksplit == o.ksplit && ld == o.ld && ep == o.ep && dt == o.dt;
    }
};

bool kernel_available(const KernelKey& k);
hipError_t launch_conv(const KernelKey& k, const ConvArgs& args, int nblocks, hipStream_t stream);

// Context model, element-wise steps of the two checkerboard passes (layout
// in conv_args.h): value into channels [off, off + C) of a [n][Hy][Wy][ld]
// float tensor at the positions of set `part`; y_hat = sym + mean of set
// `part` (checkerboard-major inputs) onto the full [n][Hy][Wy][C] grid as
// float32 (out32) and / or bf16 (out16), either may be null.
hipError_t launch_cb_fill(float* buf, int n, int Hy, int Wy, int ld, int off, int C, int part, float value,
                          hipStream_t s);
// bf16 (round to nearest even) copy of n floats.
hipError_t launch_f32_to_bf16(const float* in, void* out, long n, hipStream_t s);
hipError_t launch_cb_dequant(const int8_t* sym, const float* mean, float* out32, void* out16, int n, int Hy, int Wy,
                             int C, int part, hipStream_t s);

// Kernel tags beyond the codec's layer ids: the distilled synthesis network
// (forward layers, and the input gradients of its second and third layer).
enum { TAG_DT1 = 32, TAG_DT2 = 33, TAG_DT3 = 34, TAG_DB2 = 35, TAG_DB3 = 36 };

// What the tile policy needs to know of a packed layer.
struct ConvShape {
    int tag, ld, ep, dt, cin, cop, nphase;
    int halo1 = 0;     // stride-1 grid, every tap within one pixel (halo-tile loader allowed)
};

// Picks the tile configuration (split-K for small grids) from policy_pixels
// (the pixel grid of one image, so that results do not depend on the batch),
// sets a.ncog and launches over the a.n x a.Hg x a.Wg grid.  Returns a
// lic_status; *errp names the failure.
// With chosen non-null nothing is launched: the configuration is stored there.
int launch_conv_policy(const ConvShape& L, ConvArgs& a, long policy_pixels, hipStream_t s, std::string* errp,
                       KernelKey* chosen = nullptr);

}  // namespace lic

// Host-side interface to the HIP kernels.
#pragma once
#include <hip/hip_runtime_api.h>

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

}  // namespace lic

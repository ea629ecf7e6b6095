// Kernel instantiations for DMAS order n = 7, single-frame and multi-frame (one
// order per unit so that the orders compile in parallel).
#include "dmas_kernel.hpp"

namespace dmas {
// With p != nullptr: launch. With p == nullptr: report resident workgroups
// per CU for the shape in *blocks.
hipError_t launch_order7(const KernelParams *p, const LaunchShape &s, hipStream_t stream, int *blocks)
{
    return launch_order<7>(p, s, stream, blocks);
}

hipError_t launch_batch_order7(const BatchParams &bp, bool cf, bool env, bool nearfield, int table,
                               unsigned grid, size_t lds, hipStream_t stream)
{
    return launch_batch_order<7>(bp, cf, env, nearfield, table, grid, lds, stream);
}
}  // namespace dmas

// Kernel instantiations for DMAS order n = 1, single-frame and multi-frame (one
// order per unit so that the orders compile in parallel).
#include "dmas_kernel.hpp"

namespace dmas {
// With p != nullptr: launch. With p == nullptr: report resident workgroups
// per CU for the shape in *blocks.
hipError_t launch_order1(const KernelParams *p, const LaunchShape &s, hipStream_t stream, int *blocks)
{
    return launch_order<1>(p, s, stream, blocks);
}

hipError_t launch_batch_order1(const BatchParams &bp, bool cf, bool env, bool nearfield, int table,
                               unsigned grid, size_t lds, hipStream_t stream)
{
    return launch_batch_order<1>(bp, cf, env, nearfield, table, grid, lds, stream);
}
}  // namespace dmas

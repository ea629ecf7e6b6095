// Dispatch of the multi-frame (serving) kernels by order.
#include "dmas_internal.hpp"

namespace dmas {

hipError_t launch_batch(int order, const BatchParams &bp, bool cf, bool env, bool nearfield, int delay,
                        unsigned grid, size_t lds_bytes, hipStream_t stream)
{
    switch (order) {
    case 1: return launch_batch_order1(bp, cf, env, nearfield, delay, grid, lds_bytes, stream);
    case 2: return launch_batch_order2(bp, cf, env, nearfield, delay, grid, lds_bytes, stream);
    case 3: return launch_batch_order3(bp, cf, env, nearfield, delay, grid, lds_bytes, stream);
    case 4: return launch_batch_order4(bp, cf, env, nearfield, delay, grid, lds_bytes, stream);
    case 5: return launch_batch_order5(bp, cf, env, nearfield, delay, grid, lds_bytes, stream);
    case 6: return launch_batch_order6(bp, cf, env, nearfield, delay, grid, lds_bytes, stream);
    case 7: return launch_batch_order7(bp, cf, env, nearfield, delay, grid, lds_bytes, stream);
    case 8: return launch_batch_order8(bp, cf, env, nearfield, delay, grid, lds_bytes, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dmas

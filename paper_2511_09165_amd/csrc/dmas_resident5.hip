// Resident worker instantiations for DMAS order n = 5 (one order per unit so
// that the orders compile in parallel).
#include "dmas_resident_kernel.hpp"

namespace dmas {
hipError_t launch_resident_order5(bool cf, bool env, bool nearfield, int delay, const ResidentArgs &a, unsigned grid,
                                  size_t lds, hipStream_t stream, int *blocks)
{
    return launch_resident_order<5>(cf, env, nearfield, delay, a, grid, lds, stream, blocks);
}
}  // namespace dmas

// Root plane pass: the signed n-th root of every channel sample, eq. (4),
// stored beside the sample for the beamformer's staging step.
#include "dmas_kernel.hpp"

namespace dmas {

namespace {

template <int N>
hipError_t launch_roots_n(int dtype, const void *x, float2 *plane, size_t count, hipStream_t stream)
{
    constexpr unsigned kThreads = 256;
    const size_t want = (count + kThreads - 1) / kThreads;
    const unsigned grid = (unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192);
    if (dtype == 0) hipLaunchKernelGGL((root_plane_kernel<N, 0>), dim3(grid), dim3(kThreads), 0, stream, x, plane, count);
    else if (dtype == 1) hipLaunchKernelGGL((root_plane_kernel<N, 1>), dim3(grid), dim3(kThreads), 0, stream, x, plane, count);
    else hipLaunchKernelGGL((root_plane_kernel<N, 2>), dim3(grid), dim3(kThreads), 0, stream, x, plane, count);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_roots(int order, int dtype, const void *x, float2 *plane, size_t count, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    switch (order) {
    case 2: return launch_roots_n<2>(dtype, x, plane, count, stream);
    case 3: return launch_roots_n<3>(dtype, x, plane, count, stream);
    case 4: return launch_roots_n<4>(dtype, x, plane, count, stream);
    case 5: return launch_roots_n<5>(dtype, x, plane, count, stream);
    case 6: return launch_roots_n<6>(dtype, x, plane, count, stream);
    case 7: return launch_roots_n<7>(dtype, x, plane, count, stream);
    case 8: return launch_roots_n<8>(dtype, x, plane, count, stream);
    default: return hipErrorNotSupported;
    }
}

}  // namespace dmas

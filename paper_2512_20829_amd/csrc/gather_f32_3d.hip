// The gather kernels and launchers for binary32 in 3-D (one unit per precision and
// dimension, so that the instantiations compile in parallel).
#include "gather.hpp"

namespace flp {

template hipError_t launch_gather<float, 3>(const GatherArgs&, int, bool, int, hipStream_t);
template hipError_t launch_gather_batch<float, 3>(const BatchItem*, int, int, int, bool, int, bool, uint32_t*, int,
                                                  hipStream_t);

}  // namespace flp

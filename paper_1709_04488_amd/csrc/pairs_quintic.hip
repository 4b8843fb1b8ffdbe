// Pair kernels instantiated for the quintic spline (R = 3).
#include "pairs.hpp"

namespace sph {

template void launch_density<SPH_KERNEL_QUINTIC>(hipStream_t, int, int, unsigned, const Batch<DensArgs> &);
template void launch_forces<SPH_KERNEL_QUINTIC>(hipStream_t, int, int, bool, bool, unsigned,
                                  const Batch<ForceArgs> &);
template void launch_neighbours<SPH_KERNEL_QUINTIC>(hipStream_t, int, unsigned, const NgbArgs &, int);
template void launch_mfv<SPH_KERNEL_QUINTIC>(hipStream_t, int, unsigned, const MfvArgs &);

} // namespace sph

// Pair kernels instantiated for the M4 cubic spline (R = 2).
#include "pairs.hpp"

namespace sph {

template void launch_density<SPH_KERNEL_M4>(hipStream_t, int, int, unsigned, const Batch<DensArgs> &);
template void launch_forces<SPH_KERNEL_M4>(hipStream_t, int, int, bool, bool, unsigned,
                                  const Batch<ForceArgs> &);
template void launch_neighbours<SPH_KERNEL_M4>(hipStream_t, int, unsigned, const NgbArgs &, int);
template void launch_mfv<SPH_KERNEL_M4>(hipStream_t, int, unsigned, const MfvArgs &);

} // namespace sph

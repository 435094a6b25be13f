// Instantiation unit: sparse-row LDS table walk kernels, mode WALK_ALL.
#include "parem_walk_kernels.h"

namespace parem {
template void launch_walk_family<PAREM_LAYOUT_SPARSE_LDS, WALK_ALL>(const DeviceDfa &, const PlainPlan &, const WalkArgs &,
                                                            hipStream_t, bool);
}  // namespace parem

// Instantiation unit: batched walk kernels with 64-byte staged tiles, whole speculated sets.
#include "parem_batch_kernels.h"

namespace parem {
WalkKernel batch_walk_kernel_64(uint32_t G, int kind) { return walk_kernel_tile<64, WALK_ALL>(G, kind); }
}  // namespace parem

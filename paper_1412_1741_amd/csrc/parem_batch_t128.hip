// Instantiation unit: batched walk kernels with 128-byte staged tiles, whole speculated sets.
#include "parem_batch_kernels.h"

namespace parem {
WalkKernel batch_walk_kernel_128(uint32_t G, int kind) { return walk_kernel_tile<128, WALK_ALL>(G, kind); }
}  // namespace parem

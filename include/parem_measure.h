/*
 * parem_measure.h - measurement helpers of libparem.so (not part of the
 * method): the HBM read ceiling the walk kernels are compared against.
 *
 * The paper evaluates its matcher by execution time over input sizes
 * (Section IV); the walk here is a streaming pass over the text, so its
 * bound is the rate at which one GPU can read device memory. This call
 * measures that rate on the same bytes with plain coalesced 16-byte loads.
 */
#ifndef PAREM_MEASURE_H
#define PAREM_MEASURE_H

#include <stdint.h>

#include "parem.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Read `len` bytes at d_buf (device, 16-byte aligned, len a multiple of 16)
 * once with 16-byte loads (a grid of 8 workgroups of 256 threads per compute
 * unit, four loads in flight per thread) and write the XOR of all words to
 * *d_sink (device u32), so that the reads are not removed. Asynchronous on
 * `stream`. PAREM_EINVAL for misaligned or empty input.
 */
parem_status parem_read_sweep(const uint8_t *d_buf, uint64_t len, void *stream, uint32_t *d_sink);

#ifdef __cplusplus
}
#endif

#endif /* PAREM_MEASURE_H */

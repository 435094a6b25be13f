// Batched walk kernel (persistent, work-item queue) and the structures the
// batch kernels read. Its instantiations are split by staged tile size over
// two translation units that compile in parallel.
#pragma once

#include "parem_device.h"

namespace parem {

// one pair as the batch kernels read it
struct BatchPair {
    WalkArgs w;  // w.text is unused: a run's texts come from its pointer array
    const void *table;
    uint32_t table_bytes;
    uint32_t start;
    const uint16_t *full;  // hot-row layout: the whole table and the state encoding
    const uint16_t *enc;
    uint32_t hot_rows;
    KgParams kg;
    ComposeArgs ca;
    SegOut seg[2];  // ping-pong segment buffers
    parem_result *out;
    LookArgs la;    // lookback sets (la.K == 0: Algorithm 1's sets); la.text unused
};

struct LookItem {
    uint32_t pair;
    uint32_t quad;  // chunks 4 * quad ... 4 * quad + 3 of the pair
};

struct WalkItem {
    uint32_t pair;
    uint32_t blk;  // chunks blk * 256 ... of the pair
};

struct ComposeItem {
    uint32_t pair;
    uint32_t last;  // 1: the pair's last level (writes its result)
    uint64_t seg;
    uint64_t nin;   // maps of the pair at the previous level
};

// walk kernel variants: the table layout of the pairs they serve
enum BatchKind : int {
    BK_BYTE_LDS = 0,
    BK_BYTE_GLOBAL = 1,
    BK_KGRAM1 = 2,
    BK_KGRAM2 = 3,
    BK_KGRAM3 = 4,
    BK_HOT = 5,
    BK_CLASS = 6
};

template <int G, uint32_t TILE, int KIND, int MODE>
__global__ __launch_bounds__(kWalkThreads, (G <= 8 ? 4 : 2)) void k_batch_walk(
    const BatchPair *__restrict__ pairs, const uint8_t *const *__restrict__ texts, const WalkItem *__restrict__ items,
    uint32_t nitems, uint32_t *__restrict__ queue, uint32_t table_cap) {
    // no static LDS: the k-gram stepper addresses its table as the start of
    // the dynamic LDS; the queue slot sits after the staging area
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t &s_next = *reinterpret_cast<uint32_t *>(smem + table_cap + Stage<TILE>::kBytes);
    uint32_t staged = 0xffffffffu;
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(s_next);
        // every lane has read s_next, and every wave has left the previous
        // item (its table and staging area are free)
        __syncthreads();
        if (it >= nitems) break;
        const uint32_t pi = __builtin_amdgcn_readfirstlane(items[it].pair);
        const uint64_t c0 = (uint64_t)__builtin_amdgcn_readfirstlane(items[it].blk) * kWalkThreads;
        const BatchPair &bp = pairs[pi];
        WalkArgs a = bp.w;
        a.text = texts[pi];  // with MODE == WALK_SELECTED, a.sel / a.nsel hold the lookback sets
        if constexpr (KIND != BK_BYTE_GLOBAL) {
            if (pi != staged) {
                stage_table(reinterpret_cast<uint4 *>(smem), reinterpret_cast<const uint4 *>(bp.table),
                            bp.table_bytes / 16u);
                staged = pi;
            }
        }
        if constexpr (KIND == BK_BYTE_LDS) {
            ByteStep<uint8_t, kByteLdsRow> st{smem};
            walk_chunk<G, ByteStep<uint8_t, kByteLdsRow>, true, TILE, MODE>(st, a, smem + table_cap, c0);
        } else if constexpr (KIND == BK_BYTE_GLOBAL) {
            ByteStep<uint16_t, 256> st{reinterpret_cast<const uint16_t *>(bp.table)};
            walk_chunk<G, ByteStep<uint16_t, 256>, true, TILE, MODE>(st, a, smem, c0);
        } else if constexpr (KIND == BK_CLASS) {
            ClassStep st{smem, reinterpret_cast<const uint16_t *>(smem + 256), bp.w.start_class};  // A + 1
            walk_chunk<G, ClassStep, true, TILE, MODE>(st, a, smem + table_cap, c0);
        } else if constexpr (KIND == BK_HOT) {
            const uint16_t *hot = reinterpret_cast<const uint16_t *>(smem);
            HotStep st{hot, hot + (bp.hot_rows + 1) * kHotRow, bp.full, bp.enc, bp.hot_rows};
            walk_chunk<G, HotStep, true, TILE, MODE>(st, a, smem + table_cap, c0);
        } else {
            KgStep<KIND - 1> st{smem, bp.kg};
            walk_chunk<G, KgStep<KIND - 1>, true, TILE, MODE>(st, a, smem + table_cap, c0);
        }
    }
}

using WalkKernel = void (*)(const BatchPair *, const uint8_t *const *, const WalkItem *, uint32_t, uint32_t *,
                            uint32_t);

template <int G, uint32_t TILE, int MODE>
WalkKernel walk_kernel_kind(int kind) {
    switch (kind) {
        case BK_BYTE_LDS: return k_batch_walk<G, TILE, BK_BYTE_LDS, MODE>;
        case BK_BYTE_GLOBAL: return k_batch_walk<G, TILE, BK_BYTE_GLOBAL, MODE>;
        case BK_KGRAM1: return k_batch_walk<G, TILE, BK_KGRAM1, MODE>;
        case BK_KGRAM2: return k_batch_walk<G, TILE, BK_KGRAM2, MODE>;
        case BK_KGRAM3: return k_batch_walk<G, TILE, BK_KGRAM3, MODE>;
        case BK_CLASS: return k_batch_walk<G, TILE, BK_CLASS, MODE>;
        default: return k_batch_walk<G, TILE, BK_HOT, MODE>;
    }
}

template <uint32_t TILE, int MODE>
WalkKernel walk_kernel_tile(uint32_t G, int kind) {
    switch (G) {
        case 4: return walk_kernel_kind<4, TILE, MODE>(kind);
        case 8: return walk_kernel_kind<8, TILE, MODE>(kind);
        default: return walk_kernel_kind<16, TILE, MODE>(kind);
    }
}

// defined in the per-(tile, mode) translation units
WalkKernel batch_walk_kernel_64(uint32_t G, int kind);
WalkKernel batch_walk_kernel_128(uint32_t G, int kind);
WalkKernel batch_walk_kernel_64_sel(uint32_t G, int kind);
WalkKernel batch_walk_kernel_128_sel(uint32_t G, int kind);

}  // namespace parem

// Walk kernels of one text and their launchers. The instantiations are
// spread over several translation units (one per table family and walk
// mode) so that they compile in parallel; each includes this header and
// instantiates launch_walk_family for its pair of template arguments.
#pragma once

#include "parem_device.h"

namespace parem {

// Walk modes other than WALK_ALL (learned selection, re-walk) lock-step 8 or
// 16 walks; WALK_ALL offers every group size.
#define PAREM_GROUP_SWITCH(X)                                 \
    if constexpr (MODE == WALK_ALL) {                         \
        switch (p.G) {                                        \
            case 2: X(2); break;                              \
            case 4: X(4); break;                              \
            case 8: X(8); break;                              \
            default: X(16); break;                            \
        }                                                     \
    } else {                                                  \
        if (p.G <= 8) X(8);                                   \
        else X(16);                                           \
    }

// at least 4 waves per SIMD (at most 128 VGPRs) for groups up to 8 walks
template <typename E, uint32_t ROW, int G, bool LDS_TABLE, bool ALIGNED, uint32_t TILE, int MODE>
__global__ __launch_bounds__(kWalkThreads, (G <= 8 ? 4 : 2)) void k_walk_byte(WalkArgs a, const E *__restrict__ g_table,
                                                                              uint32_t table_bytes) {
    extern __shared__ __align__(16) uint8_t smem[];
    ByteStep<E, ROW> st{g_table};
    uint32_t tb = 0;
    if constexpr (LDS_TABLE) {
        stage_table(reinterpret_cast<uint4 *>(smem), reinterpret_cast<const uint4 *>(g_table), table_bytes / 16u);
        st.T = reinterpret_cast<const E *>(smem);
        tb = table_bytes;
    }
    walk_chunk<G, ByteStep<E, ROW>, ALIGNED, TILE, MODE>(st, a, smem + tb, (uint64_t)xcd_block() * kWalkThreads);
}

template <int G, bool ALIGNED, uint32_t TILE, int MODE>
__global__ __launch_bounds__(kWalkThreads, (G <= 8 ? 4 : 2)) void k_walk_hot(WalkArgs a, const uint8_t *__restrict__ g_table,
                                                                             uint32_t table_bytes, uint32_t hot_rows,
                                                                             const uint16_t *__restrict__ full,
                                                                             const uint16_t *__restrict__ enc) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table(reinterpret_cast<uint4 *>(smem), reinterpret_cast<const uint4 *>(g_table), table_bytes / 16u);
    const uint16_t *hot = reinterpret_cast<const uint16_t *>(smem);
    HotStep st{hot, hot + (hot_rows + 1) * kHotRow, full, enc, hot_rows};
    walk_chunk<G, HotStep, ALIGNED, TILE, MODE>(st, a, smem + table_bytes, (uint64_t)xcd_block() * kWalkThreads);
}

template <int G, bool ALIGNED, uint32_t TILE, int MODE>
__global__ __launch_bounds__(kWalkThreads, (G <= 8 ? 4 : 2)) void k_walk_class(WalkArgs a,
                                                                               const uint8_t *__restrict__ g_table,
                                                                               uint32_t table_bytes, uint32_t A1) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table(reinterpret_cast<uint4 *>(smem), reinterpret_cast<const uint4 *>(g_table), table_bytes / 16u);
    ClassStep st{smem, reinterpret_cast<const uint16_t *>(smem + 256), A1};
    walk_chunk<G, ClassStep, ALIGNED, TILE, MODE>(st, a, smem + table_bytes, (uint64_t)xcd_block() * kWalkThreads);
}

// one workgroup of kSparseThreads per CU: four waves per SIMD
template <int G, bool ALIGNED, int MODE, bool RAW, bool UNI>
__global__ __launch_bounds__(kSparseThreads) void k_walk_sparse(WalkArgs a, const uint8_t *__restrict__ g_table,
                                                                uint32_t table_bytes,
                                                                const uint16_t *__restrict__ sids, uint32_t d0) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table<kSparseThreads>(reinterpret_cast<uint4 *>(smem), reinterpret_cast<const uint4 *>(g_table),
                                table_bytes / 16u);
    SparseStep<RAW, UNI> st{smem, sids, d0};
    walk_chunk<G, SparseStep<RAW, UNI>, ALIGNED, 64, MODE>(st, a, smem + table_bytes,
                                                           (uint64_t)xcd_block() * kSparseThreads);
}

template <int G, int B, bool ALIGNED, uint32_t TILE, int MODE>
__global__ __launch_bounds__(kWalkThreads, (G <= 8 ? 4 : 2)) void k_walk_kgram(WalkArgs a,
                                                                               const uint8_t *__restrict__ g_table,
                                                                               uint32_t table_bytes, KgParams kp) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table(reinterpret_cast<uint4 *>(smem), reinterpret_cast<const uint4 *>(g_table), table_bytes / 16u);
    KgStep<B> st{smem, kp};
    walk_chunk<G, KgStep<B>, ALIGNED, TILE, MODE>(st, a, smem + table_bytes, (uint64_t)xcd_block() * kWalkThreads);
}

template <typename E, uint32_t ROW, bool LDS, bool ALIGNED, uint32_t TILE, int MODE>
inline void launch_walk_byte(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const size_t lds = (LDS ? d.table_bytes : 0) + ((ALIGNED && MODE != WALK_REDO) ? Stage<TILE>::kBytes : 0);
    const E *tab = reinterpret_cast<const E *>(d.d_table);
#define PAREM_WALK(GG)                                                                                            \
    hipLaunchKernelGGL((k_walk_byte<E, ROW, GG, LDS, ALIGNED, TILE, MODE>), dim3(grid), dim3(kWalkThreads), lds, \
                       stream, a, tab, d.table_bytes)
    PAREM_GROUP_SWITCH(PAREM_WALK)
#undef PAREM_WALK
}

template <int B, bool ALIGNED, uint32_t TILE, int MODE>
inline void launch_kgram_b(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const size_t lds = d.table_bytes + ((ALIGNED && MODE != WALK_REDO) ? Stage<TILE>::kBytes : 0);
    const uint8_t *tab = reinterpret_cast<const uint8_t *>(d.d_table);
#define PAREM_KG(GG)                                                                                              \
    hipLaunchKernelGGL((k_walk_kgram<GG, B, ALIGNED, TILE, MODE>), dim3(grid), dim3(kWalkThreads), lds, stream, a, \
                       tab, d.table_bytes, d.kg)
    PAREM_GROUP_SWITCH(PAREM_KG)
#undef PAREM_KG
}

template <bool ALIGNED, uint32_t TILE, int MODE>
inline void launch_walk_hot(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const size_t lds = d.table_bytes + ((ALIGNED && MODE != WALK_REDO) ? Stage<TILE>::kBytes : 0);
    const uint8_t *tab = reinterpret_cast<const uint8_t *>(d.d_table);
#define PAREM_HOT(GG)                                                                                           \
    hipLaunchKernelGGL((k_walk_hot<GG, ALIGNED, TILE, MODE>), dim3(grid), dim3(kWalkThreads), lds, stream, a, tab, \
                       d.table_bytes, d.hot_rows, d.d_full, d.d_enc)
    PAREM_GROUP_SWITCH(PAREM_HOT)
#undef PAREM_HOT
}

template <bool ALIGNED, uint32_t TILE, int MODE>
inline void launch_walk_class(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const size_t lds = d.table_bytes + ((ALIGNED && MODE != WALK_REDO) ? Stage<TILE>::kBytes : 0);
    const uint8_t *tab = reinterpret_cast<const uint8_t *>(d.d_table);
#define PAREM_CLS(GG)                                                                                             \
    hipLaunchKernelGGL((k_walk_class<GG, ALIGNED, TILE, MODE>), dim3(grid), dim3(kWalkThreads), lds, stream, a, tab, \
                       d.table_bytes, d.A + 1)
    PAREM_GROUP_SWITCH(PAREM_CLS)
#undef PAREM_CLS
}

// the table, then (aligned texts) a 64-byte text tile per wave
template <bool ALIGNED, int MODE, bool RAW, bool UNI>
inline void launch_walk_sparse_t(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kSparseThreads - 1) / kSparseThreads);
    using SG = Stage<64, SparseStep<RAW, UNI>::kSwizzle>;
    static_assert(kSparseLdsMax + (kSparseThreads / 64) * SG::kWave <= 160 * 1024, "slots and tiles exceed LDS");
    const size_t lds = d.table_bytes + ((ALIGNED && MODE != WALK_REDO) ? (kSparseThreads / 64) * SG::kWave : 0);
    const uint8_t *tab = reinterpret_cast<const uint8_t *>(d.d_table);
#define PAREM_SPR(GG)                                                                                           \
    hipLaunchKernelGGL((k_walk_sparse<GG, ALIGNED, MODE, RAW, UNI>), dim3(grid), dim3(kSparseThreads), lds, stream, \
                       a, tab, d.table_bytes, d.d_sids, d.sparse_d0)
    PAREM_GROUP_SWITCH(PAREM_SPR)
#undef PAREM_SPR
}

template <bool ALIGNED, int MODE>
inline void launch_walk_sparse(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    if (d.sparse_raw) {
        if (d.sparse_uniform) launch_walk_sparse_t<ALIGNED, MODE, true, true>(d, p, a, stream);
        else launch_walk_sparse_t<ALIGNED, MODE, true, false>(d, p, a, stream);
    } else {
        if (d.sparse_uniform) launch_walk_sparse_t<ALIGNED, MODE, false, true>(d, p, a, stream);
        else launch_walk_sparse_t<ALIGNED, MODE, false, false>(d, p, a, stream);
    }
}

template <int LAYOUT, bool ALIGNED, uint32_t TILE, int MODE>
inline void launch_family_t(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    if constexpr (LAYOUT == PAREM_LAYOUT_KGRAM_LDS) {
        switch (d.kg.bits) {
            case 1: launch_kgram_b<1, ALIGNED, TILE, MODE>(d, p, a, stream); break;
            case 2: launch_kgram_b<2, ALIGNED, TILE, MODE>(d, p, a, stream); break;
            default: launch_kgram_b<3, ALIGNED, TILE, MODE>(d, p, a, stream); break;
        }
    } else if constexpr (LAYOUT == PAREM_LAYOUT_BYTE_LDS) {
        launch_walk_byte<uint8_t, kByteLdsRow, true, ALIGNED, TILE, MODE>(d, p, a, stream);
    } else if constexpr (LAYOUT == PAREM_LAYOUT_HOT_LDS) {
        launch_walk_hot<ALIGNED, TILE, MODE>(d, p, a, stream);
    } else if constexpr (LAYOUT == PAREM_LAYOUT_CLASS_LDS) {
        launch_walk_class<ALIGNED, TILE, MODE>(d, p, a, stream);
    } else if constexpr (LAYOUT == PAREM_LAYOUT_SPARSE_LDS) {
        launch_walk_sparse<ALIGNED, MODE>(d, p, a, stream);
    } else {
        launch_walk_byte<uint16_t, 256, false, ALIGNED, TILE, MODE>(d, p, a, stream);
    }
}

// one table layout and walk mode
template <int LAYOUT, int MODE>
void launch_walk_family(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream,
                        bool aligned) {
    if constexpr (LAYOUT == PAREM_LAYOUT_SPARSE_LDS) {
        // no staged tiles: the tile size does not matter
        if (aligned) launch_family_t<LAYOUT, true, 64, MODE>(d, p, a, stream);
        else launch_family_t<LAYOUT, false, 64, MODE>(d, p, a, stream);
        return;
    }
    if (!aligned) launch_family_t<LAYOUT, false, 64, MODE>(d, p, a, stream);
    else if (p.tile == 128 || MODE == WALK_REDO) launch_family_t<LAYOUT, true, 128, MODE>(d, p, a, stream);
    else launch_family_t<LAYOUT, true, 64, MODE>(d, p, a, stream);
}

#undef PAREM_GROUP_SWITCH

}  // namespace parem

// Device building blocks of the speculative chunked DFA walk, shared by the
// single-text kernels and the batched persistent kernels: table steppers,
// the per-lane chunk walk with LDS-staged text tiles, and the per-segment
// composition of chunk maps.
#pragma once

#include "parem_internal.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace parem {


constexpr int kWalkThreads = 256;
// the sparse-row walk: one 1024-thread workgroup per CU, four waves per SIMD
// (measured: a second workgroup per CU does not become resident, and a
// register cap for more waves spills)
constexpr int kSparseThreads = 1024;
constexpr int kComposeThreads = 256;
// Workgroups are dealt to the eight XCDs in turn (workgroup b to XCD b % 8).
// xcd_block() renumbers them so that XCD x takes the x-th eighth of the
// grid's range (the first n % 8 XCDs one workgroup more): each XCD then
// streams one contiguous part of the text instead of every eighth 2 MiB
// block (1 GiB: the k-gram walk 199 -> 177 us; a plain read 6.15 -> 6.88 TB/s).
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t n = gridDim.x, b = blockIdx.x, q = n / 8u, r = n % 8u, x = b % 8u;
    return x * q + min(x, r) + b / 8u;
}

// A staged tile holds TILE bytes of each of a wave's 64 chunks. Rows are
// TILE + 16 bytes apart so that 8 consecutive lanes' 16-byte reads hit
// distinct banks; or, SWZ, TILE = 64 bytes apart with the 16-byte pieces of
// row r stored in the order piece ^ ((r >> 1) & 3), which spreads the same
// reads over the banks without the padding.
template <uint32_t TILE, bool SWZ = false>
struct Stage {
    static_assert(!SWZ || TILE == 64, "the swizzle permutes four pieces");
    static constexpr uint32_t kRow = SWZ ? TILE : TILE + 16;
    static constexpr uint32_t kWave = 64 * kRow;
    static constexpr uint32_t kBytes = (kWalkThreads / 64) * kWave;
    static constexpr uint32_t kPieces = TILE / 16;      // 16-byte loads per lane per tile
    static constexpr uint32_t kChunksPerLoad = 64 / kPieces;
    // byte offset of piece k within row r
    static __device__ __forceinline__ uint32_t piece_at(uint32_t r, uint32_t k) {
        return 16u * (SWZ ? (k ^ ((r >> 1) & 3u)) : k);
    }
};

// u16 at LDS byte address `addr`. The k-gram walk kernels declare no static
// LDS, so their dynamic LDS (the table first) starts at address 0 and a table
// offset is an LDS address: the read needs no base addition.
__device__ __forceinline__ uint32_t lds_u16_abs(uint32_t addr) {
    return *reinterpret_cast<const __attribute__((address_space(3))) uint16_t *>(static_cast<uintptr_t>(addr));
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// T (a scalar or ext_vector_type) at LDS byte address `addr`
template <typename T>
__device__ __forceinline__ T lds_abs(uint32_t addr) {
    return *reinterpret_cast<const __attribute__((address_space(3))) T *>(static_cast<uintptr_t>(addr));
}

__device__ __forceinline__ uint32_t lds_u16(const uint8_t *base, uint32_t byte_off) {
    return *reinterpret_cast<const uint16_t *>(base + byte_off);
}

// ---------------------------------------------------------------------------
// steppers: how one walk advances over 4 bytes / 1 byte
// ---------------------------------------------------------------------------

// Byte table with ROW entries per state row. A row stride that is not a
// multiple of the LDS bank width spreads the rows of different states over
// different banks (rows of 256 one-byte entries would all start on bank 0).
template <typename E, uint32_t ROW>
struct ByteStep {
    static constexpr bool kRedo = false;  // pieces never need a second pass
    // byte-at-a-time tables serve large speculated sets: many short passes,
    // which share one load of the chunk's first 64 bytes
    static constexpr bool kPrefixPasses = true;
    static constexpr bool kStage = true;   // text staged through LDS when aligned
    static constexpr uint32_t kAcc = sizeof(E) * 8 - 1;
    static constexpr uint32_t kMask = (1u << kAcc) - 1u;
    const E *__restrict__ T;

    __device__ __forceinline__ uint32_t init(uint32_t s) const { return s; }
    __device__ __forceinline__ uint32_t id(uint32_t r) const { return r; }
    __device__ __forceinline__ bool same(uint32_t a, uint32_t b) const { return a == b; }
    __device__ __forceinline__ void one(uint32_t &s, uint32_t &c, uint32_t byte) const {
        const uint32_t v = T[s * ROW + byte];
        c += v >> kAcc;
        s = v & kMask;
    }
    template <int G>
    __device__ __forceinline__ void dword(uint32_t d, uint32_t (&R)[G], uint32_t (&S)[G], uint32_t (&c)[G], int nw,
                                          uint32_t &bad) const {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t byte = (d >> (8 * k)) & 0xffu;
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (j < nw) one(R[j], c[j], byte);
        }
    }
    template <int G>
    __device__ __forceinline__ void flush(uint32_t (&S)[G], uint32_t (&c)[G], int nw) const {}
    __device__ __forceinline__ void byte(uint32_t x, uint32_t &R, uint32_t &c, uint32_t &bad) const {
        one(R, c, x);
    }
};

// Column-indexed table in LDS: byte -> column through a 256-entry map (one
// read per byte, shared by the lane's walks), then entry (state, column) =
// next | final << 15. Column A sends every state to the sentinel (invalid
// bytes); the sentinel row stays in the sentinel.
struct ClassStep {
    static constexpr bool kRedo = false;
    static constexpr bool kPrefixPasses = true;
    static constexpr bool kStage = true;   // text staged through LDS when aligned
    const uint8_t *__restrict__ col;   // LDS: [256]
    const uint16_t *__restrict__ T;    // LDS: (Q+1) x (A+1)
    uint32_t A1;                       // A + 1

    __device__ __forceinline__ uint32_t init(uint32_t s) const { return s; }
    __device__ __forceinline__ uint32_t id(uint32_t r) const { return r; }
    __device__ __forceinline__ bool same(uint32_t a, uint32_t b) const { return a == b; }
    __device__ __forceinline__ void one(uint32_t &s, uint32_t &c, uint32_t cl) const {
        const uint32_t v = T[s * A1 + cl];
        c += v >> 15;
        s = v & 0x7fffu;
    }
    template <int G>
    __device__ __forceinline__ void dword(uint32_t d, uint32_t (&R)[G], uint32_t (&S)[G], uint32_t (&c)[G], int nw,
                                          uint32_t &bad) const {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t cl = col[(d >> (8 * k)) & 0xffu];
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (j < nw) one(R[j], c[j], cl);
        }
    }
    template <int G>
    __device__ __forceinline__ void flush(uint32_t (&S)[G], uint32_t (&c)[G], int nw) const {}
    __device__ __forceinline__ void byte(uint32_t x, uint32_t &R, uint32_t &c, uint32_t &bad) const {
        one(R, c, col[x]);
    }
};

// Sparse rows: per state a default entry and four (column, entry)
// exceptions in 16 bytes of LDS (entry = next | final << 15; unused slots
// repeat a column with its own entry). A step is one 16-byte LDS read and
// four column compares. The table leaves room for two workgroups per CU only
// without the text staging area, so lanes load their chunks 16 bytes at a
// time themselves (the lines stay in L2 between a lane's loads).
// Sparse layout: the table's rows displaced into one vector of u32 slots.
// The slot at row base b + k holds the step on key k (a byte when every
// byte is valid, RAW, else the byte's column) when its key field is k;
// otherwise the step takes the default. Two forms:
//
// UNI (every row shares one default): the walk's state is the row's base
// (bits 0-15) with the state's final flag in bits 16-23 (bits 24-31 carry
// whatever key led there and are ignored). A slot holds the next state's
// value in bits 0-23 and its key in bits 24-31; the default's value is a
// kernel argument. A step is one LDS read, a compare, a select and the
// count's add.
//
// General: the state is the base; the slot's key is its high half, and the
// header slot b + 256 holds the row's own default (low half) and the final
// flag of the row's state (bits 16-23). A step is two independent LDS reads
// (slot and header), a compare, a select and the count's add.
//
// The add of the base and the key takes the byte straight out of the text
// dword, and the compare and the select take their fields straight out of
// the slots (SDWA operand selects, written out below because the compiler
// extracts them with extra instructions). The count takes the flag of the
// state a step leaves, so it is shifted by one step: it starts at minus the
// start state's flag and the end state's flag is added when the walk is
// stored (kDeferredCount).
//
// KSEL selects the byte of `key` used (BYTE_k of a text dword, or DWORD for a
// column). A VALU write of VCC needs two wait states before v_cndmask reads
// it: the count's add and one s_nop.
#define PAREM_SPARSE_KEYADD(KSEL)                                                                      \
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:" KSEL " src1_sel:WORD_0" \
        : "=v"(u)                                                                                      \
        : "v"(key), "v"(s))
#define PAREM_SPARSE_STEP(KSEL)                                                                                  \
    asm("v_cmp_eq_u32_sdwa vcc, %2, %3 src0_sel:WORD_1 src1_sel:" KSEL "\n\t"                                  \
        "v_add_u32_sdwa %1, %1, %4 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2\n\t"       \
        "s_nop 0\n\t"                                                                                            \
        "v_cndmask_b32_sdwa %0, %4, %2, vcc dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:WORD_0" \
        : "=&v"(v), "+v"(c)                                                                                      \
        : "v"(e), "v"(key), "v"(h)                                                                               \
        : "vcc")
#define PAREM_SPARSE_STEP_UNI(KSEL)                                                                        \
    asm("v_cmp_eq_u32_sdwa vcc, %2, %3 src0_sel:BYTE_3 src1_sel:" KSEL "\n\t"                            \
        "v_add_u32_sdwa %1, %1, %4 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2\n\t" \
        "s_nop 0\n\t"                                                                                      \
        "v_cndmask_b32_e32 %0, %5, %2, vcc"                                                                \
        : "=&v"(v), "+v"(c)                                                                                \
        : "v"(e), "v"(key), "v"(s), "v"(d0)                                                                \
        : "vcc")

template <bool RAW, bool UNI>
struct SparseStep {
    static constexpr bool kRedo = false;
    static constexpr bool kPrefixPasses = true;
    static constexpr bool kStage = true;   // text staged through LDS when aligned (64-byte tiles)
    static constexpr bool kCachedText = true;
    static constexpr bool kDeferredCount = true;
    static constexpr bool kSwizzle = true;  // unpadded tiles: the slots take the LDS
    // The kernel declares no static LDS: its dynamic LDS (the byte -> column
    // map, then the slots) starts at LDS address 0, so kSlots + 4 * slot is
    // the slot's LDS address.
    static constexpr uint32_t kSlots = 256;
    static constexpr uint32_t kHeads = kSlots + 4 * kSparseHead;
    const uint8_t *__restrict__ col;    // LDS: [256] byte -> column (unused when RAW)
    const uint16_t *__restrict__ sids;  // global: state of the row based at each slot
    uint32_t d0;                        // UNI: the default's value

    // walks start from the lists of walk values
    __device__ __forceinline__ uint32_t init(uint32_t s) const { return s; }
    __device__ __forceinline__ uint32_t id(uint32_t r) const { return sids[r & 0xffffu]; }
    __device__ __forceinline__ bool same(uint32_t a, uint32_t b) const {
        if constexpr (UNI) return ((a ^ b) & 0xffffu) == 0;
        else return a == b;
    }
    __device__ __forceinline__ uint32_t fin(uint32_t r) const {
        if constexpr (UNI) return (r >> 16) & 0xffu;
        else return (lds_abs<uint32_t>(kHeads + 4u * r) >> 16) & 0xffu;
    }
    // K = 0..3: the key is byte K of `key` (a text dword); K = 4: `key` is a column
    template <int K>
    __device__ __forceinline__ void one(uint32_t &s, uint32_t &c, uint32_t key) const {
        uint32_t u, v;
        if constexpr (K == 0) PAREM_SPARSE_KEYADD("BYTE_0");
        else if constexpr (K == 1) PAREM_SPARSE_KEYADD("BYTE_1");
        else if constexpr (K == 2) PAREM_SPARSE_KEYADD("BYTE_2");
        else if constexpr (K == 3) PAREM_SPARSE_KEYADD("BYTE_3");
        else PAREM_SPARSE_KEYADD("DWORD");
        const uint32_t e = lds_abs<uint32_t>(kSlots + 4u * u);
        if constexpr (UNI) {
            if constexpr (K == 0) PAREM_SPARSE_STEP_UNI("BYTE_0");
            else if constexpr (K == 1) PAREM_SPARSE_STEP_UNI("BYTE_1");
            else if constexpr (K == 2) PAREM_SPARSE_STEP_UNI("BYTE_2");
            else if constexpr (K == 3) PAREM_SPARSE_STEP_UNI("BYTE_3");
            else PAREM_SPARSE_STEP_UNI("DWORD");
        } else {
            const uint32_t h = lds_abs<uint32_t>(kHeads + 4u * s);
            if constexpr (K == 0) PAREM_SPARSE_STEP("BYTE_0");
            else if constexpr (K == 1) PAREM_SPARSE_STEP("BYTE_1");
            else if constexpr (K == 2) PAREM_SPARSE_STEP("BYTE_2");
            else if constexpr (K == 3) PAREM_SPARSE_STEP("BYTE_3");
            else PAREM_SPARSE_STEP("DWORD");
        }
        s = v;
    }
    template <int K, int G>
    __device__ __forceinline__ void byte_of(uint32_t d, uint32_t (&R)[G], uint32_t (&c)[G], int nw) const {
        if constexpr (RAW) {
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (j < nw) one<K>(R[j], c[j], d);
        } else {
            const uint32_t cl = col[(d >> (8 * K)) & 0xffu];
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (j < nw) one<4>(R[j], c[j], cl);
        }
    }
    template <int G>
    __device__ __forceinline__ void dword(uint32_t d, uint32_t (&R)[G], uint32_t (&S)[G], uint32_t (&c)[G], int nw,
                                          uint32_t &bad) const {
        byte_of<0, G>(d, R, c, nw);
        byte_of<1, G>(d, R, c, nw);
        byte_of<2, G>(d, R, c, nw);
        byte_of<3, G>(d, R, c, nw);
    }
    template <int G>
    __device__ __forceinline__ void flush(uint32_t (&S)[G], uint32_t (&c)[G], int nw) const {}
    __device__ __forceinline__ void byte(uint32_t x, uint32_t &R, uint32_t &c, uint32_t &bad) const {
        if constexpr (RAW) one<0>(R, c, x);
        else one<4>(R, c, (uint32_t)col[x]);
    }
};
#undef PAREM_SPARSE_KEYADD
#undef PAREM_SPARSE_STEP
#undef PAREM_SPARSE_STEP_UNI

// Hot-row layout: the byte-table rows of the H most visited states sit in
// LDS, the other rows are read through L2. A walk carries its state encoded:
// the slot (0..H-1) of a hot state, kHotFlag | id for a cold one; every
// entry holds the encoded destination plus the final flag in bit 15.
// Sixteen bytes are first stepped through LDS alone (row min(state, H); row
// H is all kHotLost, so a walk that leaves the hot rows stays marked); a
// lane whose walks did not all stay hot steps the same sixteen bytes again
// from the saved states with the global rows for cold states.
struct HotStep {
    static constexpr bool kRedo = true;
    static constexpr bool kPrefixPasses = true;
    static constexpr bool kStage = true;   // text staged through LDS when aligned
    const uint16_t *__restrict__ hot;   // LDS: H + 1 rows of kHotRow entries
    const uint16_t *__restrict__ ids;   // LDS: state id of each hot slot
    const uint16_t *__restrict__ full;  // global: (Q+1) x 256 entries
    const uint16_t *__restrict__ enc;   // global: encoded id of each state (unused by the walk)
    uint32_t H;

    // walks start from the encoded lists
    __device__ __forceinline__ uint32_t init(uint32_t s) const { return s; }
    __device__ __forceinline__ uint32_t id(uint32_t r) const { return r < H ? ids[r] : (r & 0x3fffu); }
    __device__ __forceinline__ bool same(uint32_t a, uint32_t b) const { return a == b; }
    __device__ __forceinline__ void fast(uint32_t &s, uint32_t &c, uint32_t byte) const {
        const uint32_t v = hot[min(s, H) * kHotRow + byte];
        c += v >> 15;
        s = v & 0x7fffu;
    }
    __device__ __forceinline__ void one(uint32_t &s, uint32_t &c, uint32_t byte) const {
        uint32_t v;
        if (s < H) v = hot[s * kHotRow + byte];
        else v = full[(s & 0x3fffu) * 256u + byte];
        c += v >> 15;
        s = v & 0x7fffu;
    }
    template <int G>
    __device__ __forceinline__ void step16(const uint4 q, uint32_t (&R)[G], uint32_t (&c)[G], int nw) const {
        uint32_t R0[G], c0[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            R0[j] = R[j];
            c0[j] = c[j];
        }
        const uint32_t d[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (j < nw) fast(R[j], c[j], (d[k >> 2] >> (8 * (k & 3))) & 0xffu);
        }
        bool cold = false;
#pragma unroll
        for (int j = 0; j < G; ++j) cold |= j < nw && R[j] >= H;
        if (cold) {
#pragma unroll
            for (int j = 0; j < G; ++j) {
                R[j] = R0[j];
                c[j] = c0[j];
            }
#pragma unroll 1
            for (int k = 0; k < 16; ++k) {
                const uint32_t word = k < 8 ? (k < 4 ? q.x : q.y) : (k < 12 ? q.z : q.w);
                const uint32_t byte = (word >> (8 * (k & 3))) & 0xffu;
#pragma unroll
                for (int j = 0; j < G; ++j)
                    if (j < nw) one(R[j], c[j], byte);
            }
        }
    }
    __device__ __forceinline__ void byte(uint32_t x, uint32_t &R, uint32_t &c, uint32_t &bad) const {
        one(R, c, x);
    }
};

// k-gram table: a state is carried as its row base (state << RS) plus the
// count bits of the last entry read. The table must sit at LDS address 0 (the
// start of the kernel's dynamic LDS; T is that address).
template <int B>
struct KgStep {
    static constexpr bool kRedo = false;
    static constexpr bool kPrefixPasses = false;  // small alphabets: few passes
    static constexpr bool kStage = true;
    static constexpr uint32_t K = (B == 3) ? 2 : 4;   // symbols per lookup
    static constexpr uint32_t RS = K * B + 1;         // row bytes = 1 << RS
    static constexpr uint32_t LOW = (1u << RS) - 1u;  // count field
    static constexpr uint32_t ROWMASK = 0xffffu & ~LOW;
    const uint8_t *__restrict__ T;
    KgParams kp;

    __device__ __forceinline__ uint32_t init(uint32_t s) const { return s << RS; }
    __device__ __forceinline__ uint32_t id(uint32_t r) const { return (r & ROWMASK) >> RS; }
    __device__ __forceinline__ bool same(uint32_t a, uint32_t b) const { return ((a ^ b) & ROWMASK) == 0; }
    template <int G>
    __device__ __forceinline__ void dword(uint32_t d, uint32_t (&R)[G], uint32_t (&S)[G], uint32_t (&c)[G], int nw,
                                          uint32_t &bad) const {
        const uint32_t cd = (d >> kp.shift) & kp.cmask4;
        bad |= __builtin_amdgcn_perm(kp.vhi, kp.vlo, cd) ^ d;
        if constexpr (B == 3) {
            const uint32_t i0 = __builtin_amdgcn_udot4(cd, kp.w0, 0u, false);
            const uint32_t i1 = __builtin_amdgcn_udot4(cd, kp.w1, 0u, false);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (j < nw) {
                    uint32_t e = lds_u16_abs((R[j] & ROWMASK) | i0);
                    S[j] += e;
                    e = lds_u16_abs((e & ROWMASK) | i1);
                    R[j] = e;
                    S[j] += e;
                }
            }
        } else {
            const uint32_t i0 = __builtin_amdgcn_udot4(cd, kp.w0, 0u, false);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (j < nw) {
                    const uint32_t e = lds_u16_abs((R[j] & ROWMASK) | i0);
                    R[j] = e;
                    S[j] += e;
                }
            }
        }
    }
    // at most 16 final destinations per 16 bytes: the count field never overflows
    template <int G>
    __device__ __forceinline__ void flush(uint32_t (&S)[G], uint32_t (&c)[G], int nw) const {
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (j < nw) {
                c[j] += S[j] & LOW;
                S[j] = 0;
            }
        }
    }
    __device__ __forceinline__ void byte(uint32_t x, uint32_t &R, uint32_t &c, uint32_t &bad) const {
        const uint32_t code = (x >> kp.shift) & (kp.cmask4 & 0xffu);
        bad |= (__builtin_amdgcn_perm(kp.vhi, kp.vlo, code) & 0xffu) ^ x;
        const uint32_t row = (R & ROWMASK) >> RS;
        const uint32_t e = lds_u16_abs(kp.t1_off + (((row << B) | code) << 1));
        c += e & LOW;
        R = e;
    }
};

// ---------------------------------------------------------------------------
// one lane's walks over its chunk
// ---------------------------------------------------------------------------

template <int G>
struct Walks {
    uint32_t R[G], S[G], c[G];
    int32_t off[G];
    uint32_t pending;  // bit j: follower j not merged yet
    bool wave_pending;
    bool merge;        // false: runs are never merged (every run walks the whole chunk)
};

template <int G, typename ST>
__device__ __forceinline__ void merge_check(const ST &st, Walks<G> &w) {
    if (!w.merge) return;
#pragma unroll
    for (int j = 1; j < G; ++j) {
        if (((w.pending >> j) & 1u) && st.same(w.R[j], w.R[0])) {
            w.off[j] = (int32_t)(w.c[j] - w.c[0]);
            w.pending &= ~(1u << j);
        }
    }
}

// 16 bytes for every walk (while any lane of the wave has unmerged
// followers) or for the leader alone
template <int G, typename ST>
__device__ __forceinline__ void piece(const ST &st, Walks<G> &w, const uint4 q, uint32_t &bad) {
    if constexpr (ST::kRedo) {
        if (w.wave_pending) {
            st.template step16<G>(q, w.R, w.c, G);
            merge_check<G>(st, w);
            w.wave_pending = __any(w.pending != 0);
        } else {
            st.template step16<G>(q, w.R, w.c, 1);
        }
    } else if (w.wave_pending) {
        st.template dword<G>(q.x, w.R, w.S, w.c, G, bad);
        st.template dword<G>(q.y, w.R, w.S, w.c, G, bad);
        st.template dword<G>(q.z, w.R, w.S, w.c, G, bad);
        st.template dword<G>(q.w, w.R, w.S, w.c, G, bad);
        st.template flush<G>(w.S, w.c, G);
        merge_check<G>(st, w);
        w.wave_pending = __any(w.pending != 0);
    } else {
        st.template dword<G>(q.x, w.R, w.S, w.c, 1, bad);
        st.template dword<G>(q.y, w.R, w.S, w.c, 1, bad);
        st.template dword<G>(q.z, w.R, w.S, w.c, 1, bad);
        st.template dword<G>(q.w, w.R, w.S, w.c, 1, bad);
        st.template flush<G>(w.S, w.c, 1);
    }
}

// 16 text bytes at a 16-byte aligned address, loaded non-temporally: the
// text is read once, and streaming it past the caches measured 6.15 against
// 5.44 TB/s for the walk's access pattern (64 chunks of 8 KiB a wave, one
// 128-byte line per chunk a round)
__device__ __forceinline__ uint4 load16_stream(const uint8_t *p) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

template <bool ALIGNED>
__device__ __forceinline__ uint4 load16(const uint8_t *p) {
    if constexpr (ALIGNED) {
        return load16_stream(p);
    } else {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v[k] = (uint32_t)p[4 * k] | ((uint32_t)p[4 * k + 1] << 8) | ((uint32_t)p[4 * k + 2] << 16) |
                   ((uint32_t)p[4 * k + 3] << 24);
        return make_uint4(v[0], v[1], v[2], v[3]);
    }
}

// Walk index idx (0 = leader) starts in the state at list position
// pos(idx): idx itself for the whole speculated set, sel[idx] for a learned
// selection.
struct Positions {
    const uint16_t *sel;  // null: identity
    __device__ __forceinline__ uint32_t operator()(uint32_t idx) const { return sel ? (uint32_t)sel[idx] : idx; }
};

// Steppers with kCachedText = true load text tiles with ordinary loads
// (others stream them non-temporally).
template <typename ST, typename = void>
struct CachedText : std::false_type {};
template <typename ST>
struct CachedText<ST, std::void_t<decltype(ST::kCachedText)>> : std::bool_constant<ST::kCachedText> {};

// Steppers with kDeferredCount count the final flag of the state a step
// leaves: a walk's count starts at minus its start state's flag and gets its
// end state's flag when stored. Others count the state a step enters.
template <typename ST, typename = void>
struct Deferred : std::false_type {};
template <typename ST>
struct Deferred<ST, std::void_t<decltype(ST::kDeferredCount)>> : std::bool_constant<ST::kDeferredCount> {};

// Steppers with kSwizzle stage text tiles in unpadded, swizzled rows.
template <typename ST, typename = void>
struct Swizzled : std::false_type {};
template <typename ST>
struct Swizzled<ST, std::void_t<decltype(ST::kSwizzle)>> : std::bool_constant<ST::kSwizzle> {};

template <typename ST>
__device__ __forceinline__ uint32_t count_start(const ST &st, uint32_t r) {
    if constexpr (Deferred<ST>::value) return 0u - st.fin(r);
    else return 0u;
}

template <typename ST>
__device__ __forceinline__ uint32_t count_end(const ST &st, uint32_t r) {
    if constexpr (Deferred<ST>::value) return st.fin(r);
    else return 0u;
}

template <int G, typename ST>
__device__ __forceinline__ void walks_init(const ST &st, Walks<G> &w, const uint32_t *__restrict__ list,
                                           const Positions &pos, uint32_t nwalk, uint32_t first) {
    const uint32_t lead = st.init(list[pos(0)]);
    w.pending = 0;
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const uint32_t idx = first + (uint32_t)j - 1u;
        const bool real = j > 0 && idx < nwalk;
        w.R[j] = real ? st.init(list[pos(idx)]) : lead;
        w.S[j] = 0;
        w.c[j] = count_start(st, w.R[j]);
        w.off[j] = 0;
        if (real && !st.same(w.R[j], lead)) w.pending |= 1u << j;
    }
    w.wave_pending = __any(w.pending != 0);
}

// Staged tiles: bytes [0, ntiles * TILE) of every chunk of the wave.
// `wave_text` is the first byte of the wave's first chunk; all 64 chunks hold
// at least ntiles * TILE bytes (the caller guarantees it). Load k of a tile:
// lane reads 16 bytes of chunk lane / P + k * (64 / P) at byte 16 (lane % P)
// of the tile (P = TILE / 16 lanes cover one chunk's TILE contiguous bytes).
// Named members (not an array): an 8 x 16-byte array is not promoted to
// registers and would live in scratch memory.
template <uint32_t TILE>
struct Tile;
template <>
struct Tile<64> {
    uint4 p0, p1, p2, p3;
};
template <>
struct Tile<128> {
    uint4 p0, p1, p2, p3, p4, p5, p6, p7;
};

template <uint32_t K, uint32_t TILE>
__device__ __forceinline__ uint4 &piece_of(Tile<TILE> &t) {
    if constexpr (K == 0) return t.p0;
    else if constexpr (K == 1) return t.p1;
    else if constexpr (K == 2) return t.p2;
    else if constexpr (K == 3) return t.p3;
    else if constexpr (K == 4) return t.p4;
    else if constexpr (K == 5) return t.p5;
    else if constexpr (K == 6) return t.p6;
    else return t.p7;
}

template <uint32_t TILE, bool NT, size_t... K>
__device__ __forceinline__ Tile<TILE> tile_load_seq(const uint8_t *s, size_t step, std::index_sequence<K...>) {
    Tile<TILE> r;
    if constexpr (NT) ((piece_of<K>(r) = load16_stream(s + K * step)), ...);
    else ((piece_of<K>(r) = *reinterpret_cast<const uint4 *>(s + K * step)), ...);
    return r;
}

template <uint32_t TILE, bool NT = true>
__device__ __forceinline__ Tile<TILE> tile_load(const uint8_t *s, size_t step) {
    return tile_load_seq<TILE, NT>(s, step, std::make_index_sequence<TILE / 16>{});
}

// (load K's chunks are kChunksPerLoad rows further: with the swizzle, an
// even step of rows, so every load K of a lane lands at the same piece slot)
template <uint32_t TILE, bool SWZ, size_t... K>
__device__ __forceinline__ void tile_store_seq(Tile<TILE> x, uint8_t *dst, std::index_sequence<K...>) {
    using SG = Stage<TILE, SWZ>;
    static_assert(!SWZ || SG::kChunksPerLoad % 8 == 0, "the swizzle must repeat every kChunksPerLoad rows");
    ((*reinterpret_cast<uint4 *>(dst + K * SG::kChunksPerLoad * SG::kRow) = piece_of<K>(x)), ...);
}

// write the wave's tile to LDS (this lane then reads its chunk's TILE bytes
// back one 16-byte piece at a time, just before walking it)
template <uint32_t TILE, bool SWZ = false>
__device__ __forceinline__ void tile_store(const Tile<TILE> x, uint8_t *dst) {
    __builtin_amdgcn_wave_barrier();
    tile_store_seq<TILE, SWZ>(x, dst, std::make_index_sequence<TILE / 16>{});
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G, typename ST, uint32_t TILE>
__device__ __forceinline__ void walk_staged(const ST &st, Walks<G> &w, const uint8_t *__restrict__ wave_text,
                                            uint32_t L, uint32_t ntiles, uint32_t lane, uint8_t *stage,
                                            uint32_t &bad) {
    constexpr bool SWZ = Swizzled<ST>::value;
    using SG = Stage<TILE, SWZ>;
    const uint32_t ch0 = lane / SG::kPieces, sub = (lane % SG::kPieces) * 16u;
    const uint8_t *src = wave_text + (size_t)ch0 * L + sub;
    const size_t step = (size_t)SG::kChunksPerLoad * L;
    uint8_t *dst = stage + ch0 * SG::kRow + SG::piece_at(ch0, lane % SG::kPieces);
    const uint8_t *mine = stage + lane * SG::kRow;
    // one tile ahead; the prefetch is unconditional (past the last tile it
    // reloads the last tile, an L2 hit) so the wait before each store covers
    // only the older tile
    const uint32_t last = ntiles - 1;
    constexpr bool NT = !CachedText<ST>::value;
    Tile<TILE> nxt = tile_load<TILE, NT>(src, step);
    for (uint32_t t = 0; t < ntiles; ++t) {
        tile_store<TILE, SWZ>(nxt, dst);
        nxt = tile_load<TILE, NT>(src + (size_t)min(t + 1, last) * TILE, step);
#pragma unroll
        for (uint32_t k = 0; k < SG::kPieces; ++k)
            piece<G>(st, w, *reinterpret_cast<const uint4 *>(mine + SG::piece_at(lane, k)), bad);
    }
}

// Direct loads from `pos` to the end of the chunk (or, for a short pass, until
// every follower has merged).
template <int G, typename ST, bool ALIGNED>
__device__ __forceinline__ void walk_direct(const ST &st, Walks<G> &w, const uint8_t *__restrict__ p, uint32_t pos,
                                            uint32_t len, bool full, uint32_t &bad) {
    const uint32_t len16 = len & ~15u;
    if constexpr (ALIGNED) {
        // 64-byte blocks with the next block loaded before the current one is
        // walked (a full pass reads a whole chunk through this path when it
        // is walked again alone)
        const uint32_t len64 = pos + ((len16 - pos) & ~63u);
        if (pos < len64 && (full || w.wave_pending)) {
            uint4 n0 = load16<true>(p + pos), n1 = load16<true>(p + pos + 16), n2 = load16<true>(p + pos + 32),
                  n3 = load16<true>(p + pos + 48);
            for (; pos < len64; pos += 64) {
                if (!full && !w.wave_pending) return;
                const uint4 c0 = n0, c1 = n1, c2 = n2, c3 = n3;
                const uint32_t nx = min(pos + 64, len64 - 64);  // unconditional: reloads the last block at the end
                n0 = load16<true>(p + nx);
                n1 = load16<true>(p + nx + 16);
                n2 = load16<true>(p + nx + 32);
                n3 = load16<true>(p + nx + 48);
                piece<G>(st, w, c0, bad);
                piece<G>(st, w, c1, bad);
                piece<G>(st, w, c2, bad);
                piece<G>(st, w, c3, bad);
            }
        }
    }
    for (; pos < len16; pos += 16) {
        if (!full && !w.wave_pending) return;
        piece<G>(st, w, load16<ALIGNED>(p + pos), bad);
    }
    if (!full && !w.pending) return;
    for (; pos < len; ++pos) {
        const uint32_t x = p[pos];
        if (w.pending) {
#pragma unroll
            for (int j = 0; j < G; ++j) st.byte(x, w.R[j], w.c[j], bad);
            merge_check<G>(st, w);
        } else if (full) {
            st.byte(x, w.R[0], w.c[0], bad);
        } else {
            return;
        }
    }
}

// returns true when some walk of the pass ends in another state than the leader
template <int G, typename ST>
__device__ __forceinline__ bool store_pass(const ST &st, const Walks<G> &w, const Positions &pos, uint32_t first,
                                           uint32_t nwalk, bool full, uint32_t &lead_end, uint32_t &lead_cnt,
                                           uint32_t *__restrict__ out, uint64_t stride) {
    bool differs = false;
    if (full) {
        lead_end = st.id(w.R[0]);
        lead_cnt = w.c[0] + count_end(st, w.R[0]);
        out[(uint64_t)pos(0) * stride] = lead_end | (lead_cnt << 16);
    }
#pragma unroll
    for (int j = 1; j < G; ++j) {
        const uint32_t idx = first + (uint32_t)j - 1u;
        if (idx < nwalk) {
            uint32_t e, cn;
            if ((w.pending >> j) & 1u) {
                e = st.id(w.R[j]);
                cn = w.c[j] + count_end(st, w.R[j]);
                differs |= e != lead_end;
            } else {
                e = lead_end;
                cn = (uint32_t)((int32_t)lead_cnt + w.off[j]);
            }
            out[(uint64_t)pos(idx) * stride] = e | (cn << 16);
        }
    }
    return differs;
}

// Arguments of a walk launch.
struct WalkArgs {
    const uint8_t *text;
    uint64_t n;
    uint32_t L;
    uint64_t nchunks;
    const uint8_t *cls;
    const uint32_t *loff;
    const uint32_t *llist;
    uint32_t start_class;
    uint32_t sent;
    uint32_t merge;
    uint32_t *map;        // [RM][nchunks] packed end | count << 16 (end 0xffff: not walked)
    uint16_t *map_cls;    // [nchunks] class, bit 15 = ends differ
    uint16_t *map_lead;   // [nchunks] end state of the leader walk
    const uint16_t *sel;  // selection: positions [nchunks][sel_stride] in the chunk's set
    const uint8_t *nsel;  // [nchunks] number of selected positions (0: the whole set)
    uint32_t sel_stride;
    const uint8_t *redo;  // re-walk mode: only chunks with redo[c] != 0, from the whole set
    uint32_t absent_fill; // selection: map entry of a state not walked (kAbsent16, or for
                          // the S filter of a partial table dead | 0 << 16: such a
                          // state has no transition on the chunk's first byte)
};

enum WalkMode : int { WALK_ALL = 0, WALK_SELECTED = 1, WALK_REDO = 2 };

// lane threadIdx.x walks chunk c_base + threadIdx.x (c_base a multiple of 64)
template <int G, typename ST, bool ALIGNED, uint32_t TILE, int MODE>
__device__ __forceinline__ void walk_chunk(const ST &st, const WalkArgs &a, uint8_t *stage, uint64_t c_base) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t c = c_base + threadIdx.x;
    bool active = c < a.nchunks;
    if constexpr (MODE == WALK_REDO) {
        if (!active || a.redo[c] == 0) return;  // no wave-wide staging in this mode
    }
    const uint64_t b = c * (uint64_t)a.L;
    const uint32_t len = active ? (uint32_t)min((uint64_t)a.L, a.n - b) : 0u;
    const uint32_t cls = (!active || c == 0) ? a.start_class : (uint32_t)a.cls[a.text[b - 1]];
    const uint32_t lo = a.loff[cls];
    const uint32_t nlist = a.loff[cls + 1] - lo;
    const uint32_t *list = a.llist + lo;
    Positions pos{nullptr};
    uint32_t nwalk = nlist;
    if constexpr (MODE == WALK_SELECTED) {
        // nsel 0: this chunk walks its whole set
        if (active) {
            const uint32_t ns = a.nsel[c];
            if (ns) {
                pos.sel = a.sel + c * a.sel_stride;
                nwalk = ns;
            }
        } else {
            nwalk = 1;
        }
    }
    if constexpr (MODE == WALK_REDO) {
        // a walk again from a lookback set (it holds the true entry state);
        // the entries it does not walk keep what the first walk stored
        if (a.sel) {
            const uint32_t ns = a.nsel[c];
            if (ns) {
                pos.sel = a.sel + c * a.sel_stride;
                nwalk = ns;
            }
        }
    }

    // tiles every chunk of this wave holds in full
    uint32_t ntiles = 0;
    if constexpr (ALIGNED && MODE != WALK_REDO && ST::kStage) {
        uint32_t m = len;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, o, 64));
        ntiles = m / TILE;
    }

    Walks<G> w;
    uint32_t bad = 0, lead_end = 0, lead_cnt = 0;
    walks_init<G>(st, w, list, pos, nwalk, 1);
    w.merge = a.merge != 0;
    if (ntiles) {
        const uint64_t wave_first = c - lane;
        walk_staged<G, ST, TILE>(st, w, a.text + wave_first * a.L, a.L, ntiles, lane,
                                 stage + (threadIdx.x >> 6) * Stage<TILE, Swizzled<ST>::value>::kWave, bad);
    }
    if (!active) return;
    const uint8_t *p = a.text + b;
    uint32_t *out = a.map + c;
    if constexpr (MODE == WALK_SELECTED) {
        // entries not walked are marked absent (or given their known end)
        if (pos.sel)
            for (uint32_t j = 0; j < nlist; ++j) out[(uint64_t)j * a.nchunks] = a.absent_fill;
    }
    walk_direct<G, ST, ALIGNED>(st, w, p, ntiles * TILE, len, true, bad);
    bool nonuni = store_pass<G>(st, w, pos, 1, nwalk, true, lead_end, lead_cnt, out, a.nchunks);
    if (nwalk > (uint32_t)G) {
        // further passes restart at the chunk start and usually merge within a
        // few bytes: with many passes the first 64 bytes are loaded once for
        // all of them
        const bool pre = ST::kPrefixPasses && ALIGNED && len >= 64 && nwalk > 4u * (uint32_t)G;
        uint4 q0 = make_uint4(0, 0, 0, 0), q1 = q0, q2 = q0, q3 = q0;
        if (pre) {
            q0 = load16<true>(p);
            q1 = load16<true>(p + 16);
            q2 = load16<true>(p + 32);
            q3 = load16<true>(p + 48);
        }
        for (uint32_t first = G; first < nwalk; first += G - 1) {
            walks_init<G>(st, w, list, pos, nwalk, first);
            w.merge = a.merge != 0;
            uint32_t at = 0;
            if (pre) {
                if (w.wave_pending) { piece<G>(st, w, q0, bad); at = 16; }
                if (w.wave_pending) { piece<G>(st, w, q1, bad); at = 32; }
                if (w.wave_pending) { piece<G>(st, w, q2, bad); at = 48; }
                if (w.wave_pending) { piece<G>(st, w, q3, bad); at = 64; }
            }
            walk_direct<G, ST, ALIGNED>(st, w, p, at, len, false, bad);
            nonuni |= store_pass<G>(st, w, pos, first, nwalk, false, lead_end, lead_cnt, out, a.nchunks);
        }
    }
    if constexpr (MODE == WALK_SELECTED) {
        // entries filled with a known end other than the leader's make the
        // map non-uniform (the S filter of a partial table)
        if (pos.sel && nwalk < nlist && a.absent_fill != kAbsent16 && a.absent_fill != lead_end) nonuni = true;
    }
    if (bad) {
        // a byte outside the alphabet: every walk of this chunk ends in the sentinel
        for (uint32_t j = 0; j < nwalk; ++j) out[(uint64_t)pos(j) * a.nchunks] = a.sent;
        nonuni = false;
        lead_end = a.sent;
    }
    // bit 15: the walks end in more than one state
    a.map_cls[c] = (uint16_t)(cls | (nonuni ? 0x8000u : 0u));
    a.map_lead[c] = (uint16_t)lead_end;
}

// ---------------------------------------------------------------------------
// lookback sets: chunk c >= 1 starts in some state of
// B_c = delta*(Q, t[b-K .. b-1]) (b = c*L, K <= b), the image of every state
// under the K bytes before it; B_c is a subset of R_c (its last step is the
// column of t[b-1]) and holds the true entry state, so the true run is always
// walked. Entries of other walks that end outside B_c become absent in the
// composition, which only ever follows the true run to the result. One wave
// per chunk: the set is a bitmap in LDS mapped byte by byte; the result is
// the ascending positions of B_c in R_c's sorted list, or nsel 0 (walk all of
// R_c) when |B_c| > cap.
// ---------------------------------------------------------------------------

struct LookArgs {
    const uint8_t *text;
    uint32_t L;
    uint64_t nchunks;
    uint32_t K;             // first lookback window in bytes
    uint32_t Q, A;
    uint32_t words;         // bitmap words: ceil((Q + 1) / 32)
    const uint8_t *cls;     // byte -> class (A or more: invalid)
    const uint32_t *loff;   // class lists (the image of every state under one byte)
    const uint32_t *llist;
    const uint16_t *next;   // (Q+1) x A next state by class
    const uint16_t *inv;    // (A+2) x (Q+1) position of a state in a class list
    uint16_t *sel;          // [nchunks][kLookCap]
    uint8_t *nsel;          // [nchunks]
};

// LDS bytes one wave of the lookback needs (window of up to kLookMax bytes)
__host__ __device__ inline uint32_t look_wave_bytes(uint32_t words) {
    return (2u * words * 4u + 256u + kLookMax + 15u) & ~15u;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}

// Image under win[0 .. K) of every state (from_start false) or of {q0}
// (the window starts at the text start). Leaves the set in *cur; returns
// false when a byte outside the alphabet was met.
__device__ __forceinline__ bool look_image(const LookArgs &a, uint32_t start, bool from_start, const uint8_t *win,
                                           uint32_t K, const uint8_t *cl, uint32_t *&cur, uint32_t *&nxt) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t W = a.words;
    for (uint32_t w = lane; w < W; w += 64) {
        cur[w] = (from_start && (start >> 5) == w) ? 1u << (start & 31u) : 0u;
        nxt[w] = 0;
    }
    uint32_t k0 = 0;
    if (!from_start && K > 0) {
        // the image of every state under the first byte is its column's list
        const uint32_t col = cl[win[0]];
        if (col >= a.A) return false;
        wave_sync();
        for (uint32_t i = a.loff[col] + lane; i < a.loff[col + 1]; i += 64) {
            const uint32_t q = a.llist[i];
            atomicOr(&cur[q >> 5], 1u << (q & 31u));
        }
        k0 = 1;
    }
    wave_sync();
    for (uint32_t k = k0; k < K; ++k) {
        const uint32_t col = cl[win[k]];
        if (col >= a.A) return false;  // uniform: every lane reads the same byte
        for (uint32_t w = lane; w < W; w += 64) {
            uint32_t bits = cur[w];
            if (bits) {
                cur[w] = 0;
                do {
                    const uint32_t q = w * 32u + (uint32_t)__builtin_ctz(bits);
                    bits &= bits - 1u;
                    const uint32_t nq = a.next[q * a.A + col];
                    atomicOr(&nxt[nq >> 5], 1u << (nq & 31u));
                } while (bits);
            }
        }
        wave_sync();
        uint32_t *t = cur;
        cur = nxt;
        nxt = t;
    }
    return true;
}

// The wave's lanes compute chunk c's lookback set; `ws` is the wave's LDS.
// The window starts at K bytes and grows fourfold (up to kLookMax) while the
// image has more than kLookCap states; a window that reaches the text start
// maps {q0} instead of every state, which gives the true entry state alone.
__device__ __forceinline__ void lookback_chunk(const LookArgs &a, uint32_t start, uint64_t c, uint8_t *ws) {
    const uint32_t lane = threadIdx.x & 63u;
    if (c == 0) {
        if (lane == 0) {
            a.nsel[0] = 1;  // chunk 0: {q0}, position 0 of the start class
            a.sel[0] = 0;
        }
        return;
    }
    const uint32_t W = a.words;
    uint32_t *cur = reinterpret_cast<uint32_t *>(ws);
    uint32_t *nxt = cur + W;
    uint8_t *cl = reinterpret_cast<uint8_t *>(nxt + W);
    uint8_t *win = cl + 256;
    const uint64_t b = c * (uint64_t)a.L;
    for (uint32_t x = lane; x < 256; x += 64) cl[x] = a.cls[x];
    uint16_t *out = a.sel + c * kLookCap;
    uint32_t K = a.K, total = 0;
    for (;;) {
        const bool from_start = (uint64_t)K >= b;
        const uint32_t Kc = from_start ? (uint32_t)b : K;
        const uint8_t *src = a.text + (b - Kc);
        for (uint32_t k = lane; k < Kc; k += 64) win[k] = src[k];
        wave_sync();
        if (!look_image(a, start, from_start, win, Kc, cl, cur, nxt)) {
            if (lane == 0) {
                a.nsel[c] = 1;  // any state: the walk through the invalid byte ends in the sentinel
                out[0] = 0;
            }
            return;
        }
        uint32_t cnt = 0;
        for (uint32_t w = lane; w < W; w += 64) cnt += (uint32_t)__builtin_popcount(cur[w]);
        total = wave_sum(cnt);
        if (total <= kLookCap || from_start || K >= kLookMax) break;
        K = min(K * 4u, kLookMax);
        wave_sync();  // every lane is done with the window before it is rewritten
    }
    if (total > kLookCap) {
        if (lane == 0) a.nsel[c] = 0;
        return;
    }
    const uint32_t per = (W + 63u) / 64u;
    const uint32_t w0 = min(lane * per, W), w1 = min(w0 + per, W);
    uint32_t mine = 0;
    for (uint32_t w = w0; w < w1; ++w) mine += (uint32_t)__builtin_popcount(cur[w]);
    // exclusive prefix over lanes: ascending state order across lanes
    uint32_t off = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)off, o, 64);
        if ((int)lane >= o) off += v;
    }
    off -= mine;
    const uint32_t cls_prev = cl[a.text[b - 1]];
    const uint16_t *pos = a.inv + (size_t)cls_prev * (a.Q + 1);
    uint32_t missing = 0;
    for (uint32_t w = w0; w < w1; ++w) {
        uint32_t bits = cur[w];
        while (bits) {
            const uint32_t q = w * 32u + (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1u;
            const uint32_t p = pos[q];
            missing |= p == 0xffffu;
            out[off++] = (uint16_t)p;
        }
    }
    missing = wave_sum(missing);
    if (lane == 0) a.nsel[c] = missing ? 0 : (uint8_t)total;  // a state outside R_c cannot occur
}

// copy the table into LDS with four 16-byte loads in flight per thread
// (NT threads in the workgroup)
template <uint32_t NT = kWalkThreads>
__device__ __forceinline__ void stage_table(uint4 *dst, const uint4 *__restrict__ src, uint32_t n16) {
    // loads are unconditional (index clamped) so that they stay in registers
    // and are all in flight before the first store
    for (uint32_t i0 = threadIdx.x; i0 < n16; i0 += 4 * NT) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[min(i0 + (uint32_t)u * NT, n16 - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + (uint32_t)u * NT;
            if (i < n16) dst[i] = v[u];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// composition
// ---------------------------------------------------------------------------

__device__ __forceinline__ int find_state(const uint32_t *__restrict__ list, uint32_t n, uint32_t e) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (list[mid] < e) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && list[lo] == e) ? (int)lo : -1;
}

struct ComposeArgs {
    const uint32_t *loff;
    const uint32_t *llist;
    const uint16_t *inv;   // [(A+2) * (Q+1)] position of a state in a class list, 0xffff if absent; may be null
    uint32_t inv_bytes;    // staged in LDS when non-zero
    uint32_t Q1;           // Q + 1
    uint32_t sent;
    uint32_t RM;
    uint32_t P;
    const uint8_t *final_flag;
    uint64_t chunks;
};

// LDS image of P maps. Map m has entries j < sz[m]: end[m][j] (kAbsent32:
// not walked) and count base[m] + cnt[m][j]. A uniform map (uni[m] != 0)
// sends every present entry to the same state lead[m]; composing a uniform
// map on the left with any map costs one lookup and yields a uniform map.
struct Tree {
    uint64_t *cnt;
    uint64_t *base;
    uint32_t *end;
    uint32_t *cls;
    uint32_t *sz;
    uint32_t *uni;
    uint32_t *lead;
    const uint16_t *inv;
};

__device__ __forceinline__ int lookup(const ComposeArgs &a, const Tree &t, uint32_t cls, uint32_t sz, uint32_t e) {
    if (e >= a.Q1) return -1;
    if (t.inv) {
        const uint32_t v = t.inv[cls * a.Q1 + e];
        return v == 0xffffu ? -1 : (int)v;
    }
    return find_state(a.llist + a.loff[cls], sz, e);
}

__device__ __forceinline__ Tree carve(uint8_t *smem, const ComposeArgs &a) {
    Tree t;
    const size_t pr = (size_t)a.P * a.RM;
    t.cnt = reinterpret_cast<uint64_t *>(smem);
    t.base = t.cnt + pr;
    t.end = reinterpret_cast<uint32_t *>(t.base + a.P);
    t.cls = t.end + pr;
    t.sz = t.cls + a.P;
    t.uni = t.sz + a.P;
    t.lead = t.uni + a.P;
    uint16_t *inv = reinterpret_cast<uint16_t *>(t.lead + a.P);
    if (a.inv_bytes) {
        const uint32_t nw = a.inv_bytes / 4;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(a.inv);
        uint32_t *dst = reinterpret_cast<uint32_t *>(inv);
        for (uint32_t i = threadIdx.x; i < nw; i += kComposeThreads) dst[i] = src[i];
        t.inv = inv;
    } else {
        t.inv = a.inv;
    }
    return t;
}

// end of map r's entry x (kAbsent32 when that entry was not walked)
__device__ __forceinline__ uint32_t end_at(const Tree &t, uint32_t RM, uint32_t r, uint32_t x) {
    const uint32_t e = t.end[r * RM + x];
    if (e == kAbsent32) return kAbsent32;
    return t.uni[r] ? t.lead[r] : e;
}

// binary tree over np maps already in LDS; the result is map 0
__device__ __forceinline__ void tree(const ComposeArgs &a, const Tree &t, uint32_t np) {
    const uint32_t RM = a.RM;
    for (uint32_t w = 1; w < np; w <<= 1) {
        const uint32_t npairs = (np + 2 * w - 1) / (2 * w);
        int general = 0;
        for (uint32_t i = threadIdx.x; i < npairs; i += kComposeThreads) {
            const uint32_t left = i * 2 * w, right = left + w;
            if (right >= np) continue;
            if (!t.uni[left]) {
                general = 1;
                continue;
            }
            const uint32_t e = t.lead[left];
            const int x = lookup(a, t, t.cls[right], t.sz[right], e);
            const uint32_t ex = x < 0 ? a.sent : end_at(t, RM, right, (uint32_t)x);
            if (x >= 0 && ex != kAbsent32) t.base[left] += t.base[right] + t.cnt[right * RM + (uint32_t)x];
            // a missing entry (sentinel, or a state not walked: off the true run) ends the map there
            t.lead[left] = ex == kAbsent32 ? a.sent : ex;
        }
        if (__syncthreads_or(general)) {
            for (uint32_t k = threadIdx.x; k < npairs * RM; k += kComposeThreads) {
                const uint32_t i = k / RM, j = k - i * RM;
                const uint32_t left = i * 2 * w, right = left + w;
                if (right < np && !t.uni[left] && j < t.sz[left]) {
                    const uint32_t e = t.end[left * RM + j];
                    if (e == kAbsent32) continue;
                    const int x = lookup(a, t, t.cls[right], t.sz[right], e);
                    if (x < 0) {
                        t.end[left * RM + j] = a.sent;  // only the sentinel leaves the lists
                    } else {
                        const uint32_t ex = end_at(t, RM, right, (uint32_t)x);
                        if (ex != kAbsent32)
                            t.cnt[left * RM + j] += t.base[right] + t.cnt[right * RM + (uint32_t)x];
                        t.end[left * RM + j] = ex;
                    }
                }
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < npairs; i += kComposeThreads) {
                const uint32_t left = i * 2 * w, right = left + w;
                if (right < np && !t.uni[left] && t.uni[right]) {
                    // every present entry now ends where the right map's walks end
                    t.uni[left] = 1;
                    t.lead[left] = t.lead[right];
                    for (uint32_t j = 0; j < t.sz[left]; ++j) {
                        const uint32_t e = t.end[left * RM + j];
                        if (e != kAbsent32 && e != t.lead[right]) t.uni[left] = 0;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// segment map outputs of one workgroup
struct SegOut {
    uint32_t *end;
    uint64_t *cnt;
    uint32_t *cls;   // bit 31: not uniform
    uint64_t *runs;
    uint32_t *lead;
};

// segment `seg` of the level; a non-null `result` marks the last level
__device__ __forceinline__ void emit(const ComposeArgs &a, const Tree &t, uint64_t runs_total, const SegOut &o,
                                     uint64_t seg, parem_result *__restrict__ result) {
    const bool uni = t.uni[0] != 0;
    const uint64_t base = t.base[0];
    for (uint32_t j = threadIdx.x; j < t.sz[0]; j += kComposeThreads) {
        const uint32_t e = t.end[j];
        o.end[seg * a.RM + j] = e == kAbsent32 ? kAbsent32 : (uni ? t.lead[0] : e);
        o.cnt[seg * a.RM + j] = base + t.cnt[j];
    }
    if (threadIdx.x == 0) {
        o.cls[seg] = t.cls[0] | (uni ? 0u : 0x80000000u);
        o.runs[seg] = runs_total;
        o.lead[seg] = t.lead[0];
        if (result != nullptr) {
            // the last map: domain {q0}, entry 0
            const uint32_t e = uni ? t.lead[0] : t.end[0];
            parem_result r;
            if (e >= a.sent) {
                r.final_state = 0xffffffffu;
                r.accept = 0;
                r.count = 0;
            } else {
                r.final_state = e;
                r.accept = a.final_flag[e];
                r.count = base + t.cnt[0];
            }
            r.chunks = a.chunks;
            r.spec_runs = runs_total;
            r.rerun_chunks = 0;
            *result = r;
        }
    }
}

__device__ __forceinline__ uint64_t block_sum(uint64_t v) {
    __shared__ uint64_t red[kComposeThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (uint64_t)__shfl_xor((long long)v, o, 64);
    if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kComposeThreads / 64; ++i) s += red[i];
    return s;
}

// All maps of the workgroup uniform: map i (i >= 1) is entered in map i-1's
// lead state, so it contributes the count of that one entry and no tree is
// needed (one lookup per map, a block sum). The workgroup's map keeps the
// first map's entries raised by that sum and ends in the last map's lead
// (the sentinel if a state is missing from the next list).
template <typename CntOf, typename PresentOf>
__device__ __forceinline__ void uniform_chain(const ComposeArgs &a, const Tree &t, uint32_t np, CntOf cnt_of,
                                              PresentOf present_of, uint64_t &sum, uint32_t &end) {
    uint64_t contrib = 0;
    int fail = 0;
    for (uint32_t i = threadIdx.x; i < np; i += kComposeThreads) {
        if (i == 0) continue;
        const int x = lookup(a, t, t.cls[i], t.sz[i], t.lead[i - 1]);
        if (x < 0 || !present_of(i, (uint32_t)x)) fail = 1;
        else contrib += cnt_of(i, (uint32_t)x);
    }
    sum = block_sum(contrib);
    fail = __syncthreads_or(fail);
    end = fail ? a.sent : t.lead[np - 1];
}

template <typename FirstOf>
__device__ __forceinline__ void emit_uniform(const ComposeArgs &a, const Tree &t, uint64_t sum, uint32_t end,
                                             uint64_t runs_total, FirstOf first_of, const SegOut &o,
                                             uint64_t seg, parem_result *__restrict__ result) {
    for (uint32_t j = threadIdx.x; j < t.sz[0]; j += kComposeThreads) {
        uint64_t c;
        const bool present = first_of(j, c);
        o.end[seg * a.RM + j] = present ? end : kAbsent32;
        o.cnt[seg * a.RM + j] = c + sum;
    }
    if (threadIdx.x == 0) {
        o.cls[seg] = t.cls[0];
        o.runs[seg] = runs_total;
        o.lead[seg] = end;
        if (result != nullptr) {
            uint64_t c0;
            first_of(0, c0);
            parem_result r;
            if (end >= a.sent) {
                r.final_state = 0xffffffffu;
                r.accept = 0;
                r.count = 0;
            } else {
                r.final_state = end;
                r.accept = a.final_flag[end];
                r.count = c0 + sum;
            }
            r.chunks = a.chunks;
            r.spec_runs = runs_total;
            r.rerun_chunks = 0;
            *result = r;
        }
    }
}

// level 1: chunk maps, entry-major packed (end | count << 16); one
// workgroup composes segment `seg` (maps seg * P ...)
__device__ __forceinline__ void compose_chunks_seg(uint8_t *smem, const uint32_t *__restrict__ map,
                                                   const uint16_t *__restrict__ map_cls,
                                                   const uint16_t *__restrict__ map_lead, const ComposeArgs &a,
                                                   const SegOut &o, uint64_t seg, parem_result *__restrict__ result) {
    Tree t = carve(smem, a);
    const uint64_t g0 = seg * a.P;
    const uint32_t np = (uint32_t)min((uint64_t)a.P, a.chunks - g0);
    uint64_t runs = 0;
    int nonuni = 0;
    for (uint32_t i = threadIdx.x; i < np; i += kComposeThreads) {
        const uint32_t v = map_cls[g0 + i];
        const uint32_t cl = v & 0x7fffu;
        const uint32_t sz = a.loff[cl + 1] - a.loff[cl];
        t.cls[i] = cl;
        t.sz[i] = sz;
        t.uni[i] = (v & 0x8000u) ? 0u : 1u;
        t.lead[i] = map_lead[g0 + i];
        t.base[i] = 0;
        nonuni |= (v & 0x8000u) ? 1 : 0;
        runs += sz;
    }
    const uint64_t runs_total = block_sum(runs);  // contains a barrier
    const uint64_t C = a.chunks;
    if (!__syncthreads_or(nonuni) && np <= (uint32_t)kComposeThreads) {
        auto cnt_of = [&](uint32_t i, uint32_t x) { return (uint64_t)(map[(uint64_t)x * C + g0 + i] >> 16); };
        auto present_of = [&](uint32_t i, uint32_t x) {
            return (map[(uint64_t)x * C + g0 + i] & 0xffffu) != kAbsent16;
        };
        auto first_of = [&](uint32_t j, uint64_t &c) {
            const uint32_t v = map[(uint64_t)j * C + g0];
            c = v >> 16;
            return (v & 0xffffu) != kAbsent16;
        };
        uint64_t sum;
        uint32_t end;
        uniform_chain(a, t, np, cnt_of, present_of, sum, end);
        emit_uniform(a, t, sum, end, runs_total, first_of, o, seg, result);
        return;
    }
    // 8 loads in flight per thread before the LDS stores; i fastest: coalesced
    const uint32_t total = np * a.RM;
    for (uint32_t k0 = threadIdx.x; k0 < total; k0 += 8 * kComposeThreads) {
        uint32_t v[8], slot[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t k = k0 + (uint32_t)u * kComposeThreads;
            slot[u] = 0xffffffffu;
            if (k < total) {
                const uint32_t j = k / np, i = k - j * np;
                if (j < t.sz[i]) {
                    v[u] = map[(uint64_t)j * C + g0 + i];
                    slot[u] = i * a.RM + j;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (slot[u] != 0xffffffffu) {
                const uint32_t e = v[u] & 0xffffu;
                t.end[slot[u]] = e == kAbsent16 ? kAbsent32 : e;
                t.cnt[slot[u]] = v[u] >> 16;
            }
        }
    }
    __syncthreads();
    tree(a, t, np);
    emit(a, t, runs_total, o, seg, result);
}

// levels >= 2: segment maps, row-major (end u32, count u64)
__device__ __forceinline__ void compose_segs_seg(uint8_t *smem, const SegOut &in, uint64_t nin, const ComposeArgs &a,
                                                 const SegOut &o, uint64_t seg, parem_result *__restrict__ result) {
    const uint32_t *__restrict__ in_end = in.end;
    const uint64_t *__restrict__ in_cnt = in.cnt;
    const uint32_t *__restrict__ in_cls = in.cls;
    const uint64_t *__restrict__ in_runs = in.runs;
    const uint32_t *__restrict__ in_lead = in.lead;
    Tree t = carve(smem, a);
    const uint64_t g0 = seg * a.P;
    const uint32_t np = (uint32_t)min((uint64_t)a.P, nin - g0);
    const uint32_t RM = a.RM;
    uint64_t runs = 0;
    int nonuni = 0;
    for (uint32_t i = threadIdx.x; i < np; i += kComposeThreads) {
        const uint32_t v = in_cls[g0 + i];
        const uint32_t cl = v & 0x7fffffffu;
        t.cls[i] = cl;
        t.sz[i] = a.loff[cl + 1] - a.loff[cl];
        t.uni[i] = (v & 0x80000000u) ? 0u : 1u;
        t.lead[i] = in_lead[g0 + i];
        t.base[i] = 0;
        nonuni |= (v & 0x80000000u) ? 1 : 0;
        runs += in_runs[g0 + i];
    }
    const uint64_t runs_total = block_sum(runs);
    if (!__syncthreads_or(nonuni)) {
        auto cnt_of = [&](uint32_t i, uint32_t x) { return in_cnt[(g0 + i) * RM + x]; };
        auto present_of = [&](uint32_t i, uint32_t x) { return in_end[(g0 + i) * RM + x] != kAbsent32; };
        auto first_of = [&](uint32_t j, uint64_t &c) {
            c = in_cnt[g0 * RM + j];
            return in_end[g0 * RM + j] != kAbsent32;
        };
        uint64_t sum;
        uint32_t end;
        uniform_chain(a, t, np, cnt_of, present_of, sum, end);
        emit_uniform(a, t, sum, end, runs_total, first_of, o, seg, result);
        return;
    }
    const uint32_t total = np * RM;
    for (uint32_t k0 = threadIdx.x; k0 < total; k0 += 4 * kComposeThreads) {
        uint32_t e[4];
        uint64_t cn[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t k = k0 + (uint32_t)u * kComposeThreads;
            ok[u] = false;
            if (k < total) {
                const uint32_t i = k / RM, j = k - i * RM;
                if (j < t.sz[i]) {
                    e[u] = in_end[g0 * RM + k];
                    cn[u] = in_cnt[g0 * RM + k];
                    ok[u] = true;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (ok[u]) {
                t.end[k0 + (uint32_t)u * kComposeThreads] = e[u];
                t.cnt[k0 + (uint32_t)u * kComposeThreads] = cn[u];
            }
        }
    }
    __syncthreads();
    tree(a, t, np);
    emit(a, t, runs_total, o, seg, result);
}


// walk launch of one text for a table layout and walk mode; instantiated in
// its own translation unit per (layout, mode)
template <int LAYOUT, int MODE>
void launch_walk_family(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream, bool aligned);
extern template void launch_walk_family<PAREM_LAYOUT_SPARSE_LDS, WALK_ALL>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_SPARSE_LDS, WALK_SELECTED>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_SPARSE_LDS, WALK_REDO>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_CLASS_LDS, WALK_ALL>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_CLASS_LDS, WALK_SELECTED>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_CLASS_LDS, WALK_REDO>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_KGRAM_LDS, WALK_ALL>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_KGRAM_LDS, WALK_SELECTED>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_KGRAM_LDS, WALK_REDO>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_BYTE_LDS, WALK_ALL>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_BYTE_LDS, WALK_SELECTED>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_BYTE_LDS, WALK_REDO>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_BYTE_GLOBAL, WALK_ALL>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_BYTE_GLOBAL, WALK_SELECTED>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_BYTE_GLOBAL, WALK_REDO>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_HOT_LDS, WALK_ALL>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_HOT_LDS, WALK_SELECTED>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);
extern template void launch_walk_family<PAREM_LAYOUT_HOT_LDS, WALK_REDO>(const DeviceDfa &, const PlainPlan &,
                                                     const WalkArgs &, hipStream_t, bool);

// ---------------------------------------------------------------------------
// host-side argument builders
// ---------------------------------------------------------------------------

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// LDS of a composition workgroup: P maps of RM entries (u64 count, u32 end),
// per-map fields, and the inverse index when staged
inline uint32_t compose_lds(uint32_t P, uint32_t RM, uint32_t inv_lds) { return P * RM * 12u + P * 24u + inv_lds; }

inline parem_options with_chunk_len(parem_options o, uint32_t L) {
    o.chunk_len = L;
    return o;
}

inline WalkArgs walk_args(const DeviceDfa &d, const PlainPlan &p, const uint8_t *text, uint8_t *ws) {
    WalkArgs a{};
    a.text = text;
    a.n = p.n;
    a.L = p.L;
    a.nchunks = p.chunks;
    a.cls = d.d_cls;
    a.loff = d.d_loff;
    a.llist = d.d_llist_walk;
    a.start_class = d.A + 1;
    a.sent = d.sent;
    a.merge = p.merge;
    a.map = reinterpret_cast<uint32_t *>(ws + p.off_map);
    a.map_cls = reinterpret_cast<uint16_t *>(ws + p.off_mcls);
    a.map_lead = reinterpret_cast<uint16_t *>(ws + p.off_mlead);
    a.absent_fill = kAbsent16;
    return a;
}

inline LookArgs look_args(const DeviceDfa &d, const PlainPlan &p, const uint8_t *text, uint8_t *ws) {
    LookArgs a{};
    a.text = text;
    a.L = p.L;
    a.nchunks = p.chunks;
    a.K = p.look;
    a.Q = d.Q;
    a.A = d.A;
    a.words = (d.Q + 1 + 31) / 32;
    a.cls = d.d_cls;
    a.loff = d.d_loff;
    a.llist = d.d_llist;
    a.next = d.d_next;
    a.inv = d.d_inv;
    a.sel = reinterpret_cast<uint16_t *>(ws + p.off_sel);
    a.nsel = ws + p.off_nsel;
    return a;
}

inline ComposeArgs compose_args(const DeviceDfa &d, const PlainPlan &p) {
    ComposeArgs a;
    a.loff = d.d_loff;
    a.llist = d.d_llist;
    a.inv = d.d_inv;
    a.inv_bytes = d.inv_lds;
    a.Q1 = d.Q + 1;
    a.sent = d.sent;
    a.RM = p.RM;
    a.P = p.P;
    a.final_flag = d.d_final;
    a.chunks = p.chunks;
    return a;
}

inline SegOut seg_out(const PlainPlan &p, uint8_t *ws, size_t k) {
    const PlainPlan::Seg &g = p.seg[k];
    SegOut o;
    o.end = reinterpret_cast<uint32_t *>(ws + g.end);
    o.cnt = reinterpret_cast<uint64_t *>(ws + g.cnt);
    o.cls = reinterpret_cast<uint32_t *>(ws + g.cls);
    o.runs = reinterpret_cast<uint64_t *>(ws + g.runs);
    o.lead = reinterpret_cast<uint32_t *>(ws + g.lead);
    return o;
}

}  // namespace parem

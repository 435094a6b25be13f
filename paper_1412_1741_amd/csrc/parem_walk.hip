// HIP kernels of the plain speculative chunked DFA walk for gfx950.
//
// Method (PaREM, Section II-B, Algorithm 1): the text is cut into chunks;
// chunk c > 0 is walked from every state of its speculated set R_c (the
// image of the column of the byte before the chunk: the L set; S is every
// state because tables are total), chunk 0 from q0 only. Each chunk yields a
// map r -> (end state, number of final destinations). The maps are joined
// (Section II-B, the reduction after the barrier) by composing them; map
// composition is associative, so the join is a tree.
//
// k_walk: one lane per chunk. The lane walks a "leader" candidate through the
// whole chunk and up to G-1 followers in lockstep with it; a follower whose
// state equals the leader's is merged (runs that meet stay equal: the DFA is
// deterministic) and only its count offset is kept. Candidates beyond the
// first G are walked in further short passes, again with the leader, until
// they merge. Text reaches the lanes through a per-wave LDS tile: the wave
// loads 64 bytes of each of its 64 chunks with coalesced 16-byte loads (four
// lanes per 64-byte segment), writes them to LDS and every lane reads back
// its own chunk's 64 bytes; an 80-byte row stride keeps the 16-byte reads
// free of bank conflicts. Two table layouts step the walks:
//   byte table   (Q+1) x 256 entries indexed by raw byte (the byte-to-column
//                map folded in, invalid bytes leading to an absorbing
//                sentinel state), final flag in the entry's top bit;
//   k-gram table for alphabets of at most 8 symbols with a bit-field code:
//                one shift and mask give four symbol codes per text dword,
//                one v_dot4 forms the index, one LDS read advances 4 (or 2)
//                symbols, one v_perm validates 4 bytes against the alphabet.
// Chunk maps leave the kernel entry-major (map[j * chunks + c], packed
// end | count << 16) so the stores of a wave coalesce.
//
// k_compose_chunks / k_compose_segs: a workgroup composes up to P
// consecutive maps with a binary tree in LDS (inverse index of the
// speculated lists in LDS when it fits); repeated until one map (domain
// {q0}) remains, whose single entry is the result.
#include "parem_internal.h"

#include <algorithm>
#include <utility>

namespace parem {

constexpr int kWalkThreads = 256;
constexpr int kComposeThreads = 256;
// A staged tile holds TILE bytes of each of a wave's 64 chunks; LDS rows are
// TILE + 16 bytes apart so that 8 consecutive lanes' 16-byte reads hit
// distinct banks.
template <uint32_t TILE>
struct Stage {
    static constexpr uint32_t kRow = TILE + 16;
    static constexpr uint32_t kWave = 64 * kRow;
    static constexpr uint32_t kBytes = (kWalkThreads / 64) * kWave;
    static constexpr uint32_t kPieces = TILE / 16;      // 16-byte loads per lane per tile
    static constexpr uint32_t kChunksPerLoad = 64 / kPieces;
};

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

// k-gram table: a state is carried as its row base (state << RS) plus the
// count bits of the last entry read.
template <int B>
struct KgStep {
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
                    uint32_t e = lds_u16(T, (R[j] & ROWMASK) | i0);
                    S[j] += e;
                    e = lds_u16(T, (e & ROWMASK) | i1);
                    R[j] = e;
                    S[j] += e;
                }
            }
        } else {
            const uint32_t i0 = __builtin_amdgcn_udot4(cd, kp.w0, 0u, false);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (j < nw) {
                    const uint32_t e = lds_u16(T, (R[j] & ROWMASK) | i0);
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
        const uint32_t e = lds_u16(T, kp.t1_off + (((row << B) | code) << 1));
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
    if (w.wave_pending) {
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

template <bool ALIGNED>
__device__ __forceinline__ uint4 load16(const uint8_t *p) {
    if constexpr (ALIGNED) {
        return *reinterpret_cast<const uint4 *>(p);
    } else {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v[k] = (uint32_t)p[4 * k] | ((uint32_t)p[4 * k + 1] << 8) | ((uint32_t)p[4 * k + 2] << 16) |
                   ((uint32_t)p[4 * k + 3] << 24);
        return make_uint4(v[0], v[1], v[2], v[3]);
    }
}

template <int G, typename ST>
__device__ __forceinline__ void walks_init(const ST &st, Walks<G> &w, const uint32_t *__restrict__ list,
                                           uint32_t nlist, uint32_t first) {
    const uint32_t lead = st.init(list[0]);
    w.pending = 0;
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const uint32_t idx = first + (uint32_t)j - 1u;
        const bool real = j > 0 && idx < nlist;
        w.R[j] = real ? st.init(list[idx]) : lead;
        w.S[j] = 0;
        w.c[j] = 0;
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

template <uint32_t TILE, size_t... K>
__device__ __forceinline__ Tile<TILE> tile_load_seq(const uint8_t *s, size_t step, std::index_sequence<K...>) {
    Tile<TILE> r;
    ((piece_of<K>(r) = *reinterpret_cast<const uint4 *>(s + K * step)), ...);
    return r;
}

template <uint32_t TILE>
__device__ __forceinline__ Tile<TILE> tile_load(const uint8_t *s, size_t step) {
    return tile_load_seq<TILE>(s, step, std::make_index_sequence<TILE / 16>{});
}

template <uint32_t TILE, size_t... K>
__device__ __forceinline__ void tile_store_seq(Tile<TILE> x, uint8_t *dst, std::index_sequence<K...>) {
    ((*reinterpret_cast<uint4 *>(dst + K * Stage<TILE>::kChunksPerLoad * Stage<TILE>::kRow) = piece_of<K>(x)),
     ...);
}

// write the wave's tile to LDS (this lane then reads its chunk's TILE bytes
// back one 16-byte piece at a time, just before walking it)
template <uint32_t TILE>
__device__ __forceinline__ void tile_store(const Tile<TILE> x, uint8_t *dst) {
    __builtin_amdgcn_wave_barrier();
    tile_store_seq<TILE>(x, dst, std::make_index_sequence<TILE / 16>{});
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G, typename ST, uint32_t TILE>
__device__ __forceinline__ void walk_staged(const ST &st, Walks<G> &w, const uint8_t *__restrict__ wave_text,
                                            uint32_t L, uint32_t ntiles, uint32_t lane, uint8_t *stage,
                                            uint32_t &bad) {
    using SG = Stage<TILE>;
    const uint32_t ch0 = lane / SG::kPieces, sub = (lane % SG::kPieces) * 16u;
    const uint8_t *src = wave_text + (size_t)ch0 * L + sub;
    const size_t step = (size_t)SG::kChunksPerLoad * L;
    uint8_t *dst = stage + ch0 * SG::kRow + sub;
    const uint8_t *mine = stage + lane * SG::kRow;
    // one tile ahead; the prefetch is unconditional (past the last tile it
    // reloads the last tile, an L2 hit) so the wait before each store covers
    // only the older tile
    const uint32_t last = ntiles - 1;
    Tile<TILE> nxt = tile_load<TILE>(src, step);
    for (uint32_t t = 0; t < ntiles; ++t) {
        tile_store<TILE>(nxt, dst);
        nxt = tile_load<TILE>(src + (size_t)min(t + 1, last) * TILE, step);
#pragma unroll
        for (uint32_t k = 0; k < SG::kPieces; ++k)
            piece<G>(st, w, *reinterpret_cast<const uint4 *>(mine + 16 * k), bad);
    }
}

// Direct loads from `pos` to the end of the chunk (or, for a short pass, until
// every follower has merged).
template <int G, typename ST, bool ALIGNED>
__device__ __forceinline__ void walk_direct(const ST &st, Walks<G> &w, const uint8_t *__restrict__ p, uint32_t pos,
                                            uint32_t len, bool full, uint32_t &bad) {
    const uint32_t len16 = len & ~15u;
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
__device__ __forceinline__ bool store_pass(const ST &st, const Walks<G> &w, uint32_t first, uint32_t nlist,
                                           bool full, uint32_t &lead_end, uint32_t &lead_cnt,
                                           uint32_t *__restrict__ out, uint64_t stride) {
    bool differs = false;
    if (full) {
        lead_end = st.id(w.R[0]);
        lead_cnt = w.c[0];
        out[0] = lead_end | (lead_cnt << 16);
    }
#pragma unroll
    for (int j = 1; j < G; ++j) {
        const uint32_t idx = first + (uint32_t)j - 1u;
        if (idx < nlist) {
            uint32_t e, cn;
            if ((w.pending >> j) & 1u) {
                e = st.id(w.R[j]);
                cn = w.c[j];
                differs |= e != lead_end;
            } else {
                e = lead_end;
                cn = (uint32_t)((int32_t)lead_cnt + w.off[j]);
            }
            out[(uint64_t)idx * stride] = e | (cn << 16);
        }
    }
    return differs;
}

template <int G, typename ST, bool ALIGNED, uint32_t TILE>
__device__ __forceinline__ void walk_chunk(const ST &st, const uint8_t *__restrict__ text, uint64_t n, uint32_t L,
                                           uint64_t nchunks, const uint8_t *__restrict__ g_cls,
                                           const uint32_t *__restrict__ g_loff, const uint32_t *__restrict__ g_llist,
                                           uint32_t start_class, uint32_t sent, bool merge, uint8_t *stage,
                                           uint32_t *__restrict__ map, uint16_t *__restrict__ map_cls) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t c = (uint64_t)blockIdx.x * kWalkThreads + threadIdx.x;
    const bool active = c < nchunks;
    const uint64_t b = c * (uint64_t)L;
    const uint32_t len = active ? (uint32_t)min((uint64_t)L, n - b) : 0u;
    const uint32_t cls = !active ? start_class : (c == 0 ? start_class : (uint32_t)g_cls[text[b - 1]]);
    const uint32_t lo = g_loff[cls];
    const uint32_t nlist = g_loff[cls + 1] - lo;
    const uint32_t *list = g_llist + lo;

    // tiles every chunk of this wave holds in full
    uint32_t ntiles = 0;
    if constexpr (ALIGNED) {
        uint32_t m = len;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, o, 64));
        ntiles = m / TILE;
    }

    Walks<G> w;
    uint32_t bad = 0, lead_end = 0, lead_cnt = 0;
    walks_init<G>(st, w, list, nlist, 1);
    w.merge = merge;
    if (ntiles) {
        const uint64_t wave_first = c - lane;
        walk_staged<G, ST, TILE>(st, w, text + wave_first * L, L, ntiles, lane,
                                 stage + (threadIdx.x >> 6) * Stage<TILE>::kWave, bad);
    }
    if (!active) return;
    const uint8_t *p = text + b;
    walk_direct<G, ST, ALIGNED>(st, w, p, ntiles * TILE, len, true, bad);
    uint32_t *out = map + c;
    bool nonuni = store_pass<G>(st, w, 1, nlist, true, lead_end, lead_cnt, out, nchunks);
    for (uint32_t first = G; first < nlist; first += G - 1) {
        walks_init<G>(st, w, list, nlist, first);
        w.merge = merge;
        walk_direct<G, ST, ALIGNED>(st, w, p, 0, len, false, bad);
        nonuni |= store_pass<G>(st, w, first, nlist, false, lead_end, lead_cnt, out, nchunks);
    }
    if (bad) {
        // a byte outside the alphabet: every run of this chunk ends in the sentinel
        for (uint32_t j = 0; j < nlist; ++j) out[(uint64_t)j * nchunks] = sent;
        nonuni = 0;
    }
    // bit 15: the map is not uniform (its runs end in more than one state)
    map_cls[c] = (uint16_t)(cls | (nonuni ? 0x8000u : 0u));
}

// copy the table into LDS with four 16-byte loads in flight per thread
__device__ __forceinline__ void stage_table(uint4 *dst, const uint4 *__restrict__ src, uint32_t n16) {
    // loads are unconditional (index clamped) so that they stay in registers
    // and are all in flight before the first store
    for (uint32_t i0 = threadIdx.x; i0 < n16; i0 += 4 * kWalkThreads) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[min(i0 + (uint32_t)u * kWalkThreads, n16 - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kWalkThreads;
            if (i < n16) dst[i] = v[u];
        }
    }
    __syncthreads();
}

// at least 4 waves per SIMD (at most 128 VGPRs) for groups up to 8 walks
template <typename E, uint32_t ROW, int G, bool LDS_TABLE, bool ALIGNED, uint32_t TILE>
__global__ __launch_bounds__(kWalkThreads, (G <= 8 ? 4 : 2)) void k_walk_byte(
    const uint8_t *__restrict__ text, uint64_t n, uint32_t L, uint64_t nchunks, const E *__restrict__ g_table,
    uint32_t table_bytes, const uint8_t *__restrict__ g_cls, const uint32_t *__restrict__ g_loff,
    const uint32_t *__restrict__ g_llist, uint32_t start_class, uint32_t sent, uint32_t merge,
    uint32_t *__restrict__ map, uint16_t *__restrict__ map_cls) {
    extern __shared__ __align__(16) uint8_t smem[];
    ByteStep<E, ROW> st{g_table};
    uint32_t tb = 0;
    if constexpr (LDS_TABLE) {
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        const uint4 *src = reinterpret_cast<const uint4 *>(g_table);
        stage_table(dst, src, table_bytes / 16u);
        st.T = reinterpret_cast<const E *>(smem);
        tb = table_bytes;
    }
    walk_chunk<G, ByteStep<E, ROW>, ALIGNED, TILE>(st, text, n, L, nchunks, g_cls, g_loff, g_llist, start_class,
                                                   sent, merge != 0, smem + tb, map, map_cls);
}

template <int G, int B, bool ALIGNED, uint32_t TILE>
__global__ __launch_bounds__(kWalkThreads, (G <= 8 ? 4 : 2)) void k_walk_kgram(
    const uint8_t *__restrict__ text, uint64_t n, uint32_t L, uint64_t nchunks, const uint8_t *__restrict__ g_table,
    uint32_t table_bytes, KgParams kp, const uint8_t *__restrict__ g_cls, const uint32_t *__restrict__ g_loff,
    const uint32_t *__restrict__ g_llist, uint32_t start_class, uint32_t sent, uint32_t merge,
    uint32_t *__restrict__ map, uint16_t *__restrict__ map_cls) {
    extern __shared__ __align__(16) uint8_t smem[];
    {
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        const uint4 *src = reinterpret_cast<const uint4 *>(g_table);
        stage_table(dst, src, table_bytes / 16u);
    }
    KgStep<B> st{smem, kp};
    walk_chunk<G, KgStep<B>, ALIGNED, TILE>(st, text, n, L, nchunks, g_cls, g_loff, g_llist, start_class, sent,
                                            merge != 0, smem + table_bytes, map, map_cls);
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
    const uint16_t *inv;   // [(A+2) * (Q+1)] index of a state in a class list, 0xffff if absent; may be null
    uint32_t inv_bytes;    // staged in LDS when non-zero
    uint32_t Q1;           // Q + 1
    uint32_t sent;
    uint32_t RM;
    uint32_t P;
    const uint8_t *final_flag;
    uint64_t chunks;
};

// LDS image of P maps. A map m has entries j < sz[m] with end[m][j] and
// count base[m] + cnt[m][j]. A uniform map (uni[m] != 0) sends every entry
// to the same end state, stored in end[m][0]; composing a uniform map on the
// left with any map costs one lookup, and the result is uniform again.
struct Tree {
    uint64_t *cnt;
    uint64_t *base;
    uint32_t *end;
    uint32_t *cls;
    uint32_t *sz;
    uint32_t *uni;
    const uint16_t *inv;
};

__device__ __forceinline__ int lookup(const ComposeArgs &a, const Tree &t, uint32_t cls, uint32_t sz, uint32_t e) {
    if (t.inv) {
        const uint32_t v = t.inv[cls * a.Q1 + e];
        return v == 0xffffu ? -1 : (int)v;
    }
    return find_state(a.llist + a.loff[cls], sz, e);
}

// carve the dynamic LDS of a compose workgroup
__device__ __forceinline__ Tree carve(uint8_t *smem, const ComposeArgs &a) {
    Tree t;
    const size_t pr = (size_t)a.P * a.RM;
    t.cnt = reinterpret_cast<uint64_t *>(smem);
    t.base = t.cnt + pr;
    t.end = reinterpret_cast<uint32_t *>(t.base + a.P);
    t.cls = t.end + pr;
    t.sz = t.cls + a.P;
    t.uni = t.sz + a.P;
    uint16_t *inv = reinterpret_cast<uint16_t *>(t.uni + a.P);
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
            const uint32_t e = t.end[left * RM];
            const int x = lookup(a, t, t.cls[right], t.sz[right], e);
            if (x < 0) {
                t.end[left * RM] = a.sent;  // only the sentinel leaves the lists
            } else {
                t.base[left] += t.base[right] + t.cnt[right * RM + (uint32_t)x];
                t.end[left * RM] = t.uni[right] ? t.end[right * RM] : t.end[right * RM + (uint32_t)x];
            }
        }
        if (__syncthreads_or(general)) {
            for (uint32_t k = threadIdx.x; k < npairs * RM; k += kComposeThreads) {
                const uint32_t i = k / RM, j = k - i * RM;
                const uint32_t left = i * 2 * w, right = left + w;
                if (right < np && !t.uni[left] && j < t.sz[left]) {
                    const uint32_t e = t.end[left * RM + j];
                    const int x = lookup(a, t, t.cls[right], t.sz[right], e);
                    if (x < 0) {
                        t.end[left * RM + j] = a.sent;
                    } else {
                        t.cnt[left * RM + j] += t.base[right] + t.cnt[right * RM + (uint32_t)x];
                        t.end[left * RM + j] = t.uni[right] ? t.end[right * RM] : t.end[right * RM + (uint32_t)x];
                    }
                }
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < npairs; i += kComposeThreads) {
                const uint32_t left = i * 2 * w, right = left + w;
                if (right < np && !t.uni[left]) t.uni[left] = t.uni[right];
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void emit(const ComposeArgs &a, const Tree &t, uint64_t runs_total,
                                     uint32_t *__restrict__ out_end, uint64_t *__restrict__ out_cnt,
                                     uint32_t *__restrict__ out_cls, uint64_t *__restrict__ out_runs,
                                     parem_result *__restrict__ result) {
    const bool uni = t.uni[0] != 0;
    const uint64_t base = t.base[0];
    for (uint32_t j = threadIdx.x; j < t.sz[0]; j += kComposeThreads) {
        out_end[(uint64_t)blockIdx.x * a.RM + j] = uni ? t.end[0] : t.end[j];
        out_cnt[(uint64_t)blockIdx.x * a.RM + j] = base + t.cnt[j];
    }
    if (threadIdx.x == 0) {
        out_cls[blockIdx.x] = t.cls[0] | (uni ? 0u : 0x80000000u);
        out_runs[blockIdx.x] = runs_total;
        if (result != nullptr && gridDim.x == 1) {
            const uint32_t e = t.end[0];
            parem_result r;
            if (e == a.sent) {
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

// All P maps of a workgroup uniform: map i (i >= 1) is entered in the single
// end state of map i-1, so it contributes the count of that one entry and no
// tree is needed: one lookup per map and a block sum. The segment map keeps
// the first map's entries, each raised by that sum, and ends where the last
// map ends (in the sentinel if some end state is missing from the next list,
// which only the sentinel can be).
struct Uniform {
    uint32_t end;
    uint64_t sum;
    int fail;
};

template <typename EndOf, typename CntOf>
__device__ __forceinline__ Uniform uniform_chain(const ComposeArgs &a, const Tree &t, uint32_t np, EndOf end_of,
                                                 CntOf cnt_of) {
    const uint32_t i = threadIdx.x;
    if (i < np) t.end[i] = end_of(i);
    __syncthreads();
    uint64_t contrib = 0;
    int fail = 0;
    if (i < np && i > 0) {
        const int x = lookup(a, t, t.cls[i], t.sz[i], t.end[i - 1]);
        if (x < 0) fail = 1;
        else contrib = cnt_of(i, (uint32_t)x);
    }
    Uniform u;
    u.sum = block_sum(contrib);
    u.fail = __syncthreads_or(fail);
    u.end = u.fail ? a.sent : t.end[np - 1];
    return u;
}

template <typename CntOf>
__device__ __forceinline__ void emit_uniform(const ComposeArgs &a, const Tree &t, const Uniform &u,
                                             uint64_t runs_total, CntOf first_cnt, uint32_t *__restrict__ out_end,
                                             uint64_t *__restrict__ out_cnt, uint32_t *__restrict__ out_cls,
                                             uint64_t *__restrict__ out_runs, parem_result *__restrict__ result) {
    for (uint32_t j = threadIdx.x; j < t.sz[0]; j += kComposeThreads) {
        out_end[(uint64_t)blockIdx.x * a.RM + j] = u.end;
        out_cnt[(uint64_t)blockIdx.x * a.RM + j] = first_cnt(j) + u.sum;
    }
    if (threadIdx.x == 0) {
        out_cls[blockIdx.x] = t.cls[0];
        out_runs[blockIdx.x] = runs_total;
        if (result != nullptr && gridDim.x == 1) {
            parem_result r;
            if (u.end == a.sent) {
                r.final_state = 0xffffffffu;
                r.accept = 0;
                r.count = 0;
            } else {
                r.final_state = u.end;
                r.accept = a.final_flag[u.end];
                r.count = first_cnt(0) + u.sum;
            }
            r.chunks = a.chunks;
            r.spec_runs = runs_total;
            r.rerun_chunks = 0;
            *result = r;
        }
    }
}

// level 1: chunk maps, entry-major packed (end | count << 16)
__global__ __launch_bounds__(kComposeThreads) void k_compose_chunks(
    const uint32_t *__restrict__ map, const uint16_t *__restrict__ map_cls, ComposeArgs a,
    uint32_t *__restrict__ out_end, uint64_t *__restrict__ out_cnt, uint32_t *__restrict__ out_cls,
    uint64_t *__restrict__ out_runs, parem_result *__restrict__ result) {
    extern __shared__ __align__(16) uint8_t smem[];
    Tree t = carve(smem, a);
    const uint64_t g0 = (uint64_t)blockIdx.x * a.P;
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
        t.base[i] = 0;
        nonuni |= (v & 0x8000u) ? 1 : 0;
        runs += sz;
    }
    const uint64_t runs_total = block_sum(runs);  // contains a barrier
    if (!__syncthreads_or(nonuni) && np <= (uint32_t)kComposeThreads) {
        const uint64_t C = a.chunks;
        auto end_of = [&](uint32_t i) { return map[g0 + i] & 0xffffu; };
        auto cnt_of = [&](uint32_t i, uint32_t x) { return (uint64_t)(map[(uint64_t)x * C + g0 + i] >> 16); };
        auto first = [&](uint32_t j) { return (uint64_t)(map[(uint64_t)j * C + g0] >> 16); };
        const Uniform u = uniform_chain(a, t, np, end_of, cnt_of);
        emit_uniform(a, t, u, runs_total, first, out_end, out_cnt, out_cls, out_runs, result);
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
                    v[u] = map[(uint64_t)j * a.chunks + g0 + i];
                    slot[u] = i * a.RM + j;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (slot[u] != 0xffffffffu) {
                t.end[slot[u]] = v[u] & 0xffffu;
                t.cnt[slot[u]] = v[u] >> 16;
            }
        }
    }
    __syncthreads();
    tree(a, t, np);
    emit(a, t, runs_total, out_end, out_cnt, out_cls, out_runs, result);
}

// levels >= 2: segment maps, row-major (end u32, count u64)
__global__ __launch_bounds__(kComposeThreads) void k_compose_segs(
    const uint32_t *__restrict__ in_end, const uint64_t *__restrict__ in_cnt, const uint32_t *__restrict__ in_cls,
    const uint64_t *__restrict__ in_runs, uint64_t nin, ComposeArgs a, uint32_t *__restrict__ out_end,
    uint64_t *__restrict__ out_cnt, uint32_t *__restrict__ out_cls, uint64_t *__restrict__ out_runs,
    parem_result *__restrict__ result) {
    extern __shared__ __align__(16) uint8_t smem[];
    Tree t = carve(smem, a);
    const uint64_t g0 = (uint64_t)blockIdx.x * a.P;
    const uint32_t np = (uint32_t)min((uint64_t)a.P, nin - g0);
    uint64_t runs = 0;
    int nonuni = 0;
    for (uint32_t i = threadIdx.x; i < np; i += kComposeThreads) {
        const uint32_t v = in_cls[g0 + i];
        const uint32_t cl = v & 0x7fffffffu;
        t.cls[i] = cl;
        t.sz[i] = a.loff[cl + 1] - a.loff[cl];
        t.uni[i] = (v & 0x80000000u) ? 0u : 1u;
        t.base[i] = 0;
        nonuni |= (v & 0x80000000u) ? 1 : 0;
        runs += in_runs[g0 + i];
    }
    const uint64_t runs_total = block_sum(runs);
    if (!__syncthreads_or(nonuni) && np <= (uint32_t)kComposeThreads) {
        const uint32_t RM = a.RM;
        auto end_of = [&](uint32_t i) { return in_end[(g0 + i) * RM]; };
        auto cnt_of = [&](uint32_t i, uint32_t x) { return in_cnt[(g0 + i) * RM + x]; };
        auto first = [&](uint32_t j) { return in_cnt[g0 * RM + j]; };
        const Uniform u = uniform_chain(a, t, np, end_of, cnt_of);
        emit_uniform(a, t, u, runs_total, first, out_end, out_cnt, out_cls, out_runs, result);
        return;
    }
    const uint32_t total = np * a.RM;
    for (uint32_t k0 = threadIdx.x; k0 < total; k0 += 4 * kComposeThreads) {
        uint32_t e[4];
        uint64_t cn[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t k = k0 + (uint32_t)u * kComposeThreads;
            ok[u] = false;
            if (k < total) {
                const uint32_t i = k / a.RM, j = k - i * a.RM;
                if (j < t.sz[i]) {
                    e[u] = in_end[g0 * a.RM + k];
                    cn[u] = in_cnt[g0 * a.RM + k];
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
    emit(a, t, runs_total, out_end, out_cnt, out_cls, out_runs, result);
}

__global__ void k_empty_result(uint32_t start, const uint8_t *__restrict__ final_flag,
                               parem_result *__restrict__ result) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        parem_result r;
        r.final_state = start;
        r.accept = final_flag[start];
        r.count = 0;
        r.chunks = 0;
        r.spec_runs = 0;
        r.rerun_chunks = 0;
        *result = r;
    }
}

// ---------------------------------------------------------------------------
// host side: plan and launches
// ---------------------------------------------------------------------------

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

static uint32_t compose_lds(uint32_t P, uint32_t RM, uint32_t inv_lds) {
    return P * RM * 12u + P * 20u + inv_lds;
}

parem_status plan_plain(const DeviceDfa &d, uint64_t len, PlainPlan *p) {
    PlainPlan q;
    q.n = len;
    q.RM = d.max_spec;
    uint32_t L = d.opt.chunk_len;
    if (L == 0) {
        // about 2^17 chunks for large texts (two 256-lane workgroups per CU
        // on a 1 GiB text), at least 256 bytes each
        uint64_t want = len >> 17;
        L = 256;
        while ((uint64_t)L < want && L < kMaxChunk) L <<= 1;
    }
    if (L % 64 != 0 || L == 0 || L > kMaxChunk) return PAREM_EINVAL;
    q.L = L;
    q.chunks = (len + L - 1) / L;
    q.tile = d.opt.tile ? d.opt.tile : 128;
    q.merge = d.opt.no_merge ? 0u : 1u;
    if (q.tile != 64 && q.tile != 128) return PAREM_EINVAL;
    uint32_t G = d.opt.group ? d.opt.group : 8;
    if (G != 2 && G != 4 && G != 8 && G != 16) return PAREM_EINVAL;
    q.G = G;
    uint32_t P = 256;
    while (P > 2 && compose_lds(P, q.RM, d.inv_lds) > 64 * 1024) P >>= 1;
    if (compose_lds(P, q.RM, d.inv_lds) > 150 * 1024) return PAREM_EUNSUPPORTED;
    q.P = P;
    q.level_cap = q.chunks > 1 ? (q.chunks + P - 1) / P : 1;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const uint64_t ch = std::max<uint64_t>(q.chunks, 1);
    q.off_cend = take(ch * q.RM * 4);   // packed chunk maps
    q.off_ccls = take(ch * 2);
    const uint64_t lm = q.level_cap * q.RM;
    q.off_a_end = take(lm * 4);
    q.off_a_cnt = take(lm * 8);
    q.off_a_cls = take(q.level_cap * 4);
    q.off_a_runs = take(q.level_cap * 8);
    q.off_b_end = take(lm * 4);
    q.off_b_cnt = take(lm * 8);
    q.off_b_cls = take(q.level_cap * 4);
    q.off_b_runs = take(q.level_cap * 8);
    q.bytes = off;
    *p = q;
    return PAREM_OK;
}

template <typename E, uint32_t ROW, bool LDS, bool ALIGNED, uint32_t TILE>
static void launch_walk_byte(const DeviceDfa &d, const PlainPlan &p, const uint8_t *text, uint8_t *ws,
                             hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const size_t lds = (LDS ? d.table_bytes : 0) + (ALIGNED ? Stage<TILE>::kBytes : 0);
    auto *map = reinterpret_cast<uint32_t *>(ws + p.off_cend);
    auto *mcl = reinterpret_cast<uint16_t *>(ws + p.off_ccls);
    const E *tab = reinterpret_cast<const E *>(d.d_table);
    const uint32_t start_class = d.A + 1;
#define PAREM_WALK(GG)                                                                                       \
    hipLaunchKernelGGL((k_walk_byte<E, ROW, GG, LDS, ALIGNED, TILE>), dim3(grid), dim3(kWalkThreads), lds,  \
                       stream, text, p.n, p.L, p.chunks, tab, d.table_bytes, d.d_cls, d.d_loff, d.d_llist,   \
                       start_class, d.sent, p.merge, map, mcl)
    switch (p.G) {
        case 2: PAREM_WALK(2); break;
        case 4: PAREM_WALK(4); break;
        case 8: PAREM_WALK(8); break;
        default: PAREM_WALK(16); break;
    }
#undef PAREM_WALK
}

template <int B, bool ALIGNED, uint32_t TILE>
static void launch_kgram_b(const DeviceDfa &d, const PlainPlan &p, const uint8_t *text, uint8_t *ws,
                           hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const size_t lds = d.table_bytes + (ALIGNED ? Stage<TILE>::kBytes : 0);
    auto *map = reinterpret_cast<uint32_t *>(ws + p.off_cend);
    auto *mcl = reinterpret_cast<uint16_t *>(ws + p.off_ccls);
    const uint8_t *tab = reinterpret_cast<const uint8_t *>(d.d_table);
    const uint32_t start_class = d.A + 1;
#define PAREM_KG(GG)                                                                                         \
    hipLaunchKernelGGL((k_walk_kgram<GG, B, ALIGNED, TILE>), dim3(grid), dim3(kWalkThreads), lds, stream,  \
                       text, p.n, p.L, p.chunks, tab, d.table_bytes, d.kg, d.d_cls, d.d_loff, d.d_llist,    \
                       start_class, d.sent, p.merge, map, mcl)
    switch (p.G) {
        case 2: PAREM_KG(2); break;
        case 4: PAREM_KG(4); break;
        case 8: PAREM_KG(8); break;
        default: PAREM_KG(16); break;
    }
#undef PAREM_KG
}

template <bool ALIGNED, uint32_t TILE>
static void launch_walk_t(const DeviceDfa &d, const PlainPlan &p, const uint8_t *text, uint8_t *ws,
                          hipStream_t stream) {
    if (d.layout == PAREM_LAYOUT_KGRAM_LDS) {
        switch (d.kg.bits) {
            case 1: launch_kgram_b<1, ALIGNED, TILE>(d, p, text, ws, stream); break;
            case 2: launch_kgram_b<2, ALIGNED, TILE>(d, p, text, ws, stream); break;
            default: launch_kgram_b<3, ALIGNED, TILE>(d, p, text, ws, stream); break;
        }
    } else if (d.layout == PAREM_LAYOUT_BYTE_LDS) {
        launch_walk_byte<uint8_t, kByteLdsRow, true, ALIGNED, TILE>(d, p, text, ws, stream);
    } else {
        launch_walk_byte<uint16_t, 256, false, ALIGNED, TILE>(d, p, text, ws, stream);
    }
}

static void launch_walk(const DeviceDfa &d, const PlainPlan &p, const uint8_t *text, uint8_t *ws,
                        hipStream_t stream, bool aligned) {
    if (!aligned) launch_walk_t<false, 64>(d, p, text, ws, stream);
    else if (p.tile == 128) launch_walk_t<true, 128>(d, p, text, ws, stream);
    else launch_walk_t<true, 64>(d, p, text, ws, stream);
}

parem_status launch_plain(const DeviceDfa &d, const PlainPlan &p, const uint8_t *d_text, void *d_ws,
                          hipStream_t stream, parem_result *d_out, hipEvent_t ev_begin, hipEvent_t ev_end) {
    if (p.n == 0) {
        hipLaunchKernelGGL(k_empty_result, dim3(1), dim3(64), 0, stream, d.start, d.d_final, d_out);
        return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
    }
    uint8_t *ws = reinterpret_cast<uint8_t *>(d_ws);
    const bool aligned = (reinterpret_cast<uintptr_t>(d_text) & 15u) == 0;
    if (ev_begin && hipEventRecord(ev_begin, stream) != hipSuccess) return PAREM_EDEVICE;
    launch_walk(d, p, d_text, ws, stream, aligned);
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    if (ev_end && hipEventRecord(ev_end, stream) != hipSuccess) return PAREM_EDEVICE;

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
    const size_t lds = compose_lds(p.P, p.RM, d.inv_lds);
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose_chunks),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose_segs),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return PAREM_EDEVICE;
    }
    const uint32_t *map = reinterpret_cast<const uint32_t *>(ws + p.off_cend);
    const uint16_t *mcl = reinterpret_cast<const uint16_t *>(ws + p.off_ccls);
    uint64_t nin = (p.chunks + p.P - 1) / p.P;
    {
        uint32_t *oe = reinterpret_cast<uint32_t *>(ws + p.off_a_end);
        uint64_t *oc = reinterpret_cast<uint64_t *>(ws + p.off_a_cnt);
        uint32_t *ol = reinterpret_cast<uint32_t *>(ws + p.off_a_cls);
        uint64_t *orr = reinterpret_cast<uint64_t *>(ws + p.off_a_runs);
        hipLaunchKernelGGL(k_compose_chunks, dim3((uint32_t)nin), dim3(kComposeThreads), lds, stream, map, mcl, a,
                           oe, oc, ol, orr, nin == 1 ? d_out : nullptr);
        if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    }
    bool in_a = true;
    while (nin > 1) {
        const uint64_t nout = (nin + p.P - 1) / p.P;
        const uint32_t *ie = reinterpret_cast<const uint32_t *>(ws + (in_a ? p.off_a_end : p.off_b_end));
        const uint64_t *ic = reinterpret_cast<const uint64_t *>(ws + (in_a ? p.off_a_cnt : p.off_b_cnt));
        const uint32_t *il = reinterpret_cast<const uint32_t *>(ws + (in_a ? p.off_a_cls : p.off_b_cls));
        const uint64_t *ir = reinterpret_cast<const uint64_t *>(ws + (in_a ? p.off_a_runs : p.off_b_runs));
        uint32_t *oe = reinterpret_cast<uint32_t *>(ws + (in_a ? p.off_b_end : p.off_a_end));
        uint64_t *oc = reinterpret_cast<uint64_t *>(ws + (in_a ? p.off_b_cnt : p.off_a_cnt));
        uint32_t *ol = reinterpret_cast<uint32_t *>(ws + (in_a ? p.off_b_cls : p.off_a_cls));
        uint64_t *orr = reinterpret_cast<uint64_t *>(ws + (in_a ? p.off_b_runs : p.off_a_runs));
        hipLaunchKernelGGL(k_compose_segs, dim3((uint32_t)nout), dim3(kComposeThreads), lds, stream, ie, ic, il, ir,
                           nin, a, oe, oc, ol, orr, nout == 1 ? d_out : nullptr);
        if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
        nin = nout;
        in_a = !in_a;
    }
    return PAREM_OK;
}

}  // namespace parem

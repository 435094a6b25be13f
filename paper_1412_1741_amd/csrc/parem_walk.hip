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

// Walk index idx (0 = leader) starts in the state at list position
// pos(idx): idx itself for the whole speculated set, sel[idx] for a learned
// selection.
struct Positions {
    const uint16_t *sel;  // null: identity
    __device__ __forceinline__ uint32_t operator()(uint32_t idx) const { return sel ? (uint32_t)sel[idx] : idx; }
};

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
        lead_cnt = w.c[0];
        out[(uint64_t)pos(0) * stride] = lead_end | (lead_cnt << 16);
    }
#pragma unroll
    for (int j = 1; j < G; ++j) {
        const uint32_t idx = first + (uint32_t)j - 1u;
        if (idx < nwalk) {
            uint32_t e, cn;
            if ((w.pending >> j) & 1u) {
                e = st.id(w.R[j]);
                cn = w.c[j];
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
    const uint16_t *sel;  // learned selection: positions [nchunks][sel_stride] (null: whole set)
    const uint8_t *nsel;  // [nchunks] number of selected positions
    uint32_t sel_stride;
    const uint8_t *redo;  // re-walk mode: only chunks with redo[c] != 0, from the whole set
};

enum WalkMode : int { WALK_ALL = 0, WALK_SELECTED = 1, WALK_REDO = 2 };

template <int G, typename ST, bool ALIGNED, uint32_t TILE, int MODE>
__device__ __forceinline__ void walk_chunk(const ST &st, const WalkArgs &a, uint8_t *stage) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t c = (uint64_t)blockIdx.x * kWalkThreads + threadIdx.x;
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
        if (active) {
            pos.sel = a.sel + c * a.sel_stride;
            nwalk = a.nsel[c];
        } else {
            nwalk = 1;
        }
    }

    // tiles every chunk of this wave holds in full
    uint32_t ntiles = 0;
    if constexpr (ALIGNED && MODE != WALK_REDO) {
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
                                 stage + (threadIdx.x >> 6) * Stage<TILE>::kWave, bad);
    }
    if (!active) return;
    const uint8_t *p = a.text + b;
    uint32_t *out = a.map + c;
    if constexpr (MODE == WALK_SELECTED) {
        // entries not walked are marked absent
        for (uint32_t j = 0; j < nlist; ++j) out[(uint64_t)j * a.nchunks] = kAbsent16;
    }
    walk_direct<G, ST, ALIGNED>(st, w, p, ntiles * TILE, len, true, bad);
    bool nonuni = store_pass<G>(st, w, pos, 1, nwalk, true, lead_end, lead_cnt, out, a.nchunks);
    for (uint32_t first = G; first < nwalk; first += G - 1) {
        walks_init<G>(st, w, list, pos, nwalk, first);
        w.merge = a.merge != 0;
        walk_direct<G, ST, ALIGNED>(st, w, p, 0, len, false, bad);
        nonuni |= store_pass<G>(st, w, pos, first, nwalk, false, lead_end, lead_cnt, out, a.nchunks);
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
    walk_chunk<G, ByteStep<E, ROW>, ALIGNED, TILE, MODE>(st, a, smem + tb);
}

template <int G, int B, bool ALIGNED, uint32_t TILE, int MODE>
__global__ __launch_bounds__(kWalkThreads, (G <= 8 ? 4 : 2)) void k_walk_kgram(WalkArgs a,
                                                                               const uint8_t *__restrict__ g_table,
                                                                               uint32_t table_bytes, KgParams kp) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table(reinterpret_cast<uint4 *>(smem), reinterpret_cast<const uint4 *>(g_table), table_bytes / 16u);
    KgStep<B> st{smem, kp};
    walk_chunk<G, KgStep<B>, ALIGNED, TILE, MODE>(st, a, smem + table_bytes);
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

__device__ __forceinline__ void emit(const ComposeArgs &a, const Tree &t, uint64_t runs_total, const SegOut &o,
                                     parem_result *__restrict__ result) {
    const bool uni = t.uni[0] != 0;
    const uint64_t base = t.base[0];
    for (uint32_t j = threadIdx.x; j < t.sz[0]; j += kComposeThreads) {
        const uint32_t e = t.end[j];
        o.end[(uint64_t)blockIdx.x * a.RM + j] = e == kAbsent32 ? kAbsent32 : (uni ? t.lead[0] : e);
        o.cnt[(uint64_t)blockIdx.x * a.RM + j] = base + t.cnt[j];
    }
    if (threadIdx.x == 0) {
        o.cls[blockIdx.x] = t.cls[0] | (uni ? 0u : 0x80000000u);
        o.runs[blockIdx.x] = runs_total;
        o.lead[blockIdx.x] = t.lead[0];
        if (result != nullptr && gridDim.x == 1) {
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
    const uint32_t i = threadIdx.x;
    uint64_t contrib = 0;
    int fail = 0;
    if (i < np && i > 0) {
        const int x = lookup(a, t, t.cls[i], t.sz[i], t.lead[i - 1]);
        if (x < 0 || !present_of(i, (uint32_t)x)) fail = 1;
        else contrib = cnt_of(i, (uint32_t)x);
    }
    sum = block_sum(contrib);
    fail = __syncthreads_or(fail);
    end = fail ? a.sent : t.lead[np - 1];
}

template <typename FirstOf>
__device__ __forceinline__ void emit_uniform(const ComposeArgs &a, const Tree &t, uint64_t sum, uint32_t end,
                                             uint64_t runs_total, FirstOf first_of, const SegOut &o,
                                             parem_result *__restrict__ result) {
    for (uint32_t j = threadIdx.x; j < t.sz[0]; j += kComposeThreads) {
        uint64_t c;
        const bool present = first_of(j, c);
        o.end[(uint64_t)blockIdx.x * a.RM + j] = present ? end : kAbsent32;
        o.cnt[(uint64_t)blockIdx.x * a.RM + j] = c + sum;
    }
    if (threadIdx.x == 0) {
        o.cls[blockIdx.x] = t.cls[0];
        o.runs[blockIdx.x] = runs_total;
        o.lead[blockIdx.x] = end;
        if (result != nullptr && gridDim.x == 1) {
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

// level 1: chunk maps, entry-major packed (end | count << 16)
__global__ __launch_bounds__(kComposeThreads) void k_compose_chunks(const uint32_t *__restrict__ map,
                                                                     const uint16_t *__restrict__ map_cls,
                                                                     const uint16_t *__restrict__ map_lead,
                                                                     ComposeArgs a, SegOut o,
                                                                     parem_result *__restrict__ result) {
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
        emit_uniform(a, t, sum, end, runs_total, first_of, o, result);
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
    emit(a, t, runs_total, o, result);
}

// levels >= 2: segment maps, row-major (end u32, count u64)
__global__ __launch_bounds__(kComposeThreads) void k_compose_segs(const uint32_t *__restrict__ in_end,
                                                                   const uint64_t *__restrict__ in_cnt,
                                                                   const uint32_t *__restrict__ in_cls,
                                                                   const uint64_t *__restrict__ in_runs,
                                                                   const uint32_t *__restrict__ in_lead, uint64_t nin,
                                                                   ComposeArgs a, SegOut o,
                                                                   parem_result *__restrict__ result) {
    extern __shared__ __align__(16) uint8_t smem[];
    Tree t = carve(smem, a);
    const uint64_t g0 = (uint64_t)blockIdx.x * a.P;
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
    if (!__syncthreads_or(nonuni) && np <= (uint32_t)kComposeThreads) {
        auto cnt_of = [&](uint32_t i, uint32_t x) { return in_cnt[(g0 + i) * RM + x]; };
        auto present_of = [&](uint32_t i, uint32_t x) { return in_end[(g0 + i) * RM + x] != kAbsent32; };
        auto first_of = [&](uint32_t j, uint64_t &c) {
            c = in_cnt[g0 * RM + j];
            return in_end[g0 * RM + j] != kAbsent32;
        };
        uint64_t sum;
        uint32_t end;
        uniform_chain(a, t, np, cnt_of, present_of, sum, end);
        emit_uniform(a, t, sum, end, runs_total, first_of, o, result);
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
    emit(a, t, runs_total, o, result);
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
// learned speculation: coverage check and statistics
// ---------------------------------------------------------------------------

// position of state e in chunk c's map, or -1 (not in the list, or not walked)
__device__ __forceinline__ int chunk_present(const uint32_t *__restrict__ map, uint64_t C, uint64_t c,
                                             uint32_t cls, const uint16_t *__restrict__ inv, uint32_t Q1, uint32_t e) {
    if (e >= Q1) return -1;
    const uint32_t v = inv[cls * Q1 + e];
    if (v == 0xffffu) return -1;
    if ((map[(uint64_t)v * C + c] & 0xffffu) == kAbsent16) return -1;
    return (int)v;
}

// Chunk c (>= 1) is covered when every end state of chunk c-1's walks is one
// of chunk c's walked entries; then, by induction from chunk 0 (entered in
// q0, always walked), every chunk's true entry state was walked. Uncovered
// chunks get redo[c] = 1 and are walked again from their whole speculated
// set (which holds every possible entry). `escalate` != 0: if any chunk is
// uncovered, every chunk not yet complete is marked.
__global__ void k_cover(const uint32_t *__restrict__ map, const uint16_t *__restrict__ map_cls,
                        const uint16_t *__restrict__ map_lead, uint64_t C, const uint32_t *__restrict__ loff,
                        const uint16_t *__restrict__ inv, uint32_t Q1, uint32_t sent, uint8_t *__restrict__ redo,
                        uint8_t *__restrict__ done, uint32_t *__restrict__ flags, uint32_t escalate) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    redo[c] = 0;
    if (c == 0 || done[c]) return;
    const uint32_t pv = map_cls[c - 1], cv = map_cls[c];
    const uint32_t pcls = pv & 0x7fffu, ccls = cv & 0x7fffu;
    bool covered = true;
    if (!(pv & 0x8000u)) {
        const uint32_t e = map_lead[c - 1];
        covered = e == sent || chunk_present(map, C, c, ccls, inv, Q1, e) >= 0;
    } else {
        const uint32_t sz = loff[pcls + 1] - loff[pcls];
        for (uint32_t j = 0; j < sz && covered; ++j) {
            const uint32_t v = map[(uint64_t)j * C + c - 1];
            const uint32_t e = v & 0xffffu;
            if (e == kAbsent16 || e == sent) continue;
            covered = chunk_present(map, C, c, ccls, inv, Q1, e) >= 0;
        }
    }
    if (!covered) {
        if (escalate) {
            atomicOr(&flags[1], 1u);
        } else {
            redo[c] = 1;
            done[c] = 1;
            atomicAdd(&flags[0], 1u);
        }
    }
}

// second half of an escalation: if some chunk is still uncovered, every
// chunk not yet walked from its whole set is marked
__global__ void k_escalate(uint64_t C, uint8_t *__restrict__ redo, uint8_t *__restrict__ done,
                           uint32_t *__restrict__ flags) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C || flags[1] == 0 || c == 0) return;
    if (!done[c]) {
        redo[c] = 1;
        done[c] = 1;
        atomicAdd(&flags[0], 1u);
    }
}

// walks started and chunks walked again: block partial sums, then the
// result is written by k_learned_total
__global__ void k_learned_stats(const uint8_t *__restrict__ nsel, const uint8_t *__restrict__ done,
                                const uint16_t *__restrict__ map_cls, const uint32_t *__restrict__ loff, uint64_t C,
                                unsigned long long *__restrict__ acc) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long runs = 0, redo = 0;
    if (c < C) {
        runs = nsel[c];
        if (done[c]) {
            const uint32_t cl = map_cls[c] & 0x7fffu;
            runs += loff[cl + 1] - loff[cl];
            redo = 1;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        runs += (unsigned long long)__shfl_xor((long long)runs, o, 64);
        redo += (unsigned long long)__shfl_xor((long long)redo, o, 64);
    }
    __shared__ unsigned long long part[2][4];
    if ((threadIdx.x & 63u) == 0) {
        part[0][threadIdx.x >> 6] = runs;
        part[1][threadIdx.x >> 6] = redo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&acc[0], part[0][0] + part[0][1] + part[0][2] + part[0][3]);
        atomicAdd(&acc[1], part[1][0] + part[1][1] + part[1][2] + part[1][3]);
    }
}

__global__ void k_learned_total(const unsigned long long *__restrict__ acc, parem_result *__restrict__ result) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        result->spec_runs = acc[0];
        result->rerun_chunks = acc[1];
    }
}

__global__ void k_clear_u8(uint8_t *__restrict__ p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
__global__ void k_clear_u32(uint32_t *__restrict__ p, uint32_t n) {
    if (threadIdx.x < n) p[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// boundary states: down-sweep of entry states through the kept levels
// ---------------------------------------------------------------------------

// entry state of map i at a level whose maps are grouped P to a parent;
// parent entries are known. Walk from the nearest uniform map before i in
// the group (its lead is the exit of whatever entered it) or from the group
// start, applying each map to the state.
template <bool CHUNKS>
__global__ void k_entries(uint64_t nmaps, uint32_t P, const uint32_t *__restrict__ parent_entry,
                          const uint32_t *__restrict__ seg_end, const uint32_t *__restrict__ seg_cls,
                          const uint32_t *__restrict__ seg_lead, const uint32_t *__restrict__ cmap,
                          const uint16_t *__restrict__ cmap_cls, const uint16_t *__restrict__ cmap_lead,
                          const uint16_t *__restrict__ inv, uint32_t Q1, uint32_t RM, uint32_t sent,
                          uint32_t *__restrict__ entry) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nmaps) return;
    const uint64_t g0 = i / P * P;
    auto uniform = [&](uint64_t k) {
        return CHUNKS ? !(cmap_cls[k] & 0x8000u) : !(seg_cls[k] & 0x80000000u);
    };
    auto lead = [&](uint64_t k) { return CHUNKS ? (uint32_t)cmap_lead[k] : seg_lead[k]; };
    auto apply = [&](uint64_t k, uint32_t e) -> uint32_t {
        if (e >= Q1) return sent;
        const uint32_t cl = CHUNKS ? (cmap_cls[k] & 0x7fffu) : (seg_cls[k] & 0x7fffffffu);
        const uint32_t x = inv[cl * Q1 + e];
        if (x == 0xffffu) return sent;
        uint32_t ex;
        if (CHUNKS) {
            ex = cmap[(uint64_t)x * nmaps + k] & 0xffffu;
            if (ex == kAbsent16) return sent;
        } else {
            ex = seg_end[k * RM + x];
            if (ex == kAbsent32) return sent;
        }
        return uniform(k) ? lead(k) : ex;
    };
    uint64_t k = i;
    while (k > g0 && !uniform(k - 1)) --k;
    uint32_t e;
    if (k > g0) {
        e = lead(k - 1);  // a uniform map ends in its lead whatever entered it
    } else {
        e = parent_entry[i / P];
    }
    for (uint64_t j = k; j < i; ++j) e = apply(j, e);
    entry[i] = e >= sent ? 0xffffffffu : e;
}

// The down-sweep shortcut above trusts a uniform map's lead, which holds
// only when its entry state is in its list; the sentinel (after a byte
// outside the alphabet) is in none. The first chunk whose walks end in the
// sentinel contains the first such byte: every later boundary is invalid.
__global__ void k_first_bad(const uint16_t *__restrict__ map_lead, uint64_t C, uint32_t sent,
                            uint32_t *__restrict__ first_bad) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C && map_lead[c] == sent) atomicMin(first_bad, (uint32_t)c);
}

__global__ void k_after_bad(uint32_t *__restrict__ states, uint64_t C, const uint32_t *__restrict__ first_bad) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C && c > *first_bad) states[c] = 0xffffffffu;
}

__global__ void k_set_u32(uint32_t *__restrict__ p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------------------
// host side: plan and launches
// ---------------------------------------------------------------------------

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

static uint32_t compose_lds(uint32_t P, uint32_t RM, uint32_t inv_lds) {
    return P * RM * 12u + P * 24u + inv_lds;
}

static parem_status plan_common(const DeviceDfa &d, uint64_t len, uint32_t L, bool keep, PlainPlan *p) {
    PlainPlan q;
    q.n = len;
    q.RM = d.max_spec;
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
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const uint64_t ch = std::max<uint64_t>(q.chunks, 1);
    q.off_map = take(ch * q.RM * 4);  // packed chunk maps
    q.off_mcls = take(ch * 2);
    q.off_mlead = take(ch * 2);
    // segment levels: kept separately (down-sweep) or two ping-pong buffers
    uint64_t m = q.chunks;
    q.levels.clear();
    do {
        m = (m + P - 1) / P;
        q.levels.push_back(m);
    } while (m > 1);
    const size_t nbuf = keep ? q.levels.size() : std::min<size_t>(2, q.levels.size());
    q.seg.assign(nbuf, PlainPlan::Seg{});
    for (size_t l = 0; l < nbuf; ++l) {
        const uint64_t cap = keep ? q.levels[l] : q.levels[0];
        PlainPlan::Seg &g = q.seg[l];
        g.end = take(cap * q.RM * 4);
        g.cnt = take(cap * q.RM * 8);
        g.cls = take(cap * 4);
        g.runs = take(cap * 8);
        g.lead = take(cap * 4);
    }
    q.keep = keep;
    q.bytes = off;
    *p = q;
    return PAREM_OK;
}

parem_status plan_plain(const DeviceDfa &d, uint64_t len, PlainPlan *p) {
    return plan_common(d, len, d.opt.chunk_len, false, p);
}

static WalkArgs walk_args(const DeviceDfa &d, const PlainPlan &p, const uint8_t *text, uint8_t *ws) {
    WalkArgs a{};
    a.text = text;
    a.n = p.n;
    a.L = p.L;
    a.nchunks = p.chunks;
    a.cls = d.d_cls;
    a.loff = d.d_loff;
    a.llist = d.d_llist;
    a.start_class = d.A + 1;
    a.sent = d.sent;
    a.merge = p.merge;
    a.map = reinterpret_cast<uint32_t *>(ws + p.off_map);
    a.map_cls = reinterpret_cast<uint16_t *>(ws + p.off_mcls);
    a.map_lead = reinterpret_cast<uint16_t *>(ws + p.off_mlead);
    return a;
}

template <typename E, uint32_t ROW, bool LDS, bool ALIGNED, uint32_t TILE, int MODE>
static void launch_walk_byte(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const size_t lds = (LDS ? d.table_bytes : 0) + ((ALIGNED && MODE != WALK_REDO) ? Stage<TILE>::kBytes : 0);
    const E *tab = reinterpret_cast<const E *>(d.d_table);
#define PAREM_WALK(GG)                                                                                            \
    hipLaunchKernelGGL((k_walk_byte<E, ROW, GG, LDS, ALIGNED, TILE, MODE>), dim3(grid), dim3(kWalkThreads), lds, \
                       stream, a, tab, d.table_bytes)
    switch (p.G) {
        case 2: PAREM_WALK(2); break;
        case 4: PAREM_WALK(4); break;
        case 8: PAREM_WALK(8); break;
        default: PAREM_WALK(16); break;
    }
#undef PAREM_WALK
}

template <int B, bool ALIGNED, uint32_t TILE, int MODE>
static void launch_kgram_b(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const size_t lds = d.table_bytes + ((ALIGNED && MODE != WALK_REDO) ? Stage<TILE>::kBytes : 0);
    const uint8_t *tab = reinterpret_cast<const uint8_t *>(d.d_table);
#define PAREM_KG(GG)                                                                                              \
    hipLaunchKernelGGL((k_walk_kgram<GG, B, ALIGNED, TILE, MODE>), dim3(grid), dim3(kWalkThreads), lds, stream, a, \
                       tab, d.table_bytes, d.kg)
    switch (p.G) {
        case 2: PAREM_KG(2); break;
        case 4: PAREM_KG(4); break;
        case 8: PAREM_KG(8); break;
        default: PAREM_KG(16); break;
    }
#undef PAREM_KG
}

template <bool ALIGNED, uint32_t TILE, int MODE>
static void launch_walk_t(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream) {
    if (d.layout == PAREM_LAYOUT_KGRAM_LDS) {
        switch (d.kg.bits) {
            case 1: launch_kgram_b<1, ALIGNED, TILE, MODE>(d, p, a, stream); break;
            case 2: launch_kgram_b<2, ALIGNED, TILE, MODE>(d, p, a, stream); break;
            default: launch_kgram_b<3, ALIGNED, TILE, MODE>(d, p, a, stream); break;
        }
    } else if (d.layout == PAREM_LAYOUT_BYTE_LDS) {
        launch_walk_byte<uint8_t, kByteLdsRow, true, ALIGNED, TILE, MODE>(d, p, a, stream);
    } else {
        launch_walk_byte<uint16_t, 256, false, ALIGNED, TILE, MODE>(d, p, a, stream);
    }
}

template <int MODE>
static void launch_walk(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream,
                        bool aligned) {
    if (!aligned) launch_walk_t<false, 64, MODE>(d, p, a, stream);
    else if (p.tile == 128 || MODE == WALK_REDO) launch_walk_t<true, 128, MODE>(d, p, a, stream);
    else launch_walk_t<true, 64, MODE>(d, p, a, stream);
}

static ComposeArgs compose_args(const DeviceDfa &d, const PlainPlan &p) {
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

static SegOut seg_out(const PlainPlan &p, uint8_t *ws, size_t k) {
    const PlainPlan::Seg &g = p.seg[k];
    SegOut o;
    o.end = reinterpret_cast<uint32_t *>(ws + g.end);
    o.cnt = reinterpret_cast<uint64_t *>(ws + g.cnt);
    o.cls = reinterpret_cast<uint32_t *>(ws + g.cls);
    o.runs = reinterpret_cast<uint64_t *>(ws + g.runs);
    o.lead = reinterpret_cast<uint32_t *>(ws + g.lead);
    return o;
}

// the composition levels after the walk; the last writes *d_out
static parem_status launch_compose(const DeviceDfa &d, const PlainPlan &p, uint8_t *ws, hipStream_t stream,
                                   parem_result *d_out) {
    const ComposeArgs a = compose_args(d, p);
    const size_t lds = compose_lds(p.P, p.RM, d.inv_lds);
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose_chunks),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose_segs),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return PAREM_EDEVICE;
    }
    const uint32_t *map = reinterpret_cast<const uint32_t *>(ws + p.off_map);
    const uint16_t *mcl = reinterpret_cast<const uint16_t *>(ws + p.off_mcls);
    const uint16_t *mld = reinterpret_cast<const uint16_t *>(ws + p.off_mlead);
    uint64_t nin = p.levels[0];
    hipLaunchKernelGGL(k_compose_chunks, dim3((uint32_t)nin), dim3(kComposeThreads), lds, stream, map, mcl, mld, a,
                       seg_out(p, ws, 0), nin == 1 ? d_out : nullptr);
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    for (size_t l = 1; l < p.levels.size(); ++l) {
        const size_t src = p.keep ? l - 1 : (l - 1) % 2, dst = p.keep ? l : l % 2;
        const SegOut in = seg_out(p, ws, src);
        const uint64_t nout = p.levels[l];
        hipLaunchKernelGGL(k_compose_segs, dim3((uint32_t)nout), dim3(kComposeThreads), lds, stream, in.end, in.cnt,
                           in.cls, in.runs, in.lead, nin, a, seg_out(p, ws, dst), nout == 1 ? d_out : nullptr);
        if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
        nin = nout;
    }
    return PAREM_OK;
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
    const WalkArgs a = walk_args(d, p, d_text, ws);
    launch_walk<WALK_ALL>(d, p, a, stream, aligned);
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    if (ev_end && hipEventRecord(ev_end, stream) != hipSuccess) return PAREM_EDEVICE;
    return launch_compose(d, p, ws, stream, d_out);
}

// ---- boundary states ----

parem_status plan_boundary(const DeviceDfa &d, uint64_t len, uint32_t L, PlainPlan *p) {
    parem_status st = plan_common(d, len, L, true, p);
    if (st != PAREM_OK) return st;
    // entry arrays per level (level 0 is the caller's output)
    uint64_t off = p->bytes;
    p->entries.clear();
    for (size_t l = 0; l < p->levels.size(); ++l) {
        p->entries.push_back(off);
        off = align256(off + p->levels[l] * 4);
    }
    p->off_dummy = off;
    off = align256(off + sizeof(parem_result) + 16);
    p->bytes = off;
    return PAREM_OK;
}

parem_status launch_boundary(const DeviceDfa &d, const PlainPlan &p, const uint8_t *d_text, uint32_t *d_states,
                             void *d_ws, hipStream_t stream) {
    if (p.n == 0) return PAREM_OK;
    if (!d.d_inv) return PAREM_EUNSUPPORTED;
    uint8_t *ws = reinterpret_cast<uint8_t *>(d_ws);
    const bool aligned = (reinterpret_cast<uintptr_t>(d_text) & 15u) == 0;
    const WalkArgs a = walk_args(d, p, d_text, ws);
    launch_walk<WALK_ALL>(d, p, a, stream, aligned);
    parem_status st = launch_compose(d, p, ws, stream, reinterpret_cast<parem_result *>(ws + p.off_dummy));
    if (st != PAREM_OK) return st;
    // down-sweep: the top map is entered in q0
    const size_t top = p.levels.size() - 1;
    uint32_t *top_entry = reinterpret_cast<uint32_t *>(ws + p.entries[top]);
    if (hipMemcpyAsync(top_entry, &d.start, 4, hipMemcpyHostToDevice, stream) != hipSuccess) return PAREM_EDEVICE;
    for (size_t l = top; l-- > 0;) {
        const SegOut s = seg_out(p, ws, l);
        const uint64_t nmaps = p.levels[l];
        hipLaunchKernelGGL(k_entries<false>, dim3((uint32_t)((nmaps + 255) / 256)), dim3(256), 0, stream, nmaps, p.P,
                           reinterpret_cast<const uint32_t *>(ws + p.entries[l + 1]), s.end, s.cls, s.lead, nullptr,
                           nullptr, nullptr, d.d_inv, d.Q + 1, p.RM, d.sent,
                           reinterpret_cast<uint32_t *>(ws + p.entries[l]));
    }
    const uint32_t g = (uint32_t)((p.chunks + 255) / 256);
    hipLaunchKernelGGL(k_entries<true>, dim3(g), dim3(256), 0, stream, p.chunks, p.P,
                       reinterpret_cast<const uint32_t *>(ws + p.entries[0]), nullptr, nullptr, nullptr, a.map,
                       a.map_cls, a.map_lead, d.d_inv, d.Q + 1, p.RM, d.sent, d_states);
    uint32_t *first_bad = reinterpret_cast<uint32_t *>(ws + p.off_dummy + sizeof(parem_result));
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, stream, first_bad, 0xffffffffu);
    hipLaunchKernelGGL(k_first_bad, dim3(g), dim3(256), 0, stream, a.map_lead, p.chunks, d.sent, first_bad);
    hipLaunchKernelGGL(k_after_bad, dim3(g), dim3(256), 0, stream, d_states, p.chunks, first_bad);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

// ---- learned speculation ----

parem_status plan_learned(const DeviceDfa &d, const Proposal &pr, uint64_t len, uint32_t m, PlainPlan *p) {
    parem_status st = plan_common(d, len, d.opt.chunk_len, false, p);
    if (st != PAREM_OK) return st;
    uint64_t off = p->bytes;
    const uint64_t ch = std::max<uint64_t>(p->chunks, 1);
    p->off_sel = off;
    off = align256(off + ch * m * 2);
    p->off_nsel = off;
    off = align256(off + ch);
    p->off_redo = off;
    off = align256(off + ch);
    p->off_done = off;
    off = align256(off + ch);
    p->off_flags = off;
    off = align256(off + 64);
    p->off_mlp = off;
    off = align256(off + proposal_infer_bytes(pr, ch));
    p->bytes = off;
    p->m = m;
    return PAREM_OK;
}

parem_status launch_learned(const DeviceDfa &d, const Proposal &pr, const PlainPlan &p, const uint8_t *d_text,
                            void *d_ws, hipStream_t stream, parem_result *d_out, hipEvent_t ev_begin,
                            hipEvent_t ev_end) {
    if (p.n == 0) {
        hipLaunchKernelGGL(k_empty_result, dim3(1), dim3(64), 0, stream, d.start, d.d_final, d_out);
        return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
    }
    if (!d.d_inv) return PAREM_EUNSUPPORTED;
    uint8_t *ws = reinterpret_cast<uint8_t *>(d_ws);
    const bool aligned = (reinterpret_cast<uintptr_t>(d_text) & 15u) == 0;
    uint16_t *sel = reinterpret_cast<uint16_t *>(ws + p.off_sel);
    uint8_t *nsel = ws + p.off_nsel;
    uint8_t *redo = ws + p.off_redo;
    uint8_t *done = ws + p.off_done;
    uint32_t *flags = reinterpret_cast<uint32_t *>(ws + p.off_flags);
    const uint32_t C = (uint32_t)p.chunks;
    const uint32_t g = (C + 255) / 256;
    if (ev_begin && hipEventRecord(ev_begin, stream) != hipSuccess) return PAREM_EDEVICE;
    // 1. proposal: top-m of each chunk's speculated set
    parem_status st = proposal_select(pr, d_text, p.L, C, p.m, p.m, ws + p.off_mlp, stream, sel, nsel);
    if (st != PAREM_OK) return st;
    // 2. walk the selected states
    WalkArgs a = walk_args(d, p, d_text, ws);
    a.sel = sel;
    a.nsel = nsel;
    a.sel_stride = p.m;
    launch_walk<WALK_SELECTED>(d, p, a, stream, aligned);
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    // 3. verify coverage, walk uncovered chunks again from their whole set
    hipLaunchKernelGGL(k_clear_u8, dim3(g), dim3(256), 0, stream, done, (uint64_t)C);
    hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, stream, flags, 8u);
    WalkArgs r = walk_args(d, p, d_text, ws);
    r.redo = redo;
    for (int it = 0; it <= kCoverRounds; ++it) {
        const uint32_t escalate = it == kCoverRounds ? 1u : 0u;
        hipLaunchKernelGGL(k_cover, dim3(g), dim3(256), 0, stream, a.map, a.map_cls, a.map_lead, (uint64_t)C, d.d_loff,
                           d.d_inv, d.Q + 1, d.sent, redo, done, flags, escalate);
        if (escalate) hipLaunchKernelGGL(k_escalate, dim3(g), dim3(256), 0, stream, (uint64_t)C, redo, done, flags);
        launch_walk<WALK_REDO>(d, p, r, stream, aligned);
    }
    if (ev_end && hipEventRecord(ev_end, stream) != hipSuccess) return PAREM_EDEVICE;
    // 4. compose, then the learned statistics
    st = launch_compose(d, p, ws, stream, d_out);
    if (st != PAREM_OK) return st;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(flags + 4);
    hipLaunchKernelGGL(k_learned_stats, dim3(g), dim3(256), 0, stream, nsel, done, a.map_cls, d.d_loff,
                       (uint64_t)C, acc);  // 256 threads: four waves per partial
    hipLaunchKernelGGL(k_learned_total, dim3(1), dim3(64), 0, stream, acc, d_out);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

}  // namespace parem

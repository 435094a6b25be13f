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
#include "parem_device.h"

namespace parem {

__global__ __launch_bounds__(kComposeThreads) void k_compose_chunks(const uint32_t *__restrict__ map,
                                                                     const uint16_t *__restrict__ map_cls,
                                                                     const uint16_t *__restrict__ map_lead,
                                                                     ComposeArgs a, SegOut o,
                                                                     parem_result *__restrict__ result) {
    extern __shared__ __align__(16) uint8_t smem[];
    compose_chunks_seg(smem, map, map_cls, map_lead, a, o, blockIdx.x, result);
}

__global__ __launch_bounds__(kComposeThreads) void k_compose_segs(SegOut in, uint64_t nin, ComposeArgs a, SegOut o,
                                                                   parem_result *__restrict__ result) {
    extern __shared__ __align__(16) uint8_t smem[];
    compose_segs_seg(smem, in, nin, a, o, blockIdx.x, result);
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

// walks started under lookback selection (nsel 0: the chunk's whole set)
__global__ void k_look_stats(const uint8_t *__restrict__ nsel, const uint16_t *__restrict__ map_cls,
                             const uint32_t *__restrict__ loff, uint64_t C, unsigned long long *__restrict__ acc) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long runs = 0;
    if (c < C) {
        runs = nsel[c];
        if (!runs) {
            const uint32_t cl = map_cls[c] & 0x7fffu;
            runs = loff[cl + 1] - loff[cl];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) runs += (unsigned long long)__shfl_xor((long long)runs, o, 64);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = runs;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&acc[0], part[0] + part[1] + part[2] + part[3]);
}

__global__ __launch_bounds__(256) void k_lookback(LookArgs a, uint32_t start, uint32_t wave_bytes) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint64_t c = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    if (c >= a.nchunks) return;  // whole waves leave; no workgroup barrier follows
    lookback_chunk(a, start, c, smem + (threadIdx.x >> 6) * wave_bytes);
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

parem_status plan_chunks(const DeviceDfa &d, uint64_t len, const parem_options &o, bool keep, PlainPlan *p) {
    PlainPlan q;
    q.n = len;
    q.RM = d.max_spec;
    uint32_t L = o.chunk_len;
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
    q.look = (o.lookback && d.d_next && d.d_inv) ? o.lookback : 0u;
    q.tile = o.tile ? o.tile : 128;
    q.merge = o.no_merge ? 0u : 1u;
    if (q.tile != 64 && q.tile != 128) return PAREM_EINVAL;
    uint32_t G = o.group ? o.group : 8;
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
    if (q.look) {
        q.off_sel = take(ch * kLookCap * 2);  // lookback selection (positions in R_c)
        q.off_nsel = take(ch);
        q.off_flags = take(64);               // speculated-walk tally
    }
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
    return plan_chunks(d, len, d.opt, false, p);
}

template <int MODE>
static void launch_walk(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream,
                        bool aligned) {
    switch (d.layout) {
        case PAREM_LAYOUT_KGRAM_LDS: launch_walk_family<PAREM_LAYOUT_KGRAM_LDS, MODE>(d, p, a, stream, aligned); break;
        case PAREM_LAYOUT_BYTE_LDS: launch_walk_family<PAREM_LAYOUT_BYTE_LDS, MODE>(d, p, a, stream, aligned); break;
        case PAREM_LAYOUT_HOT_LDS: launch_walk_family<PAREM_LAYOUT_HOT_LDS, MODE>(d, p, a, stream, aligned); break;
        case PAREM_LAYOUT_CLASS_LDS: launch_walk_family<PAREM_LAYOUT_CLASS_LDS, MODE>(d, p, a, stream, aligned); break;
        default: launch_walk_family<PAREM_LAYOUT_BYTE_GLOBAL, MODE>(d, p, a, stream, aligned); break;
    }
}

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
        hipLaunchKernelGGL(k_compose_segs, dim3((uint32_t)nout), dim3(kComposeThreads), lds, stream, in, nin, a,
                           seg_out(p, ws, dst), nout == 1 ? d_out : nullptr);
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
    WalkArgs a = walk_args(d, p, d_text, ws);
    if (p.look) {
        const LookArgs la = look_args(d, p, d_text, ws);
        const uint32_t wb = look_wave_bytes(la.words);
        hipLaunchKernelGGL(k_lookback, dim3((uint32_t)((p.chunks + 3) / 4)), dim3(256), 4 * wb, stream, la, d.start, wb);
        a.sel = la.sel;
        a.nsel = la.nsel;
        a.sel_stride = kLookCap;
        launch_walk<WALK_SELECTED>(d, p, a, stream, aligned);
    } else {
        launch_walk<WALK_ALL>(d, p, a, stream, aligned);
    }
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    if (ev_end && hipEventRecord(ev_end, stream) != hipSuccess) return PAREM_EDEVICE;
    parem_status st = launch_compose(d, p, ws, stream, d_out);
    if (st != PAREM_OK || !p.look) return st;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(ws + p.off_flags);
    hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, stream, reinterpret_cast<uint32_t *>(acc), 4u);
    hipLaunchKernelGGL(k_look_stats, dim3((uint32_t)((p.chunks + 255) / 256)), dim3(256), 0, stream, a.nsel,
                       a.map_cls, d.d_loff, p.chunks, acc);
    hipLaunchKernelGGL(k_learned_total, dim3(1), dim3(64), 0, stream, acc, d_out);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

// ---- boundary states ----

parem_status plan_boundary(const DeviceDfa &d, uint64_t len, uint32_t L, PlainPlan *p) {
    parem_options o = with_chunk_len(d.opt, L);
    o.lookback = 0;  // the down-sweep reads the walked maps of Algorithm 1's sets
    parem_status st = plan_chunks(d, len, o, true, p);
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

parem_status plan_learned(const DeviceDfa &d, const Proposal &pr, uint64_t len, uint32_t m, const parem_options &opt,
                          PlainPlan *p) {
    parem_options o = opt;
    o.lookback = 0;  // the proposal selects within Algorithm 1's sets
    parem_status st = plan_chunks(d, len, o, false, p);
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

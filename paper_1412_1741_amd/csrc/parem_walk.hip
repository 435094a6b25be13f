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
// Kernel 1 (k_walk_byte): one lane per chunk. The lane walks a "leader"
// candidate through the whole chunk and up to G-1 followers in lockstep with
// it; a follower whose state equals the leader's state is merged (runs that
// meet stay equal: the DFA is deterministic) and only its count offset is
// kept. Candidates beyond the first G are walked in further short passes,
// again with the leader, until they merge. The transition table is indexed
// by raw byte ((Q+1) x 256 entries, the byte-to-column map folded in, invalid
// bytes leading to an absorbing sentinel state) and carries the final-state
// flag in its top bit.
//
// Kernel 2 (k_compose): a workgroup composes P consecutive maps with a
// binary tree in LDS; repeated until one map (domain {q0}) remains, whose
// single entry is the result.
#include "parem_internal.h"

#include <algorithm>

namespace parem {

constexpr int kWalkThreads = 256;
constexpr int kComposeThreads = 256;

template <typename E>
struct EntryBits {
    static constexpr uint32_t acc_shift = sizeof(E) * 8 - 1;
    static constexpr uint32_t state_mask = (1u << acc_shift) - 1u;
};

template <typename E>
__device__ __forceinline__ void step(uint32_t &s, uint32_t &c, uint32_t byte, const E *__restrict__ T) {
    const uint32_t v = T[(s << 8) | byte];
    c += v >> EntryBits<E>::acc_shift;
    s = v & EntryBits<E>::state_mask;
}

template <typename E, int G>
__device__ __forceinline__ void step_word(uint32_t (&s)[G], uint32_t (&c)[G], uint32_t w, int nwalk,
                                          const E *__restrict__ T) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t byte = (w >> (8 * k)) & 0xffu;
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (j < nwalk) step<E>(s[j], c[j], byte, T);
    }
}

template <bool ALIGNED>
__device__ __forceinline__ uint4 load16(const uint8_t *p) {
    if constexpr (ALIGNED) {
        return *reinterpret_cast<const uint4 *>(p);
    } else {
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            w[k] = (uint32_t)p[4 * k] | ((uint32_t)p[4 * k + 1] << 8) | ((uint32_t)p[4 * k + 2] << 16) |
                   ((uint32_t)p[4 * k + 3] << 24);
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// One pass: leader list[0] plus followers list[first .. first+G-2]. With
// `full`, the leader is walked to the chunk end (pass 0); otherwise the pass
// stops as soon as every follower has merged.
template <typename E, int G, bool ALIGNED>
__device__ __forceinline__ void walk_pass(const uint8_t *__restrict__ p, uint32_t len, const E *__restrict__ T,
                                          const uint32_t *__restrict__ list, uint32_t nlist, uint32_t first,
                                          bool full, uint32_t &lead_end, uint32_t &lead_cnt,
                                          uint32_t *__restrict__ out_end, uint32_t *__restrict__ out_cnt) {
    uint32_t s[G], c[G];
    int32_t off[G];
    uint32_t pending = 0;  // bit j: follower j not merged yet
    const uint32_t lead = list[0];
    s[0] = lead;
    c[0] = 0;
    off[0] = 0;
#pragma unroll
    for (int j = 1; j < G; ++j) {
        const uint32_t idx = first + (uint32_t)j - 1u;
        const bool real = idx < nlist;
        s[j] = real ? list[idx] : lead;
        c[j] = 0;
        off[j] = 0;
        if (real && s[j] != lead) pending |= 1u << j;
    }

    const uint32_t len16 = len & ~15u;
    uint32_t pos = 0;
    bool wave_pending = __any(pending != 0);
    for (; pos < len16; pos += 16) {
        if (!full && !wave_pending) break;
        const uint4 q = load16<ALIGNED>(p + pos);
        if (wave_pending) {
            step_word<E, G>(s, c, q.x, G, T);
            step_word<E, G>(s, c, q.y, G, T);
            step_word<E, G>(s, c, q.z, G, T);
            step_word<E, G>(s, c, q.w, G, T);
#pragma unroll
            for (int j = 1; j < G; ++j) {
                if (((pending >> j) & 1u) && s[j] == s[0]) {
                    off[j] = (int32_t)(c[j] - c[0]);
                    pending &= ~(1u << j);
                }
            }
            wave_pending = __any(pending != 0);
        } else {
            step_word<E, G>(s, c, q.x, 1, T);
            step_word<E, G>(s, c, q.y, 1, T);
            step_word<E, G>(s, c, q.z, 1, T);
            step_word<E, G>(s, c, q.w, 1, T);
        }
    }
    if (full || pending) {
        // ragged tail (or the rest of a short pass that has not merged yet)
        for (uint32_t i = pos; i < len; ++i) {
            const uint32_t byte = p[i];
            if (pending) {
#pragma unroll
                for (int j = 0; j < G; ++j) step<E>(s[j], c[j], byte, T);
#pragma unroll
                for (int j = 1; j < G; ++j) {
                    if (((pending >> j) & 1u) && s[j] == s[0]) {
                        off[j] = (int32_t)(c[j] - c[0]);
                        pending &= ~(1u << j);
                    }
                }
            } else if (full) {
                step<E>(s[0], c[0], byte, T);
            } else {
                break;
            }
        }
    }
    if (full) {
        lead_end = s[0];
        lead_cnt = c[0];
        out_end[0] = s[0];
        out_cnt[0] = c[0];
    }
#pragma unroll
    for (int j = 1; j < G; ++j) {
        const uint32_t idx = first + (uint32_t)j - 1u;
        if (idx < nlist) {
            if ((pending >> j) & 1u) {
                out_end[idx] = s[j];
                out_cnt[idx] = c[j];
            } else {
                out_end[idx] = lead_end;
                out_cnt[idx] = (uint32_t)((int32_t)lead_cnt + off[j]);
            }
        }
    }
}

template <typename E, int G, bool LDS_TABLE, bool ALIGNED>
__global__ __launch_bounds__(kWalkThreads) void k_walk_byte(
    const uint8_t *__restrict__ text, uint64_t n, uint32_t L, uint64_t nchunks, const E *__restrict__ g_table,
    uint32_t table_entries, const uint8_t *__restrict__ g_cls, const uint32_t *__restrict__ g_loff,
    const uint32_t *__restrict__ g_llist, uint32_t start_class, uint32_t RM, uint32_t *__restrict__ map_end,
    uint32_t *__restrict__ map_cnt, uint32_t *__restrict__ map_cls) {
    extern __shared__ __align__(16) uint8_t smem[];
    const E *T = g_table;
    if constexpr (LDS_TABLE) {
        // stage the table in LDS with 16-byte copies (entries padded to 16 B by the compile step)
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        const uint4 *src = reinterpret_cast<const uint4 *>(g_table);
        const uint32_t n16 = (table_entries * (uint32_t)sizeof(E) + 15u) / 16u;
        for (uint32_t i = threadIdx.x; i < n16; i += kWalkThreads) dst[i] = src[i];
        __syncthreads();
        T = reinterpret_cast<const E *>(smem);
    }
    const uint64_t c = (uint64_t)blockIdx.x * kWalkThreads + threadIdx.x;
    if (c >= nchunks) return;
    const uint64_t b = c * (uint64_t)L;
    const uint32_t len = (uint32_t)min((uint64_t)L, n - b);
    const uint32_t cls = (c == 0) ? start_class : (uint32_t)g_cls[text[b - 1]];
    const uint32_t lo = g_loff[cls];
    const uint32_t nlist = g_loff[cls + 1] - lo;
    const uint32_t *list = g_llist + lo;
    uint32_t *oe = map_end + c * RM;
    uint32_t *oc = map_cnt + c * RM;
    map_cls[c] = cls;

    uint32_t lead_end = 0, lead_cnt = 0;
    const uint8_t *p = text + b;
    walk_pass<E, G, ALIGNED>(p, len, T, list, nlist, 1, true, lead_end, lead_cnt, oe, oc);
    for (uint32_t first = G; first < nlist; first += G - 1)
        walk_pass<E, G, ALIGNED>(p, len, T, list, nlist, first, false, lead_end, lead_cnt, oe, oc);
}

__device__ __forceinline__ int find_state(const uint32_t *__restrict__ list, uint32_t n, uint32_t e) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (list[mid] < e) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && list[lo] == e) ? (int)lo : -1;
}

template <typename CIn>
__global__ __launch_bounds__(kComposeThreads) void k_compose(
    const uint32_t *__restrict__ in_end, const CIn *__restrict__ in_cnt, const uint32_t *__restrict__ in_cls,
    const uint64_t *__restrict__ in_runs, uint64_t nin, uint32_t RM, uint32_t P,
    const uint32_t *__restrict__ loff, const uint32_t *__restrict__ llist, uint32_t sent,
    uint32_t *__restrict__ out_end, uint64_t *__restrict__ out_cnt, uint32_t *__restrict__ out_cls,
    uint64_t *__restrict__ out_runs, const uint8_t *__restrict__ final_flag, parem_result *__restrict__ result,
    uint64_t chunks) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint64_t *s_cnt = reinterpret_cast<uint64_t *>(smem);
    uint32_t *s_end = reinterpret_cast<uint32_t *>(smem + (size_t)P * RM * 8);
    uint32_t *s_cls = s_end + (size_t)P * RM;
    uint32_t *s_sz = s_cls + P;
    __shared__ uint64_t s_red[kComposeThreads];

    const uint64_t g0 = (uint64_t)blockIdx.x * P;
    const uint32_t np = (uint32_t)min((uint64_t)P, nin - g0);
    const uint32_t tid = threadIdx.x;

    uint64_t runs = 0;
    for (uint32_t t = tid; t < np; t += kComposeThreads) {
        const uint32_t cl = in_cls[g0 + t];
        s_cls[t] = cl;
        const uint32_t sz = loff[cl + 1] - loff[cl];
        s_sz[t] = sz;
        runs += in_runs ? in_runs[g0 + t] : (uint64_t)sz;
    }
    s_red[tid] = runs;
    __syncthreads();
    for (uint32_t t = tid; t < np * RM; t += kComposeThreads) {
        const uint32_t i = t / RM, j = t - i * RM;
        if (j < s_sz[i]) {
            s_end[t] = in_end[(g0 + i) * RM + j];
            s_cnt[t] = (uint64_t)in_cnt[(g0 + i) * RM + j];
        }
    }
    for (uint32_t w = kComposeThreads / 2; w > 0; w >>= 1) {
        if (tid < w) s_red[tid] += s_red[tid + w];
        __syncthreads();
    }
    for (uint32_t w = 1; w < np; w <<= 1) {
        const uint32_t npairs = (np + 2 * w - 1) / (2 * w);
        for (uint32_t t = tid; t < npairs * RM; t += kComposeThreads) {
            const uint32_t i = t / RM, j = t - i * RM;
            const uint32_t left = i * 2 * w, right = left + w;
            if (right < np && j < s_sz[left]) {
                const uint32_t e = s_end[left * RM + j];
                const int k = find_state(llist + loff[s_cls[right]], s_sz[right], e);
                if (k < 0) {
                    s_end[left * RM + j] = sent;  // only the sentinel leaves the lists
                } else {
                    s_end[left * RM + j] = s_end[right * RM + (uint32_t)k];
                    s_cnt[left * RM + j] += s_cnt[right * RM + (uint32_t)k];
                }
            }
        }
        __syncthreads();
    }
    for (uint32_t j = tid; j < s_sz[0]; j += kComposeThreads) {
        out_end[(uint64_t)blockIdx.x * RM + j] = s_end[j];
        out_cnt[(uint64_t)blockIdx.x * RM + j] = s_cnt[j];
    }
    if (tid == 0) {
        out_cls[blockIdx.x] = s_cls[0];
        out_runs[blockIdx.x] = s_red[0];
        if (result != nullptr && gridDim.x == 1) {
            const uint32_t e = s_end[0];
            parem_result r;
            if (e == sent) {
                r.final_state = 0xffffffffu;
                r.accept = 0;
                r.count = 0;
            } else {
                r.final_state = e;
                r.accept = final_flag[e];
                r.count = s_cnt[0];
            }
            r.chunks = chunks;
            r.spec_runs = s_red[0];
            r.rerun_chunks = 0;
            *result = r;
        }
    }
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

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

static uint32_t compose_lds(uint32_t P, uint32_t RM) { return P * RM * 12u + P * 8u; }

parem_status plan_plain(const DeviceDfa &d, uint64_t len, PlainPlan *p) {
    PlainPlan q;
    q.n = len;
    q.RM = d.max_spec;
    uint32_t L = d.opt.chunk_len;
    if (L == 0) {
        // about 2^18 chunks for large texts, at least 256 bytes each
        uint64_t want = len >> 18;
        L = 256;
        while ((uint64_t)L < want && L < (1u << 20)) L <<= 1;
    }
    if (L % 64 != 0 || L == 0) return PAREM_EINVAL;
    q.L = L;
    q.chunks = (len + L - 1) / L;
    uint32_t G = d.opt.group ? d.opt.group : 8;
    if (G != 2 && G != 4 && G != 8 && G != 16) return PAREM_EINVAL;
    q.G = G;
    uint32_t P = 256;
    while (P > 2 && compose_lds(P, q.RM) > 64 * 1024) P >>= 1;
    if (compose_lds(P, q.RM) > 150 * 1024) return PAREM_EUNSUPPORTED;
    q.P = P;
    uint64_t m = q.chunks;
    while (m > 1) {
        m = (m + P - 1) / P;
        q.level_maps.push_back(m);
    }
    q.level_cap = q.chunks > 1 ? (q.chunks + P - 1) / P : 1;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const uint64_t cm = std::max<uint64_t>(q.chunks, 1) * q.RM;
    q.off_cend = take(cm * 4);
    q.off_ccnt = take(cm * 4);
    q.off_ccls = take(std::max<uint64_t>(q.chunks, 1) * 4);
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

template <typename E, bool LDS, bool ALIGNED>
static void launch_walk_g(const DeviceDfa &d, const PlainPlan &p, const uint8_t *text, uint8_t *ws,
                          hipStream_t stream) {
    const uint32_t grid = (uint32_t)((p.chunks + kWalkThreads - 1) / kWalkThreads);
    const uint32_t entries = (d.Q + 1) * 256;
    const size_t lds = LDS ? ((size_t)entries * sizeof(E) + 15) / 16 * 16 : 0;
    auto *me = reinterpret_cast<uint32_t *>(ws + p.off_cend);
    auto *mc = reinterpret_cast<uint32_t *>(ws + p.off_ccnt);
    auto *ml = reinterpret_cast<uint32_t *>(ws + p.off_ccls);
    const E *tab = reinterpret_cast<const E *>(d.d_table);
    const uint32_t start_class = d.A + 1;
#define PAREM_WALK(GG)                                                                                        \
    hipLaunchKernelGGL((k_walk_byte<E, GG, LDS, ALIGNED>), dim3(grid), dim3(kWalkThreads), lds, stream, text, \
                       p.n, p.L, p.chunks, tab, entries, d.d_cls, d.d_loff, d.d_llist, start_class, p.RM, me, mc, ml)
    switch (p.G) {
        case 2: PAREM_WALK(2); break;
        case 4: PAREM_WALK(4); break;
        case 8: PAREM_WALK(8); break;
        default: PAREM_WALK(16); break;
    }
#undef PAREM_WALK
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
    if (d.layout == PAREM_LAYOUT_BYTE_LDS) {
        if (aligned) launch_walk_g<uint8_t, true, true>(d, p, d_text, ws, stream);
        else launch_walk_g<uint8_t, true, false>(d, p, d_text, ws, stream);
    } else if (d.layout == PAREM_LAYOUT_BYTE_GLOBAL) {
        if (aligned) launch_walk_g<uint16_t, false, true>(d, p, d_text, ws, stream);
        else launch_walk_g<uint16_t, false, false>(d, p, d_text, ws, stream);
    } else {
        return PAREM_EUNSUPPORTED;
    }
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    if (ev_end && hipEventRecord(ev_end, stream) != hipSuccess) return PAREM_EDEVICE;

    // compose levels
    const size_t lds = compose_lds(p.P, p.RM);
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose<uint32_t>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose<uint64_t>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return PAREM_EDEVICE;
    }
    const uint32_t *ie = reinterpret_cast<const uint32_t *>(ws + p.off_cend);
    const uint32_t *ic32 = reinterpret_cast<const uint32_t *>(ws + p.off_ccnt);
    const uint32_t *il = reinterpret_cast<const uint32_t *>(ws + p.off_ccls);
    const uint64_t *ic64 = nullptr;
    const uint64_t *ir = nullptr;
    uint64_t nin = p.chunks;
    bool use_a = true;
    bool first = true;
    do {
        const uint64_t nout = (nin + p.P - 1) / p.P;
        uint32_t *oe = reinterpret_cast<uint32_t *>(ws + (use_a ? p.off_a_end : p.off_b_end));
        uint64_t *oc = reinterpret_cast<uint64_t *>(ws + (use_a ? p.off_a_cnt : p.off_b_cnt));
        uint32_t *ol = reinterpret_cast<uint32_t *>(ws + (use_a ? p.off_a_cls : p.off_b_cls));
        uint64_t *orr = reinterpret_cast<uint64_t *>(ws + (use_a ? p.off_a_runs : p.off_b_runs));
        parem_result *res = nout == 1 ? d_out : nullptr;
        if (first) {
            hipLaunchKernelGGL(k_compose<uint32_t>, dim3((uint32_t)nout), dim3(kComposeThreads), lds, stream, ie,
                               ic32, il, ir, nin, p.RM, p.P, d.d_loff, d.d_llist, d.sent, oe, oc, ol, orr,
                               d.d_final, res, p.chunks);
        } else {
            hipLaunchKernelGGL(k_compose<uint64_t>, dim3((uint32_t)nout), dim3(kComposeThreads), lds, stream, ie,
                               ic64, il, ir, nin, p.RM, p.P, d.d_loff, d.d_llist, d.sent, oe, oc, ol, orr,
                               d.d_final, res, p.chunks);
        }
        if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
        ie = oe;
        ic64 = oc;
        il = ol;
        ir = orr;
        nin = nout;
        use_a = !use_a;
        first = false;
    } while (nin > 1);
    return PAREM_OK;
}

}  // namespace parem

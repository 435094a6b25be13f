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

#include <mutex>

namespace parem {

__global__ __launch_bounds__(kComposeThreads) void k_compose_chunks(const uint32_t *__restrict__ map,
                                                                     const uint16_t *__restrict__ map_cls,
                                                                     const uint16_t *__restrict__ map_lead,
                                                                     ComposeArgs a, SegOut o,
                                                                     parem_result *__restrict__ result) {
    extern __shared__ __align__(16) uint8_t smem[];
    compose_chunks_seg(smem, map, map_cls, map_lead, a, o, blockIdx.x, result);
}

// First level for wide maps (P <= 64 chunk maps a group, so the LDS tree
// allows few groups per CU): one wave per group. A group whose maps are all
// uniform composes here, as compose_chunks_seg does it (each map sends every
// walk to its lead: chain the leads through the maps, sum the counts, and
// give each entry of the group's first map the chain's end); a group with a
// non-uniform map is flagged in `todo` (one u32 per group, written by every
// group) for k_compose_chunks_list.
__global__ __launch_bounds__(256) void k_compose_chunks_uniform(const uint32_t *__restrict__ map,
                                                                const uint16_t *__restrict__ map_cls,
                                                                const uint16_t *__restrict__ map_lead, ComposeArgs a,
                                                                SegOut o, uint64_t ngroups, uint32_t *__restrict__ todo) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t seg = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    if (seg >= ngroups) return;  // whole waves leave; no workgroup barrier follows
    const uint64_t g0 = seg * a.P, C = a.chunks;
    const uint32_t np = (uint32_t)min((uint64_t)a.P, C - g0);
    uint32_t cl = 0, sz = 0, lead = 0;
    bool nonuni = false;
    if (lane < np) {
        const uint32_t v = map_cls[g0 + lane];
        cl = v & 0x7fffu;
        sz = a.loff[cl + 1] - a.loff[cl];
        nonuni = (v & 0x8000u) != 0;
        lead = map_lead[g0 + lane];
    }
    const bool tree = __any(nonuni);
    if (lane == 0) todo[seg] = tree ? 1u : 0u;
    if (tree) return;
    const uint32_t prev = (uint32_t)__shfl_up((int)lead, 1, 64);
    unsigned long long contrib = 0;
    int fail = 0;
    if (lane >= 1 && lane < np) {
        int x = -1;
        if (prev < a.Q1) {
            if (a.inv) {
                const uint32_t v = a.inv[cl * a.Q1 + prev];
                x = v == 0xffffu ? -1 : (int)v;
            } else {
                x = find_state(a.llist + a.loff[cl], sz, prev);
            }
        }
        const uint32_t v = x < 0 ? kAbsent16 : map[(uint64_t)x * C + g0 + lane];
        if ((v & 0xffffu) == kAbsent16) fail = 1;
        else contrib = v >> 16;
    }
    unsigned long long runs = sz;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        contrib += (unsigned long long)__shfl_xor((long long)contrib, off, 64);
        runs += (unsigned long long)__shfl_xor((long long)runs, off, 64);
    }
    fail = __any(fail);
    const uint32_t last = (uint32_t)__shfl((int)lead, (int)np - 1, 64);
    const uint32_t end = fail ? a.sent : last;
    const uint32_t sz0 = (uint32_t)__shfl((int)sz, 0, 64), cl0 = (uint32_t)__shfl((int)cl, 0, 64);
    for (uint32_t j = lane; j < sz0; j += 64) {
        const uint32_t v = map[(uint64_t)j * C + g0];
        o.end[seg * a.RM + j] = (v & 0xffffu) != kAbsent16 ? end : kAbsent32;
        o.cnt[seg * a.RM + j] = (uint64_t)(v >> 16) + contrib;
    }
    if (lane == 0) {
        o.cls[seg] = cl0;
        o.runs[seg] = runs;
        o.lead[seg] = end;
    }
}

// the first-level groups k_compose_chunks_uniform flagged, through the LDS
// tree; workgroups stride over the groups
__global__ __launch_bounds__(kComposeThreads) void k_compose_chunks_list(const uint32_t *__restrict__ map,
                                                                          const uint16_t *__restrict__ map_cls,
                                                                          const uint16_t *__restrict__ map_lead,
                                                                          ComposeArgs a, SegOut o, uint64_t ngroups,
                                                                          const uint32_t *__restrict__ todo) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (uint64_t k = blockIdx.x; k < ngroups; k += gridDim.x) {
        if (!todo[k]) continue;  // the same for the whole workgroup
        compose_chunks_seg(smem, map, map_cls, map_lead, a, o, k, nullptr);
        __syncthreads();  // the next group reuses the LDS
    }
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
                        uint8_t *__restrict__ done, uint32_t *__restrict__ flags, uint32_t escalate,
                        uint32_t *__restrict__ round_count, uint32_t *__restrict__ rlist, uint32_t first) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    redo[c] = 0;
    // the first round starts every chunk as not walked from its whole set
    const bool was_done = first ? false : done[c] != 0;
    if (first) done[c] = 0;
    if (c == 0 || was_done) return;
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
            const uint32_t at = atomicAdd(round_count, 1u);
            if (at < kSplitMax) rlist[at] = (uint32_t)c;
        }
    }
}

// second half of an escalation: if some chunk is still uncovered, every
// chunk not yet walked from its whole set is marked. The marks are final
// here, so the statistics are summed too: walks started (the selection, plus
// the whole set of a marked chunk) and chunks walked again; one partial pair
// per block (256 threads), added up by k_stats_total.
__global__ void k_escalate(uint64_t C, uint8_t *__restrict__ redo, uint8_t *__restrict__ done,
                           uint32_t *__restrict__ flags, uint32_t *__restrict__ round_count,
                           uint32_t *__restrict__ rlist, const uint8_t *__restrict__ nsel,
                           const uint16_t *__restrict__ map_cls, const uint32_t *__restrict__ loff,
                           const uint8_t *__restrict__ lnsel, unsigned long long *__restrict__ part_out) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long runs = 0, again = 0;
    if (c < C) {
        bool dn = done[c] != 0;
        if (c > 0 && !dn && flags[1] != 0) {
            redo[c] = 1;
            done[c] = 1;
            atomicAdd(&flags[0], 1u);
            const uint32_t at = atomicAdd(round_count, 1u);
            if (at < kSplitMax) rlist[at] = (uint32_t)c;
            dn = true;
        }
        runs = nsel[c];
        if (dn) {
            // walked again from its lookback set (lnsel, when that is not the
            // whole set) or from its whole speculated set
            const uint32_t cl = map_cls[c] & 0x7fffu;
            const uint32_t ln = lnsel ? lnsel[c] : 0u;
            runs += ln ? ln : loff[cl + 1] - loff[cl];
            again = 1;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        runs += (unsigned long long)__shfl_xor((long long)runs, o, 64);
        again += (unsigned long long)__shfl_xor((long long)again, o, 64);
    }
    __shared__ unsigned long long sum[2][4];
    if ((threadIdx.x & 63u) == 0) {
        sum[0][threadIdx.x >> 6] = runs;
        sum[1][threadIdx.x >> 6] = again;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part_out[2 * blockIdx.x] = sum[0][0] + sum[0][1] + sum[0][2] + sum[0][3];
        part_out[2 * blockIdx.x + 1] = sum[1][0] + sum[1][1] + sum[1][2] + sum[1][3];
    }
}

// the learned statistics into the result: sums of n partial pairs
__global__ void k_stats_total(const unsigned long long *__restrict__ part, uint32_t n,
                              parem_result *__restrict__ result) {
    unsigned long long r = 0, g = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        r += part[2 * i];
        g += part[2 * i + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        r += (unsigned long long)__shfl_xor((long long)r, o, 64);
        g += (unsigned long long)__shfl_xor((long long)g, o, 64);
    }
    if (threadIdx.x == 0) {
        result->spec_runs = r;
        result->rerun_chunks = g;
    }
}

// ---------------------------------------------------------------------------
// sub-chunk re-walk (learned speculation). A chunk marked for a walk from its
// whole set R_c is walked by one workgroup as up to 64 sub-chunks at once:
// sub-chunk k runs from every state of Algorithm 1's set for its own start
// (the image of the column of the byte before it; R_c for k = 0), and the
// sub-chunk maps are then chained for every state of R_c, which is the
// composition of Algorithm 1 applied inside the chunk. The entries written
// equal those of the whole-set walk (end | count << 16, the class with bit 15
// when the ends differ, the end from position 0; the sentinel for every
// entry when the chunk holds a byte outside the alphabet), and the chunk is
// unmarked, so the whole-set walk launched after this kernel skips it. One
// chunk's serial walk of L bytes becomes 64 walks of L / 64 bytes; with more
// than kSplitMax chunks marked in a round the kernel leaves every chunk to
// the whole-set walk, whose lanes then carry the load. After a chunk, its
// successor (when not marked already) is checked against the new ends, as the
// next coverage round would, and walked the same way when uncovered (at most
// kSplitHops successors, so that a chain of uncovered chunks is not walked
// serially: the escalation takes what is left): only the workgroup of chunk
// c ever reaches c + 1 this way, and a marked successor is walked from its
// whole set anyway, so no chunk is walked twice at once.
// ---------------------------------------------------------------------------
constexpr uint32_t kSplitSub = 64;
constexpr uint32_t kSplitThreads = 1024;
constexpr uint32_t kSplitHops = 4;  // successors one workgroup walks after a marked chunk

struct SplitArgs {
    const uint8_t *text;
    uint64_t n;
    uint32_t L;
    uint64_t C;
    const uint8_t *cls;
    const uint32_t *loff;
    const uint32_t *llist;
    const uint16_t *step;  // [(Q+1) x (A+1)] next | final << 15
    const uint16_t *inv;   // [(A+2) x (Q+1)] position in each class list
    uint32_t Q1, A1, sent;
    uint32_t inv_lds;      // bytes of inv staged in LDS (0: read from L2)
    uint32_t *map;
    uint16_t *map_cls;
    uint16_t *map_lead;
    uint8_t *redo;
    uint8_t *done;
    uint32_t *marked;      // chunks marked so far (flags[0])
    const uint32_t *rlist;
    const uint32_t *count;
};

struct SplitLds {
    uint32_t step, inv, ctab, cb, sub, kinfo, bytes;
};
__host__ __device__ static SplitLds split_lds(uint32_t Q1, uint32_t A1, uint32_t inv_lds, uint32_t L) {
    SplitLds o;
    uint32_t off = 0;
    o.step = off;
    off += (Q1 * A1 * 2 + 15) & ~15u;
    o.inv = off;
    off += (inv_lds + 15) & ~15u;
    o.ctab = off;
    off += 256;
    o.cb = off;
    off += (L + 15) & ~15u;
    o.sub = off;
    off += kSplitSub * 64 * 4;
    o.kinfo = off;
    off += (4 * kSplitSub + kSplitSub + 1) * 4;
    o.bytes = off;
    return o;
}

__global__ __launch_bounds__(kSplitThreads) void k_redo_split(SplitArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t marked = *a.count;
    if (marked == 0 || marked > kSplitMax || blockIdx.x >= marked) return;
    const uint32_t tid = threadIdx.x;
    const SplitLds o = split_lds(a.Q1, a.A1, a.inv_lds, a.L);
    uint16_t *T = reinterpret_cast<uint16_t *>(smem + o.step);
    uint16_t *IV = reinterpret_cast<uint16_t *>(smem + o.inv);
    uint8_t *CT = smem + o.ctab;
    uint8_t *CB = smem + o.cb;
    uint32_t *SUB = reinterpret_cast<uint32_t *>(smem + o.sub);
    uint32_t *kcls = reinterpret_cast<uint32_t *>(smem + o.kinfo);
    uint32_t *klo = kcls + kSplitSub, *ksz = klo + kSplitSub, *kfrom = ksz + kSplitSub, *koff = kfrom + kSplitSub;
    for (uint32_t i = tid; i < a.Q1 * a.A1; i += kSplitThreads) T[i] = a.step[i];
    for (uint32_t i = tid; i < a.inv_lds / 2; i += kSplitThreads) IV[i] = a.inv[i];
    if (tid < 256) CT[tid] = a.cls[tid];
    __syncthreads();
    __shared__ uint32_t s_next;
    for (uint32_t it = blockIdx.x; it < marked; it += gridDim.x) {
      for (uint64_t c = a.rlist[it], hop = 0;; ++c, ++hop) {  // c >= 1: chunk 0 is never marked
        const uint64_t b = c * (uint64_t)a.L;
        const uint32_t len = (uint32_t)min((uint64_t)a.L, a.n - b);
        const uint32_t P = min(kSplitSub, len);
        // classes of the chunk's bytes
        const uint8_t *src = a.text + b;
        if ((reinterpret_cast<uintptr_t>(src) & 15u) == 0) {
            for (uint32_t i = 16 * tid; i < len; i += 16 * kSplitThreads) {
                if (i + 16 <= len) {
                    const uint4 q = *reinterpret_cast<const uint4 *>(src + i);
                    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int h = 0; h < 16; ++h) CB[i + h] = CT[(w[h >> 2] >> (8 * (h & 3))) & 0xffu];
                } else {
                    for (uint32_t h = i; h < len; ++h) CB[h] = CT[src[h]];
                }
            }
        } else {
            for (uint32_t i = tid; i < len; i += kSplitThreads) CB[i] = CT[src[i]];
        }
        // sub-chunk k covers [k len / P, (k+1) len / P); its set follows the byte before it
        if (tid < P) {
            const uint32_t from = tid * len / P;
            const uint32_t cl = CT[a.text[b + from - 1]];
            const uint32_t lo = a.loff[cl];
            kcls[tid] = cl;
            klo[tid] = lo;
            ksz[tid] = a.loff[cl + 1] - lo;
            kfrom[tid] = from;
        }
        __syncthreads();
        if (tid < 64) {
            // offsets of the sub-chunk walks (inclusive scan over the wave)
            uint32_t v = tid < P ? ksz[tid] : 0u;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t u = (uint32_t)__shfl_up((int)v, d, 64);
                if ((int)tid >= d) v += u;
            }
            koff[tid + 1] = v;
            if (tid == 0) koff[0] = 0;
        }
        __syncthreads();
        const uint32_t total = koff[P];
        for (uint32_t task = tid; task < total; task += kSplitThreads) {
            uint32_t lo = 0, hi = P;  // koff[lo] <= task < koff[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (koff[mid] <= task) lo = mid;
                else hi = mid;
            }
            const uint32_t k = lo, j = task - koff[k];
            const uint32_t to = k + 1 < P ? kfrom[k + 1] : len;
            uint32_t e = a.llist[klo[k] + j], cnt = 0;
#pragma unroll 4
            for (uint32_t i = kfrom[k]; i < to; ++i) {
                const uint32_t v = T[e * a.A1 + CB[i]];
                e = v & 0x7fffu;
                cnt += v >> 15;
            }
            // the chain needs the end's position in the next sub-chunk's set
            // (0xffff: the sentinel, or not in the set); the last keeps the state
            uint32_t out = e;
            if (k + 1 < P) {
                const uint32_t ix = kcls[k + 1] * a.Q1 + e;
                const uint32_t pos = e == a.sent ? 0xffffu : (a.inv_lds ? IV[ix] : a.inv[ix]);
                out = pos < ksz[k + 1] ? pos : 0xffffu;
            }
            SUB[task] = out | (cnt << 16);
        }
        __syncthreads();
        if (tid < 64) {
            // chain every state of R_c through the sub-chunk maps
            const uint32_t sz0 = ksz[0];
            const bool act = tid < sz0;
            uint32_t e = 0, cnt = 0;
            if (act) {
                uint32_t pos = tid;
                for (uint32_t k = 0; k < P; ++k) {
                    const uint32_t v = SUB[koff[k] + pos];
                    cnt += v >> 16;
                    pos = v & 0xffffu;
                    if (k + 1 == P) {
                        e = pos;
                    } else if (pos == 0xffffu) {
                        e = a.sent;
                        break;
                    }
                }
            }
            const uint32_t lead = (uint32_t)__shfl((int)e, 0, 64);
            const bool nonuni = __any(act && e != lead);
            if (act) a.map[(uint64_t)tid * a.C + c] = e == a.sent ? a.sent : (e | (cnt << 16));
            // the successor's coverage of the new ends (as chunk_present)
            bool go = false;
            if (hop < kSplitHops && c + 1 < a.C && a.done[c + 1] == 0) {
                const uint32_t ncl = a.map_cls[c + 1] & 0x7fffu;
                bool miss = false;
                if (act && e != a.sent) {
                    const uint32_t ix = ncl * a.Q1 + e;
                    const uint32_t pos = a.inv_lds ? IV[ix] : a.inv[ix];
                    miss = pos == 0xffffu || (a.map[(uint64_t)pos * a.C + c + 1] & 0xffffu) == kAbsent16;
                }
                go = __any(miss);
            }
            if (tid == 0) {
                a.map_cls[c] = (uint16_t)(kcls[0] | (nonuni ? 0x8000u : 0u));
                a.map_lead[c] = (uint16_t)lead;
                a.redo[c] = 0;
                if (go) {
                    a.done[c + 1] = 1;
                    atomicAdd(a.marked, 1u);
                }
                s_next = go ? 1u : 0u;
            }
        }
        __syncthreads();
        if (!s_next) break;
      }
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

// S filter of a partial table (Algorithm 1's R = S intersect L): for chunk
// c >= 1 the positions, in the list of the class of the byte before it (L,
// completed with `dead`), of the states other than dead that have a
// transition on the chunk's first byte. At most kLookCap are selected (more: nsel 0, the whole list is
// walked, states outside S die on the first byte); none: position 0 is
// walked (it dies at once, or is dead), so the map still has a leader. The
// walks of S intersect L (1 for chunk 0) are tallied in acc[0].
__global__ void k_sfilter(const uint8_t *__restrict__ text, uint64_t n, uint32_t L, uint64_t C,
                          const uint8_t *__restrict__ cls, uint32_t A, const uint32_t *__restrict__ loff,
                          const uint32_t *__restrict__ llist, const uint16_t *__restrict__ next, uint32_t dead,
                          uint16_t *__restrict__ sel, uint8_t *__restrict__ nsel,
                          unsigned long long *__restrict__ acc) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long runs = 0;
    if (c < C) {
        if (c == 0) {
            nsel[0] = 0;
            runs = 1;
        } else {
            const uint64_t b = c * (uint64_t)L;
            const uint32_t pc = cls[text[b - 1]], x = cls[text[b]];
            if (pc >= A || x >= A) {
                nsel[c] = 0;  // a byte outside the alphabet: the walk reports it
            } else {
                const uint32_t lo = loff[pc], sz = loff[pc + 1] - lo;
                uint16_t *s = sel + c * kLookCap;
                uint32_t k = 0;
                for (uint32_t j = 0; j < sz; ++j) {
                    const uint32_t r = llist[lo + j];
                    if (r != dead && next[r * A + x] != dead) {
                        if (k < kLookCap) s[k] = (uint16_t)j;
                        ++k;
                    }
                }
                runs = k;
                if (k == 0) s[0] = 0;
                nsel[c] = k > kLookCap ? 0 : (uint8_t)max(k, 1u);
            }
        }
    }
    (void)n;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) runs += (unsigned long long)__shfl_xor((long long)runs, o, 64);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = runs;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&acc[0], part[0] + part[1] + part[2] + part[3]);
}

// the internal dead state of a partial table reads PAREM_DEAD_STATE outside
__global__ void k_dead_result(parem_result *__restrict__ r, uint32_t dead) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && r->final_state == dead) {
        r->final_state = PAREM_DEAD_STATE;
        r->accept = 0;
    }
}

__global__ void k_dead_states(uint32_t *__restrict__ states, uint64_t C, uint32_t dead) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C && states[c] == dead) states[c] = PAREM_DEAD_STATE;
}

// `only` (may be null): chunks with only[c] == 0 are skipped
__global__ __launch_bounds__(256) void k_lookback(LookArgs a, uint32_t start, uint32_t wave_bytes,
                                                  const uint8_t *__restrict__ only) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint64_t c = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    if (c >= a.nchunks) return;  // whole waves leave; no workgroup barrier follows
    if (only && only[c] == 0) return;
    lookback_chunk(a, start, c, smem + (threadIdx.x >> 6) * wave_bytes);
}

// Lookback sets over the sparse layout's slot image (uniform form, every
// byte valid; windows of 2..kSlotLookMaxK bytes, at most the chunk length):
// one lane per chunk instead of one wave, the image read from LDS. The image
// of every state under the window's first byte is that byte's class list;
// each further byte maps the states collected so far through one slot read
// each. The shared default D is kept as a flag, since most states fall back
// to it; the others (at most kSlotLookCap, else the chunk walks its whole
// set) sit in LDS, element k of thread t at k * kSparseThreads + t.
// Duplicates are dropped at the end; the states become positions in the
// class list of the chunk's previous byte (ascending, as k_lookback writes
// them). Chunk 0 starts in q0 at position 0 of the start class.
constexpr uint32_t kSlotLookCap = 32;
constexpr uint32_t kSlotLookMaxK = 16;
static_assert(kSparseLdsMax + kSlotLookCap * kSparseThreads * 2 <= 160 * 1024, "slot lookback exceeds LDS");

__global__ __launch_bounds__(kSparseThreads) void k_lookback_slots(LookArgs a, const uint32_t *__restrict__ walk_list,
                                                                   const uint8_t *__restrict__ g_table,
                                                                   uint32_t table_bytes,
                                                                   const uint16_t *__restrict__ sids, uint32_t d0) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table<kSparseThreads>(reinterpret_cast<uint4 *>(smem), reinterpret_cast<const uint4 *>(g_table),
                                table_bytes / 16u);
    // no workgroup barrier follows: lanes past the last chunk leave
    const uint64_t c = (uint64_t)blockIdx.x * kSparseThreads + threadIdx.x;
    if (c >= a.nchunks) return;
    uint16_t *out = a.sel + c * kLookCap;
    if (c == 0) {
        a.nsel[0] = 1;
        out[0] = 0;
        return;
    }
    uint16_t *buf = reinterpret_cast<uint16_t *>(smem + table_bytes) + threadIdx.x;
    constexpr uint32_t T = kSparseThreads;
    const uint32_t dbase = d0 & 0xffffu;
    // slot-image step of the uniform form (the slots start at LDS address 256)
    auto step = [&](uint32_t base, uint32_t x) -> uint32_t {
        const uint32_t e = lds_abs<uint32_t>(256u + 4u * (base + x));
        return (e >> 24) == x ? (e & 0xffffu) : dbase;
    };
    const uint8_t *win = a.text + (c * (uint64_t)a.L - a.K);
    const uint32_t cl0 = a.cls[win[0]];
    const uint32_t lo = a.loff[cl0], hi = a.loff[cl0 + 1];
    uint32_t n = 0;
    bool has_d = false, over = false;
    const uint32_t x1 = win[1];
    // eight list entries loaded before their steps (the list is read through L2)
    for (uint32_t i0 = lo; i0 < hi && !over; i0 += 8) {
        uint32_t v[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) v[u] = walk_list[min(i0 + u, hi - 1)];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) {
            if (i0 + u >= hi) break;
            const uint32_t r = step(v[u] & 0xffffu, x1);
            if (r == dbase) has_d = true;
            else if (n < kSlotLookCap) buf[T * n++] = (uint16_t)r;
            else over = true;
        }
    }
    for (uint32_t k = 2; k < a.K && !over; ++k) {
        const uint32_t x = win[k];
        uint32_t m = 0;
        bool nd = false;
        for (uint32_t j = 0; j < n; ++j) {  // in place: m <= j
            const uint32_t r = step(buf[T * j], x);
            if (r == dbase) nd = true;
            else buf[T * m++] = (uint16_t)r;
        }
        if (has_d) {
            const uint32_t r = step(dbase, x);
            if (r == dbase) nd = true;
            else if (m < kSlotLookCap) buf[T * m++] = (uint16_t)r;
            else over = true;
        }
        n = m;
        has_d = nd;
    }
    if (!over && has_d) {
        if (n < kSlotLookCap) buf[T * n++] = (uint16_t)dbase;
        else over = true;
    }
    if (over) {
        a.nsel[c] = 0;  // the whole set
        return;
    }
    // positions in the class list of the previous byte, sorted, duplicates dropped
    const uint16_t *pos = a.inv + (size_t)a.cls[win[a.K - 1]] * (a.Q + 1);
    uint32_t cnt = 0;
    bool missing = false;
    for (uint32_t j = 0; j < n; ++j) {
        const uint32_t id = sids[buf[T * j]];
        const uint32_t p = id <= a.Q ? pos[id] : 0xffffu;
        missing |= p == 0xffffu;
        uint32_t at = cnt;
        while (at > 0 && out[at - 1] > p) --at;
        if (at > 0 && out[at - 1] == p) continue;
        for (uint32_t q = cnt; q > at; --q) out[q] = out[q - 1];
        out[at] = (uint16_t)p;
        ++cnt;
    }
    a.nsel[c] = missing ? 0 : (uint8_t)cnt;  // a state outside R_c cannot occur
}

static bool slot_lookback(const DeviceDfa &d, const PlainPlan &p) {
    return d.layout == PAREM_LAYOUT_SPARSE_LDS && d.sparse_uniform && d.sparse_raw && p.look >= 2 &&
           p.look <= kSlotLookMaxK && p.look <= p.L;
}

__global__ void k_learned_total(const unsigned long long *__restrict__ acc, parem_result *__restrict__ result) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        result->spec_runs = acc[0];
        result->rerun_chunks = acc[1];
    }
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

parem_status plan_chunks(const DeviceDfa &d, uint64_t len, const parem_options &o, bool keep, PlainPlan *p,
                         bool wide_segs) {
    PlainPlan q;
    q.n = len;
    q.RM = d.max_spec;
    uint32_t L = o.chunk_len;
    if (L == 0) {
        // about 2^17 chunks for large texts (two 256-lane workgroups per CU
        // on a 1 GiB text), 2^18 for sparse rows (one 1024-lane workgroup
        // per CU), at least 256 bytes each
        uint64_t want = len >> (d.layout == PAREM_LAYOUT_SPARSE_LDS ? 18 : 17);
        L = 256;
        while ((uint64_t)L < want && L < kMaxChunk) L <<= 1;
    }
    if (L % 64 != 0 || L == 0 || L > kMaxChunk) return PAREM_EINVAL;
    q.L = L;
    q.chunks = (len + L - 1) / L;
    q.look = (o.lookback && d.d_next && d.d_inv) ? o.lookback : 0u;
    q.sfilter = d.dead != 0xffffffffu;
    q.tile = o.tile ? o.tile : 128;
    q.merge = o.no_merge ? 0u : 1u;
    if (q.tile != 64 && q.tile != 128) return PAREM_EINVAL;
    // sparse layout: eight runs a pass fit the 128 registers of four waves
    // per SIMD (a few spills outside the walk loop; 4 GiB Zipf text over the
    // 4096-state byte DFA: 1.90 against 1.98 ms with four). k-gram tables:
    // sixteen when a set holds more than eight states, so that one pass
    // walks it (the LDS already limits these kernels to two waves per SIMD,
    // which leaves the registers; 1 GiB DNA motif: 197 against 205 us)
    uint32_t G = o.group ? o.group : 8;
    if (!o.group && d.layout == PAREM_LAYOUT_KGRAM_LDS && d.max_spec > 8) G = 16;
    if (G != 2 && G != 4 && G != 8 && G != 16) return PAREM_EINVAL;
    q.G = G;
    uint32_t P = 256;
    while (P > 2 && compose_lds(P, q.RM, d.inv_lds) > 64 * 1024) P >>= 1;
    if (compose_lds(P, q.RM, d.inv_lds) > 150 * 1024) return PAREM_EUNSUPPORTED;
    q.P = P;
    // later levels: with wide_segs up to 512 segment maps a workgroup (LDS
    // up to 150 KiB), so that 2^17 chunks need two levels, not three
    uint32_t P2 = P;
    while (wide_segs && P2 < 512 && compose_lds(2 * P2, q.RM, d.inv_lds) <= 150 * 1024) P2 <<= 1;
    q.P2 = P2;
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
    if (q.look || q.sfilter) {
        q.off_sel = take(ch * kLookCap * 2);  // lookback / S-filter selection (positions in R_c)
        q.off_nsel = take(ch);
        q.off_flags = take(64);               // speculated-walk tally
    }
    // segment levels: kept separately (down-sweep) or two ping-pong buffers
    uint64_t m = q.chunks;
    q.levels.clear();
    do {
        const uint32_t fan = q.levels.empty() ? P : P2;
        m = (m + fan - 1) / fan;
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
    // wide maps: first-level groups of uniform maps compose one wave each,
    // the others are listed for the LDS tree
    q.off_todo = (P <= 64 && q.levels[0] > 1) ? take(q.levels[0] * 4) : 0;
    q.keep = keep;
    q.bytes = off;
    *p = q;
    return PAREM_OK;
}

parem_status plan_plain(const DeviceDfa &d, uint64_t len, PlainPlan *p) {
    return plan_chunks(d, len, d.opt, false, p, true);
}

template <int MODE>
static void launch_walk(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, hipStream_t stream,
                        bool aligned) {
    switch (d.layout) {
        case PAREM_LAYOUT_KGRAM_LDS: launch_walk_family<PAREM_LAYOUT_KGRAM_LDS, MODE>(d, p, a, stream, aligned); break;
        case PAREM_LAYOUT_BYTE_LDS: launch_walk_family<PAREM_LAYOUT_BYTE_LDS, MODE>(d, p, a, stream, aligned); break;
        case PAREM_LAYOUT_HOT_LDS: launch_walk_family<PAREM_LAYOUT_HOT_LDS, MODE>(d, p, a, stream, aligned); break;
        case PAREM_LAYOUT_CLASS_LDS: launch_walk_family<PAREM_LAYOUT_CLASS_LDS, MODE>(d, p, a, stream, aligned); break;
        case PAREM_LAYOUT_SPARSE_LDS: launch_walk_family<PAREM_LAYOUT_SPARSE_LDS, MODE>(d, p, a, stream, aligned); break;
        default: launch_walk_family<PAREM_LAYOUT_BYTE_GLOBAL, MODE>(d, p, a, stream, aligned); break;
    }
}

static parem_status launch_compose(const DeviceDfa &d, const PlainPlan &p, uint8_t *ws, hipStream_t stream,
                                   parem_result *d_out) {
    const ComposeArgs a = compose_args(d, p);
    ComposeArgs a2 = a;
    a2.P = p.P2;
    const size_t lds = compose_lds(p.P, p.RM, d.inv_lds);
    const size_t lds2 = compose_lds(p.P2, p.RM, d.inv_lds);
    if (lds > 64 * 1024 && hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose_chunks),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return PAREM_EDEVICE;
    if (lds2 > 64 * 1024 && hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose_segs),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2) != hipSuccess)
        return PAREM_EDEVICE;
    const uint32_t *map = reinterpret_cast<const uint32_t *>(ws + p.off_map);
    const uint16_t *mcl = reinterpret_cast<const uint16_t *>(ws + p.off_mcls);
    const uint16_t *mld = reinterpret_cast<const uint16_t *>(ws + p.off_mlead);
    uint64_t nin = p.levels[0];
    if (p.off_todo) {
        if (lds > 64 * 1024 && hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose_chunks_list),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return PAREM_EDEVICE;
        uint32_t *todo = reinterpret_cast<uint32_t *>(ws + p.off_todo);
        hipLaunchKernelGGL(k_compose_chunks_uniform, dim3((uint32_t)((nin + 3) / 4)), dim3(256), 0, stream, map, mcl,
                           mld, a, seg_out(p, ws, 0), nin, todo);
        hipLaunchKernelGGL(k_compose_chunks_list, dim3((uint32_t)std::min<uint64_t>(nin, 512)), dim3(kComposeThreads),
                           lds, stream, map, mcl, mld, a, seg_out(p, ws, 0), nin, todo);
    } else {
        hipLaunchKernelGGL(k_compose_chunks, dim3((uint32_t)nin), dim3(kComposeThreads), lds, stream, map, mcl, mld, a,
                           seg_out(p, ws, 0), nin == 1 ? d_out : nullptr);
    }
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    for (size_t l = 1; l < p.levels.size(); ++l) {
        const size_t src = p.keep ? l - 1 : (l - 1) % 2, dst = p.keep ? l : l % 2;
        const SegOut in = seg_out(p, ws, src);
        const uint64_t nout = p.levels[l];
        hipLaunchKernelGGL(k_compose_segs, dim3((uint32_t)nout), dim3(kComposeThreads), lds2, stream, in, nin, a2,
                           seg_out(p, ws, dst), nout == 1 ? d_out : nullptr);
        if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
        nin = nout;
    }
    return PAREM_OK;
}

void launch_walk_phase(const DeviceDfa &d, const PlainPlan &p, WalkArgs &a, const uint8_t *d_text, uint8_t *ws,
                       hipStream_t stream, bool aligned);
parem_status finish_result(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, uint8_t *ws,
                           hipStream_t stream, parem_result *d_out);

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
    launch_walk_phase(d, p, a, d_text, ws, stream, aligned);
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    if (ev_end && hipEventRecord(ev_end, stream) != hipSuccess) return PAREM_EDEVICE;
    parem_status st = launch_compose(d, p, ws, stream, d_out);
    if (st != PAREM_OK) return st;
    return finish_result(d, p, a, ws, stream, d_out);
}

// The walk of a plain match: Algorithm 1's sets, lookback sets, or for a
// partial table the S filter's selection. `a` receives the selection.
void launch_walk_phase(const DeviceDfa &d, const PlainPlan &p, WalkArgs &a, const uint8_t *d_text, uint8_t *ws,
                       hipStream_t stream, bool aligned) {
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(ws + p.off_flags);
    const uint32_t g = (uint32_t)((p.chunks + 255) / 256);
    if (p.look) {
        const LookArgs la = look_args(d, p, d_text, ws);
        if (slot_lookback(d, p)) {
            const size_t lds = d.table_bytes + (size_t)kSlotLookCap * kSparseThreads * 2;
            hipLaunchKernelGGL(k_lookback_slots, dim3((uint32_t)((p.chunks + kSparseThreads - 1) / kSparseThreads)),
                               dim3(kSparseThreads), lds, stream, la, d.d_llist_walk,
                               reinterpret_cast<const uint8_t *>(d.d_table), d.table_bytes, d.d_sids, d.sparse_d0);
        } else {
            const uint32_t wb = look_wave_bytes(la.words);
            hipLaunchKernelGGL(k_lookback, dim3((uint32_t)((p.chunks + 3) / 4)), dim3(256), 4 * wb, stream, la,
                               d.start, wb, nullptr);
        }
        a.sel = la.sel;
        a.nsel = la.nsel;
        a.sel_stride = kLookCap;
        launch_walk<WALK_SELECTED>(d, p, a, stream, aligned);
    } else if (p.sfilter) {
        a.sel = reinterpret_cast<uint16_t *>(ws + p.off_sel);
        a.nsel = ws + p.off_nsel;
        a.sel_stride = kLookCap;
        a.absent_fill = d.dead;  // count 0
        hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, stream, reinterpret_cast<uint32_t *>(acc), 4u);
        hipLaunchKernelGGL(k_sfilter, dim3(g), dim3(256), 0, stream, d_text, p.n, p.L, p.chunks, d.d_cls, d.A,
                           d.d_loff, d.d_llist, d.d_next, d.dead, const_cast<uint16_t *>(a.sel),
                           const_cast<uint8_t *>(a.nsel), acc);
        launch_walk<WALK_SELECTED>(d, p, a, stream, aligned);
    } else {
        launch_walk<WALK_ALL>(d, p, a, stream, aligned);
    }
}

// After the composition wrote *d_out: the walk tally of a selection and the
// outside name of the dead state.
parem_status finish_result(const DeviceDfa &d, const PlainPlan &p, const WalkArgs &a, uint8_t *ws,
                           hipStream_t stream, parem_result *d_out) {
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(ws + p.off_flags);
    const uint32_t g = (uint32_t)((p.chunks + 255) / 256);
    if (p.sfilter) {
        hipLaunchKernelGGL(k_learned_total, dim3(1), dim3(64), 0, stream, acc, d_out);
        hipLaunchKernelGGL(k_dead_result, dim3(1), dim3(64), 0, stream, d_out, d.dead);
        return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
    }
    if (!p.look) return PAREM_OK;
    hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, stream, reinterpret_cast<uint32_t *>(acc), 4u);
    hipLaunchKernelGGL(k_look_stats, dim3(g), dim3(256), 0, stream, a.nsel, a.map_cls, d.d_loff, p.chunks, acc);
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
    uint8_t *ws = reinterpret_cast<uint8_t *>(d_ws);
    parem_status st =
        launch_boundary_into(d, p, d_text, d_states, ws, stream, reinterpret_cast<parem_result *>(ws + p.off_dummy));
    if (st != PAREM_OK || p.n == 0 || d.dead == 0xffffffffu) return st;
    hipLaunchKernelGGL(k_dead_states, dim3((uint32_t)((p.chunks + 255) / 256)), dim3(256), 0, stream, d_states,
                       p.chunks, d.dead);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

// Walk, composition (the match result into d_out) and down-sweep (the entry
// state of every chunk into d_states).
parem_status launch_boundary_into(const DeviceDfa &d, const PlainPlan &p, const uint8_t *d_text, uint32_t *d_states,
                                  uint8_t *ws, hipStream_t stream, parem_result *d_out) {
    if (p.n == 0) return PAREM_OK;
    if (!d.d_inv) return PAREM_EUNSUPPORTED;
    const bool aligned = (reinterpret_cast<uintptr_t>(d_text) & 15u) == 0;
    WalkArgs a = walk_args(d, p, d_text, ws);
    launch_walk_phase(d, p, a, d_text, ws, stream, aligned);
    parem_status st = launch_compose(d, p, ws, stream, d_out);
    if (st != PAREM_OK) return st;
    st = finish_result(d, p, a, ws, stream, d_out);
    if (st != PAREM_OK) return st;
    // down-sweep: the top map is entered in q0
    const size_t top = p.levels.size() - 1;
    uint32_t *top_entry = reinterpret_cast<uint32_t *>(ws + p.entries[top]);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, stream, top_entry, d.start);
    for (size_t l = top; l-- > 0;) {
        const SegOut s = seg_out(p, ws, l);
        const uint64_t nmaps = p.levels[l];
        hipLaunchKernelGGL(k_entries<false>, dim3((uint32_t)((nmaps + 255) / 256)), dim3(256), 0, stream, nmaps, p.P2,
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
    parem_status st = plan_chunks(d, len, o, false, p, true);
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
    p->off_rlist = off;
    off = align256(off + kSplitMax * 4);
    p->off_part = off;
    off = align256(off + (ch + 255) / 256 * 16);
    p->off_mlp = off;
    off = align256(off + proposal_infer_bytes(pr, ch));
    // a handle that walks lookback sets in plain matches walks them again
    // here for chunks whose selection missed (the sub-chunk path serves
    // small sets instead)
    const bool split = d.d_step && d.max_spec <= 64;
    p->relook = (opt.lookback && d.d_next && d.d_inv && !split) ? opt.lookback : 0u;
    if (p->relook) {
        p->off_lsel = off;
        off = align256(off + ch * kLookCap * 2);
        p->off_lnsel = off;
        off = align256(off + ch);
    }
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
    // the selection also clears the coverage counters of step 3
    // (flags: 0 chunks marked, 1 escalation, 8 + round: marked in the round)
    parem_status st = proposal_select(pr, d_text, p.L, C, p.m, p.m, ws + p.off_mlp, stream, sel, nsel, flags,
                                      8u + kCoverRounds + 1);
    if (st != PAREM_OK) return st;
    // 2. walk the selected states
    WalkArgs a = walk_args(d, p, d_text, ws);
    a.sel = sel;
    a.nsel = nsel;
    a.sel_stride = p.m;
    launch_walk<WALK_SELECTED>(d, p, a, stream, aligned);
    if (hipGetLastError() != hipSuccess) return PAREM_EDEVICE;
    // 3. verify coverage, walk uncovered chunks again from their whole set
    unsigned long long *part = reinterpret_cast<unsigned long long *>(ws + p.off_part);
    WalkArgs r = walk_args(d, p, d_text, ws);
    r.redo = redo;
    uint32_t *rlist = reinterpret_cast<uint32_t *>(ws + p.off_rlist);
    // marked chunks of small-set DFAs are walked in sub-chunks first
    const bool split = d.d_step && d.max_spec <= 64;
    SplitArgs sa{};
    SplitLds sl{};
    if (split) {
        sa = SplitArgs{d_text, p.n, p.L, (uint64_t)C, d.d_cls, d.d_loff, d.d_llist, d.d_step, d.d_inv, d.Q + 1,
                       d.A + 1, d.sent, d.inv_lds, a.map, a.map_cls, a.map_lead, redo, done, flags, rlist, nullptr};
        sl = split_lds(d.Q + 1, d.A + 1, d.inv_lds, p.L);
        static std::once_flag lds_once;
        static hipError_t lds_err = hipSuccess;
        std::call_once(lds_once, [] {
            const SplitLds most = split_lds(kSplitTable, 1, 16384, kMaxChunk);
            lds_err = hipFuncSetAttribute(reinterpret_cast<const void *>(k_redo_split),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)most.bytes);
        });
        if (lds_err != hipSuccess) return PAREM_EDEVICE;
    }
    // marked chunks of handles with lookback sets are walked again from them
    LookArgs la{};
    uint32_t lwb = 0;
    uint8_t *lnsel = nullptr;
    if (p.relook) {
        PlainPlan lp = p;
        lp.look = p.relook;
        la = look_args(d, lp, d_text, ws);
        la.sel = reinterpret_cast<uint16_t *>(ws + p.off_lsel);
        lnsel = ws + p.off_lnsel;
        la.nsel = lnsel;
        lwb = look_wave_bytes(la.words);
        r.sel = la.sel;
        r.nsel = lnsel;
        r.sel_stride = kLookCap;
    }
    // (the sub-chunk walk settles what later coverage rounds would find: one
    // round before the escalation is enough then)
    const int rounds = split ? 1 : kCoverRounds;
    for (int it = 0; it <= rounds; ++it) {
        const uint32_t escalate = it == rounds ? 1u : 0u;
        uint32_t *round_count = flags + 8 + it;
        hipLaunchKernelGGL(k_cover, dim3(g), dim3(256), 0, stream, a.map, a.map_cls, a.map_lead, (uint64_t)C, d.d_loff,
                           d.d_inv, d.Q + 1, d.sent, redo, done, flags, escalate, round_count, rlist,
                           it == 0 ? 1u : 0u);
        if (escalate)
            hipLaunchKernelGGL(k_escalate, dim3(g), dim3(256), 0, stream, (uint64_t)C, redo, done, flags, round_count,
                               rlist, nsel, a.map_cls, d.d_loff, lnsel, part);
        if (split) {
            sa.count = round_count;
            hipLaunchKernelGGL(k_redo_split, dim3(512), dim3(kSplitThreads), sl.bytes, stream, sa);
        }
        if (p.relook)
            hipLaunchKernelGGL(k_lookback, dim3((C + 3) / 4), dim3(256), 4 * lwb, stream, la, d.start, lwb, redo);
        launch_walk<WALK_REDO>(d, p, r, stream, aligned);
    }
    if (ev_end && hipEventRecord(ev_end, stream) != hipSuccess) return PAREM_EDEVICE;
    // 4. compose, then the learned statistics
    st = launch_compose(d, p, ws, stream, d_out);
    if (st != PAREM_OK) return st;
    hipLaunchKernelGGL(k_stats_total, dim3(1), dim3(64), 0, stream, part, g, d_out);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

}  // namespace parem

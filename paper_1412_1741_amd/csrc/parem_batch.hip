// Batched matching of many (DFA, text) pairs on one GPU.
//
// Every pair is the method of Section II-B / Algorithm 1 on its own text:
// chunks walked from their speculated sets, chunk maps joined by
// composition. Batching changes only how the work reaches the chip:
//   * the chunks of all pairs are cut into work items of 256 chunks (one
//     workgroup, one chunk per lane); items of pairs that share a kernel
//     variant (table layout, lockstep group, staged tile) go to one
//     persistent launch whose workgroups take items from an atomic queue,
//     the most expensive first, and stage each pair's table in LDS when the
//     layout keeps it there (skipped when the previous item had the same
//     pair);
//   * composition runs level by level: one launch per level holds a
//     workgroup per (pair, segment) for every pair that still has more than
//     one map; a pair's last level writes its result;
//   * nothing in a run waits on the host, so the whole sequence is captured
//     once into a HIP graph and replayed (the per-run text pointers live in
//     a device array the graph reads, refreshed by a copy before each
//     replay).
#include "parem_batch_kernels.h"

#include <algorithm>
#include <cstring>
#include <new>

namespace parem {

__global__ void k_batch_clear(uint32_t *__restrict__ p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__global__ __launch_bounds__(kComposeThreads) void k_batch_compose(const BatchPair *__restrict__ pairs,
                                                                    const ComposeItem *__restrict__ items,
                                                                    uint32_t level) {
    extern __shared__ __align__(16) uint8_t smem[];
    const ComposeItem &it = items[blockIdx.x];
    const BatchPair &bp = pairs[it.pair];
    parem_result *res = it.last ? bp.out : nullptr;
    if (level == 0)
        compose_chunks_seg(smem, bp.w.map, bp.w.map_cls, bp.w.map_lead, bp.ca, bp.seg[0], it.seg, res);
    else
        compose_segs_seg(smem, bp.seg[(level - 1) & 1u], it.nin, bp.ca, bp.seg[level & 1u], it.seg, res);
}

// pairs with an empty text: the start state
__global__ void k_batch_empty(const BatchPair *__restrict__ pairs, const uint32_t *__restrict__ idx, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const BatchPair &bp = pairs[idx[i]];
    parem_result r;
    r.final_state = bp.start;
    r.accept = bp.ca.final_flag[bp.start];
    r.count = 0;
    r.chunks = 0;
    r.spec_runs = 0;
    r.rerun_chunks = 0;
    *bp.out = r;
}

static WalkKernel walk_kernel(uint32_t G, uint32_t tile, int kind, bool sel) {
    if (sel) return tile == 64 ? batch_walk_kernel_64_sel(G, kind) : batch_walk_kernel_128_sel(G, kind);
    return tile == 64 ? batch_walk_kernel_64(G, kind) : batch_walk_kernel_128(G, kind);
}

// lookback sets of four chunks of one pair per workgroup (one wave each)
__global__ __launch_bounds__(256) void k_batch_lookback(const BatchPair *__restrict__ pairs,
                                                        const uint8_t *const *__restrict__ texts,
                                                        const LookItem *__restrict__ items, uint32_t wave_bytes) {
    extern __shared__ __align__(16) uint8_t smem[];
    const LookItem &it = items[blockIdx.x];
    const BatchPair &bp = pairs[it.pair];
    const uint64_t c = (uint64_t)it.quad * 4u + (threadIdx.x >> 6);
    if (c >= bp.la.nchunks) return;
    LookArgs a = bp.la;
    a.text = texts[it.pair];
    lookback_chunk(a, bp.start, c, smem + (threadIdx.x >> 6) * wave_bytes);
}

// walks started by a lookback pair (nsel 0: the chunk's whole set); runs
// after the pair's result is written
__global__ __launch_bounds__(256) void k_batch_look_stats(const BatchPair *__restrict__ pairs,
                                                          const uint32_t *__restrict__ idx) {
    const BatchPair &bp = pairs[idx[blockIdx.x]];
    unsigned long long runs = 0;
    for (uint64_t c = threadIdx.x; c < bp.w.nchunks; c += 256) {
        uint32_t r = bp.w.nsel[c];
        if (!r) {
            const uint32_t cl = bp.w.map_cls[c] & 0x7fffu;
            r = bp.ca.loff[cl + 1] - bp.ca.loff[cl];
        }
        runs += r;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) runs += (unsigned long long)__shfl_xor((long long)runs, o, 64);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = runs;
    __syncthreads();
    if (threadIdx.x == 0) bp.out->spec_runs = part[0] + part[1] + part[2] + part[3];
}

// Automatic chunk length inside a batch: the other pairs supply the
// parallelism, so a pair needs only about 256 chunks (one work item) up to
// 8 KiB chunks; longer texts get more items of 8 KiB chunks.
uint32_t batch_chunk_len(uint64_t len) {
    uint32_t L = 64;
    while (L < 8192 && (uint64_t)L * 256 < len) L <<= 1;
    return L;
}

static int batch_kind(const DeviceDfa &d) {
    if (d.layout == PAREM_LAYOUT_KGRAM_LDS) return BK_KGRAM1 + (int)d.kg.bits - 1;
    if (d.layout == PAREM_LAYOUT_BYTE_LDS) return BK_BYTE_LDS;
    if (d.layout == PAREM_LAYOUT_HOT_LDS) return BK_HOT;
    if (d.layout == PAREM_LAYOUT_CLASS_LDS) return BK_CLASS;
    return BK_BYTE_GLOBAL;
}

struct BatchVariant {
    int kind = 0;
    uint32_t G = 0, tile = 0;
    bool sel = false;        // lookback selections (WALK_SELECTED)
    uint32_t table_cap = 0;  // largest LDS table of its pairs (16-byte multiple)
    std::vector<WalkItem> items;
    uint64_t off_items = 0;
    uint32_t grid = 0;
    size_t lds = 0;
    WalkKernel fn = nullptr;
};

struct BatchLevel {
    std::vector<ComposeItem> items;
    uint64_t off_items = 0;
    size_t lds = 0;
};

}  // namespace parem

struct parem_batch_s {
    int device = 0;
    uint32_t n = 0;
    std::vector<const parem::DeviceDfa *> dfas;
    std::vector<uint64_t> lens;
    std::vector<parem::PlainPlan> plans;
    std::vector<parem::BatchVariant> variants;
    std::vector<parem::BatchLevel> levels;
    std::vector<uint32_t> empties;
    std::vector<uint32_t> learned;                 // pairs with a proposal
    std::vector<const parem::Proposal *> props;    // per pair (null: plain)
    std::vector<uint64_t> ws_off;                  // per pair workspace offset
    std::vector<const uint8_t *> cap_texts;        // learned pairs' texts in the captured graph
    hipStream_t lstream = nullptr;                 // branch of the learned pairs
    hipEvent_t lfork = nullptr, ljoin = nullptr;
    std::vector<uint32_t> look_pairs;
    std::vector<parem::LookItem> look_items;
    uint32_t look_wave = 0;
    uint64_t off_look_pairs = 0, off_look_items = 0;
    uint64_t off_empties = 0, off_pairs = 0, off_queue = 0, off_texts = 0, off_results = 0;
    uint64_t chunks = 0, text_bytes = 0, ws_bytes = 0, items = 0;
    uint8_t *d_meta = nullptr;
    uint8_t *d_ws = nullptr;
    const uint8_t **h_texts = nullptr;  // pinned staging of the text pointers
    hipEvent_t staged = nullptr;        // the last pointer upload has been read
    bool staged_pending = false;
    hipStream_t cap_stream = nullptr;
    // walk launches run on up to kBranches concurrent streams (branches of
    // the graph): a launch whose items are few and long overlaps the others
    static constexpr int kBranches = 4;
    hipStream_t aux[kBranches - 1] = {};
    hipEvent_t fork = nullptr, join[kBranches - 1] = {};
    std::vector<int> branch;  // per variant
    int nbranch = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t graph_nodes = 0;
};

namespace parem {

static void batch_release(parem_batch_s *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (int i = 0; i < parem_batch_s::kBranches - 1; ++i) {
        if (b->aux[i]) (void)hipStreamDestroy(b->aux[i]);
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->lstream) (void)hipStreamDestroy(b->lstream);
    if (b->lfork) (void)hipEventDestroy(b->lfork);
    if (b->ljoin) (void)hipEventDestroy(b->ljoin);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->h_texts) (void)hipHostFree(b->h_texts);
    (void)hipFree(b->d_meta);
    (void)hipFree(b->d_ws);
    delete b;
}

static parem_status batch_plan(const parem_handle *dfas, const uint64_t *lens, uint32_t n, const parem_options *opts,
                               const parem_proposal *props, const uint32_t *m, parem_batch_s *b) {
    if (hipGetDevice(&b->device) != hipSuccess) return PAREM_EDEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
        return PAREM_EDEVICE;
    b->n = n;
    b->dfas.resize(n);
    b->lens.assign(lens, lens + n);
    b->plans.resize(n);
    std::vector<uint64_t> &ws_off = b->ws_off;
    ws_off.assign(n, 0);
    b->props.assign(n, nullptr);
    std::vector<int> pair_var(n, -1);
    uint64_t ws = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!dfas[i]) return PAREM_EINVAL;
        const DeviceDfa &d = dfas[i]->dev;
        if (d.device != b->device) return PAREM_EINVAL;
        b->dfas[i] = &d;
        parem_options o = opts ? opts[i] : d.opt;
        if (o.lookback > kLookMax) return PAREM_EINVAL;
        // the speculated sets (policy, partial table) are the handle's; per-pair
        // options may only repeat them
        if ((o.policy && o.policy != d.opt.policy) || (o.partial && o.partial != d.opt.partial)) return PAREM_EINVAL;
        if (d.dead != 0xffffffffu) return PAREM_EUNSUPPORTED;  // partial tables: single-text matches only
        if (o.chunk_len == 0) o.chunk_len = batch_chunk_len(lens[i]);
        PlainPlan &p = b->plans[i];
        const Proposal *pr = props ? props[i] : nullptr;
        if (pr) {
            // learned speculation: its own launch sequence, on the learned branch
            if (pr->dfa != &d || !m || m[i] < 1 || m[i] > 16) return PAREM_EINVAL;
            parem_status st = plan_learned(d, *pr, lens[i], m[i], o, &p);
            if (st != PAREM_OK) return st;
            b->text_bytes += lens[i];
            if (lens[i] == 0) {
                b->empties.push_back(i);
                continue;
            }
            b->props[i] = pr;
            b->learned.push_back(i);
            b->chunks += p.chunks;
            ws_off[i] = ws;
            ws = align256(ws + p.bytes);
            continue;
        }
        parem_status st = plan_chunks(d, lens[i], o, false, &p);
        if (st != PAREM_OK) return st;
        if (p.G < 4) return PAREM_EUNSUPPORTED;  // batch kernels lock-step 4, 8 or 16 walks
        b->text_bytes += lens[i];
        if (lens[i] == 0) {
            b->empties.push_back(i);
            continue;
        }
        b->chunks += p.chunks;
        ws_off[i] = ws;
        ws = align256(ws + p.bytes);
        const int kind = batch_kind(d);
        const bool sel = p.look > 0;
        if (sel) {
            b->look_pairs.push_back(i);
            for (uint64_t q4 = 0; q4 < (p.chunks + 3) / 4; ++q4) b->look_items.push_back(LookItem{i, (uint32_t)q4});
            b->look_wave = std::max(b->look_wave, look_wave_bytes((d.Q + 1 + 31) / 32));
        }
        int v = -1;
        for (size_t k = 0; k < b->variants.size(); ++k) {
            const BatchVariant &x = b->variants[k];
            if (x.kind == kind && x.G == p.G && x.tile == p.tile && x.sel == sel) v = (int)k;
        }
        if (v < 0) {
            BatchVariant x;
            x.kind = kind;
            x.G = p.G;
            x.tile = p.tile;
            x.sel = sel;
            x.fn = walk_kernel(p.G, p.tile, kind, sel);
            b->variants.push_back(x);
            v = (int)b->variants.size() - 1;
        }
        pair_var[i] = v;
        BatchVariant &x = b->variants[(size_t)v];
        if (kind != BK_BYTE_GLOBAL) x.table_cap = std::max<uint32_t>(x.table_cap, (d.table_bytes + 15u) & ~15u);
    }
    b->ws_bytes = ws;

    // walk items, most expensive first: longer chunks, then more speculated
    // states per chunk (a workgroup's time grows with both)
    for (uint32_t i = 0; i < n; ++i) {
        if (pair_var[i] < 0) continue;
        const PlainPlan &p = b->plans[i];
        const uint64_t nblk = (p.chunks + kWalkThreads - 1) / kWalkThreads;
        for (uint64_t k = 0; k < nblk; ++k)
            b->variants[(size_t)pair_var[i]].items.push_back(WalkItem{i, (uint32_t)k});
    }
    for (BatchVariant &x : b->variants) {
        std::stable_sort(x.items.begin(), x.items.end(), [&](const WalkItem &l, const WalkItem &r) {
            const PlainPlan &pl = b->plans[l.pair], &pr = b->plans[r.pair];
            if (pl.L != pr.L) return pl.L > pr.L;
            return pl.RM > pr.RM;
        });
        b->items += x.items.size();
        x.lds = x.table_cap + (size_t)(x.tile == 64 ? Stage<64>::kBytes : Stage<128>::kBytes) + 16;  // + queue slot
        if (x.lds > 64 * 1024 &&
            hipFuncSetAttribute(reinterpret_cast<const void *>(x.fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)x.lds) != hipSuccess)
            return PAREM_EUNSUPPORTED;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(x.fn), kWalkThreads,
                                                         x.lds) != hipSuccess)
            return PAREM_EDEVICE;
        if (per_cu < 1) return PAREM_EUNSUPPORTED;
        x.grid = (uint32_t)std::min<uint64_t>(x.items.size(), (uint64_t)per_cu * (uint64_t)cus);
    }

    // branches: variants by decreasing (longest chunk x items), dealt round robin
    b->branch.assign(b->variants.size(), 0);
    b->nbranch = (int)std::min<size_t>(parem_batch_s::kBranches, b->variants.size());
    if (b->nbranch > 1) {
        std::vector<size_t> ord(b->variants.size());
        std::vector<uint64_t> cost(b->variants.size(), 0);
        for (size_t v = 0; v < b->variants.size(); ++v) {
            ord[v] = v;
            for (const WalkItem &it : b->variants[v].items) cost[v] += b->plans[it.pair].L;
        }
        std::stable_sort(ord.begin(), ord.end(), [&](size_t l, size_t r) { return cost[l] > cost[r]; });
        for (size_t k = 0; k < ord.size(); ++k) b->branch[ord[k]] = (int)(k % (size_t)b->nbranch);
        for (int i = 0; i < b->nbranch - 1; ++i) {
            if (hipStreamCreateWithFlags(&b->aux[i], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) != hipSuccess)
                return PAREM_EDEVICE;
        }
    }
    if (b->nbranch > 1 && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        return PAREM_EDEVICE;

    // composition levels
    size_t nlev = 0;
    for (uint32_t i = 0; i < n; ++i)
        if (lens[i] && !b->props[i]) nlev = std::max(nlev, b->plans[i].levels.size());
    b->levels.resize(nlev);
    for (uint32_t i = 0; i < n; ++i) {
        if (!lens[i] || b->props[i]) continue;
        const PlainPlan &p = b->plans[i];
        const DeviceDfa &d = *b->dfas[i];
        const size_t lds = compose_lds(p.P, p.RM, d.inv_lds);
        for (size_t l = 0; l < p.levels.size(); ++l) {
            BatchLevel &lv = b->levels[l];
            lv.lds = std::max(lv.lds, lds);
            const uint64_t nin = l == 0 ? p.chunks : p.levels[l - 1];
            const uint32_t last = l + 1 == p.levels.size() ? 1u : 0u;
            for (uint64_t s = 0; s < p.levels[l]; ++s) lv.items.push_back(ComposeItem{i, last, s, nin});
        }
    }
    if (!b->learned.empty()) {
        if (hipStreamCreateWithFlags(&b->lstream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->lfork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->ljoin, hipEventDisableTiming) != hipSuccess)
            return PAREM_EDEVICE;
    }
    for (BatchLevel &lv : b->levels) {
        if (lv.lds > 64 * 1024 &&
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch_compose),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lv.lds) != hipSuccess)
            return PAREM_EUNSUPPORTED;
    }

    // device metadata: pair descriptors, item lists, queues, text pointers, results
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align256(off + std::max<uint64_t>(bytes, 1));
        return o;
    };
    b->off_pairs = take((uint64_t)n * sizeof(BatchPair));
    for (BatchVariant &x : b->variants) x.off_items = take(x.items.size() * sizeof(WalkItem));
    for (BatchLevel &lv : b->levels) lv.off_items = take(lv.items.size() * sizeof(ComposeItem));
    b->off_empties = take(b->empties.size() * 4);
    b->off_look_pairs = take(b->look_pairs.size() * 4);
    b->off_look_items = take(b->look_items.size() * sizeof(LookItem));
    b->off_queue = take(std::max<size_t>(b->variants.size(), 1) * 4);
    b->off_texts = take((uint64_t)n * 8);
    b->off_results = take((uint64_t)n * sizeof(parem_result));
    if (hipMalloc(reinterpret_cast<void **>(&b->d_meta), off) != hipSuccess) return PAREM_ENOMEM;
    if (ws && hipMalloc(reinterpret_cast<void **>(&b->d_ws), ws) != hipSuccess) return PAREM_ENOMEM;
    if (hipHostMalloc(reinterpret_cast<void **>(&b->h_texts), std::max<size_t>(n, 1) * 8) != hipSuccess)
        return PAREM_ENOMEM;
    if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) return PAREM_EDEVICE;

    std::vector<BatchPair> hp(n);
    parem_result *d_res = reinterpret_cast<parem_result *>(b->d_meta + b->off_results);
    for (uint32_t i = 0; i < n; ++i) {
        const DeviceDfa &d = *b->dfas[i];
        const PlainPlan &p = b->plans[i];
        BatchPair &q = hp[i];
        std::memset(&q, 0, sizeof(q));
        uint8_t *pws = b->d_ws ? b->d_ws + ws_off[i] : nullptr;
        q.start = d.start;
        q.out = d_res + i;
        q.ca = compose_args(d, p);
        if (lens[i] == 0 || b->props[i]) continue;
        q.w = walk_args(d, p, nullptr, pws);
        // sparse layout: the batch kernels walk the byte table through L2,
        // from the lists of state ids (not the lists of slot bases)
        q.table = d.layout == PAREM_LAYOUT_SPARSE_LDS ? d.d_bytes : d.d_table;
        if (d.layout == PAREM_LAYOUT_SPARSE_LDS) q.w.llist = d.d_llist;
        q.table_bytes = d.table_bytes;
        q.full = d.d_full;
        q.enc = d.d_enc;
        q.hot_rows = d.hot_rows;
        q.kg = d.kg;
        for (size_t k = 0; k < p.seg.size() && k < 2; ++k) q.seg[k] = seg_out(p, pws, k);
        if (p.look) {
            q.la = look_args(d, p, nullptr, pws);
            q.w.sel = q.la.sel;
            q.w.nsel = q.la.nsel;
            q.w.sel_stride = kLookCap;
        }
    }
    auto put = [&](uint64_t o, const void *src, size_t bytes) {
        return bytes == 0 || hipMemcpy(b->d_meta + o, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = put(b->off_pairs, hp.data(), hp.size() * sizeof(BatchPair));
    for (BatchVariant &x : b->variants) ok = ok && put(x.off_items, x.items.data(), x.items.size() * sizeof(WalkItem));
    for (BatchLevel &lv : b->levels)
        ok = ok && put(lv.off_items, lv.items.data(), lv.items.size() * sizeof(ComposeItem));
    ok = ok && put(b->off_empties, b->empties.data(), b->empties.size() * 4);
    ok = ok && put(b->off_look_pairs, b->look_pairs.data(), b->look_pairs.size() * 4);
    ok = ok && put(b->off_look_items, b->look_items.data(), b->look_items.size() * sizeof(LookItem));
    if (ok && b->look_wave * 4 > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch_lookback), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(b->look_wave * 4)) != hipSuccess)
        return PAREM_EUNSUPPORTED;
    return ok ? PAREM_OK : PAREM_EDEVICE;
}

// the launches of one run (no host synchronisation: capturable); `host_texts`
// are the run's text pointers (only learned pairs take them as arguments)
static parem_status batch_enqueue(const parem_batch_s *b, hipStream_t s, const uint8_t *const *host_texts) {
    const BatchPair *pairs = reinterpret_cast<const BatchPair *>(b->d_meta + b->off_pairs);
    if (!b->learned.empty()) {
        // learned pairs: each its own sequence (selection, walk, coverage, composition)
        parem_result *res = reinterpret_cast<parem_result *>(b->d_meta + b->off_results);
        if (hipEventRecord(b->lfork, s) != hipSuccess || hipStreamWaitEvent(b->lstream, b->lfork, 0) != hipSuccess)
            return PAREM_EDEVICE;
        for (uint32_t i : b->learned) {
            parem_status st = launch_learned(*b->dfas[i], *b->props[i], b->plans[i], host_texts[i],
                                             b->d_ws + b->ws_off[i], b->lstream, res + i, nullptr, nullptr);
            if (st != PAREM_OK) return st;
        }
        if (hipEventRecord(b->ljoin, b->lstream) != hipSuccess) return PAREM_EDEVICE;
    }
    const uint8_t *const *texts = reinterpret_cast<const uint8_t *const *>(b->d_meta + b->off_texts);
    uint32_t *queue = reinterpret_cast<uint32_t *>(b->d_meta + b->off_queue);
    // The lookback sets run first, alone: launched beside the persistent walk
    // kernels of the other variants they lose compute units to them, and the
    // variants that walk the sets (the batch's longest chain) start later
    // (4096 uneven pairs: 92.4 ms per replay that way against 83.5 ms).
    if (!b->look_items.empty())
        hipLaunchKernelGGL(k_batch_lookback, dim3((uint32_t)b->look_items.size()), dim3(256), 4 * b->look_wave, s,
                           pairs, texts, reinterpret_cast<const LookItem *>(b->d_meta + b->off_look_items),
                           b->look_wave);
    if (!b->variants.empty()) {
        hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(64), 0, s, queue, (uint32_t)b->variants.size());
        const int nb = b->nbranch;
        if (nb > 1) {
            if (hipEventRecord(b->fork, s) != hipSuccess) return PAREM_EDEVICE;
            for (int i = 0; i < nb - 1; ++i)
                if (hipStreamWaitEvent(b->aux[i], b->fork, 0) != hipSuccess) return PAREM_EDEVICE;
        }
        for (size_t v = 0; v < b->variants.size(); ++v) {
            const BatchVariant &x = b->variants[v];
            const WalkItem *items = reinterpret_cast<const WalkItem *>(b->d_meta + x.off_items);
            hipStream_t bs = b->branch[v] == 0 ? s : b->aux[b->branch[v] - 1];
            hipLaunchKernelGGL(x.fn, dim3(x.grid), dim3(kWalkThreads), x.lds, bs, pairs, texts, items,
                               (uint32_t)x.items.size(), queue + v, x.table_cap);
        }
        for (int i = 0; i < nb - 1; ++i) {
            if (hipEventRecord(b->join[i], b->aux[i]) != hipSuccess || hipStreamWaitEvent(s, b->join[i], 0) != hipSuccess)
                return PAREM_EDEVICE;
        }
    }
    if (!b->empties.empty()) {
        const uint32_t ne = (uint32_t)b->empties.size();
        hipLaunchKernelGGL(k_batch_empty, dim3((ne + 255) / 256), dim3(256), 0, s, pairs,
                           reinterpret_cast<const uint32_t *>(b->d_meta + b->off_empties), ne);
    }
    for (size_t l = 0; l < b->levels.size(); ++l) {
        const BatchLevel &lv = b->levels[l];
        if (lv.items.empty()) continue;
        hipLaunchKernelGGL(k_batch_compose, dim3((uint32_t)lv.items.size()), dim3(kComposeThreads), lv.lds, s, pairs,
                           reinterpret_cast<const ComposeItem *>(b->d_meta + lv.off_items), (uint32_t)l);
    }
    if (!b->look_pairs.empty())
        hipLaunchKernelGGL(k_batch_look_stats, dim3((uint32_t)b->look_pairs.size()), dim3(256), 0, s, pairs,
                           reinterpret_cast<const uint32_t *>(b->d_meta + b->off_look_pairs));
    if (!b->learned.empty() && hipStreamWaitEvent(s, b->ljoin, 0) != hipSuccess) return PAREM_EDEVICE;
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

static parem_status batch_capture(parem_batch_s *b, const uint8_t *const *host_texts) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return PAREM_EDEVICE;
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return PAREM_EDEVICE;
    parem_status st = batch_enqueue(b, b->cap_stream, host_texts);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st != PAREM_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != PAREM_OK ? st : PAREM_EDEVICE;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return PAREM_EDEVICE;
    }
    size_t nodes = 0;
    (void)hipGraphGetNodes(g, nullptr, &nodes);
    b->graph = g;
    b->exec = x;
    b->graph_nodes = nodes;
    b->cap_texts.clear();
    for (uint32_t i : b->learned) b->cap_texts.push_back(host_texts[i]);
    return PAREM_OK;
}

static parem_status batch_run(parem_batch_s *b, const uint8_t *const *d_texts, hipStream_t s, parem_result *d_out,
                              bool use_graph) {
    for (uint32_t i = 0; i < b->n; ++i) {
        if (b->lens[i] && (!d_texts[i] || (reinterpret_cast<uintptr_t>(d_texts[i]) & 15u) != 0))
            return PAREM_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device) return PAREM_EINVAL;
    // the previous run's pointer upload must have been read before the staging is rewritten
    if (b->staged_pending && hipEventSynchronize(b->staged) != hipSuccess) return PAREM_EDEVICE;
    std::memcpy(b->h_texts, d_texts, (size_t)b->n * 8);
    if (b->n && hipMemcpyAsync(b->d_meta + b->off_texts, b->h_texts, (size_t)b->n * 8, hipMemcpyHostToDevice, s) !=
                    hipSuccess)
        return PAREM_EDEVICE;
    if (hipEventRecord(b->staged, s) != hipSuccess) return PAREM_EDEVICE;
    b->staged_pending = true;
    if (use_graph) {
        bool same = b->exec != nullptr;
        for (size_t k = 0; same && k < b->learned.size(); ++k) same = b->cap_texts[k] == d_texts[b->learned[k]];
        if (!same) {
            parem_status st = batch_capture(b, d_texts);
            if (st != PAREM_OK) return st;
        }
        if (hipGraphLaunch(b->exec, s) != hipSuccess) return PAREM_EDEVICE;
    } else {
        parem_status st = batch_enqueue(b, s, d_texts);
        if (st != PAREM_OK) return st;
    }
    if (b->n && hipMemcpyAsync(d_out, b->d_meta + b->off_results, (size_t)b->n * sizeof(parem_result),
                               hipMemcpyDeviceToDevice, s) != hipSuccess)
        return PAREM_EDEVICE;
    return PAREM_OK;
}

}  // namespace parem

extern "C" {

parem_status parem_batch_create(const parem_handle *dfas, const uint64_t *lens, uint32_t n,
                                const parem_options *opts, const parem_proposal *props, const uint32_t *m,
                                parem_batch *out) {
    if (!out || (n && (!dfas || !lens))) return PAREM_EINVAL;
    *out = nullptr;
    parem_batch_s *b = new (std::nothrow) parem_batch_s;
    if (!b) return PAREM_ENOMEM;
    parem_status st = parem::batch_plan(dfas, lens, n, opts, props, m, b);
    if (st != PAREM_OK) {
        parem::batch_release(b);
        return st;
    }
    *out = b;
    return PAREM_OK;
}

parem_status parem_batch_run(parem_batch b, const uint8_t *const *d_texts, void *stream, parem_result *d_out,
                             int use_graph) {
    if (!b || (b->n && (!d_texts || !d_out))) return PAREM_EINVAL;
    return parem::batch_run(b, d_texts, static_cast<hipStream_t>(stream), d_out, use_graph != 0);
}

parem_status parem_batch_describe(parem_batch b, parem_batch_info *info) {
    if (!b) return PAREM_EINVAL;
    if (info) {
        info->pairs = b->n;
        info->walk_launches = (uint32_t)b->variants.size();
        info->walk_items = b->items;
        uint32_t lv = 0;
        for (const parem::BatchLevel &l : b->levels) lv += l.items.empty() ? 0u : 1u;
        info->levels = lv;
        info->graph_nodes = (uint32_t)b->graph_nodes;
        info->learned_pairs = (uint32_t)b->learned.size();
        info->chunks = b->chunks;
        info->text_bytes = b->text_bytes;
        info->workspace_bytes = b->ws_bytes;
    }
    return PAREM_OK;
}

void parem_batch_free(parem_batch b) { parem::batch_release(b); }

parem_status parem_match_batch(const parem_handle *dfas, const uint8_t *const *d_texts, const uint64_t *lens,
                               uint32_t n, void *stream, parem_result *d_out) {
    parem_batch b = nullptr;
    parem_status st = parem_batch_create(dfas, lens, n, nullptr, nullptr, nullptr, &b);
    if (st != PAREM_OK) return st;
    st = parem_batch_run(b, d_texts, stream, d_out, 1);
    if (st == PAREM_OK && hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) st = PAREM_EDEVICE;
    if (st == PAREM_OK && n) {
        std::vector<parem_result> r(n);
        if (hipMemcpy(r.data(), d_out, (size_t)n * sizeof(parem_result), hipMemcpyDeviceToHost) != hipSuccess)
            st = PAREM_EDEVICE;
        for (uint32_t i = 0; st == PAREM_OK && i < n; ++i)
            if (lens[i] && r[i].final_state == 0xffffffffu) st = PAREM_ESYMBOL;
    }
    parem_batch_free(b);
    return st;
}

static constexpr uint64_t kTuneWorkspace = 4ull << 30;

parem_status parem_tune(parem_handle h, const uint8_t *d_sample, uint64_t sample_len, uint32_t copies,
                        const parem_options *cands, uint32_t ncand, uint32_t reps, void *stream, float *ms_out,
                        uint32_t *best) {
    if (!h || !d_sample || !sample_len || !copies || !cands || !ncand || !reps || !ms_out || !best)
        return PAREM_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_sample) & 15u) != 0) return PAREM_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return PAREM_EDEVICE;
    }
    parem_result *d_out = nullptr;
    parem_status st = PAREM_OK;
    if (hipMalloc(reinterpret_cast<void **>(&d_out), (size_t)copies * sizeof(parem_result)) != hipSuccess)
        st = PAREM_ENOMEM;
    float best_ms = -1.f;
    *best = 0;
    for (uint32_t c = 0; st == PAREM_OK && c < ncand; ++c) {
        ms_out[c] = -1.f;
        // as many copies as fit a bounded workspace
        parem_options oc = cands[c];
        if (oc.chunk_len == 0) oc.chunk_len = parem::batch_chunk_len(sample_len);
        parem::PlainPlan pp;
        if (parem::plan_chunks(h->dev, sample_len, oc, false, &pp) != PAREM_OK) continue;
        const uint64_t k = std::max<uint64_t>(1, std::min<uint64_t>(copies, kTuneWorkspace / std::max<uint64_t>(pp.bytes, 1)));
        std::vector<parem_handle> hs(k, h);
        std::vector<uint64_t> lens(k, sample_len);
        std::vector<const uint8_t *> texts(k, d_sample);
        std::vector<parem_options> o(k, oc);
        parem_batch b = nullptr;
        if (parem_batch_create(hs.data(), lens.data(), (uint32_t)k, o.data(), nullptr, nullptr, &b) != PAREM_OK)
            continue;
        // warm-up run (captures the graph), then the timed replays
        st = parem_batch_run(b, texts.data(), stream, d_out, 1);
        if (st == PAREM_OK && hipEventRecord(e0, s) != hipSuccess) st = PAREM_EDEVICE;
        for (uint32_t r = 0; st == PAREM_OK && r < reps; ++r) st = parem_batch_run(b, texts.data(), stream, d_out, 1);
        if (st == PAREM_OK && hipEventRecord(e1, s) != hipSuccess) st = PAREM_EDEVICE;
        if (st == PAREM_OK && hipEventSynchronize(e1) != hipSuccess) st = PAREM_EDEVICE;
        float ms = 0.f;
        if (st == PAREM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = PAREM_EDEVICE;
        parem_batch_free(b);
        if (st != PAREM_OK) break;
        ms_out[c] = ms / (float)reps / (float)k;
        if (best_ms < 0.f || ms_out[c] < best_ms) {
            best_ms = ms_out[c];
            *best = c;
        }
    }
    (void)hipFree(d_out);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == PAREM_OK && best_ms < 0.f) st = PAREM_EUNSUPPORTED;
    return st;
}

}  // extern "C"

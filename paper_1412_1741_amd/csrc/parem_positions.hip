// Match positions: the offset of every byte whose step enters a final state
// (the steps Algorithm 1's `found` tally counts, Section II-B; the trace of
// visited states it keeps per walk is the I vector). After the plain walk and
// composition, a down-sweep gives every chunk its true entry state (chunk c
// is entered in chunk c-1's exit); the map entry of that state holds the
// chunk's count on the true route, an exclusive scan of those counts gives
// each chunk's first output slot, and one lane per chunk with matches walks
// its chunk again from the entry state alone, writing its offsets in order.
#include "parem_device.h"

namespace parem {

constexpr uint32_t kScanBlock = 1024;  // elements per scan workgroup (256 threads x 4)

// the true route's count in chunk c: the count of its entry state's map entry
__global__ void k_chunk_counts(const uint32_t *__restrict__ entry, uint64_t C, const uint32_t *__restrict__ map,
                               const uint16_t *__restrict__ map_cls, const uint16_t *__restrict__ inv, uint32_t Q1,
                               uint64_t *__restrict__ cnt) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const uint32_t e = entry[c];
    uint64_t k = 0;
    if (e < Q1) {
        const uint32_t x = inv[(size_t)(map_cls[c] & 0x7fffu) * Q1 + e];
        if (x != 0xffffu) {
            const uint32_t v = map[(uint64_t)x * C + c];
            if ((v & 0xffffu) != kAbsent16) k = v >> 16;
        }
    }
    cnt[c] = k;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t u = (uint64_t)__shfl_up((long long)v, o, 64);
        if (lane >= (uint32_t)o) v += u;
    }
    return v;
}

// exclusive scan of 256 values held one per thread; returns the block total
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t &excl) {
    __shared__ uint64_t wsum[4];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint64_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint64_t before = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < 4; ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    excl = before + inc - v;
    __syncthreads();
    return total;
}

// pass 1: exclusive scan inside each block of kScanBlock values (in place),
// block totals to sums
__global__ __launch_bounds__(256) void k_scan_local(uint64_t *__restrict__ x, uint64_t n, uint64_t *__restrict__ sums) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * 4u;
    uint64_t v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < n ? x[base + k] : 0;
        s += v[k];
    }
    uint64_t excl;
    const uint64_t total = block_excl_scan(s, excl);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) x[base + k] = excl;
        excl += v[k];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// pass 2: exclusive scan of the block totals (one workgroup, tiles of 256)
__global__ __launch_bounds__(256) void k_scan_sums(uint64_t *__restrict__ sums, uint64_t nb) {
    uint64_t carry = 0;
    for (uint64_t t0 = 0; t0 < nb; t0 += 256) {
        const uint64_t i = t0 + threadIdx.x;
        const uint64_t v = i < nb ? sums[i] : 0;
        uint64_t excl;
        const uint64_t total = block_excl_scan(v, excl);
        if (i < nb) sums[i] = carry + excl;
        carry += total;
    }
}

// pass 3: add each block's offset
__global__ __launch_bounds__(256) void k_scan_add(uint64_t *__restrict__ x, uint64_t n,
                                                  const uint64_t *__restrict__ sums) {
    const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (i < n) x[i] += sums[i / kScanBlock];
}

// One lane per chunk with matches: walk it from its entry state, writing the
// offset of every step into a final state at base[c] + k while below cap.
// The (Q+1) x (A+1) column table (next | final << 15, column A: the
// sentinel) and the byte -> column map are staged in LDS when they fit.
__global__ __launch_bounds__(256) void k_positions(const uint8_t *__restrict__ text, uint64_t n, uint32_t L,
                                                   uint64_t C, const uint32_t *__restrict__ entry,
                                                   const uint64_t *__restrict__ cnt,
                                                   const uint64_t *__restrict__ base, const uint8_t *__restrict__ cls,
                                                   const uint16_t *__restrict__ coltab, uint32_t A1, uint32_t Q1,
                                                   uint32_t tab_lds, uint64_t *__restrict__ out, uint64_t cap) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t *cl = smem;
    uint16_t *T = reinterpret_cast<uint16_t *>(smem + 256);
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) cl[i] = cls[i];
    if (tab_lds)
        for (uint32_t i = threadIdx.x; i < Q1 * A1; i += blockDim.x) T[i] = coltab[i];
    __syncthreads();
    const uint16_t *tab = tab_lds ? T : coltab;
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const uint64_t want = cnt[c];
    uint64_t slot = base[c];
    if (want == 0 || slot >= cap) return;
    const uint64_t b = c * (uint64_t)L;
    const uint32_t len = (uint32_t)min((uint64_t)L, n - b);
    const uint64_t stop = min(cap, slot + want);
    uint32_t e = entry[c];
    const uint8_t *p = text + b;
    const bool aligned = (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
    uint32_t i = 0;
    if (aligned) {
        for (; i + 16 <= len && slot < stop; i += 16) {
            const uint4 q = *reinterpret_cast<const uint4 *>(p + i);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t v = tab[e * A1 + cl[(w[k >> 2] >> (8 * (k & 3))) & 0xffu]];
                e = v & 0x7fffu;
                if (v >> 15) {
                    if (slot < stop) out[slot] = b + i + (uint32_t)k;
                    ++slot;
                }
            }
        }
    }
    for (; i < len && slot < stop; ++i) {
        const uint32_t v = tab[e * A1 + cl[p[i]]];
        e = v & 0x7fffu;
        if (v >> 15) {
            out[slot] = b + i;
            ++slot;
        }
    }
}

struct PosPlan {
    PlainPlan p;
    uint64_t off_entry = 0, off_cnt = 0, off_base = 0, off_sums = 0, bytes = 0;
};

static uint32_t positions_chunk_len(const DeviceDfa &d, uint64_t len) {
    if (d.opt.chunk_len) return d.opt.chunk_len;
    // about 2^19 chunks: the second walk of a chunk is one lane's serial
    // chain, so shorter chunks shorten the critical path
    uint32_t L = 256;
    while ((uint64_t)L < (len >> 19) && L < 4096) L <<= 1;
    return L;
}

static parem_status plan_positions(const DeviceDfa &d, uint64_t len, PosPlan *q) {
    parem_status st = plan_boundary(d, len, positions_chunk_len(d, len), &q->p);
    if (st != PAREM_OK) return st;
    const uint64_t C = std::max<uint64_t>(q->p.chunks, 1);
    uint64_t off = q->p.bytes;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = (off + bytes + 255) & ~(uint64_t)255;
        return o;
    };
    q->off_entry = take(C * 4);
    q->off_cnt = take(C * 8);
    q->off_base = take(C * 8);
    q->off_sums = take(((C + kScanBlock - 1) / kScanBlock) * 8);
    q->bytes = off;
    return PAREM_OK;
}

static parem_status launch_positions(const DeviceDfa &d, const PosPlan &q, const uint8_t *d_text, uint64_t *d_pos,
                                     uint64_t cap, uint8_t *ws, hipStream_t s, parem_result *d_out) {
    const PlainPlan &p = q.p;
    if (p.n == 0) return launch_plain(d, p, d_text, ws, s, d_out);
    if (!d.d_coltab) return PAREM_EUNSUPPORTED;
    uint32_t *entry = reinterpret_cast<uint32_t *>(ws + q.off_entry);
    parem_status st = launch_boundary_into(d, p, d_text, entry, ws, s, d_out);
    if (st != PAREM_OK) return st;
    const uint64_t C = p.chunks;
    uint64_t *cnt = reinterpret_cast<uint64_t *>(ws + q.off_cnt);
    uint64_t *base = reinterpret_cast<uint64_t *>(ws + q.off_base);
    uint64_t *sums = reinterpret_cast<uint64_t *>(ws + q.off_sums);
    const uint32_t g = (uint32_t)((C + 255) / 256);
    const WalkArgs a = walk_args(d, p, d_text, ws);
    hipLaunchKernelGGL(k_chunk_counts, dim3(g), dim3(256), 0, s, entry, C, a.map, a.map_cls, d.d_inv, d.Q + 1, cnt);
    if (hipMemcpyAsync(base, cnt, C * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) return PAREM_EDEVICE;
    const uint64_t nb = (C + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_local, dim3((uint32_t)nb), dim3(256), 0, s, base, C, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(g), dim3(256), 0, s, base, C, sums);
    if (cap) {
        const uint32_t Q1 = d.Q + 1, A1 = d.A + 1;
        const uint64_t tab_bytes = (uint64_t)Q1 * A1 * 2;
        const uint32_t tab_lds = tab_bytes <= 48 * 1024 ? 1u : 0u;
        const size_t lds = 256 + (tab_lds ? (size_t)tab_bytes : 0);
        hipLaunchKernelGGL(k_positions, dim3(g), dim3(256), lds, s, d_text, p.n, p.L, C, entry, cnt, base, d.d_cls,
                           d.d_coltab, A1, Q1, tab_lds, d_pos, cap);
    }
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

}  // namespace parem

extern "C" {

parem_status parem_positions_workspace_size(parem_handle h, uint64_t len, uint64_t *bytes) {
    if (!h || !bytes) return PAREM_EINVAL;
    parem::PosPlan q;
    parem_status st = parem::plan_positions(h->dev, len, &q);
    if (st != PAREM_OK) return st;
    *bytes = q.bytes;
    return PAREM_OK;
}

parem_status parem_match_positions_async(parem_handle h, const uint8_t *d_text, uint64_t len, uint64_t *d_positions,
                                         uint64_t cap, void *d_workspace, uint64_t workspace_bytes, void *stream,
                                         parem_result *d_out) {
    if (!h || !d_out || (len && !d_text) || (cap && !d_positions)) return PAREM_EINVAL;
    parem::PosPlan q;
    parem_status st = parem::plan_positions(h->dev, len, &q);
    if (st != PAREM_OK) return st;
    if (len && (!d_workspace || workspace_bytes < q.bytes)) return PAREM_EINVAL;
    return parem::launch_positions(h->dev, q, d_text, d_positions, cap, reinterpret_cast<uint8_t *>(d_workspace),
                                   reinterpret_cast<hipStream_t>(stream), d_out);
}

}  // extern "C"

// C-ABI of the speculative chunked DFA walk: compile (validation, per-symbol
// speculated sets, table layout, upload) and the match entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "parem_internal.h"

using parem::DeviceDfa;
using parem::KgParams;

namespace {

template <typename T>
parem_status upload(const std::vector<T> &h, T **d, size_t pad_to = 16) {
    size_t bytes = h.size() * sizeof(T);
    size_t alloc = std::max<size_t>((bytes + pad_to - 1) / pad_to * pad_to, pad_to);
    if (hipMalloc(reinterpret_cast<void **>(d), alloc) != hipSuccess) return PAREM_ENOMEM;
    if (hipMemset(*d, 0, alloc) != hipSuccess) return PAREM_EDEVICE;
    if (bytes && hipMemcpy(*d, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return PAREM_EDEVICE;
    return PAREM_OK;
}

void release(DeviceDfa &d) {
    hipFree(d.d_table);
    hipFree(d.d_cls);
    hipFree(d.d_loff);
    if (d.d_llist_walk != d.d_llist) hipFree(d.d_llist_walk);
    d.d_llist_walk = nullptr;
    hipFree(d.d_llist);
    hipFree(d.d_final);
    hipFree(d.d_verify);
    hipFree(d.d_inv);
    hipFree(d.d_full);
    hipFree(d.d_enc);
    hipFree(d.d_next);
    hipFree(d.d_step);
    hipFree(d.d_bytes);
    hipFree(d.d_sids);
    hipFree(d.d_coltab);
    d.d_sids = nullptr;
    d.d_coltab = nullptr;
    d.d_next = nullptr;
    d.d_step = nullptr;
    d.d_bytes = nullptr;
    d.d_inv = nullptr;
    d.d_full = nullptr;
    d.d_enc = nullptr;
    d.d_table = nullptr;
    d.d_cls = nullptr;
    d.d_loff = nullptr;
    d.d_llist = nullptr;
    d.d_final = nullptr;
    d.d_verify = nullptr;
}

uint32_t read_entry(const void *table, int eb, uint64_t k) {
    switch (eb) {
        case 1: return static_cast<const uint8_t *>(table)[k];
        case 2: return static_cast<const uint16_t *>(table)[k];
        default: return static_cast<const uint32_t *>(table)[k];
    }
}

// Byte-indexed table: entry (q, x) = delta(q, column of x), the sentinel for
// invalid bytes, with the destination's final flag in the entry's top bit.
template <typename E>
std::vector<E> byte_table(const DeviceDfa &d, const std::vector<uint32_t> &t, uint32_t row) {
    constexpr uint32_t acc_shift = sizeof(E) * 8 - 1;
    std::vector<E> out(((size_t)(d.Q + 1) * row * sizeof(E) + 15) / 16 * 16 / sizeof(E), (E)0);
    for (uint32_t q = 0; q <= d.Q; ++q) {
        for (uint32_t x = 0; x < 256; ++x) {
            uint32_t nx = d.sent;
            if (q < d.Q && d.cls[x] < d.A) nx = t[(size_t)q * d.A + d.cls[x]];
            out[(size_t)q * row + x] = (E)(nx | ((uint32_t)d.final_flag[nx] << acc_shift));
        }
    }
    return out;
}

// Sparse layout: the rows of a table with few exceptions per row displaced
// into one vector of u32 slots (row displacement, the compression used for
// parser and scanner tables). Row q has a base slot b(q), distinct for every
// row; its exception on key k (the byte itself when every byte is valid,
// else the byte's column) sits in slot b(q) + k. A step from q on key k
// reads slot b(q) + k and takes it when the slot's key field is k, else the
// default: a slot that another row r owns at b(r) + k' = b(q) + k has
// k' != k because bases differ, and the key field of a slot no row owns
// never matches (below). The walk's state is the base, or for the uniform
// form the base with the state's final flag in bits 16-23.
//
// Uniform form, when every row's exceptions against one common default D
// (the most frequent default) fit: a slot holds the next state's base
// (bits 0-15), its final flag (bits 16-23) and the key (bits 24-31); the
// walk keeps D's value in a register, so a step is one LDS read. The key
// field of a free slot j is a byte x such that no row has base j - x.
//
// General form: each row has a header slot at b(q) + 256 holding the base
// of its own default (its most frequent next state) in its low half, q's
// final flag in bits 16-23 and 1 in bits 24-31 (so its high half, like a
// free slot's 0xffff, is at least 256); an exception slot holds the next
// state's base in its low half and the key in its high half. A step reads
// the slot and the header.
//
// Rows are placed first-fit, rows with more exceptions first. LDS image:
// [256 B byte -> column][slots], slots padded to a multiple of four. False
// when neither form fits kSparseLdsMax or the placement search runs over its
// budget.
struct SparseImage {
    std::vector<uint8_t> image;
    std::vector<uint32_t> walk;   // [Q+1] value a walk from each state starts with
    std::vector<uint16_t> sids;   // [slots] state whose row is based at each slot
    bool uniform = false;
    uint32_t d0 = 0;              // uniform form: the default's walk value
};

// first-fit placement of rows (key lists eoff/ekey); `head` adds the header
// slot at base + 256. Bases are distinct; every lookup b + key stays below
// the returned slot count.
bool place_rows(const std::vector<uint32_t> &eoff, const std::vector<uint32_t> &ekey, bool head, uint32_t cap,
                std::vector<uint32_t> &base, std::vector<uint8_t> &used, std::vector<uint8_t> &is_base,
                uint32_t &slots) {
    const uint32_t rows = (uint32_t)eoff.size() - 1;
    std::vector<uint32_t> order(rows);
    for (uint32_t q = 0; q < rows; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return eoff[x + 1] - eoff[x] > eoff[y + 1] - eoff[y]; });
    used.assign(cap, 0);
    is_base.assign(cap, 0);
    base.assign(rows, 0);
    uint32_t first_free = 0;
    slots = 0;
    uint64_t budget = 1ull << 27;  // candidate bases tried
    for (const uint32_t q : order) {
        const uint32_t lo = eoff[q], hi = eoff[q + 1];
        uint32_t least = head ? parem::kSparseHead : 256u;
        for (uint32_t k = lo; k < hi; ++k) least = std::min(least, ekey[k]);
        if (lo == hi && !head) least = 0;
        // a base below first_free - least would put the row's lowest slot on a used one
        uint32_t b = first_free > least ? first_free - least : 0;
        for (;; ++b) {
            if (b + 256 >= cap || budget == 0) return false;
            --budget;
            bool ok = !is_base[b] && !(head && used[b + parem::kSparseHead]);
            for (uint32_t k = lo; ok && k < hi; ++k) ok = !used[b + ekey[k]];
            if (ok) break;
        }
        is_base[b] = 1;
        if (head) used[b + parem::kSparseHead] = 1;
        for (uint32_t k = lo; k < hi; ++k) used[b + ekey[k]] = 1;
        base[q] = b;
        slots = std::max(slots, b + 257);
        while (first_free < cap && used[first_free]) ++first_free;
    }
    return true;
}

bool sparse_slots(const DeviceDfa &d, const std::vector<uint32_t> &t, SparseImage &out) {
    // the invalid column A is reachable only when some byte is outside the alphabet
    bool invalid_used = false;
    for (uint32_t x = 0; x < 256; ++x) invalid_used |= d.cls[x] >= d.A;
    const uint32_t ncol = d.A + (invalid_used ? 1u : 0u);
    if (ncol > 256) return false;
    // every byte valid: keys are the bytes themselves (the walk then needs no
    // byte -> column read); else the columns
    uint32_t key[256];
    for (uint32_t a = 0; a < 256; ++a) key[a] = a;
    if (!invalid_used)
        for (uint32_t x = 0; x < 256; ++x) key[d.cls[x]] = x;
    const uint32_t rows = d.Q + 1;  // row Q, the sentinel, keeps every key in itself
    const uint32_t cap = (parem::kSparseLdsMax - 256) / 4;
    auto next_of = [&](uint32_t q, uint32_t a) { return (q < d.Q && a < d.A) ? t[(size_t)q * d.A + a] : d.sent; };
    // each row's own default (its most frequent next state)
    std::vector<uint32_t> dflt(rows), count(rows, 0), votes(rows, 0);
    for (uint32_t q = 0; q < rows; ++q) {
        uint32_t df = next_of(q, 0), best = 0;
        for (uint32_t a = 0; a < ncol; ++a)
            if (++count[next_of(q, a)] > best) {
                best = count[next_of(q, a)];
                df = next_of(q, a);
            }
        for (uint32_t a = 0; a < ncol; ++a) count[next_of(q, a)] = 0;
        dflt[q] = df;
    }
    uint32_t D = dflt[0], top = 0;
    for (uint32_t q = 0; q < d.Q; ++q)
        if (++votes[dflt[q]] > top) {
            top = votes[dflt[q]];
            D = dflt[q];
        }
    std::vector<uint32_t> base;
    std::vector<uint8_t> used, is_base;
    uint32_t slots = 0;
    for (int form = 0; form < 2; ++form) {
        const bool uni = form == 0;
        // exceptions: columns whose next state is not the default in force
        std::vector<uint32_t> eoff(rows + 1, 0), ekey, enext;
        uint64_t need = 0;
        bool fits = true;
        for (uint32_t q = 0; q < rows && fits; ++q) {
            const uint32_t df = uni ? D : dflt[q];
            for (uint32_t a = 0; a < ncol; ++a) {
                if (next_of(q, a) == df) continue;
                ekey.push_back(key[a]);
                enext.push_back(next_of(q, a));
            }
            eoff[q + 1] = (uint32_t)ekey.size();
            need += eoff[q + 1] - eoff[q] + (uni ? 0 : 1);
            fits = need <= cap;
        }
        if (!fits || !place_rows(eoff, ekey, !uni, cap, base, used, is_base, slots)) continue;
        slots = (slots + 3) / 4 * 4;
        if (256 + (size_t)slots * 4 > parem::kSparseLdsMax) continue;
        std::vector<uint32_t> w(slots, 0xffff0000u);
        if (uni) {
            // a free slot's key field: a byte x with no row based at j - x
            bool ok = true;
            for (uint32_t j = 0; j < slots && ok; ++j) {
                if (j < cap && used[j]) continue;
                uint32_t x = 0;
                while (x < 256 && x <= j && j - x < cap && is_base[j - x]) ++x;
                ok = x < 256;
                w[j] = 0xffffu | x << 24;
            }
            if (!ok) continue;
        }
        auto walk_value = [&](uint32_t q) { return base[q] | (uni ? (uint32_t)d.final_flag[q] << 16 : 0u); };
        for (uint32_t q = 0; q < rows; ++q) {
            const uint32_t b = base[q];
            for (uint32_t k = eoff[q]; k < eoff[q + 1]; ++k)
                w[b + ekey[k]] = uni ? walk_value(enext[k]) | ekey[k] << 24 : base[enext[k]] | ekey[k] << 16;
            if (!uni) w[b + parem::kSparseHead] = base[dflt[q]] | (uint32_t)d.final_flag[q] << 16 | 1u << 24;
        }
        out.image.assign(256 + (size_t)slots * 4, 0);
        for (uint32_t x = 0; x < 256; ++x) out.image[x] = (uint8_t)d.cls[x];
        std::memcpy(out.image.data() + 256, w.data(), (size_t)slots * 4);
        out.sids.assign(slots, 0xffffu);
        out.walk.assign(rows, 0);
        for (uint32_t q = 0; q < rows; ++q) {
            out.sids[base[q]] = (uint16_t)q;
            out.walk[q] = walk_value(q);
        }
        out.uniform = uni;
        out.d0 = uni ? walk_value(D) : 0u;
        return true;
    }
    return false;
}

// Hot-row layout. The hot states are the kHotMax states of largest weight
// under the stationary behaviour of the walk on uniformly random symbols
// (power iteration, averaged over the later iterates so that periodic chains
// settle); their rows go to LDS, followed by one row of kHotLost entries and
// the hot states' ids. Every destination is stored encoded (its slot for a
// hot state, kHotFlag | id for a cold one) with its final flag in bit 15.
// Weight share of the hot states (a cheap stand-in for how often a walk stays
// in LDS rows); fills `order` with the states by decreasing weight.
double hot_share(const DeviceDfa &d, const std::vector<uint32_t> &t, std::vector<uint32_t> &order) {
    const uint32_t Q = d.Q, A = d.A;
    // each row as (target, share of its columns): rows of large sparse tables
    // have few distinct targets, so the iterations touch far fewer entries
    std::vector<uint32_t> roff(Q + 1, 0), tgt;
    std::vector<double> wt;
    std::vector<uint32_t> row(A);
    for (uint32_t q = 0; q < Q; ++q) {
        std::copy(t.begin() + (size_t)q * A, t.begin() + (size_t)(q + 1) * A, row.begin());
        std::sort(row.begin(), row.end());
        for (uint32_t a = 0; a < A;) {
            uint32_t b = a;
            while (b < A && row[b] == row[a]) ++b;
            tgt.push_back(row[a]);
            wt.push_back((double)(b - a) / A);
            a = b;
        }
        roff[q + 1] = (uint32_t)tgt.size();
    }
    std::vector<double> pi(Q, 1.0 / Q), nx(Q), acc(Q, 0.0);
    for (int it = 0; it < 48; ++it) {
        std::fill(nx.begin(), nx.end(), 0.0);
        for (uint32_t q = 0; q < Q; ++q)
            for (uint32_t k = roff[q]; k < roff[q + 1]; ++k) nx[tgt[k]] += pi[q] * wt[k];
        pi.swap(nx);
        if (it >= 16)
            for (uint32_t q = 0; q < Q; ++q) acc[q] += pi[q];
    }
    order.resize(Q);
    for (uint32_t q = 0; q < Q; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return acc[a] > acc[b]; });
    double all = 0.0, top = 0.0;
    for (uint32_t q = 0; q < Q; ++q) all += acc[q];
    for (uint32_t s = 0; s < std::min<uint32_t>(parem::kHotMax, Q); ++s) top += acc[order[s]];
    return all > 0.0 ? top / all : 1.0;
}

void hot_tables(DeviceDfa &d, const std::vector<uint32_t> &t, const std::vector<uint32_t> &order,
                std::vector<uint8_t> &image, std::vector<uint16_t> &full, std::vector<uint16_t> &enc) {
    const uint32_t Q = d.Q, A = d.A;
    const uint32_t H = std::min<uint32_t>(parem::kHotMax, Q);
    enc.assign(Q + 1, 0);
    for (uint32_t q = 0; q <= Q; ++q) enc[q] = (uint16_t)(parem::kHotFlag | q);
    for (uint32_t s = 0; s < H; ++s) enc[order[s]] = (uint16_t)s;
    full.assign((size_t)(Q + 1) * 256, 0);
    for (uint32_t q = 0; q <= Q; ++q) {
        for (uint32_t x = 0; x < 256; ++x) {
            uint32_t nxs = d.sent;
            if (q < Q && d.cls[x] < A) nxs = t[(size_t)q * A + d.cls[x]];
            full[(size_t)q * 256 + x] = (uint16_t)(enc[nxs] | ((uint32_t)d.final_flag[nxs] << 15));
        }
    }
    const size_t rows_bytes = (size_t)(H + 1) * parem::kHotRow * 2;
    image.assign((rows_bytes + (size_t)H * 2 + 15) / 16 * 16, 0);
    uint16_t *rows = reinterpret_cast<uint16_t *>(image.data());
    for (uint32_t s = 0; s < H; ++s) {
        std::copy(full.begin() + (size_t)order[s] * 256, full.begin() + (size_t)order[s] * 256 + 256,
                  rows + (size_t)s * parem::kHotRow);
        rows[(size_t)(H + 1) * parem::kHotRow + s] = (uint16_t)order[s];
    }
    std::fill(rows + (size_t)H * parem::kHotRow, rows + (size_t)(H + 1) * parem::kHotRow,
              (uint16_t)parem::kHotLost);
    d.hot_rows = H;
}

// k-gram layout. Finds B bits and a shift such that (x >> shift) & (2^B - 1)
// is distinct over the alphabet, then tabulates K-symbol steps. Returns false
// when the alphabet has no such code or the table would not fit.
bool build_kgram(DeviceDfa &d, const std::vector<uint32_t> &t, std::vector<uint8_t> &bytes) {
    if (d.A > 8) return false;
    uint32_t need = d.A <= 2 ? 1 : (d.A <= 4 ? 2 : 3);
    std::vector<uint8_t> alpha(d.A);
    for (uint32_t x = 0; x < 256; ++x)
        if (d.cls[x] < d.A) alpha[d.cls[x]] = (uint8_t)x;
    for (uint32_t B = need; B <= 3; ++B) {
        const uint32_t mask = (1u << B) - 1u;
        for (uint32_t shift = 0; shift + B <= 8; ++shift) {
            std::vector<int> code2col(1u << B, -1);
            bool ok = true;
            for (uint32_t j = 0; j < d.A && ok; ++j) {
                const uint32_t code = (alpha[j] >> shift) & mask;
                if (code2col[code] != -1) ok = false;
                else code2col[code] = (int)j;
            }
            if (!ok) continue;
            const uint32_t K = (B == 3) ? 2 : 4;
            const uint32_t RS = K * B + 1;
            if (((uint64_t)(d.Q + 1) << RS) > 65536) return false;
            const uint32_t tk_bytes = (d.Q + 1) << RS;
            const uint32_t t1_bytes = (d.Q + 1) * (1u << B) * 2;
            bytes.assign(((size_t)tk_bytes + t1_bytes + 15) / 16 * 16, 0);
            auto put = [&](size_t off, uint32_t v) {
                bytes[off] = (uint8_t)(v & 0xff);
                bytes[off + 1] = (uint8_t)(v >> 8);
            };
            auto next = [&](uint32_t s, uint32_t code) -> uint32_t {
                if (s == d.sent || code2col[code] < 0) return d.sent;
                return t[(size_t)s * d.A + (uint32_t)code2col[code]];
            };
            const uint32_t ncols = 1u << (K * B);
            for (uint32_t r = 0; r <= d.Q; ++r) {
                for (uint32_t idx = 0; idx < ncols; ++idx) {
                    uint32_t s = r, cnt = 0;
                    for (uint32_t m = 0; m < K; ++m) {
                        s = next(s, (idx >> (B * m)) & mask);
                        cnt += d.final_flag[s];
                    }
                    put(((size_t)r << RS) + 2 * idx, (s << RS) | cnt);
                }
                for (uint32_t code = 0; code <= mask; ++code) {
                    const uint32_t s = next(r, code);
                    put(tk_bytes + (((size_t)r << B) | code) * 2, (s << RS) | d.final_flag[s]);
                }
            }
            KgParams kp;
            kp.shift = shift;
            kp.cmask4 = mask * 0x01010101u;
            kp.bits = B;
            kp.t1_off = tk_bytes;
            if (B == 1) kp.w0 = 0x10080402u;
            else if (B == 2) kp.w0 = 0x80200802u;
            else {
                kp.w0 = 0x00001002u;
                kp.w1 = 0x10020000u;
            }
            // expected byte of each code; an unused code expects a byte whose
            // own code differs (alphabet[0]), so it never validates
            uint8_t v[8];
            for (uint32_t code = 0; code < 8; ++code)
                v[code] = (code <= mask && code2col[code] >= 0) ? alpha[(uint32_t)code2col[code]] : alpha[0];
            kp.vlo = v[0] | (v[1] << 8) | (v[2] << 16) | ((uint32_t)v[3] << 24);
            kp.vhi = v[4] | (v[5] << 8) | (v[6] << 16) | ((uint32_t)v[7] << 24);
            d.kg = kp;
            d.kgram = K;
            return true;
        }
    }
    return false;
}

}  // namespace

extern "C" {

const char *parem_strerror(parem_status s) {
    switch (s) {
        case PAREM_OK: return "ok";
        case PAREM_EINVAL: return "invalid argument";
        case PAREM_ENOMEM: return "out of memory";
        case PAREM_EDEVICE: return "HIP runtime error";
        case PAREM_ESYMBOL: return "text byte outside the alphabet";
        case PAREM_ESTATE: return "state id out of range";
        case PAREM_EUNSUPPORTED: return "unsupported size";
        case PAREM_ESYNTAX: return "regular expression syntax error";
        default: return "unknown status";
    }
}

parem_status parem_compile(const void *table, int entry_bytes, uint32_t num_states, const uint8_t *alphabet,
                           uint32_t alphabet_size, uint32_t start, const uint32_t *accepting,
                           uint32_t num_accepting, const parem_options *opt, parem_handle *out) {
    if (!out) return PAREM_EINVAL;
    *out = nullptr;
    if (!table || !alphabet || (num_accepting && !accepting)) return PAREM_EINVAL;
    if (entry_bytes != 1 && entry_bytes != 2 && entry_bytes != 4) return PAREM_EINVAL;
    if (num_states == 0 || alphabet_size == 0 || alphabet_size > 256) return PAREM_EINVAL;
    if (num_states > 32767) return PAREM_EUNSUPPORTED;
    if (start >= num_states) return PAREM_ESTATE;
    parem_options o{};
    if (opt) {
        o = *opt;
        if (o.partial > 1) return PAREM_EINVAL;
        if (o.lookback > parem::kLookMax) return PAREM_EINVAL;
        if (o.chunk_len % 64 || o.chunk_len > parem::kMaxChunk) return PAREM_EINVAL;
        if (o.group && o.group != 2 && o.group != 4 && o.group != 8 && o.group != 16) return PAREM_EINVAL;
        if (o.layout > PAREM_LAYOUT_SPARSE_LDS) return PAREM_EINVAL;
        if (o.tile && o.tile != 64 && o.tile != 128) return PAREM_EINVAL;
        if (o.policy > PAREM_POLICY_ENUMERATE) return PAREM_EINVAL;
        if (o.no_merge > 1) return PAREM_EINVAL;
        // lookback sets shrink the speculated sets by another rule; the
        // Enumeration policy walks every state of total tables only
        if ((o.partial || o.policy == PAREM_POLICY_ENUMERATE) && o.lookback) return PAREM_EINVAL;
        if (o.partial && o.policy == PAREM_POLICY_ENUMERATE) return PAREM_EINVAL;
    }
    // a partial table gains one state (dead); the S filter reads the
    // next-state table, which holds Q + 1 <= kLookStates states
    if (o.partial && num_states + 2 > parem::kLookStates) return PAREM_EUNSUPPORTED;

    parem_dfa *h = new (std::nothrow) parem_dfa();
    if (!h) return PAREM_ENOMEM;
    DeviceDfa &d = h->dev;
    d.user_Q = num_states;
    d.Q = o.partial ? num_states + 1 : num_states;
    d.dead = o.partial ? num_states : 0xffffffffu;
    d.A = alphabet_size;
    d.start = start;
    d.sent = d.Q;
    d.opt = o;
    d.num_classes = d.A + 2;

    d.cls.assign(256, (uint8_t)0);
    std::vector<int> seen(256, 0);
    for (uint32_t j = 0; j < d.A; ++j) {
        if (seen[alphabet[j]]) {
            delete h;
            return PAREM_EINVAL;
        }
        seen[alphabet[j]] = 1;
    }
    // class A (invalid) does not fit in a byte when A == 256; all bytes are then valid
    for (uint32_t x = 0; x < 256; ++x) d.cls[x] = (uint8_t)std::min<uint32_t>(d.A, 255);
    for (uint32_t j = 0; j < d.A; ++j) d.cls[alphabet[j]] = (uint8_t)j;

    // the table (for a partial one: undefined entries -> dead, and the dead
    // row, which stays dead)
    const uint32_t undef = entry_bytes == 1 ? 0xffu : (entry_bytes == 2 ? 0xffffu : 0xffffffffu);
    std::vector<uint32_t> t((size_t)d.Q * d.A);
    for (uint64_t k = 0; k < (uint64_t)d.user_Q * d.A; ++k) {
        t[k] = read_entry(table, entry_bytes, k);
        if (o.partial && t[k] == undef) t[k] = d.dead;
        else if (t[k] >= d.user_Q) {
            delete h;
            return PAREM_ESTATE;
        }
    }
    if (o.partial)
        for (uint32_t a = 0; a < d.A; ++a) t[(size_t)d.dead * d.A + a] = d.dead;
    d.final_flag.assign(d.Q + 1, 0);
    for (uint32_t i = 0; i < num_accepting; ++i) {
        if (accepting[i] >= d.user_Q) {
            delete h;
            return PAREM_ESTATE;
        }
        d.final_flag[accepting[i]] = 1;
    }

    // speculated set per class: image of the column (L of Algorithm 1; for a
    // partial table completed with dead, which the S filter leaves out of the
    // walks), every state under the Enumeration
    // policy, the sentinel after an invalid byte, and {q0} for the first chunk
    d.loff.assign(d.num_classes + 1, 0);
    d.llist.clear();
    std::vector<uint8_t> mark(d.Q + 1);
    for (uint32_t c = 0; c < d.num_classes; ++c) {
        d.loff[c] = (uint32_t)d.llist.size();
        if (c < d.A && o.policy == PAREM_POLICY_ENUMERATE) {
            for (uint32_t q = 0; q < d.Q; ++q) d.llist.push_back(q);
        } else if (c < d.A) {
            std::fill(mark.begin(), mark.end(), 0);
            for (uint32_t q = 0; q < d.Q; ++q) mark[t[(size_t)q * d.A + c]] = 1;
            // the run may have died anywhere before: dead is a possible entry
            // of every chunk (its map entry is known, it is never walked)
            if (o.partial) mark[d.dead] = 1;
            for (uint32_t q = 0; q <= d.Q; ++q)
                if (mark[q]) d.llist.push_back(q);
        } else if (c == d.A) {
            d.llist.push_back(d.sent);
        } else {
            d.llist.push_back(d.start);
        }
        d.max_spec = std::max<uint32_t>(d.max_spec, (uint32_t)d.llist.size() - d.loff[c]);
    }
    d.loff[d.num_classes] = (uint32_t)d.llist.size();
    d.total_list = (uint32_t)d.llist.size();

    // layout: k-gram when the alphabet has a bit-field code and the table
    // fits; else the byte table in LDS (Q+1 <= 128) or read through L2
    uint32_t layout = o.layout;
    std::vector<uint8_t> kgbytes;
    const bool kg_ok = (layout == PAREM_LAYOUT_AUTO || layout == PAREM_LAYOUT_KGRAM_LDS) && build_kgram(d, t, kgbytes);
    const bool lds_ok = d.Q + 1 <= 128;
    const bool hot_ok = d.Q + 1 <= 0x3fffu;  // kHotFlag | id stays below kHotLost
    const bool class_ok = 256 + (uint64_t)(d.Q + 1) * (d.A + 1) * 2 <= parem::kClassLdsMax;
    std::vector<uint32_t> hot_order;
    // automatic choice: k-gram, LDS byte table, column-indexed LDS table, then
    // sparse rows when every row qualifies (checked once), hot rows only when
    // they hold most of the walk's weight, else the byte table through L2
    SparseImage sparse;
    const bool big_auto = layout == PAREM_LAYOUT_AUTO && !kg_ok && !lds_ok && !class_ok;
    const bool sparse_ok = (big_auto || layout == PAREM_LAYOUT_SPARSE_LDS) &&
                           sparse_slots(d, t, sparse);
    const bool hot_auto = hot_ok && !kg_ok && !lds_ok && !class_ok && !(big_auto && sparse_ok) &&
                          hot_share(d, t, hot_order) >= 0.9;
    const uint32_t big = hot_auto ? PAREM_LAYOUT_HOT_LDS : PAREM_LAYOUT_BYTE_GLOBAL;
    if (layout == PAREM_LAYOUT_AUTO || (layout == PAREM_LAYOUT_KGRAM_LDS && !kg_ok))
        layout = kg_ok ? PAREM_LAYOUT_KGRAM_LDS
                       : (lds_ok ? PAREM_LAYOUT_BYTE_LDS : (class_ok ? PAREM_LAYOUT_CLASS_LDS : big));
    if (layout == PAREM_LAYOUT_BYTE_LDS && !lds_ok) layout = class_ok ? PAREM_LAYOUT_CLASS_LDS : big;
    if (layout == PAREM_LAYOUT_CLASS_LDS && !class_ok) layout = big;
    if (layout == PAREM_LAYOUT_HOT_LDS && !hot_ok) layout = PAREM_LAYOUT_BYTE_GLOBAL;
    // sparse layout: asked for, or chosen automatically when no dense table
    // fits LDS, and only when the rows' exceptions (columns other than a row's
    // default; the invalid column counts unless every byte is in the
    // alphabet) and headers fit the slots
    if (layout == PAREM_LAYOUT_SPARSE_LDS && !sparse_ok) layout = class_ok ? PAREM_LAYOUT_CLASS_LDS : big;
    if (big_auto && sparse_ok) layout = PAREM_LAYOUT_SPARSE_LDS;
    d.layout = layout;
    if (layout == PAREM_LAYOUT_SPARSE_LDS) {
        bool all_valid = true;
        for (uint32_t x = 0; x < 256; ++x) all_valid &= d.cls[x] < d.A;
        d.sparse_raw = all_valid;
        d.sparse_uniform = sparse.uniform;
        d.sparse_d0 = sparse.d0;
    }
    if (layout != PAREM_LAYOUT_KGRAM_LDS) {
        d.kgram = 0;
        d.kg = parem::KgParams{};
    }

    parem_status st = PAREM_OK;
    std::vector<uint16_t> hot_enc;
    if (hipGetDevice(&d.device) != hipSuccess) st = PAREM_EDEVICE;
    if (st == PAREM_OK) {
        if (layout == PAREM_LAYOUT_KGRAM_LDS) {
            d.entry_bytes = 2;
            d.table_bytes = (uint32_t)kgbytes.size();
            d.lds_bytes = d.table_bytes;
            uint8_t *p = nullptr;
            st = upload(kgbytes, &p);
            d.d_table = p;
        } else if (layout == PAREM_LAYOUT_BYTE_LDS) {
            auto bt = byte_table<uint8_t>(d, t, parem::kByteLdsRow);
            d.entry_bytes = 1;
            d.row_stride = parem::kByteLdsRow;
            d.table_bytes = (uint32_t)bt.size();
            d.lds_bytes = d.table_bytes;
            uint8_t *p = nullptr;
            st = upload(bt, &p);
            d.d_table = p;
        } else if (layout == PAREM_LAYOUT_CLASS_LDS) {
            // [256 B byte -> column][(Q+1) x (A+1) u16 entries]
            const uint32_t A1 = d.A + 1;
            std::vector<uint8_t> image((256 + (size_t)(d.Q + 1) * A1 * 2 + 15) / 16 * 16, 0);
            for (uint32_t x = 0; x < 256; ++x) image[x] = d.cls[x];
            uint16_t *T = reinterpret_cast<uint16_t *>(image.data() + 256);
            for (uint32_t q = 0; q <= d.Q; ++q) {
                for (uint32_t a = 0; a < A1; ++a) {
                    const uint32_t nx = (q < d.Q && a < d.A) ? t[(size_t)q * d.A + a] : d.sent;
                    T[(size_t)q * A1 + a] = (uint16_t)(nx | ((uint32_t)d.final_flag[nx] << 15));
                }
            }
            d.entry_bytes = 2;
            d.row_stride = A1;
            d.table_bytes = (uint32_t)image.size();
            d.lds_bytes = d.table_bytes;
            uint8_t *p = nullptr;
            st = upload(image, &p);
            d.d_table = p;
        } else if (layout == PAREM_LAYOUT_SPARSE_LDS) {
            d.entry_bytes = 4;
            d.row_stride = 0;
            d.table_bytes = (uint32_t)sparse.image.size();
            d.lds_bytes = d.table_bytes;
            uint8_t *p = nullptr;
            st = upload(sparse.image, &p);
            d.d_table = p;
            if (st == PAREM_OK) st = upload(sparse.sids, &d.d_sids);
            // batches walk such a table as the byte table through L2
            if (st == PAREM_OK) st = upload(byte_table<uint16_t>(d, t, 256), &d.d_bytes);
        } else if (layout == PAREM_LAYOUT_HOT_LDS) {
            std::vector<uint8_t> image;
            std::vector<uint16_t> full, enc;
            if (hot_order.empty()) hot_share(d, t, hot_order);
            hot_tables(d, t, hot_order, image, full, enc);
            hot_enc = enc;
            d.entry_bytes = 2;
            d.row_stride = parem::kHotRow;
            d.table_bytes = (uint32_t)image.size();
            d.lds_bytes = d.table_bytes;
            uint8_t *p = nullptr;
            st = upload(image, &p);
            d.d_table = p;
            if (st == PAREM_OK) st = upload(full, &d.d_full);
            if (st == PAREM_OK) st = upload(enc, &d.d_enc);
        } else {
            auto bt = byte_table<uint16_t>(d, t, 256);
            d.entry_bytes = 2;
            d.row_stride = 256;
            d.table_bytes = (uint32_t)(bt.size() * 2);
            d.lds_bytes = 0;
            uint16_t *p = nullptr;
            st = upload(bt, &p);
            d.d_table = p;
        }
    }
    if (st == PAREM_OK) st = upload(d.cls, &d.d_cls);
    if (st == PAREM_OK) st = upload(d.loff, &d.d_loff);
    if (st == PAREM_OK) st = upload(d.llist, &d.d_llist);
    d.d_llist_walk = d.d_llist;
    if (st == PAREM_OK && (layout == PAREM_LAYOUT_HOT_LDS || layout == PAREM_LAYOUT_SPARSE_LDS)) {
        // walks start from encoded ids (hot rows) or bases (sparse layout): no
        // lookup of the encoding per walk
        std::vector<uint32_t> enc_list(d.llist.size());
        for (size_t k = 0; k < d.llist.size(); ++k)
            enc_list[k] = layout == PAREM_LAYOUT_HOT_LDS ? hot_enc[d.llist[k]] : sparse.walk[d.llist[k]];
        st = upload(enc_list, &d.d_llist_walk);
    }
    if (st == PAREM_OK) st = upload(d.final_flag, &d.d_final);
    if (st == PAREM_OK && d.Q + 1 <= parem::kLookStates) {
        // next state by class for lookback sets; the sentinel row stays in the sentinel
        std::vector<uint16_t> nx((size_t)(d.Q + 1) * d.A);
        for (uint32_t q = 0; q <= d.Q; ++q)
            for (uint32_t a = 0; a < d.A; ++a)
                nx[(size_t)q * d.A + a] = (uint16_t)(q < d.Q ? t[(size_t)q * d.A + a] : d.sent);
        st = upload(nx, &d.d_next);
    }
    if (st == PAREM_OK) {
        // next state by class with the invalid class A, final flag in bit 15:
        // match positions walk it; the sub-chunk re-walk of learned
        // speculation stages it in LDS when it is small
        std::vector<uint16_t> sx((size_t)(d.Q + 1) * (d.A + 1));
        for (uint32_t q = 0; q <= d.Q; ++q)
            for (uint32_t a = 0; a <= d.A; ++a) {
                const uint32_t e = (q < d.Q && a < d.A) ? t[(size_t)q * d.A + a] : d.sent;
                sx[(size_t)q * (d.A + 1) + a] = (uint16_t)(e | (e < d.Q && d.final_flag[e] ? 0x8000u : 0u));
            }
        st = upload(sx, &d.d_coltab);
        if (st == PAREM_OK && sx.size() <= parem::kSplitTable) st = upload(sx, &d.d_step);
    }
    // inverse index of the class lists (composition looks up the position of
    // an end state in the next chunk's list); skipped when it would be huge
    const uint64_t inv_entries = (uint64_t)d.num_classes * (d.Q + 1);
    if (st == PAREM_OK && inv_entries * 2 <= (16u << 20)) {
        std::vector<uint16_t> inv((size_t)((inv_entries + 1) / 2 * 2), (uint16_t)0xffff);
        for (uint32_t c = 0; c < d.num_classes; ++c)
            for (uint32_t k = d.loff[c]; k < d.loff[c + 1]; ++k)
                inv[(size_t)c * (d.Q + 1) + d.llist[k]] = (uint16_t)(k - d.loff[c]);
        const uint32_t bytes = (uint32_t)(inv.size() * 2);
        d.inv_lds = bytes <= 16384 ? bytes : 0;
        st = upload(inv, &d.d_inv);
    }
    if (st != PAREM_OK) {
        release(d);
        delete h;
        return st;
    }
    *out = h;
    return PAREM_OK;
}

void parem_free(parem_handle h) {
    if (!h) return;
    release(h->dev);
    delete h;
}

parem_status parem_describe(parem_handle h, uint32_t *layout, uint32_t *max_spec, uint32_t *lds_bytes,
                            uint32_t *kgram) {
    if (!h) return PAREM_EINVAL;
    if (layout) *layout = h->dev.layout;
    if (max_spec) *max_spec = h->dev.max_spec;
    if (lds_bytes) *lds_bytes = h->dev.lds_bytes;
    if (kgram) *kgram = h->dev.kgram;
    return PAREM_OK;
}

parem_status parem_workspace_size(parem_handle h, uint64_t len, uint64_t *bytes) {
    if (!h || !bytes) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_plain(h->dev, len, &p);
    if (st != PAREM_OK) return st;
    *bytes = p.bytes;
    return PAREM_OK;
}

parem_status parem_match_async(parem_handle h, const uint8_t *d_text, uint64_t len, void *d_workspace,
                               uint64_t workspace_bytes, void *stream, parem_result *d_out) {
    if (!h || !d_out || (len && !d_text)) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_plain(h->dev, len, &p);
    if (st != PAREM_OK) return st;
    if (len && (!d_workspace || workspace_bytes < p.bytes)) return PAREM_EINVAL;
    return parem::launch_plain(h->dev, p, d_text, d_workspace, reinterpret_cast<hipStream_t>(stream), d_out);
}

parem_status parem_match_async_timed(parem_handle h, const uint8_t *d_text, uint64_t len, void *d_workspace,
                                     uint64_t workspace_bytes, void *stream, parem_result *d_out,
                                     void *ev_walk_begin, void *ev_walk_end) {
    if (!h || !d_out || (len && !d_text)) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_plain(h->dev, len, &p);
    if (st != PAREM_OK) return st;
    if (len && (!d_workspace || workspace_bytes < p.bytes)) return PAREM_EINVAL;
    return parem::launch_plain(h->dev, p, d_text, d_workspace, reinterpret_cast<hipStream_t>(stream), d_out,
                               reinterpret_cast<hipEvent_t>(ev_walk_begin), reinterpret_cast<hipEvent_t>(ev_walk_end));
}

parem_status parem_boundary_workspace_size(parem_handle h, uint64_t len, uint32_t chunk_len, uint64_t *bytes) {
    if (!h || !bytes || chunk_len == 0) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_boundary(h->dev, len, chunk_len, &p);
    if (st != PAREM_OK) return st;
    *bytes = p.bytes;
    return PAREM_OK;
}

parem_status parem_boundary_states(parem_handle h, const uint8_t *d_text, uint64_t len, uint32_t chunk_len,
                                   uint32_t *d_states, void *d_workspace, uint64_t workspace_bytes, void *stream) {
    if (!h || (len && (!d_text || !d_states)) || chunk_len == 0) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_boundary(h->dev, len, chunk_len, &p);
    if (st != PAREM_OK) return st;
    if (len && (!d_workspace || workspace_bytes < p.bytes)) return PAREM_EINVAL;
    return parem::launch_boundary(h->dev, p, d_text, d_states, d_workspace, reinterpret_cast<hipStream_t>(stream));
}

parem_status parem_learned_workspace_size(parem_handle h, parem_proposal pr, uint64_t len, uint64_t *bytes) {
    if (!h || !pr || !bytes) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_learned(h->dev, *pr, len, 16, h->dev.opt, &p);
    if (st != PAREM_OK) return st;
    *bytes = p.bytes;
    return PAREM_OK;
}

parem_status parem_match_learned_async(parem_handle h, parem_proposal pr, uint32_t m, const uint8_t *d_text,
                                       uint64_t len, void *d_workspace, uint64_t workspace_bytes, void *stream,
                                       parem_result *d_out, void *ev_walk_begin, void *ev_walk_end) {
    if (!h || !pr || !d_out || (len && !d_text) || m == 0 || m > 16) return PAREM_EINVAL;
    if (pr->dfa != &h->dev) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_learned(h->dev, *pr, len, m, h->dev.opt, &p);
    if (st != PAREM_OK) return st;
    if (len && (!d_workspace || workspace_bytes < p.bytes)) return PAREM_EINVAL;
    return parem::launch_learned(h->dev, *pr, p, d_text, d_workspace, reinterpret_cast<hipStream_t>(stream), d_out,
                                 reinterpret_cast<hipEvent_t>(ev_walk_begin), reinterpret_cast<hipEvent_t>(ev_walk_end));
}

parem_status parem_match(parem_handle h, const uint8_t *text, uint64_t len, parem_result *out) {
    if (!h || !out || (len && !text)) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_plain(h->dev, len, &p);
    if (st != PAREM_OK) return st;

    bool on_device = false;
    if (len) {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, text) == hipSuccess) {
            on_device = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
        } else {
            (void)hipGetLastError();  // plain host memory
        }
    }
    uint8_t *staged = nullptr;
    void *ws = nullptr;
    parem_result *d_out = nullptr;
    st = PAREM_OK;
    if (len && !on_device) {
        if (hipMalloc(&staged, len) != hipSuccess) st = PAREM_ENOMEM;
        else if (hipMemcpy(staged, text, len, hipMemcpyHostToDevice) != hipSuccess) st = PAREM_EDEVICE;
    }
    if (st == PAREM_OK && p.bytes && hipMalloc(&ws, p.bytes) != hipSuccess) st = PAREM_ENOMEM;
    if (st == PAREM_OK && hipMalloc(&d_out, sizeof(parem_result)) != hipSuccess) st = PAREM_ENOMEM;
    if (st == PAREM_OK) {
        const uint8_t *src = on_device ? text : staged;
        st = parem::launch_plain(h->dev, p, src, ws, nullptr, d_out);
    }
    if (st == PAREM_OK && hipMemcpy(out, d_out, sizeof(parem_result), hipMemcpyDeviceToHost) != hipSuccess)
        st = PAREM_EDEVICE;
    hipFree(staged);
    hipFree(ws);
    hipFree(d_out);
    if (st == PAREM_OK && out->final_state == 0xffffffffu) st = PAREM_ESYMBOL;
    return st;
}

}  // extern "C"

// Internal definitions shared by the host compile step, the C-ABI and the
// HIP kernels of the speculative chunked DFA walk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/parem.h"

namespace parem {

// k-gram layout: a text byte x maps to the symbol code (x >> shift) & cmask
// (B bits, B = 1..3, chosen so the alphabet's codes are distinct); one table
// lookup consumes K = (B == 3 ? 2 : 4) symbols. A state is carried as its
// table row base (state << RS, RS = K*B + 1 bytes per row of u16 entries);
// entries hold (next state << RS) | (final destinations among the K steps).
struct KgParams {
    uint32_t shift = 0;
    uint32_t cmask4 = 0;   // cmask in every byte
    uint32_t w0 = 0, w1 = 0; // dot4 weights giving 2*index of symbols 0..K-1 (w1: second pair, B == 3)
    uint32_t vlo = 0, vhi = 0; // expected byte of codes 0..3 / 4..7 (validation with v_perm)
    uint32_t t1_off = 0;   // byte offset of the one-symbol table (tails)
    uint32_t bits = 0;     // B
};

// Lists of speculated states are indexed by "class": the column of the byte
// just before a chunk (0..A-1), the invalid-byte class A (list {SENT}) and the
// start class A+1 (list {q0}, used by chunk 0).
struct DeviceDfa {
    uint32_t Q = 0, A = 0, start = 0;
    uint32_t sent = 0;           // absorbing sentinel state (= Q) entered on an invalid byte
    uint32_t num_classes = 0;    // A + 2
    uint32_t max_spec = 0;       // largest list size over all classes
    uint32_t total_list = 0;     // sum of list sizes
    uint32_t layout = 0;
    uint32_t entry_bytes = 0;    // bytes per byte-table entry (1 or 2)
    uint32_t lds_bytes = 0;      // LDS the walk kernel stages its table in
    uint32_t kgram = 0;          // symbols per k-gram step (k-gram layout)
    uint32_t sym_bits = 0;       // bits per symbol code (k-gram layout)
    uint32_t hash_shift = 0;     // symbol code = (byte >> hash_shift) & mask (k-gram layout)
    uint32_t table_bytes = 0;    // bytes of d_table (16-byte padded)
    uint32_t row_stride = 256;   // byte layouts: entries per table row in memory
    KgParams kg{};
    parem_options opt{};
    int device = 0;

    // host copies
    std::vector<uint8_t> cls;        // [256] byte -> class (A when invalid)
    std::vector<uint32_t> loff;      // [num_classes + 1]
    std::vector<uint32_t> llist;     // concatenated sorted lists
    std::vector<uint8_t> final_flag; // [Q + 1]

    // device copies (owned)
    void *d_table = nullptr;         // layout-specific table
    uint8_t *d_cls = nullptr;
    uint32_t *d_loff = nullptr;
    uint32_t *d_llist = nullptr;
    uint8_t *d_final = nullptr;
    uint8_t *d_verify = nullptr;     // unused (kept null)
    uint16_t *d_inv = nullptr;       // [(A+2) * (Q+1)] position of a state in each class list, 0xffff if absent
    uint32_t inv_lds = 0;            // bytes of d_inv staged in LDS by the compose kernels (0: read from L2)
};

// Workspace carving for one plain match.
struct PlainPlan {
    uint64_t n = 0;
    uint32_t L = 0;          // chunk length
    uint64_t chunks = 0;
    uint32_t RM = 0;         // map width (max_spec)
    uint32_t P = 0;          // maps composed per workgroup in the tree
    uint32_t G = 0;          // lockstep group
    uint32_t tile = 0;       // staged tile bytes per chunk (64 or 128)
    uint32_t merge = 1;      // 0: speculated runs are never merged
    std::vector<uint64_t> level_maps; // number of maps after each compose level
    uint64_t bytes = 0;
    // offsets into the workspace
    uint64_t off_cend = 0, off_ccnt = 0, off_ccls = 0;
    uint64_t off_a_end = 0, off_a_cnt = 0, off_a_cls = 0, off_a_runs = 0;
    uint64_t off_b_end = 0, off_b_cnt = 0, off_b_cls = 0, off_b_runs = 0;
    uint64_t level_cap = 0;
};

constexpr uint32_t kByteLdsRow = 260;  // row stride of the LDS byte table
constexpr uint32_t kMaxChunk = 32768;  // chunk maps pack a count < 2^16 beside the end state

parem_status plan_plain(const DeviceDfa &d, uint64_t len, PlainPlan *p);
parem_status launch_plain(const DeviceDfa &d, const PlainPlan &p, const uint8_t *d_text,
                          void *d_ws, hipStream_t stream, parem_result *d_out,
                          hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);

}  // namespace parem

struct parem_dfa {
    parem::DeviceDfa dev;
};

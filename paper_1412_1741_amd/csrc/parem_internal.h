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
    // partial tables: the caller's Q states plus one absorbing, non-final
    // state `dead` (= the caller's Q) standing for every undefined transition;
    // Q counts it. 0xffffffff for total tables.
    uint32_t dead = 0xffffffffu;
    uint32_t user_Q = 0;         // states of the caller's table
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
    uint32_t *d_llist_walk = nullptr; // the lists as walks start from them (hot rows: encoded ids), else d_llist
    uint8_t *d_final = nullptr;
    uint8_t *d_verify = nullptr;     // unused (kept null)
    uint16_t *d_inv = nullptr;       // [(A+2) * (Q+1)] position of a state in each class list, 0xffff if absent
    uint32_t inv_lds = 0;            // bytes of d_inv staged in LDS by the compose kernels (0: read from L2)
    // hot-row layout: d_table is the LDS image (hot rows, then their state ids)
    uint16_t *d_full = nullptr;      // (Q+1) x 256 byte table with encoded destinations
    uint16_t *d_next = nullptr;      // [(Q+1) x A] next state by class (lookback sets); row Q: the sentinel
    uint16_t *d_enc = nullptr;       // [Q+1] encoded id of each state (slot when hot, 0x4000 | id else)
    uint16_t *d_step = nullptr;      // [(Q+1) x (A+1)] next state by class | final << 15 (small tables only)
    uint16_t *d_bytes = nullptr;     // sparse layout: the (Q+1) x 256 u16 byte table for batch walks
    uint16_t *d_sids = nullptr;      // sparse layout: [slots] state whose row is based at each slot
    uint16_t *d_coltab = nullptr;    // [(Q+1) x (A+1)] next state by column | final << 15 (match positions)
    uint32_t hot_rows = 0;
    bool sparse_raw = false;         // sparse rows are keyed by bytes, not columns (every byte valid)
    bool sparse_uniform = false;     // sparse rows share one default (no header slots)
    uint32_t sparse_d0 = 0;          // that default's walk value (base | final flag << 16)
};

// hot-row layout: at most kHotMax rows of kHotRow u16 entries (256 bytes plus
// padding that shifts successive rows by one LDS bank)
constexpr uint32_t kHotMax = 32;
constexpr uint32_t kClassLdsMax = 48 * 1024;  // largest column-indexed LDS table
// sparse layout (rows displaced into one vector of u32 slots): a row's
// header slot sits kSparseHead slots after its base; the LDS image is the
// 256-byte byte -> column map and the slots, at most kSparseLdsMax bytes
// (160 KiB of LDS less sixteen waves' 4 KiB text tiles)
constexpr uint32_t kSparseHead = 256;
constexpr uint32_t kSparseLdsMax = 160 * 1024 - 16 * 4096;
constexpr uint32_t kHotRow = 258;
constexpr uint32_t kHotFlag = 0x4000u;  // cold state: kHotFlag | id; hot state: its slot
constexpr uint32_t kHotLost = 0x7fffu;  // entries of the extra LDS row H

// learned proposal network dimensions (32-byte window, 16-d embeddings)
constexpr uint32_t kMlpWindow = 32;
constexpr uint32_t kMlpEmb = 16;
constexpr uint32_t kMlpIn = kMlpWindow * kMlpEmb;
constexpr uint32_t kMlpHid = 256;

// end state of an entry that was not walked (learned speculation)
constexpr uint32_t kAbsent16 = 0xffffu;
constexpr uint32_t kAbsent32 = 0xffffffffu;

struct Proposal {
    const DeviceDfa *dfa = nullptr;
    uint32_t S = 0;              // head rows (= Q)
    size_t nparams = 0;
    size_t o_emb = 0, o_W1 = 0, o_b1 = 0, o_W2 = 0, o_b2 = 0, o_W3 = 0, o_b3 = 0;
    float *d_params = nullptr;   // fp32 master weights
    uint16_t *d_params16 = nullptr;
    float *d_grad = nullptr, *d_m = nullptr, *d_v = nullptr;
    uint64_t step = 0;
    // training scratch (grown on demand)
    void *t_buf = nullptr;
    uint32_t cap_batch = 0;
    size_t t_pos = 0, t_lab = 0, t_win = 0, t_cls = 0, t_X = 0, t_pre1 = 0, t_H1 = 0, t_pre2 = 0, t_H2 = 0,
           t_Z = 0, t_dZ32 = 0, t_dZ16 = 0, t_dA2_32 = 0, t_dA2_16 = 0, t_dA1_32 = 0, t_dA1_16 = 0, t_dX = 0,
           t_loss = 0, t_part = 0;
};

void proposal_layout(Proposal &p);
parem_status proposal_adamw(Proposal &p, const float *d_grad, float lr, float wd, hipStream_t s);
size_t proposal_infer_bytes(const Proposal &p, uint64_t rows);
// `zero`: nzero u32 counters the selection also clears (the learned match's
// coverage counters, which saves a launch); may be null
parem_status proposal_select(const Proposal &p, const uint8_t *d_text, uint64_t L, uint32_t chunks, uint32_t m,
                             uint32_t RM, void *scratch, hipStream_t s, uint16_t *sel, uint8_t *nsel,
                             uint32_t *zero = nullptr, uint32_t nzero = 0);

// Workspace carving for one match.
struct PlainPlan {
    uint64_t n = 0;
    uint32_t L = 0;          // chunk length
    uint64_t chunks = 0;
    uint32_t RM = 0;         // map width (max_spec)
    uint32_t P = 0;          // chunk maps composed per workgroup (first level)
    uint32_t P2 = 0;         // segment maps composed per workgroup (later levels)
    uint32_t G = 0;          // lockstep group
    uint32_t tile = 0;       // staged tile bytes per chunk (64 or 128)
    uint32_t merge = 1;      // 0: speculated runs are never merged
    uint32_t m = 0;          // learned: states walked per chunk
    uint32_t look = 0;       // lookback bytes (0: the speculated sets of Algorithm 1)
    bool sfilter = false;    // partial table: walk only S intersect L (selection per chunk)
    uint32_t relook = 0;     // learned: chunks walked again use lookback sets of this window
    uint64_t off_lsel = 0, off_lnsel = 0;  // learned: their selections
    bool keep = false;       // keep every composition level (down-sweep)
    std::vector<uint64_t> levels;  // maps after each composition level
    struct Seg {
        uint64_t end = 0, cnt = 0, cls = 0, runs = 0, lead = 0;
    };
    std::vector<Seg> seg;          // per kept level, or two ping-pong buffers
    std::vector<uint64_t> entries; // boundary states: entry states per level
    uint64_t bytes = 0;
    uint64_t off_map = 0, off_mcls = 0, off_mlead = 0, off_dummy = 0;
    uint64_t off_sel = 0, off_nsel = 0, off_redo = 0, off_done = 0, off_flags = 0, off_mlp = 0, off_rlist = 0, off_part = 0;
    uint64_t off_todo = 0;   // wide maps (P <= 64): per first-level group, 1 when it needs the LDS tree
};

constexpr uint32_t kByteLdsRow = 260;  // row stride of the LDS byte table
constexpr uint32_t kMaxChunk = 32768;  // chunk maps pack a count < 2^16 beside the end state

constexpr int kCoverRounds = 3;         // coverage rounds before every incomplete chunk is walked again
constexpr uint32_t kSplitMax = 2048;    // most chunks of a round walked again in sub-chunks
constexpr uint32_t kSplitTable = 8192;  // largest (Q+1) x (A+1) table for the sub-chunk walk

constexpr uint32_t kLookMax = 4096;     // longest lookback window
constexpr uint32_t kLookCap = 64;       // largest lookback set walked as a selection
constexpr uint32_t kLookStates = 16384; // lookback sets need Q + 1 <= this

// chunking, map width, group, tile and workspace carving of one text under options o
parem_status plan_chunks(const DeviceDfa &d, uint64_t len, const parem_options &o, bool keep, PlainPlan *p,
                         bool wide_segs = false);
parem_status plan_plain(const DeviceDfa &d, uint64_t len, PlainPlan *p);
parem_status launch_plain(const DeviceDfa &d, const PlainPlan &p, const uint8_t *d_text,
                          void *d_ws, hipStream_t stream, parem_result *d_out,
                          hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);
parem_status plan_boundary(const DeviceDfa &d, uint64_t len, uint32_t L, PlainPlan *p);
parem_status launch_boundary(const DeviceDfa &d, const PlainPlan &p, const uint8_t *d_text, uint32_t *d_states,
                             void *d_ws, hipStream_t stream);
parem_status launch_boundary_into(const DeviceDfa &d, const PlainPlan &p, const uint8_t *d_text, uint32_t *d_states,
                                  uint8_t *ws, hipStream_t stream, parem_result *d_out);
parem_status plan_learned(const DeviceDfa &d, const Proposal &pr, uint64_t len, uint32_t m, const parem_options &o,
                          PlainPlan *p);
parem_status launch_learned(const DeviceDfa &d, const Proposal &pr, const PlainPlan &p, const uint8_t *d_text,
                            void *d_ws, hipStream_t stream, parem_result *d_out, hipEvent_t ev_begin,
                            hipEvent_t ev_end);

}  // namespace parem

struct parem_dfa {
    parem::DeviceDfa dev;
};

struct parem_proposal_s : parem::Proposal {};

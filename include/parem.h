/*
 * parem.h - C interface of the MI355X (gfx950) speculative chunked DFA walk.
 *
 * Method: PaREM (Memeti & Pllana, "PaREM: A Novel Approach for Parallel
 * Regular Expression Matching", CSE 2014), Section II-B and Algorithm 1: the
 * input is decomposed into chunks; each chunk is walked only from the states
 * that have an incoming transition on the symbol just before the chunk
 * (R = S intersect L, with S = every state for a total table); the resulting
 * per-chunk state maps are joined into the run of the whole input.
 *
 * The result equals the sequential DFA run of Section II-A exactly: the
 * state reached after the last symbol, whether it is final, and the number
 * of steps whose destination state is final (the `found` tally of
 * Algorithm 1 along the connected route; the start state is not counted).
 *
 * Conventions for every call:
 *  - Plain pointers and sizes only. "Host" pointers are ordinary CPU memory;
 *    "device" pointers are HIP device memory of the current device.
 *  - Nothing is thrown across this interface: every call returns a
 *    parem_status; on failure outputs are left unspecified.
 *  - Handles are immutable after parem_compile; calls that pass their own
 *    workspace may run concurrently on different streams with one handle.
 *  - Streams are passed as `void*` holding a hipStream_t (NULL = the null
 *    stream of the current device).
 */
#ifndef PAREM_H
#define PAREM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct parem_dfa *parem_handle;
typedef struct parem_proposal_s *parem_proposal;
typedef struct parem_batch_s *parem_batch;

typedef enum {
    PAREM_OK = 0,
    PAREM_EINVAL = -1,      /* a null pointer, a zero size, a bad option */
    PAREM_ENOMEM = -2,      /* host or device allocation failed          */
    PAREM_EDEVICE = -3,     /* a HIP runtime call failed                  */
    PAREM_ESYMBOL = -4,     /* a text byte is not in the alphabet         */
    PAREM_ESTATE = -5,      /* a table entry / start / final id >= Q      */
    PAREM_EUNSUPPORTED = -6,/* sizes or options the library does not take */
    PAREM_ESYNTAX = -7      /* a regular expression does not parse        */
} parem_status;

/* Table layouts the compile step may choose (parem_options.layout). */
enum {
    PAREM_LAYOUT_AUTO = 0,
    PAREM_LAYOUT_BYTE_LDS = 1,   /* (Q+1) x 256 byte-indexed table in LDS       */
    PAREM_LAYOUT_BYTE_GLOBAL = 2,/* same table read through L2 (large tables)   */
    PAREM_LAYOUT_KGRAM_LDS = 3,  /* k-symbol stride table in LDS (small alphabets) */
    PAREM_LAYOUT_HOT_LDS = 4,    /* rows of the most visited states in LDS, the
                                    others read through L2 (up to 16383 states) */
    PAREM_LAYOUT_CLASS_LDS = 5,  /* (Q+1) x (A+1) table indexed by column, plus the
                                    byte-to-column map, in LDS (up to 48 KiB) */
    PAREM_LAYOUT_SPARSE_LDS = 6  /* sparse rows in LDS: per state a default next
                                    state and its exceptions (columns with another
                                    next state), the rows displaced into one vector
                                    of 4-byte slots: one slot per exception and one
                                    per state, at most 24512 slots (96 KiB). AUTO
                                    takes it when no dense LDS table fits and the
                                    slots fit; asked for on another table, the
                                    compile falls back as AUTO would. Batches walk
                                    such a handle's byte table through L2. */
};

/* Speculation policy (parem_options.policy). */
enum {
    PAREM_POLICY_PAREM = 0,     /* chunk c is walked from R_c = S intersect L
                                   (Algorithm 1, Section II-B)                 */
    PAREM_POLICY_ENUMERATE = 1  /* every state for every chunk after the first:
                                   the Enumeration approach the paper compares
                                   against (Section II-C counts its runs,
                                   Section IV-A measures it). Total tables
                                   only; not with lookback.                   */
};

/* Final state of a run that met an undefined transition of a partial table
 * (parem_options.partial), and of a text with a byte outside the alphabet. */
#define PAREM_DEAD_STATE 0xFFFFFFFEu
#define PAREM_INVALID_STATE 0xFFFFFFFFu

typedef struct {
    uint32_t chunk_len;   /* bytes per chunk, multiple of 64; 0 = automatic     */
    uint32_t layout;      /* PAREM_LAYOUT_*; AUTO lets the compile step choose  */
    uint32_t group;       /* speculated states walked in lockstep per lane; 0 = auto */
    uint32_t policy;      /* PAREM_POLICY_*                                      */
    uint32_t tile;        /* bytes of each chunk staged per load round: 64 or 128; 0 = auto */
    uint32_t no_merge;    /* 1: every speculated run walks its whole chunk, as the
                             paper's Algorithm 1 does; 0 (default): runs that
                             reach the same state are merged (identical results) */
    uint32_t lookback;    /* 0 (default): chunk c is walked from R_c, the image of
                             the column of the byte before it (Algorithm 1).
                             K > 0: from the image of every state under the K
                             bytes before the chunk (K capped at the chunk's
                             offset), a subset of R_c that still holds the true
                             entry state, so results are identical; chunks
                             whose image has more than 64 states use R_c (32
                             for a sparse-layout handle whose rows share one
                             default and whose alphabet is every byte, with
                             K <= 16: its sets are read from the slot image).
                             At most 4096; ignored when Q >= 16384. Not with
                             partial tables or the Enumeration policy.       */
    uint32_t partial;     /* 1: the table is a partial DFA (Section II-B): an
                             entry equal to the all-ones value of its width
                             (0xFF, 0xFFFF, 0xFFFFFFFF) is an undefined
                             transition. A run that meets one dies: the match
                             reports final_state PAREM_DEAD_STATE, accept 0,
                             and the count of final destinations before it.
                             Chunk c is then walked only from S intersect L:
                             the states of L (destinations on the byte before
                             the chunk) that have a transition on the chunk's
                             first byte. Needs num_states <= 16381; not with
                             lookback, the Enumeration policy, proposals or
                             batches. 0: every entry must be a state.        */
} parem_options;

typedef struct {
    uint32_t final_state;  /* state after the last byte (start state if len == 0);
                              PAREM_DEAD_STATE after an undefined transition,
                              PAREM_INVALID_STATE after a byte outside the
                              alphabet (async calls)                           */
    uint32_t accept;       /* 1 iff final_state is final                           */
    uint64_t count;        /* number of steps whose destination state is final    */
    uint64_t chunks;       /* chunks the text was split into                       */
    uint64_t spec_runs;    /* speculated (chunk, state) walks started              */
    uint64_t rerun_chunks; /* chunks walked again because their true entry state
                              was not speculated (always 0 for the plain set)     */
} parem_result;

/*
 * Build a handle from a total DFA (Section II-A: Q, Sigma, delta, q0, F).
 *  table        host, row-major [num_states][alphabet_size]; entry (q, j) is
 *               delta(q, alphabet[j]); entry_bytes is 1, 2 or 4 (unsigned).
 *               Every entry must be < num_states (else PAREM_ESTATE): the
 *               table is total (the S set of Algorithm 1 is then Q), unless
 *               opt->partial allows undefined entries (all-ones values).
 *  alphabet     host, alphabet_size distinct byte values (1..256); column j
 *               of the table is the byte alphabet[j]. Bytes not listed are
 *               invalid in texts (PAREM_ESYMBOL at match time).
 *  start        q0 < num_states.
 *  accepting    host, num_accepting state ids (duplicates allowed) of F.
 *  opt          NULL for defaults.
 *  out          receives the handle; owned by the caller, release with
 *               parem_free. All inputs are copied; the caller keeps them.
 * The compile step precomputes, per symbol, the speculated set of a chunk
 * that follows that symbol (the image of the symbol's column, the L set of
 * Algorithm 1) and uploads the chosen table layout to the current device.
 * Limits: 1 <= num_states <= 32767.
 */
parem_status parem_compile(const void *table, int entry_bytes, uint32_t num_states,
                           const uint8_t *alphabet, uint32_t alphabet_size, uint32_t start,
                           const uint32_t *accepting, uint32_t num_accepting,
                           const parem_options *opt, parem_handle *out);

/*
 * Regular-expression front-end (Section III). A pattern of the operators of
 * Table III - concatenation ab, Kleene star a*, union a|b, positive closure
 * a+, range [x..y] (bytes x to y in code order; x-y and several items per
 * bracket are accepted too), optionality a?, groups (...) - is parsed into a
 * syntax tree, turned into an automaton with empty moves by the
 * McNaughton-Yamada-Thompson construction, freed of its empty moves, and
 * determinised by the subset construction over the given alphabet (states
 * numbered in breadth-first order of discovery; the start state is 0).
 * Outside brackets ( ) [ ] | * + ? \ are operators and \x is the byte x;
 * every other byte stands for itself; an empty branch is the empty word.
 *  mode PAREM_RE_ANCHORED: the automaton of the expression itself; a step
 *       counts when the text read so far is in its language, and the match
 *       accepts when the whole text is.
 *  mode PAREM_RE_SEARCH: the automaton of Sigma* followed by the expression
 *       (Sigma = the alphabet); a step counts when some match of the
 *       expression ends at that byte - e.g. "parallel" over p,a,r,e,l gives
 *       the automaton of Table I.
 *  partial  1: no dead state; transitions into the empty set are undefined
 *       (a partial table, see parem_options.partial).
 * parem_regex_dfa writes the number of states to *num_states and, when the
 * pointers are not NULL, the table [states][alphabet_size] (u32; 0xFFFFFFFF
 * for undefined transitions; table_cap entries available) and one final
 * flag per state (final_cap bytes available). Host code only: no device is
 * used. PAREM_ESYNTAX for a malformed pattern, PAREM_EUNSUPPORTED beyond
 * 32767 states (16381 for partial tables), PAREM_EINVAL for too small
 * buffers or a repeated alphabet byte.
 * parem_compile_regex builds that automaton and compiles it with
 * parem_compile (opt->partial selects the partial form); bytes of the
 * pattern outside the alphabet can never match.
 */
#define PAREM_RE_ANCHORED 0u
#define PAREM_RE_SEARCH 1u
parem_status parem_regex_dfa(const char *pattern, uint64_t pattern_len, const uint8_t *alphabet,
                             uint32_t alphabet_size, uint32_t mode, uint32_t partial, uint32_t *num_states,
                             uint32_t *table, uint64_t table_cap, uint8_t *final_flags, uint64_t final_cap);
parem_status parem_compile_regex(const char *pattern, uint64_t pattern_len, const uint8_t *alphabet,
                                 uint32_t alphabet_size, uint32_t mode, const parem_options *opt,
                                 parem_handle *out);

/* Release a handle and its device memory. NULL is accepted. */
void parem_free(parem_handle h);

/* Text of a status code (static storage). */
const char *parem_strerror(parem_status s);

/* Layout and sizes the compile step chose, for logs and the autotuner.
 * Any output pointer may be NULL. */
parem_status parem_describe(parem_handle h, uint32_t *layout, uint32_t *max_spec,
                            uint32_t *lds_bytes, uint32_t *kgram);

/*
 * Device workspace (bytes) that parem_match_async needs for a text of `len`
 * bytes with this handle and its options.
 */
parem_status parem_workspace_size(parem_handle h, uint64_t len, uint64_t *bytes);

/*
 * Enqueue one match on `stream` and return at once.
 *  d_text       device, len bytes (any alignment); read only.
 *  d_workspace  device, at least parem_workspace_size bytes; the call owns
 *               it until the stream reaches the end of the match.
 *  d_out        device, one parem_result written when the match completes.
 *               A byte outside the alphabet yields final_state = 0xFFFFFFFF
 *               and accept = 0 in *d_out (the status is then known only
 *               after the stream is synchronised; parem_match maps it to
 *               PAREM_ESYMBOL).
 */
parem_status parem_match_async(parem_handle h, const uint8_t *d_text, uint64_t len,
                               void *d_workspace, uint64_t workspace_bytes, void *stream,
                               parem_result *d_out);

/*
 * parem_match_async plus two caller-owned hipEvent_t (passed as void*)
 * recorded on `stream` right before and right after the walk kernel, the
 * dominant kernel of a match, so that it can be timed alone. Either event
 * may be NULL. Same arguments, ownership and errors as parem_match_async.
 */
parem_status parem_match_async_timed(parem_handle h, const uint8_t *d_text, uint64_t len,
                                     void *d_workspace, uint64_t workspace_bytes, void *stream,
                                     parem_result *d_out, void *ev_walk_begin, void *ev_walk_end);

/*
 * parem_match_async without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The workspace is a file-scope device
 * array of parem_noalloc_scratch_bytes() bytes (64 MiB) that every GPU the
 * library runs on holds until the process ends; the call allocates no
 * device memory. Texts whose workspace (parem_workspace_size) exceeds it get
 * PAREM_EUNSUPPORTED (e.g. the 35-state DNA automaton needs about 10 MiB for
 * 1 GiB of text at the default chunk length). Nothing in the array needs to
 * start at zero. All calls on one GPU share its array: calls that overlap
 * on one GPU (other streams, or other host threads) race and give undefined
 * results; serialise them. The current device must be the handle's device
 * (PAREM_EINVAL otherwise). Same text, result and error conventions as
 * parem_match_async.
 */
parem_status parem_match_async_noalloc(parem_handle h, const uint8_t *d_text, uint64_t len, void *stream,
                                       parem_result *d_out);
uint64_t parem_noalloc_scratch_bytes(void);

/*
 * Synchronous match. `text` may be host or device memory (detected with
 * hipPointerGetAttributes); host text is staged through pinned memory. The
 * workspace is allocated and freed inside the call. Returns PAREM_ESYMBOL if
 * a byte is not in the alphabet.
 */
parem_status parem_match(parem_handle h, const uint8_t *text, uint64_t len, parem_result *out);

/*
 * States at chunk boundaries: the true state of the run after the first
 * c * chunk_len bytes, for c = 0 .. ceil(len / chunk_len) - 1 (the entry
 * state of every chunk; Section II-B: chunk c is entered in chunk c-1's
 * exit). Computed with the plain speculative walk, an up-sweep composition
 * that keeps every level, and a down-sweep that hands each map its entry.
 *  d_states     device, u32 per chunk (0xFFFFFFFF after a byte outside the
 *               alphabet).
 *  d_workspace  device, parem_boundary_workspace_size bytes.
 */
parem_status parem_boundary_workspace_size(parem_handle h, uint64_t len, uint32_t chunk_len, uint64_t *bytes);
parem_status parem_boundary_states(parem_handle h, const uint8_t *d_text, uint64_t len, uint32_t chunk_len,
                                   uint32_t *d_states, void *d_workspace, uint64_t workspace_bytes,
                                   void *stream);

/*
 * Match positions: the offset (0-based) of every byte whose step enters a
 * final state, ascending - the steps the count counts (Algorithm 1's `found`
 * tally along the connected route; for a search automaton such as Sigma*.P,
 * the last byte of every occurrence). After the walk and composition of a
 * plain match, a down-sweep hands every chunk its true entry state (chunk c
 * is entered in chunk c-1's exit, Section II-B); the chunk's count on that
 * route comes from its map, an exclusive scan of the counts gives each
 * chunk's first output slot, and each chunk with matches is walked once more
 * from its entry state alone, writing its offsets.
 *  d_positions  device, cap u64 slots; the first min(cap, count) offsets are
 *               written (cap may be 0: count only; d_positions may then be
 *               NULL).
 *  d_out        device parem_result of the match (count = number of
 *               positions). After a byte outside the alphabet the result is
 *               invalid (final_state PAREM_INVALID_STATE) and the positions
 *               are unspecified; a partial table's run that died has no
 *               positions after its death.
 *  d_workspace  device, parem_positions_workspace_size bytes; owned by the
 *               call until the stream reaches its end.
 * Chunks of the handle's chunk_len, or (0) about len / 2^19 bytes (256 to
 * 4096), so that the second walk, one lane per chunk, stays short.
 */
parem_status parem_positions_workspace_size(parem_handle h, uint64_t len, uint64_t *bytes);
parem_status parem_match_positions_async(parem_handle h, const uint8_t *d_text, uint64_t len, uint64_t *d_positions,
                                         uint64_t cap, void *d_workspace, uint64_t workspace_bytes, void *stream,
                                         parem_result *d_out);

/*
 * Learned speculation proposal (not in the paper). A small network scores
 * the states at a chunk boundary from the 32 bytes before it:
 * 16-d embedding per byte (bytes before the text start embed as zero) ->
 * 512 -> 256 (GELU) -> 256 (GELU) -> one logit per state. Parameters are one
 * flat float vector, in this order: emb[256][16], W1[256][512], b1[256],
 * W2[256][256], b2[256], W3[Q][256], b3[Q]; nparams must equal
 * 4096 + 131328 + 65792 + 257 * Q. Layers run as bf16 MFMA products with
 * fp32 accumulation; the fp32 master copy is updated by AdamW
 * (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay).
 *
 * parem_proposal_create   copies the host params; the proposal keeps a
 *                         pointer to h (free the proposal first).
 * parem_proposal_train_step
 *                         one AdamW step on the mean masked softmax
 *                         cross-entropy of `batch` boundaries: d_positions
 *                         (u64, device) are byte offsets into d_text, and
 *                         d_labels (u32, device) the true states there. Only
 *                         the states of the boundary's speculated set (the
 *                         image of the column of the byte before it) take
 *                         part in the softmax. A row whose label is not one
 *                         of them (e.g. 0xffffffff, the boundary state after
 *                         a byte outside the alphabet) or whose position is
 *                         beyond len takes no part: zero gradient, no loss
 *                         (the mean still divides by batch). lr = 0 and
 *                         weight_decay = 0 compute the gradient without
 *                         updating. d_loss (device float, may be NULL)
 *                         receives the mean loss.
 * parem_proposal_params   copies the fp32 weights and the last gradient
 *                         (either pointer may be NULL) to the host.
 * parem_proposal_logits   logits [batch][Q] (device fp32) at d_positions
 *                         (u64, device, byte offsets into the len-byte
 *                         d_text; a position beyond len scores an all-pad
 *                         window and reads no text).
 * parem_proposal_apply_grad
 *                         one AdamW step of the fp32 master weights (and
 *                         their bf16 copy) with the caller's gradient d_grad
 *                         (device, nparams floats, the flat parameter order
 *                         above), e.g. a gradient summed over several
 *                         devices. Shares the step counter and moments with
 *                         parem_proposal_train_step. Bias corrections
 *                         1 - beta^t are formed in double precision.
 */
parem_status parem_proposal_create(parem_handle h, const float *params, uint64_t nparams, parem_proposal *out);
void parem_proposal_free(parem_proposal p);
parem_status parem_proposal_params(parem_proposal p, float *params_out, float *grad_out, uint64_t nparams);
parem_status parem_proposal_train_step(parem_proposal p, const uint8_t *d_text, uint64_t len,
                                       const uint64_t *d_positions, const uint32_t *d_labels, uint32_t batch,
                                       float lr, float weight_decay, void *stream, float *d_loss);
parem_status parem_proposal_logits(parem_proposal p, const uint8_t *d_text, uint64_t len,
                                   const uint64_t *d_positions, uint32_t batch, float *d_logits, void *stream);
parem_status parem_proposal_apply_grad(parem_proposal p, const float *d_grad, uint64_t nparams, float lr,
                                       float weight_decay, void *stream);

/*
 * The selection learned speculation walks: for each chunk c of chunk_len
 * bytes, the positions (within the chunk's speculated list, which is sorted
 * by state id) of its m best-scored states, ascending, in d_sel[c * m ..];
 * d_nsel[c] = min(m, |R_c|). Chunk 0 selects {q0}. Ties: the lower state id.
 * Workspace: parem_proposal_select_size bytes.
 */
parem_status parem_proposal_select_size(parem_proposal p, uint64_t len, uint32_t chunk_len, uint64_t *bytes);
parem_status parem_proposal_select(parem_proposal p, const uint8_t *d_text, uint64_t len, uint32_t chunk_len,
                                   uint32_t m, uint16_t *d_sel, uint8_t *d_nsel, void *d_workspace,
                                   uint64_t workspace_bytes, void *stream);

/*
 * Match with learned speculation: every chunk c >= 1 walks only the m states
 * of its speculated set R_c that the proposal scores highest (ties: lower
 * state id; all of R_c when |R_c| <= m). A chunk whose entry states are not
 * all covered (some end state of its predecessor's walks was not walked
 * here) is walked again from all of R_c, which holds every possible entry;
 * this repeats until every chunk is covered, so the result is the sequential
 * run's, exactly. rerun_chunks counts the chunks walked again. 1 <= m <= 16.
 * Workspace from parem_learned_workspace_size.
 */
parem_status parem_learned_workspace_size(parem_handle h, parem_proposal p, uint64_t len, uint64_t *bytes);
parem_status parem_match_learned_async(parem_handle h, parem_proposal p, uint32_t m, const uint8_t *d_text,
                                       uint64_t len, void *d_workspace, uint64_t workspace_bytes, void *stream,
                                       parem_result *d_out, void *ev_walk_begin, void *ev_walk_end);

/*
 * Batched matching of many (DFA, text) pairs (each pair is Algorithm 1 on its
 * own text, as above). The plan fixes, per pair, the handle, the text length
 * and the options (chunk_len, group, tile, no_merge; the layout is the
 * handle's); every run then matches a new set of texts of those lengths.
 *
 * Execution: the chunks of all pairs are cut into work items of 256 chunks;
 * one persistent walk kernel per (table layout, group, tile) combination
 * takes items from a queue in descending cost order, staging each pair's
 * table in LDS when its layout does; then one launch per composition level
 * joins the chunk maps of every pair still holding more than one map. The
 * launches are enqueued without host synchronisation, so a run can be
 * captured in a HIP graph: with use_graph = 1 the first run on a plan
 * captures and instantiates the graph and every run replays it.
 *
 * parem_batch_create   dfas[n], lens[n] (bytes of each pair's text), opts
 *                      (n entries, or NULL for each handle's own options).
 *                      props (n entries, or NULL) and m: pair i with a
 *                      non-null props[i] (a proposal of dfas[i]) is matched
 *                      with learned speculation, top-m[i] states per chunk
 *                      (1..16), as parem_match_learned_async does; these
 *                      pairs run one after another on a branch of their own.
 *                      Allocates the plan's device memory (workspace for
 *                      every pair). Pairs with lens[i] == 0 are allowed.
 *                      The handles and proposals must outlive the plan.
 *                      A handle with the sparse layout is walked with
 *                      its byte table through L2 (no batch kernel stages
 *                      the sparse slots).
 * parem_batch_run      d_texts: host array of n device pointers, each
 *                      16-byte aligned (PAREM_EINVAL otherwise), holding
 *                      lens[i] bytes. d_out: device array of n results.
 *                      Asynchronous on `stream`; the texts must stay valid
 *                      until the stream reaches the end of the run. Calls on
 *                      one plan must not overlap (they share its workspace).
 *                      A text byte outside its pair's alphabet gives that
 *                      pair final_state 0xffffffff, accept 0, count 0 (the
 *                      other pairs are unaffected). The graph reads the
 *                      texts of plain pairs through a pointer array, so it
 *                      is replayed for any texts; learned pairs take their
 *                      text pointers as launch arguments, so new pointers
 *                      for them make the run capture a new graph.
 * parem_batch_describe plan statistics (any pointer may be NULL).
 * parem_match_batch    create + run (graph) + synchronize + free; on a byte
 *                      outside an alphabet returns PAREM_ESYMBOL after
 *                      writing every result.
 */
typedef struct {
    uint32_t pairs;
    uint32_t walk_launches;  /* persistent walk kernels (layout x group x tile)   */
    uint64_t walk_items;     /* work items of 256 chunks                          */
    uint32_t levels;         /* composition launches                              */
    uint32_t graph_nodes;    /* nodes of the captured graph (0 before capture)    */
    uint32_t learned_pairs;  /* pairs matched with learned speculation             */
    uint64_t chunks;         /* chunks over all pairs                             */
    uint64_t text_bytes;     /* bytes over all pairs                              */
    uint64_t workspace_bytes;
} parem_batch_info;

parem_status parem_batch_create(const parem_handle *dfas, const uint64_t *lens, uint32_t n,
                                const parem_options *opts, const parem_proposal *props, const uint32_t *m,
                                parem_batch *out);
parem_status parem_batch_run(parem_batch b, const uint8_t *const *d_texts, void *stream, parem_result *d_out,
                             int use_graph);
parem_status parem_batch_describe(parem_batch b, parem_batch_info *info);
void parem_batch_free(parem_batch b);
parem_status parem_match_batch(const parem_handle *dfas, const uint8_t *const *d_texts, const uint64_t *lens,
                               uint32_t n, void *stream, parem_result *d_out);

/*
 * Autotuner measurement: for each candidate option set (chunk_len, group,
 * tile, no_merge; chunk_len 0 = the batch default), plans a batch of up to
 * `copies` pairs that all match d_sample (sample_len bytes, device, 16-byte
 * aligned) with handle h (fewer copies when their workspace would pass
 * 4 GiB), times `reps` graph replays after one warm-up run, and writes the
 * milliseconds per copy (replay time / copies) to ms_out[ncand] (host).
 * *best receives the index of the fastest candidate. Candidates that the
 * handle cannot run (e.g. group 2, a chunk length above the maximum) get
 * ms_out = -1; PAREM_EUNSUPPORTED when none can.
 */
parem_status parem_tune(parem_handle h, const uint8_t *d_sample, uint64_t sample_len, uint32_t copies,
                        const parem_options *cands, uint32_t ncand, uint32_t reps, void *stream, float *ms_out,
                        uint32_t *best);

#ifdef __cplusplus
}
#endif

#endif /* PAREM_H */

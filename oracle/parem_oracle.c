/*
 * CPU oracle for the speculative chunked DFA walk (PaREM, Memeti & Pllana).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it. It shares no code, header, table or helper
 * with the HIP library.
 *
 * Deliberately plain, single-threaded and slow. Tables are given row-major
 * as table[q * A + j] = delta(q, alphabet[j]) (uint32 entries). With the
 * flag ORC_PARTIAL an entry equal to ORC_UNDEF (all ones) is an undefined
 * transition (a partial DFA, Section II-B: such a state is not in the S set
 * of a symbol); a run that meets one dies: it stays in the absorbing result
 * ORC_DEAD (not final, counts nothing more). Without the flag every entry
 * must be a state (a total DFA).
 * Status codes: 0 ok, -1 bad argument, -4 a text byte outside the alphabet
 * (anywhere in the text, also after the run died), -5 a table entry or start
 * state outside [0, Q), -6 internal inconsistency (a chunk route that does
 * not connect; impossible by the method's reasoning).
 *
 * Functions:
 *   oracle_walk       the sequential DFA run (Section II-A, "Background";
 *                     Section II-B: one step per input symbol from q0,
 *                     time linear in the input length). Also counts the
 *                     positions whose destination state is final, the quantity
 *                     Algorithm 1 tallies in `found`.
 *   oracle_states_at  the same run, reporting the state after given prefix
 *                     lengths (the true entry state of a chunk starting there).
 *   oracle_parem      Algorithm 1 step by step: domain decomposition into p
 *                     slices, the S and L sets, R = S intersect L, one walk
 *                     per r in R with its visited states, then the join of
 *                     the sub-routes (Section II-B, Algorithm 1, and the
 *                     worked example of Section II-C, Tables I and II).
 *                     Policy ORC_POLICY_ENUMERATE speculates every state
 *                     for every slice after the first (the Enumeration
 *                     approach Section IV-A compares against; Section II-C
 *                     counts its runs on the example).
 *   oracle_positions  the sequential run again, listing the offset of every
 *                     symbol whose step enters a final state (the positions
 *                     the `found` tally counts; the matches' end offsets).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ESYMBOL (-4)
#define ORC_ESTATE (-5)
#define ORC_EJOIN (-6)

#define ORC_PARTIAL 1u            /* flags: undefined transitions allowed */
#define ORC_UNDEF 0xffffffffu     /* table entry of an undefined transition */
#define ORC_DEAD 0xfffffffeu      /* result of a run that met one */
#define ORC_POLICY_PAREM 0u       /* R = S intersect L (Algorithm 1) */
#define ORC_POLICY_ENUMERATE 1u   /* R = every state */

/* Column of each byte value: the j with alphabet[j] == byte, or -1. */
static int build_columns(const uint8_t *alphabet, uint32_t A, int col[256])
{
    for (int b = 0; b < 256; ++b)
        col[b] = -1;
    for (uint32_t j = 0; j < A; ++j) {
        if (col[alphabet[j]] != -1)
            return ORC_EINVAL; /* the same byte named twice */
        col[alphabet[j]] = (int)j;
    }
    return ORC_OK;
}

static int check_dfa(const uint32_t *table, uint32_t Q, const uint8_t *alphabet,
                     uint32_t A, uint32_t start, uint32_t flags, int col[256])
{
    if (!table || !alphabet || Q == 0 || A == 0 || A > 256 || (flags & ~ORC_PARTIAL))
        return ORC_EINVAL;
    int rc = build_columns(alphabet, A, col);
    if (rc)
        return rc;
    if (start >= Q)
        return ORC_ESTATE;
    for (uint64_t k = 0; k < (uint64_t)Q * A; ++k)
        if (table[k] >= Q && !((flags & ORC_PARTIAL) && table[k] == ORC_UNDEF))
            return ORC_ESTATE;
    return ORC_OK;
}

/* One step of a run: the next state, or ORC_DEAD on an undefined transition
 * (and from ORC_DEAD). */
static uint32_t step(const uint32_t *table, uint32_t A, uint32_t q, int j)
{
    if (q == ORC_DEAD)
        return ORC_DEAD;
    uint32_t nx = table[(uint64_t)q * A + (uint32_t)j];
    return nx == ORC_UNDEF ? ORC_DEAD : nx;
}

/* First byte outside the alphabet at or after offset i, or len. */
static uint64_t first_invalid(const int col[256], const uint8_t *text, uint64_t i, uint64_t len)
{
    for (; i < len; ++i)
        if (col[text[i]] < 0)
            return i;
    return len;
}

/*
 * Sequential run: q = q0; for every symbol q = delta(q, symbol); count the
 * steps whose destination is final. The start state itself is never counted.
 * On a byte outside the alphabet returns -4 and stores its offset in *bad_pos.
 * A partial table's run that meets an undefined transition ends in ORC_DEAD.
 */
int oracle_walk(const uint32_t *table, uint32_t Q, const uint8_t *alphabet, uint32_t A,
                uint32_t start, uint32_t flags, const uint8_t *is_final, const uint8_t *text,
                uint64_t len, uint32_t *out_final, uint64_t *out_count, uint64_t *bad_pos)
{
    int col[256];
    int rc = check_dfa(table, Q, alphabet, A, start, flags, col);
    if (rc)
        return rc;
    if (!is_final || (!text && len) || !out_final || !out_count)
        return ORC_EINVAL;
    uint32_t q = start;
    uint64_t count = 0;
    for (uint64_t i = 0; i < len; ++i) {
        int j = col[text[i]];
        if (j < 0) {
            if (bad_pos)
                *bad_pos = i;
            return ORC_ESYMBOL;
        }
        q = step(table, A, q, j);
        if (q == ORC_DEAD) {
            uint64_t bad = first_invalid(col, text, i + 1, len);
            if (bad < len) {
                if (bad_pos)
                    *bad_pos = bad;
                return ORC_ESYMBOL;
            }
            break;
        }
        if (is_final[q])
            ++count;
    }
    *out_final = q;
    *out_count = count;
    return ORC_OK;
}

/*
 * The sequential run again, recording the state after each prefix length in
 * `positions` (ascending, each <= len) and the count of final destinations up
 * to that point. positions[k] == 0 gives the start state and count 0; after
 * the run died the state is ORC_DEAD.
 */
int oracle_states_at(const uint32_t *table, uint32_t Q, const uint8_t *alphabet, uint32_t A,
                     uint32_t start, uint32_t flags, const uint8_t *is_final, const uint8_t *text,
                     uint64_t len, const uint64_t *positions, uint64_t npos, uint32_t *out_states,
                     uint64_t *out_counts)
{
    int col[256];
    int rc = check_dfa(table, Q, alphabet, A, start, flags, col);
    if (rc)
        return rc;
    if (!is_final || (!text && len) || (npos && (!positions || !out_states)))
        return ORC_EINVAL;
    uint32_t q = start;
    uint64_t count = 0;
    uint64_t i = 0;
    for (uint64_t k = 0; k < npos; ++k) {
        uint64_t stop = positions[k];
        if (stop > len || (k && stop < positions[k - 1]))
            return ORC_EINVAL;
        for (; i < stop; ++i) {
            int j = col[text[i]];
            if (j < 0)
                return ORC_ESYMBOL;
            q = step(table, A, q, j);
            if (q != ORC_DEAD && is_final[q])
                ++count;
        }
        out_states[k] = q;
        if (out_counts)
            out_counts[k] = count;
    }
    return ORC_OK;
}

/*
 * Offsets of the symbols whose step enters a final state, ascending: the
 * first min(cap, total) are stored in out_pos, the total in *total (equal to
 * oracle_walk's count). Errors as oracle_walk.
 */
int oracle_positions(const uint32_t *table, uint32_t Q, const uint8_t *alphabet, uint32_t A,
                     uint32_t start, uint32_t flags, const uint8_t *is_final, const uint8_t *text,
                     uint64_t len, uint64_t *out_pos, uint64_t cap, uint64_t *total, uint64_t *bad_pos)
{
    int col[256];
    int rc = check_dfa(table, Q, alphabet, A, start, flags, col);
    if (rc)
        return rc;
    if (!is_final || (!text && len) || !total || (cap && !out_pos))
        return ORC_EINVAL;
    uint64_t bad = first_invalid(col, text, 0, len);
    if (bad < len) {
        if (bad_pos)
            *bad_pos = bad;
        return ORC_ESYMBOL;
    }
    uint32_t q = start;
    uint64_t count = 0;
    for (uint64_t i = 0; i < len && q != ORC_DEAD; ++i) {
        q = step(table, A, q, col[text[i]]);
        if (q != ORC_DEAD && is_final[q]) {
            if (count < cap)
                out_pos[count] = i;
            ++count;
        }
    }
    *total = count;
    return ORC_OK;
}

/*
 * Algorithm 1 with p processing units, executed one unit after another.
 *
 * Readings of the printed algorithm:
 *  - slice c covers [floor(c*len/p), floor((c+1)*len/p)): the printed
 *    start/length drop len mod p trailing symbols, a balanced split does not;
 *  - L is built from the last symbol of the PREVIOUS slice, as the prose and
 *    the worked example (Table II, the yellow cells of Table I) do; the
 *    printed pseudocode names the slice's own last symbol;
 *  - slice 0 speculates {q0} only; an empty slice has the identity route;
 *  - `found` is kept per (slice, r) and only the counts on the connected
 *    route are summed (the printed counter is shared by all r);
 *  - partial tables: S holds the states with a transition on the slice's
 *    first symbol, L the destinations of the transitions on the symbol
 *    before it; a walk that meets an undefined transition ends in ORC_DEAD
 *    with the count it had. A route that is dead stays dead; a live route
 *    whose state is in L but not in S dies on the slice's first symbol.
 *
 * policy ORC_POLICY_PAREM: R = S intersect L (Algorithm 1);
 * ORC_POLICY_ENUMERATE: R = every state, for every slice after the first.
 *
 * Outputs: final state and count of the connected route; total number of
 * walks performed (sum of |R| over slices); for each slice its true entry
 * state (entries[c], ORC_DEAD once the route died) and |R| (rsize[c]) when
 * those pointers are non-NULL. With trace != NULL, every walk appends the
 * record
 *     slice, r, slice length, visited states...
 * (the I vector of Algorithm 1; ORC_DEAD after a death) while it fits in
 * trace_cap words; the number of words needed is stored in *trace_len.
 */
int oracle_parem(const uint32_t *table, uint32_t Q, const uint8_t *alphabet, uint32_t A,
                 uint32_t start, uint32_t flags, uint32_t policy, const uint8_t *is_final,
                 const uint8_t *text, uint64_t len, uint64_t p, uint32_t *out_final,
                 uint64_t *out_count, uint64_t *out_runs, uint32_t *entries, uint32_t *rsize,
                 uint32_t *trace, uint64_t trace_cap, uint64_t *trace_len)
{
    int col[256];
    int rc = check_dfa(table, Q, alphabet, A, start, flags, col);
    if (rc)
        return rc;
    if (!is_final || (!text && len) || p == 0 || !out_final || !out_count || policy > ORC_POLICY_ENUMERATE)
        return ORC_EINVAL;
    if (first_invalid(col, text, 0, len) < len)
        return ORC_ESYMBOL;

    uint8_t *in_S = (uint8_t *)malloc(Q);
    uint8_t *in_L = (uint8_t *)malloc(Q);
    /* per slice: the speculated states and, per state, (end, found) */
    uint32_t *run_end = (uint32_t *)malloc((size_t)Q * sizeof(uint32_t));
    uint64_t *run_found = (uint64_t *)malloc((size_t)Q * sizeof(uint64_t));
    uint8_t *in_R = (uint8_t *)malloc(Q);
    if (!in_S || !in_L || !run_end || !run_found || !in_R) {
        free(in_S); free(in_L); free(run_end); free(run_found); free(in_R);
        return ORC_EINVAL;
    }

    uint64_t runs = 0, tl = 0;
    uint32_t route_state = start; /* exit state of the connected route so far */
    uint64_t route_count = 0;
    rc = ORC_OK;

    for (uint64_t c = 0; c < p; ++c) {
        uint64_t b = (uint64_t)(((unsigned __int128)c * len) / p);
        uint64_t e = (uint64_t)(((unsigned __int128)(c + 1) * len) / p);
        uint64_t n = e - b;

        /* S: states with a transition on the slice's first symbol */
        memset(in_S, 1, Q);
        if (n > 0) {
            int j0 = col[text[b]];
            for (uint32_t q = 0; q < Q; ++q)
                if (table[(uint64_t)q * A + (uint32_t)j0] == ORC_UNDEF)
                    in_S[q] = 0;
        }
        /* possible initial states */
        memset(in_R, 0, Q);
        if (c == 0) {
            in_R[start] = 1;
        } else if (policy == ORC_POLICY_ENUMERATE) {
            memset(in_R, 1, Q);
        } else {
            /* L: destinations on the previous slice's last symbol */
            memset(in_L, 0, Q);
            if (b > 0) {
                int jl = col[text[b - 1]];
                for (uint32_t q = 0; q < Q; ++q) {
                    uint32_t nx = table[(uint64_t)q * A + (uint32_t)jl];
                    if (nx != ORC_UNDEF)
                        in_L[nx] = 1;
                }
            } else {
                in_L[start] = 1; /* no symbol read yet: only q0 is possible */
            }
            for (uint32_t q = 0; q < Q; ++q)
                in_R[q] = in_S[q] && in_L[q];
        }

        /* one walk per r in R */
        uint32_t rcount = 0;
        for (uint32_t r = 0; r < Q; ++r) {
            if (!in_R[r])
                continue;
            ++rcount;
            uint32_t s = r;
            uint64_t found = 0;
            int keep = trace && tl + 3 + n <= trace_cap;
            if (keep) {
                trace[tl] = (uint32_t)c;
                trace[tl + 1] = r;
                trace[tl + 2] = (uint32_t)n;
            }
            for (uint64_t i = 0; i < n; ++i) {
                s = step(table, A, s, col[text[b + i]]);
                if (s != ORC_DEAD && is_final[s])
                    ++found;
                if (keep)
                    trace[tl + 3 + i] = s;
            }
            tl += 3 + n;
            run_end[r] = s;
            run_found[r] = found;
        }
        runs += rcount;
        if (rsize)
            rsize[c] = rcount;

        /* join: the route enters this slice in the previous slice's exit */
        if (entries)
            entries[c] = route_state;
        if (route_state == ORC_DEAD)
            continue;
        if (!in_R[route_state]) {
            if (!in_S[route_state]) {
                route_state = ORC_DEAD; /* dies on the slice's first symbol */
                continue;
            }
            rc = ORC_EJOIN;
            break;
        }
        route_count += run_found[route_state];
        route_state = run_end[route_state];
    }

    free(in_S); free(in_L); free(run_end); free(run_found); free(in_R);
    if (rc)
        return rc;
    *out_final = route_state;
    *out_count = route_count;
    if (out_runs)
        *out_runs = runs;
    if (trace_len)
        *trace_len = tl;
    return ORC_OK;
}

/*
 * Run of a nondeterministic automaton with empty moves (the McNaughton-
 * Yamada-Thompson construction of Section III), simulated on sets of states:
 * the current set starts as the empty-move closure of `start`; each byte
 * moves every state of the set along its edges whose byte range holds the
 * byte, and the closure of the result is the next set. Nothing is
 * determinised. A step counts when the new set holds an accepting state;
 * *out_accept is whether the final set does, *out_empty whether the set
 * became empty (no continuation can match any more).
 *  edges: n_edges records (from, lo, hi, to): a move on bytes lo..hi;
 *  eps:   n_eps records (from, to): an empty move.
 * Bytes outside the alphabet give -4 (offset in *bad_pos).
 */
int oracle_nfa_walk(uint32_t n_states, uint32_t start, const uint8_t *accepting,
                    const uint32_t *edges, uint32_t n_edges, const uint32_t *eps, uint32_t n_eps,
                    const uint8_t *alphabet, uint32_t A, const uint8_t *text, uint64_t len,
                    uint8_t *out_accept, uint64_t *out_count, uint8_t *out_empty, uint64_t *bad_pos)
{
    int col[256];
    if (!accepting || n_states == 0 || start >= n_states || (n_edges && !edges) || (n_eps && !eps) ||
        !out_accept || !out_count || (!text && len) || !alphabet || A == 0 || A > 256)
        return ORC_EINVAL;
    if (build_columns(alphabet, A, col))
        return ORC_EINVAL;
    for (uint32_t k = 0; k < n_edges; ++k)
        if (edges[4 * k] >= n_states || edges[4 * k + 3] >= n_states || edges[4 * k + 1] > edges[4 * k + 2] ||
            edges[4 * k + 2] > 255)
            return ORC_EINVAL;
    for (uint32_t k = 0; k < n_eps; ++k)
        if (eps[2 * k] >= n_states || eps[2 * k + 1] >= n_states)
            return ORC_EINVAL;
    uint8_t *cur = (uint8_t *)calloc(n_states, 1);
    uint8_t *nxt = (uint8_t *)calloc(n_states, 1);
    uint32_t *stack = (uint32_t *)malloc((size_t)n_states * sizeof(uint32_t));
    if (!cur || !nxt || !stack) {
        free(cur); free(nxt); free(stack);
        return ORC_EINVAL;
    }
    /* closure of the marked set `s` in place (depth-first over empty moves) */
#define CLOSE(s)                                                              \
    do {                                                                      \
        uint32_t sp = 0;                                                      \
        for (uint32_t q = 0; q < n_states; ++q)                               \
            if (s[q])                                                         \
                stack[sp++] = q;                                              \
        while (sp) {                                                          \
            uint32_t q = stack[--sp];                                         \
            for (uint32_t k = 0; k < n_eps; ++k)                              \
                if (eps[2 * k] == q && !s[eps[2 * k + 1]]) {                  \
                    s[eps[2 * k + 1]] = 1;                                    \
                    stack[sp++] = eps[2 * k + 1];                             \
                }                                                             \
        }                                                                     \
    } while (0)
    cur[start] = 1;
    CLOSE(cur);
    uint64_t count = 0;
    int rc = ORC_OK;
    for (uint64_t i = 0; i < len; ++i) {
        if (col[text[i]] < 0) {
            if (bad_pos)
                *bad_pos = i;
            rc = ORC_ESYMBOL;
            break;
        }
        memset(nxt, 0, n_states);
        for (uint32_t k = 0; k < n_edges; ++k)
            if (cur[edges[4 * k]] && text[i] >= edges[4 * k + 1] && text[i] <= edges[4 * k + 2])
                nxt[edges[4 * k + 3]] = 1;
        CLOSE(nxt);
        uint8_t *t = cur;
        cur = nxt;
        nxt = t;
        int acc = 0;
        for (uint32_t q = 0; q < n_states && !acc; ++q)
            acc = cur[q] && accepting[q];
        count += (uint64_t)acc;
    }
#undef CLOSE
    if (rc == ORC_OK) {
        int acc = 0, any = 0;
        for (uint32_t q = 0; q < n_states; ++q) {
            acc |= cur[q] && accepting[q];
            any |= cur[q];
        }
        *out_accept = (uint8_t)acc;
        *out_count = count;
        if (out_empty)
            *out_empty = (uint8_t)!any;
    }
    free(cur); free(nxt); free(stack);
    return rc;
}

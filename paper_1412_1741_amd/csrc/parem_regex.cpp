// Regular-expression front-end (Section III): a pattern built from the
// operators of Table III (concatenation, Kleene star, union, positive
// closure, range [x..y], optionality, groups) is parsed into an abstract
// syntax tree, turned into an automaton with empty moves by the
// McNaughton-Yamada-Thompson construction, freed of its empty moves, and
// determinised by the subset construction into the transition table that
// parem_compile takes. Host code only.
#include <algorithm>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/parem.h"

namespace {

// ---------------------------------------------------------------------------
// syntax tree
// ---------------------------------------------------------------------------

struct Node {
    enum Kind { SET, EMPTY, CAT, ALT, STAR, PLUS, OPT } kind;
    uint64_t bytes[4] = {0, 0, 0, 0};  // SET: member bytes
    int a = -1, b = -1;                // operands
};

class Parser {
  public:
    Parser(const uint8_t *p, size_t n, std::vector<Node> &nodes) : p_(p), n_(n), nodes_(nodes) {}

    // root node index, or -1 on a syntax error
    int run() {
        const int r = alt();
        if (r < 0 || pos_ != n_) return -1;
        return r;
    }

  private:
    const uint8_t *p_;
    size_t n_, pos_ = 0;
    std::vector<Node> &nodes_;
    int depth_ = 0;

    static bool special(uint8_t c) { return std::strchr("()[]|*+?\\", c) != nullptr && c != 0; }
    bool more() const { return pos_ < n_; }
    uint8_t peek() const { return p_[pos_]; }

    int add(Node x) {
        nodes_.push_back(x);
        return (int)nodes_.size() - 1;
    }
    int pair(Node::Kind k, int a, int b) {
        Node x{k};
        x.a = a;
        x.b = b;
        return add(x);
    }

    // union := concat ('|' concat)*
    int alt() {
        if (++depth_ > 2000) return -1;  // nesting bound (recursion depth)
        int node = cat();
        while (node >= 0 && more() && peek() == '|') {
            ++pos_;
            const int r = cat();
            node = r < 0 ? -1 : pair(Node::ALT, node, r);
        }
        --depth_;
        return node;
    }

    // concat := repeat*   (none: the empty word)
    int cat() {
        int node = -1;
        bool any = false;
        while (more() && peek() != '|' && peek() != ')') {
            const int r = repeat();
            if (r < 0) return -1;
            node = any ? pair(Node::CAT, node, r) : r;
            any = true;
        }
        return any ? node : add(Node{Node::EMPTY});
    }

    // repeat := atom ('*' | '+' | '?')*
    int repeat() {
        int node = atom();
        while (node >= 0 && more() && (peek() == '*' || peek() == '+' || peek() == '?')) {
            const uint8_t op = p_[pos_++];
            node = pair(op == '*' ? Node::STAR : op == '+' ? Node::PLUS : Node::OPT, node, -1);
        }
        return node;
    }

    // one byte inside brackets (an escape takes the next byte as it is)
    bool bracket_byte(uint8_t &c) {
        if (!more()) return false;
        c = p_[pos_++];
        if (c == '\\') {
            if (!more()) return false;
            c = p_[pos_++];
            return true;
        }
        return c != ']';
    }

    int atom() {
        if (!more()) return -1;
        const uint8_t c = p_[pos_++];
        if (c == '(') {
            const int r = alt();
            if (r < 0 || !more() || p_[pos_++] != ')') return -1;
            return r;
        }
        if (c == '[') {
            Node x{Node::SET};
            if (!more() || peek() == ']') return -1;  // empty range
            while (true) {
                if (!more()) return -1;
                if (peek() == ']') break;
                uint8_t lo, hi;
                if (!bracket_byte(lo)) return -1;
                hi = lo;
                if (pos_ + 2 < n_ && p_[pos_] == '.' && p_[pos_ + 1] == '.' && p_[pos_ + 2] != ']') {
                    pos_ += 2;
                    if (!bracket_byte(hi)) return -1;
                } else if (pos_ + 1 < n_ && p_[pos_] == '-' && p_[pos_ + 1] != ']') {
                    pos_ += 1;
                    if (!bracket_byte(hi)) return -1;
                }
                if (hi < lo) return -1;
                for (uint32_t v = lo; v <= hi; ++v) x.bytes[v >> 6] |= 1ull << (v & 63);
            }
            ++pos_;  // ']'
            return add(x);
        }
        Node x{Node::SET};
        uint8_t v = c;
        if (c == '\\') {
            if (!more()) return -1;
            v = p_[pos_++];
        } else if (special(c)) {
            return -1;
        }
        x.bytes[v >> 6] |= 1ull << (v & 63);
        return add(x);
    }
};

// ---------------------------------------------------------------------------
// McNaughton-Yamada-Thompson construction
// ---------------------------------------------------------------------------

struct Move {
    uint8_t lo, hi;
    int to;
};

struct Nfa {
    std::vector<std::vector<Move>> moves;
    std::vector<std::vector<int>> eps;
    int start = 0, accept = 0;

    int state() {
        moves.emplace_back();
        eps.emplace_back();
        return (int)moves.size() - 1;
    }
};

struct Frag {
    int s, f;
};

// fragments are built bottom-up in node order (operands precede operators in
// `nodes`, so no recursion is needed)
bool thompson(const std::vector<Node> &nodes, Nfa &m, std::vector<Frag> &frag) {
    frag.assign(nodes.size(), Frag{-1, -1});
    for (size_t i = 0; i < nodes.size(); ++i) {
        const Node &x = nodes[i];
        Frag r{};
        switch (x.kind) {
            case Node::SET: {
                r = Frag{m.state(), m.state()};
                for (uint32_t v = 0; v < 256;) {
                    if (!((x.bytes[v >> 6] >> (v & 63)) & 1u)) {
                        ++v;
                        continue;
                    }
                    uint32_t w = v;
                    while (w + 1 < 256 && ((x.bytes[(w + 1) >> 6] >> ((w + 1) & 63)) & 1u)) ++w;
                    m.moves[r.s].push_back(Move{(uint8_t)v, (uint8_t)w, r.f});
                    v = w + 1;
                }
                break;
            }
            case Node::EMPTY:
                r = Frag{m.state(), m.state()};
                m.eps[r.s].push_back(r.f);
                break;
            case Node::CAT: {
                const Frag a = frag[x.a], b = frag[x.b];
                m.eps[a.f].push_back(b.s);
                r = Frag{a.s, b.f};
                break;
            }
            case Node::ALT: {
                const Frag a = frag[x.a], b = frag[x.b];
                r = Frag{m.state(), m.state()};
                m.eps[r.s].push_back(a.s);
                m.eps[r.s].push_back(b.s);
                m.eps[a.f].push_back(r.f);
                m.eps[b.f].push_back(r.f);
                break;
            }
            default: {
                const Frag a = frag[x.a];
                r = Frag{m.state(), m.state()};
                m.eps[r.s].push_back(a.s);
                if (x.kind != Node::PLUS) m.eps[r.s].push_back(r.f);   // zero occurrences
                if (x.kind != Node::OPT) m.eps[a.f].push_back(a.s);    // again
                m.eps[a.f].push_back(r.f);
                break;
            }
        }
        frag[i] = r;
    }
    return true;
}

// ---------------------------------------------------------------------------
// removal of empty moves: state s takes the moves of every state of its
// empty-move closure and accepts when the closure holds the accepting state
// ---------------------------------------------------------------------------

struct Plain {
    std::vector<std::vector<Move>> moves;
    std::vector<uint8_t> accepting;
    int start = 0;
};

Plain remove_empty(const Nfa &m) {
    const int n = (int)m.moves.size();
    Plain out;
    out.moves.resize(n);
    out.accepting.assign(n, 0);
    out.start = m.start;
    std::vector<int> mark(n, -1), stack;
    for (int s = 0; s < n; ++s) {
        stack.assign(1, s);
        mark[s] = s;
        while (!stack.empty()) {
            const int q = stack.back();
            stack.pop_back();
            for (const Move &mv : m.moves[q]) out.moves[s].push_back(mv);
            if (q == m.accept) out.accepting[s] = 1;
            for (int t : m.eps[q])
                if (mark[t] != s) {
                    mark[t] = s;
                    stack.push_back(t);
                }
        }
    }
    return out;
}

// ---------------------------------------------------------------------------
// subset construction over the alphabet's columns, states numbered in
// breadth-first order of discovery from {start}; the empty set is the dead
// state (or, for a partial table, no transition)
// ---------------------------------------------------------------------------

constexpr uint32_t kUndef = 0xffffffffu;

parem_status subset(const Plain &nf, const uint8_t *alphabet, uint32_t A, bool partial, uint32_t max_states,
                    std::vector<uint32_t> &table, std::vector<uint8_t> &final_flag) {
    const size_t n = nf.moves.size();
    const size_t words = (n + 63) / 64;
    using Set = std::vector<uint64_t>;
    std::unordered_map<std::string, uint32_t> id;
    std::deque<Set> sets;
    auto key = [&](const Set &s) { return std::string(reinterpret_cast<const char *>(s.data()), s.size() * 8); };
    auto add = [&](const Set &s, uint32_t &out) -> bool {
        const std::string k = key(s);
        auto it = id.find(k);
        if (it != id.end()) {
            out = it->second;
            return true;
        }
        if (sets.size() >= max_states) return false;
        out = (uint32_t)sets.size();
        id.emplace(k, out);
        sets.push_back(s);
        return true;
    };
    Set s0(words, 0);
    s0[nf.start >> 6] |= 1ull << (nf.start & 63);
    uint32_t tmp;
    add(s0, tmp);
    table.clear();
    final_flag.clear();
    Set nx(words);
    for (size_t k = 0; k < sets.size(); ++k) {
        const Set cur = sets[k];
        uint8_t fin = 0;
        for (size_t q = 0; q < n; ++q)
            if ((cur[q >> 6] >> (q & 63)) & 1u) fin |= nf.accepting[q];
        final_flag.push_back(fin);
        for (uint32_t j = 0; j < A; ++j) {
            const uint8_t x = alphabet[j];
            std::fill(nx.begin(), nx.end(), 0);
            bool any = false;
            for (size_t q = 0; q < n; ++q) {
                if (!((cur[q >> 6] >> (q & 63)) & 1u)) continue;
                for (const Move &mv : nf.moves[q])
                    if (x >= mv.lo && x <= mv.hi) {
                        nx[(size_t)mv.to >> 6] |= 1ull << (mv.to & 63);
                        any = true;
                    }
            }
            if (!any && partial) {
                table.push_back(kUndef);
                continue;
            }
            uint32_t t;
            if (!add(nx, t)) return PAREM_EUNSUPPORTED;
            table.push_back(t);
        }
    }
    return PAREM_OK;
}

parem_status regex_table(const char *pattern, uint64_t pattern_len, const uint8_t *alphabet, uint32_t A,
                         uint32_t mode, bool partial, uint32_t max_states, std::vector<uint32_t> &table,
                         std::vector<uint8_t> &final_flag) {
    if ((!pattern && pattern_len) || !alphabet || A == 0 || A > 256 || mode > PAREM_RE_SEARCH) return PAREM_EINVAL;
    bool seen[256] = {};
    for (uint32_t j = 0; j < A; ++j) {
        if (seen[alphabet[j]]) return PAREM_EINVAL;
        seen[alphabet[j]] = true;
    }
    std::vector<Node> nodes;
    Parser ps(reinterpret_cast<const uint8_t *>(pattern), (size_t)pattern_len, nodes);
    const int root = ps.run();
    if (root < 0) return PAREM_ESYNTAX;
    Nfa m;
    std::vector<Frag> frag;
    thompson(nodes, m, frag);
    m.start = frag[root].s;
    m.accept = frag[root].f;
    if (mode == PAREM_RE_SEARCH) {
        // Sigma* before the expression: a start state looping on every
        // alphabet byte, with an empty move into the expression
        const int loop = m.state();
        for (uint32_t j = 0; j < A; ++j) m.moves[loop].push_back(Move{alphabet[j], alphabet[j], loop});
        m.eps[loop].push_back(m.start);
        m.start = loop;
    }
    const Plain nf = remove_empty(m);
    return subset(nf, alphabet, A, partial, max_states, table, final_flag);
}

}  // namespace

extern "C" {

parem_status parem_regex_dfa(const char *pattern, uint64_t pattern_len, const uint8_t *alphabet,
                             uint32_t alphabet_size, uint32_t mode, uint32_t partial, uint32_t *num_states,
                             uint32_t *table, uint64_t table_cap, uint8_t *final_flags, uint64_t final_cap) {
    if (!num_states || partial > 1) return PAREM_EINVAL;
    try {
        std::vector<uint32_t> t;
        std::vector<uint8_t> f;
        parem_status st = regex_table(pattern, pattern_len, alphabet, alphabet_size, mode, partial != 0, 32767, t, f);
        if (st != PAREM_OK) return st;
        *num_states = (uint32_t)f.size();
        if (table) {
            if (table_cap < t.size()) return PAREM_EINVAL;
            std::memcpy(table, t.data(), t.size() * 4);
        }
        if (final_flags) {
            if (final_cap < f.size()) return PAREM_EINVAL;
            std::memcpy(final_flags, f.data(), f.size());
        }
        return PAREM_OK;
    } catch (const std::bad_alloc &) {
        return PAREM_ENOMEM;
    }
}

parem_status parem_compile_regex(const char *pattern, uint64_t pattern_len, const uint8_t *alphabet,
                                 uint32_t alphabet_size, uint32_t mode, const parem_options *opt,
                                 parem_handle *out) {
    if (!out) return PAREM_EINVAL;
    *out = nullptr;
    try {
        const bool partial = opt && opt->partial;
        std::vector<uint32_t> t;
        std::vector<uint8_t> f;
        parem_status st = regex_table(pattern, pattern_len, alphabet, alphabet_size, mode, partial,
                                      partial ? 16381 : 32767, t, f);
        if (st != PAREM_OK) return st;
        std::vector<uint32_t> acc;
        for (uint32_t q = 0; q < f.size(); ++q)
            if (f[q]) acc.push_back(q);
        return parem_compile(t.data(), 4, (uint32_t)f.size(), alphabet, alphabet_size, 0, acc.data(),
                             (uint32_t)acc.size(), opt, out);
    } catch (const std::bad_alloc &) {
        return PAREM_ENOMEM;
    }
}

}  // extern "C"

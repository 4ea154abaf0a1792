// Host-side RE compiler: RE text -> parser automaton tables.
//
// Follows arXiv 2503.06763: the numbered RE (Sect. 2.2), the classic
// followers over numbered symbols (Eq. classicfollowers), the segments
// (Sect. 2.3.2), the follower segments (Eq. folsegdef) and, by powerset, the
// DFA started from I and the multi-entry DFA started from every singleton,
// merged into one table per direction (Sect. 3.1; "Automaton optimization" of
// Sect. 3.3), never minimized.  Segments are enumerated forwards: a segment is
// a walk in the follower graph that starts at a symbol able to begin an LST or
// to follow a terminal, runs through meta-symbols only and stops at the first
// end-letter; this yields the same set as the right-to-left meta-prefix
// extension of Fig. segmentalgo.
#include <algorithm>
#include <array>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <unordered_map>
#include <unordered_set>

#include "../../include/slpf.h"
#include "slpf_internal.hpp"

namespace slpf {
namespace {

// ------------------------------------------------------------------ tokens

enum class T : uint8_t { Byte, Set, Open, Close, Bar, Star, Plus, Quest };
using ByteSet = std::array<uint64_t, 4>;
struct Token {
    T t;
    int byte;
    size_t off;
    ByteSet set{};           // T::Set: the bytes
    int form = 0;            // T::Set: 1 a bracketed set, 2 the wildcard
};

bool has_byte(const ByteSet &m, int b) { return (m[b >> 6] >> (b & 63)) & 1u; }

int hexdigit(int c) {
    if (c >= '0' && c <= '9') return c - '0';
    c |= 0x20;
    if (c >= 'a' && c <= 'f') return c - 'a' + 10;
    return -1;
}

// One byte after an optional backslash (\n, \t, \xHH); -1 on error.
int escaped_byte(const uint8_t *s, size_t n, size_t &i) {
    if (i >= n) return -1;
    int c = s[i++];
    if (c != '\\') return c;
    if (i >= n) return -1;
    int e = s[i++];
    if (e == 'n') return '\n';
    if (e == 't') return '\t';
    if (e == 'x') {
        if (i + 2 > n || hexdigit(s[i]) < 0 || hexdigit(s[i + 1]) < 0) return -1;
        e = hexdigit(s[i]) * 16 + hexdigit(s[i + 1]);
        i += 2;
    }
    return e;
}

bool tokenize(const uint8_t *s, size_t n, std::vector<Token> &out, size_t *err) {
    for (size_t i = 0; i < n;) {
        size_t at = i;
        int c = s[i++];
        if (c == '[') {   // a set of bytes and ranges, ^ complements (App. A, character features)
            Token t{T::Set, -2, at};
            t.form = 1;
            bool neg = i < n && s[i] == '^', first = true;
            if (neg) ++i;
            for (;;) {
                if (i >= n) { *err = at; return false; }
                if (s[i] == ']' && !first) { ++i; break; }
                first = false;
                const int lo = escaped_byte(s, n, i);
                if (lo < 0) { *err = at; return false; }
                int hi = lo;
                if (i + 1 < n && s[i] == '-' && s[i + 1] != ']') {
                    ++i;
                    hi = escaped_byte(s, n, i);
                    if (hi < lo) { *err = at; return false; }
                }
                for (int b = lo; b <= hi; ++b) t.set[b >> 6] |= uint64_t(1) << (b & 63);
            }
            uint64_t any = 0;
            for (auto &w : t.set) {
                if (neg) w = ~w;
                any |= w;
            }
            if (!any) { *err = at; return false; }
            out.push_back(t);
            continue;
        }
        if (c == '.') {   // the wildcard: any byte but the newline
            Token t{T::Set, -2, at};
            t.form = 2;
            t.set = {~uint64_t(0), ~uint64_t(0), ~uint64_t(0), ~uint64_t(0)};
            t.set['\n' >> 6] &= ~(uint64_t(1) << ('\n' & 63));
            out.push_back(t);
            continue;
        }
        switch (c) {
        case '(': out.push_back(Token{T::Open, 0, at}); break;
        case ')': out.push_back(Token{T::Close, 0, at}); break;
        case '|': out.push_back(Token{T::Bar, 0, at}); break;
        case '*': out.push_back(Token{T::Star, 0, at}); break;
        case '+': out.push_back(Token{T::Plus, 0, at}); break;
        case '?': out.push_back(Token{T::Quest, 0, at}); break;
        case '\\': {
            if (i >= n) { *err = at; return false; }
            int e = s[i++];
            if (e == 'n') e = '\n';
            else if (e == 't') e = '\t';
            else if (e == 'x') {
                if (i + 2 > n || hexdigit(s[i]) < 0 || hexdigit(s[i + 1]) < 0) { *err = at; return false; }
                e = hexdigit(s[i]) * 16 + hexdigit(s[i + 1]);
                i += 2;
            }
            out.push_back(Token{T::Byte, e, at});
            break;
        }
        default: out.push_back(Token{T::Byte, c, at});
        }
    }
    return true;
}

// -------------------------------------------------------------- syntax tree

enum class K : uint8_t { Lit, Eps, Cat, Alt, Star, Plus, Opt };
struct Node {
    K kind;
    int byte = -1;           // K::Lit: the byte, or -2 for a set
    std::vector<int> kids;
    int num = 0;
    ByteSet set{};           // K::Lit: the bytes the terminal matches
    int form = 0;            // K::Lit: 0 a byte, 1 a bracketed set, 2 the wildcard
};

struct Parser {
    const std::vector<Token> &tk;
    size_t n_bytes;
    std::vector<Node> &nodes;
    size_t i = 0;
    bool ok = true;
    size_t err = 0;

    int make(K k) {
        nodes.push_back(Node{k});
        return static_cast<int>(nodes.size()) - 1;
    }
    bool at(T t) const { return i < tk.size() && tk[i].t == t; }
    void fail() {
        if (ok) err = i < tk.size() ? tk[i].off : n_bytes;
        ok = false;
    }
    // union of sequences
    int alternation() {
        std::vector<int> alts{sequence()};
        while (ok && at(T::Bar)) {
            ++i;
            alts.push_back(sequence());
        }
        if (!ok) return -1;
        if (alts.size() == 1) return alts[0];
        int x = make(K::Alt);
        nodes[x].kids = alts;
        return x;
    }
    // concatenation of postfix items; none = epsilon
    int sequence() {
        std::vector<int> items;
        while (ok && i < tk.size() && tk[i].t != T::Bar && tk[i].t != T::Close) items.push_back(postfix());
        if (!ok) return -1;
        if (items.empty()) return make(K::Eps);
        if (items.size() == 1) return items[0];
        int x = make(K::Cat);
        nodes[x].kids = items;
        return x;
    }
    int postfix() {
        int x = primary();
        while (ok && i < tk.size()) {
            K k;
            if (tk[i].t == T::Star) k = K::Star;
            else if (tk[i].t == T::Plus) k = K::Plus;
            else if (tk[i].t == T::Quest) k = K::Opt;
            else break;
            ++i;
            int y = make(k);
            nodes[y].kids.push_back(x);
            x = y;
        }
        return x;
    }
    int primary() {
        if (i >= tk.size()) { fail(); return -1; }
        const Token &t = tk[i];
        if (t.t == T::Byte || t.t == T::Set) {
            ++i;
            int x = make(K::Lit);
            nodes[x].byte = t.byte;
            nodes[x].form = t.form;
            if (t.t == T::Set) nodes[x].set = t.set;
            else nodes[x].set[t.byte >> 6] = uint64_t(1) << (t.byte & 63);
            return x;
        }
        if (t.t == T::Open) {
            ++i;
            if (at(T::Close)) { ++i; return make(K::Eps); }
            int x = alternation();
            if (!ok) return -1;
            if (!at(T::Close)) { fail(); return -1; }
            ++i;
            return x;
        }
        fail();
        return -1;
    }
};

// ---------------------------------------------------- numbered symbols, Fol

enum SymKind : uint8_t { SOpen = 0, SLeaf = 1, SClose = 2, SEnd = 3 };
struct Sym {
    SymKind kind;
    int node;     // -1 for the end mark
};

struct Glushkov {
    std::vector<int> first, last;
    bool nullable;
};

// ------------------------------------------------------------ bitset helper

struct Bits {
    std::vector<uint64_t> w;
    explicit Bits(size_t W = 0) : w(W, 0) {}
    void set(size_t i) { w[i >> 6] |= uint64_t(1) << (i & 63); }
    bool get(size_t i) const { return (w[i >> 6] >> (i & 63)) & 1; }
    bool any() const {
        for (auto v : w) if (v) return true;
        return false;
    }
    bool meets(const Bits &o) const {
        for (size_t k = 0; k < w.size(); ++k) if (w[k] & o.w[k]) return true;
        return false;
    }
    void operator|=(const Bits &o) {
        for (size_t k = 0; k < w.size(); ++k) w[k] |= o.w[k];
    }
    bool operator==(const Bits &o) const { return w == o.w; }
};
struct BitsHash {
    size_t operator()(const Bits &b) const { return hash_words(b.w.data(), static_cast<int>(b.w.size())); }
};

struct SegKey {
    std::vector<int> syms;
    bool operator==(const SegKey &o) const { return syms == o.syms; }
};
struct SegKeyHash {
    size_t operator()(const SegKey &k) const {
        size_t h = 1469598103934665603ull;
        for (int s : k.syms) h = (h ^ static_cast<size_t>(s)) * 1099511628211ull;
        return h;
    }
};

}  // namespace

int compile_re(const uint8_t *re, size_t len, const CompileLimits &lim, HostAutomaton &A,
               size_t *err_offset) {
    std::vector<Token> tk;
    size_t err = 0;
    if (!tokenize(re, len, tk, &err)) {
        if (err_offset) *err_offset = err;
        return SLPF_E_SYNTAX;
    }
    std::vector<Node> nodes;
    Parser P{tk, len, nodes};
    int root = P.alternation();
    if (P.ok && P.i != tk.size()) P.fail();
    if (!P.ok) {
        if (err_offset) *err_offset = P.err;
        return SLPF_E_SYNTAX;
    }

    // preorder numbering (iterative)
    {
        std::vector<int> st{root};
        int ctr = 0;
        while (!st.empty()) {
            int x = st.back();
            st.pop_back();
            nodes[x].num = ++ctr;
            for (auto it = nodes[x].kids.rbegin(); it != nodes[x].kids.rend(); ++it) st.push_back(*it);
        }
    }

    // symbols in left-to-right order of the numbered RE, then the end mark
    std::vector<Sym> syms;
    std::vector<int> open_of(nodes.size(), -1), close_of(nodes.size(), -1), leaf_of(nodes.size(), -1);
    std::function<void(int)> emit = [&](int x) {
        const Node &v = nodes[x];
        if (v.kind == K::Lit || v.kind == K::Eps) {
            leaf_of[x] = static_cast<int>(syms.size());
            syms.push_back({SLeaf, x});
            return;
        }
        open_of[x] = static_cast<int>(syms.size());
        syms.push_back({SOpen, x});
        for (int k : v.kids) emit(k);
        close_of[x] = static_cast<int>(syms.size());
        syms.push_back({SClose, x});
    };
    emit(root);
    const int END = static_cast<int>(syms.size());
    syms.push_back({SEnd, -1});
    const int NS = static_cast<int>(syms.size());

    // classic followers of the LST language: node k reads  k( inner )k
    std::vector<std::vector<char>> folm(NS, std::vector<char>(NS, 0));
    auto link = [&](const std::vector<int> &from, const std::vector<int> &to) {
        for (int a : from) for (int b : to) folm[a][b] = 1;
    };
    std::function<Glushkov(int)> gl = [&](int x) -> Glushkov {
        const Node &v = nodes[x];
        if (v.kind == K::Lit || v.kind == K::Eps) return {{leaf_of[x]}, {leaf_of[x]}, false};
        Glushkov in;
        if (v.kind == K::Cat) {
            in = gl(v.kids[0]);
            for (size_t k = 1; k < v.kids.size(); ++k) {
                Glushkov nx = gl(v.kids[k]);
                link(in.last, nx.first);
                Glushkov m;
                m.first = in.first;
                if (in.nullable) m.first.insert(m.first.end(), nx.first.begin(), nx.first.end());
                m.last = nx.last;
                if (nx.nullable) m.last.insert(m.last.end(), in.last.begin(), in.last.end());
                m.nullable = in.nullable && nx.nullable;
                in = m;
            }
        } else if (v.kind == K::Alt) {
            in.nullable = false;
            for (int k : v.kids) {
                Glushkov nx = gl(k);
                in.first.insert(in.first.end(), nx.first.begin(), nx.first.end());
                in.last.insert(in.last.end(), nx.last.begin(), nx.last.end());
                in.nullable = in.nullable || nx.nullable;
            }
        } else {
            in = gl(v.kids[0]);
            if (v.kind != K::Opt) link(in.last, in.first);           // another iteration
            if (v.kind != K::Plus) in.nullable = true;               // zero iterations
        }
        std::vector<int> o{open_of[x]}, c{close_of[x]};
        link(o, in.first);
        link(in.last, c);
        if (in.nullable) link(o, c);
        return {o, c, false};
    };
    Glushkov whole = gl(root);
    link(whole.last, {END});
    const int FIRST = whole.first[0];

    std::vector<std::vector<int>> fol(NS);
    for (int a = 0; a < NS; ++a)
        for (int b = 0; b < NS; ++b)
            if (folm[a][b]) fol[a].push_back(b);

    auto is_end_letter = [&](int s) {
        return syms[s].kind == SEnd || (syms[s].kind == SLeaf && nodes[syms[s].node].kind == K::Lit);
    };

    // infinite ambiguity <=> a cycle through meta-symbols in the follower graph
    {
        std::vector<uint8_t> color(NS, 0);
        bool cyc = false;
        std::function<void(int)> dfs = [&](int s) {
            color[s] = 1;
            for (int t : fol[s]) {
                if (is_end_letter(t) || cyc) continue;
                if (color[t] == 1) { cyc = true; return; }
                if (color[t] == 0) dfs(t);
            }
            color[s] = 2;
        };
        for (int s = 0; s < NS && !cyc; ++s)
            if (!is_end_letter(s) && color[s] == 0) dfs(s);
        if (cyc) return SLPF_E_INF_AMBIG;
    }

    // segments: walks from a start symbol through meta-symbols to an end-letter
    std::vector<char> start(NS, 0);
    start[FIRST] = 1;
    for (int s = 0; s < NS; ++s)
        if (syms[s].kind == SLeaf && nodes[syms[s].node].kind == K::Lit)
            for (int t : fol[s]) start[t] = 1;
    std::unordered_set<SegKey, SegKeyHash> seen;
    std::vector<std::vector<int>> segs;
    bool overflow = false;
    std::vector<int> path;
    std::function<void(int)> walk = [&](int s) {
        if (overflow) return;
        path.push_back(s);
        if (is_end_letter(s)) {
            SegKey key{path};
            if (seen.insert(key).second) {
                segs.push_back(path);
                if (segs.size() > lim.max_segments) overflow = true;
            }
        } else {
            for (int t : fol[s]) walk(t);
        }
        path.pop_back();
    };
    for (int s = 0; s < NS; ++s)
        if (start[s]) walk(s);
    if (overflow || segs.empty()) return SLPF_E_TOO_LARGE;

    // canonical order
    auto code = [&](int s) -> std::pair<int, int> {
        if (syms[s].kind == SEnd) return {0x7fffffff, 0};
        return {nodes[syms[s].node].num, static_cast<int>(syms[s].kind)};
    };
    std::sort(segs.begin(), segs.end(), [&](const std::vector<int> &a, const std::vector<int> &b) {
        auto ea = code(a.back()), eb = code(b.back());
        if (ea != eb) return ea < eb;
        if (a.size() != b.size()) return a.size() < b.size();
        for (size_t k = 0; k + 1 < a.size(); ++k) {
            auto ca = code(a[k]), cb = code(b[k]);
            if (ca != cb) return ca < cb;
        }
        return false;
    });

    const uint32_t L = static_cast<uint32_t>(segs.size());
    const uint32_t W = (L + 63) / 64;
    if (W > static_cast<uint32_t>(kMaxWords)) return SLPF_E_TOO_LARGE;
    A.nseg = L;
    A.W = W;

    // texts
    A.seg_text.clear();
    for (auto &sg : segs) {
        std::string out;
        for (size_t k = 0; k < sg.size(); ++k) {
            if (k) out += ' ';
            const Sym &y = syms[sg[k]];
            if (y.kind == SEnd) { out += "\xe2\x8a\xa3"; continue; }
            int num = nodes[y.node].num;
            char buf[32];
            if (y.kind == SOpen) snprintf(buf, sizeof buf, "%d(", num);
            else if (y.kind == SClose) snprintf(buf, sizeof buf, ")%d", num);
            else if (nodes[y.node].kind == K::Eps) snprintf(buf, sizeof buf, "\xce\xb5%d", num);
            else if (nodes[y.node].form == 2) snprintf(buf, sizeof buf, ".%d", num);
            else if (nodes[y.node].form == 1) {
                // a set as its maximal byte ranges: one byte, two bytes, or lo-hi
                const ByteSet &m = nodes[y.node].set;
                auto one = [&](int b) {
                    char t[8];
                    const bool an = (b >= 'a' && b <= 'z') || (b >= 'A' && b <= 'Z') || (b >= '0' && b <= '9');
                    if (an) snprintf(t, sizeof t, "%c", b);
                    else snprintf(t, sizeof t, "\\x%02x", b);
                    out += t;
                };
                out += '[';
                for (int b = 0; b < 256;) {
                    if (!has_byte(m, b)) { ++b; continue; }
                    int e = b;
                    while (e + 1 < 256 && has_byte(m, e + 1)) ++e;
                    one(b);
                    if (e == b + 1) one(e);
                    else if (e > b + 1) { out += '-'; one(e); }
                    b = e + 1;
                }
                snprintf(buf, sizeof buf, "]%d", num);
            } else {
                int b = nodes[y.node].byte;
                bool letter = (b >= 'a' && b <= 'z') || (b >= 'A' && b <= 'Z');
                if (letter) snprintf(buf, sizeof buf, "%c%d", b, num);
                else snprintf(buf, sizeof buf, "\\x%02x%d", b, num);
            }
            out += buf;
        }
        A.seg_text.push_back(out);
    }

    // byte classes: bytes matched by exactly the same terminals share a class,
    // in order of their smallest byte; class 0 = bytes no terminal matches.
    // Every terminal's set is a union of classes, and classes are disjoint:
    // the partition of overlapping sets into disjoint subsets that App. A
    // (character features, Fig. charset) asks for to keep the powerset
    // automata deterministic, applied to the alphabet, so segments keep
    // their set end-letters and are never split.
    A.classmap.assign(256, 0);
    std::vector<int> leaves;
    for (size_t x = 0; x < nodes.size(); ++x)
        if (nodes[x].kind == K::Lit) leaves.push_back(static_cast<int>(x));
    std::vector<int> rep_byte{-1};                 // a byte of each class
    {
        std::map<std::vector<bool>, uint16_t> sig_class;
        for (int b = 0; b < 256; ++b) {
            std::vector<bool> sig(leaves.size());
            bool any = false;
            for (size_t k = 0; k < leaves.size(); ++k) {
                sig[k] = has_byte(nodes[leaves[k]].set, b);
                any = any || sig[k];
            }
            if (!any) continue;
            auto it = sig_class.find(sig);
            if (it == sig_class.end()) {
                it = sig_class.emplace(sig, static_cast<uint16_t>(rep_byte.size())).first;
                rep_byte.push_back(b);
            }
            A.classmap[b] = it->second;
        }
        A.C = static_cast<uint32_t>(rep_byte.size());
    }
    if (A.C > 256) return SLPF_E_TOO_LARGE;   // class ids are packed into bytes on the device
    const uint32_t C = A.C;
    // the classes a terminal matches
    auto leaf_has_class = [&](int node, uint32_t c) { return c > 0 && has_byte(nodes[node].set, rep_byte[c]); };

    // per segment: end symbol; I, F; followers grouped by end symbol
    std::vector<int> endsym(L);
    Bits I(W), F(W);
    for (uint32_t q = 0; q < L; ++q) {
        endsym[q] = segs[q].back();
        if (segs[q][0] == FIRST) I.set(q);
        if (syms[endsym[q]].kind == SEnd) F.set(q);
    }
    // segment q's end-letter matches class c
    auto label_has = [&](uint32_t q, uint32_t c) {
        return syms[endsym[q]].kind != SEnd && leaf_has_class(syms[endsym[q]].node, c);
    };
    // first symbol -> segments starting with it
    std::vector<std::vector<uint32_t>> starting(NS);
    for (uint32_t q = 0; q < L; ++q) starting[segs[q][0]].push_back(q);
    // followers of each end-letter symbol (Eq. folsegdef)
    std::unordered_map<int, Bits> folT;
    std::vector<Bits> ending_in;   // per end symbol index in `ends`
    std::vector<int> ends;         // distinct terminal end symbols
    std::unordered_map<int, int> end_index;
    for (uint32_t q = 0; q < L; ++q) {
        int e = endsym[q];
        if (syms[e].kind == SEnd) continue;
        if (!end_index.count(e)) {
            end_index[e] = static_cast<int>(ends.size());
            ends.push_back(e);
            ending_in.emplace_back(W);
            Bits f(W);
            for (int t : fol[e])
                for (uint32_t s2 : starting[t]) f.set(s2);
            folT.emplace(e, f);
        }
        ending_in[end_index[e]].set(q);
    }
    A.folseg.assign(static_cast<size_t>(L) * W, 0);
    for (uint32_t q = 0; q < L; ++q) {
        int e = endsym[q];
        if (syms[e].kind == SEnd) continue;
        const Bits &f = folT.at(e);
        std::copy(f.w.begin(), f.w.end(), A.folseg.begin() + static_cast<size_t>(q) * W);
    }
    // group masks for match extraction
    int maxnum = 0;
    for (auto &v : nodes) maxnum = std::max(maxnum, v.num);
    A.ngroups = static_cast<uint32_t>(maxnum + 1);
    A.gmask.assign(static_cast<size_t>(A.ngroups) * 3 * W, 0);
    for (uint32_t q = 0; q < L; ++q) {
        std::vector<int> first(A.ngroups, -1), last(A.ngroups, -1);   // first / last g-symbol kind
        std::vector<char> open_then_close(A.ngroups, 0);
        for (int sy : segs[q]) {
            const Sym &y = syms[sy];
            if (y.kind != SOpen && y.kind != SClose) continue;
            const int g = nodes[y.node].num;
            if (first[g] < 0) first[g] = y.kind;
            if (y.kind == SClose && last[g] == SOpen) open_then_close[g] = 1;
            last[g] = y.kind;
        }
        for (uint32_t g = 1; g < A.ngroups; ++g) {
            uint64_t *m = A.gmask.data() + static_cast<size_t>(g) * 3 * W;
            const uint64_t bit = uint64_t(1) << (q & 63);
            if (last[g] == SOpen) m[q >> 6] |= bit;
            if (first[g] == SClose) m[W + (q >> 6)] |= bit;
            if (open_then_close[g]) m[2 * W + (q >> 6)] |= bit;
        }
    }
    // the RE tree and each segment's symbols, for getChildren
    A.parent.assign(A.ngroups, 0);
    A.node_kind.assign(A.ngroups, 0);
    for (auto &v : nodes) {
        if (v.num <= 0) continue;
        A.node_kind[v.num] = v.kind == K::Lit ? 1 : v.kind == K::Eps ? 2 : 0;
        for (int k : v.kids) A.parent[nodes[k].num] = v.num;
    }
    A.sym_off.assign(1, 0);
    A.sym_code.clear();
    for (uint32_t q = 0; q < L; ++q) {
        for (int sy : segs[q]) {
            const Sym &y = syms[sy];
            const int32_t num = y.kind == SEnd ? 0 : nodes[y.node].num;
            A.sym_code.push_back(num * 4 + static_cast<int32_t>(y.kind));
        }
        A.sym_off.push_back(static_cast<uint32_t>(A.sym_code.size()));
    }
    A.I = I.w;
    A.F = F.w;
    A.ninit = A.nfinal = 0;
    for (uint32_t q = 0; q < L; ++q) {
        A.ninit += I.get(q);
        A.nfinal += F.get(q);
    }
    // terminals grouped by class
    std::vector<std::vector<int>> ends_of_class(C);
    for (size_t k = 0; k < ends.size(); ++k)
        for (uint32_t c = 1; c < C; ++c)
            if (leaf_has_class(syms[ends[k]].node, c)) ends_of_class[c].push_back(static_cast<int>(k));

    // one NFA step on sets (Eq. matrixmul): forward, and reverse (transposed)
    auto fwd_step = [&](const Bits &S, uint32_t c, Bits &out) {
        std::fill(out.w.begin(), out.w.end(), 0);
        for (int k : ends_of_class[c])
            if (S.meets(ending_in[k])) out |= folT.at(ends[k]);
    };
    auto rev_step = [&](const Bits &S, uint32_t c, Bits &out) {
        std::fill(out.w.begin(), out.w.end(), 0);
        for (int k : ends_of_class[c])
            if (folT.at(ends[k]).meets(S)) out |= ending_in[k];
    };

    // powerset over byte classes from the given seeds
    auto build = [&](HostTable &tab, const Bits &start_set, bool forward) -> int {
        std::unordered_map<Bits, uint32_t, BitsHash> ids;
        std::vector<Bits> states;
        auto intern = [&](const Bits &b) -> uint32_t {
            auto it = ids.find(b);
            if (it != ids.end()) return it->second;
            uint32_t id = static_cast<uint32_t>(states.size());
            ids.emplace(b, id);
            states.push_back(b);
            return id;
        };
        intern(Bits(W));                       // id 0 = empty set
        std::vector<std::vector<uint16_t>> delta;
        size_t head = 1;
        Bits nx(W);
        auto expand = [&]() -> bool {
            while (head < states.size()) {
                if (states.size() - 1 > lim.max_states) return false;
                delta.resize(states.size());
                std::vector<uint16_t> row(C, 0);
                for (uint32_t c = 1; c < C; ++c) {
                    if (forward) fwd_step(states[head], c, nx);
                    else rev_step(states[head], c, nx);
                    uint32_t t = intern(nx);
                    if (t > lim.max_states) return false;
                    row[c] = static_cast<uint16_t>(t);
                }
                delta[head] = row;
                ++head;
            }
            return true;
        };
        tab.start = static_cast<uint16_t>(intern(start_set));
        if (!expand()) return SLPF_E_TOO_LARGE;
        tab.dfa_states = static_cast<uint32_t>(states.size()) - 1 - (start_set.any() ? 0 : 0);
        tab.single.resize(L);
        for (uint32_t q = 0; q < L; ++q) {
            Bits s(W);
            s.set(q);
            uint32_t id = intern(s);
            if (id > lim.max_states) return SLPF_E_TOO_LARGE;
            tab.single[q] = static_cast<uint16_t>(id);
        }
        if (!expand()) return SLPF_E_TOO_LARGE;
        // ME-DFA alone: reachable from the singletons
        {
            std::vector<char> mark(states.size(), 0);
            std::vector<uint32_t> st;
            for (uint32_t q = 0; q < L; ++q)
                if (!mark[tab.single[q]]) { mark[tab.single[q]] = 1; st.push_back(tab.single[q]); }
            uint32_t cnt = 0;
            while (!st.empty()) {
                uint32_t x = st.back();
                st.pop_back();
                ++cnt;
                for (uint32_t c = 1; c < C; ++c) {
                    uint32_t t = delta[x][c];
                    if (t && !mark[t]) { mark[t] = 1; st.push_back(t); }
                }
            }
            tab.medfa_states = cnt;
        }
        // DFA alone: reachable from the start set (empty set excluded)
        {
            std::vector<char> mark(states.size(), 0);
            std::vector<uint32_t> st;
            uint32_t cnt = 0;
            if (tab.start) { mark[tab.start] = 1; st.push_back(tab.start); }
            while (!st.empty()) {
                uint32_t x = st.back();
                st.pop_back();
                ++cnt;
                for (uint32_t c = 1; c < C; ++c) {
                    uint32_t t = delta[x][c];
                    if (t && !mark[t]) { mark[t] = 1; st.push_back(t); }
                }
            }
            tab.dfa_states = cnt;
        }
        tab.nstates = static_cast<uint32_t>(states.size());
        tab.bits.assign(static_cast<size_t>(tab.nstates) * W, 0);
        tab.delta.assign(static_cast<size_t>(tab.nstates) * C, 0);
        for (uint32_t id = 0; id < tab.nstates; ++id) {
            std::copy(states[id].w.begin(), states[id].w.end(), tab.bits.begin() + static_cast<size_t>(id) * W);
            if (id)
                std::copy(delta[id].begin(), delta[id].end(), tab.delta.begin() + static_cast<size_t>(id) * C);
        }
        size_t hcap = 16;
        while (hcap < 2 * static_cast<size_t>(tab.nstates)) hcap <<= 1;
        tab.hash.assign(hcap, kHashEmpty);
        for (uint32_t id = 0; id < tab.nstates; ++id) {
            size_t h = hash_words(states[id].w.data(), static_cast<int>(W)) & (hcap - 1);
            while (tab.hash[h] != kHashEmpty) h = (h + 1) & (hcap - 1);
            tab.hash[h] = id;
        }
        return SLPF_OK;
    };
    int st = build(A.fwd, I, true);
    if (st != SLPF_OK) return st;
    st = build(A.rev, F, false);
    if (st != SLPF_OK) return st;

    // speculative entry lists X[p][q]: segments that can sit at a column whose
    // previous byte has class p (or the text start) and next byte class q (or
    // the text end)
    const uint32_t NL = C + 1;
    std::vector<Bits> after(C, Bits(W));        // followers of any segment labelled with class p
    for (uint32_t p = 1; p < C; ++p)
        for (int k : ends_of_class[p]) after[p] |= folT.at(ends[k]);
    A.xoff.assign(static_cast<size_t>(NL) * NL + 1, 0);
    A.xlist.clear();
    A.max_entries = 0;
    for (uint32_t p = 0; p < NL; ++p) {
        for (uint32_t q = 0; q < NL; ++q) {
            A.xoff[p * NL + q] = static_cast<uint32_t>(A.xlist.size());
            if (p == 0 || q == 0) continue;
            uint32_t cnt = 0;
            for (uint32_t s = 0; s < L; ++s) {
                bool label_ok = (q == C) ? F.get(s) : label_has(s, q);
                if (!label_ok) continue;
                bool prev_ok = (p == C) ? I.get(s) : after[p].get(s);
                if (!prev_ok) continue;
                A.xlist.push_back(static_cast<uint16_t>(s));
                ++cnt;
            }
            A.max_entries = std::max(A.max_entries, cnt);
        }
    }
    A.xoff[static_cast<size_t>(NL) * NL] = static_cast<uint32_t>(A.xlist.size());
    // the same lists without the previous-byte filter (initial segments at
    // the text start): the speculation ablation; usable when they fit a mask
    A.xoff_nb.assign(static_cast<size_t>(NL) * NL + 1, 0);
    A.xlist_nb.clear();
    A.max_entries_nb = 0;
    for (uint32_t p = 0; p < NL; ++p) {
        for (uint32_t q = 0; q < NL; ++q) {
            A.xoff_nb[p * NL + q] = static_cast<uint32_t>(A.xlist_nb.size());
            if (p == 0 || q == 0) continue;
            uint32_t cnt = 0;
            for (uint32_t s = 0; s < L; ++s) {
                bool label_ok = (q == C) ? F.get(s) : label_has(s, q);
                if (!label_ok || (p == C && !I.get(s))) continue;
                A.xlist_nb.push_back(static_cast<uint16_t>(s));
                ++cnt;
            }
            A.max_entries_nb = std::max(A.max_entries_nb, cnt);
        }
    }
    A.xoff_nb[static_cast<size_t>(NL) * NL] = static_cast<uint32_t>(A.xlist_nb.size());
    return SLPF_OK;
}

}  // namespace slpf

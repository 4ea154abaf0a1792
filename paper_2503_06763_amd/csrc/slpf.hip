// C ABI of the SLPF library: compile (host) and parse (device launches).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <new>
#include <vector>

#include "../../include/slpf.h"
#include "count.hpp"
#include "kernels.hpp"
#include "slpf_internal.hpp"

namespace {

using namespace slpf;

constexpr size_t kLdsBudget = 96 * 1024;   // transition tables staged in LDS up to this size
constexpr uint64_t kShiftWindow = 256;       // chunk-edge shifting: bytes searched after an edge
constexpr size_t kMaxPairTable = 4u << 20;  // largest table of clean-column sizes (bytes)
constexpr size_t kMaxArcsTable = 2u << 20;  // largest table of arcs between two columns (entries)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Workspace {
    void *base = nullptr;
    size_t bytes = 0;
    uint64_t *pinned = nullptr;       // host staging of batch descriptors
    size_t pinned_words = 0;
    hipEvent_t copied = nullptr;      // the last descriptor copy
};

}  // namespace

struct slpf_parser {
    HostAutomaton A;
    int device = 0;
    uint32_t tuned_chunk = 0, tuned_flags = 0;   // slpf_tune's result (0: not tuned)
    size_t lds_limit = 64 * 1024;     // dynamic LDS per workgroup on the device
    void *blob = nullptr;
    size_t blob_bytes = 0;
    Tabs tabs{};
    uint32_t placement = 0;
    size_t lds_bytes = 0;
    bool host_only = false;
    bool col_single = false;          // every clean column of an accepted text is one segment
    std::mutex mu;
    std::map<hipStream_t, Workspace> ws;   // per stream
};

namespace {

slpf_status hip_ok(hipError_t e) { return e == hipSuccess ? SLPF_OK : SLPF_E_DEVICE; }

// Device-side copy of the tables in one allocation.
// Per state: its only segment when the state's set has exactly one, else kNoSole.
std::vector<uint16_t> sole_segments(const HostTable &t, uint32_t W) {
    std::vector<uint16_t> out(t.nstates, kNoSole);
    for (uint32_t s = 0; s < t.nstates; ++s) {
        int cnt = 0, seg = 0;
        for (uint32_t w = 0; w < W; ++w) {
            const uint64_t v = t.bits[size_t(s) * W + w];
            cnt += __builtin_popcountll(v);
            if (v) seg = int(w * 64 + __builtin_ctzll(v));
        }
        if (cnt == 1) out[s] = static_cast<uint16_t>(seg);
    }
    return out;
}

// No clean column can hold two segments.  A clean column of an accepted
// text is the intersection of the forward set of its prefix and the reverse
// set of its suffix, i.e. of a state reachable from I in the forward table
// and one reachable from F in the reverse table (the multi-entry states never
// label a column), so only those pairs count.
bool column_unambiguous(const HostAutomaton &A) {
    auto reachable = [&](const HostTable &T) {
        std::vector<uint32_t> out{T.start};
        std::vector<uint8_t> seen(T.nstates, 0);
        seen[T.start] = 1;
        for (size_t k = 0; k < out.size(); ++k)
            for (uint32_t c = 0; c < A.C; ++c) {
                const uint32_t nx = T.delta[size_t(out[k]) * A.C + c];
                if (!seen[nx]) {
                    seen[nx] = 1;
                    out.push_back(nx);
                }
            }
        return out;
    };
    const std::vector<uint32_t> rf = reachable(A.fwd), rr = reachable(A.rev);
    for (const uint32_t fs : rf)
        for (const uint32_t bs : rr) {
            uint32_t m = 0;
            for (uint32_t w = 0; w < A.W; ++w)
                m += static_cast<uint32_t>(__builtin_popcountll(A.fwd.bits[size_t(fs) * A.W + w] &
                                                                A.rev.bits[size_t(bs) * A.W + w]));
            if (m > 1) return false;
        }
    return true;
}

slpf_status upload(slpf_parser *p) {
    const HostAutomaton &A = p->A;
    const std::vector<uint16_t> fsole = sole_segments(A.fwd, A.W), rsole = sole_segments(A.rev, A.W);
    // offset form of the transition tables when byte offsets fit in u16
    const uint32_t c2 = 2 * A.C;
    const bool off16 = size_t(A.fwd.nstates) * c2 <= 65535 && size_t(A.rev.nstates) * c2 <= 65535;
    std::vector<uint16_t> fdo, rdo, cls2;
    if (off16) {
        fdo.resize(A.fwd.delta.size());
        rdo.resize(A.rev.delta.size());
        cls2.resize(256);
        for (size_t k = 0; k < fdo.size(); ++k) fdo[k] = static_cast<uint16_t>(A.fwd.delta[k] * c2);
        for (size_t k = 0; k < rdo.size(); ++k) rdo[k] = static_cast<uint16_t>(A.rev.delta[k] * c2);
        for (size_t k = 0; k < 256; ++k) cls2[k] = static_cast<uint16_t>(A.classmap[k] * 2);
    }
    // rank of segment s in the candidate list X[p, end-letter class of s],
    // per previous class p (the compact SLPF's bit index)
    const uint32_t NL = A.C + 1;
    // (per previous class p, or per class pair (p, q) when an end-letter set
    // spans several classes, so that a segment lies in several lists X[p, q])
    bool rank_pq = false;
    {
        std::vector<int> seen(A.nseg, -1);
        for (uint32_t pq = 0; pq < NL * NL && !rank_pq; ++pq)
            for (uint32_t k = A.xoff[pq]; k < A.xoff[pq + 1]; ++k) {
                const int q = static_cast<int>(pq % NL);
                if (seen[A.xlist[k]] >= 0 && seen[A.xlist[k]] != q) rank_pq = true;
                seen[A.xlist[k]] = q;
            }
    }
    const size_t rank_rows = rank_pq ? size_t(NL) * NL : NL;
    std::vector<uint8_t> rankx(rank_rows * std::max<uint32_t>(A.nseg, 1), 0xff);
    for (uint32_t pq = 0; pq < NL * NL; ++pq)
        for (uint32_t k = A.xoff[pq]; k < A.xoff[pq + 1]; ++k)
            rankx[(rank_pq ? pq : pq / NL) * size_t(A.nseg) + A.xlist[k]] = static_cast<uint8_t>(k - A.xoff[pq]);
    // per state, the non-zero words of its set (W <= 32)
    auto nonzero_words = [&](const HostTable &t) {
        std::vector<uint32_t> nz(t.nstates, 0);
        for (uint32_t q = 0; q < t.nstates; ++q)
            for (uint32_t w = 0; w < A.W; ++w)
                if (t.bits[size_t(q) * A.W + w]) nz[q] |= 1u << w;
        return nz;
    };
    const std::vector<uint32_t> fnz = nonzero_words(A.fwd), rnz = nonzero_words(A.rev);
    // tree count: sizes of the clean columns over pairs of a forward state
    // reachable from I (ids 1 .. dfa_states: the powerset from I is built
    // first) and a reverse state reachable from F; every (forward, backward)
    // id pair of an accepted text's column is such a pair.  Kept when small:
    // one byte per pair (sizes capped at 255), or, when that is over the
    // limit, 4 bits per pair (capped at 15)
    uint32_t kfd = A.fwd.dfa_states + 1, krd = A.rev.dfa_states + 1;
    const size_t npairs = size_t(kfd) * krd;
    const bool pair_nib = npairs > kMaxPairTable;
    if ((npairs + 1) / 2 > kMaxPairTable) kfd = krd = 0;
    const size_t pair_bytes = pair_nib ? (size_t(kfd) * krd + 1) / 2 : size_t(kfd) * krd;
    std::vector<uint8_t> pairm(std::max<size_t>(pair_bytes, 1), 0);
    for (uint32_t f = 0; f < kfd; ++f)
        for (uint32_t b = 0; b < krd; ++b) {
            uint32_t m = 0;
            for (uint32_t w = 0; w < A.W; ++w)
                m += static_cast<uint32_t>(
                    __builtin_popcountll(A.fwd.bits[size_t(f) * A.W + w] & A.rev.bits[size_t(b) * A.W + w]));
            const size_t k = size_t(f) * krd + b;
            if (pair_nib)
                pairm[k >> 1] |= static_cast<uint8_t>(std::min<uint32_t>(m, 15) << ((k & 1) * 4));
            else
                pairm[k] = static_cast<uint8_t>(std::min<uint32_t>(m, 255));
        }
    // arcs between two adjacent clean columns of an accepted text, over the
    // forward state f of the left column, the reverse state b of the right
    // one and the class c of the byte between them: left = bits_f(f) &
    // bits_r(rev(b, c)), right = bits_f(fwd(f, c)) & bits_r(b)
    const size_t n_arcs = size_t(kfd) * krd * A.C;
    const bool with_arcs = n_arcs && n_arcs <= kMaxArcsTable;
    std::vector<uint16_t> arcs(with_arcs ? n_arcs : 1, 0xffffu);
    if (with_arcs) {
        std::vector<uint32_t> lft, rgt;
        for (uint32_t f = 0; f < kfd; ++f)
            for (uint32_t b = 0; b < krd; ++b)
                for (uint32_t c = 1; c < A.C; ++c) {
                    const uint32_t fr = A.fwd.delta[size_t(f) * A.C + c], bl = A.rev.delta[size_t(b) * A.C + c];
                    lft.clear();
                    rgt.clear();
                    for (uint32_t w = 0; w < A.W; ++w) {
                        for (uint64_t v = A.fwd.bits[size_t(f) * A.W + w] & A.rev.bits[size_t(bl) * A.W + w]; v;
                             v &= v - 1)
                            lft.push_back(w * 64 + static_cast<uint32_t>(__builtin_ctzll(v)));
                        for (uint64_t v = A.fwd.bits[size_t(fr) * A.W + w] & A.rev.bits[size_t(b) * A.W + w]; v;
                             v &= v - 1)
                            rgt.push_back(w * 64 + static_cast<uint32_t>(__builtin_ctzll(v)));
                    }
                    uint32_t na = 0;
                    for (const uint32_t r : lft)
                        for (const uint32_t q : rgt) na += (A.folseg[size_t(r) * A.W + (q >> 6)] >> (q & 63)) & 1u;
                    arcs[(size_t(f) * krd + b) * A.C + c] = static_cast<uint16_t>(std::min<uint32_t>(na, 0xffffu));
                }
    }
    // 0, 1, .., the larger DFA's state count: the all-DFA-states speculation
    // ablation lists DFA state m + 1 as entry m
    std::vector<uint16_t> seqids(std::max(A.fwd.dfa_states, A.rev.dfa_states) + 2);
    for (size_t k = 0; k < seqids.size(); ++k) seqids[k] = static_cast<uint16_t>(k);
    // the segments each segment follows (transpose of FolSeg)
    std::vector<uint64_t> pred(size_t(A.nseg) * A.W, 0);
    for (uint32_t r = 0; r < A.nseg; ++r)
        for (uint32_t sg = 0; sg < A.nseg; ++sg)
            if ((A.folseg[size_t(r) * A.W + (sg >> 6)] >> (sg & 63)) & 1ull)
                pred[size_t(sg) * A.W + (r >> 6)] |= 1ull << (r & 63);
    struct Part {
        const void *src;
        size_t bytes;
        size_t off;
    };
    std::vector<Part> parts = {
        {A.classmap.data(), A.classmap.size() * 2, 0},
        {A.fwd.delta.data(), A.fwd.delta.size() * 2, 0},
        {A.rev.delta.data(), A.rev.delta.size() * 2, 0},
        {A.fwd.bits.data(), A.fwd.bits.size() * 8, 0},
        {A.rev.bits.data(), A.rev.bits.size() * 8, 0},
        {A.xoff.data(), A.xoff.size() * 4, 0},
        {A.xlist.data(), std::max<size_t>(A.xlist.size(), 1) * 2, 0},
        {A.fwd.single.data(), A.fwd.single.size() * 2, 0},
        {A.rev.single.data(), A.rev.single.size() * 2, 0},
        {A.fwd.hash.data(), A.fwd.hash.size() * 4, 0},
        {A.rev.hash.data(), A.rev.hash.size() * 4, 0},
        {A.folseg.data(), A.folseg.size() * 8, 0},
        {fsole.data(), fsole.size() * 2, 0},
        {rsole.data(), rsole.size() * 2, 0},
        {fdo.data(), fdo.size() * 2, 0},
        {rdo.data(), rdo.size() * 2, 0},
        {cls2.data(), cls2.size() * 2, 0},
        {rankx.data(), rankx.size(), 0},
        {fnz.data(), fnz.size() * 4, 0},
        {rnz.data(), rnz.size() * 4, 0},
        {A.xoff_nb.data(), A.xoff_nb.size() * 4, 0},
        {A.xlist_nb.data(), std::max<size_t>(A.xlist_nb.size(), 1) * 2, 0},
        {A.gmask.data(), A.gmask.size() * 8, 0},
        {pairm.data(), pairm.size(), 0},
        {pred.data(), pred.size() * 8, 0},
        {arcs.data(), arcs.size() * 2, 0},
        {seqids.data(), seqids.size() * 2, 0},
    };
    size_t total = 0;
    for (auto &pt : parts) {
        pt.off = total;
        total = align_up(total + pt.bytes, 256);
    }
    std::vector<uint8_t> host(total, 0);
    for (auto &pt : parts)
        if (pt.src && pt.bytes) std::memcpy(host.data() + pt.off, pt.src, pt.bytes);
    if (hipSetDevice(p->device) != hipSuccess) return SLPF_E_DEVICE;
    if (hipMalloc(&p->blob, total) != hipSuccess) {
        p->blob = nullptr;
        return SLPF_E_NOMEM;
    }
    if (hipMemcpy(p->blob, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) return SLPF_E_DEVICE;
    p->blob_bytes = total;
    auto at = [&](int k) { return static_cast<uint8_t *>(p->blob) + parts[k].off; };
    Tabs &t = p->tabs;
    t.classmap = reinterpret_cast<const uint16_t *>(at(0));
    t.fdelta = reinterpret_cast<const uint16_t *>(at(1));
    t.rdelta = reinterpret_cast<const uint16_t *>(at(2));
    t.fbits = reinterpret_cast<const uint64_t *>(at(3));
    t.rbits = reinterpret_cast<const uint64_t *>(at(4));
    t.xoff = reinterpret_cast<const uint32_t *>(at(5));
    t.xlist = reinterpret_cast<const uint16_t *>(at(6));
    t.fsingle = reinterpret_cast<const uint16_t *>(at(7));
    t.rsingle = reinterpret_cast<const uint16_t *>(at(8));
    t.fhash = reinterpret_cast<const uint32_t *>(at(9));
    t.rhash = reinterpret_cast<const uint32_t *>(at(10));
    t.folseg = reinterpret_cast<const uint64_t *>(at(11));
    t.fsole = reinterpret_cast<const uint16_t *>(at(12));
    t.rsole = reinterpret_cast<const uint16_t *>(at(13));
    t.off16 = off16 ? 1u : 0u;
    t.fdo = off16 ? reinterpret_cast<const uint16_t *>(at(14)) : nullptr;
    t.rdo = off16 ? reinterpret_cast<const uint16_t *>(at(15)) : nullptr;
    t.cls2 = off16 ? reinterpret_cast<const uint16_t *>(at(16)) : nullptr;
    t.rankx = at(17);
    t.rank_pq = rank_pq ? 1u : 0u;
    t.fnz = reinterpret_cast<const uint32_t *>(at(18));
    t.rnz = reinterpret_cast<const uint32_t *>(at(19));
    t.xoff_nb = reinterpret_cast<const uint32_t *>(at(20));
    t.xlist_nb = reinterpret_cast<const uint16_t *>(at(21));
    t.emax_nb = std::max<uint32_t>(A.max_entries_nb, 1);
    t.gmask = reinterpret_cast<const uint64_t *>(at(22));
    t.ngroups = A.ngroups;
    t.pairm = at(23);
    t.kfd = kfd;
    t.krd = krd;
    t.pair_nib = pair_nib && kfd ? 1u : 0u;
    t.predseg = reinterpret_cast<const uint64_t *>(at(24));
    t.arcs2 = with_arcs ? reinterpret_cast<const uint16_t *>(at(25)) : nullptr;
    t.seqids = reinterpret_cast<const uint16_t *>(at(26));
    t.dfa_f = A.fwd.dfa_states;
    t.dfa_r = A.rev.dfa_states;
    t.col_single = p->col_single ? 1u : 0u;
    t.fhmask = static_cast<uint32_t>(A.fwd.hash.size() - 1);
    t.rhmask = static_cast<uint32_t>(A.rev.hash.size() - 1);
    t.C = A.C;
    t.W = A.W;
    t.NL = A.C + 1;
    t.nf = A.fwd.nstates;
    t.nr = A.rev.nstates;
    t.fstart = A.fwd.start;
    t.rstart = A.rev.start;
    t.emax = std::max<uint32_t>(A.max_entries, 1);
    t.wmagic = ((1ull << 32) + A.W - 1) / A.W;
    t.nseg = A.nseg;
    return SLPF_OK;
}

void set_placement(slpf_parser *p) {
    const HostAutomaton &A = p->A;
    p->lds_bytes = 512 + (static_cast<size_t>(A.fwd.nstates) + A.rev.nstates) * A.C * 2;
    size_t budget = kLdsBudget;
    if (!p->host_only) {
        int lim = 0;
        if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) == hipSuccess &&
            lim > 0) {
            p->lds_limit = static_cast<size_t>(lim);
            budget = std::min<size_t>(budget, p->lds_limit);
        }
    } else {
        p->lds_limit = 160 * 1024;
    }
    p->placement = p->lds_bytes <= budget ? 0 : 1;
}

constexpr size_t kLdsPerCu = 160 * 1024;     // LDS of one compute unit (gfx950)

uint64_t chunk_bytes_for(uint64_t n, const slpf_parse_opts *o) {
    if (o && o->chunk_bytes) return o->chunk_bytes;
    // 1 KiB lane chunks for large texts (a chunk-size sweep on MI355X: reach
    // latency falls with more lanes while build & merge stays flat), down to
    // 256 bytes so that small texts still fill several wavefronts
    uint64_t s = (n + 262143) / 262144;
    s = (s + 63) / 64 * 64;
    return std::min<uint64_t>(std::max<uint64_t>(s, 256), 1024);
}

struct Layout {
    std::vector<size_t> off;
    size_t total = 0;
    int add(size_t bytes) {
        off.push_back(total);
        total = align_up(total + std::max<size_t>(bytes, 8), 256);
        return static_cast<int>(off.size()) - 1;
    }
};

// join level sizes: N_0 = c, N_{l+1} = ceil(N_l / 64) down to a level of one item
std::vector<uint32_t> join_levels(uint32_t c) {
    std::vector<uint32_t> lv{c};
    do lv.push_back((lv.back() + 63) / 64);
    while (lv.back() > 1);
    return lv;
}

}  // namespace

extern "C" {

const char *slpf_status_str(slpf_status s) {
    switch (s) {
    case SLPF_OK: return "ok";
    case SLPF_E_ARG: return "invalid argument";
    case SLPF_E_SYNTAX: return "RE syntax error";
    case SLPF_E_INF_AMBIG: return "infinitely ambiguous RE";
    case SLPF_E_TOO_LARGE: return "automaton too large";
    case SLPF_E_NOMEM: return "out of memory";
    case SLPF_E_DEVICE: return "device error";
    case SLPF_E_CAPACITY: return "output buffer too small";
    case SLPF_E_INTERNAL: return "internal error";
    }
    return "unknown status";
}

slpf_status slpf_compile(const char *re, size_t re_len, const slpf_compile_opts *opts,
                         slpf_parser **out, size_t *err_offset) {
    if (!out) return SLPF_E_ARG;
    *out = nullptr;
    if (!re && re_len) return SLPF_E_ARG;
    if (opts && opts->struct_size != sizeof(slpf_compile_opts)) return SLPF_E_ARG;
    CompileLimits lim;
    if (opts && opts->max_segments) lim.max_segments = std::min<uint32_t>(opts->max_segments, 64 * kMaxWords);
    if (opts && opts->max_states) lim.max_states = std::min<uint32_t>(opts->max_states, 65535);
    slpf_parser *p = new (std::nothrow) slpf_parser();
    if (!p) return SLPF_E_NOMEM;
    p->device = opts ? opts->device : 0;
    int st;
    try {
        st = compile_re(reinterpret_cast<const uint8_t *>(re), re_len, lim, p->A, err_offset);
    } catch (const std::bad_alloc &) {
        st = SLPF_E_NOMEM;
    } catch (...) {
        st = SLPF_E_INTERNAL;
    }
    p->host_only = opts && (opts->flags & SLPF_COMPILE_HOST_ONLY);
    if (st == SLPF_OK) {
        set_placement(p);
        p->col_single = column_unambiguous(p->A);
    }
    if (st == SLPF_OK && !p->host_only) st = upload(p);
    if (st != SLPF_OK) {
        slpf_parser_destroy(p);
        return static_cast<slpf_status>(st);
    }
    *out = p;
    return SLPF_OK;
}

void slpf_parser_destroy(slpf_parser *p) {
    if (!p) return;
    if (p->host_only) {
        delete p;
        return;
    }
    hipSetDevice(p->device);
    for (auto &kv : p->ws) {
        if (kv.second.copied) hipEventSynchronize(kv.second.copied);
        if (kv.second.base) hipFree(kv.second.base);
        if (kv.second.pinned) hipHostFree(kv.second.pinned);
        if (kv.second.copied) hipEventDestroy(kv.second.copied);
    }
    if (p->blob) hipFree(p->blob);
    delete p;
}

slpf_status slpf_parser_info_get(const slpf_parser *p, slpf_parser_info *info) {
    if (!p || !info) return SLPF_E_ARG;
    const HostAutomaton &A = p->A;
    std::memset(info, 0, sizeof(*info));
    info->num_segments = A.nseg;
    info->words_per_column = A.W;
    info->num_initial = A.ninit;
    info->num_final = A.nfinal;
    info->fwd_states = A.fwd.nstates - 1;
    info->rev_states = A.rev.nstates - 1;
    info->dfa_states = A.fwd.dfa_states;
    info->medfa_states = A.fwd.medfa_states;
    info->rdfa_states = A.rev.dfa_states;
    info->rmedfa_states = A.rev.medfa_states;
    info->num_classes = A.C;
    info->max_entries = A.max_entries;
    info->max_entries_next_byte = A.max_entries_nb;
    info->placement = p->placement;
    info->column_unambiguous = p->col_single ? 1u : 0u;
    info->table_bytes = p->blob_bytes;
    return SLPF_OK;
}

slpf_status slpf_segment_text(const slpf_parser *p, uint32_t seg, char *buf, size_t cap, size_t *need) {
    if (!p || seg >= p->A.nseg) return SLPF_E_ARG;
    const std::string &s = p->A.seg_text[seg];
    if (need) *need = s.size();
    if (buf && cap) {
        size_t k = std::min(cap - 1, s.size());
        std::memcpy(buf, s.data(), k);
        buf[k] = 0;
    }
    return SLPF_OK;
}

slpf_status slpf_table_dump(const slpf_parser *p, int dir, uint64_t *sets, uint32_t *delta,
                            uint16_t *classmap) {
    if (!p || (dir != 0 && dir != 1)) return SLPF_E_ARG;
    const HostTable &t = dir == 0 ? p->A.fwd : p->A.rev;
    if (sets) std::memcpy(sets, t.bits.data(), t.bits.size() * 8);
    if (delta)
        for (size_t k = 0; k < t.delta.size(); ++k) delta[k] = t.delta[k];
    if (classmap) std::memcpy(classmap, p->A.classmap.data(), 512);
    return SLPF_OK;
}

uint64_t slpf_forest_bytes(const slpf_parser *p, uint64_t n) {
    if (!p) return 0;
    return (n + 1) * static_cast<uint64_t>(p->A.W) * 8;
}

uint64_t slpf_compact_bytes(uint64_t n) { return (n + 1) * 8; }

slpf_status slpf_decode_compact(const slpf_parser *cp, const uint8_t *text_dev, uint64_t n,
                                const uint64_t *compact_dev, uint64_t *columns_dev, void *hip_stream) {
    const slpf_parser *p = cp;
    if (!p || p->host_only || !compact_dev || !columns_dev || (n && !text_dev)) return SLPF_E_ARG;
    if (p->A.max_entries > static_cast<uint32_t>(kMaxEntries)) return SLPF_E_TOO_LARGE;   // no compact form
    if (hipSetDevice(p->device) != hipSuccess) return SLPF_E_DEVICE;
    const uint64_t cols = n + 1;
    const uint64_t blocks = (cols + 255) / 256;
    if (blocks > 0x7fffffffull) return SLPF_E_ARG;
    hipLaunchKernelGGL(k_decode_compact, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), p->tabs, text_dev, n, compact_dev, columns_dev);
    return hipGetLastError() == hipSuccess ? SLPF_OK : SLPF_E_DEVICE;
}

uint64_t slpf_num_chunks(const slpf_parser *p, uint64_t n, const slpf_parse_opts *opts) {  // one text
    if (!p || n == 0) return 0;
    uint64_t s = chunk_bytes_for(n, opts);
    return (n + s - 1) / s;
}

}  // extern "C"

namespace {

// One job: T texts parsed with one parser; text t owns lane chunks
// tchunk0[t] .. tchunk0[t+1]-1 of a common index space.
// ext_ws / ext_bytes: a caller-held workspace (device memory) used instead of
// the parser's per-stream one, for one text only; nothing is allocated then.
slpf_status run_job(slpf_parser *p, const slpf_text *items, size_t T, const slpf_parse_opts *opts,
                    hipStream_t stream, uint8_t *ext_ws = nullptr, size_t ext_bytes = 0) {
    const uint32_t flags = opts ? opts->flags : 0;
    const bool recog = (flags & SLPF_PARSE_RECOGNIZE) != 0;
    const bool count = !(flags & SLPF_PARSE_NO_COUNT) && !recog;
    if (hipSetDevice(p->device) != hipSuccess) return SLPF_E_DEVICE;
    Tabs tb = p->tabs;
    // speculation entry lists: reduced (default) or filtered by the next byte only
    Tabs ts = tb;
    if ((flags & SLPF_PARSE_COMPACT) && tb.emax > static_cast<uint32_t>(kMaxEntries)) return SLPF_E_TOO_LARGE;
    if (flags & SLPF_PARSE_NEXT_BYTE_ENTRIES) {
        ts.xoff = tb.xoff_nb;
        ts.xlist = tb.xlist_nb;
        ts.emax = tb.emax_nb;
    }
    // all-DFA-states ablation: inner lane-chunk edges list every DFA state
    const bool alldfa = (flags & SLPF_PARSE_ALL_DFA_STATES) != 0;
    if (alldfa) ts.emax = std::max(ts.emax, std::max(tb.dfa_f, tb.dfa_r));
    const uint32_t W = tb.W, E = ts.emax, EW = (E + 63) / 64;
    // join masks of at most 32 words (2048 entries; the entry lists of a
    // parser always fit, the all-DFA-states lists of a large DFA may not)
    if (EW > static_cast<uint32_t>(kMaxWords)) return SLPF_E_TOO_LARGE;
    uint64_t total = 0;
    for (size_t t = 0; t < T; ++t) total += items[t].n;
    const uint64_t s = chunk_bytes_for(total, opts);
    std::vector<uint32_t> tchunk0(T + 1, 0);
    uint64_t c64 = 0;
    for (size_t t = 0; t < T; ++t) {
        tchunk0[t] = static_cast<uint32_t>(c64);
        c64 += (items[t].n + s - 1) / s;
        if (c64 > 0x7fffffffull) return SLPF_E_ARG;
    }
    tchunk0[T] = static_cast<uint32_t>(c64);
    const uint32_t c = static_cast<uint32_t>(c64);
    const uint32_t nt = static_cast<uint32_t>(T);

    Job jb{};
    jb.ntexts = nt;
    jb.fwd_only = recog ? 1u : 0u;
    jb.compact = (flags & SLPF_PARSE_COMPACT) ? 1u : 0u;
    jb.s = s;
    jb.c = c;
    // chunk-edge shifting: on by default when a run group cannot hold the
    // longest entry list; the window is half a lane chunk at most
    const bool shift = !alldfa && !(flags & SLPF_PARSE_NO_EDGE_SHIFT) &&
                       ((flags & SLPF_PARSE_EDGE_SHIFT) || ts.emax > static_cast<uint32_t>(kGroup));
    jb.alldfa = alldfa ? 1u : 0u;
    jb.shift = shift ? static_cast<uint32_t>(std::min<uint64_t>(kShiftWindow, s / 2)) : 0u;
    if (T == 1) {
        jb.d0[0] = reinterpret_cast<uint64_t>(items[0].text_dev);
        jb.d0[1] = items[0].n;
        jb.d0[2] = reinterpret_cast<uint64_t>(items[0].out.columns_dev);
        jb.d0[3] = reinterpret_cast<uint64_t>(items[0].out.scalars_dev);
    }
    const std::vector<uint32_t> jl = join_levels(std::max<uint32_t>(c, 1));
    const size_t nck = size_t(c) * ((s + 63) / 64);   // window-major checkpoints

    Layout L;
    int itd = L.add(T > 1 ? T * 32 + (T + 1) * 4 + 64 : 8);
    const int itmap = T > 1 ? L.add(size_t(c) * 4) : -1;   // the text of each lane chunk
    int iR = L.add(size_t(E) * c * 2), iRh = L.add(size_t(E) * c * 2), iRt = L.add(size_t(E) * c * 2);
    int iRm = -1, iRmh = -1, ies = -1;
    if (shift) {
        iRm = L.add(size_t(E) * c * 2);
        iRmh = L.add(size_t(E) * c * 2);
        ies = L.add(c);
    }
    int iMf = L.add(size_t(c) * E * EW * 8), iMb = L.add(size_t(c) * E * EW * 8);
    int inxf = L.add(size_t(c + 1) * 2), inxb = L.add(size_t(c + 1) * 2), irsf = L.add(c + 1), irsb = L.add(c + 1);
    int ifin = L.add(size_t(c + 1) * EW * 8), ifout = L.add(size_t(c + 1) * EW * 8);
    int ibin = L.add(size_t(c + 1) * EW * 8), ibout = L.add(size_t(c + 1) * EW * 8);
    int ifid = L.add(size_t(c) * 2), irid = L.add(size_t(c) * 2);
    int ickpt = L.add(nck * 2), ibckpt = L.add(nck * 2);
    int iflags = L.add(16);
    // join levels: items of level l >= 1 (rows, nx, cst, cv, entering vectors)
    // and prefix maps of every level below the top
    const size_t TL = jl.size() - 1;
    std::vector<int> jrows[2], jnx[2], jisc[2], jcv[2], jvec[2], jprow[2], jpcst[2], jpcv[2];
    for (size_t l = 0; l <= TL; ++l)
        for (int d = 0; d < 2; ++d) {
            const size_t N = jl[l];
            jrows[d].push_back(l ? L.add(N * E * EW * 8) : -1);
            jnx[d].push_back(l ? L.add((N + 1) * 2) : -1);
            jisc[d].push_back(l ? L.add(N + 1) : -1);
            jcv[d].push_back(l ? L.add((N + 1) * EW * 8) : -1);
            jvec[d].push_back(l ? L.add((N + 1) * EW * 8) : -1);
            jprow[d].push_back(l < TL ? L.add(N * E * EW * 8) : -1);
            jpcst[d].push_back(l < TL ? L.add(N + 1) : -1);
            jpcv[d].push_back(l < TL ? L.add((N + 1) * EW * 8) : -1);
        }
    // tree count: run marks per 64-column window (as the checkpoints), chunk
    // and text products, and the lists of the run kernels.  Long runs (more
    // than lshort columns) are at most total / lshort; runs with a cell
    // boundary inside are at most total / cell, and so are the anchors, which
    // bounds the piece matrices.
    const uint64_t cols_total = total + T;
    // (cells of 256 columns up to 4096 cells per job, so the pieces of a long
    // run walk in parallel; longer texts get longer cells)
    uint64_t cell = 256;
    while (cell < cols_total / 4096) cell <<= 1;
    const uint32_t lshort = 512;
    const uint64_t cap_runs = cols_total / lshort + T + 1;
    const uint64_t cap_mats = 2 * (cols_total / cell) + 2;
    const uint64_t cap_pieces = cap_runs + cols_total / cell + 1;
    // short runs queued for one lane each: room for one per 16 columns (the
    // rest are counted where they are found)
    const uint64_t cap_sruns = tb.col_single || s > kMaxRunChunk
                                   ? 0 : std::min<uint64_t>(cols_total / 16 + 64, 0x7fffffffull);
    if (count && (cap_runs > 0xffffffffull || cap_pieces > 0xffffffffull || nck >= 0x80000000ull))
        return SLPF_E_ARG;
    int iam = -1, iaend = -1, icfac = -1, itprod = -1, itfail = -1, iccnt = -1, idch = -1, iruns = -1, ipiece = -1,
        imats = -1, ipmat = -1, isr = -1, isq2 = -1, icf = -1;
    if (count) {
        iam = L.add(nck * 8);
        iaend = L.add(size_t(T) * 8);
        icfac = L.add(size_t(c) * 16);
        itprod = L.add(size_t(T) * 16);
        itfail = L.add(size_t(T) * 4);
        iccnt = L.add(32);
        idch = L.add((nck + cap_sruns) * 4);
        isr = L.add(cap_sruns * 8);
        icf = L.add(c);
        isq2 = L.add(cap_sruns * 4);
        iruns = L.add(cap_runs * sizeof(RunRec));
        ipiece = L.add(cap_pieces * 8);
        imats = L.add(cap_mats * kPieceR * kPieceR * 16);
        ipmat = L.add(cap_pieces * 4);
    }

    uint8_t *base;
    if (ext_ws) {
        if (T != 1) return SLPF_E_ARG;
        if (L.total > ext_bytes) return SLPF_E_CAPACITY;
        base = ext_ws;
    } else {
        std::lock_guard<std::mutex> g(p->mu);
        Workspace &w = p->ws[stream];
        if (w.bytes < L.total) {
            if (w.base) {
                if (hipStreamSynchronize(stream) != hipSuccess) return SLPF_E_DEVICE;
                hipFree(w.base);
                w.base = nullptr;
                w.bytes = 0;
            }
            size_t want = align_up(L.total + L.total / 4, 1 << 20);
            if (hipMalloc(&w.base, want) != hipSuccess) {
                w.base = nullptr;
                return SLPF_E_NOMEM;
            }
            w.bytes = want;
        }
        base = static_cast<uint8_t *>(w.base);
        if (T > 1) {   // text descriptors: pinned staging, copied on the stream
            if (w.copied && hipEventSynchronize(w.copied) != hipSuccess) return SLPF_E_DEVICE;
            const size_t need = T * 4 + (T + 1 + 1) / 2 + 8;
            if (w.pinned_words < need) {
                if (w.pinned) hipHostFree(w.pinned);
                w.pinned = nullptr;
                if (hipHostMalloc(reinterpret_cast<void **>(&w.pinned), need * 8, hipHostMallocDefault) != hipSuccess) {
                    w.pinned_words = 0;
                    return SLPF_E_NOMEM;
                }
                w.pinned_words = need;
            }
            uint64_t *d = w.pinned;
            for (size_t t = 0; t < T; ++t) {
                d[4 * t] = reinterpret_cast<uint64_t>(items[t].text_dev);
                d[4 * t + 1] = items[t].n;
                d[4 * t + 2] = reinterpret_cast<uint64_t>(items[t].out.columns_dev);
                d[4 * t + 3] = reinterpret_cast<uint64_t>(items[t].out.scalars_dev);
            }
            std::memcpy(d + 4 * T, tchunk0.data(), (T + 1) * 4);
            if (hipMemcpyAsync(base + L.off[itd], d, T * 32 + (T + 1) * 4, hipMemcpyHostToDevice, stream) !=
                hipSuccess)
                return SLPF_E_DEVICE;
            if (!w.copied && hipEventCreateWithFlags(&w.copied, hipEventDisableTiming) != hipSuccess)
                return SLPF_E_DEVICE;
            if (hipEventRecord(w.copied, stream) != hipSuccess) return SLPF_E_DEVICE;
        }
    }
    auto ptr = [&](int k) { return base + L.off[k]; };
    if (T > 1) {
        jb.tdesc = reinterpret_cast<const uint64_t *>(ptr(itd));
        jb.tchunk0 = reinterpret_cast<const uint32_t *>(ptr(itd) + T * 32);
    }
    jb.R = reinterpret_cast<uint16_t *>(ptr(iR));
    jb.Rh = reinterpret_cast<uint16_t *>(ptr(iRh));
    jb.Rt = reinterpret_cast<uint16_t *>(ptr(iRt));
    jb.Rm = shift ? reinterpret_cast<uint16_t *>(ptr(iRm)) : jb.R;
    jb.Rmh = shift ? reinterpret_cast<uint16_t *>(ptr(iRmh)) : nullptr;
    jb.eshift = shift ? reinterpret_cast<uint8_t *>(ptr(ies)) : nullptr;
    jb.Mf = reinterpret_cast<uint64_t *>(ptr(iMf));
    jb.MbR = reinterpret_cast<uint64_t *>(ptr(iMb));
    jb.nxf = reinterpret_cast<uint16_t *>(ptr(inxf));
    jb.nxb = reinterpret_cast<uint16_t *>(ptr(inxb));
    jb.ew = EW;
    jb.rsf = ptr(irsf);
    jb.rsb = ptr(irsb);
    jb.fin = reinterpret_cast<uint64_t *>(ptr(ifin));
    jb.fout = reinterpret_cast<uint64_t *>(ptr(ifout));
    jb.bin = reinterpret_cast<uint64_t *>(ptr(ibin));
    jb.bout = reinterpret_cast<uint64_t *>(ptr(ibout));
    jb.fid = reinterpret_cast<uint16_t *>(ptr(ifid));
    jb.rid = reinterpret_cast<uint16_t *>(ptr(irid));
    jb.ckpt = reinterpret_cast<uint16_t *>(ptr(ickpt));
    jb.bckpt = reinterpret_cast<uint16_t *>(ptr(ibckpt));
    jb.flags = reinterpret_cast<uint32_t *>(ptr(iflags));
    jb.trace = nullptr;
    if (T == 1 && opts && opts->trace_dev && opts->trace_bytes >= 2ull * (c + 1) * W * 8) jb.trace = opts->trace_dev;
    jb.count_on = count ? 1u : 0u;
    if (count) {
        jb.amask = reinterpret_cast<uint64_t *>(ptr(iam));
        jb.aend = reinterpret_cast<uint64_t *>(ptr(iaend));
        jb.cfac = reinterpret_cast<uint64_t *>(ptr(icfac));
        jb.tprod = reinterpret_cast<uint64_t *>(ptr(itprod));
        jb.tfail = reinterpret_cast<uint32_t *>(ptr(itfail));
        jb.ccnt = reinterpret_cast<uint32_t *>(ptr(iccnt));
        jb.dchunk = reinterpret_cast<uint32_t *>(ptr(idch));
        jb.runs = reinterpret_cast<RunRec *>(ptr(iruns));
        jb.piece = reinterpret_cast<uint64_t *>(ptr(ipiece));
        jb.mats = reinterpret_cast<uint64_t *>(ptr(imats));
        jb.pmat = reinterpret_cast<uint32_t *>(ptr(ipmat));
        jb.sruns = reinterpret_cast<uint64_t *>(ptr(isr));
        jb.squeue2 = reinterpret_cast<uint32_t *>(ptr(isq2));
        jb.cfull = reinterpret_cast<uint8_t *>(ptr(icf));
        jb.nsruns = reinterpret_cast<unsigned long long *>(ptr(iccnt) + 16);
        jb.cap_sruns = static_cast<uint32_t>(cap_sruns);
        jb.fol_lds = size_t(tb.nseg) * tb.W * 8 <= kFolLdsBytes ? 1u : 0u;
        jb.cap_runs = static_cast<uint32_t>(cap_runs);
        jb.cap_pieces = static_cast<uint32_t>(cap_pieces);
        jb.cap_mats = static_cast<uint32_t>(std::min<uint64_t>(cap_mats, 0xffffffffull));
        jb.lshort = lshort;
        jb.cell = cell;
    }

    const bool timed = opts && opts->events && opts->num_events >= SLPF_NUM_PHASE_EVENTS;
    if (opts && opts->events && opts->num_events && !timed) return SLPF_E_ARG;
    if (timed)
        for (int k = 0; k < SLPF_NUM_PHASE_EVENTS; ++k)
            if (!opts->events[k]) return SLPF_E_ARG;
    hipError_t ev_err = hipSuccess;
    auto mark = [&](int k) {
        if (timed && ev_err == hipSuccess) ev_err = hipEventRecord(static_cast<hipEvent_t>(opts->events[k]), stream);
    };
    const bool lds = p->placement == 0 && !(flags & SLPF_PARSE_FORCE_L2);
    const size_t lds_bytes = lds ? p->lds_bytes : 0;
    const uint32_t blocks = (c + 255) / 256;

    if (T > 1 && c) {
        uint32_t *tmap = reinterpret_cast<uint32_t *>(ptr(itmap));
        hipLaunchKernelGGL(k_tmap, dim3(blocks), dim3(256), 0, stream, jb, tmap);
        jb.tmap = tmap;
    }
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, stream, jb);
    mark(0);
    if (c) {
        // reach
        auto reach = [&](auto mode) {
            constexpr int MU = decltype(mode)::value;
            if (lds && tb.off16)
                hipLaunchKernelGGL((k_reach<true, true, MU>), dim3(blocks), dim3(256), lds_bytes, stream, ts, jb);
            else if (lds)
                hipLaunchKernelGGL((k_reach<true, false, MU>), dim3(blocks), dim3(256), lds_bytes, stream, ts, jb);
            else
                hipLaunchKernelGGL((k_reach<false, false, MU>), dim3(blocks), dim3(256), 0, stream, ts, jb);
        };
        if (ts.emax > static_cast<uint32_t>(kGroup) || alldfa)
            reach(std::integral_constant<int, 2>{});
        else if (jb.shift)
            reach(std::integral_constant<int, 1>{});
        else
            reach(std::integral_constant<int, 0>{});
    }
    mark(1);
    if (c) {
        // join: segmented scans, forward (text order) and backward (reversed),
        // both directions in each launch; up the levels composing groups of
        // 64 items, then down applying the prefix maps
        auto u64p = [&](int k) { return reinterpret_cast<uint64_t *>(ptr(k)); };
        std::vector<ScanPair> lv(TL + 1);
        for (size_t l = 0; l <= TL; ++l)
            for (int d = 0; d < 2; ++d) {
                ScanLevel &x = lv[l].L[d];
                x.N = jl[l];
                x.level0 = l == 0;
                if (l == 0) {
                    x.rows = d == 0 ? jb.Mf : jb.MbR;
                    x.nx = d == 0 ? jb.nxf : jb.nxb;
                    x.cst = d == 0 ? jb.rsf : jb.rsb;
                    x.cv = nullptr;
                } else {
                    x.rows = u64p(jrows[d][l]);
                    x.nx = reinterpret_cast<const uint16_t *>(ptr(jnx[d][l]));
                    x.cst = ptr(jisc[d][l]);
                    x.cv = u64p(jcv[d][l]);
                }
            }
        const size_t grp_lds = size_t(2) * 64 * E * 8;
        const uint32_t ndir = recog ? 1u : 2u;    // the recogniser joins forward only
        for (size_t l = 0; l < TL; ++l) {
            ScanOut o{};
            for (int d = 0; d < 2; ++d) {
                o.rows[d] = u64p(jrows[d][l + 1]);
                o.nx[d] = reinterpret_cast<uint16_t *>(ptr(jnx[d][l + 1]));
                o.cst[d] = ptr(jisc[d][l + 1]);
                o.cv[d] = u64p(jcv[d][l + 1]);
                o.prow[d] = u64p(jprow[d][l]);
                o.pcst[d] = ptr(jpcst[d][l]);
                o.pcv[d] = u64p(jpcv[d][l]);
            }
            if (EW == 1)
                hipLaunchKernelGGL(k_compose, dim3(jl[l + 1], ndir), dim3(64), grp_lds, stream, lv[l], o, E);
            else
                hipLaunchKernelGGL(k_compose_wide, dim3(jl[l + 1], ndir), dim3(64), 2 * EW * 8, stream, lv[l], o, E,
                                   EW);
        }
        for (size_t l = TL; l-- > 0;) {
            ScanPrefix pf{};
            for (int d = 0; d < 2; ++d) {
                pf.prow[d] = u64p(jprow[d][l]);
                pf.pcst[d] = ptr(jpcst[d][l]);
                pf.pcv[d] = u64p(jpcv[d][l]);
                pf.pvec[d] = l + 1 < TL ? u64p(jvec[d][l + 1]) : nullptr;
                if (l == 0) {
                    pf.vin[d] = d == 0 ? jb.fin : jb.bin;
                    pf.vout[d] = d == 0 ? jb.fout : jb.bout;
                } else {
                    pf.vin[d] = u64p(jvec[d][l]);
                    pf.vout[d] = nullptr;
                }
            }
            if (EW == 1)
                hipLaunchKernelGGL(k_expand, dim3((jl[l] + 255) / 256, ndir), dim3(256), 0, stream, lv[l], pf, E);
            else
                hipLaunchKernelGGL(k_expand_wide, dim3((jl[l] + 255) / 256, ndir), dim3(256), 256 * EW * 8, stream,
                                   lv[l], pf, E, EW);
        }
    }
    mark(2);
    if (c && !recog) hipLaunchKernelGGL(k_starts, dim3(blocks), dim3(256), 0, stream, ts, jb);
    mark(3);

    // build & merge: transition tables and bit sets in LDS when they fit
    const size_t tab_lds = (512 + (size_t(tb.nf) + tb.nr) * tb.C * 2 + 15) & ~size_t(15);
    const size_t bits_lds = ((size_t(tb.nf) + tb.nr) * (W * 8 + 4) + 15) & ~size_t(15);   // sets, non-zero words
    if (c && !recog) {
        const bool fit_tab = lds && kStageBytes + tab_lds <= p->lds_limit;
        const bool fit_bits = fit_tab && kStageBytes + tab_lds + bits_lds <= p->lds_limit;
        const uint32_t bblocks = (c + kBuildThreads - 1) / kBuildThreads;
        // compact: the rank table goes after the tables when LDS has room and
        // it does not cost a resident block per CU
        const size_t tabs_end = kStageBytes + (fit_tab ? tab_lds : 0) + (fit_bits ? bits_lds : 0);
        const size_t rank_bytes = ((tb.rank_pq ? size_t(tb.NL) * tb.NL : tb.NL) * tb.nseg + 15) & ~size_t(15);
        const bool rank_fits = tabs_end + rank_bytes <= p->lds_limit &&
                               kLdsPerCu / (tabs_end + rank_bytes) == kLdsPerCu / tabs_end;
        jb.rank_lds = jb.compact && lds && rank_fits ? static_cast<uint32_t>(tabs_end) : 0u;
        size_t bld_lds = tabs_end + (jb.rank_lds ? rank_bytes : 0);
        // tree count: the pair table after them, on the same terms
        const size_t pair_bytes =
            ((tb.pair_nib ? (size_t(tb.kfd) * tb.krd + 1) / 2 : size_t(tb.kfd) * tb.krd) + 15) & ~size_t(15);
        const bool pair_fits = pair_bytes && bld_lds + pair_bytes <= p->lds_limit &&
                               kLdsPerCu / (bld_lds + pair_bytes) == kLdsPerCu / bld_lds;
        jb.pair_lds = count && !tb.col_single && lds && pair_fits ? static_cast<uint32_t>(bld_lds) : 0u;
        if (jb.pair_lds) bld_lds += pair_bytes;
        auto launch = [&](auto compact) {
            constexpr bool CM = decltype(compact)::value;
            if (fit_bits)
                hipLaunchKernelGGL((k_build<true, true, CM>), dim3(bblocks), dim3(kBuildThreads), bld_lds, stream,
                                   tb, jb);
            else if (fit_tab)
                hipLaunchKernelGGL((k_build<true, false, CM>), dim3(bblocks), dim3(kBuildThreads), bld_lds, stream,
                                   tb, jb);
            else
                hipLaunchKernelGGL((k_build<false, false, CM>), dim3(bblocks), dim3(kBuildThreads), bld_lds, stream,
                                   tb, jb);
        };
        if (jb.compact) launch(std::true_type{});
        else launch(std::false_type{});
    }
    mark(4);
    // tree count: the marked runs (k_build marked them and multiplied in the
    // one-column runs).  The deferred chunks, pieces and long runs are known on
    // the device only: their kernels loop over grids of a fixed size.
    if (count && c && !tb.col_single) {
        const uint64_t nwins = uint64_t(c) * (s / 64);
        hipLaunchKernelGGL(k_count_runs, dim3(static_cast<uint32_t>((nwins + kRunThreads - 1) / kRunThreads)),
                           dim3(kRunThreads), 0, stream, tb, jb);
        const uint32_t sgrid = static_cast<uint32_t>(
            std::min<uint64_t>((uint64_t(jb.cap_sruns) + kShortThreads - 1) / kShortThreads, 2048));
        const size_t fol_bytes = jb.fol_lds ? size_t(tb.nseg) * tb.W * 8 : 0;
        // FolSeg rows of at most four words are loaded once per segment.  A
        // wide count runs the first queue with kTV2 vectors at once (the
        // second queue then stays empty).
        using ShortKernel = void (*)(Tabs, Job);
        const ShortKernel first = tb.W == 1 ? k_count_short<kTV, false, 1>
                                  : tb.W == 2 ? k_count_short<kTV, false, 2>
                                  : tb.W <= 4 ? k_count_short<kTV, false, 4>
                                              : k_count_short<kTV, false, 0>;
        const ShortKernel wide = tb.W == 1 ? k_count_short<kTV2, false, 1>
                                 : tb.W == 2 ? k_count_short<kTV2, false, 2>
                                 : tb.W <= 4 ? k_count_short<kTV2, false, 4>
                                             : k_count_short<kTV2, false, 0>;
        const ShortKernel second = tb.W == 1 ? k_count_short<kTV2, true, 1>
                                   : tb.W == 2 ? k_count_short<kTV2, true, 2>
                                   : tb.W <= 4 ? k_count_short<kTV2, true, 4>
                                               : k_count_short<kTV2, true, 0>;
        if (flags & SLPF_PARSE_WIDE_COUNT) {
            hipLaunchKernelGGL(wide, dim3(std::max<uint32_t>(sgrid / 4, 1)), dim3(kShortThreads), fol_bytes, stream,
                               tb, jb);
        } else {
            hipLaunchKernelGGL(first, dim3(std::max<uint32_t>(sgrid, 1)), dim3(kShortThreads), fol_bytes, stream, tb,
                               jb);
            hipLaunchKernelGGL(second, dim3(std::max<uint32_t>(sgrid / 4, 1)), dim3(kShortThreads), fol_bytes, stream,
                               tb, jb);
        }
        const uint32_t wgrid = std::min<uint32_t>(c, 2048);
        hipLaunchKernelGGL(k_count_defer, dim3(wgrid), dim3(64), 0, stream, tb, jb);
        hipLaunchKernelGGL(k_count_pieces, dim3(wgrid), dim3(64), 0, stream, tb, jb);
        hipLaunchKernelGGL(k_count_chain, dim3(std::min<uint32_t>(c, 1024)), dim3(64), 0, stream, jb);
    }
    hipLaunchKernelGGL(k_text_scalars, dim3(nt), dim3(kScalarThreads), 0, stream, tb, jb, recog ? 2 : count ? 1 : 0);
    mark(5);
    if (ev_err != hipSuccess) return SLPF_E_ARG;
    return hip_ok(hipGetLastError());
}

slpf_status check_item(const slpf_parser *p, const uint8_t *text, uint64_t n, const slpf_forest *forest,
                       uint32_t flags) {
    if (!forest || !forest->scalars_dev) return SLPF_E_ARG;
    if (n && !text) return SLPF_E_ARG;
    if (reinterpret_cast<uintptr_t>(text) % 16 != 0) return SLPF_E_ARG;
    if (flags & SLPF_PARSE_RECOGNIZE) return SLPF_OK;   // no column is written
    if (!forest->columns_dev) return SLPF_E_ARG;
    const uint64_t need = (flags & SLPF_PARSE_COMPACT) ? slpf_compact_bytes(n) : slpf_forest_bytes(p, n);
    if (forest->capacity_bytes < need) return SLPF_E_CAPACITY;
    return SLPF_OK;
}

}  // namespace

extern "C" {

slpf_status slpf_parse(const slpf_parser *cp, const uint8_t *text, uint64_t n, const slpf_parse_opts *opts,
                       const slpf_forest *forest, void *hip_stream) {
    slpf_parser *p = const_cast<slpf_parser *>(cp);
    if (!p || p->host_only) return SLPF_E_ARG;
    if (opts && opts->struct_size != sizeof(slpf_parse_opts)) return SLPF_E_ARG;
    if (opts && opts->chunk_bytes && (opts->chunk_bytes % 64 != 0)) return SLPF_E_ARG;
    slpf_status st = check_item(p, text, n, forest, opts ? opts->flags : 0u);
    if (st != SLPF_OK) return st;
    slpf_text item{text, n, *forest};
    return run_job(p, &item, 1, opts, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

// ------------------------------------------------- parse without allocation
// The workspace of slpf_parse_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  In host code `scratch` only names
// the symbol; its device address on each GPU comes from hipGetSymbolAddress
// (taken once per device, with that device current) and only that address
// is passed to kernels.
namespace {

constexpr size_t kNoAllocScratchBytes = 128u << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the device must be current).
slpf_status scratch_on(int device, uint8_t **out) {
    if (device < 0 || device >= kMaxDevices) return SLPF_E_ARG;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SLPF_E_DEVICE;
        g_scratch_ptr[device] = static_cast<uint8_t *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return SLPF_OK;
}

}  // namespace

extern "C" {

slpf_status slpf_parse_noalloc(const slpf_parser *cp, const uint8_t *text, uint64_t n, const slpf_parse_opts *opts,
                               const slpf_forest *forest, void *hip_stream) {
    slpf_parser *p = const_cast<slpf_parser *>(cp);
    if (!p || p->host_only) return SLPF_E_ARG;
    if (opts && opts->struct_size != sizeof(slpf_parse_opts)) return SLPF_E_ARG;
    if (opts && opts->chunk_bytes && (opts->chunk_bytes % 64 != 0)) return SLPF_E_ARG;
    slpf_status st = check_item(p, text, n, forest, opts ? opts->flags : 0u);
    if (st != SLPF_OK) return st;
    if (hipSetDevice(p->device) != hipSuccess) return SLPF_E_DEVICE;
    uint8_t *ws = nullptr;
    st = scratch_on(p->device, &ws);
    if (st != SLPF_OK) return st;
    slpf_text item{text, n, *forest};
    return run_job(p, &item, 1, opts, static_cast<hipStream_t>(hip_stream), ws, kNoAllocScratchBytes);
}

slpf_status slpf_parse_texts(const slpf_parser *cp, const slpf_text *items, size_t count, const slpf_parse_opts *opts,
                             void *hip_stream) {
    slpf_parser *p = const_cast<slpf_parser *>(cp);
    if (!p || p->host_only || (!items && count)) return SLPF_E_ARG;
    if (opts && opts->struct_size != sizeof(slpf_parse_opts)) return SLPF_E_ARG;
    if (opts && opts->chunk_bytes && (opts->chunk_bytes % 64 != 0)) return SLPF_E_ARG;
    if (count == 0) return SLPF_OK;
    if (count > 0x7fffffffull) return SLPF_E_ARG;
    for (size_t t = 0; t < count; ++t) {
        slpf_status st = check_item(p, items[t].text_dev, items[t].n, &items[t].out, opts ? opts->flags : 0u);
        if (st != SLPF_OK) return st;
    }
    return run_job(p, items, count, opts, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

// ------------------------------------------------ batches over many parsers
// The jobs of one slpf_parse_batch call run on library-owned streams of the
// device, forked from and joined back into the caller's stream.  A parser
// always uses the same one (its jobs keep one work area per stream).
namespace {

constexpr int kBatchStreams = 4;

struct BatchStreams {
    std::mutex mu;
    bool made = false;
    hipStream_t s[kBatchStreams] = {};
    hipEvent_t fork = nullptr, done[kBatchStreams] = {};
    std::unordered_map<const slpf_parser *, int> home;
};

BatchStreams g_batch[kMaxDevices];

}  // namespace

extern "C" {

slpf_status slpf_parse_batch(const slpf_item *items, size_t count, const slpf_parse_opts *opts, void *hip_stream) {
    if (!items && count) return SLPF_E_ARG;
    if (opts && opts->struct_size != sizeof(slpf_parse_opts)) return SLPF_E_ARG;
    if (opts && opts->chunk_bytes && (opts->chunk_bytes % 64 != 0)) return SLPF_E_ARG;
    if (opts && opts->trace_dev) return SLPF_E_ARG;
    if (count == 0) return SLPF_OK;
    if (count > 0x7fffffffull) return SLPF_E_ARG;
    const uint32_t flags = opts ? opts->flags : 0u;
    int dev = -1;
    std::vector<const slpf_parser *> order;
    std::unordered_map<const slpf_parser *, std::vector<slpf_text>> groups;
    for (size_t t = 0; t < count; ++t) {
        const slpf_parser *p = items[t].p;
        if (!p || p->host_only) return SLPF_E_ARG;
        if (dev < 0) dev = p->device;
        if (p->device != dev || dev >= kMaxDevices) return SLPF_E_ARG;
        slpf_status st = check_item(p, items[t].text_dev, items[t].n, &items[t].out, flags);
        if (st != SLPF_OK) return st;
        auto &g = groups[p];
        if (g.empty()) order.push_back(p);
        g.push_back(slpf_text{items[t].text_dev, items[t].n, items[t].out});
    }
    if (hipSetDevice(dev) != hipSuccess) return SLPF_E_DEVICE;
    hipStream_t caller = static_cast<hipStream_t>(hip_stream);
    auto job_opts = [&](const slpf_parser *p) {
        slpf_parse_opts o{};
        if (opts) o = *opts;
        o.struct_size = sizeof(slpf_parse_opts);
        if (o.chunk_bytes == 0 && p->tuned_chunk) {
            o.chunk_bytes = p->tuned_chunk;
            o.flags |= p->tuned_flags;
        }
        o.events = nullptr;
        o.num_events = 0;
        return o;
    };
    if (order.size() == 1) {
        const slpf_parse_opts o = job_opts(order[0]);
        auto &g = groups[order[0]];
        return run_job(const_cast<slpf_parser *>(order[0]), g.data(), g.size(), &o, caller);
    }
    BatchStreams &bs = g_batch[dev];
    std::lock_guard<std::mutex> lock(bs.mu);
    if (!bs.made) {
        for (int k = 0; k < kBatchStreams; ++k)
            if (hipStreamCreateWithFlags(&bs.s[k], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&bs.done[k], hipEventDisableTiming) != hipSuccess)
                return SLPF_E_DEVICE;
        if (hipEventCreateWithFlags(&bs.fork, hipEventDisableTiming) != hipSuccess) return SLPF_E_DEVICE;
        bs.made = true;
    }
    if (hipEventRecord(bs.fork, caller) != hipSuccess) return SLPF_E_DEVICE;
    bool used[kBatchStreams] = {};
    slpf_status first_err = SLPF_OK;
    for (const slpf_parser *p : order) {
        auto it = bs.home.find(p);
        if (it == bs.home.end()) it = bs.home.emplace(p, static_cast<int>(bs.home.size() % kBatchStreams)).first;
        const int k = it->second;
        if (!used[k]) {
            if (hipStreamWaitEvent(bs.s[k], bs.fork, 0) != hipSuccess) {
                first_err = SLPF_E_DEVICE;
                break;
            }
            used[k] = true;
        }
        const slpf_parse_opts o = job_opts(p);
        auto &g = groups[p];
        const slpf_status st = run_job(const_cast<slpf_parser *>(p), g.data(), g.size(), &o, bs.s[k]);
        if (st != SLPF_OK) {
            first_err = st;
            break;
        }
    }
    for (int k = 0; k < kBatchStreams; ++k) {
        if (!used[k]) continue;
        if (hipEventRecord(bs.done[k], bs.s[k]) != hipSuccess || hipStreamWaitEvent(caller, bs.done[k], 0) != hipSuccess)
            if (first_err == SLPF_OK) first_err = SLPF_E_DEVICE;
    }
    return first_err;
}

slpf_status slpf_parser_trim(const slpf_parser *cp, void *hip_stream) {
    slpf_parser *p = const_cast<slpf_parser *>(cp);
    if (!p) return SLPF_E_ARG;
    std::lock_guard<std::mutex> g(p->mu);
    auto it = p->ws.find(static_cast<hipStream_t>(hip_stream));
    if (it == p->ws.end()) return SLPF_OK;
    Workspace &w = it->second;
    if (hipSetDevice(p->device) != hipSuccess) return SLPF_E_DEVICE;
    if (hipStreamSynchronize(it->first) != hipSuccess) return SLPF_E_DEVICE;
    if (w.copied) (void)hipEventDestroy(w.copied);
    if (w.base) (void)hipFree(w.base);
    if (w.pinned) (void)hipHostFree(w.pinned);
    p->ws.erase(it);
    return SLPF_OK;
}

slpf_status slpf_tune(const slpf_parser *cp, const slpf_text *items, size_t count, uint32_t flags,
                      slpf_parse_opts *best, float *best_ms, void *hip_stream) {
    slpf_parser *p = const_cast<slpf_parser *>(cp);
    if (!p || p->host_only || !best || best->struct_size != sizeof(slpf_parse_opts) || !items || !count)
        return SLPF_E_ARG;
    flags &= ~static_cast<uint32_t>(SLPF_PARSE_FORCE_L2);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return SLPF_E_DEVICE;
    }
    slpf_status st = SLPF_OK;
    float best_t = -1.0f;
    uint32_t best_chunk = 0, best_flags = flags;
    flags &= ~static_cast<uint32_t>(SLPF_PARSE_WIDE_COUNT);
    const uint32_t chunks[] = {256, 512, 1024, 2048, 4096};
    const int nplace = p->placement == 0 ? 2 : 1;    // LDS tables and, if they fit, L2 as well
    // the wide count too, when the texts' trees are counted in runs
    const bool counted = !(flags & (SLPF_PARSE_NO_COUNT | SLPF_PARSE_RECOGNIZE)) && !p->col_single;
    const int nwide = counted ? 2 : 1;
    for (uint32_t k : chunks) {
        for (int cand = 0; cand < nplace * nwide && st == SLPF_OK; ++cand) {
            const int pl = cand % nplace, wc = cand / nplace;
            slpf_parse_opts o{};
            o.struct_size = sizeof(o);
            o.chunk_bytes = k;
            o.flags = flags | (pl ? SLPF_PARSE_FORCE_L2 : 0u) | (wc ? SLPF_PARSE_WIDE_COUNT : 0u);
            // one untimed run (workspace growth, caches), one timed run
            st = slpf_parse_texts(p, items, count, &o, stream);
            if (st != SLPF_OK) break;
            if (hipEventRecord(e0, stream) != hipSuccess) st = SLPF_E_DEVICE;
            if (st == SLPF_OK) st = slpf_parse_texts(p, items, count, &o, stream);
            if (st == SLPF_OK && hipEventRecord(e1, stream) != hipSuccess) st = SLPF_E_DEVICE;
            if (st == SLPF_OK && hipEventSynchronize(e1) != hipSuccess) st = SLPF_E_DEVICE;
            float ms = 0;
            if (st == SLPF_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = SLPF_E_DEVICE;
            if (st == SLPF_OK && (best_t < 0 || ms < best_t)) {
                best_t = ms;
                best_chunk = k;
                best_flags = o.flags;
            }
        }
        if (st != SLPF_OK) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != SLPF_OK) return st;
    best->chunk_bytes = best_chunk;
    best->flags = best_flags;
    if (best_ms) *best_ms = best_t;
    p->tuned_chunk = best_chunk;
    p->tuned_flags = best_flags & (SLPF_PARSE_FORCE_L2 | SLPF_PARSE_WIDE_COUNT);
    return SLPF_OK;
}

}  // extern "C"

// ------------------------------------------------------------ match extraction
// Match extraction over a clean SLPF (Sect. 4, "Other functions of the tool",
// Match extraction: getMatches).
//
// A match of group g (the operator node numbered g) is a pair (start, end)
// of text positions such that some syntax tree has "g(" at position start
// and its matching ")g" at position end.  In the clean SLPF every local
// path extends to a whole tree (each segment lies on one), so the matches
// starting at column r are found by a walk: from the segments of C_r whose
// last g-symbol is "g(", follow the arcs (followers present in the next
// column) through segments without g-symbols, and every column e where a
// segment whose first g-symbol is ")g" is reached gives (r, e).  A segment
// holding "g( .. )g" gives the empty match (r, r).  Group g cannot open
// inside itself, so no other g-symbol can appear on such a path.
//
// Pass 1 flags the start columns, a device select lists them in order; one
// wavefront per start column walks and counts its matches; an exclusive
// scan gives each start its output offset; the second walk writes the pairs,
// so they come out sorted by (start, end).
namespace slpf {
namespace {

__global__ __launch_bounds__(256) void k_match_flags(Tabs tb, const uint64_t *cols, uint64_t n, uint32_t g,
                                                     uint8_t *flags) {
    const uint64_t r = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r > n) return;
    const uint32_t W = tb.W;
    const uint64_t *m = tb.gmask + static_cast<uint64_t>(g) * 3 * W;
    uint64_t any = 0;
    for (uint32_t w = 0; w < W; ++w) any |= cols[r * W + w] & (m[w] | m[2 * W + w]);
    flags[r] = any != 0 ? 1 : 0;
}

// One wavefront per start column; lane w holds word w of the walk's frontier.
template <bool WRITE>
__global__ __launch_bounds__(64) void k_match_walk(Tabs tb, const uint64_t *cols, uint64_t n, uint32_t g,
                                                   const uint64_t *starts, const int *nstarts, uint64_t *counts,
                                                   const uint64_t *offs, uint64_t *pairs, uint64_t cap) {
    const uint32_t lane = threadIdx.x, W = tb.W;
    const bool on = lane < W;
    const uint64_t *m = tb.gmask + static_cast<uint64_t>(g) * 3 * W;
    const uint64_t op = on ? m[lane] : 0ull, cl = on ? m[W + lane] : 0ull, oc = on ? m[2 * W + lane] : 0ull;
    const int ns = *nstarts;
    for (int item = blockIdx.x; item < ns; item += gridDim.x) {
        const uint64_t r = starts[item];
        uint64_t pos = WRITE ? offs[item] : 0ull;
        auto emit = [&](uint64_t e) {
            if (WRITE && lane == 0 && pos < cap) {
                pairs[2 * pos] = r;
                pairs[2 * pos + 1] = e;
            }
            ++pos;
        };
        const uint64_t c0 = on ? cols[r * W + lane] : 0ull;
        if (__any((c0 & oc) != 0)) emit(r);                  // "g( .. )g" inside a segment
        uint64_t f = c0 & op;                                // g is open after these segments
        uint64_t c = r;
        while (c < n && __any(f != 0)) {
            ++c;
            uint64_t nf = 0;
            for (uint32_t w = 0; w < W; ++w) {
                for (uint64_t fw = readlane_u64(f, static_cast<int>(w)); fw; fw &= fw - 1) {
                    const uint64_t sg = w * 64ull + static_cast<uint64_t>(__builtin_ctzll(fw));
                    if (on) nf |= tb.folseg[sg * W + lane];
                }
            }
            if (on) nf &= cols[c * W + lane];
            if (__any((nf & cl) != 0)) emit(c);
            f = nf & ~cl;
        }
        if (!WRITE && lane == 0) counts[item] = pos;
    }
}

__global__ void k_match_fill(uint64_t *a, uint64_t n) {
    const uint64_t k = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) a[k] = 0;
}

__global__ void k_match_total(const uint64_t *offs, const uint64_t *counts, const int *ns, uint64_t *total) {
    const int k = *ns;
    *total = k > 0 ? offs[k - 1] + counts[k - 1] : 0ull;
}

}  // namespace
}  // namespace slpf

extern "C" slpf_status slpf_get_matches(const slpf_parser *p, const uint64_t *columns_dev, uint64_t n, uint32_t group,
                                        uint64_t *pairs_dev, uint64_t capacity, uint64_t *num_matches,
                                        void *hip_stream) {
    using namespace slpf;
    if (!p || p->host_only || !columns_dev || !num_matches || (capacity && !pairs_dev)) return SLPF_E_ARG;
    const Tabs tb = p->tabs;
    const int device = p->device;
    if (group == 0 || group >= tb.ngroups) return SLPF_E_ARG;
    if (n >= static_cast<uint64_t>(INT_MAX)) return SLPF_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return SLPF_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const uint64_t N = n + 1;
    const int NI = static_cast<int>(N);
    // work buffers: flags, starts, their number, counts, offsets, total
    size_t sel_bytes = 0, scan_bytes = 0;
    hipcub::CountingInputIterator<uint64_t> idx(0);
    if (hipcub::DeviceSelect::Flagged(nullptr, sel_bytes, idx, static_cast<uint8_t *>(nullptr),
                                      static_cast<uint64_t *>(nullptr), static_cast<int *>(nullptr), NI, st) !=
            hipSuccess ||
        hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, static_cast<uint64_t *>(nullptr),
                                         static_cast<uint64_t *>(nullptr), NI, st) != hipSuccess)
        return SLPF_E_DEVICE;
    const size_t tmp_bytes = sel_bytes > scan_bytes ? sel_bytes : scan_bytes;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_flags = 0, o_starts = o_flags + al(N), o_counts = o_starts + al(N * 8), o_offs = o_counts + al(N * 8),
                 o_ns = o_offs + al(N * 8), o_total = o_ns + 256, o_tmp = o_total + 256, bytes = o_tmp + al(tmp_bytes);
    uint8_t *buf = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&buf), bytes) != hipSuccess) return SLPF_E_NOMEM;
    uint8_t *flags = buf + o_flags;
    uint64_t *starts = reinterpret_cast<uint64_t *>(buf + o_starts);
    uint64_t *counts = reinterpret_cast<uint64_t *>(buf + o_counts);
    uint64_t *offs = reinterpret_cast<uint64_t *>(buf + o_offs);
    int *ns = reinterpret_cast<int *>(buf + o_ns);
    uint64_t *total = reinterpret_cast<uint64_t *>(buf + o_total);
    void *tmp = buf + o_tmp;
    slpf_status status = SLPF_OK;
    uint64_t h_total = 0;
    const uint32_t blocks = static_cast<uint32_t>((N + 255) / 256);
    const uint32_t walkers = static_cast<uint32_t>(N < 4096 ? N : 4096);
    do {
        hipLaunchKernelGGL(k_match_flags, dim3(blocks), dim3(256), 0, st, tb, columns_dev, n, group, flags);
        hipLaunchKernelGGL(k_match_fill, dim3(blocks), dim3(256), 0, st, counts, N);
        size_t tb1 = tmp_bytes;
        if (hipcub::DeviceSelect::Flagged(tmp, tb1, idx, flags, starts, ns, NI, st) != hipSuccess) {
            status = SLPF_E_DEVICE;
            break;
        }
        hipLaunchKernelGGL(k_match_walk<false>, dim3(walkers), dim3(64), 0, st, tb, columns_dev, n, group, starts, ns,
                           counts, nullptr, nullptr, 0ull);
        size_t tb2 = tmp_bytes;
        if (hipcub::DeviceScan::ExclusiveSum(tmp, tb2, counts, offs, NI, st) != hipSuccess) {
            status = SLPF_E_DEVICE;
            break;
        }
        hipLaunchKernelGGL(k_match_total, dim3(1), dim3(1), 0, st, offs, counts, ns, total);
        if (hipMemcpyAsync(&h_total, total, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            status = SLPF_E_DEVICE;
            break;
        }
        if (h_total && capacity)
            hipLaunchKernelGGL(k_match_walk<true>, dim3(walkers), dim3(64), 0, st, tb, columns_dev, n, group, starts,
                               ns, counts, offs, pairs_dev, capacity);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) status = SLPF_E_DEVICE;
    } while (false);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (status != SLPF_OK) return status;
    *num_matches = h_total;
    return h_total > capacity ? SLPF_E_CAPACITY : SLPF_OK;
}

// ------------------------------------------------------------ child extraction
// The children of a match (Sect. 4, "Other functions of the tool", Match
// extraction: getChildren).
//
// Given a match (i, j) of node g, the trees that hold g over (i, j) are the
// paths of the clean SLPF that leave column i through a segment whose last
// g-symbol is "g(", cross the columns strictly between without closing g,
// and enter column j through a segment whose first g-symbol is ")g" (for
// i = j: the segments holding "g( .. )g").  This sub-forest is cut from the
// columns first; the children of g are then read inside it, each segment
// restricted to the part of its symbols that lies inside g's occurrence
// (after its last "g(" at column i, before its first ")g" at column j).
//
// Cutting the sub-forest is chunk-parallel: a column of the clean SLPF that
// holds one segment lies on every tree, so when (i, j) is a match that
// segment lies on the sub-forest.  Such columns split [i, j] into stretches;
// one wavefront per stretch walks forward from the stretch's first column
// (the segments allowed there) and back from its last, and the stretches
// need nothing from each other.  The match exists iff every stretch's
// forward walk reaches its last column.
//
// A child k of g (a node whose parent is g) has, per column a of the
// sub-forest:
//   an empty match (k, a, a) where a segment holds "k( )k" (adjacent among
//   its k-symbols) or the leaf "εk" inside g's part of it;
//   the one-byte match (k, a, a + 1) where a < j and the segment's
//   end-letter is the terminal k;
//   matches (k, a, e), e > a, walked from the segments whose last k-symbol
//   is "k(" through segments without k-symbols to those whose first
//   k-symbol is ")k", inside the sub-forest.  (At columns i and j these
//   whole-segment tests agree with the tests on g's part: a k-symbol
//   outside it belongs to another occurrence of g, which can only be an
//   earlier one closing at i or a later one opening at j.)
// The per-child masks depend on the column's place in [i, j] and are built
// on the host for the call.  The (child, column) items are flagged, listed
// in order, walked once to count and once to write, as in match extraction,
// so the triples come out sorted by (child, start, end).
namespace slpf {
namespace {

constexpr int kChildMasks = 7;   // per child: op, cl, term, empty at first / interior / last / both

// Cut columns of [start, start + L): the two ends and every column with at
// most one segment.
__global__ __launch_bounds__(256) void k_cf_cuts(const uint64_t *cols, uint32_t W, uint64_t start, uint64_t L,
                                                 uint8_t *flags) {
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= L) return;
    const uint64_t *c = cols + (start + t) * W;
    int pc = 0;
    for (uint32_t w = 0; w < W && pc < 2; ++w) pc += __builtin_popcountll(c[w]);
    flags[t] = (t == 0 || t == L - 1 || pc <= 1) ? 1 : 0;
}

// One wavefront per stretch [cuts[s], cuts[s+1]]; lane w holds word w.
// sub[t] receives the sub-forest's column start + t; *fail is set when a
// stretch's forward walk dies (then (start, start + L - 1) is no match).
__global__ __launch_bounds__(64) void k_cf_stretch(Tabs tb, const uint64_t *cols, uint64_t start, uint64_t L,
                                                   uint32_t g, const uint64_t *cuts, const int *ncuts,
                                                   uint64_t *sub, uint32_t *fail) {
    const uint32_t lane = threadIdx.x, W = tb.W;
    const bool on = lane < W;
    const uint64_t *m = tb.gmask + static_cast<uint64_t>(g) * 3 * W;
    const uint64_t op = on ? m[lane] : 0ull, cl = on ? m[W + lane] : 0ull, oc = on ? m[2 * W + lane] : 0ull;
    if (L == 1) {
        if (blockIdx.x != 0) return;
        const uint64_t f = on ? cols[start * W + lane] & oc : 0ull;
        if (on) sub[lane] = f;
        if (!__any(f != 0) && lane == 0) *fail = 1u;
        return;
    }
    const int nst = *ncuts - 1;
    for (int s = blockIdx.x; s < nst; s += gridDim.x) {
        const uint64_t u = cuts[s], v = cuts[s + 1];
        uint64_t f = on ? cols[(start + u) * W + lane] : 0ull;
        if (u == 0) {
            f &= op;
            if (on) sub[lane] = f;
        }
        uint64_t c = u;
        while (c < v && __any(f != 0)) {
            ++c;
            uint64_t nf = 0;
            for (uint32_t w = 0; w < W; ++w)
                for (uint64_t fw = readlane_u64(f, static_cast<int>(w)); fw; fw &= fw - 1) {
                    const uint64_t sg = w * 64ull + static_cast<uint64_t>(__builtin_ctzll(fw));
                    if (on) nf |= tb.folseg[sg * W + lane];
                }
            if (on) nf &= cols[(start + c) * W + lane] & (c == L - 1 ? cl : ~cl);
            if (on) sub[c * W + lane] = nf;
            f = nf;
        }
        if (c < v || !__any(f != 0)) {
            if (lane == 0) *fail = 1u;
            continue;
        }
        // back from column v: keep the segments some kept follower follows
        uint64_t b = f;
        const uint64_t lo = u == 0 ? 0 : u + 1;     // an interior cut is written by the stretch ending there
        for (uint64_t cc = v; cc > lo; --cc) {
            const uint64_t col = cc - 1;
            uint64_t pb = 0;
            for (uint32_t w = 0; w < W; ++w)
                for (uint64_t bw = readlane_u64(b, static_cast<int>(w)); bw; bw &= bw - 1) {
                    const uint64_t sg = w * 64ull + static_cast<uint64_t>(__builtin_ctzll(bw));
                    if (on) pb |= tb.predseg[sg * W + lane];
                }
            uint64_t x = 0;
            if (on) {
                x = sub[col * W + lane] & pb;
                sub[col * W + lane] = x;
            }
            b = x;
        }
    }
}

__device__ __forceinline__ int child_role(uint64_t t, uint64_t L) {
    return L == 1 ? 6 : t == 0 ? 3 : t == L - 1 ? 5 : 4;
}

// Item q * L + t (child q, column start + t): flagged when the walk there
// emits anything.
__global__ __launch_bounds__(256) void k_ch_flags(const uint64_t *masks, uint32_t W, const uint64_t *sub, uint64_t L,
                                                  uint64_t N, const uint32_t *fail, uint8_t *flags) {
    const uint64_t item = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (item >= N) return;
    if (*fail) {
        flags[item] = 0;
        return;
    }
    const uint64_t q = item / L, t = item % L;
    const uint64_t *mk = masks + q * kChildMasks * W;
    const uint64_t *e = mk + static_cast<uint64_t>(child_role(t, L)) * W;
    const bool inner = t + 1 < L;
    uint64_t any = 0;
    for (uint32_t w = 0; w < W; ++w)
        any |= sub[t * W + w] & (e[w] | (inner ? mk[w] | mk[2 * W + w] : 0ull));
    flags[item] = any != 0 ? 1 : 0;
}

// One wavefront per listed item; lane w holds word w.
template <bool WRITE>
__global__ __launch_bounds__(64) void k_ch_walk(Tabs tb, const uint64_t *masks, const uint32_t *kids,
                                                const uint64_t *sub, uint64_t start, uint64_t L, const uint64_t *items,
                                                const int *nitems, uint64_t *counts, const uint64_t *offs,
                                                uint64_t *triples, uint64_t cap) {
    const uint32_t lane = threadIdx.x, W = tb.W;
    const bool on = lane < W;
    const int ni = *nitems;
    for (int it = blockIdx.x; it < ni; it += gridDim.x) {
        const uint64_t item = items[it], q = item / L, t = item % L;
        const uint64_t *mk = masks + q * kChildMasks * W;
        const uint64_t op = on ? mk[lane] : 0ull, cl = on ? mk[W + lane] : 0ull;
        const uint64_t term = on ? mk[2 * W + lane] : 0ull;
        const uint64_t em = on ? mk[static_cast<uint64_t>(child_role(t, L)) * W + lane] : 0ull;
        const uint64_t k = kids[q];
        uint64_t pos = WRITE ? offs[it] : 0ull;
        auto emit = [&](uint64_t e) {
            if (WRITE && lane == 0 && pos < cap) {
                triples[3 * pos] = k;
                triples[3 * pos + 1] = start + t;
                triples[3 * pos + 2] = start + e;
            }
            ++pos;
        };
        const uint64_t s0 = on ? sub[t * W + lane] : 0ull;
        if (__any((s0 & em) != 0)) emit(t);
        if (t + 1 < L) {
            if (__any((s0 & term) != 0)) emit(t + 1);
            uint64_t f = s0 & op;
            uint64_t c = t;
            while (c + 1 < L && __any(f != 0)) {
                ++c;
                uint64_t nf = 0;
                for (uint32_t w = 0; w < W; ++w)
                    for (uint64_t fw = readlane_u64(f, static_cast<int>(w)); fw; fw &= fw - 1) {
                        const uint64_t sg = w * 64ull + static_cast<uint64_t>(__builtin_ctzll(fw));
                        if (on) nf |= tb.folseg[sg * W + lane];
                    }
                if (on) nf &= sub[c * W + lane];
                if (__any((nf & cl) != 0)) emit(c);
                f = nf & ~cl;
            }
        }
        if (!WRITE && lane == 0) counts[it] = pos;
    }
}

// Host: the per-child masks of a call (kChildMasks x W words per child).
void child_masks(const HostAutomaton &A, uint32_t g, const std::vector<uint32_t> &kids, std::vector<uint64_t> &out) {
    const uint32_t W = A.W, nk = static_cast<uint32_t>(kids.size());
    out.assign(static_cast<size_t>(nk) * kChildMasks * W, 0);
    std::vector<int> idx(A.ngroups, -1);
    for (uint32_t q = 0; q < nk; ++q) {
        idx[kids[q]] = static_cast<int>(q);
        const uint64_t *gm = A.gmask.data() + static_cast<size_t>(kids[q]) * 3 * W;
        std::copy(gm, gm + 2 * W, out.begin() + static_cast<size_t>(q) * kChildMasks * W);   // op, cl
    }
    std::vector<int8_t> prev(nk, -1);
    std::vector<uint32_t> touched;
    for (uint32_t s = 0; s < A.nseg; ++s) {
        const int32_t *y = A.sym_code.data() + A.sym_off[s];
        const int len = static_cast<int>(A.sym_off[s + 1] - A.sym_off[s]);
        const uint64_t bit = uint64_t(1) << (s & 63);
        const size_t word = s >> 6;
        auto set = [&](uint32_t q, int mask) { out[(static_cast<size_t>(q) * kChildMasks + mask) * W + word] |= bit; };
        int last_open = -1, first_close = -1, close_after = -1;
        for (int x = 0; x < len; ++x) {
            if (y[x] == static_cast<int32_t>(g * 4 + 0)) last_open = x;
            if (y[x] == static_cast<int32_t>(g * 4 + 2) && first_close < 0) first_close = x;
        }
        for (int x = last_open + 1; last_open >= 0 && x < len; ++x)
            if (y[x] == static_cast<int32_t>(g * 4 + 2)) {
                close_after = x;
                break;
            }
        // the end-letter is terminal k
        const int32_t e = y[len - 1];
        if ((e & 3) == 1 && A.node_kind[e >> 2] == 1 && idx[e >> 2] >= 0) set(static_cast<uint32_t>(idx[e >> 2]), 2);
        // empty children inside [lo, hi) for each place of the column
        auto empties = [&](int lo, int hi, int mask) {
            for (int x = lo; x < hi; ++x) {
                const int32_t num = y[x] >> 2, kind = y[x] & 3;
                if (kind == 3 || idx[num] < 0) continue;
                const uint32_t q = static_cast<uint32_t>(idx[num]);
                if (kind == 1) {
                    if (A.node_kind[num] == 2) set(q, mask);
                } else if (kind == 0) {
                    if (prev[q] < 0) touched.push_back(q);
                    prev[q] = 0;
                } else {
                    if (prev[q] == 0) set(q, mask);
                    if (prev[q] < 0) touched.push_back(q);
                    prev[q] = 2;
                }
            }
            for (uint32_t q : touched) prev[q] = -1;
            touched.clear();
        };
        if (last_open >= 0) empties(last_open + 1, len, 3);
        empties(0, len, 4);
        if (first_close >= 0) empties(0, first_close, 5);
        if (last_open >= 0 && close_after >= 0) empties(last_open + 1, close_after, 6);
    }
}

}  // namespace
}  // namespace slpf

extern "C" slpf_status slpf_get_children(const slpf_parser *p, const uint64_t *columns_dev, uint64_t n,
                                         uint32_t group, uint64_t start, uint64_t end, uint64_t *triples_dev,
                                         uint64_t capacity, uint64_t *num_children, void *hip_stream) {
    using namespace slpf;
    if (!p || p->host_only || !columns_dev || !num_children || (capacity && !triples_dev)) return SLPF_E_ARG;
    const HostAutomaton &A = p->A;
    const Tabs tb = p->tabs;
    if (group == 0 || group >= tb.ngroups || start > end || end > n) return SLPF_E_ARG;
    if (n >= static_cast<uint64_t>(INT_MAX)) return SLPF_E_ARG;
    std::vector<uint32_t> kids;
    for (uint32_t k = 1; k < A.ngroups; ++k)
        if (A.parent[k] == static_cast<int32_t>(group)) kids.push_back(k);
    *num_children = 0;
    if (kids.empty()) return SLPF_OK;                 // a leaf
    const uint64_t L = end - start + 1, nk = kids.size(), N = nk * L;
    if (N >= static_cast<uint64_t>(INT_MAX)) return SLPF_E_ARG;
    const uint32_t W = tb.W;
    std::vector<uint64_t> hmask;
    child_masks(A, group, kids, hmask);
    if (hipSetDevice(p->device) != hipSuccess) return SLPF_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int NI = static_cast<int>(N), LI = static_cast<int>(L);
    size_t sel_bytes = 0, sel2_bytes = 0, scan_bytes = 0;
    hipcub::CountingInputIterator<uint64_t> idx(0);
    if (hipcub::DeviceSelect::Flagged(nullptr, sel_bytes, idx, static_cast<uint8_t *>(nullptr),
                                      static_cast<uint64_t *>(nullptr), static_cast<int *>(nullptr), NI, st) !=
            hipSuccess ||
        hipcub::DeviceSelect::Flagged(nullptr, sel2_bytes, idx, static_cast<uint8_t *>(nullptr),
                                      static_cast<uint64_t *>(nullptr), static_cast<int *>(nullptr), LI, st) !=
            hipSuccess ||
        hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, static_cast<uint64_t *>(nullptr),
                                         static_cast<uint64_t *>(nullptr), NI, st) != hipSuccess)
        return SLPF_E_DEVICE;
    const size_t tmp_bytes = std::max(sel_bytes, std::max(sel2_bytes, scan_bytes));
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    // work buffers: child masks, child numbers, the sub-forest, cut flags and
    // list, item flags, list, counts, offsets, small counters, select/scan room
    const size_t o_mask = 0, o_kids = o_mask + al(hmask.size() * 8), o_sub = o_kids + al(nk * 4),
                 o_cflag = o_sub + al(L * W * 8), o_cuts = o_cflag + al(L), o_iflag = o_cuts + al(L * 8),
                 o_items = o_iflag + al(N), o_counts = o_items + al(N * 8), o_offs = o_counts + al(N * 8),
                 o_small = o_offs + al(N * 8), o_tmp = o_small + 256, bytes = o_tmp + al(tmp_bytes);
    uint8_t *buf = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&buf), bytes) != hipSuccess) return SLPF_E_NOMEM;
    uint64_t *masks = reinterpret_cast<uint64_t *>(buf + o_mask);
    uint32_t *kids_dev = reinterpret_cast<uint32_t *>(buf + o_kids);
    uint64_t *sub = reinterpret_cast<uint64_t *>(buf + o_sub);
    uint8_t *cflag = buf + o_cflag, *iflag = buf + o_iflag;
    uint64_t *cuts = reinterpret_cast<uint64_t *>(buf + o_cuts);
    uint64_t *items = reinterpret_cast<uint64_t *>(buf + o_items);
    uint64_t *counts = reinterpret_cast<uint64_t *>(buf + o_counts);
    uint64_t *offs = reinterpret_cast<uint64_t *>(buf + o_offs);
    uint64_t *total = reinterpret_cast<uint64_t *>(buf + o_small);
    int *ncuts = reinterpret_cast<int *>(buf + o_small + 8);
    int *nitems = reinterpret_cast<int *>(buf + o_small + 16);
    uint32_t *fail = reinterpret_cast<uint32_t *>(buf + o_small + 24);
    void *tmp = buf + o_tmp;
    slpf_status status = SLPF_OK;
    uint64_t h_total = 0;
    const uint32_t lblocks = static_cast<uint32_t>((L + 255) / 256), nblocks = static_cast<uint32_t>((N + 255) / 256);
    do {
        if (hipMemcpyAsync(masks, hmask.data(), hmask.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(kids_dev, kids.data(), nk * 4, hipMemcpyHostToDevice, st) != hipSuccess) {
            status = SLPF_E_DEVICE;
            break;
        }
        hipLaunchKernelGGL(k_match_fill, dim3(1), dim3(64), 0, st, total, 4);   // total, counters, fail
        hipLaunchKernelGGL(k_cf_cuts, dim3(lblocks), dim3(256), 0, st, columns_dev, W, start, L, cflag);
        size_t t1 = tmp_bytes;
        if (hipcub::DeviceSelect::Flagged(tmp, t1, idx, cflag, cuts, ncuts, LI, st) != hipSuccess) {
            status = SLPF_E_DEVICE;
            break;
        }
        const uint32_t swalk = static_cast<uint32_t>(std::min<uint64_t>(L, 4096));
        hipLaunchKernelGGL(k_cf_stretch, dim3(swalk), dim3(64), 0, st, tb, columns_dev, start, L, group, cuts, ncuts,
                           sub, fail);
        hipLaunchKernelGGL(k_ch_flags, dim3(nblocks), dim3(256), 0, st, masks, W, sub, L, N, fail, iflag);
        hipLaunchKernelGGL(k_match_fill, dim3(nblocks), dim3(256), 0, st, counts, N);
        size_t t2 = tmp_bytes;
        if (hipcub::DeviceSelect::Flagged(tmp, t2, idx, iflag, items, nitems, NI, st) != hipSuccess) {
            status = SLPF_E_DEVICE;
            break;
        }
        const uint32_t walkers = static_cast<uint32_t>(std::min<uint64_t>(N, 4096));
        hipLaunchKernelGGL(k_ch_walk<false>, dim3(walkers), dim3(64), 0, st, tb, masks, kids_dev, sub, start, L, items,
                           nitems, counts, nullptr, nullptr, 0ull);
        size_t t3 = tmp_bytes;
        if (hipcub::DeviceScan::ExclusiveSum(tmp, t3, counts, offs, NI, st) != hipSuccess) {
            status = SLPF_E_DEVICE;
            break;
        }
        hipLaunchKernelGGL(k_match_total, dim3(1), dim3(1), 0, st, offs, counts, nitems, total);
        if (hipMemcpyAsync(&h_total, total, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            status = SLPF_E_DEVICE;
            break;
        }
        if (h_total && capacity)
            hipLaunchKernelGGL(k_ch_walk<true>, dim3(walkers), dim3(64), 0, st, tb, masks, kids_dev, sub, start, L,
                               items, nitems, counts, offs, triples_dev, capacity);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) status = SLPF_E_DEVICE;
    } while (false);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (status != SLPF_OK) return status;
    *num_children = h_total;
    return h_total > capacity ? SLPF_E_CAPACITY : SLPF_OK;
}

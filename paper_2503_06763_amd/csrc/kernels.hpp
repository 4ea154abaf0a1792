// Device kernels of the SLPF parser for gfx950 (CDNA4, wave64).
//
// Work decomposition.  The text is cut into lane chunks of s bytes (s a
// multiple of 64, the last chunk shorter); one lane owns one chunk in every
// per-chunk kernel, so a wavefront covers 64 consecutive chunks.  Chunk i
// spans the columns P_i+1 .. P_{i+1} with P_i = min(i*s, n).
//
// Entry lists.  At the edge column P_b the clean column is a subset of
// X_b = X[class(x_{P_b}), class(x_{P_b+1})]: segments whose end-letter is
// the next byte and that follow some segment labelled with the previous byte
// (I at the text start, F at the text end).  Runs started from other
// segments die on the first byte, and J_b restricted to the labels of the
// next byte lies inside X_b, so speculating only from X_b reproduces the
// paper's R/J exactly while starting from the reduced (ME-DFA entry) set.
//
// Phases (Sect. 3.2):
//   k_reach  forward and backward ME-DFA runs from the singletons of X_i and
//            X_{i+1} over chunk i (Eq. reacher), deduplicated when runs meet;
//            results as end-state ids and as 64-bit masks over the entry list
//            at the far edge.
//   k_compose / k_scan_top / k_expand
//            the join (Eq. joiner) as a scan of Boolean maps between entry
//            lists: groups of 64 maps are composed per wavefront, the group
//            aggregates scanned, and the group-start vectors expanded back.
//   k_starts the join sets J, J^ at every edge and their DFA state ids
//            (set -> id by hashing; a set selected from one run is that
//            run's id), the accept flag.
//   k_build  fused builder & merger (Eq. builder, Eq. merger, Fig.
//            builders&merger): forward DFA run with a checkpoint every 64
//            bytes, then window by window backwards: recompute the window's
//            forward ids from its checkpoint, run the reverse DFA and write
//            the clean column bitsF[fwd] & bitsR[bwd] of every position.
//   k_count_runs / k_count_defer / k_count_pieces / k_count_chain / k_text_scalars (count.hpp)
//            the number of syntax trees modulo 2^64 and modulo 2^61 - 1:
//            every path through the clean SLPF passes through each singleton
//            column, so the count is the product over the maximal runs of
//            ambiguous columns of the paths through each run.  k_build
//            multiplies in the one-column runs inside a lane chunk (the
//            column's size, from a table over pairs of DFA states) and marks
//            the columns of every other run; the run kernels count the
//            marked runs from the written columns.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "slpf_internal.hpp"

namespace slpf {

struct Tabs {
    const uint16_t *classmap;   // 256
    const uint16_t *fdelta;     // nf x C
    const uint16_t *rdelta;     // nr x C
    const uint64_t *fbits;      // nf x W
    const uint64_t *rbits;      // nr x W
    const uint32_t *xoff;       // NL*NL + 1
    const uint16_t *xlist;
    const uint16_t *fsingle;    // per segment
    const uint16_t *rsingle;
    const uint32_t *fhash;
    const uint32_t *rhash;
    const uint64_t *folseg;     // nseg x W
    const uint16_t *fsole;      // per forward state: its only segment, or kNoSole
    const uint16_t *rsole;      // per backward state
    // offset form of the transition tables (present when off16): an entry is
    // the byte offset of the next state's row, the class map gives byte
    // offsets of the classes, so a step is one add and one lookup
    const uint16_t *fdo, *rdo, *cls2;
    const uint8_t *rankx;       // rank of a segment in X[p, q]: NL x nseg by previous class p (q is
                                // its end-letter's class), or NL x NL x nseg by (p, q) when rank_pq
    uint32_t rank_pq;
    const uint32_t *fnz, *rnz;  // per state: bit w set iff word w of its set is non-zero
    const uint16_t *seqids;     // 0, 1, 2, ..: DFA state m + 1 as entry m (all-DFA-states ablation)
    uint32_t dfa_f, dfa_r;      // forward / reverse DFA states (ids 1 .. dfa_f / dfa_r)
    const uint32_t *xoff_nb;    // entry lists filtered by the next byte only (ablation)
    const uint16_t *xlist_nb;
    uint32_t emax_nb;
    const uint64_t *gmask;      // match extraction: ngroups x 3 x W segment masks
    uint32_t ngroups;
    uint32_t col_single;        // reachable forward and reverse states share at most one segment
    // tree count: pairm[f * krd + b] = |bits_f(f) & bits_r(b)| (capped at 255)
    // for the forward states reachable from I (ids < kfd) and the reverse
    // states reachable from F (ids < krd); predseg[s] = the segments that s
    // follows (the transpose of folseg), nseg x W
    const uint8_t *pairm;
    uint32_t kfd, krd;
    // 1: pairm holds 4-bit entries, two per byte (low nibble first), with 15
    // standing for any size of 15 or more (used when the byte table is too big)
    uint32_t pair_nib;
    // arcs2[(f * krd + b) * C + c] = number of arcs between two adjacent clean
    // columns: the left one of forward state f, the right one of reverse state
    // b, the byte between them of class c (0xffff: unknown); null when large
    const uint16_t *arcs2;
    const uint64_t *predseg;
    uint32_t off16;
    uint32_t fhmask, rhmask;
    uint32_t C, W, NL;          // classes, words, C + 1
    uint32_t nf, nr;            // table sizes including id 0
    uint32_t fstart, rstart;    // ids of I and F
    uint32_t emax;
    uint32_t nseg;
    uint64_t wmagic;            // ceil(2^32 / W): e / W == (e * wmagic) >> 32 for e < 2^16
};

// A short run queued for k_count_short, in one word: columns lo_i + off ..
// lo_i + off + len - 1 of the text of lane chunk i (lo_i: the chunk's first
// byte); bits 0-9 len (0: a slot left unused), 10-32 off, 33-63 i.  Lane
// chunks of at most kMaxRunChunk bytes (longer ones queue nothing).
constexpr uint64_t kMaxRunChunk = 1ull << 22;
__host__ __device__ inline uint64_t short_run(uint32_t i, uint64_t off, uint32_t len) {
    return (static_cast<uint64_t>(i) << 33) | (off << 10) | len;
}

// A long run of marked columns r0 .. r1 of text t, cut into npc pieces
// (piece items pb .., matrix slots mb .. when npc > 1).
struct RunRec {
    uint64_t r0, r1;
    uint32_t t, pb, npc, mb;
};

struct Job {
    // texts: a job parses one or many texts with one parser; the lane chunks of
    // all texts form one index space, text t owning chunks tchunk0[t] ..
    // tchunk0[t+1]-1.  With one text the descriptor is carried in d0.
    uint32_t ntexts;
    const uint64_t *tdesc;      // [T][4]: text ptr, n, columns ptr, scalars ptr
    const uint32_t *tchunk0;    // [T+1]
    const uint32_t *tmap;       // [c] the text of each lane chunk (T > 1; filled by k_tmap first)
    uint64_t d0[4];
    uint64_t s;                 // lane chunk bytes
    uint32_t c;                 // lane chunks of all texts
    uint16_t *R, *Rh;           // [emax][c] end ids of the reach runs
    uint16_t *Rt;               // [emax][c] reach: ids of the runs part way
    uint16_t *Rm, *Rmh;         // [emax][c] ids of lane k's forward / backward runs at its fixed right
                                // edge (chunk-edge shifting; without it Rm is R and Rmh is unused)
    uint8_t *eshift;            // [c] the right edge of lane k's runs was shifted past its fixed edge
    uint32_t shift;             // chunk-edge shifting window (bytes), 0 = off
    uint32_t alldfa;            // ablation: inner edges list every DFA state (runs from I at the text
                                // start, from F at its end)
    uint64_t *Mf, *MbR;         // [c][emax][ew] masks; MbR indexed by c-1-i
    uint32_t ew;                // words of an entry-list mask (ceil(emax / 64))
    uint16_t *nxf, *nxb;        // entry-list sizes at the scan input of item k (forward: left edge of
                                // chunk k; backward: right edge of chunk c-1-k)
    uint8_t *rsf, *rsb;         // item k starts a text (forward: first chunk; backward: last chunk)
    uint64_t *fin, *fout;       // [c][ew] forward join masks at the left / right edge of chunk i
    uint64_t *bin, *bout;       // [c][ew] backward join masks (reversed item order: index c-1-i)
    uint16_t *fid, *rid;        // build start ids per chunk
    uint16_t *ckpt;             // forward id at the left edge of every 64-byte window
    uint16_t *bckpt;            // backward id at the right edge of every 64-byte window
    uint32_t *flags;            // [0] set not found, [1..3] unused
    uint64_t *trace;            // optional J / J^ words (one text only)
    // tree count (count_on): the count of a text is the product of the
    // numbers of paths through its maximal runs of ambiguous clean columns
    // (every path passes through every singleton column; a text edge acts as
    // one).  k_build multiplies in the runs of one column that lie inside a
    // lane chunk and marks the columns of every other run; the run kernels
    // count the marked runs from the written columns.
    uint32_t count_on;
    uint64_t *amask;            // [window-major, as ckpt] marked columns of each 64-column window
    uint64_t *aend;             // [T] bit 0: the text-end column n is marked
    uint64_t *cfac;             // [c][2] product per chunk, modulo 2^64 and 2^61 - 1
    uint64_t *tprod;            // [T][2] product of the long runs of each text
    uint32_t *tfail;            // [T] a run of the text could not be counted
    uint32_t *ccnt;             // [0] deferred windows, [1] long runs, [2] pieces, [3] matrix slots
    uint32_t *dchunk;           // windows (w c + i) whose short runs the wave kernel counts
    RunRec *runs;               // [cap_runs] long runs
    uint64_t *sruns;            // [cap_sruns] short runs queued for k_count_short (short_run words)
    uint8_t *cfull;             // [c] every column of lane chunk i is marked (run ends skip such chunks)
    uint32_t *squeue2;          // [cap_sruns] queued runs with a column too large for the first pass
    unsigned long long *nsruns; // short runs queued (may pass cap_sruns: then the rest are counted in place)
    uint32_t cap_sruns;
    uint32_t fol_lds;           // k_count_short: FolSeg staged in LDS (it fits)
    uint64_t *piece;            // [cap_pieces]: run index | piece number << 32
    uint64_t *mats;             // [cap_mats][kPieceR][kPieceR][2] piece matrices
    uint32_t *pmat;             // [cap_pieces]: rows | cols << 8 of the piece's matrix, or void
    uint32_t cap_runs, cap_pieces, cap_mats;
    uint32_t lshort;            // runs longer than this go to the piece kernels
    uint64_t cell;              // piece cell length (columns)
    uint32_t fwd_only;          // recogniser: forward runs and forward join only
    uint32_t compact;           // columns as one word over the candidate list X[x_r, x_r+1]
    uint32_t rank_lds;          // compact build: LDS byte offset of the rank table, 0 = read it from L2
    uint32_t pair_lds;          // build: LDS byte offset of the pair table, 0 = read it from L2
};

constexpr int kDedupEvery = 32;

// Window checkpoints are stored window-major (w * c + i), so the lanes of a
// wavefront write 64 consecutive entries.
__device__ inline uint64_t ck(const Job &jb, uint32_t i, uint32_t w) { return static_cast<uint64_t>(w) * jb.c + i; }
// One text of a job and one lane chunk of it.
struct TextRef {
    const uint8_t *text;
    uint64_t n;
    uint64_t *out;
    uint64_t *scalars;
};

// Text and output buffers are global memory.  The pointers are made in the
// global address space and then converted, so the compiler emits global (not
// flat) loads and stores: flat accesses share a wait counter with LDS, and
// every LDS wait would then wait for the text loads and column stores too.
template <class T>
__device__ inline T *global_ptr(uint64_t a) {
    using G = __attribute__((address_space(1))) T;
    return (T *)((G *)a);
}

__device__ inline TextRef text_ref(const Job &jb, uint32_t t) {
    const uint64_t *d = jb.ntexts == 1 ? jb.d0 : jb.tdesc + 4ull * t;
    return {global_ptr<const uint8_t>(d[0]), d[1], global_ptr<uint64_t>(d[2]), global_ptr<uint64_t>(d[3])};
}

__device__ inline uint32_t first_chunk(const Job &jb, uint32_t t) {
    return jb.ntexts == 1 ? (t == 0 ? 0 : jb.c) : jb.tchunk0[t];
}

// text owning chunk i: the largest t < T with tchunk0[t] <= i (a search)
__device__ inline uint32_t text_search(const Job &jb, uint32_t i) {
    uint32_t lo = 0, hi = jb.ntexts - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (jb.tchunk0[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// text owning chunk i (one load from the chunk map once it is filled)
__device__ inline uint32_t text_of(const Job &jb, uint32_t i) {
    if (jb.ntexts == 1) return 0;
    return jb.tmap ? jb.tmap[i] : text_search(jb, i);
}

struct ChunkCtx {
    TextRef tr;
    uint32_t t, li, ct;         // text, chunk index within the text, chunks of the text
    uint64_t lo, hi;            // byte range within the text
    bool first, last;
};

__device__ inline ChunkCtx chunk_ctx(const Job &jb, uint32_t i) {
    ChunkCtx x;
    x.t = text_of(jb, i);
    x.tr = text_ref(jb, x.t);
    const uint32_t c0 = first_chunk(jb, x.t);
    x.ct = first_chunk(jb, x.t + 1) - c0;
    x.li = i - c0;
    x.lo = static_cast<uint64_t>(x.li) * jb.s;
    x.first = x.li == 0;
    x.last = x.li + 1 == x.ct;
    x.hi = x.last ? x.tr.n : x.lo + jb.s;
    return x;
}

constexpr int kGroup = 12;                    // runs in lockstep (slot nibbles in a u64)
constexpr uint32_t kReachPre = 256;           // reach: bytes every run covers before runs are merged
constexpr int kPieceR = 8;                    // largest anchor column of a piece of a long run

__device__ inline uint32_t boundary_list(const Tabs &tb, const uint16_t *cls, const uint8_t *text,
                                         uint64_t n, uint64_t s, uint32_t c, uint32_t b) {
    uint64_t pos = (b == c) ? n : static_cast<uint64_t>(b) * s;
    uint32_t p = (b == 0) ? tb.C : cls[text[pos - 1]];
    uint32_t q = (b == c) ? tb.C : cls[text[pos]];
    return p * tb.NL + q;
}

__device__ inline uint64_t low_mask(uint32_t k) { return k >= 64 ? ~0ull : ((1ull << k) - 1); }

__device__ inline uint64_t apply_map(const uint64_t *rows, uint64_t v) {
    uint64_t r = 0;
    while (v) {
        int m = __builtin_ctzll(v);
        v &= v - 1;
        r |= rows[m];
    }
    return r;
}

__device__ inline uint32_t lookup_set(const uint32_t *htab, uint32_t mask, const uint64_t *bits,
                                      uint32_t W, const uint64_t *key, uint32_t *err) {
    uint32_t h = hash_words(key, static_cast<int>(W)) & mask;
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        uint32_t id = htab[h];
        if (id == kHashEmpty) break;
        const uint64_t *b = bits + static_cast<uint64_t>(id) * W;
        bool eq = true;
        for (uint32_t w = 0; w < W; ++w) eq = eq && (b[w] == key[w]);
        if (eq) return id;
        h = (h + 1) & mask;
    }
    atomicOr(err, 1u);
    return 0;
}

// -------------------------------------------------------------- table staging

// Transition tables and the class map staged in LDS (placement 0) or read in
// place through the caches (placement 1).
template <bool LDS>
struct Lookup {
    const uint16_t *cls;
    const uint16_t *fd;
    const uint16_t *rd;
};

template <bool LDS>
__device__ inline Lookup<LDS> stage_tables(const Tabs &tb, uint8_t *smem, bool need_f, bool need_r) {
    Lookup<LDS> lk;
    if constexpr (LDS) {
        uint16_t *cls = reinterpret_cast<uint16_t *>(smem);
        uint16_t *fd = cls + 256;
        uint16_t *rd = fd + (need_f ? tb.nf * tb.C : 0);
        const uint32_t nth = blockDim.x;
        for (uint32_t k = threadIdx.x; k < 256; k += nth) cls[k] = tb.classmap[k];
        if (need_f) {
            const uint32_t nfw = tb.nf * tb.C;
            for (uint32_t k = threadIdx.x; k < nfw; k += nth) fd[k] = tb.fdelta[k];
        }
        if (need_r) {
            const uint32_t nrw = tb.nr * tb.C;
            for (uint32_t k = threadIdx.x; k < nrw; k += nth) rd[k] = tb.rdelta[k];
        }
        __syncthreads();
        lk.cls = cls;
        lk.fd = fd;
        lk.rd = rd;
    } else {
        lk.cls = tb.classmap;
        lk.fd = tb.fdelta;
        lk.rd = tb.rdelta;
    }
    return lk;
}

__device__ inline uint32_t byte_of(const uint32_t *xw, int t) { return (xw[t >> 2] >> ((t & 3) * 8)) & 0xffu; }

// Load text[a0, a0+len) (len <= 64) into 16 words; 16-byte loads when the
// whole window is inside the text.
__device__ inline void load_window(const uint8_t *text, uint64_t a0, uint32_t len, uint32_t *xw) {
    if (len == 64) {
        const uint4 *p = reinterpret_cast<const uint4 *>(text + a0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint4 v = p[k];
            xw[4 * k] = v.x;
            xw[4 * k + 1] = v.y;
            xw[4 * k + 2] = v.z;
            xw[4 * k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) xw[k] = 0;
        for (uint32_t t = 0; t < len; ++t) xw[t >> 2] |= static_cast<uint32_t>(text[a0 + t]) << ((t & 3) * 8);
    }
}

// -------------------------------------------------------------------- reach

// Runs kGroup ME-DFA runs in lockstep over text[lo, hi) (forward) or its
// reverse (backward); the part between the first and the last 16-byte
// boundary is read with 16-byte loads.  Runs that reach the same state are merged (equal states have equal
// futures); `alias` maps entry k of the group to the slot holding its run.
// Slots dead in every lane of the wavefront are skipped.
// HEAD: lo may lie off a 16-byte boundary (else it is known to lie on one).
template <bool FWD, bool OFF, bool GRP, bool HEAD = true>
__device__ __forceinline__ void run_group(const uint8_t *text, uint64_t lo, uint64_t hi, const uint16_t *cls,
                                 const uint16_t *delta, uint32_t C, uint32_t st[kGroup],
                                 uint64_t &alias) {
    uint32_t nl = kGroup;
    auto settle = [&]() -> bool {
#pragma unroll
        for (int j = 1; j < kGroup; ++j) {
#pragma unroll
            for (int i = 0; i < j; ++i) {
                if (st[j] != 0 && st[j] == st[i]) {
#pragma unroll
                    for (int k = 0; k < kGroup; ++k)
                        if (((alias >> (4 * k)) & 15u) == static_cast<uint32_t>(j))
                            alias = (alias & ~(15ull << (4 * k))) | (static_cast<uint64_t>(i) << (4 * k));
                    st[j] = 0;
                }
            }
        }
        // compact the live runs to the front so that the wavefront bound below
        // counts live runs, not the highest live slot; entries whose run died
        // point to slot 15 (no slot: final state 0)
        uint32_t live = 0;
#pragma unroll
        for (int j = 0; j < kGroup; ++j) live |= (st[j] != 0 ? 1u : 0u) << j;
        uint64_t nidx = 0;                       // new slot of slot j in nibble j (15: dead)
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
            const uint32_t ix = ((live >> j) & 1u) ? static_cast<uint32_t>(__builtin_popcount(live & ((1u << j) - 1u)))
                                                   : 15u;
            nidx |= static_cast<uint64_t>(ix) << (4 * j);
        }
        uint32_t ns[kGroup];
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
            ns[t] = 0;
#pragma unroll
            for (int j = t; j < kGroup; ++j)
                if (((nidx >> (4 * j)) & 15u) == static_cast<uint32_t>(t)) ns[t] = st[j];
        }
        uint64_t na = 0;
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            const uint32_t a = (alias >> (4 * k)) & 15u;
            const uint32_t m = a < kGroup ? (nidx >> (4 * a)) & 15u : 15u;
            na |= static_cast<uint64_t>(m) << (4 * k);
        }
        alias = na;
#pragma unroll
        for (int t = 0; t < kGroup; ++t) st[t] = ns[t];
        const uint32_t top = static_cast<uint32_t>(__builtin_popcount(live));
        nl = 0;
#pragma unroll
        for (int j = kGroup; j >= 1; --j)
            if (nl == 0 && __any(top >= static_cast<uint32_t>(j))) nl = j;
        return nl != 0;
    };
    auto step = [&](uint32_t byte) {
        const uint32_t cl = cls[byte];
        if constexpr (OFF) {   // st and cl are byte offsets into the table
            const uint8_t *db = reinterpret_cast<const uint8_t *>(delta);
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                if (j < static_cast<int>(nl)) st[j] = *reinterpret_cast<const uint16_t *>(db + st[j] + cl);
        } else {
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                if (j < static_cast<int>(nl)) st[j] = delta[st[j] * C + cl];
        }
    };
    // [lo, a) head up to the first 16-byte boundary, [a, a + body) in blocks,
    // the rest a tail (the text itself starts on a 16-byte boundary)
    const uint64_t a = HEAD ? min(hi, (lo + 15) & ~15ull) : lo;
    const uint64_t body = (hi - a) & ~15ull;
    if (!settle()) return;
    if (FWD) {
        if constexpr (HEAD)
            for (uint64_t p = lo; p < a; ++p) step(text[p]);
    } else {
        for (uint64_t p = hi; p-- > a + body;) step(text[p]);
    }
    const uint64_t nblk = body >> 4;
    const uint4 *vp = reinterpret_cast<const uint4 *>(text + a);
    // 16-byte blocks in processing order; the next block is loaded while the
    // current ones are consumed, so the wave does not wait on HBM per block.
    // GRP: four blocks (64 bytes) a lane per load round, so that a lane uses
    // half a cache line at once and lines are not fetched again after
    // eviction (with tables in L2 the registers go to the lookups instead)
    auto blk = [&](uint64_t k) { return vp[FWD ? k : nblk - 1 - k]; };
    auto run16 = [&](const uint4 &v) {
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int tt = FWD ? t : 15 - t;
            step((wd[tt >> 2] >> ((tt & 3) * 8)) & 0xffu);
        }
    };
    if constexpr (GRP) {
        const uint64_t ngrp = nblk >> 2;
        uint4 cur[4], nxt[4];
        if (ngrp) {
#pragma unroll
            for (int j = 0; j < 4; ++j) cur[j] = blk(j);
        }
        for (uint64_t g = 0; g < ngrp; ++g) {
            if (g + 1 < ngrp) {
#pragma unroll
                for (int j = 0; j < 4; ++j) nxt[j] = blk(4 * (g + 1) + j);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j == 3 && !settle()) return;
                run16(cur[j]);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) cur[j] = nxt[j];
        }
        for (uint64_t k = 4 * ngrp; k < nblk; ++k) {
            if ((k & 3) == 3 && !settle()) return;
            run16(blk(k));
        }
    } else {
        uint4 v = nblk ? blk(0) : uint4{0, 0, 0, 0};
        for (uint64_t k = 0; k < nblk; ++k) {
            const uint4 nv = k + 1 < nblk ? blk(k + 1) : v;
            if ((k & 3) == 3 && !settle()) return;
            run16(v);
            v = nv;
        }
    }
    if (FWD) {
        for (uint64_t p = a + body; p < hi; ++p) step(text[p]);
    } else {
        if constexpr (HEAD)
            for (uint64_t p = a; p-- > lo;) step(text[p]);
    }
}

// Id of the run of group entry k (slot alias nibble k; 15: dead).
template <bool OFF>
__device__ __forceinline__ uint32_t slot_id(const uint32_t st[kGroup], uint64_t alias, int k, uint32_t c2) {
    const uint32_t sl = (alias >> (4 * k)) & 15u;
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kGroup; ++q)
        if (sl == static_cast<uint32_t>(q)) v = st[q];
    return OFF ? v / c2 : v;
}

// Runs from the singletons of the entries xl[0 .. n), kGroup in lockstep,
// over two stretches in processing order: forward [a, m) then [m, b),
// backward [m, b) (from b down) then [a, m).  out1[e * c + i] (if given) and
// out2[e * c + i] receive the id of the run from entry e after each stretch
// (0: dead).
template <bool FWD, bool OFF, bool GRP, bool SPLIT = true, bool HEAD = true>
__device__ __forceinline__ void runs_from_entries(const uint8_t *text, uint64_t a, uint64_t m, uint64_t b,
                                                  const uint16_t *cls, const uint16_t *delta, uint32_t C, uint32_t c2,
                                                  const uint16_t *single, const uint16_t *xl, uint32_t n,
                                                  uint16_t *out1, uint16_t *out2, uint32_t c, uint32_t i) {
    for (uint32_t g0 = 0; __any(g0 < n); g0 += kGroup) {
        uint32_t st[kGroup];
        uint64_t alias = 0;
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            st[k] = (g0 + k < n) ? single[xl[g0 + k]] * c2 : 0;
            alias |= static_cast<uint64_t>(k) << (4 * k);
        }
        // (without SPLIT the first stretch is empty: m is a for forward runs, b for backward ones)
        if constexpr (SPLIT) run_group<FWD, OFF, GRP, HEAD>(text, FWD ? a : m, FWD ? m : b, cls, delta, C, st, alias);
        if (SPLIT && out1) {
#pragma unroll
            for (int k = 0; k < kGroup; ++k)
                if (g0 + k < n)
                    out1[static_cast<uint64_t>(g0 + k) * c + i] =
                        static_cast<uint16_t>(slot_id<OFF>(st, alias, k, c2));
        }
        run_group<FWD, OFF, GRP, HEAD>(text, FWD ? m : a, FWD ? b : m, cls, delta, C, st, alias);
#pragma unroll
        for (int k = 0; k < kGroup; ++k)
            if (g0 + k < n)
                out2[static_cast<uint64_t>(g0 + k) * c + i] = static_cast<uint16_t>(slot_id<OFF>(st, alias, k, c2));
    }
}

// The runs of n entries whose ids are in[m * c + i] continued over text[a, b)
// (backward: from b down to a) into out (a different buffer): only the
// distinct live ids are run, kGroup at a time in increasing id order, so
// runs that have met are run once.  The selection is made again after each
// run (rather than kept in registers across it) to map every entry to its
// run's slot.
template <bool FWD, bool OFF, bool GRP>
__device__ __forceinline__ void runs_from_ids(const uint8_t *text, uint64_t a, uint64_t b, const uint16_t *cls,
                                              const uint16_t *delta, uint32_t C, uint32_t c2, uint32_t n,
                                              const uint16_t *in, uint16_t *out, uint32_t c, uint32_t i) {
    auto select = [&](uint32_t thr, uint32_t u[kGroup]) {   // the smallest distinct ids above thr, ascending
#pragma unroll
        for (int j = 0; j < kGroup; ++j) u[j] = 0xffffffffu;
        for (uint32_t m = 0; m < n; ++m) {
            const uint32_t v = in[static_cast<uint64_t>(m) * c + i];
            if (v <= thr || v >= u[kGroup - 1]) continue;
            bool dup = false;
#pragma unroll
            for (int j = 0; j < kGroup; ++j) dup |= u[j] == v;
            if (dup) continue;
#pragma unroll
            for (int j = kGroup - 1; j >= 0; --j) {   // insertion; the largest falls off
                const uint32_t below = j > 0 ? u[j - 1] : 0u;
                if (j > 0 && below > v)
                    u[j] = below;
                else if (u[j] > v)
                    u[j] = v;
            }
        }
    };
    for (uint32_t m = 0; m < n; ++m) {       // dead runs stay dead; with no bytes every id stays
        const uint64_t at = static_cast<uint64_t>(m) * c + i;
        const uint16_t v = in[at];
        if (v == 0 || a == b) out[at] = v;
    }
    bool more = a != b;
    uint32_t thr = 0;
    while (__any(more)) {
        uint32_t st[kGroup];
        uint64_t alias = 0;
        {
            uint32_t u[kGroup];
            if (more) select(thr, u);
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                st[j] = more && u[j] != 0xffffffffu ? u[j] * c2 : 0;
                alias |= static_cast<uint64_t>(j) << (4 * j);
            }
        }
        run_group<FWD, OFF, GRP>(text, a, b, cls, delta, C, st, alias);
        if (more) {
            uint32_t u[kGroup];
            select(thr, u);
            uint32_t top = thr;
#pragma unroll
            for (int j = 0; j < kGroup; ++j) top = u[j] != 0xffffffffu ? u[j] : top;
            for (uint32_t m = 0; m < n; ++m) {
                const uint64_t at = static_cast<uint64_t>(m) * c + i;
                const uint32_t v = in[at];
                if (v <= thr || v > top) continue;
                uint32_t fin = 0;
#pragma unroll
                for (int j = 0; j < kGroup; ++j)
                    if (u[j] == v) fin = slot_id<OFF>(st, alias, j, c2);
                out[at] = static_cast<uint16_t>(fin);
            }
            more = u[kGroup - 1] != 0xffffffffu;   // a full round: there may be more ids above top
            thr = top;
        }
    }
}

// Entry list of lane-chunk edge b of a text and its position.  Chunk-edge
// shifting (Sect. Tool optimization, technique (ii)): with a window w > 0
// an inner edge moves to the first position in [b s, b s + w) (inside the
// text) whose entry list X[class(x_p), class(x_{p+1})] is shortest; the
// text's first and last edges stay.
__device__ inline uint32_t edge_list(const Tabs &tb, const uint16_t *cls, const uint8_t *text, uint64_t n,
                                     uint64_t s, uint32_t ct, uint32_t b, uint32_t w, uint64_t &pos) {
    if (b == 0 || b == ct || w == 0) {
        pos = b == ct ? n : static_cast<uint64_t>(b) * s;
        return boundary_list(tb, cls, text, n, s, ct, b);
    }
    const uint64_t e = static_cast<uint64_t>(b) * s, end = min(n, e + w);
    uint32_t pc = cls[text[e - 1]];
    uint32_t best = 0, bsz = 0xffffffffu;
    uint64_t bp = e;
    for (uint64_t p = e; p < end && bsz > 1; ++p) {
        const uint32_t q = cls[text[p]];
        const uint32_t l = pc * tb.NL + q;
        const uint32_t sz = tb.xoff[l + 1] - tb.xoff[l];
        if (sz < bsz) {
            bsz = sz;
            best = l;
            bp = p;
        }
        pc = q;
    }
    pos = bp;
    return best;
}

// OFF: the runs step through the offset form of the tables; states are byte
// offsets (id * 2C) until the end ids are stored.
// MODE 0: entry lists of at most kGroup segments, no edge shifting; 1: the
// same with shifting; 2: longer lists (every run covers a first stretch,
// then only the distinct ones go on), with or without shifting.
template <bool LDS, bool OFF, int MODE>
__global__ __launch_bounds__(256) void k_reach(Tabs tb, Job jb) {
    constexpr bool MULTI = MODE == 2;
    extern __shared__ __align__(16) uint8_t smem[];
    Tabs ts = tb;
    if constexpr (OFF) {
        ts.classmap = tb.cls2;
        ts.fdelta = tb.fdo;
        ts.rdelta = tb.rdo;
    }
    Lookup<LDS> lk = stage_tables<LDS>(ts, smem, true, true);
    const uint32_t c2 = OFF ? 2 * tb.C : 1;     // state id -> offset factor
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= jb.c) return;
    const ChunkCtx cx = chunk_ctx(jb, i);
    const uint8_t *text = cx.tr.text;
    const uint64_t lo = cx.lo, hi = cx.hi;
    const uint16_t *bcls = OFF ? tb.classmap : lk.cls;
    // the lane's runs cover [pa, pb): its edges, shifted when jb.shift > 0
    uint64_t pa = lo, pb = hi;
    const uint32_t sw = MODE == 0 ? 0u : jb.shift;
    const uint32_t la = edge_list(tb, bcls, text, cx.tr.n, jb.s, cx.ct, cx.li, sw, pa);
    const uint32_t lb = edge_list(tb, bcls, text, cx.tr.n, jb.s, cx.ct, cx.li + 1, sw, pb);
    const uint32_t xa0 = tb.xoff[la], nfa = tb.xoff[la + 1] - xa0;   // the edges' lists
    const uint32_t xb0 = tb.xoff[lb], nfb = tb.xoff[lb + 1] - xb0;
    uint32_t na = nfa, nb = nfb;                                       // the runs' start lists
    // entries: run m starts in fsg[xla[m]] (forward) / rsg[xlb[m]] (backward)
    const uint16_t *xla = tb.xlist + xa0, *xlb = tb.xlist + xb0, *fsg = tb.fsingle, *rsg = tb.rsingle;
    // all-DFA-states ablation: an inner edge lists DFA state m + 1 as entry m;
    // the text's first forward runs start in I, its last backward runs in F
    // (its lists are longer than a run group: mode 2 only)
    const bool alldfa = MODE == 2 && jb.alldfa;
    const bool adA = alldfa && !cx.first, adB = alldfa && !cx.last;
    if (alldfa) {
        na = adA ? tb.dfa_f : 1u;
        xla = tb.seqids;
        fsg = adA ? tb.seqids + 1 : tb.seqids + tb.fstart;
        nb = adB ? tb.dfa_r : 1u;
        xlb = tb.seqids;
        rsg = adB ? tb.seqids + 1 : tb.seqids + tb.rstart;
    }
    // scan items: forward item i maps X_i -> X_{i+1}; backward item c-1-i maps X_{i+1} -> X_i
    jb.nxf[i] = static_cast<uint16_t>(na);
    jb.rsf[i] = cx.first ? 1 : 0;
    jb.nxb[jb.c - 1 - i] = static_cast<uint16_t>(nb);
    jb.rsb[jb.c - 1 - i] = cx.last ? 1 : 0;
    if (sw) jb.eshift[i] = pb > hi ? 1 : 0;

    // (four 16-byte blocks a lane per load round with the offset-form LDS
    // tables; the id form's address arithmetic leaves no registers for them)
    constexpr bool GRP = LDS && OFF;
    const uint32_t C = tb.C, c = jb.c;
    if constexpr (!MULTI) {
        // one group: forward to the fixed right edge hi (ids in Rm, which is R
        // without shifting) and on to the shifted edge pb (R); backward from pb
        // to hi (Rmh) and on to pa (Rh)
        constexpr bool SPLIT = MODE == 1;
        // (mode 0: the runs start and end on the lane chunk's own 64-byte edges)
        runs_from_entries<true, OFF, GRP, SPLIT, SPLIT>(text, pa, SPLIT ? hi : pa, pb, lk.cls, lk.fd, C, c2,
                                                        fsg, xla, na, SPLIT ? jb.Rm : nullptr, jb.R,
                                                        c, i);
        if (!jb.fwd_only)
            runs_from_entries<false, OFF, GRP, SPLIT, SPLIT>(text, pa, SPLIT ? hi : pb, pb, lk.cls, lk.rd, C, c2,
                                                             rsg, xlb, nb, SPLIT ? jb.Rmh : nullptr,
                                                             jb.Rh, c, i);
    } else {
        // forward runs from X_i: every entry over the first kReachPre bytes,
        // the distinct runs on to the fixed right edge hi (ids in Rm: J there
        // is the union of the selected ones), then to the shifted edge pb (ids
        // in R; without shifting Rm is R)
        const uint64_t fa = pa + kReachPre < hi ? pa + kReachPre : hi;
        runs_from_entries<true, OFF, GRP>(text, pa, fa, fa, lk.cls, lk.fd, C, c2, fsg, xla, na,
                                          nullptr, jb.Rt, c, i);
        runs_from_ids<true, OFF, GRP>(text, fa, hi, lk.cls, lk.fd, C, c2, na, jb.Rt, jb.Rm, c, i);
        if (jb.shift) runs_from_ids<true, OFF, GRP>(text, hi, pb, lk.cls, lk.fd, C, c2, na, jb.Rm, jb.R, c, i);
        // backward runs from X_{i+1} (not for the recogniser): with shifting
        // first from pb down to the fixed edge hi (ids in Rmh: J^ there), then
        // every run over the last kReachPre bytes before hi, the distinct ones
        // down to pa
        if (!jb.fwd_only) {
            const uint64_t ba = hi - pa > kReachPre ? max(pa, (hi - kReachPre) & ~15ull) : pa;
            if (jb.shift) {
                runs_from_entries<false, OFF, GRP>(text, hi, hi, pb, lk.cls, lk.rd, C, c2, rsg,
                                                   xlb, nb, nullptr, jb.Rmh, c, i);
                runs_from_ids<false, OFF, GRP>(text, ba, hi, lk.cls, lk.rd, C, c2, nb, jb.Rmh, jb.Rt, c, i);
            } else {
                runs_from_entries<false, OFF, GRP>(text, ba, hi, hi, lk.cls, lk.rd, C, c2, rsg,
                                                   xlb, nb, nullptr, jb.Rt, c, i);
            }
            runs_from_ids<false, OFF, GRP>(text, pa, ba, lk.cls, lk.rd, C, c2, nb, jb.Rt, jb.Rh, c, i);
        }
    }
    // maps between entry lists: forward X_i -> X_{i+1}, backward X_{i+1} -> X_i;
    // row m (ew words) has bit p set when the run from entry m ends in a set
    // holding the p-th segment of the far list
    const uint32_t W = tb.W, EW = jb.ew;
    for (uint32_t m = 0; m < na; ++m) {
        uint32_t id = jb.R[static_cast<uint64_t>(m) * jb.c + i];
        const uint64_t *bits = tb.fbits + static_cast<uint64_t>(id) * W;
        uint64_t *dst = jb.Mf + (static_cast<uint64_t>(i) * tb.emax + m) * EW;
        if (adB) {   // the far list is every DFA state: the run's end state itself
            for (uint32_t w = 0; w < EW; ++w) dst[w] = id && (id - 1) / 64 == w ? 1ull << ((id - 1) & 63) : 0ull;
            continue;
        }
        for (uint32_t w = 0; w < EW; ++w) {
            uint64_t row = 0;
            for (uint32_t p = 64 * w; p < nfb && p < 64 * w + 64; ++p) {
                uint32_t sg = tb.xlist[xb0 + p];
                row |= ((bits[sg >> 6] >> (sg & 63)) & 1ull) << (p & 63);
            }
            dst[w] = row;
        }
    }
    for (uint32_t m = 0; m < (jb.fwd_only ? 0u : nb); ++m) {
        uint32_t id = jb.Rh[static_cast<uint64_t>(m) * jb.c + i];
        const uint64_t *bits = tb.rbits + static_cast<uint64_t>(id) * W;
        uint64_t *dst = jb.MbR + (static_cast<uint64_t>(jb.c - 1 - i) * tb.emax + m) * EW;
        if (adA) {
            for (uint32_t w = 0; w < EW; ++w) dst[w] = id && (id - 1) / 64 == w ? 1ull << ((id - 1) & 63) : 0ull;
            continue;
        }
        for (uint32_t w = 0; w < EW; ++w) {
            uint64_t row = 0;
            for (uint32_t p = 64 * w; p < nfa && p < 64 * w + 64; ++p) {
                uint32_t sg = tb.xlist[xa0 + p];
                row |= ((bits[sg >> 6] >> (sg & 63)) & 1ull) << (p & 63);
            }
            dst[w] = row;
        }
    }
}

// Wavefront-local synchronization: LDS written by some lanes of a wavefront
// is visible to the other lanes of the same wavefront after this point.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of v in lane (lane - 1) of the wavefront (lane 0 gets its own value).
__device__ inline uint64_t shfl_up_u64(uint64_t v, int delta) {
    const uint32_t lo = static_cast<uint32_t>(__shfl_up(static_cast<int>(static_cast<uint32_t>(v)), delta));
    const uint32_t hi = static_cast<uint32_t>(__shfl_up(static_cast<int>(static_cast<uint32_t>(v >> 32)), delta));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// --------------------------------------------------------------------- join

// The join is a segmented scan over "items" (chunks, in text order for the
// forward direction and reversed for the backward one).  Item k maps masks
// over the entry list at its input edge to masks over the one at its output
// edge: f(v) = cst ? cv : OR of rows[m] over the bits m of v.  An item that
// starts a text ignores its input and starts from all of its entry list (J_0 =
// I restricted, or J^ = F restricted), so it is a constant map.  Level l+1
// holds the compositions of groups of 64 items of level l, up to a level of
// one item.  Every wavefront scans its group in LDS (Hillis-Steele, lanes =
// items) and writes the prefix maps, so the expansion back down is one
// independent map application per item.
struct ScanLevel {
    const uint64_t *rows;       // [N][E]
    uint32_t N;
    const uint16_t *nx;         // [N] input entry-list size per item
    const uint8_t *cst;         // [N] level 0: item starts a text; above: constant map
    const uint64_t *cv;         // [N] level >= 1: the constant
    int level0;
};

// Both directions of the join run in the same launches: blockIdx.y selects
// the forward (0) or the backward (1) scan.
struct ScanPair {
    ScanLevel L[2];
};
struct ScanOut {
    uint64_t *rows[2];          // next level
    uint16_t *nx[2];
    uint8_t *cst[2];
    uint64_t *cv[2];
    uint64_t *prow[2];          // prefix maps of this level's items within their group: [N][E]
    uint8_t *pcst[2];
    uint64_t *pcv[2];
};
struct ScanPrefix {
    const uint64_t *prow[2];
    const uint8_t *pcst[2];
    const uint64_t *pcv[2];
    const uint64_t *pvec[2];    // vectors entering the groups (nullptr: the empty mask)
    uint64_t *vin[2];           // mask entering every item
    uint64_t *vout[2];          // level 0: mask leaving every item
};

__device__ inline uint64_t map_apply(const uint64_t *rows, bool cst, uint64_t cv, uint64_t v) {
    if (cst) return cv;
    uint64_t r = 0;
    while (v) {
        const int m = __builtin_ctzll(v);
        v &= v - 1;
        r |= rows[m];
    }
    return r;
}

// Scan of one group of up to 64 items per wavefront: dynamic LDS holds two
// buffers of 64 x E rows.
__global__ __launch_bounds__(64) void k_compose(ScanPair S, ScanOut O, uint32_t E) {
    extern __shared__ uint64_t mrows[];
    __shared__ uint64_t mcv[2][64];
    __shared__ uint8_t mcst[2][64];
    const uint32_t d = blockIdx.y;
    const ScanLevel L = d ? S.L[1] : S.L[0];
    const uint32_t g = blockIdx.x, k = threadIdx.x;
    const uint32_t k0 = g * 64, n = min(k0 + 64, L.N) - k0;
    // stage the group's rows (contiguous in memory), 16 loads in flight per lane
    const uint64_t *src = L.rows + static_cast<uint64_t>(k0) * E;
    const uint32_t tot = n * E;
    for (uint32_t e0 = 0; e0 < tot; e0 += 64 * 16) {
        uint64_t tmp[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint32_t e = e0 + u * 64 + k;
            tmp[u] = e < tot ? src[e] : 0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint32_t e = e0 + u * 64 + k;
            if (e < tot) mrows[e] = tmp[u];
        }
    }
    const uint32_t nx0 = L.nx[k0];              // input list of the group
    bool cst = false;
    uint64_t cv = 0;
    uint32_t nxin = 0;                          // input-list size of the lane's composite
    if (k < n) {
        nxin = L.nx[k0 + k];
        cst = L.cst[k0 + k] != 0;
        if (L.level0) {
            if (cst) {   // a text start: its image of the whole entry list
                const uint64_t *r = src + static_cast<uint64_t>(k) * E;
                for (uint32_t m = 0; m < nxin; ++m) cv |= r[m];
            }
        } else {
            cv = L.cv[k0 + k];
        }
    }
    mcst[0][k] = cst ? 1 : 0;
    mcv[0][k] = cv;
    __syncthreads();
    // inclusive scan: lane k's map becomes (map_k after map_{k-dd}); after the
    // last round it is the composite of items 0..k of the group
    int cur = 0;
    for (uint32_t dd = 1; dd < 64; dd <<= 1) {
        const int nxt = cur ^ 1;
        uint64_t *mine = mrows + (nxt * 64 + k) * E;
        const uint64_t *self = mrows + (cur * 64 + k) * E;
        bool hc = mcst[cur][k] != 0;
        uint64_t hv = mcv[cur][k];
        const uint32_t nxa = __shfl_up(static_cast<int>(nxin), dd);
        if (k >= dd && k < n) {
            const uint32_t a = k - dd;
            const uint64_t *arow = mrows + (cur * 64 + a) * E;
            if (!hc) {
                if (mcst[cur][a]) {
                    hv = map_apply(self, false, 0, mcv[cur][a]);
                    hc = true;
                } else {
                    for (uint32_t m = 0; m < nxa; ++m) mine[m] = map_apply(self, false, 0, arow[m]);
                }
            }
            nxin = nxa;
        } else if (!hc) {
            for (uint32_t m = 0; m < nxin; ++m) mine[m] = self[m];
        }
        mcst[nxt][k] = hc ? 1 : 0;
        mcv[nxt][k] = hv;
        __syncthreads();
        cur = nxt;
    }
    // prefix maps of this level, coalesced from LDS
    const uint64_t *fin = mrows + cur * 64 * E;
    uint64_t *pdst = O.prow[d] + static_cast<uint64_t>(k0) * E;
    for (uint32_t e = k; e < tot; e += 64) pdst[e] = fin[e];
    if (k < n) {
        O.pcst[d][k0 + k] = mcst[cur][k];
        O.pcv[d][k0 + k] = mcv[cur][k];
    }
    // the group's composite is the next level's item g
    if (k < nx0) O.rows[d][static_cast<uint64_t>(g) * E + k] = fin[(n - 1) * E + k];
    if (k == 0) {
        O.nx[d][g] = static_cast<uint16_t>(nx0);
        O.cst[d][g] = mcst[cur][n - 1];
        O.cv[d][g] = mcv[cur][n - 1];
    }
}

// Expand one level: thread k (lanes = items of its group) applies its prefix
// map to the vector entering its group.  Level 0 (L.level0) also writes the
// mask leaving every item; a text start enters with its whole entry list.
__global__ __launch_bounds__(256) void k_expand(ScanPair S, ScanPrefix P, uint32_t E) {
    const uint32_t d = blockIdx.y;
    const ScanLevel L = d ? S.L[1] : S.L[0];
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = k >> 6;
    const bool act = k < L.N;
    uint64_t vp = 0;
    if (act && P.pvec[d]) vp = P.pvec[d][g];
    uint64_t out = 0;
    if (act)
        out = map_apply(P.prow[d] + static_cast<uint64_t>(k) * E, P.pcst[d][k] != 0, P.pcv[d][k], vp);
    const uint64_t prev = shfl_up_u64(out, 1);
    if (!act) return;
    uint64_t in = lane == 0 ? vp : prev;
    if (L.level0 && L.cst[k]) in = low_mask(L.nx[k]);
    P.vin[d][k] = in;
    if (L.level0) P.vout[d][k] = out;
}

// ---- join with entry lists of more than 64 segments (masks of EW words)
//
// The same segmented scan of maps between entry lists, with every row and
// vector held as EW words.  One wavefront composes its group of 64 items in
// order (lanes over the rows of the running prefix map, which go straight to
// the prefix array), and the expansion stages each item's output in LDS as
// the next item's input.

// bits [64 w, 64 w + 64) of the mask of the first nx entries
__device__ inline uint64_t low_mask_word(uint32_t nx, uint32_t w) {
    if (nx >= 64 * w + 64) return ~0ull;
    if (nx <= 64 * w) return 0ull;
    return low_mask(nx - 64 * w);
}

// Dynamic LDS: two buffers of EW words (the running prefix when constant).
__global__ __launch_bounds__(64) void k_compose_wide(ScanPair S, ScanOut O, uint32_t E, uint32_t EW) {
    extern __shared__ uint64_t cvs[];
    const uint32_t d = blockIdx.y;
    const ScanLevel L = d ? S.L[1] : S.L[0];
    const uint32_t g = blockIdx.x, lane = threadIdx.x;
    const uint32_t k0 = g * 64, n = min(k0 + 64, L.N) - k0;
    const uint32_t nx0 = L.nx[k0];
    const uint64_t RS = static_cast<uint64_t>(E) * EW;         // words per map
    bool pc = false;                                            // the running prefix is constant
    uint32_t cb = 0;                                            // its value is in cvs[cb * EW ..]
    for (uint32_t k = 0; k < n; ++k) {
        const uint64_t it = k0 + k;
        const uint64_t *rk = L.rows + it * RS;
        uint64_t *pk = O.prow[d] + it * RS;
        if (L.cst[it]) {
            // a constant map: at level 0 a text start, the image of its whole entry list
            for (uint32_t w = lane; w < EW; w += 64) {
                uint64_t v = 0;
                if (L.level0) {
                    for (uint32_t m = 0; m < L.nx[it]; ++m) v |= rk[static_cast<uint64_t>(m) * EW + w];
                } else {
                    v = L.cv[it * EW + w];
                }
                cvs[(cb ^ 1u) * EW + w] = v;
            }
            cb ^= 1u;
            pc = true;
        } else if (k == 0) {
            for (uint32_t m = lane; m < nx0; m += 64)
                for (uint32_t w = 0; w < EW; ++w) pk[static_cast<uint64_t>(m) * EW + w] = rk[static_cast<uint64_t>(m) * EW + w];
        } else if (pc) {
            // item k after a constant prefix: the constant's image
            const uint64_t *cv = cvs + cb * EW;
            for (uint32_t w = lane; w < EW; w += 64) {
                uint64_t v = 0;
                for (uint32_t e = 0; e < EW; ++e)
                    for (uint64_t x = cv[e]; x; x &= x - 1)
                        v |= rk[(64ull * e + __builtin_ctzll(x)) * EW + w];
                cvs[(cb ^ 1u) * EW + w] = v;
            }
            cb ^= 1u;
        } else {
            // row m of the new prefix: item k applied to row m of the previous prefix
            const uint64_t *pp = O.prow[d] + (it - 1) * RS;
            for (uint32_t m = lane; m < nx0; m += 64) {
                const uint64_t *prv = pp + static_cast<uint64_t>(m) * EW;
                for (uint32_t w = 0; w < EW; ++w) {
                    uint64_t v = 0;
                    for (uint32_t e = 0; e < EW; ++e)
                        for (uint64_t x = prv[e]; x; x &= x - 1)
                            v |= rk[(64ull * e + __builtin_ctzll(x)) * EW + w];
                    pk[static_cast<uint64_t>(m) * EW + w] = v;
                }
            }
        }
        wave_sync();
        if (lane == 0) O.pcst[d][it] = pc ? 1 : 0;
        for (uint32_t w = lane; w < EW; w += 64) O.pcv[d][it * EW + w] = pc ? cvs[cb * EW + w] : 0ull;
    }
    // the group's composite is the next level's item g
    const uint64_t last = k0 + n - 1;
    if (pc) {
        for (uint32_t w = lane; w < EW; w += 64) O.cv[d][static_cast<uint64_t>(g) * EW + w] = cvs[cb * EW + w];
    } else {
        const uint64_t *pl = O.prow[d] + last * RS;
        for (uint32_t m = lane; m < nx0; m += 64)
            for (uint32_t w = 0; w < EW; ++w)
                O.rows[d][static_cast<uint64_t>(g) * RS + static_cast<uint64_t>(m) * EW + w] =
                    pl[static_cast<uint64_t>(m) * EW + w];
        for (uint32_t w = lane; w < EW; w += 64) O.cv[d][static_cast<uint64_t>(g) * EW + w] = 0ull;
    }
    if (lane == 0) {
        O.nx[d][g] = static_cast<uint16_t>(nx0);
        O.cst[d][g] = pc ? 1 : 0;
    }
}

// Dynamic LDS: blockDim x EW words (each item's output).
__global__ __launch_bounds__(256) void k_expand_wide(ScanPair S, ScanPrefix P, uint32_t E, uint32_t EW) {
    extern __shared__ uint64_t outs[];
    const uint32_t d = blockIdx.y;
    const ScanLevel L = d ? S.L[1] : S.L[0];
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63, g = k >> 6;
    const bool act = k < L.N;
    const uint64_t *vp = act && P.pvec[d] ? P.pvec[d] + static_cast<uint64_t>(g) * EW : nullptr;
    const uint64_t RS = static_cast<uint64_t>(E) * EW;
    const bool cst = act && P.pcst[d][k] != 0;
    for (uint32_t w = 0; w < EW; ++w) {
        uint64_t o = 0;
        if (act) {
            if (cst) {
                o = P.pcv[d][static_cast<uint64_t>(k) * EW + w];
            } else if (vp) {
                const uint64_t *rows = P.prow[d] + k * RS;
                for (uint32_t e = 0; e < EW; ++e)
                    for (uint64_t x = vp[e]; x; x &= x - 1) o |= rows[(64ull * e + __builtin_ctzll(x)) * EW + w];
            }
            if (L.level0) P.vout[d][static_cast<uint64_t>(k) * EW + w] = o;
        }
        outs[threadIdx.x * EW + w] = o;
    }
    __syncthreads();
    if (!act) return;
    for (uint32_t w = 0; w < EW; ++w) {
        uint64_t in = lane == 0 ? (vp ? vp[w] : 0ull) : outs[(threadIdx.x - 1) * EW + w];
        if (L.level0 && L.cst[k]) in = low_mask_word(L.nx[k], w);
        P.vin[d][static_cast<uint64_t>(k) * EW + w] = in;
    }
}

// Join sets and build start ids.  Thread i handles chunk i: fid_i = id of
// J at P_i, rid_i = id of J^ at P_{i+1}; the last chunk of a text writes its
// accept flag.
__global__ __launch_bounds__(256) void k_starts(Tabs tb, Job jb) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t c = jb.c, W = tb.W;
    if (i >= c) return;
    const ChunkCtx cx = chunk_ctx(jb, i);
    uint64_t acc[kMaxWords];
    const uint32_t EW = jb.ew;
    // J at the right edge of chunk k: union of its runs selected by fin[k], at that edge
    auto join_fwd = [&](uint32_t k) -> uint32_t {
        for (uint32_t w = 0; w < W; ++w) acc[w] = 0;
        uint32_t first = 0xffffffffu;
        bool same = true;
        for (uint32_t e = 0; e < EW; ++e) {
            uint64_t sel = jb.fin[static_cast<uint64_t>(k) * EW + e];
            while (sel) {
                const uint32_t m = 64 * e + static_cast<uint32_t>(__builtin_ctzll(sel));
                sel &= sel - 1;
                uint32_t id = jb.Rm[static_cast<uint64_t>(m) * c + k];   // ids at the fixed right edge
                if (first == 0xffffffffu) first = id;
                same = same && (id == first);
                const uint64_t *bt = tb.fbits + static_cast<uint64_t>(id) * W;
                for (uint32_t w = 0; w < W; ++w) acc[w] |= bt[w];
            }
        }
        if (first == 0xffffffffu) return 0;
        if (same) return first;
        return lookup_set(tb.fhash, tb.fhmask, tb.fbits, W, acc, jb.flags);
    };
    // J^ at the left edge of chunk k: union of its backward runs selected by
    // the mask at its right edge (ids: ends of its runs, Rh); with `mid` the
    // same runs' ids at chunk k's fixed right edge (Rmh, when its runs start
    // at a shifted edge beyond it): J^ at that edge
    auto join_bwd = [&](uint32_t k, bool mid) -> uint32_t {
        for (uint32_t w = 0; w < W; ++w) acc[w] = 0;
        uint32_t first = 0xffffffffu;
        bool same = true;
        const uint16_t *ids = mid ? jb.Rmh : jb.Rh;
        for (uint32_t e = 0; e < EW; ++e) {
            // reversed item c-1-k enters at chunk k's right edge
            uint64_t sel = jb.bin[static_cast<uint64_t>(c - 1 - k) * EW + e];
            while (sel) {
                const uint32_t m = 64 * e + static_cast<uint32_t>(__builtin_ctzll(sel));
                sel &= sel - 1;
                uint32_t id = ids[static_cast<uint64_t>(m) * c + k];
                if (first == 0xffffffffu) first = id;
                same = same && (id == first);
                const uint64_t *bt = tb.rbits + static_cast<uint64_t>(id) * W;
                for (uint32_t w = 0; w < W; ++w) acc[w] |= bt[w];
            }
        }
        if (first == 0xffffffffu) return 0;
        if (same) return first;
        return lookup_set(tb.rhash, tb.rhmask, tb.rbits, W, acc, jb.flags);
    };
    const uint32_t f = cx.first ? tb.fstart : join_fwd(i - 1);
    const uint32_t r = cx.last ? tb.rstart : (jb.shift && jb.eshift[i]) ? join_bwd(i, true) : join_bwd(i + 1, false);
    jb.fid[i] = static_cast<uint16_t>(f);
    jb.rid[i] = static_cast<uint16_t>(r);
    if (jb.trace) {   // one text: J and J^ at every chunk edge
        uint64_t *Jt = jb.trace, *Jh = jb.trace + static_cast<uint64_t>(c + 1) * W;
        const uint64_t *fb = tb.fbits + static_cast<uint64_t>(f) * W;
        for (uint32_t w = 0; w < W; ++w) Jt[static_cast<uint64_t>(i) * W + w] = fb[w];
        const uint64_t *rb = tb.rbits + static_cast<uint64_t>(r) * W;
        for (uint32_t w = 0; w < W; ++w) Jh[static_cast<uint64_t>(i + 1) * W + w] = rb[w];
        if (i + 1 == c) {
            const uint64_t *e = tb.fbits + static_cast<uint64_t>(join_fwd(c - 1)) * W;
            for (uint32_t w = 0; w < W; ++w) Jt[static_cast<uint64_t>(c) * W + w] = e[w];
        }
        if (i == 0) {
            const uint64_t *e = tb.rbits + static_cast<uint64_t>(join_bwd(0, false)) * W;
            for (uint32_t w = 0; w < W; ++w) Jh[w] = e[w];
        }
    }
    if (cx.last) {
        uint64_t any = 0;
        for (uint32_t e = 0; e < EW; ++e) any |= jb.fout[static_cast<uint64_t>(i) * EW + e];
        cx.tr.scalars[0] = any != 0 ? 1ull : 0ull;
    }
}

// -------------------------------------------------------------------- build


// Tables for the build and count kernels: class map and transition tables
// (TAB_LDS) and the state bit sets (BITS_LDS) staged in LDS after `skip`
// bytes of the dynamic LDS area, or read in place.
template <bool TAB_LDS, bool BITS_LDS>
struct BuildTabs {
    const uint16_t *cls, *fd, *rd;
    const uint64_t *fb, *rb;
    const uint32_t *fnz, *rnz;
};

template <bool TAB_LDS, bool BITS_LDS>
__device__ inline BuildTabs<TAB_LDS, BITS_LDS> stage_build(const Tabs &tb, uint8_t *smem, uint32_t skip) {
    BuildTabs<TAB_LDS, BITS_LDS> t;
    const uint32_t nth = blockDim.x;
    uint8_t *p = smem + skip;
    if constexpr (TAB_LDS) {
        uint16_t *cls = reinterpret_cast<uint16_t *>(p);
        uint16_t *fd = cls + 256;
        uint16_t *rd = fd + tb.nf * tb.C;
        for (uint32_t k = threadIdx.x; k < 256; k += nth) cls[k] = tb.classmap[k];
        for (uint32_t k = threadIdx.x; k < tb.nf * tb.C; k += nth) fd[k] = tb.fdelta[k];
        for (uint32_t k = threadIdx.x; k < tb.nr * tb.C; k += nth) rd[k] = tb.rdelta[k];
        t.cls = cls;
        t.fd = fd;
        t.rd = rd;
        p += (512 + (tb.nf + tb.nr) * tb.C * 2 + 15) & ~15u;
    } else {
        t.cls = tb.classmap;
        t.fd = tb.fdelta;
        t.rd = tb.rdelta;
    }
    if constexpr (BITS_LDS) {
        uint64_t *fb = reinterpret_cast<uint64_t *>(p);
        uint64_t *rb = fb + tb.nf * tb.W;
        for (uint32_t k = threadIdx.x; k < tb.nf * tb.W; k += nth) fb[k] = tb.fbits[k];
        for (uint32_t k = threadIdx.x; k < tb.nr * tb.W; k += nth) rb[k] = tb.rbits[k];
        uint32_t *fz = reinterpret_cast<uint32_t *>(rb + tb.nr * tb.W), *rz = fz + tb.nf;
        for (uint32_t k = threadIdx.x; k < tb.nf; k += nth) fz[k] = tb.fnz[k];
        for (uint32_t k = threadIdx.x; k < tb.nr; k += nth) rz[k] = tb.rnz[k];
        t.fb = fb;
        t.rb = rb;
        t.fnz = fz;
        t.rnz = rz;
    } else {
        t.fb = tb.fbits;
        t.rb = tb.rbits;
        t.fnz = tb.fnz;
        t.rnz = tb.rnz;
    }
    __syncthreads();
    return t;
}

__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = __shfl(static_cast<uint32_t>(v), src);
    uint32_t hi = __shfl(static_cast<uint32_t>(v >> 32), src);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}


// Classes of the 64 window bytes, packed four per word.
template <class BT>
__device__ inline void window_classes(const BT &T, const uint32_t *xw, uint32_t *cw) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t v = xw[k];
        cw[k] = static_cast<uint32_t>(T.cls[v & 0xffu]) | (static_cast<uint32_t>(T.cls[(v >> 8) & 0xffu]) << 8) |
                (static_cast<uint32_t>(T.cls[(v >> 16) & 0xffu]) << 16) |
                (static_cast<uint32_t>(T.cls[v >> 24]) << 24);
    }
}

// Lane j's value of v.  The builtin returns int: each half goes through
// uint32_t so that the low half is not sign-extended into the high one.
__device__ inline uint64_t readlane_u64(uint64_t v, int j) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), j));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), j));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), off)));
    return v;
}

constexpr uint64_t kP61 = (1ull << 61) - 1;    // the second modulus of the tree count

// a * b modulo 2^61 - 1 (a, b < 2^61): with 2^61 = 1, the 122-bit product
// hi * 2^64 + lo folds to (lo mod 2^61) + (lo >> 61) + 8 hi.
__device__ inline uint64_t mulp(uint64_t a, uint64_t b) {
    const uint64_t lo = a * b, hi = __umul64hi(a, b);
    uint64_t r = (lo & kP61) + ((lo >> 61) | (hi << 3));
    r = (r & kP61) + (r >> 61);
    return r >= kP61 ? r - kP61 : r;
}

// x * m modulo 2^61 - 1 for x < 2^61 and m < 2^16 (the high word of the
// product is below 2^13, so one fold and one subtraction suffice).
__device__ inline uint64_t mulp_small(uint64_t x, uint32_t m) {
    const uint64_t lo = x * m, hi = __umul64hi(x, static_cast<uint64_t>(m));
    const uint64_t r = (lo & kP61) + ((lo >> 61) | (hi << 3));
    return r >= kP61 ? r - kP61 : r;
}

// Tree-count bookkeeping of one lane of k_build.  Every path through the
// clean SLPF of an accepted text passes through each singleton column, and a
// text edge acts as one, so the count is the product over the maximal runs
// of ambiguous columns of the paths through each run; a run of one column
// between two singletons has as many paths as the column has segments.  The
// lane visits its chunk's columns right to left.  A one-column run inside
// the chunk is multiplied in here; the columns of every other run (longer,
// touching a chunk edge inside the text, or of unknown size) are marked,
// one bit per column, for the run kernels.
// A run of two columns is multiplied in too: its paths are the arcs between
// them, a function of the left column's forward state, the right column's
// reverse state and the byte between them (table arcs2).
//   st 0: the column to the right is a singleton or the text end;
//   st 1: it is an ambiguous column of size pm not marked yet, whose own
//         right neighbour is a singleton;
//   st 2: it and its right neighbour are ambiguous, not marked, with pa
//         paths between them, and a singleton further right;
//   st 3: it is marked, or lies beyond the chunk.
struct RunMarks {
    uint32_t st = 3, pm = 0, pa = 0, endmark = 0;
    uint32_t e2 = 0;                   // one-column runs of two segments (a factor 2 each)
    uint64_t a64 = 1, ap = 1;          // product of the other short runs, mod 2^64 and 2^61 - 1
    uint64_t wcur = 0, wright = 0;     // marks of the current window and of the window to its right
    __device__ __forceinline__ void mul(uint32_t m) {
        a64 *= m;
        ap = mulp_small(ap, m);
    }
    // a singleton column: it closes a pending run of one or two columns
    __device__ __forceinline__ void single() {
        if (st == 1) {
            if (pm == 2) ++e2;
            else mul(pm);
        } else if (st == 2) {
            mul(pa);
        }
        st = 0;
    }
    // mark column t + d (d = 1, 2) of the current window; end: it is the text-end column
    __device__ __forceinline__ void mark_right(uint32_t t, uint32_t d, bool end) {
        if (end) endmark = 1;
        else if (t + d >= 64) wright |= 1ull << (t + d - 64);
        else wcur |= 1ull << (t + d);
    }
    // column t of the current window (text column col) has the size code m
    // (1 a singleton, 2..254 its size, other values unknown) and forward
    // state ft; the column to its right has reverse state bright (for the
    // arcs table, with the class of the byte text[col] between them); endk:
    // column t + k is the text end n (which has no bit in the windows)
    template <class Cls>
    __device__ __forceinline__ void step(const Tabs &tb, uint32_t t, uint32_t m, uint32_t ft, uint32_t bright,
                                         const uint8_t *text, uint64_t col, const Cls *cls, bool end1, bool end2) {
        const bool known = m - 2u <= 252u;
        if (m == 1) {
            single();
            return;
        }
        if (st == 0 && known) {
            st = 1;
            pm = m;
            return;
        }
        if (st == 1 && known) {   // the byte between this column and the next is text[col]
            const uint32_t a = tb.arcs2 && ft < tb.kfd && bright < tb.krd
                                   ? tb.arcs2[(static_cast<uint64_t>(ft) * tb.krd + bright) * tb.C + cls[text[col]]]
                                   : 0xffffu;
            if (a != 0xffffu) {
                st = 2;
                pa = a;
                return;
            }
        }
        // the column is marked, and so are the pending ones to its right
        if (st == 1 || st == 2) mark_right(t, 1, end1);
        if (st == 2) mark_right(t, 2, end2);
        wcur |= 1ull << t;
        st = 3;
    }
    // fold the factors 2 into the products (2^61 = 1 modulo 2^61 - 1)
    __device__ inline void finish() {
        a64 = e2 < 64 ? a64 << e2 : 0ull;
        ap = mulp(ap, 1ull << (e2 % 61));
    }
};

constexpr int kBuildThreads = 512;             // 8 wavefronts
constexpr int kStageCols = 32;                 // columns per staged part of a window
constexpr int kStageRow = kStageCols + 1;      // padded: lanes fall in distinct banks
constexpr int kStageBytes = kBuildThreads * kStageRow * 4;

// Fused builder & merger.  Each lane owns one chunk and writes its columns
// P_i .. P_{i+1}-1 (the last chunk also the text-end column n): a forward DFA
// run from J at P_i storing a checkpoint per 64-byte window, then window by
// window from the right: the reverse DFA runs from the right edge while the
// forward ids of the next window to the left are recomputed from its
// checkpoint (two independent lookup chains per lane), and the (forward,
// backward) id pair of every column goes to LDS.  Every kStageCols (32)
// columns the wavefront writes the staged columns of its 64 chunks, each
// chunk's columns as one contiguous run of W-word columns starting on a
// 32-column boundary (so on a 128-byte boundary for any W); lane e writes word
// e, 512 contiguous bytes per store instruction, as streaming (nontemporal)
// stores.  Wavefronts synchronize only with themselves.
//
// COMPACT writes the compact SLPF instead: column r as one word whose bit k
// says that the k-th segment of the candidate list X[class(x_r),
// class(x_{r+1})] is in the clean column (the clean column lies in that list,
// which holds at most 64 segments).  Parts are 16 columns (one 128-byte line
// per chunk), and the stage row holds each column's previous-byte class
// after its id pairs.
template <bool TAB_LDS, bool BITS_LDS, bool COMPACT>
__global__ __launch_bounds__(kBuildThreads) void k_build(Tabs tb, Job jb) {
    constexpr int SC = COMPACT ? 16 : kStageCols;     // columns per part
    constexpr int PARTS = 64 / SC;
    static_assert(!COMPACT || 2 * SC <= kStageRow, "a compact stage row holds ids and classes");
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *stage = reinterpret_cast<uint32_t *>(smem);
    const BuildTabs<TAB_LDS, BITS_LDS> T = stage_build<TAB_LDS, BITS_LDS>(tb, smem, kStageBytes);
    const uint32_t C = tb.C, W = tb.W;
    // compact: the rank table in LDS when the launch reserved room for it
    const uint8_t *rkl = smem + jb.rank_lds;
    if (COMPACT && jb.rank_lds) {
        uint8_t *dst = smem + jb.rank_lds;
        const uint32_t nr = (tb.rank_pq ? tb.NL * tb.NL : tb.NL) * tb.nseg;
        for (uint32_t k = threadIdx.x; k < nr; k += blockDim.x) dst[k] = tb.rankx[k];
        __syncthreads();
    }
    auto rank_of = [&](uint32_t idx) -> uint32_t { return jb.rank_lds ? rkl[idx] : tb.rankx[idx]; };
    // tree count: the pair table (sizes of the clean columns) in LDS when the
    // launch reserved room for it
    const uint8_t *pml = smem + jb.pair_lds;
    if (jb.count_on && jb.pair_lds) {
        uint8_t *dst = smem + jb.pair_lds;
        const uint32_t nb = tb.pair_nib ? (tb.kfd * tb.krd + 1) / 2 : tb.kfd * tb.krd;
        for (uint32_t k = threadIdx.x; k < nb; k += blockDim.x) dst[k] = tb.pairm[k];
        __syncthreads();
    }
    auto pair_size = [&](uint32_t fi, uint32_t bi) -> uint32_t {
        if (fi >= tb.kfd || bi >= tb.krd) return 0u;
        const uint32_t k = fi * tb.krd + bi;
        const uint8_t *pt = jb.pair_lds ? pml : tb.pairm;
        if (!tb.pair_nib) return static_cast<uint32_t>(pt[k]);
        const uint32_t v = (static_cast<uint32_t>(pt[k >> 1]) >> ((k & 1u) * 4u)) & 15u;
        return v == 15u ? 255u : v;          // 255: too many to multiply in (a general run)
    };

    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t wave_first = blockIdx.x * blockDim.x + wv * 64;
    if (wave_first >= jb.c) return;                 // whole wavefront idle
    const bool act = i < jb.c;
    ChunkCtx cx{};
    uint64_t lo = 0, hi = 0;
    uint32_t nwin = 0;
    const uint8_t *text = nullptr;
    uint64_t *out = nullptr;
    if (act) {
        cx = chunk_ctx(jb, i);
        lo = cx.lo;
        hi = cx.hi;
        text = cx.tr.text;
        out = cx.tr.out;
        nwin = static_cast<uint32_t>((hi - lo + 63) / 64);
    }
    const uint32_t nwin_wave = wave_max_u32(nwin);
    uint32_t xw[16], cw[16];
    // tree count of an accepted text (an RE whose clean columns are all
    // singletons has one tree per accepted text: nothing to count)
    const bool cnt = act && jb.count_on && !tb.col_single && cx.tr.scalars[0] != 0;
    bool allm = true;                  // so far, every column of the chunk's windows is marked
    RunMarks rm;

    // forward sweep: checkpoints
    uint32_t f = act ? jb.fid[i] : 0;
    for (uint32_t w = 0; w < nwin; ++w) {
        const uint64_t a0 = lo + 64ull * w;
        const uint32_t len = static_cast<uint32_t>(hi - a0 < 64 ? hi - a0 : 64);
        jb.ckpt[ck(jb, i, w)] = static_cast<uint16_t>(f);
        load_window(text, a0, len, xw);
        window_classes(T, xw, cw);
#pragma unroll
        for (int t = 0; t < 64; ++t)
            if (t < static_cast<int>(len)) f = T.fd[f * C + byte_of(cw, t)];
    }
    if (act && cx.last) {   // the text-end column: J_c & F
        if constexpr (COMPACT) {
            const uint32_t pc = T.cls[text[cx.tr.n - 1]];
            uint64_t m = 0;
            for (uint32_t w = 0; w < W; ++w) {
                uint64_t v = T.fb[f * W + w] & T.rb[tb.rstart * W + w];
                while (v) {
                    const uint32_t sg = w * 64 + static_cast<uint32_t>(__builtin_ctzll(v));
                    v &= v - 1;
                    m |= 1ull << tb.rankx[(tb.rank_pq ? pc * tb.NL + C : pc) * tb.nseg + sg];
                }
            }
            out[cx.tr.n] = m;
        } else {
            for (uint32_t w = 0; w < W; ++w)
                out[cx.tr.n * W + w] = T.fb[f * W + w] & T.rb[tb.rstart * W + w];
        }
        if (cnt) {   // the text-end column, with the text end to its right
            const uint32_t m = pair_size(f, tb.rstart);
            rm.st = 0;
            if (m >= 2 && m <= 254) {
                rm.st = 1;
                rm.pm = m;
            } else if (m != 1) {
                rm.endmark = 1;
                rm.st = 3;
            }
        }
    }

    // backward sweep, two windows in flight; fwA[t] = forward id at column a0+t
    uint32_t b = act ? jb.rid[i] : 0;
    uint32_t bright = b;               // tree count: backward id of the column right of the current part
    uint32_t amb = 0;                  // tree count: the current part's columns that are not singletons
    uint32_t *mine = stage + threadIdx.x * kStageRow;
    const uint32_t *wave_rows = stage + wv * 64 * kStageRow;
    uint32_t fwA[64], cwA[16];
    uint32_t lenA = 0;
    uint64_t a0A = 0;
    // class of the byte before the chunk (the text start: the sentinel C)
    const uint32_t pfirst = COMPACT && act && lo > 0 ? T.cls[text[lo - 1]] : C;
    if (nwin) {   // the last window of the chunk
        a0A = lo + 64ull * (nwin - 1);
        lenA = static_cast<uint32_t>(hi - a0A);
        load_window(text, a0A, lenA, xw);
        window_classes(T, xw, cwA);
        uint32_t g = jb.ckpt[ck(jb, i, nwin - 1)];
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            fwA[t] = g;
            if (t < static_cast<int>(lenA)) g = T.fd[g * C + byte_of(cwA, t)];
        }
    }
    for (int w = static_cast<int>(nwin_wave) - 1; w >= 0; --w) {
        const bool on = w < static_cast<int>(nwin);
        // window w-1 (full length) is prepared while window w is merged
        const bool nxt = on && w > 0;
        uint32_t cwB[16], fwB[64];
        uint32_t g = 0;
        if (nxt) {
            load_window(text, lo + 64ull * (w - 1), 64, xw);
            window_classes(T, xw, cwB);
            g = jb.ckpt[ck(jb, i, w - 1)];
        }
        if (on) jb.bckpt[ck(jb, i, w)] = static_cast<uint16_t>(b);
        if (cnt && on) {
            rm.wright = rm.wcur;
            rm.wcur = 0;
        }
        const uint32_t len_now = on ? lenA : 0;
        // class of the byte before window w: the last byte of window w-1
        const uint32_t pA0 = nxt ? byte_of(cwB, 63) : pfirst;
#pragma unroll
        for (int h = PARTS - 1; h >= 0; --h) {
            // columns a0+S*h .. a0+S*h+S-1 of window w (S = SC), right to left
#pragma unroll
            for (int u = SC - 1; u >= 0; --u) {
                const int t = h * SC + u;
                if (on && t < static_cast<int>(lenA)) {
                    b = T.rd[b * C + byte_of(cwA, t)];    // now the backward id at column a0+t
                    mine[u] = fwA[t] | (b << 16);
                    // compact: the classes of the bytes before and after the column
                    if constexpr (COMPACT) mine[SC + u] = (t > 0 ? byte_of(cwA, t - 1) : pA0) | (byte_of(cwA, t) << 16);
                    if (cnt) amb |= (pair_size(fwA[t], b) != 1 ? 1u : 0u) << u;   // not a singleton
                }
                const int tf = (PARTS - 1 - h) * SC + (SC - 1 - u);   // forward step of window w-1
                if (nxt) {
                    fwB[tf] = g;
                    g = T.fd[g * C + byte_of(cwB, tf)];
                }
            }
            if (cnt && on && static_cast<int>(lenA) > h * SC) {
                // tree count: the part's ambiguous columns right to left, from
                // their staged id pairs; a gap between two of them is a run of
                // singletons, which closes a pending run
                const int top = min(SC - 1, static_cast<int>(lenA) - 1 - h * SC);
                int prev = top + 1;
#pragma unroll 1
                for (uint32_t am = amb; am;) {
                    const int u = 31 - __builtin_clz(am);
                    am &= ~(1u << u);
                    if (u + 1 < prev) rm.single();
                    const uint32_t t = static_cast<uint32_t>(h * SC + u), v = mine[u];
                    const uint32_t fi = v & 0xffffu, bi = v >> 16;
                    const uint32_t br = u + 1 <= top ? mine[u + 1] >> 16 : bright;   // the column to the right
                    const uint64_t col = a0A + t;
                    rm.step(tb, t, pair_size(fi, bi), fi, br, text, col, T.cls, col + 1 == cx.tr.n,
                            col + 2 == cx.tr.n);
                    prev = u;
                }
                if (prev > 0) rm.single();
                bright = mine[0] >> 16;
            }
            amb = 0;
            wave_sync();
            if constexpr (COMPACT) {
                // 16 words per chunk: lanes 16g..16g+15 write chunk 4q+g
                const uint32_t e = lane & 15;
                const uint64_t base = reinterpret_cast<uint64_t>(out + a0A) + static_cast<uint64_t>(h * SC) * 8;
#pragma unroll 1
                for (int q = 0; q < 16; ++q) {
                    const int j = q * 4 + static_cast<int>(lane >> 4);
                    const uint32_t lj = static_cast<uint32_t>(__shfl(static_cast<int>(len_now), j));
                    const uint64_t rj = shfl_u64(base, j);
                    const uint32_t np = lj > static_cast<uint32_t>(h * SC)
                                            ? (lj - h * SC < static_cast<uint32_t>(SC) ? lj - h * SC : SC) : 0;
                    if (e < np) {
                        const uint32_t *sj = wave_rows + j * kStageRow;
                        const uint32_t v = sj[e], pc = sj[SC + e];
                        const uint32_t fi = v & 0xffffu, bi = v >> 16;
                        uint64_t m = 0;
                        // only the words where both sets are non-zero (id 0 is
                        // the empty set: a dead run)
                        const uint32_t nz0 = fi != 0 && bi != 0 ? T.fnz[fi] & T.rnz[bi] : 0u;
                        for (uint32_t nz = nz0; nz; nz &= nz - 1) {
                            const uint32_t ww = static_cast<uint32_t>(__builtin_ctz(nz));
                            for (uint64_t y = T.fb[fi * W + ww] & T.rb[bi * W + ww]; y; y &= y - 1) {
                                const uint32_t sg = ww * 64 + static_cast<uint32_t>(__builtin_ctzll(y));
                                m |= 1ull << rank_of((tb.rank_pq ? (pc & 0xffffu) * tb.NL + (pc >> 16)
                                                                 : (pc & 0xffffu)) * tb.nseg + sg);
                            }
                        }
                        __builtin_nontemporal_store(m, global_ptr<uint64_t>(rj) + e);
                    }
                }
            } else {
                // write columns a0+S*h .. of every chunk of the wavefront
                for (int j = 0; j < 64; ++j) {
                    const uint32_t lj = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(len_now), j));
                    const uint32_t np = lj > static_cast<uint32_t>(h * SC)
                                            ? (lj - h * SC < static_cast<uint32_t>(SC) ? lj - h * SC : SC) : 0;
                    if (np == 0) continue;
                    uint64_t *region = global_ptr<uint64_t>(readlane_u64(reinterpret_cast<uint64_t>(out + a0A * W), j)) +
                                       static_cast<uint64_t>(h * SC) * W;
                    const uint32_t *sj = wave_rows + j * kStageRow;
                    const uint32_t nwords = np * W;
                    if constexpr (BITS_LDS) {
                        for (uint32_t e = lane; e < nwords; e += 64) {
                            const uint32_t p = static_cast<uint32_t>((static_cast<uint64_t>(e) * tb.wmagic) >> 32);
                            const uint32_t ww = e - p * W;
                            const uint32_t v = sj[p];
                            // streaming store: the SLPF is not read back by this kernel
                            __builtin_nontemporal_store(T.fb[(v & 0xffffu) * W + ww] & T.rb[(v >> 16) * W + ww],
                                                        region + e);
                        }
                        continue;
                    }
                    // bit sets in L2: four store rounds at a time, their loads
                    // first (the stores may alias the tables, so the compiler
                    // does not move loads above them)
                    for (uint32_t e0 = lane; e0 < nwords; e0 += 256) {
                        uint64_t y[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const uint32_t e = e0 + 64u * q;
                            y[q] = 0;
                            if (e < nwords) {
                                const uint32_t p = static_cast<uint32_t>((static_cast<uint64_t>(e) * tb.wmagic) >> 32);
                                const uint32_t ww = e - p * W;
                                const uint32_t v = sj[p];
                                y[q] = T.fb[(v & 0xffffu) * W + ww] & T.rb[(v >> 16) * W + ww];
                            }
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const uint32_t e = e0 + 64u * q;
                            // streaming store: the SLPF is not read back by this kernel
                            if (e < nwords) __builtin_nontemporal_store(y[q], region + e);
                        }
                    }
                }
            }
            wave_sync();
        }
        // window w+1 can take no more marks
        if (cnt && on && w + 1 < static_cast<int>(nwin)) {
            jb.amask[ck(jb, i, w + 1)] = rm.wright;
            const uint64_t len = min(64ull, hi - (lo + 64ull * (w + 1)));
            allm = allm && (rm.wright | ~low_mask(static_cast<uint32_t>(len))) == ~0ull;
        }
        if (nxt) {
#pragma unroll
            for (int t = 0; t < 64; ++t) fwA[t] = fwB[t];
#pragma unroll
            for (int k = 0; k < 16; ++k) cwA[k] = cwB[k];
            lenA = 64;
            a0A = lo + 64ull * (w - 1);
        }
    }
    if (act && jb.count_on) {
        if (cx.first) {   // the text's product of long runs and its failure flag
            jb.tprod[2ull * cx.t] = 1;
            jb.tprod[2ull * cx.t + 1] = 1;
            jb.tfail[cx.t] = 0;
        }
        if (cnt) {
            // the column left of the chunk: the text start acts as a singleton;
            // inside the text it is another chunk's, so a pending column is marked
            if (rm.st == 1 || rm.st == 2) {
                if (cx.first) {
                    rm.mul(rm.st == 1 ? rm.pm : rm.pa);
                } else {   // the pending columns lo (and lo + 1, possibly the text end)
                    rm.wcur |= 1ull;
                    if (rm.st == 2) rm.mark_right(0, 1, lo + 1 == cx.tr.n);
                }
            }
            jb.amask[ck(jb, i, 0)] = rm.wcur;
            allm = allm && (rm.wcur | ~low_mask(static_cast<uint32_t>(min(64ull, hi - lo)))) == ~0ull;
            jb.cfull[i] = allm ? 1 : 0;     // every column of the chunk is marked
            if (cx.last) jb.aend[cx.t] = rm.endmark;
            rm.finish();
        }
        jb.cfac[2ull * i] = rm.a64;
        jb.cfac[2ull * i + 1] = rm.ap;
    }
}

// ------------------------------------------------------------ wave helpers

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint32_t>(v)), m));
    const uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint32_t>(v >> 32)), m));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t o = shfl_xor_u64(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ inline uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += shfl_xor_u64(v, off);
    return v;
}

// Compact SLPF to W-word columns: one thread per column r, whose bit k names
// the k-th segment of X[class(x_r), class(x_r+1)] (the sentinel C before the
// text and after it).
__global__ __launch_bounds__(256) void k_decode_compact(Tabs tb, const uint8_t *text, uint64_t n,
                                                        const uint64_t *cmp, uint64_t *out) {
    const uint64_t r = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r > n) return;
    const uint32_t p = r > 0 ? tb.classmap[text[r - 1]] : tb.C;
    const uint32_t q = r < n ? tb.classmap[text[r]] : tb.C;
    const uint16_t *xl = tb.xlist + tb.xoff[p * tb.NL + q];
    const uint64_t m = cmp[r];
    for (uint32_t w = 0; w < tb.W; ++w) {
        uint64_t v = 0;
        for (uint64_t x = m; x; x &= x - 1) {
            const uint32_t sg = xl[__builtin_ctzll(x)];
            if ((sg >> 6) == w) v |= 1ull << (sg & 63);
        }
        out[r * tb.W + w] = v;
    }
}

// The chunk map of a job of several texts: tmap[i] = the text owning chunk
// i (jb.tmap is null in this launch; out is where it goes).
__global__ __launch_bounds__(256) void k_tmap(Job jb, uint32_t *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < jb.c) out[i] = text_search(jb, i);
}

__global__ void k_init(Job jb) {
    if (blockIdx.x == 0 && threadIdx.x < 4) jb.flags[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 8 && jb.count_on) jb.ccnt[threadIdx.x] = 0;   // with the u64 nsruns
}

}  // namespace slpf

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
//   k_count_fast / k_count_list / k_count_general / k_count_factor /
//   k_count_chain / k_text_scalars
//            the number of syntax trees modulo 2^64: the product of the
//            chunks' path-count matrices between their clean edge columns,
//            each factored through an anchor column (a singleton: rank 1;
//            else the smallest column, rank <= kGenR), so that the product
//            falls apart into per-chunk numbers and short chains of small
//            anchor-to-anchor matrices.
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
    const uint8_t *rankx;       // NL x nseg: rank of a segment in X[p, its end-letter class]
    const uint32_t *fnz, *rnz;  // per state: bit w set iff word w of its set is non-zero
    const uint32_t *xoff_nb;    // entry lists filtered by the next byte only (ablation)
    const uint16_t *xlist_nb;
    uint32_t emax_nb;
    const uint64_t *gmask;      // match extraction: ngroups x 3 x W segment masks
    uint32_t ngroups;
    uint32_t col_single;        // reachable forward and reverse states share at most one segment
    uint32_t off16;
    uint32_t fhmask, rhmask;
    uint32_t C, W, NL;          // classes, words, C + 1
    uint32_t nf, nr;            // table sizes including id 0
    uint32_t fstart, rstart;    // ids of I and F
    uint32_t emax;
    uint32_t nseg;
    uint64_t wmagic;            // ceil(2^32 / W): e / W == (e * wmagic) >> 32 for e < 2^16
};

struct Job {
    // texts: a job parses one or many texts with one parser; the lane chunks of
    // all texts form one index space, text t owning chunks tchunk0[t] ..
    // tchunk0[t+1]-1.  With one text the descriptor is carried in d0.
    uint32_t ntexts;
    const uint64_t *tdesc;      // [T][4]: text ptr, n, columns ptr, scalars ptr
    const uint32_t *tchunk0;    // [T+1]
    uint64_t d0[4];
    uint64_t s;                 // lane chunk bytes
    uint32_t c;                 // lane chunks of all texts
    uint16_t *R, *Rh;           // [emax][c] end ids of the reach runs
    uint64_t *Mf, *MbR;         // [c][emax] masks; MbR indexed by c-1-i
    uint8_t *nxf, *nxb;         // entry-list sizes at the scan input of item k (forward: left edge of
                                // chunk k; backward: right edge of chunk c-1-k)
    uint8_t *rsf, *rsb;         // item k starts a text (forward: first chunk; backward: last chunk)
    uint64_t *fin, *fout;       // forward join masks at the left / right edge of chunk i
    uint64_t *bin, *bout;       // backward join masks (reversed item order: index c-1-i)
    uint16_t *fid, *rid;        // build start ids per chunk
    uint16_t *ckpt;             // forward id at the left edge of every 64-byte window
    uint16_t *bckpt;            // backward id at the right edge of every 64-byte window
    uint32_t *flags;            // [0] set not found, [1] chain starts, [2] unused,
                                // [3] chunks for the general count kernel
    uint64_t *trace;            // optional J / J^ words (one text only)
    // tree count
    uint8_t *dims;              // [c][2]: edge column sizes
    uint64_t *uv;               // [c][2][kVec]: u (right edge) then v (left edge) of a rank-1 chunk
    uint64_t *pi;               // [c] scalar factor of a rank-1 chunk
    uint64_t *factor;           // [c + T] chunk factors, then one text-start factor per text
    uint32_t *kind;             // [c]: kRank1, kPending (left to the general kernel), kGeneral,
                                // kSkip, or kOverflow (a column beyond kGenSeg: the count fails)
    uint32_t *ovf;              // chunks left to the general count kernel (count in flags[3])
    uint32_t *chains;           // general chunks that start a chain (count in flags[1])
    uint64_t *gmat;             // [c][kGenR][kGenR]: anchor-to-anchor matrix of a general chunk
    uint64_t *gin;              // [c][kGenR]: row vector into a chain's first anchor
    uint32_t *pend;             // [c]: the chunk after a stretch of general chunks (piece products)
    uint32_t fwd_only;          // recogniser: forward runs and forward join only
    uint32_t compact;           // columns as one word over the candidate list X[x_r, x_r+1]
    uint32_t rank_lds;          // compact build: LDS byte offset of the rank table, 0 = read it from L2
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

// text owning chunk i: the largest t < T with tchunk0[t] <= i
__device__ inline uint32_t text_of(const Job &jb, uint32_t i) {
    if (jb.ntexts == 1) return 0;
    uint32_t lo = 0, hi = jb.ntexts - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (jb.tchunk0[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
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
constexpr int kVec = 12;                      // clean-column segments handled by the fast count
constexpr uint32_t kRank1 = 0xffffffffu;       // chunk matrix held as v * pi * u^T
constexpr uint32_t kOverflow = 0xfffffffeu;    // general chunk beyond the kernel's limits
constexpr uint32_t kPending = 0xfffffffdu;     // chunk left to the general count kernel
constexpr uint32_t kGeneral = 0xfffffffcu;     // chunk matrix held as A * B through an anchor column
constexpr uint32_t kSkip = 0xfffffffbu;        // general chunk with no anchor: walked through
constexpr uint32_t kUncounted = 0u;            // chunk not counted yet
constexpr int kGenR = 8;                       // largest anchor column of a general chunk
constexpr int kGenSeg = 64;                    // largest clean column on a general chunk's walks
static_assert(kGenR * kGenR == 64, "the chain kernels hold one anchor matrix per wavefront, an entry a lane");

__device__ inline bool kind_failed(uint32_t k) { return k != kRank1 && k != kGeneral && k != kSkip; }

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
// reverse (backward); lo is 16-byte aligned, so the body is read with 16-byte
// loads.  Runs that reach the same state are merged (equal states have equal
// futures); `alias` maps entry k of the group to the slot holding its run.
// Slots dead in every lane of the wavefront are skipped.
template <bool FWD, bool OFF, bool GRP>
__device__ inline void run_group(const uint8_t *text, uint64_t lo, uint64_t hi, const uint16_t *cls,
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
    const uint64_t body = (hi - lo) & ~15ull;
    if (!settle()) return;
    if (!FWD)
        for (uint64_t p = hi; p-- > lo + body;) step(text[p]);
    const uint64_t nblk = body >> 4;
    const uint4 *vp = reinterpret_cast<const uint4 *>(text + lo);
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
    if (FWD)
        for (uint64_t p = lo + body; p < hi; ++p) step(text[p]);
}

// OFF: the runs step through the offset form of the tables; states are byte
// offsets (id * 2C) until the end ids are stored.
template <bool LDS, bool OFF>
__global__ __launch_bounds__(256) void k_reach(Tabs tb, Job jb) {
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
    const uint32_t la = boundary_list(tb, bcls, text, cx.tr.n, jb.s, cx.ct, cx.li);
    const uint32_t lb = boundary_list(tb, bcls, text, cx.tr.n, jb.s, cx.ct, cx.li + 1);
    const uint32_t xa0 = tb.xoff[la], na = tb.xoff[la + 1] - xa0;
    const uint32_t xb0 = tb.xoff[lb], nb = tb.xoff[lb + 1] - xb0;
    // scan items: forward item i maps X_i -> X_{i+1}; backward item c-1-i maps X_{i+1} -> X_i
    jb.nxf[i] = static_cast<uint8_t>(na);
    jb.rsf[i] = cx.first ? 1 : 0;
    jb.nxb[jb.c - 1 - i] = static_cast<uint8_t>(nb);
    jb.rsb[jb.c - 1 - i] = cx.last ? 1 : 0;

    // forward runs from X_i
    for (uint32_t g0 = 0; __any(g0 < na); g0 += kGroup) {
        uint32_t st[kGroup];
        uint64_t alias = 0;
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            st[k] = (g0 + k < na) ? tb.fsingle[tb.xlist[xa0 + g0 + k]] * c2 : 0;
            alias |= static_cast<uint64_t>(k) << (4 * k);
        }
        run_group<true, OFF, LDS>(text, lo, hi, lk.cls, lk.fd, tb.C, st, alias);
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            if (g0 + k < na) {
                uint32_t sl = (alias >> (4 * k)) & 15u, v = 0;
#pragma unroll
                for (int q = 0; q < kGroup; ++q)
                    if (sl == static_cast<uint32_t>(q)) v = st[q];
                jb.R[static_cast<uint64_t>(g0 + k) * jb.c + i] = static_cast<uint16_t>(OFF ? v / c2 : v);
            }
        }
    }
    // backward runs from X_{i+1} (not for the recogniser)
    for (uint32_t g0 = 0; !jb.fwd_only && __any(g0 < nb); g0 += kGroup) {
        uint32_t st[kGroup];
        uint64_t alias = 0;
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            st[k] = (g0 + k < nb) ? tb.rsingle[tb.xlist[xb0 + g0 + k]] * c2 : 0;
            alias |= static_cast<uint64_t>(k) << (4 * k);
        }
        run_group<false, OFF, LDS>(text, lo, hi, lk.cls, lk.rd, tb.C, st, alias);
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            if (g0 + k < nb) {
                uint32_t sl = (alias >> (4 * k)) & 15u, v = 0;
#pragma unroll
                for (int q = 0; q < kGroup; ++q)
                    if (sl == static_cast<uint32_t>(q)) v = st[q];
                jb.Rh[static_cast<uint64_t>(g0 + k) * jb.c + i] = static_cast<uint16_t>(OFF ? v / c2 : v);
            }
        }
    }
    // maps between entry lists: forward X_i -> X_{i+1}, backward X_{i+1} -> X_i
    const uint32_t W = tb.W;
    for (uint32_t m = 0; m < na; ++m) {
        uint32_t id = jb.R[static_cast<uint64_t>(m) * jb.c + i];
        const uint64_t *bits = tb.fbits + static_cast<uint64_t>(id) * W;
        uint64_t row = 0;
        for (uint32_t p = 0; p < nb; ++p) {
            uint32_t sg = tb.xlist[xb0 + p];
            row |= ((bits[sg >> 6] >> (sg & 63)) & 1ull) << p;
        }
        jb.Mf[static_cast<uint64_t>(i) * tb.emax + m] = row;
    }
    for (uint32_t m = 0; m < (jb.fwd_only ? 0u : nb); ++m) {
        uint32_t id = jb.Rh[static_cast<uint64_t>(m) * jb.c + i];
        const uint64_t *bits = tb.rbits + static_cast<uint64_t>(id) * W;
        uint64_t row = 0;
        for (uint32_t p = 0; p < na; ++p) {
            uint32_t sg = tb.xlist[xa0 + p];
            row |= ((bits[sg >> 6] >> (sg & 63)) & 1ull) << p;
        }
        jb.MbR[static_cast<uint64_t>(jb.c - 1 - i) * tb.emax + m] = row;
    }
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
    const uint8_t *nx;          // [N] input entry-list size per item
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
    uint8_t *nx[2];
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
        O.nx[d][g] = static_cast<uint8_t>(nx0);
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

// Join sets and build start ids.  Thread i handles chunk i: fid_i = id of
// J at P_i, rid_i = id of J^ at P_{i+1}; the last chunk of a text writes its
// accept flag.
__global__ __launch_bounds__(256) void k_starts(Tabs tb, Job jb) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t c = jb.c, W = tb.W;
    if (i >= c) return;
    const ChunkCtx cx = chunk_ctx(jb, i);
    uint64_t acc[kMaxWords];
    // J at the right edge of chunk k: union of the ends of its runs selected by fin[k]
    auto join_fwd = [&](uint32_t k) -> uint32_t {
        uint64_t sel = jb.fin[k];
        for (uint32_t w = 0; w < W; ++w) acc[w] = 0;
        uint32_t first = 0xffffffffu;
        bool same = true;
        while (sel) {
            int m = __builtin_ctzll(sel);
            sel &= sel - 1;
            uint32_t id = jb.R[static_cast<uint64_t>(m) * c + k];
            if (first == 0xffffffffu) first = id;
            same = same && (id == first);
            const uint64_t *bt = tb.fbits + static_cast<uint64_t>(id) * W;
            for (uint32_t w = 0; w < W; ++w) acc[w] |= bt[w];
        }
        if (first == 0xffffffffu) return 0;
        if (same) return first;
        return lookup_set(tb.fhash, tb.fhmask, tb.fbits, W, acc, jb.flags);
    };
    // J^ at the left edge of chunk k: union of its backward runs selected by the mask at its right edge
    auto join_bwd = [&](uint32_t k) -> uint32_t {
        uint64_t sel = jb.bin[c - 1 - k];      // reversed item c-1-k enters at chunk k's right edge
        for (uint32_t w = 0; w < W; ++w) acc[w] = 0;
        uint32_t first = 0xffffffffu;
        bool same = true;
        while (sel) {
            int m = __builtin_ctzll(sel);
            sel &= sel - 1;
            uint32_t id = jb.Rh[static_cast<uint64_t>(m) * c + k];
            if (first == 0xffffffffu) first = id;
            same = same && (id == first);
            const uint64_t *bt = tb.rbits + static_cast<uint64_t>(id) * W;
            for (uint32_t w = 0; w < W; ++w) acc[w] |= bt[w];
        }
        if (first == 0xffffffffu) return 0;
        if (same) return first;
        return lookup_set(tb.rhash, tb.rhmask, tb.rbits, W, acc, jb.flags);
    };
    const uint32_t f = cx.first ? tb.fstart : join_fwd(i - 1);
    const uint32_t r = cx.last ? tb.rstart : join_bwd(i + 1);
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
            const uint64_t *e = tb.rbits + static_cast<uint64_t>(join_bwd(0)) * W;
            for (uint32_t w = 0; w < W; ++w) Jh[w] = e[w];
        }
    }
    if (cx.last) cx.tr.scalars[0] = jb.fout[i] != 0 ? 1ull : 0ull;
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

// Wavefront-local synchronization: LDS written by some lanes of a wavefront
// is visible to the other lanes of the same wavefront after this point.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
        for (uint32_t k = threadIdx.x; k < tb.NL * tb.nseg; k += blockDim.x) dst[k] = tb.rankx[k];
        __syncthreads();
    }
    auto rank_of = [&](uint32_t idx) -> uint32_t { return jb.rank_lds ? rkl[idx] : tb.rankx[idx]; };
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
                    m |= 1ull << tb.rankx[pc * tb.nseg + sg];
                }
            }
            out[cx.tr.n] = m;
        } else {
            for (uint32_t w = 0; w < W; ++w)
                out[cx.tr.n * W + w] = T.fb[f * W + w] & T.rb[tb.rstart * W + w];
        }
    }

    // backward sweep, two windows in flight; fwA[t] = forward id at column a0+t
    uint32_t b = act ? jb.rid[i] : 0;
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
                    if constexpr (COMPACT) mine[SC + u] = t > 0 ? byte_of(cwA, t - 1) : pA0;
                }
                const int tf = (PARTS - 1 - h) * SC + (SC - 1 - u);   // forward step of window w-1
                if (nxt) {
                    fwB[tf] = g;
                    g = T.fd[g * C + byte_of(cwB, tf)];
                }
            }
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
                                m |= 1ull << rank_of(pc * tb.nseg + sg);
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
                    for (uint32_t e = lane; e < nwords; e += 64) {
                        const uint32_t p = static_cast<uint32_t>((static_cast<uint64_t>(e) * tb.wmagic) >> 32);
                        const uint32_t ww = e - p * W;
                        const uint32_t v = sj[p];
                        // streaming store: the SLPF is not read back by this kernel
                        __builtin_nontemporal_store(T.fb[(v & 0xffffu) * W + ww] & T.rb[(v >> 16) * W + ww], region + e);
                    }
                }
            }
            wave_sync();
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
}

// ------------------------------------------------------ tree count, fast path

// List the segments of the clean column (fi, bi) into seg[0..kVec); returns
// the number of segments (values beyond kVec are not listed).
template <class BT>
__device__ inline uint32_t list_clean(const BT &T, uint32_t W, uint32_t fi, uint32_t bi, uint32_t seg[kVec]) {
    uint32_t m = 0;
    for (uint32_t w = 0; w < W; ++w) {
        uint64_t v = T.fb[fi * W + w] & T.rb[bi * W + w];
        while (v) {
            const uint32_t sg = w * 64 + __builtin_ctzll(v);
            v &= v - 1;
#pragma unroll
            for (int k = 0; k < kVec; ++k)
                if (m == static_cast<uint32_t>(k)) seg[k] = sg;
            ++m;
        }
    }
    return m;
}

__device__ inline bool follows(const uint64_t *folseg, uint32_t W, uint32_t rho, uint32_t sigma) {
    return (folseg[static_cast<uint64_t>(rho) * W + (sigma >> 6)] >> (sigma & 63)) & 1ull;
}

// Wavefront-uniform maximum and minimum.
__device__ inline uint32_t wave_max_small(uint32_t v) {   // v <= 31
    uint32_t r = 0;
#pragma unroll
    for (int bit = 4; bit >= 0; --bit) {
        const uint32_t cand = r | (1u << bit);
        if (__any(v >= cand)) r = cand;
    }
    return r;
}
__device__ inline uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), off)));
    return v;
}

constexpr int kCountThreads = 256;
constexpr int kQuarter = 16;                                // columns staged per row fill
constexpr int kCountRow = kQuarter + 1;                     // padded per-lane row of 16 columns
constexpr int kCountY = 2 * kVec + 1;                       // two count vectors (u64), padded
constexpr int kCountLaneBytes = kCountY * 8 + kCountRow * 4;
constexpr int kCountLdsBytes = kCountThreads * kCountLaneBytes;

// LDS offsets of the count kernel's staged tables after the per-lane areas:
// class map and transition tables, then the sole-segment tables, then (FULL)
// the state bit sets and the follower sets.
struct CountLds {
    uint32_t tab, sole, bits, fol, end;
};
__host__ __device__ inline CountLds count_lds(uint32_t nf, uint32_t nr, uint32_t C, uint32_t W, uint32_t nseg) {
    CountLds o;
    o.tab = kCountLdsBytes;
    o.sole = o.tab + ((512 + (nf + nr) * C * 2 + 15) & ~15u);
    o.bits = o.sole + (((nf + nr) * 2 + 15) & ~15u);
    o.fol = o.bits + (nf + nr) * W * 8;
    o.end = o.fol + nseg * W * 8;
    return o;
}

// When every forward state reachable from I and every reverse state reachable
// from F share at most one segment (col_single), every clean column is a
// singleton and every chunk of
// an accepted text has one path between its edges: the rank-1 factor
// v = u = (1), pi = 1, stored here without reading the text or the columns.
// Empty chunks are left to the count kernels (kUncounted).
constexpr int kSingleThreads = 256;
__global__ __launch_bounds__(kSingleThreads) void k_count_single(Job jb) {
    const uint32_t i = blockIdx.x * kSingleThreads + threadIdx.x;
    if (i >= jb.c) return;
    const ChunkCtx cx = chunk_ctx(jb, i);
    if (cx.tr.scalars[0] != 0 && cx.hi > cx.lo) {
        uint64_t *uv = jb.uv + static_cast<uint64_t>(i) * 2 * kVec;
        for (int k = 0; k < 2 * kVec; ++k) uv[k] = (k == 0 || k == kVec) ? 1ull : 0ull;
        jb.pi[i] = 1;
        jb.dims[2 * i] = 1;
        jb.dims[2 * i + 1] = 1;
        jb.kind[i] = kRank1;
    } else {
        jb.kind[i] = kUncounted;
    }
}

// Fast tree count.  Paths through a singleton clean column all pass through
// its one segment, so a chunk whose columns P_i .. P_{i+1}-1 include a
// singleton column has the rank-1 transfer matrix T = v * pi * u^T from
// column P_i to column P_{i+1}:
//   v[k]  paths from the k-th segment of column P_i to the leftmost singleton;
//   pi    product of the path counts between consecutive singleton columns
//         (a backward vector DP that collapses at every singleton);
//   u[q]  paths from the rightmost singleton r1 to the q-th segment of
//         column P_{i+1} (a forward vector DP from r1).
// A clean column of an accepted text is non-empty and inside both of its
// state sets, so it is the only segment of either state when that state's set
// has one (the sole-segment tables).  Between a singleton and any column
// every arc exists (each segment of a clean column has a neighbour in the next
// and in the previous one), so arcs are looked at only between two ambiguous
// columns, and there only the arcs themselves: a column is its bit set
// bitsF[f] & bitsR[b], the arcs of a segment into the other column are its
// follower row ANDed with that set, and count vectors are indexed by rank in
// the column (kept in the lane's LDS, so a rank is an address).  Per 64-byte
// window the forward ids come from the build's checkpoint and the backward ids
// from its backward checkpoint; each quarter window's (forward, backward) ids
// go to the lane's LDS row, which the DP then walks.  Chunks with no singleton
// or with a column above kVec segments go to the general kernel.
template <bool TAB_LDS, bool FULL>
__global__ __launch_bounds__(kCountThreads) void k_count_fast(Tabs tb, Job jb) {
    extern __shared__ __align__(16) uint8_t smem[];
    if (jb.ntexts == 1 && text_ref(jb, 0).scalars[0] == 0) return;    // rejected text: no tree
    const uint32_t C = tb.C, W = tb.W;
    uint64_t *yb = reinterpret_cast<uint64_t *>(smem) + threadIdx.x * kCountY;   // yb[0..kVec), yb[kVec..2kVec)
    uint32_t *row = reinterpret_cast<uint32_t *>(smem + kCountThreads * kCountY * 8) + threadIdx.x * kCountRow;
    // transition tables and sole-segment tables (and with FULL the bit sets
    // and follower sets) staged in LDS
    const uint16_t *cls, *fd, *rd, *fso, *rso;
    const uint64_t *fbits = tb.fbits, *rbits = tb.rbits, *fol = tb.folseg;
    if constexpr (TAB_LDS) {
        const CountLds o = count_lds(tb.nf, tb.nr, C, W, tb.nseg);
        uint16_t *c16 = reinterpret_cast<uint16_t *>(smem + o.tab);
        uint16_t *f16 = c16 + 256, *r16 = f16 + tb.nf * C;
        uint16_t *fs16 = reinterpret_cast<uint16_t *>(smem + o.sole);
        uint16_t *rs16 = fs16 + tb.nf;
        for (uint32_t k = threadIdx.x; k < 256; k += blockDim.x) c16[k] = tb.classmap[k];
        for (uint32_t k = threadIdx.x; k < tb.nf * C; k += blockDim.x) f16[k] = tb.fdelta[k];
        for (uint32_t k = threadIdx.x; k < tb.nr * C; k += blockDim.x) r16[k] = tb.rdelta[k];
        for (uint32_t k = threadIdx.x; k < tb.nf; k += blockDim.x) fs16[k] = tb.fsole[k];
        for (uint32_t k = threadIdx.x; k < tb.nr; k += blockDim.x) rs16[k] = tb.rsole[k];
        if constexpr (FULL) {
            uint64_t *fb64 = reinterpret_cast<uint64_t *>(smem + o.bits), *rb64 = fb64 + tb.nf * W;
            uint64_t *fl64 = reinterpret_cast<uint64_t *>(smem + o.fol);
            for (uint32_t k = threadIdx.x; k < tb.nf * W; k += blockDim.x) fb64[k] = tb.fbits[k];
            for (uint32_t k = threadIdx.x; k < tb.nr * W; k += blockDim.x) rb64[k] = tb.rbits[k];
            for (uint32_t k = threadIdx.x; k < tb.nseg * W; k += blockDim.x) fl64[k] = tb.folseg[k];
            fbits = fb64, rbits = rb64, fol = fl64;
        }
        __syncthreads();
        cls = c16, fd = f16, rd = r16, fso = fs16, rso = rs16;
    } else {
        cls = tb.classmap, fd = tb.fdelta, rd = tb.rdelta, fso = tb.fsole, rso = tb.rsole;
    }
    struct ClsTab {
        const uint16_t *cls;
    } ct{cls};
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t wave_first = blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
    if (wave_first >= jb.c) return;
    ChunkCtx cx{};
    bool act = i < jb.c;
    if (act) {
        cx = chunk_ctx(jb, i);
        // trees only in accepted texts; with col_single the chunks already counted
        act = cx.tr.scalars[0] != 0 && !(tb.col_single && jb.kind[i] == kRank1);
    }
    const uint8_t *text = cx.tr.text;
    uint64_t lo = 0, hi = 0;
    uint32_t nwin = 0;
    if (act) {
        lo = cx.lo;
        hi = cx.hi;
        nwin = static_cast<uint32_t>((hi - lo + 63) / 64);
    }
    const uint32_t nwin_wave = wave_max_u32(nwin);
    uint32_t xw[16], cw[16], qs[4];              // window bytes, classes, forward id at each quarter start
    uint32_t mp = 0, yc = 0;                     // previous column's size; its vector is yb + yc*kVec
    bool lz = false;                             // that vector is all ylz (a singleton's count, not written)
    uint64_t ylz = 0;
    uint32_t fp = 0, bp = 0;                     // previous column's state ids when it was ambiguous
    uint64_t pi = 1, r1 = 0;
    bool found = false, over = !act;

    // a staged column: (f | b << 16) for the state ids, or (s << 16) when the
    // clean column is the single segment s (f = 0, the empty set, never
    // labels a column of an accepted text)
    auto entry = [&](uint32_t f, uint32_t b) -> uint32_t {
        uint32_t s = fso[f];
        if (s == kNoSole) s = rso[b];
        return s != kNoSole ? (s << 16) : (f | (b << 16));
    };
    auto word = [&](uint32_t f, uint32_t b, uint32_t w) -> uint64_t { return fbits[f * W + w] & rbits[b * W + w]; };
    // number of segments of a staged column
    auto column = [&](bool live, uint32_t e) -> uint32_t {
        const bool multi = live && (e & 0xffffu) != 0;
        uint32_t m = live ? 1u : 0u;
        if (__any(multi)) {
            if (multi) {
                m = 0;
                for (uint32_t w = 0; w < W; ++w) m += __popcll(word(e & 0xffffu, e >> 16, w));
            }
        }
        return m;
    };
    // one DP step onto the column e (m segments) from the previous column (mp
    // segments); fwd: the previous column is the left one; collapse: multiply
    // pi at singletons (backward pass).  Each case other than singleton to
    // singleton sits behind a wavefront-uniform test.
    auto step = [&](bool live, uint32_t m, uint32_t e, bool fwd, bool collapse) {
        uint64_t *yprev = yb + yc * kVec, *ycur = yb + (yc ^ 1u) * kVec;
        const uint32_t f = e & 0xffffu, b = e >> 16;
        const bool gen = live && m > 1 && mp > 1;
        if (__any(gen)) {
            if (gen && lz) {   // write out the broadcast count before the arcs read it
                for (uint32_t j = 0; j < mp; ++j) yprev[j] = ylz;
                lz = false;
            }
            if (gen && !fwd) {
                // backward: y[k] over the current (left) column gathers the counts of
                // the followers of its k-th segment in the previous (right) column
                uint32_t k = 0;
                for (uint32_t w = 0; w < W; ++w) {
                    uint64_t cv = word(f, b, w);
                    while (cv) {
                        const uint32_t sk = w * 64 + __builtin_ctzll(cv);
                        cv &= cv - 1;
                        uint64_t acc = 0;
                        uint32_t pre = 0;
                        for (uint32_t v = 0; v < W; ++v) {
                            const uint64_t pv = word(fp, bp, v);
                            uint64_t a = fol[static_cast<uint64_t>(sk) * W + v] & pv;
                            while (a) {
                                const uint32_t s = __builtin_ctzll(a);
                                a &= a - 1;
                                acc += yprev[pre + __popcll(pv & low_mask(s))];
                            }
                            pre += __popcll(pv);
                        }
                        ycur[k++] = acc;
                    }
                }
            } else if (gen) {
                // forward: each segment of the previous (left) column adds its count
                // to its followers in the current (right) column
                for (uint32_t k = 0; k < m; ++k) ycur[k] = 0;
                uint32_t j = 0;
                for (uint32_t v = 0; v < W; ++v) {
                    uint64_t pv = word(fp, bp, v);
                    while (pv) {
                        const uint32_t sj = v * 64 + __builtin_ctzll(pv);
                        pv &= pv - 1;
                        const uint64_t val = yprev[j++];
                        uint32_t pre = 0;
                        for (uint32_t w = 0; w < W; ++w) {
                            const uint64_t cwv = word(f, b, w);
                            uint64_t a = fol[static_cast<uint64_t>(sj) * W + w] & cwv;
                            while (a) {
                                const uint32_t s = __builtin_ctzll(a);
                                a &= a - 1;
                                ycur[pre + __popcll(cwv & low_mask(s))] += val;
                            }
                            pre += __popcll(cwv);
                        }
                    }
                }
            }
        }
        const bool sum = live && m == 1 && mp > 1;     // every segment of the previous column reaches the singleton
        if (__any(sum)) {
            if (sum) {
                uint64_t t = 0;
                if (lz) {
                    t = ylz * mp;
                } else {
                    for (uint32_t j = 0; j < mp; ++j) t += yprev[j];
                }
                yprev[0] = t;
                lz = false;
            }
        }
        // the singleton reaches every segment of this column: the vector is
        // its count everywhere, kept as one number until arcs need it
        if (live && m > 1 && mp == 1) {
            lz = true;
            ylz = yprev[0];
        }
        if (collapse && live && m == 1 && mp > 1) {
            pi *= yprev[0];
            yprev[0] = 1;
        }
        if (live) {
            if (m > 1) {
                yc ^= 1u;          // the current column's vector becomes the previous one
                fp = f;
                bp = b;
            }
            mp = m;
        }
    };
    // forward ids at the quarter starts of window w (columns a0, a0+16, a0+32,
    // a0+48) into qs; returns the id after the window
    auto quarter_starts = [&](uint32_t w, uint32_t len) -> uint32_t {
        uint32_t g = jb.ckpt[ck(jb, i, w)];
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            if ((t & (kQuarter - 1)) == 0) qs[t / kQuarter] = g;
            if (t < static_cast<int>(len)) g = fd[g * C + byte_of(cw, t)];
        }
        return g;
    };

    // backward over the chunk's columns hi-1 .. lo
    for (int w = static_cast<int>(nwin_wave) - 1; w >= 0; --w) {
        const bool on = !over && w < static_cast<int>(nwin);
        uint64_t a0 = 0;
        uint32_t len = 0, b = 0;
        if (on) {
            a0 = lo + 64ull * w;
            len = static_cast<uint32_t>(hi - a0 < 64 ? hi - a0 : 64);
            load_window(text, a0, len, xw);
            window_classes(ct, xw, cw);
            quarter_starts(w, len);
            b = jb.bckpt[ck(jb, i, w)];
        }
#pragma unroll 1
        for (int q = 3; q >= 0; --q) {
            if (on) {
                // one static copy per quarter: register arrays indexed by constants only
                // (an index that depends on q would put them in scratch memory)
                auto stage_bwd = [&](auto qc) {
                    constexpr int Q = decltype(qc)::value;
                    uint32_t fq[kQuarter];               // forward ids at columns a0+16Q .. a0+16Q+15
                    uint32_t g = qs[Q];
#pragma unroll
                    for (int u = 0; u < kQuarter; ++u) {
                        fq[u] = g;
                        if (Q * kQuarter + u < static_cast<int>(len)) g = fd[g * C + byte_of(cw, Q * kQuarter + u)];
                    }
#pragma unroll
                    for (int u = kQuarter - 1; u >= 0; --u) {
                        const int t = Q * kQuarter + u;
                        if (t < static_cast<int>(len)) {
                            b = rd[b * C + byte_of(cw, t)];
                            row[u] = entry(fq[u], b);
                        }
                    }
                };
                if (q == 3) stage_bwd(std::integral_constant<int, 3>{});
                else if (q == 2) stage_bwd(std::integral_constant<int, 2>{});
                else if (q == 1) stage_bwd(std::integral_constant<int, 1>{});
                else stage_bwd(std::integral_constant<int, 0>{});
            }
#pragma unroll 1
            for (int u = kQuarter - 1; u >= 0; --u) {
                const int t = q * kQuarter + u;
                bool live = on && !over && t < static_cast<int>(len);
                const uint32_t e = live ? row[u] : 0u;
                uint32_t m = column(live, e);
                if (live && (m > static_cast<uint32_t>(kVec) || m == 0)) {
                    over = true;
                    live = false;
                }
                if (live && !found) {
                    if (m == 1) {
                        found = true;
                        r1 = a0 + t;
                        yb[yc * kVec] = 1;
                        mp = 1;
                        lz = false;
                    }
                    live = false;
                }
                step(live, m, e, false, true);
            }
        }
    }
    if (act && !over && !found) over = true;          // no singleton column in the chunk
    const uint32_t mL = mp;
    if (act && !over) {
        uint64_t *uv = jb.uv + static_cast<uint64_t>(i) * 2 * kVec;
        const uint64_t *yv = yb + yc * kVec;
        for (int k = 0; k < kVec; ++k) uv[kVec + k] = k < static_cast<int>(mL) ? (lz ? ylz : yv[k]) : 0ull;
    }

    // forward from r1 to column hi = P_{i+1}
    yc = 0;
    yb[0] = 1;
    mp = 1;
    lz = false;
    const bool fw_on = act && !over;
    const uint32_t w_first = wave_min(fw_on ? static_cast<uint32_t>((r1 - lo) / 64) : 0xffffffffu);
    for (uint32_t w = w_first; w < nwin_wave; ++w) {
        const bool on = fw_on && w < nwin;
        uint64_t a0 = 0;
        uint32_t len = 0, f_end = 0, b_end = 0;
        if (on) {
            a0 = lo + 64ull * w;
            len = static_cast<uint32_t>(hi - a0 < 64 ? hi - a0 : 64);
            load_window(text, a0, len, xw);
            window_classes(ct, xw, cw);
            f_end = quarter_starts(w, len);
            b_end = jb.bckpt[ck(jb, i, w)];
        }
#pragma unroll 1
        for (int q = 0; q < 4; ++q) {
            // (forward, backward) ids of the columns a0+16q+1 .. a0+16q+16 below
            // a0+len into row[0..16); the column a0+len is (f_end, b_end).  The
            // backward ids run from the window's right edge, first over the
            // bytes above the quarter.  One static copy per quarter.
            if (on) {
                auto stage_fwd = [&](auto qc) {
                    constexpr int Q = decltype(qc)::value;
                    uint32_t fq[kQuarter];               // forward ids at columns a0+16Q+1 .. a0+16Q+16
                    uint32_t g = qs[Q];
#pragma unroll
                    for (int u = 0; u < kQuarter; ++u) {
                        if (Q * kQuarter + u < static_cast<int>(len)) g = fd[g * C + byte_of(cw, Q * kQuarter + u)];
                        fq[u] = g;
                    }
                    uint32_t b = b_end;
#pragma unroll
                    for (int t = 63; t >= Q * kQuarter + 1; --t) {
                        if (t < static_cast<int>(len)) {
                            b = rd[b * C + byte_of(cw, t)];       // backward id at column a0+t
                            if (t <= Q * kQuarter + kQuarter) row[t - Q * kQuarter - 1] = entry(fq[t - Q * kQuarter - 1], b);
                        }
                    }
                };
                if (q == 3) stage_fwd(std::integral_constant<int, 3>{});
                else if (q == 2) stage_fwd(std::integral_constant<int, 2>{});
                else if (q == 1) stage_fwd(std::integral_constant<int, 1>{});
                else stage_fwd(std::integral_constant<int, 0>{});
            }
#pragma unroll 1
            for (int u = 0; u < kQuarter; ++u) {   // column a0 + 16q + u + 1
                const int t = q * kQuarter + u + 1;
                const uint64_t col = a0 + t;
                bool live = on && !over && t <= static_cast<int>(len) && col > r1;
                uint32_t e = 0;
                if (live) e = t == static_cast<int>(len) ? entry(f_end, b_end) : row[u];
                uint32_t m = column(live, e);
                if (live && (m > static_cast<uint32_t>(kVec) || m == 0)) {
                    over = true;
                    live = false;
                }
                step(live, m, e, true, false);
            }
        }
    }
    if (act && over) {
        jb.kind[i] = kPending;
        jb.ovf[atomicAdd(&jb.flags[3], 1u)] = i;
        return;
    }
    if (!act) return;
    uint64_t *uv = jb.uv + static_cast<uint64_t>(i) * 2 * kVec;
    const uint64_t *yv = yb + yc * kVec;
    for (int k = 0; k < kVec; ++k) uv[k] = k < static_cast<int>(mp) ? (lz ? ylz : yv[k]) : 0ull;
    jb.pi[i] = pi;
    jb.dims[2 * i] = static_cast<uint8_t>(mL);
    jb.dims[2 * i + 1] = static_cast<uint8_t>(mp);
    jb.kind[i] = kRank1;
}

// ---- tree count for wide columns (W > 2): segment lists in LDS

constexpr int kListThreads = 512;
constexpr int kListRow = kQuarter + 1;                     // padded per-lane row of 16 columns
constexpr int kListSegWords = kVec;                        // two lists of kVec u16 segment ids
constexpr int kListLaneBytes = (kListRow + kListSegWords) * 4;
constexpr int kListLdsBytes = kListThreads * kListLaneBytes;

// LDS offsets of the count kernel's staged tables after the per-lane areas:
// class map and transition tables, then the sole-segment tables, then (FULL)
// the state bit sets and the follower sets.
struct ListLds {
    uint32_t tab, sole, bits, fol, end;
};
__host__ __device__ inline ListLds list_lds(uint32_t nf, uint32_t nr, uint32_t C, uint32_t W, uint32_t nseg) {
    ListLds o;
    o.tab = kListLdsBytes;
    o.sole = o.tab + ((512 + (nf + nr) * C * 2 + 15) & ~15u);
    o.bits = o.sole + (((nf + nr) * 2 + 15) & ~15u);
    o.fol = o.bits + (nf + nr) * W * 8;
    o.end = o.fol + nseg * W * 8;
    return o;
}

// Fast tree count.  Paths through a singleton clean column all pass through
// its one segment, so a chunk whose columns P_i .. P_{i+1}-1 include a
// singleton column has the rank-1 transfer matrix T = v * pi * u^T from
// column P_i to column P_{i+1}:
//   v[k]  paths from the k-th segment of column P_i to the leftmost singleton;
//   pi    product of the path counts between consecutive singleton columns
//         (a backward vector DP that collapses at every singleton);
//   u[q]  paths from the rightmost singleton r1 to the q-th segment of
//         column P_{i+1} (a forward vector DP from r1).
// A clean column of an accepted text is non-empty and inside both of its
// state sets, so it is the only segment of either state when that state's set
// has one (the sole-segment tables); only columns where both sets hold
// several segments are listed from the bit sets.  Between a singleton and any
// column every arc exists (each segment of a clean column has a neighbour in
// the next and in the previous one), so the follower relation is read only
// between two ambiguous columns.  Per 64-byte window the forward ids come
// from the build's checkpoint and the backward ids from its backward
// checkpoint; each half window's (forward, backward) id pairs go to the
// lane's LDS row, which the DP then walks.  Segment lists of the current and
// the previous column live in the lane's LDS too, so the vector state in
// registers is only the path counts.  Chunks with no singleton or with a
// column above kVec segments go to the general kernel.
template <bool TAB_LDS, bool FULL>
__global__ __launch_bounds__(kListThreads) void k_count_list(Tabs tb, Job jb) {
    extern __shared__ __align__(16) uint8_t smem[];
    if (jb.ntexts == 1 && text_ref(jb, 0).scalars[0] == 0) return;    // rejected text: no tree
    const uint32_t C = tb.C, W = tb.W;
    uint32_t *row = reinterpret_cast<uint32_t *>(smem) + threadIdx.x * kListRow;
    uint16_t *segl = reinterpret_cast<uint16_t *>(smem + kListThreads * kListRow * 4) + threadIdx.x * 2 * kVec;
    // transition tables and sole-segment tables (and with FULL the bit sets
    // and follower sets) staged in LDS
    const uint16_t *cls, *fd, *rd, *fso, *rso;
    const uint64_t *fbits = tb.fbits, *rbits = tb.rbits, *fol = tb.folseg;
    if constexpr (TAB_LDS) {
        const ListLds o = list_lds(tb.nf, tb.nr, C, W, tb.nseg);
        uint16_t *c16 = reinterpret_cast<uint16_t *>(smem + o.tab);
        uint16_t *f16 = c16 + 256, *r16 = f16 + tb.nf * C;
        uint16_t *fs16 = reinterpret_cast<uint16_t *>(smem + o.sole);
        uint16_t *rs16 = fs16 + tb.nf;
        for (uint32_t k = threadIdx.x; k < 256; k += blockDim.x) c16[k] = tb.classmap[k];
        for (uint32_t k = threadIdx.x; k < tb.nf * C; k += blockDim.x) f16[k] = tb.fdelta[k];
        for (uint32_t k = threadIdx.x; k < tb.nr * C; k += blockDim.x) r16[k] = tb.rdelta[k];
        for (uint32_t k = threadIdx.x; k < tb.nf; k += blockDim.x) fs16[k] = tb.fsole[k];
        for (uint32_t k = threadIdx.x; k < tb.nr; k += blockDim.x) rs16[k] = tb.rsole[k];
        if constexpr (FULL) {
            uint64_t *fb64 = reinterpret_cast<uint64_t *>(smem + o.bits), *rb64 = fb64 + tb.nf * W;
            uint64_t *fl64 = reinterpret_cast<uint64_t *>(smem + o.fol);
            for (uint32_t k = threadIdx.x; k < tb.nf * W; k += blockDim.x) fb64[k] = tb.fbits[k];
            for (uint32_t k = threadIdx.x; k < tb.nr * W; k += blockDim.x) rb64[k] = tb.rbits[k];
            for (uint32_t k = threadIdx.x; k < tb.nseg * W; k += blockDim.x) fl64[k] = tb.folseg[k];
            fbits = fb64, rbits = rb64, fol = fl64;
        }
        __syncthreads();
        cls = c16, fd = f16, rd = r16, fso = fs16, rso = rs16;
    } else {
        cls = tb.classmap, fd = tb.fdelta, rd = tb.rdelta, fso = tb.fsole, rso = tb.rsole;
    }
    struct ClsTab {
        const uint16_t *cls;
    } ct{cls};
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t wave_first = blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
    if (wave_first >= jb.c) return;
    ChunkCtx cx{};
    bool act = i < jb.c;
    if (act) {
        cx = chunk_ctx(jb, i);
        // trees only in accepted texts; with col_single the chunks already counted
        act = cx.tr.scalars[0] != 0 && !(tb.col_single && jb.kind[i] == kRank1);
    }
    const uint8_t *text = cx.tr.text;
    uint64_t lo = 0, hi = 0;
    uint32_t nwin = 0;
    if (act) {
        lo = cx.lo;
        hi = cx.hi;
        nwin = static_cast<uint32_t>((hi - lo + 63) / 64);
    }
    const uint32_t nwin_wave = wave_max_u32(nwin);
    uint32_t xw[16], cw[16], qs[4];              // window bytes, classes, forward id at each quarter start
    uint64_t y[kVec];                            // path counts over the previous column's segments
#pragma unroll
    for (int k = 0; k < kVec; ++k) y[k] = 0;
    uint32_t mp = 0, ep = 0;                     // previous column's size, and its entry when ambiguous
    uint64_t pi = 1, r1 = 0;
    bool found = false, over = !act;

    // a staged column: (f | b << 16) for the state ids, or (s << 16) when the
    // clean column is the single segment s (f = 0, the empty set, never
    // labels a column of an accepted text)
    auto entry = [&](uint32_t f, uint32_t b) -> uint32_t {
        uint32_t s = fso[f];
        if (s == kNoSole) s = rso[b];
        return s != kNoSole ? (s << 16) : (f | (b << 16));
    };
    // number of segments of a staged column
    auto column = [&](bool live, uint32_t e) -> uint32_t {
        const bool multi = live && (e & 0xffffu) != 0;
        uint32_t m = live ? 1u : 0u;
        if (__any(multi)) {
            if (multi) {
                const uint32_t f = e & 0xffffu, b = e >> 16;
                m = 0;
                for (uint32_t w = 0; w < W; ++w) m += static_cast<uint32_t>(__popcll(fbits[f * W + w] & rbits[b * W + w]));
            }
        }
        return m;
    };
    // the segments of an ambiguous column (entry e) into lst[0..kVec)
    auto list_into = [&](uint32_t e, uint16_t *lst) {
        const uint32_t f = e & 0xffffu, b = e >> 16;
        uint32_t m = 0;
        for (uint32_t w = 0; w < W; ++w) {
            uint64_t v = fbits[f * W + w] & rbits[b * W + w];
            while (v) {
                if (m < static_cast<uint32_t>(kVec)) lst[m] = static_cast<uint16_t>(w * 64 + __builtin_ctzll(v));
                v &= v - 1;
                ++m;
            }
        }
    };
    // one DP step onto the column e (m segments) from the previous column
    // (mp segments, entry ep when mp > 1); fwd: the previous column is the
    // left one; collapse: multiply pi at singletons (backward pass).  The
    // segment lists are made only for a step between two ambiguous columns (a
    // step from or to a singleton needs no arcs).  Each case other than
    // singleton-to-singleton sits behind a wavefront-uniform test, so a
    // wavefront skips the cases none of its lanes needs.
    auto step = [&](bool live, uint32_t m, uint32_t e, bool fwd, bool collapse) {
        const bool gen = live && m > 1 && mp > 1;
        if (__any(gen)) {   // ambiguous to ambiguous: follower checks, uniform bounds over those lanes
            const uint32_t mw = wave_max_small(gen ? m : 0), mpw = wave_max_small(gen ? mp : 0);
            uint16_t *lc = segl, *lp = segl + kVec;
            if (gen) {
                list_into(e, lc);
                list_into(ep, lp);
            }
            uint64_t z[kVec];
#pragma unroll
            for (int k = 0; k < kVec; ++k) z[k] = 0;
#pragma unroll 1
            for (uint32_t k = 0; k < mw; ++k) {
                const bool on_k = gen && k < m;
                const uint32_t sk = on_k ? lc[k] : 0u;
                uint64_t acc = 0;
#pragma unroll
                for (int j = 0; j < kVec; ++j) {
                    if (j < static_cast<int>(mpw) && on_k && j < static_cast<int>(mp)) {
                        const uint32_t sj = lp[j];
                        const bool arc = fwd ? follows(fol, W, sj, sk) : follows(fol, W, sk, sj);
                        if (arc) acc += y[j];
                    }
                }
#pragma unroll
                for (int kk = 0; kk < kVec; ++kk)
                    if (static_cast<uint32_t>(kk) == k) z[kk] = acc;
            }
            if (gen) {
#pragma unroll
                for (int k = 0; k < kVec; ++k) y[k] = z[k];
            }
        }
        const bool sum = live && m == 1 && mp > 1;     // every segment of the previous column reaches the singleton
        if (__any(sum)) {
            if (sum) {
                uint64_t t = 0;
#pragma unroll
                for (int j = 0; j < kVec; ++j) t += j < static_cast<int>(mp) ? y[j] : 0ull;
                y[0] = t;
            }
        }
        const bool bcast = live && m > 1 && mp == 1;   // the singleton reaches every segment of this column
        if (__any(bcast)) {
            if (bcast) {
                const uint64_t y0 = y[0];
#pragma unroll
                for (int k = 0; k < kVec; ++k) y[k] = k < static_cast<int>(m) ? y0 : 0ull;
            }
        }
        if (collapse && live && m == 1) {
            pi *= y[0];
            y[0] = 1;
        }
        if (live) {
            if (m > 1) ep = e;
            mp = m;
        }
    };
    // forward ids at the quarter starts of window w (columns a0, a0+16, a0+32,
    // a0+48) into qs; returns the id after the window
    auto quarter_starts = [&](uint32_t w, uint32_t len) -> uint32_t {
        uint32_t g = jb.ckpt[ck(jb, i, w)];
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            if ((t & (kQuarter - 1)) == 0) qs[t / kQuarter] = g;
            if (t < static_cast<int>(len)) g = fd[g * C + byte_of(cw, t)];
        }
        return g;
    };

    // backward over the chunk's columns hi-1 .. lo
    for (int w = static_cast<int>(nwin_wave) - 1; w >= 0; --w) {
        const bool on = !over && w < static_cast<int>(nwin);
        uint64_t a0 = 0;
        uint32_t len = 0, b = 0;
        if (on) {
            a0 = lo + 64ull * w;
            len = static_cast<uint32_t>(hi - a0 < 64 ? hi - a0 : 64);
            load_window(text, a0, len, xw);
            window_classes(ct, xw, cw);
            quarter_starts(w, len);
            b = jb.bckpt[ck(jb, i, w)];
        }
#pragma unroll 1
        for (int q = 3; q >= 0; --q) {
            // backward ids of the quarter, with the forward ids, into the lane's row
            // (q selects between static register indices: no indexed registers)
            if (on) {
                // one static copy per quarter: register arrays indexed by constants only
                auto stage_bwd = [&](auto qc) {
                    constexpr int Q = decltype(qc)::value;
                    uint32_t fq[kQuarter];               // forward ids at columns a0+16Q .. a0+16Q+15
                    uint32_t g = qs[Q];
#pragma unroll
                    for (int u = 0; u < kQuarter; ++u) {
                        fq[u] = g;
                        if (Q * kQuarter + u < static_cast<int>(len)) g = fd[g * C + byte_of(cw, Q * kQuarter + u)];
                    }
#pragma unroll
                    for (int u = kQuarter - 1; u >= 0; --u) {
                        const int t = Q * kQuarter + u;
                        if (t < static_cast<int>(len)) {
                            b = rd[b * C + byte_of(cw, t)];
                            row[u] = entry(fq[u], b);
                        }
                    }
                };
                if (q == 3) stage_bwd(std::integral_constant<int, 3>{});
                else if (q == 2) stage_bwd(std::integral_constant<int, 2>{});
                else if (q == 1) stage_bwd(std::integral_constant<int, 1>{});
                else stage_bwd(std::integral_constant<int, 0>{});
            }
#pragma unroll 1
            for (int u = kQuarter - 1; u >= 0; --u) {
                const int t = q * kQuarter + u;
                bool live = on && !over && t < static_cast<int>(len);
                const uint32_t e = live ? row[u] : 0u;
                uint32_t m = column(live, e);
                if (live && (m > static_cast<uint32_t>(kVec) || m == 0)) {
                    over = true;
                    live = false;
                }
                if (live && !found) {
                    if (m == 1) {
                        found = true;
                        r1 = a0 + t;
                        y[0] = 1;
                        mp = 1;
                    }
                    live = false;
                }
                step(live, m, e, false, true);
            }
        }
    }
    if (act && !over && !found) over = true;          // no singleton column in the chunk
    const uint32_t mL = mp;
    if (act && !over) {
        uint64_t *uv = jb.uv + static_cast<uint64_t>(i) * 2 * kVec;
#pragma unroll
        for (int k = 0; k < kVec; ++k) uv[kVec + k] = k < static_cast<int>(mL) ? y[k] : 0ull;
    }

    // forward from r1 to column hi = P_{i+1}
#pragma unroll
    for (int k = 0; k < kVec; ++k) y[k] = 0;
    y[0] = 1;
    mp = 1;
    const bool fw_on = act && !over;
    const uint32_t w_first = wave_min(fw_on ? static_cast<uint32_t>((r1 - lo) / 64) : 0xffffffffu);
    for (uint32_t w = w_first; w < nwin_wave; ++w) {
        const bool on = fw_on && w < nwin;
        uint64_t a0 = 0;
        uint32_t len = 0, f_end = 0, b_end = 0;
        if (on) {
            a0 = lo + 64ull * w;
            len = static_cast<uint32_t>(hi - a0 < 64 ? hi - a0 : 64);
            load_window(text, a0, len, xw);
            window_classes(ct, xw, cw);
            f_end = quarter_starts(w, len);
            b_end = jb.bckpt[ck(jb, i, w)];
        }
#pragma unroll 1
        for (int q = 0; q < 4; ++q) {
            // (forward, backward) ids of the columns a0+16q+1 .. a0+16q+16 below
            // a0+len into row[0..16); the column a0+len is (f_end, b_end).  One
            // static copy per quarter.
            if (on) {
                auto stage_fwd = [&](auto qc) {
                    constexpr int Q = decltype(qc)::value;
                    uint32_t fq[kQuarter];               // forward ids at columns a0+16Q+1 .. a0+16Q+16
                    uint32_t g = qs[Q];
#pragma unroll
                    for (int u = 0; u < kQuarter; ++u) {
                        if (Q * kQuarter + u < static_cast<int>(len)) g = fd[g * C + byte_of(cw, Q * kQuarter + u)];
                        fq[u] = g;
                    }
                    uint32_t b = b_end;
#pragma unroll
                    for (int t = 63; t >= Q * kQuarter + 1; --t) {
                        if (t < static_cast<int>(len)) {
                            b = rd[b * C + byte_of(cw, t)];       // backward id at column a0+t
                            if (t <= Q * kQuarter + kQuarter) row[t - Q * kQuarter - 1] = entry(fq[t - Q * kQuarter - 1], b);
                        }
                    }
                };
                if (q == 3) stage_fwd(std::integral_constant<int, 3>{});
                else if (q == 2) stage_fwd(std::integral_constant<int, 2>{});
                else if (q == 1) stage_fwd(std::integral_constant<int, 1>{});
                else stage_fwd(std::integral_constant<int, 0>{});
            }
#pragma unroll 1
            for (int u = 0; u < kQuarter; ++u) {   // column a0 + 16q + u + 1
                const int t = q * kQuarter + u + 1;
                const uint64_t col = a0 + t;
                bool live = on && !over && t <= static_cast<int>(len) && col > r1;
                uint32_t e = 0;
                if (live) e = t == static_cast<int>(len) ? entry(f_end, b_end) : row[u];
                uint32_t m = column(live, e);
                if (live && (m > static_cast<uint32_t>(kVec) || m == 0)) {
                    over = true;
                    live = false;
                }
                step(live, m, e, true, false);
            }
        }
    }
    if (act && over) {
        jb.kind[i] = kPending;
        jb.ovf[atomicAdd(&jb.flags[3], 1u)] = i;
        return;
    }
    if (!act) return;
    uint64_t *uv = jb.uv + static_cast<uint64_t>(i) * 2 * kVec;
#pragma unroll
    for (int k = 0; k < kVec; ++k) uv[k] = k < static_cast<int>(mp) ? y[k] : 0ull;
    jb.pi[i] = pi;
    jb.dims[2 * i] = static_cast<uint8_t>(mL);
    jb.dims[2 * i + 1] = static_cast<uint8_t>(mp);
    jb.kind[i] = kRank1;
}

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

// Count factors.  The count of a text is the all-ones row over its column 0
// times the chunk matrices times the all-ones column over column n.  A rank-1
// chunk g contributes factor[g] = pi_g times u_g^T carried to the next anchor:
// u_g . v_{g+1} when the next chunk is rank-1, the sum of u_g at the text end.
// factor[c + t] for text t is the all-ones row carried to the first anchor:
// the sum of v over the first chunk when it is rank-1.  When the next chunk
// (or the first chunk) is general, the chain kernel writes these factors.
// General chunks contribute 1.
__global__ __launch_bounds__(256) void k_count_factor(Job jb) {
    const uint32_t c = jb.c;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= c + jb.ntexts) return;
    const uint32_t t = g < c ? text_of(jb, g) : g - c;
    const TextRef tr = text_ref(jb, t);
    if (tr.n == 0 || tr.scalars[0] == 0) {
        jb.factor[g] = 1;
        return;
    }
    const uint32_t c0 = first_chunk(jb, t), c1 = first_chunk(jb, t + 1);
    if (g >= c) {
        if (jb.kind[c0] != kRank1) return;                 // the chain kernel's
        const uint32_t dim = jb.dims[2 * c0];
        const uint64_t *v = jb.uv + static_cast<uint64_t>(c0) * 2 * kVec + kVec;
        uint64_t d = 0;
        for (uint32_t k = 0; k < dim; ++k) d += v[k];
        jb.factor[g] = d;
        return;
    }
    if (jb.kind[g] != kRank1) {
        jb.factor[g] = 1;
        return;
    }
    const uint64_t *u = jb.uv + static_cast<uint64_t>(g) * 2 * kVec;
    const uint32_t dim = jb.dims[2 * g + 1];
    uint64_t d = 0;
    if (g + 1 == c1) {
        for (uint32_t k = 0; k < dim; ++k) d += u[k];
    } else if (jb.kind[g + 1] == kRank1) {
        const uint64_t *v = jb.uv + static_cast<uint64_t>(g + 1) * 2 * kVec + kVec;
        for (uint32_t k = 0; k < dim; ++k) d += u[k] * v[k];
    } else {
        return;                                            // the chain kernel's
    }
    jb.factor[g] = jb.pi[g] * d;
}

// Products of the anchor-to-anchor matrices over pieces of 64 chunks: one
// wavefront per piece multiplies, in order, the matrices of each stretch of
// general chunks of one text inside the piece (a run cut at the piece's
// edges), a chunk without an anchor counting as the identity.  The product
// replaces the matrix of the stretch's first chunk, and pend[first] is the
// chunk after the stretch.  Lane 8k+b holds entry (k, b); entry (k, b) of
// P G is the sum over m of P(k, m) G(m, b), P(k, m) taken from lane 8k+m.
__global__ __launch_bounds__(64) void k_count_piece(Job jb) {
    const uint32_t L = threadIdx.x, k = L >> 3, b = L & 7;
    const uint32_t p0 = blockIdx.x * 64;
    if (p0 >= jb.c) return;
    const uint32_t np = jb.c - p0 < 64 ? jb.c - p0 : 64;
    // lane l: kind of chunk p0+l (rank-1 for chunks of rejected texts) and
    // its text
    uint32_t kd = kRank1, tl = 0;
    if (L < np) {
        tl = text_of(jb, p0 + L);
        if (text_ref(jb, tl).scalars[0] != 0) kd = jb.kind[p0 + L];
    }
    if (!__any(kd != kRank1)) return;
    const uint64_t ident = k == b ? 1ull : 0ull;
    uint64_t P = ident;
    int st = -1;
    uint32_t ts = 0;
    uint64_t gc[kGenR], gn[kGenR];
#pragma unroll
    for (int m = 0; m < kGenR; ++m) gc[m] = jb.gmat[static_cast<uint64_t>(p0) * kGenR * kGenR + m * kGenR + b];
    for (uint32_t l = 0; l < np; ++l) {
        // the next chunk's column b in flight while this one is applied
        const uint32_t ln = l + 1 < np ? l + 1 : l;
#pragma unroll
        for (int m = 0; m < kGenR; ++m) gn[m] = jb.gmat[static_cast<uint64_t>(p0 + ln) * kGenR * kGenR + m * kGenR + b];
        const uint32_t kl = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(kd), static_cast<int>(l)));
        const uint32_t tcur = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(tl), static_cast<int>(l)));
        const bool gen = kl != kRank1;
        if (st >= 0 && (!gen || tcur != ts)) {
            jb.gmat[static_cast<uint64_t>(p0 + st) * kGenR * kGenR + L] = P;
            if (L == 0) jb.pend[p0 + st] = p0 + l;
            st = -1;
        }
        if (gen) {
            if (st < 0) {
                st = static_cast<int>(l);
                ts = tcur;
                P = ident;
            }
            if (kl == kGeneral) {
                uint64_t q = 0;
#pragma unroll
                for (int m = 0; m < kGenR; ++m) q += shfl_u64(P, static_cast<int>(k * kGenR + m)) * gc[m];
                P = q;
            }
        }
#pragma unroll
        for (int m = 0; m < kGenR; ++m) gc[m] = gn[m];
    }
    if (st >= 0) {
        jb.gmat[static_cast<uint64_t>(p0 + st) * kGenR * kGenR + L] = P;
        if (L == 0) jb.pend[p0 + st] = p0 + np;
    }
}

// Chains through general chunks: one wavefront per run of general chunks (a
// text's first chunks, or the chunks after a rank-1 chunk, up to the next
// rank-1 chunk or the text end).  The row vector gin[j0] of its first chunk
// j0 is multiplied by the run's piece products in order; the last anchor
// matrix has one column, so the product is a number (and when the run has no
// anchor, gin[j0] is that number already): the factor of the rank-1 chunk
// before j0 (times its pi), or the text-start factor.  Lane 8k+b holds entry
// (k, b) of the current matrix and entry k of the row vector; entry b of
// the product is the sum over the lanes b, b+8, ..., b+56.
__global__ __launch_bounds__(64) void k_count_chain(Job jb) {
    const uint32_t L = threadIdx.x, k = L >> 3;
    for (uint32_t item = blockIdx.x; item < jb.flags[1]; item += gridDim.x) {
        const uint32_t j0 = jb.chains[item];
        const uint32_t t = text_of(jb, j0);
        const uint32_t c0 = first_chunk(jb, t), c1 = first_chunk(jb, t + 1);
        uint64_t vk = jb.gin[static_cast<uint64_t>(j0) * kGenR + k];
        uint32_t j = j0;
        while (true) {
            const uint64_t gm = jb.gmat[static_cast<uint64_t>(j) * kGenR * kGenR + L];
            const uint32_t e = jb.pend[j];
            uint64_t p = vk * gm;
            p += shfl_xor_u64(p, 8);
            p += shfl_xor_u64(p, 16);
            p += shfl_xor_u64(p, 32);
            vk = shfl_u64(p, static_cast<int>(k));   // entry k of the new row vector
            // the run goes on into the next piece
            if (e < c1 && e % 64 == 0 && jb.kind[e] != kRank1) j = e;
            else break;
        }
        if (L == 0) {
            if (j0 == c0) jb.factor[jb.c + t] = vk;   // entry 0 of the final row (one column)
            else jb.factor[j0 - 1] = jb.pi[j0 - 1] * vk;
        }
    }
}

// Per-text scalars: one block per text (count: 0 not requested, 1 requested,
// 2 recogniser).  Empty text: column 0 = I & F and
// one tree per initial-and-final segment.  Otherwise the count is the
// product of the text's factors modulo 2^64 (0 for a rejected text); status
// 2 when not requested, 1 when the general count failed on a chunk of the
// text, 3 when a join set was not a table state.
constexpr int kScalarThreads = 1024;

__global__ __launch_bounds__(kScalarThreads) void k_text_scalars(Tabs tb, Job jb, int count) {
    __shared__ uint64_t part[kScalarThreads];
    __shared__ uint32_t failed;
    const uint32_t t = blockIdx.x, th = threadIdx.x;
    const TextRef tr = text_ref(jb, t);
    if (count == 2) {   // recogniser: accept from the forward join alone
        if (th == 0) {
            uint64_t any = 0;
            if (tr.n == 0) {
                const uint64_t *fb = tb.fbits + static_cast<uint64_t>(tb.fstart) * tb.W;
                const uint64_t *rb = tb.rbits + static_cast<uint64_t>(tb.rstart) * tb.W;
                for (uint32_t w = 0; w < tb.W; ++w) any |= fb[w] & rb[w];
            } else {
                any = jb.fout[first_chunk(jb, t + 1) - 1];
            }
            tr.scalars[0] = any ? 1 : 0;
            tr.scalars[1] = 0;
            tr.scalars[2] = jb.flags[0] ? 3 : 2;
        }
        return;
    }
    if (tr.n == 0) {
        if (th == 0) {
            const uint64_t *fb = tb.fbits + static_cast<uint64_t>(tb.fstart) * tb.W;
            const uint64_t *rb = tb.rbits + static_cast<uint64_t>(tb.rstart) * tb.W;
            uint64_t any = 0, pc = 0, cm = 0;
            for (uint32_t w = 0; w < tb.W; ++w) {
                const uint64_t v = fb[w] & rb[w];
                if (!jb.compact) tr.out[w] = v;
                any |= v;
                pc += __popcll(v);
                for (uint64_t x = v; x; x &= x - 1)   // compact: ranks in X[start, end]
                    cm |= 1ull << tb.rankx[tb.C * tb.nseg + w * 64 + static_cast<uint32_t>(__builtin_ctzll(x))];
            }
            if (jb.compact) tr.out[0] = cm;
            tr.scalars[0] = any ? 1 : 0;
            tr.scalars[1] = count ? pc : 0;
            tr.scalars[2] = count ? 0 : 2;
        }
        return;
    }
    uint64_t st = 0, val = 0;
    if (!count) {
        st = 2;
    } else if (tr.scalars[0] == 0) {
        st = 0;
    } else {
        const uint32_t c0 = first_chunk(jb, t), c1 = first_chunk(jb, t + 1);
        if (th == 0) failed = 0;
        __syncthreads();
        // eight independent products per thread keep eight loads in flight
        uint64_t acc[8] = {1, 1, 1, 1, 1, 1, 1, 1};
        bool bad = false;
        const uint32_t stride = blockDim.x;
        uint32_t k = c0 + th;
        for (; k + 7 * stride < c1; k += 8 * stride) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                acc[u] *= jb.factor[k + u * stride];
                bad = bad || kind_failed(jb.kind[k + u * stride]);
            }
        }
        for (; k < c1; k += stride) {
            acc[0] *= jb.factor[k];
            bad = bad || kind_failed(jb.kind[k]);
        }
        if (bad) atomicOr(&failed, 1u);
        part[th] = acc[0] * acc[1] * acc[2] * acc[3] * acc[4] * acc[5] * acc[6] * acc[7];
        __syncthreads();
        for (uint32_t h = kScalarThreads / 2; h; h >>= 1) {
            if (th < h) part[th] *= part[th + h];
            __syncthreads();
        }
        if (failed) st = 1;
        else val = part[0] * jb.factor[jb.c + t];
    }
    if (jb.flags[0]) st = 3;
    if (th == 0) {
        tr.scalars[1] = val;
        tr.scalars[2] = st;
    }
}

// ---- tree count, general chunks: a chunk with no singleton column, or with
// a column above kVec segments.  Its matrix M = T(lo -> hi) (paths between
// the segments of its edge columns) is factored through an anchor column a,
// the leftmost column of [lo, hi] with the fewest segments, when that column
// has r <= kGenR segments: M = A B with A = T(lo -> a), B = T(a -> hi).  The
// kernel stores the anchor-to-anchor matrix G = T(a -> a'), with a' the next
// anchor of the run (unit vectors), or the next rank-1 chunk's left edge
// weighed by its v, or the text end weighed by ones; r x r' zero-padded to
// kGenR x kGenR.  A chunk whose smallest column is larger has no anchor and
// is walked through by its neighbours' products, so the count never depends
// on where the lane chunks fall.  The first chunk of a run stores the row
// vector w^T T(lo -> first anchor) with w the previous chunk's u or the
// all-ones row.  Each product is one backward walk over the clean columns:
// count vectors y_c[k] (paths from the k-th segment of column c to the start
// vectors) go from column c+1 to c along the arcs rho -> sigma with sigma a
// follower of rho.  One wavefront per chunk; lane k holds segment k of the
// current column; the columns are staged kGenBlock at a time in LDS with
// their segment lists.

constexpr int kGenBlock = 32;                  // columns staged per block
constexpr int kGenYRows = kGenSeg;             // count vector rows

// LDS of the general kernel (one wavefront): staged column words and prefix
// counts (row 0 is the column above the block), segment lists, two count
// vector buffers, and the follower table when it fits.
struct GenLds {
    uint32_t colw, pre, segl, mcnt, y, fol, end;
};

__host__ __device__ inline GenLds gen_lds(uint32_t W, uint32_t nseg, bool fol_lds) {
    GenLds o{};
    uint32_t at = 0;
    o.colw = at;
    at += (kGenBlock + 1) * W * 8;
    o.y = at;
    at += 2 * kGenYRows * kGenR * 8;
    o.pre = at;
    at += (kGenBlock + 1) * W * 2;
    o.segl = at;
    at += kGenBlock * kGenSeg * 2;
    o.mcnt = at;
    at += (kGenBlock + 1) * 4 + 4;
    at = (at + 15u) & ~15u;
    o.fol = at;
    if (fol_lds) at += nseg * W * 8;
    o.end = at;
    return o;
}

struct GenCtx {
    const uint64_t *out;     // the text's clean columns
    const uint64_t *fol;     // follower table (LDS or global)
    uint64_t *colw, *y;
    uint16_t *pre, *segl;
    uint32_t *mcnt;
    uint32_t W;
    // compact columns: one word over the candidate list X[class(x_r), class(x_r+1)]
    bool compact;
    const uint8_t *text;
    uint64_t n;
    const uint16_t *cls, *xlist;
    const uint32_t *xoff;
    uint32_t C, NL;
};

// Segment count of column col.
__device__ inline uint32_t gen_colsize(const GenCtx &g, uint64_t col) {
    if (g.compact) return static_cast<uint32_t>(__popcll(g.out[col]));
    const uint64_t *cw = g.out + col * g.W;
    uint32_t m = 0;
    for (uint32_t w = 0; w < g.W; ++w) m += __popcll(cw[w]);
    return m;
}

// Leftmost column of [lo, hi] with the fewest segments, as
// (segments << 40) | (column - lo).
__device__ inline uint64_t gen_anchor(const GenCtx &g, uint64_t lo, uint64_t hi) {
    uint64_t best = ~0ull;
    for (uint64_t col = lo + threadIdx.x; col <= hi; col += 64) {
        const uint32_t m = gen_colsize(g, col);
        const uint64_t key = (static_cast<uint64_t>(m) << 40) | (col - lo);
        best = key < best ? key : best;
    }
    return wave_min_u64(best);
}

// Backward walk from column `from` down to column `to` (to <= from).  VB <=
// kGenR count vectors start at column `from`: start(k, v) for its k-th
// segment.  On return lane k < m_to holds y_to[k][v] in acc[v] (zero for v
// >= VB).  Returns false when a column of the walk has more than kGenSeg
// segments.
template <int VB, class Start>
__device__ inline bool gen_walk(const GenCtx &g, uint64_t from, uint64_t to, Start start, uint64_t acc[kGenR],
                                uint32_t *m_to) {
    const uint32_t lane = threadIdx.x, W = g.W;
    uint32_t yc = 0;
    bool first = true;
    uint32_t m = 0;
    for (uint64_t top = from;; top -= kGenBlock) {
        const uint32_t rows = static_cast<uint32_t>(top - to + 1 < kGenBlock ? top - to + 1 : kGenBlock);
        // row 0: the column above the block (the previous block's last row)
        if (!first) {
            for (uint32_t w = lane; w < W; w += 64) {
                g.colw[w] = g.colw[kGenBlock * W + w];
                g.pre[w] = g.pre[kGenBlock * W + w];
            }
            if (lane == 0) g.mcnt[0] = g.mcnt[kGenBlock];
        }
        __syncthreads();
        // rows 1..rows: columns top, top-1, ...; lane l lists its column
        bool big = false;
        if (lane < rows) {
            const uint32_t row = lane + 1;
            const uint64_t col = top - lane;
            uint64_t *rw = g.colw + row * W;
            if (g.compact) {   // the column's words from its candidate list
                for (uint32_t w = 0; w < W; ++w) rw[w] = 0;
                const uint32_t p = col > 0 ? g.cls[g.text[col - 1]] : g.C;
                const uint32_t q = col < g.n ? g.cls[g.text[col]] : g.C;
                const uint16_t *xl = g.xlist + g.xoff[p * g.NL + q];
                for (uint64_t m = g.out[col]; m; m &= m - 1) {
                    const uint32_t sg = xl[__builtin_ctzll(m)];
                    rw[sg >> 6] |= 1ull << (sg & 63);
                }
            } else {
                const uint64_t *cw = g.out + col * W;
                for (uint32_t w = 0; w < W; ++w) rw[w] = cw[w];
            }
            uint32_t cnt = 0;
            for (uint32_t w = 0; w < W; ++w) {
                uint64_t v = rw[w];
                g.pre[row * W + w] = static_cast<uint16_t>(cnt);
                while (v) {
                    const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(v));
                    v &= v - 1;
                    if (cnt < kGenSeg) g.segl[lane * kGenSeg + cnt] = static_cast<uint16_t>(w * 64 + b);
                    ++cnt;
                }
            }
            g.mcnt[row] = cnt;
            big = cnt > kGenSeg;
        }
        if (__any(big)) return false;
        __syncthreads();
        for (uint32_t r = 1; r <= rows; ++r) {
            m = g.mcnt[r];
            uint64_t a[kGenR];
#pragma unroll
            for (int v = 0; v < kGenR; ++v) a[v] = 0;
            if (first && r == 1) {
                if (lane < m) {
#pragma unroll
                    for (int v = 0; v < VB; ++v) a[v] = start(lane, v);
                }
            } else if (lane < m) {
                const uint64_t *yprev = g.y + yc * kGenYRows * kGenR;
                const uint32_t s = g.segl[(r - 1) * kGenSeg + lane];
                const uint64_t *nx = g.colw + (r - 1) * W;
                const uint16_t *np = g.pre + (r - 1) * W;
                for (uint32_t w = 0; w < W; ++w) {
                    const uint64_t cwd = nx[w];
                    uint64_t f = g.fol[s * W + w] & cwd;
                    while (f) {
                        const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(f));
                        f &= f - 1;
                        const uint32_t rk = np[w] + static_cast<uint32_t>(__popcll(cwd & low_mask(b)));
                        const uint64_t *yr = yprev + rk * kGenR;
#pragma unroll
                        for (int v = 0; v < VB; ++v) a[v] += yr[v];
                    }
                }
            }
            yc ^= 1u;
            if (lane < m) {
                uint64_t *ycur = g.y + yc * kGenYRows * kGenR + lane * kGenR;
#pragma unroll
                for (int v = 0; v < VB; ++v) ycur[v] = a[v];
            }
#pragma unroll
            for (int v = 0; v < kGenR; ++v) acc[v] = a[v];
            __syncthreads();
        }
        first = false;
        if (top - rows + 1 == to) break;
    }
    *m_to = m;
    return true;
}

// The first anchor at or after chunk jj of a run (the chunks after a rank-1
// chunk or the text start that are not rank-1): the leftmost smallest column
// of the first chunk whose smallest column has at most kGenR segments; else
// the left edge of the run's closing rank-1 chunk, whose v weighs it; else
// the text end, weighed by ones.
struct GenTarget {
    uint64_t col;
    uint32_t how;            // 0: unit vectors over r segments, 1: v of chunk h, 2: ones
    uint32_t h;
    uint32_t r;              // start vectors
};

__device__ inline GenTarget gen_next(const GenCtx &g, const Job &jb, const ChunkCtx &cx, uint32_t c0, uint32_t jj) {
    for (;; ++jj) {
        const uint32_t li = jj - c0;
        if (li == cx.ct) return {cx.tr.n, 2u, 0u, 1u};
        const uint64_t lo = static_cast<uint64_t>(li) * jb.s;
        if (jb.kind[jj] == kRank1) return {lo, 1u, jj, 1u};
        const uint64_t hi = li + 1 == cx.ct ? cx.tr.n : lo + jb.s;
        const uint64_t key = gen_anchor(g, lo, hi);
        const uint32_t r = static_cast<uint32_t>(key >> 40);
        if (r <= static_cast<uint32_t>(kGenR)) return {lo + (key & ((1ull << 40) - 1)), 0u, 0u, r};
    }
}

template <bool FOL_LDS>
__global__ __launch_bounds__(64) void k_count_general(Tabs tb, Job jb) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t W = tb.W, lane = threadIdx.x;
    const GenLds o = gen_lds(W, tb.nseg, FOL_LDS);
    GenCtx g;
    g.colw = reinterpret_cast<uint64_t *>(smem + o.colw);
    g.y = reinterpret_cast<uint64_t *>(smem + o.y);
    g.pre = reinterpret_cast<uint16_t *>(smem + o.pre);
    g.segl = reinterpret_cast<uint16_t *>(smem + o.segl);
    g.mcnt = reinterpret_cast<uint32_t *>(smem + o.mcnt);
    g.W = W;
    g.compact = jb.compact != 0;
    g.cls = tb.classmap;
    g.xlist = tb.xlist;
    g.xoff = tb.xoff;
    g.C = tb.C;
    g.NL = tb.NL;
    if constexpr (FOL_LDS) {
        uint64_t *f = reinterpret_cast<uint64_t *>(smem + o.fol);
        for (uint32_t k = lane; k < tb.nseg * W; k += 64) f[k] = tb.folseg[k];
        g.fol = f;
    } else {
        g.fol = tb.folseg;
    }
    __syncthreads();
    for (uint32_t item = blockIdx.x; item < jb.flags[3]; item += gridDim.x) {
        const uint32_t j = jb.ovf[item];
        const ChunkCtx cx = chunk_ctx(jb, j);
        const uint32_t c0 = j - cx.li;
        g.out = cx.tr.out;
        g.text = cx.tr.text;
        g.n = cx.tr.n;
        const bool starts = cx.first || jb.kind[j - 1] == kRank1;
        const uint64_t key = gen_anchor(g, cx.lo, cx.hi);
        const bool anchored = (key >> 40) <= static_cast<uint64_t>(kGenR);
        const uint64_t a = cx.lo + (key & ((1ull << 40) - 1));
        bool ok = true;
        uint64_t acc[kGenR];
        uint32_t mt = 0;
        auto walk_to = [&](const GenTarget &tg, uint64_t to) -> bool {
            const uint64_t *vh = jb.uv + static_cast<uint64_t>(tg.h) * 2 * kVec + kVec;
            auto start = [&](uint32_t k, int v) -> uint64_t {
                if (tg.how == 0) return k == static_cast<uint32_t>(v) ? 1ull : 0ull;
                if (v != 0) return 0ull;
                return tg.how == 1 ? vh[k] : 1ull;
            };
            if (tg.r <= 1) return gen_walk<1>(g, tg.col, to, start, acc, &mt);
            if (tg.r <= 2) return gen_walk<2>(g, tg.col, to, start, acc, &mt);
            if (tg.r <= 4) return gen_walk<4>(g, tg.col, to, start, acc, &mt);
            return gen_walk<kGenR>(g, tg.col, to, start, acc, &mt);
        };
        // the row into the run: w^T T(lo -> first anchor), w the previous
        // chunk's u or ones (a number when the run has no anchor)
        if (starts) {
            const GenTarget tg = anchored ? GenTarget{a, 0u, 0u, static_cast<uint32_t>(key >> 40)}
                                          : gen_next(g, jb, cx, c0, j + 1);
            ok = walk_to(tg, cx.lo);
            if (ok) {
                const uint64_t wk = lane >= mt ? 0ull
                                    : cx.first ? 1ull
                                               : jb.uv[static_cast<uint64_t>(j - 1) * 2 * kVec + lane];
                uint64_t row[kGenR];
#pragma unroll
                for (int v = 0; v < kGenR; ++v) row[v] = wave_sum_u64(wk * acc[v]);
                if (lane == 0) {
#pragma unroll
                    for (int v = 0; v < kGenR; ++v) jb.gin[static_cast<uint64_t>(j) * kGenR + v] = row[v];
                }
            }
        }
        // anchor-to-anchor matrix G = T(a -> next anchor), weighed at the far end
        if (ok && anchored) {
            const GenTarget tg = gen_next(g, jb, cx, c0, j + 1);
            ok = walk_to(tg, a);
            if (ok && lane < static_cast<uint32_t>(kGenR)) {
                // lane k < r holds row k; rows r..kGenR-1 are zero
                uint64_t *gm = jb.gmat + static_cast<uint64_t>(j) * kGenR * kGenR;
#pragma unroll
                for (int v = 0; v < kGenR; ++v) gm[lane * kGenR + v] = lane < mt ? acc[v] : 0ull;
            }
        }
        if (lane == 0) {
            jb.kind[j] = !ok ? kOverflow : anchored ? kGeneral : kSkip;
            if (starts) jb.chains[atomicAdd(&jb.flags[1], 1u)] = j;
        }
        __syncthreads();
    }
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

__global__ void k_init(Job jb) {
    if (blockIdx.x == 0 && threadIdx.x < 4) jb.flags[threadIdx.x] = 0;
}

}  // namespace slpf

// Tree count of the SLPF parser: the number of syntax trees of every
// accepted text modulo 2^64 and modulo the prime 2^61 - 1.
//
// A syntax tree is one accepting run of the parser NFA (Sect. 2.3.4), i.e.
// one path through the clean SLPF that starts in column 0, ends in column n
// and steps from a segment rho of column r-1 to a follower sigma of rho in
// column r.  Every such path passes through the one segment of each singleton
// column, and every segment of a clean column lies on some path, so all arcs
// exist between a singleton column and its neighbours.  The count is
// therefore the product, over the maximal runs of ambiguous columns (two or
// more segments), of the number of paths that enter the run's first column
// anywhere and leave its last column anywhere; the text start and end act as
// singletons.
//
//   k_build          multiplies in the one-column runs inside a lane chunk
//                    (such a run has as many paths as the column has
//                    segments) and marks every other column of a run
//                    (RunMarks);
//   k_count_runs     one thread per 64-column window finds the marked runs
//                    that start in it; a short run whose columns hold at
//                    most kTV segments is counted by a vector walk in
//                    registers, the window's other short runs go to
//                    k_count_defer, long runs (more than Job::lshort
//                    columns) to the piece kernels;
//   k_count_defer    one wavefront per deferred window walks its short runs
//                    with the count vector in LDS, a segment a lane;
//   k_count_pieces   a long run is cut at anchor columns, the leftmost
//                    smallest column of each cell of Job::cell columns when
//                    it holds at most kPieceR segments; one wavefront per
//                    piece computes the path counts between its two anchors
//                    (a matrix of at most kPieceR x kPieceR);
//   k_count_chain    one wavefront per long run multiplies its pieces;
//   k_text_scalars   one block per text multiplies the chunk products and the
//                    long-run products.
// Products and sums are taken modulo 2^64 and modulo 2^61 - 1 side by side.
#pragma once

#include "kernels.hpp"

namespace slpf {

// ------------------------------------------------------ modular arithmetic

__device__ inline uint64_t addp(uint64_t a, uint64_t b) {   // a, b < 2^61 - 1
    const uint64_t s = a + b;
    return s >= kP61 ? s - kP61 : s;
}

struct Cnt {                 // a count modulo 2^64 and modulo 2^61 - 1
    uint64_t a, p;
};
__device__ inline Cnt cmul(Cnt x, Cnt y) { return {x.a * y.a, mulp(x.p, y.p)}; }
__device__ inline Cnt cadd(Cnt x, Cnt y) { return {x.a + y.a, addp(x.p, y.p)}; }

// Sum over the wavefront of both moduli.
__device__ inline Cnt wave_sum_cnt(Cnt x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        x.a += shfl_xor_u64(x.a, off);
        x.p = addp(x.p, shfl_xor_u64(x.p, off));
    }
    return x;
}

// Multiply the count pair at p (mod 2^64, mod 2^61 - 1) by x; several
// threads may do it at once (both products are commutative).
__device__ inline void cmul_at(uint64_t *p, Cnt x) {
    unsigned long long *pa = reinterpret_cast<unsigned long long *>(p);
    unsigned long long *pp = pa + 1;
    unsigned long long old = *pa, seen;
    do {
        seen = old;
        old = atomicCAS(pa, seen, seen * x.a);
    } while (old != seen);
    old = *pp;
    do {
        seen = old;
        old = atomicCAS(pp, seen, static_cast<unsigned long long>(mulp(seen, x.p)));
    } while (old != seen);
}

__device__ inline void tprod_mul(const Job &jb, uint32_t t, Cnt x) { cmul_at(jb.tprod + 2ull * t, x); }

// ------------------------------------------------------------ marked runs

struct TextCols {
    const uint64_t *out;     // the text's clean columns (W words each, or one compact word)
    const uint8_t *text;
    uint64_t n;
    uint32_t t, c0;          // text index, its first lane chunk
};

__device__ inline TextCols text_cols(const Job &jb, uint32_t t) {
    const TextRef tr = text_ref(jb, t);
    return {tr.out, tr.text, tr.n, t, first_chunk(jb, t)};
}

// Marks of the 64-column window that holds column r < n (bit r % 64).
__device__ inline uint64_t mark_word(const Job &jb, const TextCols &tc, uint64_t r) {
    // in windows: the lane chunk of r and the window inside it (s is a multiple of 64)
    const uint32_t rw = static_cast<uint32_t>(r >> 6), sw = static_cast<uint32_t>(jb.s >> 6);
    const uint32_t li = rw / sw;
    return jb.amask[ck(jb, tc.c0 + li, rw - li * sw)];
}

__device__ inline bool marked(const Job &jb, const TextCols &tc, uint64_t r) {
    if (r == tc.n) return (jb.aend[tc.t] & 1ull) != 0;
    return ((mark_word(jb, tc, r) >> (r & 63)) & 1ull) != 0;
}

// Last column of the marked run that starts at r0.  Mark words are scanned
// 64 columns at a time; a lane chunk whose columns are all marked is
// skipped whole.
__device__ inline uint64_t run_end(const Job &jb, const TextCols &tc, uint64_t r0) {
    uint64_t e = r0;
    while (true) {
        const uint64_t nx = e + 1;
        if (nx > tc.n) break;
        if (nx == tc.n) {
            if (jb.aend[tc.t] & 1ull) e = nx;
            break;
        }
        const uint32_t nw = static_cast<uint32_t>(nx >> 6), sw = static_cast<uint32_t>(jb.s >> 6);
        if ((nx & 63) == 0 && nw % sw == 0) {       // a lane chunk starts at nx
            const uint32_t li = nw / sw;
            if (jb.cfull[tc.c0 + li]) {
                e = min(nx + jb.s, tc.n) - 1;       // through its last column
                continue;
            }
        }
        const uint32_t sh = static_cast<uint32_t>(nx & 63);
        const uint64_t v = mark_word(jb, tc, nx) >> sh;
        const uint32_t ones = ~v == 0 ? 64u : static_cast<uint32_t>(__builtin_ctzll(~v));
        if (ones == 0) break;
        e = nx + ones - 1;
        // the run ends inside this word, unless it reaches column n - 1: the
        // text-end column n has its mark outside the windows
        if (sh + ones < 64 && e + 1 < tc.n) break;
    }
    return e;
}

// Calls f(r0) for the first column of every marked run that starts in
// window w of lane chunk i (its columns lo + 64 w .., and n after the last
// window of a text), in column order.
template <class F>
__device__ inline void for_window_run_starts(const Job &jb, const TextCols &tc, uint32_t i, uint32_t w,
                                             const ChunkCtx &cx, F f) {
    const uint32_t nwin = static_cast<uint32_t>((cx.hi - cx.lo + 63) / 64);
    uint64_t carry;
    if (w > 0) carry = jb.amask[ck(jb, i, w - 1)] >> 63;
    else carry = cx.li > 0 && marked(jb, tc, cx.lo - 1) ? 1ull : 0ull;
    const uint64_t v = jb.amask[ck(jb, i, w)];
    uint64_t st = v & ~((v << 1) | carry);
    while (st) {
        const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(st));
        st &= st - 1;
        f(cx.lo + 64ull * w + b);
    }
    if (cx.last && w + 1 == nwin && (jb.aend[tc.t] & 1ull) && !marked(jb, tc, tc.n - 1)) f(tc.n);
}

// Calls f(k, segment) for the segments of column r in ascending order;
// returns their number.  Compact columns: bit k of the word names the k-th
// segment of the candidate list X[class(x_r), class(x_{r+1})].
template <class F>
__device__ inline uint32_t for_segments(const Tabs &tb, const Job &jb, const TextCols &tc, uint64_t r, F f) {
    uint32_t k = 0;
    if (jb.compact) {
        const uint32_t p = r > 0 ? tb.classmap[tc.text[r - 1]] : tb.C;
        const uint32_t q = r < tc.n ? tb.classmap[tc.text[r]] : tb.C;
        const uint16_t *xl = tb.xlist + tb.xoff[p * tb.NL + q];
        for (uint64_t m = tc.out[r]; m; m &= m - 1) f(k++, static_cast<uint32_t>(xl[__builtin_ctzll(m)]));
    } else {
        const uint64_t *cw = tc.out + r * tb.W;
        auto word = [&](uint32_t w, uint64_t v) {
            for (; v; v &= v - 1) f(k++, w * 64 + static_cast<uint32_t>(__builtin_ctzll(v)));
        };
        uint32_t w = 0;
        if ((reinterpret_cast<uintptr_t>(cw) & 15u) == 0)      // two words per 16-byte load
            for (; w + 2 <= tb.W; w += 2) {
                const uint4 q = *reinterpret_cast<const uint4 *>(cw + w);
                word(w, (static_cast<uint64_t>(q.y) << 32) | q.x);
                word(w + 1, (static_cast<uint64_t>(q.w) << 32) | q.z);
            }
        for (; w < tb.W; ++w) word(w, cw[w]);
    }
    return k;
}

__device__ inline uint32_t column_size(const Tabs &tb, const Job &jb, const TextCols &tc, uint64_t r) {
    if (jb.compact) return static_cast<uint32_t>(__popcll(tc.out[r]));
    const uint64_t *cw = tc.out + r * tb.W;
    uint32_t m = 0;
    for (uint32_t w = 0; w < tb.W; ++w) m += static_cast<uint32_t>(__popcll(cw[w]));
    return m;
}

__device__ inline bool follows(const Tabs &tb, uint32_t rho, uint32_t sigma) {
    return (tb.folseg[static_cast<uint64_t>(rho) * tb.W + (sigma >> 6)] >> (sigma & 63)) & 1ull;
}

// The same over a copy of FolSeg (nseg x W words, e.g. in LDS).
__device__ inline bool follows(const uint64_t *fol, uint32_t W, uint32_t rho, uint32_t sigma) {
    return (fol[rho * W + (sigma >> 6)] >> (sigma & 63)) & 1ull;
}

// ------------------------------------------------------- short runs, lanes

constexpr int kTV = 8;               // largest column of a run counted in registers (first pass)
constexpr int kTV2 = 16;             // the same, second pass
constexpr uint32_t kDeferRun = 0x80000000u;   // deferred item: a queued short run, not a window

// x mod 2^61 - 1 for any 64-bit x (2^61 = 1: one fold leaves at most
// 2^61 + 6, one subtraction the rest).
__device__ __forceinline__ uint64_t foldp(uint64_t x) {
    const uint64_t r = (x & kP61) + (x >> 61);
    return r >= kP61 ? r - kP61 : r;
}

// One column step of a lane's path counts: ya/yp over the mp segments sp of
// the previous column become the counts over the m segments sn of the next
// (each the sum over its predecessors).  The pair loops stop at the largest
// columns among the wavefront's active lanes (the bounds are uniform, so the
// rest is skipped).  NW = 1, 2 or 4: FolSeg rows of at most NW words;
// segment j's row is loaded once and tested for every k in registers.  NW
// = 0: any width, one FolSeg word loaded per pair.  The adds are masked
// (NW > 0) or branched (NW = 0, where the per-pair loads dominate); the
// sums modulo 2^61 - 1 are folded once per 7 terms (the folded sum and 7
// terms below 2^61 stay below 2^64).
template <int TV, int NW>
__device__ __forceinline__ void paths_step(const uint64_t *fol, uint32_t W, const uint32_t (&sp)[TV], uint32_t mp,
                                           const uint32_t (&sn)[TV], uint32_t m, uint64_t (&ya)[TV],
                                           uint64_t (&yp)[TV]) {
    uint64_t za[TV], zp[TV];
#pragma unroll
    for (int k = 0; k < TV; ++k) {
        za[k] = 0;
        zp[k] = 0;
    }
#pragma unroll
    for (int j = 0; j < TV; ++j) {
        if (!__any(static_cast<uint32_t>(j) < mp)) break;
        const bool jon = static_cast<uint32_t>(j) < mp;
        uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
        if (NW > 0 && jon) {
            const uint64_t *row = fol + static_cast<uint64_t>(sp[j]) * W;
            w0 = row[0];
            if (NW > 1 && W > 1) w1 = row[1];
            if (NW > 2 && W > 2) w2 = row[2];
            if (NW > 2 && W > 3) w3 = row[3];
        }
        const uint64_t a = jon ? ya[j] : 0ull, b = jon ? yp[j] : 0ull;
#pragma unroll
        for (int k = 0; k < TV; ++k) {
            if (!__any(static_cast<uint32_t>(k) < m)) break;
            const uint32_t sg = sn[k];
            if (NW == 0) {
                // one FolSeg word per pair; hits are sparse, so the adds branch
                // (sn[k >= m] is stale and is not read)
                if (jon && static_cast<uint32_t>(k) < m && follows(fol, W, sp[j], sg)) {
                    za[k] += a;
                    zp[k] += b;
                }
                continue;
            }
            uint64_t x;
            if (NW == 1) x = w0;
            else if (NW == 2) x = (sg & 64u) ? w1 : w0;
            else x = (sg & 128u) ? ((sg & 64u) ? w3 : w2) : ((sg & 64u) ? w1 : w0);
            const uint64_t msk = (static_cast<uint32_t>(k) < m && ((x >> (sg & 63)) & 1ull)) ? ~0ull : 0ull;
            za[k] += a & msk;
            zp[k] += b & msk;
        }
        if (j % 7 == 6) {
#pragma unroll
            for (int k = 0; k < TV; ++k) zp[k] = foldp(zp[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < TV; ++k) {
        ya[k] = za[k];
        yp[k] = foldp(zp[k]);
    }
}

// Paths through columns r0 .. r1 entering anywhere and leaving anywhere
// (one lane); false when a column holds more than TV segments.
template <int TV = kTV, int NW = 0>
__device__ inline bool run_paths_lane(const Tabs &tb, const uint64_t *fol, const Job &jb, const TextCols &tc,
                                      uint64_t r0, uint64_t r1, Cnt &out) {
    uint32_t sp[TV], sn[TV];
    uint64_t ya[TV], yp[TV];
    const uint32_t mp0 = for_segments(tb, jb, tc, r0, [&](uint32_t k, uint32_t sg) {
#pragma unroll
        for (int j = 0; j < TV; ++j)
            if (static_cast<uint32_t>(j) == k) sp[j] = sg;
    });
    if (mp0 > static_cast<uint32_t>(TV)) return false;
    uint32_t mp = mp0;
#pragma unroll
    for (int j = 0; j < TV; ++j) {
        ya[j] = static_cast<uint32_t>(j) < mp ? 1ull : 0ull;
        yp[j] = ya[j];
    }
    for (uint64_t r = r0 + 1; r <= r1; ++r) {
        const uint32_t m = for_segments(tb, jb, tc, r, [&](uint32_t k, uint32_t sg) {
#pragma unroll
            for (int j = 0; j < TV; ++j)
                if (static_cast<uint32_t>(j) == k) sn[j] = sg;
        });
        if (m > static_cast<uint32_t>(TV)) return false;
        paths_step<TV, NW>(fol, tb.W, sp, mp, sn, m, ya, yp);
#pragma unroll
        for (int k = 0; k < TV; ++k) sp[k] = sn[k];
        mp = m;
    }
    Cnt s{0, 0};
#pragma unroll
    for (int j = 0; j < TV; ++j)
        if (static_cast<uint32_t>(j) < mp) s = cadd(s, Cnt{ya[j], yp[j]});
    out = s;
    return true;
}

// A long run r0 .. r1 of text t: its record and one piece per anchor cell.
// Cells are [k G, (k+1) G) with G = Job::cell; the cells whose start lies
// strictly inside the run may hold an anchor, and piece j (j >= 1) starts at
// the anchor of the j-th of them.
__device__ inline void emit_long(const Job &jb, uint32_t t, uint64_t r0, uint64_t r1) {
    const uint64_t G = jb.cell;
    const uint64_t kf = r0 / G + 1, kl = (r1 - 1) / G;
    const uint32_t nb = kl >= kf ? static_cast<uint32_t>(kl - kf + 1) : 0u;
    const uint32_t npc = nb + 1;
    const uint32_t ri = atomicAdd(&jb.ccnt[1], 1u);
    if (ri >= jb.cap_runs) {
        jb.tfail[t] = 1;
        return;
    }
    const uint32_t pb = atomicAdd(&jb.ccnt[2], npc);
    const uint32_t mb = npc > 1 ? atomicAdd(&jb.ccnt[3], npc) : 0u;
    RunRec &rr = jb.runs[ri];
    if (pb + static_cast<uint64_t>(npc) > jb.cap_pieces ||
        (npc > 1 && mb + static_cast<uint64_t>(npc) > jb.cap_mats)) {
        jb.tfail[t] = 1;
        rr.npc = 0;                                  // no pieces: the chain kernel skips it
        return;
    }
    rr.t = t;
    rr.r0 = r0;
    rr.r1 = r1;
    rr.pb = pb;
    rr.npc = npc;
    rr.mb = mb;
    for (uint32_t j = 0; j < npc; ++j) jb.piece[pb + j] = static_cast<uint64_t>(ri) | (static_cast<uint64_t>(j) << 32);
}

constexpr int kRunThreads = 256;

// Lane chunk and columns r0 .. r1 of a queued run; false for a void slot.
__device__ inline bool queued_run(const Job &jb, uint64_t v, uint32_t &i, uint64_t &r0, uint64_t &r1) {
    const uint32_t len = static_cast<uint32_t>(v & 1023u);
    i = static_cast<uint32_t>(v >> 33);
    if (len == 0) return false;
    const uint32_t t = text_of(jb, i);
    r0 = static_cast<uint64_t>(i - first_chunk(jb, t)) * jb.s + ((v >> 10) & ((1ull << 23) - 1));
    r1 = r0 + len - 1;
    return true;
}

// One thread per 64-column window, window-major as the marks (g = w c + i):
// the lanes of a wavefront read consecutive mark words.  Long runs are
// emitted for the piece kernels; the short runs starting in the window are
// queued for k_count_short (one atomic per wavefront).  When the queue is
// full the wavefront counts its short runs itself (a lane each; windows with
// a column too large for the lane go to the deferred list).
__global__ __launch_bounds__(kRunThreads) void k_count_runs(Tabs tb, Job jb) {
    const uint32_t sw = static_cast<uint32_t>(jb.s >> 6);
    const uint64_t gg = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u;
    bool act = gg < static_cast<uint64_t>(jb.c) * sw;
    uint32_t g = 0, w = 0, i = 0;
    ChunkCtx cx{};
    TextCols tc{};
    if (act) {
        g = static_cast<uint32_t>(gg);
        w = g / jb.c;
        i = g - w * jb.c;
        cx = chunk_ctx(jb, i);
        act = cx.tr.scalars[0] != 0 && 64ull * w < cx.hi - cx.lo;          // accepted, inside the chunk
    }
    if (act) tc = text_cols(jb, cx.t);
    uint32_t ns = 0;
    if (act)
        for_window_run_starts(jb, tc, i, w, cx, [&](uint64_t r0) {
            const uint64_t r1 = run_end(jb, tc, r0);
            if (r1 - r0 + 1 > jb.lshort)
                emit_long(jb, cx.t, r0, r1);
            else
                ++ns;
        });
    uint32_t incl = ns;   // inclusive prefix over the wavefront
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), d));
        if (lane >= static_cast<uint32_t>(d)) incl += v;
    }
    const uint32_t total = static_cast<uint32_t>(__shfl(static_cast<int>(incl), 63));
    if (total == 0) return;
    unsigned long long base = 0;
    if (lane == 63) base = atomicAdd(jb.nsruns, static_cast<unsigned long long>(total));
    base = shfl_u64(base, 63);
    uint64_t slot = base + incl - ns;
    if (base + total <= jb.cap_sruns) {
        if (ns)
            for_window_run_starts(jb, tc, i, w, cx, [&](uint64_t r0) {
                const uint64_t r1 = run_end(jb, tc, r0);
                if (r1 - r0 + 1 <= jb.lshort)
                    jb.sruns[slot++] = short_run(i, r0 - cx.lo, static_cast<uint32_t>(r1 - r0 + 1));
            });
        return;
    }
    for (uint32_t k = 0; k < ns; ++k)
        if (slot + k < jb.cap_sruns) jb.sruns[slot + k] = 0;              // reserved below the capacity
    if (!ns) return;
    Cnt acc{1, 1};
    bool defer = false;
    for_window_run_starts(jb, tc, i, w, cx, [&](uint64_t r0) {
        const uint64_t r1 = run_end(jb, tc, r0);
        if (r1 - r0 + 1 > jb.lshort || defer) return;
        Cnt x;
        if (run_paths_lane(tb, tb.folseg, jb, tc, r0, r1, x)) acc = cmul(acc, x);
        else defer = true;
    });
    if (defer) jb.dchunk[atomicAdd(&jb.ccnt[0], 1u)] = g;      // one entry per window
    else if (acc.a != 1 || acc.p != 1) cmul_at(jb.cfac + 2ull * i, acc);
}

constexpr int kShortThreads = 256;
constexpr uint32_t kFolLdsBytes = 32768;   // FolSeg staged in LDS up to this size

// A slot of the list counted by *ctr for every active lane of the
// wavefront (the lanes calling it), with one atomic per wavefront.
__device__ __forceinline__ uint32_t wave_slot(uint32_t *ctr) {
    const uint64_t act = __ballot(1);
    const uint32_t lane = __lane_id();
    const int leader = __ffsll(static_cast<unsigned long long>(act)) - 1;
    uint32_t base = 0;
    if (static_cast<int>(lane) == leader) base = atomicAdd(ctr, static_cast<uint32_t>(__popcll(act)));
    base = static_cast<uint32_t>(__shfl(static_cast<int>(base), leader));
    return base + static_cast<uint32_t>(__popcll(act & ((1ull << lane) - 1ull)));
}

// The queued short runs, one per lane (grid-stride).  A run's paths go
// into the product of its lane chunk.  TV = kTV: the runs of the first
// queue, counted with vectors of kTV segments; a run with a larger column
// goes to the second queue.  TV = kTV2: the runs of the second queue
// (FROM_Q2) or of the first (a wide count, without the kTV pass), with
// vectors of kTV2; a run with a still larger column is deferred to the
// wavefront walk (its queue index, tagged).  NW: FolSeg rows of at most NW
// words (0: any).
//
// Runs differ in length, so a lane that finishes its run takes the next
// one at once: every iteration of the loop advances each active lane by one
// column (the first column of a fresh run, or the next column of its run),
// and the wavefront runs as long as its lanes' summed work, not as long as
// its longest run times the number of runs per lane.
template <int TV, bool FROM_Q2, int NW>
__global__ __launch_bounds__(kShortThreads) void k_count_short(Tabs tb, Job jb) {
    static_assert(TV == kTV || TV == kTV2, "vectors of kTV or kTV2 segments");
    static_assert(!FROM_Q2 || TV == kTV2, "the second queue is counted with kTV2");
    extern __shared__ __align__(16) uint64_t fol_lds[];
    const uint64_t *fol = tb.folseg;
    if (jb.fol_lds) {
        const uint32_t nw = tb.nseg * tb.W;
        for (uint32_t k = threadIdx.x; k < nw; k += blockDim.x) fol_lds[k] = tb.folseg[k];
        __syncthreads();
        fol = fol_lds;
    }
    const uint32_t W = tb.W;
    const uint64_t nq = FROM_Q2 ? static_cast<uint64_t>(jb.ccnt[6])
                                : min(*jb.nsruns, static_cast<unsigned long long>(jb.cap_sruns));
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    uint64_t q = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    uint32_t sp[TV], sn[TV];
    uint64_t ya[TV], yp[TV];
    uint32_t mp = 0, k = 0, i = 0;
    uint64_t r = 0, r1 = 0;
    TextCols tc{};
    bool live = false, fresh = false;
    // plain columns of at most four words: the words of column r, loaded
    // one step ahead so that the load overlaps the previous step
    const bool pre = NW > 0 && !jb.compact;
    uint64_t cw0 = 0, cw1 = 0, cw2 = 0, cw3 = 0;
    auto load_col = [&](uint64_t rr) {
        const uint64_t *cw = tc.out + rr * W;
        cw0 = cw[0];
        if (NW > 1 && W > 1) cw1 = cw[1];
        if (NW > 2 && W > 2) cw2 = cw[2];
        if (NW > 2 && W > 3) cw3 = cw[3];
    };
    // the lane's next queued run (void slots skipped); live = false when none is left
    auto take = [&]() {
        live = false;
        while (q < nq) {
            k = FROM_Q2 ? jb.squeue2[q] : static_cast<uint32_t>(q);
            q += stride;
            uint64_t r0;
            if (queued_run(jb, jb.sruns[k], i, r0, r1)) {
                r = r0;
                tc = text_cols(jb, text_of(jb, i));
                live = true;
                fresh = true;
                if (pre) load_col(r);
                return;
            }
        }
    };
    take();
    while (__any(live)) {
        if (!live) continue;
        uint32_t m = 0;
        auto put = [&](uint32_t kk, uint32_t sg) {
#pragma unroll
            for (int j = 0; j < TV; ++j)
                if (static_cast<uint32_t>(j) == kk) sn[j] = sg;
        };
        if (pre) {
            auto word = [&](uint32_t w, uint64_t v) {
                for (; v; v &= v - 1) put(m++, w * 64 + static_cast<uint32_t>(__builtin_ctzll(v)));
            };
            word(0, cw0);
            if (NW > 1) word(1, cw1);
            if (NW > 2) {
                word(2, cw2);
                word(3, cw3);
            }
            if (r < r1) load_col(r + 1);
        } else {
            m = for_segments(tb, jb, tc, r, put);
        }
        const bool fail = m > static_cast<uint32_t>(TV);
        if (!fail) {
            if (fresh) {
#pragma unroll
                for (int j = 0; j < TV; ++j) {
                    ya[j] = static_cast<uint32_t>(j) < m ? 1ull : 0ull;
                    yp[j] = ya[j];
                }
            } else {
                paths_step<TV, NW>(fol, W, sp, mp, sn, m, ya, yp);
            }
#pragma unroll
            for (int j = 0; j < TV; ++j) sp[j] = sn[j];
            mp = m;
            fresh = false;
        }
        if (fail) {
            if (TV == kTV) jb.squeue2[wave_slot(&jb.ccnt[6])] = k;
            else jb.dchunk[wave_slot(&jb.ccnt[0])] = kDeferRun | k;
            take();
        } else if (r == r1) {
            Cnt x{0, 0};
#pragma unroll
            for (int j = 0; j < TV; ++j)
                if (static_cast<uint32_t>(j) < mp) x = cadd(x, Cnt{ya[j], yp[j]});
            if (x.a != 1 || x.p != 1) cmul_at(jb.cfac + 2ull * i, x);
            take();
        } else {
            ++r;
        }
    }
}

// ----------------------------------------------------- wavefront walks

constexpr uint32_t kWalkLdsWords = 4096;   // count vectors: 2 buffers x segments x VB x 2 moduli

template <int VB>
struct WalkCap {
    static constexpr uint32_t segs = kWalkLdsWords / (4 * VB);   // VB = 1: 1024, VB = 8: 128
};

struct WalkLds {
    uint64_t colw[2][kMaxWords];
    uint32_t pre[2][kMaxWords];
    uint32_t m[2];
    uint16_t seg[2][1024];
    uint64_t y[kWalkLdsWords];
};

// One wavefront walks columns a .. e of a text: VB count vectors start on
// column a (VB = 1: all ones; else unit vector v on the v-th segment of
// column a, v < m(a)), and each step to column r gives segment sigma the sum
// of the previous column's counts over the segments that sigma follows.  On
// return the vectors over column e are in y[buf] (segment k, vector v,
// modulus d at (k * VB + v) * 2 + d) with buf and m(e) returned; false when
// a column holds more segments than the LDS holds.
template <int VB>
__device__ inline bool wave_walk(const Tabs &tb, const Job &jb, const TextCols &tc, uint64_t a, uint64_t e,
                                 WalkLds &L, uint32_t &buf, uint32_t &m_end) {
    constexpr uint32_t cap = WalkCap<VB>::segs;
    const uint32_t lane = threadIdx.x, W = tb.W;
    uint32_t cur = 0;
    for (uint64_t r = a;; ++r) {
        // the column's words
        if (jb.compact) {
            const uint32_t p = r > 0 ? tb.classmap[tc.text[r - 1]] : tb.C;
            const uint32_t q = r < tc.n ? tb.classmap[tc.text[r]] : tb.C;
            const uint16_t *xl = tb.xlist + tb.xoff[p * tb.NL + q];
            const uint64_t cm = tc.out[r];
            for (uint32_t w = lane; w < W; w += 64) {
                uint64_t v = 0;
                for (uint64_t x = cm; x; x &= x - 1) {
                    const uint32_t sg = xl[__builtin_ctzll(x)];
                    if ((sg >> 6) == w) v |= 1ull << (sg & 63);
                }
                L.colw[cur][w] = v;
            }
        } else {
            for (uint32_t w = lane; w < W; w += 64) L.colw[cur][w] = tc.out[r * W + w];
        }
        wave_sync();
        // segments before each word, and the segment list
        uint32_t mt = 0;
        for (uint32_t w = 0; w < W; ++w) {
            if (lane == w) L.pre[cur][w] = mt;
            mt += static_cast<uint32_t>(__popcll(L.colw[cur][w]));
        }
        if (mt > cap) return false;
        for (uint32_t w = lane; w < W; w += 64) {
            uint32_t k = L.pre[cur][w];
            for (uint64_t v = L.colw[cur][w]; v; v &= v - 1) L.seg[cur][k++] = static_cast<uint16_t>(w * 64 + __builtin_ctzll(v));
        }
        wave_sync();
        uint64_t *yc = L.y + cur * (kWalkLdsWords / 2);
        const uint64_t *yq = L.y + (cur ^ 1u) * (kWalkLdsWords / 2);
        const uint32_t prv = cur ^ 1u;
        for (uint32_t k = lane; k < mt; k += 64) {
            uint64_t za[VB], zp[VB];
            if (r == a) {
#pragma unroll
                for (int v = 0; v < VB; ++v) {
                    za[v] = VB == 1 ? 1ull : (k == static_cast<uint32_t>(v) ? 1ull : 0ull);
                    zp[v] = za[v];
                }
            } else {
#pragma unroll
                for (int v = 0; v < VB; ++v) za[v] = zp[v] = 0;
                const uint32_t sg = L.seg[cur][k];
                for (uint32_t w = 0; w < W; ++w) {
                    const uint64_t pw = L.colw[prv][w];
                    uint64_t x = tb.predseg[static_cast<uint64_t>(sg) * W + w] & pw;
                    while (x) {
                        const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(x));
                        x &= x - 1;
                        const uint32_t rk = L.pre[prv][w] + static_cast<uint32_t>(__popcll(pw & low_mask(b)));
#pragma unroll
                        for (int v = 0; v < VB; ++v) {
                            za[v] += yq[(rk * VB + v) * 2];
                            zp[v] = addp(zp[v], yq[(rk * VB + v) * 2 + 1]);
                        }
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < VB; ++v) {
                yc[(k * VB + v) * 2] = za[v];
                yc[(k * VB + v) * 2 + 1] = zp[v];
            }
        }
        wave_sync();
        if (r == e) {
            buf = cur;
            m_end = mt;
            return true;
        }
        cur ^= 1u;
    }
}

// Sum of vector v over the segments of the last column of a walk.
template <int VB>
__device__ inline Cnt walk_sum(const WalkLds &L, uint32_t buf, uint32_t m, int v) {
    const uint64_t *y = L.y + buf * (kWalkLdsWords / 2);
    Cnt s{0, 0};
    for (uint32_t k = threadIdx.x; k < m; k += 64) s = cadd(s, Cnt{y[(k * VB + v) * 2], y[(k * VB + v) * 2 + 1]});
    return wave_sum_cnt(s);
}

// Deferred windows (their short runs) and deferred queued runs, one
// wavefront per item.
__global__ __launch_bounds__(64) void k_count_defer(Tabs tb, Job jb) {
    __shared__ WalkLds L;
    for (uint32_t item = blockIdx.x; item < jb.ccnt[0]; item += gridDim.x) {
        const uint32_t g = jb.dchunk[item];
        if (g & kDeferRun) {
            uint32_t ri;
            uint64_t r0, r1;
            queued_run(jb, jb.sruns[g & ~kDeferRun], ri, r0, r1);   // a deferred run is never a void slot
            const uint32_t t = text_of(jb, ri);
            const TextCols tc = text_cols(jb, t);
            uint32_t buf = 0, m = 0;
            const bool ok = wave_walk<1>(tb, jb, tc, r0, r1, L, buf, m);
            const Cnt x = ok ? walk_sum<1>(L, buf, m, 0) : Cnt{1, 1};
            if (threadIdx.x == 0) {
                cmul_at(jb.cfac + 2ull * ri, x);
                if (!ok) jb.tfail[t] = 1;
            }
            __syncthreads();
            continue;
        }
        const uint32_t w = g / jb.c, i = g - w * jb.c;
        const ChunkCtx cx = chunk_ctx(jb, i);
        const TextCols tc = text_cols(jb, cx.t);
        Cnt acc{1, 1};
        bool ok = true;
        for_window_run_starts(jb, tc, i, w, cx, [&](uint64_t r0) {
            const uint64_t r1 = run_end(jb, tc, r0);
            if (r1 - r0 + 1 > jb.lshort || !ok) return;    // long runs: the piece kernels'
            uint32_t buf = 0, m = 0;
            if (!wave_walk<1>(tb, jb, tc, r0, r1, L, buf, m)) {
                ok = false;
                return;
            }
            acc = cmul(acc, walk_sum<1>(L, buf, m, 0));
        });
        if (threadIdx.x == 0) {
            cmul_at(jb.cfac + 2ull * i, acc);
            if (!ok) jb.tfail[cx.t] = 1;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ long runs

// Anchor of cell k of the run r0 .. r1: the leftmost column of the cell
// (inside the run) with the fewest segments, if it holds at most kPieceR;
// returns (size << 40) | column, or ~0 for none.
__device__ inline uint64_t cell_anchor(const Tabs &tb, const Job &jb, const TextCols &tc, uint64_t r1, uint64_t k) {
    const uint64_t c0 = k * jb.cell, c1 = min(c0 + jb.cell, r1);   // c0 > r0 for the cells asked
    uint64_t best = ~0ull;
    for (uint64_t r = c0 + threadIdx.x; r < c1; r += 64) {
        const uint64_t key = (static_cast<uint64_t>(column_size(tb, jb, tc, r)) << 40) | r;
        best = key < best ? key : best;
    }
    best = wave_min_u64(best);
    return (best >> 40) <= static_cast<uint64_t>(kPieceR) ? best : ~0ull;
}

constexpr uint32_t kVoidPiece = 0xffffffffu;

// One wavefront per piece: the path counts from its first column (all ones
// for piece 0, else the unit vectors of its start anchor) to the next anchor
// of the run (one row per start vector and one column per anchor segment),
// or summed over the run's last column.  A one-piece run multiplies its
// count into the text's product directly.
__global__ __launch_bounds__(64) void k_count_pieces(Tabs tb, Job jb) {
    __shared__ WalkLds L;
    const uint32_t lane = threadIdx.x;
    const uint32_t np = min(jb.ccnt[2], jb.cap_pieces);
    for (uint32_t item = blockIdx.x; item < np; item += gridDim.x) {
        const uint64_t pc = jb.piece[item];
        const uint32_t ri = static_cast<uint32_t>(pc), j = static_cast<uint32_t>(pc >> 32);
        const RunRec &rr = jb.runs[ri];
        const uint32_t t = rr.t;
        const uint64_t r0 = rr.r0, r1 = rr.r1;
        const uint32_t npc = rr.npc, mb = rr.mb;
        const TextCols tc = text_cols(jb, t);
        const uint64_t kf = r0 / jb.cell + 1;
        uint64_t a = r0;
        uint32_t ra = 1;
        if (j > 0) {
            const uint64_t an = cell_anchor(tb, jb, tc, r1, kf + j - 1);
            if (an == ~0ull) {                            // no anchor: walked through by an earlier piece
                if (lane == 0) jb.pmat[item] = kVoidPiece;
                continue;
            }
            a = an & ((1ull << 40) - 1);
            ra = static_cast<uint32_t>(an >> 40);
        }
        // the next anchor, or the run's end
        uint64_t e = r1;
        uint32_t re = 0;
        for (uint64_t k = kf + j; k * jb.cell < r1; ++k) {
            const uint64_t an = cell_anchor(tb, jb, tc, r1, k);
            if (an != ~0ull) {
                e = an & ((1ull << 40) - 1);
                re = static_cast<uint32_t>(an >> 40);
                break;
            }
        }
        uint32_t buf = 0, m = 0;
        bool ok;
        Cnt res[kPieceR];
        if (j == 0) ok = wave_walk<1>(tb, jb, tc, a, e, L, buf, m);
        else ok = wave_walk<kPieceR>(tb, jb, tc, a, e, L, buf, m);
        if (!ok) {
            if (lane == 0) {
                jb.tfail[t] = 1;
                jb.pmat[item] = kVoidPiece;
            }
            __syncthreads();
            continue;
        }
        const int vb = j == 0 ? 1 : kPieceR;
        if (re == 0) {   // the run's end: sums over its last column
            for (int v = 0; v < kPieceR; ++v) {
                if (v >= static_cast<int>(ra)) break;
                res[v] = vb == 1 ? walk_sum<1>(L, buf, m, v) : walk_sum<kPieceR>(L, buf, m, v);
            }
        }
        if (npc == 1) {                                   // a single piece: the run's count
            if (lane == 0) tprod_mul(jb, t, res[0]);
        } else {
            // matrix rows = start vectors (ra), columns = end segments (re, or 1 when summed)
            uint64_t *M = jb.mats + (static_cast<uint64_t>(mb) + j) * kPieceR * kPieceR * 2;
            const uint64_t *y = L.y + buf * (kWalkLdsWords / 2);
            if (lane < static_cast<uint32_t>(kPieceR * kPieceR)) {
                const uint32_t v = lane / kPieceR, k = lane % kPieceR;
                uint64_t xa = 0, xp = 0;
                if (v < ra) {
                    if (re == 0) {
                        if (k == 0) {
                            // res[v] is wavefront-uniform
                            for (uint32_t q = 0; q < static_cast<uint32_t>(kPieceR); ++q)
                                if (q == v) {
                                    xa = res[q].a;
                                    xp = res[q].p;
                                }
                        }
                    } else if (k < re) {
                        xa = y[(k * vb + v) * 2];
                        xp = y[(k * vb + v) * 2 + 1];
                    }
                }
                M[(v * kPieceR + k) * 2] = xa;
                M[(v * kPieceR + k) * 2 + 1] = xp;
            }
            if (lane == 0) jb.pmat[item] = ra | ((re == 0 ? 1u : re) << 8);
        }
        __syncthreads();
    }
}

// One wavefront per long run of several pieces: the row vector of piece 0
// times the matrices of the pieces that start at an anchor; the last one
// sums over the run's end, leaving the run's count.
__global__ __launch_bounds__(64) void k_count_chain(Job jb) {
    const uint32_t lane = threadIdx.x;
    const uint32_t nr = min(jb.ccnt[1], jb.cap_runs);
    for (uint32_t ri = blockIdx.x; ri < nr; ri += gridDim.x) {
        const RunRec &rr = jb.runs[ri];
        const uint32_t npc = rr.npc;
        if (npc < 2) continue;
        const uint32_t t = rr.t, pb = rr.pb, mb = rr.mb;
        // lane k < kPieceR holds entry k of the row vector
        Cnt vk{0, 0};
        uint32_t dim = 0;
        bool ok = true;
        for (uint32_t j = 0; j < npc; ++j) {
            const uint32_t info = jb.pmat[pb + j];
            if (info == kVoidPiece) {
                if (j == 0) ok = false;
                continue;
            }
            const uint32_t rows = info & 0xffu, cols = info >> 8;
            const uint64_t *M = jb.mats + (static_cast<uint64_t>(mb) + j) * kPieceR * kPieceR * 2;
            if (j == 0) {
                vk = lane < cols ? Cnt{M[lane * 2], M[lane * 2 + 1]} : Cnt{0, 0};
            } else {
                if (rows != dim) ok = false;
                Cnt s{0, 0};
                for (uint32_t r = 0; r < rows; ++r) {
                    const Cnt vr{readlane_u64(vk.a, static_cast<int>(r)), readlane_u64(vk.p, static_cast<int>(r))};
                    if (lane < cols) s = cadd(s, cmul(vr, Cnt{M[(r * kPieceR + lane) * 2], M[(r * kPieceR + lane) * 2 + 1]}));
                }
                vk = lane < cols ? s : Cnt{0, 0};
            }
            dim = cols;
        }
        if (lane == 0) {
            if (!ok || dim != 1) jb.tfail[t] = 1;
            else tprod_mul(jb, t, vk);
        }
    }
}

// Per-text scalars: one block per text (count: 0 not requested, 1 requested,
// 2 recogniser).  Empty text: column 0 = I & F and one tree per
// initial-and-final segment.  Otherwise the count is the product of the
// text's chunk products and long-run products (0 for a rejected text).
// scalars[2]: 0 counted, 1 a run could not be counted, 2 not requested, 3 a
// join set was not a table state.
constexpr int kScalarThreads = 1024;

__global__ __launch_bounds__(kScalarThreads) void k_text_scalars(Tabs tb, Job jb, int count) {
    __shared__ uint64_t pa[kScalarThreads], pq[kScalarThreads];
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
                const uint64_t last = first_chunk(jb, t + 1) - 1;
                for (uint32_t e = 0; e < jb.ew; ++e) any |= jb.fout[last * jb.ew + e];
            }
            tr.scalars[0] = any ? 1 : 0;
            tr.scalars[1] = 0;
            tr.scalars[2] = jb.flags[0] ? 3 : 2;
            tr.scalars[3] = 0;
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
                    cm |= 1ull << tb.rankx[(tb.rank_pq ? tb.C * tb.NL + tb.C : tb.C) * tb.nseg + w * 64 +
                                           static_cast<uint32_t>(__builtin_ctzll(x))];
            }
            if (jb.compact) tr.out[0] = cm;
            tr.scalars[0] = any ? 1 : 0;
            tr.scalars[1] = count ? pc : 0;
            tr.scalars[2] = count ? 0 : 2;
            tr.scalars[3] = count ? pc : 0;
        }
        return;
    }
    uint64_t st = 0, va = 0, vp = 0;
    if (!count) {
        st = 2;
    } else if (tr.scalars[0] != 0) {
        const uint32_t c0 = first_chunk(jb, t), c1 = first_chunk(jb, t + 1);
        // four independent products per thread keep four multiplications in flight
        Cnt acc[4] = {{1, 1}, {1, 1}, {1, 1}, {1, 1}};
        const uint32_t st4 = 4 * blockDim.x;
        uint32_t k = c0 + th;
        for (; k + 3 * blockDim.x < c1; k += st4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t q = k + u * blockDim.x;
                acc[u] = cmul(acc[u], Cnt{jb.cfac[2 * q], jb.cfac[2 * q + 1]});
            }
        }
        for (; k < c1; k += blockDim.x) acc[0] = cmul(acc[0], Cnt{jb.cfac[2ull * k], jb.cfac[2ull * k + 1]});
        const Cnt a01 = cmul(acc[0], acc[1]), a23 = cmul(acc[2], acc[3]), all = cmul(a01, a23);
        pa[th] = all.a;
        pq[th] = all.p;
        __syncthreads();
        for (uint32_t h = kScalarThreads / 2; h; h >>= 1) {
            if (th < h) {
                pa[th] *= pa[th + h];
                pq[th] = mulp(pq[th], pq[th + h]);
            }
            __syncthreads();
        }
        va = pa[0];
        vp = pq[0];
        if (!tb.col_single) {
            va *= jb.tprod[2ull * t];
            vp = mulp(vp, jb.tprod[2ull * t + 1]);
            if (jb.tfail[t]) st = 1;
        }
    }
    if (jb.flags[0]) st = 3;
    if (th == 0) {
        tr.scalars[1] = va;
        tr.scalars[2] = st;
        tr.scalars[3] = vp;
    }
}

}  // namespace slpf

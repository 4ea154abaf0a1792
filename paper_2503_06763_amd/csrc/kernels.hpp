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
//   k_count_chunk / k_prod
//            the number of syntax trees: per chunk a transfer matrix of path
//            counts between its clean edge columns, then their ordered
//            product modulo 2^64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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
    uint32_t fhmask, rhmask;
    uint32_t C, W, NL;          // classes, words, C + 1
    uint32_t nf, nr;            // table sizes including id 0
    uint32_t fstart, rstart;    // ids of I and F
    uint32_t emax;
};

struct Job {
    const uint8_t *text;
    uint64_t n;
    uint64_t s;                 // lane chunk bytes
    uint32_t c;                 // lane chunks
    uint16_t *R, *Rh;           // [emax][c] end ids of the reach runs
    uint64_t *Mf, *MbR;         // [c][emax] masks; MbR indexed by c-1-i
    uint8_t *nxf, *nxb;         // |X_b| for b = 0..c (nxb reversed: nxb[k] = |X_{c-k}|)
    uint64_t *vf, *vb;          // join vectors, vf[b] = J_b & X_b, vb[k] = J^_{c-k} & X_{c-k}
    uint16_t *fid, *rid;        // build start ids per chunk
    uint16_t *ckpt;             // forward id every 64 bytes
    uint64_t *out;              // SLPF columns
    uint64_t *scalars;          // [0] accepted [1] count [2] count status
    uint32_t *flags;            // [0] set not found, [1] big-slot counter, [2] count overflow
    uint64_t *trace;            // optional J / J^ words
    // tree count
    uint8_t *dims;              // [c][2]: edge column sizes
    uint64_t *tsmall;           // [c][8*8]
    uint32_t *tbig_idx;         // [c], 0xffffffff = small slot
    uint64_t *tbig;             // [pool][64*64]
    uint32_t big_pool;
};

constexpr int kDedupEvery = 32;
constexpr int kGroup = 8;
constexpr int kSmallT = 8;
constexpr int kBigT = 64;

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

// Runs kGroup ME-DFA runs in lockstep over `len` bytes starting at `base`
// (forward) or ending at `base + len` (backward).  Runs that reach the same
// state are merged (equal states have equal futures); `alias` maps entry k
// of the group to the slot holding its run.
template <bool FWD>
__device__ inline void run_group(const uint8_t *text, uint64_t lo, uint64_t hi, const uint16_t *cls,
                                 const uint16_t *delta, uint32_t C, uint32_t st[kGroup],
                                 uint32_t &alias) {
    uint32_t nl = kGroup;   // wave-uniform bound on live slots
    uint64_t len = hi - lo;
    uint64_t done = 0;
    while (done < len) {
        // dedup + liveness, uniform across the wave
#pragma unroll
        for (int j = 1; j < kGroup; ++j) {
#pragma unroll
            for (int i = 0; i < j; ++i) {
                if (st[j] != 0 && st[j] == st[i]) {
#pragma unroll
                    for (int k = 0; k < kGroup; ++k)
                        if (((alias >> (4 * k)) & 15u) == static_cast<uint32_t>(j))
                            alias = (alias & ~(15u << (4 * k))) | (static_cast<uint32_t>(i) << (4 * k));
                    st[j] = 0;
                }
            }
        }
        uint32_t top = 0;
#pragma unroll
        for (int j = 0; j < kGroup; ++j)
            if (st[j]) top = j + 1;
        // wave max of top
        nl = 0;
#pragma unroll
        for (int j = kGroup; j >= 1; --j)
            if (nl == 0 && __any(top >= static_cast<uint32_t>(j))) nl = j;
        if (nl == 0) return;
        uint64_t step = len - done < kDedupEvery ? len - done : kDedupEvery;
        for (uint64_t t = 0; t < step; ++t) {
            uint64_t pos = FWD ? lo + done + t : hi - 1 - done - t;
            uint32_t cl = cls[text[pos]];
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                if (j < static_cast<int>(nl)) st[j] = delta[st[j] * C + cl];
        }
        done += step;
    }
}

template <bool LDS>
__global__ __launch_bounds__(256) void k_reach(Tabs tb, Job jb) {
    extern __shared__ __align__(16) uint8_t smem[];
    Lookup<LDS> lk = stage_tables<LDS>(tb, smem, true, true);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= jb.c) return;
    const uint64_t lo = static_cast<uint64_t>(i) * jb.s;
    const uint64_t hi = (i + 1 == jb.c) ? jb.n : lo + jb.s;
    const uint32_t la = boundary_list(tb, lk.cls, jb.text, jb.n, jb.s, jb.c, i);
    const uint32_t lb = boundary_list(tb, lk.cls, jb.text, jb.n, jb.s, jb.c, i + 1);
    const uint32_t xa0 = tb.xoff[la], na = tb.xoff[la + 1] - xa0;
    const uint32_t xb0 = tb.xoff[lb], nb = tb.xoff[lb + 1] - xb0;
    // entry-list sizes per edge, forward order and reversed (nxb[k] = |X_{c-k}|)
    jb.nxf[i] = static_cast<uint8_t>(na);
    jb.nxb[jb.c - 1 - i] = static_cast<uint8_t>(nb);
    if (i + 1 == jb.c) jb.nxf[jb.c] = static_cast<uint8_t>(nb);
    if (i == 0) jb.nxb[jb.c] = static_cast<uint8_t>(na);

    // forward runs from X_i
    for (uint32_t g0 = 0; __any(g0 < na); g0 += kGroup) {
        uint32_t st[kGroup];
        uint32_t alias = 0;
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            st[k] = (g0 + k < na) ? tb.fsingle[tb.xlist[xa0 + g0 + k]] : 0;
            alias |= static_cast<uint32_t>(k) << (4 * k);
        }
        run_group<true>(jb.text, lo, hi, lk.cls, lk.fd, tb.C, st, alias);
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            if (g0 + k < na) {
                uint32_t sl = (alias >> (4 * k)) & 15u, v = 0;
#pragma unroll
                for (int q = 0; q < kGroup; ++q)
                    if (sl == static_cast<uint32_t>(q)) v = st[q];
                jb.R[static_cast<uint64_t>(g0 + k) * jb.c + i] = static_cast<uint16_t>(v);
            }
        }
    }
    // backward runs from X_{i+1}
    for (uint32_t g0 = 0; __any(g0 < nb); g0 += kGroup) {
        uint32_t st[kGroup];
        uint32_t alias = 0;
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            st[k] = (g0 + k < nb) ? tb.rsingle[tb.xlist[xb0 + g0 + k]] : 0;
            alias |= static_cast<uint32_t>(k) << (4 * k);
        }
        run_group<false>(jb.text, lo, hi, lk.cls, lk.rd, tb.C, st, alias);
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            if (g0 + k < nb) {
                uint32_t sl = (alias >> (4 * k)) & 15u, v = 0;
#pragma unroll
                for (int q = 0; q < kGroup; ++q)
                    if (sl == static_cast<uint32_t>(q)) v = st[q];
                jb.Rh[static_cast<uint64_t>(g0 + k) * jb.c + i] = static_cast<uint16_t>(v);
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
    for (uint32_t m = 0; m < nb; ++m) {
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

// --------------------------------------------------------------------- join

// Compose groups of 64 consecutive maps: out[g] = M[64g+63] o ... o M[64g].
// One wavefront per group, lane = row (entry of the group's first list).
__global__ __launch_bounds__(64) void k_compose(const uint64_t *M, uint32_t stride, uint32_t N,
                                                const uint8_t *nx, uint64_t *out, uint8_t *out_nx) {
    const uint32_t g = blockIdx.x, m = threadIdx.x;
    const uint32_t k0 = g * 64, k1 = min(k0 + 64, N);
    const uint32_t rows = nx[k0];
    if (m == 0) {
        out_nx[g] = nx[k0];
        if (k1 == N) out_nx[g + 1] = nx[N];
    }
    uint64_t v = 0;
    if (m < rows) {
        v = 1ull << m;
        for (uint32_t k = k0; k < k1; ++k) v = apply_map(M + static_cast<uint64_t>(k) * stride, v);
    }
    out[static_cast<uint64_t>(g) * 64 + m] = v;
}

// Sequential scan over the top level: vec[0] = all entries of the first list.
__global__ void k_scan_top(const uint64_t *M, uint32_t stride, uint32_t N, const uint8_t *nx,
                           uint64_t *vec) {
    if (threadIdx.x || blockIdx.x) return;
    uint64_t v = low_mask(nx[0]);
    vec[0] = v;
    for (uint32_t k = 0; k < N; ++k) {
        v = apply_map(M + static_cast<uint64_t>(k) * stride, v);
        vec[k + 1] = v;
    }
}

// Expand parent vectors down one level: one thread per parent group.
__global__ __launch_bounds__(64) void k_expand(const uint64_t *M, uint32_t stride, uint32_t N,
                                               const uint64_t *pvec, uint32_t NP, uint64_t *vec) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    uint64_t v = pvec[p];
    const uint32_t k0 = p * 64, k1 = min(k0 + 64, N);
    for (uint32_t k = k0; k < k1; ++k) {
        vec[k] = v;
        v = apply_map(M + static_cast<uint64_t>(k) * stride, v);
    }
    if (k1 == N) vec[N] = v;
}

// Join sets and build start ids.  Thread i handles chunk i: fid_i = id of
// J at P_i, rid_i = id of J^ at P_{i+1}.
__global__ __launch_bounds__(256) void k_starts(Tabs tb, Job jb) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t c = jb.c, W = tb.W;
    if (i >= c) return;
    uint64_t acc[kMaxWords];
    // forward: J at P_i is the union of the ends of the runs of chunk i-1 selected by vf[i-1]
    auto join_fwd = [&](uint32_t b) -> uint32_t {   // J at P_b, b >= 1
        uint64_t sel = jb.vf[b - 1];
        for (uint32_t w = 0; w < W; ++w) acc[w] = 0;
        uint32_t first = 0xffffffffu;
        bool same = true;
        while (sel) {
            int m = __builtin_ctzll(sel);
            sel &= sel - 1;
            uint32_t id = jb.R[static_cast<uint64_t>(m) * c + (b - 1)];
            if (first == 0xffffffffu) first = id;
            same = same && (id == first);
            const uint64_t *bt = tb.fbits + static_cast<uint64_t>(id) * W;
            for (uint32_t w = 0; w < W; ++w) acc[w] |= bt[w];
        }
        if (first == 0xffffffffu) return 0;
        if (same) return first;
        return lookup_set(tb.fhash, tb.fhmask, tb.fbits, W, acc, jb.flags);
    };
    // backward: J^ at P_b (b <= c-1) from the runs of chunk b selected by g at P_{b+1}
    auto join_bwd = [&](uint32_t b) -> uint32_t {
        uint64_t sel = jb.vb[c - (b + 1)];
        for (uint32_t w = 0; w < W; ++w) acc[w] = 0;
        uint32_t first = 0xffffffffu;
        bool same = true;
        while (sel) {
            int m = __builtin_ctzll(sel);
            sel &= sel - 1;
            uint32_t id = jb.Rh[static_cast<uint64_t>(m) * c + b];
            if (first == 0xffffffffu) first = id;
            same = same && (id == first);
            const uint64_t *bt = tb.rbits + static_cast<uint64_t>(id) * W;
            for (uint32_t w = 0; w < W; ++w) acc[w] |= bt[w];
        }
        if (first == 0xffffffffu) return 0;
        if (same) return first;
        return lookup_set(tb.rhash, tb.rhmask, tb.rbits, W, acc, jb.flags);
    };
    const uint32_t f = (i == 0) ? tb.fstart : join_fwd(i);
    const uint32_t r = (i + 1 == c) ? tb.rstart : join_bwd(i + 1);
    jb.fid[i] = static_cast<uint16_t>(f);
    jb.rid[i] = static_cast<uint16_t>(r);
    if (jb.trace) {
        uint64_t *Jt = jb.trace, *Jh = jb.trace + static_cast<uint64_t>(c + 1) * W;
        const uint64_t *fb = tb.fbits + static_cast<uint64_t>(f) * W;
        for (uint32_t w = 0; w < W; ++w) Jt[static_cast<uint64_t>(i) * W + w] = fb[w];
        const uint64_t *rb = tb.rbits + static_cast<uint64_t>(r) * W;
        for (uint32_t w = 0; w < W; ++w) Jh[static_cast<uint64_t>(i + 1) * W + w] = rb[w];
        if (i + 1 == c) {
            uint32_t fe = join_fwd(c);
            const uint64_t *fe_b = tb.fbits + static_cast<uint64_t>(fe) * W;
            for (uint32_t w = 0; w < W; ++w) Jt[static_cast<uint64_t>(c) * W + w] = fe_b[w];
        }
        if (i == 0) {
            uint32_t r0 = join_bwd(0);
            const uint64_t *r0b = tb.rbits + static_cast<uint64_t>(r0) * W;
            for (uint32_t w = 0; w < W; ++w) Jh[w] = r0b[w];
        }
    }
    if (i == 0) {
        jb.scalars[0] = jb.vf[c] != 0 ? 1ull : 0ull;
    }
}

// -------------------------------------------------------------------- build

template <int WT, bool LDS>
__global__ __launch_bounds__(256) void k_build(Tabs tb, Job jb) {
    extern __shared__ __align__(16) uint8_t smem[];
    Lookup<LDS> lk = stage_tables<LDS>(tb, smem, true, true);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= jb.c) return;
    const uint32_t C = tb.C, W = tb.W;
    const uint64_t lo = static_cast<uint64_t>(i) * jb.s;
    const uint64_t hi = (i + 1 == jb.c) ? jb.n : lo + jb.s;
    const uint16_t *cls = lk.cls, *fd = lk.fd, *rd = lk.rd;
    uint32_t xw[16];

    // forward DFA run from J at P_i, one checkpoint per 64-byte window
    uint32_t f = jb.fid[i];
    for (uint64_t a0 = lo; a0 < hi; a0 += 64) {
        const uint32_t len = static_cast<uint32_t>(hi - a0 < 64 ? hi - a0 : 64);
        jb.ckpt[a0 >> 6] = static_cast<uint16_t>(f);
        load_window(jb.text, a0, len, xw);
#pragma unroll
        for (int t = 0; t < 64; ++t)
            if (t < static_cast<int>(len)) f = fd[f * C + cls[byte_of(xw, t)]];
    }

    // backward reverse-DFA run from J^ at P_{i+1}; merge window by window
    uint32_t b = jb.rid[i];
    const uint64_t last = lo + ((hi - lo - 1) & ~63ull);
    for (uint64_t a0 = last;; a0 -= 64) {
        const uint32_t len = static_cast<uint32_t>(hi - a0 < 64 ? hi - a0 : 64);
        load_window(jb.text, a0, len, xw);
        uint32_t fw[64];
        uint32_t g = jb.ckpt[a0 >> 6];
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            if (t < static_cast<int>(len)) g = fd[g * C + cls[byte_of(xw, t)]];
            fw[t] = g;
        }
#pragma unroll
        for (int t = 63; t >= 0; --t) {
            if (t < static_cast<int>(len)) {
                const uint64_t r = a0 + t + 1;
                const uint64_t *fb = tb.fbits + static_cast<uint64_t>(fw[t]) * W;
                const uint64_t *rb = tb.rbits + static_cast<uint64_t>(b) * W;
                uint64_t *o = jb.out + r * W;
#pragma unroll
                for (int w = 0; w < WT; ++w)
                    if (w < static_cast<int>(W)) o[w] = fb[w] & rb[w];
                b = rd[b * C + cls[byte_of(xw, t)]];
            }
        }
        if (a0 == lo) break;
    }
    if (i == 0) {   // compose: C_0 = J_0 & J^_1
        const uint64_t *fb = tb.fbits + static_cast<uint64_t>(tb.fstart) * W;
        const uint64_t *rb = tb.rbits + static_cast<uint64_t>(b) * W;
        for (uint32_t w = 0; w < W; ++w) jb.out[w] = fb[w] & rb[w];
    }
}

// --------------------------------------------------------------- tree count

// Transfer matrix of chunk i: T[k][q] = number of paths in the clean SLPF from
// the k-th segment of column P_i to the q-th segment of column P_{i+1}
// (segments ranked by id).  A path crosses an arc rho -> sigma between
// consecutive clean columns iff sigma is a follower of rho (the label of rho
// equals the byte read, as every segment of a clean column does).  One
// wavefront per chunk; lane q keeps column q of the running matrix U in LDS.
__global__ __launch_bounds__(64) void k_count_chunk(Tabs tb, Job jb) {
    __shared__ uint64_t U[2][kBigT][kBigT];
    __shared__ uint32_t segs[2][kBigT];
    __shared__ uint64_t arcs[kBigT];
    __shared__ uint32_t nseg[2];
    __shared__ uint32_t fail;
    const uint32_t i = blockIdx.x, q = threadIdx.x;
    if (jb.scalars[0] == 0) return;
    const uint32_t W = tb.W;
    const uint64_t lo = static_cast<uint64_t>(i) * jb.s;
    const uint64_t hi = (i + 1 == jb.c) ? jb.n : lo + jb.s;
    if (q == 0) fail = 0;
    __syncthreads();
    // list the segments of column r into segs[slot]; returns the count or > 64
    auto list_column = [&](uint64_t r, int slot) {
        if (q == 0) {
            uint32_t cnt = 0;
            const uint64_t *col = jb.out + r * W;
            for (uint32_t w = 0; w < W && cnt <= kBigT; ++w) {
                uint64_t v = col[w];
                while (v) {
                    int bpos = __builtin_ctzll(v);
                    v &= v - 1;
                    if (cnt < kBigT) segs[slot][cnt] = w * 64 + bpos;
                    ++cnt;
                }
            }
            nseg[slot] = cnt;
        }
        __syncthreads();
    };
    int cur = 0;
    list_column(hi, cur);
    const uint32_t mR = nseg[cur];
    if (mR > kBigT) {
        if (q == 0) atomicOr(&jb.flags[2], 1u);
        return;
    }
    for (uint32_t k = 0; k < kBigT; ++k) U[cur][k][q] = (k == q && q < mR) ? 1ull : 0ull;
    __syncthreads();
    for (uint64_t r = hi; r-- > lo;) {
        const int nxt = cur ^ 1;
        list_column(r, nxt);
        const uint32_t m = nseg[nxt], mp = nseg[cur];
        if (m > kBigT) {
            if (q == 0) atomicOr(&jb.flags[2], 1u);
            return;
        }
        if (q < m) {   // arcs of the q-th segment of column r into column r+1
            const uint64_t *fs = tb.folseg + static_cast<uint64_t>(segs[nxt][q]) * W;
            uint64_t a = 0;
            for (uint32_t j = 0; j < mp; ++j) {
                uint32_t sg = segs[cur][j];
                a |= ((fs[sg >> 6] >> (sg & 63)) & 1ull) << j;
            }
            arcs[q] = a;
        }
        __syncthreads();
        if (q < mR) {
            for (uint32_t k = 0; k < m; ++k) {
                uint64_t sum = 0, a = arcs[k];
                while (a) {
                    int j = __builtin_ctzll(a);
                    a &= a - 1;
                    sum += U[cur][j][q];
                }
                U[nxt][k][q] = sum;
            }
        }
        __syncthreads();
        cur = nxt;
    }
    const uint32_t mL = nseg[cur];
    if (q == 0) {
        jb.dims[2 * i] = static_cast<uint8_t>(mL);
        jb.dims[2 * i + 1] = static_cast<uint8_t>(mR);
    }
    if (mL <= kSmallT && mR <= kSmallT) {
        if (q == 0) jb.tbig_idx[i] = 0xffffffffu;
        if (q < kSmallT)
            for (uint32_t k = 0; k < kSmallT; ++k)
                jb.tsmall[static_cast<uint64_t>(i) * kSmallT * kSmallT + k * kSmallT + q] =
                    (k < mL && q < mR) ? U[cur][k][q] : 0ull;
    } else {
        __shared__ uint32_t slot;
        if (q == 0) {
            slot = atomicAdd(&jb.flags[1], 1u);
            jb.tbig_idx[i] = slot;
        }
        __syncthreads();
        if (slot >= jb.big_pool) {
            if (q == 0) atomicOr(&jb.flags[2], 1u);
            return;
        }
        for (uint32_t k = 0; k < kBigT; ++k)
            jb.tbig[static_cast<uint64_t>(slot) * kBigT * kBigT + k * kBigT + q] =
                (k < mL && q < mR) ? U[cur][k][q] : 0ull;
    }
}

// Ordered product of transfer matrices.  Level 0 reads the per-chunk slots;
// higher levels read the previous level's 64x64 outputs.  One wavefront per
// group of `G` consecutive matrices; lane q computes column q.
__global__ __launch_bounds__(64) void k_prod(Job jb, int level0, const uint64_t *in,
                                             const uint8_t *in_dims, uint32_t N, uint32_t G,
                                             uint64_t *out, uint8_t *out_dims, int final_level) {
    __shared__ uint64_t P[kBigT][kBigT + 1];
    __shared__ uint32_t drows, dcols;
    const uint32_t g = blockIdx.x, q = threadIdx.x;
    if (jb.scalars[0] == 0 || jb.flags[2] != 0) {
        if (final_level && g == 0 && q == 0) {
            jb.scalars[1] = 0;
            jb.scalars[2] = jb.flags[2] ? 1ull : 0ull;
        }
        return;
    }
    auto elem = [&](uint32_t idx, uint32_t k, uint32_t col) -> uint64_t {
        if (level0) {
            uint32_t bi = jb.tbig_idx[idx];
            if (bi == 0xffffffffu)
                return (k < kSmallT && col < kSmallT)
                           ? jb.tsmall[static_cast<uint64_t>(idx) * kSmallT * kSmallT + k * kSmallT + col]
                           : 0ull;
            return jb.tbig[static_cast<uint64_t>(bi) * kBigT * kBigT + k * kBigT + col];
        }
        return in[static_cast<uint64_t>(idx) * kBigT * kBigT + k * kBigT + col];
    };
    const uint32_t k0 = g * G, k1 = min(k0 + G, N);
    if (q == 0) {
        drows = in_dims[2 * k0];
        dcols = in_dims[2 * k0 + 1];
    }
    __syncthreads();
    for (uint32_t k = 0; k < kBigT; ++k) P[k][q] = (k < drows && q < dcols) ? elem(k0, k, q) : 0ull;
    __syncthreads();
    uint64_t col[kBigT];
    for (uint32_t idx = k0 + 1; idx < k1; ++idx) {
        const uint32_t br = in_dims[2 * idx], bc = in_dims[2 * idx + 1];
        const uint32_t rows = drows;
        for (uint32_t k = 0; k < kBigT; ++k) col[k] = 0;
        if (q < bc) {
            for (uint32_t l = 0; l < br; ++l) {
                uint64_t e = elem(idx, l, q);
                if (!e) continue;
                for (uint32_t k = 0; k < rows; ++k) col[k] += P[k][l] * e;
            }
        }
        __syncthreads();
        for (uint32_t k = 0; k < kBigT; ++k) P[k][q] = col[k];
        if (q == 0) dcols = bc;
        __syncthreads();
    }
    if (final_level) {
        if (q == 0) {
            uint64_t tot = 0;
            for (uint32_t k = 0; k < drows; ++k)
                for (uint32_t l = 0; l < dcols; ++l) tot += P[k][l];
            jb.scalars[1] = tot;
            jb.scalars[2] = 0;
        }
        return;
    }
    for (uint32_t k = 0; k < kBigT; ++k) out[static_cast<uint64_t>(g) * kBigT * kBigT + k * kBigT + q] = P[k][q];
    if (q == 0) {
        out_dims[2 * g] = static_cast<uint8_t>(drows);
        out_dims[2 * g + 1] = static_cast<uint8_t>(dcols);
    }
}

__global__ void k_init(Job jb) {
    if (blockIdx.x == 0 && threadIdx.x < 4) jb.flags[threadIdx.x] = 0;
}

__global__ void k_set_scalars(Job jb, uint64_t v1, uint64_t v2) {
    if (threadIdx.x || blockIdx.x) return;
    jb.scalars[1] = v1;
    jb.scalars[2] = v2;
}

// An edge set that is not a state of the table means a broken table: report
// it as count status 3 so that callers never take such a result as valid.
__global__ void k_finish(Job jb) {
    if (threadIdx.x || blockIdx.x) return;
    if (jb.flags[0]) jb.scalars[2] = 3;
}

// Empty text: one column I & F; one tree per initial-and-final segment.
__global__ void k_empty(Tabs tb, Job jb, int count) {
    if (threadIdx.x || blockIdx.x) return;
    const uint64_t *fb = tb.fbits + static_cast<uint64_t>(tb.fstart) * tb.W;
    const uint64_t *rb = tb.rbits + static_cast<uint64_t>(tb.rstart) * tb.W;
    uint64_t any = 0, pc = 0;
    for (uint32_t w = 0; w < tb.W; ++w) {
        uint64_t v = fb[w] & rb[w];
        jb.out[w] = v;
        any |= v;
        pc += __popcll(v);
    }
    jb.scalars[0] = any ? 1 : 0;
    jb.scalars[1] = count ? pc : 0;
    jb.scalars[2] = count ? 0 : 2;
}

}  // namespace slpf

// Internal definitions shared by the host compiler and the device runtime of
// the SLPF library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace slpf {

constexpr int kMaxEntries = 64;     // entries of a list that one u64 mask holds (the compact SLPF's limit)
constexpr int kMaxWords = 32;       // words per SLPF column handled by the kernels
constexpr uint32_t kHashEmpty = 0xffffffffu;
constexpr uint16_t kNoSole = 0xffffu;  // state set with zero or several segments

// Hash of a W-word segment set, identical on host and device.
__host__ __device__ inline uint32_t hash_words(const uint64_t *w, int W) {
    uint64_t h = 0x243f6a8885a308d3ull;
    for (int i = 0; i < W; ++i) {
        h ^= w[i] + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        h *= 0xd6e8feb86659fd93ull;
    }
    return static_cast<uint32_t>(h ^ (h >> 29));
}

// One direction's merged DFA / multi-entry DFA table, host side.
struct HostTable {
    uint32_t nstates = 0;                 // including id 0 = empty set
    uint32_t dfa_states = 0, medfa_states = 0;
    std::vector<uint64_t> bits;           // nstates x W
    std::vector<uint16_t> delta;          // nstates x C
    std::vector<uint16_t> single;         // id of {q}, per segment
    uint16_t start = 0;                   // id of I (forward) or F (reverse)
    std::vector<uint32_t> hash;           // open addressing, power-of-two size
};

struct HostAutomaton {
    uint32_t nseg = 0, W = 0, C = 0;      // segments, words per set, byte classes
    std::vector<std::string> seg_text;
    std::vector<uint64_t> I, F;           // W words
    std::vector<uint64_t> folseg;         // nseg x W, followers of each segment
    std::vector<uint16_t> classmap;       // 256
    std::vector<uint32_t> xoff;           // (C+1)^2 + 1 offsets of the entry lists
    std::vector<uint16_t> xlist;          // segment ids
    uint32_t max_entries = 0;
    // entry lists filtered by the next byte only (every ME-DFA entry whose
    // end-letter is the next byte): the speculation ablation
    std::vector<uint32_t> xoff_nb;
    std::vector<uint16_t> xlist_nb;
    uint32_t max_entries_nb = 0;
    uint32_t ninit = 0, nfinal = 0;
    HostTable fwd, rev;
    // match extraction: per node number g (1 .. ngroups-1) three W-word
    // segment masks: the segment leaves g open (its last g-symbol is "g("),
    // it closes an open g (its first g-symbol is ")g"), it holds "g( .. )g"
    // (an empty match); all zero for leaves
    uint32_t ngroups = 0;
    std::vector<uint64_t> gmask;          // ngroups x 3 x W
    // child extraction: per node number, its parent's number (0 for the
    // root) and its kind (0 operator, 1 terminal, 2 epsilon); per segment,
    // its symbols in order as num * 4 + kind (0 "num(", 1 a leaf, 2 ")num",
    // 3 the end mark with num 0), segment q at [sym_off[q], sym_off[q+1])
    std::vector<int32_t> parent;          // ngroups
    std::vector<uint8_t> node_kind;       // ngroups
    std::vector<uint32_t> sym_off;        // nseg + 1
    std::vector<int32_t> sym_code;
};

struct CompileLimits {
    uint32_t max_segments = 2048;
    uint32_t max_states = 65535;
};

// Returns an slpf_status value.
int compile_re(const uint8_t *re, size_t len, const CompileLimits &lim, HostAutomaton &out,
               size_t *err_offset);

}  // namespace slpf

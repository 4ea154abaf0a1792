// Host-side checks run under AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_host_sanitizers.py builds this with g++ together with the RE
// compiler):
//   - the RE compiler on every RE of a file (one per line, hex-encoded bytes:
//     generated REs, malformed ones and random byte strings); each must
//     compile or return an error status, and a compiled automaton must be
//     self-consistent in its sizes;
//   - the request server's arena on a seeded random sequence of allocations
//     and frees, against a brute-force model of first-fit allocation.
#include <cstdint>
#include <cstdio>
#include <fstream>
#include <string>
#include <vector>

#include "../../paper_2503_06763_amd/csrc/arena.hpp"
#include "../../paper_2503_06763_amd/csrc/slpf_internal.hpp"

namespace {

int fails = 0;

void check(bool ok, const char *what, long k) {
    if (!ok) {
        std::fprintf(stderr, "FAIL %s (case %ld)\n", what, k);
        ++fails;
    }
}

std::vector<uint8_t> unhex(const std::string &h) {
    std::vector<uint8_t> out;
    for (size_t i = 0; i + 1 < h.size(); i += 2) out.push_back(static_cast<uint8_t>(std::stoi(h.substr(i, 2), nullptr, 16)));
    return out;
}

void compile_all(const char *path) {
    std::ifstream f(path);
    std::string line;
    long k = 0, ok = 0;
    while (std::getline(f, line)) {
        const std::vector<uint8_t> re = unhex(line);
        slpf::HostAutomaton A;
        slpf::CompileLimits lim;
        size_t off = 0;
        const int st = slpf::compile_re(re.data(), re.size(), lim, A, &off);
        if (st == 0) {
            ++ok;
            check(A.W == (A.nseg + 63) / 64 && A.nseg > 0, "words per column", k);
            check(A.folseg.size() == size_t(A.nseg) * A.W, "FolSeg size", k);
            check(A.fwd.bits.size() == size_t(A.fwd.nstates) * A.W, "forward bit sets", k);
            check(A.fwd.delta.size() == size_t(A.fwd.nstates) * A.C, "forward table", k);
            check(A.rev.delta.size() == size_t(A.rev.nstates) * A.C, "reverse table", k);
            check(A.classmap.size() == 256, "class map", k);
            check(A.xoff.size() == size_t(A.C + 1) * (A.C + 1) + 1 && A.xoff.back() == A.xlist.size(), "entry lists",
                  k);
            for (uint16_t q : A.fwd.delta) check(q < A.fwd.nstates, "forward transition", k);
            for (uint16_t q : A.rev.delta) check(q < A.rev.nstates, "reverse transition", k);
        } else {
            check(off <= re.size(), "error offset", k);
        }
        ++k;
    }
    std::printf("compiled %ld of %ld REs\n", ok, k);
}

uint64_t splitmix(uint64_t &x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

void arena_model(long steps) {
    const uint64_t G = 256, N = 4096;               // granules of 256 bytes
    slpf::Arena a;
    a.reset(N * G);
    std::vector<uint8_t> busy(N, 0);
    std::vector<std::pair<uint64_t, uint64_t>> live;
    uint64_t seed = 12345;
    for (long k = 0; k < steps; ++k) {
        if (live.empty() || splitmix(seed) % 3 != 0) {
            const uint64_t g = 1 + splitmix(seed) % 96;
            uint64_t want = N;                      // first fit in the model
            for (uint64_t s = 0, run = 0; s < N; ++s) {
                run = busy[s] ? 0 : run + 1;
                if (run == g) {
                    want = s + 1 - g;
                    break;
                }
            }
            uint64_t off = 0;
            const bool got = a.alloc(g * G, &off);
            check(got == (want < N), "alloc succeeds iff a hole fits", k);
            if (got) {
                check(off == want * G, "first-fit offset", k);
                for (uint64_t s = want; s < want + g; ++s) busy[s] = 1;
                live.emplace_back(off, g * G);
            }
        } else {
            const size_t j = splitmix(seed) % live.size();
            a.release(live[j].first, live[j].second);
            for (uint64_t s = live[j].first / G; s < (live[j].first + live[j].second) / G; ++s) busy[s] = 0;
            live[j] = live.back();
            live.pop_back();
        }
        uint64_t held = 0, holes = 0, prev_end = ~0ull;
        for (auto &l : live) held += l.second;
        for (auto &h : a.holes()) {
            check(h.first != prev_end, "holes coalesced", k);
            prev_end = h.first + h.second;
            holes += h.second;
        }
        check(a.used() == held && held + holes == N * G, "arena accounting", k);
    }
    std::printf("arena: %ld steps\n", steps);
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 3) return 2;
    compile_all(argv[1]);
    arena_model(std::stol(argv[2]));
    std::printf(fails ? "FAILED\n" : "ok\n");
    return fails ? 1 : 0;
}

// Byte ranges of the request server's device arena (host-side bookkeeping
// only): first-fit allocation over [0, size), frees coalesced with their
// neighbours.  The server admits a request when its SLPF fits here.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace slpf {

class Arena {
public:
    void reset(uint64_t size) {
        holes_.clear();
        if (size) holes_[0] = size;
        used_ = 0;
    }

    // The lowest free range of `bytes` bytes; false when none is large enough.
    bool alloc(uint64_t bytes, uint64_t *off) {
        for (auto it = holes_.begin(); it != holes_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                holes_.erase(it);
                if (rest) holes_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }

    // Return a range that alloc handed out.
    void release(uint64_t off, uint64_t bytes) {
        used_ -= bytes;
        auto it = holes_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != holes_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            holes_.erase(nx);
        }
        if (it != holes_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                holes_.erase(it);
            }
        }
    }

    uint64_t used() const { return used_; }
    const std::map<uint64_t, uint64_t> &holes() const { return holes_; }   // offset -> size

private:
    std::map<uint64_t, uint64_t> holes_;
    uint64_t used_ = 0;
};

}  // namespace slpf

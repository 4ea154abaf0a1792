// Request server of the SLPF library: continuous batching of parse requests
// on one GPU.
//
// Requests wait in a FIFO queue.  A request is admitted when a job slot is
// free and its output (the SLPF columns and the scalars, sized by
// slpf_forest_bytes) fits in the server's device arena, whose size is the
// memory budget.  Admitted requests of one slot form one job: per parser,
// one slpf_parse_texts on the slot's stream.  Slots run concurrently on
// their own streams, so requests that arrive while others are on the GPU
// are admitted as slots and arena space free up, and their work overlaps on
// the device.  A finished request keeps its arena range until the caller
// releases it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/slpf.h"
#include "arena.hpp"

namespace {

constexpr uint64_t kAlign = 256;

uint64_t round_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
    const slpf_parser *p;
    const uint8_t *text;
    uint64_t n;
    uint64_t tag;
    uint64_t off = 0, bytes = 0, forest = 0;   // arena range; SLPF bytes inside it
    slpf_status st = SLPF_OK;                  // why the request could not be parsed
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request> reqs;
};

}  // namespace

struct slpf_server {
    slpf_server_opts o{};
    uint8_t *arena = nullptr;
    uint64_t arena_bytes = 0;
    slpf::Arena ranges;                          // the arena's free and admitted byte ranges
    std::deque<Request> queue;
    std::vector<Slot> slots;
    std::unordered_map<uint64_t, Request> finished;
    std::deque<uint64_t> done;                   // finished tags not yet reported
    std::vector<const slpf_parser *> used;       // parsers that ran on the slots' streams
};

namespace {

// Admit requests from the queue head into a free slot and launch them as one
// job; *launched is false when the head does not fit in the arena, or when
// no admitted request could be launched (those are reported finished with
// their error status).
slpf_status launch(slpf_server *s, Slot &sl, bool *launched) {
    *launched = false;
    std::vector<Request> batch;
    while (!s->queue.empty() && batch.size() < s->o.max_batch_texts) {
        Request r = s->queue.front();
        if (!s->ranges.alloc(r.bytes, &r.off)) break;   // FIFO: the head waits for space
        s->queue.pop_front();
        batch.push_back(r);
    }
    if (batch.empty()) return SLPF_OK;
    // one batched parse per parser, in order of first appearance
    std::vector<const slpf_parser *> order;
    for (const Request &r : batch)
        if (std::find(order.begin(), order.end(), r.p) == order.end()) order.push_back(r.p);
    slpf_parse_opts po{};
    po.struct_size = sizeof(po);
    po.flags = s->o.parse_flags;
    // a parser whose job cannot be launched fails its own requests only; they
    // are reported finished with that status (no GPU work reads their range)
    std::vector<slpf_text> items;
    std::vector<Request> ran, failed;
    for (const slpf_parser *p : order) {
        if (std::find(s->used.begin(), s->used.end(), p) == s->used.end()) s->used.push_back(p);
        items.clear();
        for (const Request &r : batch) {
            if (r.p != p) continue;
            slpf_text t{};
            t.text_dev = r.text;
            t.n = r.n;
            t.out.columns_dev = reinterpret_cast<uint64_t *>(s->arena + r.off);
            t.out.capacity_bytes = r.forest;
            t.out.scalars_dev = reinterpret_cast<uint64_t *>(s->arena + r.off + round_up(r.forest));
            items.push_back(t);
        }
        const slpf_status st = slpf_parse_texts(p, items.data(), items.size(), &po, sl.stream);
        for (Request r : batch) {
            if (r.p != p) continue;
            r.st = st;
            (st == SLPF_OK ? ran : failed).push_back(r);
        }
    }
    for (const Request &r : failed) {
        s->finished[r.tag] = r;
        s->done.push_back(r.tag);
    }
    if (ran.empty()) return SLPF_OK;
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) {
        // the launched jobs cannot be tracked: wait for them here
        const slpf_status st = hipStreamSynchronize(sl.stream) == hipSuccess ? SLPF_OK : SLPF_E_DEVICE;
        for (Request r : ran) {
            if (st != SLPF_OK) r.st = st;
            s->finished[r.tag] = r;
            s->done.push_back(r.tag);
        }
        return SLPF_OK;
    }
    sl.reqs = std::move(ran);
    sl.busy = true;
    *launched = true;
    return SLPF_OK;
}

}  // namespace

extern "C" {

slpf_status slpf_server_create(const slpf_server_opts *opts, slpf_server **out) {
    if (!opts || !out || opts->struct_size != sizeof(slpf_server_opts)) return SLPF_E_ARG;
    if (opts->slots == 0 || opts->max_batch_texts == 0 || opts->memory_budget < kAlign) return SLPF_E_ARG;
    if (hipSetDevice(opts->device) != hipSuccess) return SLPF_E_DEVICE;
    slpf_server *s = new (std::nothrow) slpf_server();
    if (!s) return SLPF_E_NOMEM;
    s->o = *opts;
    s->arena_bytes = opts->memory_budget / kAlign * kAlign;
    if (hipMalloc(reinterpret_cast<void **>(&s->arena), s->arena_bytes) != hipSuccess) {
        delete s;
        return SLPF_E_NOMEM;
    }
    s->ranges.reset(s->arena_bytes);
    s->slots.resize(opts->slots);
    for (Slot &sl : s->slots) {
        // default-priority streams
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            slpf_server_destroy(s);
            return SLPF_E_DEVICE;
        }
    }
    *out = s;
    return SLPF_OK;
}

void slpf_server_destroy(slpf_server *s) {
    if (!s) return;
    if (hipSetDevice(s->o.device) != hipSuccess) return;
    for (Slot &sl : s->slots) {
        if (sl.stream) {
            (void)hipStreamSynchronize(sl.stream);
            for (const slpf_parser *p : s->used) (void)slpf_parser_trim(p, sl.stream);   // per-stream buffers
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->arena) (void)hipFree(s->arena);
    delete s;
}

slpf_status slpf_server_submit(slpf_server *s, const slpf_parser *p, const uint8_t *text_dev, uint64_t n,
                               uint64_t tag) {
    if (!s || !p || (n && !text_dev) || reinterpret_cast<uintptr_t>(text_dev) % 16 != 0) return SLPF_E_ARG;
    Request r;
    r.p = p;
    r.text = text_dev;
    r.n = n;
    r.tag = tag;
    r.forest = (s->o.parse_flags & SLPF_PARSE_COMPACT) ? slpf_compact_bytes(n) : slpf_forest_bytes(p, n);
    if (r.forest == 0) return SLPF_E_ARG;
    r.bytes = round_up(r.forest) + kAlign;        // columns, then the four scalars
    if (r.bytes > s->arena_bytes) return SLPF_E_CAPACITY;
    s->queue.push_back(r);
    return SLPF_OK;
}

slpf_status slpf_server_poll(slpf_server *s, uint64_t *done_tags, size_t cap, size_t *n_done) {
    if (!s || !n_done || (cap && !done_tags)) return SLPF_E_ARG;
    *n_done = 0;
    if (hipSetDevice(s->o.device) != hipSuccess) return SLPF_E_DEVICE;
    // retire finished jobs
    for (Slot &sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return SLPF_E_DEVICE;
        for (const Request &r : sl.reqs) {
            s->finished[r.tag] = r;
            s->done.push_back(r.tag);
        }
        sl.reqs.clear();
        sl.busy = false;
    }
    // admit and launch while slots are free
    for (Slot &sl : s->slots) {
        if (sl.busy || s->queue.empty()) continue;
        bool launched = false;
        slpf_status st = launch(s, sl, &launched);
        if (st != SLPF_OK) return st;
        if (!launched) break;    // the queue head does not fit yet (or the admitted requests all failed)
    }
    while (*n_done < cap && !s->done.empty()) {
        done_tags[(*n_done)++] = s->done.front();
        s->done.pop_front();
    }
    return SLPF_OK;
}

slpf_status slpf_server_result(const slpf_server *s, uint64_t tag, slpf_forest *out) {
    if (!s || !out) return SLPF_E_ARG;
    auto it = s->finished.find(tag);
    if (it == s->finished.end()) return SLPF_E_ARG;
    const Request &r = it->second;
    out->columns_dev = reinterpret_cast<uint64_t *>(s->arena + r.off);
    out->capacity_bytes = r.forest;
    out->scalars_dev = reinterpret_cast<uint64_t *>(s->arena + r.off + round_up(r.forest));
    return r.st;
}

slpf_status slpf_server_release(slpf_server *s, uint64_t tag) {
    if (!s) return SLPF_E_ARG;
    auto it = s->finished.find(tag);
    if (it == s->finished.end()) return SLPF_E_ARG;
    s->ranges.release(it->second.off, it->second.bytes);
    s->finished.erase(it);
    return SLPF_OK;
}

slpf_status slpf_server_stats(const slpf_server *s, slpf_server_state *st) {
    if (!s || !st) return SLPF_E_ARG;
    st->queued = s->queue.size();
    uint64_t inflight = 0, busy = 0;
    for (const Slot &sl : s->slots)
        if (sl.busy) {
            ++busy;
            inflight += sl.reqs.size();
        }
    st->in_flight = inflight;
    st->busy_slots = busy;
    st->finished_unreleased = s->finished.size();
    st->admitted_bytes = s->ranges.used();
    st->arena_bytes = s->arena_bytes;
    return SLPF_OK;
}

}  // extern "C"

// Serving core: continuous batching of decode requests over the batched
// decode (hamming_decode_batch).  Host code only.
//
// Flow of one request: submit -> FIFO queue -> admission (its outputs are
// carved from the output pool) -> placed in the next batch of a free slot ->
// the slot copies its descriptors to the device and replays its batch graph
// on its own stream -> progress() sees the slot's event complete -> a
// completion record is queued (and the outputs freed when auto_release).
// New batches launch whenever a slot is free, so arrivals overlap with
// batches already on the GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "hamming.h"

namespace {

constexpr uint64_t kAlign = 256;   // output allocations start on 256-byte boundaries

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing frees.
class RangeAllocator {
public:
    explicit RangeAllocator(uint64_t size) : size_(size) { if (size) free_[0] = size; }

    bool alloc(uint64_t bytes, uint64_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes;
                const uint64_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }

    void release(uint64_t off, uint64_t bytes)
    {
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                bytes += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            free_.erase(next);
        }
        free_[off] = bytes;
    }

    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }

private:
    uint64_t size_;
    uint64_t used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Request {
    uint64_t in_word_off, n_cw;
    uint32_t r;
    uint64_t arrival_ns;
    uint64_t out_off = 0, out_bytes = 0;
    uint64_t data_bytes = 0;
    bool done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    unsigned char* host = nullptr;     // pinned: n_packets (uint32, padded to 8) + descriptors
    hamming_packet* descs_dev = nullptr;
    uint32_t* n_dev = nullptr;
    int32_t* status_dev = nullptr;
    int32_t* status_host = nullptr;    // pinned
    void* ws = nullptr;
    uint64_t ws_bytes = 0;
    std::vector<uint64_t> reqs;
    bool busy = false;
};

uint64_t now_ns()
{
    return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                        std::chrono::steady_clock::now().time_since_epoch())
                        .count());
}

}  // namespace

struct hamming_server {
    hamming_server_config cfg;
    const uint64_t* pool = nullptr;
    uint64_t pool_words = 0;
    unsigned char* out_base = nullptr;
    RangeAllocator alloc{0};
    std::vector<Slot> slots;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::deque<hamming_completion> completions;
    uint64_t next_id = 0;
    uint64_t inflight = 0;
    uint64_t batches = 0;
};

namespace {

int message_bits(uint32_t r) { return (1 << r) - 1 - int(r); }

void free_server(hamming_server* s)
{
    for (auto& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.status_host) (void)hipHostFree(sl.status_host);
        if (sl.n_dev) (void)hipFree(sl.n_dev);          // also holds descs_dev
        if (sl.status_dev) (void)hipFree(sl.status_dev);
        if (sl.ws) (void)hipFree(sl.ws);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
}

// Record completions of slots whose batch finished.
int reap(hamming_server* s)
{
    for (auto& sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return HAMMING_EDEVICE;
        const uint64_t t = now_ns();
        for (size_t i = 0; i < sl.reqs.size(); ++i) {
            const uint64_t id = sl.reqs[i];
            Request& rq = s->reqs[id];
            rq.done = true;
            hamming_completion c;
            memset(&c, 0, sizeof c);
            c.request_id = id;
            c.data_offset = rq.out_off;
            c.errpos_offset = rq.out_off + round_up(rq.data_bytes, 16);
            c.submit_ns = rq.arrival_ns;
            c.complete_ns = t;
            c.status = sl.status_host[i];
            s->completions.push_back(c);
            if (s->cfg.auto_release) {
                s->alloc.release(rq.out_off, rq.out_bytes);
                s->reqs.erase(id);
            }
        }
        s->inflight -= sl.reqs.size();
        sl.reqs.clear();
        sl.busy = false;
    }
    return HAMMING_OK;
}

// Fill free slots with admitted requests and launch them.
int launch(hamming_server* s)
{
    for (auto& sl : s->slots) {
        if (sl.busy || s->queue.empty()) continue;
        uint32_t n = 0;
        uint64_t cws = 0;
        auto* descs = reinterpret_cast<hamming_packet*>(sl.host + 8);
        while (!s->queue.empty() && n < s->cfg.max_batch_packets) {
            Request& rq = s->reqs[s->queue.front()];
            if (n > 0 && cws + rq.n_cw > s->cfg.max_batch_codewords) break;
            uint64_t off = 0;
            if (!s->alloc.alloc(rq.out_bytes, &off)) break;      // wait for memory (FIFO)
            rq.out_off = off;
            hamming_packet& d = descs[n];
            d.in_word_off = rq.in_word_off;
            d.n_cw = rq.n_cw;
            d.r = rq.r;
            d.flags = 0;
            d.data_word_off = off / 8;
            d.errpos_off = off + round_up(rq.data_bytes, 16);
            sl.reqs.push_back(s->queue.front());
            s->queue.pop_front();
            cws += rq.n_cw;
            ++n;
        }
        if (n == 0) break;                                       // head of the queue does not fit
        *reinterpret_cast<uint32_t*>(sl.host) = n;
        const uint64_t bytes = 8 + uint64_t(n) * sizeof(hamming_packet);
        // n_packets and the descriptors travel in one copy (n_dev sits just
        // before descs_dev in the same device allocation).
        if (hipMemcpyAsync(sl.n_dev, sl.host, bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            return HAMMING_EDEVICE;
        const int rc = hamming_decode_batch(s->pool, s->pool_words, sl.descs_dev, sl.n_dev,
                                            s->cfg.max_batch_packets, s->cfg.max_batch_codewords,
                                            reinterpret_cast<uint64_t*>(s->out_base), s->alloc.size() / 8,
                                            s->out_base, s->alloc.size(), sl.status_dev, sl.ws, sl.ws_bytes,
                                            sl.stream);
        if (rc != HAMMING_OK) return rc;
        if (hipMemcpyAsync(sl.status_host, sl.status_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                           sl.stream) != hipSuccess)
            return HAMMING_EDEVICE;
        if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return HAMMING_EDEVICE;
        sl.busy = true;
        s->inflight += n;
        ++s->batches;
    }
    return HAMMING_OK;
}

}  // namespace

extern "C" {

uint64_t hamming_server_now_ns(void) { return now_ns(); }

int hamming_server_create(const hamming_server_config* config, const uint64_t* cw_pool, uint64_t cw_pool_words,
                          void* output_pool, uint64_t output_pool_bytes, hamming_server** out)
{
    if (!config || !cw_pool || !output_pool || !out || cw_pool_words == 0 || output_pool_bytes < kAlign)
        return HAMMING_EINVAL;
    const hamming_server_config& c = *config;
    if (c.slots < 1 || c.slots > 16 || c.max_batch_packets < 1 || c.max_batch_packets > 65536 ||
        c.max_batch_codewords < 1 || c.max_queue < 1 || c.auto_release > 1)
        return HAMMING_EINVAL;
    if ((reinterpret_cast<uintptr_t>(cw_pool) & 7u) || (reinterpret_cast<uintptr_t>(output_pool) & (kAlign - 1)))
        return HAMMING_EALIGN;
    *out = nullptr;
    hamming_server* s = new (std::nothrow) hamming_server;
    if (!s) return HAMMING_ENOMEM;
    s->cfg = c;
    s->pool = cw_pool;
    s->pool_words = cw_pool_words;
    s->out_base = static_cast<unsigned char*>(output_pool);
    s->alloc = RangeAllocator(output_pool_bytes / kAlign * kAlign);
    s->slots.resize(c.slots);
    const uint64_t ws_bytes = hamming_batch_workspace_bytes(c.max_batch_packets);
    for (auto& sl : s->slots) {
        char* dev = nullptr;
        const uint64_t dbytes = 8 + uint64_t(c.max_batch_packets) * sizeof(hamming_packet);
        bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
                  hipHostMalloc(reinterpret_cast<void**>(&sl.host), dbytes, hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(reinterpret_cast<void**>(&sl.status_host), 4ull * c.max_batch_packets,
                                hipHostMallocDefault) == hipSuccess &&
                  hipMalloc(reinterpret_cast<void**>(&dev), dbytes) == hipSuccess;
        if (ok) {
            sl.n_dev = reinterpret_cast<uint32_t*>(dev);
            sl.descs_dev = reinterpret_cast<hamming_packet*>(dev + 8);
            ok = hipMalloc(reinterpret_cast<void**>(&sl.status_dev), 4ull * c.max_batch_packets) == hipSuccess &&
                 hipMalloc(&sl.ws, ws_bytes) == hipSuccess;
            sl.ws_bytes = ws_bytes;
        }
        if (!ok) {
            (void)hipGetLastError();
            free_server(s);
            return HAMMING_ENOMEM;
        }
    }
    *out = s;
    return HAMMING_OK;
}

int hamming_server_destroy(hamming_server* s)
{
    if (!s) return HAMMING_EINVAL;
    free_server(s);
    return HAMMING_OK;
}

int hamming_server_submit(hamming_server* s, uint64_t in_word_off, uint64_t n_cw, uint32_t r, uint64_t arrival_ns,
                          uint64_t* request_id)
{
    if (!s || !request_id) return HAMMING_EINVAL;
    if (r < 3 || r > 7) return HAMMING_EINVAL;
    const uint64_t wpc = r == 7 ? 2 : 1;
    if (n_cw > HAMMING_MAX_CODEWORDS || in_word_off > s->pool_words || n_cw * wpc > s->pool_words - in_word_off)
        return HAMMING_ERANGE;
    const uint64_t data_bytes = ((n_cw * uint64_t(message_bits(r)) + 63) / 64) * 8;
    uint64_t out_bytes = round_up(round_up(data_bytes, 16) + n_cw, kAlign);
    if (out_bytes == 0) out_bytes = kAlign;                      // every request owns a range
    if (out_bytes > s->alloc.size()) return HAMMING_ERANGE;
    if (s->queue.size() >= s->cfg.max_queue) return HAMMING_ENOMEM;
    Request rq;
    rq.in_word_off = in_word_off;
    rq.n_cw = n_cw;
    rq.r = r;
    rq.arrival_ns = arrival_ns;
    rq.data_bytes = data_bytes;
    rq.out_bytes = out_bytes;
    const uint64_t id = s->next_id++;
    s->reqs.emplace(id, rq);
    s->queue.push_back(id);
    *request_id = id;
    return HAMMING_OK;
}

int hamming_server_progress(hamming_server* s)
{
    if (!s) return HAMMING_EINVAL;
    const int rc = reap(s);
    if (rc != HAMMING_OK) return rc;
    return launch(s);
}

int hamming_server_poll(hamming_server* s, hamming_completion* out, uint32_t max, uint32_t* n_out)
{
    if (!s || !n_out || (max && !out)) return HAMMING_EINVAL;
    uint32_t n = 0;
    while (n < max && !s->completions.empty()) {
        out[n++] = s->completions.front();
        s->completions.pop_front();
    }
    *n_out = n;
    return HAMMING_OK;
}

int hamming_server_release(hamming_server* s, uint64_t request_id)
{
    if (!s) return HAMMING_EINVAL;
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end() || !it->second.done) return HAMMING_EINVAL;
    s->alloc.release(it->second.out_off, it->second.out_bytes);
    s->reqs.erase(it);
    return HAMMING_OK;
}

int hamming_server_output_pool(hamming_server* s, void** base, uint64_t* bytes)
{
    if (!s || !base || !bytes) return HAMMING_EINVAL;
    *base = s->out_base;
    *bytes = s->alloc.size();
    return HAMMING_OK;
}

int hamming_server_stats(hamming_server* s, uint64_t* queued, uint64_t* inflight, uint64_t* used, uint64_t* batches)
{
    if (!s || !queued || !inflight || !used || !batches) return HAMMING_EINVAL;
    *queued = s->queue.size();
    *inflight = s->inflight;
    *used = s->alloc.used();
    *batches = s->batches;
    return HAMMING_OK;
}

int hamming_server_run_trace(hamming_server* s, uint32_t n, const uint64_t* arrival_ns, const uint64_t* in_word_off,
                             const uint64_t* n_cw, const uint32_t* r, uint64_t timeout_ns, uint64_t* latency_ns,
                             uint64_t* elapsed_ns)
{
    if (!s || !s->cfg.auto_release || (n && (!arrival_ns || !in_word_off || !n_cw || !r || !latency_ns)) ||
        !elapsed_ns)
        return HAMMING_EINVAL;
    std::unordered_map<uint64_t, uint32_t> index;   // request id -> trace position
    index.reserve(n * 2 + 1);
    std::vector<hamming_completion> buf(1024);
    const uint64_t start = now_ns();
    uint32_t next = 0, finished = 0;
    while (finished < n) {
        const uint64_t t = now_ns();
        if (t - start > timeout_ns) return HAMMING_ERANGE;
        while (next < n && arrival_ns[next] <= t - start) {
            uint64_t id = 0;
            const int rc = hamming_server_submit(s, in_word_off[next], n_cw[next], r[next], start + arrival_ns[next],
                                                 &id);
            if (rc != HAMMING_OK) return rc;
            index[id] = next;
            ++next;
        }
        int rc = hamming_server_progress(s);
        if (rc != HAMMING_OK) return rc;
        uint32_t got = 0;
        do {
            rc = hamming_server_poll(s, buf.data(), uint32_t(buf.size()), &got);
            if (rc != HAMMING_OK) return rc;
            for (uint32_t i = 0; i < got; ++i) {
                auto it = index.find(buf[i].request_id);
                if (it == index.end()) continue;          // a request submitted before this trace
                latency_ns[it->second] = buf[i].complete_ns - buf[i].submit_ns;
                index.erase(it);
                ++finished;
            }
        } while (got == buf.size());
    }
    *elapsed_ns = now_ns() - start;
    return HAMMING_OK;
}

}  // extern "C"

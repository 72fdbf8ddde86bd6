// Serving core: continuous batching of decode requests over the batched
// decode (hamming_decode_batch).  Host code only.
//
// Flow of one request: submit -> FIFO queue -> admission (its outputs are
// carved from the output pool) -> placed in the next batch of a free slot ->
// the slot launches the batch on its own stream: a batch of at most 16
// requests and 2^20 codewords is one decode launch with its descriptors in
// the kernel arguments; a larger one is planned on the host (tile prefix sums
// and a coarse tile-to-packet map next to the descriptors), copied to the
// device in one transfer and decoded by one launch -> progress() sees the
// slot's event complete -> a completion record is queued (and the outputs
// freed when auto_release).  The server validated every request at
// submission, so no planning or validation runs on the device.
// New batches launch whenever a slot is free, so arrivals overlap with
// batches already on the GPU.
//
// Every per-request step is O(1): requests live in a ring indexed by id,
// admission is FIFO so a batch is a contiguous id range, and outputs come
// from a ring allocator over the output pool that reclaims space in id
// order (a request released early keeps its space until every older request
// is released too).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <new>
#include <vector>

#include "batch.h"
#include "hamming.h"
#include "host_plan.h"
#include "ring_alloc.h"

namespace {

constexpr uint64_t kAlign = 256;   // output allocations start on 256-byte boundaries

// Batches of at most hm::kSmallBatchMax requests and this many codewords are
// decoded in one launch with their descriptors in the kernel arguments;
// others are planned on the host and decoded by one planned-batch launch.  Measured on the serving trace of
// the bench (256 streams, requests of 256..2^18 codewords): p50 at 10% load
// 22-31 us against 63-70 us; without the codeword bound the one-launch form
// also took large batches and its p50 at 70% load rose from 170-187 us to
// 224-242 us.
constexpr uint64_t kDirectMaxCodewords = uint64_t(1) << 20;

// XCD chunk of the planned-batch launches (consecutive workgroups each XCD
// takes in turn).  Saturated on the serving trace of the bench, two boxes,
// two runs each: 16 was 0.007-0.017 of the plain rate above 128 (the chunk
// tuned for the graph-batched path) on each box, 0.840-0.907 against
// 0.825-0.891, with 32 and 64 in between and 1 lowest.  Served batches are many small requests at random
// places on four streams at once, so they keep a chunk of their own.
constexpr uint32_t kServeXcdChunk = 16;

// Arrivals a trace replay submits between two progress calls.
constexpr uint32_t kSubmitBurst = 256;

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

uint64_t now_ns()
{
    return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                        std::chrono::steady_clock::now().time_since_epoch())
                        .count());
}

enum : uint8_t { kQueued = 0, kInflight = 1, kDone = 2, kReleased = 3 };

struct Request {
    uint64_t in_word_off, n_cw;
    uint64_t arrival_ns;
    uint64_t out_off, out_bytes, data_bytes;
    uint32_t r;
    uint8_t state;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    unsigned char* plan_host = nullptr;   // pinned: the host plan of the slot's batch
    unsigned char* plan_dev = nullptr;    // device: its copy, read by the decode kernel
    uint64_t first = 0, count = 0;        // request ids [first, first + count)
    bool busy = false;
};

}  // namespace

struct hamming_server {
    hamming_server_config cfg;
    const uint64_t* pool = nullptr;
    uint64_t pool_words = 0;
    unsigned char* out_base = nullptr;
    hm::RingAllocator alloc;
    std::vector<Slot> slots;
    std::vector<Request> ring;         // request id -> ring[id % ring.size()]
    uint64_t next_id = 0;              // ids [next_admit, next_id) are queued
    uint64_t next_admit = 0;
    uint64_t oldest_live = 0;          // smallest id not yet released
    std::deque<hamming_completion> completions;
    uint64_t inflight = 0;
    uint64_t batches = 0;

    Request& req(uint64_t id) { return ring[id % ring.size()]; }
};

namespace {

uint64_t message_bytes(uint64_t n_cw, uint32_t r)
{
    const uint64_t k = (uint64_t(1) << r) - 1 - r;
    return ((n_cw * k + 63) / 64) * 8;
}

void free_server(hamming_server* s)
{
    for (auto& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.plan_host) (void)hipHostFree(sl.plan_host);
        if (sl.plan_dev) (void)hipFree(sl.plan_dev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
}

// Reclaim output space of released requests, oldest first.
void reclaim(hamming_server* s)
{
    while (s->oldest_live < s->next_admit) {
        Request& rq = s->req(s->oldest_live);
        if (rq.state != kReleased) break;
        s->alloc.release_oldest(rq.out_off, rq.out_bytes);
        ++s->oldest_live;
    }
}

int reap(hamming_server* s)
{
    for (auto& sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return HAMMING_EDEVICE;
        const uint64_t t = now_ns();
        for (uint64_t id = sl.first; id < sl.first + sl.count; ++id) {
            Request& rq = s->req(id);
            hamming_completion c;
            c.request_id = id;
            c.data_offset = rq.out_off;
            c.errpos_offset = rq.out_off + round_up(rq.data_bytes, 16);
            c.submit_ns = rq.arrival_ns;
            c.complete_ns = t;
            c.status = HAMMING_OK;
            c.reserved = 0;
            s->completions.push_back(c);
            rq.state = s->cfg.auto_release ? kReleased : kDone;
        }
        s->inflight -= sl.count;
        sl.busy = false;
        sl.count = 0;
    }
    if (s->cfg.auto_release) reclaim(s);
    return HAMMING_OK;
}

// Tile prefix sums of a batch's descriptors under the batch schedule in
// force (tiles of 64 lanes of schedule_lane_width codewords each).
bool tile_prefix(const hamming_packet* descs, uint32_t n, int schedule, uint64_t* ts)
{
    ts[0] = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t cwt = 64ull * hm::schedule_lane_width(schedule, descs[i].r);
        if (cwt == 0) return false;
        ts[i + 1] = ts[i] + (descs[i].n_cw + cwt - 1) / cwt;
    }
    return true;
}

// A batch of at most hm::kSmallBatchMax requests: the descriptors (checked
// at submission, outputs carved from the pool) and their tile prefix sums go
// to the decode kernel in its arguments, in one launch.
int launch_small(hamming_server* s, const hamming_packet* descs, uint32_t n, int schedule, hipStream_t stream)
{
    hm::SmallBatch b{};
    b.cw_arena = s->pool;
    b.data_arena = reinterpret_cast<uint64_t*>(s->out_base);
    b.errpos_arena = s->out_base;
    b.n = n;
    for (uint32_t i = 0; i < n; ++i) b.descs[i] = descs[i];
    if (!tile_prefix(descs, n, schedule, b.tile_start)) return HAMMING_EINVAL;
    if (b.tile_start[n] == 0) return HAMMING_OK;                 // nothing but empty requests
    return hm::launch_small_batch(b, schedule, stream) == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

// A larger batch: the host plan (descriptors, already in the slot's pinned
// buffer, then the tile prefix sums and a coarse tile-to-packet map) goes to
// the device in one copy, followed by one decode launch.
int launch_planned(hamming_server* s, Slot& sl, uint32_t n, int schedule, uint32_t xcd_chunk)
{
    const auto* descs = reinterpret_cast<const hamming_packet*>(sl.plan_host);
    const uint64_t ts_off = sizeof(hamming_packet) * uint64_t(n);
    auto* ts = reinterpret_cast<uint64_t*>(sl.plan_host + ts_off);
    if (!tile_prefix(descs, n, schedule, ts)) return HAMMING_EINVAL;
    const uint64_t total = ts[n];
    if (total == 0) return HAMMING_OK;
    // entry j = the packet holding tile j << g, at most planned_coarse_capacity(n) entries
    const uint32_t g = hm::planned_coarse_log2(total, n);
    const uint64_t coarse_off = ts_off + 8ull * (n + 1);
    const uint64_t entries = hm::plan_coarse_map(ts, n, g, reinterpret_cast<uint32_t*>(sl.plan_host + coarse_off));
    const uint64_t bytes = coarse_off + 4 * entries;
    if (hipMemcpyAsync(sl.plan_dev, sl.plan_host, bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
        return HAMMING_EDEVICE;
    hm::PlannedBatch b{};
    b.cw_arena = s->pool;
    b.data_arena = reinterpret_cast<uint64_t*>(s->out_base);
    b.errpos_arena = s->out_base;
    b.descs = reinterpret_cast<const hamming_packet*>(sl.plan_dev);
    b.tile_start = reinterpret_cast<const uint64_t*>(sl.plan_dev + ts_off);
    b.coarse = reinterpret_cast<const uint32_t*>(sl.plan_dev + coarse_off);
    b.total_tiles = total;
    b.n = n;
    b.coarse_log2 = g;
    b.xcd_chunk = xcd_chunk;
    b.chunk_log2 = hm::batch_chunk_log2();
    return hm::launch_planned_batch(b, schedule, sl.stream) == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

// Requests [first, first + n) were admitted but their batch could not be
// launched: complete them with the error status (releasing their outputs when
// auto_release is set, else leaving that to the caller) so the queue and the
// output pool keep moving.
void fail_batch(hamming_server* s, uint64_t first, uint32_t n, int status)
{
    const uint64_t t = now_ns();
    for (uint64_t id = first; id < first + n; ++id) {
        Request& rq = s->req(id);
        hamming_completion c;
        c.request_id = id;
        c.data_offset = rq.out_off;
        c.errpos_offset = rq.out_off + round_up(rq.data_bytes, 16);
        c.submit_ns = rq.arrival_ns;
        c.complete_ns = t;
        c.status = status;
        c.reserved = 0;
        s->completions.push_back(c);
        rq.state = s->cfg.auto_release ? kReleased : kDone;
    }
    if (s->cfg.auto_release) reclaim(s);
}

int launch(hamming_server* s)
{
    int schedule = 0, use_graph = 0;
    uint32_t xcd_chunk = 0, grid_cap = 0;   // only the schedule applies to served batches
    if (hamming_batch_config_get(&schedule, &xcd_chunk, &grid_cap, &use_graph) != HAMMING_OK) return HAMMING_EDEVICE;
    for (auto& sl : s->slots) {
        if (sl.busy || s->next_admit == s->next_id) continue;
        auto* descs = reinterpret_cast<hamming_packet*>(sl.plan_host);
        uint32_t n = 0;
        uint64_t cws = 0;
        const uint64_t first = s->next_admit;
        while (s->next_admit < s->next_id && n < s->cfg.max_batch_packets) {
            Request& rq = s->req(s->next_admit);
            if (n > 0 && cws + rq.n_cw > s->cfg.max_batch_codewords) break;
            uint64_t off = 0;
            if (!s->alloc.alloc(rq.out_bytes, &off)) break;     // wait for memory (FIFO)
            rq.out_off = off;
            rq.state = kInflight;
            hamming_packet& d = descs[n];
            d.in_word_off = rq.in_word_off;
            d.n_cw = rq.n_cw;
            d.r = rq.r;
            d.flags = 0;
            d.data_word_off = off / 8;
            d.errpos_off = off + round_up(rq.data_bytes, 16);
            ++s->next_admit;
            cws += rq.n_cw;
            ++n;
        }
        if (n == 0) break;                                      // the head of the queue does not fit
        int rc;
        if (n <= hm::kSmallBatchMax && cws <= kDirectMaxCodewords)
            rc = launch_small(s, descs, n, schedule, sl.stream);
        else
            rc = launch_planned(s, sl, n, schedule, kServeXcdChunk);
        if (rc == HAMMING_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) rc = HAMMING_EDEVICE;
        if (rc != HAMMING_OK) {
            (void)hipGetLastError();
            fail_batch(s, first, n, rc);
            return rc;
        }
        sl.first = first;
        sl.count = n;
        sl.busy = true;
        s->inflight += n;
        ++s->batches;
    }
    return HAMMING_OK;
}

int run_trace_loop(hamming_server* s, uint32_t n, const uint64_t* arrival_ns, const uint64_t* in_word_off,
                   const uint64_t* n_cw, const uint32_t* r, uint64_t timeout_ns, uint64_t* latency_ns,
                   uint64_t* elapsed_ns, std::deque<hamming_completion>& keep);

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
    s->alloc = hm::RingAllocator(output_pool_bytes / kAlign * kAlign);
    try {
        // queued + in flight + completed but not yet released
        s->ring.resize(uint64_t(c.max_queue) + uint64_t(c.slots) * c.max_batch_packets);
    } catch (...) {
        delete s;
        return HAMMING_ENOMEM;
    }
    s->slots.resize(c.slots);
    const uint64_t plan_bytes = hm::planned_bytes(c.max_batch_packets);
    for (auto& sl : s->slots) {
        const bool ok =
            hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&sl.plan_host), plan_bytes, hipHostMallocDefault) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&sl.plan_dev), plan_bytes) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            free_server(s);
            return HAMMING_ENOMEM;
        }
    }
    // One-time costs are paid here rather than by the first batches: loading
    // the batch kernels' code object (about 1.2 ms), and the first plan-sized
    // copy on each slot's stream (a fresh process's first trace started about
    // 5 ms behind without it).
    bool started = hm::launch_batch_module_start(s->slots[0].stream) == hipSuccess;
    for (auto& sl : s->slots)
        started = started &&
                  hipMemcpyAsync(sl.plan_dev, sl.plan_host, plan_bytes, hipMemcpyHostToDevice, sl.stream) == hipSuccess;
    for (auto& sl : s->slots) started = hipStreamSynchronize(sl.stream) == hipSuccess && started;
    if (!started) {
        (void)hipGetLastError();
        free_server(s);
        return HAMMING_EDEVICE;
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
    const uint64_t data_bytes = message_bytes(n_cw, r);
    uint64_t out_bytes = round_up(round_up(data_bytes, 16) + n_cw, kAlign);
    if (out_bytes == 0) out_bytes = kAlign;                      // every request owns a range
    if (out_bytes >= s->alloc.size()) return HAMMING_ERANGE;
    if (s->next_id - s->next_admit >= s->cfg.max_queue || s->next_id - s->oldest_live >= s->ring.size())
        return HAMMING_ENOMEM;
    Request& rq = s->req(s->next_id);
    rq.in_word_off = in_word_off;
    rq.n_cw = n_cw;
    rq.arrival_ns = arrival_ns;
    rq.out_off = 0;
    rq.out_bytes = out_bytes;
    rq.data_bytes = data_bytes;
    rq.r = r;
    rq.state = kQueued;
    *request_id = s->next_id++;
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
    if (!s || request_id < s->oldest_live || request_id >= s->next_admit) return HAMMING_EINVAL;
    Request& rq = s->req(request_id);
    if (rq.state != kDone) return HAMMING_EINVAL;
    rq.state = kReleased;
    reclaim(s);
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
    *queued = s->next_id - s->next_admit;
    *inflight = s->inflight;
    *used = s->alloc.used();
    *batches = s->batches;
    return HAMMING_OK;
}

int hamming_server_run_trace(hamming_server* s, uint32_t n, const uint64_t* arrival_ns, const uint64_t* in_word_off,
                             const uint64_t* n_cw, const uint32_t* r, uint64_t timeout_ns, uint64_t* latency_ns,
                             uint64_t* elapsed_ns)
{
    if (!s || (n && (!arrival_ns || !in_word_off || !n_cw || !r || !latency_ns)) || !elapsed_ns)
        return HAMMING_EINVAL;
    // completions recorded before the trace stay for the caller; without
    // auto_release the trace's own are kept after them (their outputs stay
    // allocated until released)
    std::deque<hamming_completion> keep;
    keep.swap(s->completions);
    const int rc = run_trace_loop(s, n, arrival_ns, in_word_off, n_cw, r, timeout_ns, latency_ns, elapsed_ns, keep);
    for (const auto& c : s->completions) keep.push_back(c);
    s->completions.swap(keep);
    return rc;
}

}  // extern "C"

namespace {

int run_trace_loop(hamming_server* s, uint32_t n, const uint64_t* arrival_ns, const uint64_t* in_word_off,
                   const uint64_t* n_cw, const uint32_t* r, uint64_t timeout_ns, uint64_t* latency_ns,
                   uint64_t* elapsed_ns, std::deque<hamming_completion>& keep)
{
    const uint64_t first_id = s->next_id;             // trace request i gets id first_id + i
    const uint64_t start = now_ns();
    uint32_t next = 0, finished = 0;
    while (finished < n) {
        const uint64_t t = now_ns();
        if (t - start > timeout_ns) return HAMMING_ERANGE;
        // at most kSubmitBurst arrivals between two progress calls, so a
        // burst of arrivals (a saturated trace has all of them at time 0)
        // does not hold back the first launches
        for (uint32_t burst = 0; burst < kSubmitBurst && next < n && arrival_ns[next] <= t - start; ++burst) {
            uint64_t id = 0;
            const int rc = hamming_server_submit(s, in_word_off[next], n_cw[next], r[next], start + arrival_ns[next],
                                                 &id);
            if (rc == HAMMING_ENOMEM) break;            // queue full: retry after progress
            if (rc != HAMMING_OK) return rc;
            ++next;
        }
        const int rc = hamming_server_progress(s);
        if (rc != HAMMING_OK) return rc;
        while (!s->completions.empty()) {
            const hamming_completion& c = s->completions.front();
            if (c.request_id >= first_id && c.request_id - first_id < n) {
                latency_ns[c.request_id - first_id] = c.complete_ns - c.submit_ns;
                ++finished;
            }
            if (!s->cfg.auto_release) keep.push_back(c);
            s->completions.pop_front();
        }
    }
    *elapsed_ns = now_ns() - start;
    return HAMMING_OK;
}

}  // namespace

// Host side of the batched decode: argument validation, the persistent grid
// size, the hipGraph cache and hamming_batch_layout.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "batch.h"
#include "hamming.h"
#include "launch.h"

namespace {

using hm::BatchArgs;

std::atomic<int> g_schedule{3};
std::atomic<uint32_t> g_grid_cap{0};
std::atomic<uint32_t> g_xcd_chunk{1};
std::atomic<int> g_use_graph{1};
std::atomic<uint32_t> g_chunk_log2{3};

struct GraphKey {
    BatchArgs a;
    int schedule;
    uint32_t grid;
    hipStream_t stream;
    int device;
    bool operator==(const GraphKey& o) const { return memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
};

// Executable graphs are kept until hamming_batch_release_graphs (or the end of
// the process); once the cache is full, calls with new argument sets launch
// directly.  They are not destroyed from a static destructor: at process exit
// that would call into the HIP runtime after its own teardown may have run.
constexpr size_t kMaxGraphs = 64;
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;

hipGraphExec_t find_or_capture(const GraphKey& key, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (const auto& e : g_graphs)
        if (e.key == key) return e.exec;
    if (g_graphs.size() >= kMaxGraphs) return nullptr;
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    const hipError_t le = hm::launch_batch(key.a, key.schedule, key.grid, stream);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(stream, &graph);
    if (le != hipSuccess || ce != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess || !exec) {
        (void)hipGetLastError();
        return nullptr;
    }
    GraphEntry ent;
    memset(&ent, 0, sizeof ent);
    ent.key = key;
    ent.exec = exec;
    g_graphs.push_back(ent);
    return exec;
}

// Workspace of hamming_decode_batch_noalloc: one copy per GPU, held by the
// library's code object until the process ends.  Host code must not use this
// name as an address (it is a host-side stand-in); scratch_address() gives
// the current device's copy.
static __device__ __align__(256) uint8_t scratch[HAMMING_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
std::atomic<void*> g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on device `dev` (the current device), looked up
// on the first call for that device; nullptr when the lookup fails.
void* scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
    return p;
}

bool misaligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) != 0; }

// Upper bound on the tiles of any batch the arguments allow: the input arena
// bounds the codewords as well as the caller's hint does, so the tighter of
// the two is taken, plus one partial tile per packet.
uint64_t batch_tile_bound(uint64_t cw_words, uint32_t max_packets, uint64_t max_codewords, int schedule)
{
    uint64_t tiles = cw_words / hm::schedule_min_tile_words(schedule);
    const uint64_t min_cw = hm::schedule_min_tile_codewords(schedule);
    if (max_codewords && max_codewords / min_cw < tiles) tiles = max_codewords / min_cw;
    return tiles + uint64_t(max_packets);
}

// Workgroups of the batched decode kernel: one wave per chunk of the tile
// bound (waves beyond the real chunk count only read the totals and exit,
// but at 4x the count they cost a visible tail), capped by the configured cap
// and by the dispatch limit, beyond which waves loop over chunks.
uint64_t batch_grid_blocks(uint64_t cw_words, uint32_t max_packets, uint64_t max_codewords, uint64_t cap,
                           uint32_t chunk_log2, int schedule)
{
    const uint64_t chunks =
        (batch_tile_bound(cw_words, max_packets, max_codewords, schedule) + (uint64_t(1) << chunk_log2) - 1) >>
        chunk_log2;
    uint64_t blocks = (chunks + hm::kWavesPerBlockHost - 1) / hm::kWavesPerBlockHost;
    if (cap && blocks > cap) blocks = cap;
    if (blocks > hm::max_launch_blocks(256)) blocks = hm::max_launch_blocks(256);
    if (blocks < 1) blocks = 1;
    return blocks;
}

}  // namespace

namespace hm {

// Validate the arguments of a batched decode and lay the workspace out.
int batch_prepare(const uint64_t* cw_arena, uint64_t cw_words, const hamming_packet* descs,
                  const uint32_t* n_packets_dev, uint32_t max_packets, uint64_t max_codewords, uint64_t* data_arena,
                  uint64_t data_words, uint8_t* errpos_arena, uint64_t errpos_bytes, int32_t* status_out,
                  void* workspace, uint64_t workspace_bytes, int schedule, BatchArgs* out, uint32_t* grid)
{
    if (max_packets > HAMMING_MAX_BATCH) return HAMMING_ERANGE;
    if (!cw_arena || !descs || !n_packets_dev || !data_arena || !workspace) return HAMMING_EINVAL;
    if (misaligned(cw_arena, 8) || misaligned(data_arena, 8) || misaligned(descs, 8) ||
        misaligned(n_packets_dev, 4) || misaligned(workspace, 8) || (status_out && misaligned(status_out, 4)))
        return HAMMING_EALIGN;
    if (workspace_bytes < hm::batch_workspace_min_bytes(max_packets)) return HAMMING_ENOMEM;

    BatchArgs& a = *out;
    memset(&a, 0, sizeof a);
    a.cw_arena = cw_arena;
    a.cw_words = cw_words;
    a.descs = descs;
    a.n_packets_dev = n_packets_dev;
    a.max_packets = max_packets;
    a.data_arena = data_arena;
    a.data_words = data_words;
    a.errpos_arena = errpos_arena;
    a.errpos_bytes = errpos_arena ? errpos_bytes : 0;
    a.status_out = status_out;
    a.xcd_chunk = g_xcd_chunk.load();
    a.chunk_log2 = g_chunk_log2.load();
    a.coarse_cap = hm::batch_coarse_capacity(max_packets);
    a.fine_cap = hm::batch_fine_capacity(max_packets, workspace_bytes);
    a.ws = static_cast<hm::BatchWs*>(workspace);
    a.tile_start = reinterpret_cast<uint64_t*>(static_cast<char*>(workspace) + sizeof(hm::BatchWs));
    a.coarse = reinterpret_cast<uint32_t*>(a.tile_start + (uint64_t(max_packets) + 1));
    a.fine = a.coarse + a.coarse_cap;

    const uint64_t blocks =
        batch_grid_blocks(cw_words, max_packets, max_codewords, g_grid_cap.load(), a.chunk_log2, schedule);
    *grid = uint32_t(blocks);
    // the fine map has at most one entry per chunk of the bound (its kernel
    // is grid-stride, so this only sizes its grid)
    const uint64_t chunks =
        (batch_tile_bound(cw_words, max_packets, max_codewords, schedule) + (uint64_t(1) << a.chunk_log2) - 1) >>
        a.chunk_log2;
    const uint64_t fine_entries = chunks < a.fine_cap ? chunks : a.fine_cap;
    a.fine_blocks = uint32_t((fine_entries + 255) / 256);
    return HAMMING_OK;
}

int batch_schedule() { return g_schedule.load(); }
uint32_t batch_chunk_log2() { return g_chunk_log2.load(); }

}  // namespace hm

extern "C" {

uint64_t hamming_batch_workspace_bytes(uint32_t max_packets)
{
    if (max_packets > HAMMING_MAX_BATCH) return 0;
    return hm::batch_workspace_bytes(max_packets);
}

uint64_t hamming_batch_workspace_min_bytes(uint32_t max_packets)
{
    if (max_packets > HAMMING_MAX_BATCH) return 0;
    return hm::batch_workspace_min_bytes(max_packets);
}

int hamming_batch_layout(hamming_packet* descs, uint32_t n, uint64_t* data_words, uint64_t* errpos_bytes)
{
    if (n > HAMMING_MAX_BATCH) return HAMMING_ERANGE;
    if ((n && !descs) || !data_words || !errpos_bytes) return HAMMING_EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
        if (descs[i].r < 3 || descs[i].r > 7 || descs[i].flags != 0) return HAMMING_EINVAL;
        if (descs[i].n_cw > HAMMING_MAX_CODEWORDS) return HAMMING_ERANGE;
    }
    uint64_t dw = 0, eb = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t k = (uint64_t(1) << descs[i].r) - 1 - descs[i].r;
        const uint64_t words = (descs[i].n_cw * k + 63) / 64;
        descs[i].data_word_off = dw;
        descs[i].errpos_off = eb;
        dw += (words + 1) & ~uint64_t(1);
        eb += (descs[i].n_cw + 15) & ~uint64_t(15);
    }
    *data_words = dw;
    *errpos_bytes = eb;
    return HAMMING_OK;
}

int hamming_batch_config_set(int schedule, uint32_t xcd_chunk, uint32_t grid_cap_blocks, int use_graph)
{
    if (schedule < 0 || schedule > 3 || xcd_chunk < 1 || xcd_chunk > (1u << 20) ||
        (use_graph != 0 && use_graph != 1))
        return HAMMING_EINVAL;
    g_schedule.store(schedule);
    g_xcd_chunk.store(xcd_chunk);
    g_grid_cap.store(grid_cap_blocks);
    g_use_graph.store(use_graph);
    return HAMMING_OK;
}

int hamming_batch_chunk_set(uint32_t tiles_log2)
{
    if (tiles_log2 > hm::kMaxChunkLog2) return HAMMING_EINVAL;
    g_chunk_log2.store(tiles_log2);
    return HAMMING_OK;
}

int hamming_batch_chunk_get(uint32_t* tiles_log2)
{
    if (!tiles_log2) return HAMMING_EINVAL;
    *tiles_log2 = g_chunk_log2.load();
    return HAMMING_OK;
}

int hamming_batch_config_get(int* schedule, uint32_t* xcd_chunk, uint32_t* grid_cap_blocks, int* use_graph)
{
    if (!schedule || !xcd_chunk || !grid_cap_blocks || !use_graph) return HAMMING_EINVAL;
    *schedule = g_schedule.load();
    *xcd_chunk = g_xcd_chunk.load();
    *grid_cap_blocks = g_grid_cap.load();
    *use_graph = g_use_graph.load();
    return HAMMING_OK;
}

int hamming_decode_batch(const uint64_t* cw_arena, uint64_t cw_words, const hamming_packet* descs,
                         const uint32_t* n_packets_dev, uint32_t max_packets, uint64_t max_codewords,
                         uint64_t* data_arena, uint64_t data_words, uint8_t* errpos_arena, uint64_t errpos_bytes,
                         int32_t* status_out, void* workspace, uint64_t workspace_bytes, hipStream_t stream)
{
    if (max_packets > HAMMING_MAX_BATCH) return HAMMING_ERANGE;
    if (max_packets == 0) return HAMMING_OK;
    BatchArgs a;
    uint32_t grid = 0;
    const int schedule = g_schedule.load();
    const int rc = hm::batch_prepare(cw_arena, cw_words, descs, n_packets_dev, max_packets, max_codewords, data_arena,
                                     data_words, errpos_arena, errpos_bytes, status_out, workspace, workspace_bytes,
                                     schedule, &a, &grid);
    if (rc != HAMMING_OK) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HAMMING_EDEVICE;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (stream && hipStreamIsCapturing(stream, &cs) != hipSuccess) return HAMMING_EDEVICE;
    if (stream && cs == hipStreamCaptureStatusNone && g_use_graph.load()) {
        GraphKey key;
        memset(&key, 0, sizeof key);
        key.a = a;
        key.schedule = schedule;
        key.grid = grid;
        key.stream = stream;
        key.device = dev;
        hipGraphExec_t exec = find_or_capture(key, stream);
        if (exec) return hipGraphLaunch(exec, stream) == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
    }
    return hm::launch_batch(a, schedule, grid, stream) == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

int hamming_decode_batch_noalloc(const uint64_t* cw_arena, uint64_t cw_words, const hamming_packet* descs,
                                 const uint32_t* n_packets_dev, uint32_t max_packets, uint64_t max_codewords,
                                 uint64_t* data_arena, uint64_t data_words, uint8_t* errpos_arena,
                                 uint64_t errpos_bytes, int32_t* status_out, hipStream_t stream)
{
    if (max_packets > HAMMING_NOALLOC_MAX_PACKETS) return HAMMING_ERANGE;
    if (max_packets == 0) return HAMMING_OK;
    static_assert(HAMMING_NOALLOC_SCRATCH_BYTES >= hm::batch_workspace_min_bytes(HAMMING_NOALLOC_MAX_PACKETS),
                  "the scratch array must hold the workspace of the largest batch it accepts");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HAMMING_EDEVICE;
    void* ws = scratch_address(dev);
    if (!ws) return HAMMING_EDEVICE;
    BatchArgs a;
    uint32_t grid = 0;
    const int schedule = g_schedule.load();
    const int rc = hm::batch_prepare(cw_arena, cw_words, descs, n_packets_dev, max_packets, max_codewords, data_arena,
                                     data_words, errpos_arena, errpos_bytes, status_out, ws,
                                     HAMMING_NOALLOC_SCRATCH_BYTES, schedule, &a, &grid);
    if (rc != HAMMING_OK) return rc;
    return hm::launch_batch(a, schedule, grid, stream) == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

int hamming_batch_release_graphs(void)
{
    std::lock_guard<std::mutex> lock(g_graph_mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return HAMMING_EDEVICE;
    int rc = HAMMING_OK;
    for (auto& e : g_graphs) {
        // a replay may still be in flight on its device
        if (hipSetDevice(e.key.device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
            hipGraphExecDestroy(e.exec) != hipSuccess)
            rc = HAMMING_EDEVICE;
    }
    g_graphs.clear();
    if (hipSetDevice(cur) != hipSuccess) rc = HAMMING_EDEVICE;
    (void)hipGetLastError();
    return rc;
}

uint64_t hamming_decode_batch_grid(uint64_t cw_words, uint32_t max_packets, uint64_t max_codewords)
{
    if (max_packets == 0 || max_packets > HAMMING_MAX_BATCH) return 0;
    return batch_grid_blocks(cw_words, max_packets, max_codewords, g_grid_cap.load(), g_chunk_log2.load(),
                             g_schedule.load());
}

}  // extern "C"

// Internal interface of the batched decode (kernels in decode_batch.hip,
// host side in batch_host.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming.h"
#include "host_plan.h"

namespace hm {

// Head of the caller's workspace.  After it: tile_start[max_packets + 1]
// (uint64, exclusive prefix sum of tiles per packet), coarse[coarse_cap] and
// fine[fine_cap] (uint32): coarse[j] is the packet holding tile j << coarse_log2,
// fine[j] the packet holding tile j << fine_log2 (fine_log2 >= chunk_log2).
struct BatchWs {
    uint64_t total_tiles;   // tiles of the whole batch
    uint64_t n_packets;     // packets planned (clamped to max_packets)
    uint32_t coarse_log2;
    uint32_t fine_log2;
    uint64_t n_coarse;      // valid coarse entries
    uint64_t n_fine;        // valid fine entries
    uint64_t reserved[3];
};

struct BatchArgs {
    const uint64_t* cw_arena;
    uint64_t cw_words;
    const hamming_packet* descs;
    const uint32_t* n_packets_dev;
    uint32_t max_packets;
    uint32_t xcd_chunk;      // blocks per XCD slice of the decode grid
    uint64_t* data_arena;
    uint64_t data_words;
    uint8_t* errpos_arena;
    uint64_t errpos_bytes;
    int32_t* status_out;
    BatchWs* ws;
    uint64_t* tile_start;
    uint32_t* coarse;
    uint32_t* fine;
    uint32_t coarse_cap;
    uint32_t fine_cap;
    uint32_t fine_blocks;   // grid of the fine-map kernel (it loops over entries beyond the grid)
    uint32_t chunk_log2;    // a wave's unit of work: 2^chunk_log2 consecutive tiles
};

constexpr uint32_t batch_coarse_capacity(uint32_t max_packets) { return 2 * max_packets + 1024; }

// Fine-map entries of the recommended workspace: one per tile of batches up
// to 2^24 tiles (or 4 per packet), so the map is exact for every usual batch.
inline uint32_t batch_fine_capacity_full(uint32_t max_packets)
{
    return (4 * max_packets > (1u << 24)) ? 4 * max_packets : (1u << 24);
}

// Workspace bytes before the fine map: header, tile prefix sums, coarse map.
constexpr uint64_t batch_workspace_fixed_bytes(uint32_t max_packets)
{
    return sizeof(BatchWs) + 8ull * (uint64_t(max_packets) + 1) + 4ull * batch_coarse_capacity(max_packets);
}

// Smallest workspace a call accepts: the fixed part plus one fine entry.
constexpr uint64_t batch_workspace_min_bytes(uint32_t max_packets) { return batch_workspace_fixed_bytes(max_packets) + 4; }

// Recommended workspace (hamming_batch_workspace_bytes).
inline uint64_t batch_workspace_bytes(uint32_t max_packets)
{
    const uint64_t b = batch_workspace_fixed_bytes(max_packets) + 4ull * batch_fine_capacity_full(max_packets);
    return (b + 255) & ~uint64_t(255);
}

// Fine-map entries that a workspace of `bytes` (at least the minimum) holds,
// capped at the recommended count.  A map with fewer entries than tiles
// groups 2^g tiles per entry; the decode kernel then finds a tile's packet by
// a 64-lane probe of the prefix sums from the entry's packet on.
inline uint32_t batch_fine_capacity(uint32_t max_packets, uint64_t bytes)
{
    const uint64_t room = (bytes - batch_workspace_fixed_bytes(max_packets)) / 4;
    const uint64_t full = batch_fine_capacity_full(max_packets);
    return uint32_t(room < full ? room : full);
}

// Waves per workgroup of the decode kernels (tile.h's kWavesPerBlock).
constexpr uint64_t kWavesPerBlockHost = 4;

hipError_t launch_batch(const BatchArgs& a, int schedule, uint32_t grid, hipStream_t stream);

// Validate the arguments of hamming_decode_batch, lay the caller's workspace
// out and size the decode grid.  Returns a status code; *out and *grid are
// set on HAMMING_OK.
int batch_prepare(const uint64_t* cw_arena, uint64_t cw_words, const hamming_packet* descs,
                  const uint32_t* n_packets_dev, uint32_t max_packets, uint64_t max_codewords, uint64_t* data_arena,
                  uint64_t data_words, uint8_t* errpos_arena, uint64_t errpos_bytes, int32_t* status_out,
                  void* workspace, uint64_t workspace_bytes, int schedule, BatchArgs* out, uint32_t* grid);

// The batch schedule in force (hamming_batch_config_set) and the chunk size
// (hamming_batch_chunk_set).
int batch_schedule();
uint32_t batch_chunk_log2();

// Largest chunk: 2^6 tiles.
constexpr uint32_t kMaxChunkLog2 = 6;

// A batch small enough to travel in the kernel arguments: its descriptors
// and the exclusive prefix sum of their tile counts, computed on the host by
// a caller that has validated the descriptors itself (the server).  One
// launch then replaces the descriptor copy, the plan and the two map kernels.
constexpr uint32_t kSmallBatchMax = 16;
struct SmallBatch {
    const uint64_t* cw_arena;
    uint64_t* data_arena;
    uint8_t* errpos_arena;
    uint32_t n;
    uint32_t reserved;
    uint64_t tile_start[kSmallBatchMax + 1];
    hamming_packet descs[kSmallBatchMax];
};

// A batch planned on the host by a caller that has validated its
// descriptors itself (the server): the exclusive prefix sum of the packets'
// tile counts, a coarse tile-to-packet map (entry j = the packet holding tile
// j << coarse_log2) and the descriptors, uploaded in one copy.  One launch of
// decode_planned_batch_kernel then replaces the plan and map kernels: a wave
// reads its map entry and probes the prefix sums 64 entries at a time from
// there.  The map has at most about two entries per packet, so the probe
// almost always ends in its first step.
struct PlannedBatch {
    const uint64_t* cw_arena;
    uint64_t* data_arena;
    uint8_t* errpos_arena;
    const uint64_t* tile_start;     // device, n + 1 entries
    const uint32_t* coarse;         // device, ceil(total_tiles / 2^coarse_log2) entries
    const hamming_packet* descs;    // device, n entries
    uint64_t total_tiles;           // tile_start[n], at least 1
    uint32_t n;
    uint32_t coarse_log2;
    uint32_t xcd_chunk;
    uint32_t chunk_log2;            // a wave's unit of work: 2^chunk_log2 consecutive tiles
};

// Bytes of a host plan of n packets: prefix sums, coarse map (padded to 8
// bytes), descriptors.
inline uint64_t planned_bytes(uint32_t n)
{
    return 8ull * (n + 1) + ((4ull * planned_coarse_capacity(n) + 7) & ~7ull) + sizeof(hamming_packet) * n;
}

hipError_t launch_planned_batch(const PlannedBatch& b, int schedule, hipStream_t stream);

// Codewords per lane of a tile of r-bit codewords in a batch schedule (a
// tile is 64 lanes); 0 for an unknown schedule or r.
uint32_t schedule_lane_width(int schedule, uint32_t r);

// Smallest codeword count and smallest input words of one tile over every r
// of a schedule: they size the grid from an upper bound on the batch's
// codewords or input words.
uint64_t schedule_min_tile_codewords(int schedule);
uint64_t schedule_min_tile_words(int schedule);

// Decodes a small batch whose tile_start[n] tiles are at least one.
hipError_t launch_small_batch(const SmallBatch& b, int schedule, hipStream_t stream);

// Launches an empty kernel from the batched decode's code object: the first
// launch of any kernel of that object in a process loads it (about 1.2 ms),
// so a server does this at creation rather than in its first batch.
hipError_t launch_batch_module_start(hipStream_t stream);

}  // namespace hm

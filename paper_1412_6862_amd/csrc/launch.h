// Internal launch interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {

// Kernel flag bits, decided on the host from pointer alignment.
constexpr uint32_t kFlagIn16 = 1u;    // codeword input is 16-byte aligned
constexpr uint32_t kFlagEpVec = 2u;   // errpos output is aligned to U bytes
constexpr uint32_t kFlagOut16 = 4u;   // message output is 16-byte aligned

struct DecodeLaunch {
    int r;
    int u;                  // codewords per lane
    const uint64_t* cw;
    uint64_t n_cw;
    uint64_t* data;
    uint64_t data_words;
    uint8_t* errpos;
    uint64_t max_blocks;    // 0 = one wave per tile
    uint32_t xcd_chunk;     // blocks per XCD slice (1 = hardware order)
};

// A dispatch packet holds its grid size in work-items as a 32-bit field, so
// one launch has at most this many workgroups of `threads` work-items.
constexpr uint64_t kMaxDispatchItems = 0xFFFFFFFFull;
constexpr uint64_t max_launch_blocks(uint64_t threads) { return kMaxDispatchItems / threads; }

// Workgroups (of 4 waves) of a plain decode launch over n_tiles wave tiles:
// one wave per tile, capped by max_blocks (0 = no cap) and by the dispatch
// limit; the kernel's waves loop over the tiles beyond the grid.
constexpr uint64_t plain_grid_blocks(uint64_t n_tiles, uint64_t max_blocks)
{
    uint64_t blocks = (n_tiles + 3) / 4;
    if (max_blocks && blocks > max_blocks) blocks = max_blocks;
    if (blocks > max_launch_blocks(256)) blocks = max_launch_blocks(256);
    return blocks;
}

// Smallest lane width that gives every lane chunk at least one dword.
constexpr bool valid_u(int r, int u)
{
    const int k = (1 << r) - 1 - r;
    return (u == 2 || u == 4 || u == 8 || u == 16) && u * k >= 32;
}

hipError_t launch_decode(const DecodeLaunch& L, hipStream_t stream);
hipError_t launch_encode(int r, const void* stream_in, uint64_t n_cw, uint64_t* out, hipStream_t stream);

}  // namespace hm

// Plain packet decode kernel for gfx950.  The per-wave tile decode lives in
// tile.h; this file holds the plain grid over one packet and its launcher.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming_device.h"
#include "launch.h"
#include "tile.h"

namespace hm {

// Wave w of the grid takes tiles w, w + waves, w + 2*waves, ... (one tile
// per wave when the grid covers the packet).  With a 16-byte aligned input,
// the full tiles run as a two-stage pipeline: a wave issues the loads of its
// next tile before it decodes the current one, so a grid smaller than the
// packet keeps two tiles of loads in flight per wave and pays its set-up once
// for many tiles.  The ragged last tile, and every tile of an unaligned
// input, go through the checked path.
template <int R, int U>
__global__ __launch_bounds__(kBlockThreads) void decode_plain_kernel(
    const uint64_t* __restrict__ cw, uint64_t n_cw, uint64_t* __restrict__ data, uint64_t data_words,
    uint8_t* __restrict__ errpos, uint64_t n_tiles, uint32_t flags, uint32_t xcd_chunk)
{
    using T = TileShape<R, U>;
    __shared__ u32x4 lds_raw[kWavesPerBlock][T::LDS_DW / 4];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar bookkeeping
    uint32_t* lds = reinterpret_cast<uint32_t*>(&lds_raw[wave][0]);
    const uint64_t waves = uint64_t(gridDim.x) * kWavesPerBlock;
    uint64_t t = uint64_t(xcd_block(blockIdx.x, gridDim.x, xcd_chunk)) * kWavesPerBlock + wave;
    if (flags & kFlagIn16) {
        const uint64_t n_full = n_cw / T::CW;
        if (t < n_full) {
            TileIn<R, U> cur;
            load_full_tile<R, U>(cw, t, cur);
            for (;;) {
                const uint64_t tn = t + waves;
                if (tn >= n_full) break;
                TileIn<R, U> nxt;
                load_full_tile<R, U>(cw, tn, nxt);          // in flight while `cur` is decoded
                finish_tile<R, U>(cur, n_cw, t, data, data_words, errpos, lds, flags);
                cur = nxt;
                t = tn;
            }
            finish_tile<R, U>(cur, n_cw, t, data, data_words, errpos, lds, flags);
            t += waves;
        }
        // the ragged tile n_full, if any, falls to the wave whose turn it is
        while (t < n_full) t += waves;
    }
    for (; t < n_tiles; t += waves)
        decode_tile<R, U>(cw, n_cw, t, data, data_words, errpos, lds, flags);
}

// ---- launchers ----------------------------------------------------------------

template <int R, int U>
static hipError_t launch_decode_ru(const DecodeLaunch& L, hipStream_t stream)
{
    using T = TileShape<R, U>;
    static_assert(kWavesPerBlock == 4 && kBlockThreads == 256, "plain_grid_blocks assumes 4-wave workgroups");
    const uint64_t n_tiles = (L.n_cw + T::CW - 1) / T::CW;
    const uint64_t blocks = plain_grid_blocks(n_tiles, L.max_blocks);
    if (blocks == 0) return hipSuccess;
    uint32_t flags = 0;
    if ((reinterpret_cast<uintptr_t>(L.cw) & 15u) == 0) flags |= kFlagIn16;
    if (L.errpos && (reinterpret_cast<uintptr_t>(L.errpos) % U) == 0) flags |= kFlagEpVec;
    if ((reinterpret_cast<uintptr_t>(L.data) & 15u) == 0) flags |= kFlagOut16;
    hipLaunchKernelGGL((decode_plain_kernel<R, U>), dim3(uint32_t(blocks)), dim3(kBlockThreads), 0, stream,
                       L.cw, L.n_cw, L.data, L.data_words, L.errpos, n_tiles, flags, L.xcd_chunk);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_decode_r(const DecodeLaunch& L, hipStream_t stream)
{
    if (!valid_u(R, L.u)) return hipErrorInvalidValue;
    switch (L.u) {
    case 2: if constexpr (valid_u(R, 2)) return launch_decode_ru<R, 2>(L, stream); break;
    case 4: if constexpr (valid_u(R, 4)) return launch_decode_ru<R, 4>(L, stream); break;
    case 8: if constexpr (valid_u(R, 8)) return launch_decode_ru<R, 8>(L, stream); break;
    case 16: if constexpr (valid_u(R, 16)) return launch_decode_ru<R, 16>(L, stream); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_decode(const DecodeLaunch& L, hipStream_t stream)
{
    switch (L.r) {
    case 3: return launch_decode_r<3>(L, stream);
    case 4: return launch_decode_r<4>(L, stream);
    case 5: return launch_decode_r<5>(L, stream);
    case 6: return launch_decode_r<6>(L, stream);
    case 7: return launch_decode_r<7>(L, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hm

// Plain packet decode kernel for gfx950.  The per-wave tile decode lives in
// tile.h; this file holds the plain grid over one packet and its launcher.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming_device.h"
#include "launch.h"
#include "tile.h"

namespace hm {

// Wave w of the grid takes tiles w, w + waves, w + 2*waves, ... (one tile
// per wave when the grid covers the packet); a grid smaller than the packet
// keeps two tiles of loads in flight per wave and pays its set-up once for
// many tiles.
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
    const uint64_t t = uint64_t(xcd_block(blockIdx.x, gridDim.x, xcd_chunk)) * kWavesPerBlock + wave;
    decode_run<R, U>(cw, n_cw, t, n_tiles, waves, data, data_words, errpos, lds, flags);
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
    if (L.errpos && (reinterpret_cast<uintptr_t>(L.errpos) % U) == 0) flags |= kFlagEpVec;
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

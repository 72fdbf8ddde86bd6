// Plain packet decode and encode kernels for gfx950.
//
// Decode work split.  A wave owns a tile of 64*U consecutive codewords; lane
// L decodes the U consecutive codewords [64*U*t + U*L, +U) of tile t, so its
// input is one contiguous run of U*8*WPC bytes, read with 16-byte loads.  The
// checksum, correction and redundancy removal (Sec. II; Sec. III.C) run
// per lane in registers; the checksum never leaves the lane.
//
// Merge (Sec. II, the merger).  The lane's U messages are concatenated into a
// chunk of B = U*k bits with compile-time shifts.  Chunks of consecutive
// lanes are consecutive in the output stream, and 64 lanes produce exactly
// B 64-bit words, so every tile writes a disjoint, word-aligned range.  Lane
// L owns the output dwords that start inside its chunk; the last of them
// reaches into lane L+1's chunk, whose first dword arrives by one cross-lane
// shuffle.  Owned dwords are written to a wave-private LDS buffer and read
// back as 64-bit words by consecutive lanes, so global stores are coalesced.
// No atomics, no block barrier.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming_device.h"
#include "launch.h"

namespace hm {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = 64 * kWavesPerBlock;

template <int R, int U>
struct TileShape {
    using C = Code<R>;
    static constexpr int CW = 64 * U;               // codewords per wave tile
    static constexpr int B = U * C::K;              // message bits per lane chunk
    static constexpr int CHW = (B + 31) / 32;       // dwords per chunk
    static constexpr int BR = B % 32;
    static constexpr int WORDS = B;                 // 64-bit output words per full tile
    static constexpr int LDS_DW = 2 * B;            // LDS staging dwords per wave
    static_assert(B >= 32, "a lane chunk must span at least one dword");
    static_assert((U * C::DW) % 4 == 0, "lane input must be whole 16-byte vectors");
};

// Insert a k-bit message at compile-time bit offset OFF of a chunk.
template <int R, int OFF, int CHA>
__device__ __forceinline__ void chunk_insert(uint32_t (&chunk)[CHA], const uint32_t (&p)[Code<R>::PW])
{
    constexpr int q = OFF / 32;
    constexpr int sh = OFF % 32;
#pragma unroll
    for (int i = 0; i < Code<R>::PW; ++i) {
        chunk[q + i] |= p[i] << sh;
        if constexpr (sh != 0) chunk[q + i + 1] |= p[i] >> (32 - sh);
    }
}

template <int R, int U, int u, int CHA>
__device__ __forceinline__ void decode_lane_codewords(uint32_t (&in)[U * Code<R>::DW],
                                                      uint32_t (&chunk)[CHA], uint32_t (&s)[U])
{
    if constexpr (u < U) {
        using C = Code<R>;
        uint32_t a[C::DW];
#pragma unroll
        for (int d = 0; d < C::DW; ++d) a[d] = in[u * C::DW + d];
        mask_padding<R>(a);
        const uint32_t syn = checksum<R>(a);     // error detection
        correct<R>(a, syn);                      // error correction
        uint32_t p[C::PW];
        extract<R>(a, p);                        // redundancy removal
        s[u] = syn;
        chunk_insert<R, u * C::K>(chunk, p);     // merge, within the lane
        decode_lane_codewords<R, U, u + 1>(in, chunk, s);
    }
}

template <int R, int U>
__device__ __forceinline__ void decode_tile(const uint64_t* __restrict__ cw, uint64_t n_cw, uint64_t tile,
                                            uint64_t* __restrict__ data, uint64_t data_words,
                                            uint8_t* __restrict__ errpos, uint32_t* lds, uint32_t flags)
{
    using C = Code<R>;
    using T = TileShape<R, U>;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t c0 = tile * T::CW + uint64_t(lane) * U;
    const bool full = (tile + 1) * T::CW <= n_cw;

    // ---- load U codewords --------------------------------------------------
    uint32_t in[U * C::DW];
    if (full && (flags & kFlagIn16)) {
        const u32x4* src = reinterpret_cast<const u32x4*>(cw + c0 * C::WPC);
#pragma unroll
        for (int v = 0; v < U * C::DW / 4; ++v) {
            const u32x4 x = __builtin_nontemporal_load(src + v);
            in[4 * v + 0] = x.x;
            in[4 * v + 1] = x.y;
            in[4 * v + 2] = x.z;
            in[4 * v + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int q = 0; q < C::WPC; ++q) {
                const uint64_t x = (c0 + u < n_cw) ? cw[(c0 + u) * C::WPC + q] : 0;
                in[u * C::DW + 2 * q] = uint32_t(x);
                in[u * C::DW + 2 * q + 1] = uint32_t(x >> 32);
            }
        }
    }

    // ---- decode, merge within the lane ------------------------------------
    constexpr int CHA = T::CHW + 2;
    uint32_t chunk[CHA];
#pragma unroll
    for (int i = 0; i < CHA; ++i) chunk[i] = 0;
    uint32_t s[U];
    decode_lane_codewords<R, U, 0>(in, chunk, s);

    // ---- error positions ---------------------------------------------------
    if (errpos) {
        if (full && (flags & kFlagEpVec)) {
            if constexpr (U == 2) {
                *reinterpret_cast<uint16_t*>(errpos + c0) = uint16_t(s[0] | (s[1] << 8));
            } else {
                uint32_t packed[U / 4];
#pragma unroll
                for (int g = 0; g < U / 4; ++g)
                    packed[g] = s[4 * g] | (s[4 * g + 1] << 8) | (s[4 * g + 2] << 16) | (s[4 * g + 3] << 24);
                if constexpr (U == 4) {
                    *reinterpret_cast<uint32_t*>(errpos + c0) = packed[0];
                } else {
#pragma unroll
                    for (int g = 0; g < U / 8; ++g)
                        reinterpret_cast<uint2*>(errpos + c0)[g] = make_uint2(packed[2 * g], packed[2 * g + 1]);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (c0 + u < n_cw) errpos[c0 + u] = uint8_t(s[u]);
        }
    }

    // ---- merge across lanes: owned dwords -> LDS ---------------------------
    uint32_t e[T::CHW + 1];
#pragma unroll
    for (int i = 0; i < T::CHW; ++i) e[i] = chunk[i];
    e[T::CHW] = 0;
    if constexpr (T::BR != 0) {
        const uint32_t nxt = __shfl_down(chunk[0], 1);   // first dword of lane L+1's chunk
        e[T::CHW - 1] |= nxt << T::BR;
        e[T::CHW] = nxt >> (32 - T::BR);
    }
    const uint32_t bitpos = lane * uint32_t(T::B);
    const uint32_t first = (bitpos + 31u) >> 5;
    const uint32_t a = (first << 5) - bitpos;
    const uint32_t n_own = ((bitpos + T::B + 31u) >> 5) - first;
#pragma unroll
    for (int i = 0; i < T::CHW; ++i) {
        const uint32_t v = (T::BR == 0) ? e[i] : __builtin_amdgcn_alignbit(e[i + 1], e[i], a);
        if (T::BR == 0 || uint32_t(i) < n_own) lds[first + i] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // ---- LDS -> global, 64-bit words by consecutive lanes -------------------
    const uint64_t w0 = tile * uint64_t(T::WORDS);
    const uint64_t nw = (data_words - w0 < uint64_t(T::WORDS)) ? (data_words - w0) : uint64_t(T::WORDS);
    const uint2* l2 = reinterpret_cast<const uint2*>(lds);
#pragma unroll
    for (int q = 0; q < (T::WORDS + 63) / 64; ++q) {
        const uint32_t j = lane + 64u * q;
        if (j < nw) {
            const uint2 v = l2[j];
            __builtin_nontemporal_store(uint64_t(v.x) | (uint64_t(v.y) << 32), data + w0 + j);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int R, int U>
__global__ __launch_bounds__(kBlockThreads) void decode_plain_kernel(
    const uint64_t* __restrict__ cw, uint64_t n_cw, uint64_t* __restrict__ data, uint64_t data_words,
    uint8_t* __restrict__ errpos, uint64_t n_tiles, uint32_t flags)
{
    using T = TileShape<R, U>;
    __shared__ uint2 lds_raw[kWavesPerBlock][(T::LDS_DW + 1) / 2];
    const uint32_t wave = threadIdx.x >> 6;
    uint32_t* lds = reinterpret_cast<uint32_t*>(&lds_raw[wave][0]);
    const uint64_t stride = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t tile = uint64_t(blockIdx.x) * kWavesPerBlock + wave; tile < n_tiles; tile += stride)
        decode_tile<R, U>(cw, n_cw, tile, data, data_words, errpos, lds, flags);
}

// ---- encoder: one codeword per thread --------------------------------------
template <int R>
__global__ __launch_bounds__(256) void encode_plain_kernel(const uint32_t* __restrict__ stream,
                                                           uint64_t stream_dwords, uint64_t n_cw,
                                                           uint64_t* __restrict__ cw_out)
{
    using C = Code<R>;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_cw; i += stride) {
        const uint64_t o = i * C::K;
        const uint64_t d = o >> 5;
        const uint32_t sh = uint32_t(o & 31u);
        uint32_t raw[C::PW + 1];
#pragma unroll
        for (int q = 0; q <= C::PW; ++q) raw[q] = (d + q < stream_dwords) ? stream[d + q] : 0u;
        uint32_t p[C::PW];
#pragma unroll
        for (int q = 0; q < C::PW; ++q) p[q] = __builtin_amdgcn_alignbit(raw[q + 1], raw[q], sh);
        if constexpr (C::K % 32 != 0) p[C::PW - 1] &= (1u << (C::K % 32)) - 1u;
        uint32_t a[C::DW];
        deposit<R>(p, a);
        set_checksum_bits<R>(a, checksum<R>(a));
#pragma unroll
        for (int q = 0; q < C::WPC; ++q) cw_out[i * C::WPC + q] = uint64_t(a[2 * q]) | (uint64_t(a[2 * q + 1]) << 32);
    }
}

// ---- launchers ----------------------------------------------------------------

template <int R, int U>
static hipError_t launch_decode_ru(const DecodeLaunch& L, hipStream_t stream)
{
    using T = TileShape<R, U>;
    const uint64_t n_tiles = (L.n_cw + T::CW - 1) / T::CW;
    uint64_t blocks = (n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const uint64_t cap = L.max_blocks ? L.max_blocks : blocks;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) return hipSuccess;
    uint32_t flags = 0;
    if ((reinterpret_cast<uintptr_t>(L.cw) & 15u) == 0) flags |= kFlagIn16;
    if (L.errpos && (reinterpret_cast<uintptr_t>(L.errpos) % U) == 0) flags |= kFlagEpVec;
    hipLaunchKernelGGL((decode_plain_kernel<R, U>), dim3(uint32_t(blocks)), dim3(kBlockThreads), 0, stream,
                       L.cw, L.n_cw, L.data, L.data_words, L.errpos, n_tiles, flags);
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

template <int R>
static hipError_t launch_encode_r(const void* stream_in, uint64_t n_cw, uint64_t* out, hipStream_t stream)
{
    using C = Code<R>;
    const uint64_t dwords = 2 * ((n_cw * C::K + 63) / 64);
    uint64_t blocks = (n_cw + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((encode_plain_kernel<R>), dim3(uint32_t(blocks)), dim3(256), 0, stream,
                       static_cast<const uint32_t*>(stream_in), dwords, n_cw, out);
    return hipGetLastError();
}

hipError_t launch_encode(int r, const void* stream_in, uint64_t n_cw, uint64_t* out, hipStream_t stream)
{
    switch (r) {
    case 3: return launch_encode_r<3>(stream_in, n_cw, out, stream);
    case 4: return launch_encode_r<4>(stream_in, n_cw, out, stream);
    case 5: return launch_encode_r<5>(stream_in, n_cw, out, stream);
    case 6: return launch_encode_r<6>(stream_in, n_cw, out, stream);
    case 7: return launch_encode_r<7>(stream_in, n_cw, out, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hm

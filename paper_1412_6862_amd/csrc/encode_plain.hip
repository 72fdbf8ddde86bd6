// Plain packet encoder for gfx950 (the transmitter's half of Sec. II): the
// message of codeword i is bits [i*k, i*k+k) of the dense LSB-first stream;
// the checksum bits follow Sec. III.C.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming_device.h"
#include "launch.h"

namespace hm {

typedef uint32_t enc_u32x4 __attribute__((ext_vector_type(4)));

// ---- encoder: a thread builds the codewords of one 16-byte output vector ---
// (two codewords for r <= 6, one for r = 7) and writes them with one
// nontemporal 16-byte store when the output is 16-byte aligned.
template <int R>
__device__ __forceinline__ void encode_one(const uint32_t* __restrict__ stream, uint64_t stream_dwords, uint64_t i,
                                           uint32_t (&a)[Code<R>::DW])
{
    using C = Code<R>;
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
    deposit<R>(p, a);
    set_checksum_bits<R>(a, checksum<R>(a));
}

template <int R>
__global__ __launch_bounds__(256) void encode_plain_kernel(const uint32_t* __restrict__ stream,
                                                           uint64_t stream_dwords, uint64_t n_cw,
                                                           uint64_t* __restrict__ cw_out, uint32_t out16)
{
    using C = Code<R>;
    constexpr int PER = C::WPC == 1 ? 2 : 1;          // codewords per 16-byte vector
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    const uint64_t n_vec = (n_cw + PER - 1) / PER;
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n_vec; j += stride) {
        uint32_t a[PER][C::DW];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint64_t i = j * PER + u;
            if (i < n_cw) {
                encode_one<R>(stream, stream_dwords, i, a[u]);
            } else {
#pragma unroll
                for (int q = 0; q < C::DW; ++q) a[u][q] = 0;
            }
        }
        const bool full = (j + 1) * PER <= n_cw;
        if (out16 && full) {
            enc_u32x4 v;
            v.x = a[0][0];
            v.y = a[0][1];
            v.z = PER == 2 ? a[PER - 1][0] : a[0][C::DW > 2 ? 2 : 0];
            v.w = PER == 2 ? a[PER - 1][1] : a[0][C::DW > 3 ? 3 : 0];
            __builtin_nontemporal_store(v, reinterpret_cast<enc_u32x4*>(cw_out) + j);
        } else {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint64_t i = j * PER + u;
                if (i >= n_cw) break;
#pragma unroll
                for (int q = 0; q < C::WPC; ++q)
                    cw_out[i * C::WPC + q] = uint64_t(a[u][2 * q]) | (uint64_t(a[u][2 * q + 1]) << 32);
            }
        }
    }
}

template <int R>
static hipError_t launch_encode_r(const void* stream_in, uint64_t n_cw, uint64_t* out, hipStream_t stream)
{
    using C = Code<R>;
    constexpr uint64_t per = C::WPC == 1 ? 2 : 1;
    const uint64_t dwords = 2 * ((n_cw * C::K + 63) / 64);
    const uint64_t n_vec = (n_cw + per - 1) / per;
    uint64_t blocks = (n_vec + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) return hipSuccess;
    const uint32_t out16 = (reinterpret_cast<uintptr_t>(out) & 15u) == 0 ? 1u : 0u;
    hipLaunchKernelGGL((encode_plain_kernel<R>), dim3(uint32_t(blocks)), dim3(256), 0, stream,
                       static_cast<const uint32_t*>(stream_in), dwords, n_cw, out, out16);
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

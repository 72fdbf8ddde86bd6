// Plain packet encoder for gfx950 (the transmitter's half of Sec. II): the
// message of codeword i is bits [i*k, i*k+k) of the dense LSB-first stream;
// the checksum bits follow Sec. III.C.  A thread builds the codewords of one
// 16-byte output vector at a time (two codewords for r <= 6, one for r = 7)
// and writes them with one nontemporal 16-byte store when the output is
// 16-byte aligned.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming_device.h"
#include "launch.h"

namespace hm {

typedef uint32_t enc_u32x4 __attribute__((ext_vector_type(4)));

template <int R>
struct EncShape {
    using C = Code<R>;
    static constexpr int PER = C::WPC == 1 ? 2 : 1;                        // codewords per vector
    static constexpr uint32_t VPT = 2;                                     // vectors per thread (staged)
    static constexpr uint32_t CW = 256u * PER * VPT;                       // codewords per tile (staged)
    static constexpr uint32_t LDS_Q = (CW * C::K) / 64 + C::PW / 2 + 3;    // staged 64-bit words
};

// raw holds the PW+1 stream dwords starting at the one that holds message bit
// 0; sh is that bit's offset in raw[0].
template <int R>
__device__ __forceinline__ void build_codeword(const uint32_t (&raw)[Code<R>::PW + 1], uint32_t sh,
                                               uint32_t (&a)[Code<R>::DW])
{
    using C = Code<R>;
    uint32_t p[C::PW];
#pragma unroll
    for (int q = 0; q < C::PW; ++q) p[q] = __builtin_amdgcn_alignbit(raw[q + 1], raw[q], sh);
    if constexpr (C::K % 32 != 0) p[C::PW - 1] &= (1u << (C::K % 32)) - 1u;
    deposit<R>(p, a);
    set_checksum_bits<R>(a, checksum<R>(a));
}

// Output vector j holds codewords j*PER .. j*PER+PER-1; codewords at or past
// n_cw are not written.
template <int R>
__device__ __forceinline__ void store_vector(const uint32_t (&a)[EncShape<R>::PER][Code<R>::DW], uint64_t j,
                                             uint64_t n_cw, uint32_t out16, uint64_t* __restrict__ cw_out)
{
    using C = Code<R>;
    constexpr int PER = EncShape<R>::PER;
    if (out16 && (j + 1) * PER <= n_cw) {
        enc_u32x4 v;
        v.x = a[0][0];
        v.y = a[0][1];
        v.z = PER == 2 ? a[PER - 1][0] : a[0][C::DW > 2 ? 2 : 0];
        v.w = PER == 2 ? a[PER - 1][1] : a[0][C::DW > 3 ? 3 : 0];
        __builtin_nontemporal_store(v, reinterpret_cast<enc_u32x4*>(cw_out) + j);
        return;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint64_t i = j * PER + u;
        if (i >= n_cw) break;
#pragma unroll
        for (int q = 0; q < C::WPC; ++q)
            cw_out[i * C::WPC + q] = uint64_t(a[u][2 * q]) | (uint64_t(a[u][2 * q + 1]) << 32);
    }
}

// ---- short messages (r = 3..5): each thread loads its own stream words -----
template <int R>
__global__ __launch_bounds__(256) void encode_plain_kernel(const uint32_t* __restrict__ stream,
                                                           uint64_t stream_dwords, uint64_t n_cw,
                                                           uint64_t* __restrict__ cw_out, uint32_t out16)
{
    using C = Code<R>;
    constexpr int PER = EncShape<R>::PER;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    const uint64_t n_vec = (n_cw + PER - 1) / PER;
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n_vec; j += stride) {
        uint32_t a[PER][C::DW];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint64_t o = (j * PER + u) * C::K;
            const uint64_t d = o >> 5;
            uint32_t raw[C::PW + 1];
#pragma unroll
            for (int q = 0; q <= C::PW; ++q) raw[q] = (d + q < stream_dwords) ? stream[d + q] : 0u;
            build_codeword<R>(raw, uint32_t(o & 31u), a[u]);
        }
        store_vector<R>(a, j, n_cw, out16, cw_out);
    }
}

// ---- long messages (r = 6, 7): the stream is staged through LDS ------------
// A workgroup of 256 threads encodes one tile of 512 output vectors (two per
// thread, 256 apart, so stores stay coalesced).  The tile's slice of the
// message stream is staged in LDS with coalesced 64-bit loads; each thread
// then funnel-shifts its messages out of LDS instead of issuing PW+1 32-bit
// loads per codeword at a k-bit stride.  A workgroup loops over tiles and
// loads the next tile's words into registers while it encodes the current
// one.  Words past the end of the stream are staged as zero (their bits are
// masked off or belong to no codeword).
template <int R>
__global__ __launch_bounds__(256) void encode_staged_kernel(const uint64_t* __restrict__ stream, uint64_t stream_q,
                                                            uint64_t n_cw, uint64_t* __restrict__ cw_out,
                                                            uint32_t out16)
{
    using C = Code<R>;
    using S = EncShape<R>;
    constexpr int PER = S::PER;
    constexpr uint32_t LPT = (S::LDS_Q + 255) / 256;      // staged words per thread
    __shared__ uint64_t lds_q[S::LDS_Q];
    const uint32_t* lds = reinterpret_cast<const uint32_t*>(lds_q);
    const uint64_t n_tiles = (n_cw + S::CW - 1) / S::CW;
    const uint64_t n_vec = (n_cw + PER - 1) / PER;
    uint64_t nxt[LPT];
    auto fetch = [&](uint64_t t) {
        const uint64_t q0 = (t * S::CW * C::K) >> 6;
#pragma unroll
        for (uint32_t l = 0; l < LPT; ++l) {
            const uint32_t e = threadIdx.x + 256u * l;
            const uint64_t q = q0 + e;
            nxt[l] = (e < S::LDS_Q && q < stream_q) ? __builtin_nontemporal_load(stream + q) : uint64_t(0);
        }
    };
    uint64_t t = blockIdx.x;
    if (t < n_tiles) fetch(t);
    for (; t < n_tiles; t += gridDim.x) {
        const uint64_t q0 = (t * S::CW * C::K) >> 6;      // first staged word
        __syncthreads();                                   // the previous tile's reads are done
#pragma unroll
        for (uint32_t l = 0; l < LPT; ++l) {
            const uint32_t e = threadIdx.x + 256u * l;
            if (e < S::LDS_Q) lds_q[e] = nxt[l];
        }
        __syncthreads();
        if (t + gridDim.x < n_tiles) fetch(t + gridDim.x);   // next tile's words load during this tile's work
#pragma unroll
        for (uint32_t w = 0; w < S::VPT; ++w) {
            const uint64_t j = (t * S::VPT + w) * 256 + threadIdx.x;
            if (j >= n_vec) break;
            uint32_t a[PER][C::DW];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint64_t o = (j * PER + u) * C::K;
                const uint32_t* src = lds + uint32_t((o >> 5) - 2 * q0);
                uint32_t raw[C::PW + 1];
#pragma unroll
                for (int q = 0; q <= C::PW; ++q) raw[q] = src[q];
                build_codeword<R>(raw, uint32_t(o & 31u), a[u]);
            }
            store_vector<R>(a, j, n_cw, out16, cw_out);
        }
    }
}

// Workgroup caps of one launch; larger inputs loop.  The staged kernel's
// prefetch needs a few tiles per workgroup: 2^15 workgroups (2 tiles each for
// 2^26 codewords of r = 6) measured faster than one tile per workgroup, and
// than 2^12-2^14 workgroups.
constexpr uint64_t kEncodeMaxBlocks = 32768;
constexpr uint64_t kEncodeDirectMaxBlocks = 65536;

template <int R>
static hipError_t launch_encode_r(const void* stream_in, uint64_t n_cw, uint64_t* out, hipStream_t stream)
{
    using C = Code<R>;
    const uint64_t stream_q = (n_cw * C::K + 63) / 64;
    const uint32_t out16 = (reinterpret_cast<uintptr_t>(out) & 15u) == 0 ? 1u : 0u;
    if constexpr (R >= 6) {
        using T = EncShape<R>;
        uint64_t blocks = (n_cw + T::CW - 1) / T::CW;
        if (blocks > kEncodeMaxBlocks) blocks = kEncodeMaxBlocks;
        if (blocks == 0) return hipSuccess;
        hipLaunchKernelGGL((encode_staged_kernel<R>), dim3(uint32_t(blocks)), dim3(256), 0, stream,
                           static_cast<const uint64_t*>(stream_in), stream_q, n_cw, out, out16);
    } else {
        constexpr uint64_t per = EncShape<R>::PER;
        uint64_t blocks = ((n_cw + per - 1) / per + 255) / 256;
        if (blocks > kEncodeDirectMaxBlocks) blocks = kEncodeDirectMaxBlocks;
        if (blocks == 0) return hipSuccess;
        hipLaunchKernelGGL((encode_plain_kernel<R>), dim3(uint32_t(blocks)), dim3(256), 0, stream,
                           static_cast<const uint32_t*>(stream_in), 2 * stream_q, n_cw, out, out16);
    }
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

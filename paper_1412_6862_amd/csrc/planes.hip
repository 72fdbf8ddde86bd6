// Bit-plane input layout: the index-set clustering of Sec. III.A (Fig. 4)
// taken to single positions.  Plane p-1 holds position p of every codeword
// (codeword i at bit i%64 of 64-bit word i/64), so a codeword occupies n bits
// of input instead of one or two padded 64-bit words, and a lane that loads
// one 32-bit word of each plane holds 32 codewords bit-sliced:
//   checksum bit j of all 32 codewords = XOR of the planes in index set I_j
//   (Algorithm 1 applied to 32 codewords at once);
//   correction mask of position p = AND over j of (s_j or ~s_j as bit j of p
//   says), built from two half-width minterm tables;
//   message bit m of the 32 codewords = corrected plane of its position.
// A 32x32 bit transpose turns message planes into per-codeword messages,
// which are packed into the same dense stream as the plain decode and
// written through LDS with coalesced stores; errpos bytes come from the
// syndrome planes with a multiply-spread.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming.h"
#include "hamming_device.h"
#include "tile.h"

namespace hm {
namespace {

constexpr bool is_pow2(int p) { return (p & (p - 1)) == 0; }

// Message positions in order (1-based positions, powers of two skipped).
template <int R>
struct MsgPositions {
    int v[Code<R>::K];
    constexpr MsgPositions() : v()
    {
        int c = 0;
        for (int p = 1; p <= Code<R>::N; ++p)
            if (!is_pow2(p)) v[c++] = p;
    }
};

template <int R>
struct PlaneShape {
    static constexpr int N = Code<R>::N;
    static constexpr int K = Code<R>::K;
    static constexpr int NB = (K + 31) / 32;                     // 32-row transpose blocks
    static constexpr int WAVES = R == 7 ? 1 : (R == 6 ? 2 : 4);   // waves per block (LDS bound)
    static constexpr int MSG_DW = 64 * K;                         // staged message dwords per wave
    static constexpr int EP_DW = 64 * 8;                          // staged errpos dwords per wave
    static constexpr int LDS_DW = MSG_DW + EP_DW;
};

// In-place transpose of a 32x32 bit matrix: bit c of row i moves to bit i of
// row c.  Stage j swaps, for rows k and k+j (bit j of k clear), the columns
// with bit j set in row k against the columns with bit j clear in row k+j.
__device__ __forceinline__ void transpose32(uint32_t* A)
{
    constexpr uint32_t masks[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int st = 0; st < 5; ++st) {
        const int j = 16 >> st;
        const uint32_t m = masks[st];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if (k & j) continue;
            const uint32_t t = ((A[k] >> j) ^ A[k + j]) & m;
            A[k + j] ^= t;
            A[k] ^= t << j;
        }
    }
}

template <int R>
__global__ __launch_bounds__(64 * PlaneShape<R>::WAVES) void decode_planes_kernel(
    const uint32_t* __restrict__ planes, uint64_t plane_dwords, uint64_t n_cw, uint32_t* __restrict__ data,
    uint64_t data_dwords, uint8_t* __restrict__ errpos, uint32_t flags)
{
    using S = PlaneShape<R>;
    constexpr int N = S::N, K = S::K, NB = S::NB;
    __shared__ uint32_t lds[S::WAVES * S::LDS_DW];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t wave = uint64_t(blockIdx.x) * S::WAVES + wib;
    const uint64_t groups = (n_cw + 31) / 32;
    if (wave * 64 >= groups) return;
    const uint64_t g = wave * 64 + lane;
    uint32_t* Mw = lds + wib * S::LDS_DW;
    uint32_t* Ew = Mw + S::MSG_DW;

    // a1: one dword of every plane = 32 codewords, bit-sliced
    uint32_t P[N];
    if (g < groups) {
        const uint32_t* src = planes + g;
#pragma unroll
        for (int p = 0; p < N; ++p) P[p] = __builtin_nontemporal_load(src + uint64_t(p) * plane_dwords);
        if (g == groups - 1 && (n_cw & 31u)) {
            const uint32_t valid = (1u << (n_cw & 31u)) - 1u;
#pragma unroll
            for (int p = 0; p < N; ++p) P[p] &= valid;
        }
    } else {
#pragma unroll
        for (int p = 0; p < N; ++p) P[p] = 0;
    }

    // a2: checksum planes
    uint32_t s[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        uint32_t x = 0;
#pragma unroll
        for (int p = 1; p <= N; ++p)
            if ((p >> j) & 1) x ^= P[p - 1];
        s[j] = x;
    }

    // a3: errpos bytes, codeword c = byte c%4 of dword c/4
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        uint32_t e = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) e |= ((((s[j] >> (4 * d)) & 0xFu) * 0x00204081u) & 0x01010101u) << j;
        Ew[lane * 8 + d] = e;
    }

    // a4: correction masks from minterms of the low and high checksum planes
    constexpr int H = R / 2, HH = R - H;
    uint32_t lo[1 << H], hi[1 << HH];
    lo[0] = ~s[0];
    lo[1] = s[0];
#pragma unroll
    for (int j = 1; j < H; ++j) {
#pragma unroll
        for (int a = (1 << j) - 1; a >= 0; --a) {
            lo[a | (1 << j)] = lo[a] & s[j];
            lo[a] &= ~s[j];
        }
    }
    hi[0] = ~s[H];
    hi[1] = s[H];
#pragma unroll
    for (int j = 1; j < HH; ++j) {
#pragma unroll
        for (int a = (1 << j) - 1; a >= 0; --a) {
            hi[a | (1 << j)] = hi[a] & s[H + j];
            hi[a] &= ~s[H + j];
        }
    }

    // a5: corrected message planes, padded to whole transpose blocks
    constexpr MsgPositions<R> kPos{};
    uint32_t X[NB * 32];
#pragma unroll
    for (int m = 0; m < NB * 32; ++m) {
        if (m < K) {
            constexpr int kLoMask = (1 << H) - 1;
            const int p = kPos.v[m];
            X[m] = P[p - 1] ^ (lo[p & kLoMask] & hi[p >> H]);
        } else {
            X[m] = 0;
        }
    }
    if constexpr (K == 4) {
        // Hamming(7,4): output dword w holds codewords 8w..8w+7, four bits
        // each; spread byte w of message plane m to every fourth bit
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            uint32_t out = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                uint32_t x = (X[m] >> (8 * w)) & 0xFFu;
                x = (x | (x << 12)) & 0x000F000Fu;
                x = (x | (x << 6)) & 0x03030303u;
                x = (x | (x << 3)) & 0x11111111u;
                out |= x << m;
            }
            Mw[lane * K + w] = out;
        }
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) transpose32(X + 32 * b);

        // a6: codeword c's message bits [32b, 32b+32) are X[32b + c]; append
        // them in stream order (c*K + 32b) and emit each completed dword
        uint32_t acc = 0;
        int filled = 0, wout = 0;
#pragma unroll
        for (int c = 0; c < 32; ++c) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const uint32_t v = X[32 * b + c];
                const int len = (K - 32 * b) < 32 ? (K - 32 * b) : 32;
                acc |= filled ? (v << filled) : v;
                if (filled + len >= 32) {
                    Mw[lane * K + wout] = acc;
                    ++wout;
                    acc = filled ? (v >> (32 - filled)) : 0u;
                    filled = filled + len - 32;
                } else {
                    filled += len;
                }
            }
        }
    }
    wave_sync();

    // coalesced stores of the wave's message dwords and errpos bytes
    const uint64_t dw0 = wave * 64 * K;
    const bool out16 = (flags & kFlagOut16) != 0;
    for (uint32_t v = lane; v < 16u * K; v += 64) {
        const uint64_t at = dw0 + 4ull * v;
        if (at >= data_dwords) break;
        const u32x4 x = *reinterpret_cast<const u32x4*>(Mw + 4 * v);
        if (out16 && at + 4 <= data_dwords) {
            __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(data + at));
        } else {
            for (int q = 0; q < 4 && at + q < data_dwords; ++q) data[at + q] = x[q];
        }
    }
    if (errpos) {
        const uint64_t e0 = wave * 2048;
        const bool ev = (flags & kFlagEpVec) != 0;
        for (uint32_t v = lane; v < 128; v += 64) {
            const uint64_t at = e0 + 16ull * v;
            if (at >= n_cw) break;
            const u32x4 x = *reinterpret_cast<const u32x4*>(Ew + 4 * v);
            if (ev && at + 16 <= n_cw) {
                __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(errpos + at));
            } else {
                for (int q = 0; q < 16 && at + q < n_cw; ++q) errpos[at + q] = uint8_t(x[q / 4] >> (8 * (q % 4)));
            }
        }
    }
}

// Natural layout -> planes: one lane transposes 32 codewords, one storage
// dword at a time.
template <int R>
__global__ __launch_bounds__(256) void to_planes_kernel(const uint32_t* __restrict__ cw, uint64_t n_cw,
                                                        uint32_t* __restrict__ planes, uint64_t plane_dwords)
{
    constexpr int N = Code<R>::N, DW = Code<R>::DW;
    const uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t groups = (n_cw + 31) / 32;
    if (g >= groups) return;
#pragma unroll
    for (int d = 0; d < DW; ++d) {
        if (32 * d >= N) break;
        uint32_t A[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            const uint64_t i = 32 * g + c;
            A[c] = i < n_cw ? cw[i * DW + d] : 0u;
        }
        transpose32(A);
#pragma unroll
        for (int b = 0; b < 32; ++b)
            if (32 * d + b < N) planes[uint64_t(32 * d + b) * plane_dwords + g] = A[b];
    }
}

template <int R>
void launch_planes(const uint64_t* planes, uint64_t plane_words, uint64_t n_cw, void* data, uint8_t* errpos,
                   uint32_t flags, hipStream_t stream)
{
    using S = PlaneShape<R>;
    const uint64_t waves = ((n_cw + 31) / 32 + 63) / 64;
    const uint64_t blocks = (waves + S::WAVES - 1) / S::WAVES;
    const uint64_t data_dwords = hamming_data_bytes(n_cw, R) / 4;
    hipLaunchKernelGGL(decode_planes_kernel<R>, dim3(uint32_t(blocks)), dim3(64 * S::WAVES), 0, stream,
                       reinterpret_cast<const uint32_t*>(planes), plane_words * 2, n_cw,
                       static_cast<uint32_t*>(data), data_dwords, errpos, flags);
}

template <int R>
void launch_to_planes(const uint64_t* cw, uint64_t n_cw, uint64_t* planes, uint64_t plane_words, hipStream_t stream)
{
    const uint64_t groups = (n_cw + 31) / 32;
    hipLaunchKernelGGL(to_planes_kernel<R>, dim3(uint32_t((groups + 255) / 256)), dim3(256), 0, stream,
                       reinterpret_cast<const uint32_t*>(cw), n_cw, reinterpret_cast<uint32_t*>(planes),
                       plane_words * 2);
}

}  // namespace
}  // namespace hm

extern "C" {

// One launch covers at most this many codewords: both plane kernels then
// stay within a dispatch's 32-bit work-item count (one lane per 32 codewords).
constexpr uint64_t kPlanesMaxCodewords = (uint64_t(1) << 37) - (uint64_t(1) << 13);

uint64_t hamming_planes_words(uint64_t n_cw, int r)
{
    if (r < 3 || r > 7 || n_cw > HAMMING_MAX_CODEWORDS) return 0;
    return uint64_t((1 << r) - 1) * ((n_cw + 63) / 64);
}

int hamming_decode_planes(const uint64_t* planes, uint64_t plane_words, uint64_t n_cw, int r, void* data_out,
                          uint8_t* errpos_out, hipStream_t stream)
{
    if (r < 3 || r > 7) return HAMMING_EINVAL;
    if (n_cw > kPlanesMaxCodewords) return HAMMING_ERANGE;
    if (n_cw == 0) return HAMMING_OK;
    if (!planes || !data_out) return HAMMING_EINVAL;
    if (plane_words < (n_cw + 63) / 64) return HAMMING_ERANGE;
    if ((reinterpret_cast<uintptr_t>(planes) & 7u) || (reinterpret_cast<uintptr_t>(data_out) & 7u))
        return HAMMING_EALIGN;
    uint32_t flags = 0;
    if (!(reinterpret_cast<uintptr_t>(data_out) & 15u)) flags |= hm::kFlagOut16;
    if (errpos_out && !(reinterpret_cast<uintptr_t>(errpos_out) & 15u)) flags |= hm::kFlagEpVec;
    switch (r) {
    case 3: hm::launch_planes<3>(planes, plane_words, n_cw, data_out, errpos_out, flags, stream); break;
    case 4: hm::launch_planes<4>(planes, plane_words, n_cw, data_out, errpos_out, flags, stream); break;
    case 5: hm::launch_planes<5>(planes, plane_words, n_cw, data_out, errpos_out, flags, stream); break;
    case 6: hm::launch_planes<6>(planes, plane_words, n_cw, data_out, errpos_out, flags, stream); break;
    default: hm::launch_planes<7>(planes, plane_words, n_cw, data_out, errpos_out, flags, stream); break;
    }
    return hipGetLastError() == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

int hamming_to_planes(const uint64_t* codewords, uint64_t n_cw, int r, uint64_t* planes, uint64_t plane_words,
                      hipStream_t stream)
{
    if (r < 3 || r > 7) return HAMMING_EINVAL;
    if (n_cw > kPlanesMaxCodewords) return HAMMING_ERANGE;
    if (n_cw == 0) return HAMMING_OK;
    if (!codewords || !planes) return HAMMING_EINVAL;
    if (plane_words < (n_cw + 63) / 64) return HAMMING_ERANGE;
    if ((reinterpret_cast<uintptr_t>(codewords) & 7u) || (reinterpret_cast<uintptr_t>(planes) & 7u))
        return HAMMING_EALIGN;
    switch (r) {
    case 3: hm::launch_to_planes<3>(codewords, n_cw, planes, plane_words, stream); break;
    case 4: hm::launch_to_planes<4>(codewords, n_cw, planes, plane_words, stream); break;
    case 5: hm::launch_to_planes<5>(codewords, n_cw, planes, plane_words, stream); break;
    case 6: hm::launch_to_planes<6>(codewords, n_cw, planes, plane_words, stream); break;
    default: hm::launch_to_planes<7>(codewords, n_cw, planes, plane_words, stream); break;
    }
    return hipGetLastError() == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

}  // extern "C"

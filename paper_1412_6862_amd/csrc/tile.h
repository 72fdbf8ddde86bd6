// Wave-tile decode shared by the plain and the batched kernels.
//
// A wave owns a tile of 64*U consecutive codewords of one packet; lane L
// decodes the U consecutive codewords [64*U*t + U*L, +U) of tile t, so its
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
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming_device.h"
#include "launch.h"

namespace hm {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// The same 16-byte vector at 8-byte alignment: packets and message streams
// start at any 64-bit word, and a global dwordx4 access needs only dword
// alignment, so every full tile takes the vector path.
typedef uint32_t u32x4a8 __attribute__((ext_vector_type(4), aligned(8)));

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
    static constexpr int NV = U * C::DW / 4;        // 16-byte input vectors per lane
    static constexpr int LDS_IN_DW = NV * 64 * 4;   // input transpose staging
    static constexpr int LDS_OUT_DW = 2 * B;        // merge staging
    static constexpr int LDS_DW = LDS_IN_DW > LDS_OUT_DW ? LDS_IN_DW : LDS_OUT_DW;  // per wave
    static_assert(LDS_DW % 4 == 0, "per-wave LDS must be whole 16-byte vectors");
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

// Part i of `total` units split into `parts` near-equal contiguous ranges:
// [split_range(total, i, parts), split_range(total, i + 1, parts)).
__device__ __forceinline__ uint64_t split_range(uint64_t total, uint64_t i, uint64_t parts)
{
    return (total / parts) * i + ((total % parts) * i) / parts;
}

// Workgroups are handed to the 8 XCDs of gfx950 round-robin (block b runs on
// XCD b % 8), and each XCD has its own L2 and address-translation caches.
// xcd_block renumbers blocks in groups of 8*chunk: inside a group, XCD x takes
// the `chunk` consecutive logical blocks x*chunk .. x*chunk+chunk-1, so each
// XCD streams through its own slice of every group instead of every XCD
// touching every page, while all XCDs still advance through memory together.
// chunk = 1 keeps the hardware order.  A bijection on [0, nblocks); a final
// partial group keeps the hardware order.
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblocks, uint32_t chunk)
{
    const uint32_t group = kXcds * chunk;
    const uint32_t g = b / group;
    if (chunk <= 1 || (g + 1) * uint64_t(group) > nblocks) return b;
    const uint32_t j = b - g * group;
    return g * group + (j % kXcds) * chunk + j / kXcds;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Input registers of one lane for one tile: the lane's 16-byte vectors
// v*64 + lane of the tile (consecutive lanes read consecutive vectors);
// finish_tile transposes them through LDS to the lane's own U codewords.
template <int R, int U>
struct TileIn {
    uint32_t in[U * Code<R>::DW];
};

// Issue the loads of tile `tile`.  In the ragged last tile of a packet the
// vectors past its last codeword read as zero (a vector holding only the
// last word is read as one 8-byte load), so every access stays inside the
// packet and the tile still goes through the coalesced transpose.
template <int R, int U>
__device__ __forceinline__ void load_tile(const uint64_t* __restrict__ cw, uint64_t n_cw, uint64_t tile,
                                          uint32_t lane, TileIn<R, U>& t)
{
    using C = Code<R>;
    using T = TileShape<R, U>;
    const uint64_t w0 = tile * T::CW * C::WPC;          // first input word of the tile
    const u32x4a8* src = reinterpret_cast<const u32x4a8*>(cw + w0) + lane;
    if ((tile + 1) * T::CW <= n_cw) {
#pragma unroll
        for (int v = 0; v < T::NV; ++v) {
            const u32x4 x = __builtin_nontemporal_load(src + 64 * v);
            t.in[4 * v + 0] = x.x;
            t.in[4 * v + 1] = x.y;
            t.in[4 * v + 2] = x.z;
            t.in[4 * v + 3] = x.w;
        }
    } else {
        const uint64_t rem = n_cw * C::WPC - w0;          // input words left in the packet, < the tile's
#pragma unroll
        for (int v = 0; v < T::NV; ++v) {
            const uint64_t w = 2 * (64u * uint64_t(v) + lane);   // first word of this lane's vector v
            u32x4 x = {0u, 0u, 0u, 0u};
            if (w + 1 < rem) {
                x = __builtin_nontemporal_load(src + 64 * v);
            } else if (w < rem) {
                const uint64_t y = cw[w0 + w];
                x.x = uint32_t(y);
                x.y = uint32_t(y >> 32);
            }
            t.in[4 * v + 0] = x.x;
            t.in[4 * v + 1] = x.y;
            t.in[4 * v + 2] = x.z;
            t.in[4 * v + 3] = x.w;
        }
    }
}

// Issue the loads of a tile known to be full (the vector form of load_tile
// with no checks).
template <int R, int U>
__device__ __forceinline__ void load_full_tile(const uint64_t* __restrict__ cw, uint64_t tile, uint32_t lane,
                                               TileIn<R, U>& t)
{
    using C = Code<R>;
    using T = TileShape<R, U>;
    const u32x4a8* src = reinterpret_cast<const u32x4a8*>(cw + tile * T::CW * C::WPC) + lane;
#pragma unroll
    for (int v = 0; v < T::NV; ++v) {
        const u32x4 x = __builtin_nontemporal_load(src + 64 * v);
        t.in[4 * v + 0] = x.x;
        t.in[4 * v + 1] = x.y;
        t.in[4 * v + 2] = x.z;
        t.in[4 * v + 3] = x.w;
    }
}

// Decode the loaded codewords of tile `tile` and write its outputs.
template <int R, int U>
__device__ __forceinline__ void finish_tile(TileIn<R, U>& tin, uint64_t n_cw, uint64_t tile, uint32_t lane,
                                            uint64_t* __restrict__ data, uint64_t data_words,
                                            uint8_t* __restrict__ errpos, uint32_t* lds, uint32_t flags)
{
    using T = TileShape<R, U>;
    const uint64_t c0 = tile * T::CW + uint64_t(lane) * U;
    const bool full = (tile + 1) * T::CW <= n_cw;
    auto& in = tin.in;

    // ---- transpose coalesced vectors to lane-contiguous codewords ----------
    // Vector j is kept in LDS slot j ^ ((j / NV) % NV): the low bits are
    // rotated per block of NV vectors, so the lane-strided reads below hit
    // different banks while the lane-consecutive writes stay conflict free.
    // For NV <= 8 (NV^2 divides 64) the rotation of vector 64v + lane does
    // not depend on v, so one lane address serves every write.
    {
        u32x4* lv = reinterpret_cast<u32x4*>(lds);
        constexpr uint32_t NV = T::NV;
        const uint32_t wslot = lane ^ ((lane / NV) % NV);
#pragma unroll
        for (int v = 0; v < T::NV; ++v) {
            u32x4 x;
            x.x = in[4 * v + 0];
            x.y = in[4 * v + 1];
            x.z = in[4 * v + 2];
            x.w = in[4 * v + 3];
            const uint32_t j = 64u * v + lane;
            if constexpr (NV <= 8)
                lv[64u * v + wslot] = x;
            else
                lv[j ^ ((j / NV) % NV)] = x;
        }
        wave_sync();
#pragma unroll
        for (int v = 0; v < T::NV; ++v) {
            // slot of vector lane*NV + v: lane*NV + (v ^ (lane % NV))
            const u32x4 x = lv[lane * NV + (uint32_t(v) ^ (lane % NV))];
            in[4 * v + 0] = x.x;
            in[4 * v + 1] = x.y;
            in[4 * v + 2] = x.z;
            in[4 * v + 3] = x.w;
        }
        wave_sync();
    }

    // ---- decode, merge within the lane ------------------------------------
    constexpr int CHA = T::CHW + 2;
    uint32_t chunk[CHA];
#pragma unroll
    for (int i = 0; i < CHA; ++i) chunk[i] = 0;
    uint32_t s[U];
    decode_lane_codewords<R, U, 0>(in, chunk, s);

    // ---- error positions ---------------------------------------------------
    // lanes whose U codewords all exist store them at once (every lane of a
    // full tile; in the ragged tile all but the lanes past its end)
    if (errpos) {
        if ((flags & kFlagEpVec) && c0 + U <= n_cw) {
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
    const uint32_t bitpos = __umul24(lane, uint32_t(T::B));     // lane < 64, B < 2^11
    const uint32_t first = (bitpos + 31u) >> 5;
    const uint32_t a = (first << 5) - bitpos;
    const uint32_t n_own = ((bitpos + T::B + 31u) >> 5) - first;
    // a chunk of B bits holds floor(B/32) or ceil(B/32) dword starts, so only
    // the last candidate dword is owned by some lanes and not others
#pragma unroll
    for (int i = 0; i < T::CHW; ++i) {
        const uint32_t v = (T::BR == 0) ? e[i] : __builtin_amdgcn_alignbit(e[i + 1], e[i], a);
        if (T::BR == 0 || i < T::CHW - 1 || uint32_t(i) < n_own) lds[first + i] = v;
    }
    wave_sync();

    // ---- LDS -> global by consecutive lanes ---------------------------------
    const uint64_t w0 = tile * uint64_t(T::WORDS);
    if (full) {
        // whole tile: T::WORDS is even (U is even)
        const u32x4* l4 = reinterpret_cast<const u32x4*>(lds);
        u32x4a8* dst = reinterpret_cast<u32x4a8*>(data + w0);
#pragma unroll
        for (int q = 0; q < (T::WORDS / 2 + 63) / 64; ++q) {
            const uint32_t j = lane + 64u * q;
            if ((q + 1) * 64 <= T::WORDS / 2 || j < uint32_t(T::WORDS / 2)) __builtin_nontemporal_store(l4[j], dst + j);
        }
    } else {
        // ragged tile: whole 16-byte vectors below the stream's end, then at
        // most one last 64-bit word
        const uint64_t nw = (data_words - w0 < uint64_t(T::WORDS)) ? (data_words - w0) : uint64_t(T::WORDS);
        const u32x4* l4 = reinterpret_cast<const u32x4*>(lds);
        u32x4a8* dst = reinterpret_cast<u32x4a8*>(data + w0);
#pragma unroll
        for (int q = 0; q < (T::WORDS / 2 + 63) / 64; ++q) {
            const uint32_t j = lane + 64u * q;
            if (2 * uint64_t(j) + 1 < nw) __builtin_nontemporal_store(l4[j], dst + j);
        }
        if ((nw & 1) && lane == 0) {
            const uint2 v = reinterpret_cast<const uint2*>(lds)[nw - 1];
            __builtin_nontemporal_store(uint64_t(v.x) | (uint64_t(v.y) << 32), data + w0 + nw - 1);
        }
    }
    wave_sync();
}

template <int R, int U>
__device__ __forceinline__ void decode_tile(const uint64_t* __restrict__ cw, uint64_t n_cw, uint64_t tile,
                                            uint32_t lane, uint64_t* __restrict__ data, uint64_t data_words,
                                            uint8_t* __restrict__ errpos, uint32_t* lds, uint32_t flags)
{
    TileIn<R, U> t;
    load_tile<R, U>(cw, n_cw, tile, lane, t);
    finish_tile<R, U>(t, n_cw, tile, lane, data, data_words, errpos, lds, flags);
}

// Lane index within the wave, made opaque to the optimiser: lane-derived
// addresses are then computed where a run starts instead of being hoisted
// out of the loops around it (a batch kernel holds a run for every r, and
// values hoisted for all of them at once would exceed its register budget).
__device__ __forceinline__ uint32_t run_lane()
{
    uint32_t l = threadIdx.x & 63u;
    asm volatile("" : "+v"(l));
    return l;
}

// Tiles t, t + stride, ... below t_end of one packet.  The full ones run as a
// two-stage pipeline: the wave issues the loads of its next full tile before
// it decodes the current one, so two tiles of loads are in flight while it
// computes.  Tiles past the last full one (at most the ragged tile) go
// through the checked path.
template <int R, int U>
__device__ __forceinline__ void decode_run(const uint64_t* __restrict__ cw, uint64_t n_cw, uint64_t t,
                                           uint64_t t_end, uint64_t stride, uint64_t* __restrict__ data,
                                           uint64_t data_words, uint8_t* __restrict__ errpos, uint32_t* lds,
                                           uint32_t flags)
{
    using T = TileShape<R, U>;
    const uint32_t lane = run_lane();
    const uint64_t n_full = n_cw / T::CW;
    const uint64_t full_end = t_end < n_full ? t_end : n_full;
    if (t < full_end) {
        TileIn<R, U> cur;
        load_full_tile<R, U>(cw, t, lane, cur);
        for (;;) {
            const uint64_t tn = t + stride;
            if (tn >= full_end) break;
            TileIn<R, U> nxt;
            load_full_tile<R, U>(cw, tn, lane, nxt);    // in flight while `cur` is decoded
            finish_tile<R, U>(cur, n_cw, t, lane, data, data_words, errpos, lds, flags);
            cur = nxt;
            t = tn;
        }
        finish_tile<R, U>(cur, n_cw, t, lane, data, data_words, errpos, lds, flags);
        t += stride;
    }
    for (; t < t_end; t += stride) decode_tile<R, U>(cw, n_cw, t, lane, data, data_words, errpos, lds, flags);
}

}  // namespace hm

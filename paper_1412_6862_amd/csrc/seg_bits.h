// Bit helpers of the segmented-packet kernels (segmented.hip): pure functions
// on 64-bit words, compiled for the device and for the host, so that host
// unit tests can check them against bit-by-bit definitions.
//
// A segment's positions are read in windows of 128: window v holds positions
// 128v .. 128v+127 (position 0 does not exist; it keeps window 0 aligned like
// the others), position 128v + q at bit q of the pair (x0, x1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {

__host__ __device__ inline uint32_t seg_umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Index, within its segment, of the first message bit of window v, and pw =
// 1 when position 128v is a checksum position.  For v >= 1 that can only be
// 128v itself (when v is a power of two), so the window's message bits are
// consecutive from position 128v + pw, whose message index is 128v + pw minus
// the floor(log2 v) + 8 checksum positions below it minus one.  Window 0
// starts at message bit 0.
__host__ __device__ inline uint32_t run_start(uint32_t v, uint32_t& pw)
{
    const uint32_t lv = 31u - uint32_t(__builtin_clz(v | 1u));
    pw = (v & (v - 1u)) == 0u ? 1u : 0u;
    return v == 0 ? 0u : 128u * v + pw - lv - 9u;
}

// 128 bits starting at bit s (0..63) of word a, continuing into b and c.
__host__ __device__ inline void funnel128(uint64_t a, uint64_t b, uint64_t c, uint32_t s, uint64_t& lo,
                                          uint64_t& hi)
{
    lo = (a >> s) | ((b << 1) << (63u - s));
    hi = (b >> s) | ((c << 1) << (63u - s));
}

// Keeps bits 0..top of a window (top = last position of the segment minus
// 128v; any top >= 127 keeps the whole window).
__host__ __device__ inline void mask_top(uint64_t& x0, uint64_t& x1, uint32_t top)
{
    x0 &= ~uint64_t(0) >> (63u - seg_umin(top, 63u));
    x1 &= top < 64u ? uint64_t(0) : (~uint64_t(0) >> (63u - seg_umin(top - 64u, 63u)));
}

// The message positions below 64 (3, 5..7, 9..15, 17..31, 33..63) carry a
// segment's first 57 message bits.  head_message compacts them from a word
// holding positions 1..64 at bits 0..63; head_expand places message bits
// 0..56 at those positions in window 0's layout (position q at bit q).
__host__ __device__ inline uint64_t head_message(uint64_t w)
{
    return ((w >> 2) & 0x1ull) | (((w >> 4) & 0x7ull) << 1) | (((w >> 8) & 0x7Full) << 4) |
           (((w >> 16) & 0x7FFFull) << 11) | (((w >> 32) & 0x7FFFFFFFull) << 26);
}

__host__ __device__ inline uint64_t head_expand(uint64_t m)
{
    return ((m & 0x1ull) << 3) | (((m >> 1) & 0x7ull) << 5) | (((m >> 4) & 0x7Full) << 9) |
           (((m >> 11) & 0x7FFFull) << 17) | (((m >> 26) & 0x7FFFFFFFull) << 33);
}

}  // namespace hm

// Device-side arithmetic of the Hamming decoder for gfx950.
//
// One codeword lives in registers as dwords a[0..DW-1]: position p (1..n) is
// bit (p-1)%32 of dword (p-1)/32.  Everything here is integer GF(2) work on
// 32-bit VALU operations; no step touches memory.
//
// Checksum (Sec. III.C, Algorithm 1).  Checksum bit j is the XOR of the bits
// of index set I_j = {p : bit j of p is 1} (Sec. III.A).  Inside one dword,
// positions 32q+b+1 for the same b share bits 0..4, so for j <= 4 the dwords
// are XOR-folded first and bit j is the parity of (fold & M_j).  Bits 5 and 6
// depend on which dword a bit came from and are taken from explicit
// high/low-bit selections.  Parity is the low bit of a popcount
// (v_bcnt_u32_b32); the parities are gathered by a funnel shift that moves
// each one in as the new top bit of an accumulator (v_alignbit_b32), so bit j
// needs no masking or shifting of its own and stale low bits fall out at the
// end.
//
// Correction (Sec. II, error correction unit): the checksum value s names the
// flipped position; storage bit s-1 is inverted, branch-free, when s != 0.
// For r = 6 and 7, s = 0 inverts the top padding bit instead (bit 63 or
// 127): padding takes no part in the checksum or the extracted message, so
// the no-error case needs no select.
//
// Redundancy removal (Sec. II): the message positions form r-1 runs between
// consecutive powers of two, run j = positions 2^j+1 .. 2^(j+1)-1; each run
// is moved with one bit-field extract and one shift-or.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {

template <int R>
struct Code {
    static constexpr int N = (1 << R) - 1;      // code bits
    static constexpr int K = N - R;             // message bits
    static constexpr int WPC = (R == 7) ? 2 : 1;  // 64-bit storage words per codeword
    static constexpr int DW = 2 * WPC;          // dwords per codeword
    static constexpr int PW = (K + 31) / 32;    // message dwords
};

// Index-set masks over one dword: bit b is set when bit j of (b+1) is 1.
__device__ constexpr uint32_t kSetMask0 = 0x55555555u;
__device__ constexpr uint32_t kSetMask1 = 0x66666666u;
__device__ constexpr uint32_t kSetMask2 = 0x78787878u;
__device__ constexpr uint32_t kSetMask3 = 0x7F807F80u;
__device__ constexpr uint32_t kSetMask4 = 0x7FFF8000u;
constexpr uint32_t kTop = 0x80000000u;
constexpr uint32_t kLow31 = 0x7FFFFFFFu;

__device__ __forceinline__ uint32_t bfe(uint32_t x, int off, int len)
{
    return (x >> off) & ((len >= 32) ? 0xFFFFFFFFu : ((1u << len) - 1u));
}

// acc >> 1 with the parity of x as the new bit 31.  After J pushes, bits
// 32-J .. 31 hold the J parities in push order (first pushed lowest).
__device__ __forceinline__ uint32_t push_parity(uint32_t acc, uint32_t x)
{
    return __builtin_amdgcn_alignbit(uint32_t(__builtin_popcount(x)), acc, 1);
}

// Push checksum bits 0..J-1 of a folded dword (J <= 5).
template <int J>
__device__ __forceinline__ uint32_t push_low_checksum(uint32_t acc, uint32_t f)
{
    acc = push_parity(acc, f & kSetMask0);
    if constexpr (J > 1) acc = push_parity(acc, f & kSetMask1);
    if constexpr (J > 2) acc = push_parity(acc, f & kSetMask2);
    if constexpr (J > 3) acc = push_parity(acc, f & kSetMask3);
    if constexpr (J > 4) acc = push_parity(acc, f & kSetMask4);
    return acc;
}

// Clear the padding bits (storage bits >= n) of a codeword.  For r = 6 the
// checksum and the extraction below read around the one padding bit, so
// nothing is cleared.
template <int R>
__device__ __forceinline__ void mask_padding(uint32_t (&a)[Code<R>::DW])
{
    if constexpr (R <= 5) {
        a[0] &= (1u << Code<R>::N) - 1u;
        a[1] = 0;
    } else if constexpr (R == 7) {
        a[3] &= kLow31;
    }
}

// Checksum value s in [0, n] of a codeword whose padding is clear (for r = 6:
// whatever its padding bit holds).
template <int R>
__device__ __forceinline__ uint32_t checksum(const uint32_t (&a)[Code<R>::DW])
{
    if constexpr (R <= 5) {
        return push_low_checksum<R>(0u, a[0]) >> (32 - R);
    } else if constexpr (R == 6) {
        // bit 31 of the fold is position 32 or 64: outside every set I_0..I_4
        uint32_t acc = push_low_checksum<5>(0u, a[0] ^ a[1]);
        // positions 32..63: bit 31 of dword 0 and bits 0..30 of dword 1
        // (dword 1's bit 31 is padding)
        acc = push_parity(acc, (a[0] & kTop) | (a[1] & kLow31));
        return acc >> 26;
    } else {
        uint32_t acc = push_low_checksum<5>(0u, a[0] ^ a[1] ^ a[2] ^ a[3]);
        // bit 5: positions 32, 33..63, 96, 97..127
        const uint32_t h = a[0] ^ a[2];
        const uint32_t l = a[1] ^ a[3];
        acc = push_parity(acc, (h & kTop) | (l & kLow31));
        // bit 6: positions 64..127
        acc = push_parity(acc, a[2] ^ a[3] ^ (a[1] & kTop));
        return acc >> 25;
    }
}

// Flip storage bit s-1 when s != 0.
template <int R>
__device__ __forceinline__ void correct(uint32_t (&a)[Code<R>::DW], uint32_t s)
{
    if constexpr (R <= 5) {
        a[0] ^= (1u << s) >> 1;
    } else if constexpr (R == 6) {
        const uint32_t t = s - 1u;                        // s = 0: bit 63, padding
        const uint64_t v = uint64_t(1) << (t & 63u);
        a[0] ^= uint32_t(v);
        a[1] ^= uint32_t(v >> 32);
    } else {
        const uint32_t t = s - 1u;                        // s = 0: bit 127, padding
        const uint64_t v = uint64_t(1) << (t & 63u);
        const uint32_t hi = uint32_t(int32_t(t << 25) >> 31);   // all ones when bit 6 of t is set
        a[0] ^= uint32_t(v) & ~hi;
        a[1] ^= uint32_t(v >> 32) & ~hi;
        a[2] ^= uint32_t(v) & hi;
        a[3] ^= uint32_t(v >> 32) & hi;
    }
}

// Message bits of a corrected codeword, LSB first, into p[0..PW-1]; bits at
// or above k are 0.
template <int R>
__device__ __forceinline__ void extract(const uint32_t (&a)[Code<R>::DW], uint32_t (&p)[Code<R>::PW])
{
    const uint32_t lo = a[0];
    // runs 1..4 of dword 0: (storage start bit, length, message offset)
    uint32_t m = bfe(lo, 2, 1);
    if constexpr (R >= 3) m |= bfe(lo, 4, 3) << 1;
    if constexpr (R >= 4) m |= bfe(lo, 8, 7) << 4;
    if constexpr (R >= 5) m |= bfe(lo, 16, 15) << 11;
    if constexpr (R <= 5) {
        p[0] = m;
    } else {
        const uint32_t hi = a[1];              // positions 33..63 (run 5); bit 31 is position 64 or padding
        p[0] = m | (hi << 26);
        p[1] = bfe(hi, 6, 25);
        if constexpr (R == 7) {                // positions 65..127 (run 6)
            p[1] |= a[2] << 25;
            p[2] = (a[2] >> 7) | (a[3] << 25);
            p[3] = (a[3] & kLow31) >> 7;
        }
    }
}

// Inverse of extract for a zero codeword: place message bits at the message
// positions (checksum positions stay 0).
template <int R>
__device__ __forceinline__ void deposit(const uint32_t (&p)[Code<R>::PW], uint32_t (&a)[Code<R>::DW])
{
    uint32_t lo = bfe(p[0], 0, 1) << 2;
    if constexpr (R >= 3) lo |= bfe(p[0], 1, 3) << 4;
    if constexpr (R >= 4) lo |= bfe(p[0], 4, 7) << 8;
    if constexpr (R >= 5) lo |= bfe(p[0], 11, 15) << 16;
    a[0] = lo;
    if constexpr (R <= 5) {
        a[1] = 0;
    } else {
        a[1] = ((p[0] >> 26) | (p[1] << 6)) & kLow31;
        if constexpr (R == 7) {
            a[2] = (p[1] >> 25) | (p[2] << 7);
            a[3] = ((p[2] >> 25) | (p[3] << 7)) & kLow31;
        }
    }
}

// Set checksum position 2^j for every set bit j of s.
template <int R>
__device__ __forceinline__ void set_checksum_bits(uint32_t (&a)[Code<R>::DW], uint32_t s)
{
    a[0] |= (s & 1u) | ((s & 2u)) | (((s >> 2) & 1u) << 3) | (((s >> 3) & 1u) << 7) |
            (((s >> 4) & 1u) << 15);
    if constexpr (R >= 6) a[0] |= ((s >> 5) & 1u) << 31;
    if constexpr (R == 7) a[1] |= ((s >> 6) & 1u) << 31;
}

}  // namespace hm

// Segmented packets (Sec. II, Fig. 1): a packet of M message bytes travels
// as t shortened Hamming segments H_1..H_t laid end to end as one bit
// string; each segment is checked and corrected on its own and the recovered
// message segments are merged back into the M-byte packet.  The checksum of a
// segment is the XOR over its index sets (Sec. III.A, III.C, Algorithm 1).
//
// A group of threads per packet (part of a wave, a wave or a workgroup): the
// 128-position windows of all segments form one flat list dealt to the
// threads.  Decoding, a thread reads each of its windows once from HBM (an
// unaligned three-word span), folds it into its partial syndrome of the
// segment and ORs the window's message bits (one run of consecutive message
// indices per window) into the packet's message buffer in LDS; the segment
// owners then finish the syndromes and flip the one message bit a
// correctable error hits, and the buffer is stored.  Encoding runs the same
// walk the other way: a thread reads the message run of each window, places
// it at the window's positions, folds it into the partial syndrome and ORs it
// into the packet's encoded buffer in LDS; the owners set checksum position
// 2^j to bit j of the syndrome.  Segment offsets are closed-form (message
// sizes take two values), so no lookup table is read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "hamming.h"
#include "launch.h"
#include "seg_bits.h"
#include "tile.h"

using hm::funnel128;
using hm::head_expand;
using hm::head_message;
using hm::mask_top;
using hm::run_start;
using hm::u32x4;
using hm::u32x4a8;
using hm::wave_sync;

namespace {

constexpr uint32_t kSegWaves = 4;                          // waves per block

// Encoded words of the longest packet of at most max_msg_bytes message
// bytes, plus a word in front (stream bit -1, where the first window of the
// packet starts) and two behind (a window ORed in at a bit offset touches
// three words).
__host__ __device__ inline uint32_t enc_slice_words(uint32_t max_msg_bytes)
{
    return (8u * max_msg_bytes + 16u * HAMMING_SEG_MAX_T + 63u) / 64u + 3u;
}

// Message words of the longest packet plus three (a message run ORed in at a
// bit offset touches up to three words) plus one (the buffer is cleared in
// pairs of words).
__host__ __device__ inline uint32_t msg_slice_words(uint32_t max_msg_bytes)
{
    return (max_msg_bytes + 7u) / 8u + 4u;
}

// Checksum bits of a shortened segment with k >= 1 message bits: the
// smallest r >= 2 with 2^r - 1 - r >= k.  With b the bit length of k, r is b,
// or b + 1 when 2^b - 1 - b < k (2^(b-1) - b < k always rules out b - 1).
__host__ __device__ inline uint32_t seg_checksum_bits(uint32_t k)
{
    const uint32_t b = 32u - uint32_t(__builtin_clz(k));
    const uint32_t r = b + (((1u << b) - 1u - b) < k ? 1u : 0u);
    return r < 2 ? 2 : r;
}

// Segment layout of one packet in closed form.  The first `rem` segments
// carry q+1 message bits and nA positions, the others q bits and nB
// positions, so every offset is a product and a min.  vA and vB count the
// 128-position windows of a segment (window v = positions 128v..128v+127,
// position 0 included so that window 0 is aligned like the others).
struct Layout {
    uint32_t t, q, rem, nA, nB, vA, vB, total;

    __device__ uint32_t K(uint32_t i) const { return i * q + min(i, rem); }            // first message bit
    __device__ uint32_t o(uint32_t i) const { return i * nB + min(i, rem) * (nA - nB); }  // first stream bit
    __device__ uint32_t n(uint32_t i) const { return i < rem ? nA : nB; }
    __device__ uint32_t windows() const { return rem * vA + (t - rem) * vB; }
};

// Validates the packet shape; returns false for one this launch cannot take.
__device__ __forceinline__ bool make_layout(uint32_t msg_bytes, uint32_t t, uint32_t max_msg_bytes, Layout& L)
{
    if (t < 1 || t > HAMMING_SEG_MAX_T || msg_bytes < 1 || msg_bytes > max_msg_bytes || 8u * msg_bytes < t) return false;
    const uint32_t bits = 8u * msg_bytes;
    L.t = t;
    L.q = bits / t;
    L.rem = bits % t;
    if (L.q + (L.rem ? 1u : 0u) > HAMMING_SEG_MAX_K) return false;
    L.nA = L.q + 1 + seg_checksum_bits(L.q + 1);
    L.nB = L.q + seg_checksum_bits(L.q);
    L.vA = L.nA / 128 + 1;
    L.vB = L.nB / 128 + 1;
    L.total = L.o(t);
    return true;
}

// A thread's position in the flat list of windows: segment i, window v of
// it (nv windows), and the segment's first stream bit, positions and first
// message bit.
struct WindowWalk {
    uint32_t i, v, nv, o, n, K;

    __device__ WindowWalk(const Layout& Lo, uint32_t first)
        : i(0), v(first), nv(Lo.rem > 0 ? Lo.vA : Lo.vB), o(0), n(Lo.n(0)), K(0) {}

    // Moves forward to the segment holding window v (a window past the
    // packet's last one stays in the last segment; it is never used).
    __device__ void settle(const Layout& Lo)
    {
        while (v >= nv && i + 1 < Lo.t) {
            v -= nv;
            ++i;
            nv = i < Lo.rem ? Lo.vA : Lo.vB;
            o = Lo.o(i);
            n = Lo.n(i);
            K = Lo.K(i);
        }
    }
};

// ORs 128 bits into a word array at word bq, bit bs (three LDS atomics:
// neighbouring threads' runs share the boundary words).
__device__ __forceinline__ void or128(uint64_t* W, uint32_t bq, uint32_t bs, uint64_t x0, uint64_t x1)
{
    atomicOr(reinterpret_cast<unsigned long long*>(&W[bq]), x0 << bs);
    atomicOr(reinterpret_cast<unsigned long long*>(&W[bq + 1]), ((x0 >> 1) >> (63u - bs)) | (x1 << bs));
    atomicOr(reinterpret_cast<unsigned long long*>(&W[bq + 2]), (x1 >> 1) >> (63u - bs));
}

// Folds window v (bit q of (x0, x1) = position 128v + q) into a partial
// syndrome: bits 0..5 of a position are those of q mod 64 (the XOR of the
// halves), bit 6 says which half, bits 7 and up are those of v.
__device__ __forceinline__ void fold_window(uint64_t x0, uint64_t x1, uint32_t v, uint64_t& xacc, uint32_t& hacc)
{
    const uint64_t f = x0 ^ x1;
    xacc ^= f;
    hacc ^= ((uint32_t(__popcll(x1)) & 1u) << 6) ^ ((__popcll(f) & 1u) ? 128u * v : 0u);
}

// Syndrome of a segment from the XOR X of its 64-position halves and the
// high part H: bits 0..4 of a position are shared by bits q and q+32 of a
// half, so those five parities are taken on the XOR of its 32-bit halves; bit
// 5 is the parity of the upper 32 bits.
__device__ __forceinline__ uint32_t fold_syndrome(uint64_t x, uint32_t h)
{
    const uint32_t hi = uint32_t(x >> 32), f = uint32_t(x) ^ hi;
    uint32_t v = h;
    v ^= __popc(f & 0xAAAAAAAAu) & 1u;
    v ^= (__popc(f & 0xCCCCCCCCu) & 1u) << 1;
    v ^= (__popc(f & 0xF0F0F0F0u) & 1u) << 2;
    v ^= (__popc(f & 0xFF00FF00u) & 1u) << 3;
    v ^= (__popc(f & 0xFFFF0000u) & 1u) << 4;
    v ^= (__popc(hi) & 1u) << 5;
    return v;
}

// Adds a thread's partial syndrome of segment i to the segment's accumulators.
// Threads whose windows cancelled (or that had none) skip the LDS atomics,
// which all threads of a segment aim at the same two addresses.
__device__ __forceinline__ void flush_partial(uint64_t* X, uint32_t* H, uint32_t i, uint64_t x, uint32_t h)
{
    if (x | h) {
        atomicXor(reinterpret_cast<unsigned long long*>(&X[i]), x);
        atomicXor(&H[i], h);
    }
}

// Barrier of the threads that work on one packet: part of a wave or one wave
// (the wave runs in lockstep), or the workgroup.
template <uint32_t GROUP>
__device__ __forceinline__ void group_sync()
{
    if constexpr (GROUP <= 64) {
        wave_sync();
    } else {
        __syncthreads();
    }
}

// Decoding pass over the windows of a packet (thread gl takes flat windows
// gl, gl + GROUP, ...; it issues the loads of BATCH windows before it uses
// the first).  Each window is read from the encoded stream src as three
// words, folded into the thread's partial syndrome of its segment (flushed
// to X/H in LDS when the thread moves on to the next segment), and its
// message run is ORed into the message buffer Mb; window 0 holds the 57 head
// bits, checksum position 64 and 63 more message bits.  Mb (mw + 3 words), X
// and H must be zero and visible on entry; the result is visible to the
// group on return.
template <uint32_t GROUP, uint32_t BATCH>
__device__ __forceinline__ void decode_windows(const uint64_t* src, uint32_t ew, const Layout& Lo, uint64_t* Mb,
                                               uint64_t* X, uint32_t* H, uint32_t gl)
{
    const uint32_t wins = Lo.windows(), last = ew - 1u;
    WindowWalk walk(Lo, gl);
    uint32_t ci = 0;              // segment of the partial syndrome in xacc/hacc
    uint64_t xacc = 0;
    uint32_t hacc = 0;
    for (uint32_t g0 = gl; g0 < wins; g0 += BATCH * GROUP) {
        uint64_t a[BATCH], b[BATCH], c[BATCH];
        int32_t qw[BATCH];
        uint32_t seg[BATCH], wd[BATCH], sh[BATCH], nn[BATCH], kk[BATCH];
#pragma unroll
        for (uint32_t u = 0; u < BATCH; ++u) {
            walk.settle(Lo);
            // position 128v of segment i is stream bit s0 (-1, before the
            // packet, for the first window of segment 0)
            const int32_t s0 = int32_t(walk.o + 128u * walk.v) - 1;
            qw[u] = s0 >> 6;
            seg[u] = walk.i;
            wd[u] = walk.v;
            sh[u] = uint32_t(s0) & 63u;
            nn[u] = walk.n;
            kk[u] = walk.K;
            walk.v += GROUP;
        }
        // Unconditional loads clamped into the packet: for s0 = -1 the stray
        // bit lands on position 0, and a word past the packet supplies only
        // positions past the last segment; both are masked below.
#pragma unroll
        for (uint32_t u = 0; u < BATCH; ++u) {
            a[u] = src[min(uint32_t(max(qw[u], 0)), last)];
            b[u] = src[min(uint32_t(qw[u] + 1), last)];
            c[u] = src[min(uint32_t(qw[u] + 2), last)];
        }
#pragma unroll
        for (uint32_t u = 0; u < BATCH; ++u) {
            if (g0 + u * GROUP >= wins) break;
            const uint32_t v = wd[u];
            uint64_t x0, x1;
            funnel128(a[u], b[u], c[u], sh[u], x0, x1);
            mask_top(x0, x1, nn[u] - 128u * v);
            x0 &= ~uint64_t(v == 0 ? 1u : 0u);            // there is no position 0

            if (seg[u] != ci) {
                flush_partial(X, H, ci, xacc, hacc);
                ci = seg[u];
                xacc = 0;
                hacc = 0;
            }
            fold_window(x0, x1, v, xacc, hacc);

            uint32_t pw;
            const uint32_t b0 = kk[u] + run_start(v, pw);
            uint64_t c0 = (x0 >> pw) | ((x1 << 1) << (63u - pw));
            uint64_t c1 = x1 >> pw;
            if (v == 0) {
                c0 = head_message(c0) | (c1 << 57);
                c1 >>= 7;
            }
            or128(Mb, b0 >> 6, b0 & 63u, c0, c1);
        }
    }
    flush_partial(X, H, ci, xacc, hacc);
    group_sync<GROUP>();
}

// Encoding pass, the decoding pass reversed: each window's message run is
// read from the message words src (mw words; clamped reads past the packet
// supply only bits that land past the last segment's positions), placed at
// the window's positions with its checksum positions 0, folded into the
// partial syndrome, and ORed into the encoded buffer E at stream bit
// o + 128v - 1 (E[0] stands for stream bit -64..-1).  E (ew + 3 words), X and
// H must be zero and visible on entry.
template <uint32_t GROUP, uint32_t BATCH>
__device__ __forceinline__ void encode_windows(const uint64_t* src, uint32_t mw, const Layout& Lo, uint64_t* E,
                                               uint64_t* X, uint32_t* H, uint32_t gl)
{
    const uint32_t wins = Lo.windows(), last = mw - 1u;
    WindowWalk walk(Lo, gl);
    uint32_t ci = 0;
    uint64_t xacc = 0;
    uint32_t hacc = 0;
    for (uint32_t g0 = gl; g0 < wins; g0 += BATCH * GROUP) {
        uint64_t a[BATCH], b[BATCH], c[BATCH];
        uint32_t qm[BATCH], seg[BATCH], wd[BATCH], sh[BATCH], nn[BATCH], oo[BATCH], pp[BATCH];
#pragma unroll
        for (uint32_t u = 0; u < BATCH; ++u) {
            walk.settle(Lo);
            uint32_t pw;
            const uint32_t m0 = walk.K + run_start(walk.v, pw);
            qm[u] = m0 >> 6;
            sh[u] = m0 & 63u;
            pp[u] = pw;
            seg[u] = walk.i;
            wd[u] = walk.v;
            nn[u] = walk.n;
            oo[u] = walk.o;
            walk.v += GROUP;
        }
#pragma unroll
        for (uint32_t u = 0; u < BATCH; ++u) {
            a[u] = src[min(qm[u], last)];
            b[u] = src[min(qm[u] + 1u, last)];
            c[u] = src[min(qm[u] + 2u, last)];
        }
#pragma unroll
        for (uint32_t u = 0; u < BATCH; ++u) {
            if (g0 + u * GROUP >= wins) break;
            const uint32_t v = wd[u], pw = pp[u];
            uint64_t m0, m1;
            funnel128(a[u], b[u], c[u], sh[u], m0, m1);
            uint64_t x0, x1;
            if (v == 0) {
                x0 = head_expand(m0);
                x1 = ((m0 >> 57) | (m1 << 7)) << 1;        // positions 65..127
            } else {
                x0 = m0 << pw;
                x1 = (m1 << pw) | ((m0 >> 63) & pw);
            }
            mask_top(x0, x1, nn[u] - 128u * v);

            if (seg[u] != ci) {
                flush_partial(X, H, ci, xacc, hacc);
                ci = seg[u];
                xacc = 0;
                hacc = 0;
            }
            fold_window(x0, x1, v, xacc, hacc);

            const uint32_t sp = oo[u] + 128u * v + 63u;     // stream bit of position 128v, plus 64
            or128(E, sp >> 6, sp & 63u, x0, x1);
        }
    }
    flush_partial(X, H, ci, xacc, hacc);
    group_sync<GROUP>();
}

struct SegArgs {
    const uint64_t* enc;       // encoded arena (decode input, encode output)
    uint64_t enc_words;
    const hamming_seg_packet* descs;
    uint32_t n_packets;
    uint32_t max_msg_bytes;
    uint64_t* msg;             // message arena (decode output, encode input)
    uint64_t msg_words;
    uint16_t* syndromes;
    uint64_t syndrome_count;
    uint8_t* status;
    uint32_t slice_words;      // per-packet LDS buffer (accumulators excluded)
};

// Per-packet accumulators after the buffer: X, one 64-bit word per segment,
// then H, one 32-bit word per segment.
constexpr uint32_t kAccWords = HAMMING_SEG_MAX_T + HAMMING_SEG_MAX_T / 2;

// Decode packet pk with GROUP threads (gl = 0..GROUP-1); Mb is the packet's
// message buffer in LDS (at least mw + 3 words) and acc its accumulators.
// With GROUP < 64 several packets share a wave, so pk, the descriptor and the
// layout are per-lane values and wave-wide ballots are masked to the group.
// Every thread of a group takes the same branches at the barriers.
template <uint32_t GROUP, uint32_t BATCH>
__device__ __forceinline__ void decode_packet(const SegArgs& a, uint64_t pk, uint32_t gl, uint64_t* Mb, uint64_t* acc)
{
    const hamming_seg_packet d = a.descs[pk];
    const uint32_t M = d.msg_bytes, t = d.t;
    Layout Lo;
    const bool shape_ok = make_layout(M, t, a.max_msg_bytes, Lo);
    const uint64_t ew = (uint64_t(Lo.total) + 63) / 64, mw = (uint64_t(M) + 7) / 8;
    const bool ok = shape_ok && d.enc_word_off <= a.enc_words && ew <= a.enc_words - d.enc_word_off &&
                    d.msg_word_off <= a.msg_words && mw <= a.msg_words - d.msg_word_off &&
                    (!a.syndromes || (d.seg_off <= a.syndrome_count && t <= a.syndrome_count - d.seg_off));
    if (!ok) {
        if (a.status && gl == 0) a.status[pk] = HAMMING_SEG_INVALID;
        return;
    }
    uint64_t* X = acc;
    uint32_t* H = reinterpret_cast<uint32_t*>(acc + HAMMING_SEG_MAX_T);
    for (uint32_t w = 2 * gl; w < mw + 3; w += 2 * GROUP) {   // in pairs: the slice has mw + 4 words
        Mb[w] = 0;
        Mb[w + 1] = 0;
    }
    for (uint32_t i = gl; i < t; i += GROUP) {
        X[i] = 0;
        H[i] = 0;
    }
    group_sync<GROUP>();

    decode_windows<GROUP, BATCH>(a.enc + d.enc_word_off, uint32_t(ew), Lo, Mb, X, H, gl);

    // checksum owners: thread gl takes segments gl, gl + GROUP, ...; an error
    // at a message position flips that message bit, one at a checksum
    // position changes no message bit
    uint32_t st = 0;
    for (uint32_t i = gl; i < t; i += GROUP) {
        const uint32_t s = fold_syndrome(X[i], H[i]), n = Lo.n(i);
        if (s >= 1 && s <= n) {
            if (s & (s - 1u)) {
                const uint32_t bit = Lo.K(i) + s - (31u - __clz(s)) - 2u;
                atomicXor(reinterpret_cast<unsigned long long*>(&Mb[bit >> 6]), 1ull << (bit & 63));
            }
            st = max(st, 1u);
        } else if (s > n) {
            st = 2;
        }
        if (a.syndromes) a.syndromes[d.seg_off + i] = uint16_t(s);
    }
    uint64_t mask = ~uint64_t(0);
    if constexpr (GROUP < 64) mask = ((uint64_t(1) << GROUP) - 1) << ((threadIdx.x & 63u) & ~(GROUP - 1));
    if constexpr (GROUP > 64) {
        // t <= 32: every owner is in the first wave, whose ballot decides
        mask = (threadIdx.x < 64) ? mask : 0;
    }
    const uint64_t any2 = __ballot(st == 2) & mask, any1 = __ballot(st == 1) & mask;
    if (a.status && gl == 0) a.status[pk] = any2 ? 2 : (any1 ? 1 : 0);
    group_sync<GROUP>();

    // the message words in 16-byte stores (two words per thread and step)
    uint64_t* dst = a.msg + d.msg_word_off;
    const uint64_t pairs = mw / 2;
    for (uint32_t q = gl; q < pairs; q += GROUP) {
        const uint64_t w0 = Mb[2 * q], w1 = Mb[2 * q + 1];
        u32x4 v;
        v.x = uint32_t(w0);
        v.y = uint32_t(w0 >> 32);
        v.z = uint32_t(w1);
        v.w = uint32_t(w1 >> 32);
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4a8*>(dst) + q);
    }
    if ((mw & 1) && gl == 0) __builtin_nontemporal_store(Mb[mw - 1], dst + mw - 1);
}

// Encode packet pk with GROUP threads; E is the packet's encoded buffer in
// LDS (at least ew + 3 words, E[0] in front of the stream) and acc its
// accumulators.  A descriptor this launch cannot take is skipped.
template <uint32_t GROUP, uint32_t BATCH>
__device__ __forceinline__ void encode_packet(const SegArgs& a, uint64_t pk, uint32_t gl, uint64_t* E, uint64_t* acc)
{
    const hamming_seg_packet d = a.descs[pk];
    const uint32_t M = d.msg_bytes, t = d.t;
    Layout Lo;
    const bool shape_ok = make_layout(M, t, a.max_msg_bytes, Lo);
    const uint64_t ew = (uint64_t(Lo.total) + 63) / 64, mw = (uint64_t(M) + 7) / 8;
    const bool ok = shape_ok && d.enc_word_off <= a.enc_words && ew <= a.enc_words - d.enc_word_off &&
                    d.msg_word_off <= a.msg_words && mw <= a.msg_words - d.msg_word_off;
    if (!ok) return;
    uint64_t* X = acc;
    uint32_t* H = reinterpret_cast<uint32_t*>(acc + HAMMING_SEG_MAX_T);
    for (uint32_t w = gl; w < ew + 3; w += GROUP) E[w] = 0;
    for (uint32_t i = gl; i < t; i += GROUP) {
        X[i] = 0;
        H[i] = 0;
    }
    group_sync<GROUP>();

    encode_windows<GROUP, BATCH>(a.msg + d.msg_word_off, uint32_t(mw), Lo, E, X, H, gl);

    // checksum position 2^j of segment i takes bit j of the syndrome of its
    // message bits, which makes the segment's syndrome 0
    for (uint32_t i = gl; i < t; i += GROUP) {
        const uint32_t s = fold_syndrome(X[i], H[i]), o = Lo.o(i);
        for (uint32_t j = 0; (s >> j) != 0; ++j) {
            if (!((s >> j) & 1u)) continue;
            const uint32_t bit = o + (1u << j) + 63u;       // stream bit of position 2^j, plus 64
            atomicOr(reinterpret_cast<unsigned long long*>(&E[bit >> 6]), 1ull << (bit & 63));
        }
    }
    group_sync<GROUP>();

    // the encoded words in 16-byte stores (two words per thread and step)
    uint64_t* dst = const_cast<uint64_t*>(a.enc) + d.enc_word_off;
    const uint64_t pairs = ew / 2;
    for (uint32_t q = gl; q < pairs; q += GROUP) {
        const uint64_t w0 = E[2 * q + 1], w1 = E[2 * q + 2];
        u32x4 v;
        v.x = uint32_t(w0);
        v.y = uint32_t(w0 >> 32);
        v.z = uint32_t(w1);
        v.w = uint32_t(w1 >> 32);
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4a8*>(dst) + q);
    }
    if ((ew & 1) && gl == 0) __builtin_nontemporal_store(E[ew], dst + ew - 1);
}

// 256 / GROUP packets per block, GROUP threads each: part of a wave, a wave,
// or (GROUP = 256) the whole block on one packet, the latency form.
template <uint32_t GROUP, uint32_t BATCH>
__global__ __launch_bounds__(64 * kSegWaves) void seg_decode_kernel(SegArgs a)
{
    extern __shared__ uint64_t lds[];
    const uint32_t slot = threadIdx.x / GROUP;
    const uint64_t pk = uint64_t(blockIdx.x) * (64 * kSegWaves / GROUP) + slot;
    if (pk >= a.n_packets) return;
    uint64_t* slice = lds + slot * (a.slice_words + kAccWords);
    decode_packet<GROUP, BATCH>(a, pk, threadIdx.x % GROUP, slice, slice + a.slice_words);
}

template <uint32_t GROUP, uint32_t BATCH>
__global__ __launch_bounds__(64 * kSegWaves) void seg_encode_kernel(SegArgs a)
{
    extern __shared__ uint64_t lds[];
    const uint32_t slot = threadIdx.x / GROUP;
    const uint64_t pk = uint64_t(blockIdx.x) * (64 * kSegWaves / GROUP) + slot;
    if (pk >= a.n_packets) return;
    uint64_t* slice = lds + slot * (a.slice_words + kAccWords);
    encode_packet<GROUP, BATCH>(a, pk, threadIdx.x % GROUP, slice, slice + a.slice_words);
}

// Threads per packet when the caller leaves the choice to the library: a
// workgroup per packet for batches too small to fill the GPU's wave slots
// (latency), otherwise a group sized to the packets (throughput).
constexpr uint32_t kWideMaxPackets = 2048;
std::atomic<uint32_t> g_seg_threads{0};

uint32_t auto_threads_per_packet(uint32_t n_packets, uint32_t max_msg_bytes, bool decode)
{
    if (n_packets <= kWideMaxPackets) return 256;
    // measured on the Table 1 grid (400..2000-byte packets) and between its
    // sizes: 8 threads per packet are fastest at 400 bytes (the per-packet
    // overhead is shared by eight packets of a wave) and, decoding, at 640
    // and 800 bytes for every t; 16 beat 8, 32 and 64 from 1000 bytes on
    if (max_msg_bytes <= (decode ? 896u : 640u)) return 8u;
    return max_msg_bytes <= 2048 ? 16u : (max_msg_bytes <= 3072 ? 32u : 64u);
}

template <uint32_t GROUP, uint32_t BATCH, bool DECODE>
constexpr void (*seg_kernel())(SegArgs)
{
    if constexpr (DECODE)
        return seg_decode_kernel<GROUP, BATCH>;
    else
        return seg_encode_kernel<GROUP, BATCH>;
}

// Launches the decode or encode of n_packets with the configured (or
// automatic) group size.  Windows a thread loads ahead: 2 while a thread has
// at most about five windows (the unused slots of a last batch cost loads and
// walk steps), 4 above (more loads in flight); measured on the Table 1 grid.
template <bool DECODE>
void launch(const SegArgs& a, uint32_t n_packets, uint32_t max_msg_bytes, hipStream_t stream)
{
    uint32_t group = g_seg_threads.load();
    if (group == 0) group = auto_threads_per_packet(n_packets, max_msg_bytes, DECODE);
    const bool deep = (8u * max_msg_bytes) / (128u * group) > 5u;
    void (*kernel)(SegArgs);
    if (group == 8)
        kernel = deep ? seg_kernel<8, 4, DECODE>() : seg_kernel<8, 2, DECODE>();
    else if (group == 16)
        kernel = deep ? seg_kernel<16, 4, DECODE>() : seg_kernel<16, 2, DECODE>();
    else if (group == 32)
        kernel = deep ? seg_kernel<32, 4, DECODE>() : seg_kernel<32, 2, DECODE>();
    else if (group == 64)   // at most four windows each (HAMMING_SEG_MAX_BYTES)
        kernel = seg_kernel<64, 2, DECODE>();
    else
        kernel = seg_kernel<256, 2, DECODE>();
    const uint32_t per_block = 64 * kSegWaves / group;
    const size_t lds = size_t(per_block) * (a.slice_words + kAccWords) * 8;
    // one launch per slice of packets that fits a dispatch's 32-bit work-item
    // count; a slice addresses its packets through offset descriptor and
    // status pointers (syndromes are placed by each descriptor's seg_off)
    const uint64_t per_launch = hm::max_launch_blocks(64 * kSegWaves) * per_block;
    for (uint64_t first = 0; first < n_packets; first += per_launch) {
        SegArgs s = a;
        s.descs = a.descs + first;
        s.status = a.status ? a.status + first : nullptr;
        s.n_packets = uint32_t(n_packets - first < per_launch ? n_packets - first : per_launch);
        const uint32_t blocks = (s.n_packets + per_block - 1) / per_block;
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(64 * kSegWaves), lds, stream, s);
    }
}

int check_common(const void* enc, const void* descs, uint32_t n_packets, const void* msg, uint32_t max_msg_bytes)
{
    if (n_packets > HAMMING_MAX_BATCH) return HAMMING_ERANGE;
    if (max_msg_bytes < 1 || max_msg_bytes > HAMMING_SEG_MAX_BYTES) return HAMMING_EINVAL;
    if (n_packets == 0) return HAMMING_OK;
    if (!enc || !descs || !msg) return HAMMING_EINVAL;
    if ((reinterpret_cast<uintptr_t>(enc) & 7u) || (reinterpret_cast<uintptr_t>(msg) & 7u) ||
        (reinterpret_cast<uintptr_t>(descs) & 7u))
        return HAMMING_EALIGN;
    return HAMMING_OK;
}

}  // namespace

extern "C" {

int64_t hamming_seg_layout(uint32_t msg_bytes, uint32_t t, uint32_t* k_out, uint32_t* r_out)
{
    if (t < 1 || t > HAMMING_SEG_MAX_T || msg_bytes < 1 || msg_bytes > HAMMING_SEG_MAX_BYTES || 8ull * msg_bytes < t)
        return -1;
    const uint32_t bits = 8u * msg_bytes;
    if ((bits + t - 1) / t > HAMMING_SEG_MAX_K) return -1;
    int64_t total = 0;
    for (uint32_t i = 0; i < t; ++i) {
        const uint32_t k = bits / t + (i < bits % t ? 1u : 0u);
        const uint32_t r = seg_checksum_bits(k);
        if (k_out) k_out[i] = k;
        if (r_out) r_out[i] = r;
        total += int64_t(k) + r;
    }
    return total;
}

int hamming_seg_config_set(uint32_t threads_per_packet)
{
    if (threads_per_packet != 0 && threads_per_packet != 8 && threads_per_packet != 16 && threads_per_packet != 32 &&
        threads_per_packet != 64 && threads_per_packet != 256)
        return HAMMING_EINVAL;
    g_seg_threads.store(threads_per_packet);
    return HAMMING_OK;
}

int hamming_seg_config_get(uint32_t* threads_per_packet)
{
    if (!threads_per_packet) return HAMMING_EINVAL;
    *threads_per_packet = g_seg_threads.load();
    return HAMMING_OK;
}

int hamming_decode_segmented(const uint64_t* enc_arena, uint64_t enc_words, const hamming_seg_packet* descs,
                             uint32_t n_packets, uint32_t max_msg_bytes, uint64_t* msg_arena, uint64_t msg_words,
                             uint16_t* syndromes, uint64_t syndrome_count, uint8_t* status, hipStream_t stream)
{
    int rc = check_common(enc_arena, descs, n_packets, msg_arena, max_msg_bytes);
    if (rc != HAMMING_OK || n_packets == 0) return rc;
    if (syndromes && (reinterpret_cast<uintptr_t>(syndromes) & 1u)) return HAMMING_EALIGN;
    SegArgs a{enc_arena, enc_words, descs, n_packets, max_msg_bytes, msg_arena, msg_words,
              syndromes, syndromes ? syndrome_count : 0, status, msg_slice_words(max_msg_bytes)};
    launch<true>(a, n_packets, max_msg_bytes, stream);
    return hipGetLastError() == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

int hamming_encode_segmented(const uint64_t* msg_arena, uint64_t msg_words, const hamming_seg_packet* descs,
                             uint32_t n_packets, uint32_t max_msg_bytes, uint64_t* enc_arena, uint64_t enc_words,
                             hipStream_t stream)
{
    int rc = check_common(enc_arena, descs, n_packets, msg_arena, max_msg_bytes);
    if (rc != HAMMING_OK || n_packets == 0) return rc;
    SegArgs a{enc_arena, enc_words, descs, n_packets, max_msg_bytes, const_cast<uint64_t*>(msg_arena), msg_words,
              nullptr, 0, nullptr, enc_slice_words(max_msg_bytes)};
    launch<false>(a, n_packets, max_msg_bytes, stream);
    return hipGetLastError() == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

}  // extern "C"

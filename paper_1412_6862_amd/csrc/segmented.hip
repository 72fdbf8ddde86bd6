// Segmented packets (Sec. II, Fig. 1): a packet of M message bytes travels
// as t shortened Hamming segments H_1..H_t laid end to end as one bit
// string; each segment is checked and corrected on its own and the recovered
// message segments are merged back into the M-byte packet.  The checksum of a
// segment is the XOR over its index sets (Sec. III.A, III.C, Algorithm 1),
// computed here one 64-position word at a time and reduced across the wave.
//
// A group of threads per packet (part of a wave, a wave or a workgroup): the
// 128-position windows of all segments are dealt to the threads and read from
// HBM once, as unaligned three-word spans.  Each window is folded into the
// thread's partial syndrome of its segment and its message bits (one run of
// consecutive message indices per window) are ORed into the packet's message
// buffer in LDS; the segment owners then finish the syndromes, flip the one
// message bit a correctable error hits, and the buffer is stored.  Segment
// offsets are closed-form (message sizes take two values), so no lookup
// table is read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "hamming.h"
#include "tile.h"

using hm::wave_sync;

namespace {

constexpr uint32_t kSegWaves = 4;                          // packets per block
constexpr uint32_t kSynWords = HAMMING_SEG_MAX_T / 2;      // per-wave syndrome accumulators, in 64-bit words

// Longest encoded packet of at most max_msg_bytes message bytes, in 64-bit
// words, plus a zero word in front (so the word holding positions 0..63 of the
// first segment reads as any other) and two behind (that unaligned two-word
// reads may touch).
__host__ __device__ inline uint32_t enc_slice_words(uint32_t max_msg_bytes)
{
    return (8u * max_msg_bytes + 16u * HAMMING_SEG_MAX_T + 63u) / 64u + 3u;
}

// Message words of the longest packet plus three (a message run ORed in at a
// bit offset touches up to three words).
__host__ __device__ inline uint32_t msg_slice_words(uint32_t max_msg_bytes)
{
    return (max_msg_bytes + 7u) / 8u + 3u;
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

// 64 bits starting at an arbitrary bit of an LDS word array (both words read,
// no branch: the high word is shifted in two steps so a shift of 0 is defined).
__device__ __forceinline__ uint64_t read_bits64(const uint64_t* L, uint64_t bit)
{
    const uint32_t q = uint32_t(bit >> 6), sh = uint32_t(bit & 63);
    return (L[q] >> sh) | ((L[q + 1] << 1) << (63 - sh));
}

// Segment layout of one packet in closed form.  The first `rem` segments
// carry q+1 message bits and nA positions, the others q bits and nB
// positions, so every offset is a product and a min, and the segment that
// holds a given bit is one division.  All fields are wave-uniform.
struct Layout {
    uint32_t t, q, rem, nA, nB, nwA, nwB, total;

    __device__ uint32_t K(uint32_t i) const { return i * q + min(i, rem); }            // first message bit
    __device__ uint32_t k(uint32_t i) const { return q + (i < rem ? 1u : 0u); }
    __device__ uint32_t o(uint32_t i) const { return i * nB + min(i, rem) * (nA - nB); }  // first stream bit
    __device__ uint32_t n(uint32_t i) const { return i < rem ? nA : nB; }
    __device__ uint32_t seg_of_msg(uint32_t m) const
    {
        const uint32_t a = rem * (q + 1);
        return m < a ? m / (q + 1) : rem + (m - a) / q;
    }
    __device__ uint32_t seg_of_bit(uint32_t b) const
    {
        const uint32_t a = rem * nA;
        return b < a ? b / nA : rem + (b - a) / nB;
    }
    __device__ uint32_t syndrome_words() const { return rem * nwA + (t - rem) * nwB; }
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
    L.nwA = L.nA / 64 + 1;
    L.nwB = L.nB / 64 + 1;
    L.total = L.o(t);
    return true;
}

// Contribution of position word w of a segment (positions 64w..64w+63, bit
// q of the word = position 64w + q) to its syndrome: the low six bits of a
// position are those of q, the higher bits those of 64w (Algorithm 1's XOR
// over index sets, 64 positions at a time).  Bits q and q+32 share bits 0..4
// of q, so those five parities are taken on the XOR of the two halves.
__device__ __forceinline__ uint32_t word_syndrome(const uint64_t* L, uint32_t o, uint32_t n, uint32_t w)
{
    // position 64w + q is bit o + 64w + q - 1 of L, read from the zero word in
    // front of L for o = w = 0
    uint64_t x = read_bits64(L - 1, uint64_t(o) + 64u * w + 63u);
    if (w == 0) x &= ~uint64_t(1);                     // there is no position 0
    const uint32_t hi = n - 64u * w;                    // last valid bit index in this word
    if (hi < 63) x &= (uint64_t(2) << hi) - 1;
    const uint32_t h = uint32_t(x >> 32), f = uint32_t(x) ^ h;
    uint32_t v = __popc(f & 0xAAAAAAAAu) & 1u;
    v |= (__popc(f & 0xCCCCCCCCu) & 1u) << 1;
    v |= (__popc(f & 0xF0F0F0F0u) & 1u) << 2;
    v |= (__popc(f & 0xFF00FF00u) & 1u) << 3;
    v |= (__popc(f & 0xFFFF0000u) & 1u) << 4;
    v |= (__popc(h) & 1u) << 5;
    if (__popc(f) & 1u) v |= 64u * w;
    return v;
}

// Barrier of the threads that decode one packet: part of a wave or one wave
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

// Syndromes of all segments: the position words of every segment form one
// flat list dealt to the GROUP threads (thread L takes words L, L+GROUP, ...); each
// walks its (segment, word) position forward and XORs its words'
// contributions into the segment's accumulator in LDS.  S must be zero and
// visible on entry; the result is visible to the whole wave on return.
template <uint32_t GROUP>
__device__ __forceinline__ void all_syndromes(const uint64_t* L, const Layout& Lo, uint32_t* S, uint32_t lane)
{
    const uint32_t words = Lo.syndrome_words();
    uint32_t i = 0, w = lane, nw = Lo.rem > 0 ? Lo.nwA : Lo.nwB;
    for (uint32_t g = lane; g < words; g += GROUP) {
        while (w >= nw) {          // move to the segment holding word g
            w -= nw;
            ++i;
            nw = i < Lo.rem ? Lo.nwA : Lo.nwB;
        }
        atomicXor(&S[i], word_syndrome(L, Lo.o(i), Lo.n(i), w));
        w += GROUP;
    }
    group_sync<GROUP>();
}

// The message positions below 64 (3, 5..7, 9..15, 17..31, 33..63) carry a
// segment's first 57 message bits; given positions 1..64 as bits 0..63 of w,
// this compacts them with constant masks and shifts.
__device__ __forceinline__ uint64_t head_message(uint64_t w)
{
    return ((w >> 2) & 0x1ull) | (((w >> 4) & 0x7ull) << 1) | (((w >> 8) & 0x7Full) << 4) |
           (((w >> 16) & 0x7FFFull) << 11) | (((w >> 32) & 0x7FFFFFFFull) << 26);
}

// Syndrome of a segment from the XOR of its position words (X) and the XOR of
// 64w over its words of odd weight (H): bits 0..4 of a position are those of
// its bit q in the word, and q and q+32 share them, so those five parities are
// taken on the XOR of the halves; bit 5 is the parity of the high half.
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
// Threads whose words cancelled (or that had none) skip the LDS atomics, which
// all threads of a segment aim at the same two addresses.
__device__ __forceinline__ void flush_partial(uint64_t* X, uint32_t* H, uint32_t i, uint64_t x, uint32_t h)
{
    if (x | h) {
        atomicXor(reinterpret_cast<unsigned long long*>(&X[i]), x);
        atomicXor(&H[i], h);
    }
}

// One pass over the windows of every segment of a packet: window v of a
// segment is positions 128v..128v+127 (bit q of the pair (x0, x1) is position
// 128v + q), and thread gl takes flat windows gl, gl + GROUP, ...  A window is
// read from HBM as three words and shifted into place; a thread issues the
// loads of BATCH windows before it uses the first.  It is folded into the
// thread's partial syndrome of its segment (bits 0..5 of a position are those
// of q mod 64, bit 6 says which half, the rest are v), flushed to X/H in LDS
// when the thread moves on to the next segment.  Its message positions are
// ORed into the message buffer Mb: for v >= 1 only position 128v can be a
// checksum position (when v is a power of two), so a window holds one run of
// consecutive message bits whose first index is closed-form; window 0 holds
// the 57 head bits, the checksum position 64 and 63 more message bits.
// Mb (mw + 3 words), X and H must be zero and visible on entry; the result is
// visible to the group on return.
template <uint32_t GROUP, uint32_t BATCH>
__device__ __forceinline__ void scan_packet(const uint64_t* src, uint32_t ew, const Layout& Lo, uint64_t* Mb,
                                            uint64_t* X, uint32_t* H, uint32_t gl)
{
    const uint32_t vA = Lo.nA / 128u + 1u, vB = Lo.nB / 128u + 1u;
    const uint32_t wins = Lo.rem * vA + (Lo.t - Lo.rem) * vB;
    // walk state of the next window to load: segment, window, windows in the
    // segment, first stream bit, positions, first message bit
    uint32_t wi = 0, vv = gl, wnv = Lo.rem > 0 ? vA : vB, wo = 0, wn = Lo.n(0), wK = 0;
    uint32_t ci = 0;              // segment of the partial syndrome in xacc/hacc
    uint64_t xacc = 0;
    uint32_t hacc = 0;
    const uint32_t last = ew - 1u;
    for (uint32_t g0 = gl; g0 < wins; g0 += BATCH * GROUP) {
        uint64_t a[BATCH], b[BATCH], c[BATCH];
        int32_t qw[BATCH];
        uint32_t seg[BATCH], wd[BATCH], sh[BATCH], nn[BATCH], kk[BATCH];
#pragma unroll
        for (uint32_t u = 0; u < BATCH; ++u) {
            // (a slot past the packet's last window stays in the last
            // segment; it is never used)
            while (vv >= wnv && wi + 1 < Lo.t) {
                vv -= wnv;
                ++wi;
                wnv = wi < Lo.rem ? vA : vB;
                wo = Lo.o(wi);
                wn = Lo.n(wi);
                wK = Lo.K(wi);
            }
            // position 128vv of segment wi is stream bit s0 (-1, before the
            // packet, for the first window of segment 0)
            const int32_t s0 = int32_t(wo + 128u * vv) - 1;
            qw[u] = s0 >> 6;
            seg[u] = wi;
            wd[u] = vv;
            sh[u] = uint32_t(s0) & 63u;
            nn[u] = wn;
            kk[u] = wK;
            vv += GROUP;
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
            const uint32_t v = wd[u], s = sh[u];
            uint64_t x0 = (a[u] >> s) | ((b[u] << 1) << (63u - s));
            uint64_t x1 = (b[u] >> s) | ((c[u] << 1) << (63u - s));
            // positions past the segment's last one, and position 0
            const uint32_t top = nn[u] - 128u * v;
            x0 &= (~uint64_t(0) >> (63u - min(top, 63u))) & ~uint64_t(v == 0 ? 1u : 0u);
            x1 &= top < 64u ? uint64_t(0) : (~uint64_t(0) >> (63u - min(top - 64u, 63u)));

            if (seg[u] != ci) {
                flush_partial(X, H, ci, xacc, hacc);
                ci = seg[u];
                xacc = 0;
                hacc = 0;
            }
            const uint64_t f = x0 ^ x1;
            xacc ^= f;
            hacc ^= ((uint32_t(__popcll(x1)) & 1u) << 6) ^ ((__popcll(f) & 1u) ? 128u * v : 0u);

            // message bits of the window and the index of the first one (pw:
            // position 128v is a checksum position, as for v = 0 none is)
            const uint32_t lv = 31u - __clz(v | 1u);
            const uint32_t pw = (v & (v - 1u)) == 0u ? 1u : 0u;
            uint64_t c0 = (x0 >> pw) | ((x1 << 1) << (63u - pw));
            uint64_t c1 = x1 >> pw;
            if (v == 0) {
                c0 = head_message(c0) | (c1 << 57);
                c1 >>= 7;
            }
            const uint32_t bb = kk[u] + (v == 0 ? 0u : 128u * v + pw - lv - 9u);
            const uint32_t bq = bb >> 6, bs = bb & 63u;
            atomicOr(reinterpret_cast<unsigned long long*>(&Mb[bq]), c0 << bs);
            atomicOr(reinterpret_cast<unsigned long long*>(&Mb[bq + 1]), ((c0 >> 1) >> (63u - bs)) | (c1 << bs));
            atomicOr(reinterpret_cast<unsigned long long*>(&Mb[bq + 2]), (c1 >> 1) >> (63u - bs));
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
    uint32_t slice_words;      // per-packet LDS slice (accumulators excluded)
};

// Per-packet decode accumulators after the message buffer: X, one 64-bit
// word per segment, then H, one 32-bit word per segment.
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
    for (uint32_t w = gl; w < mw + 3; w += GROUP) Mb[w] = 0;
    for (uint32_t i = gl; i < t; i += GROUP) {
        X[i] = 0;
        H[i] = 0;
    }
    group_sync<GROUP>();

    scan_packet<GROUP, BATCH>(a.enc + d.enc_word_off, uint32_t(ew), Lo, Mb, X, H, gl);

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

    uint64_t* dst = a.msg + d.msg_word_off;
    for (uint32_t ow = gl; ow < mw; ow += GROUP) __builtin_nontemporal_store(Mb[ow], dst + ow);
}

// Throughput form: 256 / GROUP packets per block, GROUP threads each (a
// wave, or a part of one: 8, 16 or 32 threads).
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

// Latency form: one packet per block, all four waves on it.
__global__ __launch_bounds__(64 * kSegWaves) void seg_decode_wide_kernel(SegArgs a)
{
    extern __shared__ uint64_t lds[];
    const uint64_t pk = blockIdx.x;
    if (pk >= a.n_packets) return;
    decode_packet<64 * kSegWaves, 2>(a, pk, threadIdx.x, lds, lds + a.slice_words);
}

__global__ __launch_bounds__(64 * kSegWaves) void seg_encode_kernel(SegArgs a)
{
    extern __shared__ uint64_t lds[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t pk = uint64_t(blockIdx.x) * kSegWaves + wib;
    if (pk >= a.n_packets) return;
    uint64_t* slice = lds + wib * (a.slice_words + kSynWords);  // zero word, encoded words, message words
    uint64_t* E = slice + 1;
    uint32_t* S = reinterpret_cast<uint32_t*>(slice + a.slice_words);

    const hamming_seg_packet d = a.descs[pk];
    const uint32_t M = d.msg_bytes, t = d.t;
    Layout Lo;
    const bool shape_ok = make_layout(M, t, a.max_msg_bytes, Lo);
    const uint64_t ew = (uint64_t(Lo.total) + 63) / 64, mw = (uint64_t(M) + 7) / 8;
    const bool ok = shape_ok && d.enc_word_off <= a.enc_words && ew <= a.enc_words - d.enc_word_off &&
                    d.msg_word_off <= a.msg_words && mw <= a.msg_words - d.msg_word_off;
    if (!ok) return;
    uint64_t* Mw = slice + enc_slice_words(a.max_msg_bytes);
    const uint64_t* src = a.msg + d.msg_word_off;
    for (uint32_t w = lane; w < mw; w += 64) Mw[w] = src[w];
    if (lane < 2) {
        Mw[mw + lane] = 0;
        E[ew + lane] = 0;
    }
    if (lane == 2) E[-1] = 0;
    if (lane < HAMMING_SEG_MAX_T) S[lane] = 0;
    wave_sync();

    // message bits into their positions, checksum positions left 0
    for (uint32_t e = lane; e < ew; e += 64) {
        uint32_t b = 64u * e;
        const uint32_t end = min(b + 64u, Lo.total);
        uint32_t i = Lo.seg_of_bit(b);
        uint64_t acc = 0;
        while (b < end) {
            const uint32_t o = Lo.o(i), n = Lo.n(i);
            const uint32_t p = b - o + 1;
            if (p > n) {
                ++i;
                continue;
            }
            if ((p & (p - 1)) == 0) {   // checksum position
                ++b;
                continue;
            }
            const uint32_t j = 31u - __clz(p);
            const uint32_t last = min((2u << j) - 1u, n);
            const uint32_t len = min(last - p + 1u, end - b);
            uint64_t v = read_bits64(Mw, uint64_t(Lo.K(i)) + p - j - 2u);
            if (len < 64) v &= (uint64_t(1) << len) - 1;
            acc |= v << (b - 64u * e);
            b += len;
        }
        E[e] = acc;
    }
    wave_sync();

    // checksum position 2^j takes bit j of the syndrome of the message bits alone
    all_syndromes<64>(E, Lo, S, lane);
    if (lane < t) {
        const uint32_t s = S[lane], o = Lo.o(lane);
        for (uint32_t j = 0; s >> j; ++j) {
            if (!((s >> j) & 1)) continue;
            const uint32_t bit = o + (1u << j) - 1u;
            atomicOr(reinterpret_cast<unsigned long long*>(&E[bit >> 6]), 1ull << (bit & 63));
        }
    }
    wave_sync();
    uint64_t* dst = const_cast<uint64_t*>(a.enc) + d.enc_word_off;
    for (uint32_t w = lane; w < ew; w += 64) __builtin_nontemporal_store(E[w], dst + w);
}

// Threads per packet when the caller leaves the choice to the library: a
// workgroup per packet for batches too small to fill the GPU's wave slots
// (latency), otherwise a group sized to the packets (throughput).
constexpr uint32_t kWideMaxPackets = 2048;
std::atomic<uint32_t> g_seg_threads{0};

uint32_t auto_threads_per_packet(uint32_t n_packets, uint32_t max_msg_bytes)
{
    if (n_packets <= kWideMaxPackets) return 256;
    // measured on the Table 1 grid (400..2000-byte packets): 8 threads per
    // packet are fastest at 400 bytes (the per-packet overhead is shared by
    // eight packets of a wave), tie with 16 at 800, and 16 beat 8, 32 and 64
    // from 1200 bytes on
    if (max_msg_bytes <= 640) return 8u;
    return max_msg_bytes <= 2048 ? 16u : (max_msg_bytes <= 3072 ? 32u : 64u);
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
    uint32_t group = g_seg_threads.load();
    if (group == 0) group = auto_threads_per_packet(n_packets, max_msg_bytes);
    if (group == 256) {
        const size_t lds = size_t(a.slice_words + kAccWords) * 8;
        hipLaunchKernelGGL(seg_decode_wide_kernel, dim3(n_packets), dim3(64 * kSegWaves), lds, stream, a);
    } else {
        const uint32_t per_block = 64 * kSegWaves / group;
        const size_t lds = size_t(per_block) * (a.slice_words + kAccWords) * 8;
        const uint32_t blocks = (n_packets + per_block - 1) / per_block;
        // windows a thread loads ahead: 2 while a thread has at most about
        // five windows (the unused slots of a last batch cost loads and walk
        // steps), 4 above (more loads in flight); measured on the Table 1 grid
        const bool deep = (8u * max_msg_bytes) / (128u * group) > 5u;
        if (group == 8 && deep)
            hipLaunchKernelGGL((seg_decode_kernel<8, 4>), dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
        else if (group == 8)
            hipLaunchKernelGGL((seg_decode_kernel<8, 2>), dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
        else if (group == 16 && deep)
            hipLaunchKernelGGL((seg_decode_kernel<16, 4>), dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
        else if (group == 16)
            hipLaunchKernelGGL((seg_decode_kernel<16, 2>), dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
        else if (group == 32 && deep)
            hipLaunchKernelGGL((seg_decode_kernel<32, 4>), dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
        else if (group == 32)
            hipLaunchKernelGGL((seg_decode_kernel<32, 2>), dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
        else   // 64 threads: at most four windows each (HAMMING_SEG_MAX_BYTES)
            hipLaunchKernelGGL((seg_decode_kernel<64, 2>), dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
    }
    return hipGetLastError() == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

int hamming_encode_segmented(const uint64_t* msg_arena, uint64_t msg_words, const hamming_seg_packet* descs,
                             uint32_t n_packets, uint32_t max_msg_bytes, uint64_t* enc_arena, uint64_t enc_words,
                             hipStream_t stream)
{
    int rc = check_common(enc_arena, descs, n_packets, msg_arena, max_msg_bytes);
    if (rc != HAMMING_OK || n_packets == 0) return rc;
    SegArgs a{enc_arena, enc_words, descs, n_packets, max_msg_bytes, const_cast<uint64_t*>(msg_arena), msg_words,
              nullptr, 0, nullptr, enc_slice_words(max_msg_bytes) + msg_slice_words(max_msg_bytes)};
    const size_t lds = size_t(kSegWaves) * (a.slice_words + kSynWords) * 8;
    const uint32_t blocks = (n_packets + kSegWaves - 1) / kSegWaves;
    hipLaunchKernelGGL(seg_encode_kernel, dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
    return hipGetLastError() == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

}  // extern "C"

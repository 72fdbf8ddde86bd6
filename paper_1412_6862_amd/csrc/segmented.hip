// Segmented packets (Sec. II, Fig. 1): a packet of M message bytes travels
// as t shortened Hamming segments H_1..H_t laid end to end as one bit
// string; each segment is checked and corrected on its own and the recovered
// message segments are merged back into the M-byte packet.  The checksum of a
// segment is the XOR over its index sets (Sec. III.A, III.C, Algorithm 1),
// computed here one 64-position word at a time and reduced across the wave.
//
// One wave per packet: the encoded packet is staged in the wave's slice of
// LDS, syndromes are reduced with cross-lane XORs, the corrections are LDS
// atomics, and each lane then assembles whole 64-bit words of the merged
// message from the runs of message positions between checksum positions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hamming.h"
#include "tile.h"

using hm::wave_sync;

namespace {

constexpr uint32_t kSegWaves = 4;                      // packets per block
constexpr uint32_t kTableU32 = 3 * (HAMMING_SEG_MAX_T + 1);
constexpr uint32_t kTableWords = (kTableU32 + 1) / 2;  // per-wave segment table, in 64-bit words

// Longest encoded packet of at most max_msg_bytes message bytes, in 64-bit
// words, plus two zero words that unaligned two-word reads may touch.
__host__ __device__ inline uint32_t enc_slice_words(uint32_t max_msg_bytes)
{
    return (8u * max_msg_bytes + 16u * HAMMING_SEG_MAX_T + 63u) / 64u + 2u;
}

__host__ __device__ inline uint32_t msg_slice_words(uint32_t max_msg_bytes)
{
    return (max_msg_bytes + 7u) / 8u + 2u;
}

// Checksum bits of a shortened segment with k message bits: the smallest r
// with 2^r - 1 - r >= k.
__host__ __device__ inline uint32_t seg_checksum_bits(uint32_t k)
{
    uint32_t r = 2;
    while ((1u << r) - 1u - r < k) ++r;
    return r;
}

__device__ __forceinline__ uint64_t read_bits64(const uint64_t* L, uint64_t bit)
{
    const uint32_t q = uint32_t(bit >> 6), sh = uint32_t(bit & 63);
    return sh ? (L[q] >> sh) | (L[q + 1] << (64 - sh)) : L[q];
}

__device__ __forceinline__ uint32_t wave_xor(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v ^= __shfl_xor(v, d, 64);
    return v;
}

// Per-wave segment table in LDS: K[i] (first message bit of segment i,
// K[t] = 8M), o[i] (first stream bit, o[t] = encoded length), k[i].
struct SegTable {
    uint32_t* K;
    uint32_t* o;
    uint32_t* k;
};

// Validates the descriptor and fills the segment table; returns the encoded
// length in bits, or 0 for a packet this launch cannot take (uniform).
__device__ __forceinline__ uint32_t build_table(uint32_t msg_bytes, uint32_t t, uint32_t max_msg_bytes, uint32_t lane,
                                                SegTable tab)
{
    if (t < 1 || t > HAMMING_SEG_MAX_T || msg_bytes < 1 || msg_bytes > max_msg_bytes || 8u * msg_bytes < t) return 0;
    const uint32_t bits = 8u * msg_bytes;
    if ((bits + t - 1) / t > HAMMING_SEG_MAX_K) return 0;
    uint32_t ki = 0, ni = 0;
    if (lane < t) {
        ki = bits / t + (lane < bits % t ? 1u : 0u);
        ni = ki + seg_checksum_bits(ki);
    }
    uint32_t sk = ki, sn = ni;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t a = __shfl_up(sk, d, 64), b = __shfl_up(sn, d, 64);
        if (lane >= uint32_t(d)) {
            sk += a;
            sn += b;
        }
    }
    if (lane < t) {
        tab.K[lane] = sk - ki;
        tab.o[lane] = sn - ni;
        tab.k[lane] = ki;
    }
    if (lane == t - 1) {
        tab.K[t] = sk;
        tab.o[t] = sn;
    }
    return __shfl(sn, int(t - 1), 64);
}

// Syndrome of segment i: positions 1..n of the segment are stream bits
// o + p - 1.  Word w of the segment covers positions 64w..64w+63, so bit q
// of the word is position 64w + q: its low six bits are q, its higher bits
// are those of 64w.  Uniform result on every lane.
__device__ __forceinline__ uint32_t segment_syndrome(const uint64_t* L, uint32_t o, uint32_t n, uint32_t lane)
{
    uint32_t s = 0;
    const uint32_t nw = n / 64 + 1;
    for (uint32_t w = lane; w < nw; w += 64) {
        uint64_t x = (o == 0 && w == 0) ? (L[0] << 1) : read_bits64(L, uint64_t(o) + 64u * w - 1u);
        if (w == 0) x &= ~uint64_t(1);                     // there is no position 0
        const uint32_t hi = n - 64u * w;                    // last valid bit index in this word
        if (hi < 63) x &= (uint64_t(2) << hi) - 1;
        uint32_t v = 0;
        v |= uint32_t(__popcll(x & 0xAAAAAAAAAAAAAAAAull) & 1) << 0;
        v |= uint32_t(__popcll(x & 0xCCCCCCCCCCCCCCCCull) & 1) << 1;
        v |= uint32_t(__popcll(x & 0xF0F0F0F0F0F0F0F0ull) & 1) << 2;
        v |= uint32_t(__popcll(x & 0xFF00FF00FF00FF00ull) & 1) << 3;
        v |= uint32_t(__popcll(x & 0xFFFF0000FFFF0000ull) & 1) << 4;
        v |= uint32_t(__popcll(x & 0xFFFFFFFF00000000ull) & 1) << 5;
        if (__popcll(x) & 1) v |= 64u * w;
        s ^= v;
    }
    return wave_xor(s);
}

// Run of message positions containing message bit mu of a segment: the
// positions strictly between 2^j and 2^(j+1) carry message bits
// mu = p - j - 2.  Returns j.
__device__ __forceinline__ uint32_t run_of(uint32_t mu)
{
    uint32_t j = 31u - __clz(mu + 2u);
    if (j < 1) j = 1;
    while ((2u << j) - j - 2u <= mu) ++j;
    return j;
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
    uint32_t slice_words;      // per-wave LDS slice (table excluded)
};

__global__ __launch_bounds__(64 * kSegWaves) void seg_decode_kernel(SegArgs a)
{
    extern __shared__ uint64_t lds[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t pk = uint64_t(blockIdx.x) * kSegWaves + wib;
    if (pk >= a.n_packets) return;
    uint64_t* L = lds + wib * (a.slice_words + kTableWords);
    uint32_t* t32 = reinterpret_cast<uint32_t*>(L + a.slice_words);
    const SegTable tab{t32, t32 + (HAMMING_SEG_MAX_T + 1), t32 + 2 * (HAMMING_SEG_MAX_T + 1)};

    const hamming_seg_packet d = a.descs[pk];
    const uint32_t M = d.msg_bytes, t = d.t;
    const uint32_t total = build_table(M, t, a.max_msg_bytes, lane, tab);
    const uint64_t ew = (uint64_t(total) + 63) / 64, mw = (uint64_t(M) + 7) / 8;
    const bool ok = total != 0 && d.enc_word_off <= a.enc_words && ew <= a.enc_words - d.enc_word_off &&
                    d.msg_word_off <= a.msg_words && mw <= a.msg_words - d.msg_word_off &&
                    (!a.syndromes || (d.seg_off <= a.syndrome_count && t <= a.syndrome_count - d.seg_off));
    if (!ok) {
        if (a.status && lane == 0) a.status[pk] = HAMMING_SEG_INVALID;
        return;
    }

    const uint64_t* src = a.enc + d.enc_word_off;
    for (uint32_t w = lane; w < ew; w += 64) L[w] = __builtin_nontemporal_load(src + w);
    if (lane < 2) L[ew + lane] = 0;
    wave_sync();

    uint32_t my_s = 0;
    for (uint32_t i = 0; i < t; ++i) {
        const uint32_t o = tab.o[i];
        const uint32_t s = segment_syndrome(L, o, tab.o[i + 1] - o, lane);
        if (lane == i) my_s = s;
    }
    wave_sync();   // every lane has read the received bits before any correction

    uint32_t st = 0;
    if (lane < t) {
        const uint32_t o = tab.o[lane], n = tab.o[lane + 1] - o;
        if (my_s >= 1 && my_s <= n) {
            const uint32_t bit = o + my_s - 1;
            atomicXor(reinterpret_cast<unsigned long long*>(&L[bit >> 6]), 1ull << (bit & 63));
            st = 1;
        } else if (my_s > n) {
            st = 2;
        }
        if (a.syndromes) a.syndromes[d.seg_off + lane] = uint16_t(my_s);
    }
    const uint64_t any2 = __ballot(st == 2), any1 = __ballot(st == 1);
    if (a.status && lane == 0) a.status[pk] = any2 ? 2 : (any1 ? 1 : 0);
    wave_sync();

    // merge: lane-owned 64-bit words of the packet's message
    const uint32_t nbits = 8u * M;
    uint64_t* dst = a.msg + d.msg_word_off;
    for (uint32_t ow = lane; ow < mw; ow += 64) {
        uint32_t m = 64u * ow;
        const uint32_t end = min(m + 64u, nbits);
        uint32_t i = 0;
        while (i + 1 < t && tab.K[i + 1] <= m) ++i;
        uint64_t acc = 0;
        while (m < end) {
            const uint32_t K = tab.K[i], k = tab.k[i];
            const uint32_t mu = m - K;
            if (mu >= k) {
                ++i;
                continue;
            }
            const uint32_t j = run_of(mu);
            const uint32_t len = min(min((2u << j) - j - 2u, k) - mu, end - m);
            uint64_t v = read_bits64(L, uint64_t(m) + (tab.o[i] - K) + j + 1);
            if (len < 64) v &= (uint64_t(1) << len) - 1;
            acc |= v << (m - 64u * ow);
            m += len;
        }
        __builtin_nontemporal_store(acc, dst + ow);
    }
}

__global__ __launch_bounds__(64 * kSegWaves) void seg_encode_kernel(SegArgs a)
{
    extern __shared__ uint64_t lds[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t pk = uint64_t(blockIdx.x) * kSegWaves + wib;
    if (pk >= a.n_packets) return;
    uint64_t* E = lds + wib * (a.slice_words + kTableWords);     // encoded words, then the message words
    uint32_t* t32 = reinterpret_cast<uint32_t*>(E + a.slice_words);
    const SegTable tab{t32, t32 + (HAMMING_SEG_MAX_T + 1), t32 + 2 * (HAMMING_SEG_MAX_T + 1)};

    const hamming_seg_packet d = a.descs[pk];
    const uint32_t M = d.msg_bytes, t = d.t;
    const uint32_t total = build_table(M, t, a.max_msg_bytes, lane, tab);
    const uint64_t ew = (uint64_t(total) + 63) / 64, mw = (uint64_t(M) + 7) / 8;
    const bool ok = total != 0 && d.enc_word_off <= a.enc_words && ew <= a.enc_words - d.enc_word_off &&
                    d.msg_word_off <= a.msg_words && mw <= a.msg_words - d.msg_word_off;
    if (!ok) {
        if (a.status && lane == 0) a.status[pk] = HAMMING_SEG_INVALID;
        return;
    }
    uint64_t* Mw = E + enc_slice_words(a.max_msg_bytes);
    const uint64_t* src = a.msg + d.msg_word_off;
    for (uint32_t w = lane; w < mw; w += 64) Mw[w] = src[w];
    if (lane < 2) {
        Mw[mw + lane] = 0;
        E[ew + lane] = 0;
    }
    wave_sync();

    // message bits into their positions, checksum positions left 0
    for (uint32_t e = lane; e < ew; e += 64) {
        uint32_t b = 64u * e;
        const uint32_t end = min(b + 64u, total);
        uint32_t i = 0;
        while (i + 1 < t && tab.o[i + 1] <= b) ++i;
        uint64_t acc = 0;
        while (b < end) {
            const uint32_t o = tab.o[i], n = tab.o[i + 1] - o;
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
            uint64_t v = read_bits64(Mw, uint64_t(tab.K[i]) + p - j - 2u);
            if (len < 64) v &= (uint64_t(1) << len) - 1;
            acc |= v << (b - 64u * e);
            b += len;
        }
        E[e] = acc;
    }
    wave_sync();

    // checksum position 2^j takes bit j of the syndrome of the message bits alone
    uint32_t my_s = 0;
    for (uint32_t i = 0; i < t; ++i) {
        const uint32_t o = tab.o[i];
        const uint32_t s = segment_syndrome(E, o, tab.o[i + 1] - o, lane);
        if (lane == i) my_s = s;
    }
    wave_sync();
    if (lane < t) {
        const uint32_t o = tab.o[lane];
        for (uint32_t j = 0; my_s >> j; ++j) {
            if (!((my_s >> j) & 1)) continue;
            const uint32_t bit = o + (1u << j) - 1u;
            atomicOr(reinterpret_cast<unsigned long long*>(&E[bit >> 6]), 1ull << (bit & 63));
        }
    }
    if (a.status && lane == 0) a.status[pk] = 0;
    wave_sync();
    uint64_t* dst = const_cast<uint64_t*>(a.enc) + d.enc_word_off;
    for (uint32_t w = lane; w < ew; w += 64) __builtin_nontemporal_store(E[w], dst + w);
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

int hamming_decode_segmented(const uint64_t* enc_arena, uint64_t enc_words, const hamming_seg_packet* descs,
                             uint32_t n_packets, uint32_t max_msg_bytes, uint64_t* msg_arena, uint64_t msg_words,
                             uint16_t* syndromes, uint64_t syndrome_count, uint8_t* status, hipStream_t stream)
{
    int rc = check_common(enc_arena, descs, n_packets, msg_arena, max_msg_bytes);
    if (rc != HAMMING_OK || n_packets == 0) return rc;
    if (syndromes && (reinterpret_cast<uintptr_t>(syndromes) & 1u)) return HAMMING_EALIGN;
    SegArgs a{enc_arena, enc_words, descs, n_packets, max_msg_bytes, msg_arena, msg_words,
              syndromes, syndromes ? syndrome_count : 0, status, enc_slice_words(max_msg_bytes)};
    const size_t lds = size_t(kSegWaves) * (a.slice_words + kTableWords) * 8;
    const uint32_t blocks = (n_packets + kSegWaves - 1) / kSegWaves;
    hipLaunchKernelGGL(seg_decode_kernel, dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
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
    const size_t lds = size_t(kSegWaves) * (a.slice_words + kTableWords) * 8;
    const uint32_t blocks = (n_packets + kSegWaves - 1) / kSegWaves;
    hipLaunchKernelGGL(seg_encode_kernel, dim3(blocks), dim3(64 * kSegWaves), lds, stream, a);
    return hipGetLastError() == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE;
}

}  // extern "C"

/*
 * Segmented-packet Hamming decoder oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, bit-by-bit CPU implementation of the paper's own packet
 * workload: the splitter cuts an encoded packet H into t segments H_1..H_t,
 * each segment is decoded on its own (error detection, error correction,
 * redundancy removal) and the merger concatenates the recovered message
 * segments M_1..M_t into the packet M (Sec. II, Fig. 1).  Each segment is a
 * shortened Hamming codeword whose number of checksum bits r(H_i) depends on
 * its length (Sec. III.A, III.C).  Only the test suite and the bench's
 * CPU-baseline leg may load this code; the product library never does and
 * shares nothing with it.
 *
 * Readings of the paper that every function below follows:
 *   - A packet carries M message bytes = 8M message bits, split into t
 *     segments of k_i message bits: k_i = floor(8M/t), plus one for the first
 *     (8M mod t) segments.  Segment i holds message bits [K_i, K_i + k_i) of
 *     the packet, K_i = k_0 + ... + k_{i-1}.
 *   - r_i is the smallest r >= 2 with 2^r - 1 - r >= k_i; the segment has
 *     n_i = k_i + r_i positions 1..n_i, checksum bits at the positions 2^j
 *     (j < r_i) and message bits at the other positions, in ascending order.
 *     This is the shortened code of the paper's worked example, whose 11-bit
 *     segment has 4 checksum bits.
 *   - The encoded packet is the dense LSB-first bit string H_1 H_2 ... H_t:
 *     position p of segment i is bit o_i + p - 1, o_i = n_0 + ... + n_{i-1}.
 *   - Error detection: checksum bit C[j] is the XOR of the bits of index set
 *     I_j = { p in [1, n_i] : bit j of p is 1 }, j = 0..r_i-1; the syndrome is
 *     s = sum of C[j] 2^j.
 *   - s = 0: no error.  1 <= s <= n_i: bit s is flipped (corrected).
 *     s > n_i: no position of the shortened segment explains the checksum;
 *     the segment is reported as detected-uncorrectable and its bits are
 *     passed on as received.
 *   - The decoded packet is M bytes, message bit K_i + m of the packet being
 *     bit (K_i + m) % 8 of byte (K_i + m) / 8.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SEG_MAX_T 32
#define SEG_MAX_K 65519   /* 2^16 - 1 - 16: every segment fits r <= 16 */

int oracle_index_set(int n, int j, int32_t *out);   /* hamming_oracle.c */

static int is_pow2(uint32_t p) { return p > 0 && (p & (p - 1)) == 0; }

static int get_bit(const uint8_t *s, uint64_t b) { return (s[b / 8] >> (b % 8)) & 1; }

static void put_bit(uint8_t *s, uint64_t b, int v)
{
    if (v)
        s[b / 8] |= (uint8_t)(1u << (b % 8));
    else
        s[b / 8] &= (uint8_t)~(1u << (b % 8));
}

/*
 * Segment layout of a packet of msg_bytes bytes in t segments.  Fills k, r,
 * n (t entries each, or NULL) and returns the total number of encoded bits,
 * or -1 for an unsupported packet (t outside [1, 32], fewer message bits than
 * segments, or a segment longer than SEG_MAX_K message bits).
 */
int64_t oracle_seg_layout(uint32_t msg_bytes, uint32_t t, uint32_t *k, uint32_t *r, uint32_t *n)
{
    if (t < 1 || t > SEG_MAX_T) return -1;
    const uint64_t bits = 8ull * msg_bytes;
    if (bits < t) return -1;
    int64_t total = 0;
    for (uint32_t i = 0; i < t; ++i) {
        uint64_t ki = bits / t + (i < bits % t ? 1 : 0);
        if (ki > SEG_MAX_K) return -1;
        uint32_t ri = 2;
        while (((uint64_t)1 << ri) - 1 - ri < ki) ++ri;
        if (k) k[i] = (uint32_t)ki;
        if (r) r[i] = ri;
        if (n) n[i] = (uint32_t)ki + ri;
        total += (int64_t)ki + ri;
    }
    return total;
}

/* Syndrome of one segment y[1..n] with r checksum bits (Algorithm 1). */
static uint32_t segment_checksum(const uint8_t *y, uint32_t n, uint32_t r, int32_t *scratch)
{
    uint32_t s = 0;
    for (uint32_t j = 0; j < r; ++j) {
        int cnt = oracle_index_set((int)n, (int)j, scratch);
        int c = 0;
        for (int q = 0; q < cnt; ++q) c ^= y[scratch[q]];
        s |= (uint32_t)c << j;
    }
    return s;
}

typedef struct {
    uint32_t k[SEG_MAX_T], r[SEG_MAX_T], n[SEG_MAX_T];
    uint32_t t, msg_bytes;
    uint64_t enc_bits;
} seg_layout;

static int make_layout(uint32_t msg_bytes, uint32_t t, seg_layout *L)
{
    int64_t tot = oracle_seg_layout(msg_bytes, t, L->k, L->r, L->n);
    if (tot < 0) return -1;
    L->t = t;
    L->msg_bytes = msg_bytes;
    L->enc_bits = (uint64_t)tot;
    return 0;
}

/* Decode one packet; y and scratch hold room for the longest segment. */
static int decode_packet(const seg_layout *L, const uint8_t *enc, uint8_t *msg, uint16_t *syn, uint8_t *status,
                         uint8_t *y, int32_t *scratch)
{
    uint64_t o = 0, K = 0;
    uint8_t st = 0;
    memset(msg, 0, L->msg_bytes);
    for (uint32_t i = 0; i < L->t; ++i) {
        const uint32_t n = L->n[i];
        /* splitter: segment i's positions 1..n */
        y[0] = 0;
        for (uint32_t p = 1; p <= n; ++p) y[p] = (uint8_t)get_bit(enc, o + p - 1);
        /* error detection */
        const uint32_t s = segment_checksum(y, n, L->r[i], scratch);
        /* error correction */
        if (s >= 1 && s <= n) {
            y[s] ^= 1;
            if (st < 1) st = 1;
        } else if (s > n) {
            st = 2;
        }
        if (syn) syn[i] = (uint16_t)s;
        /* redundancy removal and merge */
        uint64_t m = 0;
        for (uint32_t p = 1; p <= n; ++p) {
            if (is_pow2(p)) continue;
            put_bit(msg, K + m, y[p]);
            ++m;
        }
        o += n;
        K += L->k[i];
    }
    if (status) *status = st;
    return 0;
}

static void encode_packet(const seg_layout *L, const uint8_t *msg, uint8_t *enc, uint64_t enc_bytes, uint8_t *c,
                          int32_t *scratch)
{
    uint64_t o = 0, K = 0;
    memset(enc, 0, enc_bytes);
    for (uint32_t i = 0; i < L->t; ++i) {
        const uint32_t n = L->n[i];
        uint64_t m = 0;
        for (uint32_t p = 1; p <= n; ++p) {
            c[p] = 0;
            if (!is_pow2(p)) c[p] = (uint8_t)get_bit(msg, K + m++);
        }
        /* checksum bit 2^j makes the XOR over I_j zero */
        for (uint32_t j = 0; j < L->r[i]; ++j) {
            int cnt = oracle_index_set((int)n, (int)j, scratch);
            int par = 0;
            for (int q = 0; q < cnt; ++q) par ^= c[scratch[q]];
            c[1u << j] = (uint8_t)par;
        }
        for (uint32_t p = 1; p <= n; ++p) put_bit(enc, o + p - 1, c[p]);
        o += n;
        K += L->k[i];
    }
}

/*
 * Decode one packet.
 *   enc        : the encoded packet, at least ceil(enc_bits / 8) bytes.
 *   msg_out    : msg_bytes bytes, fully written.
 *   syndrome_out: t entries (the syndrome s of each segment), or NULL.
 *   status_out : 0 clean, 1 at least one segment corrected, 2 at least one
 *                segment detected-uncorrectable; or NULL.
 * Returns 0, or -1 for a bad argument.
 */
int oracle_seg_decode(const uint8_t *enc, uint64_t enc_bytes, uint32_t msg_bytes, uint32_t t, uint8_t *msg_out,
                      uint16_t *syndrome_out, uint8_t *status_out)
{
    seg_layout L;
    if (make_layout(msg_bytes, t, &L) || !enc || !msg_out) return -1;
    if (enc_bytes < (L.enc_bits + 7) / 8) return -1;
    uint32_t nmax = 0;
    for (uint32_t i = 0; i < t; ++i)
        if (L.n[i] > nmax) nmax = L.n[i];
    uint8_t *y = malloc(nmax + 1);
    int32_t *scratch = malloc(sizeof(int32_t) * (nmax + 1));
    int rc = -1;
    if (y && scratch) rc = decode_packet(&L, enc, msg_out, syndrome_out, status_out, y, scratch);
    free(y);
    free(scratch);
    return rc;
}

/* Encode one packet of msg_bytes bytes into enc_out (enc_bytes >= the
 * encoded length rounded up to bytes; bytes beyond it are written 0). */
int oracle_seg_encode(const uint8_t *msg, uint32_t msg_bytes, uint32_t t, uint8_t *enc_out, uint64_t enc_bytes)
{
    seg_layout L;
    if (make_layout(msg_bytes, t, &L) || !msg || !enc_out) return -1;
    if (enc_bytes < (L.enc_bits + 7) / 8) return -1;
    uint8_t *c = malloc(SEG_MAX_K + 17 + 1);
    int32_t *scratch = malloc(sizeof(int32_t) * (SEG_MAX_K + 17 + 1));
    if (!c || !scratch) {
        free(c);
        free(scratch);
        return -1;
    }
    encode_packet(&L, msg, enc_out, enc_bytes, c, scratch);
    free(c);
    free(scratch);
    return 0;
}

/* ---- many packets of one shape, for test inputs and the CPU baseline ---- */

typedef struct {
    const seg_layout *L;
    const uint8_t *in;
    uint8_t *out;
    uint64_t in_stride, out_stride;
    uint16_t *syn;
    uint8_t *status;
    uint64_t begin, end;
    int encode;
} seg_job;

static void *seg_range(void *arg)
{
    seg_job *jb = (seg_job *)arg;
    const seg_layout *L = jb->L;
    uint8_t *buf = malloc(SEG_MAX_K + 17 + 1);
    int32_t *scratch = malloc(sizeof(int32_t) * (SEG_MAX_K + 17 + 1));
    if (!buf || !scratch) {
        free(buf);
        free(scratch);
        return (void *)1;
    }
    for (uint64_t q = jb->begin; q < jb->end; ++q) {
        if (jb->encode)
            encode_packet(L, jb->in + q * jb->in_stride, jb->out + q * jb->out_stride, jb->out_stride, buf, scratch);
        else
            decode_packet(L, jb->in + q * jb->in_stride, jb->out + q * jb->out_stride,
                          jb->syn ? jb->syn + q * L->t : NULL, jb->status ? jb->status + q : NULL, buf, scratch);
    }
    free(buf);
    free(scratch);
    return NULL;
}

/*
 * Decode (encode = 0) or encode (encode = 1) n_packets packets of one shape
 * stored at fixed strides: packet q's input at in + q*in_stride, its output at
 * out + q*out_stride (decode: in_stride >= encoded bytes, out_stride >=
 * msg_bytes; encode: the reverse).  syndrome_out holds t entries per packet.
 */
int oracle_seg_many(int encode, const uint8_t *in, uint64_t in_stride, uint64_t n_packets, uint32_t msg_bytes,
                    uint32_t t, uint8_t *out, uint64_t out_stride, uint16_t *syndrome_out, uint8_t *status_out,
                    int nthreads)
{
    seg_layout L;
    if (make_layout(msg_bytes, t, &L)) return -1;
    const uint64_t enc_bytes = (L.enc_bits + 7) / 8;
    if (encode ? (in_stride < msg_bytes || out_stride < enc_bytes) : (in_stride < enc_bytes || out_stride < msg_bytes))
        return -1;
    if (n_packets == 0) return 0;
    if (!in || !out) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if ((uint64_t)nthreads > n_packets) nthreads = (int)n_packets;
    seg_job jobs[64];
    pthread_t th[64];
    const uint64_t per = (n_packets + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int q = 0; q < nthreads; ++q) {
        jobs[q] = (seg_job){&L, in, out, in_stride, out_stride, syndrome_out, status_out, 0, 0, encode};
        jobs[q].begin = (uint64_t)q * per < n_packets ? (uint64_t)q * per : n_packets;
        jobs[q].end = (uint64_t)(q + 1) * per < n_packets ? (uint64_t)(q + 1) * per : n_packets;
    }
    int launched = 0, failed = 0;
    for (int q = 1; q < nthreads; ++q) {
        if (pthread_create(&th[q], NULL, seg_range, &jobs[q]) != 0) break;
        ++launched;
    }
    if (seg_range(&jobs[0])) failed = 1;
    for (int q = 1; q <= launched; ++q) {
        void *res = NULL;
        pthread_join(th[q], &res);
        if (res) failed = 1;
    }
    for (int q = launched + 1; q < nthreads; ++q)
        if (seg_range(&jobs[q])) failed = 1;
    return failed ? -1 : 0;
}

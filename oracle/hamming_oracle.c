/*
 * Hamming decoder oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, bit-by-bit CPU implementation of what the decode path
 * computes, written from Islam, Kim & Kim, "Computationally Efficient
 * Implementation of a Hamming Code Decoder using Graphics Processing Unit"
 * (J. Communications and Networks, 2014).  Only the test suite, the smoke
 * check and the bench's CPU-baseline leg may load this library; the product
 * decode path never does, and this file shares no code, header, table or
 * helper with the HIP library.
 *
 * Conventions (the readings of the paper that every function below follows):
 *   - r parity bits, n = 2^r - 1 code bits, k = n - r message bits, r in [3,7].
 *   - Bits are addressed by position p = 1..n.  In storage, position p is bit
 *     (p-1) of a little-endian sequence of 64-bit words: one word per codeword
 *     for r <= 6, two words for r = 7 (word 0 = positions 1..64, word 1 =
 *     positions 65..127).  Storage bits at or above n are padding and ignored.
 *   - Index set I_j = { p in [1,n] : bit j of p is 1 }, j = 0..r-1 (the sets
 *     the paper prints for an 11-bit segment in Sec. III.A).
 *   - The parity (checksum) bits sit at positions 2^j; the message bits fill
 *     the remaining positions in ascending order.
 *   - The decoded message of codeword i occupies bits [i*k, i*k+k) of a dense
 *     LSB-first byte stream (the merger of Sec. II); bits after the last
 *     message up to the end of the last 64-bit word are 0.
 *   - errpos = the checksum value s read as a position (0 = no error).  Two or
 *     more flipped bits are handled by the same rule: position s is flipped.
 *
 * Decode follows the paper's decomposition (Sec. II, Fig. 1; Sec. III.C):
 *   error detection (checksum over each index set, Algorithm 1) ->
 *   error correction -> redundancy removal -> merge.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_R 7
#define ORACLE_MAX_N 127

/* ---- code parameters ---------------------------------------------------- */

static int code_n(int r) { return (1 << r) - 1; }
static int code_k(int r) { return (1 << r) - 1 - r; }
static int words_per_cw(int r) { return r == 7 ? 2 : 1; }

static int is_power_of_two(int p) { return p > 0 && (p & (p - 1)) == 0; }

int oracle_code_n(int r) { return (r >= 3 && r <= ORACLE_MAX_R) ? code_n(r) : -1; }
int oracle_code_k(int r) { return (r >= 3 && r <= ORACLE_MAX_R) ? code_k(r) : -1; }

/* Size in bytes of the decoded stream for n_cw codewords: whole 64-bit words. */
uint64_t oracle_data_bytes(uint64_t n_cw, int r)
{
    uint64_t bits = n_cw * (uint64_t)code_k(r);
    return ((bits + 63) / 64) * 8;
}

/*
 * Index set I_j of a segment of n bits (Sec. III.A): every position p in
 * [1, n] whose binary expansion has bit j set, in ascending order.
 * Writes the positions to out (room for n entries) and returns their count.
 */
int oracle_index_set(int n, int j, int32_t *out)
{
    int count = 0;
    if (n < 1 || j < 0 || j > 30) return -1;
    for (int p = 1; p <= n; ++p) {
        if ((p >> j) & 1) out[count++] = p;
    }
    return count;
}

/* ---- bit access ----------------------------------------------------------- */

static int get_storage_bit(const uint64_t *words, int bit)
{
    return (int)((words[bit / 64] >> (bit % 64)) & 1u);
}

static int get_stream_bit(const uint8_t *stream, uint64_t bit)
{
    return (stream[bit / 8] >> (bit % 8)) & 1;
}

static void set_stream_bit(uint8_t *stream, uint64_t bit)
{
    stream[bit / 8] |= (uint8_t)(1u << (bit % 8));
}

/* ---- one codeword, as an array of bits y[1..n] -------------------------- */

/*
 * Per-r tables: the index sets of Sec. III.A and the ascending list of
 * message positions (every position that is not a power of two).
 */
typedef struct {
    int r, n, k;
    int set_len[ORACLE_MAX_R];
    int set_pos[ORACLE_MAX_R][ORACLE_MAX_N];
    int msg_pos[ORACLE_MAX_N];
} code_tables;

static void build_tables(int r, code_tables *t)
{
    t->r = r;
    t->n = code_n(r);
    t->k = code_k(r);
    for (int j = 0; j < r; ++j) {
        int32_t tmp[ORACLE_MAX_N];
        t->set_len[j] = oracle_index_set(t->n, j, tmp);
        for (int q = 0; q < t->set_len[j]; ++q) t->set_pos[j][q] = tmp[q];
    }
    int m = 0;
    for (int p = 1; p <= t->n; ++p)
        if (!is_power_of_two(p)) t->msg_pos[m++] = p;
}

/*
 * Error detection: checksum bit C[j] is the modulo-2 sum (XOR) of the bits
 * selected by index set I_j (Algorithm 1, steps 2-5).  The checksum vector,
 * read as a binary number with C[j] as bit j, is returned.
 */
static int checksum(const code_tables *t, const uint8_t *y)
{
    int s = 0;
    for (int j = 0; j < t->r; ++j) {
        int c = 0;
        for (int q = 0; q < t->set_len[j]; ++q) c ^= y[t->set_pos[j][q]];
        s |= c << j;
    }
    return s;
}

/*
 * Decode one received word y[1..n] in place (Sec. II): ED, then EC (flip the
 * bit the checksum points at), then RR (keep the message positions, in
 * order).  Writes k message bits to msg[0..k-1] and returns the error
 * position (0 when the checksum is zero).
 */
static int decode_word(const code_tables *t, uint8_t *y, uint8_t *msg)
{
    int s = checksum(t, y);             /* error detection  */
    if (s != 0) y[s] ^= 1;              /* error correction */
    for (int m = 0; m < t->k; ++m)      /* redundancy removal */
        msg[m] = y[t->msg_pos[m]];
    return s;
}

/*
 * Encode one message msg[0..k-1] into c[1..n]: message bits at the message
 * positions, then each parity position 2^j set so that the XOR over I_j is 0.
 */
static void encode_word(const code_tables *t, const uint8_t *msg, uint8_t *c)
{
    for (int p = 1; p <= t->n; ++p) c[p] = 0;
    for (int m = 0; m < t->k; ++m) c[t->msg_pos[m]] = msg[m];
    for (int j = 0; j < t->r; ++j) {
        int parity = 0;
        for (int q = 0; q < t->set_len[j]; ++q) parity ^= c[t->set_pos[j][q]];
        c[1 << j] = (uint8_t)parity;   /* c[2^j] was 0, so parity excludes it */
    }
}

/* ---- whole packets -------------------------------------------------------- */

typedef struct {
    const code_tables *t;
    const uint64_t *cw;       /* decode input / encode output */
    uint64_t *cw_out;
    const uint8_t *stream_in; /* encode input */
    uint8_t *stream_out;      /* decode output */
    uint8_t *errpos_out;
    uint64_t begin, end;      /* codeword range */
} job;

static void *decode_range(void *arg)
{
    job *jb = (job *)arg;
    const code_tables *t = jb->t;
    const int wpc = words_per_cw(t->r);
    uint8_t y[ORACLE_MAX_N + 1];
    uint8_t msg[ORACLE_MAX_N];
    for (uint64_t i = jb->begin; i < jb->end; ++i) {
        const uint64_t *w = jb->cw + i * (uint64_t)wpc;
        y[0] = 0;
        for (int p = 1; p <= t->n; ++p) y[p] = (uint8_t)get_storage_bit(w, p - 1);
        int s = decode_word(t, y, msg);
        if (jb->errpos_out) jb->errpos_out[i] = (uint8_t)s;
        /* merge: message m of codeword i goes to stream bit i*k + m */
        for (int m = 0; m < t->k; ++m)
            if (msg[m]) set_stream_bit(jb->stream_out, i * (uint64_t)t->k + (uint64_t)m);
    }
    return NULL;
}

static void *encode_range(void *arg)
{
    job *jb = (job *)arg;
    const code_tables *t = jb->t;
    const int wpc = words_per_cw(t->r);
    uint8_t c[ORACLE_MAX_N + 1];
    uint8_t msg[ORACLE_MAX_N];
    for (uint64_t i = jb->begin; i < jb->end; ++i) {
        for (int m = 0; m < t->k; ++m)
            msg[m] = (uint8_t)get_stream_bit(jb->stream_in, i * (uint64_t)t->k + (uint64_t)m);
        encode_word(t, msg, c);
        uint64_t *w = jb->cw_out + i * (uint64_t)wpc;
        for (int q = 0; q < wpc; ++q) w[q] = 0;
        for (int p = 1; p <= t->n; ++p)
            if (c[p]) w[(p - 1) / 64] |= (uint64_t)1 << ((p - 1) % 64);
    }
    return NULL;
}

/* Split [0, n_cw) into nthreads ranges whose boundaries are multiples of 64
 * codewords, so that every thread writes whole bytes of the output stream. */
static int run_parallel(void *(*fn)(void *), job proto, uint64_t n_cw, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    uint64_t groups = (n_cw + 63) / 64;
    if ((uint64_t)nthreads > groups) nthreads = groups ? (int)groups : 1;
    job jobs[256];
    pthread_t th[256];
    uint64_t per = (groups + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    int launched = 0;
    for (int q = 0; q < nthreads; ++q) {
        jobs[q] = proto;
        jobs[q].begin = (uint64_t)q * per * 64;
        jobs[q].end = (uint64_t)(q + 1) * per * 64;
        if (jobs[q].begin > n_cw) jobs[q].begin = n_cw;
        if (jobs[q].end > n_cw) jobs[q].end = n_cw;
    }
    if (nthreads == 1) {
        fn(&jobs[0]);
        return 0;
    }
    for (int q = 0; q < nthreads; ++q) {
        if (pthread_create(&th[q], NULL, fn, &jobs[q]) != 0) break;
        ++launched;
    }
    for (int q = 0; q < launched; ++q) pthread_join(th[q], NULL);
    for (int q = launched; q < nthreads; ++q) fn(&jobs[q]);   /* thread creation failed: run inline */
    return 0;
}

/*
 * Decode a packet of n_cw received words.
 *   cw         : n_cw words (2*n_cw for r = 7), layout as above.
 *   data_out   : data_bytes = oracle_data_bytes(n_cw, r) bytes; fully written.
 *   errpos_out : n_cw bytes, or NULL.
 * Returns 0, or -1 for a bad argument.
 */
int oracle_decode(const uint64_t *cw, uint64_t n_cw, int r,
                  uint8_t *data_out, uint64_t data_bytes,
                  uint8_t *errpos_out, int nthreads)
{
    if (r < 3 || r > ORACLE_MAX_R) return -1;
    if (data_bytes < oracle_data_bytes(n_cw, r)) return -1;
    if (n_cw && (!cw || !data_out)) return -1;
    if (data_out) memset(data_out, 0, (size_t)data_bytes);
    if (n_cw == 0) return 0;
    code_tables t;
    build_tables(r, &t);
    job proto;
    memset(&proto, 0, sizeof proto);
    proto.t = &t;
    proto.cw = cw;
    proto.stream_out = data_out;
    proto.errpos_out = errpos_out;
    return run_parallel(decode_range, proto, n_cw, nthreads);
}

/*
 * Encode n_cw messages read from a dense LSB-first stream (message of
 * codeword i at bits [i*k, i*k+k)) into codewords; padding bits are 0.
 */
int oracle_encode(const uint8_t *stream, uint64_t n_cw, int r,
                  uint64_t *cw_out, int nthreads)
{
    if (r < 3 || r > ORACLE_MAX_R) return -1;
    if (n_cw && (!stream || !cw_out)) return -1;
    if (n_cw == 0) return 0;
    code_tables t;
    build_tables(r, &t);
    job proto;
    memset(&proto, 0, sizeof proto);
    proto.t = &t;
    proto.cw_out = cw_out;
    proto.stream_in = stream;
    return run_parallel(encode_range, proto, n_cw, nthreads);
}

/*
 * hamming.h -- C ABI of the MI355X (gfx950) Hamming decoder library
 * (libhamming.so).
 *
 * The operation is the per-codeword decode of Islam, Kim & Kim, "Computationally
 * Efficient Implementation of a Hamming Code Decoder using Graphics Processing
 * Unit" (J. Communications and Networks, 2014): error detection by a modulo-2
 * checksum over each index set (Sec. III.C, Algorithm 1; index sets as in
 * Sec. III.A), correction of the bit the checksum names, removal of the
 * checksum bits and merging of the recovered messages (Sec. II, Fig. 1), run
 * over whole packets of codewords.
 *
 * Codes.  r parity bits, r in [3, 7]: n = 2^r - 1 code bits and k = n - r
 * message bits per codeword, i.e. Hamming(7,4), (15,11), (31,26), (63,57) and
 * (127,120).
 *
 * Codeword storage.  Position p (1..n) of a codeword is bit p-1 of a
 * little-endian sequence of 64-bit words: one word per codeword for r <= 6,
 * two for r = 7 (word 0 holds positions 1..64, word 1 positions 65..127).
 * Checksum bits sit at positions 2^j, message bits fill the other positions
 * in ascending order.  Storage bits at or above n are padding: ignored on
 * input, never written.
 *
 * Decoded output.
 *   data_out   : dense LSB-first bit stream; message bit m of codeword i is
 *                stream bit i*k + m (bit (i*k+m)%8 of byte (i*k+m)/8).  The
 *                stream is padded with zero bits to a whole number of 64-bit
 *                words: hamming_data_bytes(n_cw, r) bytes are written.
 *   errpos_out : one byte per codeword, the checksum value s (0 = no error
 *                detected, else the position that was flipped).
 * A received word with two or more flipped bits is decoded by the same rule
 * (position s is flipped), which yields the unique codeword within distance 1
 * of the received word: Hamming codes are perfect, so every received word
 * decodes and the decoder never reports "uncorrectable".
 *
 * Memory and ownership.  All data pointers passed to the decode and encode
 * calls are device pointers owned by the caller; the library never frees or
 * keeps them.  Inputs are never written.  Calls are asynchronous on the given
 * stream (NULL = the default stream) and return once the work is enqueued;
 * faults during execution surface at the caller's next synchronisation.  Calls
 * on different streams may run concurrently; the library keeps no per-call
 * global state.
 *
 * Errors.  Every call validates its arguments on the host before any launch
 * and returns one of the status codes below synchronously; nothing is enqueued
 * when the status is not HAMMING_OK.
 */
#ifndef HAMMING_H
#define HAMMING_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum hamming_status {
    HAMMING_OK = 0,
    HAMMING_EINVAL = -1,   /* r out of [3,7], NULL pointer, bad descriptor field */
    HAMMING_EALIGN = -2,   /* a pointer breaks the alignment stated for it */
    HAMMING_ERANGE = -3,   /* size too large, or an offset outside its arena */
    HAMMING_ENOMEM = -4,   /* a caller-provided buffer is too small */
    HAMMING_EDEVICE = -5   /* the HIP runtime refused the launch */
};

/* Largest n_cw accepted by one call (2^40 codewords). */
#define HAMMING_MAX_CODEWORDS ((uint64_t)1 << 40)

/* Number of message bits k of the code with r parity bits; -1 if r is not in
 * [3,7]. */
int hamming_message_bits(int r);

/* Bytes of the decoded stream for n_cw codewords: ceil(n_cw*k/64)*8.  Returns
 * 0 for an invalid r or n_cw above HAMMING_MAX_CODEWORDS. */
uint64_t hamming_data_bytes(uint64_t n_cw, int r);

/*
 * Decode one packet of n_cw codewords of the code with r parity bits
 * (error detection, correction, redundancy removal and merge; Sec. II and
 * Sec. III.C).
 *   codewords  : device, n_cw words (2*n_cw for r = 7), 8-byte aligned.
 *   n_cw       : number of codewords; 0 is valid and enqueues nothing.
 *   r          : 3..7.
 *   data_out   : device, hamming_data_bytes(n_cw, r) bytes, 8-byte aligned.
 *   errpos_out : device, n_cw bytes, any alignment; NULL = not written.
 *   stream     : HIP stream to enqueue on.
 * Returns HAMMING_OK, HAMMING_EINVAL (bad r, NULL codewords/data_out with
 * n_cw > 0), HAMMING_EALIGN, HAMMING_ERANGE (n_cw too large) or
 * HAMMING_EDEVICE.
 */
int hamming_decode(const uint64_t *codewords, uint64_t n_cw, int r,
                   void *data_out, uint8_t *errpos_out, hipStream_t stream);

/*
 * Encode n_cw messages (the transmitter's half of Sec. II): the message of
 * codeword i is read from bits [i*k, i*k+k) of the dense LSB-first stream
 * data_in, placed at the message positions, and checksum position 2^j is set
 * so that the XOR over index set I_j is 0.  Padding bits are written as 0.
 *   data_in       : device, at least ceil(n_cw*k/64)*8 bytes, 8-byte aligned.
 *   codewords_out : device, n_cw words (2*n_cw for r = 7), 8-byte aligned.
 * Same status codes as hamming_decode.
 */
int hamming_encode(const void *data_in, uint64_t n_cw, int r,
                   uint64_t *codewords_out, hipStream_t stream);

/*
 * Launch shape of the plain decode for the code with r parity bits (a tuning
 * knob, no effect on results).  lane_codewords is the number of consecutive
 * codewords one lane decodes: 2, 4, 8 or 16, with lane_codewords*k >= 32.
 * max_blocks caps the workgroups of one launch (waves then loop over tiles);
 * 0 launches one wave per tile.  The shape is process-wide state read at each
 * hamming_decode call; set it before decoding.  Returns HAMMING_OK,
 * HAMMING_EINVAL or HAMMING_ERANGE.
 */
int hamming_plain_config_set(int r, int lane_codewords, uint64_t max_blocks);
int hamming_plain_config_get(int r, int *lane_codewords, uint64_t *max_blocks);

/* Static, human-readable text for a status code. */
const char *hamming_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* HAMMING_H */

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
 * 0 launches one wave per tile.  xcd_chunk (1..2^20) is the number of
 * consecutive workgroups each of the 8 XCDs takes in turn (1 = the hardware's
 * round-robin order).  The shape is process-wide state read at each
 * hamming_decode call; set it before decoding.  Returns HAMMING_OK,
 * HAMMING_EINVAL or HAMMING_ERANGE.
 */
int hamming_plain_config_set(int r, int lane_codewords, uint64_t max_blocks, uint32_t xcd_chunk);
int hamming_plain_config_get(int r, int *lane_codewords, uint64_t *max_blocks, uint32_t *xcd_chunk);

/* Workgroups (of 256 work-items) that hamming_decode would launch for n_cw
 * codewords of code r under the current launch shape: one wave per tile of
 * 64*lane_codewords codewords, capped by max_blocks and by the 2^32-1
 * work-items a dispatch can hold; waves loop over the tiles beyond the grid.
 * Host-only and informative (tests, capacity planning); 0 for an invalid r,
 * n_cw = 0 or n_cw above HAMMING_MAX_CODEWORDS. */
uint64_t hamming_decode_grid(uint64_t n_cw, int r);

/* ---- batched decode ------------------------------------------------------ */

/*
 * One packet of a batch (40 bytes).  The batched decode applies exactly the
 * plain decode to every packet, so each packet's outputs are byte-identical
 * to a hamming_decode call on that packet alone.
 *   in_word_off   : first 64-bit word of the packet's codewords in cw_arena.
 *   n_cw          : codewords in the packet; 0 is allowed (nothing written).
 *   r             : 3..7.
 *   flags         : reserved, must be 0.
 *   data_word_off : first 64-bit word of the packet's message stream in
 *                   data_arena; hamming_data_bytes(n_cw, r)/8 words are written.
 *   errpos_off    : first byte of the packet's n_cw errpos bytes in
 *                   errpos_arena, or HAMMING_NO_ERRPOS.
 * Output ranges of different packets must not overlap (hamming_batch_layout
 * produces disjoint ones); input ranges may.
 */
typedef struct hamming_packet {
    uint64_t in_word_off;
    uint64_t n_cw;
    uint32_t r;
    uint32_t flags;
    uint64_t data_word_off;
    uint64_t errpos_off;
} hamming_packet;

#define HAMMING_NO_ERRPOS UINT64_MAX
#define HAMMING_MAX_BATCH (1u << 24)

/*
 * Host helper: fill data_word_off and errpos_off of n descriptors (host
 * memory) with disjoint, consecutive ranges in packet order, each rounded up to
 * 16 bytes; in_word_off, n_cw and r are read, not changed.  Writes the arena
 * sizes the batch needs to *data_words (64-bit words) and *errpos_bytes.
 * Returns HAMMING_OK, HAMMING_EINVAL (NULL pointer, bad r or flags) or
 * HAMMING_ERANGE (n above HAMMING_MAX_BATCH or n_cw too large); on error no
 * descriptor is changed.
 */
int hamming_batch_layout(hamming_packet *descs, uint32_t n, uint64_t *data_words,
                         uint64_t *errpos_bytes);

/* Recommended device workspace bytes of hamming_decode_batch for max_packets
 * packets: batch totals, tile prefix sums, a coarse tile-to-packet map and a
 * fine map with one entry per tile of any batch of up to
 * max(2^24, 4*max_packets) tiles.  0 if max_packets > HAMMING_MAX_BATCH. */
uint64_t hamming_batch_workspace_bytes(uint32_t max_packets);

/* Smallest workspace hamming_decode_batch accepts for max_packets packets (a
 * fine map of one entry).  Any size from this one up works: a fine map with
 * fewer entries than the batch has tiles groups 2^g tiles per entry, and each
 * wave then finds its tile's packet by probing the prefix sums 64 entries at
 * a time from the entry's packet on (slower, same results).  0 if max_packets
 * > HAMMING_MAX_BATCH. */
uint64_t hamming_batch_workspace_min_bytes(uint32_t max_packets);

/*
 * Batched decode: decode every packet of a device-resident descriptor array.
 * A planning kernel validates each descriptor, writes its status and computes
 * a prefix sum of tiles (64-codeword multiples aligned to each packet's
 * start); two more kernels build tile-to-packet maps; the decode kernel then
 * gives one tile to each wave in global tile order, so packets of any size and
 * r share the GPU as one stream of work.  On a non-NULL stream that is not
 * already capturing, the four kernels are captured once into a hipGraph
 * (cached per argument set) and replayed on later calls; the number of packets
 * is read on the device, so one graph serves every batch of up to max_packets
 * packets in the same arenas.
 *   cw_arena, cw_words     : device codeword arena and its size in 64-bit words.
 *   descs                  : device, max_packets descriptors, 8-byte aligned.
 *   n_packets_dev          : device uint32, packets to decode this call
 *                            (values above max_packets are clamped).
 *   max_codewords          : an upper bound on the total codewords of any batch
 *                            decoded with these arguments, used only to size the
 *                            grid; 0 derives one from cw_words (exact when
 *                            packets do not share input words).  Any value is
 *                            correct; a low one is slower, a high one launches
 *                            idle waves.
 *   data_arena, data_words : device message arena, 8-byte aligned, and its size.
 *   errpos_arena, errpos_bytes : device errpos arena and size (may be NULL/0
 *                            when every packet uses HAMMING_NO_ERRPOS).
 *   status_out             : device int32[max_packets] or NULL; per packet
 *                            HAMMING_OK, HAMMING_EINVAL (bad r or flags) or
 *                            HAMMING_ERANGE (a range outside its arena).  A
 *                            rejected packet is skipped; the others decode as
 *                            usual.
 *   workspace, workspace_bytes : device scratch, 8-byte aligned, at least
 *                            hamming_batch_workspace_min_bytes(max_packets)
 *                            (hamming_batch_workspace_bytes(max_packets) for the
 *                            exact map); owned by the caller, not shared by
 *                            concurrent calls.  Its first 64 bytes receive the
 *                            batch totals: tiles (uint64), packets (uint64),
 *                            then the log2 group sizes of the coarse and fine
 *                            maps (two uint32).
 * Returns HAMMING_OK, HAMMING_EINVAL, HAMMING_EALIGN, HAMMING_ERANGE,
 * HAMMING_ENOMEM (workspace too small) or HAMMING_EDEVICE.
 */
int hamming_decode_batch(const uint64_t *cw_arena, uint64_t cw_words,
                         const hamming_packet *descs, const uint32_t *n_packets_dev,
                         uint32_t max_packets, uint64_t max_codewords, uint64_t *data_arena,
                         uint64_t data_words, uint8_t *errpos_arena, uint64_t errpos_bytes,
                         int32_t *status_out, void *workspace, uint64_t workspace_bytes,
                         hipStream_t stream);

/*
 * Launch shape of the batched decode (a tuning knob, no effect on results):
 * schedule selects the per-r lane widths and occupancy (0..3); xcd_chunk (1..2^20) the
 * consecutive workgroups each of the 8 XCDs takes in turn (1 = hardware
 * order); grid_cap_blocks caps the decode kernel's workgroups (0 = no cap;
 * waves then loop over tiles); use_graph whether to capture and replay a
 * hipGraph (1) or launch directly (0).  Process-wide; set before decoding.
 * Returns HAMMING_OK or HAMMING_EINVAL.
 */
int hamming_batch_config_set(int schedule, uint32_t xcd_chunk, uint32_t grid_cap_blocks, int use_graph);
int hamming_batch_config_get(int *schedule, uint32_t *xcd_chunk, uint32_t *grid_cap_blocks, int *use_graph);

/*
 * Work unit of the batched decode kernels (a tuning knob, no effect on
 * results): a wave takes 2^tiles_log2 consecutive tiles of the batch's tile
 * order, finds the packet of the first once and decodes each packet's share
 * with the next tile's loads in flight (tiles_log2 in [0, 6], default 3).
 * The one-launch form for at most 16 served requests keeps one tile per
 * wave.  Process-wide; set before decoding (cached hipGraphs are keyed on
 * it).  Returns HAMMING_OK or HAMMING_EINVAL.
 */
int hamming_batch_chunk_set(uint32_t tiles_log2);
int hamming_batch_chunk_get(uint32_t *tiles_log2);

/* Workgroups of the batched decode kernel for these arguments of
 * hamming_decode_batch: one wave per chunk (hamming_batch_chunk_set) of the
 * largest batch they allow (min(cw_words/W, max_codewords/C) + max_packets
 * tiles, W and C the smallest input words and codewords of a tile under the
 * schedule in force: 256 and 128 for schedules 0-2, 512 and 256 for schedule
 * 3; max_codewords 0 = no hint), capped by grid_cap_blocks and by the 2^32-1
 * work-items a dispatch can hold.  Host-only and informative; 0 if max_packets is 0 or above
 * HAMMING_MAX_BATCH. */
uint64_t hamming_decode_batch_grid(uint64_t cw_words, uint32_t max_packets, uint64_t max_codewords);

/* Destroy the hipGraph executables hamming_decode_batch has cached (they
 * otherwise live until the process ends): waits for each cached graph's
 * device to go idle, then frees them; later calls capture afresh.  Must not
 * run while another thread is inside hamming_decode_batch.  Returns
 * HAMMING_OK or HAMMING_EDEVICE. */
int hamming_batch_release_graphs(void);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batched
 * decode of hamming_decode_batch, with the same arguments, results, per-packet
 * status and kernels, but with its workspace taken from a fixed device array
 * of HAMMING_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on until the process ends.  The call itself allocates nothing: no
 * hipMalloc, no hipFree, no graph instantiation (the kernels are launched
 * directly on `stream`, so a capturing stream records them).  The first call
 * on a device looks up that device's copy of the array once.
 *   max_packets : at most HAMMING_NOALLOC_MAX_PACKETS (HAMMING_ERANGE above).
 *                 The tile-to-packet map gets what the array holds beyond the
 *                 prefix sums; a batch with more tiles than map entries
 *                 decodes through the probe path (slower, same results).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (nothing in it needs to start at zero: each call writes the prefix
 * sums and maps before reading them).  Calls that overlap in time on one GPU
 * (on different streams, or from several host threads) race on the array and
 * may decode wrongly; serialise them, for example on one stream.
 * Returns HAMMING_OK, HAMMING_EINVAL, HAMMING_EALIGN, HAMMING_ERANGE or
 * HAMMING_EDEVICE (also when the array's address cannot be looked up).
 */
#define HAMMING_NOALLOC_MAX_PACKETS 65536u
#define HAMMING_NOALLOC_SCRATCH_BYTES (4u << 20)
int hamming_decode_batch_noalloc(const uint64_t *cw_arena, uint64_t cw_words,
                                 const hamming_packet *descs, const uint32_t *n_packets_dev,
                                 uint32_t max_packets, uint64_t max_codewords, uint64_t *data_arena,
                                 uint64_t data_words, uint8_t *errpos_arena, uint64_t errpos_bytes,
                                 int32_t *status_out, hipStream_t stream);

/* ---- bit-plane input layout -------------------------------------------------
 *
 * The index-set clustering of Sec. III.A (Fig. 4) carried to single
 * positions, as a device format: plane p-1 (p = 1..n) holds position p of
 * every codeword, codeword i at bit i%64 of 64-bit word i/64 of the plane;
 * planes are plane_words words apart (plane_words >= ceil(n_cw/64)).  A
 * codeword takes n bits of input instead of 64 (r <= 6) or 128 (r = 7).
 * Bits of the last plane word past n_cw are ignored.  The decode's outputs are
 * those of hamming_decode: dense message stream and errpos bytes.
 */

/* Words of a plane-layout packet with plane_words = ceil(n_cw/64); 0 for bad
 * arguments. */
uint64_t hamming_planes_words(uint64_t n_cw, int r);

/*
 * Decode n_cw codewords given in the plane layout (n_cw at most
 * 2^37 - 2^13 per call, the reach of one launch).
 *   planes     : device, n planes of plane_words 64-bit words (8-byte aligned).
 *   data_out   : device, hamming_data_bytes(n_cw, r) bytes (8-byte aligned;
 *                16-byte alignment enables vector stores).
 *   errpos_out : device, n_cw bytes, or NULL.
 * Returns HAMMING_OK, HAMMING_EINVAL, HAMMING_EALIGN, HAMMING_ERANGE (n_cw
 * too large, or plane_words below ceil(n_cw/64)) or HAMMING_EDEVICE.
 */
int hamming_decode_planes(const uint64_t *planes, uint64_t plane_words, uint64_t n_cw, int r, void *data_out,
                          uint8_t *errpos_out, hipStream_t stream);

/* Convert n_cw codewords from the storage layout of hamming_decode into the
 * plane layout (device buffers, 8-byte aligned; padding bits dropped; plane
 * words past ceil(n_cw/32) 32-bit words are not written).  Same status codes
 * as hamming_decode_planes. */
int hamming_to_planes(const uint64_t *codewords, uint64_t n_cw, int r, uint64_t *planes, uint64_t plane_words,
                      hipStream_t stream);

/* ---- segmented packets ------------------------------------------------------
 *
 * The paper's own packet format (Sec. II, Fig. 1; shortened segments as in
 * the worked example of Sec. III.A): a packet of M message bytes is split into
 * t segments; segment i carries k_i = floor(8M/t) message bits, plus one for
 * the first (8M mod t) segments, message bits [K_i, K_i + k_i) of the packet.
 * It is a shortened Hamming codeword of n_i = k_i + r_i positions, r_i the
 * smallest r >= 2 with 2^r - 1 - r >= k_i: checksum bits at positions 2^j,
 * message bits at the other positions in ascending order.  The encoded packet
 * is the dense LSB-first bit string of segment 1, then segment 2, ...:
 * position p of segment i is bit o_i + p - 1, o_i = n_0 + ... + n_{i-1}, of a
 * little-endian sequence of 64-bit words.  Bits after the last segment up to
 * the end of its last word are ignored on input and written 0 by the encoder.
 *
 * Decoding a segment: s = syndrome (XOR over its index sets).  s = 0: clean;
 * 1 <= s <= n_i: bit s is flipped; s > n_i: no single flip explains the
 * checksum, the segment is detected-uncorrectable and passed on as received
 * (a shortened code is not perfect, so this case exists).  The merged message
 * is M bytes, message bit b of the packet being bit b%8 of byte b/8, written
 * as ceil(M/8) whole 64-bit words whose bytes past M are 0.
 */
#define HAMMING_SEG_MAX_T 32          /* segments per packet */
#define HAMMING_SEG_MAX_K 65519       /* message bits per segment (r_i <= 16) */
#define HAMMING_SEG_MAX_BYTES 4096    /* message bytes per packet */
#define HAMMING_SEG_INVALID 0xFF      /* status of a descriptor the call rejected */

typedef struct hamming_seg_packet {
    uint64_t enc_word_off;  /* first 64-bit word of the encoded packet in the encoded arena */
    uint64_t msg_word_off;  /* first 64-bit word of the message in the message arena */
    uint32_t msg_bytes;     /* M, 1..max_msg_bytes */
    uint32_t t;             /* segments, 1..HAMMING_SEG_MAX_T, at most 8M */
    uint64_t seg_off;       /* first entry of this packet's segments in the syndrome array */
} hamming_seg_packet;       /* 32 bytes */

/* Host helper: segment layout of a packet (k_out, r_out: t entries each, or
 * NULL).  Returns the encoded length in bits, or -1 for a shape the decoder
 * does not take (t outside [1, 32], 8M < t, M > HAMMING_SEG_MAX_BYTES or a
 * segment above HAMMING_SEG_MAX_K message bits). */
int64_t hamming_seg_layout(uint32_t msg_bytes, uint32_t t, uint32_t *k_out, uint32_t *r_out);

/*
 * Decode n_packets segmented packets, a group of threads per packet (see
 * hamming_seg_config_set).
 *   enc_arena, enc_words : device, the encoded packets (8-byte aligned).
 *   descs               : device, n_packets descriptors (8-byte aligned).
 *   max_msg_bytes       : an upper bound of every packet's msg_bytes,
 *                         1..HAMMING_SEG_MAX_BYTES (sizes the LDS of a launch).
 *   msg_arena, msg_words: device, receives the merged messages.
 *   syndromes           : device, syndrome_count entries, or NULL; packet q's
 *                         segment i writes entry seg_off + i with its s.
 *   status              : device, n_packets bytes, or NULL: 0 clean, 1 some
 *                         segment corrected, 2 some segment
 *                         detected-uncorrectable, HAMMING_SEG_INVALID for a
 *                         descriptor with a bad shape or a range outside its
 *                         arena (nothing else is written for that packet).
 * Packets must not overlap in the output arenas.  Returns HAMMING_OK,
 * HAMMING_EINVAL, HAMMING_EALIGN, HAMMING_ERANGE (n_packets above
 * HAMMING_MAX_BATCH) or HAMMING_EDEVICE.
 */
int hamming_decode_segmented(const uint64_t *enc_arena, uint64_t enc_words, const hamming_seg_packet *descs,
                             uint32_t n_packets, uint32_t max_msg_bytes, uint64_t *msg_arena, uint64_t msg_words,
                             uint16_t *syndromes, uint64_t syndrome_count, uint8_t *status, hipStream_t stream);

/* Work assignment of hamming_decode_segmented and hamming_encode_segmented
 * (no effect on results): the threads that cooperate on one packet, 8, 16 or 32 (part of a wave), 64 (a
 * wave) or 256 (a workgroup).  0 lets the library choose: a workgroup per
 * packet for batches of at most 2048 packets (latency), else a group sized to
 * max_msg_bytes (throughput).  Process-wide.  Returns HAMMING_OK or
 * HAMMING_EINVAL. */
int hamming_seg_config_set(uint32_t threads_per_packet);
int hamming_seg_config_get(uint32_t *threads_per_packet);

/*
 * Encode n_packets messages into segmented packets (the transmitter half):
 * reads ceil(M/8) words at msg_word_off (bytes past M ignored), writes the
 * encoded words at enc_word_off.  A descriptor with a bad shape or a range
 * outside its arena is skipped.  Same argument rules and status codes as
 * hamming_decode_segmented.
 */
int hamming_encode_segmented(const uint64_t *msg_arena, uint64_t msg_words, const hamming_seg_packet *descs,
                             uint32_t n_packets, uint32_t max_msg_bytes, uint64_t *enc_arena, uint64_t enc_words,
                             hipStream_t stream);

/* ---- host-resident packets: transfer pipeline ------------------------------ */

/* Transfer scheduling of hamming_decode_host (Sec. III.B): one chunk after
 * another on one stream (SYNC), or chunks spread over several streams so that
 * host-to-device copies, decodes and device-to-host copies of different chunks
 * overlap (ASYNC).  MAPPED uses no copies: the decode kernel reads the
 * received words from, and writes its results to, pinned host memory through
 * its device mapping, so both link directions carry data at once. */
enum hamming_transfer_mode { HAMMING_TRANSFER_SYNC = 0, HAMMING_TRANSFER_ASYNC = 1, HAMMING_TRANSFER_MAPPED = 2 };

/* Device workspace bytes hamming_decode_host needs for chunks of chunk_cw
 * codewords of code r on `streams` streams; 0 for invalid arguments. */
uint64_t hamming_host_workspace_bytes(uint64_t chunk_cw, int r, uint32_t streams);

/*
 * Decode a packet that lives in host memory: the packet is cut into chunks of
 * chunk_cw codewords (a multiple of 64, so every chunk's messages start on a
 * 64-bit word of the output stream); each chunk is copied to the device,
 * decoded with hamming_decode's kernels and copied back into host_data_out /
 * host_errpos_out.  Results are identical to hamming_decode on the whole
 * packet.  Returns after every copy has finished (the call synchronises its
 * streams).
 *   host_cw         : host, n_cw words (2*n_cw for r = 7).  For copies to
 *                     overlap with kernels the three host buffers should be
 *                     pinned (hipHostMalloc); pageable memory works but copies
 *                     then serialise.
 *   host_data_out   : host, hamming_data_bytes(n_cw, r) bytes.
 *   host_errpos_out : host, n_cw bytes, or NULL.
 *   mode            : HAMMING_TRANSFER_SYNC, _ASYNC or _MAPPED.  MAPPED needs
 *                     all three host buffers in pinned, device-mapped memory
 *                     (hipHostMalloc); any other memory is rejected with
 *                     HAMMING_EINVAL before anything runs.  MAPPED ignores
 *                     chunk_cw, streams and the workspace (may be NULL).
 *   streams         : streams used by the asynchronous mode (1..8); the
 *                     synchronous mode uses one.
 *   workspace       : device, hamming_host_workspace_bytes(chunk_cw, r,
 *                     streams) bytes, 256-byte aligned, owned by the caller.
 *   times_ms        : NULL, or double[3] receiving the summed milliseconds of
 *                     host-to-device copies, decodes and device-to-host copies
 *                     (per-operation events; meaningful in the synchronous
 *                     mode, where the operations do not overlap; MAPPED
 *                     reports the whole kernel as the decode time).
 * Returns HAMMING_OK, HAMMING_EINVAL, HAMMING_EALIGN, HAMMING_ERANGE,
 * HAMMING_ENOMEM (workspace too small) or HAMMING_EDEVICE.
 */
int hamming_decode_host(const uint64_t *host_cw, uint64_t n_cw, int r, void *host_data_out,
                        uint8_t *host_errpos_out, uint64_t chunk_cw, int mode, uint32_t streams,
                        void *workspace, uint64_t workspace_bytes, double *times_ms);

/* ---- autotuning ------------------------------------------------------------ */

/*
 * Autotuner: on the current device and `stream`, time the plain decode of
 * random 2^26-codeword packets (2^25 for r = 7) for every lane width, grid
 * cap and XCD chunking, keeping, among the shapes within 1% of the fastest,
 * the widest lane of at most four 16-byte loads (fewer instructions per
 * codeword); and the batched decode of two batches in one 2^28-word (2 GiB)
 * arena of random words, (A) up to 2,000 packets packed end to end (sizes
 * log-uniform in [64, 2^20] codewords, r uniform in 3..7) and (B) 2,000
 * requests of a serving mix at random places (sizes log-uniform in
 * [256, 2^18], r uniform in 4..7), for every schedule, XCD chunking and work
 * chunk; the shapes within 3% of the least summed time (at most 8) are timed
 * twice more with 20 launches per batch, and the lowest mean of those is
 * kept.  Apply the shapes (as hamming_plain_config_set /
 * hamming_batch_config_set / hamming_batch_chunk_set would) and, when
 * cache_path is neither NULL nor empty, write them there (a shape not tuned
 * by this call is written as it stands, with the time hamming_tune_load read
 * for it).  flags: bit 0 tunes the plain decode, bit 1 the batched decode.  Allocates up to about 5 GB of device memory for the
 * duration of the call (1.1 GB for the plain trials, the batch arena and its
 * outputs) and synchronises `stream`.  The cache is keyed by the device
 * architecture only: shapes tuned on these batches serve every later batch.
 * Returns HAMMING_OK, HAMMING_EINVAL, HAMMING_ENOMEM or HAMMING_EDEVICE.
 */
int hamming_tune(const char *cache_path, uint32_t flags, hipStream_t stream);

/* Apply the shapes of a cache written by hamming_tune, if it was written on a
 * device of the same name and architecture.  Returns HAMMING_OK or
 * HAMMING_EINVAL (unreadable file, other device, nothing applied). */
int hamming_tune_load(const char *cache_path);

/* ---- serving: continuous batching of decode requests ---------------------- */

/*
 * A server decodes requests (one packet each) taken from a device-resident
 * codeword pool, batching whatever is waiting as soon as one of its in-flight
 * batch slots is free, so requests that arrive while earlier batches run are
 * admitted and overlap with them on the device.  A batch of at most 16
 * requests and 2^20 codewords is one decode launch with its descriptors in
 * the kernel arguments.  A larger one is planned on the host, which validated
 * every request at submission: the tile prefix sums and a coarse
 * tile-to-packet map go to the device with the descriptors in one copy, and
 * one decode launch follows (no planning or map kernels).  Served batches use
 * the schedule of hamming_batch_config_set and an XCD chunk of 16 of their
 * own (measured on served traffic; the configured chunk is the graph-batched
 * path's).  A request is
 * admitted when its outputs fit in the server's output pool (the
 * device-memory admission cap); until then it waits in FIFO order.
 * The server is driven by the caller (hamming_server_progress) and keeps no
 * thread of its own; one server must not be used from two threads at once.
 * The arithmetic of every request is exactly the plain decode's.
 */
typedef struct hamming_server hamming_server;

typedef struct hamming_server_config {
    uint32_t slots;               /* batches in flight, each on its own stream (1..16) */
    uint32_t max_batch_packets;   /* requests per batch (1..65536) */
    uint64_t max_batch_codewords; /* a batch closes once it holds this many codewords (>= 1) */
    uint32_t max_queue;           /* requests waiting for admission (submit fails beyond) */
    uint32_t auto_release;        /* 1: free a request's outputs once its completion is recorded */
} hamming_server_config;

typedef struct hamming_completion {
    uint64_t request_id;
    uint64_t data_offset;         /* byte offset of the message stream in the output pool */
    uint64_t errpos_offset;       /* byte offset of the errpos bytes in the output pool */
    uint64_t submit_ns;           /* arrival time given to hamming_server_submit */
    uint64_t complete_ns;         /* time the server observed the batch complete */
    int32_t status;               /* HAMMING_OK, or the error of the launch of the request's batch */
    uint32_t reserved;
} hamming_completion;

/* Monotonic clock (nanoseconds) used for arrival and completion times. */
uint64_t hamming_server_now_ns(void);

/*
 * Create a server on the current device.  cw_pool/cw_pool_words is the
 * device codeword pool requests point into (read only); output_pool /
 * output_pool_bytes (device, 256-byte aligned) is where results are written,
 * and its size is the admission cap.  Both stay owned by the caller and must
 * outlive the server.  The server allocates per-slot streams, descriptor
 * arrays, pinned staging and workspaces; hamming_server_destroy frees them.
 * Before returning it runs an empty kernel of the batched decode's code
 * object and one plan-sized copy on each slot's stream, and waits for them,
 * so that those one-time costs (loading the code object, a stream's first
 * copy) are not charged to the first batches.  Returns HAMMING_OK,
 * HAMMING_EINVAL (bad config, NULL pointer), HAMMING_EALIGN, HAMMING_ENOMEM
 * or HAMMING_EDEVICE (a start-up launch or copy failed).
 */
int hamming_server_create(const hamming_server_config *config, const uint64_t *cw_pool,
                          uint64_t cw_pool_words, void *output_pool, uint64_t output_pool_bytes,
                          hamming_server **out);

/* Wait for every batch in flight, then free everything the server owns.
 * Returns HAMMING_OK or HAMMING_EINVAL (NULL). */
int hamming_server_destroy(hamming_server *server);

/*
 * Queue a request: n_cw codewords of code r starting at word in_word_off of
 * the pool, arriving at arrival_ns (hamming_server_now_ns() time base).  On
 * success *request_id receives the request's id (ids count up from 0).  Does
 * not launch anything.  Returns HAMMING_OK, HAMMING_EINVAL (bad r, NULL),
 * HAMMING_ERANGE (outside the pool, or outputs larger than the whole output
 * pool) or HAMMING_ENOMEM (queue full).
 */
int hamming_server_submit(hamming_server *server, uint64_t in_word_off, uint64_t n_cw, uint32_t r,
                          uint64_t arrival_ns, uint64_t *request_id);

/*
 * Non-blocking step: record completions of finished batches (freeing outputs
 * when auto_release is set), admit waiting requests in FIFO order while their
 * outputs fit, and launch one batch per free slot.  Returns HAMMING_OK or
 * HAMMING_EDEVICE.  When a batch cannot be launched, its requests are
 * completed with that error status (and released under auto_release), so the
 * server keeps serving the requests behind them.
 */
int hamming_server_progress(hamming_server *server);

/* Move up to max recorded completions into out[]; *n_out receives the count. */
int hamming_server_poll(hamming_server *server, hamming_completion *out, uint32_t max, uint32_t *n_out);

/* Free the outputs of a completed request (when auto_release is 0).  Returns
 * HAMMING_OK or HAMMING_EINVAL (unknown or unfinished request). */
int hamming_server_release(hamming_server *server, uint64_t request_id);

/* Device base address and size of the output pool. */
int hamming_server_output_pool(hamming_server *server, void **base, uint64_t *bytes);

/* Requests queued, requests in flight, output bytes in use, batches launched. */
int hamming_server_stats(hamming_server *server, uint64_t *queued, uint64_t *inflight,
                         uint64_t *output_bytes_used, uint64_t *batches);

/*
 * Open-loop load generator: submit n requests at times start + arrival_ns[i]
 * (start = now), driving progress between arrivals, until all complete or
 * timeout_ns passes.  latency_ns[i] receives completion - scheduled arrival,
 * *elapsed_ns the wall time of the run.  With auto_release = 1 the trace's
 * completions are consumed here; with auto_release = 0 they are left for
 * hamming_server_poll (after any recorded before the call) and the outputs
 * stay allocated until released, so the output pool must hold the outputs of
 * the whole trace.  Returns HAMMING_OK, HAMMING_EINVAL, HAMMING_ERANGE
 * (timeout), a submit error or a progress error.
 */
int hamming_server_run_trace(hamming_server *server, uint32_t n, const uint64_t *arrival_ns,
                             const uint64_t *in_word_off, const uint64_t *n_cw, const uint32_t *r,
                             uint64_t timeout_ns, uint64_t *latency_ns, uint64_t *elapsed_ns);

/* Static, human-readable text for a status code. */
const char *hamming_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* HAMMING_H */

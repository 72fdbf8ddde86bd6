/* A plain C consumer of libhamming.so: compiled and linked against
 * include/hamming.h by tests/test_c_abi.py.  It makes only calls that are
 * answered on the host (sizes, layouts, argument validation), so it runs
 * without a GPU; it proves the header is valid C and the exported symbols
 * resolve with the declared signatures. */
#include <stdio.h>
#include <string.h>

#include "hamming.h"

#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                   \
        }                                                               \
    } while (0)

int main(void)
{
    static const int k[5] = {4, 11, 26, 57, 120};
    for (int r = 3; r <= 7; ++r) {
        CHECK(hamming_message_bits(r) == k[r - 3]);
        CHECK(hamming_data_bytes(1000, r) == ((1000ull * k[r - 3] + 63) / 64) * 8);
    }
    CHECK(hamming_message_bits(8) == -1);

    uint64_t words[4] = {0};
    uint8_t out[64];
    /* validation happens on the host before anything is enqueued */
    CHECK(hamming_decode(words, 4, 9, out, NULL, NULL) == HAMMING_EINVAL);
    CHECK(hamming_decode((const uint64_t *)((char *)words + 4), 4, 4, out, NULL, NULL) == HAMMING_EALIGN);
    CHECK(hamming_decode(NULL, 0, 5, NULL, NULL, NULL) == HAMMING_OK);
    CHECK(strlen(hamming_strerror(HAMMING_EINVAL)) > 0);

    uint32_t kk[8], rr[8];
    CHECK(hamming_seg_layout(7, 8, kk, rr) == 88);
    CHECK(kk[0] == 7 && rr[0] == 4);
    CHECK(hamming_seg_layout(1, 9, NULL, NULL) == -1);
    CHECK(hamming_planes_words(65, 3) == 14);
    CHECK(hamming_host_workspace_bytes(100, 4, 1) == 0);

    hamming_packet p[2];
    memset(p, 0, sizeof p);
    p[0].n_cw = 100; p[0].r = 4;
    p[1].in_word_off = 100; p[1].n_cw = 7; p[1].r = 7;
    uint64_t dw = 0, eb = 0;
    CHECK(hamming_batch_layout(p, 2, &dw, &eb) == HAMMING_OK);
    CHECK(p[1].data_word_off > 0 && dw >= p[1].data_word_off + 14 && eb >= 107);
    CHECK(sizeof(hamming_packet) == 40 && sizeof(hamming_seg_packet) == 32);
    printf("c abi ok\n");
    return 0;
}

// Host-side unit checks of the library's host-only helpers, built with the
// address and undefined-behaviour sanitizers by tests/test_host_sanitize.py:
//  * the segmented kernels' window bit helpers (seg_bits.h) against
//    bit-by-bit definitions, mask_top over every window end;
//  * the server's output ring allocator against a model of live ranges;
//  * the server's coarse tile-to-packet map against the prefix sums.
// Prints "host units ok" and exits 0 when every check holds.
#include <stdint.h>
#include <stdio.h>

#include <deque>
#include <random>
#include <vector>

#include "host_plan.h"
#include "ring_alloc.h"
#include "seg_bits.h"

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            fprintf(stderr, "check failed at %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            return 1;                                                                \
        }                                                                            \
    } while (0)

static bool is_pow2(uint64_t p) { return p && !(p & (p - 1)); }

static uint64_t bit128(uint64_t lo, uint64_t hi, uint32_t q) { return q < 64 ? (lo >> q) & 1 : (hi >> (q - 64)) & 1; }

static int check_mask_top()
{
    std::mt19937_64 g(1);
    for (uint32_t top = 0; top < 400; ++top)
        for (int rep = 0; rep < 32; ++rep) {
            const uint64_t a = g(), b = g();
            uint64_t x0 = a, x1 = b;
            hm::mask_top(x0, x1, top);
            for (uint32_t q = 0; q < 128; ++q) CHECK(bit128(x0, x1, q) == (q <= top ? bit128(a, b, q) : 0));
        }
    return 0;
}

static int check_funnel128()
{
    std::mt19937_64 g(2);
    for (uint32_t s = 0; s < 64; ++s)
        for (int rep = 0; rep < 64; ++rep) {
            const uint64_t w[3] = {g(), g(), g()};
            uint64_t lo = 0, hi = 0;
            hm::funnel128(w[0], w[1], w[2], s, lo, hi);
            for (uint32_t q = 0; q < 128; ++q) {
                const uint32_t b = s + q;
                CHECK(bit128(lo, hi, q) == ((w[b / 64] >> (b % 64)) & 1));
            }
        }
    return 0;
}

static int check_run_start()
{
    // message index of position p = non-power-of-two positions below it
    for (uint32_t v = 0; v < 3000; ++v) {
        uint32_t pw = 7;
        const uint32_t got = hm::run_start(v, pw);
        if (v == 0) {
            CHECK(got == 0);
            continue;
        }
        const uint64_t p0 = 128ull * v;
        CHECK(pw == (is_pow2(p0) ? 1u : 0u));
        const uint64_t first = p0 + pw;             // first message position of the window
        CHECK(!is_pow2(first));
        uint64_t below = 0;
        for (uint64_t p = 1; p < first; ++p) below += !is_pow2(p);
        CHECK(got == below);
    }
    return 0;
}

static int check_head()
{
    std::mt19937_64 g(3);
    std::vector<uint32_t> pos;                      // message positions below 64, ascending
    for (uint32_t p = 1; p < 64; ++p)
        if (!is_pow2(p)) pos.push_back(p);
    CHECK(pos.size() == 57);
    for (int rep = 0; rep < 20000; ++rep) {
        const uint64_t w = g();                     // positions 1..64 at bits 0..63
        uint64_t want = 0;
        for (size_t m = 0; m < pos.size(); ++m) want |= ((w >> (pos[m] - 1)) & 1) << m;
        CHECK(hm::head_message(w) == want);
        const uint64_t msg = g() & ((uint64_t(1) << 57) - 1);
        uint64_t placed = 0;                        // position q at bit q
        for (size_t m = 0; m < pos.size(); ++m) placed |= ((msg >> m) & 1) << pos[m];
        CHECK(hm::head_expand(msg) == placed);
    }
    return 0;
}

static int check_ring_allocator()
{
    std::mt19937_64 g(4);
    for (uint64_t size : {uint64_t(256), uint64_t(4096), uint64_t(1) << 20}) {
        hm::RingAllocator ra(size);
        std::deque<std::pair<uint64_t, uint64_t>> live;   // (off, bytes), oldest first
        uint64_t used = 0;
        for (int step = 0; step < 200000; ++step) {
            if (live.empty() || (g() % 3) != 0) {
                const uint64_t bytes = 1 + g() % (size / 3 + 1);
                uint64_t off = ~uint64_t(0);
                if (ra.alloc(bytes, &off)) {
                    CHECK(off + bytes <= size);
                    for (const auto& l : live) CHECK(off + bytes <= l.first || l.first + l.second <= off);
                    live.emplace_back(off, bytes);
                    used += bytes;
                } else {
                    CHECK(!live.empty() || bytes > size);  // an empty ring takes anything that fits
                }
            } else {
                ra.release_oldest(live.front().first, live.front().second);
                used -= live.front().second;
                live.pop_front();
            }
            CHECK(ra.used() == used && ra.live() == live.size());
        }
        while (!live.empty()) {
            ra.release_oldest(live.front().first, live.front().second);
            live.pop_front();
        }
        uint64_t off = 1;
        CHECK(ra.alloc(size, &off) && off == 0);
        uint64_t off2 = 0;
        CHECK(!ra.alloc(1, &off2));
        CHECK(!ra.alloc(0, &off2));
    }
    return 0;
}

static int check_coarse_map()
{
    std::mt19937_64 g(5);
    for (int rep = 0; rep < 3000; ++rep) {
        const uint32_t n = 1 + uint32_t(g() % 700);
        std::vector<uint64_t> ts(n + 1, 0);
        for (uint32_t p = 0; p < n; ++p) {
            const uint64_t k = g() % 4;
            const uint64_t tiles = k == 0 ? 0 : (k == 1 ? 1 : (k == 2 ? g() % 40 : g() % 5000));
            ts[p + 1] = ts[p] + tiles;
        }
        if (ts[n] == 0) continue;
        const uint32_t lg = hm::planned_coarse_log2(ts[n], n);
        CHECK((ts[n] >> lg) < hm::planned_coarse_capacity(n));
        CHECK(lg == 0 || (ts[n] >> (lg - 1)) >= hm::planned_coarse_capacity(n));
        std::vector<uint32_t> coarse(hm::planned_coarse_capacity(n) + 1, 0xFFFFFFFFu);
        const uint64_t entries = hm::plan_coarse_map(ts.data(), n, lg, coarse.data());
        CHECK(entries <= hm::planned_coarse_capacity(n));
        CHECK(coarse[entries] == 0xFFFFFFFFu);                 // nothing written past the entries
        for (uint64_t j = 0; j < entries; ++j) {
            const uint32_t p = coarse[j];
            CHECK(p < n && ts[p] <= (j << lg) && (j << lg) < ts[p + 1]);
        }
        // every tile's packet is reached by probing forward from its entry
        for (uint64_t t = 0; t < ts[n]; t += 1 + g() % 7) {
            uint32_t p = coarse[t >> lg];
            CHECK(ts[p] <= t);
            while (p + 1 < n && ts[p + 1] <= t) ++p;
            CHECK(ts[p] <= t && t < ts[p + 1]);
        }
    }
    return 0;
}

int main()
{
    if (check_mask_top() || check_funnel128() || check_run_start() || check_head() || check_ring_allocator() ||
        check_coarse_map())
        return 1;
    printf("host units ok\n");
    return 0;
}

// Host side of a planned batch (see PlannedBatch in batch.h): the coarse
// tile-to-packet map built from the packets' tile prefix sums.  Host code only.
#pragma once

#include <stdint.h>

namespace hm {

// Coarse-map entries a host plan of n packets may use.
inline uint64_t planned_coarse_capacity(uint32_t n) { return 2ull * n + 64; }

// Smallest g with ceil(total / 2^g) <= planned_coarse_capacity(n).
inline uint32_t planned_coarse_log2(uint64_t total, uint32_t n)
{
    const uint64_t cap = planned_coarse_capacity(n);
    uint32_t g = 0;
    while ((total >> g) >= cap) ++g;
    return g;
}

// Fill coarse[j] with the packet holding tile j << g, for every j below
// ceil(ts[n] / 2^g); ts[0..n] is the exclusive prefix sum of the packets'
// tile counts (packets without tiles included).  Entry j gets the first
// packet p, in order, with (j << g) < ts[p + 1]; every earlier packet ends at
// or before that tile, so ts[p] <= (j << g) as well.  Returns the entries.
inline uint64_t plan_coarse_map(const uint64_t* ts, uint32_t n, uint32_t g, uint32_t* coarse)
{
    const uint64_t entries = (ts[n] + (uint64_t(1) << g) - 1) >> g;
    uint64_t j = 0;
    for (uint32_t p = 0; p < n && j < entries; ++p)
        while (j < entries && (j << g) < ts[p + 1]) coarse[j++] = p;
    return entries;
}

}  // namespace hm

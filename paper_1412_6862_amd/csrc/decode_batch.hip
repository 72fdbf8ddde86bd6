// Batched decode: many packets of mixed size and r in one launch sequence.
//
// The arithmetic is the plain decode's (tile.h); only the work distribution
// differs.  Tiles are 64*U codewords aligned to their packet's start, and the
// batch's tiles are numbered in packet order.  Work is dealt in chunks of
// 2^c consecutive tiles: a wave finds the packet of its chunk's first tile
// once, then decodes the chunk packet by packet, each packet's share as one
// pipelined run (the next tile's loads in flight while the current one is
// decoded), so the lookup and its dependent loads are paid per chunk rather
// than per tile.  Chunks go to waves in order, as the hardware dispatches the
// plain grid, so the chunks in flight form one advancing window of memory.
// Four kernels, all replayable from a hipGraph with no host work:
//  * batch_plan_kernel (one workgroup) validates every descriptor, writes its
//    status and an exclusive prefix sum of its tile count, and picks the
//    group sizes of two chunk-to-packet maps so that each fits its capacity;
//  * batch_coarse_kernel fills the coarse map by binary search over the
//    prefix sums; batch_fine_kernel fills the fine map (normally one entry
//    per chunk) by a short binary search between two coarse entries;
//  * decode_batch_kernel reads a chunk's packet from the fine map (plus a
//    64-lane probe when a fine entry spans several chunks) and decodes it.  A
//    grid smaller than the batch loops.
// A batch of at most kSmallBatchMax packets validated by its caller can
// instead carry its descriptors and tile prefix sums in the kernel arguments
// of decode_small_batch_kernel: one launch, no copy and no maps, one tile
// per wave (the latency form).
// Each packet's output is the same words a plain call would write.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.h"
#include "hamming.h"
#include "hamming_device.h"
#include "launch.h"
#include "tile.h"

namespace hm {

// Per-r lane widths of a batch schedule, and the waves per SIMD the decode
// kernel's register allocation must allow.
template <int U3, int U4, int U5, int U6, int U7, int WAVES>
struct Schedule {
    static constexpr int u[5] = {U3, U4, U5, U6, U7};
    static constexpr int waves_per_simd = WAVES;
    static constexpr int max2(int a, int b) { return a > b ? a : b; }
    static constexpr int LDS_MAX =
        max2(max2(max2(TileShape<3, U3>::LDS_DW, TileShape<4, U4>::LDS_DW),
                  max2(TileShape<5, U5>::LDS_DW, TileShape<6, U6>::LDS_DW)),
             TileShape<7, U7>::LDS_DW);
    static_assert(valid_u(3, U3) && valid_u(4, U4) && valid_u(5, U5) && valid_u(6, U6) && valid_u(7, U7),
                  "invalid lane width");
};

using Sched0 = Schedule<8, 8, 8, 8, 2, 4>;
using Sched1 = Schedule<8, 4, 4, 4, 2, 5>;
using Sched2 = Schedule<8, 8, 8, 4, 2, 5>;
using Sched3 = Schedule<8, 8, 8, 8, 4, 4>;

__device__ __forceinline__ uint64_t message_words(uint64_t n_cw, uint32_t r)
{
    const uint64_t k = (uint64_t(1) << r) - 1 - r;
    return (n_cw * k + 63) / 64;
}

template <class S>
__device__ __forceinline__ uint64_t packet_tiles(uint64_t n_cw, uint32_t r)
{
    const uint64_t cwt = 64u * uint64_t(S::u[r - 3]);
    return (n_cw + cwt - 1) / cwt;
}

// Validate one descriptor; returns a status and the packet's tile count.
template <class S>
__device__ int32_t plan_packet(const hamming_packet& d, const BatchArgs& a, uint64_t* tiles)
{
    *tiles = 0;
    if (d.r < 3 || d.r > 7 || d.flags != 0) return HAMMING_EINVAL;
    if (d.n_cw > HAMMING_MAX_CODEWORDS) return HAMMING_ERANGE;
    if (d.n_cw == 0) return HAMMING_OK;
    const uint64_t wpc = d.r == 7 ? 2 : 1;
    if (d.in_word_off > a.cw_words || d.n_cw * wpc > a.cw_words - d.in_word_off) return HAMMING_ERANGE;
    const uint64_t mw = message_words(d.n_cw, d.r);
    if (d.data_word_off > a.data_words || mw > a.data_words - d.data_word_off) return HAMMING_ERANGE;
    if (d.errpos_off != HAMMING_NO_ERRPOS) {
        if (!a.errpos_arena || d.errpos_off > a.errpos_bytes || d.n_cw > a.errpos_bytes - d.errpos_off)
            return HAMMING_ERANGE;
    }
    *tiles = packet_tiles<S>(d.n_cw, d.r);
    return HAMMING_OK;
}

template <class S>
__global__ __launch_bounds__(1024) void batch_plan_kernel(BatchArgs a)
{
    __shared__ uint64_t wave_sums[16];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    uint32_t n = *a.n_packets_dev;
    if (n > a.max_packets) n = a.max_packets;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t p = base + tid;
        uint64_t t = 0;
        if (p < n) {
            const int32_t st = plan_packet<S>(a.descs[p], a, &t);
            if (a.status_out) a.status_out[p] = st;
        }
        uint64_t x = t;   // inclusive scan within the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t y = __shfl_up(x, off);
            if (lane >= uint32_t(off)) x += y;
        }
        if (lane == 63) wave_sums[wave] = x;
        __syncthreads();
        if (wave == 0) {
            uint64_t v = lane < 16 ? wave_sums[lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const uint64_t y = __shfl_up(v, off);
                if (lane >= uint32_t(off)) v += y;
            }
            if (lane < 16) wave_sums[lane] = v;
        }
        __syncthreads();
        const uint64_t before = wave ? wave_sums[wave - 1] : 0;
        if (p < n) a.tile_start[p] = carry + before + x - t;
        carry += wave_sums[15];
        __syncthreads();
    }
    if (tid == 0) {
        // entries = ceil(total / 2^g) <= capacity; the fine map needs at most
        // one entry per chunk (lookups are made at chunk starts only)
        uint32_t gc = 0, gf = a.chunk_log2;
        while ((carry >> gc) >= a.coarse_cap) ++gc;
        while ((carry >> gf) >= a.fine_cap) ++gf;
        a.tile_start[n] = carry;
        a.ws->total_tiles = carry;
        a.ws->n_packets = n;
        a.ws->coarse_log2 = gc;
        a.ws->fine_log2 = gf;
        a.ws->n_coarse = (carry + (uint64_t(1) << gc) - 1) >> gc;
        a.ws->n_fine = (carry + (uint64_t(1) << gf) - 1) >> gf;
    }
}

// Last p in [lo, hi) with ts[p] <= t, given ts[lo] <= t (per lane).
__device__ __forceinline__ uint32_t search_packet(const uint64_t* ts, uint64_t t, uint32_t lo, uint32_t hi)
{
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ts[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void batch_coarse_kernel(BatchArgs a)
{
    const uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= a.ws->n_coarse) return;
    a.coarse[j] = search_packet(a.tile_start, j << a.ws->coarse_log2, 0, uint32_t(a.ws->n_packets));
}

__global__ __launch_bounds__(256) void batch_fine_kernel(BatchArgs a)
{
    const uint64_t n_fine = a.ws->n_fine;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n_fine; j += stride) {
        const uint64_t t = j << a.ws->fine_log2;
        const uint64_t jc = t >> a.ws->coarse_log2;
        const uint32_t lo = a.coarse[jc];
        // the packet holding tile t lies between the coarse entries around it
        const uint32_t hi = (jc + 1 < a.ws->n_coarse) ? a.coarse[jc + 1] + 1 : uint32_t(a.ws->n_packets);
        a.fine[j] = search_packet(a.tile_start, t, lo, hi);
    }
}

// Last packet p in [0, n) with tile_start[p] <= t, given tile_start[lo] <= t
// and t < tile_start[n] (t uniform across the wave): 64 lanes probe 64
// consecutive entries per step.
__device__ __forceinline__ uint32_t probe_packet(const uint64_t* ts, uint32_t n, uint64_t t, uint32_t lo)
{
    const uint32_t lane = threadIdx.x & 63u;
    for (;;) {
        const uint32_t q = lo + lane;
        const bool le = (q < n) && (ts[q] <= t);
        const uint64_t m = __ballot(le);                 // a prefix of the lanes: ts is non-decreasing
        const uint32_t cnt = uint32_t(__popcll(m));
        if (cnt < 64) return lo + cnt - 1;
        lo += 63;
    }
}

// Tiles [tl0, tl1) of one packet as one pipelined run.
template <int R, int U>
__device__ __forceinline__ void decode_packet_run(const hamming_packet& d, uint64_t tl0, uint64_t tl1,
                                                  const uint64_t* cw_arena, uint64_t* data_arena,
                                                  uint8_t* errpos_arena, uint32_t* lds)
{
    const uint64_t* cw = cw_arena + d.in_word_off;
    uint64_t* data = data_arena + d.data_word_off;
    uint8_t* ep = (d.errpos_off == HAMMING_NO_ERRPOS) ? nullptr : errpos_arena + d.errpos_off;
    const uint32_t flags = (ep && (reinterpret_cast<uintptr_t>(ep) % U) == 0) ? kFlagEpVec : 0u;
    decode_run<R, U>(cw, d.n_cw, tl0, tl1, 1, data, message_words(d.n_cw, R), ep, lds, flags);
}

template <class S>
__device__ __forceinline__ void decode_any_run(const hamming_packet& d, uint64_t tl0, uint64_t tl1,
                                               const uint64_t* cw_arena, uint64_t* data_arena,
                                               uint8_t* errpos_arena, uint32_t* lds)
{
    switch (d.r) {
    case 3: decode_packet_run<3, S::u[0]>(d, tl0, tl1, cw_arena, data_arena, errpos_arena, lds); break;
    case 4: decode_packet_run<4, S::u[1]>(d, tl0, tl1, cw_arena, data_arena, errpos_arena, lds); break;
    case 5: decode_packet_run<5, S::u[2]>(d, tl0, tl1, cw_arena, data_arena, errpos_arena, lds); break;
    case 6: decode_packet_run<6, S::u[3]>(d, tl0, tl1, cw_arena, data_arena, errpos_arena, lds); break;
    default: decode_packet_run<7, S::u[4]>(d, tl0, tl1, cw_arena, data_arena, errpos_arena, lds); break;
    }
}

// Tiles [t, t_end) of the batch in tile order, p being the packet that holds
// tile t (ts[p] <= t < ts[p + 1]): one run per packet, packets without tiles
// passed over.  All values are uniform across the wave.
template <class S>
__device__ __forceinline__ void decode_span(uint64_t t, uint64_t t_end, uint32_t p, const uint64_t* ts,
                                            const hamming_packet* descs, const uint64_t* cw_arena,
                                            uint64_t* data_arena, uint8_t* errpos_arena, uint32_t* lds)
{
    while (t < t_end) {
        const uint64_t t1 = ts[p + 1];
        if (t1 > t) {
            const hamming_packet d = descs[p];
            const uint64_t t0 = ts[p];
            const uint64_t e = t1 < t_end ? t1 : t_end;
            decode_any_run<S>(d, t - t0, e - t0, cw_arena, data_arena, errpos_arena, lds);
            t = e;
        }
        ++p;
    }
}

template <class S>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(S::waves_per_simd)))
void decode_batch_kernel(
    BatchArgs a, const BatchWs* __restrict__ ws, const uint32_t* __restrict__ fine,
    const uint64_t* __restrict__ ts, const hamming_packet* __restrict__ descs)
{
    __shared__ u32x4 lds_raw[kWavesPerBlock][S::LDS_MAX / 4];
    // the wave index is uniform: keep chunk bookkeeping in scalar registers so
    // the table and descriptor reads below are scalar loads
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* lds = reinterpret_cast<uint32_t*>(&lds_raw[wave][0]);
    const uint64_t waves = uint64_t(gridDim.x) * kWavesPerBlock;
    const uint32_t cl = a.chunk_log2;
    uint64_t c = uint64_t(xcd_block(blockIdx.x, gridDim.x, a.xcd_chunk)) * kWavesPerBlock + wave;
    // Read this chunk's map entry together with the batch totals instead of
    // after them: when the map has one entry per chunk (fine_log2 = chunk
    // log2, the usual case) it is the entry needed.  The index is clamped to
    // the map, so the read stays in bounds whatever the totals turn out to be.
    const uint32_t p_first = fine[c < a.fine_cap ? c : a.fine_cap - 1];
    const uint64_t total = ws->total_tiles;
    if ((c << cl) >= total) return;
    const uint32_t n = uint32_t(ws->n_packets);
    const uint32_t gf = ws->fine_log2;            // >= cl
    bool first = true;
    for (; (c << cl) < total; c += waves) {
        const uint64_t t = c << cl;
        uint32_t p = (first && gf == cl) ? p_first : fine[t >> gf];
        first = false;
        if (gf > cl) p = probe_packet(ts, n, t, p);
        const uint64_t t_end = (t + (uint64_t(1) << cl) < total) ? t + (uint64_t(1) << cl) : total;
        decode_span<S>(t, t_end, p, ts, descs, a.cw_arena, a.data_arena, a.errpos_arena, lds);
    }
}

// The small-batch form: one tile per wave, the packet found by a scan of the
// prefix sums in the kernel arguments (at most kSmallBatchMax entries, scalar
// loads), then the same tile decode.
template <class S>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(S::waves_per_simd)))
void decode_small_batch_kernel(SmallBatch b)
{
    __shared__ u32x4 lds_raw[kWavesPerBlock][S::LDS_MAX / 4];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* lds = reinterpret_cast<uint32_t*>(&lds_raw[wave][0]);
    const uint64_t t = uint64_t(blockIdx.x) * kWavesPerBlock + wave;
    if (t >= b.tile_start[b.n]) return;
    uint32_t p = 0;
    while (p + 1 < b.n && b.tile_start[p + 1] <= t) ++p;    // packets without tiles are passed over
    const hamming_packet d = b.descs[p];
    decode_any_run<S>(d, t - b.tile_start[p], t + 1 - b.tile_start[p], b.cw_arena, b.data_arena, b.errpos_arena,
                      lds);
}

// Last packet p with tile_start[p] <= t, given tile_start[lo] <= t < tile_start[n]
// (t and lo uniform): eight entries per step by scalar loads, which do not
// queue behind the wave's streaming vector loads.  The host plan's coarse map
// puts lo within a packet or two of the answer, so one step almost always
// suffices.
__device__ __forceinline__ uint32_t scan_packet(const uint64_t* __restrict__ ts, uint32_t n, uint64_t t, uint32_t lo)
{
    for (;;) {
        // entries lo+1 .. lo+8 at or below t form a prefix (ts is non-decreasing);
        // indices past n read ts[n] = total > t, so all eight loads issue at once
        uint64_t e[8];
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) e[i] = ts[min(lo + 1 + i, n)];
        uint32_t k = 0;
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) k += e[i] <= t ? 1u : 0u;
        if (k < 8) return lo + k;
        lo += 8;
    }
}

// The host-planned form: chunks of 2^c tiles in order (waves loop when the
// batch has more chunks than a dispatch can hold), the packet of a chunk's
// first tile found from the coarse map entry by a scalar scan of the prefix
// sums.  The plan's arrays are separate read-only kernel arguments so that
// every read of them (map entry, prefix sums, descriptors) is a scalar load.
template <class S>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(S::waves_per_simd)))
void decode_planned_batch_kernel(PlannedBatch b, const uint64_t* __restrict__ ts, const uint32_t* __restrict__ coarse,
                                 const hamming_packet* __restrict__ descs)
{
    __shared__ u32x4 lds_raw[kWavesPerBlock][S::LDS_MAX / 4];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* lds = reinterpret_cast<uint32_t*>(&lds_raw[wave][0]);
    const uint64_t waves = uint64_t(gridDim.x) * kWavesPerBlock;
    const uint32_t cl = b.chunk_log2;
    for (uint64_t c = uint64_t(xcd_block(blockIdx.x, gridDim.x, b.xcd_chunk)) * kWavesPerBlock + wave;
         (c << cl) < b.total_tiles; c += waves) {
        const uint64_t t = c << cl;
        const uint32_t p = scan_packet(ts, b.n, t, coarse[t >> b.coarse_log2]);
        const uint64_t t_end = (t + (uint64_t(1) << cl) < b.total_tiles) ? t + (uint64_t(1) << cl) : b.total_tiles;
        decode_span<S>(t, t_end, p, ts, descs, b.cw_arena, b.data_arena, b.errpos_arena, lds);
    }
}

template <class S>
static hipError_t launch_planned_s(const PlannedBatch& b, hipStream_t stream)
{
    const uint64_t chunks = (b.total_tiles + (uint64_t(1) << b.chunk_log2) - 1) >> b.chunk_log2;
    uint64_t blocks = (chunks + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > max_launch_blocks(kBlockThreads)) blocks = max_launch_blocks(kBlockThreads);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((decode_planned_batch_kernel<S>), dim3(uint32_t(blocks)), dim3(kBlockThreads), 0, stream, b,
                       b.tile_start, b.coarse, b.descs);
    return hipGetLastError();
}

hipError_t launch_planned_batch(const PlannedBatch& b, int schedule, hipStream_t stream)
{
    if (b.n < 1) return hipErrorInvalidValue;
    switch (schedule) {
    case 0: return launch_planned_s<Sched0>(b, stream);
    case 1: return launch_planned_s<Sched1>(b, stream);
    case 2: return launch_planned_s<Sched2>(b, stream);
    case 3: return launch_planned_s<Sched3>(b, stream);
    default: return hipErrorInvalidValue;
    }
}

template <class S>
static hipError_t launch_batch_s(const BatchArgs& a, uint32_t grid, hipStream_t stream)
{
    hipLaunchKernelGGL((batch_plan_kernel<S>), dim3(1), dim3(1024), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_coarse_kernel, dim3((a.coarse_cap + 255) / 256), dim3(256), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_fine_kernel, dim3(a.fine_blocks), dim3(256), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((decode_batch_kernel<S>), dim3(grid), dim3(kBlockThreads), 0, stream, a, a.ws, a.fine,
                       a.tile_start, a.descs);
    return hipGetLastError();
}

template <class S>
static hipError_t launch_small_s(const SmallBatch& b, hipStream_t stream)
{
    const uint64_t blocks = (b.tile_start[b.n] + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks == 0 || blocks > max_launch_blocks(kBlockThreads)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((decode_small_batch_kernel<S>), dim3(uint32_t(blocks)), dim3(kBlockThreads), 0, stream, b);
    return hipGetLastError();
}

__global__ void batch_module_start_kernel() {}

hipError_t launch_batch_module_start(hipStream_t stream)
{
    hipLaunchKernelGGL(batch_module_start_kernel, dim3(1), dim3(64), 0, stream);
    return hipGetLastError();
}

hipError_t launch_small_batch(const SmallBatch& b, int schedule, hipStream_t stream)
{
    if (b.n < 1 || b.n > kSmallBatchMax) return hipErrorInvalidValue;
    switch (schedule) {
    case 0: return launch_small_s<Sched0>(b, stream);
    case 1: return launch_small_s<Sched1>(b, stream);
    case 2: return launch_small_s<Sched2>(b, stream);
    case 3: return launch_small_s<Sched3>(b, stream);
    default: return hipErrorInvalidValue;
    }
}

uint32_t schedule_lane_width(int schedule, uint32_t r)
{
    if (r < 3 || r > 7) return 0;
    switch (schedule) {
    case 0: return uint32_t(Sched0::u[r - 3]);
    case 1: return uint32_t(Sched1::u[r - 3]);
    case 2: return uint32_t(Sched2::u[r - 3]);
    case 3: return uint32_t(Sched3::u[r - 3]);
    default: return 0;
    }
}

uint64_t schedule_min_tile_codewords(int schedule)
{
    uint64_t m = ~uint64_t(0);
    for (uint32_t r = 3; r <= 7; ++r) {
        const uint64_t c = 64ull * schedule_lane_width(schedule, r);
        if (c && c < m) m = c;
    }
    return m == ~uint64_t(0) ? 0 : m;
}

uint64_t schedule_min_tile_words(int schedule)
{
    uint64_t m = ~uint64_t(0);
    for (uint32_t r = 3; r <= 7; ++r) {
        const uint64_t c = 64ull * schedule_lane_width(schedule, r) * (r == 7 ? 2 : 1);
        if (c && c < m) m = c;
    }
    return m == ~uint64_t(0) ? 0 : m;
}

hipError_t launch_batch(const BatchArgs& a, int schedule, uint32_t grid, hipStream_t stream)
{
    switch (schedule) {
    case 0: return launch_batch_s<Sched0>(a, grid, stream);
    case 1: return launch_batch_s<Sched1>(a, grid, stream);
    case 2: return launch_batch_s<Sched2>(a, grid, stream);
    case 3: return launch_batch_s<Sched3>(a, grid, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hm

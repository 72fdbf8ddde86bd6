// C ABI of libhamming.so: host-side argument validation, launch-shape
// selection and error mapping.  Declarations and the contract of every entry
// point are in include/hamming.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "hamming.h"
#include "launch.h"

namespace {

using hm::DecodeLaunch;

// Plain-decode launch shape per r (index r-3): codewords per lane and a cap
// on workgroups (0 = one wave per tile).  Read at every call; the setters are
// meant for start-up configuration and the tuner.
struct PlainShape {
    std::atomic<int> u;
    std::atomic<uint64_t> max_blocks;
    std::atomic<uint32_t> xcd_chunk;
};

PlainShape g_plain[5] = {{8, 0, 1}, {8, 0, 1}, {8, 0, 1}, {8, 0, 1}, {2, 0, 1}};

bool valid_r(int r) { return r >= 3 && r <= 7; }

int message_bits(int r) { return (1 << r) - 1 - r; }

int words_per_cw(int r) { return r == 7 ? 2 : 1; }

int map_hip(hipError_t e) { return e == hipSuccess ? HAMMING_OK : HAMMING_EDEVICE; }

}  // namespace

extern "C" {

int hamming_message_bits(int r) { return valid_r(r) ? message_bits(r) : -1; }

uint64_t hamming_data_bytes(uint64_t n_cw, int r)
{
    if (!valid_r(r) || n_cw > HAMMING_MAX_CODEWORDS) return 0;
    const uint64_t bits = n_cw * uint64_t(message_bits(r));
    return ((bits + 63) / 64) * 8;
}

int hamming_decode(const uint64_t* codewords, uint64_t n_cw, int r, void* data_out, uint8_t* errpos_out,
                   hipStream_t stream)
{
    if (!valid_r(r)) return HAMMING_EINVAL;
    if (n_cw > HAMMING_MAX_CODEWORDS) return HAMMING_ERANGE;
    if (n_cw == 0) return HAMMING_OK;
    if (!codewords || !data_out) return HAMMING_EINVAL;
    if ((reinterpret_cast<uintptr_t>(codewords) & 7u) || (reinterpret_cast<uintptr_t>(data_out) & 7u))
        return HAMMING_EALIGN;
    DecodeLaunch L;
    L.r = r;
    L.u = g_plain[r - 3].u.load(std::memory_order_relaxed);
    L.cw = codewords;
    L.n_cw = n_cw;
    L.data = static_cast<uint64_t*>(data_out);
    L.data_words = hamming_data_bytes(n_cw, r) / 8;
    L.errpos = errpos_out;
    L.max_blocks = g_plain[r - 3].max_blocks.load(std::memory_order_relaxed);
    L.xcd_chunk = g_plain[r - 3].xcd_chunk.load(std::memory_order_relaxed);
    return map_hip(hm::launch_decode(L, stream));
}

int hamming_encode(const void* data_in, uint64_t n_cw, int r, uint64_t* codewords_out, hipStream_t stream)
{
    if (!valid_r(r)) return HAMMING_EINVAL;
    if (n_cw > HAMMING_MAX_CODEWORDS) return HAMMING_ERANGE;
    if (n_cw == 0) return HAMMING_OK;
    if (!data_in || !codewords_out) return HAMMING_EINVAL;
    if ((reinterpret_cast<uintptr_t>(data_in) & 7u) || (reinterpret_cast<uintptr_t>(codewords_out) & 7u))
        return HAMMING_EALIGN;
    (void)words_per_cw;
    return map_hip(hm::launch_encode(r, data_in, n_cw, codewords_out, stream));
}

int hamming_plain_config_set(int r, int lane_codewords, uint64_t max_blocks, uint32_t xcd_chunk)
{
    if (!valid_r(r) || !hm::valid_u(r, lane_codewords) || xcd_chunk < 1) return HAMMING_EINVAL;
    if (max_blocks > (uint64_t(1) << 31) || xcd_chunk > (1u << 20)) return HAMMING_ERANGE;
    g_plain[r - 3].u.store(lane_codewords, std::memory_order_relaxed);
    g_plain[r - 3].max_blocks.store(max_blocks, std::memory_order_relaxed);
    g_plain[r - 3].xcd_chunk.store(xcd_chunk, std::memory_order_relaxed);
    return HAMMING_OK;
}

int hamming_plain_config_get(int r, int* lane_codewords, uint64_t* max_blocks, uint32_t* xcd_chunk)
{
    if (!valid_r(r) || !lane_codewords || !max_blocks || !xcd_chunk) return HAMMING_EINVAL;
    *lane_codewords = g_plain[r - 3].u.load(std::memory_order_relaxed);
    *max_blocks = g_plain[r - 3].max_blocks.load(std::memory_order_relaxed);
    *xcd_chunk = g_plain[r - 3].xcd_chunk.load(std::memory_order_relaxed);
    return HAMMING_OK;
}

uint64_t hamming_decode_grid(uint64_t n_cw, int r)
{
    if (!valid_r(r) || n_cw > HAMMING_MAX_CODEWORDS) return 0;
    const uint64_t cw_per_tile = 64ull * uint64_t(g_plain[r - 3].u.load(std::memory_order_relaxed));
    return hm::plain_grid_blocks((n_cw + cw_per_tile - 1) / cw_per_tile,
                                 g_plain[r - 3].max_blocks.load(std::memory_order_relaxed));
}

const char* hamming_strerror(int status)
{
    switch (status) {
    case HAMMING_OK: return "success";
    case HAMMING_EINVAL: return "invalid argument (r outside [3,7], NULL pointer or bad descriptor field)";
    case HAMMING_EALIGN: return "pointer is not aligned as required";
    case HAMMING_ERANGE: return "size or offset out of range";
    case HAMMING_ENOMEM: return "caller-provided buffer is too small";
    case HAMMING_EDEVICE: return "the HIP runtime rejected the launch";
    default: return "unknown status";
    }
}

}  // extern "C"

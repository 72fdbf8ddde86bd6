// Decode of host-resident packets with copies scheduled as in Sec. III.B:
// synchronous (copy in, decode, copy out, chunk after chunk) or asynchronous
// (chunks spread over several streams so that copies and decodes of different
// chunks overlap, the pipelined transfer of Fig. 5 / Eq. 1), plus a mapped
// mode in which the kernel itself reads and writes pinned host memory.  Host
// code only; the decodes are hamming_decode's kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "hamming.h"

namespace {

constexpr uint32_t kMaxStreams = 8;

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

struct StagingLayout {
    uint64_t in_bytes, data_bytes, ep_bytes, per_stream;
};

StagingLayout staging(uint64_t chunk_cw, int r)
{
    StagingLayout L;
    L.in_bytes = round_up(chunk_cw * (r == 7 ? 16 : 8), 256);
    L.data_bytes = round_up(hamming_data_bytes(chunk_cw, r), 256);
    L.ep_bytes = round_up(chunk_cw, 256);
    L.per_stream = L.in_bytes + L.data_bytes + L.ep_bytes;
    return L;
}

struct Timers {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ok = true;
    Timers()
    {
        for (auto& x : e)
            if (hipEventCreate(&x) != hipSuccess) ok = false;
    }
    ~Timers()
    {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// Device address of pinned, device-mapped host memory, or nullptr for
// anything else (pageable memory, device memory, unknown pointers).
void* mapped_address(const void* p)
{
    hipPointerAttribute_t at;
    if (!p || hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (at.type != hipMemoryTypeHost || !at.devicePointer || !at.hostPointer) return nullptr;
    const char* hp = static_cast<const char*>(at.hostPointer);
    const char* q = static_cast<const char*>(p);
    return static_cast<char*>(at.devicePointer) + (q - hp);
}

// Mapped mode: the decode kernel reads the received words from host memory
// and writes the results to host memory itself, so the two PCIe directions
// are in use at the same time without copy engines.
int decode_mapped(const uint64_t* host_cw, uint64_t n_cw, int r, void* host_data_out, uint8_t* host_errpos_out,
                  double* times_ms)
{
    const void* dcw = mapped_address(host_cw);
    void* ddata = mapped_address(host_data_out);
    void* dep = host_errpos_out ? mapped_address(host_errpos_out) : nullptr;
    if (!dcw || !ddata || (host_errpos_out && !dep)) return HAMMING_EINVAL;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HAMMING_EDEVICE;
    Timers tm;
    int rc = tm.ok ? HAMMING_OK : HAMMING_EDEVICE;
    if (rc == HAMMING_OK && times_ms) (void)hipEventRecord(tm.e[0], s);
    if (rc == HAMMING_OK)
        rc = hamming_decode(static_cast<const uint64_t*>(dcw), n_cw, r, ddata, static_cast<uint8_t*>(dep), s);
    if (rc == HAMMING_OK && times_ms) (void)hipEventRecord(tm.e[1], s);
    if (hipStreamSynchronize(s) != hipSuccess && rc == HAMMING_OK) rc = HAMMING_EDEVICE;
    if (rc == HAMMING_OK && times_ms) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, tm.e[0], tm.e[1]) == hipSuccess) times_ms[1] = ms;
    }
    (void)hipStreamDestroy(s);
    return rc;
}

}  // namespace

extern "C" {

uint64_t hamming_host_workspace_bytes(uint64_t chunk_cw, int r, uint32_t streams)
{
    if (r < 3 || r > 7 || chunk_cw == 0 || chunk_cw % 64 || chunk_cw > HAMMING_MAX_CODEWORDS || streams < 1 ||
        streams > kMaxStreams)
        return 0;
    return staging(chunk_cw, r).per_stream * streams;
}

int hamming_decode_host(const uint64_t* host_cw, uint64_t n_cw, int r, void* host_data_out,
                        uint8_t* host_errpos_out, uint64_t chunk_cw, int mode, uint32_t streams, void* workspace,
                        uint64_t workspace_bytes, double* times_ms)
{
    if (r < 3 || r > 7 ||
        (mode != HAMMING_TRANSFER_SYNC && mode != HAMMING_TRANSFER_ASYNC && mode != HAMMING_TRANSFER_MAPPED))
        return HAMMING_EINVAL;
    if (n_cw > HAMMING_MAX_CODEWORDS) return HAMMING_ERANGE;
    if (mode == HAMMING_TRANSFER_MAPPED) {
        if (times_ms) times_ms[0] = times_ms[1] = times_ms[2] = 0.0;
        if (n_cw == 0) return HAMMING_OK;
        if (!host_cw || !host_data_out) return HAMMING_EINVAL;
        if ((reinterpret_cast<uintptr_t>(host_cw) & 7u) || (reinterpret_cast<uintptr_t>(host_data_out) & 7u))
            return HAMMING_EALIGN;
        return decode_mapped(host_cw, n_cw, r, host_data_out, host_errpos_out, times_ms);
    }
    if (chunk_cw == 0 || chunk_cw % 64 || streams < 1 || streams > kMaxStreams) return HAMMING_EINVAL;
    if (times_ms) times_ms[0] = times_ms[1] = times_ms[2] = 0.0;
    if (n_cw == 0) return HAMMING_OK;
    if (!host_cw || !host_data_out || !workspace) return HAMMING_EINVAL;
    if ((reinterpret_cast<uintptr_t>(host_cw) & 7u) || (reinterpret_cast<uintptr_t>(host_data_out) & 7u) ||
        (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return HAMMING_EALIGN;
    const uint32_t ns = mode == HAMMING_TRANSFER_SYNC ? 1u : streams;
    const StagingLayout L = staging(chunk_cw, r);
    if (workspace_bytes < L.per_stream * ns) return HAMMING_ENOMEM;

    const uint64_t wpc = r == 7 ? 2 : 1;
    const uint64_t k = (uint64_t(1) << r) - 1 - r;
    const uint64_t total_bytes = hamming_data_bytes(n_cw, r);
    std::vector<hipStream_t> st(ns, nullptr);
    int rc = HAMMING_OK;
    for (auto& s : st)
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) rc = HAMMING_EDEVICE;
    Timers tm;
    if (!tm.ok) rc = HAMMING_EDEVICE;

    const uint64_t chunks = (n_cw + chunk_cw - 1) / chunk_cw;
    for (uint64_t c = 0; c < chunks && rc == HAMMING_OK; ++c) {
        const uint32_t si = uint32_t(c % ns);
        hipStream_t s = st[si];
        char* base = static_cast<char*>(workspace) + si * L.per_stream;
        uint64_t* d_in = reinterpret_cast<uint64_t*>(base);
        char* d_data = base + L.in_bytes;
        uint8_t* d_ep = reinterpret_cast<uint8_t*>(base + L.in_bytes + L.data_bytes);
        const uint64_t c0 = c * chunk_cw;
        const uint64_t m = (n_cw - c0 < chunk_cw) ? n_cw - c0 : chunk_cw;
        // this chunk's messages start at stream byte c0*k/8 (a whole 64-bit word)
        const uint64_t out_off = c0 * k / 8;
        const uint64_t out_len = (c + 1 == chunks) ? total_bytes - out_off : m * k / 8;
        const bool timed = times_ms && mode == HAMMING_TRANSFER_SYNC;
        if (timed) (void)hipEventRecord(tm.e[0], s);
        if (hipMemcpyAsync(d_in, host_cw + c0 * wpc, m * wpc * 8, hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = HAMMING_EDEVICE;
            break;
        }
        if (timed) (void)hipEventRecord(tm.e[1], s);
        rc = hamming_decode(d_in, m, r, d_data, host_errpos_out ? d_ep : nullptr, s);
        if (rc != HAMMING_OK) break;
        if (timed) (void)hipEventRecord(tm.e[2], s);
        if (hipMemcpyAsync(static_cast<char*>(host_data_out) + out_off, d_data, out_len, hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            (host_errpos_out &&
             hipMemcpyAsync(host_errpos_out + c0, d_ep, m, hipMemcpyDeviceToHost, s) != hipSuccess)) {
            rc = HAMMING_EDEVICE;
            break;
        }
        if (timed) {
            (void)hipEventRecord(tm.e[3], s);
            float a = 0, b = 0, d = 0;
            if (hipEventSynchronize(tm.e[3]) != hipSuccess || hipEventElapsedTime(&a, tm.e[0], tm.e[1]) != hipSuccess ||
                hipEventElapsedTime(&b, tm.e[1], tm.e[2]) != hipSuccess ||
                hipEventElapsedTime(&d, tm.e[2], tm.e[3]) != hipSuccess) {
                rc = HAMMING_EDEVICE;
                break;
            }
            times_ms[0] += a;
            times_ms[1] += b;
            times_ms[2] += d;
        } else if (mode == HAMMING_TRANSFER_SYNC) {
            if (hipStreamSynchronize(s) != hipSuccess) rc = HAMMING_EDEVICE;
        }
    }
    for (auto& s : st) {
        if (!s) continue;
        if (hipStreamSynchronize(s) != hipSuccess && rc == HAMMING_OK) rc = HAMMING_EDEVICE;
        (void)hipStreamDestroy(s);
    }
    return rc;
}

}  // extern "C"

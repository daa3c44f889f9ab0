// Random record reads: the rate at which the memory system serves reads of
// short records at random positions of a large buffer, the access pattern of
// the neighbour-record gather. A measurement aid for roofline reports.
#include "device.hpp"

namespace {

__device__ inline uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// read r (of n_reads) is record mix64(r + salt) mod nrec, one 8-byte word per
// lane of its group of wpr lanes; the guarded store keeps the loads and fires
// only for the (zero-filled) buffer's impossible value
__global__ void __launch_bounds__(256) k_random_reads(const uint64_t *buf, uint64_t nrec, int wpr, int64_t n_reads,
                                                      uint64_t salt, uint64_t *sink)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t r = t / (uint64_t)wpr, j = t % (uint64_t)wpr;
    if (r >= (uint64_t)n_reads) return;
    const uint64_t rec = mix64(r + salt) % nrec;
    const uint64_t x = buf[rec * (uint64_t)wpr + j];
    if (x == 0x9e3779b97f4a7c15ull) sink[0] = x;
}

}  // namespace

extern "C" scc_status scc_probe_random_reads(const void *buf, uint64_t buf_bytes, int record_bytes, int64_t n_reads,
                                             uint64_t salt, uint64_t *sink, void *stream, float *ms_out)
{
    if (!buf || !sink || !ms_out) return set_error(SCC_EINVAL, "NULL argument");
    if (record_bytes < 8 || record_bytes > 256 || record_bytes % 8)
        return set_error(SCC_EINVAL, "record_bytes = %d not a multiple of 8 in [8, 256]", record_bytes);
    if ((uintptr_t)buf % 8) return set_error(SCC_EINVAL, "buffer not 8-byte aligned");
    const uint64_t nrec = buf_bytes / (uint64_t)record_bytes;
    if (nrec == 0) return set_error(SCC_EINVAL, "buffer smaller than one record");
    const int wpr = record_bytes / 8;
    if (n_reads < 0 || (uint64_t)n_reads * (uint64_t)wpr > (1ull << 31))
        return set_error(SCC_EINVAL, "n_reads = %lld out of range", (long long)n_reads);
    *ms_out = 0;
    if (n_reads == 0) return SCC_OK;
    const uint64_t threads = (uint64_t)n_reads * (uint64_t)wpr;
    hipStream_t st = (hipStream_t)stream;
    struct Ev {
        hipEvent_t e = nullptr;
        ~Ev() { if (e) (void)hipEventDestroy(e); }
    } e0, e1;
    HIP_TRY(hipEventCreate(&e0.e));
    HIP_TRY(hipEventCreate(&e1.e));
    HIP_TRY(hipEventRecord(e0.e, st));
    hipLaunchKernelGGL(k_random_reads, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st,
                       (const uint64_t *)buf, nrec, wpr, n_reads, salt, sink);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e1.e, st));
    HIP_TRY(hipEventSynchronize(e1.e));
    HIP_TRY(hipEventElapsedTime(ms_out, e0.e, e1.e));
    return SCC_OK;
}

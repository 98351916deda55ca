// Random row-gather throughput of the device (jag_gather_ceiling): the
// practical ceiling for the search's memory stream, which reads rows of a
// few hundred bytes at data-dependent indices.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "jag_internal.h"

namespace jag {
namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Each group of G lanes reads one row of ch * G * 16 bytes per step; the next
// row index mixes the first word the group read into its hash, so the loads
// of one group form a dependent chain.
template <int G>
__global__ __launch_bounds__(64) void gather_probe_kernel(const uint4 *__restrict__ base, uint32_t nrows,
                                                          int ch, int iters, uint32_t *sink)
{
    const int lane = threadIdx.x, sub = lane & (G - 1), grp = lane / G;
    uint32_t idx = mix32(blockIdx.x * 977u + (uint32_t)grp * 131u + 7u) % nrows;
    uint32_t acc = 0;
    for (int it = 0; it < iters; it++) {
        const uint4 *row = base + (size_t)idx * (size_t)(G * ch);
        uint32_t first = 0;
        for (int j = 0; j < ch; j++) {
            const uint4 v = row[j * G + sub];
            acc += v.x ^ v.y ^ v.z ^ v.w;
            if (j == 0) first = v.x;
        }
        // the group's lane 0 word of the row steers the next index
        first = __shfl(first, lane & ~(G - 1), 64);
        idx = mix32(idx * 2654435761u + (uint32_t)it + (first & 1u)) % nrows;
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads; practically never taken
}

}  // namespace
}  // namespace jag

extern "C" jag_status jag_gather_ceiling(const void *buffer, int64_t buffer_bytes, int32_t row_bytes,
                                         int32_t waves, int32_t iters, int32_t reps, void *stream,
                                         double *gbs_out)
{
    using namespace jag;
    if (!buffer || !gbs_out || row_bytes < 64 || row_bytes > 16384 || row_bytes % 64 || waves < 1 ||
        waves > (1 << 20) || iters < 1 || iters > 100000 || reps < 1 || reps > 100 ||
        buffer_bytes < 64 * (int64_t)row_bytes || buffer_bytes / row_bytes > (int64_t)UINT32_MAX) {
        set_error("jag_gather_ceiling: bad arguments");
        return JAG_EINVAL;
    }
    const int G = row_bytes <= 384 ? 4 : row_bytes <= 512 ? 8 : 16;
    if (row_bytes % (16 * G)) {
        set_error("jag_gather_ceiling: row_bytes must be a multiple of %d", 16 * G);
        return JAG_EINVAL;
    }
    const int ch = row_bytes / (16 * G);
    const uint32_t nrows = (uint32_t)(buffer_bytes / row_bytes);
    hipStream_t sm = (hipStream_t)stream;
    uint32_t *sink = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    float ms = 0.f;
    auto launch = [&]() {
        const uint4 *base = static_cast<const uint4 *>(buffer);
        if (G == 4) hipLaunchKernelGGL(gather_probe_kernel<4>, dim3(waves), dim3(64), 0, sm, base, nrows, ch, iters, sink);
        else if (G == 8) hipLaunchKernelGGL(gather_probe_kernel<8>, dim3(waves), dim3(64), 0, sm, base, nrows, ch, iters, sink);
        else hipLaunchKernelGGL(gather_probe_kernel<16>, dim3(waves), dim3(64), 0, sm, base, nrows, ch, iters, sink);
        return hipGetLastError();
    };
    hipError_t e = hipMalloc((void **)&sink, 64);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(a, sm);
    for (int r = 0; r < reps && e == hipSuccess; r++) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, sm);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (sink) (void)hipFree(sink);
    if (e != hipSuccess) {
        set_error("jag_gather_ceiling: %s", hipGetErrorString(e));
        return JAG_EDEVICE;
    }
    const double bytes = (double)waves * (64 / G) * (double)iters * row_bytes * reps;
    *gbs_out = ms > 0.f ? bytes / (ms * 1e-3) / 1e9 : 0.0;
    return JAG_OK;
}

// Resident serving waves: slot-level admission for the request server.
//
// A launch places up to the device's resident capacity of one-wave
// workgroups, each with the LDS of one query's search.  Every wave loops:
// take a ticket (one atomic add on a device counter), wait until request
// number `ticket` has been published, copy its query and distance table into
// the wave's own device memory, run the search of Algorithm 2 over
// Algorithm 1 (search_device.h) and write the answer straight into the
// host's result rows.  A wave therefore takes a new request the moment its
// previous one ends, and requests are served in arrival order: a request
// waits only for a free wave, never for the rest of a batch.
//
// The device-side count of available requests is raised by one wave only:
// the one whose ticket is the next request to arrive (the head of the line).
// It polls the host's publish counter once per poll interval; the waves
// behind it sleep for longer the further back they are, so the waiting
// waves cost little memory traffic.  The head also ends the launch: after
// the idle interval without a new request, or when the host asks for a stop,
// it sets the closing bit of the available count, which freezes the count.
// Waves holding a ticket below the frozen count serve it; the others leave.
// The host then finds the launch ended with requests left over, moves the
// ticket counter back to the frozen count and launches again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "jag_internal.h"
#include "search_device.h"

namespace jag {
namespace {

constexpr uint64_t kClosing = 1ull << 63;

__device__ __forceinline__ uint64_t bcast64(uint64_t v)
{
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

__device__ __forceinline__ void nap(int n)
{
    for (int i = 0; i < n; i++) __builtin_amdgcn_s_sleep(127);  // about 8,000 clocks each
}

// The request this wave may serve next, or -1 when the launch is closing and
// the wave's ticket is beyond the frozen count.
__device__ int64_t wait_for_request(const ServeRing &r)
{
    const int lane = threadIdx.x;
    uint64_t *ticket = r.dctl + kServeTicketWord;
    uint64_t *avail = r.dctl + kServeAvailWord;
    uint64_t *raised = r.dctl + kServeRaisedWord;
    const uint64_t t =
        bcast64(lane == 0 ? __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0);
    const uint64_t since = wall_clock64();
    uint64_t last_poll = since - (uint64_t)r.poll_ticks;
    for (;;) {
        const uint64_t v = bcast64(
            lane == 0 ? __hip_atomic_load(avail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) : 0);
        const uint64_t av = v & ~kClosing;
        if (av > t) return (int64_t)t;
        if (v & kClosing) return -1;
        if (t == av) {
            // head of the line: poll the host, close when idle or asked to stop
            if (lane == 0) {
                const uint64_t now = wall_clock64();
                if ((int64_t)(now - last_poll) >= r.poll_ticks) {
                    last_poll = now;
                    const uint64_t pub = __hip_atomic_load(r.ctl + 0, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                    const uint64_t stop = __hip_atomic_load(r.ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    if (pub > av && !stop) {
                        __hip_atomic_store(raised, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_max(avail, pub, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        // idle since this wave took its ticket and since the last new request
                        const uint64_t last = __hip_atomic_load(raised, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const uint64_t from = (int64_t)(last - since) > 0 ? last : since;
                        if (stop || (int64_t)(now - from) >= r.idle_ticks)
                            __hip_atomic_fetch_or(avail, kClosing, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
            __builtin_amdgcn_s_sleep(16);
        } else {
            const uint64_t dist = t - av;
            nap(dist < 248 ? 1 + (int)(dist >> 3) : 32);
        }
    }
}

template <int STORE, int G, int CH, int WPE, int SL, int AK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void serve_kernel(SearchArgs a,
                                                                                           ServeRing r)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    float *qcopy = reinterpret_cast<float *>(r.wave_mem + (int64_t)blockIdx.x * r.wave_bytes);
    uint8_t *tcopy = r.wave_mem + (int64_t)blockIdx.x * r.wave_bytes + ((int64_t)4 * a.d + 255) / 256 * 256;
    for (;;) {
        const int64_t h = wait_for_request(r);
        if (h < 0) break;
        const uint32_t slot = (uint32_t)h & r.cmask;
        const unsigned char *req = r.req + (int64_t)slot * r.req_stride;
        // drop any cached copy of host memory before reading the slot
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        const uint64_t seq = lane == 0 ? __hip_atomic_load(reinterpret_cast<const uint64_t *>(req + 128),
                                                           __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM)
                                       : 0ull;
        const bool seq_ok = __builtin_amdgcn_readfirstlane((uint32_t)(seq == (uint64_t)h + 1)) != 0;
        // the record, one word per lane, gathered into uniform registers
        const uint32_t word = lane < 32 ? reinterpret_cast<const uint32_t *>(req)[lane] : 0u;
        FilterRecord f;
        uint32_t *fw = reinterpret_cast<uint32_t *>(&f);
#pragma unroll
        for (int i = 0; i < 32; i++) fw[i] = __builtin_amdgcn_readlane(word, i);
        int32_t *ids_out = r.ids + (int64_t)slot * a.k;
        float *dists_out = r.dists + (int64_t)slot * a.k;
        if (seq_ok) {
            const float *qsrc = reinterpret_cast<const float *>(req + kServeSlotHeader);
            for (int i = lane; i < a.d; i += 64) qcopy[i] = qsrc[i];
            const uint8_t *tab = nullptr;
            if (f.type == F_TABLE) {
                const int tb = (1 << f.nlit) > 16 ? (1 << f.nlit) : 16;
                const uint4 *src = reinterpret_cast<const uint4 *>(r.tab + f.table_off);
                uint4 *dst = reinterpret_cast<uint4 *>(tcopy);
                for (int i = lane; i < tb / 16; i += 64) dst[i] = src[i];
                tab = tcopy;
            }
            // the copies are read back by this wave only
            __syncthreads();
            search_query<STORE, G, CH, SL, AK>(a, 0, f, tab, qcopy, ids_out, dists_out, r.count + slot, smem);
        } else if (lane == 0) {
            r.count[slot] = -1;
        }
        // the answer reaches host memory before the done word does
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        if (lane == 0)
            __hip_atomic_store(r.done + slot, (uint64_t)h + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Before a launch: tickets start again at the first request not served (the
// frozen count of the last launch), and the closing bit is cleared.
__global__ void serve_reset_kernel(uint64_t *dctl)
{
    if (threadIdx.x == 0) {
        const uint64_t av =
            __hip_atomic_load(dctl + kServeAvailWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ~kClosing;
        __hip_atomic_store(dctl + kServeTicketWord, av, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(dctl + kServeAvailWord, av, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

using ServeFn = void (*)(SearchArgs, ServeRing);

struct ServeFamily {
    using Fn = ServeFn;
    template <int STORE, int G, int CH, int WPE, int SL, int AK>
    static Fn get()
    {
        return serve_kernel<STORE, G, CH, WPE, SL, AK>;
    }
};

ServeFn pick_serve(int store, int stride, int R, int ak)
{
    int G = pick_group(stride);
    int ch = stride / (16 * G);
    using F = ServeFamily;
    if (R > 64) return family_pick_sl<F, kWavesPerSimd, 2, AK_ANY>(store, G, ch);
    if (ak == AK_SCALAR) return family_pick_sl<F, kWavesPerSimd, 1, AK_SCALAR>(store, G, ch);
    if (ak == AK_LABELS) return family_pick_sl<F, kWavesPerSimd, 1, AK_LABELS>(store, G, ch);
    return family_pick_sl<F, kWavesPerSimd, 1, AK_ANY>(store, G, ch);
}

// The search a server wave runs: a fixed beam, or the learned beam in one
// pass (the prediction taken inside the wave's own search).
jag_status plan_serve(Index &ix, int32_t k, const jag_search_params &S, SearchArgs &a, ServeFn &fn,
                      size_t &lds)
{
    if (S.learned != 0 && S.learned != 1) {
        set_error("resident server waves run fixed (learned = 0) or learned one-pass (1) searches");
        return JAG_EINVAL;
    }
    jag_search_params s2 = S;
    s2.single_pass = 1;
    float dummy = 0.f;
    int ak = AK_ANY;
    jag_status st = plan_search(ix, &dummy, 1, &dummy, k, s2, nullptr, nullptr, nullptr, a, lds, ak);
    if (st != JAG_OK) return st;
    fn = pick_serve(ix.store, ix.vec_stride, ix.R, ak);
    if (!fn) {
        set_error("no serving kernel for row stride %d", ix.vec_stride);
        return JAG_EUNSUPPORTED;
    }
    a.Q = nullptr;
    a.rec = nullptr;
    return JAG_OK;
}

}  // namespace

jag_status serve_capacity(Index &ix, int32_t k, const jag_search_params &S, int64_t *resident)
{
    SearchArgs a;
    ServeFn fn = nullptr;
    size_t lds = 0;
    jag_status st = plan_serve(ix, k, S, a, fn, lds);
    if (st != JAG_OK) return st;
    int per_cu = 0;
    hipDeviceProp_t prop;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), 64, lds) !=
            hipSuccess ||
        hipGetDeviceProperties(&prop, ix.device) != hipSuccess) {
        set_error("cannot query the serving kernel's occupancy");
        return JAG_EDEVICE;
    }
    *resident = (int64_t)per_cu * prop.multiProcessorCount;
    return JAG_OK;
}

jag_status launch_serve(Index &ix, int32_t k, const jag_search_params &S, const ServeRing &r, int64_t waves,
                        void *stream)
{
    SearchArgs a;
    ServeFn fn = nullptr;
    size_t lds = 0;
    jag_status st = plan_serve(ix, k, S, a, fn, lds);
    if (st != JAG_OK) return st;
    if (waves < 1 || waves > INT_MAX || !r.req || !r.ids || !r.dists || !r.count || !r.done || !r.ctl ||
        !r.dctl || !r.wave_mem || r.wave_bytes < serve_wave_bytes(ix.d) || (r.cmask & (r.cmask + 1)) != 0) {
        set_error("bad serving launch");
        return JAG_EINVAL;
    }
    hipLaunchKernelGGL(serve_reset_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, r.dctl);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fn, dim3((unsigned)waves), dim3(64), lds, (hipStream_t)stream, a, r);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        set_error("serving kernel launch failed: %s", hipGetErrorString(e));
        return JAG_EDEVICE;
    }
    return JAG_OK;
}

}  // namespace jag

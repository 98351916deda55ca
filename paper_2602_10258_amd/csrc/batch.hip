// jag_search_batch: host filters encoded into pinned staging buffers and
// uploaded on the index's copy stream, then the batched search of
// search.hip.  Host code only (no kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "jag_internal.h"

namespace jag {

// Pinned host buffers of jag_search_batch (see the staging section below).
struct StagingBuf {
    unsigned char *host = nullptr;
    size_t cap = 0;
    hipEvent_t copied = nullptr;  // recorded after the copy out of `host`
    bool filling = false;         // a caller is encoding into it
};

struct StagingRing {
    std::mutex mu;
    std::vector<StagingBuf> bufs;
    // the uploads run on a stream of their own, so that a call's copy does
    // not wait behind the caller's earlier work (created on first use)
    hipStream_t copy = nullptr;
};

StagingRing *new_staging() { return new StagingRing(); }

}  // namespace jag

// ---------------------------------------------------------------- staging
// jag_search_batch encodes host filters into pinned host memory and copies
// them to the device asynchronously; an event recorded after the copy says
// when a buffer may be filled again, so the call never waits for the stream.
namespace jag {

constexpr size_t kStagingMax = 8;  // buffers per index; beyond that a caller waits

void free_staging(StagingRing *r)
{
    if (!r) return;
    if (r->copy) {
        (void)hipStreamSynchronize(r->copy);
        (void)hipStreamDestroy(r->copy);
    }
    for (auto &b : r->bufs) {
        if (b.copied) {
            (void)hipEventSynchronize(b.copied);
            (void)hipEventDestroy(b.copied);
        }
        if (b.host) (void)hipHostFree(b.host);
    }
    delete r;
}

// A pinned buffer of at least `bytes` that no pending copy reads: a free one,
// a new one while the ring is short, else the least recently filled one once
// its copy has completed.  Returns its slot, or -1 with the error set.
static int staging_acquire(StagingRing *r, size_t bytes)
{
    int pick = -1;
    {
        std::lock_guard<std::mutex> g(r->mu);
        for (size_t i = 0; i < r->bufs.size() && pick < 0; i++) {
            StagingBuf &b = r->bufs[i];
            if (!b.filling && (!b.copied || hipEventQuery(b.copied) == hipSuccess)) pick = (int)i;
        }
        if (pick < 0 && r->bufs.size() < kStagingMax) {
            r->bufs.emplace_back();
            pick = (int)r->bufs.size() - 1;
        }
        if (pick < 0)
            for (size_t i = 0; i < r->bufs.size() && pick < 0; i++)
                if (!r->bufs[i].filling) pick = (int)i;
        if (pick < 0) {
            set_error("all %zu filter staging buffers are being filled by other calls", r->bufs.size());
            return -1;
        }
        r->bufs[(size_t)pick].filling = true;
    }
    StagingBuf &b = r->bufs[(size_t)pick];
    if (b.copied && hipEventSynchronize(b.copied) != hipSuccess) {
        std::lock_guard<std::mutex> g(r->mu);
        b.filling = false;
        set_error("filter staging copy failed");
        return -1;
    }
    if (!b.copied && hipEventCreateWithFlags(&b.copied, hipEventDisableTiming) != hipSuccess) {
        std::lock_guard<std::mutex> g(r->mu);
        b.filling = false;
        set_error("event creation failed");
        return -1;
    }
    if (b.cap < bytes) {
        if (b.host) (void)hipHostFree(b.host);
        b.host = nullptr;
        b.cap = 0;
        const size_t cap = std::max<size_t>((bytes + 4095) / 4096 * 4096, size_t(1) << 20);
        if (hipHostMalloc((void **)&b.host, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            std::lock_guard<std::mutex> g(r->mu);
            b.filling = false;
            set_error("pinned staging allocation of %zu bytes failed", cap);
            return -1;
        }
        b.cap = cap;
    }
    return pick;
}

static void staging_release(StagingRing *r, int slot)
{
    std::lock_guard<std::mutex> g(r->mu);
    r->bufs[(size_t)slot].filling = false;
}

}  // namespace jag

extern "C" jag_status jag_search_batch(jag_index *idx, const float *Q, int64_t nq,
                                       const jag_filter *F, const int32_t *pool, int64_t pool_len,
                                       int32_t k, const jag_search_params *S, int32_t *ids,
                                       float *dists, int32_t *count, void *stream)
{
    if (nq == 0) return JAG_OK;
    if (!idx || !S || nq < 0 || !F) {
        jag::set_error("null argument");
        return JAG_EINVAL;
    }
    jag::Index &ix = idx->ix;
    int64_t bytes = 0;
    jag_status st = jag_encoded_bytes(idx, F, nq, pool, pool_len, &bytes);
    if (st != JAG_OK) return st;
    if (!ix.staging) {
        jag::set_error("index has no staging ring");
        return JAG_EDEVICE;
    }
    const int slot = jag::staging_acquire(ix.staging, (size_t)bytes);
    if (slot < 0) return JAG_ENOMEM;
    jag::StagingBuf &buf = ix.staging->bufs[(size_t)slot];
    st = jag_encode_filters_sized(idx, F, nq, pool, pool_len, buf.host, bytes);
    if (st != JAG_OK) {
        jag::staging_release(ix.staging, slot);
        return st;
    }
    // The records go up on the ring's copy stream: the copy of one call then
    // overlaps the searches still running on the caller's stream, which
    // waits for the copy only where its search begins.
    hipStream_t s = (hipStream_t)stream;
    {
        std::lock_guard<std::mutex> g(ix.staging->mu);
        if (!ix.staging->copy && hipStreamCreateWithFlags(&ix.staging->copy, hipStreamNonBlocking) != hipSuccess) {
            ix.staging->copy = nullptr;
            (void)hipGetLastError();
        }
    }
    hipStream_t cs = ix.staging->copy ? ix.staging->copy : s;
    void *drec = nullptr;
    if (hipMallocAsync(&drec, (size_t)bytes, cs) != hipSuccess) {
        (void)hipGetLastError();
        jag::staging_release(ix.staging, slot);
        jag::set_error("device allocation for filter records failed");
        return JAG_ENOMEM;
    }
    hipError_t e = hipMemcpyAsync(drec, buf.host, (size_t)bytes, hipMemcpyHostToDevice, cs);
    // the buffer may be filled again, and the search may start, once this copy has run
    hipError_t er = hipEventRecord(buf.copied, cs);
    if (e == hipSuccess && er == hipSuccess && cs != s) er = hipStreamWaitEvent(s, buf.copied, 0);
    jag::staging_release(ix.staging, slot);
    if (e != hipSuccess || er != hipSuccess) {
        (void)hipFreeAsync(drec, cs);
        jag::set_error("filter upload failed: %s", hipGetErrorString(e != hipSuccess ? e : er));
        return JAG_EDEVICE;
    }
    st = jag_search_encoded(idx, Q, nq, drec, k, S, ids, dists, count, stream);
    (void)hipFreeAsync(drec, s);
    return st;
}

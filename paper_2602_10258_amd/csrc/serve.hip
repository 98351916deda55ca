// Request server: single filtered queries admitted to the GPU as they come.
//
// Callers queue requests (jag_server_submit) from any thread; a scheduler
// thread admits them in one of two ways.
//
// Batches: the thread keeps up to n_streams batches on the GPU, one HIP
// stream each.  Whenever a stream is idle and requests are pending it
// gathers up to max_batch of them -- without exceeding max_inflight requests
// on the GPU --, stages their vectors and filter records in pinned host
// memory, copies them to the stream's device buffers, launches the search
// kernel and copies the results back, all asynchronously on that stream.
// Finished streams are found with hipEventQuery and their requests
// completed.
//
// Slots: one launch of resident waves (serve_kernels.hip) takes requests one
// at a time.  The thread writes each request into the next free slot of a
// ring in fine-grained pinned host memory and publishes it by raising a
// counter there; a free wave claims it, searches, writes the answer into the
// slot's result rows and marks the slot done.  The thread collects done
// slots, frees them in order and starts the waves again whenever they have
// ended (after an idle interval) with published requests left.
//
// Each query's beam lives in its own wavefront's LDS for the whole search,
// so a result does not depend on the batch or the company it ran in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "jag_internal.h"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    uint64_t ticket;
    jag::FilterRecord rec;
    std::vector<uint8_t> table;  // distance table of a TABLE filter (2^nvar bytes)
    std::vector<float> q;
    clk::time_point t_submit;
};

struct Done {
    std::vector<int32_t> ids;
    std::vector<float> dists;
    int32_t count;
    double latency_us;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    // pinned host staging and device buffers sized for max_batch requests
    float *h_q = nullptr;
    jag::FilterRecord *h_rec = nullptr;
    int32_t *h_ids = nullptr, *h_cnt = nullptr;
    float *h_d = nullptr;
    float *d_q = nullptr;
    jag::FilterRecord *d_rec = nullptr;
    int32_t *d_ids = nullptr, *d_cnt = nullptr;
    float *d_d = nullptr;
    // distance tables of the batch's TABLE filters, grown on demand
    uint8_t *h_tab = nullptr, *d_tab = nullptr;
    size_t tab_cap = 0;
    std::vector<Request> batch;
    int64_t batch_no = 0;  // 1-based count of the server's launches
    bool busy = false;
};

// Slot admission: the ring in fine-grained pinned host memory, the waves'
// device memory, and the thread's bookkeeping per slot.
struct Ring {
    int64_t C = 0;
    int64_t req_stride = 0;
    unsigned char *h_req = nullptr;
    unsigned char *h_tab = nullptr;
    int64_t tab_cap = 0;
    int32_t *h_ids = nullptr, *h_cnt = nullptr;
    float *h_d = nullptr;
    uint64_t *h_done = nullptr, *h_ctl = nullptr;
    uint64_t *d_ctl = nullptr;
    unsigned char *d_wave = nullptr;
    jag::ServeRing view{};  // what the waves see (device addresses)
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    int64_t waves = 0;
    bool running = false;
    int64_t launches = 0;
    // per slot: the request it holds, whether its answer was collected, and
    // the table area's write position after its table
    std::vector<uint64_t> ticket;
    std::vector<clk::time_point> t_submit;
    std::vector<uint8_t> collected;
    std::vector<int64_t> tab_end;
    int64_t published = 0;   // requests written to the ring
    int64_t freed = 0;       // requests whose slots are free again (a prefix)
    int64_t finished = 0;    // requests collected
    int64_t tab_head = 0, tab_tail = 0;  // table area: next write, oldest live byte
};

constexpr int64_t kRingTableBytes = 8ll << 20;
constexpr int64_t kServePollUs = 2;
constexpr int64_t kServeIdleUs = 10000;
constexpr int kServeStallS = 10;

}  // namespace

struct jag_server {
    jag_index *idx = nullptr;
    jag_server_params P{};
    int64_t max_inflight = 0, resident = 0;
    std::vector<Slot> slots;
    bool slot_mode = false;
    Ring ring;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::unordered_map<uint64_t, Done> done;
    std::vector<double> latencies;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, batches = 0, inflight = 0, max_inflight_seen = 0;
    int64_t batched_requests = 0;
    clk::time_point t_first{}, t_last{};
    bool have_first = false;
    bool stop = false;
    std::string error;
    std::thread worker;
    int64_t device_bytes = 0;
    // Failure handling test hook: JAG_SERVER_TEST_FAIL_BATCH = b (b >= 1) makes
    // the completion check of the server's b-th batch report a device error
    // once that batch has finished normally (nothing faults on the device).
    int64_t test_fail_batch = 0;
};

namespace {

#define HIPOK(expr) ((expr) == hipSuccess)

void free_slot(Slot &s)
{
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.event) (void)hipEventDestroy(s.event);
    for (void *p : {(void *)s.h_q, (void *)s.h_rec, (void *)s.h_ids, (void *)s.h_cnt, (void *)s.h_d,
                    (void *)s.h_tab})
        if (p) (void)hipHostFree(p);
    for (void *p : {(void *)s.d_q, (void *)s.d_rec, (void *)s.d_ids, (void *)s.d_cnt, (void *)s.d_d,
                    (void *)s.d_tab})
        if (p) (void)hipFree(p);
    s = Slot();
}

bool alloc_slot(Slot &s, int B, int d, int k)
{
    return HIPOK(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) &&
           HIPOK(hipEventCreateWithFlags(&s.event, hipEventDisableTiming)) &&
           HIPOK(hipHostMalloc((void **)&s.h_q, sizeof(float) * B * d, hipHostMallocDefault)) &&
           HIPOK(hipHostMalloc((void **)&s.h_rec, sizeof(jag::FilterRecord) * B, hipHostMallocDefault)) &&
           HIPOK(hipHostMalloc((void **)&s.h_ids, sizeof(int32_t) * B * k, hipHostMallocDefault)) &&
           HIPOK(hipHostMalloc((void **)&s.h_cnt, sizeof(int32_t) * B, hipHostMallocDefault)) &&
           HIPOK(hipHostMalloc((void **)&s.h_d, sizeof(float) * B * k, hipHostMallocDefault)) &&
           HIPOK(hipMalloc((void **)&s.d_q, sizeof(float) * B * d)) &&
           HIPOK(hipMalloc((void **)&s.d_rec, sizeof(jag::FilterRecord) * B)) &&
           HIPOK(hipMalloc((void **)&s.d_ids, sizeof(int32_t) * B * k)) &&
           HIPOK(hipMalloc((void **)&s.d_cnt, sizeof(int32_t) * B)) &&
           HIPOK(hipMalloc((void **)&s.d_d, sizeof(float) * B * k));
}

int64_t slot_device_bytes(int B, int d, int k)
{
    return (int64_t)B * (4 * d + (int64_t)sizeof(jag::FilterRecord) + 8 * k + 4);
}

// Launch one batch on a free slot (called with the lock released).
bool launch(jag_server *S, Slot &s)
{
    jag::Index &ix = S->idx->ix;
    const int d = ix.d, k = S->P.k;
    const int n = (int)s.batch.size();
    // TABLE filters: their distance tables go to the slot's table arena, and
    // each record points there (table_off counts from the record's own address)
    size_t tab_bytes = 0;
    for (int i = 0; i < n; i++)
        if (!s.batch[i].table.empty()) tab_bytes = (tab_bytes + 15) / 16 * 16 + s.batch[i].table.size();
    if (tab_bytes > s.tab_cap) {
        if (s.h_tab) (void)hipHostFree(s.h_tab);
        if (s.d_tab) (void)hipFree(s.d_tab);
        s.h_tab = nullptr;
        s.d_tab = nullptr;
        s.tab_cap = 0;
        const size_t cap = std::max<size_t>(tab_bytes, (size_t)1 << 20);
        if (!HIPOK(hipHostMalloc((void **)&s.h_tab, cap, hipHostMallocDefault)) ||
            !HIPOK(hipMalloc((void **)&s.d_tab, cap))) {
            jag::set_error("server table arena allocation failed");
            return false;
        }
        s.tab_cap = cap;
    }
    size_t tpos = 0;
    for (int i = 0; i < n; i++) {
        std::memcpy(s.h_q + (size_t)i * d, s.batch[i].q.data(), sizeof(float) * d);
        s.h_rec[i] = s.batch[i].rec;
        if (!s.batch[i].table.empty()) {
            tpos = (tpos + 15) / 16 * 16;
            std::memcpy(s.h_tab + tpos, s.batch[i].table.data(), s.batch[i].table.size());
            s.h_rec[i].table_off = (int64_t)((intptr_t)(s.d_tab + tpos) - (intptr_t)(s.d_rec + i));
            tpos += s.batch[i].table.size();
        }
    }
    bool ok = HIPOK(hipMemcpyAsync(s.d_q, s.h_q, sizeof(float) * n * d, hipMemcpyHostToDevice, s.stream)) &&
              HIPOK(hipMemcpyAsync(s.d_rec, s.h_rec, sizeof(jag::FilterRecord) * n, hipMemcpyHostToDevice,
                                   s.stream)) &&
              (tab_bytes == 0 ||
               HIPOK(hipMemcpyAsync(s.d_tab, s.h_tab, tab_bytes, hipMemcpyHostToDevice, s.stream)));
    if (ok) {
        jag_search_params sp = S->P.search;
        ok = jag::launch_search(ix, s.d_q, n, s.d_rec, k, sp, s.d_ids, s.d_d, s.d_cnt, s.stream) == JAG_OK;
    }
    ok = ok && HIPOK(hipMemcpyAsync(s.h_ids, s.d_ids, sizeof(int32_t) * n * k, hipMemcpyDeviceToHost, s.stream)) &&
         HIPOK(hipMemcpyAsync(s.h_d, s.d_d, sizeof(float) * n * k, hipMemcpyDeviceToHost, s.stream)) &&
         HIPOK(hipMemcpyAsync(s.h_cnt, s.d_cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s.stream)) &&
         HIPOK(hipEventRecord(s.event, s.stream));
    return ok;
}

// Completion state of a slot's batch: hipSuccess, hipErrorNotReady, or the
// error that ended it (the test hook turns success into a failure).
hipError_t batch_status(const jag_server *S, const Slot &s)
{
    hipError_t e = hipEventQuery(s.event);
    if (e == hipSuccess && S->test_fail_batch > 0 && s.batch_no == S->test_fail_batch)
        e = hipErrorLaunchFailure;
    return e;
}

// A batch ended in a device error: the server stops.  Its requests, and every
// request still pending, never complete; poll and drain report JAG_EDEVICE,
// submit refuses new requests, and stop waits for the other streams.
void fail(jag_server *S, Slot &s, hipError_t e)
{
    std::lock_guard<std::mutex> g(S->mu);
    char msg[256];
    std::snprintf(msg, sizeof msg, "batch %lld of %zu requests failed on the device: %s",
                  (long long)s.batch_no, s.batch.size(), hipGetErrorString(e));
    S->error = msg;
    S->inflight -= (int64_t)s.batch.size();
    s.batch.clear();
    s.busy = false;
    S->stop = true;
    S->cv_done.notify_all();
}

void finish(jag_server *S, Slot &s)
{
    const int k = S->P.k;
    auto now = clk::now();
    std::lock_guard<std::mutex> g(S->mu);
    for (size_t i = 0; i < s.batch.size(); i++) {
        Done r;
        r.ids.assign(s.h_ids + i * k, s.h_ids + (i + 1) * k);
        r.dists.assign(s.h_d + i * k, s.h_d + (i + 1) * k);
        r.count = s.h_cnt[i];
        r.latency_us = std::chrono::duration<double, std::micro>(now - s.batch[i].t_submit).count();
        S->latencies.push_back(r.latency_us);
        S->done.emplace(s.batch[i].ticket, std::move(r));
    }
    S->completed += (int64_t)s.batch.size();
    S->inflight -= (int64_t)s.batch.size();
    S->t_last = now;
    s.batch.clear();
    s.busy = false;
    S->cv_done.notify_all();
}

void worker_loop(jag_server *S)
{
    (void)hipSetDevice(S->idx->ix.device);
    const auto max_wait = std::chrono::microseconds(S->P.max_wait_us);
    for (;;) {
        bool progressed = false;
        // 1. retire finished batches; any status but "not ready" from a
        // batch that did not succeed stops the server
        for (auto &s : S->slots) {
            if (!s.busy) continue;
            const hipError_t e = batch_status(S, s);
            if (e == hipSuccess) {
                finish(S, s);
                progressed = true;
            } else if (e != hipErrorNotReady) {
                fail(S, s, e);
                return;
            }
        }
        // 2. admit pending requests onto idle streams
        for (auto &s : S->slots) {
            if (s.busy) continue;
            {
                std::unique_lock<std::mutex> lk(S->mu);
                if (S->pending.empty()) break;
                int64_t room = S->max_inflight - S->inflight;
                if (room <= 0) break;
                int64_t want = std::min<int64_t>({(int64_t)S->P.max_batch, room, (int64_t)S->pending.size()});
                // a partial batch waits briefly for company while other batches run
                bool others = S->inflight > 0;
                if (want < S->P.max_batch && others &&
                    clk::now() - S->pending.front().t_submit < max_wait)
                    break;
                for (int64_t i = 0; i < want; i++) {
                    s.batch.push_back(std::move(S->pending.front()));
                    S->pending.pop_front();
                }
                S->inflight += want;
                S->max_inflight_seen = std::max(S->max_inflight_seen, S->inflight);
                S->batches++;
                S->batched_requests += want;
                s.batch_no = S->batches;
                s.busy = true;
            }
            if (!launch(S, s)) {
                std::lock_guard<std::mutex> g(S->mu);
                S->error = jag_last_error();
                S->stop = true;
                S->cv_done.notify_all();
                return;
            }
            progressed = true;
        }
        {
            std::unique_lock<std::mutex> lk(S->mu);
            bool busy = false;
            for (auto &s : S->slots) busy |= s.busy;
            if (S->stop && S->pending.empty() && !busy) return;
            if (!progressed) {
                if (!busy && S->pending.empty())
                    S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                else {
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
                }
            }
        }
    }
}

// ---------------------------------------------------------------- slots
void free_ring(Ring &R)
{
    if (R.stream) (void)hipStreamSynchronize(R.stream);
    if (R.stream) (void)hipStreamDestroy(R.stream);
    if (R.event) (void)hipEventDestroy(R.event);
    for (void *p : {(void *)R.h_req, (void *)R.h_tab, (void *)R.h_ids, (void *)R.h_cnt, (void *)R.h_d,
                    (void *)R.h_done, (void *)R.h_ctl})
        if (p) (void)hipHostFree(p);
    for (void *p : {(void *)R.d_ctl, (void *)R.d_wave})
        if (p) (void)hipFree(p);
    R = Ring();
}

// Fine-grained pinned host memory, zeroed, and its device address.
template <class T>
bool host_coherent(T **h, int64_t bytes)
{
    if (!HIPOK(hipHostMalloc((void **)h, (size_t)bytes, hipHostMallocCoherent | hipHostMallocMapped))) {
        *h = nullptr;
        return false;
    }
    std::memset((void *)*h, 0, (size_t)bytes);
    return true;
}

template <class T>
bool device_address(T *h, T **d)
{
    void *p = nullptr;
    if (!HIPOK(hipHostGetDevicePointer(&p, (void *)h, 0))) return false;
    *d = static_cast<T *>(p);
    return true;
}

int64_t ring_device_bytes(int64_t waves, int32_t d)
{
    return waves * jag::serve_wave_bytes(d) + jag::kServeCtlWords * (int64_t)sizeof(uint64_t);
}

jag_status alloc_ring(jag_server *S, int64_t waves)
{
    Ring &R = S->ring;
    const int d = S->idx->ix.d, k = S->P.k;
    int64_t C = 1024;
    while (C < 2 * waves) C *= 2;
    R.C = C;
    R.req_stride = jag::kServeSlotHeader + ((int64_t)4 * d + 15) / 16 * 16;
    R.tab_cap = kRingTableBytes;
    R.waves = waves;
    int rate_khz = 0;
    bool ok = HIPOK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, S->idx->ix.device)) &&
              rate_khz > 0 && host_coherent(&R.h_req, C * R.req_stride) &&
              host_coherent(&R.h_tab, R.tab_cap) && host_coherent(&R.h_ids, C * k * 4) &&
              host_coherent(&R.h_d, C * k * 4) && host_coherent(&R.h_cnt, C * 4) &&
              host_coherent(&R.h_done, C * 8) && host_coherent(&R.h_ctl, 64) &&
              HIPOK(hipMalloc((void **)&R.d_ctl, jag::kServeCtlWords * sizeof(uint64_t))) &&
              HIPOK(hipMemset(R.d_ctl, 0, jag::kServeCtlWords * sizeof(uint64_t))) &&
              HIPOK(hipMalloc((void **)&R.d_wave, (size_t)(waves * jag::serve_wave_bytes(d)))) &&
              HIPOK(hipStreamCreateWithFlags(&R.stream, hipStreamNonBlocking)) &&
              HIPOK(hipEventCreateWithFlags(&R.event, hipEventDisableTiming));
    jag::ServeRing &v = R.view;
    ok = ok && device_address(R.h_req, const_cast<unsigned char **>(&v.req)) &&
         device_address(R.h_tab, const_cast<unsigned char **>(&v.tab)) && device_address(R.h_ids, &v.ids) &&
         device_address(R.h_d, &v.dists) && device_address(R.h_cnt, &v.count) &&
         device_address(R.h_done, &v.done) && device_address(R.h_ctl, const_cast<uint64_t **>(&v.ctl));
    if (!ok) {
        free_ring(R);
        jag::set_error("server ring allocation failed");
        return JAG_ENOMEM;
    }
    const int64_t per_us = std::max<int64_t>(1, rate_khz / 1000);
    v.dctl = R.d_ctl;
    v.wave_mem = R.d_wave;
    v.wave_bytes = jag::serve_wave_bytes(d);
    v.poll_ticks = kServePollUs * per_us;
    v.idle_ticks = kServeIdleUs * per_us;
    v.cmask = (uint32_t)(C - 1);
    v.req_stride = (int32_t)R.req_stride;
    R.ticket.assign(C, 0);
    R.t_submit.assign(C, clk::time_point{});
    R.collected.assign(C, 1);
    R.tab_end.assign(C, 0);
    return JAG_OK;
}

// Write pending requests into free ring slots (lock held); returns how many.
int64_t ring_publish(jag_server *S)
{
    Ring &R = S->ring;
    const int d = S->idx->ix.d;
    int64_t n = 0;
    while (!S->pending.empty() && R.published - R.freed < R.C) {
        Request &q = S->pending.front();
        int64_t tpos = -1, tend = R.tab_head;
        if (!q.table.empty()) {
            const int64_t size = std::max<int64_t>(16, ((int64_t)q.table.size() + 15) / 16 * 16);
            int64_t head = R.tab_head;
            if (head % R.tab_cap + size > R.tab_cap) head += R.tab_cap - head % R.tab_cap;  // wrap
            if (head + size - R.tab_tail > R.tab_cap) break;  // wait for tables to be freed
            tpos = head % R.tab_cap;
            std::memcpy(R.h_tab + tpos, q.table.data(), q.table.size());
            tend = head + size;
        }
        const int64_t h = R.published;
        const int64_t slot = h & (R.C - 1);
        unsigned char *p = R.h_req + slot * R.req_stride;
        jag::FilterRecord rec = q.rec;
        if (tpos >= 0) rec.table_off = tpos;
        std::memcpy(p, &rec, sizeof rec);
        const uint64_t seq = (uint64_t)h + 1;
        std::memcpy(p + 128, &seq, sizeof seq);
        std::memcpy(p + jag::kServeSlotHeader, q.q.data(), sizeof(float) * d);
        R.ticket[slot] = q.ticket;
        R.t_submit[slot] = q.t_submit;
        R.collected[slot] = 0;
        R.tab_end[slot] = tend;
        R.tab_head = tend;
        R.published++;
        S->pending.pop_front();
        n++;
    }
    if (n) {
        S->inflight = R.published - R.finished;
        S->max_inflight_seen = std::max(S->max_inflight_seen, S->inflight);
        S->batched_requests += n;
        // the slots' contents before the count that publishes them
        __atomic_store_n(&R.h_ctl[0], (uint64_t)R.published, __ATOMIC_RELEASE);
    }
    return n;
}

// Collect answered slots; returns how many, or -1 when a slot held a wrong
// sequence word (a broken ring: the server stops).
int64_t ring_collect(jag_server *S)
{
    Ring &R = S->ring;
    const int k = S->P.k;
    std::vector<std::pair<uint64_t, Done>> got;
    int64_t bad = -1;
    {
        std::lock_guard<std::mutex> g(S->mu);
        const int64_t lo = R.freed, hi = R.published;
        auto now = clk::now();
        for (int64_t h = lo; h < hi; h++) {
            const int64_t slot = h & (R.C - 1);
            if (R.collected[slot]) continue;
            if (__atomic_load_n(&R.h_done[slot], __ATOMIC_ACQUIRE) != (uint64_t)h + 1) continue;
            if (R.h_cnt[slot] < 0) {
                bad = h;
                break;
            }
            Done r;
            r.ids.assign(R.h_ids + slot * k, R.h_ids + (slot + 1) * k);
            r.dists.assign(R.h_d + slot * k, R.h_d + (slot + 1) * k);
            r.count = R.h_cnt[slot];
            r.latency_us = std::chrono::duration<double, std::micro>(now - R.t_submit[slot]).count();
            got.emplace_back(R.ticket[slot], std::move(r));
            R.collected[slot] = 1;
        }
        if (bad >= 0) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "request %lld found a wrong sequence word in its ring slot",
                          (long long)bad);
            S->error = msg;
            S->stop = true;
            S->cv_done.notify_all();
            return -1;
        }
        while (R.freed < R.published && R.collected[R.freed & (R.C - 1)]) {
            R.tab_tail = std::max(R.tab_tail, R.tab_end[R.freed & (R.C - 1)]);
            R.freed++;
        }
        for (auto &x : got) {
            S->latencies.push_back(x.second.latency_us);
            S->done.emplace(x.first, std::move(x.second));
        }
        if (!got.empty()) {
            R.finished += (int64_t)got.size();
            S->completed += (int64_t)got.size();
            S->inflight = R.published - R.finished;
            S->t_last = now;
            S->cv_done.notify_all();
        }
    }
    return (int64_t)got.size();
}

void ring_fail(jag_server *S, const char *what, hipError_t e)
{
    std::lock_guard<std::mutex> g(S->mu);
    char msg[256];
    std::snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
    S->error = msg;
    S->stop = true;
    S->cv_done.notify_all();
}

void ring_loop(jag_server *S)
{
    (void)hipSetDevice(S->idx->ix.device);
    Ring &R = S->ring;
    auto last_answer = clk::now();
    for (;;) {
        bool progressed = false;
        int64_t published;
        {
            std::lock_guard<std::mutex> g(S->mu);
            const int64_t n = ring_publish(S);
            progressed |= n > 0;
            published = R.published;
            if (n > 0 && R.published - n == R.finished) last_answer = clk::now();  // the device was idle
        }
        const int64_t got = ring_collect(S);
        if (got < 0) break;
        progressed |= got > 0;
        if (got > 0) last_answer = clk::now();
        // a search takes milliseconds: requests on the device with no answer
        // for kServeStallS mean the waves cannot see them; stop with an error
        // instead of waiting forever
        if (published > R.finished && clk::now() - last_answer > std::chrono::seconds(kServeStallS)) {
            char what[96];
            std::snprintf(what, sizeof what, "resident waves answered nothing for %d s", kServeStallS);
            ring_fail(S, what, hipErrorLaunchTimeOut);
            break;
        }
        // the waves: find out whether they have ended, start them when needed
        if (R.running) {
            hipError_t e = hipEventQuery(R.event);
            if (e == hipSuccess && S->test_fail_batch > 0 && R.launches == S->test_fail_batch)
                e = hipErrorLaunchFailure;
            if (e == hipSuccess) {
                R.running = false;
                // every claimed request was answered before its wave ended
                if (ring_collect(S) < 0) break;
            } else if (e != hipErrorNotReady) {
                char what[96];
                std::snprintf(what, sizeof what, "resident waves (launch %lld) failed on the device",
                              (long long)R.launches);
                ring_fail(S, what, e);
                break;
            }
        }
        if (!R.running) {
            int64_t finished;
            {
                std::lock_guard<std::mutex> g(S->mu);
                finished = R.finished;
            }
            if (published > finished) {
                bool ok = jag::launch_serve(S->idx->ix, S->P.k, S->P.search, R.view, R.waves, R.stream) == JAG_OK;
                ok = ok && HIPOK(hipEventRecord(R.event, R.stream));
                if (!ok) {
                    std::lock_guard<std::mutex> g(S->mu);
                    S->error = jag_last_error();
                    if (S->error.empty()) S->error = "resident waves could not be launched";
                    S->stop = true;
                    S->cv_done.notify_all();
                    break;
                }
                R.running = true;
                R.launches++;
                std::lock_guard<std::mutex> g(S->mu);
                S->batches = R.launches;
                progressed = true;
            }
        }
        {
            std::unique_lock<std::mutex> lk(S->mu);
            const bool idle = S->pending.empty() && R.finished == R.published;
            if (S->stop && idle) break;
            if (!progressed) {
                if (idle)
                    S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                else {
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(10));
                }
            }
        }
    }
    // ask running waves to leave (they also leave by themselves once idle)
    __atomic_store_n(&R.h_ctl[1], (uint64_t)1, __ATOMIC_RELEASE);
}

}  // namespace

extern "C" {

jag_status jag_server_start(jag_index *idx, const jag_server_params *P, jag_server **out)
{
    using jag::set_error;
    if (!idx || !P || !out) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    *out = nullptr;
    const bool slots = P->slot_admission == 1;
    if (P->k < 1 || P->k > 64 || P->max_inflight < 0 || P->queue_capacity < 1 || P->search.stats ||
        P->search.features || P->search.learned == 2 || (P->slot_admission != 0 && !slots) || P->reserved ||
        (!slots && (P->max_batch < 1 || P->max_batch > 4096 || P->n_streams < 1 || P->n_streams > 8 ||
                    P->max_wait_us < 0))) {
        set_error("bad server parameters");
        return JAG_EINVAL;
    }
    jag::Index &ix = idx->ix;
    if (hipSetDevice(ix.device) != hipSuccess) {
        set_error("cannot select device %d", ix.device);
        return JAG_EDEVICE;
    }
    if (slots) {
        int64_t resident = 0;
        jag_status st = jag::serve_capacity(ix, P->k, P->search, &resident);
        if (st != JAG_OK) return st;
        if (resident < 1) {
            set_error("no serving wave fits on a compute unit with this search's LDS");
            return JAG_EUNSUPPORTED;
        }
        const int64_t waves = P->max_inflight > 0 ? std::min(P->max_inflight, resident) : resident;
        const int64_t dev_bytes = ring_device_bytes(waves, ix.d);
        if (P->hbm_budget_bytes > 0 && dev_bytes > P->hbm_budget_bytes) {
            set_error("server waves need %lld bytes, over the %lld-byte budget", (long long)dev_bytes,
                      (long long)P->hbm_budget_bytes);
            return JAG_EUNSUPPORTED;
        }
        auto *S = new (std::nothrow) jag_server;
        if (!S) return JAG_ENOMEM;
        S->idx = idx;
        S->P = *P;
        S->slot_mode = true;
        S->resident = resident;
        S->max_inflight = waves;
        S->device_bytes = dev_bytes;
        if (const char *fb = std::getenv("JAG_SERVER_TEST_FAIL_BATCH")) S->test_fail_batch = std::atoll(fb);
        st = alloc_ring(S, waves);
        if (st != JAG_OK) {
            delete S;
            return st;
        }
        S->worker = std::thread(ring_loop, S);
        *out = S;
        return JAG_OK;
    }
    int64_t resident = 0;
    size_t lds = 0;
    jag_status st = jag::search_capacity(ix, P->k, P->search, &resident, &lds);
    if (st != JAG_OK) return st;
    int64_t scratch = 0;  // two-pass learned search: saved states of one batch
    st = jag::search_scratch_bytes(ix, P->k, P->search, P->max_batch, &scratch);
    if (st != JAG_OK) return st;
    int64_t dev_bytes = (int64_t)P->n_streams * (slot_device_bytes(P->max_batch, ix.d, P->k) + scratch);
    if (P->hbm_budget_bytes > 0 && dev_bytes > P->hbm_budget_bytes) {
        set_error("server buffers need %lld bytes, over the %lld-byte budget", (long long)dev_bytes,
                  (long long)P->hbm_budget_bytes);
        return JAG_EUNSUPPORTED;
    }
    auto *S = new (std::nothrow) jag_server;
    if (!S) return JAG_ENOMEM;
    S->idx = idx;
    S->P = *P;
    S->resident = resident;
    S->max_inflight = P->max_inflight > 0 ? P->max_inflight : std::max<int64_t>(resident, P->max_batch);
    S->device_bytes = dev_bytes;
    if (const char *fb = std::getenv("JAG_SERVER_TEST_FAIL_BATCH")) S->test_fail_batch = std::atoll(fb);
    S->slots.resize(P->n_streams);
    for (auto &s : S->slots) {
        if (!alloc_slot(s, P->max_batch, ix.d, P->k)) {
            for (auto &x : S->slots) free_slot(x);
            delete S;
            set_error("server buffer allocation failed");
            return JAG_ENOMEM;
        }
    }
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return JAG_OK;
}

jag_status jag_server_submit(jag_server *S, const float *Q, const jag_filter *F, int64_t n,
                             const int32_t *pool, int64_t pool_len, uint64_t *tickets_out)
{
    using jag::set_error;
    if (!S || n < 0 || (n > 0 && (!Q || !F || !tickets_out))) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    if (n == 0) return JAG_OK;
    const int d = S->idx->ix.d;
    // records followed by the distance tables of any TABLE filters
    int64_t bytes = 0;
    jag_status st = jag::encoded_bytes(S->idx->ix, F, n, pool, pool_len, &bytes);
    if (st != JAG_OK) return st;
    std::vector<uint8_t> enc((size_t)bytes);
    st = jag::encode_filters_sized(S->idx->ix, F, n, pool, pool_len, enc.data(), bytes);
    if (st != JAG_OK) return st;
    const jag::FilterRecord *rec = reinterpret_cast<const jag::FilterRecord *>(enc.data());
    for (int64_t i = 0; i < n * d; i++)
        if (!std::isfinite(Q[i])) {
            set_error("query element %lld is not finite", (long long)i);
            return JAG_EINVAL;
        }
    auto now = clk::now();
    std::lock_guard<std::mutex> g(S->mu);
    if (!S->error.empty()) {
        set_error("server stopped after an error: %s", S->error.c_str());
        return JAG_EDEVICE;
    }
    if ((int64_t)S->pending.size() + n > S->P.queue_capacity) {
        set_error("queue full (%lld pending)", (long long)S->pending.size());
        return JAG_EBUSY;
    }
    if (!S->have_first) {
        S->t_first = now;
        S->have_first = true;
    }
    for (int64_t i = 0; i < n; i++) {
        Request r;
        r.ticket = S->next_ticket++;
        r.rec = rec[i];
        if (rec[i].type == jag::F_TABLE) {
            const uint8_t *t = enc.data() + i * (int64_t)sizeof(jag::FilterRecord) + rec[i].table_off;
            r.table.assign(t, t + ((size_t)1 << rec[i].nlit));
            r.rec.table_off = 0;  // set at launch
        }
        r.q.assign(Q + i * d, Q + (i + 1) * d);
        r.t_submit = now;
        tickets_out[i] = r.ticket;
        S->pending.push_back(std::move(r));
    }
    S->submitted += n;
    S->cv_work.notify_one();
    return JAG_OK;
}

jag_status jag_server_poll(jag_server *S, uint64_t ticket, int32_t *ids, float *dists, int32_t *count,
                           double *latency_us)
{
    using jag::set_error;
    if (!S || !ids || !dists || !count) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) {
        if (ticket == 0 || ticket >= S->next_ticket) {
            set_error("unknown ticket %llu", (unsigned long long)ticket);
            return JAG_EINVAL;
        }
        if (!S->error.empty()) {
            set_error("server stopped after an error: %s", S->error.c_str());
            return JAG_EDEVICE;
        }
        return JAG_EAGAIN;
    }
    std::copy(it->second.ids.begin(), it->second.ids.end(), ids);
    std::copy(it->second.dists.begin(), it->second.dists.end(), dists);
    *count = it->second.count;
    if (latency_us) *latency_us = it->second.latency_us;
    S->done.erase(it);
    return JAG_OK;
}

jag_status jag_server_drain(jag_server *S)
{
    if (!S) {
        jag::set_error("null argument");
        return JAG_EINVAL;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->completed == S->submitted || !S->error.empty(); });
    if (!S->error.empty()) {
        jag::set_error("server stopped after an error: %s", S->error.c_str());
        return JAG_EDEVICE;
    }
    return JAG_OK;
}

jag_status jag_server_stats_get(jag_server *S, jag_server_stats *o)
{
    if (!S || !o) {
        jag::set_error("null argument");
        return JAG_EINVAL;
    }
    std::lock_guard<std::mutex> g(S->mu);
    std::memset(o, 0, sizeof(*o));
    o->submitted = S->submitted;
    o->completed = S->completed;
    o->batches = S->batches;
    o->max_inflight_seen = S->max_inflight_seen;
    o->resident_capacity = S->resident;
    o->device_bytes = S->device_bytes;
    o->mean_batch = S->batches ? (double)S->batched_requests / (double)S->batches : 0.0;
    if (!S->latencies.empty()) {
        std::vector<double> v = S->latencies;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            size_t i = (size_t)std::ceil(p * (double)v.size()) - 1;
            return v[std::min(i, v.size() - 1)];
        };
        o->p50_us = pct(0.50);
        o->p99_us = pct(0.99);
        o->max_us = v.back();
        double s = 0;
        for (double x : v) s += x;
        o->mean_us = s / (double)v.size();
        double span = std::chrono::duration<double>(S->t_last - S->t_first).count();
        o->qps = span > 0 ? (double)S->completed / span : 0.0;
    }
    return JAG_OK;
}

void jag_server_stop(jag_server *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    if (S->slot_mode) free_ring(S->ring);
    for (auto &s : S->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        free_slot(s);
    }
    delete S;
}

}  // extern "C"

// Batched filtered greedy search on gfx950: the batch launches of the search
// kernel (search_device.h) with their launch order and two-pass learned
// schedule, exact k-NN (Pre-Filtering), the vector store quantizers, index
// upload, and the C entry points of the search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "jag_internal.h"
#include "search_device.h"

namespace jag {

namespace {

// ---------------------------------------------------------------- exact k-NN
// Pre-Filtering: every item is tested against the filter; valid items are
// scored from the FP32 rows and merged into a k-entry list.
template <int G, int CH>
__global__ __launch_bounds__(64) void exact_kernel(SearchArgs a, int64_t n)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x;
    Lds s = carve(smem, a.Lcap, 1);
    const FilterRecord f = a.rec[q];
    // TABLE filters: the distance table sits table_off bytes after the record
    const uint8_t *tab = f.type == F_TABLE ? reinterpret_cast<const uint8_t *>(a.rec + q) + f.table_off : nullptr;
    QueryRegs<JAG_STORE_F32, G, CH> qr;
    qr.load(a.Q + q * a.d, a.d, lane & (G - 1));
    int cnt = 0;
    for (int64_t i0 = 0; i0 < n; i0 += 64) {
        int64_t i = i0 + lane;
        bool ok = i < n;
        uint32_t df = 1u;
        if (ok) {
            ItemAttr at;
            load_item_attr<AK_ANY>(at, f, (int32_t)i, a);
            df = dist_f<AK_ANY>(f, tab, at, a);
        }
        ok = ok && df == 0;
        uint64_t bm = ballot64(ok);
        int m = __popcll(bm);
        if (m == 0) continue;
        if (ok) {
            int slot = lanes_below(bm);
            s.cid[slot] = (int32_t)i;
            s.cdf[slot] = 0u;
        }
        __syncthreads();
        eval_rows<JAG_STORE_F32, G, CH>(a.f32, a.f32_stride, s.cid, s.cd2, m, qr);
        __syncthreads();
        int mp;
        cnt = merge_candidates(s, m, cnt, a.k, &mp);
    }
    bool ok = lane < cnt && lane < a.k;
    if (lane < a.k) {
        a.ids[q * a.k + lane] = ok ? (int32_t)(s.idf[lane] & kIdMask) : -1;
        a.dists[q * a.k + lane] = ok ? __uint_as_float((uint32_t)s.key[lane]) : __builtin_inff();
    }
    if (lane == 0) a.count[q] = cnt < a.k ? cnt : a.k;
}

// ---------------------------------------------------------------- quantizers
// FP32 -> BF16, round to nearest even (NaN stays NaN, quieted).
__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP32 -> OCP E4M3, round to nearest even, saturating at +-448.
__device__ __forceinline__ uint8_t to_e4m3(float y)
{
    uint32_t u = __float_as_uint(y);
    uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    uint32_t a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return 0x7F;
    if (a >= 0x43E00000u) return (uint8_t)(sign | 0x7E);  // |y| >= 448
    if (a < 0x3C800000u) {                                // |y| < 2^-6: subnormal step 2^-9
        float m = __builtin_rintf(__uint_as_float(a) * 512.0f);
        return (uint8_t)(sign | (uint8_t)m);               // m == 8 is the smallest normal
    }
    // keep 3 mantissa bits, round to nearest even on the 20 dropped bits
    uint32_t r = a + 0x7FFFFu + ((a >> 20) & 1u);
    uint32_t code = (r >> 20) - (120u << 3);
    return (uint8_t)(sign | (uint8_t)code);
}

__global__ void quant_bf16_kernel(const float *X, int64_t n, int d, unsigned char *out, int stride)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tot = n * (int64_t)(stride / 2);
    if (i >= tot) return;
    int64_t r = i / (stride / 2);
    int c = (int)(i % (stride / 2));
    uint16_t v = c < d ? to_bf16(X[r * d + c]) : (uint16_t)0;
    reinterpret_cast<uint16_t *>(out + r * stride)[c] = v;
}

// One 64-lane wave per row: max |x| by a butterfly, scale = max/448 (FP32
// division), code_i = E4M3(x_i / scale); an all-zero row gets scale 1.
__global__ __launch_bounds__(64) void quant_fp8_kernel(const float *X, int64_t n, int d,
                                                       unsigned char *out, int stride)
{
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    float mx = 0.f;
    for (int c = lane; c < d; c += 64) mx = fmaxf(mx, fabsf(X[r * d + c]));
    for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m, 64));
    float s = mx > 0.f ? mx / 448.0f : 1.0f;
    unsigned char *row = out + r * stride;
    for (int c = lane; c < stride - 4; c += 64) row[c] = c < d ? to_e4m3(X[r * d + c] / s) : (uint8_t)0;
    if (lane == 0) *reinterpret_cast<float *>(row + stride - 4) = s;
}

__global__ void copy_rows_kernel(const float *X, int64_t n, int d, unsigned char *out, int stride)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tot = n * (int64_t)(stride / 4);
    if (i >= tot) return;
    int64_t r = i / (stride / 4);
    int c = (int)(i % (stride / 4));
    reinterpret_cast<float *>(out + r * stride)[c] = c < d ? X[r * d + c] : 0.f;
}

__global__ void to_bf16_kernel(const float *x, int n, uint16_t *out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = to_bf16(x[i]);
}

// ---------------------------------------------------------------- schedule
// Longest-first orders for a launch, by a counting sort over 17 classes,
// largest class first.  Two-pass learned search: class = 1 + predicted
// ladder index (0 = finished before the prediction point).  One launch of
// many queries at a fixed beam, or one-pass learned: class = the filter's
// log2 selectivity estimate in steps of about two octaves, ranked so that
// the searches expected to be long run first and the launch does not end on
// them.  For range filters the broad ones search longer (the log estimate
// correlates +0.26 to +0.55 with a query's expansions), for label-based
// filters (label, subset, Boolean, truth table) the narrow ones (-0.24 for
// labels, -0.18 for Boolean filters, about 0 for subsets), so range filters
// rank broadest first and the others narrowest first.  class_kernel, one
// thread per query, first copies these classes out of the 128-byte
// records, so that the sort reads 4 bytes per query (one compute unit
// reading every record line itself takes 35 us at 10,000 queries).
// The sort is one workgroup; thread t owns queries t, t + 512, t + 1024,
// ... (coalesced reads), taken 20 at a time so that 20 independent loads
// are in flight per thread; within a class the order is (thread, then
// position), not the query order, which no result depends on.
constexpr int kOrderThreads = 512;
constexpr int kOrderBatch = 20;
constexpr int kOrderBins = JAG_LADDER_MAX + 1;
// Fixed-beam and one-pass learned launches of at least this many queries
// are ordered by selectivity (smaller ones fit on the device at once, where
// the order hardly matters).
constexpr int64_t kSelOrderMin = 4096;

static bool sel_ordered(const jag_search_params &S, int64_t nq)
{
    return (S.learned == 0 || (S.learned == 1 && S.single_pass)) && nq >= kSelOrderMin;
}

// Range filters in one-pass learned launches: once the index's own such
// launches have run enough searches of a class (kMinClassRuns), the class
// ranks by its mean expansions instead: key = 16 * mean / (largest mean
// over the range classes with data), so that the classes that searched
// longest run first whatever shape the relation to selectivity takes (on
// the range workload it is not monotonic: the broadest and the middle
// classes search longest).  Range classes without data take the mean over
// those with data; with no data at all the fixed rank above applies.
// Label-based filters keep the fixed rank (narrowest first measured 10 %
// faster than the learned rank for one-pass subset searches).
// order_kernel halves the sums and counts before each such launch adds its
// own, so the ranking follows the recent launches (a sweep over offsets
// does not freeze it).
constexpr unsigned long long kMinClassRuns = 64;

__global__ __launch_bounds__(256) void class_kernel(const FilterRecord *rec, int64_t nq, int32_t *key,
                                                    const unsigned long long *stats)
{
    __shared__ float mean[2 * kSelClasses];
    __shared__ float top, avg;
    const int t = threadIdx.x;
    if (stats) {
        if (t < 2 * kSelClasses) {
            const unsigned long long n = stats[2 * t + 1];
            mean[t] = n >= kMinClassRuns ? (float)stats[2 * t] / (float)n : -1.f;
        }
        __syncthreads();
        if (t == 0) {
            float hi = 0.f, sum = 0.f;
            int with = 0;
            for (int c = 0; c < kSelClasses; c++)  // the range classes
                if (mean[c] >= 0.f) {
                    hi = mean[c] > hi ? mean[c] : hi;
                    sum += mean[c];
                    with++;
                }
            top = hi;
            avg = with ? sum / (float)with : 0.f;
        }
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * 256 + t;
    if (i >= nq) return;
    const int kind = sel_kind(rec[i].type), broad = sel_class(rec[i].sel_feature);  // 16: selectivity 1
    int k = kind == 0 ? broad : 16 - broad;
    if (stats && kind == 0 && top > 0.f) {
        const float m = mean[broad];
        const int b = (int)(16.f * (m >= 0.f ? m : avg) / top);
        k = b < 0 ? 0 : (b > 16 ? 16 : b);
    }
    key[i] = k;
}

__device__ __forceinline__ int order_class(const int32_t *key, int64_t i)
{
    const int k = key[i];
    return k < 0 ? 0 : (k >= kOrderBins ? kOrderBins - 1 : k);
}

// Both loops clamp the index instead of branching on it, so that the
// batch's loads issue back to back.  The counters are bumped with LDS
// atomics (each thread owns its column, so nothing contends): one wave's
// atomics run in program order, so the increments of a batch issue back to
// back instead of as a chain of dependent reads and writes, and the ranks
// come out as with plain increments.  A launch of at most kOrderThreads *
// kOrderBatch queries (10,240) reads its classes once and keeps them in
// registers for the second pass.
__global__ __launch_bounds__(kOrderThreads) void order_kernel(const int32_t *key, int64_t nq, int32_t *perm,
                                                              unsigned long long *stats)
{
    __shared__ int32_t cnt[kOrderBins][kOrderThreads];
    __shared__ int32_t part[kOrderThreads];
    const int t = threadIdx.x;
    if (stats && t < 4 * kSelClasses) stats[t] >>= 1;  // older launches weigh half
    for (int b = 0; b < kOrderBins; b++) cnt[b][t] = 0;
    const bool once = nq <= (int64_t)kOrderThreads * kOrderBatch;
    int c[kOrderBatch];
    for (int64_t i0 = t; i0 < nq; i0 += (int64_t)kOrderThreads * kOrderBatch) {
#pragma unroll
        for (int j = 0; j < kOrderBatch; j++) {
            const int64_t i = i0 + (int64_t)j * kOrderThreads;
            c[j] = order_class(key, i < nq ? i : nq - 1);
        }
#pragma unroll
        for (int j = 0; j < kOrderBatch; j++)
            if (i0 + (int64_t)j * kOrderThreads < nq) atomicAdd(&cnt[c[j]][t], 1);
    }
    __syncthreads();
    // output rank r enumerates (bin descending, thread ascending); thread t
    // scans ranks [t*kOrderBins, (t+1)*kOrderBins)
    int sum = 0;
    for (int j = 0; j < kOrderBins; j++) {
        int r = t * kOrderBins + j;
        sum += cnt[kOrderBins - 1 - r / kOrderThreads][r % kOrderThreads];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < kOrderThreads; off <<= 1) {  // inclusive scan of the partial sums
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    __syncthreads();
    for (int j = 0; j < kOrderBins; j++) {
        int r = t * kOrderBins + j;
        int *c = &cnt[kOrderBins - 1 - r / kOrderThreads][r % kOrderThreads];
        int v = *c;
        *c = run;  // exclusive offset of (bin, thread)
        run += v;
    }
    __syncthreads();
    for (int64_t i0 = t; i0 < nq; i0 += (int64_t)kOrderThreads * kOrderBatch) {
        if (!once) {
#pragma unroll
            for (int j = 0; j < kOrderBatch; j++) {
                const int64_t i = i0 + (int64_t)j * kOrderThreads;
                c[j] = order_class(key, i < nq ? i : nq - 1);
            }
        }
#pragma unroll
        for (int j = 0; j < kOrderBatch; j++) {
            const int64_t i = i0 + (int64_t)j * kOrderThreads;
            if (i < nq) perm[atomicAdd(&cnt[c[j]][t], 1)] = (int32_t)i;
        }
    }
}

// The device's default memory pool keeps freed memory reserved, so that the
// stream-ordered scratch of repeated searches is not returned to the system
// and allocated again.
static void keep_pool_reserved(int device)
{
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
}

// ---------------------------------------------------------------- host glue
#define HIPCHK(expr)                                                               \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));             \
            return e_ == hipErrorOutOfMemory ? JAG_ENOMEM : JAG_EDEVICE;           \
        }                                                                          \
    } while (0)

template <class T>
jag_status dalloc(T **p, size_t bytes, int64_t &acct)
{
    HIPCHK(hipMalloc((void **)p, bytes));
    acct += (int64_t)bytes;
    return JAG_OK;
}



using SearchFn = void (*)(SearchArgs);
using ExactFn = void (*)(SearchArgs, int64_t);

struct SearchFamily {
    using Fn = SearchFn;
    template <int STORE, int G, int CH, int WPE, int SL, int AK>
    static Fn get()
    {
        return search_kernel<STORE, G, CH, WPE, SL, AK>;
    }
};

// Rows of more than 64 neighbours take the two-slice build (the one-slice
// build has no slice loop, which keeps its register allocation); rows of up
// to 64 take the build for the index's attribute kind.
SearchFn pick_search(int store, int stride, int R, int ak)
{
    int G = pick_group(stride);
    int ch = stride / (16 * G);
    using F = SearchFamily;
    if (R > 64) return family_pick_sl<F, kWavesPerSimd, 2, AK_ANY>(store, G, ch);
    if (ak == AK_SCALAR) return family_pick_sl<F, kWavesPerSimd, 1, AK_SCALAR>(store, G, ch);
    if (ak == AK_LABELS) return family_pick_sl<F, kWavesPerSimd, 1, AK_LABELS>(store, G, ch);
    return family_pick_sl<F, kWavesPerSimd, 1, AK_ANY>(store, G, ch);
}

template <int G>
ExactFn exact_for_ch(int ch)
{
    if (G == 4 && ch >= 1 && ch <= 6) {
        switch (ch) {
        case 1: return exact_kernel<G, 1>;
        case 2: return exact_kernel<G, 2>;
        case 3: return exact_kernel<G, 3>;
        case 4: return exact_kernel<G, 4>;
        case 5: return exact_kernel<G, 5>;
        case 6: return exact_kernel<G, 6>;
        }
    }
    if (G == 8 && ch == 4) return exact_kernel<G, 4>;
    if (G == 16) {
        switch (ch) {
        case 3: return exact_kernel<G, 3>;
        case 4: return exact_kernel<G, 4>;
        case 5: return exact_kernel<G, 5>;
        case 6: return exact_kernel<G, 6>;
        case 7: return exact_kernel<G, 7>;
        case 8: return exact_kernel<G, 8>;
        }
    }
    return nullptr;
}

// Seen-table slots.  The kernel holds at most 5 waves per SIMD (20 per CU)
// by registers; 2^10 slots keep LDS from lowering that for lists up to 128
// entries.  Longer lists take 2^9 slots: the LDS a wave needs (12 bytes per
// list entry, 4 per slot, 2.4 KB of staging) then lets more of them share a
// compute unit, which pays more than the extra evaluations of vertices the
// smaller table forgets.  Measured on the label-set workload (1M x 128,
// BF16 + rerank; results do not depend on the table): Boolean filters at
// L = 192 2.06 M -> 2.58 M queries/s, their learned beam (one pass) 2.45 M
// -> 2.69 M; subset filters' learned beam (two passes, lists of 512)
// 0.985 M -> 1.046 M; 2^8 slots were slower than 2^9, 2^11 slower than
// 2^10.  On the range workload (lists of 64) the occupancy is bound by
// registers either way and the larger table forgets less.
constexpr int kDefaultHash = 1024;
constexpr int kLongListHash = 512;
constexpr int kLongList = 128;
// Smallest list width of the first four expansions in learned and trace
// modes (the widest ladder beam, or L in trace mode, if larger).
constexpr int kWarmWidth = 64;
// Device memory a two-pass learned search may hold for saved states; larger
// batches are processed in chunks of queries that fit.
constexpr int64_t kStateBudget = int64_t(512) << 20;

// Words of one saved search state: 8 counters and the list (8-byte keys and
// 4-byte ids of up to Lcap entries).
constexpr int64_t state_words(int Lcap) { return 8 + 3 * (int64_t)Lcap; }

}  // namespace

jag_status upload_index(Index &ix)
{
    HIPCHK(hipGetDevice(&ix.device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, ix.device));
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0) {
        set_error("device %d is %s; this library is built for gfx950 only", ix.device, prop.gcnArchName);
        return JAG_EDEVICE;
    }
    const int64_t n = ix.n;
    const int d = ix.d;
    jag_status st;
    if (!ix.staging) ix.staging = new_staging();
    // adjacency rows with the neighbours' attributes inlined:
    //   [R ids][R scalars, if any][R x W/2 label words, if any], each part
    //   starting on a 16-byte boundary; -1 / 0 / 0xFFFF padding
    auto up4 = [](int x) { return (x + 3) / 4 * 4; };
    ix.scal_word_off = ix.has_scalar ? up4(ix.R) : 0;
    ix.lab_word_off = ix.has_labels ? up4(ix.has_scalar ? ix.scal_word_off + ix.R : ix.R) : 0;
    ix.adj_words = up4(ix.has_labels ? ix.lab_word_off + ix.R * (ix.W / 2)
                                     : (ix.has_scalar ? ix.scal_word_off + ix.R : ix.R));
    if ((st = dalloc(&ix.d_adj, sizeof(int32_t) * n * ix.adj_words, ix.device_bytes)) != JAG_OK) return st;
    {
        const int64_t chunk = 1 << 16;
        std::vector<int32_t> buf((size_t)std::min<int64_t>(chunk, n) * ix.adj_words);
        for (int64_t r0 = 0; r0 < n; r0 += chunk) {
            int64_t r1 = std::min<int64_t>(n, r0 + chunk);
            std::fill(buf.begin(), buf.end(), 0);
            for (int64_t i = r0; i < r1; i++) {
                int32_t *o = buf.data() + (size_t)(i - r0) * ix.adj_words;
                const int32_t *nb = ix.adj.data() + (size_t)i * ix.R;
                uint16_t *lw = reinterpret_cast<uint16_t *>(o + ix.lab_word_off);
                for (int j = 0; j < ix.R; j++) {
                    int32_t v = nb[j];
                    o[j] = v;
                    if (ix.has_scalar) o[ix.scal_word_off + j] = v >= 0 ? ix.scalar[v] : 0;
                    if (ix.has_labels) {
                        uint16_t *dst = lw + (size_t)j * ix.W;
                        for (int t = 0; t < ix.W; t++) dst[t] = 0xFFFF;
                        if (v >= 0)
                            for (int64_t x = ix.loff[v]; x < ix.loff[v + 1]; x++)
                                dst[x - ix.loff[v]] = (uint16_t)ix.lab[x];
                    }
                }
            }
            HIPCHK(hipMemcpy(ix.d_adj + r0 * ix.adj_words, buf.data(),
                             sizeof(int32_t) * (r1 - r0) * ix.adj_words, hipMemcpyHostToDevice));
        }
    }
    if (ix.has_scalar) {
        if ((st = dalloc(&ix.d_scalar, sizeof(int32_t) * n, ix.device_bytes)) != JAG_OK) return st;
        HIPCHK(hipMemcpy(ix.d_scalar, ix.scalar.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    }
    if (ix.has_labels) {
        std::vector<uint16_t> rows((size_t)n * ix.W, 0xFFFF);
        for (int64_t i = 0; i < n; i++)
            for (int64_t j = ix.loff[i]; j < ix.loff[i + 1]; j++)
                rows[(size_t)i * ix.W + (j - ix.loff[i])] = (uint16_t)ix.lab[j];
        if ((st = dalloc(&ix.d_lab, sizeof(uint16_t) * rows.size(), ix.device_bytes)) != JAG_OK) return st;
        HIPCHK(hipMemcpy(ix.d_lab, rows.data(), sizeof(uint16_t) * rows.size(), hipMemcpyHostToDevice));
    }
    // stage FP32 vectors, then lay out the store(s)
    float *dX = nullptr;
    HIPCHK(hipMalloc((void **)&dX, sizeof(float) * n * d));
    hipError_t e = hipMemcpy(dX, ix.X.data(), sizeof(float) * n * d, hipMemcpyHostToDevice);
    auto cleanup = [&]() { (void)hipFree(dX); };
    if (e != hipSuccess) {
        cleanup();
        set_error("copy of vectors failed: %s", hipGetErrorString(e));
        return JAG_EDEVICE;
    }
    ix.vec_stride = store_row_bytes(ix.store, d);
    ix.vec_stride = padded_stride(ix.vec_stride);
    if ((st = dalloc(&ix.d_vec, (size_t)n * ix.vec_stride, ix.device_bytes)) != JAG_OK) {
        cleanup();
        return st;
    }
    const int TB = 256;
    if (ix.store == JAG_STORE_F32) {
        int64_t tot = n * (ix.vec_stride / 4);
        copy_rows_kernel<<<(unsigned)((tot + TB - 1) / TB), TB>>>(dX, n, d, ix.d_vec, ix.vec_stride);
        ix.d_f32 = ix.d_vec;
        ix.f32_stride = ix.vec_stride;
    } else {
        if (ix.store == JAG_STORE_BF16) {
            int64_t tot = n * (ix.vec_stride / 2);
            quant_bf16_kernel<<<(unsigned)((tot + TB - 1) / TB), TB>>>(dX, n, d, ix.d_vec, ix.vec_stride);
        } else {
            quant_fp8_kernel<<<(unsigned)n, 64>>>(dX, n, d, ix.d_vec, ix.vec_stride);
        }
        if (ix.keep_f32) {
            ix.f32_stride = padded_stride((4 * d + 63) / 64 * 64);
            if ((st = dalloc(&ix.d_f32, (size_t)n * ix.f32_stride, ix.device_bytes)) != JAG_OK) {
                cleanup();
                return st;
            }
            ix.f32_owned = true;
            int64_t tot = n * (ix.f32_stride / 4);
            copy_rows_kernel<<<(unsigned)((tot + TB - 1) / TB), TB>>>(dX, n, d, ix.d_f32, ix.f32_stride);
        }
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    cleanup();
    if (e != hipSuccess) {
        set_error("store layout kernels failed: %s", hipGetErrorString(e));
        return JAG_EDEVICE;
    }
    if (!ix.d_order_stats) {
        const size_t sb = sizeof(unsigned long long) * 4 * kSelClasses;
        if ((st = dalloc(&ix.d_order_stats, sb, ix.device_bytes)) != JAG_OK) return st;
        HIPCHK(hipMemset(ix.d_order_stats, 0, sb));
    }
    return JAG_OK;
}

void free_device(Index &ix)
{
    free_staging(ix.staging);
    ix.staging = nullptr;
    auto f = [](void *p) {
        if (p) (void)hipFree(p);
    };
    f(ix.d_adj);
    f(ix.d_scalar);
    f(ix.d_lab);
    if (ix.f32_owned) f(ix.d_f32);
    f(ix.d_vec);
    f(ix.pred.d_bf16);
    f(ix.d_order_stats);
    ix.d_order_stats = nullptr;
    ix.d_adj = nullptr;
    ix.d_scalar = nullptr;
    ix.d_lab = nullptr;
    ix.d_f32 = nullptr;
    ix.d_vec = nullptr;
    ix.pred.d_bf16 = nullptr;
}

jag_status download_store(const Index &ix, void *rows_out, float *scales_out)
{
    const int64_t n = ix.n;
    const int d = ix.d;
    std::vector<unsigned char> buf((size_t)n * ix.vec_stride);
    HIPCHK(hipMemcpy(buf.data(), ix.d_vec, buf.size(), hipMemcpyDeviceToHost));
    int eb = ix.store == JAG_STORE_F32 ? 4 : ix.store == JAG_STORE_BF16 ? 2 : 1;
    unsigned char *o = static_cast<unsigned char *>(rows_out);
    for (int64_t i = 0; i < n; i++) {
        memcpy(o + (size_t)i * d * eb, buf.data() + (size_t)i * ix.vec_stride, (size_t)d * eb);
        if (ix.store == JAG_STORE_FP8_E4M3 && scales_out)
            memcpy(scales_out + i, buf.data() + (size_t)i * ix.vec_stride + ix.vec_stride - 4, 4);
    }
    return JAG_OK;
}

jag_status upload_predictor(Index &ix)
{
    if (!ix.pred.d_bf16) {
        jag_status st = dalloc(&ix.pred.d_bf16, sizeof(uint16_t) * 5376, ix.device_bytes);
        if (st != JAG_OK) return st;
    }
    float *tmp = nullptr;
    HIPCHK(hipMalloc((void **)&tmp, sizeof(float) * kPredParams));
    hipError_t e = hipMemcpy(tmp, ix.pred.params.data(), sizeof(float) * kPredParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        to_bf16_kernel<<<(kPredParams + 255) / 256, 256>>>(tmp, kPredParams, ix.pred.d_bf16);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    (void)hipFree(tmp);
    if (e != hipSuccess) {
        set_error("predictor upload failed: %s", hipGetErrorString(e));
        return JAG_EDEVICE;
    }
    return JAG_OK;
}

static jag_status fill_args(Index &ix, SearchArgs &a, const float *Q, const void *records, int32_t k,
                            int32_t *ids, float *dists, int32_t *count)
{
    a.adj = ix.d_adj;
    a.vec = ix.d_vec;
    a.f32 = ix.d_f32;
    a.scalar = ix.d_scalar;
    a.lab = ix.d_lab;
    a.Q = Q;
    a.rec = static_cast<const FilterRecord *>(records);
    a.ids = ids;
    a.dists = dists;
    a.count = count;
    a.stats = nullptr;
    a.features = nullptr;
    a.pred = ix.pred.d_bf16;
    a.vec_stride = ix.vec_stride;
    a.f32_stride = ix.f32_stride;
    a.W = ix.W;
    a.d = ix.d;
    a.R = ix.R;
    a.adj_words = ix.adj_words;
    a.scal_word_off = ix.scal_word_off;
    a.lab_word_off = ix.lab_word_off;
    a.entry = ix.entry;
    a.k = k;
    a.perm = nullptr;
    a.state = nullptr;
    a.state_stride = 0;
    a.order_key = nullptr;
    a.order_stats = nullptr;
    return JAG_OK;
}

// Validate a search request and choose its kernel, LDS size and arguments.
jag_status plan_search(Index &ix, const float *Q, int64_t nq, const void *records, int32_t k,
                       const jag_search_params &S, int32_t *ids, float *dists, int32_t *count,
                       SearchArgs &a, size_t &lds, int &ak)
{
    if (k < 1 || k > 64 || S.L < k || S.L > 1024 || S.learned < 0 || S.learned > 2 ||
        S.rerank_mult < 0 || S.rerank_mult * k > 64 || S.max_hops < 0 || nq > INT_MAX ||
        (S.hash_log2 != 0 && (S.hash_log2 < 8 || S.hash_log2 > 13))) {
        set_error("need 1 <= k <= 64, k <= L <= 1024, learned in {0,1,2}, rerank_mult*k <= 64, "
                  "hash_log2 in {0, 8..13}");
        return JAG_EINVAL;
    }
    if (S.rerank_mult > 0 && !ix.d_f32) {
        set_error("reranking needs an FP32 copy (build with keep_f32 or an FP32 store)");
        return JAG_EUNSUPPORTED;
    }
    if (S.learned == 1 && !ix.pred.present) {
        set_error("learned search needs a predictor (jag_set_predictor)");
        return JAG_EUNSUPPORTED;
    }
    if (S.learned == 2 && !S.features) {
        set_error("learned == 2 needs a features buffer");
        return JAG_EINVAL;
    }
    int dev;
    HIPCHK(hipGetDevice(&dev));
    if (dev != ix.device) {
        set_error("index lives on device %d, current device is %d", ix.device, dev);
        return JAG_EINVAL;
    }
    fill_args(ix, a, Q, records, k, ids, dists, count);
    a.stats = S.stats;
    a.features = S.features;
    a.L = S.L;
    a.mode = S.learned;
    a.delta = S.delta;
    a.rerank = S.rerank_mult;
    a.max_hops = S.max_hops;
    a.nladder = ix.pred.nladder;
    a.rho = ix.pred.rho;
    for (int i = 0; i < JAG_LADDER_MAX; i++) a.ladder[i] = ix.pred.ladder[i];
    int Lcap = S.L;
    if (S.learned == 1) {
        Lcap = ix.pred.ladder[ix.pred.nladder - 1];
        if (Lcap < k) {
            set_error("predictor ladder tops out below k");
            return JAG_EINVAL;
        }
        for (int i = 0; i < ix.pred.nladder; i++)
            if (a.ladder[i] < k) a.ladder[i] = k;
    }
    // learned and trace modes run the first four expansions with a list of
    // max(kWarmWidth, widest beam) entries: both modes see the same list when
    // the features are taken, and cutting it to any beam <= that width then
    // gives exactly the fixed-beam search's state
    if (S.learned != 0 && Lcap < kWarmWidth) Lcap = kWarmWidth;
    a.warm = Lcap;
    Lcap = (Lcap + 63) / 64 * 64;
    int H = S.hash_log2 ? (1 << S.hash_log2) : Lcap > kLongList ? kLongListHash : kDefaultHash;
    a.Lcap = Lcap;
    a.Hmask = H - 1;
    ak = ix.has_scalar && !ix.has_labels ? AK_SCALAR : !ix.has_scalar && ix.has_labels ? AK_LABELS : AK_ANY;
    lds = lds_bytes(Lcap, H);
    return JAG_OK;
}

// plan_search and the batch kernel for the index's layout.
static jag_status plan_batch(Index &ix, const float *Q, int64_t nq, const void *records, int32_t k,
                             const jag_search_params &S, int32_t *ids, float *dists, int32_t *count,
                             SearchArgs &a, SearchFn &fn, size_t &lds)
{
    int ak = AK_ANY;
    jag_status st = plan_search(ix, Q, nq, records, k, S, ids, dists, count, a, lds, ak);
    if (st != JAG_OK) return st;
    fn = pick_search(ix.store, ix.vec_stride, ix.R, ak);
    if (!fn) {
        set_error("no kernel for row stride %d", ix.vec_stride);
        return JAG_EUNSUPPORTED;
    }
    return JAG_OK;
}

// fixed_scratch (device, fixed_bytes long), when given, replaces the
// stream-ordered allocations: the launch order of a large batch and the
// saved states of a two-pass learned search (processed in chunks that fit).
jag_status launch_search(Index &ix, const float *Q, int64_t nq, const void *records, int32_t k,
                         const jag_search_params &S, int32_t *ids, float *dists, int32_t *count,
                         void *stream, void *fixed_scratch, int64_t fixed_bytes)
{
    SearchArgs a;
    SearchFn fn = nullptr;
    size_t lds = 0;
    jag_status st = plan_batch(ix, Q, nq, records, k, S, ids, dists, count, a, fn, lds);
    if (st != JAG_OK) return st;
    if (nq == 0) return JAG_OK;
    hipStream_t sm = (hipStream_t)stream;
    const bool fixed = fixed_scratch != nullptr;
    int32_t *order = nullptr;
    if (sel_ordered(S, nq)) {
        const int64_t need = 2 * (int64_t)sizeof(int32_t) * nq;
        if (fixed) {
            if (need > fixed_bytes) {
                set_error("a batch of %lld queries needs %lld bytes of scratch for its launch order; "
                          "the fixed scratch holds %lld", (long long)nq, (long long)need,
                          (long long)fixed_bytes);
                return JAG_EINVAL;
            }
            order = static_cast<int32_t *>(fixed_scratch);
        } else {
            keep_pool_reserved(ix.device);
            if (hipMallocAsync((void **)&order, (size_t)need, sm) != hipSuccess) {
                (void)hipGetLastError();  // no memory for the order: submission order below
                order = nullptr;
            }
        }
    }
    if (order) {
        // one launch, the searches expected to be long first; one-pass
        // learned launches rank range filters' classes by what the index's
        // earlier one-pass launches measured (fixed-beam launches keep the
        // fixed rank, which measured 10 % faster for them than this one on
        // the range workload)
        unsigned long long *st = S.learned == 1 ? ix.d_order_stats : nullptr;
        int32_t *key = order + nq;
        hipLaunchKernelGGL(class_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, sm, a.rec, nq, key,
                           (const unsigned long long *)st);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(order_kernel, dim3(1), dim3(kOrderThreads), 0, sm, key, nq, order, st);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            SearchArgs b = a;
            b.perm = order;
            b.order_stats = st;
            hipLaunchKernelGGL(fn, dim3((unsigned)nq), dim3(64), lds, sm, b);
            e = hipGetLastError();
        }
        hipError_t ef = fixed ? hipSuccess : hipFreeAsync(order, sm);
        HIPCHK(e);
        HIPCHK(ef);
        return JAG_OK;
    }
    if (S.learned != 1 || S.single_pass || nq < 2) {
        hipLaunchKernelGGL(fn, dim3((unsigned)nq), dim3(64), lds, sm, a);
        HIPCHK(hipGetLastError());
        return JAG_OK;
    }
    // two passes over chunks of queries: run each to its prediction and save
    // its state (list and counters), order the chunk by predicted
    // beam, widest first, then resume every search in that order; the
    // scratch is stream-ordered memory from the default pool
    const int64_t stride = state_words(a.Lcap);
    const int64_t per_q = (stride + 2) * (int64_t)sizeof(int32_t);
    int32_t *saved = nullptr;
    int64_t chunk;
    if (fixed) {
        chunk = std::min<int64_t>(nq, fixed_bytes / per_q);
        if (chunk < 1) {
            set_error("one saved search state needs %lld bytes; the fixed scratch holds %lld",
                      (long long)per_q, (long long)fixed_bytes);
            return JAG_EINVAL;
        }
        saved = static_cast<int32_t *>(fixed_scratch);
    } else {
        keep_pool_reserved(ix.device);
        chunk = std::max<int64_t>(1, std::min<int64_t>(nq, kStateBudget / per_q));
        HIPCHK(hipMallocAsync((void **)&saved, (size_t)(chunk * per_q), sm));
    }
    int32_t *perm = saved + chunk * stride;
    int32_t *okey = perm + chunk;
    hipError_t e = hipSuccess;
    for (int64_t c0 = 0; c0 < nq && e == hipSuccess; c0 += chunk) {
        const int64_t nc = std::min(chunk, nq - c0);
        SearchArgs b = a;
        b.Q = a.Q + c0 * a.d;
        b.rec = a.rec + c0;
        b.ids = a.ids + c0 * k;
        b.dists = a.dists + c0 * k;
        b.count = a.count + c0;
        b.stats = a.stats ? a.stats + c0 * 4 : nullptr;
        b.state = saved;
        b.state_stride = stride;
        b.order_key = okey;
        SearchArgs b3 = b;
        b3.mode = 3;
        b3.stats = nullptr;
        hipLaunchKernelGGL(fn, dim3((unsigned)nc), dim3(64), lds, sm, b3);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(order_kernel, dim3(1), dim3(kOrderThreads), 0, sm, okey, nc, perm,
                           (unsigned long long *)nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        b.mode = 4;
        b.perm = perm;
        hipLaunchKernelGGL(fn, dim3((unsigned)nc), dim3(64), lds, sm, b);
        e = hipGetLastError();
    }
    hipError_t ef = fixed ? hipSuccess : hipFreeAsync(saved, sm);
    HIPCHK(e);
    HIPCHK(ef);
    return JAG_OK;
}

jag_status search_capacity(Index &ix, int32_t k, const jag_search_params &S, int64_t *resident,
                           size_t *lds_per_query)
{
    SearchArgs a;
    SearchFn fn = nullptr;
    size_t lds = 0;
    jag_search_params s2 = S;
    float dummy_f = 0.f;
    if (s2.learned == 2 && !s2.features) s2.features = &dummy_f;
    jag_status st = plan_batch(ix, &dummy_f, 1, &dummy_f, k, s2, nullptr, nullptr, nullptr, a, fn, lds);
    if (st != JAG_OK) return st;
    int per_cu = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), 64, lds));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, ix.device));
    *resident = (int64_t)per_cu * prop.multiProcessorCount;
    *lds_per_query = lds;
    return JAG_OK;
}

jag_status search_scratch_bytes(Index &ix, int32_t k, const jag_search_params &S, int64_t nq,
                                int64_t *bytes)
{
    SearchArgs a;
    SearchFn fn = nullptr;
    size_t lds = 0;
    jag_search_params s2 = S;
    float dummy_f = 0.f;
    if (s2.learned == 2 && !s2.features) s2.features = &dummy_f;
    jag_status st = plan_batch(ix, &dummy_f, 1, &dummy_f, k, s2, nullptr, nullptr, nullptr, a, fn, lds);
    if (st != JAG_OK) return st;
    *bytes = 0;
    if (S.learned == 1 && !S.single_pass && nq >= 2) {
        const int64_t per_q = (state_words(a.Lcap) + 2) * (int64_t)sizeof(int32_t);
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nq, kStateBudget / per_q));
        *bytes = chunk * per_q;
    } else if (sel_ordered(S, nq)) {
        *bytes = 2 * nq * (int64_t)sizeof(int32_t);  // the launch order and the classes
    }
    return JAG_OK;
}

jag_status launch_exact(Index &ix, const float *Q, int64_t nq, const void *records, int32_t k,
                        int32_t *ids, float *dists, int32_t *count, void *stream)
{
    if (k < 1 || k > 64 || nq > INT_MAX) {
        set_error("need 1 <= k <= 64");
        return JAG_EINVAL;
    }
    if (!ix.d_f32) {
        set_error("exact search needs the FP32 copy");
        return JAG_EUNSUPPORTED;
    }
    SearchArgs a;
    fill_args(ix, a, Q, records, k, ids, dists, count);
    a.Lcap = 64;
    a.Hmask = 0;
    int G = pick_group(ix.f32_stride);
    int ch = ix.f32_stride / (16 * G);
    ExactFn fn = G == 4 ? exact_for_ch<4>(ch) : G == 8 ? exact_for_ch<8>(ch) : exact_for_ch<16>(ch);
    if (!fn || ix.f32_stride % (16 * G)) {
        set_error("no exact kernel for FP32 row stride %d", ix.f32_stride);
        return JAG_EUNSUPPORTED;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)nq), dim3(64), lds_bytes(64, 1), (hipStream_t)stream, a, ix.n);
    HIPCHK(hipGetLastError());
    return JAG_OK;
}

}  // namespace jag

// ---------------------------------------------------------------- no-allocation search
// jag_search_encoded_noalloc keeps its scratch (launch order, saved states of
// a two-pass learned search) in this file-scope device array instead of
// allocating it.  In host code `scratch` only names the symbol: its device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.  Every call on a device shares that device's copy.
namespace jag {
constexpr int64_t kNoAllocScratchBytes = int64_t(32) << 20;
}
static __device__ __align__(256) unsigned char scratch[jag::kNoAllocScratchBytes];

namespace jag {
namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[256];

// Device address of this device's `scratch` (the current device).
jag_status scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= 256) {
        set_error("device %d out of range", dev);
        return JAG_EDEVICE;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return JAG_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return JAG_OK;
}
}  // namespace
}  // namespace jag

extern "C" jag_status jag_search_encoded_noalloc(jag_index *idx, const float *Q, int64_t nq,
                                                 const void *records, int32_t k,
                                                 const jag_search_params *S, int32_t *ids, float *dists,
                                                 int32_t *count, void *stream)
{
    if (!idx || !S || nq < 0 || (nq > 0 && (!Q || !records || !ids || !dists || !count))) {
        jag::set_error("null argument");
        return JAG_EINVAL;
    }
    if (nq == 0) return JAG_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        jag::set_error("no current device");
        return JAG_EDEVICE;
    }
    if (dev != idx->ix.device) {
        jag::set_error("index lives on device %d, current device is %d", idx->ix.device, dev);
        return JAG_EINVAL;
    }
    void *p = nullptr;
    jag_status st = jag::scratch_address(dev, &p);
    if (st != JAG_OK) return st;
    return jag::launch_search(idx->ix, Q, nq, records, k, *S, ids, dists, count, stream, p,
                              jag::kNoAllocScratchBytes);
}

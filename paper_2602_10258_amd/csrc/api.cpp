// Host side of the C ABI declared in include/jag.h: argument checking,
// index assembly, filter encoding with selectivity estimates, persistence.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "jag_internal.h"

#if defined(__AVX2__)
#include <immintrin.h>
#endif

namespace jag {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int32_t store_row_bytes(int32_t store, int32_t d)
{
    int64_t raw = store == JAG_STORE_F32 ? 4 * (int64_t)d
                : store == JAG_STORE_BF16 ? 2 * (int64_t)d
                : (int64_t)d + 4;  // FP8 codes + trailing scale
    return (int32_t)((raw + 63) / 64 * 64);
}

namespace {

jag_status check_attrs(int64_t n, const jag_attrs *A)
{
    if (!A) return JAG_OK;
    if (A->label_off || A->labels) {
        if (!A->label_off || !A->labels) {
            set_error("label_off and labels must both be given");
            return JAG_EINVAL;
        }
        if (A->vocab < 1 || A->vocab > 65535) {
            set_error("vocab must be in [1, 65535], got %d", A->vocab);
            return JAG_EINVAL;
        }
        if (A->label_off[0] != 0) {
            set_error("label_off[0] must be 0");
            return JAG_EINVAL;
        }
        for (int64_t i = 0; i < n; i++) {
            int64_t s = A->label_off[i], e = A->label_off[i + 1];
            if (e < s || e - s > kMaxLabelsPerItem) {
                set_error("item %lld has %lld labels (0..%d allowed)", (long long)i,
                          (long long)(e - s), kMaxLabelsPerItem);
                return JAG_EINVAL;
            }
            for (int64_t j = s; j < e; j++) {
                int32_t l = A->labels[j];
                if (l < 0 || l >= A->vocab) {
                    set_error("item %lld: label %d outside [0, %d)", (long long)i, l, A->vocab);
                    return JAG_EINVAL;
                }
                if (j > s && A->labels[j - 1] >= l) {
                    set_error("item %lld: labels not sorted and distinct", (long long)i);
                    return JAG_EINVAL;
                }
            }
        }
    }
    return JAG_OK;
}

void copy_attrs(Index &ix, const jag_attrs *A)
{
    int64_t n = ix.n;
    if (A && A->scalar) {
        ix.has_scalar = true;
        ix.scalar.assign(A->scalar, A->scalar + n);
        ix.scalar_sorted = ix.scalar;
        std::sort(ix.scalar_sorted.begin(), ix.scalar_sorted.end());
        ix.scal_min = ix.scalar_sorted.front();
        ix.scal_max = ix.scalar_sorted.back();
        const int64_t span = ix.scal_max - ix.scal_min;
        ix.scal_shift = 0;
        while ((span >> ix.scal_shift) >= (int64_t(1) << 16)) ix.scal_shift++;
        const int64_t nb = (span >> ix.scal_shift) + 1;
        ix.scal_cum.assign((size_t)nb + 1, n);
        int64_t b = 0;
        for (int64_t i = 0; i < n; i++) {
            const int64_t bi = ((int64_t)ix.scalar_sorted[i] - ix.scal_min) >> ix.scal_shift;
            while (b <= bi) ix.scal_cum[(size_t)b++] = i;
        }
    }
    if (A && A->label_off) {
        ix.has_labels = true;
        ix.vocab = A->vocab;
        ix.loff.assign(A->label_off, A->label_off + n + 1);
        ix.lab.assign(A->labels, A->labels + A->label_off[n]);
        int64_t mx = 0;
        for (int64_t i = 0; i < n; i++) mx = std::max(mx, ix.loff[i + 1] - ix.loff[i]);
        ix.W = mx <= 2 ? 2 : mx <= 4 ? 4 : mx <= 8 ? 8 : 16;
        ix.label_count.assign(ix.vocab, 0);
        for (int32_t l : ix.lab) ix.label_count[l]++;
    }
}

jag_status check_common(const float *X, int64_t n, int32_t d)
{
    if (!X || n < 1 || n > (int64_t)INT32_MAX - 1 || d < 1 || d > kMaxDim) {
        set_error("need X != NULL, 1 <= n < 2^31, 1 <= d <= %d", kMaxDim);
        return JAG_EINVAL;
    }
    for (int64_t i = 0; i < n * (int64_t)d; i++)
        if (!std::isfinite(X[i])) {
            set_error("X[%lld] is not finite", (long long)i);
            return JAG_EINVAL;
        }
    return JAG_OK;
}

jag_status finish(std::unique_ptr<jag_index> &h, const jag_build_params *P, jag_index **out)
{
    Index &ix = h->ix;
    ix.store = P ? P->store : JAG_STORE_F32;
    ix.keep_f32 = P ? (P->keep_f32 != 0) : false;
    if (ix.store < 0 || ix.store > 2) {
        set_error("unknown store %d", ix.store);
        return JAG_EINVAL;
    }
    jag_status st = upload_index(ix);
    if (st != JAG_OK) {
        free_device(ix);
        return st;
    }
    *out = h.release();
    return JAG_OK;
}

// ---- selectivity estimate (used for the predictor's features) ----
}  // namespace

int64_t scalar_rank_below(const Index &ix, int64_t v)
{
    if (v <= ix.scal_min) return 0;
    if (v > ix.scal_max) return ix.n;
    const size_t b = (size_t)((v - ix.scal_min) >> ix.scal_shift);
    const int32_t *base = ix.scalar_sorted.data();
    return std::lower_bound(base + ix.scal_cum[b], base + ix.scal_cum[b + 1], v) - base;
}

namespace {
double label_freq(const Index &ix, int32_t l)
{
    return (double)ix.label_count[l] / (double)ix.n;
}

}  // namespace

// Encode queries [q0, q1); stops at the first bad filter (message via set_error).
// Distance table of a Boolean function of nv variables (Section 3.1): on
// entry D[x] = 0 where the function is true and 255 elsewhere; on exit D[x]
// is the fewest variable flips from assignment x to a true assignment (255:
// none).  Hamming distance is a sum over the variables, so one min-plus pass
// per variable, D[x] = min(D[x], D[x ^ 2^v] + 1), in any order of the
// variables, gives the exact transform.  Variables 0..4 stay inside each
// 32-byte block and take one byte shuffle per pass; the others pair
// contiguous runs.
static void distance_transform(uint8_t *D, int nv)
{
    const int N = 1 << nv;
    int v = 0;
#if defined(__AVX2__)
    if (nv >= 5) {
        const __m256i one = _mm256_set1_epi8(1);
        __m256i swap[4];
        for (int k = 0; k < 4; k++) {
            alignas(32) uint8_t idx[32];
            for (int i = 0; i < 32; i++) idx[i] = (uint8_t)((i ^ (1 << k)) & 15);
            swap[k] = _mm256_load_si256(reinterpret_cast<const __m256i *>(idx));
        }
        for (int base = 0; base < N; base += 32) {
            __m256i d = _mm256_loadu_si256(reinterpret_cast<const __m256i *>(D + base));
            for (int k = 0; k < 4; k++)  // partners 1, 2, 4, 8 bytes away (inside 16-byte lanes)
                d = _mm256_min_epu8(d, _mm256_adds_epu8(_mm256_shuffle_epi8(d, swap[k]), one));
            // partner 16 bytes away: the other 16-byte lane
            d = _mm256_min_epu8(d, _mm256_adds_epu8(_mm256_permute2x128_si256(d, d, 1), one));
            _mm256_storeu_si256(reinterpret_cast<__m256i *>(D + base), d);
        }
        v = 5;
    }
#endif
    for (; v < nv; v++) {
        const int b = 1 << v;
        for (int base = 0; base < N; base += 2 * b) {
            uint8_t *__restrict lo = D + base;
            uint8_t *__restrict hi = D + base + b;
            for (int i = 0; i < b; i++) {
                const uint8_t d0 = lo[i], d1 = hi[i];
                const uint8_t a0 = d0 == 255 ? 255 : (uint8_t)(d0 + 1);
                const uint8_t a1 = d1 == 255 ? 255 : (uint8_t)(d1 + 1);
                lo[i] = d0 < a1 ? d0 : a1;
                hi[i] = d1 < a0 ? d1 : a0;
            }
        }
    }
}

// TABLE filters write their distance table at tab_base + tpos[q] (tab_base is
// also the address of record 0); without a table area they are rejected.
static jag_status encode_range(const Index &ix, const jag_filter *F, int64_t q0, int64_t q1,
                               const int32_t *pool, int64_t pool_len, FilterRecord *out,
                               unsigned char *tab_base, const int64_t *tpos)
{
    // range estimates read the rank index at two places per filter: the
    // lines a few filters ahead are requested early, bucket bounds first
    constexpr int64_t kAhead = 8;
    auto bucket = [&](int64_t v) -> int64_t {
        return v <= ix.scal_min || v > ix.scal_max ? -1 : (v - ix.scal_min) >> ix.scal_shift;
    };
    auto ahead = [&](int64_t qa, bool rows) {
        if (qa >= q1 || F[qa].type != F_RANGE || !ix.has_scalar) return;
        for (int64_t v : {(int64_t)F[qa].lo, (int64_t)F[qa].hi + 1}) {
            const int64_t b = bucket(v);
            if (b < 0) continue;
            if (rows) __builtin_prefetch(ix.scalar_sorted.data() + ix.scal_cum[(size_t)b]);
            else __builtin_prefetch(ix.scal_cum.data() + b);
        }
    };
    for (int64_t q = q0; q < q1; q++) {
        ahead(q + 2 * kAhead, false);
        ahead(q + kAhead, true);
        const jag_filter &f = F[q];
        FilterRecord r;
        std::memset(&r, 0, sizeof(r));
        r.type = f.type;
        double sel = 1.0;
        auto need_labels = [&]() -> bool {
            if (!ix.has_labels) {
                set_error("query %lld: label filter on an index without labels", (long long)q);
                return false;
            }
            return true;
        };
        auto check_label = [&](int32_t l) -> bool {
            if (l < 0 || l >= ix.vocab) {
                set_error("query %lld: label %d outside [0, %d)", (long long)q, l, ix.vocab);
                return false;
            }
            return true;
        };
        auto check_span = [&]() -> bool {
            if (!pool || f.off < 0 || f.len < 1 || (int64_t)f.off + f.len > pool_len) {
                set_error("query %lld: pool span [%d, %d+%d) outside pool of %lld", (long long)q,
                          f.off, f.off, f.len, (long long)pool_len);
                return false;
            }
            return true;
        };
        if (f.type == F_LABEL) {
            if (!need_labels() || !check_label(f.label)) return JAG_EINVAL;
            r.a = f.label;
            r.lits[0] = (uint16_t)f.label;
            r.nlit = 1;
            sel = label_freq(ix, f.label);
        } else if (f.type == F_RANGE) {
            if (!ix.has_scalar) {
                set_error("query %lld: range filter on an index without scalars", (long long)q);
                return JAG_EINVAL;
            }
            r.a = f.lo;
            r.b = f.hi;
            sel = f.hi < f.lo ? 0.0
                              : (double)(scalar_rank_below(ix, (int64_t)f.hi + 1) - scalar_rank_below(ix, f.lo)) /
                                    (double)ix.n;
        } else if (f.type == F_SUBSET) {
            if (!need_labels() || !check_span()) return JAG_EINVAL;
            if (f.len > kMaxFilterLits) {
                set_error("query %lld: subset of %d labels (max %d)", (long long)q, f.len, kMaxFilterLits);
                return JAG_EINVAL;
            }
            int n = 0;
            for (int j = 0; j < f.len; j++) {
                int32_t l = pool[f.off + j];
                if (!check_label(l)) return JAG_EINVAL;
                bool dup = false;
                for (int x = 0; x < n; x++) dup |= (r.lits[x] == l);
                if (!dup) {
                    r.lits[n++] = (uint16_t)l;
                    sel *= label_freq(ix, l);
                }
            }
            r.nlit = n;
        } else if (f.type == F_BOOLEAN) {
            if (!need_labels() || !check_span()) return JAG_EINVAL;
            const int32_t *p = pool + f.off, *pe = pool + f.off + f.len;
            int32_t ncl = *p++;
            if (ncl < 1 || ncl > kMaxClauses) {
                set_error("query %lld: %d clauses (1..%d allowed)", (long long)q, ncl, kMaxClauses);
                return JAG_EINVAL;
            }
            int nl = 0, nc = 0;
            // literal i: label lits[i], negated if bit i of negmask
            std::vector<std::vector<int>> clause_lits;
            for (int c = 0; c < ncl; c++) {
                if (p >= pe) {
                    set_error("query %lld: truncated Boolean program", (long long)q);
                    return JAG_EINVAL;
                }
                int32_t m = *p++;
                if (m < 1 || p + m > pe) {
                    set_error("query %lld: bad clause length %d", (long long)q, m);
                    return JAG_EINVAL;
                }
                uint16_t mask = 0;
                bool contradictory = false;
                std::vector<int> cl;
                for (int j = 0; j < m; j++) {
                    int32_t lit = p[j];
                    bool neg = lit < 0;
                    int32_t l = neg ? ~lit : lit;
                    if (!check_label(l)) return JAG_EINVAL;
                    int idx = -1;
                    for (int x = 0; x < nl; x++)
                        if (r.lits[x] == l && (((r.negmask >> x) & 1u) != 0) == neg) idx = x;
                    if (idx < 0) {
                        if (nl >= kMaxFilterLits) {
                            set_error("query %lld: more than %d distinct literals", (long long)q,
                                      kMaxFilterLits);
                            return JAG_EINVAL;
                        }
                        idx = nl++;
                        r.lits[idx] = (uint16_t)l;
                        if (neg) r.negmask |= 1u << idx;
                    }
                    mask |= (uint16_t)(1u << idx);
                }
                p += m;
                // a clause holding both l and ~l can never be satisfied
                for (int x = 0; x < nl; x++)
                    for (int y = 0; y < nl; y++)
                        if (((mask >> x) & 1) && ((mask >> y) & 1) && r.lits[x] == r.lits[y] && x != y)
                            contradictory = true;
                if (!contradictory) {
                    r.clmask[nc++] = mask;
                    for (int x = 0; x < nl; x++)
                        if ((mask >> x) & 1) cl.push_back(x);
                    clause_lits.push_back(cl);
                }
            }
            if (p != pe) {
                set_error("query %lld: Boolean program length mismatch", (long long)q);
                return JAG_EINVAL;
            }
            r.nlit = nl;
            r.ncl = nc;
            // P(OR of clauses) by inclusion-exclusion, literals independent
            auto pl = [&](int x) {
                double pf = label_freq(ix, r.lits[x]);
                return ((r.negmask >> x) & 1u) ? 1.0 - pf : pf;
            };
            sel = 0.0;
            for (int s = 1; s < (1 << nc); s++) {
                uint32_t u = 0;
                for (int c = 0; c < nc; c++)
                    if ((s >> c) & 1) u |= r.clmask[c];
                bool bad = false;
                for (int x = 0; x < nl; x++)
                    for (int y = 0; y < nl; y++)
                        if (((u >> x) & 1) && ((u >> y) & 1) && x != y && r.lits[x] == r.lits[y]) bad = true;
                double pr = 0.0;
                if (!bad) {
                    pr = 1.0;
                    for (int x = 0; x < nl; x++)
                        if ((u >> x) & 1) pr *= pl(x);
                }
                sel += (__builtin_popcount(s) & 1) ? pr : -pr;
            }
            sel = std::min(1.0, std::max(0.0, sel));
        } else if (f.type == F_TABLE) {
            // general Boolean function of nvar labels (Section 3.1): the
            // distance of assignment x is the fewest flips to a true one
            if (!need_labels() || !check_span()) return JAG_EINVAL;
            const int32_t *p = pool + f.off;
            const int nv = p[0];
            if (nv < 1 || nv > kMaxTableVars || f.len != 1 + nv + ((1 << nv) + 31) / 32) {
                set_error("query %lld: a table filter holds nvar (1..%d), nvar labels and "
                          "ceil(2^nvar / 32) truth-table words", (long long)q, kMaxTableVars);
                return JAG_EINVAL;
            }
            for (int v = 0; v < nv; v++) {
                int32_t l = p[1 + v];
                if (!check_label(l)) return JAG_EINVAL;
                for (int x = 0; x < v; x++)
                    if (r.lits[x] == l) {
                        set_error("query %lld: table variable label %d repeated", (long long)q, l);
                        return JAG_EINVAL;
                    }
                r.lits[v] = (uint16_t)l;
            }
            r.nlit = nv;
            if (!tab_base) {
                set_error("query %lld: table filters need jag_encode_filters_sized (their distance "
                          "tables do not fit the fixed records)", (long long)q);
                return JAG_EINVAL;
            }
            const uint32_t *w = reinterpret_cast<const uint32_t *>(p + 1 + nv);
            uint8_t *D = tab_base + tpos[q];
            const int N = 1 << nv;
            for (int x = 0; x < N; x++) D[x] = ((w[x >> 5] >> (x & 31)) & 1u) ? 0 : 255;
            distance_transform(D, nv);
            // probability of each assignment under independent labels, built
            // by doubling (each product is formed in variable order, as a
            // per-assignment loop would), summed over the true assignments
            thread_local std::vector<double> pa;
            pa.assign((size_t)N, 1.0);
            for (int v = 0; v < nv; v++) {
                const double pf = label_freq(ix, r.lits[v]);
                const int b = 1 << v;
                double *__restrict lo = pa.data();
                double *__restrict hi = pa.data() + b;
                for (int x = 0; x < b; x++) {
                    hi[x] = lo[x] * pf;
                    lo[x] = lo[x] * (1.0 - pf);
                }
            }
            // in increasing order of the true assignments, visiting set bits only
            sel = 0.0;
            for (int wi = 0; wi < (N + 31) / 32; wi++) {
                uint32_t word = N >= 32 ? w[wi] : (w[wi] & ((1u << N) - 1u));
                for (; word; word &= word - 1) sel += pa[(size_t)(wi * 32 + __builtin_ctz(word))];
            }
            sel = std::min(1.0, sel);
            r.table_off = tpos[q] - q * (int64_t)sizeof(FilterRecord);
        } else {
            set_error("query %lld: unknown filter type %d", (long long)q, f.type);
            return JAG_EINVAL;
        }
        r.selectivity = (float)sel;
        r.sel_feature = (float)(std::log2(std::max(sel, 1e-9)) / 16.0);
        out[q] = r;
    }
    return JAG_OK;
}

// Host threads that encode the chunks of large batches.  Started on first
// use and kept (one call's chunks at a time; a call that finds the pool busy
// encodes its chunks itself), so a batch does not pay for starting threads.
class EncodePool {
  public:
    static EncodePool &get()
    {
        static EncodePool p;
        return p;
    }
    // fn(c) for every chunk c in [0, n); the caller takes chunks too
    void run(int n, const std::function<void(int)> &fn)
    {
        std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
        if (!busy.owns_lock() || workers_.empty()) {
            for (int c = 0; c < n; c++) fn(c);
            return;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            fn_ = &fn;
            n_ = n;
            next_.store(0);
            left_ = n;
            gen_++;
        }
        cv_.notify_all();
        drain();
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return left_ == 0; });
        fn_ = nullptr;
    }
    ~EncodePool()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }

  private:
    EncodePool()
    {
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        for (unsigned t = 1; t < std::min(hw, 8u); t++) workers_.emplace_back([this] { loop(); });
    }
    void drain()
    {
        for (;;) {
            const int c = next_.fetch_add(1);
            if (c >= n_) return;
            (*fn_)(c);
            std::lock_guard<std::mutex> g(mu_);
            if (--left_ == 0) done_.notify_all();
        }
    }
    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || (gen_ != seen && fn_); });
                if (stop_) return;
                seen = gen_;
            }
            drain();
        }
    }
    std::mutex run_mu_, mu_;
    std::condition_variable cv_, done_;
    std::vector<std::thread> workers_;
    const std::function<void(int)> *fn_ = nullptr;
    int n_ = 0, left_ = 0;
    std::atomic<int> next_{0};
    uint64_t gen_ = 0;
    bool stop_ = false;
};

static jag_status run_encode(const Index &ix, const jag_filter *F, int64_t nq, const int32_t *pool,
                             int64_t pool_len, FilterRecord *out, unsigned char *tab_base,
                             const int64_t *tpos)
{
    // large batches are encoded in chunks by the pool's host threads
    constexpr int64_t kChunk = 1024;
    const int nch = (int)((nq + kChunk - 1) / kChunk);
    if (nch <= 1) return encode_range(ix, F, 0, nq, pool, pool_len, out, tab_base, tpos);
    std::vector<jag_status> st(nch, JAG_OK);
    std::vector<std::string> msg(nch);
    EncodePool::get().run(nch, [&](int c) {
        st[c] = encode_range(ix, F, c * kChunk, std::min(nq, (c + 1) * kChunk), pool, pool_len, out, tab_base,
                             tpos);
        if (st[c] != JAG_OK) msg[c] = g_err;  // the worker's own thread-local message
    });
    for (int c = 0; c < nch; c++)
        if (st[c] != JAG_OK) {  // the first bad query in batch order
            set_error("%s", msg[c].c_str());
            return st[c];
        }
    return JAG_OK;
}

jag_status encode_filters(const Index &ix, const jag_filter *F, int64_t nq, const int32_t *pool,
                          int64_t pool_len, FilterRecord *out)
{
    return run_encode(ix, F, nq, pool, pool_len, out, nullptr, nullptr);
}

// Byte offset of every TABLE filter's distance table from the start of the
// encoded buffer (-1 for other filters) and the buffer's total size.
static jag_status table_layout(const jag_filter *F, int64_t nq, const int32_t *pool, int64_t pool_len,
                               std::vector<int64_t> *tpos, int64_t *bytes)
{
    int64_t at = nq * (int64_t)sizeof(FilterRecord);
    if (tpos) tpos->assign((size_t)nq, -1);
    for (int64_t q = 0; q < nq; q++) {
        if (F[q].type != F_TABLE) continue;
        const jag_filter &f = F[q];
        if (!pool || f.off < 0 || f.len < 1 || (int64_t)f.off + f.len > pool_len || pool[f.off] < 1 ||
            pool[f.off] > kMaxTableVars) {
            set_error("query %lld: bad table filter span or variable count", (long long)q);
            return JAG_EINVAL;
        }
        if (tpos) (*tpos)[(size_t)q] = at;
        at += ((int64_t(1) << pool[f.off]) + 15) / 16 * 16;
    }
    *bytes = at;
    return JAG_OK;
}

jag_status encoded_bytes(const Index &, const jag_filter *F, int64_t nq, const int32_t *pool, int64_t pool_len,
                         int64_t *bytes)
{
    return table_layout(F, nq, pool, pool_len, nullptr, bytes);
}

jag_status encode_filters_sized(const Index &ix, const jag_filter *F, int64_t nq, const int32_t *pool,
                                int64_t pool_len, void *out, int64_t out_bytes)
{
    std::vector<int64_t> tpos;
    int64_t need = 0;
    jag_status st = table_layout(F, nq, pool, pool_len, &tpos, &need);
    if (st != JAG_OK) return st;
    if (out_bytes < need) {
        set_error("encoded filters need %lld bytes, the buffer holds %lld", (long long)need,
                  (long long)out_bytes);
        return JAG_EINVAL;
    }
    unsigned char *base = static_cast<unsigned char *>(out);
    return run_encode(ix, F, nq, pool, pool_len, reinterpret_cast<FilterRecord *>(base), base, tpos.data());
}

}  // namespace jag

using jag::Index;
using jag::set_error;

namespace {
template <class T>
bool wr(FILE *f, const T *p, size_t cnt) { return fwrite(p, sizeof(T), cnt, f) == cnt; }
template <class T>
bool rd(FILE *f, T *p, size_t cnt) { return fread(p, sizeof(T), cnt, f) == cnt; }
}  // namespace

extern "C" {

const char *jag_last_error(void) { return jag::g_err; }
const char *jag_version(void) { return "jag-mi355x 0.1 (gfx950)"; }

static jag_status make_config(const float *X, int64_t n, int32_t d, const jag_attrs *A,
                              const jag_build_params *P, jag::BuildConfig &cfg)
{
    if (!P) {
        set_error("params are required");
        return JAG_EINVAL;
    }
    jag_status st = jag::check_common(X, n, d);
    if (st != JAG_OK) return st;
    if ((st = jag::check_attrs(n, A)) != JAG_OK) return st;
    if (P->R < 1 || P->R > jag::kMaxR || P->n_thr < 1 || P->n_thr > 8 || !P->thr ||
        !(P->alpha >= 1.0f) || P->L_build < 0) {
        set_error("need 1 <= R <= %d, 1 <= n_thr <= 8, alpha >= 1, L_build >= 0", jag::kMaxR);
        return JAG_EINVAL;
    }
    cfg.R = P->R;
    cfg.L_build = P->L_build > 0 ? P->L_build : 2 * P->R;
    cfg.alpha = P->alpha;
    cfg.seed = P->seed;
    cfg.n_threads = P->n_threads;
    cfg.max_batch = P->max_batch;
    cfg.progress = P->progress;
    for (int i = 0; i < P->n_thr; i++) {
        const int full = P->thr[i].kind;
        const int kind = full & ~JAG_THRESHOLD_WEIGHT;
        if (kind == JAG_ATTR_SCALAR && !(A && A->scalar)) {
            set_error("threshold %d names scalar attributes the index does not have", i);
            return JAG_EINVAL;
        }
        if ((kind == JAG_ATTR_LABELS || kind == JAG_ATTR_LABELS_WEIGHTED) && !(A && A->label_off)) {
            set_error("threshold %d names labels the index does not have", i);
            return JAG_EINVAL;
        }
        if (kind != JAG_ATTR_SCALAR && kind != JAG_ATTR_LABELS && kind != JAG_ATTR_LABELS_WEIGHTED) {
            set_error("threshold %d: unknown attribute kind %d", i, kind);
            return JAG_EINVAL;
        }
        if (!(P->thr[i].quantile >= 0.f)) {
            set_error("threshold %d: quantile must be >= 0", i);
            return JAG_EINVAL;
        }
        cfg.kinds.push_back(full);
        cfg.quantiles.push_back(P->thr[i].quantile);
    }
    if (P->device != 0 && P->device != 1) {
        set_error("device must be 0 (host threads) or 1 (GPU)");
        return JAG_EINVAL;
    }
    cfg.device = P->device;
    if (P->order) {
        std::vector<char> hit((size_t)n, 0);
        for (int64_t i = 0; i < n; i++) {
            const int32_t v = P->order[i];
            if (v < 0 || v >= n || hit[(size_t)v]) {
                set_error("order is not a permutation of 0..n-1 (position %lld)", (long long)i);
                return JAG_EINVAL;
            }
            hit[(size_t)v] = 1;
        }
        cfg.order = P->order;
    }
    if (P->thresholds) {
        for (int64_t i = 0; i < n * (int64_t)P->n_thr; i++) {
            const float t = P->thresholds[i];
            const bool weight = (P->thr[i % P->n_thr].kind & JAG_THRESHOLD_WEIGHT) != 0;
            if (!(t >= 0.f) || (weight && std::isinf(t))) {
                set_error("thresholds[%lld] = %g is not a valid %s", (long long)i, (double)t,
                          weight ? "weight (finite, >= 0)" : "threshold (>= 0 or +inf)");
                return JAG_EINVAL;
            }
        }
        cfg.thresholds = P->thresholds;
    }
    return JAG_OK;
}

// The graph of cfg on host threads or on the current device.
static jag_status run_build(const float *X, int64_t n, int32_t d, const jag::AttrView &av,
                            const jag::BuildConfig &cfg, std::vector<int32_t> &adj, int32_t &entry)
{
    if (cfg.device) return jag::build_graph_device(X, n, d, av, cfg, adj, entry);
    jag::build_graph(X, n, d, av, cfg, adj, entry);
    return JAG_OK;
}

jag_status jag_build_graph(const float *X, int64_t n, int32_t d, const jag_attrs *A,
                           const jag_build_params *P, int32_t *adj_out, int32_t *entry)
{
    if (!adj_out || !entry) {
        set_error("adj_out and entry are required");
        return JAG_EINVAL;
    }
    jag::BuildConfig cfg;
    jag_status st = make_config(X, n, d, A, P, cfg);
    if (st != JAG_OK) return st;
    try {
        jag::AttrView av{n, A ? A->scalar : nullptr, A ? A->label_off : nullptr, A ? A->labels : nullptr};
        std::vector<int32_t> adj;
        st = run_build(X, n, d, av, cfg, adj, *entry);
        if (st != JAG_OK) return st;
        std::memcpy(adj_out, adj.data(), adj.size() * sizeof(int32_t));
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return JAG_ENOMEM;
    }
    return JAG_OK;
}

jag_status jag_build(const float *X, int64_t n, int32_t d, const jag_attrs *A,
                     const jag_build_params *P, jag_index **out)
{
    if (!out) {
        set_error("out is required");
        return JAG_EINVAL;
    }
    *out = nullptr;
    jag::BuildConfig cfg;
    jag_status st = make_config(X, n, d, A, P, cfg);
    if (st != JAG_OK) return st;
    std::unique_ptr<jag_index> h(new (std::nothrow) jag_index);
    if (!h) return JAG_ENOMEM;
    Index &ix = h->ix;
    ix.n = n;
    ix.d = d;
    ix.R = P->R;
    try {
        ix.X.assign(X, X + n * (int64_t)d);
        jag::copy_attrs(ix, A);
        jag::AttrView av{n, ix.has_scalar ? ix.scalar.data() : nullptr,
                         ix.has_labels ? ix.loff.data() : nullptr,
                         ix.has_labels ? ix.lab.data() : nullptr};
        st = run_build(ix.X.data(), n, d, av, cfg, ix.adj, ix.entry);
        if (st != JAG_OK) return st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return JAG_ENOMEM;
    }
    return jag::finish(h, P, out);
}

jag_status jag_build_from_graph(const float *X, int64_t n, int32_t d, const jag_attrs *A,
                                const int32_t *adj, int32_t R, int32_t entry,
                                const jag_build_params *P, jag_index **out)
{
    if (!out || !adj) {
        set_error("out and adj are required");
        return JAG_EINVAL;
    }
    *out = nullptr;
    jag_status st = jag::check_common(X, n, d);
    if (st != JAG_OK) return st;
    if ((st = jag::check_attrs(n, A)) != JAG_OK) return st;
    if (R < 1 || R > jag::kMaxR || entry < 0 || entry >= n) {
        set_error("need 1 <= R <= %d and 0 <= entry < n", jag::kMaxR);
        return JAG_EINVAL;
    }
    for (int64_t i = 0; i < n; i++) {
        const int32_t *row = adj + i * R;
        for (int j = 0; j < R; j++) {
            int32_t v = row[j];
            if (v < -1 || v >= n) {
                set_error("adj[%lld][%d] = %d out of range", (long long)i, j, v);
                return JAG_EINVAL;
            }
            if (v < 0) continue;
            for (int x = 0; x < j; x++)
                if (row[x] == v) {
                    set_error("adj row %lld repeats id %d", (long long)i, v);
                    return JAG_EINVAL;
                }
        }
    }
    std::unique_ptr<jag_index> h(new (std::nothrow) jag_index);
    if (!h) return JAG_ENOMEM;
    Index &ix = h->ix;
    ix.n = n;
    ix.d = d;
    ix.R = R;
    ix.entry = entry;
    try {
        ix.X.assign(X, X + n * (int64_t)d);
        ix.adj.assign(adj, adj + n * (int64_t)R);
        jag::copy_attrs(ix, A);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return JAG_ENOMEM;
    }
    return jag::finish(h, P, out);
}

void jag_free(jag_index *idx)
{
    if (!idx) return;
    jag::free_device(idx->ix);
    delete idx;
}

jag_status jag_info(const jag_index *idx, jag_index_info *out)
{
    if (!idx || !out) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    const Index &ix = idx->ix;
    out->n = ix.n;
    out->d = ix.d;
    out->R = ix.R;
    out->entry = ix.entry;
    out->store = ix.store;
    out->has_f32 = ix.d_f32 != nullptr;
    out->has_scalar = ix.has_scalar;
    out->has_labels = ix.has_labels;
    out->label_width = ix.W;
    out->vocab = ix.vocab;
    out->has_predictor = ix.pred.present;
    out->device_bytes = ix.device_bytes;
    return JAG_OK;
}

jag_status jag_get_graph(const jag_index *idx, int32_t *adj_out, int32_t *entry)
{
    if (!idx || !adj_out || !entry) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    std::memcpy(adj_out, idx->ix.adj.data(), idx->ix.adj.size() * sizeof(int32_t));
    *entry = idx->ix.entry;
    return JAG_OK;
}

jag_status jag_get_store(const jag_index *idx, void *rows_out, float *scales_out)
{
    if (!idx || !rows_out) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    return jag::download_store(idx->ix, rows_out, scales_out);
}

jag_status jag_encode_filters(const jag_index *idx, const jag_filter *F, int64_t nq,
                              const int32_t *pool, int64_t pool_len, void *records_out)
{
    if (!idx || (nq > 0 && (!F || !records_out)) || nq < 0) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    return jag::encode_filters(idx->ix, F, nq, pool, pool_len,
                               static_cast<jag::FilterRecord *>(records_out));
}

jag_status jag_encoded_bytes(const jag_index *idx, const jag_filter *F, int64_t nq, const int32_t *pool,
                             int64_t pool_len, int64_t *bytes)
{
    if (!idx || !bytes || nq < 0 || (nq > 0 && !F)) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    return jag::encoded_bytes(idx->ix, F, nq, pool, pool_len, bytes);
}

jag_status jag_encode_filters_sized(const jag_index *idx, const jag_filter *F, int64_t nq,
                                    const int32_t *pool, int64_t pool_len, void *out, int64_t out_bytes)
{
    if (!idx || nq < 0 || (nq > 0 && (!F || !out))) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    return jag::encode_filters_sized(idx->ix, F, nq, pool, pool_len, out, out_bytes);
}

jag_status jag_search_encoded(jag_index *idx, const float *Q, int64_t nq, const void *records,
                              int32_t k, const jag_search_params *S, int32_t *ids, float *dists,
                              int32_t *count, void *stream)
{
    if (!idx || !S || nq < 0 || (nq > 0 && (!Q || !records || !ids || !dists || !count))) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    if (nq == 0) return JAG_OK;
    return jag::launch_search(idx->ix, Q, nq, records, k, *S, ids, dists, count, stream);
}

jag_status jag_exact_knn(jag_index *idx, const float *Q, int64_t nq, const void *records,
                         int32_t k, int32_t *ids, float *dists, int32_t *count, void *stream)
{
    if (!idx || nq < 0 || (nq > 0 && (!Q || !records || !ids || !dists || !count))) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    if (nq == 0) return JAG_OK;
    return jag::launch_exact(idx->ix, Q, nq, records, k, ids, dists, count, stream);
}

jag_status jag_set_predictor(jag_index *idx, const float *params, int32_t nladder,
                             const int32_t *ladder, float rho)
{
    if (!idx || !params || !ladder || nladder < 1 || nladder > JAG_LADDER_MAX || !(rho > 0.f)) {
        set_error("need params, 1 <= nladder <= %d, ladder, rho > 0", JAG_LADDER_MAX);
        return JAG_EINVAL;
    }
    for (int i = 0; i < nladder; i++)
        if (ladder[i] < 1 || ladder[i] > 1024 || (i > 0 && ladder[i] <= ladder[i - 1])) {
            set_error("ladder must be increasing within [1, 1024]");
            return JAG_EINVAL;
        }
    for (int i = 0; i < jag::kPredParams; i++)
        if (!std::isfinite(params[i])) {
            set_error("predictor parameter %d is not finite", i);
            return JAG_EINVAL;
        }
    jag::Predictor &p = idx->ix.pred;
    p.params.assign(params, params + jag::kPredParams);
    p.nladder = nladder;
    std::copy(ladder, ladder + nladder, p.ladder);
    p.rho = rho;
    jag_status st = jag::upload_predictor(idx->ix);
    if (st == JAG_OK) p.present = true;
    return st;
}

jag_status jag_train_predictor(const float *features, const float *targets, int64_t m,
                               float *params_inout, int32_t epochs, int32_t batch, float lr,
                               uint64_t seed, float *loss_out, void *stream)
{
    if (!features || !targets || !params_inout || m < 1 || epochs < 1 || batch < 1 ||
        !(lr > 0.f)) {
        set_error("bad training arguments");
        return JAG_EINVAL;
    }
    return jag::train_predictor(features, targets, m, params_inout, epochs, batch, lr, seed,
                                loss_out, stream);
}

jag_status jag_predictor_grad(const float *features, const float *targets, int64_t m,
                              const float *params, float *loss_out, float *grad_out, void *stream)
{
    if (!features || !targets || !params || !loss_out || !grad_out || m < 1) {
        set_error("bad arguments");
        return JAG_EINVAL;
    }
    return jag::predictor_grad(features, targets, m, params, loss_out, grad_out, stream);
}

// ---- persistence ----------------------------------------------------------
// File: "JAGIDX01", then int64 n, int32 d, R, entry, store, keep_f32,
// has_scalar, has_labels, vocab, has_pred, nladder, float rho, int32 ladder[16],
// then X[n*d] f32, adj[n*R] i32, [scalar[n] i32], [loff[n+1] i64, lab[] i32],
// [params[5313] f32].


jag_status jag_save(const jag_index *idx, const char *path)
{
    if (!idx || !path) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    const Index &ix = idx->ix;
    FILE *f = fopen(path, "wb");
    if (!f) {
        set_error("cannot open %s for writing", path);
        return JAG_EIO;
    }
    int32_t hdr[10] = {ix.d, ix.R, ix.entry, ix.store, ix.keep_f32, ix.has_scalar, ix.has_labels,
                       ix.vocab, ix.pred.present, ix.pred.nladder};
    bool ok = wr(f, "JAGIDX01", 8) && wr(f, &ix.n, 1) && wr(f, hdr, 10) && wr(f, &ix.pred.rho, 1) &&
              wr(f, ix.pred.ladder, JAG_LADDER_MAX) && wr(f, ix.X.data(), ix.X.size()) &&
              wr(f, ix.adj.data(), ix.adj.size());
    if (ok && ix.has_scalar) ok = wr(f, ix.scalar.data(), ix.scalar.size());
    if (ok && ix.has_labels) ok = wr(f, ix.loff.data(), ix.loff.size()) && wr(f, ix.lab.data(), ix.lab.size());
    if (ok && ix.pred.present) ok = wr(f, ix.pred.params.data(), ix.pred.params.size());
    ok = (fclose(f) == 0) && ok;
    if (!ok) {
        set_error("write to %s failed", path);
        return JAG_EIO;
    }
    return JAG_OK;
}

jag_status jag_load(const char *path, jag_index **out)
{
    if (!path || !out) {
        set_error("null argument");
        return JAG_EINVAL;
    }
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) {
        set_error("cannot open %s", path);
        return JAG_EIO;
    }
    std::unique_ptr<FILE, int (*)(FILE *)> guard(f, fclose);
    char magic[8];
    int64_t n;
    int32_t hdr[10];
    float rho;
    int32_t ladder[JAG_LADDER_MAX];
    if (!rd(f, magic, 8) || std::memcmp(magic, "JAGIDX01", 8) != 0 || !rd(f, &n, 1) ||
        !rd(f, hdr, 10) || !rd(f, &rho, 1) || !rd(f, ladder, JAG_LADDER_MAX)) {
        set_error("%s: not a JAG index file", path);
        return JAG_EINVAL;
    }
    int32_t d = hdr[0], R = hdr[1];
    if (n < 1 || d < 1 || d > jag::kMaxDim || R < 1 || R > jag::kMaxR || hdr[2] < 0 || hdr[2] >= n ||
        hdr[9] < 0 || hdr[9] > JAG_LADDER_MAX) {
        set_error("%s: corrupt header", path);
        return JAG_EINVAL;
    }
    std::vector<float> X;
    std::vector<int32_t> adj, scalar, lab;
    std::vector<int64_t> loff;
    std::vector<float> params;
    try {
        X.resize((size_t)n * d);
        adj.resize((size_t)n * R);
        if (!rd(f, X.data(), X.size()) || !rd(f, adj.data(), adj.size())) throw 1;
        if (hdr[5]) {
            scalar.resize(n);
            if (!rd(f, scalar.data(), scalar.size())) throw 1;
        }
        if (hdr[6]) {
            loff.resize(n + 1);
            if (!rd(f, loff.data(), loff.size()) || loff[0] != 0 || loff[n] < 0) throw 1;
            lab.resize(loff[n]);
            if (!rd(f, lab.data(), lab.size())) throw 1;
        }
        if (hdr[8]) {
            params.resize(jag::kPredParams);
            if (!rd(f, params.data(), params.size())) throw 1;
        }
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return JAG_ENOMEM;
    } catch (int) {
        set_error("%s: truncated or corrupt file", path);
        return JAG_EINVAL;
    }
    jag_attrs A{hdr[5] ? scalar.data() : nullptr, hdr[6] ? loff.data() : nullptr,
                hdr[6] ? lab.data() : nullptr, hdr[7]};
    jag_build_params P;
    std::memset(&P, 0, sizeof(P));
    P.store = hdr[3];
    P.keep_f32 = hdr[4];
    jag_status st = jag_build_from_graph(X.data(), n, d, &A, adj.data(), R, hdr[2], &P, out);
    if (st != JAG_OK) return st;
    if (hdr[8]) {
        st = jag_set_predictor(*out, params.data(), hdr[9], ladder, rho);
        if (st != JAG_OK) {
            jag_free(*out);
            *out = nullptr;
            return st;
        }
    }
    return JAG_OK;
}

}  // extern "C"

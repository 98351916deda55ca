// Threshold-JAG construction on host threads (paper Section 3.3,
// Algorithms 3 and 4, Appendix D.3).
//
// Insertions run in rounds: the first point (the entry vertex) alone, then
// rounds that double in size up to a cap.  Within a round every point runs
// its |T| greedy searches against the graph frozen at the start of the
// round and prunes its own out-list (Algorithm 3, lines up to the prune);
// then the reverse edges of the whole round are grouped by target and each
// target vertex merges its new in-links, re-pruning when it would exceed R.
// Every write touches one vertex's row from one task, so the graph depends
// only on the seed, not on thread count or timing.
#include <algorithm>
#include <cstdio>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <thread>

#include "jag_internal.h"

namespace jag {
namespace {

inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

// Squared Euclidean distance in the library's fixed FP32 order: partial sum
// k (0..31) takes the elements i = k mod 32 with one fused multiply-add each;
// the 32 partials fold as ((s0 + s1) + (s2 + s3)) per group of four, then the
// eight group sums pairwise at strides 4, 2 and 1.  The device builder reads
// a row as eight float4 per 32 elements (lane g of 8 holds partials 4g..4g+3)
// and folds across lanes in the same order, so both give identical bits.
float l2sq_canonical(const float *__restrict a, const float *__restrict b, int d)
{
    float acc[32] = {};
    int i = 0;
    for (; i + 32 <= d; i += 32)
        for (int k = 0; k < 32; k++) {
            const float t = a[i + k] - b[i + k];
            acc[k] = std::fma(t, t, acc[k]);
        }
    for (int k = 0; i + k < d; k++) {
        const float t = a[i + k] - b[i + k];
        acc[k] = std::fma(t, t, acc[k]);
    }
    float u[8];
    for (int g = 0; g < 8; g++) u[g] = (acc[4 * g] + acc[4 * g + 1]) + (acc[4 * g + 2] + acc[4 * g + 3]);
    float v[4];
    for (int g = 0; g < 4; g++) v[g] = u[g] + u[g + 4];
    const float w0 = v[0] + v[2], w1 = v[1] + v[3];
    return w0 + w1;
}

namespace {

inline float l2sq(const float *__restrict a, const float *__restrict b, int d)
{
    return l2sq_canonical(a, b, d);
}

void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int)> &fn,
                  int64_t grain = 1)
{
    if (n <= 0) return;
    if (nthreads <= 1 || n <= grain) {
        for (int64_t i = 0; i < n; i++) fn(i, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    int nt = (int)std::min<int64_t>(nthreads, (n + grain - 1) / grain);
    for (int t = 0; t < nt; t++) {
        th.emplace_back([&, t] {
            for (;;) {
                int64_t s = next.fetch_add(grain);
                if (s >= n) break;
                int64_t e = std::min(n, s + grain);
                for (int64_t i = s; i < e; i++) fn(i, t);
            }
        });
    }
    for (auto &x : th) x.join();
}

struct Key {
    float f;   // capped attribute distance
    float d2;  // squared vector distance
    int32_t id;
};
inline bool key_lt(const Key &a, const Key &b)
{
    if (a.f != b.f) return a.f < b.f;
    if (a.d2 != b.d2) return a.d2 < b.d2;
    return a.id < b.id;
}

// dist_A(a_i, a_j) of an attribute kind (Section 3.1; App. D.3 for the
// frequency-weighted label distance), in FP32 as the device builder computes it.
float dist_a_host(const AttrView &A, const BuildPlan &P, int kind, int64_t i, int64_t j)
{
    if (kind == JAG_ATTR_SCALAR) return std::fabs((float)((int64_t)A.scalar[i] - (int64_t)A.scalar[j]));
    int64_t x = A.loff[i], xe = A.loff[i + 1], y = A.loff[j], ye = A.loff[j + 1];
    if (kind == JAG_ATTR_LABELS_WEIGHTED) {
        // C minus the weight of the shared labels (merge of the sorted rows)
        float shared = 0.f;
        while (x < xe && y < ye) {
            if (A.lab[x] == A.lab[y]) {
                shared += P.lw[(size_t)A.lab[x]];
                x++;
                y++;
            } else if (A.lab[x] < A.lab[y]) x++;
            else y++;
        }
        return P.lw_c - shared;
    }
    // |a_i XOR a_j| by merging the two sorted rows
    int64_t common = 0;
    while (x < xe && y < ye) {
        if (A.lab[x] == A.lab[y]) {
            common++;
            x++;
            y++;
        } else if (A.lab[x] < A.lab[y]) x++;
        else y++;
    }
    return (float)((A.loff[i + 1] - A.loff[i]) + (A.loff[j + 1] - A.loff[j]) - 2 * common);
}

// First component of entry ti's comparator for base point p and the squared
// distance d2 between them: Threshold-JAG, the capped dist_A (Section 3.2);
// Weight-JAG, w * dist_A + dist with one rounding of the product-sum (Section 3.4).
float first_host(const AttrView &A, const BuildPlan &P, int ti, int64_t p, int64_t v, float d2)
{
    const float t = P.thr[(size_t)p * P.nT + ti];
    const int kind = P.kinds[ti];
    if (kind & JAG_THRESHOLD_WEIGHT) return std::fma(t, dist_a_host(A, P, kind & 0xFF, p, v), std::sqrt(d2));
    if (std::isinf(t)) return 0.f;
    const float x = dist_a_host(A, P, kind, p, v) - t;
    return x > 0.f ? x : 0.f;
}

struct Builder {
    const float *X;
    int64_t n;
    int d;
    AttrView A;
    const BuildPlan *P;
    int R, lb, nT, cap, hopcap;
    float alpha2;
    std::vector<int32_t> adj;
    std::vector<int32_t> deg;

    float dist_a(int kind, int64_t i, int64_t j) const { return dist_a_host(A, *P, kind, i, j); }
    float first(int ti, int64_t p, int64_t v, float d2) const { return first_host(A, *P, ti, p, v, d2); }
    const float *row(int64_t i) const { return X + (size_t)i * d; }
};

struct Scratch {
    std::vector<uint32_t> seen;  // epoch stamps, size n
    uint32_t epoch = 0;
    std::vector<Key> L;
    std::vector<uint8_t> expanded;
    std::vector<int32_t> visited;
    std::vector<int32_t> cand;
    // prune scratch
    std::vector<float> pd2;
    std::vector<float> pf;
    std::vector<int32_t> order;
    std::vector<uint8_t> chosen_flag;
    std::vector<int32_t> bucket, chosen;
};

// GreedySearch(G, x_p, 1, l_b, D_A^t) over the frozen graph; appends the
// expanded vertices to s.visited.  A vertex seen earlier in this search is
// not re-evaluated: the beam always holds the l_b best vertices discovered,
// so one that fell out can never get back in.  At most hopcap = 4 l_b + 64
// expansions (a bound the searches stay far below; it sizes the device
// builder's candidate buffers).
void greedy_build_search(const Builder &B, Scratch &s, int64_t p, int ti)
{
    if (++s.epoch == 0) {
        std::fill(s.seen.begin(), s.seen.end(), 0u);
        s.epoch = 1;
    }
    const uint32_t ep = s.epoch;
    auto &L = s.L;
    auto &ex = s.expanded;
    L.clear();
    ex.clear();
    const float *xp = B.row(p);
    auto make = [&](int32_t u) {
        const float d2 = l2sq(xp, B.row(u), B.d);
        return Key{B.first(ti, p, u, d2), d2, u};
    };
    int32_t entry = B.P->entry;
    L.push_back(make(entry));
    ex.push_back(0);
    s.seen[entry] = ep;
    size_t hint = 0;
    int hops = 0;
    for (;;) {
        while (hint < L.size() && ex[hint]) hint++;
        if (hint >= L.size() || hops >= B.hopcap) break;
        hops++;
        size_t pi = hint;
        ex[pi] = 1;
        int32_t v = L[pi].id;
        s.visited.push_back(v);
        const int32_t *nb = &B.adj[(size_t)v * B.R];
        int dv = B.deg[v];
        size_t min_ins = L.size();
        for (int j = 0; j < dv; j++) {
            int32_t u = nb[j];
            if (s.seen[u] == ep) continue;
            s.seen[u] = ep;
            Key c = make(u);
            if ((int)L.size() >= B.lb && !key_lt(c, L.back())) continue;
            size_t pos = std::upper_bound(L.begin(), L.end(), c, key_lt) - L.begin();
            L.insert(L.begin() + pos, c);
            ex.insert(ex.begin() + pos, 0);
            if ((int)L.size() > B.lb) {
                L.pop_back();
                ex.pop_back();
            }
            if (pos < min_ins) min_ins = pos;
        }
        hint = std::min(min_ins, pi + 1);
    }
}

// JointRobustPrune(G, p, V, R, alpha, T) with the Appendix D.3 notes.
int prune(const Builder &B, Scratch &s, int64_t p, const int32_t *V, int nv, int32_t *out)
{
    const float *xp = B.row(p);
    auto &pd2 = s.pd2;
    auto &pf = s.pf;
    auto &order = s.order;
    auto &flag = s.chosen_flag;
    auto &bucket = s.bucket;
    auto &chosen = s.chosen;
    pd2.resize(nv);
    pf.resize(nv);
    order.resize(nv);
    flag.assign(nv, 0);
    chosen.clear();
    for (int j = 0; j < nv; j++) pd2[j] = l2sq(xp, B.row(V[j]), B.d);
    for (int ti = 0; ti < B.nT; ti++) {
        for (int j = 0; j < nv; j++) {
            pf[j] = B.first(ti, p, V[j], pd2[j]);
            order[j] = j;
        }
        std::sort(order.begin(), order.end(), [&](int a, int b) {
            if (pf[a] != pf[b]) return pf[a] < pf[b];
            if (pd2[a] != pd2[b]) return pd2[a] < pd2[b];
            return V[a] < V[b];
        });
        bucket.clear();
        for (int oi = 0; oi < nv; oi++) {
            int j = order[oi];
            bool keep = true;
            if (!flag[j]) {
                const float *xv = B.row(V[j]);
                for (int bj : bucket) {
                    if (!(B.alpha2 * l2sq(B.row(V[bj]), xv, B.d) > pd2[j])) {
                        keep = false;
                        break;
                    }
                }
            }
            if (keep) bucket.push_back(j);
            if ((int)bucket.size() >= B.cap) break;
        }
        for (int j : bucket) {
            if (!flag[j]) {
                flag[j] = 1;
                chosen.push_back(V[j]);
            }
        }
    }
    int m = std::min<int>((int)chosen.size(), B.R);
    std::copy(chosen.begin(), chosen.begin() + m, out);
    return m;
}

}  // namespace

int plan_build(const float *X, int64_t n, int32_t d, const AttrView &A, const BuildConfig &cfg,
               BuildPlan &P)
{
    P.R = cfg.R;
    P.lb = cfg.L_build > 0 ? cfg.L_build : 2 * cfg.R;
    P.nT = (int)cfg.kinds.size();
    P.cap = (9 * P.R + 10 * P.nT - 1) / (10 * P.nT);
    P.hopcap = 4 * P.lb + 64;
    P.alpha2 = cfg.alpha * cfg.alpha;
    P.kinds = cfg.kinds;
    P.max_batch = cfg.max_batch > 0 ? cfg.max_batch : std::max<int64_t>(64, n / 50);
    const int nth = cfg.n_threads > 0 ? cfg.n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    P.lw.clear();
    P.lw_c = 0.f;
    if (std::any_of(P.kinds.begin(), P.kinds.end(),
                    [](int32_t k) { return (k & 0xFF) == JAG_ATTR_LABELS_WEIGHTED; })) {
        // frequency-weighted label distance (App. D.3): weight log(1/p_l),
        // p_l = fraction of items holding l; C = the largest item total, summed
        // in FP32 in label order like the shared weights, so that no distance
        // falls below zero
        int32_t vocab = 1;
        for (int64_t x = 0; x < A.loff[n]; x++) vocab = std::max(vocab, A.lab[x] + 1);
        std::vector<double> cnt((size_t)vocab, 0.0);
        for (int64_t x = 0; x < A.loff[n]; x++) cnt[(size_t)A.lab[x]] += 1.0;
        P.lw.assign(cnt.size(), 0.f);
        for (size_t l = 0; l < cnt.size(); l++)
            P.lw[l] = cnt[l] > 0.0 ? (float)std::log((double)n / cnt[l]) : 0.f;
        float c = 0.f;
        for (int64_t i = 0; i < n; i++) {
            float t = 0.f;
            for (int64_t x = A.loff[i]; x < A.loff[i + 1]; x++) t += P.lw[(size_t)A.lab[x]];
            c = std::max(c, t);
        }
        P.lw_c = c;
    }

    if (cfg.order) {
        P.order.assign(cfg.order, cfg.order + n);
        P.entry = P.order[0];
    } else {
        // entry vertex: nearest to the FP64 centroid, smaller id on ties
        std::vector<double> cen(d, 0.0);
        for (int64_t i = 0; i < n; i++)
            for (int j = 0; j < d; j++) cen[j] += X[(size_t)i * d + j];
        for (int j = 0; j < d; j++) cen[j] /= (double)n;
        std::vector<double> best(nth, std::numeric_limits<double>::infinity());
        std::vector<int64_t> bid(nth, -1);
        int64_t chunk = (n + nth - 1) / nth;
        parallel_for(nth, nth, [&](int64_t t, int) {
            for (int64_t i = t * chunk; i < std::min(n, (t + 1) * chunk); i++) {
                double acc = 0.0;
                for (int j = 0; j < d; j++) {
                    double u = (double)X[(size_t)i * d + j] - cen[j];
                    acc += u * u;
                }
                if (acc < best[t]) {
                    best[t] = acc;
                    bid[t] = i;
                }
            }
        });
        int64_t e = 0;
        double be = std::numeric_limits<double>::infinity();
        for (int t = 0; t < nth; t++)
            if (bid[t] >= 0 && best[t] < be) {
                be = best[t];
                e = bid[t];
            }
        P.entry = (int32_t)e;
        // insertion order: entry first, then a seeded permutation
        P.order.clear();
        P.order.reserve(n);
        P.order.push_back(P.entry);
        for (int64_t i = 0; i < n; i++)
            if (i != P.entry) P.order.push_back((int32_t)i);
        uint64_t st = mix64(cfg.seed ^ 0xC0FFEEull);
        for (int64_t i = n - 1; i > 1; i--) {
            st = mix64(st);
            int64_t j = 1 + (int64_t)(st % (uint64_t)i);
            std::swap(P.order[i], P.order[j]);
        }
    }

    if (cfg.thresholds) {
        P.thr.assign(cfg.thresholds, cfg.thresholds + (size_t)n * P.nT);
        return 0;
    }
    // per-point thresholds: nearest-rank quantile of dist_A over 500 samples
    P.thr.assign((size_t)n * P.nT, 0.f);
    parallel_for(n, nth, [&](int64_t p, int) {
        float vals[500];
        const float *xp = X + (size_t)p * d;
        for (int ti = 0; ti < P.nT; ti++) {
            float q = cfg.quantiles[ti];
            float t;
            if (P.kinds[ti] & JAG_THRESHOLD_WEIGHT) {
                // Weight-JAG (App. D.3): h = sigma / sigma_A over the same
                // 500 sampled points; the weight is q * h
                uint64_t ctr = mix64(cfg.seed * 0x100000001B3ull + (uint64_t)p * 8 + ti);
                double s1 = 0, s2 = 0, a1 = 0, a2 = 0;
                int m = 0;
                for (int s = 0; s < 500 && n > 1; s++) {
                    int64_t v;
                    do {
                        ctr = mix64(ctr);
                        v = (int64_t)(ctr % (uint64_t)n);
                    } while (v == p);
                    double dv = std::sqrt((double)l2sq(xp, X + (size_t)v * d, d));
                    double da = dist_a_host(A, P, P.kinds[ti] & 0xFF, p, v);
                    s1 += dv;
                    s2 += dv * dv;
                    a1 += da;
                    a2 += da * da;
                    m++;
                }
                double sd = m ? std::sqrt(std::max(s2 / m - (s1 / m) * (s1 / m), 0.0)) : 0.0;
                double sa = m ? std::sqrt(std::max(a2 / m - (a1 / m) * (a1 / m), 0.0)) : 0.0;
                t = sa > 0.0 ? (float)(q * sd / sa) : 0.f;
            } else if (q >= 1.f) t = std::numeric_limits<float>::infinity();
            else if (q <= 0.f || n < 2) t = 0.f;
            else {
                uint64_t ctr = mix64(cfg.seed * 0x100000001B3ull + (uint64_t)p * 8 + ti);
                for (int s = 0; s < 500; s++) {
                    int64_t v;
                    do {
                        ctr = mix64(ctr);
                        v = (int64_t)(ctr % (uint64_t)n);
                    } while (v == p);
                    vals[s] = dist_a_host(A, P, P.kinds[ti], p, v);
                }
                int r = (int)std::ceil((double)q * 500.0);
                r = std::max(1, std::min(500, r));
                std::nth_element(vals, vals + (r - 1), vals + 500);
                t = vals[r - 1];
            }
            P.thr[(size_t)p * P.nT + ti] = t;
        }
    }, 256);
    return 0;
}

int build_graph(const float *X, int64_t n, int32_t d, const AttrView &A, const BuildConfig &cfg,
                std::vector<int32_t> &adj, int32_t &entry)
{
    BuildPlan plan;
    plan_build(X, n, d, A, cfg, plan);
    entry = plan.entry;
    Builder B;
    B.X = X;
    B.n = n;
    B.d = d;
    B.A = A;
    B.P = &plan;
    B.R = plan.R;
    B.lb = plan.lb;
    B.nT = plan.nT;
    B.cap = plan.cap;
    B.hopcap = plan.hopcap;
    B.alpha2 = plan.alpha2;
    const int nth = cfg.n_threads > 0 ? cfg.n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    const std::vector<int32_t> &order = plan.order;

    B.adj.assign((size_t)n * B.R, -1);
    B.deg.assign(n, 0);
    std::vector<Scratch> scr(nth);
    for (auto &s : scr) s.seen.assign(n, 0);
    const int64_t max_batch = plan.max_batch;
    std::vector<std::vector<int32_t>> newrow;
    int64_t pos = 1;  // order[0] = entry, inserted with no out-edges
    int64_t bs = 1;
    std::vector<std::pair<int32_t, int32_t>> rev;
    while (pos < n) {
        int64_t be = std::min<int64_t>(n, pos + bs);
        int64_t nb = be - pos;
        newrow.assign(nb, {});
        // phase 1: searches against the frozen graph and the new vertex's own prune
        parallel_for(nb, nth, [&](int64_t bi, int t) {
            Scratch &s = scr[t];
            int32_t p = order[pos + bi];
            s.visited.clear();
            for (int ti = 0; ti < B.nT; ti++) greedy_build_search(B, s, p, ti);
            // union of the expanded sets without p and without repeats
            std::sort(s.visited.begin(), s.visited.end());
            s.visited.erase(std::unique(s.visited.begin(), s.visited.end()), s.visited.end());
            s.visited.erase(std::remove(s.visited.begin(), s.visited.end(), p), s.visited.end());
            int32_t outbuf[kMaxR];
            int m = prune(B, s, p, s.visited.data(), (int)s.visited.size(), outbuf);
            newrow[bi].assign(outbuf, outbuf + m);
        });
        for (int64_t bi = 0; bi < nb; bi++) {
            int32_t p = order[pos + bi];
            auto &r = newrow[bi];
            std::copy(r.begin(), r.end(), &B.adj[(size_t)p * B.R]);
            B.deg[p] = (int32_t)r.size();
        }
        // phase 2: reverse edges grouped by target vertex
        rev.clear();
        for (int64_t bi = 0; bi < nb; bi++)
            for (int32_t v : newrow[bi]) rev.emplace_back(v, order[pos + bi]);
        std::sort(rev.begin(), rev.end());
        std::vector<int64_t> starts;
        for (size_t i = 0; i < rev.size(); i++)
            if (i == 0 || rev[i].first != rev[i - 1].first) starts.push_back((int64_t)i);
        starts.push_back((int64_t)rev.size());
        parallel_for((int64_t)starts.size() - 1, nth, [&](int64_t gi, int t) {
            Scratch &s = scr[t];
            int32_t v = rev[starts[gi]].first;
            int32_t *rv = &B.adj[(size_t)v * B.R];
            std::vector<int32_t> merged(rv, rv + B.deg[v]);
            for (int64_t i = starts[gi]; i < starts[gi + 1]; i++) {
                int32_t p = rev[i].second;
                if (std::find(merged.begin(), merged.end(), p) == merged.end()) merged.push_back(p);
            }
            if ((int)merged.size() <= B.R) {
                std::copy(merged.begin(), merged.end(), rv);
                B.deg[v] = (int32_t)merged.size();
            } else {
                int32_t outbuf[kMaxR];
                int m = prune(B, s, v, merged.data(), (int)merged.size(), outbuf);
                std::copy(outbuf, outbuf + m, rv);
                for (int j = m; j < B.R; j++) rv[j] = -1;
                B.deg[v] = m;
            }
        }, 16);
        if (cfg.progress && (pos * 10) / n != (be * 10) / n) {
            std::fprintf(stderr, "[build] %lld of %lld points inserted\n", (long long)be, (long long)n);
            std::fflush(stderr);
        }
        pos = be;
        bs = std::min<int64_t>(bs * 2, max_batch);
    }
    adj.swap(B.adj);
    return 0;
}

}  // namespace jag

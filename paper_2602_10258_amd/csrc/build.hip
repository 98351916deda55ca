// Threshold-/Weight-JAG construction with the insertion rounds on the GPU
// (paper Section 3.3, Algorithm 3's Insert and Algorithm 4's
// JointRobustPrune with the App. D.3 notes; Section 3.4 for weight entries).
//
// The rounds, comparators and tie rules are those of the host builder, and
// every floating-point value is formed in the same order (the canonical
// squared distance of l2sq_canonical, one fused multiply-add for a weight
// entry, FP32 sums of label weights in label order), so the two builders give
// the same graph edge for edge.  Per round of nb new points:
//
//   build_search_kernel  one wave per (new point, comparator entry): greedy
//                        search of the graph as it stood before the round,
//                        beam l_b, ordered by (first component, squared
//                        distance, id); writes the expanded vertices.
//   build_prune_kernel   one wave per new point: union of its expanded sets
//                        (sorted, duplicates dropped), JointRobustPrune into
//                        its out-row.
//   rev_count / rev_offset / rev_fill
//                        group the round's reverse edges by target vertex.
//   build_prune_kernel   (reverse mode) one wave per target vertex: its row
//                        plus its new in-links in id order, pruned again with
//                        its own thresholds when that exceeds R.
//
// A prune keeps its candidates in LDS when they number at most kMaxCand;
// the rare larger ones (a hub vertex gaining thousands of in-links in one
// round) run in a second launch with their arrays in global scratch.  Rows
// of more than 64 neighbours are read in slices of 64.
//
// The new points of a round cannot be reached from the graph before the
// round (nothing links to them yet), so their out-rows are written in place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "jag_internal.h"

namespace jag {
namespace {

constexpr int kSW = 4;               // search waves per workgroup
constexpr int kMaxLb = 256;          // largest build beam l_b
constexpr int kSeenSlots = 1024;     // lossy seen-table of a search wave
constexpr int kMaxCand = 4096;       // largest candidate set of one prune in LDS
constexpr int kMaxBigCand = 65536;   // largest in global memory (16-bit positions)
constexpr int kMaxOut = 136;         // chosen list of one prune (|T| * cap <= 0.9 R + |T|)
constexpr uint32_t kExp = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;

#define HIP_OK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            set_error("%s failed: %s", #x, hipGetErrorString(e_));                  \
            return e_ == hipErrorOutOfMemory ? JAG_ENOMEM : JAG_EDEVICE;            \
        }                                                                           \
    } while (0)

struct BArgs {
    const float *X;  // [n][d4], rows zero padded to a multiple of 4 floats
    int64_t n;
    int32_t d4;
    int32_t R, lb, nT, cap, hopcap;
    float alpha2;
    int32_t entry;
    int32_t kinds[8];
    const int32_t *scal;
    const int64_t *loff;
    const int32_t *lab;
    const float *lw;
    float lw_c;
    const float *thr;      // [n][nT]
    const int32_t *order;  // [n]
    int32_t *adj;          // [n][R], -1 padded
    int32_t *exp;          // [maxnb][nT][hopcap]
    int32_t *expcnt;       // [maxnb][nT]
    unsigned long long *ptot;  // [maxnb]: (finished searches << 32) | expanded total
    int32_t *incnt;        // [n] new in-links of a target in this round
    int32_t *fillpos;      // [n]
    int32_t *segoff;       // [n]
    int32_t *touched;      // [maxnb * R]
    int32_t *inl;          // [maxnb * R]
    int32_t *ctr;          // [0] targets, [1] in-link cursor, [2] largest in-count, [3] largest union,
                           // [4] insertions and [6] targets above lds_cap candidates, [5] scratch slots
    int32_t lds_cap;       // largest candidate set a prune keeps in LDS (kMaxCand)
};

__device__ __forceinline__ bool key_less(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

// Squared distances from row xa to the rows xb[0..3] in the canonical order:
// lane g of each group of eight takes elements 32m + 4g .. 32m + 4g + 3 into
// four partial sums; the partials fold as ((s0 + s1) + (s2 + s3)), then across
// the eight lanes at strides 4, 2, 1.  Every xb[k] must be a valid row (an
// unused slot points at row 0; its result is ignored); the shuffles run in
// every lane.
__device__ __forceinline__ void dist8x4(const float *__restrict xa, const float *const xb[4], int d4, int g,
                                        float out[4])
{
    float acc[4][4];
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int c = 0; c < 4; c++) acc[k][c] = 0.f;
    for (int e = 4 * g; e < d4; e += 32) {
        const float4 u = *reinterpret_cast<const float4 *>(xa + e);
        float4 v[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            v[k] = *reinterpret_cast<const float4 *>(xb[k] + e);  // inactive rows point at row 0
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const float t0 = u.x - v[k].x, t1 = u.y - v[k].y, t2 = u.z - v[k].z, t3 = u.w - v[k].w;
            acc[k][0] = __builtin_fmaf(t0, t0, acc[k][0]);
            acc[k][1] = __builtin_fmaf(t1, t1, acc[k][1]);
            acc[k][2] = __builtin_fmaf(t2, t2, acc[k][2]);
            acc[k][3] = __builtin_fmaf(t3, t3, acc[k][3]);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        float s = (acc[k][0] + acc[k][1]) + (acc[k][2] + acc[k][3]);
        s = s + __shfl_xor(s, 4);
        s = s + __shfl_xor(s, 2);
        s = s + __shfl_xor(s, 1);
        out[k] = s;
    }
}

// dist_A(a_i, a_j) (Section 3.1; App. D.3 for the weighted label distance).
__device__ float dist_a_dev(const BArgs &a, int kind, int64_t i, int64_t j)
{
    if (kind == JAG_ATTR_SCALAR) return fabsf((float)((long long)a.scal[i] - (long long)a.scal[j]));
    const int64_t x0 = a.loff[i], xe = a.loff[i + 1], y0 = a.loff[j], ye = a.loff[j + 1];
    int64_t x = x0, y = y0;
    if (kind == JAG_ATTR_LABELS_WEIGHTED) {
        float shared = 0.f;
        while (x < xe && y < ye) {
            const int32_t lx = a.lab[x], ly = a.lab[y];
            if (lx == ly) {
                shared = shared + a.lw[lx];
                x++;
                y++;
            } else if (lx < ly) x++;
            else y++;
        }
        return a.lw_c - shared;
    }
    long long common = 0;
    while (x < xe && y < ye) {
        const int32_t lx = a.lab[x], ly = a.lab[y];
        if (lx == ly) {
            common++;
            x++;
            y++;
        } else if (lx < ly) x++;
        else y++;
    }
    return (float)((xe - x0) + (ye - y0) - 2 * common);
}

// First component of a comparator entry for base point p: the capped dist_A
// (Section 3.2) or w * dist_A + dist (Section 3.4).
__device__ float first_dev(const BArgs &a, int kind, float t, int64_t p, int64_t v, float d2)
{
    if (kind & JAG_THRESHOLD_WEIGHT) return __builtin_fmaf(t, dist_a_dev(a, kind & 0xFF, p, v), __fsqrt_rn(d2));
    if (__builtin_isinf(t)) return 0.f;
    const float x = dist_a_dev(a, kind, p, v) - t;
    return x > 0.f ? x : 0.f;
}

__device__ __forceinline__ int seen_slot(int32_t u)
{
    return (int)(((uint32_t)u * 2654435761u) >> 22);  // 10 bits: kSeenSlots
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The prune's arrays live in LDS (GM = false) or, for candidate sets too
// large for LDS, in global scratch (GM = true), where the lanes of the wave
// exchange data through memory and order it with workgroup-scope fences.
template <bool GM>
__device__ __forceinline__ void wsync()
{
    if (GM) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        wave_sync();
    }
}

// Bytes of LDS one search wave uses.
__host__ __device__ constexpr int search_wave_bytes(int d4)
{
    return kMaxLb * 8 + kMaxLb * 4 + kSeenSlots * 4 + 64 * (8 + 4 + 4 + 4 + 4 + 4) + d4 * 4;
}

// GreedySearch(G, x_p, 1, l_b, D_A^t) of Algorithm 3: the beam holds the l_b
// best vertices discovered so far, sorted; the first unexpanded one is
// expanded next.  A lossy seen-table skips most repeats; a forgotten vertex
// is recognised in the beam by its (key, id), and one that fell out of the
// beam cannot get back in (its key is worse than the beam's last).
__global__ __launch_bounds__(256) void build_search_kernel(BArgs a, int64_t pos0, int32_t nb)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t task = (int64_t)blockIdx.x * kSW + wave;
    if (task >= (int64_t)nb * a.nT) return;
    const int bi = (int)(task / a.nT), ti = (int)(task % a.nT);
    const int64_t p = a.order[pos0 + bi];

    unsigned char *base = smem + (size_t)wave * search_wave_bytes(a.d4);
    uint64_t *lkey = reinterpret_cast<uint64_t *>(base);
    int32_t *lid = reinterpret_cast<int32_t *>(lkey + kMaxLb);
    int32_t *seen = lid + kMaxLb;
    uint64_t *ck = reinterpret_cast<uint64_t *>(seen + kSeenSlots);
    int32_t *cu = reinterpret_cast<int32_t *>(ck + 64);
    float *cf = reinterpret_cast<float *>(cu + 64);
    float *cd2 = cf + 64;
    int32_t *cid = reinterpret_cast<int32_t *>(cd2 + 64);
    int32_t *spos = cid + 64;
    float *xp = reinterpret_cast<float *>(spos + 64);

    for (int i = lane; i < kSeenSlots; i += 64) seen[i] = -1;
    const float *xrow = a.X + p * a.d4;
    for (int e = lane; e < a.d4; e += 64) xp[e] = xrow[e];
    wave_sync();

    const int kind = a.kinds[ti];
    const bool wgt = (kind & JAG_THRESHOLD_WEIGHT) != 0;
    const float t = a.thr[p * a.nT + ti];
    const int lb = a.lb;
    int32_t *expo = a.exp + task * a.hopcap;
    int nL = 0, hops = 0;
    int32_t v = -1;  // the vertex being expanded; -1 for the first step, whose candidate is the entry

    for (;;) {
        // rows wider than a wave go in slices of 64 neighbours, merged in turn
        for (int h = 0; h < (v < 0 ? 1 : a.R); h += 64) {
            const int32_t u = v < 0 ? (lane == 0 ? a.entry : -1)
                                    : (h + lane < a.R ? a.adj[(int64_t)v * a.R + h + lane] : -1);
            // ---- candidates: one neighbour per lane
            bool ok = u >= 0;
            if (ok) {
                const int s = seen_slot(u);
                if (seen[s] == u) ok = false;
                else seen[s] = u;
            }
            const bool full = nL == lb;
            const uint64_t wk = full ? lkey[lb - 1] : ~0ull;
            const int32_t wi = full ? (int32_t)((uint32_t)lid[lb - 1] & kIdMask) : 0x7FFFFFFF;
            float f = 0.f;
            if (ok && !wgt) {
                f = first_dev(a, kind, t, p, u, 0.f);
                if (full && __float_as_uint(f) > (uint32_t)(wk >> 32)) ok = false;  // cannot enter the beam
            }
            const uint64_t m = __ballot(ok);
            const int nc = __popcll(m);
            if (nc > 0) {
                const int ci = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                if (ok) {
                    cu[ci] = u;
                    cf[ci] = f;
                }
                wave_sync();
                for (int c0 = 0; c0 < nc; c0 += 32) {
                    const float *xb[4];
                    bool act[4];
                    int cc[4];
    #pragma unroll
                    for (int k = 0; k < 4; k++) {
                        cc[k] = c0 + k * 8 + (lane >> 3);
                        act[k] = cc[k] < nc;
                        xb[k] = a.X + (int64_t)(act[k] ? cu[cc[k]] : 0) * a.d4;
                    }
                    float d2[4];
                    dist8x4(xp, xb, a.d4, lane & 7, d2);
    #pragma unroll
                    for (int k = 0; k < 4; k++)
                        if (act[k] && (lane & 7) == 0) cd2[cc[k]] = d2[k];
                }
                wave_sync();
                // ---- one lane per candidate: key, beam test, repeat test
                bool ok2 = lane < nc;
                uint64_t key = 0;
                int32_t id = 0;
                int lbp = 0;
                if (ok2) {
                    id = cu[lane];
                    const float d2 = cd2[lane];
                    const float ff = wgt ? first_dev(a, kind, t, p, id, d2) : cf[lane];
                    key = ((uint64_t)__float_as_uint(ff) << 32) | __float_as_uint(d2);
                    if (full && !key_less(key, id, wk, wi)) ok2 = false;
                    else {
                        int lo = 0, hi = nL;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (key_less(lkey[mid], (int32_t)((uint32_t)lid[mid] & kIdMask), key, id)) lo = mid + 1;
                            else hi = mid;
                        }
                        lbp = lo;
                        if (lo < nL && lkey[lo] == key && (int32_t)((uint32_t)lid[lo] & kIdMask) == id) ok2 = false;
                    }
                }
                const uint64_t m2 = __ballot(ok2);
                const int nc2 = __popcll(m2);
                if (nc2 > 0) {
                    const int c2 = __builtin_amdgcn_mbcnt_hi((uint32_t)(m2 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m2, 0));
                    if (ok2) {
                        ck[c2] = key;
                        cid[c2] = id;
                    }
                    wave_sync();
                    int rank = 0;
                    if (ok2)
                        for (int j = 0; j < nc2; j++) rank += key_less(ck[j], cid[j], key, id) ? 1 : 0;
                    if (ok2) spos[rank] = lbp;  // beam positions of the candidates in key order
                    // beam entries into registers before anything moves
                    uint64_t ek[kMaxLb / 64];
                    int32_t ei[kMaxLb / 64];
    #pragma unroll
                    for (int r = 0; r < kMaxLb / 64; r++) {
                        const int i = r * 64 + lane;
                        if (i < nL) {
                            ek[r] = lkey[i];
                            ei[r] = lid[i];
                        }
                    }
                    wave_sync();
    #pragma unroll
                    for (int r = 0; r < kMaxLb / 64; r++) {
                        const int i = r * 64 + lane;
                        if (i < nL) {
                            // candidates before entry i: those whose beam position is <= i
                            int lo = 0, hi = nc2;
                            while (lo < hi) {
                                const int mid = (lo + hi) >> 1;
                                if (spos[mid] <= i) lo = mid + 1;
                                else hi = mid;
                            }
                            const int np = i + lo;
                            if (np < lb) {
                                lkey[np] = ek[r];
                                lid[np] = ei[r];
                            }
                        }
                    }
                    if (ok2) {
                        const int np = lbp + rank;
                        if (np < lb) {
                            lkey[np] = key;
                            lid[np] = id;
                        }
                    }
                    nL = min(lb, nL + nc2);
                    wave_sync();
                }
            }
        }
        // ---- the first unexpanded entry of the beam
        int pi = -1;
        for (int c0 = 0; c0 < nL; c0 += 64) {
            const int i = c0 + lane;
            const bool un = i < nL && !((uint32_t)lid[i] & kExp);
            const uint64_t mm = __ballot(un);
            if (mm) {
                pi = c0 + __ffsll((long long)mm) - 1;
                break;
            }
        }
        if (pi < 0 || hops >= a.hopcap) break;
        v = (int32_t)((uint32_t)lid[pi] & kIdMask);
        wave_sync();
        if (lane == 0) {
            lid[pi] = (int32_t)((uint32_t)v | kExp);
            expo[hops] = v;
        }
        hops++;
        wave_sync();
    }
    if (lane == 0) {
        a.expcnt[task] = hops;
        const unsigned long long old = atomicAdd(&a.ptot[bi], (1ull << 32) + (unsigned long long)hops);
        if ((int)(old >> 32) == a.nT - 1) {
            const int32_t total = (int32_t)(old & 0xFFFFFFFFull) + hops;
            atomicMax(&a.ctr[3], total);
            if (total > a.lds_cap) atomicAdd(&a.ctr[4], 1);  // prunes for the global-memory pass
        }
    }
}

// Bytes of LDS one prune wave uses for P candidate slots and memf floats of
// member rows.
__host__ __device__ constexpr int prune_wave_bytes(int P, int memf)
{
    return memf * 4 + P * (4 + 4 + 4 + 2 + 1) + kMaxOut * 4 + 128 * 4 + 16;
}

// Ascending bitonic sort of ids (P a power of two, padded with INT_MAX).
template <bool GM>
__device__ void sort_ids(int32_t *x, int P, int lane)
{
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < P; i += 64) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t xi = x[i], xl = x[l];
                    const bool up = (i & k) == 0;
                    if ((xi > xl) == up) {
                        x[i] = xl;
                        x[l] = xi;
                    }
                }
            }
            wsync<GM>();
        }
}

// Drop INT_MAX padding and repeats from sorted x[0..P); returns the count.
template <bool GM>
__device__ int unique_ids(int32_t *x, int P, int lane)
{
    int out = 0;
    int32_t prev_last = (int32_t)0x80000000;
    for (int c0 = 0; c0 < P; c0 += 64) {
        const int i = c0 + lane;
        const int32_t xi = i < P ? x[i] : 0x7FFFFFFF;
        int32_t prev = __shfl_up(xi, 1);
        if (lane == 0) prev = prev_last;
        const bool keep = xi != 0x7FFFFFFF && xi != prev;
        prev_last = __shfl(xi, 63);
        const uint64_t m = __ballot(keep);
        const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
        wsync<GM>();
        if (keep) x[out + r] = xi;
        out += __popcll(m);
        wsync<GM>();
    }
    return out;
}

// Squared distance between the candidate row a group of eight lanes holds
// in registers (lane g: elements 32c + 4g .. +3) and a row at m, folded in the
// canonical order (as dist8x4).
template <int CH>
__device__ __forceinline__ float dist_reg(const float4 (&r)[CH], const float *__restrict m, int d4, int g)
{
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int c = 0; c < CH; c++) {
        const int e = 32 * c + 4 * g;
        if (e < d4) {
            const float4 u = *reinterpret_cast<const float4 *>(m + e);
            const float t0 = u.x - r[c].x, t1 = u.y - r[c].y, t2 = u.z - r[c].z, t3 = u.w - r[c].w;
            a0 = __builtin_fmaf(t0, t0, a0);
            a1 = __builtin_fmaf(t1, t1, a1);
            a2 = __builtin_fmaf(t2, t2, a2);
            a3 = __builtin_fmaf(t3, t3, a3);
        }
    }
    float s = (a0 + a1) + (a2 + a3);
    s = s + __shfl_xor(s, 4);
    s = s + __shfl_xor(s, 2);
    s = s + __shfl_xor(s, 1);
    return s;
}

// JointRobustPrune(G, v, V, R, alpha, T) with the App. D.3 notes over the
// sorted distinct ids V[0..nv): per comparator entry, candidates in order of
// (first component, squared distance, id); one chosen by an earlier entry
// joins without the alpha test; the others join when alpha^2 d^2(u, c) >
// d^2(v, c) for every member u already in the bucket; the bucket closes at
// cap members.  The ordered list is walked in chunks of 8U candidates whose
// rows are loaded once into registers (group g of eight lanes holds the
// candidates at chunk positions 8k + g); each is tested against the members
// accepted before the chunk, then the chunk is decided in list order, every
// member it accepts being tested against the candidates after it.  Member rows
// sit in LDS (mem) when they fit, else they are read from X.  Writes the
// first R chosen ids into v's row.
template <int CH, int U, bool GM>
__device__ void prune_core(const BArgs &a, int64_t v, int32_t *V, int nv, float *pd2, float *fst,
                           uint16_t *ord, uint8_t *flg, int32_t *outl, int32_t *mid, float *mem, int lane)
{
    const int g = lane & 7, grp = lane >> 3;
    const float *xv = a.X + v * a.d4;
    for (int c0 = 0; c0 < nv; c0 += 32) {
        const float *xb[4];
        int cc[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            cc[k] = c0 + k * 8 + grp;
            xb[k] = a.X + (int64_t)(cc[k] < nv ? V[cc[k]] : 0) * a.d4;
        }
        float d2[4];
        dist8x4(xv, xb, a.d4, g, d2);
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (cc[k] < nv && g == 0) pd2[cc[k]] = d2[k];
    }
    for (int j = lane; j < nv; j += 64) flg[j] = 0;
    wsync<GM>();
    int nout = 0;
    for (int ti = 0; ti < a.nT; ti++) {
        const int kind = a.kinds[ti];
        const float t = a.thr[v * a.nT + ti];
        for (int j = lane; j < nv; j += 64) fst[j] = first_dev(a, kind, t, v, V[j], pd2[j]);
        int P2 = 64;
        while (P2 < nv) P2 <<= 1;
        for (int j = lane; j < P2; j += 64) ord[j] = (uint16_t)j;
        wsync<GM>();
        // bitonic sort of positions by (first, d2, id); positions >= nv last
        for (int k = 2; k <= P2; k <<= 1)
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int i = lane; i < P2; i += 64) {
                    const int l = i ^ jj;
                    if (l > i) {
                        const int oi = ord[i], ol = ord[l];
                        bool gt;  // entry at i after entry at l
                        if (oi >= nv || ol >= nv) gt = oi >= nv && (ol < nv || oi > ol);
                        else {
                            const float fi = fst[oi], fl = fst[ol];
                            if (fi != fl) gt = fi > fl;
                            else {
                                const float di = pd2[oi], dl = pd2[ol];
                                gt = di != dl ? di > dl : oi > ol;
                            }
                        }
                        const bool up = (i & k) == 0;
                        if (gt == up) {
                            ord[i] = (uint16_t)ol;
                            ord[l] = (uint16_t)oi;
                        }
                    }
                }
                wsync<GM>();
            }
        int nm = 0;  // members of this bucket
        for (int c0 = 0; c0 < nv && nm < a.cap; c0 += 8 * U) {
            float4 row[U][CH];
            int oc[U];
            bool in[U], fl[U], alive[U];
#pragma unroll
            for (int k = 0; k < U; k++) {
                const int q = c0 + 8 * k + grp;
                in[k] = q < nv;
                oc[k] = in[k] ? ord[q] : 0;
                fl[k] = in[k] && (flg[oc[k]] & 1);
                alive[k] = in[k];
                const float *src = a.X + (int64_t)(in[k] ? V[oc[k]] : 0) * a.d4;
#pragma unroll
                for (int c = 0; c < CH; c++) {
                    const int e = 32 * c + 4 * g;
                    row[k][c] = e < a.d4 ? *reinterpret_cast<const float4 *>(src + e) : float4{0.f, 0.f, 0.f, 0.f};
                }
            }
            // the members accepted before this chunk
            for (int j = 0; j < nm; j++) {
                bool any = false;
#pragma unroll
                for (int k = 0; k < U; k++) any = any || (alive[k] && !fl[k]);
                if (!__ballot(any)) break;
                const float *mrow = mem ? mem + (size_t)j * a.d4 : a.X + (int64_t)mid[j] * a.d4;
#pragma unroll
                for (int k = 0; k < U; k++) {
                    const float d2 = dist_reg<CH>(row[k], mrow, a.d4, g);
                    if (alive[k] && !fl[k] && !(a.alpha2 * d2 > pd2[oc[k]])) alive[k] = false;
                }
            }
            // decide the chunk in list order
#pragma unroll
            for (int k = 0; k < U; k++) {
                for (int gg = 0; gg < 8; gg++) {
                    const bool take = __shfl((int)(alive[k] || fl[k]), 8 * gg) != 0;
                    if (!take) continue;
                    const int o = __shfl(oc[k], 8 * gg);
                    if (!(flg[o] & 1)) {
                        if (lane == 0) {
                            flg[o] = 1;
                            if (nout < kMaxOut) outl[nout] = V[o];
                        }
                        nout++;
                    }
                    if (lane == 0) mid[nm] = V[o];
                    if (mem && grp == gg) {
#pragma unroll
                        for (int c = 0; c < CH; c++) {
                            const int e = 32 * c + 4 * g;
                            if (e < a.d4) *reinterpret_cast<float4 *>(mem + (size_t)nm * a.d4 + e) = row[k][c];
                        }
                    }
                    nm++;
                    wsync<GM>();
                    if (nm >= a.cap) break;
                    // the candidates after it in this chunk meet the new member
                    const float *mrow = mem ? mem + (size_t)(nm - 1) * a.d4 : a.X + (int64_t)V[o] * a.d4;
#pragma unroll
                    for (int k2 = 0; k2 < U; k2++) {
                        if (k2 < k) continue;
                        const float d2 = dist_reg<CH>(row[k2], mrow, a.d4, g);
                        const bool later = k2 > k || grp > gg;
                        if (later && alive[k2] && !fl[k2] && !(a.alpha2 * d2 > pd2[oc[k2]])) alive[k2] = false;
                    }
                }
                if (nm >= a.cap) break;
            }
        }
        wsync<GM>();
    }
    const int m = min(nout, a.R);
    int32_t *row = a.adj + v * a.R;
    for (int j = lane; j < a.R; j += 64) row[j] = j < m ? outl[j] : -1;
}

// Mode 0: prune the union of a new point's expanded sets into its row.
// Mode 1: merge a target's new in-links into its row (re-pruned above R).
// GM = false: prunes of at most lds_cap candidates, arrays in LDS (P slots,
// memf floats of member rows); blocks with larger candidate sets return at
// once.  GM = true: only those larger prunes, each with P slots in its own
// gbytes of global scratch (slots handed out by ctr[5]) and member rows read
// from X.  The two passes together prune every block exactly once.
template <int CH, int U, bool GM>
__global__ __launch_bounds__(64) void build_prune_kernel(BArgs a, int64_t pos0, int32_t mode, int32_t P,
                                                         int32_t memf, unsigned char *gs, int64_t gbytes)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    bool big;
    if (mode == 0) {
        int tot = 0;
        for (int ti = 0; ti < a.nT; ti++) tot += a.expcnt[(int64_t)blockIdx.x * a.nT + ti];
        big = tot > a.lds_cap;
    } else {
        big = a.incnt[a.touched[blockIdx.x]] + a.R > a.lds_cap;
    }
    if (big != GM) return;
    unsigned char *base = smem;
    if (GM) {
        int slot = 0;
        if (lane == 0) slot = atomicAdd(&a.ctr[5], 1);
        slot = __shfl(slot, 0);
        base = gs + (size_t)slot * (size_t)gbytes;
    }
    float *mem = memf > 0 ? reinterpret_cast<float *>(base) : nullptr;
    int32_t *V = reinterpret_cast<int32_t *>(base + (size_t)memf * 4);
    float *pd2 = reinterpret_cast<float *>(V + P);
    float *fst = pd2 + P;
    int32_t *outl = reinterpret_cast<int32_t *>(fst + P);
    int32_t *mid = outl + kMaxOut;
    uint16_t *ord = reinterpret_cast<uint16_t *>(mid + 128);
    uint8_t *flg = reinterpret_cast<uint8_t *>(ord + P);

    if (mode == 0) {
        const int bi = blockIdx.x;
        const int64_t p = a.order[pos0 + bi];
        int tot = 0;
        for (int ti = 0; ti < a.nT; ti++) {
            const int c = a.expcnt[(int64_t)bi * a.nT + ti];
            const int32_t *src = a.exp + ((int64_t)bi * a.nT + ti) * a.hopcap;
            for (int j = lane; j < c; j += 64) V[tot + j] = src[j] == p ? 0x7FFFFFFF : src[j];
            tot += c;
        }
        int P2 = 64;
        while (P2 < tot) P2 <<= 1;
        for (int j = tot + lane; j < P2; j += 64) V[j] = 0x7FFFFFFF;
        wsync<GM>();
        sort_ids<GM>(V, P2, lane);
        const int nv = unique_ids<GM>(V, P2, lane);
        prune_core<CH, U, GM>(a, p, V, nv, pd2, fst, ord, flg, outl, mid, mem, lane);
        return;
    }
    const int64_t v = a.touched[blockIdx.x];
    const int cnt = a.incnt[v];
    const int32_t *src = a.inl + a.segoff[v];
    int32_t *row = a.adj + v * a.R;
    int deg = 0;
    for (int c0 = 0; c0 < a.R; c0 += 64) {
        const int j = c0 + lane;
        deg += __popcll(__ballot(j < a.R && row[j] >= 0));
    }
    int P2 = 64;
    while (P2 < cnt) P2 <<= 1;
    for (int j = lane; j < P2; j += 64) V[j] = j < cnt ? src[j] : 0x7FFFFFFF;
    wsync<GM>();
    sort_ids<GM>(V, P2, lane);
    // in-links not already in the row, in id order
    int nnew = 0;
    for (int c0 = 0; c0 < cnt; c0 += 64) {
        const int j = c0 + lane;
        bool fresh = j < cnt;
        const int32_t x = fresh ? V[j] : 0;
        for (int r = 0; r < deg && fresh; r++)
            if (row[r] == x) fresh = false;
        const uint64_t m = __ballot(fresh);
        const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
        wsync<GM>();
        if (fresh) V[nnew + r] = x;
        nnew += __popcll(m);
        wsync<GM>();
    }
    if (deg + nnew <= a.R) {
        for (int j = lane; j < nnew; j += 64) row[deg + j] = V[j];
    } else {
        // the row and the new in-links, sorted and distinct, pruned with v's thresholds
        for (int j = lane; j < deg; j += 64) V[nnew + j] = row[j];
        const int tot = nnew + deg;
        int P3 = 64;
        while (P3 < tot) P3 <<= 1;
        for (int j = tot + lane; j < P3; j += 64) V[j] = 0x7FFFFFFF;
        wsync<GM>();
        sort_ids<GM>(V, P3, lane);
        const int nv = unique_ids<GM>(V, P3, lane);
        prune_core<CH, U, GM>(a, v, V, nv, pd2, fst, ord, flg, outl, mid, mem, lane);
    }
    if (lane == 0) {
        a.incnt[v] = 0;
        a.fillpos[v] = 0;
    }
}

// Reverse edges of the round: count per target, list the targets.
__global__ void rev_count_kernel(BArgs a, int64_t pos0, int32_t nb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nb * a.R) return;
    const int64_t p = a.order[pos0 + t / a.R];
    const int32_t v = a.adj[p * a.R + t % a.R];
    if (v < 0) return;
    if (atomicAdd(&a.incnt[v], 1) == 0) a.touched[atomicAdd(&a.ctr[0], 1)] = v;
}

// Segment of each target in the in-link buffer; the largest in-count.
__global__ void rev_offset_kernel(BArgs a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int nt = a.ctr[0];
    const int c = t < nt ? a.incnt[a.touched[t]] : 0;
    int incl = c;  // inclusive prefix sum over the wave
    for (int s = 1; s < 64; s <<= 1) {
        const int y = __shfl_up(incl, s);
        if (lane >= s) incl += y;
    }
    int mx = c;
    for (int s = 32; s > 0; s >>= 1) mx = max(mx, __shfl_xor(mx, s));
    int base = 0;
    if (lane == 63) base = atomicAdd(&a.ctr[1], incl);
    base = __shfl(base, 63);
    if (t < nt) a.segoff[a.touched[t]] = base + incl - c;
    if (lane == 0) atomicMax(&a.ctr[2], mx);
    const uint64_t big = __ballot(t < nt && c + a.R > a.lds_cap);  // prunes for the global-memory pass
    if (lane == 0 && big) atomicAdd(&a.ctr[6], (int)__popcll(big));
}

__global__ void rev_fill_kernel(BArgs a, int64_t pos0, int32_t nb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nb * a.R) return;
    const int64_t p = a.order[pos0 + t / a.R];
    const int32_t v = a.adj[p * a.R + t % a.R];
    if (v < 0) return;
    a.inl[a.segoff[v] + atomicAdd(&a.fillpos[v], 1)] = (int32_t)p;
}

struct DevBufs {
    std::vector<void *> ptrs;
    ~DevBufs()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t alloc(T **out, size_t count)
    {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) {
            ptrs.push_back(p);
            *out = static_cast<T *>(p);
        }
        return e;
    }
};

template <bool GM>
void launch_prune_kind(const BArgs &a, dim3 gr, size_t lds, int64_t pos, int32_t mode, int32_t P, int32_t memf,
                       unsigned char *gs, int64_t gbytes)
{
    const dim3 bl(64);
    // a candidate row takes ceil(d4 / 32) float4 per lane; four candidates per
    // group of eight lanes up to d4 = 128, one above
    if (a.d4 <= 64)
        hipLaunchKernelGGL((build_prune_kernel<2, 4, GM>), gr, bl, lds, 0, a, pos, mode, P, memf, gs, gbytes);
    else if (a.d4 <= 96)
        hipLaunchKernelGGL((build_prune_kernel<3, 4, GM>), gr, bl, lds, 0, a, pos, mode, P, memf, gs, gbytes);
    else if (a.d4 <= 128)
        hipLaunchKernelGGL((build_prune_kernel<4, 4, GM>), gr, bl, lds, 0, a, pos, mode, P, memf, gs, gbytes);
    else
        hipLaunchKernelGGL((build_prune_kernel<16, 1, GM>), gr, bl, lds, 0, a, pos, mode, P, memf, gs, gbytes);
}

// The LDS pass over all blocks (prunes of up to lds_cap candidates, P slots;
// member rows go to LDS when the wave's LDS stays within 64 KB).
hipError_t launch_prune(const BArgs &a, int32_t grid, int64_t pos, int32_t mode, int32_t P)
{
    const int memf = prune_wave_bytes(P, a.cap * a.d4) <= 65536 ? a.cap * a.d4 : 0;
    launch_prune_kind<false>(a, dim3((unsigned)grid), (size_t)prune_wave_bytes(P, memf), pos, mode, P, memf,
                             nullptr, 0);
    return hipGetLastError();
}

// The global-memory pass over the same blocks for the nbig larger prunes of
// up to Pbig candidates; the scratch buffer grows to hold them.
jag_status launch_prune_big(const BArgs &a, DevBufs &B, unsigned char *&gs, size_t &gs_bytes, int32_t grid,
                            int64_t pos, int32_t mode, int32_t Pbig, int32_t nbig)
{
    const int64_t gbytes = ((int64_t)prune_wave_bytes(Pbig, 0) + 255) / 256 * 256;
    const size_t need = (size_t)gbytes * (size_t)nbig;
    if (need > gs_bytes) {
        unsigned char *p = nullptr;
        HIP_OK(B.alloc(&p, need));
        gs = p;  // the smaller buffer stays with B until the build ends
        gs_bytes = need;
    }
    HIP_OK(hipMemset(a.ctr + 5, 0, 4));
    launch_prune_kind<true>(a, dim3((unsigned)grid), 0, pos, mode, Pbig, 0, gs, gbytes);
    HIP_OK(hipGetLastError());
    return JAG_OK;
}

int pow2_at_least(int x)
{
    int p = 64;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

jag_status build_graph_device(const float *X, int64_t n, int32_t d, const AttrView &A,
                              const BuildConfig &cfg, std::vector<int32_t> &adj, int32_t &entry)
{
    BuildPlan plan;
    plan_build(X, n, d, A, cfg, plan);
    entry = plan.entry;
    if (plan.lb > kMaxLb) {
        set_error("the device builder takes L_build <= %d (got %d)", kMaxLb, plan.lb);
        return JAG_EINVAL;
    }
    if (n >= (int64_t)0x7FFFFFFF) {
        set_error("the device builder takes n < 2^31");
        return JAG_EINVAL;
    }
    const int d4 = (d + 3) / 4 * 4;
    const int R = plan.R, nT = plan.nT;
    const int64_t maxnb = std::min<int64_t>(plan.max_batch, std::max<int64_t>(n - 1, 1));

    DevBufs B;
    BArgs a{};
    float *dX;
    int32_t *dscal = nullptr, *dlab = nullptr;
    int64_t *dloff = nullptr;
    float *dlw = nullptr;
    float *dthr;
    int32_t *dorder, *dadj, *dexp, *dexpcnt, *dincnt, *dfill, *dseg, *dtouch, *dinl, *dctr;
    unsigned long long *dptot;
    HIP_OK(B.alloc(&dX, (size_t)n * d4));
    if (d4 == d) {
        HIP_OK(hipMemcpy(dX, X, (size_t)n * d * sizeof(float), hipMemcpyHostToDevice));
    } else {
        // one contiguous copy of rows padded on the host (a pitched copy from
        // pageable memory goes row by row)
        std::vector<float> pad((size_t)n * d4, 0.f);
        for (int64_t i = 0; i < n; i++) std::copy(X + i * d, X + (i + 1) * d, pad.begin() + i * d4);
        HIP_OK(hipMemcpy(dX, pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    if (A.scalar) {
        HIP_OK(B.alloc(&dscal, (size_t)n));
        HIP_OK(hipMemcpy(dscal, A.scalar, (size_t)n * 4, hipMemcpyHostToDevice));
    }
    if (A.loff) {
        const int64_t nnz = A.loff[n];
        HIP_OK(B.alloc(&dloff, (size_t)n + 1));
        HIP_OK(hipMemcpy(dloff, A.loff, (size_t)(n + 1) * 8, hipMemcpyHostToDevice));
        HIP_OK(B.alloc(&dlab, (size_t)nnz));
        if (nnz > 0) HIP_OK(hipMemcpy(dlab, A.lab, (size_t)nnz * 4, hipMemcpyHostToDevice));
    }
    if (!plan.lw.empty()) {
        HIP_OK(B.alloc(&dlw, plan.lw.size()));
        HIP_OK(hipMemcpy(dlw, plan.lw.data(), plan.lw.size() * 4, hipMemcpyHostToDevice));
    }
    HIP_OK(B.alloc(&dthr, (size_t)n * nT));
    HIP_OK(hipMemcpy(dthr, plan.thr.data(), (size_t)n * nT * 4, hipMemcpyHostToDevice));
    HIP_OK(B.alloc(&dorder, (size_t)n));
    HIP_OK(hipMemcpy(dorder, plan.order.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    HIP_OK(B.alloc(&dadj, (size_t)n * R));
    HIP_OK(hipMemset(dadj, 0xFF, (size_t)n * R * 4));
    HIP_OK(B.alloc(&dexp, (size_t)maxnb * nT * plan.hopcap));
    HIP_OK(B.alloc(&dexpcnt, (size_t)maxnb * nT));
    HIP_OK(B.alloc(&dptot, (size_t)maxnb));
    HIP_OK(B.alloc(&dincnt, (size_t)n));
    HIP_OK(B.alloc(&dfill, (size_t)n));
    HIP_OK(B.alloc(&dseg, (size_t)n));
    HIP_OK(hipMemset(dincnt, 0, (size_t)n * 4));
    HIP_OK(hipMemset(dfill, 0, (size_t)n * 4));
    HIP_OK(B.alloc(&dtouch, (size_t)maxnb * R));
    HIP_OK(B.alloc(&dinl, (size_t)maxnb * R));
    HIP_OK(B.alloc(&dctr, 8));
    unsigned char *gscratch = nullptr;  // global-memory prunes, grown on demand
    size_t gscratch_bytes = 0;

    a.X = dX;
    a.n = n;
    a.d4 = d4;
    a.R = R;
    a.lb = plan.lb;
    a.nT = nT;
    a.cap = plan.cap;
    a.hopcap = plan.hopcap;
    a.alpha2 = plan.alpha2;
    a.entry = plan.entry;
    for (int i = 0; i < nT; i++) a.kinds[i] = plan.kinds[i];
    a.scal = dscal;
    a.loff = dloff;
    a.lab = dlab;
    a.lw = dlw;
    a.lw_c = plan.lw_c;
    a.thr = dthr;
    a.order = dorder;
    a.adj = dadj;
    a.exp = dexp;
    a.expcnt = dexpcnt;
    a.ptot = dptot;
    a.incnt = dincnt;
    a.fillpos = dfill;
    a.segoff = dseg;
    a.touched = dtouch;
    a.inl = dinl;
    a.ctr = dctr;
    // JAG_BUILD_LDS_CANDIDATES (64..4096) lowers the LDS capacity of a prune,
    // which sends more prunes through the global-memory pass (for testing it)
    a.lds_cap = kMaxCand;
    if (const char *e = std::getenv("JAG_BUILD_LDS_CANDIDATES")) {
        const int v = std::atoi(e);
        if (v >= 64 && v <= kMaxCand) a.lds_cap = v;
    }

    const int search_lds = kSW * search_wave_bytes(d4);
    int64_t pos = 1, bs = 1;
    while (pos < n) {
        const int64_t be = std::min<int64_t>(n, pos + bs);
        const int32_t nb = (int32_t)(be - pos);
        int32_t hctr[8];
        HIP_OK(hipMemset(dctr, 0, 32));
        HIP_OK(hipMemset(dptot, 0, (size_t)nb * 8));
        const int64_t waves = (int64_t)nb * nT;
        hipLaunchKernelGGL(build_search_kernel, dim3((unsigned)((waves + kSW - 1) / kSW)), dim3(64 * kSW),
                           search_lds, 0, a, pos, nb);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpy(hctr, dctr, 32, hipMemcpyDeviceToHost));
        if (hctr[3] > kMaxBigCand) {
            set_error("an insertion expanded %d vertices in all; the device builder holds %d", hctr[3], kMaxBigCand);
            return JAG_EUNSUPPORTED;
        }
        HIP_OK(launch_prune(a, nb, pos, 0, pow2_at_least(std::min(hctr[3], a.lds_cap))));
        if (hctr[4] > 0) {
            jag_status st = launch_prune_big(a, B, gscratch, gscratch_bytes, nb, pos, 0, pow2_at_least(hctr[3]),
                                             hctr[4]);
            if (st != JAG_OK) return st;
        }
        const unsigned eb = (unsigned)(((int64_t)nb * R + 255) / 256);
        hipLaunchKernelGGL(rev_count_kernel, dim3(eb), dim3(256), 0, 0, a, pos, nb);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(rev_offset_kernel, dim3(eb), dim3(256), 0, 0, a);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(rev_fill_kernel, dim3(eb), dim3(256), 0, 0, a, pos, nb);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpy(hctr, dctr, 32, hipMemcpyDeviceToHost));
        if (hctr[0] > 0) {
            if (hctr[2] + R > kMaxBigCand) {
                set_error("a vertex gained %d in-links in one round; the device builder holds %d (lower max_batch)",
                          hctr[2], kMaxBigCand - R);
                return JAG_EUNSUPPORTED;
            }
            HIP_OK(launch_prune(a, hctr[0], pos, 1, pow2_at_least(std::min(hctr[2] + R, a.lds_cap))));
            if (hctr[6] > 0) {
                jag_status st = launch_prune_big(a, B, gscratch, gscratch_bytes, hctr[0], pos, 1,
                                                 pow2_at_least(hctr[2] + R), hctr[6]);
                if (st != JAG_OK) return st;
            }
        }
        if (cfg.progress && (pos * 10) / n != (be * 10) / n) {
            HIP_OK(hipDeviceSynchronize());
            std::fprintf(stderr, "[build] %lld of %lld points inserted (GPU)\n", (long long)be, (long long)n);
            std::fflush(stderr);
        }
        pos = be;
        bs = std::min<int64_t>(bs * 2, plan.max_batch);
    }
    adj.assign((size_t)n * R, -1);
    HIP_OK(hipMemcpy(adj.data(), dadj, (size_t)n * R * 4, hipMemcpyDeviceToHost));
    return JAG_OK;
}

}  // namespace jag

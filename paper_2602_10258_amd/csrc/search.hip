// Batched filtered greedy search on gfx950 (paper Algorithms 1 and 2 with
// the comparator D_F of Section 3.2), one 64-lane wavefront per query.
//
// Per query the wavefront keeps, in LDS:
//   key[Lcap] : (dist_F << 32) | float bits of the squared distance; equal
//               keys are ordered by vertex id, so the order is total
//   idf[Lcap] : vertex id, bit 31 = expanded
//   hash[H]   : ids already discovered.  It may forget ids (a full probe
//               window overwrites its first slot) but never reports an id it
//               was not given.  Forgetting is harmless: the candidate list is
//               always the l_s best of every vertex discovered so far, so a
//               vertex that fell out of it cannot re-enter, and one that is
//               still in it is recognised by its identical (key, id) when it
//               is merged again.
// One hop: take the first unexpanded entry p, read p's adjacency row (one
// coalesced 256-byte load), drop ids already discovered, evaluate dist_F of
// the rest from their attributes (exact integers), drop those whose dist_F
// exceeds that of the worst entry of a full list (they can never enter: the
// order is lexicographic), gather the surviving vectors four lanes per row
// and merge the new keys into the sorted list, cutting it to l_s.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
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
};

namespace {

constexpr uint32_t kExpanded = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;

struct SearchArgs {
    const int32_t *adj;
    const unsigned char *vec;
    const unsigned char *f32;
    const int32_t *scalar;
    const uint16_t *lab;
    const float *Q;
    const FilterRecord *rec;
    int32_t *ids;
    float *dists;
    int32_t *count;
    int32_t *stats;
    float *features;
    const uint16_t *pred;
    int32_t vec_stride, f32_stride, W, d, R, entry;
    int32_t adj_words, scal_word_off, lab_word_off;  // adjacency row layout (words)
    int32_t L, Lcap, Hmask, k, rerank, max_hops, mode, nladder, warm;
    const int32_t *perm;  // query handled by each workgroup (null: identity)
    int32_t *state;       // modes 3 and 4: saved search state, state_stride words per query
    int32_t *order_key;   // mode 3: 1 + predicted ladder index per query (0: ended before)
    int64_t state_stride;
    float delta, rho;
    int32_t ladder[JAG_LADDER_MAX];
};

__device__ __forceinline__ bool key_lt(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------- dist_F
// Section 3.1: label -> [label missing]; range -> distance to [lo, hi];
// subset -> number of required labels missing; Boolean DNF -> fewest
// literals to flip in the cheapest satisfiable clause; general Boolean
// function (truth table) -> its precomputed distance table at the item's
// assignment of the function's variables.
// Which attributes an index's items carry; kernels are built per kind so
// that an index with scalars only (range filters) or labels only carries no
// code or registers for the other kind.  On an index of one kind the
// encoder accepts only that kind's filters; a record of the other kind
// would get dist_F = "never satisfied".
enum AttrKind { AK_ANY = 0, AK_SCALAR = 1, AK_LABELS = 2 };

// The attribute words of one item as the filter needs them: the scalar for
// a range filter, else the label row (two uint16 labels per word, 0xFFFF
// padded).
struct ItemAttr {
    int32_t scalar;
    uint32_t w[8];
};

__device__ __forceinline__ void load_label_words(uint32_t *w, const unsigned char *row, int nw)
{
    if (nw == 1) {
        w[0] = *reinterpret_cast<const uint32_t *>(row);
    } else if (nw == 2) {
        uint2 t = *reinterpret_cast<const uint2 *>(row);
        w[0] = t.x;
        w[1] = t.y;
    } else {
        uint4 t = *reinterpret_cast<const uint4 *>(row);
        w[0] = t.x;
        w[1] = t.y;
        w[2] = t.z;
        w[3] = t.w;
        if (nw == 8) {
            uint4 s = *reinterpret_cast<const uint4 *>(row + 16);
            w[4] = s.x;
            w[5] = s.y;
            w[6] = s.z;
            w[7] = s.w;
        }
    }
}

// from the per-item attribute arrays
template <int AK>
__device__ __forceinline__ void load_item_attr(ItemAttr &at, const FilterRecord &f, int32_t u,
                                               const SearchArgs &a)
{
    if (AK == AK_SCALAR || (AK == AK_ANY && f.type == F_RANGE)) {
        at.scalar = a.scalar[u];
        return;
    }
    load_label_words(at.w, reinterpret_cast<const unsigned char *>(a.lab) + (int64_t)u * a.W * 2, a.W >> 1);
}

// from the adjacency row of the vertex being expanded: the row carries, after
// the R neighbour ids, each neighbour's scalar and label words (slot j)
template <int AK>
__device__ __forceinline__ void load_row_attr(ItemAttr &at, const FilterRecord &f, const int32_t *row,
                                              int j, const SearchArgs &a)
{
    if (AK == AK_SCALAR || (AK == AK_ANY && f.type == F_RANGE)) {
        at.scalar = row[a.scal_word_off + j];
        return;
    }
    load_label_words(at.w, reinterpret_cast<const unsigned char *>(row + a.lab_word_off) + j * a.W * 2,
                     a.W >> 1);
}

template <int AK>
__device__ __forceinline__ uint32_t dist_f(const FilterRecord &f, const uint8_t *tab, const ItemAttr &at,
                                           const SearchArgs &a)
{
    if (AK != AK_LABELS && f.type == F_RANGE) {
        int64_t v = at.scalar;
        if (v < f.a) return (uint32_t)((int64_t)f.a - v);
        if (v > f.b) return (uint32_t)(v - (int64_t)f.b);
        return 0u;
    }
    if (AK == AK_SCALAR || (AK == AK_LABELS && f.type == F_RANGE)) return kUnsat;
    const uint32_t *w = at.w;
    int nw = a.W >> 1;
    // static loop bounds keep the (uniform) record in scalar registers
    uint32_t present = 0;
#pragma unroll
    for (int i = 0; i < kMaxFilterLits; i++) {
        if (i < f.nlit) {
            uint32_t l = f.lits[i];
            bool hit = false;
#pragma unroll
            for (int j = 0; j < 8; j++)
                if (j < nw) hit |= ((w[j] & 0xFFFFu) == l) | ((w[j] >> 16) == l);
            present |= (uint32_t)hit << i;
        }
    }
    if (f.type == F_LABEL) return (present & 1u) ? 0u : 1u;
    if (f.type == F_SUBSET) return (uint32_t)(f.nlit - __builtin_popcount(present));
    if (f.type == F_TABLE) {  // present = the item's assignment of the table's variables
        const uint32_t v = tab[present];
        return v == 255u ? kUnsat : v;
    }
    uint32_t truth = present ^ f.negmask;
    uint32_t best = kUnsat;
#pragma unroll
    for (int c = 0; c < kMaxClauses; c++) {
        if (c < f.ncl) {
            uint32_t cost = (uint32_t)__builtin_popcount((uint32_t)f.clmask[c] & ~truth);
            best = cost < best ? cost : best;
        }
    }
    return best;
}

// ---------------------------------------------------------------- distances
template <int STORE>
struct StoreTraits;
template <>
struct StoreTraits<JAG_STORE_F32> {
    static constexpr int EPC = 4;
};
template <>
struct StoreTraits<JAG_STORE_BF16> {
    static constexpr int EPC = 8;
};
template <>
struct StoreTraits<JAG_STORE_FP8_E4M3> {
    static constexpr int EPC = 16;
};

// The query in registers: lane `sub` of a G-lane group holds the elements
// of the 16-byte chunks j*G + sub of a row (zero beyond d).
template <int STORE, int G, int CH>
struct QueryRegs {
    float v[CH][StoreTraits<STORE>::EPC];
    __device__ __forceinline__ void load(const float *q, int d, int sub)
    {
        constexpr int EPC = StoreTraits<STORE>::EPC;
#pragma unroll
        for (int j = 0; j < CH; j++)
#pragma unroll
            for (int e = 0; e < EPC; e++) {
                int idx = (j * G + sub) * EPC + e;
                v[j][e] = idx < d ? q[idx] : 0.f;
            }
    }
};

__device__ __forceinline__ float acc_sq(float acc, float qv, float x)
{
    float t = qv - x;
    return __builtin_fmaf(t, t, acc);
}

// Partial squared distance of one row held by a G-lane group; the partial
// sums of the group are then added in a fixed butterfly order.
template <int STORE, int G, int CH>
__device__ __forceinline__ float row_dist(const unsigned char *row, const QueryRegs<STORE, G, CH> &q,
                                          int sub)
{
    uint4 c[CH];
#pragma unroll
    for (int j = 0; j < CH; j++)
        c[j] = *reinterpret_cast<const uint4 *>(row + (j * G + sub) * 16);
    float acc = 0.f;
    if constexpr (STORE == JAG_STORE_F32) {
#pragma unroll
        for (int j = 0; j < CH; j++) {
            acc = acc_sq(acc, q.v[j][0], __uint_as_float(c[j].x));
            acc = acc_sq(acc, q.v[j][1], __uint_as_float(c[j].y));
            acc = acc_sq(acc, q.v[j][2], __uint_as_float(c[j].z));
            acc = acc_sq(acc, q.v[j][3], __uint_as_float(c[j].w));
        }
    } else if constexpr (STORE == JAG_STORE_BF16) {
#pragma unroll
        for (int j = 0; j < CH; j++) {
            uint32_t w[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
#pragma unroll
            for (int t = 0; t < 4; t++) {
                acc = acc_sq(acc, q.v[j][2 * t], __uint_as_float(w[t] << 16));
                acc = acc_sq(acc, q.v[j][2 * t + 1], __uint_as_float(w[t] & 0xFFFF0000u));
            }
        }
    } else {
        // the row's FP32 scale sits in the last 4 bytes: chunk CH-1 of lane G-1
        uint32_t sbits = c[CH - 1].w;
        float s = __uint_as_float(__shfl(sbits, (threadIdx.x & ~(G - 1)) | (G - 1), 64));
#pragma unroll
        for (int j = 0; j < CH; j++) {
            uint32_t w[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
#pragma unroll
            for (int t = 0; t < 4; t++) {
                if (j == CH - 1 && t == 3 && sub == G - 1) continue;  // the scale, not codes
                auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[t], false);
                auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[t], true);
                acc = acc_sq(acc, q.v[j][4 * t + 0], s * lo[0]);
                acc = acc_sq(acc, q.v[j][4 * t + 1], s * lo[1]);
                acc = acc_sq(acc, q.v[j][4 * t + 2], s * hi[0]);
                acc = acc_sq(acc, q.v[j][4 * t + 3], s * hi[1]);
            }
        }
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) acc += __shfl_xor(acc, m, 64);
    return acc;
}

// Squared distances of the m candidates cid[0..m) into cd2[], G lanes per row.
template <int STORE, int G, int CH>
__device__ __forceinline__ void eval_rows(const unsigned char *base, int stride, const int32_t *cid,
                                          float *cd2, int m, const QueryRegs<STORE, G, CH> &q)
{
    const int lane = threadIdx.x;
    const int sub = lane & (G - 1), grp = lane / G;
    constexpr int P = 64 / G;
    for (int r = 0; r < m; r += 2 * P) {
        int c0 = r + grp, c1 = r + P + grp;
        // rows past m re-read row cid[0] so every lane stays in bounds
        int i0 = cid[c0 < m ? c0 : 0], i1 = cid[c1 < m ? c1 : 0];
        float d0 = row_dist<STORE, G, CH>(base + (int64_t)i0 * stride, q, sub);
        float d1 = 0.f;
        if (r + P < m) d1 = row_dist<STORE, G, CH>(base + (int64_t)i1 * stride, q, sub);
        if (sub == 0 && c0 < m) cd2[c0] = d0;
        if (sub == 0 && c1 < m) cd2[c1] = d1;
    }
}

// Generic FP32 row distance with a runtime chunk count (for reranking).
__device__ __forceinline__ float row_dist_f32_rt(const unsigned char *row, const float *q, int d,
                                                 int nch, int sub)
{
    float acc = 0.f;
    for (int j = 0; j < nch; j++) {
        int e0 = (j * 4 + sub) * 4;
        float4 x = *reinterpret_cast<const float4 *>(row + (j * 4 + sub) * 16);
        float xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int e = 0; e < 4; e++) acc = acc_sq(acc, e0 + e < d ? q[e0 + e] : 0.f, xs[e]);
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    return acc;
}

// ---------------------------------------------------------------- LDS list
struct Lds {
    uint64_t *key;
    uint32_t *idf;
    int32_t *hash;
    int32_t *cid;
    uint32_t *cdf;
    float *cd2;
    uint64_t *skey;
    uint32_t *sid;
    int32_t *spos;
    float *feat;
    float *h1;
    uint64_t *exkey;
};

__device__ __forceinline__ Lds carve(unsigned char *smem, int Lcap, int H)
{
    Lds s;
    s.key = reinterpret_cast<uint64_t *>(smem);
    s.skey = s.key + Lcap;
    s.exkey = s.skey + 64;
    s.idf = reinterpret_cast<uint32_t *>(s.exkey + 4);
    s.hash = reinterpret_cast<int32_t *>(s.idf + Lcap);
    s.cid = s.hash + H;
    s.cdf = reinterpret_cast<uint32_t *>(s.cid + 64);
    s.cd2 = reinterpret_cast<float *>(s.cdf + 64);
    s.sid = reinterpret_cast<uint32_t *>(s.cd2 + 64);
    s.spos = reinterpret_cast<int32_t *>(s.sid + 64);
    s.feat = reinterpret_cast<float *>(s.spos + 64);
    s.h1 = s.feat + 16;
    return s;
}

__host__ __device__ constexpr size_t lds_bytes(int Lcap, int H)
{
    return (size_t)Lcap * 8 + 64 * 8 + 4 * 8 + (size_t)Lcap * 4 + (size_t)H * 4 + 64 * 4 * 6 + 16 * 4 +
           64 * 4;
}

// Insert id u into the lossy seen-table; true if u was not found (newly
// seen).  The table is a set of 4-slot buckets read with one 16-byte LDS
// load: u is looked for in its bucket, then stored in the first empty slot,
// or over a slot chosen by its hash when the bucket is full.  Lanes that
// insert into one bucket at once may overwrite each other's ids; either way
// the table only forgets ids, it never reports one it was not given.
__device__ __forceinline__ bool hash_insert(int32_t *hash, int mask, int32_t u)
{
    uint32_t h = (uint32_t)u * 0x9E3779B1u;
    h ^= h >> 15;
    const int b = (int)(h & (uint32_t)mask) & ~3;
    const int4 v = *reinterpret_cast<const int4 *>(hash + b);
    if (v.x == u || v.y == u || v.z == u || v.w == u) return false;
    const int slot = v.x == -1 ? 0 : v.y == -1 ? 1 : v.z == -1 ? 2 : v.w == -1 ? 3 : (int)((h >> 20) & 3u);
    hash[b + slot] = u;
    return true;
}

// First entry at or after `from` whose expanded bit is clear, or cnt.
__device__ __forceinline__ int first_unexpanded(const Lds &s, int from, int cnt)
{
    const int lane = threadIdx.x;
    for (int j0 = from; j0 < cnt; j0 += 64) {
        int j = j0 + lane;
        bool un = j < cnt && !(s.idf[j] & kExpanded);
        uint64_t b = ballot64(un);
        if (b) return j0 + __builtin_ctzll(b);
    }
    return cnt;
}

// Merge for a list of at most 64 entries and at most kSmallMerge survivors:
// lane j holds list entry j in registers; the survivors are visited one by
// one (their key broadcast with readlane), and one ballot over the list gives
// each survivor's insertion point and another tells whether it is already in
// the list.  In the same pass list lanes count the survivors ahead of them
// and candidate lanes their rank among the survivors; then every entry is
// written once to its final slot.  No LDS round trips inside the pass.
// Larger survivor sets take the binary-search merge below.  On the range
// workload (BF16, L = 44) thresholds 8 / 16 / 32 measured 0.727 / 0.734 /
// 0.764 ms per launch against 0.751 ms with the binary-search merge alone.
constexpr int kSmallMerge = 8;

__device__ __forceinline__ int merge_small(const Lds &s, int cnt, int ls, bool have, uint64_t ck, uint32_t ci,
                                           uint64_t vm, int *minpos)
{
    const int lane = threadIdx.x;
    const bool inl = lane < cnt;
    const uint64_t lk = inl ? s.key[lane] : 0ull;
    const uint32_t lidf = inl ? s.idf[lane] : 0u;
    const uint32_t li = lidf & kIdMask;
    int sh = 0, rank = 0, mypos = 0, nkeep = 0, mp = ls;
    bool dup = false;
    for (uint64_t mm = vm; mm; mm &= mm - 1) {
        const int d = __builtin_ctzll(mm);
        const uint32_t dkh = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(ck >> 32), d);
        const uint32_t dkl = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)ck, d);
        const uint32_t di = (uint32_t)__builtin_amdgcn_readlane((int)ci, d);
        const uint64_t dk = ((uint64_t)dkh << 32) | dkl;
        const int pd = __popcll(ballot64(inl && key_lt(lk, li, dk, di)));
        const bool isdup = ballot64(inl && lk == dk && li == di) != 0;
        mypos = lane == d ? pd : mypos;
        dup = lane == d ? isdup : dup;
        if (!isdup) {
            nkeep++;
            sh += (inl && pd <= lane) ? 1 : 0;
            rank += (have && key_lt(dk, di, ck, ci)) ? 1 : 0;
            mp = pd < mp ? pd : mp;
        }
    }
    __syncthreads();
    if (inl && lane + sh < ls) {
        s.key[lane + sh] = lk;
        s.idf[lane + sh] = lidf;
    }
    if (have && !dup && mypos + rank < ls) {
        s.key[mypos + rank] = ck;
        s.idf[mypos + rank] = ci;
    }
    __syncthreads();
    *minpos = nkeep ? mp : ls;
    const int nc = cnt + nkeep;
    return nc < ls ? nc : ls;
}

// Merge candidates (lane c < m holds cid/cdf/cd2 slot c) into the sorted
// list of cnt entries, keeping at most ls.  Returns the new size; *minpos is
// the list position of the best inserted candidate (ls if none).
__device__ int merge_candidates(const Lds &s, int m, int cnt, int ls, int *minpos)
{
    const int lane = threadIdx.x;
    bool have = lane < m;
    uint64_t ck = 0;
    uint32_t ci = 0;
    if (have) {
        ck = ((uint64_t)s.cdf[lane] << 32) | __float_as_uint(s.cd2[lane]);
        ci = (uint32_t)s.cid[lane];
    }
    if (have && cnt == ls) {
        uint64_t wk = s.key[cnt - 1];
        uint32_t wi = s.idf[cnt - 1] & kIdMask;
        if (!key_lt(ck, ci, wk, wi)) have = false;
    }
    {
        const uint64_t vm0 = ballot64(have);
        if (vm0 == 0) {
            *minpos = ls;
            return cnt;
        }
        if (cnt <= 64 && __popcll(vm0) <= kSmallMerge) return merge_small(s, cnt, ls, have, ck, ci, vm0, minpos);
    }
    int pos = 0;
    if (have) {
        int lo = 0, hi = cnt;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (key_lt(s.key[mid], s.idf[mid] & kIdMask, ck, ci)) lo = mid + 1;
            else hi = mid;
        }
        pos = lo;
        if (pos < cnt && s.key[pos] == ck && (s.idf[pos] & kIdMask) == ci) have = false;
    }
    uint64_t vm = ballot64(have);
    int mv = __popcll(vm);
    if (mv == 0) {
        *minpos = ls;
        return cnt;
    }
    // rank among the surviving candidates (written compacted to skey/sid first)
    int slot = lanes_below(vm);
    if (have) {
        s.skey[slot] = ck;
        s.sid[slot] = ci;
    }
    __syncthreads();
    int rank = 0;
    if (have)
        for (int j = 0; j < mv; j++) rank += key_lt(s.skey[j], s.sid[j], ck, ci) ? 1 : 0;
    __syncthreads();
    if (have) {
        s.skey[rank] = ck;
        s.sid[rank] = ci;
        s.spos[rank] = pos;
    }
    __syncthreads();
    int mp = s.spos[0];
    int newcnt = cnt + mv < ls ? cnt + mv : ls;
    // shift list entries right by the number of candidates before them,
    // chunk by chunk from the end so no unread entry is overwritten
    int top = ((cnt - 1) >> 6) << 6;
    for (int j0 = top; j0 >= (mp & ~63); j0 -= 64) {
        int j = j0 + lane;
        uint64_t kj = 0;
        uint32_t ij = 0;
        bool mv_ = j < cnt && j >= mp;
        if (mv_) {
            kj = s.key[j];
            ij = s.idf[j];
        }
        int sh = 0;
        if (mv_) {
            int lo = 0, hi = mv;
            uint32_t id = ij & kIdMask;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (key_lt(s.skey[mid], s.sid[mid], kj, id)) lo = mid + 1;
                else hi = mid;
            }
            sh = lo;
        }
        __syncthreads();
        if (mv_ && j + sh < ls) {
            s.key[j + sh] = kj;
            s.idf[j + sh] = ij;
        }
        __syncthreads();
    }
    if (have && pos + rank < ls) {
        s.key[pos + rank] = ck;
        s.idf[pos + rank] = ci;
    }
    __syncthreads();
    *minpos = mp;
    return newcnt;
}

__device__ __forceinline__ float squash(uint32_t df)
{
    float x = (float)df;
    return x / (x + 1.0f);
}

__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Beam predictor: 16 -> 64 -> 64 -> 1, ReLU, BF16 weights, FP32 sums.
// Lane j computes hidden unit j; the output is a butterfly sum over lanes.
__device__ float predict(const Lds &s, const uint16_t *P)
{
    const int lane = threadIdx.x;
    const uint16_t *W1 = P, *b1 = P + 1024, *W2 = P + 1088, *b2 = P + 5184, *w3 = P + 5248,
                   *b3 = P + 5312;
    float acc = bf16f(b1[lane]);
#pragma unroll
    for (int i = 0; i < 16; i++) acc = __builtin_fmaf(bf16f(W1[lane * 16 + i]), s.feat[i], acc);
    s.h1[lane] = acc > 0.f ? acc : 0.f;
    __syncthreads();
    float acc2 = bf16f(b2[lane]);
    for (int i = 0; i < 64; i++) acc2 = __builtin_fmaf(bf16f(W2[lane * 64 + i]), s.h1[i], acc2);
    float h2 = acc2 > 0.f ? acc2 : 0.f;
    float t = bf16f(w3[lane]) * h2;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
    __syncthreads();
    return t + bf16f(b3[0]);
}

// WPE: occupancy target (waves per SIMD) the register allocator works to;
// SL: 64-neighbour slices per row (2 for R up to 128); AK: AttrKind.
template <int STORE, int G, int CH, int WPE, int SL, int AK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void search_kernel(SearchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int64_t q = a.perm ? (int64_t)a.perm[blockIdx.x] : (int64_t)blockIdx.x;
    const int H = a.Hmask + 1;
    Lds s = carve(smem, a.Lcap, H);
    const FilterRecord f = a.rec[q];
    // TABLE filters: the distance table sits table_off bytes after the record
    const uint8_t *tab = f.type == F_TABLE ? reinterpret_cast<const uint8_t *>(a.rec + q) + f.table_off : nullptr;
    const float *qv = a.Q + q * a.d;
    QueryRegs<STORE, G, CH> qr;
    qr.load(qv, a.d, lane & (G - 1));

    int cnt = 1, hint = 0, hops = 0, ndist = 1, nattr = 1;
    // learned and trace modes: the first four expansions use the full list
    // width (see plan_search), so the features do not depend on the final beam
    int ls = a.mode == 0 ? a.L : a.warm;
    int hopcap = a.max_hops > 0 ? a.max_hops : INT_MAX;
    // modes: 0 fixed beam, 1 predicted beam, 2 trace; a two-pass learned
    // search runs mode 3 (up to the prediction, then save the state and stop)
    // and mode 4 (resume a saved state, else the same as mode 1)
    int lhat = a.mode == 0 || a.mode == 2 ? a.L : 0;
    bool predicted = a.mode == 0;
    const int32_t *rs = a.mode == 4 ? a.state + q * a.state_stride : nullptr;
    if (rs && rs[0] > 0) {
        cnt = rs[1];
        hint = rs[2];
        hops = rs[3];
        ndist = rs[4];
        nattr = rs[5];
        hopcap = rs[6];
        lhat = rs[7];
        ls = lhat;
        predicted = true;
        const uint64_t *sk = reinterpret_cast<const uint64_t *>(rs + 8);
        const uint32_t *si = reinterpret_cast<const uint32_t *>(rs + 8 + 2 * a.Lcap);
        for (int j = lane; j < cnt; j += 64) {
            s.key[j] = sk[j];
            s.idf[j] = si[j];
        }
        // the seen-table starts again from the list's ids: a forgotten vertex
        // is recognised at the merge or cannot re-enter (I1), so the results
        // are those of the one-pass search; a table that holds only the list
        // also forgets less later on than the full one would
        for (int i = lane; i < H; i += 64) s.hash[i] = -1;
        __syncthreads();
        for (int j = lane; j < cnt; j += 64) hash_insert(s.hash, a.Hmask, (int32_t)(si[j] & kIdMask));
        __syncthreads();
    } else {
        for (int i = lane; i < H; i += 64) s.hash[i] = -1;
        // L <- {s}
        if (lane == 0) {
            s.cid[0] = a.entry;
            ItemAttr at;
            load_item_attr<AK>(at, f, a.entry, a);
            s.cdf[0] = dist_f<AK>(f, tab, at, a);
        }
        __syncthreads();
        eval_rows<STORE, G, CH>(a.vec, a.vec_stride, s.cid, s.cd2, 1, qr);
        __syncthreads();
        if (lane == 0) {
            s.key[0] = ((uint64_t)s.cdf[0] << 32) | __float_as_uint(s.cd2[0]);
            s.idf[0] = (uint32_t)a.entry;
            hash_insert(s.hash, a.Hmask, a.entry);
        }
        __syncthreads();
    }
    for (;;) {
        hint = first_unexpanded(s, hint, cnt);
        if (hint >= cnt || hops >= hopcap) break;
        const int p = (int)(s.idf[hint] & kIdMask);
        __syncthreads();
        if (lane == 0) {
            s.idf[hint] |= kExpanded;
            if (hops < 4) s.exkey[hops] = s.key[hint];
        }
        hops++;
        // one row holds the neighbour ids and their attribute words: both
        // loads are issued together, before the ids are known.  Rows wider
        // than a wave (SL = 2: R up to 128) go in slices of 64 neighbours,
        // each merged in turn (one slice after the other keeps the same best l_s)
        const int32_t *row = a.adj + (int64_t)p * a.adj_words;
        int minpos = INT_MAX;
#pragma unroll
        for (int h = 0; h < SL * 64; h += 64) {
            if (h >= a.R) break;
            int32_t u = -1;
            ItemAttr at;
            if (h + lane < a.R) {
                u = row[h + lane];
                load_row_attr<AK>(at, f, row, h + lane, a);
            }
            bool fresh = u >= 0 && hash_insert(s.hash, a.Hmask, u);
            uint32_t df = fresh ? dist_f<AK>(f, tab, at, a) : 0u;
            nattr += __popcll(ballot64(fresh));
            if (cnt == ls) fresh = fresh && df <= (uint32_t)(s.key[cnt - 1] >> 32);
            uint64_t bm = ballot64(fresh);
            int m = __popcll(bm);
            if (fresh) {
                int slot = lanes_below(bm);
                s.cid[slot] = u;
                s.cdf[slot] = df;
            }
            __syncthreads();
            if (m > 0) {
                eval_rows<STORE, G, CH>(a.vec, a.vec_stride, s.cid, s.cd2, m, qr);
                __syncthreads();
                ndist += m;
                int mp = INT_MAX;
                cnt = merge_candidates(s, m, cnt, ls, &mp);
                minpos = mp < minpos ? mp : minpos;
            }
        }
        hint = minpos < hint + 1 ? minpos : hint + 1;
        if (!predicted && hops == 4) {
            predicted = true;
            // predictor features after the fourth expansion
            int valid = 0;
            for (int j0 = 0; j0 < cnt; j0 += 64) {
                int j = j0 + lane;
                valid += __popcll(ballot64(j < cnt && (s.key[j] >> 32) == 0));
            }
            if (lane == 0) {
                for (int i = 0; i < 16; i++) s.feat[i] = 0.f;
                s.feat[f.type] = 1.f;
                s.feat[4] = f.sel_feature;
                float b = __uint_as_float((uint32_t)s.exkey[0]);
                b = b > 1e-30f ? b : 1e-30f;
                for (int j = 1; j < 4; j++) s.feat[4 + j] = __uint_as_float((uint32_t)s.exkey[j]) / b;
                s.feat[8] = __uint_as_float((uint32_t)s.key[0]) / b;
                for (int j = 0; j < 4; j++) s.feat[9 + j] = squash((uint32_t)(s.exkey[j] >> 32));
                s.feat[13] = squash((uint32_t)(s.key[0] >> 32));
                s.feat[14] = (float)valid / (float)cnt;
                s.feat[15] = 1.f;
            }
            __syncthreads();
            if (a.mode == 2) {
                if (lane < 16) a.features[q * 16 + lane] = s.feat[lane];
                if (cnt > a.L) cnt = a.L;
                ls = a.L;
            } else {
                float y = predict(s, a.pred);
                float z = y + a.delta;
                int idx;
                if (!(z == z)) idx = a.nladder - 1;
                else {
                    float c = ceilf(z);
                    idx = c < 0.f ? 0 : (c > (float)(a.nladder - 1) ? a.nladder - 1 : (int)c);
                }
                lhat = a.ladder[idx];  // read from the kernel arguments when needed
                float capf = ceilf(a.rho * (float)lhat);
                int cap = capf >= 2147483647.0f ? INT_MAX : (int)capf;
                cap = cap < 4 ? 4 : cap;
                hopcap = cap < hopcap ? cap : hopcap;
                if (cnt > lhat) cnt = lhat;
                ls = lhat;
                if (a.mode == 3) {  // save the state after the cut and stop
                    int32_t *ws = a.state + q * a.state_stride;
                    uint64_t *sk = reinterpret_cast<uint64_t *>(ws + 8);
                    uint32_t *si = reinterpret_cast<uint32_t *>(ws + 8 + 2 * a.Lcap);
                    for (int j = lane; j < cnt; j += 64) {
                        sk[j] = s.key[j];
                        si[j] = s.idf[j];
                    }
                    if (lane < 8) {
                        int v = lane == 0 ? idx + 1 : lane == 1 ? cnt : lane == 2 ? hint : lane == 3 ? hops
                              : lane == 4 ? ndist : lane == 5 ? nattr : lane == 6 ? hopcap : lhat;
                        ws[lane] = v;
                    }
                    if (lane == 0) a.order_key[q] = idx + 1;
                    return;
                }
            }
        }
    }
    if (a.mode == 2 && !predicted && lane < 16)  // fewer than four expansions: no features
        a.features[q * 16 + lane] = lane == 15 ? -1.f : 0.f;
    if (a.mode == 3) {  // ended before the prediction point: the search pass redoes it
        if (lane == 0) {
            a.state[q * a.state_stride] = 0;
            a.order_key[q] = 0;
        }
        return;
    }
    // ---- output: top-k valid entries, optionally rescored in FP32
    int outn = cnt;
    if (a.rerank > 0) {
        int rk = a.rerank * a.k;
        rk = rk < cnt ? rk : cnt;
        if (lane < rk) {
            s.cid[lane] = (int32_t)(s.idf[lane] & kIdMask);
            s.cdf[lane] = (uint32_t)(s.key[lane] >> 32);
        }
        __syncthreads();
        const int sub = lane & 3, grp = lane >> 2;
        const int nch = a.f32_stride >> 6;
        for (int r = 0; r < rk; r += 16) {
            int c = r + grp;
            int id = s.cid[c < rk ? c : 0];
            float dd = row_dist_f32_rt(a.f32 + (int64_t)id * a.f32_stride, qv, a.d, nch, sub);
            if (sub == 0 && c < rk) s.cd2[c] = dd;
        }
        __syncthreads();
        uint64_t ck = 0;
        uint32_t ci = 0;
        int rank = 0;
        if (lane < rk) {
            ck = ((uint64_t)s.cdf[lane] << 32) | __float_as_uint(s.cd2[lane]);
            ci = (uint32_t)s.cid[lane];
            for (int j = 0; j < rk; j++) {
                uint64_t kj = ((uint64_t)s.cdf[j] << 32) | __float_as_uint(s.cd2[j]);
                rank += key_lt(kj, (uint32_t)s.cid[j], ck, ci) ? 1 : 0;
            }
        }
        __syncthreads();
        if (lane < rk) {
            s.key[rank] = ck;
            s.idf[rank] = ci;
        }
        __syncthreads();
        outn = rk;
    }
    bool ok = lane < a.k && lane < outn && (s.key[lane < outn ? lane : 0] >> 32) == 0;
    if (lane < a.k) {
        a.ids[q * a.k + lane] = ok ? (int32_t)(s.idf[lane] & kIdMask) : -1;
        a.dists[q * a.k + lane] = ok ? __uint_as_float((uint32_t)s.key[lane]) : __builtin_inff();
    }
    int cntv = __popcll(ballot64(ok));
    if (lane == 0) {
        a.count[q] = cntv;
        if (a.stats) {
            a.stats[q * 4 + 0] = hops;
            a.stats[q * 4 + 1] = ndist;
            a.stats[q * 4 + 2] = nattr;
            a.stats[q * 4 + 3] = lhat;
        }
    }
}

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
// ... (coalesced reads), taken 16 at a time so that 16 independent loads
// are in flight per thread; within a class the order is (thread, then
// position), not the query order, which no result depends on.
constexpr int kOrderThreads = 512;
constexpr int kOrderBatch = 16;
constexpr int kOrderBins = JAG_LADDER_MAX + 1;
// Fixed-beam and one-pass learned launches of at least this many queries
// are ordered by selectivity (smaller ones fit on the device at once, where
// the order hardly matters).
constexpr int64_t kSelOrderMin = 4096;

static bool sel_ordered(const jag_search_params &S, int64_t nq)
{
    return (S.learned == 0 || (S.learned == 1 && S.single_pass)) && nq >= kSelOrderMin;
}

__global__ __launch_bounds__(256) void class_kernel(const FilterRecord *rec, int64_t nq, int32_t *key)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nq) return;
    const float x = rec[i].sel_feature;  // log2(selectivity) / 16, in [-1.9, 0]
    const float c = floorf(16.f + x * (256.f / 30.f));
    const int broad = c >= 0.f ? (c <= 16.f ? (int)c : 16) : 0;  // 16: selectivity 1
    key[i] = rec[i].type == F_RANGE ? broad : 16 - broad;
}

__device__ __forceinline__ int order_class(const int32_t *key, int64_t i)
{
    const int k = key[i];
    return k < 0 ? 0 : (k >= kOrderBins ? kOrderBins - 1 : k);
}

// Both loops clamp the index instead of branching on it, so that the
// batch's loads issue back to back.
__global__ __launch_bounds__(kOrderThreads) void order_kernel(const int32_t *key, int64_t nq, int32_t *perm)
{
    __shared__ int32_t cnt[kOrderBins][kOrderThreads];
    __shared__ int32_t part[kOrderThreads];
    const int t = threadIdx.x;
    for (int b = 0; b < kOrderBins; b++) cnt[b][t] = 0;
    for (int64_t i0 = t; i0 < nq; i0 += (int64_t)kOrderThreads * kOrderBatch) {
        int c[kOrderBatch];
#pragma unroll
        for (int j = 0; j < kOrderBatch; j++) {
            const int64_t i = i0 + (int64_t)j * kOrderThreads;
            c[j] = order_class(key, i < nq ? i : nq - 1);
        }
#pragma unroll
        for (int j = 0; j < kOrderBatch; j++)
            if (i0 + (int64_t)j * kOrderThreads < nq) cnt[c[j]][t]++;
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
        int c[kOrderBatch];
#pragma unroll
        for (int j = 0; j < kOrderBatch; j++) {
            const int64_t i = i0 + (int64_t)j * kOrderThreads;
            c[j] = order_class(key, i < nq ? i : nq - 1);
        }
#pragma unroll
        for (int j = 0; j < kOrderBatch; j++) {
            const int64_t i = i0 + (int64_t)j * kOrderThreads;
            if (i < nq) perm[cnt[c[j]][t]++] = (int32_t)i;
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

// Lanes per vector row: 4 for rows of up to 384 bytes, 8 up to 512 bytes,
// 16 beyond; rows are padded to a multiple of 16 * G bytes.  On the label-set
// workload (FP32 rows of 512 bytes) 8 lanes of 4 chunks ran 10-17 % faster
// than 4 lanes of 8 chunks, which spill registers; on 384-byte rows 4 lanes
// of 6 chunks stay 2 % ahead of 8 lanes of 3.
int pick_group(int stride) { return stride <= 384 ? 4 : stride <= 512 ? 8 : 16; }

int padded_stride(int stride)
{
    const int unit = 16 * pick_group(stride);
    return (stride + unit - 1) / unit * unit;
}

using SearchFn = void (*)(SearchArgs);
using ExactFn = void (*)(SearchArgs, int64_t);

// Chunks of 16 bytes per lane: 4 lanes take rows of up to 384 bytes (1..6
// chunks), 8 lanes rows of 512 (4), 16 lanes wider rows padded to 256 bytes
// (3..8).
template <int STORE, int G, int WPE, int SL, int AK>
SearchFn search_for_ch(int ch)
{
    if (G == 4 && ch >= 1 && ch <= 6) {
        switch (ch) {
        case 1: return search_kernel<STORE, G, 1, WPE, SL, AK>;
        case 2: return search_kernel<STORE, G, 2, WPE, SL, AK>;
        case 3: return search_kernel<STORE, G, 3, WPE, SL, AK>;
        case 4: return search_kernel<STORE, G, 4, WPE, SL, AK>;
        case 5: return search_kernel<STORE, G, 5, WPE, SL, AK>;
        case 6: return search_kernel<STORE, G, 6, WPE, SL, AK>;
        }
    }
    if (G == 8 && ch == 4) return search_kernel<STORE, G, 4, WPE, SL, AK>;
    if (G == 16) {
        switch (ch) {
        case 3: return search_kernel<STORE, G, 3, WPE, SL, AK>;
        case 4: return search_kernel<STORE, G, 4, WPE, SL, AK>;
        case 5: return search_kernel<STORE, G, 5, WPE, SL, AK>;
        case 6: return search_kernel<STORE, G, 6, WPE, SL, AK>;
        case 7: return search_kernel<STORE, G, 7, WPE, SL, AK>;
        case 8: return search_kernel<STORE, G, 8, WPE, SL, AK>;
        }
    }
    return nullptr;
}

template <int WPE, int SL, int AK>
SearchFn pick_search_sl(int store, int G, int ch)
{
    if (store == JAG_STORE_F32)
        return G == 4   ? search_for_ch<JAG_STORE_F32, 4, WPE, SL, AK>(ch)
               : G == 8 ? search_for_ch<JAG_STORE_F32, 8, WPE, SL, AK>(ch)
                        : search_for_ch<JAG_STORE_F32, 16, WPE, SL, AK>(ch);
    if (store == JAG_STORE_BF16)
        return G == 4   ? search_for_ch<JAG_STORE_BF16, 4, WPE, SL, AK>(ch)
               : G == 8 ? search_for_ch<JAG_STORE_BF16, 8, WPE, SL, AK>(ch)
                        : search_for_ch<JAG_STORE_BF16, 16, WPE, SL, AK>(ch);
    return G == 4   ? search_for_ch<JAG_STORE_FP8_E4M3, 4, WPE, SL, AK>(ch)
           : G == 8 ? search_for_ch<JAG_STORE_FP8_E4M3, 8, WPE, SL, AK>(ch)
                    : search_for_ch<JAG_STORE_FP8_E4M3, 16, WPE, SL, AK>(ch);
}

// All modes use the build for 5 waves per SIMD (at most 96 VGPRs; the
// allocator spills 20-60 bytes per lane to scratch): on the range workload
// 8-12 % faster than the 4-wave build (100-128 VGPRs, no scratch) for fixed
// beams, and 7-10 % faster for two-pass learned search with a 64-entry
// warm-up list.  (With a 128-entry warm-up the 4-wave build had been faster
// for learned search.)
constexpr int kWavesPerSimd = 5;

// Rows of more than 64 neighbours take the two-slice build (the one-slice
// build has no slice loop, which keeps its register allocation); rows of up
// to 64 take the build for the index's attribute kind.
SearchFn pick_search(int store, int stride, int R, int ak)
{
    int G = pick_group(stride);
    int ch = stride / (16 * G);
    if (R > 64) return pick_search_sl<kWavesPerSimd, 2, AK_ANY>(store, G, ch);
    if (ak == AK_SCALAR) return pick_search_sl<kWavesPerSimd, 1, AK_SCALAR>(store, G, ch);
    if (ak == AK_LABELS) return pick_search_sl<kWavesPerSimd, 1, AK_LABELS>(store, G, ch);
    return pick_search_sl<kWavesPerSimd, 1, AK_ANY>(store, G, ch);
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

// Seen-table slots.  The kernel holds at most 4 waves per SIMD (16 per CU)
// by registers; 2^10 slots keep LDS from lowering that for lists up to 128
// entries.  Measured on the range workload (1M x 96, 10k queries): equal to
// 2^11 at fixed L = 44 and 64 (6-9 % more repeated evaluations, 14 % more
// resident queries), 17-20 % faster for learned beams (128-entry list).
constexpr int kDefaultHash = 1024;
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
    if (!ix.staging) ix.staging = new StagingRing();
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
    return JAG_OK;
}

// Validate a search request and choose its kernel, LDS size and arguments.
static jag_status plan_search(Index &ix, const float *Q, int64_t nq, const void *records, int32_t k,
                              const jag_search_params &S, int32_t *ids, float *dists, int32_t *count,
                              SearchArgs &a, SearchFn &fn, size_t &lds)
{
    if (k < 1 || k > 64 || S.L < k || S.L > 1024 || S.learned < 0 || S.learned > 2 ||
        S.rerank_mult < 0 || S.rerank_mult * k > 64 || S.max_hops < 0 || nq > INT_MAX ||
        (S.hash_log2 != 0 && (S.hash_log2 < 10 || S.hash_log2 > 13))) {
        set_error("need 1 <= k <= 64, k <= L <= 1024, learned in {0,1,2}, rerank_mult*k <= 64, "
                  "hash_log2 in {0, 10..13}");
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
    int H = S.hash_log2 ? (1 << S.hash_log2) : kDefaultHash;
    a.Lcap = Lcap;
    a.Hmask = H - 1;
    const int ak = ix.has_scalar && !ix.has_labels ? AK_SCALAR : !ix.has_scalar && ix.has_labels ? AK_LABELS
                                                                                                  : AK_ANY;
    fn = pick_search(ix.store, ix.vec_stride, ix.R, ak);
    if (!fn) {
        set_error("no kernel for row stride %d", ix.vec_stride);
        return JAG_EUNSUPPORTED;
    }
    lds = lds_bytes(Lcap, H);
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
    jag_status st = plan_search(ix, Q, nq, records, k, S, ids, dists, count, a, fn, lds);
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
        // one launch, the searches expected to be long first
        int32_t *key = order + nq;
        hipLaunchKernelGGL(class_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, sm, a.rec, nq, key);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(order_kernel, dim3(1), dim3(kOrderThreads), 0, sm, key, nq, order);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            SearchArgs b = a;
            b.perm = order;
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
        hipLaunchKernelGGL(order_kernel, dim3(1), dim3(kOrderThreads), 0, sm, okey, nc, perm);
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
    jag_status st = plan_search(ix, &dummy_f, 1, &dummy_f, k, s2, nullptr, nullptr, nullptr, a, fn, lds);
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
    jag_status st = plan_search(ix, &dummy_f, 1, &dummy_f, k, s2, nullptr, nullptr, nullptr, a, fn, lds);
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

// ---------------------------------------------------------------- staging
// jag_search_batch encodes host filters into pinned host memory and copies
// them to the device asynchronously; an event recorded after the copy says
// when a buffer may be filled again, so the call never waits for the stream.
namespace jag {

constexpr size_t kStagingMax = 8;  // buffers per index; beyond that a caller waits

void free_staging(StagingRing *r)
{
    if (!r) return;
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
    void *drec = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (hipMallocAsync(&drec, (size_t)bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        jag::staging_release(ix.staging, slot);
        jag::set_error("device allocation for filter records failed");
        return JAG_ENOMEM;
    }
    hipError_t e = hipMemcpyAsync(drec, buf.host, (size_t)bytes, hipMemcpyHostToDevice, s);
    // the buffer may be filled again once this copy has run
    hipError_t er = hipEventRecord(buf.copied, s);
    jag::staging_release(ix.staging, slot);
    if (e != hipSuccess || er != hipSuccess) {
        (void)hipFreeAsync(drec, s);
        jag::set_error("filter upload failed: %s", hipGetErrorString(e != hipSuccess ? e : er));
        return JAG_EDEVICE;
    }
    st = jag_search_encoded(idx, Q, nq, drec, k, S, ids, dists, count, stream);
    (void)hipFreeAsync(drec, s);
    return st;
}

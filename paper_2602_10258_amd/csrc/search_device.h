// Device side of the batched filtered search, shared by the batch launches
// (search.hip) and the resident server waves (serve_kernels.hip): the
// filter distances of Section 3.1, the lexicographic comparator D_F of
// Section 3.2, and one query's greedy search (Algorithms 1 and 2) by one
// 64-lane wavefront.
//
// Per query the wavefront keeps, in LDS:
//   key[Lcap] : (dist_F << 32) | float bits of the squared distance; equal
//               keys are ordered by vertex id, so the order is total
//   idf[Lcap] : vertex id, bit 31 = expanded
//   hash[H]   : ids already discovered, as 4-slot buckets.  It may forget ids
//               (a full bucket overwrites a slot) but never reports an id it
//               was not given.  Forgetting is harmless: the candidate list is
//               always the l_s best of every vertex discovered so far, so a
//               vertex that fell out of it cannot re-enter, and one that is
//               still in it is recognised by its identical (key, id) when it
//               is merged again.
// One hop: take the first unexpanded entry p, read p's adjacency row (one
// coalesced load of ids and the neighbours' attributes), drop ids already
// discovered, evaluate dist_F of the rest from their attributes (exact
// integers), drop those whose dist_F exceeds that of the worst entry of a
// full list (they can never enter: the order is lexicographic), gather the
// surviving vectors G lanes per row and merge the new keys into the sorted
// list, cutting it to l_s.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "jag_internal.h"

namespace jag {

// Kernel arguments of one search launch (plan_search fills them).
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
    // ordered launches: per (filter kind, selectivity class), the sum of
    // expansions and the count of searches (null: not recorded)
    unsigned long long *order_stats;
    int64_t state_stride;
    float delta, rho;
    int32_t ladder[JAG_LADDER_MAX];
};

// Selectivity class of a filter record for the launch order: its log2
// selectivity estimate in steps of about two octaves (0 = narrowest, 16 =
// selectivity 1), and its kind (0 range, 1 the label-based filters).
constexpr int kSelClasses = 17;
__host__ __device__ inline int sel_class(float sel_feature)
{
    const float c = floorf(16.f + sel_feature * (256.f / 30.f));  // sel_feature = log2(s) / 16
    return c >= 0.f ? (c <= 16.f ? (int)c : 16) : 0;
}
__host__ __device__ inline int sel_kind(int32_t type) { return type == F_RANGE ? 0 : 1; }

// Which attributes an index's items carry; kernels are built per kind so
// that an index with scalars only (range filters) or labels only carries no
// code or registers for the other kind.  On an index of one kind the
// encoder accepts only that kind's filters; a record of the other kind
// would get dist_F = "never satisfied".
enum AttrKind { AK_ANY = 0, AK_SCALAR = 1, AK_LABELS = 2 };

// Checks a search's parameters against the index and fills the kernel
// arguments, the LDS bytes per query and the attribute kind of the kernel
// to use (search.hip).
jag_status plan_search(Index &ix, const float *Q, int64_t nq, const void *records, int32_t k,
                       const jag_search_params &S, int32_t *ids, float *dists, int32_t *count,
                       SearchArgs &a, size_t &lds, int &ak);

namespace {

constexpr uint32_t kExpanded = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;


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
    // 32-bit byte offsets from the row (the same in every lane): the loads
    // take the row's address from scalar registers
    const unsigned char *rb = reinterpret_cast<const unsigned char *>(row);
    if (AK == AK_SCALAR || (AK == AK_ANY && f.type == F_RANGE)) {
        at.scalar = *reinterpret_cast<const int32_t *>(rb + (uint32_t)(4 * (a.scal_word_off + j)));
        return;
    }
    load_label_words(at.w, rb + (uint32_t)(4 * a.lab_word_off + j * a.W * 2), a.W >> 1);
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

// Lane `sub` of a G-lane group loads its chunks j*G + sub of a row.
template <int G, int CH>
__device__ __forceinline__ void row_load(uint4 (&c)[CH], const unsigned char *row, int sub)
{
#pragma unroll
    for (int j = 0; j < CH; j++)
        c[j] = *reinterpret_cast<const uint4 *>(row + (j * G + sub) * 16);
}

// Partial squared distance of the chunks a lane loaded; the partial sums of
// the group are then added in a fixed butterfly order.
template <int STORE, int G, int CH>
__device__ __forceinline__ float row_sum(const uint4 (&c)[CH], const QueryRegs<STORE, G, CH> &q, int sub)
{
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

// Whether a search kernel keeps two rows per lane group in flight (PAIR
// below): where the query registers and two rows' chunks fit in half of the
// 96-register budget, and the label words of the filter step or the FP8
// decoding do not crowd them out (elsewhere pairs measured as many more
// spills in the expansion loop than they save in round trips).
template <int STORE, int CH, int AK>
constexpr bool pair_rows()
{
    return CH * StoreTraits<STORE>::EPC + 8 * CH <= 48 && STORE != JAG_STORE_FP8_E4M3 &&
           (AK == AK_SCALAR || STORE == JAG_STORE_F32);
}

// Squared distances of the m candidates cid[0..m) into cd2[], G lanes per
// row, 64/G rows per group of lanes at a time.  With PAIR, when two rows per
// lane group remain both rows' loads are issued before either sum, so the
// pair costs one round trip to memory.
template <int STORE, int G, int CH, bool PAIR = false>
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
        uint4 x0[CH];
        row_load<G, CH>(x0, base + (int64_t)i0 * stride, sub);
        float d0, d1 = 0.f;
        if (PAIR && r + P < m) {
            uint4 x1[CH];
            row_load<G, CH>(x1, base + (int64_t)i1 * stride, sub);
            d0 = row_sum<STORE, G, CH>(x0, q, sub);
            d1 = row_sum<STORE, G, CH>(x1, q, sub);
        } else {
            d0 = row_sum<STORE, G, CH>(x0, q, sub);
            if (r + P < m) {
                uint4 x1[CH];
                row_load<G, CH>(x1, base + (int64_t)i1 * stride, sub);
                d1 = row_sum<STORE, G, CH>(x1, q, sub);
            }
        }
        if (sub == 0 && c0 < m) cd2[c0] = d0;
        if (sub == 0 && c1 < m) cd2[c1] = d1;
    }
}

// One row of the FP32 rerank copy, in the lane layout of the search store:
// lane `sub` of a G-lane group loads the elements of chunks j*G + sub (EPC
// each), so the query registers serve both passes; row_sum_f32 then adds the
// lane's squared differences and the group's partial sums (butterfly).
// Groups of four floats that start at or beyond d (offsets from the lane's
// first element at or beyond lim = d - sub*EPC) are not read: they add
// nothing.
template <int STORE, int G, int CH>
__device__ __forceinline__ void row_load_f32(float4 (&x)[CH][StoreTraits<STORE>::EPC / 4],
                                             const unsigned char *row, int lim, int sub)
{
    constexpr int EPC = StoreTraits<STORE>::EPC;
    constexpr int NV = EPC / 4;
    row += 4 * sub * EPC;
#pragma unroll
    for (int j = 0; j < CH; j++)
#pragma unroll
        for (int t = 0; t < NV; t++) {
            const int o = j * G * EPC + 4 * t;
            x[j][t] = o < lim ? *reinterpret_cast<const float4 *>(row + 4 * o) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
}

template <int STORE, int G, int CH>
__device__ __forceinline__ float row_sum_f32(const float4 (&x)[CH][StoreTraits<STORE>::EPC / 4],
                                             const QueryRegs<STORE, G, CH> &q)
{
    constexpr int NV = StoreTraits<STORE>::EPC / 4;
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < CH; j++)
#pragma unroll
        for (int t = 0; t < NV; t++) {
            acc = acc_sq(acc, q.v[j][4 * t + 0], x[j][t].x);
            acc = acc_sq(acc, q.v[j][4 * t + 1], x[j][t].y);
            acc = acc_sq(acc, q.v[j][4 * t + 2], x[j][t].z);
            acc = acc_sq(acc, q.v[j][4 * t + 3], x[j][t].w);
        }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) acc += __shfl_xor(acc, m, 64);
    return acc;
}

// Rows whose lane share in the store's layout is wide (more than 32 floats
// per lane, where the query registers are mostly spilled already) are
// rescored in a layout of their own: 4 lanes per row over the 64-byte
// chunks of the FP32 row (lane sub takes the 16-byte pieces 4j + sub), the
// query's values read from its vector, one piece at a time.
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

// FP32 distances of the m entries cid[0..m) into cd2[] (PAIR as in
// eval_rows).
template <int STORE, int G, int CH, bool PAIR = false>
__device__ __forceinline__ void rerank_rows(const unsigned char *base, int stride, const int32_t *cid,
                                            float *cd2, int m, const QueryRegs<STORE, G, CH> &q,
                                            const float *qv, int d)
{
    constexpr int NV = StoreTraits<STORE>::EPC / 4;
    const int lane = threadIdx.x;
    const int sub = lane & (G - 1), grp = lane / G;
    constexpr int P = 64 / G;
    // elements this lane may read: chunk offsets below lim (kept opaque so
    // that the compiler does not keep the query loader's indices alive, in
    // spilled registers, until the rerank)
    if constexpr (CH * StoreTraits<STORE>::EPC > 32) {
        const int sub4 = lane & 3, grp4 = lane >> 2, nch = stride >> 6;
        for (int r = 0; r < m; r += 16) {
            const int c = r + grp4;
            const float dd = row_dist_f32_rt(base + (int64_t)cid[c < m ? c : 0] * stride, qv, d, nch, sub4);
            if (sub4 == 0 && c < m) cd2[c] = dd;
        }
        return;
    }
    int lim = d - sub * StoreTraits<STORE>::EPC;
    asm volatile("" : "+v"(lim));
    for (int r = 0; r < m; r += 2 * P) {
        int c0 = r + grp, c1 = r + P + grp;
        int i0 = cid[c0 < m ? c0 : 0], i1 = cid[c1 < m ? c1 : 0];
        float4 x0[CH][NV];
        row_load_f32<STORE, G, CH>(x0, base + (int64_t)i0 * stride, lim, sub);
        float d0, d1 = 0.f;
        if (PAIR && r + P < m) {
            float4 x1[CH][NV];
            row_load_f32<STORE, G, CH>(x1, base + (int64_t)i1 * stride, lim, sub);
            d0 = row_sum_f32<STORE, G, CH>(x0, q);
            d1 = row_sum_f32<STORE, G, CH>(x1, q);
        } else {
            d0 = row_sum_f32<STORE, G, CH>(x0, q);
            if (r + P < m) {
                float4 x1[CH][NV];
                row_load_f32<STORE, G, CH>(x1, base + (int64_t)i1 * stride, lim, sub);
                d1 = row_sum_f32<STORE, G, CH>(x1, q);
            }
        }
        if (sub == 0 && c0 < m) cd2[c0] = d0;
        if (sub == 0 && c1 < m) cd2[c1] = d1;
    }
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

// Merge of at most kSmallMerge survivors whose insertion positions pos (the
// number of list entries ahead of them) are known, into a list of any
// length: each survivor's rank among the survivors comes from a readlane
// loop (no LDS round trips); the positions go to spos in rank order (so they
// are non-decreasing), padded to eight with INT_MAX; a list entry at j then
// moves down by the number of survivors with position <= j, counted against
// the eight positions read with two 16-byte LDS loads, instead of a binary
// search over the survivors' keys per entry.  A survivor lands at pos + rank.
__device__ __forceinline__ int merge_few(const Lds &s, int cnt, int ls, bool have, uint64_t ck, uint32_t ci,
                                         int pos, uint64_t vm, int mv, int *minpos)
{
    const int lane = threadIdx.x;
    int rank = 0;
    for (uint64_t mm = vm; mm; mm &= mm - 1) {
        const int d = __builtin_ctzll(mm);
        const uint32_t dkh = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(ck >> 32), d);
        const uint32_t dkl = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)ck, d);
        const uint32_t di = (uint32_t)__builtin_amdgcn_readlane((int)ci, d);
        const uint64_t dk = ((uint64_t)dkh << 32) | dkl;
        rank += (have && key_lt(dk, di, ck, ci)) ? 1 : 0;
    }
    if (have) s.spos[rank] = pos;
    if (lane >= mv && lane < kSmallMerge) s.spos[lane] = INT_MAX;
    __syncthreads();
    const int4 pa = *reinterpret_cast<const int4 *>(s.spos);
    const int4 pb = *reinterpret_cast<const int4 *>(s.spos + 4);
    const int mp = pa.x;
    const int newcnt = cnt + mv < ls ? cnt + mv : ls;
    // shift list entries from the end, chunk by chunk, so no unread entry is overwritten
    const int top = ((cnt - 1) >> 6) << 6;
    for (int j0 = top; j0 >= (mp & ~63); j0 -= 64) {
        const int j = j0 + lane;
        const bool move = j < cnt && j >= mp;
        uint64_t kj = 0;
        uint32_t ij = 0;
        if (move) {
            kj = s.key[j];
            ij = s.idf[j];
        }
        const int sh = (pa.x <= j) + (pa.y <= j) + (pa.z <= j) + (pa.w <= j) + (pb.x <= j) + (pb.y <= j) +
                       (pb.z <= j) + (pb.w <= j);
        __syncthreads();
        if (move && j + sh < ls) {
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
    if (mv <= kSmallMerge) return merge_few(s, cnt, ls, have, ck, ci, pos, vm, mv, minpos);
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
        // survivors ahead of entry j: those inserted at a position <= j
        // (spos is in rank order, so non-decreasing)
        int sh = 0;
        if (mv_) {
            int lo = 0, hi = mv;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (s.spos[mid] <= j) lo = mid + 1;
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
    // opaque copies of the lane and the base: the weight addresses are then
    // formed here, not hoisted out of the search loop into registers that
    // would stay live (or spilled) through every expansion
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    asm volatile("" : "+s"(P));
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

// One query's search by the calling wave (Algorithm 2 over Algorithm 1):
// f its filter record, tab its truth-table distance table (TABLE filters),
// qv its vector; ids_out/dists_out (k each) and count_out receive the
// answer.  q indexes the per-query arrays of a that only batch launches use
// (stats, features, saved states, launch order).  SL: 64-neighbour slices per
// row (2 for R up to 128); AK: AttrKind.
template <int STORE, int G, int CH, int SL, int AK>
__device__ __forceinline__ int search_query(const SearchArgs &a, const int64_t q, const FilterRecord &f,
                                             const uint8_t *tab, const float *qv, int32_t *ids_out,
                                             float *dists_out, int32_t *count_out, unsigned char *smem)
{
    const int lane = threadIdx.x;
    const int H = a.Hmask + 1;
    Lds s = carve(smem, a.Lcap, H);
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
        // the vertex to expand, the same in every lane: held in a scalar
        // register, so its row's address costs no vector registers
        const int p = __builtin_amdgcn_readfirstlane((int)(s.idf[hint] & kIdMask));
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
                u = *reinterpret_cast<const int32_t *>(reinterpret_cast<const unsigned char *>(row) +
                                                       (uint32_t)(4 * (h + lane)));
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
                eval_rows<STORE, G, CH, pair_rows<STORE, CH, AK>()>(a.vec, a.vec_stride, s.cid, s.cd2, m, qr);
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
                        // an opaque lane: the address is formed here, not
                        // hoisted out of the search loop (where it would
                        // sit in a spilled register pair)
                        int ln = lane;
                        asm volatile("" : "+v"(ln));
                        ws[ln] = v;
                    }
                    if (lane == 0) a.order_key[q] = idx + 1;
                    return hops;
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
        return hops;
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
        rerank_rows<STORE, G, CH, pair_rows<STORE, CH, AK>()>(a.f32, a.f32_stride, s.cid, s.cd2, rk, qr, qv, a.d);
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
        ids_out[lane] = ok ? (int32_t)(s.idf[lane] & kIdMask) : -1;
        dists_out[lane] = ok ? __uint_as_float((uint32_t)s.key[lane]) : __builtin_inff();
    }
    int cntv = __popcll(ballot64(ok));
    if (lane == 0) {
        *count_out = cntv;
        if (a.stats) {
            a.stats[q * 4 + 0] = hops;
            a.stats[q * 4 + 1] = ndist;
            a.stats[q * 4 + 2] = nattr;
            a.stats[q * 4 + 3] = lhat;
        }
    }
    return hops;
}

// WPE: occupancy target (waves per SIMD) the register allocator works to.
// One workgroup of one wave per query; perm (when given) is the launch order.
template <int STORE, int G, int CH, int WPE, int SL, int AK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void search_kernel(SearchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t q = a.perm ? (int64_t)a.perm[blockIdx.x] : (int64_t)blockIdx.x;
    const FilterRecord f = a.rec[q];
    // TABLE filters: the distance table sits table_off bytes after the record
    const uint8_t *tab = f.type == F_TABLE ? reinterpret_cast<const uint8_t *>(a.rec + q) + f.table_off : nullptr;
    const int hops = search_query<STORE, G, CH, SL, AK>(a, q, f, tab, a.Q + q * a.d, a.ids + q * a.k,
                                                        a.dists + q * a.k, a.count + q, smem);
    if (a.order_stats && threadIdx.x == 0) {  // what the next ordered launches rank classes by
        const int c = sel_kind(f.type) * kSelClasses + sel_class(f.sel_feature);
        atomicAdd(a.order_stats + 2 * c, (unsigned long long)hops);
        atomicAdd(a.order_stats + 2 * c + 1, 1ull);
    }
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

// The kernel of a family (a struct whose template member get<STORE, G, CH,
// WPE, SL, AK>() names one instantiation) for a row layout: chunks of 16
// bytes per lane, 4 lanes for rows of up to 384 bytes (1..6 chunks), 8 lanes
// for rows of 512 (4), 16 lanes for wider rows padded to 256 bytes (3..8).
template <class Fam, int STORE, int G, int WPE, int SL, int AK>
typename Fam::Fn family_for_ch(int ch)
{
    if (G == 4 && ch >= 1 && ch <= 6) {
        switch (ch) {
        case 1: return Fam::template get<STORE, G, 1, WPE, SL, AK>();
        case 2: return Fam::template get<STORE, G, 2, WPE, SL, AK>();
        case 3: return Fam::template get<STORE, G, 3, WPE, SL, AK>();
        case 4: return Fam::template get<STORE, G, 4, WPE, SL, AK>();
        case 5: return Fam::template get<STORE, G, 5, WPE, SL, AK>();
        case 6: return Fam::template get<STORE, G, 6, WPE, SL, AK>();
        }
    }
    if (G == 8 && ch == 4) return Fam::template get<STORE, G, 4, WPE, SL, AK>();
    if (G == 16) {
        switch (ch) {
        case 3: return Fam::template get<STORE, G, 3, WPE, SL, AK>();
        case 4: return Fam::template get<STORE, G, 4, WPE, SL, AK>();
        case 5: return Fam::template get<STORE, G, 5, WPE, SL, AK>();
        case 6: return Fam::template get<STORE, G, 6, WPE, SL, AK>();
        case 7: return Fam::template get<STORE, G, 7, WPE, SL, AK>();
        case 8: return Fam::template get<STORE, G, 8, WPE, SL, AK>();
        }
    }
    return nullptr;
}

template <class Fam, int WPE, int SL, int AK>
typename Fam::Fn family_pick_sl(int store, int G, int ch)
{
    if (store == JAG_STORE_F32)
        return G == 4   ? family_for_ch<Fam, JAG_STORE_F32, 4, WPE, SL, AK>(ch)
               : G == 8 ? family_for_ch<Fam, JAG_STORE_F32, 8, WPE, SL, AK>(ch)
                        : family_for_ch<Fam, JAG_STORE_F32, 16, WPE, SL, AK>(ch);
    if (store == JAG_STORE_BF16)
        return G == 4   ? family_for_ch<Fam, JAG_STORE_BF16, 4, WPE, SL, AK>(ch)
               : G == 8 ? family_for_ch<Fam, JAG_STORE_BF16, 8, WPE, SL, AK>(ch)
                        : family_for_ch<Fam, JAG_STORE_BF16, 16, WPE, SL, AK>(ch);
    return G == 4   ? family_for_ch<Fam, JAG_STORE_FP8_E4M3, 4, WPE, SL, AK>(ch)
           : G == 8 ? family_for_ch<Fam, JAG_STORE_FP8_E4M3, 8, WPE, SL, AK>(ch)
                    : family_for_ch<Fam, JAG_STORE_FP8_E4M3, 16, WPE, SL, AK>(ch);
}

// All searches use the build for 5 waves per SIMD (at most 96 VGPRs; the
// allocator spills 20-60 bytes per lane to scratch): on the range workload
// 8-12 % faster than the 4-wave build (100-128 VGPRs, no scratch) for fixed
// beams, and 7-10 % faster for two-pass learned search with a 64-entry
// warm-up list.  (With a 128-entry warm-up the 4-wave build had been faster
// for learned search.)
constexpr int kWavesPerSimd = 5;


}  // namespace
}  // namespace jag

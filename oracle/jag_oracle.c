/*
 * jag_oracle.c -- plain CPU reference for Joint Attribute Graph (JAG) search.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  The product
 * library never links, loads or calls it, and the two share no code.
 *
 * Everything here is written for a reader holding the paper, not for speed:
 *   - filter distances dist_F and attribute distances dist_A: Section 3.1
 *     (the four worked examples: equality, range, subset, Boolean)
 *   - capped attribute distance and the lexicographic comparators D_A^t and
 *     D_F: Section 3.2
 *   - GreedySearch (Algorithm 1) and Query (Algorithm 2)
 *   - Insert (Algorithm 3) and JointRobustPrune (Algorithm 4), with the two
 *     implementation notes of Appendix D.3 and the per-point quantile
 *     thresholds of Appendix D.3
 *   - exact filtered k-NN ("Pre-Filtering", Appendix D.4) as ground truth
 *   - BF16 / FP8-E4M3 encoders written from the format definitions, and a
 *     16-64-64-1 ReLU network in FP64 (forward + backward) for the learned
 *     beam predictor; the paper does not describe either.
 *
 * Floating point: every vector distance is a sequential FP64 sum of squared
 * differences of the FP32 inputs.  Searches additionally report the smallest
 * relative gap between two keys whose order decided the search trajectory
 * ("margin"), so a test can tell which results an FP32 implementation must
 * reproduce exactly.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_F_LABEL 0
#define OR_F_RANGE 1
#define OR_F_SUBSET 2
#define OR_F_BOOLEAN 3
#define OR_F_TABLE 4

#define OR_KIND_SCALAR 0
#define OR_KIND_LABELS 1
#define OR_KIND_LABELS_WEIGHTED 2
/* flag on a build entry's kind: a Weight-JAG entry (Section 3.4) whose
 * comparator is w * dist_A + dist, with w = multiplier * h_p (below) */
#define OR_WEIGHT_ENTRY 0x100

/* dist_F of an item against a filter that no attribute can satisfy */
#define OR_UNSAT 4294967295.0

typedef struct {
    int64_t n;
    const int32_t *scalar; /* [n] or NULL */
    const int64_t *loff;   /* [n+1] or NULL */
    const int32_t *lab;    /* label sets, each row sorted */
    const double *lw;      /* per-label weight log(1/p_l), for OR_KIND_LABELS_WEIGHTED */
    double lw_c;           /* the constant C of the weighted distance */
} or_attrs;

typedef struct {
    int32_t type, label, lo, hi, off, len;
} or_filter;

/* ------------------------------------------------------------------ */
/* Section 3.1: filter and attribute distances                        */
/* ------------------------------------------------------------------ */

static int item_has(const or_attrs *A, int64_t i, int32_t l)
{
    for (int64_t j = A->loff[i]; j < A->loff[i + 1]; j++)
        if (A->lab[j] == l) return 1;
    return 0;
}

/* Is literal `lit` (label, or ~label for "label absent") true for item i? */
static int literal_true(const or_attrs *A, int64_t i, int32_t lit)
{
    if (lit >= 0) return item_has(A, i, lit);
    return !item_has(A, i, ~lit);
}

/*
 * dist_F(a_i, f).
 *  Equality/label: 0 if the item carries the label, else 1.
 *  Range: f_min - a below the range, a - f_max above it, 0 inside (inclusive).
 *  Subset: |f \ a|, the number of required labels the item lacks.
 *  Boolean: the fewest label flips that make f true.  f is given in
 *  disjunctive normal form; a clause needs each of its distinct literals,
 *  so its cost is the number of its distinct literals that are false, and
 *  f costs the cheapest clause.  A clause holding a literal and its
 *  negation can never be satisfied and is skipped.
 *  Table: a general Boolean function of nvar labels given by its truth
 *  table; the item's assignment x has bit v set when it holds label var_v,
 *  and the distance is the least Hamming distance from x to an assignment
 *  on which the function is true (Section 3.1's definition, by brute force
 *  over all 2^nvar assignments).
 */
static double table_dist(const or_attrs *A, int64_t i, const or_filter *f, const int32_t *pool)
{
    const int32_t *p = pool + f->off;
    int32_t nv = p[0];
    const int32_t *vars = p + 1;
    const uint32_t *w = (const uint32_t *)(p + 1 + nv);
    uint32_t x = 0;
    for (int32_t v = 0; v < nv; v++)
        if (item_has(A, i, vars[v])) x |= 1u << v;
    double best = OR_UNSAT;
    for (uint32_t y = 0; y < (1u << nv); y++) {
        if (!((w[y >> 5] >> (y & 31)) & 1u)) continue;
        double h = (double)__builtin_popcount(x ^ y);
        if (h < best) best = h;
    }
    return best;
}

/* g(a_i, f) of Section 2 for a table filter: the function's value on the item. */
static int table_true(const or_attrs *A, int64_t i, const or_filter *f, const int32_t *pool)
{
    const int32_t *p = pool + f->off;
    int32_t nv = p[0];
    const uint32_t *w = (const uint32_t *)(p + 1 + nv);
    uint32_t x = 0;
    for (int32_t v = 0; v < nv; v++)
        if (item_has(A, i, p[1 + v])) x |= 1u << v;
    return (int)((w[x >> 5] >> (x & 31)) & 1u);
}

static double dist_f(const or_attrs *A, int64_t i, const or_filter *f, const int32_t *pool)
{
    if (f->type == OR_F_TABLE) return table_dist(A, i, f, pool);
    if (f->type == OR_F_LABEL) {
        return item_has(A, i, f->label) ? 0.0 : 1.0;
    }
    if (f->type == OR_F_RANGE) {
        double a = (double)A->scalar[i];
        if (a < (double)f->lo) return (double)f->lo - a;
        if (a > (double)f->hi) return a - (double)f->hi;
        return 0.0;
    }
    if (f->type == OR_F_SUBSET) {
        double missing = 0.0;
        for (int32_t j = 0; j < f->len; j++)
            if (!item_has(A, i, pool[f->off + j])) missing += 1.0;
        return missing;
    }
    if (f->type == OR_F_BOOLEAN) {
        const int32_t *p = pool + f->off;
        int32_t ncl = *p++;
        double best = OR_UNSAT;
        for (int32_t c = 0; c < ncl; c++) {
            int32_t nlit = *p++;
            const int32_t *lit = p;
            p += nlit;
            int contradictory = 0;
            double cost = 0.0;
            for (int32_t a = 0; a < nlit; a++) {
                int dup = 0;
                for (int32_t b = 0; b < a; b++) {
                    if (lit[b] == lit[a]) dup = 1;
                    if (lit[b] == ~lit[a]) contradictory = 1;
                }
                if (dup) continue;
                if (!literal_true(A, i, lit[a])) cost += 1.0;
            }
            if (!contradictory && cost < best) best = cost;
        }
        return best;
    }
    return OR_UNSAT;
}

/*
 * Label weights of the frequency-weighted label distance (App. D.3, the
 * variant the paper uses for label-heavy datasets): p_l = fraction of items
 * holding label l, weight log(1/p_l); C = the largest total weight of one
 * item's labels, so that C - (weight of any shared set) >= 0.  Returns a
 * malloc'd array indexed by label (0 for labels nobody holds).
 */
static double *label_weights(const or_attrs *A, double *c_out)
{
    int32_t vocab = 0;
    for (int64_t x = 0; x < A->loff[A->n]; x++)
        if (A->lab[x] + 1 > vocab) vocab = A->lab[x] + 1;
    double *cnt = calloc((size_t)(vocab > 0 ? vocab : 1), sizeof(double));
    for (int64_t x = 0; x < A->loff[A->n]; x++) cnt[A->lab[x]] += 1.0;
    for (int32_t l = 0; l < vocab; l++) cnt[l] = cnt[l] > 0.0 ? log((double)A->n / cnt[l]) : 0.0;
    double c = 0.0;
    for (int64_t i = 0; i < A->n; i++) {
        double t = 0.0;
        for (int64_t x = A->loff[i]; x < A->loff[i + 1]; x++) t += cnt[A->lab[x]];
        if (t > c) c = t;
    }
    *c_out = c;
    return cnt;
}

/*
 * dist_A: |a1 - a2| for scalars; |a1 XOR a2| (symmetric difference) for label
 * sets; C - sum of log(1/p_l) over shared labels l for weighted label sets.
 */
static double dist_a(const or_attrs *A, int kind, int64_t i, int64_t j)
{
    if (kind == OR_KIND_SCALAR) return fabs((double)A->scalar[i] - (double)A->scalar[j]);
    if (kind == OR_KIND_LABELS_WEIGHTED) {
        double shared = 0.0;
        for (int64_t x = A->loff[i]; x < A->loff[i + 1]; x++)
            if (item_has(A, j, A->lab[x])) shared += A->lw[A->lab[x]];
        return A->lw_c - shared;
    }
    double common = 0.0;
    for (int64_t x = A->loff[i]; x < A->loff[i + 1]; x++)
        if (item_has(A, j, A->lab[x])) common += 1.0;
    double ni = (double)(A->loff[i + 1] - A->loff[i]);
    double nj = (double)(A->loff[j + 1] - A->loff[j]);
    return ni + nj - 2.0 * common;
}

/* Capped attribute distance dist_A(a1, a2; t) = max(dist_A - t, 0), Section 3.2. */
static double dist_a_capped(const or_attrs *A, int kind, int64_t i, int64_t j, double t)
{
    if (isinf(t)) return 0.0;
    double v = dist_a(A, kind, i, j) - t;
    return v > 0.0 ? v : 0.0;
}

/* Squared Euclidean distance in FP64, summed in index order. */
static double sqdist(const float *x, const float *y, int32_t d)
{
    double s = 0.0;
    for (int32_t k = 0; k < d; k++) {
        double t = (double)x[k] - (double)y[k];
        s += t * t;
    }
    return s;
}

/*
 * Optional FP32 evaluation order ("contract mode").  A row of d values is
 * split over G lanes: lane s takes the EPC consecutive elements of chunks
 * j*G + s, j = 0..CH-1, and folds (x - y)^2 of each into its FP32 partial
 * sum with one fused multiply-add, in chunk then element order (elements
 * at or beyond d add nothing); the G partial sums are then added pairwise,
 * neighbours first: ((p0 + p1) + (p2 + p3)) + ...  An implementation that
 * evaluates distances in this documented order obtains the same FP32 value
 * bit for bit, so its search can be compared with this one id for id with
 * no tolerance.  The FP64 sum above remains the reference for accuracy.
 */
typedef struct {
    int32_t G, EPC, CH;
} or_contract;

static double sqdist_contract(const float *x, const float *y, int32_t d, const or_contract *c)
{
    float part[64];
    for (int32_t s = 0; s < c->G; s++) {
        float acc = 0.0f;
        for (int32_t j = 0; j < c->CH; j++)
            for (int32_t e = 0; e < c->EPC; e++) {
                int32_t i = (j * c->G + s) * c->EPC + e;
                if (i < d) {
                    float t = x[i] - y[i];
                    acc = fmaf(t, t, acc);
                }
            }
        part[s] = acc;
    }
    for (int32_t m = 1; m < c->G; m <<= 1)
        for (int32_t s = 0; s < c->G; s += 2 * m) part[s] = part[s] + part[s + m];
    return (double)part[0];
}

static double search_dist(const float *x, const float *y, int32_t d, const or_contract *c)
{
    return c ? sqdist_contract(x, y, d, c) : sqdist(x, y, d);
}

/* ------------------------------------------------------------------ */
/* Lexicographic keys (Section 3.2), ties broken by id                */
/* ------------------------------------------------------------------ */

typedef struct {
    double f;  /* first component: dist_F or capped dist_A */
    double d2; /* squared vector distance (order-equivalent to dist) */
    int32_t id;
    int32_t pad;
} or_key;

static int key_less(const or_key *a, const or_key *b)
{
    if (a->f != b->f) return a->f < b->f;
    if (a->d2 != b->d2) return a->d2 < b->d2;
    return a->id < b->id;
}

static int key_cmp(const void *pa, const void *pb)
{
    const or_key *a = pa, *b = pb;
    if (key_less(a, b)) return -1;
    if (key_less(b, a)) return 1;
    return 0;
}

/* Relative gap between two keys that an FP32 evaluation could swap. */
static double key_gap(const or_key *a, const or_key *b)
{
    if (a->f != b->f) return INFINITY;
    double m = fmax(fabs(a->d2), fabs(b->d2));
    if (m == 0.0) return 0.0;
    return fabs(b->d2 - a->d2) / m;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: GreedySearch                                          */
/* ------------------------------------------------------------------ */

typedef double (*first_fn)(const void *ctx, int32_t u);

typedef struct {
    const int32_t *adj; /* [n][R], -1 = no edge */
    int32_t R;
    int64_t n;
    int32_t entry;
    const float *base; /* vectors the search ranks by, [n][d] */
    int32_t d;
    const or_contract *contract; /* NULL: FP64 distances */
} or_graph;

typedef struct { /* learned beam predictor (not in the paper) */
    int32_t enabled;
    const float *params; /* 5313 values: W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3 */
    float delta;         /* offset added to the predicted ladder index */
    float rho;           /* hop cap = ceil(rho * Lhat) */
    int32_t nladder;
    const int32_t *ladder;
    float sel_feature; /* log2(selectivity estimate) / 16, computed by the caller */
    int32_t ftype;     /* filter type, for the one-hot features */
} or_learned;

typedef struct {
    int32_t hops;
    int32_t dc;
    double margin;
    double y;
    int32_t lhat;
    double feat[16]; /* predictor features at the prediction point (NaN if none) */
} or_trace;

/* per-thread membership stamps for L and V (sized n) */
typedef struct {
    int32_t *inL;
    int32_t *inV;
    int32_t stamp;
} or_scratch;

static void scratch_init(or_scratch *s, int64_t n)
{
    s->inL = calloc((size_t)n, sizeof(int32_t));
    s->inV = calloc((size_t)n, sizeof(int32_t));
    s->stamp = 0;
}

static void scratch_free(or_scratch *s)
{
    free(s->inL);
    free(s->inV);
}

static double relu(double v) { return v > 0.0 ? v : 0.0; }

/* y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 */
static double mlp_forward(const float *P, const double *x)
{
    const float *W1 = P, *b1 = P + 1024, *W2 = P + 1088, *b2 = P + 5184, *w3 = P + 5248,
                *b3 = P + 5312;
    double h1[64], h2[64];
    for (int j = 0; j < 64; j++) {
        double s = b1[j];
        for (int i = 0; i < 16; i++) s += (double)W1[j * 16 + i] * x[i];
        h1[j] = relu(s);
    }
    for (int j = 0; j < 64; j++) {
        double s = b2[j];
        for (int i = 0; i < 64; i++) s += (double)W2[j * 64 + i] * h1[i];
        h2[j] = relu(s);
    }
    double y = b3[0];
    for (int j = 0; j < 64; j++) y += (double)w3[j] * h2[j];
    return y;
}

static double squash(double v) { return v / (v + 1.0); }

/*
 * Predictor features after the fourth expansion (our definition; the paper
 * has no predictor).  e[0..3] are the keys of the four expanded vertices in
 * expansion order, L the sorted candidate list.
 */
static void learned_features(const or_learned *M, const or_key *e, const or_key *L, int32_t cnt,
                             double *x)
{
    for (int i = 0; i < 16; i++) x[i] = 0.0;
    x[M->ftype] = 1.0;
    x[4] = (double)M->sel_feature;
    double base = e[0].d2 > 1e-30 ? e[0].d2 : 1e-30;
    x[5] = e[1].d2 / base;
    x[6] = e[2].d2 / base;
    x[7] = e[3].d2 / base;
    x[8] = L[0].d2 / base;
    for (int j = 0; j < 4; j++) x[9 + j] = squash(e[j].f);
    x[13] = squash(L[0].f);
    int32_t valid = 0;
    for (int32_t j = 0; j < cnt; j++)
        if (L[j].f == 0.0) valid++;
    x[14] = (double)valid / (double)cnt;
    x[15] = 1.0;
}

/*
 * GreedySearch(G, x, k, l_s, D): beam search from the fixed entry vertex.
 * The candidate list L is kept sorted by D(x, .); V is the set of expanded
 * vertices.  While L \ V is not empty, the best unexpanded vertex is
 * expanded, each out-neighbour not already in L is added, and L is cut back
 * to its l_s best entries.
 *
 * Writes the final sorted L (up to l_s entries) into L_out and returns its
 * size; expanded vertices (in order) go to V_out when non-NULL.
 */
static int32_t greedy_search(const or_graph *G, const float *x, first_fn first, const void *ctx,
                             int32_t ls, or_scratch *S, or_key *L_out, int32_t *V_out,
                             int32_t *nV_out, const or_learned *M, or_trace *tr, int32_t track)
{
    int32_t cap = ls;
    if (M && M->enabled) {
        for (int32_t i = 0; i < M->nladder; i++)
            if (M->ladder[i] > cap) cap = M->ladder[i];
    }
    or_key *L = malloc(sizeof(or_key) * (size_t)(cap + G->R + 1));
    int32_t nL = 0, nV = 0, hops = 0, dc = 0;
    int32_t hopcap = INT32_MAX;
    double margin = INFINITY;
    or_key ex[4];
    int32_t cur_ls = (M && M->enabled) ? cap : ls;
    if (tr) {
        tr->y = NAN;
        tr->lhat = -1;
        for (int i = 0; i < 16; i++) tr->feat[i] = NAN;
    }
    S->stamp++;
    int32_t st = S->stamp;

    /* L <- {s}, V <- {} */
    L[0].id = G->entry;
    L[0].f = first(ctx, G->entry);
    L[0].d2 = search_dist(x, G->base + (size_t)G->entry * G->d, G->d, G->contract);
    dc++;
    S->inL[G->entry] = st;
    nL = 1;

    for (;;) {
        /* p <- argmin over L \ V (L is sorted, so the first unexpanded entry) */
        int32_t pi = -1, pnext = -1;
        for (int32_t j = 0; j < nL; j++) {
            if (S->inV[L[j].id] == st) continue;
            if (pi < 0) pi = j;
            else {
                pnext = j;
                break;
            }
        }
        if (pi < 0) break;
        if (hops >= hopcap) break;
        if (track && pnext >= 0) margin = fmin(margin, key_gap(&L[pi], &L[pnext]));
        or_key p = L[pi];
        S->inV[p.id] = st; /* V <- V u {p} */
        if (V_out) V_out[nV] = p.id;
        nV++;
        if (hops < 4) ex[hops] = p;
        hops++;
        /* for each out-neighbour u of p not in L: L <- L u {u} */
        const int32_t *row = G->adj + (size_t)p.id * G->R;
        for (int32_t j = 0; j < G->R; j++) {
            int32_t u = row[j];
            if (u < 0) continue;
            if (S->inL[u] == st) continue;
            or_key c;
            c.id = u;
            c.f = first(ctx, u);
            c.d2 = search_dist(x, G->base + (size_t)u * G->d, G->d, G->contract);
            dc++;
            L[nL++] = c;
            S->inL[u] = st;
        }
        /* keep the best l_s entries of L */
        qsort(L, (size_t)nL, sizeof(or_key), key_cmp);
        if (nL > cur_ls) {
            if (track) margin = fmin(margin, key_gap(&L[cur_ls - 1], &L[cur_ls]));
            for (int32_t j = cur_ls; j < nL; j++) S->inL[L[j].id] = 0;
            nL = cur_ls;
        }
        /* learned beam: after the fourth expansion, predict l_s and a hop cap */
        if (M && M->enabled && hops == 4) {
            double feat[16];
            learned_features(M, ex, L, nL, feat);
            double y = mlp_forward(M->params, feat);
            double z = y + (double)M->delta;
            double c = ceil(z);
            int32_t idx = c < 0.0 ? 0 : (c > (double)(M->nladder - 1) ? M->nladder - 1 : (int32_t)c);
            int32_t lhat = M->ladder[idx];
            if (tr) {
                tr->y = y;
                tr->lhat = lhat;
                memcpy(tr->feat, feat, sizeof(feat));
            }
            float capf = ceilf(M->rho * (float)lhat);
            hopcap = capf >= 2147483647.0f ? INT32_MAX : (int32_t)capf;
            if (hopcap < 4) hopcap = 4;
            if (nL > lhat) {
                if (track) margin = fmin(margin, key_gap(&L[lhat - 1], &L[lhat]));
                for (int32_t j = lhat; j < nL; j++) S->inL[L[j].id] = 0;
                nL = lhat;
            }
            cur_ls = lhat;
        }
    }
    memcpy(L_out, L, sizeof(or_key) * (size_t)nL);
    if (nV_out) *nV_out = nV;
    if (tr) {
        tr->hops = hops;
        tr->dc = dc;
        tr->margin = margin;
    }
    free(L);
    return nL;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2: Query (comparator D_F)                                */
/* ------------------------------------------------------------------ */

typedef struct {
    const or_attrs *A;
    const or_filter *f;
    const int32_t *pool;
} df_ctx;

static double first_df(const void *ctx, int32_t u)
{
    const df_ctx *c = ctx;
    return dist_f(c->A, u, c->f, c->pool);
}

typedef struct {
    or_graph G;
    or_attrs A;
    const float *Q;
    const or_filter *F;
    const int32_t *pool;
    const float *rerank; /* FP32 vectors for the final rescoring, or NULL */
    int32_t rerank_mult;
    const or_contract *rerank_contract; /* NULL: FP64 distances */
    int32_t ls, k;
    const float *sel_feature; /* [nq] */
    or_learned M;
    /* outputs */
    int32_t *ids;
    double *d2;
    int32_t *count;
    int32_t *hops, *dc, *lhat;
    double *margin, *y;
    double *feat; /* [nq][16] or NULL */
    int64_t q0, q1;
} search_job;

static void query_one(search_job *J, int64_t q, or_scratch *S)
{
    const float *x = J->Q + (size_t)q * J->G.d;
    df_ctx ctx = {&J->A, &J->F[q], J->pool};
    or_learned M = J->M;
    M.ftype = J->F[q].type;
    M.sel_feature = J->sel_feature ? J->sel_feature[q] : 0.0f;
    int32_t cap = J->ls;
    if (M.enabled)
        for (int32_t i = 0; i < M.nladder; i++)
            if (M.ladder[i] > cap) cap = M.ladder[i];
    or_key *L = malloc(sizeof(or_key) * (size_t)(cap + J->G.R + 1));
    or_trace tr;
    int32_t nL = greedy_search(&J->G, x, first_df, &ctx, J->ls, S, L, NULL, NULL,
                               M.enabled ? &M : NULL, &tr, 1);
    double margin = tr.margin;
    /* optional rerank: rescore the best rerank_mult*k entries of L */
    int32_t nres = nL;
    if (J->rerank) {
        int32_t rk = J->rerank_mult * J->k;
        if (nL > rk) {
            margin = fmin(margin, key_gap(&L[rk - 1], &L[rk]));
            nres = rk;
        }
        for (int32_t j = 0; j < nres; j++)
            L[j].d2 = search_dist(x, J->rerank + (size_t)L[j].id * J->G.d, J->G.d, J->rerank_contract);
        qsort(L, (size_t)nres, sizeof(or_key), key_cmp);
    }
    /* top-k of V by D_F equals the top-k of the final L; only valid ids are returned */
    int32_t cnt = 0;
    for (int32_t j = 0; j < nres && cnt < J->k; j++) {
        if (L[j].f != 0.0) break;
        J->ids[q * J->k + cnt] = L[j].id;
        J->d2[q * J->k + cnt] = L[j].d2;
        cnt++;
    }
    for (int32_t j = 0; j + 1 < nres && j < J->k; j++) margin = fmin(margin, key_gap(&L[j], &L[j + 1]));
    for (int32_t j = cnt; j < J->k; j++) {
        J->ids[q * J->k + j] = -1;
        J->d2[q * J->k + j] = INFINITY;
    }
    J->count[q] = cnt;
    if (J->hops) J->hops[q] = tr.hops;
    if (J->dc) J->dc[q] = tr.dc;
    if (J->margin) J->margin[q] = margin;
    if (J->y) J->y[q] = tr.y;
    if (J->lhat) J->lhat[q] = tr.lhat;
    if (J->feat) memcpy(J->feat + q * 16, tr.feat, sizeof(tr.feat));
    free(L);
}

static void *search_worker(void *arg)
{
    search_job *J = arg;
    or_scratch S;
    scratch_init(&S, J->G.n);
    for (int64_t q = J->q0; q < J->q1; q++) query_one(J, q, &S);
    scratch_free(&S);
    return NULL;
}

static void run_jobs(void *(*fn)(void *), void *jobs, size_t jsz, int32_t nthreads)
{
    pthread_t th[256];
    if (nthreads > 256) nthreads = 256;
    for (int32_t t = 0; t < nthreads; t++)
        pthread_create(&th[t], NULL, fn, (char *)jobs + (size_t)t * jsz);
    for (int32_t t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
}

/*
 * Batched Query.  Queries are independent, so they are spread over
 * `nthreads` threads; each query runs the sequential algorithm above.
 * learned_params == NULL disables the predictor; with it, feat (optional,
 * [nq][16]) receives each query's features at the prediction point (NaN
 * for a query that ended before its fourth expansion).  contract (optional)
 * = {G, EPC, CH} of the ranking vectors then of the rescoring vectors:
 * distances in that FP32 order instead of FP64 (see sqdist_contract).
 */
int or_search(int64_t n, int32_t d, const float *base, const int32_t *adj, int32_t R,
              int32_t entry, const int32_t *scalar, const int64_t *loff, const int32_t *lab,
              int64_t nq, const float *Q, const int32_t *F, const int32_t *pool, int32_t ls,
              int32_t k, const float *rerank, int32_t rerank_mult, const float *learned_params,
              float delta, float rho, int32_t nladder, const int32_t *ladder,
              const float *sel_feature, int32_t nthreads, int32_t *ids, double *d2, int32_t *count,
              int32_t *hops, int32_t *dc, double *margin, double *y, int32_t *lhat,
              double *feat, const int32_t *contract)
{
    or_contract cs, cr;
    if (contract) {
        cs = (or_contract){contract[0], contract[1], contract[2]};
        cr = (or_contract){contract[3], contract[4], contract[5]};
    }
    if (nthreads < 1) nthreads = 1;
    if (nq < nthreads) nthreads = (int32_t)(nq > 0 ? nq : 1);
    search_job *jobs = calloc((size_t)nthreads, sizeof(search_job));
    for (int32_t t = 0; t < nthreads; t++) {
        search_job *J = &jobs[t];
        J->G = (or_graph){adj, R, n, entry, base, d, contract ? &cs : NULL};
        J->rerank_contract = contract ? &cr : NULL;
        J->A = (or_attrs){n, scalar, loff, lab, NULL, 0.0};
        J->Q = Q;
        J->F = (const or_filter *)F;
        J->pool = pool;
        J->rerank = rerank;
        J->rerank_mult = rerank_mult;
        J->ls = ls;
        J->k = k;
        J->sel_feature = sel_feature;
        J->M = (or_learned){learned_params != NULL, learned_params, delta, rho, nladder, ladder,
                            0.0f, 0};
        J->ids = ids;
        J->d2 = d2;
        J->count = count;
        J->hops = hops;
        J->dc = dc;
        J->margin = margin;
        J->y = y;
        J->lhat = lhat;
        J->feat = feat;
        J->q0 = nq * t / nthreads;
        J->q1 = nq * (t + 1) / nthreads;
    }
    run_jobs(search_worker, jobs, sizeof(search_job), nthreads);
    free(jobs);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Exact filtered k-NN: Pre-Filtering (Appendix D.4), FP64            */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int32_t d;
    const float *X;
    or_attrs A;
    const float *Q;
    const or_filter *F;
    const int32_t *pool;
    int32_t k;
    int32_t *ids;
    double *d2;
    int64_t *nvalid;
    int64_t q0, q1;
} bf_job;

static void *bf_worker(void *arg)
{
    bf_job *J = arg;
    or_key *best = malloc(sizeof(or_key) * (size_t)(J->k + 1));
    for (int64_t q = J->q0; q < J->q1; q++) {
        const float *x = J->Q + (size_t)q * J->d;
        int32_t nb = 0;
        int64_t valid = 0;
        for (int64_t i = 0; i < J->n; i++) {
            // validity g = 1: for a table filter read the function's value
            // directly (its distance needs a pass over all assignments)
            const or_filter *fq = &J->F[q];
            if (fq->type == OR_F_TABLE ? !table_true(&J->A, i, fq, J->pool)
                                       : dist_f(&J->A, i, fq, J->pool) != 0.0)
                continue;
            valid++;
            or_key c = {0.0, sqdist(x, J->X + (size_t)i * J->d, J->d), (int32_t)i, 0};
            /* keep the k smallest (d2, id) in a sorted array */
            if (nb == J->k && !key_less(&c, &best[nb - 1])) continue;
            int32_t pos = nb < J->k ? nb++ : J->k - 1;
            while (pos > 0 && key_less(&c, &best[pos - 1])) {
                best[pos] = best[pos - 1];
                pos--;
            }
            best[pos] = c;
        }
        for (int32_t j = 0; j < J->k; j++) {
            J->ids[q * J->k + j] = j < nb ? best[j].id : -1;
            J->d2[q * J->k + j] = j < nb ? best[j].d2 : INFINITY;
        }
        J->nvalid[q] = valid;
    }
    free(best);
    return NULL;
}

int or_bruteforce(int64_t n, int32_t d, const float *X, const int32_t *scalar,
                  const int64_t *loff, const int32_t *lab, int64_t nq, const float *Q,
                  const int32_t *F, const int32_t *pool, int32_t k, int32_t nthreads,
                  int32_t *ids, double *d2, int64_t *nvalid)
{
    if (nthreads < 1) nthreads = 1;
    if (nq < nthreads) nthreads = (int32_t)(nq > 0 ? nq : 1);
    bf_job *jobs = calloc((size_t)nthreads, sizeof(bf_job));
    for (int32_t t = 0; t < nthreads; t++) {
        jobs[t] = (bf_job){n, d, X, {n, scalar, loff, lab}, Q, (const or_filter *)F, pool, k,
                           ids, d2, nvalid, nq * t / nthreads, nq * (t + 1) / nthreads};
    }
    run_jobs(bf_worker, jobs, sizeof(bf_job), nthreads);
    free(jobs);
    return 0;
}

/*
 * Selectivity estimate of each filter (the paper has none; the learned
 * search's feature 4): the fraction of items the filter passes, exact for
 * label and range filters (a count), and for subset, DNF and truth-table
 * filters the probability that an item passes when each label is held
 * independently with its observed frequency: every assignment of the
 * filter's distinct labels is enumerated, weighted by the product of the
 * frequencies, and counted when the filter holds on it.
 */
void or_selectivity(int64_t n, const int32_t *scalar, const int64_t *loff, const int32_t *lab,
                    int64_t nq, const int32_t *F, const int32_t *pool, double *out)
{
    or_attrs A = {n, scalar, loff, lab, NULL, 0.0};
    int32_t vocab = 0;
    if (loff)
        for (int64_t x = 0; x < loff[n]; x++)
            if (lab[x] + 1 > vocab) vocab = lab[x] + 1;
    double *freq = calloc((size_t)(vocab > 0 ? vocab : 1), sizeof(double));
    if (loff)
        for (int64_t x = 0; x < loff[n]; x++) freq[lab[x]] += 1.0 / (double)n;
    for (int64_t q = 0; q < nq; q++) {
        const or_filter *f = (const or_filter *)F + q;
        if (f->type == OR_F_RANGE || f->type == OR_F_LABEL) {
            int64_t c = 0;
            for (int64_t i = 0; i < n; i++) c += dist_f(&A, i, f, pool) == 0.0;
            out[q] = (double)c / (double)n;
            continue;
        }
        /* the filter's distinct labels v_0..v_{m-1} */
        int32_t vars[32], m = 0;
        const int32_t *p = pool + f->off;
        int32_t nlab = 0;
        const int32_t *labs = NULL;
        if (f->type == OR_F_SUBSET) {
            labs = p;
            nlab = f->len;
        } else if (f->type == OR_F_TABLE) {
            labs = p + 1;
            nlab = p[0];
        }
        for (int32_t j = 0; j < nlab; j++) {
            int dup = 0;
            for (int32_t x = 0; x < m; x++) dup |= vars[x] == labs[j];
            if (!dup) vars[m++] = labs[j];
        }
        if (f->type == OR_F_BOOLEAN) {
            int32_t ncl = p[0], pos = 1;
            for (int32_t c = 0; c < ncl; c++) {
                int32_t nl = p[pos++];
                for (int32_t j = 0; j < nl; j++) {
                    int32_t l = p[pos + j] >= 0 ? p[pos + j] : ~p[pos + j];
                    int dup = 0;
                    for (int32_t x = 0; x < m; x++) dup |= vars[x] == l;
                    if (!dup) vars[m++] = l;
                }
                pos += nl;
            }
        }
        /* enumerate assignments: a one-item world holding exactly the labels set in x */
        double total = 0.0;
        int32_t one_lab[32];
        int64_t one_off[2] = {0, 0};
        or_attrs one = {1, NULL, one_off, one_lab, NULL, 0.0};
        for (uint32_t x = 0; x < (1u << m); x++) {
            double pr = 1.0;
            int32_t c = 0;
            for (int32_t v = 0; v < m; v++) {
                if ((x >> v) & 1u) {
                    pr *= freq[vars[v]];
                    one_lab[c++] = vars[v];
                } else
                    pr *= 1.0 - freq[vars[v]];
            }
            one_off[1] = c;
            if (dist_f(&one, 0, f, pool) == 0.0) total += pr;
        }
        out[q] = total;
    }
    free(freq);
}

/* dist_F for a list of (item, filter) pairs; exported for the distance tests */
void or_dist_f_pairs(int64_t n, const int32_t *scalar, const int64_t *loff, const int32_t *lab,
                     int64_t m, const int64_t *items, const int32_t *F, const int32_t *fidx,
                     const int32_t *pool, double *out)
{
    or_attrs A = {n, scalar, loff, lab, NULL, 0.0};
    for (int64_t j = 0; j < m; j++)
        out[j] = dist_f(&A, items[j], (const or_filter *)F + fidx[j], pool);
}

void or_dist_a_pairs(int64_t n, const int32_t *scalar, const int64_t *loff, const int32_t *lab,
                     int32_t kind, int64_t m, const int64_t *i1, const int64_t *i2, double t,
                     double *out)
{
    or_attrs A = {n, scalar, loff, lab, NULL, 0.0};
    double *lw = NULL;
    if (kind == OR_KIND_LABELS_WEIGHTED) A.lw = lw = label_weights(&A, &A.lw_c);
    for (int64_t j = 0; j < m; j++) out[j] = dist_a_capped(&A, kind, i1[j], i2[j], t);
    free(lw);
}

/* ------------------------------------------------------------------ */
/* Algorithms 3 and 4: Insert and JointRobustPrune                     */
/* ------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea, Flood 2014): counter-based 64-bit generator. */
static uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    int64_t n;
    int32_t d, R, lb, nT;
    double alpha;
    const float *X;
    or_attrs A;
    const int32_t *kinds; /* [nT] attribute kind of each threshold */
    double *thr;          /* [n][nT] per-point threshold values */
    int32_t *adj;         /* [n][R] */
    int32_t *deg;         /* [n] */
    int32_t entry;
} build_state;

typedef struct {
    const build_state *B;
    int32_t p;
    int kind;
    double t;
} da_ctx;

/*
 * First component of the build comparator of entry `kind` for base point p:
 * Threshold-JAG, the capped dist_A(a_p, a_v; t) (Section 3.2); Weight-JAG,
 * w * dist_A(a_p, a_v) + dist(x_p, x_v) (Section 3.4), the squared distance
 * then breaking ties.
 */
static double build_first(const build_state *B, int kind, int32_t p, int32_t v, double t, double d2)
{
    if (kind & OR_WEIGHT_ENTRY)
        return t * dist_a(&B->A, kind & 0xFF, p, v) + sqrt(d2);
    return dist_a_capped(&B->A, kind, p, v, t);
}

static double first_da(const void *ctx, int32_t u)
{
    const da_ctx *c = ctx;
    double d2 = (c->kind & OR_WEIGHT_ENTRY)
                    ? sqdist(c->B->X + (size_t)c->p * c->B->d, c->B->X + (size_t)u * c->B->d, c->B->d)
                    : 0.0;
    return build_first(c->B, c->kind, c->p, u, c->t, d2);
}

/* D_A^t(p, v) (or D_A^w) with the base point's value, then id */
static or_key da_key(const build_state *B, int32_t p, int32_t ti, int32_t v)
{
    or_key k;
    k.d2 = sqdist(B->X + (size_t)p * B->d, B->X + (size_t)v * B->d, B->d);
    k.f = build_first(B, B->kinds[ti], p, v, B->thr[(size_t)p * B->nT + ti], k.d2);
    k.id = v;
    k.pad = 0;
    return k;
}

/*
 * JointRobustPrune(G, p, V, R, alpha, T).  One bucket per threshold: the
 * candidates are visited in D_A^t order and v joins the bucket when every
 * vertex u already in it satisfies alpha * dist(u, v) > dist(p, v)
 * (compared on squared distances as alpha^2 d2(u,v) > d2(p,v)).
 * Appendix D.3 notes applied:
 *   - a v already chosen by an earlier bucket joins this bucket without the
 *     alpha test (and then prunes like any member);
 *   - a bucket closes once it holds ceil(0.9 * R / |T|) vertices.
 * The union of the buckets, in bucket order, is cut to R entries.
 * Returns the number of vertices written to out[].
 */
static int32_t joint_robust_prune(const build_state *B, int32_t p, const int32_t *V, int32_t nVc,
                                  int32_t *out)
{
    int32_t nT = B->nT;
    int32_t cap = (9 * B->R + 10 * nT - 1) / (10 * nT);
    double a2 = B->alpha * B->alpha;
    or_key *srt = malloc(sizeof(or_key) * (size_t)(nVc > 0 ? nVc : 1));
    int32_t *bucket = malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *chosen = malloc(sizeof(int32_t) * (size_t)(nT * cap + 1));
    int32_t nchosen = 0;
    for (int32_t ti = 0; ti < nT; ti++) {
        int32_t m = 0;
        for (int32_t j = 0; j < nVc; j++) {
            if (V[j] == p) continue;
            int dup = 0;
            for (int32_t x = 0; x < m; x++)
                if (srt[x].id == V[j]) dup = 1;
            if (!dup) srt[m++] = da_key(B, p, ti, V[j]);
        }
        qsort(srt, (size_t)m, sizeof(or_key), key_cmp);
        int32_t nb = 0;
        for (int32_t j = 0; j < m; j++) {
            int32_t v = srt[j].id;
            int earlier = 0;
            for (int32_t x = 0; x < nchosen; x++)
                if (chosen[x] == v) earlier = 1;
            int keep = 1;
            if (!earlier) {
                for (int32_t x = 0; x < nb; x++) {
                    int32_t u = bucket[x];
                    double duv = sqdist(B->X + (size_t)u * B->d, B->X + (size_t)v * B->d, B->d);
                    if (!(a2 * duv > srt[j].d2)) {
                        keep = 0;
                        break;
                    }
                }
            }
            if (keep) bucket[nb++] = v;
            if (nb >= cap) break;
        }
        for (int32_t x = 0; x < nb; x++) {
            int already = 0;
            for (int32_t y = 0; y < nchosen; y++)
                if (chosen[y] == bucket[x]) already = 1;
            if (!already) chosen[nchosen++] = bucket[x];
        }
    }
    int32_t nout = nchosen < B->R ? nchosen : B->R;
    memcpy(out, chosen, sizeof(int32_t) * (size_t)nout);
    free(srt);
    free(bucket);
    free(chosen);
    return nout;
}

/*
 * Insert(G, p, T, l_b, R, alpha): one GreedySearch per threshold with the
 * comparator D_A^t (the search "query" is p itself, k = 1, beam l_b); the
 * union of the expanded sets, without p, is pruned into p's out-list; then
 * p is added to each chosen neighbour's out-list, and a neighbour whose list
 * grows past R is pruned again with its own thresholds.
 */
static void insert_point(build_state *B, int32_t p, or_scratch *S, or_key *Lbuf, int32_t *Vbuf,
                         int32_t *cand)
{
    or_graph G = {B->adj, B->R, B->n, B->entry, B->X, B->d};
    int32_t ncand = 0;
    for (int32_t ti = 0; ti < B->nT; ti++) {
        da_ctx ctx = {B, p, B->kinds[ti], B->thr[(size_t)p * B->nT + ti]};
        int32_t nV = 0;
        greedy_search(&G, B->X + (size_t)p * B->d, first_da, &ctx, B->lb, S, Lbuf, Vbuf, &nV,
                      NULL, NULL, 0);
        for (int32_t j = 0; j < nV; j++) {
            int32_t v = Vbuf[j];
            if (v == p) continue;
            int dup = 0;
            for (int32_t x = 0; x < ncand; x++)
                if (cand[x] == v) dup = 1;
            if (!dup) cand[ncand++] = v;
        }
    }
    int32_t *row = B->adj + (size_t)p * B->R;
    int32_t nout = joint_robust_prune(B, p, cand, ncand, row);
    for (int32_t j = nout; j < B->R; j++) row[j] = -1;
    B->deg[p] = nout;
    int32_t *tmp = malloc(sizeof(int32_t) * (size_t)(B->R + 1));
    for (int32_t j = 0; j < nout; j++) {
        int32_t v = row[j];
        int32_t *rv = B->adj + (size_t)v * B->R;
        int present = 0;
        for (int32_t x = 0; x < B->deg[v]; x++)
            if (rv[x] == p) present = 1;
        if (present) continue;
        if (B->deg[v] < B->R) {
            rv[B->deg[v]++] = p;
            continue;
        }
        /* |N_out(v)| would exceed R: prune N_out(v) u {p} with v's thresholds */
        memcpy(tmp, rv, sizeof(int32_t) * (size_t)B->deg[v]);
        tmp[B->deg[v]] = p;
        int32_t nv = joint_robust_prune(B, v, tmp, B->deg[v] + 1, rv);
        for (int32_t x = nv; x < B->R; x++) rv[x] = -1;
        B->deg[v] = nv;
    }
    free(tmp);
}

static int dbl_cmp(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/*
 * Threshold list, Appendix D.3: for each point p and each (kind, quantile)
 * pair, sample 500 other points, sort dist_A(a_p, a_v) and take the
 * nearest-rank quantile.  Quantile 100% means t = +inf (pure vector
 * order), 0% means t = 0 (strict attribute order).
 */
static void point_thresholds(build_state *B, const double *quant, uint64_t seed)
{
    const int32_t S = 500;
    double *vals = malloc(sizeof(double) * S);
    for (int64_t p = 0; p < B->n; p++) {
        for (int32_t ti = 0; ti < B->nT; ti++) {
            double q = quant[ti];
            double t;
            if (B->kinds[ti] & OR_WEIGHT_ENTRY) {
                /* Weight-JAG (App. D.3): h = sigma / sigma_A, the standard
                 * deviations of dist(x_p, x_V) and dist_A(a_p, a_V) over
                 * the same 500 sampled points; the weight is q * h */
                double s1 = 0.0, s2 = 0.0, a1 = 0.0, a2 = 0.0;
                uint64_t ctr = ((uint64_t)p * 0x10000ull + (uint64_t)ti) * 4096ull;
                int32_t m = 0;
                for (int32_t s = 0; s < S && B->n > 1; s++) {
                    int64_t v;
                    do {
                        v = (int64_t)(splitmix64(seed ^ (ctr++)) % (uint64_t)B->n);
                    } while (v == p);
                    double dv = sqrt(sqdist(B->X + (size_t)p * B->d, B->X + (size_t)v * B->d, B->d));
                    double da = dist_a(&B->A, B->kinds[ti] & 0xFF, p, v);
                    s1 += dv;
                    s2 += dv * dv;
                    a1 += da;
                    a2 += da * da;
                    m++;
                }
                double sd = m ? sqrt(fmax(s2 / m - (s1 / m) * (s1 / m), 0.0)) : 0.0;
                double sa = m ? sqrt(fmax(a2 / m - (a1 / m) * (a1 / m), 0.0)) : 0.0;
                t = sa > 0.0 ? q * sd / sa : 0.0;
            } else if (q >= 1.0) t = INFINITY;
            else if (q <= 0.0 || B->n < 2) t = 0.0;
            else {
                uint64_t ctr = ((uint64_t)p * 0x10000ull + (uint64_t)ti) * 4096ull;
                for (int32_t s = 0; s < S; s++) {
                    int64_t v;
                    do {
                        v = (int64_t)(splitmix64(seed ^ (ctr++)) % (uint64_t)B->n);
                    } while (v == p);
                    vals[s] = dist_a(&B->A, B->kinds[ti], p, v);
                }
                qsort(vals, S, sizeof(double), dbl_cmp);
                int32_t r = (int32_t)ceil(q * S);
                if (r < 1) r = 1;
                t = vals[r - 1];
            }
            B->thr[(size_t)p * B->nT + ti] = t;
        }
    }
    free(vals);
}

/*
 * Sequential JAG construction.  The entry vertex is the point nearest the
 * FP64 centroid (ties to the smaller id); it is inserted first, the other
 * points follow in a seeded random order.  Writes adj[n][R] (-1 padded) and
 * returns the entry vertex; thr_out (the per-point thresholds) and
 * order_out (the insertion order) are optional.
 * Optional inputs: order_in, an insertion order (a permutation of 0..n-1
 * starting with the entry vertex) used instead of the seeded one, and
 * thr_in[n][nT], per-point threshold values used instead of the sampled
 * quantiles.  Returns -1 when order_in is not such a permutation.
 */
int32_t or_build(int64_t n, int32_t d, const float *X, const int32_t *scalar, const int64_t *loff,
                 const int32_t *lab, int32_t R, int32_t lb, double alpha, int32_t nT,
                 const int32_t *kinds, const double *quant, uint64_t seed, int32_t *adj,
                 double *thr_out, int32_t *order_out, const int32_t *order_in,
                 const double *thr_in)
{
    build_state B;
    B.n = n;
    B.d = d;
    B.R = R;
    B.lb = lb;
    B.nT = nT;
    B.alpha = alpha;
    B.X = X;
    B.A = (or_attrs){n, scalar, loff, lab, NULL, 0.0};
    double *lw = NULL;
    for (int32_t ti = 0; ti < nT; ti++)
        if ((kinds[ti] & 0xFF) == OR_KIND_LABELS_WEIGHTED && !lw) B.A.lw = lw = label_weights(&B.A, &B.A.lw_c);
    B.kinds = kinds;
    B.thr = malloc(sizeof(double) * (size_t)n * (size_t)nT);
    B.adj = adj;
    B.deg = calloc((size_t)n, sizeof(int32_t));
    for (int64_t i = 0; i < n * R; i++) adj[i] = -1;

    double *cen = calloc((size_t)d, sizeof(double));
    for (int64_t i = 0; i < n; i++)
        for (int32_t j = 0; j < d; j++) cen[j] += (double)X[(size_t)i * d + j];
    for (int32_t j = 0; j < d; j++) cen[j] /= (double)n;
    int32_t s = 0;
    double bs = INFINITY;
    for (int64_t i = 0; i < n; i++) {
        double acc = 0.0;
        for (int32_t j = 0; j < d; j++) {
            double t = (double)X[(size_t)i * d + j] - cen[j];
            acc += t * t;
        }
        if (acc < bs) {
            bs = acc;
            s = (int32_t)i;
        }
    }
    free(cen);
    B.entry = s;
    if (thr_in) memcpy(B.thr, thr_in, sizeof(double) * (size_t)n * (size_t)nT);
    else point_thresholds(&B, quant, seed);

    int32_t *order = malloc(sizeof(int32_t) * (size_t)n);
    if (order_in) {
        char *seen = calloc((size_t)n, 1);
        int ok = order_in[0] == s;
        for (int64_t i = 0; i < n && ok; i++) {
            int32_t v = order_in[i];
            ok = v >= 0 && v < n && !seen[v];
            if (ok) seen[v] = 1;
        }
        free(seen);
        if (!ok) {
            free(order);
            free(B.thr);
            free(B.deg);
            free(lw);
            return -1;
        }
        memcpy(order, order_in, sizeof(int32_t) * (size_t)n);
    } else {
        int64_t m = 0;
        order[m++] = s;
        for (int64_t i = 0; i < n; i++)
            if (i != s) order[m++] = (int32_t)i;
        for (int64_t i = n - 1; i > 1; i--) { /* Fisher-Yates over positions 1..n-1 */
            int64_t j = 1 + (int64_t)(splitmix64(seed + 0x5bd1e995ull * (uint64_t)i) % (uint64_t)i);
            int32_t t = order[i];
            order[i] = order[j];
            order[j] = t;
        }
    }

    or_scratch S;
    scratch_init(&S, n);
    or_key *Lbuf = malloc(sizeof(or_key) * (size_t)(lb + R + 1));
    int32_t *Vbuf = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *cand = malloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; i++) insert_point(&B, order[i], &S, Lbuf, Vbuf, cand);
    scratch_free(&S);
    if (thr_out) memcpy(thr_out, B.thr, sizeof(double) * (size_t)n * (size_t)nT);
    if (order_out) memcpy(order_out, order, sizeof(int32_t) * (size_t)n);
    free(Lbuf);
    free(Vbuf);
    free(cand);
    free(order);
    free(B.thr);
    free(B.deg);
    free(lw);
    return s;
}

/* ------------------------------------------------------------------ */
/* Number formats (not in the paper): BF16 and OCP FP8 E4M3           */
/* ------------------------------------------------------------------ */

static double bf16_value(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/*
 * FP32 -> BF16, round to nearest, ties to even.  The two BF16 neighbours
 * of x are the truncation toward zero and the next code away from zero;
 * the nearer one wins and an exact tie picks the even code.
 */
uint16_t or_bf16_encode(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if (isnan(x)) return (uint16_t)((u >> 16) | 0x0040u);
    uint16_t lo = (uint16_t)(u >> 16);
    if ((u & 0xFFFFu) == 0) return lo;
    uint16_t hi = (uint16_t)(lo + 1); /* next magnitude; 0x7F7F+1 = inf */
    double a = fabs((double)x), vl = fabs(bf16_value(lo)), vh = fabs(bf16_value(hi));
    if (isinf(vh)) {
        /* above the largest finite BF16: RNE overflows to inf at the halfway point */
        double half = vl + (ldexp(1.0, 127 - 7) / 2.0);
        return (a >= half) ? hi : lo;
    }
    double dl = a - vl, dh = vh - a;
    if (dl < dh) return lo;
    if (dh < dl) return hi;
    return (lo & 1u) ? hi : lo;
}

void or_bf16_encode_array(int64_t m, const float *x, uint16_t *out)
{
    for (int64_t i = 0; i < m; i++) out[i] = or_bf16_encode(x[i]);
}

/*
 * OCP E4M3 ("e4m3fn"): 1 sign, 4 exponent bits (bias 7), 3 mantissa bits.
 * Exponent 0 holds subnormals m * 2^-9; exponents 1..15 hold (1 + m/8) * 2^(e-7),
 * except S.1111.111 which is NaN; there is no infinity; largest finite is 448.
 */
double or_e4m3_value(uint8_t c)
{
    int s = c >> 7, e = (c >> 3) & 15, m = c & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m, -9);
    else v = ldexp(1.0 + m / 8.0, e - 7);
    return s ? -v : v;
}

/* Nearest E4M3 code, ties to the even code, saturating at +-448. */
uint8_t or_e4m3_encode(float y)
{
    double a = fabs((double)y);
    uint8_t sign = (y < 0.0f || (y == 0.0f && signbit(y))) ? 0x80 : 0x00;
    if (isnan(y)) return 0x7F;
    if (a >= 448.0) return (uint8_t)(sign | 0x7E);
    uint8_t best = 0;
    double bd = INFINITY;
    for (int c = 0; c <= 0x7E; c++) {
        double dv = fabs(or_e4m3_value((uint8_t)c) - a);
        if (dv < bd || (dv == bd && (c & 1) == 0)) {
            bd = dv;
            best = (uint8_t)c;
        }
    }
    return (uint8_t)(sign | best);
}

/*
 * Per-vector scaled FP8: scale = max|x| / 448 (FP32 division), code_i =
 * E4M3(x_i / scale) with the FP32 quotient; an all-zero row gets scale 1.
 * A stored element decodes to the FP32 product scale * e4m3(code).
 */
void or_fp8_encode_rows(int64_t n, int32_t d, const float *X, uint8_t *codes, float *scales)
{
    for (int64_t i = 0; i < n; i++) {
        const float *x = X + (size_t)i * d;
        float mx = 0.0f;
        for (int32_t j = 0; j < d; j++) {
            float a = fabsf(x[j]);
            if (a > mx) mx = a;
        }
        float s = mx > 0.0f ? mx / 448.0f : 1.0f;
        scales[i] = s;
        for (int32_t j = 0; j < d; j++) {
            volatile float y = x[j] / s;
            codes[(size_t)i * d + j] = or_e4m3_encode(y);
        }
    }
}

void or_fp8_decode_rows(int64_t n, int32_t d, const uint8_t *codes, const float *scales, float *X)
{
    for (int64_t i = 0; i < n; i++)
        for (int32_t j = 0; j < d; j++)
            X[(size_t)i * d + j] = (float)((double)scales[i] * or_e4m3_value(codes[(size_t)i * d + j]));
}

/* ------------------------------------------------------------------ */
/* Beam predictor network in FP64 (not in the paper)                  */
/* ------------------------------------------------------------------ */

/*
 * The network output y for each of B feature rows X[B][16], with the FP32
 * parameters the learned search uses (the forward pass above, exported so
 * that it can be checked on its own).
 */
void or_mlp_forward(const float *P, int64_t B, const double *X, double *Y)
{
    for (int64_t b = 0; b < B; b++) Y[b] = mlp_forward(P, X + b * 16);
}

/*
 * Mean squared error of a 16-64-64-1 ReLU network over a batch, and its
 * gradient with respect to every parameter (same layout as the parameters:
 * W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3).  Returns the loss.
 */
double or_mlp_loss_grad(const double *P, int64_t B, const double *X, const double *T, double *G,
                        double *Y)
{
    const double *W1 = P, *b1 = P + 1024, *W2 = P + 1088, *b2 = P + 5184, *w3 = P + 5248,
                 *b3 = P + 5312;
    double *gW1 = G, *gb1 = G + 1024, *gW2 = G + 1088, *gb2 = G + 5184, *gw3 = G + 5248,
           *gb3 = G + 5312;
    memset(G, 0, sizeof(double) * 5313);
    double loss = 0.0;
    for (int64_t b = 0; b < B; b++) {
        const double *x = X + b * 16;
        double z1[64], h1[64], z2[64], h2[64];
        for (int j = 0; j < 64; j++) {
            z1[j] = b1[j];
            for (int i = 0; i < 16; i++) z1[j] += W1[j * 16 + i] * x[i];
            h1[j] = relu(z1[j]);
        }
        for (int j = 0; j < 64; j++) {
            z2[j] = b2[j];
            for (int i = 0; i < 64; i++) z2[j] += W2[j * 64 + i] * h1[i];
            h2[j] = relu(z2[j]);
        }
        double y = b3[0];
        for (int j = 0; j < 64; j++) y += w3[j] * h2[j];
        if (Y) Y[b] = y;
        double r = y - T[b];
        loss += r * r;
        double dy = 2.0 * r / (double)B;
        gb3[0] += dy;
        double dz2[64], dh1[64];
        for (int j = 0; j < 64; j++) {
            gw3[j] += dy * h2[j];
            dz2[j] = z2[j] > 0.0 ? dy * w3[j] : 0.0;
        }
        for (int i = 0; i < 64; i++) dh1[i] = 0.0;
        for (int j = 0; j < 64; j++) {
            gb2[j] += dz2[j];
            for (int i = 0; i < 64; i++) {
                gW2[j * 64 + i] += dz2[j] * h1[i];
                dh1[i] += dz2[j] * W2[j * 64 + i];
            }
        }
        for (int j = 0; j < 64; j++) {
            double dz1 = z1[j] > 0.0 ? dh1[j] : 0.0;
            gb1[j] += dz1;
            for (int i = 0; i < 16; i++) gW1[j * 16 + i] += dz1 * x[i];
        }
    }
    return loss / (double)B;
}

/*
 * JointRobustPrune on its own, with explicit per-point thresholds
 * thr[n][nT]; exported so hand-worked cases can check it.
 */
int32_t or_prune(int64_t n, int32_t d, const float *X, const int32_t *scalar, const int64_t *loff,
                 const int32_t *lab, int32_t R, double alpha, int32_t nT, const int32_t *kinds,
                 const double *thr, int32_t p, const int32_t *cand, int32_t ncand, int32_t *out)
{
    build_state B;
    memset(&B, 0, sizeof(B));
    B.n = n;
    B.d = d;
    B.R = R;
    B.nT = nT;
    B.alpha = alpha;
    B.X = X;
    B.A = (or_attrs){n, scalar, loff, lab, NULL, 0.0};
    double *lw = NULL;
    for (int32_t ti = 0; ti < nT; ti++)
        if ((kinds[ti] & 0xFF) == OR_KIND_LABELS_WEIGHTED && !lw) B.A.lw = lw = label_weights(&B.A, &B.A.lw_c);
    B.kinds = kinds;
    B.thr = (double *)thr;
    int32_t m = joint_robust_prune(&B, p, cand, ncand, out);
    free(lw);
    return m;
}

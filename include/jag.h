/*
 * jag.h -- C ABI of the JAG (Joint Attribute Graph) filtered vector search
 * library for AMD Instinct MI355X (gfx950).
 *
 * Problem (paper Section 2, "Filtered Nearest Neighbors Search"): each point
 * p = (x_p, a_p) has a vector x_p in R^d and an attribute a_p; each query
 * q = (x_q, f_q) has a vector and a filter.  The answer is the k points with
 * g(a_p, f_q) = 1 nearest to x_q.  The library builds a Threshold-JAG index
 * (Section 3.3, Algorithms 3 and 4) and answers batches of queries with the
 * filtered greedy search of Algorithms 1 and 2 on the GPU, ordering
 * candidates by D_F = (dist_F(f_q, a_u), dist(x_q, x_u)) lexicographically
 * (Section 3.2).
 *
 * Conventions shared by every entry point:
 *  - Every call returns a jag_status; 0 is success.  On failure the call has
 *    no effect on its outputs beyond what it documents, and jag_last_error()
 *    returns a thread-local message.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device memory on the current device (e.g. torch tensors on cuda:0).
 *  - The caller owns every buffer it passes in; inputs are only read during
 *    the call (or, for asynchronous calls, until the stream reaches the
 *    work).  The library owns the jag_index until jag_free.
 *  - Vector distances are squared Euclidean distances; "dist" below means
 *    that (it orders candidates exactly like the Euclidean distance).
 *  - Labels are integers in [0, vocab) with vocab <= 65535; each item's
 *    label list must be sorted ascending without repeats.
 *  - One jag_index may be searched from several host threads / streams at
 *    once; building, loading, saving and freeing must not overlap other use
 *    of the same index.
 */
#ifndef JAG_H
#define JAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jag_index jag_index; /* opaque, owned by the library */

typedef enum {
    JAG_OK = 0,
    JAG_EINVAL = -1,      /* bad argument, shape, filter or label */
    JAG_ENOMEM = -2,      /* host or device allocation failed */
    JAG_EDEVICE = -3,     /* HIP runtime error or no gfx950 device */
    JAG_EIO = -4,          /* file could not be read or written */
    JAG_EUNSUPPORTED = -5, /* valid request the index cannot serve (e.g. no FP32 copy) */
    JAG_EBUSY = -6,        /* jag_server_submit: queue full, nothing queued */
    JAG_EAGAIN = 1         /* jag_server_poll: request still pending (not an error) */
} jag_status;

/* Vector store used by the search (Section 8-style precision choices are the
 * library's own; the paper does not fix a precision). */
typedef enum {
    JAG_STORE_F32 = 0,      /* FP32 rows */
    JAG_STORE_BF16 = 1,     /* BF16 rows, round to nearest even */
    JAG_STORE_FP8_E4M3 = 2  /* OCP E4M3 rows with one FP32 scale per row */
} jag_store;

/* Filter types of Section 2 ("Filter Constraints"). */
typedef enum {
    JAG_LABEL = 0,   /* item's label set contains `label` (equality for one-label items) */
    JAG_RANGE = 1,   /* lo <= scalar attribute <= hi (inclusive) */
    JAG_SUBSET = 2,  /* item's label set contains every label of pool[off, off+len) */
    JAG_BOOLEAN = 3, /* DNF program in pool[off, off+len): see jag_filter */
    JAG_TABLE = 4    /* general Boolean function given by its truth table: see jag_filter */
} jag_filter_type;

/* Attribute distances dist_A the threshold list can name, one per entry
 * (Section 3.1): SCALAR |a1 - a2|; LABELS |a1 XOR a2|; LABELS_WEIGHTED the
 * frequency-weighted label distance of App. D.3, C - sum over shared labels l
 * of log(1/p_l), p_l = fraction of items holding l, C = the largest total
 * weight of one item's labels (meant for large, skewed label vocabularies). */
typedef enum { JAG_ATTR_SCALAR = 0, JAG_ATTR_LABELS = 1, JAG_ATTR_LABELS_WEIGHTED = 2 } jag_attr_kind;

/* Flag on a threshold-list entry's kind: a Weight-JAG entry (Section 3.4)
 * whose comparator is w_p * dist_A(a_p, a_v) + dist(x_p, x_v) instead of the
 * capped dist_A; `quantile` then holds the multiplier m and w_p = m * h_p,
 * h_p = sigma / sigma_A of dist and dist_A from p to the same 500 sampled
 * points (App. D.3).  m = 0 orders by vector distance alone; a very large m
 * orders by attribute first. */
#define JAG_THRESHOLD_WEIGHT 0x100

/* Per-item attributes (host).  Either part may be absent (NULL). */
typedef struct {
    const int32_t *scalar;    /* [n] int32 range attribute */
    const int64_t *label_off; /* [n+1] CSR row offsets into labels */
    const int32_t *labels;    /* [label_off[n]] label ids */
    int32_t vocab;            /* label vocabulary size, 1..65535 */
} jag_attrs;

/* One entry of the threshold list T (Section 3.3; Appendix D.3): the capped
 * attribute distance uses, for each point p, the `quantile` of dist_A(a_p, .)
 * over 500 sampled points.  quantile >= 1 means t = +inf (pure vector order),
 * quantile <= 0 means t = 0 (strict attribute order). */
typedef struct {
    int32_t kind;   /* jag_attr_kind, optionally | JAG_THRESHOLD_WEIGHT */
    float quantile; /* in [0, 1]; weight entries: the multiplier m >= 0 */
} jag_threshold;

typedef struct {
    int32_t R;                /* out-degree bound ("deg", Algorithm 4), 1..128 */
    int32_t L_build;          /* beam l_b of the insertion searches (Algorithm 3); 0 = 2R */
    float alpha;              /* pruning parameter (paper: 1.2) */
    int32_t n_thr;            /* |T|, 1..8 */
    const jag_threshold *thr; /* [n_thr] */
    int32_t store;            /* jag_store used by the search */
    int32_t keep_f32;         /* also keep an FP32 copy on the device for reranking */
    uint64_t seed;            /* insertion order and threshold sampling */
    int32_t n_threads;        /* host builder threads; 0 = all hardware threads */
    int32_t max_batch;        /* cap on points inserted per parallel round; 0 = max(64, n/50) */
    int32_t progress;         /* 1 = print one line to stderr per tenth of the points inserted */
    int32_t device;           /* 0 = rounds on host threads; 1 = rounds on the current GPU
                                 (the same graph, edge for edge; needs L_build <= 256) */
    const int32_t *order;     /* optional host [n]: insertion order, a permutation of 0..n-1
                                 whose first element becomes the entry vertex; NULL = the
                                 point nearest the centroid first, then a seeded shuffle */
    const float *thresholds;  /* optional host [n][n_thr]: per-point t of each threshold entry
                                 (>= 0 or +inf) or w of each weight entry (finite, >= 0);
                                 NULL = sampled as described under jag_threshold */
} jag_build_params;

/*
 * Query filter (host).  Fields by type:
 *   LABEL:   label
 *   RANGE:   lo, hi (inclusive)
 *   SUBSET:  off, len -> 1..16 required labels in pool
 *   BOOLEAN: off, len -> DNF program in pool:
 *              ncl, nlit_1, lit..., nlit_2, lit..., ...
 *            1..8 clauses, at most 16 literals in all; a literal l >= 0 asks
 *            for label l, l < 0 asks for the absence of label ~l.  Repeated
 *            literals count once; a clause holding l and ~l never holds.
 *   TABLE:   off, len -> an arbitrary Boolean function of nvar labels
 *            (Section 2's general Boolean filter): pool holds
 *              nvar, var_0, ..., var_{nvar-1}, w_0, ..., w_{W-1}
 *            with 1 <= nvar <= 15 distinct labels and W = ceil(2^nvar / 32)
 *            words; an item's assignment x has bit v set when it holds
 *            label var_v, and the function is true on x when bit x % 32 of
 *            word w_{x / 32} is set.  dist_F = the fewest label flips that
 *            make it true (Section 3.1).  Encode with jag_encode_filters_sized.
 */
typedef struct {
    int32_t type, label, lo, hi, off, len;
} jag_filter;

/* Bytes of one encoded filter record on the device (see jag_encode_filters). */
#define JAG_FILTER_RECORD_BYTES 128

/* Ladder of beam widths the learned predictor chooses from. */
#define JAG_LADDER_MAX 16

typedef struct {
    int32_t L;           /* beam width l_s (fixed mode), k..1024 */
    int32_t learned;     /* 0 = fixed beam L; 1 = predicted beam (index needs a predictor);
                            2 = fixed beam L plus predictor features written to `features`.
                            In modes 1 and 2 the first four expansions keep a list of
                            max(64, widest beam) entries (mode 1: the ladder's last
                            entry, mode 2: L); the features are taken after the fourth
                            expansion and the list is then cut to the beam, which gives
                            exactly the fixed-beam search's state.  Features from
                            traces at L <= 64 match those of a learned search whose
                            ladder tops out at 64 or less. */
    float delta;         /* learned mode: offset added to the predicted ladder index */
    int32_t rerank_mult; /* 0 = none; m > 0 rescores the best m*k entries of the final list
                            from the FP32 copy (needs keep_f32 or an FP32 store); m*k <= 64 */
    int32_t max_hops;    /* 0 = unlimited; else stop after this many expansions */
    int32_t *stats;      /* optional device int32 [nq][4]: expansions, vector distances,
                            attribute evaluations, chosen beam (learned) or L */
    float *features;     /* learned == 2: device float [nq][16] predictor features */
    int32_t hash_log2;   /* 0 = automatic (2^10 slots for lists of up to 128 entries,
                            2^9 for longer ones); else 8..13: the per-query LDS table
                            of discovered ids has 2^hash_log2 slots.  It only trades
                            LDS (occupancy) against repeated evaluations; results do
                            not depend on it. */
    int32_t single_pass; /* learned == 1 only.  0 = two launches: the first runs every
                            query to its prediction point and saves its list and
                            counters; the second resumes the saved searches in order
                            of decreasing predicted beam (longest first, so the batch
                            does not end on a few long searches); 1 = one launch
                            (ordered as a fixed-beam launch is, below).  Ids,
                            distances, counts, expansions and
                            beams are identical; the distance and attribute counts of
                            stats may differ, since a resumed search starts its
                            seen-table again from its list.  Two passes allocate
                            stream-ordered device scratch (hipMallocAsync on the call's
                            stream) for each query's saved state: (8 + 3*W + 2) * 4
                            bytes, W = list width (64 or the widest beam, rounded up
                            to 64; 0.8 KB at W = 64); batches needing more than
                            512 MiB run in chunks.  Which is faster depends on how
                            much the predicted beams spread: measured, one launch on
                            a range workload (ladder to 64), two on label-set
                            workloads (ladders to 512). */
} jag_search_params;

typedef struct {
    int64_t n;
    int32_t d, R, entry, store, has_f32, has_scalar, has_labels, label_width, vocab;
    int32_t has_predictor;
    int64_t device_bytes; /* HBM held by the index */
} jag_index_info;

/* ---- build, import, persistence -------------------------------------- */

/*
 * Build a Threshold-JAG index over n host vectors X[n][d] (FP32, row-major)
 * with attributes A (Algorithms 3 and 4, with the Appendix D.3 notes: a
 * neighbour picked for an earlier threshold joins later buckets without the
 * alpha test, and each bucket stops at ceil(0.9 R / |T|)).  Points are
 * inserted in parallel rounds of growing size; within a round every
 * insertion searches the graph as it stood before the round, so the result
 * depends only on the seed (or the given order and thresholds), not on the
 * thread count.  Each insertion search stops after 4 l_b + 64 expansions.  The
 * rounds run on host threads (P->device = 0) or on the current GPU
 * (P->device = 1); both form every distance in one fixed FP32 order and give
 * the same graph.  With max_batch = 1 every round holds one point: the
 * sequential construction of Algorithm 3.  The graph, attributes and vector
 * store are then placed in device memory of the current device.
 * Errors: EINVAL (n < 1, d < 1, d > 512, bad params, attributes, order or
 * thresholds; L_build > 256 on the device), ENOMEM, EDEVICE, EUNSUPPORTED
 * (device rounds only: one insertion expanding more than 65536 vertices over
 * all its searches, or a vertex gaining more than 65536 - R in-links in one
 * round; a smaller max_batch avoids the latter).  A prune of more than 4096
 * candidates runs with its arrays in device memory instead of LDS, with the
 * same result; the environment variable JAG_BUILD_LDS_CANDIDATES (64..4096)
 * lowers that limit, which only serves to exercise that path in tests.
 */
jag_status jag_build(const float *X, int64_t n, int32_t d, const jag_attrs *A,
                     const jag_build_params *P, jag_index **out);

/*
 * The graph construction of jag_build alone: writes adj_out[n][P->R] (host,
 * -1 padded) and the entry vertex to *entry.  With P->device = 0 no device
 * is involved; with P->device = 1 the rounds run on the current GPU, which
 * holds the FP32 vectors (padded to a multiple of 4 floats), the attributes
 * and the graph while it builds.  P->store and P->keep_f32 are ignored.
 * Same errors as jag_build.
 */
jag_status jag_build_graph(const float *X, int64_t n, int32_t d, const jag_attrs *A,
                           const jag_build_params *P, int32_t *adj_out, int32_t *entry);

/*
 * Make an index from a given graph (host adj[n][R], -1 padded, no
 * repeated ids in a row, ids in [0, n)) and entry vertex, instead of
 * building one.  Only P->store and P->keep_f32 are read from P (P may be
 * NULL: FP32 store).  Errors: EINVAL on a malformed graph.
 */
jag_status jag_build_from_graph(const float *X, int64_t n, int32_t d, const jag_attrs *A,
                                const int32_t *adj, int32_t R, int32_t entry,
                                const jag_build_params *P, jag_index **out);

/* Write / read the index (graph, FP32 vectors, attributes, entry vertex,
 * store choice, predictor) to / from a versioned file.  jag_load places the
 * index on the current device.  Errors: EIO, EINVAL (bad file), ENOMEM. */
jag_status jag_save(const jag_index *idx, const char *path);
jag_status jag_load(const char *path, jag_index **out);

/* Release the index and its device memory.  NULL is allowed. */
void jag_free(jag_index *idx);

jag_status jag_info(const jag_index *idx, jag_index_info *out);

/* Copy the graph to host adj_out[n][R] and the entry vertex to *entry. */
jag_status jag_get_graph(const jag_index *idx, int32_t *adj_out, int32_t *entry);

/* Copy the device vector store to the host, unpadded: F32 -> float[n][d],
 * BF16 -> uint16[n][d], FP8 -> uint8[n][d] codes plus float[n] scales
 * (scales_out is only written for FP8 and may be NULL otherwise). */
jag_status jag_get_store(const jag_index *idx, void *rows_out, float *scales_out);

/* ---- search ------------------------------------------------------------ */

/*
 * Validate and encode nq host filters into fixed-size records
 * (records_out, host, nq * JAG_FILTER_RECORD_BYTES bytes), including the
 * index's selectivity estimate for each filter (exact for LABEL and RANGE;
 * independence-based for SUBSET and BOOLEAN).  The records may be copied to
 * the device once and reused by jag_search_encoded.
 * Errors: EINVAL (unknown type, malformed pool program, label outside
 * [0, vocab), RANGE on an index without scalars, label filters on an index
 * without labels, too many labels/literals/clauses, TABLE filters: their
 * distance tables need jag_encode_filters_sized).
 */
jag_status jag_encode_filters(const jag_index *idx, const jag_filter *F, int64_t nq,
                              const int32_t *pool, int64_t pool_len, void *records_out);

/* Size in bytes of the encoding of F by jag_encode_filters_sized: nq records
 * followed by one distance table of 2^nvar bytes per TABLE filter (16-byte
 * aligned).  Errors: EINVAL (malformed TABLE span). */
jag_status jag_encoded_bytes(const jag_index *idx, const jag_filter *F, int64_t nq,
                             const int32_t *pool, int64_t pool_len, int64_t *bytes);

/* Like jag_encode_filters, for any filter type: out (host, out_bytes >=
 * jag_encoded_bytes) receives the nq records, then the distance tables of
 * the TABLE filters; each such record locates its table by a byte offset
 * from itself, so the whole buffer is copied to the device as one block
 * and passed to jag_search_encoded as `records`.  Errors: as
 * jag_encode_filters, plus EINVAL when out_bytes is too small. */
jag_status jag_encode_filters_sized(const jag_index *idx, const jag_filter *F, int64_t nq,
                                    const int32_t *pool, int64_t pool_len, void *out,
                                    int64_t out_bytes);

/*
 * Filtered greedy search (Algorithm 2 over Algorithm 1) for nq queries,
 * one GPU wavefront per query.  Q: device float[nq][d].  records: device,
 * from jag_encode_filters or jag_encode_filters_sized (the whole buffer).
 * Outputs (device): ids[nq][k] valid item ids
 * (those with dist_F = 0) in increasing (dist, id) order, padded with -1;
 * dists[nq][k] the matching squared distances (from the FP32 copy when
 * reranking, else from the store; +inf for padding); count[nq] the number
 * of valid ids.  Asynchronous on `stream` (a hipStream_t; NULL = default
 * stream).  Launch order: a batch of at least 4096 queries at a fixed
 * beam (or learned with single_pass = 1) runs the searches expected to be
 * long first, by classes of the records' selectivity estimate (range
 * filters broadest first, label-based filters narrowest first), so that
 * the batch does not end on a few long searches; it takes nq * 8 bytes of
 * stream-ordered device scratch for the order (if that cannot be
 * allocated, the batch runs in submission order).  No result depends on
 * the order.
 * Errors: EINVAL (k < 1, k > 64, L < k, L > 1024, bad params),
 * EUNSUPPORTED (rerank without an FP32 copy, learned without predictor),
 * EDEVICE.
 */
jag_status jag_search_encoded(jag_index *idx, const float *Q, int64_t nq, const void *records,
                              int32_t k, const jag_search_params *S, int32_t *ids, float *dists,
                              int32_t *count, void *stream);

/*
 * jag_search_encoded for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results as jag_search_encoded; it
 * calls no hipMalloc, hipFree or allocating library routine.  The scratch
 * that jag_search_encoded allocates per call -- the launch order of a batch
 * of at least 4096 queries at a fixed beam (or single-pass learned), 8 bytes
 * per query, and the saved states of a two-pass learned search -- lives
 * instead in one fixed 32 MiB device array per GPU, held from the first call
 * until the process ends.  Limits: a batch needing a launch order may hold
 * at most 4,194,304 queries (EINVAL beyond); two-pass learned searches run
 * in chunks of queries whose states fit (about 41,000 per chunk at a 64-entry
 * list).  Every call on one GPU shares that array and leaves its contents
 * behind (nothing in it needs clearing: each launch writes what it reads),
 * so calls whose work overlaps on one GPU -- on different streams or host
 * threads -- race and must be serialised by the caller.
 * Errors: as jag_search_encoded, plus EINVAL for a batch beyond the limit
 * and EDEVICE if the array's address cannot be obtained.
 */
jag_status jag_search_encoded_noalloc(jag_index *idx, const float *Q, int64_t nq, const void *records,
                                      int32_t k, const jag_search_params *S, int32_t *ids, float *dists,
                                      int32_t *count, void *stream);

/* Convenience: encode host filters into a pinned staging buffer, copy them
 * to the device and run jag_search_encoded; asynchronous on `stream` (the
 * call does not wait for the stream; a staging buffer is refilled only once
 * its copy has run).  The copy (into stream-ordered memory) runs on a
 * stream the index owns, so it overlaps work already queued on `stream`;
 * `stream` waits for it, by an event, only where the search begins. */
jag_status jag_search_batch(jag_index *idx, const float *Q, int64_t nq, const jag_filter *F,
                            const int32_t *pool, int64_t pool_len, int32_t k,
                            const jag_search_params *S, int32_t *ids, float *dists,
                            int32_t *count, void *stream);

/*
 * Exact filtered k-NN on the GPU over the FP32 vectors (needs the FP32
 * copy): every item passing the filter is scored.  Same output layout as
 * jag_search_encoded.  This is the Pre-Filtering method (Appendix D.4); the
 * library uses it to label predictor training data.
 */
jag_status jag_exact_knn(jag_index *idx, const float *Q, int64_t nq, const void *records,
                         int32_t k, int32_t *ids, float *dists, int32_t *count, void *stream);

/* ---- learned beam predictor (not in the paper) -------------------------- */

/*
 * Attach predictor weights: params = host float[5313] in the layout
 * W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3 (stored on the device in
 * BF16, round to nearest even); ladder = host int32[nladder] increasing
 * beam widths (nladder <= JAG_LADDER_MAX); the network output y selects
 * ladder[clamp(ceil(y + delta), 0, nladder-1)]; the search then stops after
 * ceil(rho * Lhat) expansions.
 */
jag_status jag_set_predictor(jag_index *idx, const float *params, int32_t nladder,
                             const int32_t *ladder, float rho);

/*
 * Train the predictor on the GPU: minibatch Adam on the mean squared error
 * between the network output and targets.  features: device float[m][16],
 * targets: device float[m].  params_inout: host float[5313] (initial values
 * in, trained values out, FP32).  loss_out: host float[epochs] mean loss of
 * each epoch (may be NULL).  Synchronous.
 */
jag_status jag_train_predictor(const float *features, const float *targets, int64_t m,
                               float *params_inout, int32_t epochs, int32_t batch, float lr,
                               uint64_t seed, float *loss_out, void *stream);

/*
 * One forward/backward pass on the GPU without updating: loss (host) and
 * gradient grad_out (host float[5313]) of the mean squared error over m
 * samples for the given FP32 params.  For checking the training kernels.
 */
jag_status jag_predictor_grad(const float *features, const float *targets, int64_t m,
                              const float *params, float *loss_out, float *grad_out,
                              void *stream);

/* ---- serving (not in the paper) ------------------------------------------ */

/*
 * A server owns a scheduler thread and admits single queries to the GPU in
 * one of two ways (slot_admission):
 *
 *  0  batches: the thread gathers requests into batches and keeps several on
 *     the GPU at once (one HIP stream each).  A batch is admitted when a
 *     stream is free and the number of requests on the GPU stays within
 *     max_inflight, which defaults to the number of query wavefronts the
 *     device can hold resident at once (from the kernel's LDS and register
 *     needs).
 *  1  slots: one launch keeps up to max_inflight query wavefronts resident
 *     (default: as many as the device holds, each with its own LDS), and
 *     each wave takes the next request the moment its previous search ends.
 *     Requests are published through a ring of pinned host memory that the
 *     waves poll; answers are written straight back into pinned host memory.
 *     The launch ends by itself after 10 ms without a new request and is
 *     started again when requests arrive.  While it runs it holds the CUs it
 *     occupies: other work on the device waits for free CUs.  learned must be
 *     0 or 1 (1 runs the learned search in one pass); max_batch, n_streams
 *     and max_wait_us are not used.
 *
 * Results are identical to a jag_search_encoded call on the same query with
 * the same search parameters (learned one-pass for slot admission): queries
 * share no state.  Per-request latency is measured from submit to the host
 * seeing the result.
 */
typedef struct jag_server jag_server;

typedef struct {
    int32_t k;                /* neighbours per query, 1..64 */
    jag_search_params search; /* L, learned, delta, rerank_mult, max_hops, hash_log2
                                 (stats and features must be NULL) */
    int32_t max_batch;        /* requests per launch, 1..4096 */
    int32_t n_streams;        /* batches in flight at once, 1..8 */
    int32_t max_wait_us;      /* a partial batch waits at most this long for company */
    int64_t max_inflight;     /* 0 = resident capacity of the device for this search */
    int64_t queue_capacity;   /* pending requests beyond this are refused (JAG_EBUSY) */
    int64_t hbm_budget_bytes; /* 0 = no limit; else the server's device buffers (batches: per
                                 stream a batch's queries, records and results, plus the saved
                                 states of a two-pass learned search; slots: per wave a copy of
                                 its query and a 32 KiB table copy) must fit */
    int32_t slot_admission;   /* 0 = batches per stream, 1 = resident waves (see above) */
    int32_t reserved;         /* must be 0 */
} jag_server_params;

typedef struct {
    /* batches: launches of the search (slot admission: of the resident waves);
     * max_inflight_seen: most requests published to the GPU and not yet
     * returned at once (slot admission: including those waiting for a wave) */
    int64_t submitted, completed, batches, max_inflight_seen, resident_capacity;
    double p50_us, p99_us, mean_us, max_us; /* latency of completed requests */
    double qps;                             /* completed / (last completion - first submit) */
    double mean_batch;
    int64_t device_bytes;
} jag_server_stats;

/* Start a server on idx (which must outlive it).  Errors: EINVAL, ENOMEM,
 * EUNSUPPORTED (e.g. buffers beyond hbm_budget_bytes), EDEVICE. */
jag_status jag_server_start(jag_index *idx, const jag_server_params *P, jag_server **out);

/* Queue n requests: Q host float[n][d], F host filters (pool as in
 * jag_encode_filters).  Filters are validated here; on EINVAL nothing is
 * queued.  A TABLE filter's distance table (2^nvar bytes) travels with its
 * request and is packed, per batch, into a table area of the stream that runs
 * it (pinned host and device memory grown on demand, outside hbm_budget_bytes).  tickets_out[n] receives one ticket per request.  EBUSY when the
 * queue would exceed queue_capacity (nothing queued). */
jag_status jag_server_submit(jag_server *s, const float *Q, const jag_filter *F, int64_t n,
                             const int32_t *pool, int64_t pool_len, uint64_t *tickets_out);

/* Result of one request: JAG_OK (and the result is released), JAG_EAGAIN if
 * still pending, EINVAL for an unknown ticket.  ids/dists: host [k];
 * latency_us may be NULL. */
jag_status jag_server_poll(jag_server *s, uint64_t ticket, int32_t *ids, float *dists,
                           int32_t *count, double *latency_us);

/* Block until every request submitted so far has completed. */
jag_status jag_server_drain(jag_server *s);

jag_status jag_server_stats_get(jag_server *s, jag_server_stats *out);

/* Drain, stop the scheduler and free the server.  NULL is allowed. */
void jag_server_stop(jag_server *s);

/* ---- measurement (not in the paper) ---------------------------------------- */

/*
 * The device's throughput for the access pattern the search lives on: rows
 * of row_bytes bytes read at random row indices.  `waves` one-wave workgroups
 * each read `iters` rows per group of G lanes (G = 4 for rows of up to 384
 * bytes, 8 up to 512, 16 beyond, as the search does), 16 bytes per lane per
 * load; every row index depends on the data of the group's previous row, as
 * the next expansion of a search depends on the last.  buffer: device
 * memory of buffer_bytes bytes (its contents are read, never written; use
 * far more than the last-level cache, e.g. 1 GiB); row_bytes: 64..16384, a
 * multiple of 64 and of 16 bytes per lane (128 for rows of 385..512 bytes, 256
 * beyond); waves: 1..2^20; iters: 1..100000.  The kernel runs once
 * untimed, then `reps` (1..100) times between events on `stream`; the call
 * waits for them and returns the mean rate in *gbs_out (10^9 bytes/s of rows
 * read).  Errors: EINVAL (bad sizes, NULL), EDEVICE.
 */
jag_status jag_gather_ceiling(const void *buffer, int64_t buffer_bytes, int32_t row_bytes, int32_t waves,
                              int32_t iters, int32_t reps, void *stream, double *gbs_out);

/* ---- misc ---------------------------------------------------------------- */

const char *jag_last_error(void);
const char *jag_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JAG_H */

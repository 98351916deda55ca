// Internal declarations shared by the host and device parts of libjag.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "jag.h"

namespace jag {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);

// ---------------------------------------------------------------- filters
enum : int32_t { F_LABEL = 0, F_RANGE = 1, F_SUBSET = 2, F_BOOLEAN = 3, F_TABLE = 4 };

constexpr int kMaxFilterLits = 16;
constexpr int kMaxClauses = 8;
constexpr int kMaxTableVars = 15;  // TABLE filters: distance table of 2^nvar bytes
constexpr uint32_t kUnsat = 0xFFFFFFFFu;  // dist_F when no attribute can satisfy the filter

// Device filter record, JAG_FILTER_RECORD_BYTES bytes, read with scalar loads.
struct alignas(16) FilterRecord {
    int32_t type;                   // F_*
    int32_t a;                      // LABEL: label; RANGE: lo
    int32_t b;                      // RANGE: hi
    int32_t nlit;                   // SUBSET: labels; BOOLEAN: distinct literals
    int32_t ncl;                    // BOOLEAN: satisfiable clauses (0 = never satisfiable)
    uint32_t negmask;               // BOOLEAN: bit i set = literal i asks for absence
    float sel_feature;              // log2(selectivity estimate) / 16
    float selectivity;              // estimate in [0, 1]
    uint16_t lits[kMaxFilterLits];  // labels of the literals / required labels
    uint16_t clmask[kMaxClauses];   // BOOLEAN: literals of each clause (bitmask)
    int64_t table_off;              // TABLE: byte offset from this record to its distance table
    int32_t pad[10];
};
static_assert(sizeof(FilterRecord) == JAG_FILTER_RECORD_BYTES, "record size");

// ---------------------------------------------------------------- index
constexpr int kMaxDim = 512;
constexpr int kMaxR = 128;
constexpr int kMaxLabelsPerItem = 16;
constexpr int kPredParams = 5313;

struct Predictor {
    bool present = false;
    std::vector<float> params;  // FP32 as given
    uint16_t *d_bf16 = nullptr; // device BF16 copy (5313 padded to 5376)
    int32_t nladder = 0;
    int32_t ladder[JAG_LADDER_MAX] = {0};
    float rho = 0.f;
};

// Pinned host buffers that jag_search_batch stages encoded filters in
// (batch.hip); each is reused once the copy out of it has completed.
struct StagingRing;
StagingRing *new_staging();
void free_staging(StagingRing *r);

struct Index {
    int64_t n = 0;
    int32_t d = 0, R = 0, entry = 0, store = JAG_STORE_F32;
    bool keep_f32 = false;
    bool has_scalar = false, has_labels = false;
    int32_t W = 0;      // label row width on the device (uint16 slots, 0xFFFF padded)
    int32_t vocab = 0;
    // host copies (kept for persistence, selectivity estimates and export)
    std::vector<float> X;
    std::vector<int32_t> adj;
    std::vector<int32_t> scalar;
    std::vector<int64_t> loff;
    std::vector<int32_t> lab;
    std::vector<int32_t> scalar_sorted;
    // rank index over scalar_sorted: the scalars of bucket b, the values in
    // [scal_min + (b << scal_shift), scal_min + ((b + 1) << scal_shift)),
    // sit at positions [scal_cum[b], scal_cum[b + 1]) (at most 2^16 buckets)
    std::vector<int64_t> scal_cum;
    int64_t scal_min = 0, scal_max = 0;
    int32_t scal_shift = 0;
    std::vector<int64_t> label_count;
    // device memory
    int device = 0;
    int32_t *d_adj = nullptr;  // rows of adj_words: ids, then the neighbours' attribute words
    int32_t adj_words = 0, scal_word_off = 0, lab_word_off = 0;
    unsigned char *d_vec = nullptr;  // search store rows, vec_stride bytes each
    int32_t vec_stride = 0;
    unsigned char *d_f32 = nullptr;  // FP32 rows (== d_vec for an FP32 store), f32_stride bytes
    int32_t f32_stride = 0;
    bool f32_owned = false;
    int32_t *d_scalar = nullptr;
    uint16_t *d_lab = nullptr;
    int64_t device_bytes = 0;
    Predictor pred;
    StagingRing *staging = nullptr;
    // Launch order statistics (search.hip): per filter kind (range, other)
    // and selectivity class, the sum of expansions and the number of
    // searches of the index's one-pass learned launches, older launches
    // weighing half per launch.
    unsigned long long *d_order_stats = nullptr;
};

// Number of items whose scalar is below v (exact; the rank index narrows
// the binary search to one bucket).
int64_t scalar_rank_below(const Index &ix, int64_t v);

// Row stride of a store: rows are padded to a multiple of 64 bytes; an FP8
// row keeps its FP32 scale in its last 4 bytes.
int32_t store_row_bytes(int32_t store, int32_t d);

// ---------------------------------------------------------------- builder
struct BuildConfig {
    int32_t R = 32, L_build = 64;
    float alpha = 1.2f;
    std::vector<int32_t> kinds;
    std::vector<float> quantiles;
    uint64_t seed = 0;
    int32_t n_threads = 0;
    int32_t max_batch = 0;
    int32_t progress = 0;
    int32_t device = 0;                 // 1: rounds run on the current GPU
    const int32_t *order = nullptr;     // optional insertion order (order[0] = entry)
    const float *thresholds = nullptr;  // optional per-point t / w values [n][|T|]
};

// What both builders need before the first insertion: comparator entries,
// per-point threshold (or weight) values, the insertion order with the entry
// vertex first, and the label weights of the weighted label distance.
struct BuildPlan {
    int32_t R = 0, lb = 0, nT = 0, cap = 0, hopcap = 0;
    float alpha2 = 0.f;
    int32_t entry = 0;
    int64_t max_batch = 0;
    std::vector<int32_t> kinds;
    std::vector<float> thr;      // [n][nT]
    std::vector<int32_t> order;  // [n]
    std::vector<float> lw;       // log(1/p_l) per label (weighted labels only)
    float lw_c = 0.f;            // the constant C of the weighted label distance
};

struct AttrView {
    int64_t n = 0;
    const int32_t *scalar = nullptr;
    const int64_t *loff = nullptr;
    const int32_t *lab = nullptr;
};

int plan_build(const float *X, int64_t n, int32_t d, const AttrView &A, const BuildConfig &cfg,
               BuildPlan &plan);

// Squared distance in the fixed FP32 order shared by the host and device builders.
float l2sq_canonical(const float *a, const float *b, int d);

// Threshold-JAG construction on host threads; fills adj[n*R] (-1 padded).
int build_graph(const float *X, int64_t n, int32_t d, const AttrView &A, const BuildConfig &cfg,
                std::vector<int32_t> &adj, int32_t &entry);

// The same construction with the rounds on the current device: the same
// graph as build_graph, edge for edge.
jag_status build_graph_device(const float *X, int64_t n, int32_t d, const AttrView &A,
                              const BuildConfig &cfg, std::vector<int32_t> &adj, int32_t &entry);

// ---------------------------------------------------------------- device side
// All of these run on the calling thread's current device and report errors
// through set_error, returning a jag_status.
jag_status upload_index(Index &ix);
void free_device(Index &ix);
jag_status launch_search(Index &ix, const float *Q, int64_t nq, const void *records, int32_t k,
                         const jag_search_params &S, int32_t *ids, float *dists, int32_t *count,
                         void *stream, void *fixed_scratch = nullptr, int64_t fixed_bytes = 0);
// Query wavefronts of this search the device can hold resident at once.
jag_status search_capacity(Index &ix, int32_t k, const jag_search_params &S, int64_t *resident,
                           size_t *lds_per_query);
// Stream-ordered device scratch one launch_search of nq queries allocates
// (the saved states of a two-pass learned search; 0 otherwise).
jag_status search_scratch_bytes(Index &ix, int32_t k, const jag_search_params &S, int64_t nq,
                                int64_t *bytes);
jag_status launch_exact(Index &ix, const float *Q, int64_t nq, const void *records, int32_t k,
                        int32_t *ids, float *dists, int32_t *count, void *stream);

// Resident serving waves (serve_kernels.hip).  Requests sit in a ring of C
// slots (C a power of two) in fine-grained pinned host memory; request h
// uses slot h & (C - 1).  A slot holds the filter record (its table_off, for
// a TABLE filter, is the table's byte offset in `tab`), at byte 128 the
// sequence word h + 1, and from byte kServeSlotHeader the query vector.
// The host writes a slot, then publishes it by raising ctl[0] (requests
// published).  Waves claim published requests one at a time, search, write
// the answer to the slot's result rows and then set done[slot] = h + 1.
constexpr int kServeSlotHeader = 144;
constexpr int kServeTableBytes = 1 << kMaxTableVars;  // per-wave table copy
struct ServeRing {
    const unsigned char *req;  // host: C slots of req_stride bytes
    const unsigned char *tab;  // host: distance tables of TABLE requests (16-byte aligned)
    int32_t *ids;              // host [C][k]
    float *dists;              // host [C][k]
    int32_t *count;            // host [C] (-1: the slot's sequence word was wrong)
    uint64_t *done;            // host [C]: h + 1 once request h's answer is in place
    const uint64_t *ctl;       // host: [0] requests published, [1] stop asked
    // device: [kServeTicketWord] tickets handed out (request numbers),
    // [kServeAvailWord] requests known to be published, top bit = closing,
    // [kServeRaisedWord] wall-clock time of the last rise of that count
    uint64_t *dctl;
    unsigned char *wave_mem;   // device: per wave, a copy of its query, then of its table
    int64_t wave_bytes;
    int64_t poll_ticks;        // wall-clock ticks between polls of ctl
    int64_t idle_ticks;        // the launch ends after this long without a new request
    uint32_t cmask;            // C - 1
    int32_t req_stride;
};
// The two device counters sit 256 bytes apart (separate cache lines).
constexpr int kServeTicketWord = 0;
constexpr int kServeAvailWord = 32;
constexpr int kServeRaisedWord = 48;
constexpr int kServeCtlWords = 64;
// Bytes of wave_mem per wave for vectors of d elements.
inline int64_t serve_wave_bytes(int32_t d) { return ((int64_t)4 * d + 255) / 256 * 256 + kServeTableBytes; }
// Resident waves of the serving kernel the device holds at once.
jag_status serve_capacity(Index &ix, int32_t k, const jag_search_params &S, int64_t *resident);
// Launch `waves` serving waves on `stream`; they run until a stop is asked
// or no request is claimed for idle_ticks.
jag_status launch_serve(Index &ix, int32_t k, const jag_search_params &S, const ServeRing &r,
                        int64_t waves, void *stream);
jag_status upload_predictor(Index &ix);
jag_status download_store(const Index &ix, void *rows_out, float *scales_out);
jag_status train_predictor(const float *features, const float *targets, int64_t m,
                           float *params_inout, int32_t epochs, int32_t batch, float lr,
                           uint64_t seed, float *loss_out, void *stream);
jag_status predictor_grad(const float *features, const float *targets, int64_t m,
                          const float *params, float *loss_out, float *grad_out, void *stream);

// Host-side filter encoding with the index's selectivity estimate.
jag_status encode_filters(const Index &ix, const jag_filter *F, int64_t nq, const int32_t *pool,
                          int64_t pool_len, FilterRecord *out);
// Bytes of the records of F followed by the distance tables of its TABLE
// filters (each 2^nvar bytes, 16-byte aligned).
jag_status encoded_bytes(const Index &ix, const jag_filter *F, int64_t nq, const int32_t *pool,
                         int64_t pool_len, int64_t *bytes);
// Records and tables into out (at least encoded_bytes long).
jag_status encode_filters_sized(const Index &ix, const jag_filter *F, int64_t nq, const int32_t *pool,
                                int64_t pool_len, void *out, int64_t out_bytes);

}  // namespace jag

struct jag_index {
    jag::Index ix;
};

/*
 * snn.h - C ABI of the MI355X (gfx950) Sinnamon library.
 *
 * Sinnamon (Bruch, Nardini, Ingber, Liberty; arXiv 2301.10622) answers
 * approximate top-k maximum inner product queries over a streaming collection
 * of sparse real-valued vectors. The problem statement (Eq. 1-2 and the online
 * setting of Section 1) fixes the three calls this library is built around:
 * insert(id, x), delete(id) and search(q, k).
 *
 * Conventions shared by every call:
 *   - Vectors are sparse: `nnz` coordinates in [0, dim) with float32 values.
 *     Coordinates need not be sorted. A value of exactly 0 is not a
 *     coordinate (nz() of Alg. 1 / Alg. 5) and is dropped. Duplicate
 *     coordinates, coordinates >= dim and non-finite values are rejected.
 *   - Ids are caller-chosen uint32 in [0, 0xFFFFFFFE]. 0xFFFFFFFF is reserved.
 *   - Host pointers are read before the call returns; the caller keeps
 *     ownership of every buffer it passes. The index owns all device memory it
 *     allocates and frees it in snn_destroy.
 *   - "_dev" entry points take device pointers (hipMalloc'd or a PyTorch CUDA
 *     tensor's data pointer on ROCm) and a hipStream_t (as void*, NULL = the
 *     stream given at creation). They enqueue work and return; results are
 *     valid once that stream has been synchronised.
 *   - Every call returns a status. On an error the index is unchanged and
 *     snn_last_error() describes the problem. No C++ exception crosses the ABI.
 *   - One index is used by one host thread at a time.
 *
 * Search results are sorted by Sinnamon score descending, ties by the lower
 * external id (the selection of Alg. 3 with k' = k, Alg. 7 reduced), and hold
 * min(k, live documents) entries. Documents that share no coordinate with the
 * query score exactly 0 and still take part in the ranking (Section 3).
 */
#ifndef SNN_H
#define SNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SNN_OK = 0,
  SNN_E_INVALID = -1,   /* bad argument or malformed vector */
  SNN_E_EXISTS = -2,    /* insert of an id that is already live */
  SNN_E_NOT_FOUND = -3, /* delete of an id that is not live */
  SNN_E_FULL = -4,      /* no free slot left (capacity reached) */
  SNN_E_NOMEM = -5,     /* device or host allocation failed */
  SNN_E_BUSY = -6,      /* serving admission: over the device memory budget */
  SNN_E_DEVICE = -7     /* a HIP call failed */
} snn_status;

/* Sketch configuration: Sinnamon_(2m, h) of Alg. 5/6.
 *   dim       n, the dimensionality of the vectors
 *   m         buckets per half of the sketch (U and L each hold m rows), 1..1024
 *   h         number of random mappings pi_o : [n] -> [m], 1..4
 *   hash_seed the mappings are pi_o(j) = mix64(mix64(hash_seed + o) XOR j) mod m
 *             with mix64 the SplitMix64 output function (Steele, Lea, Flood
 *             2014); the paper leaves the mappings unspecified
 *   capacity  maximum number of live documents (document slots); rounded up
 *             to a multiple of 16384 internally
 *   flags     0 or an OR of SNN_FORWARD_STORE, SNN_SKETCH_BF16, SNN_UPPER_ONLY */
/* Keep every live document's (coordinate, value) pairs on the device as well:
 * the vector storage S of Alg. 7, which the re-ranking search reads. Costs
 * 8 bytes per non-zero in HBM and the matching upload on insert. */
#define SNN_FORWARD_STORE 1u
/* Store the sketch in bfloat16, as the paper does (Section 4.1): U rounded
 * toward +infinity and L toward -infinity, so every stored bound is still a
 * bound (Theorem 1 holds) and the sketch takes half the bytes. */
#define SNN_SKETCH_BF16 2u
/* Keep only the upper half U (Sinnamon+ for non-negative collections): half
 * the sketch memory; vectors and queries with a negative value are rejected
 * (SNN_E_INVALID; in a device batch the query counts as malformed). */
#define SNN_UPPER_ONLY 4u
typedef struct {
  uint32_t dim;
  uint32_t m;
  uint32_t h;
  uint32_t capacity;
  uint64_t hash_seed;
  uint32_t flags;
  uint32_t reserved;
} snn_config;

typedef struct snn_index snn_index;

/* Create an empty index. `hip_stream` (a hipStream_t, may be NULL for the
 * default stream) is where the index's own work is enqueued. Device memory for
 * the posting bitmaps (dim x capacity bits), the sketch matrix (2m x capacity
 * float32, the row-major layout of Section 4.1 "Notes on Implementation") and
 * the slot maps is allocated here. Errors: SNN_E_INVALID (dim is 0, m not in
 * 1..1024, h not in 1..4, capacity 0 or above 2^31), SNN_E_NOMEM,
 * SNN_E_DEVICE. */
snn_status snn_create(const snn_config *cfg, void *hip_stream, snn_index **out);
void snn_destroy(snn_index *ix);

/* Insert one vector under `id` (Alg. 5): its id goes onto the inverted list of
 * every non-zero coordinate and its sketch (u = bucket max, l = bucket min;
 * buckets no coordinate maps to are written 0) into a free column of U and L.
 * A column freed by a delete is reused first (Section 4.3). Host pointers.
 * Errors: SNN_E_INVALID, SNN_E_EXISTS, SNN_E_FULL, SNN_E_DEVICE. */
snn_status snn_insert(snn_index *ix, uint32_t id, uint32_t nnz, const uint32_t *coords, const float *vals);

/* Insert `n` vectors in CSR form: vector r is coords/vals[indptr[r] ..
 * indptr[r+1]). Host pointers. All-or-nothing: on error nothing is inserted. */
snn_status snn_insert_batch(snn_index *ix, uint32_t n, const uint32_t *ids, const uint64_t *indptr,
                            const uint32_t *coords, const float *vals);

/* Delete `id` (Section 4.3): its slot leaves every inverted list it is on and
 * the live set; the sketch column is left as it is and the slot is reused by a
 * later insert. Errors: SNN_E_NOT_FOUND, SNN_E_DEVICE. */
snn_status snn_delete(snn_index *ix, uint32_t id);
snn_status snn_delete_batch(snn_index *ix, uint32_t n, const uint32_t *ids);

/* Compaction of the inverted lists (Section 4.1, Notes on Implementation:
 * the paper holds each list as a compressed list that is a bitmap where dense
 * and an array of offsets where sparse). Every coordinate keeps its posting
 * bitmap, which inserts and deletes update; this call gives each coordinate
 * whose postings cover at most 1/16 of the used slots an array container too
 * (per block of 1,024 slots, the offsets of its postings), so that scoring it
 * costs work per posting rather than per slot. Searches are correct with or
 * without it; blocks changed after it are read from the bitmaps until the next
 * compaction, with identical results. It waits for all work on the device,
 * reads every bitmap once and replaces the containers; it may be called any
 * time the index is not used by another thread (not during snn_serve_run).
 * classes (nullable, host, dim bytes): pin the coordinates that get arrays
 * (non-zero = array) instead of choosing by density. Which coordinates hold
 * arrays decides how a score's terms are grouped (the array terms are summed
 * apart, then added), so it changes the last bits of scores (within the FP32
 * tolerance); two indexes with equal live documents and equal classes give
 * identical results. A coordinate whose array table would exceed 4 GiB of
 * block offsets, or 2^32 postings in all, keeps its bitmap only.
 * Errors: SNN_E_NOMEM, SNN_E_DEVICE (the index is unchanged). */
snn_status snn_compact(snn_index *ix, const uint8_t *classes);

/* The container class of every coordinate after the last snn_compact (dim
 * bytes: 1 = array container, 0 = bitmap only; all 0 before any compaction). */
snn_status snn_container_classes(snn_index *ix, uint8_t *out);

/* Search one query (Alg. 6 scoring with T = infinity, then Alg. 3 / Alg. 7 with
 * k' = k). Writes up to k results to out_ids / out_scores (caller-allocated, k
 * entries each) and the result count to *out_count. Host pointers; returns
 * after the results are on the host. Errors: SNN_E_INVALID (k = 0 or a
 * malformed query), SNN_E_NOMEM, SNN_E_DEVICE. */
snn_status snn_search(snn_index *ix, uint32_t nnz, const uint32_t *coords, const float *vals, uint32_t k,
                      uint32_t *out_ids, float *out_scores, uint32_t *out_count);

/* Search nq queries given in CSR form (query r owns entries indptr[r] ..
 * indptr[r+1]). Outputs are nq x k row-major plus nq counts. Host pointers. */
snn_status snn_search_batch(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                            const float *vals, uint32_t k, uint32_t *out_ids, float *out_scores,
                            uint32_t *out_counts);

/* Search modes for the _dev batch search. */
typedef enum {
  SNN_MODE_PLAIN = 0,     /* one launch per query, tiles of one query at a time */
  SNN_MODE_BATCHED = 1,   /* one persistent launch for the whole batch (HIP graph) */
  SNN_MODE_LEARNED = 2    /* batched, with the learned k-th-score pre-filter */
} snn_mode;

/* Device-pointer batch search. indptr (nq + 1 uint64), coords, vals, and the
 * outputs out_ids (nq x k uint32), out_scores (nq x k float32), out_counts (nq
 * uint32) live in device memory; `total` must equal indptr[nq] (the entry
 * count, known to the caller, so the call never reads device memory back).
 * Enqueued on `stream` (NULL: the index stream); the call does not wait for
 * completion. In SNN_MODE_LEARNED the queries that need the plain path are
 * listed and re-run on the device, in the same enqueued work (no host
 * synchronisation). Malformed queries produce a
 * count of 0 and set the bit in the status returned by snn_last_batch_status.
 * Errors: SNN_E_INVALID (k = 0, nq = 0, mode unknown, no trained filter for
 * SNN_MODE_LEARNED), SNN_E_NOMEM, SNN_E_DEVICE. */
snn_status snn_search_batch_dev(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                const uint32_t *coords, const float *vals, uint32_t k, uint32_t mode, uint32_t *out_ids,
                                float *out_scores, uint32_t *out_counts, void *stream);

/* Allocation-free form of snn_search_batch_dev, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Arguments, layouts, ownership and results
 * are those of snn_search_batch_dev with mode SNN_MODE_PLAIN or
 * SNN_MODE_BATCHED. The batch's workspace (prepared query entries, per-query
 * thresholds and counters, work queues, tile candidates) is carved from one
 * array of SNN_NOALLOC_SCRATCH_BYTES of device memory that the library holds
 * on each device it runs on until the process ends; the call allocates
 * nothing and uses no HIP graph (its kernels are enqueued one by one, so a
 * capturing caller records them). Every call on one device shares that array
 * and overwrites the previous call's contents: calls that overlap on one
 * device (concurrent streams, threads) race and must be serialised by the
 * caller; the results of a call stay valid, they are in the caller's buffers.
 * The device current at the call must be the one current at snn_create.
 * Errors: SNN_E_INVALID (as snn_search_batch_dev; SNN_MODE_LEARNED; another
 * device current; a batch whose workspace exceeds the array: about
 * nq x tiles x min(k, tile) x 8 bytes of tile candidates plus 16 bytes per
 * query entry and a few words per query, with tiles = ceil(slots used / tile)
 * and a tile of 256 R slots, R from the schedule), SNN_E_DEVICE. */
#define SNN_NOALLOC_SCRATCH_BYTES (64ull << 20)
snn_status snn_search_batch_dev_noalloc(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                        const uint32_t *coords, const float *vals, uint32_t k, uint32_t mode,
                                        uint32_t *out_ids, float *out_scores, uint32_t *out_counts, void *stream);

/* Options of one batch search (all the forms above in one call):
 *   mode        SNN_MODE_PLAIN, SNN_MODE_BATCHED or SNN_MODE_LEARNED
 *   k_prime     0: ranking by the Sinnamon scores (Alg. 7 with k' = k, i.e.
 *               Alg. 3); k <= k_prime <= 65,536: Alg. 7 with k_prime
 *               candidates re-scored exactly (an index with
 *               SNN_FORWARD_STORE; SNN_MODE_BATCHED, or SNN_MODE_LEARNED,
 *               where the filter's threshold -- trained with k = k_prime --
 *               starts the selection of the k_prime candidates and a query
 *               that keeps fewer runs again without it, so the results are
 *               those of SNN_MODE_BATCHED)
 *   max_coords  0: every query coordinate is scored; c > 0: the anytime
 *               variant, scoring stops after the first c coordinates in the
 *               order of Alg. 6 (|q_j| descending, ties by the lower j). This
 *               is the time budget T of Alg. 4 / Alg. 6 expressed as a count
 *               of coordinates, so results do not depend on timing. The
 *               re-rank of Alg. 7 still uses every coordinate of q.
 *   reserved    must be 0 */
typedef struct {
  uint32_t mode;
  uint32_t k_prime;
  uint32_t max_coords;
  uint32_t reserved;
} snn_search_params;

/* Device-pointer batch search with options; arguments otherwise as in
 * snn_search_batch_dev. Errors: SNN_E_INVALID (k = 0 or > 4096, nq = 0, an
 * unknown mode, 0 < k' < k, k' > 65,536, re-rank in SNN_MODE_PLAIN or
 * without a forward store, no trained filter for SNN_MODE_LEARNED, reserved
 * != 0), SNN_E_NOMEM, SNN_E_DEVICE. */
snn_status snn_search_ex_dev(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                             const uint32_t *coords, const float *vals, uint32_t k, const snn_search_params *params,
                             uint32_t *out_ids, float *out_scores, uint32_t *out_counts, void *stream);

/* The same from host buffers (CSR queries as in snn_search_batch); returns
 * after the results are on the host. */
snn_status snn_search_ex(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                         const float *vals, uint32_t k, const snn_search_params *params, uint32_t *out_ids,
                         float *out_scores, uint32_t *out_counts);

/* Ranking with k' >= k (Alg. 7): the k_prime documents with the largest
 * Sinnamon scores are fetched from the forward store, scored exactly (the
 * inner product of Eq. 2, FP32 sums) and the k best by exact score are
 * returned, ties by the lower external id. out_scores hold those exact
 * scores. Needs an index created with SNN_FORWARD_STORE. Device pointers and
 * stream as in snn_search_batch_dev; outputs are nq x k and nq counts of
 * min(k, k_prime, live). When k_prime exceeds a tile (256 R slots), which no
 * tile's own selection can cut, the search first selects on a sample of the
 * tiles (one in 16) and starts the full pass from the lowest score of about
 * 2 k_prime / 16 best there; a query that then keeps fewer than
 * min(k_prime, live) candidates runs again without it, so the results are
 * those of Alg. 7 either way. Errors: SNN_E_INVALID (no forward store, k = 0,
 * k_prime < k or k_prime > 65,536, nq = 0), SNN_E_NOMEM, SNN_E_DEVICE. */
snn_status snn_search_rerank_dev(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                 const uint32_t *coords, const float *vals, uint32_t k, uint32_t k_prime,
                                 uint32_t *out_ids, float *out_scores, uint32_t *out_counts, void *stream);

/* The same from host buffers (CSR queries as in snn_search_batch); returns
 * after the results are on the host. */
snn_status snn_search_rerank(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                             const float *vals, uint32_t k, uint32_t k_prime, uint32_t *out_ids, float *out_scores,
                             uint32_t *out_counts);

/* Number of queries of the last snn_search_batch_dev call that were malformed
 * (needs the stream synchronised), and, for SNN_MODE_LEARNED and for a
 * re-ranking search whose k' exceeds a tile, how many fell back to the pass
 * without a starting threshold. */
snn_status snn_last_batch_status(snn_index *ix, uint32_t *invalid_queries, uint32_t *fallbacks);

/* Selection work of the last batch search (the filtered and the fallback pass
 * counted apart: SNN_MODE_LEARNED, and a re-ranking search whose k' exceeds a
 * tile, which starts from thresholds found on a sample of the tiles; the
 * *_fallback fields are 0 otherwise):
 *   candidates  keys the tiles handed to the merge, i.e. the insertions into
 *               the top-k selection of Alg. 3 that survived each tile's own
 *               selection;
 *   selects     tiles that had more than k keys at or above the query's
 *               threshold and so ran the radix select (the others pass all
 *               their keys on without one).
 * Synchronises the device. */
typedef struct {
  uint64_t candidates;
  uint64_t candidates_fallback;
  uint64_t selects;
  uint64_t selects_fallback;
} snn_batch_work;
snn_status snn_last_batch_work(snn_index *ix, snn_batch_work *out);

/* Launch schedule of the search kernels. R is the number of slots each lane
 * scores (a workgroup of 256 lanes covers a tile of 256 * R slots); grid is the
 * workgroup count of the persistent batched kernel; persistent = 0 launches one
 * workgroup per (query, tile) instead. qgroup > 1 (h = 1 only) makes each
 * batched workgroup score qgroup queries on its tile at once, loading each
 * sketch row once for all of them; results are the same bits either way.
 * Valid combinations: qgroup 1 with R_batch 16, 32, 64; qgroup 2 with
 * R_batch 8 or 16; qgroup 3 with R_batch 16; qgroup 4 with R_batch 8.
 * R_plain is 16, 32 or 64. */
typedef struct {
  int32_t R_plain;
  int32_t R_batch;
  uint32_t grid;
  uint32_t persistent;
  float best_ms;      /* tuned batched pass, ms (0 if not tuned) */
  float default_ms;   /* same batch with the default schedule, ms */
  uint32_t tried;     /* candidate schedules timed */
  uint32_t qgroup;    /* queries per batched workgroup (1 to 4) */
} snn_schedule;

/* Autotuner: time the candidate schedules (R in {16, 32, 64} with qgroup 1,
 * and (R, qgroup) in {(16, 2), (16, 3), (8, 4)} when h = 1; persistent grids of
 * 1024, 2048 and 4096 workgroups or one workgroup per item) on the given
 * device-resident batch, keep the fastest for later searches of this index,
 * and report it in *out (may be NULL). Same arguments as snn_search_batch_dev
 * without the mode; scratch outputs are allocated internally. Blocking. */
snn_status snn_autotune(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total, const uint32_t *coords,
                        const float *vals, uint32_t k, snn_schedule *out);
/* Read or set the schedule (set ignores best_ms, default_ms, tried). */
snn_status snn_get_schedule(snn_index *ix, snn_schedule *out);
snn_status snn_set_schedule(snn_index *ix, const snn_schedule *in);

/* ------------------------------------------------------------------------
 * Learned k-th-score pre-filter (not part of the paper). A small MLP over
 * hashed query features predicts y = ln(s_k), the log of the k-th Sinnamon
 * score of the query. The search starts its selection threshold (theta of
 * Alg. 3, otherwise minus infinity) at tau = exp(yhat - delta): only documents
 * scoring >= tau are candidates. When at least min(k, live) documents reach
 * tau, the k-th score is >= tau and the result is exactly the plain result;
 * otherwise the query is re-run on the plain path. Results never change.
 *
 * Features (256): f[g(j)] += xi(j) q_j and f[128 + g(j)] += q_j^2 over nz(q),
 * g(j) = mix64(mix64(feature_seed) ^ j) mod 128, xi(j) = -1 if the top bit of
 * mix64(mix64(feature_seed + 1) ^ j) is set, else +1 (signed feature hashing).
 * MLP: 256 -> 128 -> 128 -> 1 with ReLU, bf16 weights, fp32 accumulation; fp32
 * master weights trained with Adam on mean squared error. Parameters are packed
 * W1[128][256] | b1[128] | W2[128][128] | b2[128] | W3[128] | b3 (49,537
 * floats, weights row-major [out][in]).
 * ------------------------------------------------------------------------ */
#define SNN_MLP_PARAMS 49537u
#define SNN_MLP_FEATURES 256u

typedef struct {
  uint64_t feature_seed;
  uint64_t seed;          /* weight initialisation and minibatch order */
  uint32_t k;             /* the k whose k-th score is predicted */
  uint32_t epochs;
  uint32_t batch;         /* minibatch size */
  float lr;               /* Adam learning rate */
  float holdout;          /* fraction of labelled queries kept for calibration */
  float target_fallback;  /* delta is the (1 - target) quantile of yhat - y on the holdout */
} snn_filter_params;

typedef struct {
  uint32_t n_train, n_holdout, n_unlabelled;  /* unlabelled: s_k <= 0 or fewer than k results */
  uint32_t steps;
  float train_mse, holdout_mse;               /* on ln s_k */
  float delta;
  float holdout_fallback;                     /* fraction of holdout queries with s_k < tau */
  float label_ms, train_ms;                   /* GPU time of labelling and of training */
} snn_filter_report;

/* Train the filter on nq device-resident training queries (CSR as in
 * snn_search_batch_dev). Labels come from the plain search of this index.
 * Blocking. Errors: SNN_E_INVALID (bad params, too few labelled queries). */
snn_status snn_filter_train(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                            const uint32_t *coords, const float *vals, const snn_filter_params *params,
                            snn_filter_report *report);
/* Hashed features (device out: nq x 256 float32) and predictions yhat (device
 * out: nq float32) of the current filter, enqueued on the index stream. */
snn_status snn_filter_features(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                               const float *vals, float *out_features);
snn_status snn_filter_predict(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                              const float *vals, float *out_yhat);
/* Host copies of the parameters: get returns the bf16-rounded compute copies
 * widened to float32; set loads float32 masters (the compute copies are their
 * bf16 rounding) and resets the optimiser state. feature_seed and k come with
 * set so a filter can be installed without training. */
snn_status snn_filter_get_params(snn_index *ix, float *params);
snn_status snn_filter_set_params(snn_index *ix, const float *params, uint64_t feature_seed, uint32_t k);
snn_status snn_filter_set_delta(snn_index *ix, float delta);
/* Switch the learned form on (on != 0) or off for the host-buffer calls
 * snn_search and snn_search_batch, the search(q, k) of the problem statement
 * (Section 1): while on they run SNN_MODE_LEARNED instead of
 * SNN_MODE_BATCHED. Results are the same either way; snn_last_batch_status
 * reports how many queries of the last call fell back to the plain pass.
 * snn_search_ex / _dev calls keep the mode they are given. Errors:
 * SNN_E_INVALID (on != 0 without a trained or installed filter). */
snn_status snn_filter_enable(snn_index *ix, int on);
/* Loss and gradient of the MLP on B device-resident feature rows X (B x 256)
 * and targets y, with the current compute copies: *loss (host) and grad
 * (device, SNN_MLP_PARAMS floats). Used to check the training kernels. */
snn_status snn_mlp_loss_grad(snn_index *ix, uint32_t B, const float *X, const float *y, float *grad, float *loss);

/* ------------------------------------------------------------------------
 * Serving: one call runs a trace of searches, inserts and deletes against the
 * device-resident index with continuous batching. Requests are admitted in
 * arrival order. Inserts and deletes are applied as they arrive on the index
 * stream; searches that arrive while earlier batches are on the GPU form the
 * next batch, which is launched as soon as an in-flight slot and enough of the
 * device memory budget are free, on its own stream, so batches overlap on the
 * device. Every search sees exactly the inserts and deletes that precede it in
 * the trace (the online setting of Section 1): slots changed during the run
 * carry (insert, delete) sequence numbers, and a deleted slot is reused only
 * once no search that may still see its old document is in flight.
 * ------------------------------------------------------------------------ */
typedef struct {
  uint32_t n;                /* requests, in arrival order */
  const uint8_t *kind;       /* 0 = search, 1 = insert, 2 = delete */
  const double *arrival_s;   /* arrival time, seconds from the start, non-decreasing */
  const uint32_t *id;        /* insert / delete: the document id */
  const uint32_t *k;         /* search: k (1..4096) */
  const uint64_t *indptr;    /* n + 1 offsets: the vector of request r (empty for deletes) */
  const uint32_t *coords;
  const float *vals;
} snn_trace;

typedef struct {
  uint32_t max_batch;        /* most searches in one batch */
  uint32_t max_inflight;     /* most batches on the device at once, 1..8 */
  uint32_t streams;          /* HIP streams the batches rotate over, 1..4 */
  uint32_t realtime;         /* 1: admit each request at its arrival time; 0: all arrive at once */
  uint64_t budget_bytes;     /* device memory the in-flight search workspaces may use */
} snn_serve_params;

typedef struct {
  uint32_t searches, inserts, deletes, rejected, batches, max_batch_seen, max_inflight_seen;
  uint32_t reserved;
  double wall_s, search_qps;
  double p50_ms, p90_ms, p99_ms, max_ms, mean_ms; /* search latency: completion - arrival */
  double mutation_p50_ms, mutation_p99_ms;        /* insert / delete latency */
  uint64_t peak_workspace_bytes;
} snn_serve_report;

/* Run a trace (host pointers). The i-th search of the trace writes its results
 * to row i of out_ids / out_scores (rows of kmax entries, kmax = the largest k
 * in the trace), its count to out_counts[i] (0xFFFFFFFF when rejected because
 * its own workspace exceeds the budget) and its latency to out_latency_ms[i]
 * (any output pointer may be NULL). The trace is validated first
 * (all-or-nothing): unknown kinds, inserts of live ids, deletes of ids that
 * are not live at that point and malformed vectors give SNN_E_INVALID. */
snn_status snn_serve_run(snn_index *ix, const snn_trace *trace, const snn_serve_params *params, uint32_t *out_ids,
                         float *out_scores, uint32_t *out_counts, double *out_latency_ms, snn_serve_report *report);

/* Read back state for tests: the bucket table pi_o(j) as h x dim uint32
 * (row-major), and the stored sketch column (m floats each for U and L) of a
 * live id; bfloat16 sketches are widened exactly, and without an L half l
 * gets zeros. Host pointers. */
snn_status snn_bucket_table(snn_index *ix, uint32_t *out);
snn_status snn_read_sketch(snn_index *ix, uint32_t id, float *u, float *l);

/* Kernel timing for measurement. While enabled, every launch of the scoring
 * and selection kernel is bracketed by HIP events recorded on the stream it is
 * launched on. snn_profile_read synchronises those events and returns the
 * summed kernel time in milliseconds and the number of launches since the
 * previous read (then resets both). */
snn_status snn_profile_enable(snn_index *ix, int on);
snn_status snn_profile_read(snn_index *ix, double *tile_ms, uint32_t *launches);

/* Update-kernel timing (Alg. 5 insert, Section 4.3 delete). While profiling is
 * enabled, every launch of the insert kernel and of the delete kernel made by
 * snn_insert_batch / snn_delete_batch (and the single forms) is bracketed by
 * HIP events on the index's stream. This call synchronises them and returns,
 * per kernel, the summed time in milliseconds and the documents the launches
 * covered since the previous read (then resets both). Host validation and
 * the upload are outside the brackets. Any output pointer may be NULL. */
snn_status snn_profile_read_updates(snn_index *ix, double *insert_ms, uint64_t *insert_docs, double *delete_ms,
                                    uint64_t *delete_docs);

size_t snn_live_count(const snn_index *ix);
const char *snn_last_error(const snn_index *ix); /* never NULL */

#ifdef __cplusplus
}
#endif
#endif /* SNN_H */

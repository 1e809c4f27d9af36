/*
 * bbc.h - C ABI of the MI355X (gfx950) query path for large-k approximate
 * nearest-neighbour search over quantized IVF indexes with a bucket-based
 * result collector (BBC, arxiv 2604.01960).
 *
 * Problem (background section of the paper, "Problem Statement"): index N
 * d-dimensional vectors; for a query q return its k nearest vectors under
 * squared Euclidean distance (the default) or inner product, k typically
 * >= 5,000.  The path: IVF probe -> quantized-code scan (PQ tables) ->
 * bucket-based collector of the K_c = min(ceil(r*k), S) best estimated keys
 * (result-buffer section: Push / Update / Collect, bucket-id equation) ->
 * exact re-rank -> k results.
 *
 * Conventions shared by every entry point
 *  - Every function returns a status (BBC_OK or a negative BBC_E* code);
 *    nothing throws across the ABI.  bbc_last_error() gives a message for
 *    the last failing call on the calling thread.
 *  - Ids are original row numbers 0..n-1.  Results are sorted ascending by
 *    (key, id): key = squared L2, or -<q, x> for inner product, ties broken
 *    by the smaller id.  Distances returned are squared L2, or <q, x>.
 *  - If fewer than k objects are scanned, out_counts[q] is that number and
 *    the remaining slots hold id -1 and +inf (L2) / -inf (IP).
 *  - Arrays are row-major and densely packed.  The caller owns every buffer
 *    it passes; the library copies what it keeps and holds no caller pointer
 *    after a call returns.
 *  - Floating-point inputs must be finite (BBC_EINVAL otherwise).
 *  - Environment switches, read when an index is made (bbc_index_*), select
 *    kernel forms for tuning and tests; unless noted, results are the same
 *    bit for bit under every setting: BBC_SCAN_VARIANT (PQ scan block
 *    shape 0..4), BBC_PAIR_SORT (0: pair sorts with device-wide atomics),
 *    BBC_RERANK_FORM (1: per-query PQ re-rank), BBC_RERANK_SORT_BINS,
 *    BBC_RERANK_RUN_LIST (0: tile re-rank runs found by binary search),
 *    BBC_COLLECT_BCAP, BBC_FINAL_LDS_CAP, BBC_FILTER_FRACTION (tighter
 *    filter of the lists after the codebook sample, with a rescan),
 *    BBC_WALK_FORM, BBC_WALK_PRESORT, BBC_WALK_QCAP, BBC_WALK_ALPHA,
 *    BBC_SCAN_BY_LIST, BBC_RQ_SCAN_1D (RaBitQ forms).  Out-of-range values
 *    are ignored.
 *  - One index may be searched from several threads and on several streams
 *    at once.  The host side of each call is serialised per index; searches
 *    without a caller workspace share the index's device workspace, and each
 *    such search makes its stream wait for the previous one's use of it, so
 *    they never overlap on the device (plans and servers own their
 *    workspaces and run concurrently with them).
 */
#ifndef BBC_H_
#define BBC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBC_OK 0
#define BBC_EINVAL (-1)      /* bad argument */
#define BBC_ENOMEM (-2)      /* device or host allocation failed */
#define BBC_EDEVICE (-3)     /* HIP runtime error */
#define BBC_EUNSUPPORTED (-4)
#define BBC_EBUSY (-6)       /* serving: result not ready yet */

#define BBC_METRIC_L2 0
#define BBC_METRIC_IP 1

#define BBC_QUANT_PQ 0
#define BBC_QUANT_RABITQ 1

/* Result collectors (result-collector background and Algorithm 1).  All
 * three return the same candidates, the K_c smallest estimated (key, id);
 * they differ in how they find them:
 *  BUCKET  the bucket-based result buffer: codebook from the nearest lists,
 *          keys above its d_max dropped during the scan, one histogram of
 *          the rest, all buckets below the threshold bucket plus the best s
 *          of the threshold bucket;
 *  HEAP    comparator: every scanned key offered to a bounded max-heap of
 *          K_c (key, id) per query (one wave per query, 64-ary heap in
 *          global memory, many waves per compute unit);
 *  SORT    comparator: exact selection over every scanned key (radix
 *          select of the K_c-th key, ties by id);
 *  HEAP_LDS the heap comparator with each query's heap in LDS (when the
 *          batch's largest K_c fits in 152 KiB, else as HEAP): one wave per
 *          compute unit at large K_c. */
#define BBC_COLLECT_BUCKET 0
#define BBC_COLLECT_HEAP 1
#define BBC_COLLECT_SORT 2
#define BBC_COLLECT_HEAP_LDS 3

typedef struct bbc_index bbc_index; /* opaque; owns its device memory */

/* Create a PQ index on `device` from an already built IVF-PQ index held in
 * host memory (background section: IVF lists of k-means clusters, residual
 * product quantization with M sub-spaces of 2^bits codewords).
 *   centroids [nlist][d] float32
 *   list_off  [nlist+1] int64, list_off[0] = 0, non-decreasing, = n at the end
 *   list_ids  [n] int64: row id of each list slot (a permutation of 0..n-1)
 *   codebook  [pq_m][2^pq_bits][d/pq_m] float32 (codewords of residuals)
 *   codes     [n][pq_m] uint8, list-slot order, one code per byte
 *   base      [n][d] float32 in row-id order (for the exact re-rank)
 * Requirements: d % 4 == 0, d <= 1024, d % pq_m == 0, pq_bits in {4, 8},
 * 1 <= nlist <= 8192, n < 2^31.  metric must be BBC_METRIC_L2 for PQ. */
int32_t bbc_index_create_pq(int32_t device, int64_t n, int32_t d, int32_t nlist, int32_t metric,
                            const float* centroids, const int64_t* list_off, const int64_t* list_ids,
                            int32_t pq_m, int32_t pq_bits, const float* codebook, const uint8_t* codes,
                            const float* base, bbc_index** out);

/* Build an index on `device` from base [n][d] (row-id order; float32, or
 * float16 when storage = BBC_STORAGE_FP16): IVF k-means (kmeans_iters Lloyd
 * rounds on the training rows, then every row assigned to its nearest
 * centroid; empty clusters split the largest one), then
 *  - PQ: residual PQ trained on the PQ rows (pq_rows [n_pq] ascending rows,
 *    pq_init [pq_m][2^pq_bits] distinct positions in pq_rows seeding each
 *    sub-space codebook; d/pq_m <= 16; L2 only, float32 only);
 *  - RaBitQ: 1-bit codes of the rotated residuals with their factors
 *    (rotation [d][d] orthogonal float32, d % 64 == 0), bounds at
 *    confidence eps0 (0 = the cited method's 1.9); L2 or IP.
 * The random draws are inputs: train_rows [n_train] ascending rows,
 * init_pos [nlist] distinct positions in train_rows seeding the centroids.
 * Assignment uses canonical float32 squared L2 with ties to the smaller id;
 * centroid and codeword means are float64 sums in row order rounded once. */
#define BBC_STORAGE_FP32 0
#define BBC_STORAGE_FP16 1
typedef struct {
  int32_t nlist;
  int32_t kmeans_iters;
  int32_t metric;   /* BBC_METRIC_L2, or BBC_METRIC_IP (RaBitQ) */
  int32_t quant;    /* BBC_QUANT_PQ or BBC_QUANT_RABITQ */
  int32_t pq_m;
  int32_t pq_bits;  /* 4 or 8 */
  const int64_t* train_rows; int64_t n_train; const int64_t* init_pos;
  const int64_t* pq_rows; int64_t n_pq; const int64_t* pq_init;
  const float* rotation;  /* RaBitQ: [d][d] */
  float rabitq_eps0;      /* RaBitQ: 0 = 1.9 */
  int32_t storage;        /* BBC_STORAGE_FP32 / BBC_STORAGE_FP16 (RaBitQ) */
} bbc_build_params;

int32_t bbc_build_index(int32_t device, const void* base, int64_t n, int32_t d, const bbc_build_params* params,
                        bbc_index** out);

/* Create a RaBitQ index on `device` from an already built one in host
 * memory (the cited RaBitQ method: 1-bit codes of randomly rotated
 * residuals and their factors).
 *   centroids [nlist][d] float32; list_off, list_ids as for PQ
 *   rotation  [d][d] float32 orthogonal P; codes encode P^T (x - c_j)
 *   codes     [n][d/32] uint32, list-slot order: bit i of a code is word
 *             i/32, bit i%32 (1 when the rotated residual's i-th entry > 0)
 *   factors   [n][4] float32, list-slot order: (|x - c_j|, f, g, popcount)
 *   base      [n][d] float32, or float16 when storage = BBC_STORAGE_FP16,
 *             row-id order (exact distances convert float16 exactly)
 *   eps0      bound confidence (0 = 1.9)
 * Requirements: d % 64 == 0, d <= 1024, 1 <= nlist <= 8192, n < 2^31. */
int32_t bbc_index_create_rabitq(int32_t device, int64_t n, int32_t d, int32_t nlist, int32_t metric,
                                const float* centroids, const int64_t* list_off, const int64_t* list_ids,
                                const float* rotation, const uint32_t* codes, const float* factors,
                                const void* base, int32_t storage, float eps0, bbc_index** out);

typedef struct {
  double ncand_ratio;  /* r >= 1: the collector keeps K_c = min(ceil(r*k), S) candidates */
  int32_t collector;   /* BBC_COLLECT_* */
  int32_t buckets;     /* m in [1, 256]; 0 picks the default */
  int32_t nsample;     /* codebook sample: at least this many nearest probed lists (0 = 8), */
  int32_t sample_factor; /* ... extended until they hold sample_factor * K_c keys (0 = 2) */
  int32_t device_io;   /* 1: queries and outputs are device pointers on `stream` and the
                          call returns once the work is enqueued; 0: host pointers, the
                          call returns when the results are in place */
  void* stream;        /* hipStream_t; NULL = the default stream */
  int32_t lut_u8;      /* PQ only, 1: one-byte distance tables with integer sums (row f2 of the
                          fast-scan accounting).  Per (query, list) table: lo_m = the smallest
                          entry of sub-space m, span = the largest (max - lo_m) over m, delta =
                          span / 255 (1 if not positive), u = min(255, floor((entry - lo_m) *
                          (1 / delta) + 0.5)); key = sum_m lo_m + K * delta with K the integer
                          sum of u over the code's sub-spaces (float32 steps in that order).
                          Candidates follow these keys; exact re-rank unchanged.  Supported for
                          the grouped scan shapes (8-bit M=16 or 32, 4-bit M=32 or 48) */
  int32_t early_rerank; /* PQ with the bucket collector, 1: the early re-rank of Algorithm 4 (the
                          improved IVF+PQ search).  The codebook also predicts the threshold
                          bucket tau_pred = the bucket of the sample's j-th smallest key,
                          j = ceil(K_c * (sample keys) / S); while the lists after the sample are
                          scanned, every object whose bucket is below tau_pred gets its exact
                          distance at once, and a candidate among them is not re-ranked again.
                          Results are identical to the plain search.  Needs float32 tables, a
                          grouped scan shape and float32 rows (BBC_EUNSUPPORTED otherwise) */
  int32_t keep_all_keys; /* bucket collector, 1: the scan keeps every key (no relaxed-threshold
                          filter at d_max), so the collector reads every scanned key, as the heap
                          and sort collectors do: a like-for-like collector comparison.  Results
                          are identical */
} bbc_search_params;

/* Search nq queries [nq][d] float32.  k[nq] and nprobe[nq] are host arrays
 * (per-query values; 1 <= nprobe <= nlist, k >= 1).  out_offsets[nq+1] is
 * the host prefix sum of k; out_ids [sum k] int64, out_dists [sum k] float32,
 * out_counts [nq] int32 receive the results (see the conventions above). */
int32_t bbc_search(const bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                   const int32_t* nprobe, const bbc_search_params* params, const int64_t* out_offsets,
                   int64_t* out_ids, float* out_dists, int32_t* out_counts);

/* Allocation-free search, for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as bbc_search with
 * params->device_io = 1 (queries and outputs are device pointers on
 * params->stream; k, nprobe and out_offsets are host arrays), but the
 * workspace is a fixed device array of BBC_NOALLOC_MAX_BYTES held by each
 * GPU the library runs on until the process ends, and the metadata block is
 * staged through a fixed host buffer: the call makes no hipMalloc, hipFree
 * or other allocating call.  Errors: BBC_EINVAL when device_io is 0 (and as
 * bbc_search); BBC_ENOMEM, before anything is enqueued, when the batch needs
 * more workspace than BBC_NOALLOC_MAX_BYTES (bbc_query_bytes bounds each
 * query's share; split such batches).  Every allocation-free call on one GPU
 * shares that GPU's array and the array keeps the last call's contents:
 * calls that overlap on the device (different streams, or different indexes
 * on the same GPU) race, so order them on one stream or by events.  The
 * host side of these calls is serialised process-wide.  Only the 256-byte
 * aligned sub-buffers the search lays out are used; what must start at zero
 * is cleared by its kernels. */
#define BBC_NOALLOC_MAX_BYTES ((size_t)128 << 20)
int32_t bbc_search_noalloc(const bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                           const int32_t* nprobe, const bbc_search_params* params, const int64_t* out_offsets,
                           int64_t* out_ids, float* out_dists, int32_t* out_counts);

/* Intermediate state of a search, for checking every step (host arrays;
 * any pointer may be NULL).  Ragged arrays use the prefix sums given:
 * probe_*: by nprobe; cand_*: by cand_cap[q] = the per-query candidate
 * capacity reported in n_cand_cap.  For the bucket collector: codebook
 * (dmin, delta, map[nq][256]), threshold bucket tau, s, bucket counts
 * [nq][m] of all scanned keys, and the size of the threshold bucket; the
 * heap and sort collectors leave these fields (and n_sample_lists,
 * n_survivors, n_sample_keys) untouched. */
typedef struct {
  int32_t* probe_lists; float* probe_keys;   /* [sum nprobe], nearest first */
  int64_t* n_scanned;                        /* [nq] S */
  int64_t* n_cand;                           /* [nq] K_c */
  int32_t* n_recheck;                        /* [nq] lists rechecked in FP32 by the probe */
  float* dmin; float* delta; uint8_t* map;   /* [nq], [nq], [nq][256] */
  int32_t* tau; int64_t* s; int32_t* bucket_counts; int64_t* n_boundary; /* [nq],[nq],[nq][m],[nq] */
  float* est_keys;                           /* [sum S]: estimated keys in probe order */
  int64_t* est_off;                          /* [nq+1] prefix sums of S (output) */
  int64_t* cand_ids;                         /* candidate ids, ragged by cand_off */
  float* cand_exact;                         /* their exact keys (same order) */
  int64_t* cand_off;                         /* [nq+1] prefix sums of K_c (output) */
  int32_t* n_sample_lists;                   /* [nq] probed lists in the codebook sample */
  int64_t* n_survivors;                      /* [nq] keys kept by the relaxed-threshold filter */
  int64_t* n_sample_keys;                    /* [nq] keys in the codebook sample lists */
  float* est_lb; float* est_ub;              /* RaBitQ: [sum S] bounds in the est_keys order */
  int64_t* n_visited;                        /* RaBitQ: [nq] exact distances computed (the objects the
                                                bounded walk visited; all of C in the wide form) */
  int32_t* kernel_forms;                     /* [4] kernel variants the batch ran: codebook sample slots
                                                per thread (16, 32, 48; 0 = sample read from memory;
                                                -1 = none), final top-k candidates per thread (8, 16,
                                                24, 32; 0 = memory form), RaBitQ scan grid (1 = one
                                                block per pair on a 1-D grid, 2 = 2-D grid, 3 = pairs
                                                grouped by list; -1 = none), 0 */
  int32_t* walk_path;                        /* RaBitQ: [nq] how the bounded walk found its exact stop
                                                point: 0 no search, 1 in LDS, 2 in global memory,
                                                3 item-by-item walk (a bound check failed) */
  int32_t* tau_pred;                         /* early re-rank: [nq] predicted threshold bucket */
  int64_t* n_early;                          /* early re-rank: [nq] exact distances computed during the
                                                scan (objects after the sample below tau_pred) */
  int64_t* n_early_used;                     /* early re-rank: [nq] candidates whose early exact key was
                                                used (all early candidates of buckets below tau) */
} bbc_search_trace;

/* bbc_search with host I/O that also fills `trace` (est_keys, cand_ids and
 * cand_exact need the sizes reported by a first call with them NULL). */
int32_t bbc_search_traced(const bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                          const int32_t* nprobe, const bbc_search_params* params,
                          const int64_t* out_offsets, int64_t* out_ids, float* out_dists,
                          int32_t* out_counts, bbc_search_trace* trace);

/* Device bytes of per-query scratch a search with this k and nprobe needs
 * (upper bound); used for admission by memory. Negative on error. */
int64_t bbc_query_bytes(const bbc_index* ix, int32_t k, int32_t nprobe, const bbc_search_params* params);

#define BBC_FIELD_CENTROIDS 0 /* [nlist][d] float32 */
#define BBC_FIELD_LIST_OFF 1  /* [nlist+1] int64 */
#define BBC_FIELD_LIST_IDS 2  /* [n] int64 */
#define BBC_FIELD_CODES 3     /* [n][pq_m] uint8, one code per byte */
#define BBC_FIELD_CODEBOOK 4  /* [pq_m][2^bits][d/pq_m] float32 */
#define BBC_FIELD_RABITQ_CODES 5    /* [n][d/32] uint32, list-slot order */
#define BBC_FIELD_RABITQ_FACTORS 6  /* [n][4] float32 (nr, f, g, popcount), list-slot order */
#define BBC_FIELD_ROT_CENTROIDS 7   /* [nlist][d] float32: P^T c_j */
#define BBC_FIELD_ROTATION 8        /* [d][d] float32: P (RaBitQ) */
#define BBC_FIELD_BASE 9            /* [n][d] float32 (float16 when stored so), row-id order */

/* Sizes of an index: any pointer may be NULL (storage: BBC_STORAGE_*). */
int32_t bbc_index_info(const bbc_index* ix, int64_t* n, int32_t* d, int32_t* nlist, int32_t* metric,
                       int32_t* quant, int32_t* pq_m, int32_t* pq_bits, int32_t* storage);
/* Copy one array of the index (BBC_FIELD_*) to host memory of `bytes` bytes. */
int32_t bbc_index_get(const bbc_index* ix, int32_t field, void* dst, int64_t bytes);
void bbc_index_free(bbc_index* ix);

/* Index files: bbc_index_save writes the index's host-side image (what the
 * create calls take) to `path`; bbc_index_load reads one and creates the
 * index on `device` (BBC_EINVAL for a missing, foreign, truncated,
 * inconsistent or altered file).  Layout, little-endian, arrays packed in
 * this order:
 *   char[8] "BBCIDX2\0"; int32 quant, metric, storage, d, nlist, pq_m,
 *   pq_bits, 0; int64 n; float32 eps0; int32 0            (56 bytes)
 *   float32 centroids [nlist][d]; int64 list_off [nlist+1]; int64 list_ids [n]
 *   PQ:     float32 codebook [pq_m][2^pq_bits][d/pq_m]; uint8 codes [n][pq_m]
 *   RaBitQ: float32 rotation [d][d]; uint32 codes [n][d/32]; float32 factors [n][4]
 *   base [n][d] float32, or float16 when storage = BBC_STORAGE_FP16, row-id order
 *   uint64 checksum: FNV-1a over the bytes after the header taken as
 *     little-endian 64-bit words (the last one zero-padded): h = 0xcbf29ce484222325,
 *     then h = (h ^ word) * 0x100000001b3 (mod 2^64) for each word
 * The caller owns `path`; the file holds the whole base (about n*d*4 bytes). */
int32_t bbc_index_save(const bbc_index* ix, const char* path);
int32_t bbc_index_load(int32_t device, const char* path, bbc_index** out);

/* Per-stage device time: when enabled, every kernel launch of a search is
 * bracketed by HIP events recorded on the search stream; bbc_stage_times
 * waits for them and returns, per stage, the summed milliseconds and the
 * launch count since the last reset (stages: 0 probe (coarse GEMM and
 * select), 1 pair sort and scan of the codebook sample lists (RaBitQ: the
 * rotation of the queries), 2 scan of the remaining lists through the
 * relaxed threshold (RaBitQ: the bounds of every scanned object; one kernel
 * launch per search), 3 collector (the bucket collection or a comparator;
 * RaBitQ in the wide form: the lower-bound bins of the candidates),
 * 6 the collector codebook, 4 re-rank
 * (RaBitQ: the bounded walk, after the exact keys of all candidates in the
 * wide form), 5 final top-k).  A RaBitQ batch of at most as many queries as
 * the device has compute units takes the wide form with the exact keys
 * from a device-wide grid; a larger batch takes the wide form with the
 * exact keys computed tile-major (each tile of a list's rows staged once per
 * group of queries).  A PQ batch re-ranks tile-major where the rows have at
 * most 128 elements. */
int32_t bbc_stage_timing(int32_t enable);
int32_t bbc_stage_times(double* ms, int64_t* launches, int32_t nstages, int32_t reset);

/* Plans: one batch shape (nq, k[], nprobe[], fixed device buffers) whose
 * per-query metadata is uploaded once and whose whole launch sequence is
 * captured into a HIP graph, replayed by bbc_plan_execute on any stream.
 * The plan owns its workspace (searches through the index itself keep
 * working meanwhile).  params->device_io must be 1; queries, outputs and
 * out_offsets are fixed at creation: each execution searches whatever the
 * query buffer holds then and overwrites the outputs.  With autotune = 1
 * (PQ, bucket collector) the scan block geometry (5 shapes: one block per
 * CU of 512 threads with 2 or 1 codes per pass or of 1024 threads, two
 * blocks per CU of 512 threads with 2 or 1 codes, their float tables of
 * 8-bit codes over 32 sub-spaces in two slices), the bucket
 * count (64, 128, 256), the codebook sample's size (2, 3 or 4 times K_c
 * keys) and the collector's LDS budget for sorting the threshold bucket
 * (1024 or 4096 members) are chosen by a coordinate search, two passes,
 * each candidate timed on the batch itself (the choice is read back by
 * bbc_plan_info).  Results are identical for every choice. */
typedef struct bbc_plan bbc_plan;
int32_t bbc_plan_create(bbc_index* ix, int64_t nq, const int32_t* k, const int32_t* nprobe,
                        const bbc_search_params* params, const float* queries, const int64_t* out_offsets,
                        int64_t* out_ids, float* out_dists, int32_t* out_counts, int32_t autotune, bbc_plan** out);
int32_t bbc_plan_execute(bbc_plan* plan, void* stream);
int32_t bbc_plan_info(const bbc_plan* plan, int32_t* scan_variant, int32_t* buckets, int32_t* sample_factor,
                      int32_t* bcap, int64_t* workspace_bytes);
void bbc_plan_free(bbc_plan* plan);

/* Serving form (continuous batching; a request loop with admission by the
 * device memory of the candidate buffers).  Single requests (one query, its
 * k and nprobe) are submitted one by one and answered from device batches.
 * A worker thread owned by the server keeps up to `lanes` batches in flight
 * (0 = 2), each on its own stream with its own workspace, so requests
 * admitted while others run overlap with them on the device.  Admission
 * takes the pending requests in arrival order into a new batch while a lane
 * is free, at most max_slots requests are in flight, and the sum of
 * bbc_query_bytes over the requests in flight stays within
 * mem_budget_bytes; a finished batch frees its slots and bytes.  Each
 * result is the one bbc_search returns for that request alone with
 * `params` (collector, ncand_ratio, buckets, sampling); params->device_io
 * and params->stream are ignored.  The index must outlive the server.
 *
 * bbc_server_create: the server and its worker on the current device.
 * bbc_server_submit: copies the query [d] float32 (host) and returns a
 *   ticket > 0 without waiting for the device; BBC_ENOMEM if the request
 *   alone exceeds the budget, BBC_EINVAL for bad k / nprobe or non-finite
 *   values.
 * bbc_server_poll: if the ticket's result is ready, copies it to the host
 *   arrays ids [k] int64 and dists [k] float32 and fills `info`, any of
 *   them NULL to skip, hands the ticket back and returns the request's
 *   status; BBC_EBUSY if it is not ready yet; BBC_EINVAL for a ticket never
 *   issued or already collected.
 * bbc_server_wait: as poll, waiting up to timeout_ms (BBC_EBUSY after).
 * bbc_server_stats: batches run, requests answered, largest batch, most
 *   requests in flight at once, requests waiting (any pointer may be NULL).
 * bbc_server_destroy: answers every request already submitted, stops the
 *   worker and frees the server (uncollected results are dropped). */
typedef struct bbc_server bbc_server;
typedef struct {
  int32_t count;       /* results found (<= k; the rest of ids is -1) */
  int32_t status;      /* BBC_OK or the batch's error */
  int64_t latency_ns;  /* submission to completion, as seen by the worker */
  int64_t n_scanned;   /* codes scanned (S) */
  int64_t n_reranked;  /* exact distances computed: K_c (PQ); RaBitQ: the objects the bounded walk
                          visited, or all of the candidate set C in the wide form */
  int64_t batch_size;  /* requests in the batch that answered this one */
} bbc_request_info;
int32_t bbc_server_create(bbc_index* ix, const bbc_search_params* params, int64_t mem_budget_bytes,
                          int32_t max_slots, int32_t lanes, bbc_server** out);
int32_t bbc_server_submit(bbc_server* srv, const float* query, int32_t k, int32_t nprobe, uint64_t* ticket);
int32_t bbc_server_poll(bbc_server* srv, uint64_t ticket, int64_t* ids, float* dists, bbc_request_info* info);
int32_t bbc_server_wait(bbc_server* srv, uint64_t ticket, int32_t timeout_ms, int64_t* ids, float* dists,
                        bbc_request_info* info);
int32_t bbc_server_stats(bbc_server* srv, int64_t* batches, int64_t* requests, int64_t* max_batch,
                         int64_t* max_inflight, int64_t* pending);
void bbc_server_destroy(bbc_server* srv);

const char* bbc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BBC_H_ */

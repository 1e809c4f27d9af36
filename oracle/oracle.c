/*
 * Oracle for the large-k IVF query path with a bucket-based result collector
 * (BBC, arxiv 2604.01960).  TEST INFRASTRUCTURE ONLY: the tests, the smoke
 * check and the CPU-baseline leg of the benchmark call it; the product path
 * never does.  It shares no source with the GPU library.
 *
 * Plain and slow on purpose: every step is a direct loop, selection is a full
 * qsort by (key, id), and there is no blocking or fusion.  OpenMP runs
 * independent queries (or independent rows of the index build) in parallel;
 * inside one query everything is sequential.
 *
 * Arithmetic is IEEE binary32 with round-to-nearest-even, in the fixed
 * operation order below; the compiler contracts nothing (built with
 * -ffp-contract=off, no fast-math), and a fused multiply-add appears only
 * where written as fmaf (one rounding of a*b + c).  The GPU path implements
 * the same order independently; that is what makes bit-exact ids possible
 * when thousands of neighbours sit within a relative distance band of 1e-6
 * of each other.
 *
 *   canon_l2(a,b): vectors padded with zeros to a multiple of 256; 4-element
 *     chunk c goes to virtual lane c%64 at step c/64; each lane starts at +0
 *     and for each step and element e=0..3 does  t=(a-b); acc=fmaf(t,t,acc);
 *     lanes are combined by acc[l] = acc[l] + acc[l+off] for off=32,16,..,1.
 *   canon_ip: same with acc = fmaf(a,b,acc).
 *   PQ table entry: r = q - c (once per element), then sequentially over the
 *     sub-vector elements  t = r - C; acc = fmaf(t,t,acc), from acc = +0.
 *   PQ key: acc = +0; acc = acc + LUT[m][code_m] for m = 0..M-1.
 *   Total order: (key, id) with numeric key comparison, ties by smaller id.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

#define NLANES 64
#define KM_SPLIT_UP (1.0f + 1.0f / 1024.0f)
#define KM_SPLIT_DOWN (1.0f - 1.0f / 1024.0f)
#define NCELLS 256

/* ------------------------------------------------------------------------ */
/* Canonical distances                                                       */
/* ------------------------------------------------------------------------ */

float orc_canon_l2(const float* a, const float* b, int32_t d) {
  float acc[NLANES];
  for (int l = 0; l < NLANES; ++l) acc[l] = 0.0f;
  int nchunk = (d + 3) / 4;
  for (int c = 0; c < nchunk; ++c) {
    int lane = c % NLANES;
    for (int e = 0; e < 4; ++e) {
      int i = 4 * c + e;
      float av = i < d ? a[i] : 0.0f;
      float bv = i < d ? b[i] : 0.0f;
      float t = av - bv;
      acc[lane] = fmaf(t, t, acc[lane]);
    }
  }
  for (int off = NLANES / 2; off >= 1; off /= 2)
    for (int l = 0; l < off; ++l) acc[l] = acc[l] + acc[l + off];
  return acc[0];
}

float orc_canon_ip(const float* a, const float* b, int32_t d) {
  float acc[NLANES];
  for (int l = 0; l < NLANES; ++l) acc[l] = 0.0f;
  int nchunk = (d + 3) / 4;
  for (int c = 0; c < nchunk; ++c) {
    int lane = c % NLANES;
    for (int e = 0; e < 4; ++e) {
      int i = 4 * c + e;
      float av = i < d ? a[i] : 0.0f;
      float bv = i < d ? b[i] : 0.0f;
      acc[lane] = fmaf(av, bv, acc[lane]);
    }
  }
  for (int off = NLANES / 2; off >= 1; off /= 2)
    for (int l = 0; l < off; ++l) acc[l] = acc[l] + acc[l + off];
  return acc[0];
}

/* Sequential squared distance over a short sub-vector (PQ sub-spaces). */
static float seq_l2(const float* a, const float* b, int32_t n) {
  float acc = 0.0f;
  for (int e = 0; e < n; ++e) {
    float t = a[e] - b[e];
    acc = fmaf(t, t, acc);
  }
  return acc;
}

void orc_canon_l2_batch(const float* q, const float* x, int64_t n, int32_t d, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = orc_canon_l2(q, x + i * (int64_t)d, d);
}

void orc_canon_ip_batch(const float* q, const float* x, int64_t n, int32_t d, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = orc_canon_ip(q, x + i * (int64_t)d, d);
}

/* ------------------------------------------------------------------------ */
/* Total order on (key, id)                                                  */
/* ------------------------------------------------------------------------ */

typedef struct { float key; int32_t pad; int64_t id; } kv_t;

static int kv_cmp(const void* pa, const void* pb) {
  const kv_t* a = (const kv_t*)pa;
  const kv_t* b = (const kv_t*)pb;
  if (a->key < b->key) return -1;
  if (a->key > b->key) return 1;
  if (a->id < b->id) return -1;
  if (a->id > b->id) return 1;
  return 0;
}

typedef struct { double key; int64_t id; } kv64_t;

static int kv64_cmp(const void* pa, const void* pb) {
  const kv64_t* a = (const kv64_t*)pa;
  const kv64_t* b = (const kv64_t*)pb;
  if (a->key < b->key) return -1;
  if (a->key > b->key) return 1;
  if (a->id < b->id) return -1;
  if (a->id > b->id) return 1;
  return 0;
}

/* First kc of (key, id) ascending: the definition of what the collector must
 * return (exact top-kc of the estimated keys). */
int orc_topk_sort(const float* keys, const int64_t* ids, int64_t n, int64_t kc,
                  float* out_keys, int64_t* out_ids) {
  if (kc > n) kc = n;
  kv_t* v = (kv_t*)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
  if (!v) return ORC_ENOMEM;
  for (int64_t i = 0; i < n; ++i) { v[i].key = keys[i]; v[i].pad = 0; v[i].id = ids[i]; }
  qsort(v, (size_t)n, sizeof(kv_t), kv_cmp);
  for (int64_t i = 0; i < kc; ++i) { out_keys[i] = v[i].key; out_ids[i] = v[i].id; }
  free(v);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Result buffer (bucket-based collector)                                    */
/* ------------------------------------------------------------------------ */

/* Update: walk buckets in order accumulating their sizes; the threshold
 * bucket is the first one at which the running total reaches k.  Returns m
 * (standing for "infinity": accept everything) when the total is below k. */
int32_t orc_update(const int64_t* counts, int32_t m, int64_t k) {
  int64_t s = 0;
  for (int32_t i = 0; i < m; ++i) {
    s += counts[i];
    if (s >= k) return i;
  }
  return m;
}

/* Equal-width cell of a key (the floor/clamp of the bucket-id equation). */
static inline int32_t cell_of(float key, float dmin, float delta) {
  float t = (key - dmin) / delta;
  if (t < 0.0f) return 0;
  if (t >= 255.0f) return 255;
  return (int32_t)t;
}

int32_t orc_cell_of(float key, float dmin, float delta) { return cell_of(key, dmin, delta); }

/* Codebook from a sample of estimated keys (the keys of the nearest probed
 * lists): d_min and d_max are the extremes of the sample's top-kc keys, the
 * range is cut into 256 equal-width cells, and the cells are mapped onto m
 * buckets of (about) equal depth with respect to the sample's top-kc keys:
 * map[e] = min(m-1, floor(m * C_<e / T)) with C_<e the number of those keys
 * in cells before e and T their count. */
int orc_codebook(const float* sample_keys, const int64_t* sample_ids, int64_t ns, int64_t kc,
                 int32_t m, float* dmin_out, float* delta_out, uint8_t* map_out) {
  if (m < 1 || m > 256) return ORC_EINVAL;
  int64_t t = kc < ns ? kc : ns;
  if (t <= 0) {
    *dmin_out = 0.0f;
    *delta_out = 1.0f;
    for (int e = 0; e < NCELLS; ++e) map_out[e] = 0;
    return ORC_OK;
  }
  float* tk = (float*)malloc(sizeof(float) * (size_t)t);
  int64_t* ti = (int64_t*)malloc(sizeof(int64_t) * (size_t)t);
  if (!tk || !ti) { free(tk); free(ti); return ORC_ENOMEM; }
  int rc = orc_topk_sort(sample_keys, sample_ids, ns, t, tk, ti);
  if (rc) { free(tk); free(ti); return rc; }
  float dmin = tk[0];
  float dmax = tk[t - 1];
  float delta = (dmax - dmin) / 256.0f;
  if (!(delta > 0.0f)) delta = 1.0f;
  int64_t hist[NCELLS];
  for (int e = 0; e < NCELLS; ++e) hist[e] = 0;
  for (int64_t i = 0; i < t; ++i) hist[cell_of(tk[i], dmin, delta)] += 1;
  int64_t below = 0;
  for (int e = 0; e < NCELLS; ++e) {
    int64_t b = ((int64_t)m * below) / t;
    map_out[e] = (uint8_t)(b < m - 1 ? b : m - 1);
    below += hist[e];
  }
  *dmin_out = dmin;
  *delta_out = delta;
  free(tk);
  free(ti);
  return ORC_OK;
}

int32_t orc_bucket_of(float key, float dmin, float delta, const uint8_t* map) {
  return map[cell_of(key, dmin, delta)];
}

/* Number of nearest lists forming the codebook sample: at least nsample of
 * them, extended list by list until they hold sample_factor * kc keys (the
 * sample's kc-th key then lies at or beyond the kc-th key of the whole scan;
 * reading of the codebook section's "5 to 10 nearest clusters"). */
static int32_t sample_lists(const int64_t* grp_off, int32_t ngrp, int64_t kc, int32_t nsample,
                            int32_t sample_factor) {
  int32_t ns_grp = nsample < ngrp ? nsample : ngrp;
  while (ns_grp < ngrp && grp_off[ns_grp] < (int64_t)sample_factor * kc) ++ns_grp;
  return ns_grp;
}

/* What the bucket-based collector (Algorithm 1) produces for one query,
 * stated by its definition rather than by its procedure:
 *  - the codebook is built from the sample (the nearest probed lists, see
 *    sample_lists) by orc_codebook;
 *  - counts[b] is the number of scanned keys whose bucket (bucket-id
 *    equation) is b;
 *  - the threshold bucket tau is the first bucket whose running count
 *    reaches kc (Update, reading "cumulative >= k"); m when it never does;
 *  - s = kc - (keys in buckets below tau): how many of bucket tau's keys are
 *    kept;
 *  - the collected candidates are the kc smallest (key, id), ascending
 *    (Collect returns every key of the buckets below tau plus the best s of
 *    bucket tau, which is that set).
 * Keys arrive grouped by probed list, nearest list first (grp_off). */
int orc_collect_bbc(const float* keys, const int64_t* ids, const int64_t* grp_off, int32_t ngrp,
                    int64_t kc, int32_t m, int32_t nsample, int32_t sample_factor,
                    float* dmin_out, float* delta_out, uint8_t* map_out,
                    int32_t* tau_out, int64_t* s_out,
                    float* cand_keys, int64_t* cand_ids, int64_t* counts_full) {
  int64_t total = grp_off[ngrp];
  if (kc > total) kc = total;
  int32_t ns_grp = sample_lists(grp_off, ngrp, kc, nsample, sample_factor);
  int rc = orc_codebook(keys, ids, grp_off[ns_grp], kc, m, dmin_out, delta_out, map_out);
  if (rc) return rc;
  for (int32_t b = 0; b < m; ++b) counts_full[b] = 0;
  for (int64_t i = 0; i < total; ++i) counts_full[map_out[cell_of(keys[i], *dmin_out, *delta_out)]] += 1;
  int32_t tau = orc_update(counts_full, m, kc);
  int64_t below = 0;
  for (int32_t b = 0; b < tau && b < m; ++b) below += counts_full[b];
  *tau_out = tau;
  *s_out = kc - below;
  return orc_topk_sort(keys, ids, total, kc, cand_keys, cand_ids);
}

/* Early re-rank accounting of the improved IVF+PQ search (Algorithm 4) for
 * one query, keys grouped by probed list as for orc_collect_bbc.  The
 * predicted threshold bucket is the bucket of the sample's j-th smallest key
 * with j = ceil(kc * n_sample / S) (the sample's share of the scan times the
 * candidate count); tau_pred = 0 when j = 0.  Reading for a scan that runs in
 * two phases: the sample lists are scanned before tau_pred exists, so only
 * the lists after the sample re-rank early; there, every object whose bucket
 * lies below tau_pred gets its exact distance during the scan.  The
 * candidates and the final result are those of the plain definition (the kc
 * smallest estimated keys, then the k smallest exact keys): early re-ranking
 * only moves work.  Outputs: tau_pred, the early set's size, how many of it
 * are candidates, and how many candidates are left to re-rank afterwards. */
int orc_early_rerank(const float* keys, const int64_t* ids, const int64_t* grp_off, int32_t ngrp,
                     int64_t kc, int32_t m, int32_t nsample, int32_t sample_factor,
                     int32_t* tau_pred_out, int64_t* n_early, int64_t* n_early_cand, int64_t* n_late) {
  int64_t total = grp_off[ngrp];
  if (kc > total) kc = total;
  *tau_pred_out = 0; *n_early = 0; *n_early_cand = 0; *n_late = kc;
  if (kc <= 0) return ORC_OK;
  int32_t ns_grp = sample_lists(grp_off, ngrp, kc, nsample, sample_factor);
  int64_t ns = grp_off[ns_grp];
  float dmin, delta;
  uint8_t map[NCELLS];
  int rc = orc_codebook(keys, ids, ns, kc, m, &dmin, &delta, map);
  if (rc) return rc;
  /* j = ceil(kc * ns / total) in exact integer arithmetic */
  int64_t j = (kc * ns + total - 1) / total;
  int32_t tau_pred = 0;
  if (j > 0) {
    float* sk = (float*)malloc(sizeof(float) * (size_t)j);
    int64_t* si = (int64_t*)malloc(sizeof(int64_t) * (size_t)j);
    if (!sk || !si) { free(sk); free(si); return ORC_ENOMEM; }
    rc = orc_topk_sort(keys, ids, ns, j, sk, si);
    if (!rc) tau_pred = map[cell_of(sk[j - 1], dmin, delta)];
    free(sk); free(si);
    if (rc) return rc;
  }
  float* ck = (float*)malloc(sizeof(float) * (size_t)kc);
  int64_t* ci = (int64_t*)malloc(sizeof(int64_t) * (size_t)kc);
  if (!ck || !ci) { free(ck); free(ci); return ORC_ENOMEM; }
  rc = orc_topk_sort(keys, ids, total, kc, ck, ci);
  if (rc) { free(ck); free(ci); return rc; }
  /* candidate membership by (key, id): kc-th pair bounds the set */
  const float kk = ck[kc - 1];
  const int64_t ki = ci[kc - 1];
  int64_t ne = 0, nec = 0;
  for (int64_t i = ns; i < total; ++i) {
    if (map[cell_of(keys[i], dmin, delta)] >= tau_pred) continue;
    ++ne;
    if (keys[i] < kk || (keys[i] == kk && ids[i] <= ki)) ++nec;
  }
  free(ck); free(ci);
  *tau_pred_out = tau_pred;
  *n_early = ne;
  *n_early_cand = nec;
  *n_late = kc - nec;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* IVF probe                                                                 */
/* ------------------------------------------------------------------------ */

/* Probe key of list j: canonical squared L2 to its centroid, or the negated
 * canonical inner product for the inner-product metric. */
static float probe_key(const float* q, const float* c, int32_t d, int32_t metric) {
  return metric == 0 ? orc_canon_l2(q, c, d) : -orc_canon_ip(q, c, d);
}

/* The nprobe lists with the smallest (key, list id), in that order. */
static int probe_one(const float* q, const float* centroids, int32_t nlist, int32_t d,
                     int32_t metric, int32_t nprobe, int32_t* out_lists, float* out_keys) {
  kv_t* v = (kv_t*)malloc(sizeof(kv_t) * (size_t)nlist);
  if (!v) return ORC_ENOMEM;
  for (int32_t j = 0; j < nlist; ++j) {
    v[j].key = probe_key(q, centroids + (int64_t)j * d, d, metric);
    v[j].pad = 0;
    v[j].id = j;
  }
  qsort(v, (size_t)nlist, sizeof(kv_t), kv_cmp);
  for (int32_t i = 0; i < nprobe; ++i) {
    out_lists[i] = (int32_t)v[i].id;
    if (out_keys) out_keys[i] = v[i].key;
  }
  free(v);
  return ORC_OK;
}

/* Batched probe; out arrays are ragged by probe_off (nq+1 prefix of nprobe). */
int orc_probe(const float* queries, int64_t nq, int32_t d, const float* centroids, int32_t nlist,
              int32_t metric, const int32_t* nprobe, const int64_t* probe_off,
              int32_t* out_lists, float* out_keys) {
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic)
  for (int64_t qi = 0; qi < nq; ++qi) {
    int rc = probe_one(queries + qi * d, centroids, nlist, d, metric, nprobe[qi],
                       out_lists + probe_off[qi], out_keys ? out_keys + probe_off[qi] : NULL);
    if (rc) {
#pragma omp critical
      err = rc;
    }
  }
  return err;
}

/* ------------------------------------------------------------------------ */
/* PQ: tables and estimated keys                                             */
/* ------------------------------------------------------------------------ */

/* Residual table for one (query, list): lut[m][b] over ksub codewords. */
void orc_pq_lut(const float* q, const float* centroid, int32_t d, int32_t M, int32_t ksub,
                const float* codebook, float* lut) {
  int32_t dsub = d / M;
  float* r = (float*)malloc(sizeof(float) * (size_t)d);
  for (int i = 0; i < d; ++i) r[i] = q[i] - centroid[i];
  for (int32_t m = 0; m < M; ++m)
    for (int32_t b = 0; b < ksub; ++b)
      lut[(int64_t)m * ksub + b] =
          seq_l2(r + m * dsub, codebook + ((int64_t)m * ksub + b) * dsub, dsub);
  free(r);
}

float orc_pq_key(const float* lut, const uint8_t* code, int32_t M, int32_t ksub) {
  float acc = 0.0f;
  for (int32_t m = 0; m < M; ++m) acc = acc + lut[(int64_t)m * ksub + code[m]];
  return acc;
}

void orc_pq_keys(const float* lut, const uint8_t* codes, int64_t n, int32_t M, int32_t ksub,
                 float* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = orc_pq_key(lut, codes + i * M, M, ksub);
}

/* One-byte table with integer sums (row f2; the paper counts one byte per
 * table entry for its 4-bit fast-scan codes, and sums of small integers are
 * exact in any order).  Reading, one scale per (query, list) table so that
 * the sub-space codes add up as integers:
 *   lo_m  = min over b of lut[m][b]
 *   span  = max over m of (max_b lut[m][b] - lo_m)      (float32 subtraction)
 *   delta = span / 255, or 1 when that is not positive; inv = 1 / delta
 *   u[m][b] = min(255, floor(((lut[m][b] - lo_m) * inv) + 0.5))
 *             (float32 subtract, multiply, add in that order; the value is
 *             never negative, so floor is truncation)
 *   base  = lo_0 + lo_1 + ... + lo_{M-1}, sequential from +0.
 * A code's estimated key is base + K * delta with K = sum_m u[m][code_m]
 * (an exact integer; K * delta rounded once, then the add rounded once). */
void orc_pq_lut_u8(const float* lut, int32_t M, int32_t ksub, uint8_t* u, float* base_out,
                   float* delta_out) {
  float span = 0.0f, base = 0.0f;
  for (int32_t m = 0; m < M; ++m) {
    const float* row = lut + (int64_t)m * ksub;
    float lo = row[0], hi = row[0];
    for (int32_t b = 1; b < ksub; ++b) {
      if (row[b] < lo) lo = row[b];
      if (row[b] > hi) hi = row[b];
    }
    const float w = hi - lo;
    if (w > span) span = w;
    base = base + lo;
  }
  float delta = span / 255.0f;
  if (!(delta > 0.0f)) delta = 1.0f;
  const float inv = 1.0f / delta;
  for (int32_t m = 0; m < M; ++m) {
    const float* row = lut + (int64_t)m * ksub;
    float lo = row[0];
    for (int32_t b = 1; b < ksub; ++b)
      if (row[b] < lo) lo = row[b];
    for (int32_t b = 0; b < ksub; ++b) {
      float t = row[b] - lo;
      t = t * inv;
      t = t + 0.5f;
      uint32_t v = (uint32_t)t;
      u[(int64_t)m * ksub + b] = (uint8_t)(v > 255u ? 255u : v);
    }
  }
  *base_out = base;
  *delta_out = delta;
}

float orc_pq_key_u8(const uint8_t* u, const uint8_t* code, int32_t M, int32_t ksub, float base,
                    float delta) {
  uint32_t K = 0;
  for (int32_t m = 0; m < M; ++m) K += u[(int64_t)m * ksub + code[m]];
  const float t = (float)K * delta;
  return base + t;
}

void orc_pq_keys_u8(const uint8_t* u, const uint8_t* codes, int64_t n, int32_t M, int32_t ksub, float base,
                    float delta, float* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = orc_pq_key_u8(u, codes + i * M, M, ksub, base, delta);
}

/* ------------------------------------------------------------------------ */
/* Index build: IVF k-means and PQ                                           */
/* ------------------------------------------------------------------------ */

/* Nearest centroid by canonical squared L2, ties to the smaller list id. */
void orc_kmeans_assign(const float* x, const int64_t* rows, int64_t n, int32_t d,
                       const float* c, int32_t nc, int32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const float* xi = x + (rows ? rows[i] : i) * (int64_t)d;
    int32_t best = 0;
    float bk = orc_canon_l2(xi, c, d);
    for (int32_t j = 1; j < nc; ++j) {
      float kj = orc_canon_l2(xi, c + (int64_t)j * d, d);
      if (kj < bk) { bk = kj; best = j; }
    }
    out[i] = best;
  }
}

/* Centroid = mean of its members: float64 sum over members in the given row
 * order, divided by the member count in float64, rounded once to float32.
 * Empty clusters are refilled by splitting the largest one (see below). */
int orc_kmeans_update(const float* x, const int64_t* rows, int64_t n, int32_t d,
                      const int32_t* assign, int32_t nc, float* c) {
  double* sum = (double*)calloc((size_t)nc * d, sizeof(double));
  int64_t* cnt = (int64_t*)calloc((size_t)nc, sizeof(int64_t));
  if (!sum || !cnt) { free(sum); free(cnt); return ORC_ENOMEM; }
  for (int64_t i = 0; i < n; ++i) {
    const float* xi = x + (rows ? rows[i] : i) * (int64_t)d;
    double* s = sum + (int64_t)assign[i] * d;
    for (int e = 0; e < d; ++e) s[e] = s[e] + (double)xi[e];
    cnt[assign[i]] += 1;
  }
  for (int32_t j = 0; j < nc; ++j) {
    if (cnt[j] == 0) continue;
    for (int e = 0; e < d; ++e)
      c[(int64_t)j * d + e] = (float)(sum[(int64_t)j * d + e] / (double)cnt[j]);
  }
  /* Empty clusters, in ascending id order, each split the currently largest
   * cluster (ties to the smaller id): the two centroids become the largest
   * one scaled by (1 + eps) and (1 - eps) on alternating elements, and the
   * member count is shared between them (floor half to the empty one). */
  for (int32_t e = 0; e < nc; ++e) {
    if (cnt[e] != 0) continue;
    int32_t big = 0;
    for (int32_t j = 1; j < nc; ++j)
      if (cnt[j] > cnt[big]) big = j;
    if (cnt[big] < 2) break;
    float* ce = c + (int64_t)e * d;
    float* cb = c + (int64_t)big * d;
    for (int i = 0; i < d; ++i) {
      float v = cb[i];
      if (i % 2 == 0) { ce[i] = v * KM_SPLIT_UP; cb[i] = v * KM_SPLIT_DOWN; }
      else            { ce[i] = v * KM_SPLIT_DOWN; cb[i] = v * KM_SPLIT_UP; }
    }
    cnt[e] = cnt[big] / 2;
    cnt[big] -= cnt[e];
  }
  free(sum);
  free(cnt);
  return ORC_OK;
}

/* Lloyd iterations on the training rows, seeded by the rows at init_pos. */
int orc_kmeans_train(const float* x, int32_t d, const int64_t* train_rows, int64_t ntrain,
                     const int64_t* init_pos, int32_t nc, int32_t iters, float* c) {
  for (int32_t j = 0; j < nc; ++j)
    memcpy(c + (int64_t)j * d, x + train_rows[init_pos[j]] * (int64_t)d, sizeof(float) * d);
  int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)ntrain);
  if (!a) return ORC_ENOMEM;
  for (int32_t it = 0; it < iters; ++it) {
    orc_kmeans_assign(x, train_rows, ntrain, d, c, nc, a);
    int rc = orc_kmeans_update(x, train_rows, ntrain, d, a, nc, c);
    if (rc) { free(a); return rc; }
  }
  free(a);
  return ORC_OK;
}

/* Per-sub-space k-means on residual sub-vectors: resid is [n][d] (already
 * the residuals of the training rows, in ascending row order). */
int orc_pq_train(const float* resid, int64_t n, int32_t d, int32_t M, int32_t ksub,
                 const int64_t* init_pos, int32_t iters, float* codebook) {
  int32_t dsub = d / M;
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic)
  for (int32_t m = 0; m < M; ++m) {
    float* cb = codebook + (int64_t)m * ksub * dsub;
    float* sub = (float*)malloc(sizeof(float) * (size_t)n * dsub);
    int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double* sum = (double*)malloc(sizeof(double) * (size_t)ksub * dsub);
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)ksub);
    if (!sub || !a || !sum || !cnt) {
#pragma omp critical
      err = ORC_ENOMEM;
      free(sub); free(a); free(sum); free(cnt);
      continue;
    }
    for (int64_t i = 0; i < n; ++i)
      memcpy(sub + i * dsub, resid + i * (int64_t)d + (int64_t)m * dsub, sizeof(float) * dsub);
    for (int32_t b = 0; b < ksub; ++b)
      memcpy(cb + (int64_t)b * dsub, sub + init_pos[(int64_t)m * ksub + b] * dsub, sizeof(float) * dsub);
    for (int32_t it = 0; it < iters; ++it) {
      for (int64_t i = 0; i < n; ++i) {
        int32_t best = 0;
        float bk = seq_l2(sub + i * dsub, cb, dsub);
        for (int32_t b = 1; b < ksub; ++b) {
          float kb = seq_l2(sub + i * dsub, cb + (int64_t)b * dsub, dsub);
          if (kb < bk) { bk = kb; best = b; }
        }
        a[i] = best;
      }
      for (int64_t z = 0; z < (int64_t)ksub * dsub; ++z) sum[z] = 0.0;
      for (int32_t b = 0; b < ksub; ++b) cnt[b] = 0;
      for (int64_t i = 0; i < n; ++i) {
        for (int e = 0; e < dsub; ++e) sum[(int64_t)a[i] * dsub + e] += (double)sub[i * dsub + e];
        cnt[a[i]] += 1;
      }
      for (int32_t b = 0; b < ksub; ++b) {
        if (cnt[b] == 0) continue;
        for (int e = 0; e < dsub; ++e)
          cb[(int64_t)b * dsub + e] = (float)(sum[(int64_t)b * dsub + e] / (double)cnt[b]);
      }
    }
    free(sub); free(a); free(sum); free(cnt);
  }
  return err;
}

/* Code of each residual: per sub-space, the nearest codeword (sequential
 * sub-vector distance), ties to the smaller codeword index. */
void orc_pq_encode(const float* resid, int64_t n, int32_t d, int32_t M, int32_t ksub,
                   const float* codebook, uint8_t* codes) {
  int32_t dsub = d / M;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t m = 0; m < M; ++m) {
      const float* r = resid + i * (int64_t)d + (int64_t)m * dsub;
      const float* cb = codebook + (int64_t)m * ksub * dsub;
      int32_t best = 0;
      float bk = seq_l2(r, cb, dsub);
      for (int32_t b = 1; b < ksub; ++b) {
        float kb = seq_l2(r, cb + (int64_t)b * dsub, dsub);
        if (kb < bk) { bk = kb; best = b; }
      }
      codes[i * M + m] = (uint8_t)best;
    }
  }
}

/* Residuals x[row] - c[assign[row]] for the given rows (elementwise float32). */
void orc_residuals(const float* x, const int64_t* rows, int64_t n, int32_t d,
                   const float* c, const int32_t* assign_all, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t row = rows ? rows[i] : i;
    const float* xi = x + row * (int64_t)d;
    const float* ci = c + (int64_t)assign_all[row] * d;
    for (int e = 0; e < d; ++e) out[i * (int64_t)d + e] = xi[e] - ci[e];
  }
}

/* ------------------------------------------------------------------------ */
/* Search, PQ flavour (probe -> tables and keys -> collect -> re-rank)       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t n; int32_t d; int32_t nlist;
  const float* centroids;      /* [nlist][d] */
  const int64_t* list_off;     /* [nlist+1] */
  const int64_t* list_ids;     /* [n] original row of each list slot */
  const uint8_t* codes;        /* [n][M], list order, one code per byte */
  int32_t M; int32_t ksub;
  const float* codebook;       /* [M][ksub][d/M] */
  const float* base;           /* [n][d] original row order */
  int32_t metric;              /* 0 = L2 (PQ path supports L2 only) */
  int32_t lut_u8;              /* 1: one-byte tables with integer sums (orc_pq_lut_u8) */
} orc_pq_index;

/* Optional per-query intermediate outputs (any pointer may be NULL). */
typedef struct {
  int32_t* probe_lists;   /* ragged by probe_off */
  float* probe_keys;      /* ragged by probe_off */
  const int64_t* probe_off;
  int64_t* n_scanned;     /* [nq] S */
  int64_t* n_cand;        /* [nq] K_c */
  float* cand_keys;       /* ragged by cand_off: the K_c candidates, (key,id) ascending */
  int64_t* cand_ids;
  const int64_t* cand_off;
} orc_pq_debug;

static int search_pq_one(const orc_pq_index* ix, const float* q, int32_t k, int32_t nprobe,
                         double ratio, int64_t* out_ids, float* out_dists, int32_t* out_count,
                         const orc_pq_debug* dbg, int64_t qi) {
  const int32_t d = ix->d;
  int32_t* lists = (int32_t*)malloc(sizeof(int32_t) * (size_t)nprobe);
  float* lkeys = (float*)malloc(sizeof(float) * (size_t)nprobe);
  float* lut = (float*)malloc(sizeof(float) * (size_t)ix->M * ix->ksub);
  uint8_t* lut8 = (uint8_t*)malloc((size_t)ix->M * ix->ksub);
  if (!lists || !lkeys || !lut || !lut8) {
    free(lists); free(lkeys); free(lut); free(lut8);
    return ORC_ENOMEM;
  }
  int rc = probe_one(q, ix->centroids, ix->nlist, d, ix->metric, nprobe, lists, lkeys);
  if (rc) { free(lists); free(lkeys); free(lut); free(lut8); return rc; }
  if (dbg && dbg->probe_lists)
    for (int32_t i = 0; i < nprobe; ++i) dbg->probe_lists[dbg->probe_off[qi] + i] = lists[i];
  if (dbg && dbg->probe_keys)
    for (int32_t i = 0; i < nprobe; ++i) dbg->probe_keys[dbg->probe_off[qi] + i] = lkeys[i];

  int64_t S = 0;
  for (int32_t i = 0; i < nprobe; ++i) S += ix->list_off[lists[i] + 1] - ix->list_off[lists[i]];
  kv_t* est = (kv_t*)malloc(sizeof(kv_t) * (size_t)(S > 0 ? S : 1));
  if (!est) { free(lists); free(lkeys); free(lut); free(lut8); return ORC_ENOMEM; }
  int64_t w = 0;
  for (int32_t i = 0; i < nprobe; ++i) {
    int32_t j = lists[i];
    orc_pq_lut(q, ix->centroids + (int64_t)j * d, d, ix->M, ix->ksub, ix->codebook, lut);
    float base = 0.0f, delta = 1.0f;
    if (ix->lut_u8) orc_pq_lut_u8(lut, ix->M, ix->ksub, lut8, &base, &delta);
    for (int64_t p = ix->list_off[j]; p < ix->list_off[j + 1]; ++p) {
      est[w].key = ix->lut_u8 ? orc_pq_key_u8(lut8, ix->codes + p * ix->M, ix->M, ix->ksub, base, delta)
                              : orc_pq_key(lut, ix->codes + p * ix->M, ix->M, ix->ksub);
      est[w].pad = 0;
      est[w].id = ix->list_ids[p];
      ++w;
    }
  }
  int64_t kc = (int64_t)ceil(ratio * (double)k);
  if (kc > S) kc = S;
  qsort(est, (size_t)S, sizeof(kv_t), kv_cmp);
  if (dbg && dbg->n_scanned) dbg->n_scanned[qi] = S;
  if (dbg && dbg->n_cand) dbg->n_cand[qi] = kc;
  if (dbg && dbg->cand_keys)
    for (int64_t i = 0; i < kc; ++i) {
      dbg->cand_keys[dbg->cand_off[qi] + i] = est[i].key;
      dbg->cand_ids[dbg->cand_off[qi] + i] = est[i].id;
    }

  /* exact re-rank of the kc candidates */
  for (int64_t i = 0; i < kc; ++i) {
    const float* x = ix->base + est[i].id * (int64_t)d;
    est[i].key = ix->metric == 0 ? orc_canon_l2(q, x, d) : -orc_canon_ip(q, x, d);
  }
  qsort(est, (size_t)kc, sizeof(kv_t), kv_cmp);
  int64_t cnt = kc < k ? kc : k;
  for (int64_t i = 0; i < k; ++i) {
    if (i < cnt) {
      out_ids[i] = est[i].id;
      out_dists[i] = ix->metric == 0 ? est[i].key : -est[i].key;
    } else {
      out_ids[i] = -1;
      out_dists[i] = ix->metric == 0 ? INFINITY : -INFINITY;
    }
  }
  *out_count = (int32_t)cnt;
  free(est);
  free(lists);
  free(lkeys);
  free(lut);
  free(lut8);
  return ORC_OK;
}

int orc_search_pq(int64_t n, int32_t d, int32_t nlist, const float* centroids,
                  const int64_t* list_off, const int64_t* list_ids, const uint8_t* codes,
                  int32_t M, int32_t ksub, const float* codebook, const float* base, int32_t metric,
                  const float* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                  double ratio, int32_t lut_u8, const int64_t* out_off, int64_t* out_ids,
                  float* out_dists, int32_t* out_counts,
                  int32_t* dbg_probe_lists, float* dbg_probe_keys, const int64_t* dbg_probe_off,
                  int64_t* dbg_n_scanned, int64_t* dbg_n_cand,
                  float* dbg_cand_keys, int64_t* dbg_cand_ids, const int64_t* dbg_cand_off) {
  orc_pq_index ix = {n, d, nlist, centroids, list_off, list_ids, codes, M, ksub, codebook, base, metric,
                     lut_u8};
  orc_pq_debug dbg = {dbg_probe_lists, dbg_probe_keys, dbg_probe_off, dbg_n_scanned, dbg_n_cand,
                      dbg_cand_keys, dbg_cand_ids, dbg_cand_off};
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic)
  for (int64_t qi = 0; qi < nq; ++qi) {
    int rc = search_pq_one(&ix, queries + qi * d, k[qi], nprobe[qi], ratio,
                           out_ids + out_off[qi], out_dists + out_off[qi], out_counts + qi,
                           &dbg, qi);
    if (rc) {
#pragma omp critical
      err = rc;
    }
  }
  return err;
}

/* ------------------------------------------------------------------------ */
/* RaBitQ codes and bounds (the bounded quantizer the paper integrates with, */
/* cited in the background and Algorithms 2-3), in the fixed FP32 order:     */
/*                                                                          */
/*   rotation: y = P^T v, y_i = sum over e = 0..D-1 of (P[e][i] * v[e]),      */
/*     product rounded, then added, sequentially from +0;                    */
/*   code of object x in list j: r = x - c_j, y = P^T r, bit i = (y_i > 0);  */
/*     nr = sqrt(canon_l2(x, c_j)); s1 = sum_i |y_i| (sequential);          */
/*     <o_bar, o> = s1 / (nr * sqrt(D)), clamped to <= 1 (1 when nr = 0,    */
/*     with all bits 0); f = 1 / <o_bar, o>;                                 */
/*     g = sqrt(1 - <o_bar,o>^2) / <o_bar,o>; pc = popcount of the code;     */
/*   query side, per (query, list) for L2 (y = P^T q - P^T c_j) or once per  */
/*     query for IP (y = P^T q): vl = min y, vu = max y,                     */
/*     delta = (vu - vl) * fl(1/15); u_i = clamp(floor((y_i - vl) / delta   */
/*     + 0.5), 0, 15) (0 when delta = 0); four bit planes of u;             */
/*     c1 = 2 delta / sqrt(D), c2 = 2 vl / sqrt(D),                          */
/*     c3 = (delta / sqrt(D)) * sum_i u_i, c4 = sqrt(D) * vl;                */
/*   per object: ip = sum_b 2^b popcount(code & plane_b) (integer);         */
/*     est = (((c1 * ip + c2 * pc) - c3) - c4) * f;                          */
/*     L2: key = (nr*nr + nq2) - (2 nr) * est, with nq2 = canon_l2(q, c_j);  */
/*         err = (((2 nr) * sqrt(nq2)) * g) * epsc;                          */
/*     IP: key = -(ipc + nr * est), ipc = canon_ip(q, c_j);                  */
/*         err = ((nr * sqrt(canon_ip(q, q))) * g) * epsc;                   */
/*     epsc = eps0 / sqrt(D - 1); lb = key - err; ub = key + err.            */
/* ------------------------------------------------------------------------ */

void orc_rotate(const float* P, int32_t D, const float* v, int64_t n, float* y) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    const float* vv = v + r * D;
    float* yy = y + r * D;
    for (int32_t i = 0; i < D; ++i) {
      float acc = 0.0f;
      for (int32_t e = 0; e < D; ++e) {
        float t = P[(int64_t)e * D + i] * vv[e];
        acc = acc + t;
      }
      yy[i] = acc;
    }
  }
}

/* Codes [n][D/32] (bit i of object p at word i/32, bit i%32) and factors
 * [n][4] = (nr, f, g, pc) of the objects in list-slot order. */
int orc_rabitq_encode(const float* x, const int64_t* list_ids, const int64_t* list_off, int32_t nlist,
                      const float* centroids, int32_t D, const float* P, uint32_t* codes, float* factors) {
  if (D % 64) return ORC_EINVAL;
  const int32_t W = D / 32;
  const float sD = sqrtf((float)D);
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic)
  for (int32_t j = 0; j < nlist; ++j) {
    float* r = (float*)malloc(sizeof(float) * (size_t)D * 2);
    if (!r) {
#pragma omp critical
      err = ORC_ENOMEM;
      continue;
    }
    float* y = r + D;
    const float* c = centroids + (int64_t)j * D;
    for (int64_t p = list_off[j]; p < list_off[j + 1]; ++p) {
      const float* xv = x + list_ids[p] * (int64_t)D;
      for (int32_t e = 0; e < D; ++e) r[e] = xv[e] - c[e];
      for (int32_t i = 0; i < D; ++i) {
        float acc = 0.0f;
        for (int32_t e = 0; e < D; ++e) {
          float t = P[(int64_t)e * D + i] * r[e];
          acc = acc + t;
        }
        y[i] = acc;
      }
      const float nr = sqrtf(orc_canon_l2(xv, c, D));
      uint32_t* code = codes + p * W;
      float* fac = factors + p * 4;
      for (int32_t w = 0; w < W; ++w) code[w] = 0u;
      if (nr == 0.0f) {
        fac[0] = 0.0f; fac[1] = 1.0f; fac[2] = 0.0f; fac[3] = 0.0f;
        continue;
      }
      float s1 = 0.0f;
      uint32_t pc = 0;
      for (int32_t i = 0; i < D; ++i) {
        s1 = s1 + fabsf(y[i]);
        if (y[i] > 0.0f) { code[i / 32] |= 1u << (i % 32); ++pc; }
      }
      float den = nr * sD;
      float ipoo = s1 / den;
      if (ipoo > 1.0f) ipoo = 1.0f;
      float g = ipoo * ipoo;
      g = 1.0f - g;
      g = sqrtf(g);
      g = g / ipoo;
      fac[0] = nr;
      fac[1] = 1.0f / ipoo;
      fac[2] = g;
      fac[3] = (float)pc;
    }
    free(r);
  }
  return err;
}

/* Query-side quantization of one rotated vector y[D]: planes [4][D/32] and
 * scal = (vl, delta, c1, c2, c3, c4). */
void orc_rabitq_prep(const float* y, int32_t D, uint32_t* planes, float* scal) {
  const int32_t W = D / 32;
  float vl = y[0], vu = y[0];
  for (int32_t i = 1; i < D; ++i) {
    if (y[i] < vl) vl = y[i];
    if (y[i] > vu) vu = y[i];
  }
  const float inv15 = 1.0f / 15.0f;
  float delta = vu - vl;
  delta = delta * inv15;
  for (int32_t b = 0; b < 4 * W; ++b) planes[b] = 0u;
  int32_t sum_u = 0;
  for (int32_t i = 0; i < D; ++i) {
    int32_t u = 0;
    if (delta > 0.0f) {
      float t = y[i] - vl;
      t = t / delta;
      t = t + 0.5f;
      t = floorf(t);
      u = t < 0.0f ? 0 : (t > 15.0f ? 15 : (int32_t)t);
    }
    sum_u += u;
    for (int32_t b = 0; b < 4; ++b)
      if ((u >> b) & 1) planes[b * W + i / 32] |= 1u << (i % 32);
  }
  const float sD = sqrtf((float)D);
  float c1 = 2.0f * delta;
  c1 = c1 / sD;
  float c2 = 2.0f * vl;
  c2 = c2 / sD;
  float c3 = delta / sD;
  c3 = c3 * (float)sum_u;
  float c4 = sD * vl;
  scal[0] = vl; scal[1] = delta; scal[2] = c1; scal[3] = c2; scal[4] = c3; scal[5] = c4;
}

static inline int32_t popc32(uint32_t v) {
  int32_t c = 0;
  while (v) { v &= v - 1u; ++c; }
  return c;
}

/* Estimated inner product term est for one object (before the metric). */
static float rabitq_est(const uint32_t* code, const float* fac, const uint32_t* planes, const float* scal,
                        int32_t W) {
  int64_t ip = 0;
  for (int32_t b = 0; b < 4; ++b) {
    int64_t c = 0;
    for (int32_t w = 0; w < W; ++w) c += popc32(code[w] & planes[b * W + w]);
    ip += c << b;
  }
  float est = scal[2] * (float)ip;
  float t = scal[3] * fac[3];
  est = est + t;
  est = est - scal[4];
  est = est - scal[5];
  est = est * fac[1];
  return est;
}

/* key, lb, ub of n objects (codes/factors of consecutive slots) for one
 * prepared query side.  L2: a = nq2 (canon_l2(q, c_j)); IP: a = ipc
 * (canon_ip(q, c_j)) and qn = sqrt(canon_ip(q, q)). */
void orc_rabitq_bounds(const uint32_t* codes, const float* factors, int64_t n, int32_t D, const uint32_t* planes,
                       const float* scal, int32_t metric, float a, float qn, float eps0, float* key,
                       float* lb, float* ub) {
  const int32_t W = D / 32;
  const float epsc = eps0 / sqrtf((float)(D - 1));
  const float nq = sqrtf(a);
  for (int64_t p = 0; p < n; ++p) {
    const float* fac = factors + p * 4;
    const float nr = fac[0];
    const float est = rabitq_est(codes + p * W, fac, planes, scal, W);
    float kk, e;
    if (metric == 0) {
      float t = nr * nr;
      t = t + a;
      float u = 2.0f * nr;
      u = u * est;
      kk = t - u;
      e = 2.0f * nr;
      e = e * nq;
      e = e * fac[2];
      e = e * epsc;
    } else {
      float v = nr * est;
      v = a + v;
      kk = -v;
      e = nr * qn;
      e = e * fac[2];
      e = e * epsc;
    }
    key[p] = kk;
    lb[p] = kk - e;
    ub[p] = kk + e;
  }
}

typedef struct {
  int64_t n; int32_t d; int32_t nlist;
  const float* centroids;      /* [nlist][d] */
  const float* rot_centroids;  /* [nlist][d] = P^T c_j (orc_rotate) */
  const float* P;              /* [d][d] */
  const int64_t* list_off;
  const int64_t* list_ids;
  const uint32_t* codes;       /* [n][d/32], list order */
  const float* factors;        /* [n][4], list order */
  const float* base;           /* [n][d] original row order (fp32) */
  int32_t metric;
  float eps0;
} orc_rabitq_index;

/* binary max-heap of (key, id) */
static void heap_down(kv_t* h, int64_t n, int64_t i) {
  while (1) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < n && kv_cmp(&h[l], &h[m]) > 0) m = l;
    if (r < n && kv_cmp(&h[r], &h[m]) > 0) m = r;
    if (m == i) return;
    kv_t t = h[i]; h[i] = h[m]; h[m] = t;
    i = m;
  }
}
static void heap_up(kv_t* h, int64_t i) {
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (kv_cmp(&h[i], &h[p]) <= 0) return;
    kv_t t = h[i]; h[i] = h[p]; h[p] = t;
    i = p;
  }
}

/* The bounded re-rank: objects in ascending (lb, id); walking them with R =
 * the best k by (exact key, id) so far, stop before object t when R holds k
 * objects and lb_t > the k-th exact key of R (equality does not stop);
 * otherwise compute t's exact key and offer it to R.  Returns the number of
 * exact keys computed; R (unsorted) in res[0, *nres). */
static int64_t bounded_walk(const kv_t* order, int64_t S, int64_t k, const float* q, const orc_rabitq_index* ix,
                            kv_t* res, int64_t* nres) {
  int64_t nr = 0, t = 0;
  for (; t < S; ++t) {
    if (nr == k && order[t].key > res[0].key) break;
    const float* x = ix->base + order[t].id * (int64_t)ix->d;
    kv_t e;
    e.key = ix->metric == 0 ? orc_canon_l2(q, x, ix->d) : -orc_canon_ip(q, x, ix->d);
    e.pad = 0;
    e.id = order[t].id;
    if (nr < k) {
      res[nr] = e;
      heap_up(res, nr);
      ++nr;
    } else if (kv_cmp(&e, &res[0]) < 0) {
      res[0] = e;
      heap_down(res, nr, 0);
    }
  }
  *nres = nr;
  return t;
}

typedef struct {
  int32_t* probe_lists; float* probe_keys; const int64_t* probe_off;
  int64_t* n_scanned;
  float* est_key; float* est_lb; float* est_ub; const int64_t* est_off;  /* by scanned slot, probe order */
  int64_t* n_visited;
} orc_rabitq_debug;

static int search_rabitq_one(const orc_rabitq_index* ix, const float* q, int32_t k, int32_t nprobe,
                             int64_t* out_ids, float* out_dists, int32_t* out_count,
                             const orc_rabitq_debug* dbg, int64_t qi) {
  const int32_t D = ix->d, W = D / 32;
  int32_t* lists = (int32_t*)malloc(sizeof(int32_t) * (size_t)nprobe);
  float* lkeys = (float*)malloc(sizeof(float) * (size_t)nprobe);
  float* qr = (float*)malloc(sizeof(float) * (size_t)D * 2);
  uint32_t* planes = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)4 * W);
  if (!lists || !lkeys || !qr || !planes) { free(lists); free(lkeys); free(qr); free(planes); return ORC_ENOMEM; }
  float* y = qr + D;
  int rc = probe_one(q, ix->centroids, ix->nlist, D, ix->metric, nprobe, lists, lkeys);
  if (rc) { free(lists); free(lkeys); free(qr); free(planes); return rc; }
  if (dbg && dbg->probe_lists)
    for (int32_t i = 0; i < nprobe; ++i) dbg->probe_lists[dbg->probe_off[qi] + i] = lists[i];
  if (dbg && dbg->probe_keys)
    for (int32_t i = 0; i < nprobe; ++i) dbg->probe_keys[dbg->probe_off[qi] + i] = lkeys[i];
  int64_t S = 0;
  for (int32_t i = 0; i < nprobe; ++i) S += ix->list_off[lists[i] + 1] - ix->list_off[lists[i]];
  kv_t* ord = (kv_t*)malloc(sizeof(kv_t) * (size_t)(S > 0 ? S : 1));
  float* kb = (float*)malloc(sizeof(float) * (size_t)(S > 0 ? S : 1) * 3);
  kv_t* res = (kv_t*)malloc(sizeof(kv_t) * (size_t)(k > 0 ? k : 1));
  if (!ord || !kb || !res) {
    free(lists); free(lkeys); free(qr); free(planes); free(ord); free(kb); free(res);
    return ORC_ENOMEM;
  }
  orc_rotate(ix->P, D, q, 1, qr);
  float scal[6];
  float qn = 0.0f;
  if (ix->metric != 0) {
    orc_rabitq_prep(qr, D, planes, scal);
    qn = sqrtf(orc_canon_ip(q, q, D));
  }
  int64_t w = 0;
  for (int32_t i = 0; i < nprobe; ++i) {
    const int32_t j = lists[i];
    const int64_t n = ix->list_off[j + 1] - ix->list_off[j];
    float a;
    if (ix->metric == 0) {
      const float* cr = ix->rot_centroids + (int64_t)j * D;
      for (int32_t e = 0; e < D; ++e) y[e] = qr[e] - cr[e];
      orc_rabitq_prep(y, D, planes, scal);
      a = lkeys[i];                 /* canon_l2(q, c_j) */
    } else {
      a = -lkeys[i];                /* canon_ip(q, c_j) */
    }
    float* key = kb + w;
    float* lb = kb + S + w;
    float* ub = kb + 2 * S + w;
    orc_rabitq_bounds(ix->codes + ix->list_off[j] * W, ix->factors + ix->list_off[j] * 4, n, D, planes, scal,
                      ix->metric, a, qn, ix->eps0, key, lb, ub);
    for (int64_t p = 0; p < n; ++p) {
      ord[w + p].key = lb[p];
      ord[w + p].pad = 0;
      ord[w + p].id = ix->list_ids[ix->list_off[j] + p];
    }
    w += n;
  }
  if (dbg && dbg->n_scanned) dbg->n_scanned[qi] = S;
  if (dbg && dbg->est_key)
    for (int64_t p = 0; p < S; ++p) {
      dbg->est_key[dbg->est_off[qi] + p] = kb[p];
      dbg->est_lb[dbg->est_off[qi] + p] = kb[S + p];
      dbg->est_ub[dbg->est_off[qi] + p] = kb[2 * S + p];
    }
  qsort(ord, (size_t)S, sizeof(kv_t), kv_cmp);
  int64_t nres = 0;
  const int64_t visited = bounded_walk(ord, S, k, q, ix, res, &nres);
  if (dbg && dbg->n_visited) dbg->n_visited[qi] = visited;
  qsort(res, (size_t)nres, sizeof(kv_t), kv_cmp);
  for (int64_t i = 0; i < k; ++i) {
    if (i < nres) {
      out_ids[i] = res[i].id;
      out_dists[i] = ix->metric == 0 ? res[i].key : -res[i].key;
    } else {
      out_ids[i] = -1;
      out_dists[i] = ix->metric == 0 ? INFINITY : -INFINITY;
    }
  }
  *out_count = (int32_t)nres;
  free(lists); free(lkeys); free(qr); free(planes); free(ord); free(kb); free(res);
  return ORC_OK;
}

int orc_search_rabitq(int64_t n, int32_t d, int32_t nlist, const float* centroids, const float* rot_centroids,
                      const float* P, const int64_t* list_off, const int64_t* list_ids, const uint32_t* codes,
                      const float* factors, const float* base, int32_t metric, float eps0,
                      const float* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                      const int64_t* out_off, int64_t* out_ids, float* out_dists, int32_t* out_counts,
                      int32_t* dbg_probe_lists, float* dbg_probe_keys, const int64_t* dbg_probe_off,
                      int64_t* dbg_n_scanned, float* dbg_key, float* dbg_lb, float* dbg_ub,
                      const int64_t* dbg_est_off, int64_t* dbg_n_visited) {
  if (d % 64) return ORC_EINVAL;
  orc_rabitq_index ix = {n, d, nlist, centroids, rot_centroids, P, list_off, list_ids, codes, factors, base,
                         metric, eps0};
  orc_rabitq_debug dbg = {dbg_probe_lists, dbg_probe_keys, dbg_probe_off, dbg_n_scanned,
                          dbg_key, dbg_lb, dbg_ub, dbg_est_off, dbg_n_visited};
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic)
  for (int64_t qi = 0; qi < nq; ++qi) {
    int rc = search_rabitq_one(&ix, queries + qi * d, k[qi], nprobe[qi], out_ids + out_off[qi],
                               out_dists + out_off[qi], out_counts + qi, &dbg, qi);
    if (rc) {
#pragma omp critical
      err = rc;
    }
  }
  return err;
}

/* The minimal re-rank set of Observation 1 for one query: with Dist_k the
 * k-th smallest (exact key, id) over the n scanned objects, the objects whose
 * bound interval [lb, ub] contains Dist_k.  Needs the exact key of every
 * scanned object (the definition, not Algorithm 2's two-heap procedure).
 * n_min = |minimal set|; n_min_out = |minimal set united with the exact
 * top-k| (what a path that returns exact distances must compute at least);
 * both 0 when n < k (no boundary object).  dist_k = Dist_k (NaN when n < k). */
int orc_min_rerank(const float* lb, const float* ub, const float* exact, const int64_t* ids, int64_t n,
                   int64_t k, int64_t* n_min, int64_t* n_min_out, float* dist_k) {
  *n_min = 0;
  *n_min_out = 0;
  *dist_k = NAN;
  if (k <= 0 || n < k) return ORC_OK;
  float* tk = (float*)malloc(sizeof(float) * (size_t)k);
  int64_t* ti = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  if (!tk || !ti) { free(tk); free(ti); return ORC_ENOMEM; }
  int rc = orc_topk_sort(exact, ids, n, k, tk, ti);
  if (rc) { free(tk); free(ti); return rc; }
  const float dk = tk[k - 1];
  const int64_t dki = ti[k - 1];
  int64_t a = 0, b = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int in_min = lb[i] <= dk && dk <= ub[i];
    const int in_top = exact[i] < dk || (exact[i] == dk && ids[i] <= dki);
    a += in_min;
    b += in_min || in_top;
  }
  free(tk); free(ti);
  *n_min = a;
  *n_min_out = b;
  *dist_k = dk;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Ground truth: exact float64 k nearest over all rows                       */
/* ------------------------------------------------------------------------ */

int orc_exact_knn64(const float* base, int64_t n, int32_t d, const float* queries, int64_t nq,
                    int32_t k, int32_t metric, int64_t* out_ids, double* out_dists) {
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic)
  for (int64_t qi = 0; qi < nq; ++qi) {
    kv64_t* v = (kv64_t*)malloc(sizeof(kv64_t) * (size_t)n);
    if (!v) {
#pragma omp critical
      err = ORC_ENOMEM;
      continue;
    }
    const float* q = queries + qi * d;
    for (int64_t i = 0; i < n; ++i) {
      const float* x = base + i * (int64_t)d;
      double acc = 0.0;
      if (metric == 0) {
        for (int e = 0; e < d; ++e) { double t = (double)x[e] - (double)q[e]; acc += t * t; }
      } else {
        for (int e = 0; e < d; ++e) acc += (double)x[e] * (double)q[e];
        acc = -acc;
      }
      v[i].key = acc;
      v[i].id = i;
    }
    qsort(v, (size_t)n, sizeof(kv64_t), kv64_cmp);
    int32_t kk = k < n ? k : (int32_t)n;
    for (int32_t i = 0; i < k; ++i) {
      out_ids[qi * k + i] = i < kk ? v[i].id : -1;
      out_dists[qi * k + i] = i < kk ? (metric == 0 ? v[i].key : -v[i].key) : NAN;
    }
    free(v);
  }
  return err;
}

/* Threads of the OpenMP loops over queries (n < 1: all host cores). */
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n >= 1 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

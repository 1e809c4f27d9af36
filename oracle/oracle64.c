/*
 * O_64: the float64 shadow of the oracle's query paths (TEST
 * INFRASTRUCTURE ONLY, like oracle.c, and sharing nothing with the GPU
 * library).  The same steps as the float32 paths in oracle.c, carried out in
 * IEEE binary64 with plain sequential sums: probe, PQ residual tables and
 * estimated keys, the kc smallest estimated keys, the exact re-rank and the
 * k smallest exact keys (IVF+PQ); probe, rotation, 4-bit query
 * quantization, RaBitQ estimate and bounds, the bounded walk (IVF+RaBitQ).
 * Index arrays (centroids, codebooks, codes, factors, rows) are the float32
 * index both paths read; they are widened exactly to float64.
 *
 * It is never used for parity (that is the float32 oracle's job, in the
 * canonical order); it gives the float64 reference for the distance error
 * and recall of the float32 paths.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O64_OK 0
#define O64_ENOMEM (-2)
#define O64_EINVAL (-1)

typedef struct { double key; int64_t id; } kd_t;

static int kd_cmp(const void* pa, const void* pb) {
  const kd_t* a = (const kd_t*)pa;
  const kd_t* b = (const kd_t*)pb;
  if (a->key < b->key) return -1;
  if (a->key > b->key) return 1;
  if (a->id < b->id) return -1;
  if (a->id > b->id) return 1;
  return 0;
}

static double l2_64(const float* a, const float* b, int32_t d) {
  double acc = 0.0;
  for (int32_t e = 0; e < d; ++e) {
    double t = (double)a[e] - (double)b[e];
    acc += t * t;
  }
  return acc;
}

static double ip_64(const float* a, const float* b, int32_t d) {
  double acc = 0.0;
  for (int32_t e = 0; e < d; ++e) acc += (double)a[e] * (double)b[e];
  return acc;
}

/* exact key of row id: squared L2, or -<q, x> (float16 rows are passed as
 * their exact float32 values) */
static double exact_key64(const float* q, const float* base, int64_t id, int32_t d, int32_t metric) {
  const float* x = base + id * (int64_t)d;
  return metric == 0 ? l2_64(q, x, d) : -ip_64(q, x, d);
}

/* binary max-heap of (key, id) */
static void kd_down(kd_t* h, int64_t n, int64_t i) {
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < n && kd_cmp(&h[l], &h[m]) > 0) m = l;
    if (r < n && kd_cmp(&h[r], &h[m]) > 0) m = r;
    if (m == i) return;
    kd_t t = h[i]; h[i] = h[m]; h[m] = t;
    i = m;
  }
}

static void kd_up(kd_t* h, int64_t i) {
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (kd_cmp(&h[i], &h[p]) <= 0) return;
    kd_t t = h[i]; h[i] = h[p]; h[p] = t;
    i = p;
  }
}

/* nprobe lists with the smallest (key, list id) in float64 */
static int probe64(const float* q, const float* cent, int32_t nlist, int32_t d, int32_t metric, int32_t nprobe,
                   int32_t* lists, double* lkeys) {
  kd_t* v = (kd_t*)malloc(sizeof(kd_t) * (size_t)nlist);
  if (!v) return O64_ENOMEM;
  for (int32_t j = 0; j < nlist; ++j) {
    const float* c = cent + (int64_t)j * d;
    v[j].key = metric == 0 ? l2_64(q, c, d) : -ip_64(q, c, d);
    v[j].id = j;
  }
  qsort(v, (size_t)nlist, sizeof(kd_t), kd_cmp);
  for (int32_t i = 0; i < nprobe; ++i) {
    lists[i] = (int32_t)v[i].id;
    lkeys[i] = v[i].key;
  }
  free(v);
  return O64_OK;
}

static void write_out(const kd_t* r, int64_t nres, int32_t k, int32_t metric, int64_t* ids, double* dists,
                      int32_t* count) {
  for (int64_t i = 0; i < k; ++i) {
    if (i < nres) {
      ids[i] = r[i].id;
      dists[i] = metric == 0 ? r[i].key : -r[i].key;
    } else {
      ids[i] = -1;
      dists[i] = metric == 0 ? INFINITY : -INFINITY;
    }
  }
  *count = (int32_t)nres;
}

/* ------------------------------------------------------------------------ */
/* IVF+PQ in float64                                                        */
/* ------------------------------------------------------------------------ */

static int search_pq64_one(int32_t d, int32_t nlist, const float* cent, const int64_t* list_off,
                           const int64_t* list_ids, const uint8_t* codes, int32_t M, int32_t ksub,
                           const float* codebook, const float* base, const float* q, int32_t k, int32_t nprobe,
                           double ratio, int64_t* out_ids, double* out_dists, int32_t* out_count) {
  const int32_t dsub = d / M;
  int32_t* lists = (int32_t*)malloc(sizeof(int32_t) * (size_t)nprobe);
  double* lkeys = (double*)malloc(sizeof(double) * (size_t)nprobe);
  double* lut = (double*)malloc(sizeof(double) * (size_t)M * ksub);
  double* r = (double*)malloc(sizeof(double) * (size_t)d);
  if (!lists || !lkeys || !lut || !r) { free(lists); free(lkeys); free(lut); free(r); return O64_ENOMEM; }
  int rc = probe64(q, cent, nlist, d, 0, nprobe, lists, lkeys);
  int64_t S = 0;
  for (int32_t i = 0; i < nprobe; ++i) S += list_off[lists[i] + 1] - list_off[lists[i]];
  kd_t* est = (kd_t*)malloc(sizeof(kd_t) * (size_t)(S > 0 ? S : 1));
  if (rc || !est) { free(lists); free(lkeys); free(lut); free(r); free(est); return rc ? rc : O64_ENOMEM; }
  int64_t w = 0;
  for (int32_t i = 0; i < nprobe; ++i) {
    const int32_t j = lists[i];
    const float* c = cent + (int64_t)j * d;
    for (int32_t e = 0; e < d; ++e) r[e] = (double)q[e] - (double)c[e];
    for (int32_t m = 0; m < M; ++m)
      for (int32_t b = 0; b < ksub; ++b) {
        const float* cw = codebook + ((int64_t)m * ksub + b) * dsub;
        double acc = 0.0;
        for (int32_t e = 0; e < dsub; ++e) {
          double t = r[m * dsub + e] - (double)cw[e];
          acc += t * t;
        }
        lut[(int64_t)m * ksub + b] = acc;
      }
    for (int64_t p = list_off[j]; p < list_off[j + 1]; ++p) {
      const uint8_t* code = codes + p * M;
      double acc = 0.0;
      for (int32_t m = 0; m < M; ++m) acc += lut[(int64_t)m * ksub + code[m]];
      est[w].key = acc;
      est[w].id = list_ids[p];
      ++w;
    }
  }
  int64_t kc = (int64_t)ceil(ratio * (double)k);
  if (kc > S) kc = S;
  qsort(est, (size_t)S, sizeof(kd_t), kd_cmp);
  for (int64_t i = 0; i < kc; ++i) est[i].key = l2_64(q, base + est[i].id * (int64_t)d, d);
  qsort(est, (size_t)kc, sizeof(kd_t), kd_cmp);
  write_out(est, kc < k ? kc : k, k, 0, out_ids, out_dists, out_count);
  free(lists); free(lkeys); free(lut); free(r); free(est);
  return O64_OK;
}

int o64_search_pq(int64_t n, int32_t d, int32_t nlist, const float* centroids, const int64_t* list_off,
                  const int64_t* list_ids, const uint8_t* codes, int32_t M, int32_t ksub, const float* codebook,
                  const float* base, const float* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                  double ratio, const int64_t* out_off, int64_t* out_ids, double* out_dists, int32_t* out_counts) {
  (void)n;
  if (M <= 0 || d % M) return O64_EINVAL;
  int err = O64_OK;
#pragma omp parallel for schedule(dynamic)
  for (int64_t qi = 0; qi < nq; ++qi) {
    int rc = search_pq64_one(d, nlist, centroids, list_off, list_ids, codes, M, ksub, codebook, base,
                             queries + qi * d, k[qi], nprobe[qi], ratio, out_ids + out_off[qi],
                             out_dists + out_off[qi], out_counts + qi);
    if (rc) {
#pragma omp critical
      err = rc;
    }
  }
  return err;
}

/* ------------------------------------------------------------------------ */
/* IVF+RaBitQ in float64                                                    */
/* ------------------------------------------------------------------------ */

/* y = P^T v in float64 (sequential over e) */
static void rotate64(const float* P, int32_t D, const double* v, double* y) {
  for (int32_t i = 0; i < D; ++i) {
    double acc = 0.0;
    for (int32_t e = 0; e < D; ++e) acc += (double)P[(int64_t)e * D + i] * v[e];
    y[i] = acc;
  }
}

static int popc32_64(uint32_t v) {
  int c = 0;
  while (v) { v &= v - 1u; ++c; }
  return c;
}

/* quantized query side of a rotated vector: planes [4][D/32] and the five
 * scalars (delta, c1, c2, c3, c4) of the estimator, in float64 */
static void prep64(const double* y, int32_t D, uint32_t* planes, double* sc) {
  const int32_t W = D / 32;
  double vl = y[0], vu = y[0];
  for (int32_t i = 1; i < D; ++i) {
    if (y[i] < vl) vl = y[i];
    if (y[i] > vu) vu = y[i];
  }
  const double delta = (vu - vl) / 15.0;
  for (int32_t b = 0; b < 4 * W; ++b) planes[b] = 0u;
  int64_t sum_u = 0;
  for (int32_t i = 0; i < D; ++i) {
    int32_t u = 0;
    if (delta > 0.0) {
      double t = floor((y[i] - vl) / delta + 0.5);
      u = t < 0.0 ? 0 : (t > 15.0 ? 15 : (int32_t)t);
    }
    sum_u += u;
    for (int32_t b = 0; b < 4; ++b)
      if ((u >> b) & 1) planes[b * W + i / 32] |= 1u << (i % 32);
  }
  const double sD = sqrt((double)D);
  sc[0] = delta;
  sc[1] = 2.0 * delta / sD;
  sc[2] = 2.0 * vl / sD;
  sc[3] = delta / sD * (double)sum_u;
  sc[4] = sD * vl;
}

static double est64(const uint32_t* code, const float* fac, const uint32_t* planes, const double* sc, int32_t W) {
  int64_t ip = 0;
  for (int32_t b = 0; b < 4; ++b) {
    int64_t c = 0;
    for (int32_t w = 0; w < W; ++w) c += popc32_64(code[w] & planes[b * W + w]);
    ip += c << b;
  }
  return (sc[1] * (double)ip + sc[2] * (double)fac[3] - sc[3] - sc[4]) * (double)fac[1];
}

static int search_rabitq64_one(int32_t d, int32_t nlist, const float* cent, const float* P,
                               const int64_t* list_off, const int64_t* list_ids, const uint32_t* codes,
                               const float* factors, const float* base, int32_t metric,
                               double eps0, const float* q, int32_t k, int32_t nprobe, int64_t* out_ids,
                               double* out_dists, int32_t* out_count, int64_t* n_visited) {
  const int32_t D = d, W = D / 32;
  int32_t* lists = (int32_t*)malloc(sizeof(int32_t) * (size_t)nprobe);
  double* lkeys = (double*)malloc(sizeof(double) * (size_t)nprobe);
  double* buf = (double*)malloc(sizeof(double) * (size_t)D * 4);
  uint32_t* planes = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)4 * W);
  if (!lists || !lkeys || !buf || !planes) { free(lists); free(lkeys); free(buf); free(planes); return O64_ENOMEM; }
  double* qd = buf;
  double* qr = buf + D;
  double* cr = buf + 2 * D;
  double* y = buf + 3 * D;
  int rc = probe64(q, cent, nlist, D, metric, nprobe, lists, lkeys);
  int64_t S = 0;
  for (int32_t i = 0; i < nprobe; ++i) S += list_off[lists[i] + 1] - list_off[lists[i]];
  kd_t* ord = (kd_t*)malloc(sizeof(kd_t) * (size_t)(S > 0 ? S : 1));
  kd_t* res = (kd_t*)malloc(sizeof(kd_t) * (size_t)(k > 0 ? k : 1));
  if (rc || !ord || !res) {
    free(lists); free(lkeys); free(buf); free(planes); free(ord); free(res);
    return rc ? rc : O64_ENOMEM;
  }
  for (int32_t e = 0; e < D; ++e) qd[e] = (double)q[e];
  rotate64(P, D, qd, qr);
  double sc[5];
  double qn = 0.0;
  if (metric != 0) {
    prep64(qr, D, planes, sc);
    qn = sqrt(ip_64(q, q, D));
  }
  const double epsc = eps0 / sqrt((double)(D - 1));
  int64_t w = 0;
  for (int32_t i = 0; i < nprobe; ++i) {
    const int32_t j = lists[i];
    const float* c = cent + (int64_t)j * D;
    double a;
    if (metric == 0) {
      for (int32_t e = 0; e < D; ++e) y[e] = (double)c[e];
      rotate64(P, D, y, cr);
      for (int32_t e = 0; e < D; ++e) y[e] = qr[e] - cr[e];
      prep64(y, D, planes, sc);
      a = lkeys[i];               /* |q - c_j|^2 */
    } else {
      a = -lkeys[i];              /* <q, c_j> */
    }
    const double nq = sqrt(a);
    for (int64_t p = list_off[j]; p < list_off[j + 1]; ++p) {
      const float* fac = factors + p * 4;
      const double nr = (double)fac[0];
      const double est = est64(codes + p * W, fac, planes, sc, W);
      double key, err;
      if (metric == 0) {
        key = nr * nr + a - 2.0 * nr * est;
        err = 2.0 * nr * nq * (double)fac[2] * epsc;
      } else {
        key = -(a + nr * est);
        err = nr * qn * (double)fac[2] * epsc;
      }
      ord[w].key = key - err;   /* lower bound */
      ord[w].id = list_ids[p];
      ++w;
    }
  }
  qsort(ord, (size_t)S, sizeof(kd_t), kd_cmp);
  /* bounded walk in (lb, id) order: R = the best k by (exact, id); stop
   * before an object whose lb exceeds R's k-th exact key once R is full */
  int64_t nres = 0, t = 0;
  for (; t < S; ++t) {
    if (nres == k && ord[t].key > res[0].key) break;
    kd_t e;
    e.key = exact_key64(q, base, ord[t].id, D, metric);
    e.id = ord[t].id;
    if (nres < k) {
      res[nres] = e;
      kd_up(res, nres);
      ++nres;
    } else if (kd_cmp(&e, &res[0]) < 0) {
      res[0] = e;
      kd_down(res, nres, 0);
    }
  }
  *n_visited = t;
  qsort(res, (size_t)nres, sizeof(kd_t), kd_cmp);
  write_out(res, nres, k, metric, out_ids, out_dists, out_count);
  free(lists); free(lkeys); free(buf); free(planes); free(ord); free(res);
  return O64_OK;
}

int o64_search_rabitq(int64_t n, int32_t d, int32_t nlist, const float* centroids, const float* P,
                      const int64_t* list_off, const int64_t* list_ids, const uint32_t* codes, const float* factors,
                      const float* base, int32_t metric, double eps0,
                      const float* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                      const int64_t* out_off, int64_t* out_ids, double* out_dists, int32_t* out_counts,
                      int64_t* n_visited) {
  (void)n;
  if (d % 64) return O64_EINVAL;
  int err = O64_OK;
#pragma omp parallel for schedule(dynamic)
  for (int64_t qi = 0; qi < nq; ++qi) {
    int64_t nv = 0;
    int rc = search_rabitq64_one(d, nlist, centroids, P, list_off, list_ids, codes, factors, base, metric,
                                 eps0, queries + qi * d, k[qi], nprobe[qi], out_ids + out_off[qi],
                                 out_dists + out_off[qi], out_counts + qi, &nv);
    if (n_visited) n_visited[qi] = nv;
    if (rc) {
#pragma omp critical
      err = rc;
    }
  }
  return err;
}

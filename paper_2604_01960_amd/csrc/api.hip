// Host runtime and C ABI (include/bbc.h): index residency in HBM, per-call
// workspace planning, kernel sequencing on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bbc.h"
#include "kernels.h"

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

int32_t bbc::set_error(int32_t code, const std::string& msg) { return fail(code, msg); }

namespace {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return fail(_e == hipErrorOutOfMemory ? BBC_ENOMEM : BBC_EDEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(_e));              \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * count);
}

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline bool HIP_FAILED(hipError_t e) { return e != hipSuccess; }

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

bool all_finite(const float* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Grow-only device arena for per-call scratch.  `done` is recorded on the
// stream of each search after its last use of the arena, and the next search
// makes its own stream wait for it, so searches on different streams never
// overlap on the arena; growing it waits for that last use only (no
// device-wide synchronisation).
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  hipError_t reserve(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    size_t want = std::max(bytes, cap + cap / 2);
    if (base) {
      hipError_t e = done ? hipEventSynchronize(done) : hipDeviceSynchronize();
      if (e != hipSuccess) return e;
      hipFree(base);
      base = nullptr;
      cap = 0;
    }
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&base), want);
    if (e != hipSuccess) {
      base = nullptr;
      e = hipMalloc(reinterpret_cast<void**>(&base), bytes);
      if (e != hipSuccess) { base = nullptr; return e; }
      want = bytes;
    }
    cap = want;
    return hipSuccess;
  }
  // order a search on stream s after the previous search's use of the arena
  hipError_t acquire(hipStream_t s) { return done ? hipStreamWaitEvent(s, done, 0) : hipSuccess; }
  hipError_t release(hipStream_t s) { return done ? hipEventRecord(done, s) : hipSuccess; }
};

// Simple layout planner: offsets of 256-byte aligned sub-buffers.
struct Plan {
  size_t total = 0;
  size_t add(size_t bytes) {
    size_t off = total;
    total += (size_t)round_up((int64_t)std::max<size_t>(bytes, 1), 256);
    return off;
  }
};

struct StageTimer {
  bool enabled = false;
  std::mutex mu;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double ms[8] = {0};
  int64_t launches[8] = {0};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
StageTimer g_timer;
thread_local bool t_capturing = false;  // a plan is capturing its launches: no stage events

struct StageScope {
  hipStream_t s;
  int stage;
  hipEvent_t a = nullptr, b = nullptr;
  StageScope(hipStream_t s_, int st) : s(s_), stage(st) {
    if (!g_timer.enabled || t_capturing) return;
    std::lock_guard<std::mutex> g(g_timer.mu);
    a = g_timer.get();
    b = g_timer.get();
    if (a) hipEventRecord(a, s);
  }
  ~StageScope() {
    if (!a || !b) return;
    hipEventRecord(b, s);
    std::lock_guard<std::mutex> g(g_timer.mu);
    g_timer.pending.push_back({stage, a, b});
  }
};

}  // namespace

struct bbc_index {
  int device = 0;
  int64_t n = 0;
  int32_t d = 0, nlist = 0, metric = 0, quant = 0, M = 0, bits = 0, ksub = 0, dpad = 0;
  int32_t code_bytes = 0, code_stride = 0;
  int fp16 = 0;
  // device residency
  float* cent = nullptr;
  uint16_t* cent_bf16 = nullptr;
  float* cent_norm2 = nullptr;
  float* cent_norm = nullptr;
  int64_t* list_off = nullptr;
  int32_t* list_ids = nullptr;
  int32_t* pos_of_id = nullptr;
  int32_t* list_of_pos = nullptr;  // list holding each list slot
  uint8_t* codes = nullptr;
  float* codebook = nullptr;
  void* vectors = nullptr;  // list-slot order
  // RaBitQ
  uint32_t* rq_codes = nullptr;  // [n][rq_words]
  int32_t rq_words = 0;
  float* rq_factors = nullptr;   // [n][4]
  float* rot = nullptr;          // [d][d]
  float* rot_cent = nullptr;     // [nlist][d]
  float eps0 = 1.9f;
  // host metadata
  std::vector<int64_t> h_list_off;
  std::vector<int64_t> h_maxS;  // h_maxS[p] = sum of the p largest list sizes
  std::vector<int64_t> h_maxT;  // h_maxT[p] = sum of the p largest tile counts (tiles of 1 << h_maxT_ts rows)
  int h_maxT_ts = -1;
  int max_lds = 65536;
  int num_cu = 256;
  int nxcd = 8;
  int scan_variant = 0;  // grouped PQ scan block geometry (BBC_SCAN_VARIANT: 0 .. 4)
  int walk_form = 0;     // RaBitQ re-rank form (BBC_WALK_FORM: 0 by batch size, 1 per query, 2 wide, 3 wide with tile-major keys)
  int collect_bcap = 4096;  // threshold-bucket members sorted in LDS (BBC_COLLECT_BCAP: a power of two, 64..4096)
  int walk_qcap = 0;        // RaBitQ walk: objects above the k-th exact key resolved in LDS (BBC_WALK_QCAP:
                            // a power of two, 2..4096; 0 = the LDS capacity)
  int rq_scan_1d = 0;       // RaBitQ scan on a 1-D grid of pairs (BBC_RQ_SCAN_1D; taken anyway beyond 65535 queries)
  int rerank_form = 0;      // PQ re-rank form (BBC_RERANK_FORM: 0 tile-major where it applies, 1 per query)
  int64_t rt_sort_bins = (int64_t)1 << 30;  // tile-major sort: most bin counters (BBC_RERANK_SORT_BINS)
  // RaBitQ tile-major keys: C put in tile order by the walk's bin pass (1) or
  // by the candidate sort (0) (BBC_WALK_PRESORT)
  int walk_presort = 1;
  // RaBitQ scan order with tile-major keys: pairs by list, a run of lists per
  // XCD (1), or by query (0) (BBC_SCAN_BY_LIST)
  int scan_by_list = 1;
  // pair sorts by list: per-block LDS histograms (1) or device-wide atomics
  // (0) (BBC_PAIR_SORT)
  int pair_sort_lds = 1;
  // tile-major re-rank: runs found by binary search instead of the tile's
  // run list (BBC_RERANK_RUN_LIST=0; for tests of that path)
  int no_run_list = 0;
  // PQ float-table searches: the lists after the sample are filtered at the
  // upper edge of the first cell by which the sample's running count reaches
  // this fraction of K_c (BBC_FILTER_FRACTION; 0 or >= 1: at d_max), with a
  // rescan at d_max for a query it leaves short of K_c keys
  float filt_fraction = 0.0f;
  // final top-k: most results ranked in LDS (BBC_FINAL_LDS_CAP; 0: as many
  // as the LDS holds); larger result sets group their winners in memory
  int64_t final_lds_cap = 0;
  // RaBitQ wide form: the first round's keys reach this fraction of the way
  // from the k-th smallest lb's bin to U's bin (BBC_WALK_ALPHA; >= 1: one
  // round over all of C).  Unset (< 0): 0.8 with tile-major keys (large
  // batches), one round with the grid's keys (small batches, where a second
  // round's launches cost more latency than the keys they save)
  float walk_alpha = -1.0f;
  // per-call state
  Arena arena;
  char* pinned = nullptr;
  size_t pinned_cap = 0;
  hipEvent_t meta_done = nullptr;
  std::mutex mu;
};

namespace {

int32_t set_device(int dev) {
  int cnt = 0;
  HIP_TRY(hipGetDeviceCount(&cnt));
  if (dev < 0 || dev >= cnt) return fail(BBC_EINVAL, "device index out of range");
  HIP_TRY(hipSetDevice(dev));
  return BBC_OK;
}

void index_release(bbc_index* ix) {
  if (!ix) return;
  hipSetDevice(ix->device);
  hipDeviceSynchronize();
  hipFree(ix->cent); hipFree(ix->cent_bf16); hipFree(ix->cent_norm2); hipFree(ix->cent_norm);
  hipFree(ix->list_off); hipFree(ix->list_ids); hipFree(ix->pos_of_id); hipFree(ix->list_of_pos);
  hipFree(ix->codes);
  hipFree(ix->codebook); hipFree(ix->vectors);
  hipFree(ix->rq_codes); hipFree(ix->rq_factors); hipFree(ix->rot); hipFree(ix->rot_cent);
  if (ix->arena.base) hipFree(ix->arena.base);
  if (ix->arena.done) hipEventDestroy(ix->arena.done);
  if (ix->pinned) hipHostFree(ix->pinned);
  if (ix->meta_done) hipEventDestroy(ix->meta_done);
  delete ix;
}

int32_t upload_ivf_common(bbc_index* ix, const float* centroids, const int64_t* list_off,
                          const int64_t* list_ids) {
  const int64_t n = ix->n;
  const int32_t d = ix->d, nlist = ix->nlist;
  ix->dpad = (int32_t)round_up(d, 32);
  std::vector<uint16_t> cb16((size_t)nlist * ix->dpad, 0);
  std::vector<float> cn2(nlist), cn(nlist);
  for (int32_t j = 0; j < nlist; ++j) {
    float s = 0.0f;
    for (int32_t e = 0; e < d; ++e) {
      float v = centroids[(int64_t)j * d + e];
      cb16[(size_t)j * ix->dpad + e] = bf16_rne(v);
      s = s + v * v;
    }
    cn2[j] = s;
    cn[j] = std::sqrt(s);
  }
  std::vector<int32_t> ids32(n), pos(n, -1);
  for (int64_t p = 0; p < n; ++p) {
    int64_t id = list_ids[p];
    if (id < 0 || id >= n || pos[id] != -1) return fail(BBC_EINVAL, "list_ids is not a permutation of 0..n-1");
    pos[id] = (int32_t)p;
    ids32[p] = (int32_t)id;
  }
  HIP_TRY(dalloc(&ix->cent, (size_t)nlist * d));
  HIP_TRY(dalloc(&ix->cent_bf16, cb16.size()));
  HIP_TRY(dalloc(&ix->cent_norm2, nlist));
  HIP_TRY(dalloc(&ix->cent_norm, nlist));
  HIP_TRY(dalloc(&ix->list_off, nlist + 1));
  HIP_TRY(dalloc(&ix->list_ids, n));
  HIP_TRY(dalloc(&ix->pos_of_id, n));
  HIP_TRY(dalloc(&ix->list_of_pos, n));
  {
    std::vector<int32_t> lop(n);
    for (int32_t j = 0; j < nlist; ++j)
      for (int64_t p = list_off[j]; p < list_off[j + 1]; ++p) lop[p] = j;
    HIP_TRY(hipMemcpy(ix->list_of_pos, lop.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(ix->cent, centroids, sizeof(float) * nlist * d, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ix->cent_bf16, cb16.data(), sizeof(uint16_t) * cb16.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ix->cent_norm2, cn2.data(), sizeof(float) * nlist, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ix->cent_norm, cn.data(), sizeof(float) * nlist, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ix->list_off, list_off, sizeof(int64_t) * (nlist + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ix->list_ids, ids32.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ix->pos_of_id, pos.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  ix->h_list_off.assign(list_off, list_off + nlist + 1);
  std::vector<int64_t> sizes(nlist);
  for (int32_t j = 0; j < nlist; ++j) sizes[j] = list_off[j + 1] - list_off[j];
  std::sort(sizes.begin(), sizes.end(), std::greater<int64_t>());
  ix->h_maxS.assign(nlist + 1, 0);
  for (int32_t j = 0; j < nlist; ++j) ix->h_maxS[j + 1] = ix->h_maxS[j] + sizes[j];
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device) == hipSuccess && lds > 0)
    ix->max_lds = lds;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, ix->device) == hipSuccess && v > 0)
    ix->num_cu = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeNumberOfXccs, ix->device) == hipSuccess && v > 0)
    ix->nxcd = v;
  if (const char* sv = std::getenv("BBC_SCAN_VARIANT")) {
    const int x = std::atoi(sv);
    if (x >= 0 && x <= 4) ix->scan_variant = x;
  }
  if (const char* sv = std::getenv("BBC_WALK_FORM")) {
    const int x = std::atoi(sv);
    if (x >= 0 && x <= 3) ix->walk_form = x;
  }
  if (const char* sv = std::getenv("BBC_SCAN_BY_LIST")) {
    const int x = std::atoi(sv);
    if (x >= 0 && x <= 1) ix->scan_by_list = x;
  }
  if (const char* sv = std::getenv("BBC_FINAL_LDS_CAP")) {
    const long long x = std::atoll(sv);
    if (x >= 1024) ix->final_lds_cap = x;
  }
  if (const char* sv = std::getenv("BBC_RERANK_RUN_LIST")) ix->no_run_list = std::atoi(sv) == 0;
  if (const char* sv = std::getenv("BBC_FILTER_FRACTION")) {
    const float x = std::strtof(sv, nullptr);
    if (x >= 0.0f && x <= 1.0f) ix->filt_fraction = x;
  }
  if (const char* sv = std::getenv("BBC_PAIR_SORT")) {
    const int x = std::atoi(sv);
    if (x >= 0 && x <= 1) ix->pair_sort_lds = x;
  }
  if (const char* sv = std::getenv("BBC_WALK_PRESORT")) {
    const int x = std::atoi(sv);
    if (x >= 0 && x <= 1) ix->walk_presort = x;
  }
  if (const char* sv = std::getenv("BBC_RERANK_SORT_BINS")) {
    const long long x = std::atoll(sv);
    if (x >= 1) ix->rt_sort_bins = x;
  }
  if (const char* sv = std::getenv("BBC_RERANK_FORM")) {
    const int x = std::atoi(sv);
    if (x >= 0 && x <= 1) ix->rerank_form = x;
  }
  if (const char* sv = std::getenv("BBC_COLLECT_BCAP")) {
    const int x = std::atoi(sv);
    if (x >= 64 && x <= 4096 && (x & (x - 1)) == 0) ix->collect_bcap = x;
  }
  if (const char* sv = std::getenv("BBC_WALK_QCAP")) {
    const int x = std::atoi(sv);
    if (x >= 2 && x <= 4096 && (x & (x - 1)) == 0) ix->walk_qcap = x;
  }
  if (const char* sv = std::getenv("BBC_RQ_SCAN_1D")) ix->rq_scan_1d = std::atoi(sv) == 1;
  if (const char* sv = std::getenv("BBC_WALK_ALPHA")) {
    const float x = std::strtof(sv, nullptr);
    if (x >= 0.0f && x <= 64.0f) ix->walk_alpha = x;
  }
  HIP_TRY(hipEventCreateWithFlags(&ix->meta_done, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&ix->arena.done, hipEventDisableTiming));
  return BBC_OK;
}

}  // namespace

extern "C" {

const char* bbc_last_error(void) { return g_err.c_str(); }

int32_t bbc_build_index(int32_t device, const void* base, int64_t n, int32_t d, const bbc_build_params* p,
                        bbc_index** out) {
  if (!p) return fail(BBC_EINVAL, "params is NULL");
  if (p->quant == BBC_QUANT_RABITQ) return bbc::build_index_rabitq(device, base, n, d, p, out);
  if (p->quant != BBC_QUANT_PQ) return fail(BBC_EINVAL, "unknown quantizer");
  if (p->metric != BBC_METRIC_L2) return fail(BBC_EUNSUPPORTED, "the PQ path supports the L2 metric only");
  if (p->storage != BBC_STORAGE_FP32) return fail(BBC_EUNSUPPORTED, "the PQ path stores float32 only");
  return bbc::build_index_pq(device, static_cast<const float*>(base), n, d, p, out);
}

int32_t bbc_index_create_pq(int32_t device, int64_t n, int32_t d, int32_t nlist, int32_t metric,
                            const float* centroids, const int64_t* list_off, const int64_t* list_ids,
                            int32_t pq_m, int32_t pq_bits, const float* codebook, const uint8_t* codes,
                            const float* base, bbc_index** out) {
  if (!out) return fail(BBC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!centroids || !list_off || !list_ids || !codebook || !codes || !base)
    return fail(BBC_EINVAL, "NULL array");
  if (n < 1 || n >= (int64_t)1 << 31) return fail(BBC_EINVAL, "n must be in [1, 2^31)");
  if (d < 4 || d > 1024 || d % 4) return fail(BBC_EINVAL, "d must be a multiple of 4 in [4, 1024]");
  if (nlist < 1 || nlist > 8192) return fail(BBC_EINVAL, "nlist must be in [1, 8192]");
  if (metric != BBC_METRIC_L2) return fail(BBC_EUNSUPPORTED, "the PQ path supports the L2 metric only");
  if (pq_bits != 4 && pq_bits != 8) return fail(BBC_EINVAL, "pq_bits must be 4 or 8");
  if (pq_m < 1 || d % pq_m) return fail(BBC_EINVAL, "pq_m must divide d");
  if (list_off[0] != 0 || list_off[nlist] != n) return fail(BBC_EINVAL, "list_off must run from 0 to n");
  for (int32_t j = 0; j < nlist; ++j)
    if (list_off[j + 1] < list_off[j]) return fail(BBC_EINVAL, "list_off must be non-decreasing");
  const int32_t ksub = 1 << pq_bits;
  const int32_t dsub = d / pq_m;
  if (!all_finite(centroids, (int64_t)nlist * d) || !all_finite(base, n * d) ||
      !all_finite(codebook, (int64_t)pq_m * ksub * dsub))
    return fail(BBC_EINVAL, "non-finite value in the index arrays");
  for (int64_t i = 0; i < n * pq_m; ++i)
    if (codes[i] >= ksub) return fail(BBC_EINVAL, "code out of range for pq_bits");
  int32_t rc = set_device(device);
  if (rc) return rc;
  bbc_index* ix = new bbc_index();
  ix->device = device;
  ix->n = n; ix->d = d; ix->nlist = nlist; ix->metric = metric; ix->quant = BBC_QUANT_PQ;
  ix->M = pq_m; ix->bits = pq_bits; ix->ksub = ksub;
  ix->code_bytes = pq_bits == 8 ? pq_m : (pq_m + 1) / 2;
  ix->code_stride = (int32_t)round_up(ix->code_bytes, 16);
  rc = upload_ivf_common(ix, centroids, list_off, list_ids);
  if (rc) { index_release(ix); return rc; }
  // codes, re-strided (and nibble-packed for 4 bits: low nibble = even sub-space)
  std::vector<uint8_t> packed((size_t)n * ix->code_stride, 0);
  for (int64_t p = 0; p < n; ++p) {
    uint8_t* row = packed.data() + (size_t)p * ix->code_stride;
    const uint8_t* src = codes + p * pq_m;
    if (pq_bits == 8) {
      std::memcpy(row, src, pq_m);
    } else {
      for (int32_t m = 0; m < pq_m; ++m) row[m / 2] |= (uint8_t)((src[m] & 15) << (4 * (m & 1)));
    }
  }
  // base vectors in list-slot order
  std::vector<float> vec((size_t)n * d);
  for (int64_t p = 0; p < n; ++p) std::memcpy(vec.data() + (size_t)p * d, base + list_ids[p] * d, sizeof(float) * d);
  auto up = [&]() -> int32_t {
    HIP_TRY(dalloc(&ix->codes, packed.size()));
    HIP_TRY(hipMemcpy(ix->codes, packed.data(), packed.size(), hipMemcpyHostToDevice));
    HIP_TRY(dalloc(&ix->codebook, (size_t)pq_m * ksub * dsub));
    HIP_TRY(hipMemcpy(ix->codebook, codebook, sizeof(float) * pq_m * ksub * dsub, hipMemcpyHostToDevice));
    float* v = nullptr;
    HIP_TRY(dalloc(&v, vec.size()));
    ix->vectors = v;
    HIP_TRY(hipMemcpy(v, vec.data(), sizeof(float) * vec.size(), hipMemcpyHostToDevice));
    return BBC_OK;
  };
  rc = up();
  if (rc) { index_release(ix); return rc; }
  *out = ix;
  return BBC_OK;
}

int32_t bbc_index_create_rabitq(int32_t device, int64_t n, int32_t d, int32_t nlist, int32_t metric,
                                const float* centroids, const int64_t* list_off, const int64_t* list_ids,
                                const float* rotation, const uint32_t* codes, const float* factors,
                                const void* base, int32_t storage, float eps0, bbc_index** out) {
  if (!out) return fail(BBC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!centroids || !list_off || !list_ids || !rotation || !codes || !factors || !base)
    return fail(BBC_EINVAL, "NULL array");
  if (n < 1 || n >= (int64_t)1 << 31) return fail(BBC_EINVAL, "n must be in [1, 2^31)");
  if (d < 64 || d > 1024 || d % 64) return fail(BBC_EINVAL, "RaBitQ needs d a multiple of 64 in [64, 1024]");
  if (nlist < 1 || nlist > 8192) return fail(BBC_EINVAL, "nlist must be in [1, 8192]");
  if (metric != BBC_METRIC_L2 && metric != BBC_METRIC_IP) return fail(BBC_EINVAL, "unknown metric");
  if (storage != BBC_STORAGE_FP32 && storage != BBC_STORAGE_FP16) return fail(BBC_EINVAL, "unknown storage");
  if (!(eps0 >= 0.0f) || !std::isfinite(eps0)) return fail(BBC_EINVAL, "eps0 must be finite and >= 0");
  if (list_off[0] != 0 || list_off[nlist] != n) return fail(BBC_EINVAL, "list_off must run from 0 to n");
  for (int32_t j = 0; j < nlist; ++j)
    if (list_off[j + 1] < list_off[j]) return fail(BBC_EINVAL, "list_off must be non-decreasing");
  if (!all_finite(centroids, (int64_t)nlist * d) || !all_finite(rotation, (int64_t)d * d) ||
      !all_finite(factors, n * 4))
    return fail(BBC_EINVAL, "non-finite value in the index arrays");
  if (storage == BBC_STORAGE_FP32 && !all_finite(static_cast<const float*>(base), n * d))
    return fail(BBC_EINVAL, "non-finite value in base");
  int32_t rc = set_device(device);
  if (rc) return rc;
  bbc_index* ix = new bbc_index();
  ix->device = device;
  ix->n = n; ix->d = d; ix->nlist = nlist; ix->metric = metric; ix->quant = BBC_QUANT_RABITQ;
  ix->fp16 = storage == BBC_STORAGE_FP16;
  ix->eps0 = eps0 > 0.0f ? eps0 : 1.9f;
  ix->rq_words = (int32_t)round_up(d / 32, 4);
  rc = upload_ivf_common(ix, centroids, list_off, list_ids);
  if (rc) { index_release(ix); return rc; }
  const int32_t W = d / 32;
  std::vector<uint32_t> cs((size_t)n * ix->rq_words, 0u);
  for (int64_t p = 0; p < n; ++p) std::memcpy(cs.data() + (size_t)p * ix->rq_words, codes + p * W, 4 * W);
  const size_t esz = ix->fp16 ? 2 : 4;
  std::vector<char> vec((size_t)n * d * esz);
  for (int64_t p = 0; p < n; ++p)
    std::memcpy(vec.data() + (size_t)p * d * esz, static_cast<const char*>(base) + list_ids[p] * d * esz, d * esz);
  auto up = [&]() -> int32_t {
    HIP_TRY(dalloc(&ix->rq_codes, cs.size()));
    HIP_TRY(hipMemcpy(ix->rq_codes, cs.data(), 4 * cs.size(), hipMemcpyHostToDevice));
    HIP_TRY(dalloc(&ix->rq_factors, (size_t)n * 4));
    HIP_TRY(hipMemcpy(ix->rq_factors, factors, sizeof(float) * n * 4, hipMemcpyHostToDevice));
    HIP_TRY(dalloc(&ix->rot, (size_t)d * d));
    HIP_TRY(hipMemcpy(ix->rot, rotation, sizeof(float) * d * d, hipMemcpyHostToDevice));
    HIP_TRY(dalloc(&ix->rot_cent, (size_t)nlist * d));
    HIP_TRY(bbc::launch_rotate(ix->cent, nlist, d, ix->rot, ix->rot_cent, 0));
    char* v = nullptr;
    HIP_TRY(dalloc(&v, vec.size()));
    ix->vectors = v;
    HIP_TRY(hipMemcpy(v, vec.data(), vec.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipDeviceSynchronize());
    return BBC_OK;
  };
  rc = up();
  if (rc) { index_release(ix); return rc; }
  *out = ix;
  return BBC_OK;
}

int32_t bbc_index_info(const bbc_index* ix, int64_t* n, int32_t* d, int32_t* nlist, int32_t* metric,
                       int32_t* quant, int32_t* pq_m, int32_t* pq_bits, int32_t* storage) {
  if (!ix) return fail(BBC_EINVAL, "index is NULL");
  if (storage) *storage = ix->fp16 ? BBC_STORAGE_FP16 : BBC_STORAGE_FP32;
  if (n) *n = ix->n;
  if (d) *d = ix->d;
  if (nlist) *nlist = ix->nlist;
  if (metric) *metric = ix->metric;
  if (quant) *quant = ix->quant;
  if (pq_m) *pq_m = ix->M;
  if (pq_bits) *pq_bits = ix->bits;
  return BBC_OK;
}

int32_t bbc_index_get(const bbc_index* ix, int32_t field, void* dst, int64_t bytes) {
  if (!ix || !dst) return fail(BBC_EINVAL, "NULL argument");
  int32_t rc = set_device(ix->device);
  if (rc) return rc;
  const int64_t n = ix->n;
  switch (field) {
    case BBC_FIELD_CENTROIDS: {
      int64_t need = sizeof(float) * (int64_t)ix->nlist * ix->d;
      if (bytes != need) return fail(BBC_EINVAL, "wrong size for centroids");
      HIP_TRY(hipMemcpy(dst, ix->cent, need, hipMemcpyDeviceToHost));
      return BBC_OK;
    }
    case BBC_FIELD_LIST_OFF: {
      int64_t need = sizeof(int64_t) * (ix->nlist + 1);
      if (bytes != need) return fail(BBC_EINVAL, "wrong size for list_off");
      std::memcpy(dst, ix->h_list_off.data(), need);
      return BBC_OK;
    }
    case BBC_FIELD_LIST_IDS: {
      if (bytes != (int64_t)sizeof(int64_t) * n) return fail(BBC_EINVAL, "wrong size for list_ids");
      std::vector<int32_t> t(n);
      HIP_TRY(hipMemcpy(t.data(), ix->list_ids, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
      int64_t* o = static_cast<int64_t*>(dst);
      for (int64_t i = 0; i < n; ++i) o[i] = t[i];
      return BBC_OK;
    }
    case BBC_FIELD_CODES: {
      if (ix->quant != BBC_QUANT_PQ) return fail(BBC_EUNSUPPORTED, "not a PQ index");
      if (bytes != n * ix->M) return fail(BBC_EINVAL, "wrong size for codes");
      std::vector<uint8_t> t((size_t)n * ix->code_stride);
      HIP_TRY(hipMemcpy(t.data(), ix->codes, t.size(), hipMemcpyDeviceToHost));
      uint8_t* o = static_cast<uint8_t*>(dst);
      for (int64_t p = 0; p < n; ++p)
        for (int32_t m = 0; m < ix->M; ++m) {
          uint8_t b = ix->bits == 8 ? t[(size_t)p * ix->code_stride + m]
                                    : (uint8_t)((t[(size_t)p * ix->code_stride + m / 2] >> (4 * (m & 1))) & 15);
          o[p * ix->M + m] = b;
        }
      return BBC_OK;
    }
    case BBC_FIELD_CODEBOOK: {
      if (ix->quant != BBC_QUANT_PQ) return fail(BBC_EUNSUPPORTED, "not a PQ index");
      int64_t need = sizeof(float) * (int64_t)ix->M * ix->ksub * (ix->d / ix->M);
      if (bytes != need) return fail(BBC_EINVAL, "wrong size for codebook");
      HIP_TRY(hipMemcpy(dst, ix->codebook, need, hipMemcpyDeviceToHost));
      return BBC_OK;
    }
    case BBC_FIELD_RABITQ_CODES: {
      if (ix->quant != BBC_QUANT_RABITQ) return fail(BBC_EUNSUPPORTED, "not a RaBitQ index");
      const int32_t W = ix->d / 32;
      if (bytes != 4 * n * W) return fail(BBC_EINVAL, "wrong size for RaBitQ codes");
      std::vector<uint32_t> t((size_t)n * ix->rq_words);
      HIP_TRY(hipMemcpy(t.data(), ix->rq_codes, 4 * t.size(), hipMemcpyDeviceToHost));
      uint32_t* o = static_cast<uint32_t*>(dst);
      for (int64_t p = 0; p < n; ++p) std::memcpy(o + p * W, t.data() + (size_t)p * ix->rq_words, 4 * W);
      return BBC_OK;
    }
    case BBC_FIELD_RABITQ_FACTORS: {
      if (ix->quant != BBC_QUANT_RABITQ) return fail(BBC_EUNSUPPORTED, "not a RaBitQ index");
      if (bytes != 16 * n) return fail(BBC_EINVAL, "wrong size for RaBitQ factors");
      HIP_TRY(hipMemcpy(dst, ix->rq_factors, 16 * n, hipMemcpyDeviceToHost));
      return BBC_OK;
    }
    case BBC_FIELD_ROT_CENTROIDS: {
      if (ix->quant != BBC_QUANT_RABITQ) return fail(BBC_EUNSUPPORTED, "not a RaBitQ index");
      const int64_t need = sizeof(float) * (int64_t)ix->nlist * ix->d;
      if (bytes != need) return fail(BBC_EINVAL, "wrong size for rotated centroids");
      HIP_TRY(hipMemcpy(dst, ix->rot_cent, need, hipMemcpyDeviceToHost));
      return BBC_OK;
    }
    case BBC_FIELD_ROTATION: {
      if (ix->quant != BBC_QUANT_RABITQ) return fail(BBC_EUNSUPPORTED, "not a RaBitQ index");
      const int64_t need = sizeof(float) * (int64_t)ix->d * ix->d;
      if (bytes != need) return fail(BBC_EINVAL, "wrong size for the rotation");
      HIP_TRY(hipMemcpy(dst, ix->rot, need, hipMemcpyDeviceToHost));
      return BBC_OK;
    }
    case BBC_FIELD_BASE: {
      // rows are held in list-slot order: copied in chunks, placed by row id
      const int64_t row = (ix->fp16 ? 2 : 4) * (int64_t)ix->d;
      if (bytes != row * n) return fail(BBC_EINVAL, "wrong size for the base rows");
      std::vector<int32_t> ids(n);
      HIP_TRY(hipMemcpy(ids.data(), ix->list_ids, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
      const int64_t chunk = std::max<int64_t>(1, (int64_t)(256 << 20) / row);
      std::vector<char> t((size_t)(std::min(chunk, std::max<int64_t>(n, 1)) * row));
      char* o = static_cast<char*>(dst);
      for (int64_t p0 = 0; p0 < n; p0 += chunk) {
        const int64_t c = std::min(chunk, n - p0);
        HIP_TRY(hipMemcpy(t.data(), static_cast<const char*>(ix->vectors) + p0 * row, c * row, hipMemcpyDeviceToHost));
        for (int64_t p = 0; p < c; ++p) std::memcpy(o + (int64_t)ids[p0 + p] * row, t.data() + p * row, row);
      }
      return BBC_OK;
    }
    default:
      return fail(BBC_EINVAL, "unknown field");
  }
}

void bbc_index_free(bbc_index* ix) { index_release(ix); }

}  // extern "C"

namespace {

constexpr char kIndexMagic[8] = {'B', 'B', 'C', 'I', 'D', 'X', '2', '\0'};

// Checksum of an index file's arrays: FNV-1a over little-endian 64-bit words
// of the bytes after the header (the last word zero-padded), the FNV-1a
// 64-bit offset basis and prime; fed section by section.
struct WordFnv64 {
  uint64_t h = 0xcbf29ce484222325ull;
  uint8_t carry[8] = {};
  int nc = 0;
  void word(uint64_t w) { h = (h ^ w) * 0x100000001b3ull; }
  void add(const void* data, size_t n) {
    const uint8_t* p = static_cast<const uint8_t*>(data);
    while (n && nc) {  // complete a carried word
      carry[nc++] = *p++;
      --n;
      if (nc == 8) {
        uint64_t w;
        std::memcpy(&w, carry, 8);
        word(w);
        nc = 0;
      }
    }
    for (; n >= 8; n -= 8, p += 8) {
      uint64_t w;
      std::memcpy(&w, p, 8);
      word(w);
    }
    while (n--) carry[nc++] = *p++;
  }
  uint64_t final() {
    if (nc) {
      std::memset(carry + nc, 0, (size_t)(8 - nc));
      uint64_t w;
      std::memcpy(&w, carry, 8);
      word(w);
      nc = 0;
    }
    return h;
  }
};

struct IndexFileHeader {
  char magic[8];
  int32_t quant, metric, storage, d, nlist, pq_m, pq_bits, reserved0;
  int64_t n;
  float eps0;
  int32_t reserved1;
};
static_assert(sizeof(IndexFileHeader) == 56, "index file header layout");

// Bytes of each array of an index file after the header, in file order.
std::vector<int64_t> index_file_sections(const IndexFileHeader& h) {
  const int64_t n = h.n, d = h.d, nl = h.nlist;
  std::vector<int64_t> s = {4 * nl * d, 8 * (nl + 1), 8 * n};
  if (h.quant == BBC_QUANT_PQ) {
    s.push_back(4 * (int64_t)h.pq_m * (1LL << h.pq_bits) * (d / h.pq_m));
    s.push_back(n * h.pq_m);
  } else {
    s.push_back(4 * d * d);
    s.push_back(4 * n * (d / 32));
    s.push_back(16 * n);
  }
  s.push_back((h.storage == BBC_STORAGE_FP16 ? 2 : 4) * n * d);
  return s;
}

struct FileCloser {
  void operator()(FILE* f) const { if (f) std::fclose(f); }
};

}  // namespace

extern "C" {

int32_t bbc_index_save(const bbc_index* ix, const char* path) {
  if (!ix || !path) return fail(BBC_EINVAL, "NULL argument");
  IndexFileHeader h{};
  std::memcpy(h.magic, kIndexMagic, 8);
  h.quant = ix->quant; h.metric = ix->metric; h.storage = ix->fp16 ? BBC_STORAGE_FP16 : BBC_STORAGE_FP32;
  h.d = ix->d; h.nlist = ix->nlist; h.pq_m = ix->M; h.pq_bits = ix->bits; h.n = ix->n; h.eps0 = ix->eps0;
  const std::vector<int64_t> sec = index_file_sections(h);
  const int32_t fields_pq[] = {BBC_FIELD_CENTROIDS, BBC_FIELD_LIST_OFF, BBC_FIELD_LIST_IDS, BBC_FIELD_CODEBOOK,
                               BBC_FIELD_CODES, BBC_FIELD_BASE};
  const int32_t fields_rq[] = {BBC_FIELD_CENTROIDS, BBC_FIELD_LIST_OFF, BBC_FIELD_LIST_IDS, BBC_FIELD_ROTATION,
                               BBC_FIELD_RABITQ_CODES, BBC_FIELD_RABITQ_FACTORS, BBC_FIELD_BASE};
  const int32_t* fields = ix->quant == BBC_QUANT_PQ ? fields_pq : fields_rq;
  std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "wb"));
  if (!f) return fail(BBC_EINVAL, std::string("cannot open for writing: ") + path);
  if (std::fwrite(&h, sizeof(h), 1, f.get()) != 1) return fail(BBC_EINVAL, "write failed");
  WordFnv64 sum;
  for (size_t i = 0; i < sec.size(); ++i) {
    std::vector<char> buf((size_t)sec[i]);
    const int32_t rc = bbc_index_get(ix, fields[i], buf.data(), sec[i]);
    if (rc) return rc;
    sum.add(buf.data(), buf.size());
    if (sec[i] && std::fwrite(buf.data(), 1, buf.size(), f.get()) != buf.size()) return fail(BBC_EINVAL, "write failed");
  }
  const uint64_t cs = sum.final();
  if (std::fwrite(&cs, sizeof(cs), 1, f.get()) != 1) return fail(BBC_EINVAL, "write failed");
  if (std::fflush(f.get()) != 0) return fail(BBC_EINVAL, "write failed");
  return BBC_OK;
}

int32_t bbc_index_load(int32_t device, const char* path, bbc_index** out) {
  if (!out) return fail(BBC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!path) return fail(BBC_EINVAL, "path is NULL");
  std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "rb"));
  if (!f) return fail(BBC_EINVAL, std::string("cannot open: ") + path);
  IndexFileHeader h{};
  if (std::fread(&h, sizeof(h), 1, f.get()) != 1 || std::memcmp(h.magic, kIndexMagic, 8) != 0)
    return fail(BBC_EINVAL, "not an index file");
  const bool pq = h.quant == BBC_QUANT_PQ;
  if ((!pq && h.quant != BBC_QUANT_RABITQ) || h.n < 1 || h.n >= (1LL << 31) || h.d < 4 || h.d > 1024 ||
      h.nlist < 1 || h.nlist > 8192 || (h.storage != BBC_STORAGE_FP32 && h.storage != BBC_STORAGE_FP16) ||
      (pq && (h.pq_m < 1 || h.d % h.pq_m || (h.pq_bits != 4 && h.pq_bits != 8))) || (!pq && h.d % 64))
    return fail(BBC_EINVAL, "index file header out of range");
  const std::vector<int64_t> sec = index_file_sections(h);
  int64_t total = (int64_t)sizeof(h) + (int64_t)sizeof(uint64_t);  // header, arrays, checksum
  for (int64_t b : sec) total += b;
  if (std::fseek(f.get(), 0, SEEK_END) != 0 || std::ftell(f.get()) != total)
    return fail(BBC_EINVAL, "index file size does not match its header");
  std::fseek(f.get(), (long)sizeof(h), SEEK_SET);
  std::vector<std::vector<char>> a(sec.size());
  WordFnv64 sum;
  for (size_t i = 0; i < sec.size(); ++i) {
    a[i].resize((size_t)sec[i]);
    if (sec[i] && std::fread(a[i].data(), 1, a[i].size(), f.get()) != a[i].size())
      return fail(BBC_EINVAL, "index file read failed");
    sum.add(a[i].data(), a[i].size());
  }
  uint64_t cs = 0;
  if (std::fread(&cs, sizeof(cs), 1, f.get()) != 1) return fail(BBC_EINVAL, "index file read failed");
  f.reset();
  if (cs != sum.final()) return fail(BBC_EINVAL, "index file checksum mismatch (the arrays were altered)");
  const float* cent = reinterpret_cast<const float*>(a[0].data());
  const int64_t* list_off = reinterpret_cast<const int64_t*>(a[1].data());
  const int64_t* list_ids = reinterpret_cast<const int64_t*>(a[2].data());
  if (pq) {
    if (h.storage != BBC_STORAGE_FP32) return fail(BBC_EINVAL, "PQ index files hold float32 rows");
    return bbc_index_create_pq(device, h.n, h.d, h.nlist, h.metric, cent, list_off, list_ids, h.pq_m, h.pq_bits,
                               reinterpret_cast<const float*>(a[3].data()),
                               reinterpret_cast<const uint8_t*>(a[4].data()),
                               reinterpret_cast<const float*>(a[5].data()), out);
  }
  return bbc_index_create_rabitq(device, h.n, h.d, h.nlist, h.metric, cent, list_off, list_ids,
                                 reinterpret_cast<const float*>(a[3].data()),
                                 reinterpret_cast<const uint32_t*>(a[4].data()),
                                 reinterpret_cast<const float*>(a[5].data()), a[6].data(), h.storage, h.eps0, out);
}

int32_t bbc_stage_timing(int32_t enable) {
  g_timer.enabled = enable != 0;
  return BBC_OK;
}

int32_t bbc_stage_times(double* ms, int64_t* launches, int32_t nstages, int32_t reset) {
  std::lock_guard<std::mutex> g(g_timer.mu);
  for (auto& r : g_timer.pending) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return fail(BBC_EDEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    float t = 0.f;
    hipEventElapsedTime(&t, r.a, r.b);
    if (r.stage >= 0 && r.stage < 8) { g_timer.ms[r.stage] += t; g_timer.launches[r.stage] += 1; }
    g_timer.pool.push_back(r.a);
    g_timer.pool.push_back(r.b);
  }
  g_timer.pending.clear();
  for (int i = 0; i < nstages && i < 8; ++i) {
    if (ms) ms[i] = g_timer.ms[i];
    if (launches) launches[i] = g_timer.launches[i];
  }
  if (reset) {
    for (int i = 0; i < 8; ++i) { g_timer.ms[i] = 0; g_timer.launches[i] = 0; }
  }
  return BBC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// search
// ---------------------------------------------------------------------------
namespace {

struct Layout {
  // offsets into the arena
  size_t nsample_q, pair_cnt, pair_split, bs_table, rescan_q, sminmax, sorted_pairs, sorted_q, sample_keys, surv_key, surv_pos, pair_nsurv, surv_total, surv_bucket, n_rejected, books;
  size_t q, meta, dprime, probe_lists, probe_keys, rank_off, n_scanned, n_recheck, keys, cand_pos,
      cand_packed, n_cand, out_ids, out_dists, out_counts, t_dmin, t_delta, t_map, t_tau, t_s, t_counts, t_nsk,
      t_nb, qorder, rt_sorted, rt_bins, rt_ptb, rt_lcnt, rt_lpairs;
  size_t surv_exact, n_early, n_used, rt_sidx, t_tpred;  // early re-rank
};

int32_t validate_search(const bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                        const int32_t* nprobe, const bbc_search_params* p, const int64_t* out_off) {
  if (!ix) return fail(BBC_EINVAL, "index is NULL");
  if (!p) return fail(BBC_EINVAL, "params is NULL");
  if (nq < 0) return fail(BBC_EINVAL, "nq < 0");
  if (nq == 0) return BBC_OK;
  if (!queries || !k || !nprobe || !out_off) return fail(BBC_EINVAL, "NULL argument");
  if (!(p->ncand_ratio >= 1.0) || !std::isfinite(p->ncand_ratio)) return fail(BBC_EINVAL, "ncand_ratio must be >= 1");
  if (p->buckets < 0 || p->buckets > 256) return fail(BBC_EINVAL, "buckets must be in [0, 256]");
  if (p->nsample < 0) return fail(BBC_EINVAL, "nsample must be >= 0");
  if (p->sample_factor < 0 || p->sample_factor > 64) return fail(BBC_EINVAL, "sample_factor must be in [0, 64]");
  if (p->collector != BBC_COLLECT_BUCKET && p->collector != BBC_COLLECT_HEAP && p->collector != BBC_COLLECT_SORT &&
      p->collector != BBC_COLLECT_HEAP_LDS)
    return fail(BBC_EINVAL, "unknown collector");
  if (p->lut_u8 != 0 && p->lut_u8 != 1) return fail(BBC_EINVAL, "lut_u8 must be 0 or 1");
  if (p->lut_u8 && ix->quant != BBC_QUANT_PQ) return fail(BBC_EINVAL, "lut_u8 applies to PQ indexes only");
  if (p->lut_u8 && !bbc::pq_scan_grouped_shape(ix->bits, ix->M, ix->d))
    return fail(BBC_EUNSUPPORTED, "one-byte tables need a grouped scan shape (8-bit M=16 or 32, 4-bit M=32 or 48)");
  if (p->early_rerank != 0 && p->early_rerank != 1) return fail(BBC_EINVAL, "early_rerank must be 0 or 1");
  if (p->keep_all_keys != 0 && p->keep_all_keys != 1) return fail(BBC_EINVAL, "keep_all_keys must be 0 or 1");
  if (p->early_rerank) {
    if (ix->quant != BBC_QUANT_PQ) return fail(BBC_EINVAL, "early_rerank applies to PQ indexes only");
    if (p->collector != BBC_COLLECT_BUCKET) return fail(BBC_EINVAL, "early_rerank needs the bucket collector");
    if (p->lut_u8 || ix->fp16 || !bbc::pq_scan_grouped_shape(ix->bits, ix->M, ix->d))
      return fail(BBC_EUNSUPPORTED, "early_rerank needs float32 tables, float32 rows and a grouped scan shape");
  }
  if (out_off[0] != 0) return fail(BBC_EINVAL, "out_offsets[0] must be 0");
  for (int64_t i = 0; i < nq; ++i) {
    if (k[i] < 1) return fail(BBC_EINVAL, "k must be >= 1");
    if (nprobe[i] < 1 || nprobe[i] > ix->nlist) return fail(BBC_EINVAL, "nprobe must be in [1, nlist]");
    if (out_off[i + 1] - out_off[i] != k[i]) return fail(BBC_EINVAL, "out_offsets must be the prefix sums of k");
  }
  if (!p->device_io && !all_finite(queries, nq * ix->d)) return fail(BBC_EINVAL, "non-finite query value");
  return BBC_OK;
}

int64_t kc_cap_of(const bbc_index* ix, int32_t k, int32_t np, double r) {
  int64_t t = (int64_t)std::ceil(r * (double)k);
  return std::min(t, ix->h_maxS[np]);
}

// How a search call is run: normally (the index's arena, asynchronous
// metadata upload), as a sizing pass (workspace bytes only), or captured
// into a graph on a plan's own workspace (metadata uploaded synchronously,
// then every launch recorded).
struct SearchCtx {
  bool size_only = false;
  size_t ws_bytes = 0;
  char* ws = nullptr;
  int64_t* work_out = nullptr;  // [2][nq]: codes scanned, exact distances computed
  bool capture = false;
  hipGraph_t graph = nullptr;
  // fixed pinned staging for the metadata block (allocation-free searches):
  // used instead of the index's growable pinned buffer when set
  char* meta_host = nullptr;
  size_t meta_cap = 0;
  hipEvent_t meta_ev = nullptr;
};

// The final top-k's launches: queries grouped by the kernel form their
// candidate capacity selects (register-resident forms for small sets, the
// memory form for large ones), each group with the LDS its own largest
// min(k, K_c) needs, so that a few large queries do not set the form and the
// LDS of a whole batch.  order lists the queries group by group.
struct FinalGroups {
  std::vector<int32_t> order;
  struct G { int64_t beg = 0, n = 0, max_kc = 0, max_cnt = 1; };
  std::vector<G> groups;
};

void final_groups(int64_t nq, const int32_t* k, const std::vector<int64_t>& cap_of, int64_t split_from,
                  FinalGroups& fg) {
  // batches smaller than split_from queries take one launch (for them the
  // launches cost more than the forms save)
  const bool split = nq >= split_from;
  const int forms[5] = {8, 16, 24, 32, 0};
  fg.order.resize((size_t)nq);
  fg.groups.clear();
  int64_t at = 0;
  for (int f : forms) {
    if (!split && f != 0) continue;
    FinalGroups::G g;
    g.beg = at;
    for (int64_t i = 0; i < nq; ++i) {
      if (split && bbc::final_topk_form(cap_of[(size_t)i]) != f) continue;
      fg.order[(size_t)at++] = (int32_t)i;
      g.max_kc = std::max(g.max_kc, cap_of[(size_t)i]);
      g.max_cnt = std::max(g.max_cnt, std::min<int64_t>(k[i], cap_of[(size_t)i]));
    }
    g.n = at - g.beg;
    // largest candidate sets first, so that the launch does not end on a
    // few long blocks while the other CUs idle
    std::stable_sort(fg.order.begin() + g.beg, fg.order.begin() + at,
                     [&](int32_t x, int32_t y) { return cap_of[(size_t)x] > cap_of[(size_t)y]; });
    if (g.n) fg.groups.push_back(g);
  }
}

// One launch per group (a group's form from its largest K_c, its LDS from its
// largest min(k, K_c)).
int32_t launch_final_groups(bbc_index* ix, const FinalGroups& fg, const int32_t* d_order, bbc::FinalArgs fa,
                            hipStream_t s) {
  // the LDS buffer: the group's largest result set when it fits (larger ones
  // group their winners in the scratch buffer and sort in memory)
  int64_t cap_max = std::max<int64_t>(1024, (ix->max_lds - bbc::FINAL_STATIC_LDS) / 8);
  if (ix->final_lds_cap > 0) cap_max = std::min(cap_max, ix->final_lds_cap);
  for (const auto& g : fg.groups) {
    const int cap = (int)std::min(g.max_cnt, cap_max);
    int run = 1;
    while (2 * run <= cap) run *= 2;
    fa.nq = g.n;
    fa.qmap = d_order + g.beg;
    fa.cap = cap;
    fa.run = run;
    fa.max_kc = g.max_kc;
    HIP_TRY(bbc::launch_final_topk(fa, s));
  }
  return BBC_OK;
}

// Host staging of a search's metadata block: the caller-given fixed buffer,
// or the index's pinned buffer (grown when too small).  Waits until the
// previous upload out of that buffer is done before it is rewritten.
int32_t stage_meta(bbc_index* ix, const SearchCtx* ctx, size_t bytes, char** H, hipEvent_t* ev) {
  if (ctx && ctx->meta_host) {
    if (bytes > ctx->meta_cap)
      return fail(BBC_EINVAL, "the batch's metadata (" + std::to_string(bytes) +
                                  " bytes) exceeds the allocation-free staging buffer (" +
                                  std::to_string(ctx->meta_cap) + " bytes)");
    HIP_TRY(hipEventSynchronize(ctx->meta_ev));
    *H = ctx->meta_host;
    *ev = ctx->meta_ev;
    return BBC_OK;
  }
  HIP_TRY(hipEventSynchronize(ix->meta_done));
  if (ix->pinned_cap < bytes) {
    if (ix->pinned) hipHostFree(ix->pinned);
    ix->pinned = nullptr;
    ix->pinned_cap = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&ix->pinned), bytes * 2));
    ix->pinned_cap = bytes * 2;
  }
  *H = ix->pinned;
  *ev = ix->meta_done;
  return BBC_OK;
}

// Tile counts of the largest lists for tiles of 1 << ts rows: h_maxT[p] =
// sum of the p largest ceil(size / 2^ts), a bound on the bins of a query
// probing p lists.
const std::vector<int64_t>& tile_bounds(bbc_index* ix, int ts) {
  if (ix->h_maxT_ts != ts) {
    std::vector<int64_t> t(ix->nlist);
    for (int32_t j = 0; j < ix->nlist; ++j)
      t[j] = (ix->h_list_off[j + 1] - ix->h_list_off[j] + ((int64_t)1 << ts) - 1) >> ts;
    std::sort(t.begin(), t.end(), std::greater<int64_t>());
    ix->h_maxT.assign(ix->nlist + 1, 0);
    for (int32_t j = 0; j < ix->nlist; ++j) ix->h_maxT[j + 1] = ix->h_maxT[j] + t[j];
    ix->h_maxT_ts = ts;
  }
  return ix->h_maxT;
}

// Shape of the tile-major form for a batch: bin offsets per query and the
// candidate sort's LDS; false where the form does not apply.
bool tile_plan(bbc_index* ix, int64_t nq, const int32_t* nprobe, int max_np, int max_chunks,
               std::vector<int64_t>& bin_off, int* ts, int* max_bins, size_t* lds) {
  if (!ix->list_of_pos || nq > 65535 || ix->nlist > bbc::QUERY_ORDER_MAX_LISTS || max_np <= 0) return false;
  if (ix->d / 4 > max_chunks) return false;
  *ts = bbc::tile_rerank_shift(ix->d, ix->fp16);
  if (*ts < 0) return false;
  const std::vector<int64_t>& mt = tile_bounds(ix, *ts);
  bin_off.assign(nq + 1, 0);
  int64_t mb = 0;
  for (int64_t i = 0; i < nq; ++i) {
    const int64_t nb = mt[nprobe[i]];
    bin_off[i + 1] = bin_off[i] + nb + 1;
    mb = std::max(mb, nb);
  }
  // bin counters: as many as any query can have, or as many as fit in LDS
  // (the candidate sort then takes a query's ranks in ranges); one list's
  // tiles must fit
  const size_t fixed = bbc::tile_rerank_sort_lds(0, max_np, ix->nlist) + 1024;
  if (fixed >= (size_t)ix->max_lds) return false;
  mb = std::min<int64_t>(mb, (int64_t)(((size_t)ix->max_lds - fixed) / sizeof(uint32_t)));
  mb = std::max<int64_t>(std::min(mb, ix->rt_sort_bins), std::min(mb, mt[1]));
  if (mb < mt[1] || mb > (int64_t)1 << 30) return false;
  *max_bins = (int)mb;
  *lds = bbc::tile_rerank_sort_lds(*max_bins, max_np, ix->nlist);
  return *lds + 1024 <= (size_t)ix->max_lds;
}

// RaBitQ: probe, rotation of the queries, per-(query, list) bounds, bounded
// re-rank per query, final sort.  Per-query slot arrays are sized by the
// largest lists (maxS(nprobe)).
int32_t run_search_rabitq(bbc_index* ix, const float* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                          const bbc_search_params* p, const int64_t* out_off, int64_t* out_ids, float* out_dists,
                          int32_t* out_counts, bbc_search_trace* tr, SearchCtx* ctx) {
  int32_t rc = BBC_OK;
  hipStream_t s = static_cast<hipStream_t>(p->stream);
  const bool host_io = p->device_io == 0;
  const int d = ix->d;
  const bool tracing = tr != nullptr;
  std::vector<int64_t> probe_off(nq + 1, 0), key_off(nq + 1, 0);
  int64_t max_cap = 0, max_cnt = 1;
  int max_np = 0;
  for (int64_t i = 0; i < nq; ++i) {
    probe_off[i + 1] = probe_off[i] + nprobe[i];
    const int64_t cap = ix->h_maxS[nprobe[i]];
    key_off[i + 1] = key_off[i] + cap;
    max_cap = std::max(max_cap, cap);
    max_cnt = std::max(max_cnt, std::min<int64_t>(k[i], cap));
    max_np = std::max(max_np, nprobe[i]);
  }
  const int64_t npairs = probe_off[nq], nkeys = key_off[nq], nout = out_off[nq];
  // Re-rank form: one block per query walking and gathering its rows, or the
  // wide form (exact keys of the candidate set C first, then the walk over
  // them), whose keys come from a device-wide grid per query (small
  // batches) or tile-major from rows staged once per group of queries
  // (large batches, where queries share rows).
  std::vector<int64_t> bin_off;
  int rt_shift = 0, rt_bins = 0;
  size_t rt_lds = 0;
  const bool want_tiles = ix->walk_form == 3 || (ix->walk_form == 0 && nq > ix->num_cu);
  const bool tile_keys = want_tiles && tile_plan(ix, nq, nprobe, max_np, 256, bin_off, &rt_shift, &rt_bins, &rt_lds);
  if (!tile_keys) bin_off.assign(nq + 1, 0);
  FinalGroups fg;
  {
    std::vector<int64_t> cap_of((size_t)nq);
    for (int64_t i = 0; i < nq; ++i) cap_of[(size_t)i] = key_off[i + 1] - key_off[i];
    final_groups(nq, k, cap_of, ix->num_cu, fg);
  }
  Plan mp;
  const size_t m_k = mp.add(4 * nq), m_np = mp.add(4 * nq), m_po = mp.add(8 * (nq + 1)),
               m_ko = mp.add(8 * (nq + 1)), m_oo = mp.add(8 * (nq + 1)), m_bo = mp.add(8 * (nq + 1)),
               m_fq = mp.add(4 * nq);
  Plan pl;
  const size_t L_meta = pl.add(mp.total);
  const size_t L_q = host_io ? pl.add(sizeof(float) * nq * d) : 0;
  const size_t L_dprime = pl.add(sizeof(float) * nq * ix->nlist);
  const size_t L_pl = pl.add(4 * npairs), L_pk = pl.add(4 * npairs), L_ro = pl.add(8 * npairs);
  const size_t L_ns = pl.add(8 * nq), L_nr = pl.add(4 * nq);
  const size_t L_qrot = pl.add(sizeof(float) * nq * d);
  const size_t L_lb = pl.add(4 * nkeys), L_ub = pl.add(4 * nkeys);
  const size_t L_key = tracing ? pl.add(4 * nkeys) : 0;
  const size_t L_cbuf = pl.add(4 * nkeys), L_cp = pl.add(8 * nkeys), L_z = pl.add(16 * nkeys);
  const size_t L_nc = pl.add(8 * nq), L_nv = pl.add(8 * nq);
  const size_t L_qp = tracing ? pl.add(4 * nq) : 0;
  // the wide re-rank form when the batch alone leaves compute units idle
  // with one block per query, or when its keys come tile-major
  const bool wide = ix->walk_form == 2 || tile_keys || (ix->walk_form == 0 && nq <= ix->num_cu);
  // tile-major keys: the walk's bin pass also writes C in tile order (when
  // each query's probe ranks fit its LDS tables), else the candidate sort does
  const bool presort = tile_keys && ix->walk_presort && max_np <= bbc::WALK_RANKS_LDS;
  size_t L_cpos = 0, L_wbins = 0, L_wst = 0, L_wround = 0;
  // the wide form's keys in two rounds
  const bool rounds = wide && (ix->walk_alpha < 0.0f ? tile_keys : ix->walk_alpha < 1.0f);
  if (wide) {
    // C's list positions in place order: the grid keys' input (also the
    // second round's when the first round's keys come tile-major)
    if (!presort || rounds) L_cpos = pl.add(4 * nkeys);
    L_wbins = pl.add(4 * 2048 * nq);
    L_wst = pl.add(16 * nq);
    if (rounds) L_wround = pl.add(16 * nq);
  }
  const int rt_group = bbc::tile_rerank_group(d);
  const int64_t rt_lpairs_cap = npairs + (int64_t)ix->nlist * (rt_group - 1);
  size_t L_rts = 0, L_rti = 0, L_rtb = 0, L_rtp = 0, L_rtc = 0, L_rtl = 0;
  if (tile_keys) {
    L_rts = pl.add(4 * nkeys); L_rti = pl.add(4 * nkeys); L_rtb = pl.add(4 * bin_off[nq]);
    L_rtp = pl.add(4 * npairs); L_rtc = pl.add(4 * ((int64_t)ix->nlist + 1)); L_rtl = pl.add(8 * rt_lpairs_cap);
  }
  const int64_t bs_words = ix->pair_sort_lds && tile_keys ? bbc::pair_sort_table_words(nq, ix->nlist) : 0;
  const size_t L_bst = bs_words ? pl.add(4 * bs_words) : 0;
  size_t L_oid = 0, L_od = 0, L_oc = 0;
  if (host_io) { L_oid = pl.add(8 * nout); L_od = pl.add(4 * nout); L_oc = pl.add(4 * nq); }
  const size_t L_fs = pl.add(8 * nout);  // final top-k: winners grouped by bin
  if (ctx && ctx->size_only) {
    ctx->ws_bytes = pl.total;
    return BBC_OK;
  }
  char* A;
  if (ctx && ctx->ws) {
    A = ctx->ws;
  } else {
    HIP_TRY(ix->arena.reserve(pl.total));
    A = ix->arena.base;
    HIP_TRY(ix->arena.acquire(s));
  }
  char* H = nullptr;
  hipEvent_t meta_ev = nullptr;
  if ((rc = stage_meta(ix, ctx, mp.total, &H, &meta_ev))) return rc;
  std::memcpy(H + m_k, k, 4 * nq);
  std::memcpy(H + m_np, nprobe, 4 * nq);
  std::memcpy(H + m_po, probe_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_ko, key_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_oo, out_off, 8 * (nq + 1));
  std::memcpy(H + m_bo, bin_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_fq, fg.order.data(), 4 * nq);
  char* M = A + L_meta;
  if (ctx && ctx->capture) {
    HIP_TRY(hipMemcpy(M, H, mp.total, hipMemcpyHostToDevice));
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    t_capturing = true;
  } else {
    HIP_TRY(hipMemcpyAsync(M, H, mp.total, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(meta_ev, s));
  }
  const float* dq = queries;
  if (host_io) {
    HIP_TRY(hipMemcpyAsync(A + L_q, queries, sizeof(float) * nq * d, hipMemcpyHostToDevice, s));
    dq = reinterpret_cast<const float*>(A + L_q);
  }
  const int32_t* d_k = reinterpret_cast<const int32_t*>(M + m_k);
  const int32_t* d_np = reinterpret_cast<const int32_t*>(M + m_np);
  const int64_t* d_po = reinterpret_cast<const int64_t*>(M + m_po);
  const int64_t* d_ko = reinterpret_cast<const int64_t*>(M + m_ko);
  const int64_t* d_bo = reinterpret_cast<const int64_t*>(M + m_bo);
  const int64_t* d_oo = reinterpret_cast<const int64_t*>(M + m_oo);
  int64_t* d_oid = host_io ? reinterpret_cast<int64_t*>(A + L_oid) : out_ids;
  float* d_odist = host_io ? reinterpret_cast<float*>(A + L_od) : out_dists;
  int32_t* d_ocnt = host_io ? reinterpret_cast<int32_t*>(A + L_oc) : out_counts;

  bbc::ProbeArgs pa{};
  pa.q = dq; pa.nq = nq; pa.d = d; pa.cent = ix->cent; pa.cent_bf16 = ix->cent_bf16; pa.dpad = ix->dpad;
  pa.cent_norm2 = ix->cent_norm2; pa.cent_norm = ix->cent_norm; pa.nlist = ix->nlist; pa.metric = ix->metric;
  pa.nprobe = d_np; pa.probe_off = d_po; pa.list_off = ix->list_off;
  pa.dprime = reinterpret_cast<float*>(A + L_dprime);
  pa.probe_lists = reinterpret_cast<int32_t*>(A + L_pl);
  pa.probe_keys = reinterpret_cast<float*>(A + L_pk);
  pa.rank_off = reinterpret_cast<int64_t*>(A + L_ro);
  pa.n_scanned = reinterpret_cast<int64_t*>(A + L_ns);
  pa.n_recheck = reinterpret_cast<int32_t*>(A + L_nr);
  pa.nsample_q = nullptr;
  pa.num_cu = ix->num_cu;
  {
    StageScope st(s, 0);
    HIP_TRY(bbc::launch_probe(pa, s));
  }
  float* qrot = reinterpret_cast<float*>(A + L_qrot);
  {
    StageScope st(s, 1);
    HIP_TRY(bbc::launch_rotate(dq, nq, d, ix->rot, qrot, s));
  }
  // tile-major keys: the (query, rank) pairs grouped by list, before the scan
  // when it takes them in that order
  bbc::TileRerankArgs ta{};
  if (tile_keys) {
    ta.q = dq; ta.nq = nq; ta.d = d; ta.metric = ix->metric; ta.vectors = ix->vectors; ta.fp16 = ix->fp16;
    ta.list_ids = ix->list_ids; ta.list_off = ix->list_off; ta.list_of_pos = ix->list_of_pos;
    ta.nprobe = d_np; ta.probe_off = d_po; ta.probe_lists = pa.probe_lists; ta.nlist = ix->nlist;
    ta.npairs = npairs; ta.max_np = max_np; ta.tshift = rt_shift; ta.max_bins = rt_bins;
    ta.lcnt = reinterpret_cast<uint32_t*>(A + L_rtc);
    ta.lpairs = reinterpret_cast<uint64_t*>(A + L_rtl);
    ta.bs_table = bs_words ? reinterpret_cast<uint32_t*>(A + L_bst) : nullptr;
    ta.no_run_list = ix->no_run_list;
    ta.lpairs_cap = rt_lpairs_cap;
    ta.group = rt_group;
  }
  const bool scan_by_list = tile_keys && ix->scan_by_list;
  bbc::RabitqScanArgs sa{};
  if (scan_by_list) {
    sa.lpairs = ta.lpairs; sa.ngroups = ta.lcnt + ix->nlist; sa.group = rt_group; sa.lpairs_cap = rt_lpairs_cap;
  }
  sa.npairs = npairs; sa.nq = nq; sa.probe_off = d_po; sa.probe_lists = pa.probe_lists; sa.probe_keys = pa.probe_keys;
  sa.rank_off = pa.rank_off; sa.key_off = d_ko; sa.q = dq; sa.qrot = qrot; sa.rot_cent = ix->rot_cent;
  sa.D = d; sa.metric = ix->metric; sa.eps0 = ix->eps0; sa.list_off = ix->list_off; sa.codes = ix->rq_codes;
  sa.code_words = ix->rq_words; sa.factors = ix->rq_factors;
  sa.force_1d = ix->rq_scan_1d;
  sa.max_np = 1;
  for (int64_t i = 0; i < nq; ++i) sa.max_np = std::max(sa.max_np, (int)nprobe[i]);
  sa.lb = reinterpret_cast<float*>(A + L_lb);
  sa.ub = reinterpret_cast<float*>(A + L_ub);
  sa.key = tracing ? reinterpret_cast<float*>(A + L_key) : nullptr;
  {
    StageScope st(s, 2);
    if (scan_by_list) {
      HIP_TRY(bbc::launch_tile_pairs(ta, s));
      ta.pairs_ready = 1;
    }
    HIP_TRY(bbc::launch_rabitq_scan(sa, s));
  }
  bbc::RabitqWalkArgs wa{};
  wa.nq = nq; wa.n_scanned = pa.n_scanned; wa.k = d_k; wa.nprobe = d_np; wa.probe_off = d_po;
  wa.rank_off = pa.rank_off; wa.probe_lists = pa.probe_lists; wa.list_off = ix->list_off; wa.list_ids = ix->list_ids;
  wa.pos_of_id = ix->pos_of_id; wa.lb = sa.lb; wa.ub = sa.ub; wa.key_off = d_ko;
  wa.cbuf = reinterpret_cast<uint32_t*>(A + L_cbuf);
  wa.cand_off = d_ko; wa.cand_packed = reinterpret_cast<uint64_t*>(A + L_cp);
  wa.n_cand = reinterpret_cast<int64_t*>(A + L_nc);
  wa.n_visited = reinterpret_cast<int64_t*>(A + L_nv);
  wa.zbuf = reinterpret_cast<uint64_t*>(A + L_z);
  wa.q = dq; wa.vectors = ix->vectors; wa.fp16 = ix->fp16; wa.D = d; wa.metric = ix->metric;
  wa.wide = wide ? 1 : 0;
  wa.max_c = max_cap;
  wa.qcap = ix->walk_qcap;
  wa.t_qpath = tracing ? reinterpret_cast<int32_t*>(A + L_qp) : nullptr;
  if (wide) {
    wa.cpos = presort && !rounds ? nullptr : reinterpret_cast<int32_t*>(A + L_cpos);
    wa.wbins = reinterpret_cast<uint32_t*>(A + L_wbins);
    wa.wstate = reinterpret_cast<uint32_t*>(A + L_wst);
    if (rounds) {
      wa.wround = reinterpret_cast<uint32_t*>(A + L_wround);
      wa.round1_alpha = ix->walk_alpha < 0.0f ? 0.8f : ix->walk_alpha;
    }
  }
  if (presort) {
    wa.t_pos = reinterpret_cast<uint32_t*>(A + L_rts);
    wa.t_idx = reinterpret_cast<uint32_t*>(A + L_rti);
    wa.t_bins = reinterpret_cast<uint32_t*>(A + L_rtb);
    wa.t_rank_tb = reinterpret_cast<uint32_t*>(A + L_rtp);
    wa.t_bin_off = d_bo;
    wa.t_shift = rt_shift;
  }
  if (wide) {
    StageScope st(s, 3);
    HIP_TRY(bbc::launch_rabitq_walk_prep(wa, s));
  }
  {
    StageScope st(s, 4);
    // the wide form's keys in two rounds: C's first bins, a walk that settles
    // most queries, then the rest of C for the others and a second walk
    for (int round = rounds ? 1 : 0; round <= (rounds ? 2 : 0); ++round) {
      wa.round = round;
      wa.keys_ready = 0;  // round 2: C's other keys by the device-wide grid
      if (tile_keys && round < 2) {
        // the exact keys of C, tile-major, at C's indices (what the walk reads)
        ta.cand_pos = reinterpret_cast<const uint32_t*>(wa.cpos); ta.pos_off = d_ko;
        ta.ncand_w = wa.wstate + 3; ta.ncand_stride = 4;
        ta.cand_off = d_ko; ta.cand_packed = wa.cand_packed;
        ta.sorted_pos = reinterpret_cast<uint32_t*>(A + L_rts);
        ta.sorted_idx = reinterpret_cast<uint32_t*>(A + L_rti);
        ta.pair_tb = reinterpret_cast<uint32_t*>(A + L_rtp);
        ta.bin_off = d_bo;
        ta.bin_beg = reinterpret_cast<uint32_t*>(A + L_rtb);
        ta.presorted = presort ? 1 : 0;
        ta.round = round;
        ta.wround = wa.wround;
        HIP_TRY(bbc::launch_tile_rerank(ta, rt_lds, s));
        ta.pairs_ready = 1;
        wa.keys_ready = 1;
      }
      HIP_TRY(bbc::launch_rabitq_walk(wa, s));
    }
  }
  bbc::FinalArgs fa{};
  fa.k = d_k; fa.n_cand = wa.n_cand; fa.cand_off = d_ko; fa.cand_packed = wa.cand_packed;
  fa.out_off = d_oo; fa.out_ids = d_oid; fa.out_dists = d_odist; fa.out_counts = d_ocnt; fa.metric = ix->metric;
  fa.scratch = reinterpret_cast<uint64_t*>(A + L_fs);
  {
    StageScope st(s, 5);
    if ((rc = launch_final_groups(ix, fg, reinterpret_cast<const int32_t*>(M + m_fq), fa, s))) return rc;
  }
  fa.max_kc = max_cap;
  if (host_io) {
    HIP_TRY(hipMemcpyAsync(out_ids, d_oid, 8 * nout, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(out_dists, d_odist, 4 * nout, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(out_counts, d_ocnt, 4 * nq, hipMemcpyDeviceToHost, s));
  }
  if (tracing) {
    auto cp = [&](void* dst, size_t off, size_t bytes) -> int32_t {
      if (dst) HIP_TRY(hipMemcpyAsync(dst, A + off, bytes, hipMemcpyDeviceToHost, s));
      return BBC_OK;
    };
    if ((rc = cp(tr->probe_lists, L_pl, 4 * npairs))) return rc;
    if ((rc = cp(tr->probe_keys, L_pk, 4 * npairs))) return rc;
    if ((rc = cp(tr->n_recheck, L_nr, 4 * nq))) return rc;
    if ((rc = cp(tr->n_cand, L_nc, 8 * nq))) return rc;
    if ((rc = cp(tr->n_visited, L_nv, 8 * nq))) return rc;
    if ((rc = cp(tr->walk_path, L_qp, 4 * nq))) return rc;
    if (tr->kernel_forms) {
      tr->kernel_forms[0] = -1;
      tr->kernel_forms[1] = bbc::final_topk_form(fa.max_kc);
      tr->kernel_forms[2] = sa.lpairs ? 3 : (!sa.force_1d && nq <= 65535) ? 2 : 1;
      tr->kernel_forms[3] = 0;
    }
    std::vector<int64_t> nsc(nq);
    HIP_TRY(hipMemcpyAsync(nsc.data(), A + L_ns, 8 * nq, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (tr->n_scanned) std::memcpy(tr->n_scanned, nsc.data(), 8 * nq);
    if (tr->est_off) {
      tr->est_off[0] = 0;
      for (int64_t i = 0; i < nq; ++i) tr->est_off[i + 1] = tr->est_off[i] + nsc[i];
    }
    auto ragged = [&](float* dst, size_t off) -> int32_t {
      if (!dst) return BBC_OK;
      std::vector<float> all(nkeys);
      HIP_TRY(hipMemcpy(all.data(), A + off, 4 * nkeys, hipMemcpyDeviceToHost));
      int64_t w = 0;
      for (int64_t i = 0; i < nq; ++i) {
        std::memcpy(dst + w, all.data() + key_off[i], 4 * nsc[i]);
        w += nsc[i];
      }
      return BBC_OK;
    };
    if ((rc = ragged(tr->est_keys, L_key))) return rc;
    if ((rc = ragged(tr->est_lb, L_lb))) return rc;
    if ((rc = ragged(tr->est_ub, L_ub))) return rc;
  }
  if (ctx && ctx->work_out) {
    HIP_TRY(hipMemcpyAsync(ctx->work_out, A + L_ns, 8 * nq, hipMemcpyDefault, s));
    HIP_TRY(hipMemcpyAsync(ctx->work_out + nq, A + L_nv, 8 * nq, hipMemcpyDefault, s));
  }
  if (!(ctx && ctx->ws)) HIP_TRY(ix->arena.release(s));
  if (ctx && ctx->capture) {
    t_capturing = false;
    HIP_TRY(hipStreamEndCapture(s, &ctx->graph));
  }
  if (host_io) HIP_TRY(hipStreamSynchronize(s));
  return BBC_OK;
}

int32_t run_search(bbc_index* ix, const float* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                   const bbc_search_params* p, const int64_t* out_off, int64_t* out_ids, float* out_dists,
                   int32_t* out_counts, bbc_search_trace* tr, SearchCtx* ctx = nullptr) {
  int32_t rc = validate_search(ix, queries, nq, k, nprobe, p, out_off);
  if (rc || nq == 0) return rc;
  rc = set_device(ix->device);
  if (rc) return rc;
  std::lock_guard<std::mutex> guard(ix->mu);
  if (ix->quant == BBC_QUANT_RABITQ)
    return run_search_rabitq(ix, queries, nq, k, nprobe, p, out_off, out_ids, out_dists, out_counts, tr, ctx);
  hipStream_t s = static_cast<hipStream_t>(p->stream);
  const bool host_io = p->device_io == 0;
  const int m = p->buckets ? p->buckets : 256;
  const int nsample = p->nsample ? p->nsample : 8;
  const int sample_factor = p->sample_factor ? p->sample_factor : 2;
  const int d = ix->d;
  const bool tracing = tr != nullptr;
  // the comparator collectors read every scanned key: all probed lists form
  // the "sample" phase and no key is filtered
  const bool bucket = p->collector == BBC_COLLECT_BUCKET;

  // host-side metadata: per query k, nprobe, and prefix offsets
  std::vector<int64_t> probe_off(nq + 1, 0), key_off(nq + 1, 0), cand_off(nq + 1, 0), kc_target(nq),
      sample_off(nq + 1, 0), surv_off(nq + 1, 0);
  int64_t max_kc = 0, max_scap = 0;
  int max_np = 0;
  const int64_t max_list = ix->h_maxS[1];
  for (int64_t i = 0; i < nq; ++i) {
    probe_off[i + 1] = probe_off[i] + nprobe[i];
    max_np = std::max(max_np, nprobe[i]);
    int64_t cap = kc_cap_of(ix, k[i], nprobe[i], p->ncand_ratio);
    // the sample stops at the first list that brings it to K_c keys
    const int64_t scap = !bucket ? ix->h_maxS[nprobe[i]]
                                 : std::min(ix->h_maxS[nprobe[i]],
                                            std::max(ix->h_maxS[std::min(nsample, nprobe[i])],
                                                     (int64_t)sample_factor * cap + max_list));
    sample_off[i + 1] = sample_off[i] + scap;
    max_scap = std::max(max_scap, scap);
    surv_off[i + 1] = surv_off[i] + (bucket ? ix->h_maxS[nprobe[i]] : 0);
    key_off[i + 1] = key_off[i] + (tracing ? ix->h_maxS[nprobe[i]] : 0);
    kc_target[i] = (int64_t)std::ceil(p->ncand_ratio * (double)k[i]);
    cand_off[i + 1] = cand_off[i] + cap;
    max_kc = std::max(max_kc, cap);
  }
  const int64_t npairs = probe_off[nq];
  const int64_t nkeys = key_off[nq];
  const int64_t ncand = cand_off[nq];
  const int64_t nout = out_off[nq];
  // tile-major re-rank (rows of at most 32 chunks): bins per query
  std::vector<int64_t> bin_off;
  int rt_shift = 0, rt_bins = 0;
  size_t rt_lds = 0;
  const bool tile_rr = ix->rerank_form == 0 &&
                       tile_plan(ix, nq, nprobe, max_np, 32, bin_off, &rt_shift, &rt_bins, &rt_lds);
  if (!tile_rr) bin_off.assign(nq + 1, 0);

  // metadata block (one upload): k, nprobe, then the prefix arrays
  FinalGroups fg;
  // the per-query kernels (codebook, collector, candidate sort) take the
  // queries largest candidate set first
  std::vector<int32_t> big_first((size_t)nq);
  {
    std::vector<int64_t> cap_of((size_t)nq);
    for (int64_t i = 0; i < nq; ++i) cap_of[(size_t)i] = cand_off[i + 1] - cand_off[i];
    final_groups(nq, k, cap_of, ix->num_cu, fg);
    for (int64_t i = 0; i < nq; ++i) big_first[(size_t)i] = (int32_t)i;
    std::stable_sort(big_first.begin(), big_first.end(),
                     [&](int32_t x, int32_t y) { return cap_of[(size_t)x] > cap_of[(size_t)y]; });
  }
  Plan mp;
  size_t m_k = mp.add(4 * nq), m_np = mp.add(4 * nq), m_po = mp.add(8 * (nq + 1)), m_ko = mp.add(8 * (nq + 1)),
         m_kt = mp.add(8 * nq), m_co = mp.add(8 * (nq + 1)), m_oo = mp.add(8 * (nq + 1)),
         m_so = mp.add(8 * (nq + 1)), m_vo = mp.add(8 * (nq + 1)), m_bo = mp.add(8 * (nq + 1)),
         m_fq = mp.add(4 * nq), m_bq = mp.add(4 * nq);
  Plan pl;
  Layout L{};
  L.meta = pl.add(mp.total);
  L.q = host_io ? pl.add(sizeof(float) * nq * d) : 0;
  L.dprime = pl.add(sizeof(float) * nq * ix->nlist);
  L.probe_lists = pl.add(4 * npairs);
  L.probe_keys = pl.add(4 * npairs);
  L.rank_off = pl.add(8 * npairs);
  L.n_scanned = pl.add(8 * nq);
  L.n_recheck = pl.add(4 * nq);
  L.nsample_q = pl.add(4 * nq);
  L.keys = tracing ? pl.add(4 * nkeys) : 0;
  L.sample_keys = pl.add(4 * sample_off[nq]);
  L.surv_key = pl.add(4 * surv_off[nq]);
  L.surv_pos = pl.add(4 * surv_off[nq]);
  L.pair_nsurv = pl.add(4 * npairs);
  L.surv_bucket = pl.add(surv_off[nq]);
  L.surv_total = pl.add(4 * nq);
  L.n_rejected = pl.add(4 * nq);
  L.books = pl.add(sizeof(bbc::QueryBook) * nq);
  L.pair_cnt = pl.add(4 * 2 * (size_t)ix->nlist);
  L.sorted_pairs = pl.add(4 * bbc::pair_slots(npairs, ix->nlist));
  L.sorted_q = pl.add(4 * bbc::pair_slots(npairs, ix->nlist));
  L.pair_split = pl.add(8);
  // pair sorts' per-block counts: the scan's (2 * nlist bins) then the
  // re-rank's (nlist) reuse it
  const int64_t bs_words = ix->pair_sort_lds ? bbc::pair_sort_table_words(nq, 2 * ix->nlist) : 0;
  L.bs_table = bs_words ? pl.add(4 * bs_words) : 0;
  // the tighter filter of the lists after the sample (float tables only: its
  // rescan runs the generic float-table kernel)
  const bool tight = bucket && !p->early_rerank && !p->lut_u8 && !p->keep_all_keys && ix->filt_fraction > 0.0f &&
                     ix->filt_fraction < 1.0f;
  L.rescan_q = tight ? pl.add(4 * nq) : 0;
  L.sminmax = bucket ? pl.add(8 * nq) : 0;  // the sample's smallest and largest key image
  L.cand_pos = pl.add(4 * ncand);
  L.cand_packed = pl.add(8 * ncand);
  L.n_cand = pl.add(8 * nq);
  L.qorder = pl.add(4 * nq);
  const bool early = bucket && p->early_rerank;
  if (early) {
    L.surv_exact = pl.add(4 * surv_off[nq]);
    L.n_early = pl.add(4 * nq);
    L.n_used = pl.add(4 * nq);
    L.t_tpred = pl.add(4 * nq);
  }
  // tile-major re-rank: its sort buffers
  const int rt_group = bbc::tile_rerank_group(d);
  const int64_t rt_lpairs_cap = npairs + (int64_t)ix->nlist * (rt_group - 1);
  if (tile_rr) {
    if (early) L.rt_sidx = pl.add(4 * ncand);  // results at the candidates' own places
    L.rt_sorted = pl.add(4 * ncand);
    L.rt_bins = pl.add(4 * bin_off[nq]);
    L.rt_ptb = pl.add(4 * npairs);
    L.rt_lcnt = pl.add(4 * ((int64_t)ix->nlist + 1));
    L.rt_lpairs = pl.add(8 * rt_lpairs_cap);
  }
  if (host_io) {
    L.out_ids = pl.add(8 * nout);
    L.out_dists = pl.add(4 * nout);
    L.out_counts = pl.add(4 * nq);
  }
  const size_t L_fs = pl.add(8 * nout);  // final top-k: winners grouped by bin
  if (tracing) {
    L.t_dmin = pl.add(4 * nq); L.t_delta = pl.add(4 * nq); L.t_map = pl.add(256 * nq);
    L.t_tau = pl.add(4 * nq); L.t_s = pl.add(8 * nq); L.t_counts = pl.add(4 * nq * m); L.t_nb = pl.add(8 * nq); L.t_nsk = pl.add(8 * nq);
  }
  if (ctx && ctx->size_only) {
    ctx->ws_bytes = pl.total;
    return BBC_OK;
  }
  char* A;
  if (ctx && ctx->ws) {
    A = ctx->ws;
  } else {
    HIP_TRY(ix->arena.reserve(pl.total));
    A = ix->arena.base;
    HIP_TRY(ix->arena.acquire(s));
  }

  // stage metadata through pinned memory (wait for the previous call's copy)
  char* H = nullptr;
  hipEvent_t meta_ev = nullptr;
  if ((rc = stage_meta(ix, ctx, mp.total, &H, &meta_ev))) return rc;
  std::memcpy(H + m_k, k, 4 * nq);
  std::memcpy(H + m_np, nprobe, 4 * nq);
  std::memcpy(H + m_po, probe_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_ko, key_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_kt, kc_target.data(), 8 * nq);
  std::memcpy(H + m_co, cand_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_oo, out_off, 8 * (nq + 1));
  std::memcpy(H + m_so, sample_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_vo, surv_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_bo, bin_off.data(), 8 * (nq + 1));
  std::memcpy(H + m_fq, fg.order.data(), 4 * nq);
  std::memcpy(H + m_bq, big_first.data(), 4 * nq);
  char* M = A + L.meta;
  if (ctx && ctx->capture) {
    HIP_TRY(hipMemcpy(M, H, mp.total, hipMemcpyHostToDevice));
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    t_capturing = true;
  } else {
    HIP_TRY(hipMemcpyAsync(M, H, mp.total, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(meta_ev, s));
  }
  const float* dq = queries;
  if (host_io) {
    HIP_TRY(hipMemcpyAsync(A + L.q, queries, sizeof(float) * nq * d, hipMemcpyHostToDevice, s));
    dq = reinterpret_cast<const float*>(A + L.q);
  }
  const int32_t* d_k = reinterpret_cast<const int32_t*>(M + m_k);
  const int32_t* d_np = reinterpret_cast<const int32_t*>(M + m_np);
  const int64_t* d_po = reinterpret_cast<const int64_t*>(M + m_po);
  const int64_t* d_ko = reinterpret_cast<const int64_t*>(M + m_ko);
  const int64_t* d_kt = reinterpret_cast<const int64_t*>(M + m_kt);
  const int64_t* d_co = reinterpret_cast<const int64_t*>(M + m_co);
  const int64_t* d_oo = reinterpret_cast<const int64_t*>(M + m_oo);
  const int64_t* d_so = reinterpret_cast<const int64_t*>(M + m_so);
  const int64_t* d_vo = reinterpret_cast<const int64_t*>(M + m_vo);
  const int64_t* d_bo = reinterpret_cast<const int64_t*>(M + m_bo);
  int64_t* d_oid = host_io ? reinterpret_cast<int64_t*>(A + L.out_ids) : out_ids;
  float* d_odist = host_io ? reinterpret_cast<float*>(A + L.out_dists) : out_dists;
  int32_t* d_ocnt = host_io ? reinterpret_cast<int32_t*>(A + L.out_counts) : out_counts;

  bbc::ProbeArgs pa{};
  pa.q = dq; pa.nq = nq; pa.d = d; pa.cent = ix->cent; pa.cent_bf16 = ix->cent_bf16; pa.dpad = ix->dpad;
  pa.cent_norm2 = ix->cent_norm2; pa.cent_norm = ix->cent_norm; pa.nlist = ix->nlist; pa.metric = ix->metric;
  pa.nprobe = d_np; pa.probe_off = d_po; pa.list_off = ix->list_off;
  pa.dprime = reinterpret_cast<float*>(A + L.dprime);
  pa.probe_lists = reinterpret_cast<int32_t*>(A + L.probe_lists);
  pa.probe_keys = reinterpret_cast<float*>(A + L.probe_keys);
  pa.rank_off = reinterpret_cast<int64_t*>(A + L.rank_off);
  pa.n_scanned = reinterpret_cast<int64_t*>(A + L.n_scanned);
  pa.n_recheck = reinterpret_cast<int32_t*>(A + L.n_recheck);
  pa.kc_target = d_kt; pa.nsample = bucket ? nsample : ix->nlist; pa.sample_factor = sample_factor;
  pa.nsample_q = reinterpret_cast<int32_t*>(A + L.nsample_q);
  pa.num_cu = ix->num_cu;
  {
    StageScope st(s, 0);  // coarse GEMM and probe select
    HIP_TRY(bbc::launch_probe(pa, s));
  }

  const int bcap = ix->collect_bcap;
  bbc::QueryBook* books = reinterpret_cast<bbc::QueryBook*>(A + L.books);
  float* surv_key = reinterpret_cast<float*>(A + L.surv_key);
  uint32_t* surv_pos = reinterpret_cast<uint32_t*>(A + L.surv_pos);
  uint32_t* pair_nsurv = reinterpret_cast<uint32_t*>(A + L.pair_nsurv);
  uint32_t* n_rejected = reinterpret_cast<uint32_t*>(A + L.n_rejected);
  float* sample_keys = reinterpret_cast<float*>(A + L.sample_keys);

  bbc::PqScanArgs sa{};
  sa.q = dq; sa.nq = nq; sa.d = d; sa.cent = ix->cent; sa.M = ix->M; sa.bits = ix->bits;
  sa.codebook = ix->codebook; sa.codes = ix->codes; sa.code_stride = ix->code_stride;
  sa.list_off = ix->list_off; sa.probe_off = d_po; sa.probe_lists = pa.probe_lists; sa.rank_off = pa.rank_off;
  sa.key_off = d_ko;
  sa.nlist = ix->nlist; sa.npairs = npairs; sa.num_cu = ix->num_cu; sa.nxcd = ix->nxcd;
  sa.scan_variant = ix->scan_variant;
  sa.lut_u8 = p->lut_u8;
  sa.pair_cnt = reinterpret_cast<uint32_t*>(A + L.pair_cnt);
  sa.sorted_pairs = reinterpret_cast<uint32_t*>(A + L.sorted_pairs);
  sa.sorted_q = reinterpret_cast<uint32_t*>(A + L.sorted_q);
  sa.pair_split = reinterpret_cast<uint32_t*>(A + L.pair_split);
  sa.bs_table = bs_words ? reinterpret_cast<uint32_t*>(A + L.bs_table) : nullptr;
  sa.nsample_q = pa.nsample_q; sa.sample_keys = sample_keys; sa.sample_off = d_so; sa.books = books;
  sa.surv_key = surv_key; sa.surv_pos = surv_pos; sa.surv_off = d_vo; sa.pair_nsurv = pair_nsurv;
  sa.n_rejected = n_rejected;
  sa.trace_keys = tracing ? reinterpret_cast<float*>(A + L.keys) : nullptr;
  sa.early = early;
  sa.metric = ix->metric;
  sa.vectors = reinterpret_cast<const float*>(ix->vectors);
  sa.surv_exact = early ? reinterpret_cast<float*>(A + L.surv_exact) : nullptr;
  sa.n_early = early ? reinterpret_cast<uint32_t*>(A + L.n_early) : nullptr;

  bbc::CollectArgs ca{};
  ca.nq = nq; ca.n_scanned = pa.n_scanned; ca.nprobe = d_np;
  ca.probe_off = d_po; ca.probe_lists = pa.probe_lists; ca.rank_off = pa.rank_off; ca.list_off = ix->list_off;
  ca.list_ids = ix->list_ids; ca.pos_of_id = ix->pos_of_id; ca.kc_target = d_kt; ca.cand_off = d_co; ca.m = m;
  ca.nsample_q = pa.nsample_q; ca.bcap = bcap; ca.max_sample = max_scap; ca.cand_pos = reinterpret_cast<uint32_t*>(A + L.cand_pos);
  ca.bnd_scratch = reinterpret_cast<uint64_t*>(A + L.cand_packed);
  ca.n_cand = reinterpret_cast<int64_t*>(A + L.n_cand);
  ca.sample_keys = sample_keys; ca.sample_off = d_so; ca.books = books;
  ca.surv_key = surv_key; ca.surv_pos = surv_pos; ca.surv_off = d_vo; ca.pair_nsurv = pair_nsurv;
  ca.surv_total = reinterpret_cast<uint32_t*>(A + L.surv_total);
  ca.surv_bucket = reinterpret_cast<uint8_t*>(A + L.surv_bucket);
  ca.n_rejected = n_rejected;
  if (tracing) {
    ca.t_dmin = reinterpret_cast<float*>(A + L.t_dmin); ca.t_delta = reinterpret_cast<float*>(A + L.t_delta);
    ca.t_map = reinterpret_cast<uint8_t*>(A + L.t_map); ca.t_tau = reinterpret_cast<int32_t*>(A + L.t_tau);
    ca.t_s = reinterpret_cast<int64_t*>(A + L.t_s); ca.t_counts = reinterpret_cast<int32_t*>(A + L.t_counts);
    ca.t_nboundary = reinterpret_cast<int64_t*>(A + L.t_nb);
    ca.t_nsample_keys = reinterpret_cast<int64_t*>(A + L.t_nsk);
  }
  ca.early = early;
  ca.keep_all = p->keep_all_keys != 0;
  ca.filt_fraction = tight ? ix->filt_fraction : 0.0f;
  ca.qorder = reinterpret_cast<const int32_t*>(M + m_bq);
  if (bucket) {
    sa.smin = reinterpret_cast<uint32_t*>(A + L.sminmax);
    sa.smax = sa.smin + nq;
    ca.smin = sa.smin;
    ca.smax = sa.smax;
  }
  ca.t_tau_pred = early ? reinterpret_cast<int32_t*>(A + L.t_tpred) : nullptr;

  // scan of the sample lists, codebook, scan of the rest through the filter,
  // then the collector over the survivors
  {
    StageScope st(s, 1);
    HIP_TRY(bbc::launch_pair_sort(sa, s));
    sa.mode = 0;
    HIP_TRY(bbc::launch_pq_scan(sa, s));
    sa.smin = sa.smax = nullptr;  // the filter scan keeps no extremes
  }
  if (bucket) {
    {
      StageScope st(s, 6);
      HIP_TRY(bbc::launch_codebook(ca, s));
    }
    {
      StageScope st(s, 2);
      sa.mode = 1;
      if (early) HIP_TRY(bbc::launch_zero_u32(sa.n_early, nq, s));
      HIP_TRY(bbc::launch_pq_scan(sa, s));
      if (tight) HIP_TRY(bbc::launch_filter_rescan(sa, d_kt, reinterpret_cast<uint32_t*>(A + L.rescan_q), s));
    }
    {
      StageScope st(s, 3);
      HIP_TRY(bbc::launch_collect_bucket(ca, s));
    }
    if (early) {  // candidates re-ranked during the scan: (exact key, id) in place
      StageScope st(s, 4);
      bbc::EarlyFillArgs ea{};
      ea.nq = nq; ea.n_cand = ca.n_cand; ea.cand_off = d_co; ea.cand_pos = ca.cand_pos; ea.surv_off = d_vo;
      ea.surv_pos = surv_pos; ea.surv_exact = sa.surv_exact; ea.list_ids = ix->list_ids;
      ea.cand_packed = reinterpret_cast<uint64_t*>(A + L.cand_packed);
      ea.n_used = reinterpret_cast<uint32_t*>(A + L.n_used);
      HIP_TRY(bbc::launch_zero_u32(ea.n_used, nq, s));
      HIP_TRY(bbc::launch_early_fill(ea, max_kc, s));
    }
  } else {
    bbc::CompareArgs xa{};
    xa.nq = nq; xa.n_scanned = pa.n_scanned; xa.kc_target = d_kt; xa.nprobe = d_np; xa.probe_off = d_po;
    xa.rank_off = pa.rank_off; xa.probe_lists = pa.probe_lists; xa.list_off = ix->list_off;
    xa.list_ids = ix->list_ids; xa.pos_of_id = ix->pos_of_id;
    xa.keys = reinterpret_cast<const float*>(A + L.sample_keys); xa.key_off = d_so;
    xa.cand_off = d_co; xa.cand_pos = ca.cand_pos; xa.n_cand = ca.n_cand;
    xa.heap = reinterpret_cast<uint64_t*>(A + L.cand_packed);
    xa.max_kc = max_kc;
    StageScope st(s, 3);
    HIP_TRY(bbc::launch_compare_collect(xa, p->collector, s));
  }

  bbc::RerankArgs ra{};
  ra.q = dq; ra.nq = nq; ra.d = d; ra.metric = ix->metric; ra.vectors = ix->vectors; ra.fp16 = ix->fp16;
  ra.list_ids = ix->list_ids; ra.cand_pos = ca.cand_pos; ra.cand_off = d_co; ra.n_cand = ca.n_cand;
  ra.cand_packed = reinterpret_cast<uint64_t*>(A + L.cand_packed);
  {
    StageScope st(s, 4);
    if (tile_rr) {
      bbc::TileRerankArgs ta{};
      ta.q = dq; ta.nq = nq; ta.d = d; ta.metric = ix->metric; ta.vectors = ix->vectors; ta.fp16 = ix->fp16;
      ta.list_ids = ix->list_ids; ta.list_off = ix->list_off; ta.list_of_pos = ix->list_of_pos;
      ta.nprobe = d_np; ta.probe_off = d_po; ta.probe_lists = pa.probe_lists; ta.nlist = ix->nlist;
      ta.cand_pos = ca.cand_pos; ta.pos_off = d_co; ta.n_cand = ca.n_cand;
      ta.cand_off = d_co; ta.cand_packed = ra.cand_packed;
      ta.npairs = npairs; ta.max_np = max_np; ta.tshift = rt_shift; ta.max_bins = rt_bins;
      ta.qorder = reinterpret_cast<const int32_t*>(M + m_bq);
      ta.sorted_pos = reinterpret_cast<uint32_t*>(A + L.rt_sorted);
      ta.pair_tb = reinterpret_cast<uint32_t*>(A + L.rt_ptb);
      ta.bin_off = d_bo;
      ta.bin_beg = reinterpret_cast<uint32_t*>(A + L.rt_bins);
      ta.lcnt = reinterpret_cast<uint32_t*>(A + L.rt_lcnt);
      ta.lpairs = reinterpret_cast<uint64_t*>(A + L.rt_lpairs);
      ta.lpairs_cap = rt_lpairs_cap;
      ta.bs_table = bs_words ? reinterpret_cast<uint32_t*>(A + L.bs_table) : nullptr;
      ta.no_run_list = ix->no_run_list;
      ta.group = rt_group;
      if (early) ta.sorted_idx = reinterpret_cast<uint32_t*>(A + L.rt_sidx);
      HIP_TRY(bbc::launch_tile_rerank(ta, rt_lds, s));
    } else {
      if (ix->nlist <= bbc::QUERY_ORDER_MAX_LISTS && nq > 1) {
        int32_t* qo = reinterpret_cast<int32_t*>(A + L.qorder);
        HIP_TRY(bbc::launch_query_order(pa.probe_lists, d_po, d_np, nq, ix->nlist, qo, s));
        ra.qorder = qo;
      }
      HIP_TRY(bbc::launch_rerank(ra, max_kc, s));
    }
  }

  // trace copies of the exact candidate keys happen before the final step
  // reuses the candidate buffer as merge scratch
  std::vector<uint64_t> cand_packed_h;
  std::vector<uint32_t> cand_pos_h;
  std::vector<int64_t> n_cand_h(nq);
  if (tracing && (tr->cand_ids || tr->cand_exact || tr->cand_off)) {
    cand_packed_h.resize(ncand);
    HIP_TRY(hipMemcpyAsync(cand_packed_h.data(), ra.cand_packed, 8 * ncand, hipMemcpyDeviceToHost, s));
  }

  // final top-k LDS: `cap` packed items (dynamic; the largest min(k, K_c) of
  // the batch when it fits) + the kernel's static tables
  bbc::FinalArgs fa{};
  fa.k = d_k; fa.n_cand = ca.n_cand; fa.cand_off = d_co; fa.cand_packed = ra.cand_packed;
  fa.out_off = d_oo; fa.out_ids = d_oid; fa.out_dists = d_odist; fa.out_counts = d_ocnt; fa.metric = ix->metric;
  fa.scratch = reinterpret_cast<uint64_t*>(A + L_fs);
  {
    StageScope st(s, 5);
    if ((rc = launch_final_groups(ix, fg, reinterpret_cast<const int32_t*>(M + m_fq), fa, s))) return rc;
  }
  fa.max_kc = max_kc;

  if (host_io) {
    HIP_TRY(hipMemcpyAsync(out_ids, d_oid, 8 * nout, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(out_dists, d_odist, 4 * nout, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(out_counts, d_ocnt, 4 * nq, hipMemcpyDeviceToHost, s));
  }
  if (tracing) {
    auto cp = [&](void* dst, size_t off, size_t bytes) -> int32_t {
      if (dst) HIP_TRY(hipMemcpyAsync(dst, A + off, bytes, hipMemcpyDeviceToHost, s));
      return BBC_OK;
    };
    if (tr->kernel_forms) {
      tr->kernel_forms[0] = bucket ? bbc::codebook_form(ca.max_sample) : -1;
      tr->kernel_forms[1] = bbc::final_topk_form(fa.max_kc);
      tr->kernel_forms[2] = -1;
      tr->kernel_forms[3] = 0;
    }
    if ((rc = cp(tr->probe_lists, L.probe_lists, 4 * npairs))) return rc;
    if ((rc = cp(tr->probe_keys, L.probe_keys, 4 * npairs))) return rc;
    if ((rc = cp(tr->n_recheck, L.n_recheck, 4 * nq))) return rc;
    std::vector<uint32_t> nsurv(nq, 0);
    if (bucket) {  // the bucket collector's own intermediates
      if ((rc = cp(tr->dmin, L.t_dmin, 4 * nq))) return rc;
      if ((rc = cp(tr->delta, L.t_delta, 4 * nq))) return rc;
      if ((rc = cp(tr->map, L.t_map, 256 * nq))) return rc;
      if ((rc = cp(tr->tau, L.t_tau, 4 * nq))) return rc;
      if ((rc = cp(tr->s, L.t_s, 8 * nq))) return rc;
      if ((rc = cp(tr->bucket_counts, L.t_counts, 4 * nq * m))) return rc;
      if ((rc = cp(tr->n_boundary, L.t_nb, 8 * nq))) return rc;
      if ((rc = cp(tr->n_sample_lists, L.nsample_q, 4 * nq))) return rc;
      if ((rc = cp(tr->n_sample_keys, L.t_nsk, 8 * nq))) return rc;
      HIP_TRY(hipMemcpyAsync(nsurv.data(), A + L.surv_total, 4 * nq, hipMemcpyDeviceToHost, s));
    }
    std::vector<uint32_t> nearly(nq, 0), nused(nq, 0);
    if (early) {
      if ((rc = cp(tr->tau_pred, L.t_tpred, 4 * nq))) return rc;
      HIP_TRY(hipMemcpyAsync(nearly.data(), A + L.n_early, 4 * nq, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(nused.data(), A + L.n_used, 4 * nq, hipMemcpyDeviceToHost, s));
    }
    std::vector<int64_t> nsc(nq);
    HIP_TRY(hipMemcpyAsync(nsc.data(), A + L.n_scanned, 8 * nq, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(n_cand_h.data(), A + L.n_cand, 8 * nq, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (tr->n_scanned) std::memcpy(tr->n_scanned, nsc.data(), 8 * nq);
    if (tr->n_cand) std::memcpy(tr->n_cand, n_cand_h.data(), 8 * nq);
    if (tr->n_survivors && bucket)
      for (int64_t i = 0; i < nq; ++i) tr->n_survivors[i] = nsurv[i];
    if (early) {
      for (int64_t i = 0; i < nq; ++i) {
        if (tr->n_early) tr->n_early[i] = nearly[i];
        if (tr->n_early_used) tr->n_early_used[i] = nused[i];
      }
    }
    if (tr->est_off) {
      tr->est_off[0] = 0;
      for (int64_t i = 0; i < nq; ++i) tr->est_off[i + 1] = tr->est_off[i] + nsc[i];
    }
    if (tr->est_keys) {
      std::vector<float> kk(nkeys);
      HIP_TRY(hipMemcpy(kk.data(), A + L.keys, 4 * nkeys, hipMemcpyDeviceToHost));
      int64_t w = 0;
      for (int64_t i = 0; i < nq; ++i) {
        std::memcpy(tr->est_keys + w, kk.data() + key_off[i], 4 * nsc[i]);
        w += nsc[i];
      }
    }
    if (tr->cand_off) {
      tr->cand_off[0] = 0;
      for (int64_t i = 0; i < nq; ++i) tr->cand_off[i + 1] = tr->cand_off[i] + n_cand_h[i];
    }
    if (tr->cand_ids || tr->cand_exact) {
      int64_t w = 0;
      for (int64_t i = 0; i < nq; ++i) {
        for (int64_t j = 0; j < n_cand_h[i]; ++j) {
          uint64_t v = cand_packed_h[cand_off[i] + j];
          uint32_t kb = (uint32_t)(v >> 32);
          uint32_t fb = (kb & 0x80000000u) ? (kb & 0x7fffffffu) : ~kb;
          float key;
          std::memcpy(&key, &fb, 4);
          if (tr->cand_ids) tr->cand_ids[w] = (int64_t)(v & 0xffffffffu);
          if (tr->cand_exact) tr->cand_exact[w] = key;
          ++w;
        }
      }
    }
  }
  if (ctx && ctx->work_out) {
    HIP_TRY(hipMemcpyAsync(ctx->work_out, A + L.n_scanned, 8 * nq, hipMemcpyDefault, s));
    HIP_TRY(hipMemcpyAsync(ctx->work_out + nq, A + L.n_cand, 8 * nq, hipMemcpyDefault, s));
  }
  if (!(ctx && ctx->ws)) HIP_TRY(ix->arena.release(s));
  if (ctx && ctx->capture) {
    t_capturing = false;
    HIP_TRY(hipStreamEndCapture(s, &ctx->graph));
  }
  if (host_io) HIP_TRY(hipStreamSynchronize(s));
  return BBC_OK;
}

}  // namespace

namespace bbc {

int32_t search_in_workspace(bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                            const int32_t* nprobe, const bbc_search_params* p, const int64_t* out_off,
                            int64_t* out_ids, float* out_dists, int32_t* out_counts, char* ws, size_t* ws_bytes,
                            int64_t* work_out, const MetaStaging* meta) {
  if (!p || !ws_bytes) return fail(BBC_EINVAL, "NULL argument");
  if (!p->device_io) return fail(BBC_EINVAL, "a workspace search needs device I/O");
  // a sizing pass reads no query: any non-null pointer passes validation
  static const float no_query = 0.0f;
  if (!ws && !queries) queries = &no_query;
  SearchCtx ctx;
  ctx.size_only = ws == nullptr;
  ctx.ws = ws;
  ctx.work_out = work_out;
  if (meta) {
    ctx.meta_host = meta->host;
    ctx.meta_cap = meta->bytes;
    ctx.meta_ev = meta->done;
  }
  const int32_t rc = run_search(ix, queries, nq, k, nprobe, p, out_off, out_ids, out_dists, out_counts, nullptr, &ctx);
  if (ctx.size_only) *ws_bytes = ctx.ws_bytes;
  return rc;
}

int index_device(const bbc_index* ix) { return ix ? ix->device : -1; }

}  // namespace bbc

extern "C" {

int32_t bbc_search(const bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                   const int32_t* nprobe, const bbc_search_params* params, const int64_t* out_offsets,
                   int64_t* out_ids, float* out_dists, int32_t* out_counts) {
  return run_search(const_cast<bbc_index*>(ix), queries, nq, k, nprobe, params, out_offsets, out_ids,
                    out_dists, out_counts, nullptr);
}

int32_t bbc_search_traced(const bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                          const int32_t* nprobe, const bbc_search_params* params,
                          const int64_t* out_offsets, int64_t* out_ids, float* out_dists,
                          int32_t* out_counts, bbc_search_trace* trace) {
  if (!params || params->device_io) return fail(BBC_EINVAL, "traced search needs host I/O");
  if (!trace) return fail(BBC_EINVAL, "trace is NULL");
  return run_search(const_cast<bbc_index*>(ix), queries, nq, k, nprobe, params, out_offsets, out_ids,
                    out_dists, out_counts, trace);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free search: the workspace is a fixed device array
// ---------------------------------------------------------------------------
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = BBC_NOALLOC_MAX_BYTES;  // device scratch per GPU
constexpr size_t NOALLOC_META_BYTES = (size_t)1 << 20;       // host staging of the metadata block
constexpr int NOALLOC_MAX_DEVICES = 64;

}  // namespace

// The allocation-free search's workspace.  In host code this name stands for
// the array but is not its device address: kernels get the address that
// hipGetSymbolAddress returns for the current device (each GPU holds its own
// copy, at its own address, until the process ends).
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

struct NoAllocDevice {
  char* ptr = nullptr;             // device address of this GPU's copy of `scratch`
  hipEvent_t meta_done = nullptr;  // recorded after each metadata upload out of g_noalloc_meta
};
std::mutex g_noalloc_mu;  // serialises the host side of every allocation-free call
NoAllocDevice g_noalloc[NOALLOC_MAX_DEVICES];
alignas(256) char g_noalloc_meta[NOALLOC_META_BYTES];

// Once per device, with that device current: the device address of its copy
// of `scratch` and the staging buffer's event.
int32_t noalloc_setup(int dev) {
  NoAllocDevice& nd = g_noalloc[dev];
  if (nd.ptr) return BBC_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(BBC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  hipEvent_t ev = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  nd.meta_done = ev;
  nd.ptr = static_cast<char*>(ptr);
  return BBC_OK;
}

}  // namespace

extern "C" {

int32_t bbc_search_noalloc(const bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                           const int32_t* nprobe, const bbc_search_params* params, const int64_t* out_offsets,
                           int64_t* out_ids, float* out_dists, int32_t* out_counts) {
  if (!ix) return fail(BBC_EINVAL, "index is NULL");
  if (!params) return fail(BBC_EINVAL, "params is NULL");
  if (!params->device_io) return fail(BBC_EINVAL, "the allocation-free search needs device I/O (device_io = 1)");
  const int dev = ix->device;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(BBC_EUNSUPPORTED, "device ordinal out of range");
  std::lock_guard<std::mutex> guard(g_noalloc_mu);
  int32_t rc = set_device(dev);
  if (rc) return rc;
  if ((rc = noalloc_setup(dev))) return rc;
  bbc_index* mix = const_cast<bbc_index*>(ix);
  size_t need = 0;
  rc = bbc::search_in_workspace(mix, queries, nq, k, nprobe, params, out_offsets, out_ids, out_dists, out_counts,
                                nullptr, &need);
  if (rc || nq == 0) return rc;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(BBC_ENOMEM, "the batch needs " + std::to_string(need) +
                                " bytes of workspace, above the allocation-free maximum of " +
                                std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes: split it into smaller batches");
  const bbc::MetaStaging ms{g_noalloc_meta, NOALLOC_META_BYTES, g_noalloc[dev].meta_done};
  return bbc::search_in_workspace(mix, queries, nq, k, nprobe, params, out_offsets, out_ids, out_dists, out_counts,
                                  g_noalloc[dev].ptr, &need, nullptr, &ms);
}

struct bbc_plan {
  bbc_index* ix = nullptr;
  int64_t nq = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;  // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t scan_variant = 0, buckets = 0, sample_factor = 0, bcap = 0;
};

static void plan_release(bbc_plan* pl) {
  if (!pl) return;
  if (pl->ix) hipSetDevice(pl->ix->device);
  if (pl->exec) hipGraphExecDestroy(pl->exec);
  if (pl->graph) hipGraphDestroy(pl->graph);
  if (pl->stream) { hipStreamSynchronize(pl->stream); hipStreamDestroy(pl->stream); }
  if (pl->ws) hipFree(pl->ws);
  delete pl;
}

int32_t bbc_plan_create(bbc_index* ix, int64_t nq, const int32_t* k, const int32_t* nprobe,
                        const bbc_search_params* params, const float* queries, const int64_t* out_offsets,
                        int64_t* out_ids, float* out_dists, int32_t* out_counts, int32_t autotune, bbc_plan** out) {
  if (!out) return fail(BBC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params || !params->device_io) return fail(BBC_EINVAL, "a plan needs device pointers (device_io = 1)");
  if (!out_ids || !out_dists || !out_counts) return fail(BBC_EINVAL, "NULL output");
  int32_t rc = validate_search(ix, queries, nq, k, nprobe, params, out_offsets);
  if (rc) return rc;
  if (nq < 1) return fail(BBC_EINVAL, "a plan needs nq >= 1");
  if ((rc = set_device(ix->device))) return rc;
  bbc_plan* pl = new bbc_plan();
  pl->ix = ix;
  pl->nq = nq;
  bbc_search_params prm = *params;
  if (HIP_FAILED(hipStreamCreateWithFlags(&pl->stream, hipStreamNonBlocking))) {
    plan_release(pl);
    return fail(BBC_EDEVICE, "hipStreamCreateWithFlags failed");
  }
  prm.stream = pl->stream;
  const int saved_variant = ix->scan_variant, saved_bcap = ix->collect_bcap;
  pl->scan_variant = ix->scan_variant;
  pl->buckets = prm.buckets;
  pl->sample_factor = prm.sample_factor;
  pl->bcap = ix->collect_bcap;
  // autotune (PQ, bucket collector): a coordinate search, timed on the batch
  // itself, over the scan block geometry, the bucket count, the codebook
  // sample's size (a larger sample gives a tighter relaxed threshold and
  // fewer survivors but a costlier codebook) and the collector's LDS budget
  // for sorting the threshold bucket; two passes over the four.  Every
  // choice returns the same results.
  if (autotune && ix->quant == BBC_QUANT_PQ && prm.collector == BBC_COLLECT_BUCKET) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    int cur[4] = {ix->scan_variant, prm.buckets ? prm.buckets : 256, prm.sample_factor ? prm.sample_factor : 2,
                  ix->collect_bcap};
    const std::vector<int> choices[4] = {{0, 1, 2, 3, 4}, {64, 128, 256}, {2, 3, 4}, {1024, 4096}};
    auto time_of = [&](const int* c, float* out_ms) -> int32_t {
      ix->scan_variant = c[0];
      prm.buckets = c[1];
      prm.sample_factor = c[2];
      ix->collect_bcap = c[3];
      float ms = 0.0f;
      for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(e0, pl->stream);
        const int32_t r = run_search(ix, queries, nq, k, nprobe, &prm, out_offsets, out_ids, out_dists, out_counts,
                                     nullptr);
        if (r) return r;
        hipEventRecord(e1, pl->stream);
        hipEventSynchronize(e1);
        hipEventElapsedTime(&ms, e0, e1);
      }
      *out_ms = ms;
      return BBC_OK;
    };
    float best = 1e30f;
    rc = time_of(cur, &best);
    for (int pass = 0; pass < 2 && rc == BBC_OK; ++pass)
      for (int dim = 0; dim < 4 && rc == BBC_OK; ++dim)
        for (int v : choices[dim]) {
          if (v == cur[dim]) continue;
          int trial[4] = {cur[0], cur[1], cur[2], cur[3]};
          trial[dim] = v;
          float ms = 0.0f;
          if ((rc = time_of(trial, &ms))) break;
          if (ms < best) {
            best = ms;
            cur[dim] = v;
          }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) {
      ix->scan_variant = saved_variant;
      ix->collect_bcap = saved_bcap;
      plan_release(pl);
      return rc;
    }
    pl->scan_variant = cur[0];
    pl->buckets = cur[1];
    pl->sample_factor = cur[2];
    pl->bcap = cur[3];
  }
  ix->scan_variant = pl->scan_variant;
  ix->collect_bcap = pl->bcap;
  prm.buckets = pl->buckets;
  prm.sample_factor = pl->sample_factor;
  SearchCtx sz;
  sz.size_only = true;
  rc = run_search(ix, queries, nq, k, nprobe, &prm, out_offsets, out_ids, out_dists, out_counts, nullptr, &sz);
  if (rc == BBC_OK && HIP_FAILED(hipMalloc(reinterpret_cast<void**>(&pl->ws), sz.ws_bytes)))
    rc = fail(BBC_ENOMEM, "plan workspace allocation failed");
  pl->ws_bytes = sz.ws_bytes;
  SearchCtx cap;
  cap.ws = pl->ws;
  cap.capture = true;
  if (rc == BBC_OK) {
    rc = run_search(ix, queries, nq, k, nprobe, &prm, out_offsets, out_ids, out_dists, out_counts, nullptr, &cap);
    if (t_capturing) {  // a launch failed during the capture: close it
      t_capturing = false;
      hipGraph_t g = nullptr;
      hipStreamEndCapture(pl->stream, &g);
      if (g) hipGraphDestroy(g);
    }
  }
  ix->scan_variant = saved_variant;
  ix->collect_bcap = saved_bcap;
  pl->graph = cap.graph;
  if (rc == BBC_OK && HIP_FAILED(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0)))
    rc = fail(BBC_EDEVICE, "hipGraphInstantiate failed");
  if (rc) { plan_release(pl); return rc; }
  *out = pl;
  return BBC_OK;
}

int32_t bbc_plan_execute(bbc_plan* pl, void* stream) {
  if (!pl || !pl->exec) return fail(BBC_EINVAL, "plan is NULL");
  int32_t rc = set_device(pl->ix->device);
  if (rc) return rc;
  HIP_TRY(hipGraphLaunch(pl->exec, static_cast<hipStream_t>(stream)));
  return BBC_OK;
}

int32_t bbc_plan_info(const bbc_plan* pl, int32_t* scan_variant, int32_t* buckets, int32_t* sample_factor,
                      int32_t* bcap, int64_t* workspace_bytes) {
  if (!pl) return fail(BBC_EINVAL, "plan is NULL");
  if (scan_variant) *scan_variant = pl->scan_variant;
  if (buckets) *buckets = pl->buckets;
  if (sample_factor) *sample_factor = pl->sample_factor;
  if (bcap) *bcap = pl->bcap;
  if (workspace_bytes) *workspace_bytes = (int64_t)pl->ws_bytes;
  return BBC_OK;
}

void bbc_plan_free(bbc_plan* pl) { plan_release(pl); }

int64_t bbc_query_bytes(const bbc_index* ix, int32_t k, int32_t nprobe, const bbc_search_params* p) {
  if (!ix || !p) return fail(BBC_EINVAL, "NULL argument");
  // the workspace a one-query search with device I/O reserves, from the
  // search's own sizing pass (the same layout the search then allocates)
  bbc_search_params q = *p;
  q.device_io = 1;
  q.stream = nullptr;
  const float dummy = 0.0f;
  const int64_t off[2] = {0, k};
  SearchCtx sz;
  sz.size_only = true;
  const int32_t rc = run_search(const_cast<bbc_index*>(ix), &dummy, 1, &k, &nprobe, &q, off, nullptr, nullptr,
                                nullptr, nullptr, &sz);
  if (rc) return rc;
  return (int64_t)sz.ws_bytes;
}

}  // extern "C"

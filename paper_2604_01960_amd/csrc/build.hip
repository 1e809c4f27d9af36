// Index build: IVF k-means and residual PQ (background section: the IVF
// index partitions the vectors with k-means; PQ keeps per-sub-space
// codebooks and codes).  Random draws (training rows, seeds) are inputs.
//
// Rules (shared with any other implementation of the same build):
//  * assignment: nearest centroid by canonical FP32 squared L2, ties to the
//    smaller list id -- on the GPU through the probe kernels with nprobe = 1
//    (BF16 MFMA pre-filter, error-bounded FP32 recheck);
//  * update: centroid = float64 sum of its members in ascending row order,
//    divided by the count in float64, rounded once to float32; each empty
//    cluster (ascending id) splits the currently largest one: both become the
//    largest centroid scaled by (1 + 2^-10) and (1 - 2^-10) on alternating
//    elements (even elements: the empty one gets the up-scaled value) and the
//    member count is shared (floor half to the empty one);
//  * PQ: per sub-space k-means on the residuals x - c(x) of the PQ rows with
//    the sequential sub-vector distance, empty codewords keep their value;
//    codes = nearest codeword, ties to the smaller index.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bbc.h"
#include "kernels.h"

namespace bbc {

// Gather rows[i] of x into out (row-major), float4 granularity.
__global__ void gather_rows_kernel(const float* __restrict__ x, const int64_t* __restrict__ rows, int64_t nrows,
                                   int d, float* __restrict__ out) {
  const int64_t nc = d / 4;
  const int64_t total = nrows * nc;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / nc, c = t % nc;
    reinterpret_cast<float4*>(out)[i * nc + c] = reinterpret_cast<const float4*>(x + rows[i] * d)[c];
  }
}

// Code of each (row, sub-space): blockIdx.y = sub-space m, the sub-space's
// codebook in LDS; residual element r = x - c(x), then t = r - C and
// acc = fma(t, t, acc) sequentially from +0; ties to the smaller codeword.
__global__ __launch_bounds__(256) void pq_assign_kernel(const float* __restrict__ x, const int64_t* __restrict__ rows,
                                                        int64_t nrows, const int32_t* __restrict__ assign_of_row,
                                                        const float* __restrict__ cent, const float* __restrict__ codebook,
                                                        int d, int M, int ksub, uint8_t* __restrict__ codes) {
  extern __shared__ float cbm[];
  const int m = blockIdx.y;
  const int dsub = d / M;
  for (int i = threadIdx.x; i < ksub * dsub; i += blockDim.x) cbm[i] = codebook[(int64_t)m * ksub * dsub + i];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = rows[i];
    const float* xr = x + row * d + m * dsub;
    const float* cr = cent + (int64_t)assign_of_row[row] * d + m * dsub;
    float r[16];
    for (int e = 0; e < dsub; ++e) r[e] = xr[e] - cr[e];
    int best = 0;
    float bk = 0.0f;
    for (int b = 0; b < ksub; ++b) {
      float acc = 0.0f;
      for (int e = 0; e < dsub; ++e) {
        const float t = r[e] - cbm[b * dsub + e];
        acc = __builtin_fmaf(t, t, acc);
      }
      if (b == 0 || acc < bk) { bk = acc; best = b; }
    }
    codes[i * M + m] = (uint8_t)best;
  }
}

}  // namespace bbc

namespace {

int32_t bfail(int32_t code, const std::string& m) { return bbc::set_error(code, m); }

#define BTRY(expr)                                                                      \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return bfail(_e == hipErrorOutOfMemory ? BBC_ENOMEM : BBC_EDEVICE,                \
                   std::string(#expr) + ": " + hipGetErrorString(_e));                  \
  } while (0)

template <typename T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
  hipError_t alloc(size_t n) {
    if (p) { (void)hipFree(p); p = nullptr; }
    return hipMalloc(reinterpret_cast<void**>(&p), sizeof(T) * std::max<size_t>(n, 1));
  }
};

uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Nearest-centroid assignment on the GPU for `nrows` contiguous rows at dx.
struct Assigner {
  int32_t d, nlist, dpad;
  DevBuf<float> cent, cn2, cn, dprime, pkeys;
  DevBuf<uint16_t> cb16;
  DevBuf<int64_t> probe_off, list_off, rank_off, nsc;
  DevBuf<int32_t> nprobe, lists;
  int64_t chunk;

  int32_t init(int32_t d_, int32_t nlist_, int64_t chunk_) {
    d = d_; nlist = nlist_; dpad = (d + 31) / 32 * 32; chunk = chunk_;
    BTRY(cent.alloc((size_t)nlist * d));
    BTRY(cb16.alloc((size_t)nlist * dpad));
    BTRY(cn2.alloc(nlist));
    BTRY(cn.alloc(nlist));
    BTRY(dprime.alloc((size_t)chunk * nlist));
    BTRY(pkeys.alloc(chunk));
    BTRY(probe_off.alloc(chunk + 1));
    BTRY(list_off.alloc(nlist + 1));
    BTRY(rank_off.alloc(chunk));
    BTRY(nsc.alloc(chunk));
    BTRY(nprobe.alloc(chunk));
    BTRY(lists.alloc(chunk));
    std::vector<int64_t> po(chunk + 1);
    for (int64_t i = 0; i <= chunk; ++i) po[i] = i;
    std::vector<int32_t> ones(chunk, 1);
    std::vector<int64_t> lo(nlist + 1, 0);
    BTRY(hipMemcpy(probe_off.p, po.data(), 8 * (chunk + 1), hipMemcpyHostToDevice));
    BTRY(hipMemcpy(nprobe.p, ones.data(), 4 * chunk, hipMemcpyHostToDevice));
    BTRY(hipMemcpy(list_off.p, lo.data(), 8 * (nlist + 1), hipMemcpyHostToDevice));
    return BBC_OK;
  }

  int32_t set_centroids(const std::vector<float>& c) {
    std::vector<uint16_t> b16((size_t)nlist * dpad, 0);
    std::vector<float> n2(nlist), n1(nlist);
    for (int32_t j = 0; j < nlist; ++j) {
      float s = 0.0f;
      for (int32_t e = 0; e < d; ++e) {
        float v = c[(size_t)j * d + e];
        b16[(size_t)j * dpad + e] = to_bf16(v);
        s = s + v * v;
      }
      n2[j] = s;
      n1[j] = std::sqrt(s);
    }
    BTRY(hipMemcpy(cent.p, c.data(), 4 * c.size(), hipMemcpyHostToDevice));
    BTRY(hipMemcpy(cb16.p, b16.data(), 2 * b16.size(), hipMemcpyHostToDevice));
    BTRY(hipMemcpy(cn2.p, n2.data(), 4 * nlist, hipMemcpyHostToDevice));
    BTRY(hipMemcpy(cn.p, n1.data(), 4 * nlist, hipMemcpyHostToDevice));
    return BBC_OK;
  }

  // rows [0, nrows) of dx -> out (host)
  int32_t assign(const float* dx, int64_t nrows, int32_t* out) {
    for (int64_t r0 = 0; r0 < nrows; r0 += chunk) {
      int64_t nr = std::min(chunk, nrows - r0);
      bbc::ProbeArgs a{};
      a.q = dx + r0 * d; a.nq = nr; a.d = d; a.cent = cent.p; a.cent_bf16 = cb16.p; a.dpad = dpad;
      a.cent_norm2 = cn2.p; a.cent_norm = cn.p; a.nlist = nlist; a.metric = 0;
      a.nprobe = nprobe.p; a.probe_off = probe_off.p; a.list_off = list_off.p;
      a.dprime = dprime.p; a.probe_lists = lists.p; a.probe_keys = pkeys.p; a.rank_off = rank_off.p;
      a.n_scanned = nsc.p; a.n_recheck = nullptr; a.kc_target = nullptr; a.nsample_q = nullptr;
      BTRY(bbc::launch_probe(a, 0));
      BTRY(hipMemcpy(out + r0, lists.p, 4 * nr, hipMemcpyDeviceToHost));
    }
    return BBC_OK;
  }
};

// float64 member sums in ascending row order, then the empty-cluster split.
void kmeans_update(const float* x, const int64_t* rows, int64_t n, int32_t d, const int32_t* a, int32_t nc,
                   std::vector<float>& c) {
  std::vector<double> sum((size_t)nc * d, 0.0);
  std::vector<int64_t> cnt(nc, 0);
  for (int64_t i = 0; i < n; ++i) {
    const float* xi = x + rows[i] * d;
    double* s = sum.data() + (size_t)a[i] * d;
    for (int32_t e = 0; e < d; ++e) s[e] = s[e] + (double)xi[e];
    cnt[a[i]] += 1;
  }
  for (int32_t j = 0; j < nc; ++j) {
    if (!cnt[j]) continue;
    for (int32_t e = 0; e < d; ++e) c[(size_t)j * d + e] = (float)(sum[(size_t)j * d + e] / (double)cnt[j]);
  }
  const float up = 1.0f + 1.0f / 1024.0f, down = 1.0f - 1.0f / 1024.0f;
  for (int32_t e = 0; e < nc; ++e) {
    if (cnt[e]) continue;
    int32_t big = (int32_t)(std::max_element(cnt.begin(), cnt.end()) - cnt.begin());  // first maximum
    if (cnt[big] < 2) break;
    float* ce = c.data() + (size_t)e * d;
    float* cb = c.data() + (size_t)big * d;
    for (int32_t i = 0; i < d; ++i) {
      float v = cb[i];
      if (i % 2 == 0) { ce[i] = v * up; cb[i] = v * down; }
      else { ce[i] = v * down; cb[i] = v * up; }
    }
    cnt[e] = cnt[big] / 2;
    cnt[big] -= cnt[e];
  }
}

// IVF lists: k-means on the training rows, every row assigned to its nearest
// centroid, lists in ascending row order.  dx: the base rows on the device.
int32_t build_ivf_lists(const float* base, const float* dx, int64_t n, int32_t d, const bbc_build_params* p,
                        std::vector<float>& cent, std::vector<int32_t>& a_all, std::vector<int64_t>& list_off,
                        std::vector<int64_t>& list_ids) {
  const int32_t nlist = p->nlist, iters = p->kmeans_iters;
  const int64_t ntr = p->n_train;
  Assigner as;
  int32_t rc = as.init(d, nlist, std::min<int64_t>(std::max<int64_t>(ntr, 1), 65536));
  if (rc) return rc;
  cent.assign((size_t)nlist * d, 0.0f);
  for (int32_t j = 0; j < nlist; ++j)
    std::memcpy(cent.data() + (size_t)j * d, base + p->train_rows[p->init_pos[j]] * d, sizeof(float) * d);
  DevBuf<float> dtrain;
  DevBuf<int64_t> drows;
  BTRY(dtrain.alloc((size_t)ntr * d));
  BTRY(drows.alloc(ntr));
  BTRY(hipMemcpy(drows.p, p->train_rows, 8 * ntr, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(bbc::gather_rows_kernel, dim3(1024), dim3(256), 0, 0, dx, drows.p, ntr, d, dtrain.p);
  BTRY(hipGetLastError());
  std::vector<int32_t> a_tr(ntr);
  for (int32_t it = 0; it < iters; ++it) {
    if ((rc = as.set_centroids(cent))) return rc;
    if ((rc = as.assign(dtrain.p, ntr, a_tr.data()))) return rc;
    kmeans_update(base, p->train_rows, ntr, d, a_tr.data(), nlist, cent);
  }
  if ((rc = as.set_centroids(cent))) return rc;
  a_all.assign(n, 0);
  if ((rc = as.assign(dx, n, a_all.data()))) return rc;
  list_off.assign(nlist + 1, 0);
  list_ids.assign(n, 0);
  for (int64_t i = 0; i < n; ++i) list_off[a_all[i] + 1] += 1;
  for (int32_t j = 0; j < nlist; ++j) list_off[j + 1] += list_off[j];
  std::vector<int64_t> fill(list_off.begin(), list_off.end() - 1);
  for (int64_t i = 0; i < n; ++i) list_ids[fill[a_all[i]]++] = i;  // ascending rows within a list
  return BBC_OK;
}

}  // namespace

int32_t bbc::build_index_pq(int32_t device, const float* base, int64_t n, int32_t d,
                            const bbc_build_params* p, bbc_index** out) {
  if (!out || !base || !p) return bfail(BBC_EINVAL, "NULL argument");
  *out = nullptr;
  const int32_t nlist = p->nlist, M = p->pq_m, bits = p->pq_bits, iters = p->kmeans_iters;
  if (n < 1 || n >= (int64_t)1 << 31) return bfail(BBC_EINVAL, "n must be in [1, 2^31)");
  if (d < 4 || d > 1024 || d % 4) return bfail(BBC_EINVAL, "d must be a multiple of 4 in [4, 1024]");
  if (nlist < 1 || nlist > 8192) return bfail(BBC_EINVAL, "nlist must be in [1, 8192]");
  if (bits != 4 && bits != 8) return bfail(BBC_EINVAL, "pq_bits must be 4 or 8");
  if (M < 1 || d % M || d / M > 16) return bfail(BBC_EINVAL, "pq_m must divide d with d/pq_m <= 16");
  if (iters < 0) return bfail(BBC_EINVAL, "kmeans_iters < 0");
  if (!p->train_rows || p->n_train < nlist || !p->init_pos) return bfail(BBC_EINVAL, "bad k-means training draws");
  const int32_t ksub = 1 << bits;
  if (!p->pq_rows || p->n_pq < ksub || !p->pq_init) return bfail(BBC_EINVAL, "bad PQ training draws");
  for (int64_t i = 0; i < p->n_train; ++i)
    if (p->train_rows[i] < 0 || p->train_rows[i] >= n || (i && p->train_rows[i] <= p->train_rows[i - 1]))
      return bfail(BBC_EINVAL, "train_rows must be ascending rows of base");
  for (int64_t i = 0; i < p->n_pq; ++i)
    if (p->pq_rows[i] < 0 || p->pq_rows[i] >= n || (i && p->pq_rows[i] <= p->pq_rows[i - 1]))
      return bfail(BBC_EINVAL, "pq_rows must be ascending rows of base");
  for (int32_t j = 0; j < nlist; ++j)
    if (p->init_pos[j] < 0 || p->init_pos[j] >= p->n_train) return bfail(BBC_EINVAL, "init_pos out of range");
  for (int64_t j = 0; j < (int64_t)M * ksub; ++j)
    if (p->pq_init[j] < 0 || p->pq_init[j] >= p->n_pq) return bfail(BBC_EINVAL, "pq_init out of range");
  for (int64_t i = 0; i < n * d; ++i)
    if (!std::isfinite(base[i])) return bfail(BBC_EINVAL, "non-finite value in base");
  {
    int cnt = 0;
    BTRY(hipGetDeviceCount(&cnt));
    if (device < 0 || device >= cnt) return bfail(BBC_EINVAL, "device index out of range");
    BTRY(hipSetDevice(device));
  }

  DevBuf<float> dx;
  BTRY(dx.alloc((size_t)n * d));
  BTRY(hipMemcpy(dx.p, base, sizeof(float) * n * d, hipMemcpyHostToDevice));
  std::vector<float> cent;
  std::vector<int32_t> a_all;
  std::vector<int64_t> list_off, list_ids;
  int32_t rc = build_ivf_lists(base, dx.p, n, d, p, cent, a_all, list_off, list_ids);
  if (rc) return rc;
  // ---- PQ training on residuals of the PQ rows -------------------------------
  const int32_t dsub = d / M;
  DevBuf<float> dcent, dcb;
  DevBuf<int32_t> dassign;
  DevBuf<int64_t> dpq, dall;
  DevBuf<uint8_t> dcodes;
  BTRY(dcent.alloc((size_t)nlist * d));
  BTRY(dcb.alloc((size_t)M * ksub * dsub));
  BTRY(dassign.alloc(n));
  BTRY(dpq.alloc(p->n_pq));
  BTRY(hipMemcpy(dcent.p, cent.data(), 4 * cent.size(), hipMemcpyHostToDevice));
  BTRY(hipMemcpy(dassign.p, a_all.data(), 4 * n, hipMemcpyHostToDevice));
  BTRY(hipMemcpy(dpq.p, p->pq_rows, 8 * p->n_pq, hipMemcpyHostToDevice));
  const int64_t npq = p->n_pq;
  std::vector<float> resid((size_t)npq * d);
  for (int64_t i = 0; i < npq; ++i) {
    const float* xi = base + p->pq_rows[i] * d;
    const float* ci = cent.data() + (size_t)a_all[p->pq_rows[i]] * d;
    for (int32_t e = 0; e < d; ++e) resid[(size_t)i * d + e] = xi[e] - ci[e];
  }
  std::vector<float> cb((size_t)M * ksub * dsub);
  for (int32_t m = 0; m < M; ++m)
    for (int32_t b = 0; b < ksub; ++b)
      std::memcpy(cb.data() + ((size_t)m * ksub + b) * dsub,
                  resid.data() + (size_t)p->pq_init[(size_t)m * ksub + b] * d + (size_t)m * dsub, 4 * dsub);
  size_t lds = sizeof(float) * ksub * dsub;
  BTRY(dcodes.alloc((size_t)std::max<int64_t>(npq, n) * M));
  std::vector<uint8_t> cpq((size_t)npq * M);
  for (int32_t it = 0; it < iters; ++it) {
    BTRY(hipMemcpy(dcb.p, cb.data(), 4 * cb.size(), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(bbc::pq_assign_kernel, dim3((unsigned)std::min<int64_t>((npq + 255) / 256, 4096), M),
                       dim3(256), lds, 0, dx.p, dpq.p, npq, dassign.p, dcent.p, dcb.p, d, M, ksub, dcodes.p);
    BTRY(hipGetLastError());
    BTRY(hipMemcpy(cpq.data(), dcodes.p, cpq.size(), hipMemcpyDeviceToHost));
    std::vector<double> sum((size_t)M * ksub * dsub, 0.0);
    std::vector<int64_t> cnt((size_t)M * ksub, 0);
    for (int64_t i = 0; i < npq; ++i)
      for (int32_t m = 0; m < M; ++m) {
        size_t b = (size_t)m * ksub + cpq[(size_t)i * M + m];
        for (int32_t e = 0; e < dsub; ++e) sum[b * dsub + e] = sum[b * dsub + e] + (double)resid[(size_t)i * d + m * dsub + e];
        cnt[b] += 1;
      }
    for (size_t b = 0; b < (size_t)M * ksub; ++b) {
      if (!cnt[b]) continue;
      for (int32_t e = 0; e < dsub; ++e) cb[b * dsub + e] = (float)(sum[b * dsub + e] / (double)cnt[b]);
    }
  }
  // ---- codes of every row in list order --------------------------------------
  BTRY(hipMemcpy(dcb.p, cb.data(), 4 * cb.size(), hipMemcpyHostToDevice));
  BTRY(dall.alloc(n));
  BTRY(hipMemcpy(dall.p, list_ids.data(), 8 * n, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(bbc::pq_assign_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192), M), dim3(256),
                     lds, 0, dx.p, dall.p, n, dassign.p, dcent.p, dcb.p, d, M, ksub, dcodes.p);
  BTRY(hipGetLastError());
  std::vector<uint8_t> codes((size_t)n * M);
  BTRY(hipMemcpy(codes.data(), dcodes.p, codes.size(), hipMemcpyDeviceToHost));
  rc = bbc_index_create_pq(device, n, d, nlist, BBC_METRIC_L2, cent.data(), list_off.data(), list_ids.data(), M,
                           bits, cb.data(), codes.data(), base, out);
  if (rc) return rc;
  return BBC_OK;
}

// IVF lists, then the RaBitQ codes of every row in list order, encoded on the
// device in chunks of rows (residual, rotation, code bits and factors).
int32_t bbc::build_index_rabitq(int32_t device, const void* base_v, int64_t n, int32_t d,
                                const bbc_build_params* p, bbc_index** out) {
  if (!out || !base_v || !p) return bfail(BBC_EINVAL, "NULL argument");
  *out = nullptr;
  const int32_t nlist = p->nlist;
  if (n < 1 || n >= (int64_t)1 << 31) return bfail(BBC_EINVAL, "n must be in [1, 2^31)");
  if (d < 64 || d > 1024 || d % 64) return bfail(BBC_EINVAL, "RaBitQ needs d a multiple of 64 in [64, 1024]");
  if (nlist < 1 || nlist > 8192) return bfail(BBC_EINVAL, "nlist must be in [1, 8192]");
  if (p->kmeans_iters < 0) return bfail(BBC_EINVAL, "kmeans_iters < 0");
  if (p->metric != BBC_METRIC_L2 && p->metric != BBC_METRIC_IP) return bfail(BBC_EINVAL, "unknown metric");
  if (p->storage != BBC_STORAGE_FP32 && p->storage != BBC_STORAGE_FP16) return bfail(BBC_EINVAL, "unknown storage");
  if (!p->rotation) return bfail(BBC_EINVAL, "RaBitQ needs a rotation");
  if (!p->train_rows || p->n_train < nlist || !p->init_pos) return bfail(BBC_EINVAL, "bad k-means training draws");
  for (int64_t i = 0; i < p->n_train; ++i)
    if (p->train_rows[i] < 0 || p->train_rows[i] >= n || (i && p->train_rows[i] <= p->train_rows[i - 1]))
      return bfail(BBC_EINVAL, "train_rows must be ascending rows of base");
  for (int32_t j = 0; j < nlist; ++j)
    if (p->init_pos[j] < 0 || p->init_pos[j] >= p->n_train) return bfail(BBC_EINVAL, "init_pos out of range");
  // float32 rows for the build (float16 converts exactly)
  std::vector<float> base32;
  const float* base = static_cast<const float*>(base_v);
  if (p->storage == BBC_STORAGE_FP16) {
    base32.resize((size_t)n * d);
    const __half* h = static_cast<const __half*>(base_v);
    for (int64_t i = 0; i < n * d; ++i) base32[i] = __half2float(h[i]);
    base = base32.data();
  }
  for (int64_t i = 0; i < n * d; ++i)
    if (!std::isfinite(base[i])) return bfail(BBC_EINVAL, "non-finite value in base");
  {
    int cnt = 0;
    BTRY(hipGetDeviceCount(&cnt));
    if (device < 0 || device >= cnt) return bfail(BBC_EINVAL, "device index out of range");
    BTRY(hipSetDevice(device));
  }
  DevBuf<float> dx;
  BTRY(dx.alloc((size_t)n * d));
  BTRY(hipMemcpy(dx.p, base, sizeof(float) * n * d, hipMemcpyHostToDevice));
  std::vector<float> cent;
  std::vector<int32_t> a_all;
  std::vector<int64_t> list_off, list_ids;
  int32_t rc = build_ivf_lists(base, dx.p, n, d, p, cent, a_all, list_off, list_ids);
  if (rc) return rc;
  const int32_t cw = (int32_t)(((d / 32) + 3) / 4 * 4);
  DevBuf<float> dcent, dP, dfac, dres, drot;
  DevBuf<int64_t> dids, doff;
  DevBuf<uint32_t> dcodes;
  BTRY(dcent.alloc((size_t)nlist * d));
  BTRY(dP.alloc((size_t)d * d));
  BTRY(dids.alloc(n));
  BTRY(doff.alloc(nlist + 1));
  BTRY(dcodes.alloc((size_t)n * cw));
  BTRY(dfac.alloc((size_t)n * 4));
  BTRY(hipMemcpy(dcent.p, cent.data(), 4 * cent.size(), hipMemcpyHostToDevice));
  BTRY(hipMemcpy(dP.p, p->rotation, sizeof(float) * d * d, hipMemcpyHostToDevice));
  BTRY(hipMemcpy(dids.p, list_ids.data(), 8 * n, hipMemcpyHostToDevice));
  BTRY(hipMemcpy(doff.p, list_off.data(), 8 * (nlist + 1), hipMemcpyHostToDevice));
  const int64_t chunk = std::min<int64_t>(n, 1 << 18);
  BTRY(dres.alloc((size_t)chunk * d));
  BTRY(drot.alloc((size_t)chunk * d));
  bbc::RabitqBuildArgs ba{};
  ba.x = dx.p; ba.list_ids = dids.p; ba.list_off = doff.p; ba.nlist = nlist; ba.cent = dcent.p; ba.P = dP.p;
  ba.D = d; ba.codes = dcodes.p; ba.code_words = cw; ba.factors = dfac.p;
  for (int64_t p0 = 0; p0 < n; p0 += chunk)
    BTRY(bbc::launch_rabitq_encode(ba, p0, std::min(chunk, n - p0), dres.p, drot.p, 0));
  BTRY(hipDeviceSynchronize());
  std::vector<uint32_t> codes_s((size_t)n * cw), codes((size_t)n * (d / 32));
  std::vector<float> fac((size_t)n * 4);
  BTRY(hipMemcpy(codes_s.data(), dcodes.p, 4 * codes_s.size(), hipMemcpyDeviceToHost));
  BTRY(hipMemcpy(fac.data(), dfac.p, 4 * fac.size(), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i)
    std::memcpy(codes.data() + (size_t)i * (d / 32), codes_s.data() + (size_t)i * cw, 4 * (d / 32));
  return bbc_index_create_rabitq(device, n, d, nlist, p->metric, cent.data(), list_off.data(), list_ids.data(),
                                 p->rotation, codes.data(), fac.data(), base_v, p->storage, p->rabitq_eps0, out);
}

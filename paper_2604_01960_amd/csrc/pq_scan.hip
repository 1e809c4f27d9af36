// PQ estimated distances (background section: quantization methods
// precompute query-to-codeword distances and sum them per code; IVF+PQ uses
// residual codes, one table per (query, probed list)).
//
// One block per (query, probe rank).  The block builds the residual table
// LUT[m][b] = sum_e ((q_e - c_e) - C_m[b][e])^2 in LDS (r = q - c once per
// element, then sequentially over the sub-vector elements, unfused), and
// then every thread walks its objects' codes and sums LUT[m][code_m] for
// m = 0..M-1 in order, starting from +0.  Keys go to the per-query key
// scratch in probe order, so the keys of the nearest lists come first.
#include "common.h"
#include "kernels.h"

namespace bbc {

__device__ __forceinline__ int64_t find_query(const int64_t* __restrict__ off, int64_t nq, int64_t p) {
  // largest qi with off[qi] <= p (off is non-decreasing, off[0] = 0)
  int64_t lo = 0, hi = nq - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int BITS>
__global__ __launch_bounds__(256) void pq_scan_kernel(PqScanArgs a) {
  constexpr int NT = 256;
  constexpr int KSUB = 1 << BITS;
  extern __shared__ __align__(16) unsigned char smem[];
  float* lut = reinterpret_cast<float*>(smem);              // [M][KSUB]
  float* res = lut + a.M * KSUB;                            // [d]

  const int64_t p = blockIdx.x;
  const int64_t qi = find_query(a.probe_off, a.nq, p);
  const int rank = (int)(p - a.probe_off[qi]);
  if (rank < a.rank_begin || rank >= a.rank_end) return;
  const int j = a.probe_lists[p];
  const float* qv = a.q + qi * a.d;
  const float* cv = a.cent + (int64_t)j * a.d;
  for (int i = threadIdx.x; i < a.d; i += NT) res[i] = qv[i] - cv[i];
  __syncthreads();
  const int dsub = a.d / a.M;
  const int nent = a.M * KSUB;
  for (int e = threadIdx.x; e < nent; e += NT) {
    const int m = e / KSUB;
    const float* cw = a.codebook + (int64_t)e * dsub;
    const float* rr = res + m * dsub;
    float acc = 0.0f;
    for (int t = 0; t < dsub; ++t) {
      float u = rr[t] - cw[t];
      u = u * u;
      acc = acc + u;
    }
    lut[e] = acc;
  }
  __syncthreads();
  const int64_t lbeg = a.list_off[j];
  const int64_t nobj = a.list_off[j + 1] - lbeg;
  float* out = a.keys + a.key_off[qi] + a.rank_off[p];
  const int stride = a.code_stride;  // bytes per code row, multiple of 16
  const uint8_t* codes = a.codes + lbeg * stride;
  for (int64_t i = threadIdx.x; i < nobj; i += NT) {
    const uint4* row = reinterpret_cast<const uint4*>(codes + i * stride);
    float key = 0.0f;
    int m = 0;
    for (int c = 0; c < stride / 16 && m < a.M; ++c) {
      uint4 v = row[c];
      uint32_t wds[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int wi = 0; wi < 4; ++wi) {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) {
          uint32_t byte = (wds[wi] >> (8 * bi)) & 0xffu;
          if (BITS == 8) {
            if (m < a.M) { key = key + lut[m * KSUB + byte]; ++m; }
          } else {
            if (m < a.M) { key = key + lut[m * KSUB + (byte & 15u)]; ++m; }
            if (m < a.M) { key = key + lut[m * KSUB + (byte >> 4)]; ++m; }
          }
        }
      }
    }
    out[i] = key;
  }
}

hipError_t launch_pq_scan(const PqScanArgs& a, int64_t npairs, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  size_t lds = sizeof(float) * ((size_t)a.M * (1 << a.bits) + a.d);
  if (a.bits == 8)
    hipLaunchKernelGGL(pq_scan_kernel<8>, dim3((unsigned)npairs), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL(pq_scan_kernel<4>, dim3((unsigned)npairs), dim3(256), lds, s, a);
  return hipGetLastError();
}

}  // namespace bbc

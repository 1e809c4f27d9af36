// Exact re-rank of the collected candidates (the unbounded-method search of
// the background section: the n_cand candidates found by estimated distance
// are re-ranked by exact distance; the exact distance is the canonical FP32
// squared L2, or the negated canonical inner product as the ordering key).
//
// Rows of at most 32 four-element chunks (d <= 128) are handled by half a
// wave each, two rows per wave; longer rows by a full wave, lane l taking
// chunks l, l+64, ...  Each lane keeps its query chunks in registers for the
// whole block; four rows are in flight per row group so that the gathers of
// whole contiguous rows (d*4 bytes each) overlap.
#include <hip/hip_fp16.h>
#include "common.h"
#include "kernels.h"

namespace bbc {

template <typename T> __device__ __forceinline__ float4 load4(const T* p, int64_t chunk);
template <> __device__ __forceinline__ float4 load4<float>(const float* p, int64_t chunk) {
  return reinterpret_cast<const float4*>(p)[chunk];
}
template <> __device__ __forceinline__ float4 load4<__half>(const __half* p, int64_t chunk) {
  const uint2 v = reinterpret_cast<const uint2*>(p)[chunk];
  __half2 h0 = __builtin_bit_cast(__half2, v.x);
  __half2 h1 = __builtin_bit_cast(__half2, v.y);
  float2 f0 = __half22float2(h0);
  float2 f1 = __half22float2(h1);
  return make_float4(f0.x, f0.y, f1.x, f1.y);
}

constexpr int RR_ROWS_PER_BLOCK = 256;
constexpr int RR_UNROLL = 4;

// Half-wave rows (nchunk <= 32).
template <typename T>
__global__ __launch_bounds__(256) void rerank_half_kernel(RerankArgs a) {
  const int64_t qi = a.qorder ? a.qorder[blockIdx.y] : blockIdx.y;
  const int64_t kc = a.n_cand[qi];
  const int64_t row0 = (int64_t)blockIdx.x * RR_ROWS_PER_BLOCK;
  if (row0 >= kc) return;
  const int lane = threadIdx.x & 63;
  const int hl = lane & 31;
  const int wv = threadIdx.x >> 6;   // 4 waves per block
  const int half = lane >> 5;
  const int nchunk = a.d >> 2;
  const bool ip = a.metric != 0;
  float4 qc = make_float4(0.f, 0.f, 0.f, 0.f);
  if (hl < nchunk) qc = reinterpret_cast<const float4*>(a.q + qi * a.d)[hl];
  const uint32_t* cpos = a.cand_pos + a.cand_off[qi];
  uint64_t* outp = a.cand_packed + a.cand_off[qi];
  const T* vec = reinterpret_cast<const T*>(a.vectors);
  const int64_t row_end = min(kc, row0 + RR_ROWS_PER_BLOCK);
  // the loop bound is uniform across the wave; each half takes RR_UNROLL rows
  for (int64_t wbase = row0 + wv * 2 * RR_UNROLL; wbase < row_end; wbase += 4 * 2 * RR_UNROLL) {
    const int64_t base = wbase + half * RR_UNROLL;
    float4 xv[RR_UNROLL];
    uint32_t pos[RR_UNROLL];
#pragma unroll
    for (int u = 0; u < RR_UNROLL; ++u) {
      int64_t r = base + u;
      pos[u] = r < row_end ? cpos[r] : 0u;
      xv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < row_end && hl < nchunk) xv[u] = load4<T>(vec + (int64_t)pos[u] * a.d, hl);
    }
#pragma unroll
    for (int u = 0; u < RR_UNROLL; ++u) {
      float acc = ip ? chunk_ip(qc, xv[u], 0.0f) : chunk_l2(qc, xv[u], 0.0f);
      acc = canon_reduce32(acc);
      int64_t r = base + u;
      if (hl == 0 && r < row_end) {
        float key = ip ? -acc : acc;
        outp[r] = pack_key_id(key, (uint32_t)a.list_ids[pos[u]]);
      }
    }
  }
}

// Full-wave rows (nchunk > 32), at most 4 steps (d <= 1024).
template <typename T>
__global__ __launch_bounds__(256) void rerank_full_kernel(RerankArgs a) {
  const int64_t qi = a.qorder ? a.qorder[blockIdx.y] : blockIdx.y;
  const int64_t kc = a.n_cand[qi];
  const int64_t row0 = (int64_t)blockIdx.x * RR_ROWS_PER_BLOCK;
  if (row0 >= kc) return;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;  // 4 waves per block
  const int nchunk = a.d >> 2;
  const bool ip = a.metric != 0;
  float4 qc[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    int c = lane + 64 * st;
    qc[st] = c < nchunk ? reinterpret_cast<const float4*>(a.q + qi * a.d)[c] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const uint32_t* cpos = a.cand_pos + a.cand_off[qi];
  uint64_t* outp = a.cand_packed + a.cand_off[qi];
  const T* vec = reinterpret_cast<const T*>(a.vectors);
  const int64_t row_end = min(kc, row0 + RR_ROWS_PER_BLOCK);
  for (int64_t base = row0 + wv * 2; base < row_end; base += 4 * 2) {
    float4 xv[2][4];
    uint32_t pos[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int64_t r = base + u;
      pos[u] = r < row_end ? cpos[r] : 0u;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        int c = lane + 64 * st;
        xv[u][st] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < row_end && c < nchunk) xv[u][st] = load4<T>(vec + (int64_t)pos[u] * a.d, c);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      float acc = 0.0f;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        int c = lane + 64 * st;
        if (c < nchunk) acc = ip ? chunk_ip(qc[st], xv[u][st], acc) : chunk_l2(qc[st], xv[u][st], acc);
      }
      acc = canon_reduce64(acc);
      int64_t r = base + u;
      if (lane == 0 && r < row_end) {
        float key = ip ? -acc : acc;
        outp[r] = pack_key_id(key, (uint32_t)a.list_ids[pos[u]]);
      }
    }
  }
}

// Queries ordered by their nearest probed list (a counting sort in one
// block): queries that share it tend to share candidates, and re-ranking them
// together lets the caches serve the rows they have in common.
__global__ __launch_bounds__(1024) void query_order_kernel(const int32_t* __restrict__ probe_lists,
                                                           const int64_t* __restrict__ probe_off,
                                                           const int32_t* __restrict__ nprobe, int64_t nq,
                                                           int nlist, int32_t* __restrict__ order) {
  extern __shared__ uint32_t cnt[];  // [nlist + 1]
  const int NT = 1024;
  auto top = [&](int64_t q) { return nprobe[q] > 0 ? probe_lists[probe_off[q]] : nlist; };
  for (int i = threadIdx.x; i <= nlist; i += NT) cnt[i] = 0;
  __syncthreads();
  for (int64_t q = threadIdx.x; q < nq; q += NT) atomicAdd(&cnt[top(q)], 1u);
  __syncthreads();
  if (threadIdx.x < 64) {
    uint32_t carry = 0;
    for (int base = 0; base <= nlist; base += 64) {
      const int i = base + (int)threadIdx.x;
      const uint32_t v = i <= nlist ? cnt[i] : 0u;
      const uint32_t incl = wave_incl_scan(v);
      if (i <= nlist) cnt[i] = carry + incl - v;
      carry += __shfl(incl, 63);
    }
  }
  __syncthreads();
  for (int64_t q = threadIdx.x; q < nq; q += NT) order[atomicAdd(&cnt[top(q)], 1u)] = (int32_t)q;
}

hipError_t launch_query_order(const int32_t* probe_lists, const int64_t* probe_off, const int32_t* nprobe,
                              int64_t nq, int nlist, int32_t* order, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  if (nlist > QUERY_ORDER_MAX_LISTS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(query_order_kernel, dim3(1), dim3(1024), sizeof(uint32_t) * (nlist + 1), s, probe_lists,
                     probe_off, nprobe, nq, nlist, order);
  return hipGetLastError();
}

hipError_t launch_rerank(const RerankArgs& a, int64_t max_kc, hipStream_t s) {
  if (a.nq <= 0 || max_kc <= 0) return hipSuccess;
  dim3 grid((unsigned)((max_kc + RR_ROWS_PER_BLOCK - 1) / RR_ROWS_PER_BLOCK), (unsigned)a.nq);
  const int nchunk = a.d / 4;
  if (nchunk <= 32) {
    if (a.fp16) hipLaunchKernelGGL(rerank_half_kernel<__half>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(rerank_half_kernel<float>, grid, dim3(256), 0, s, a);
  } else {
    if (a.fp16) hipLaunchKernelGGL(rerank_full_kernel<__half>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(rerank_full_kernel<float>, grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace bbc

// Final top-k of the re-ranked candidates, sorted ascending by (exact key, id)
// (the last step of the unbounded search in the background section: the
// re-ranked candidates yield the k results).
//
// One block of 1024 threads per query:
//  1. threshold: the (cnt-1)-th smallest packed (key, id), cnt = min(k, K_c),
//     by an exact 64-bit radix select over the K_c re-ranked candidates;
//  2. compaction of the cnt winners into the query's output slots;
//  3. sort: runs of `run` items sorted in LDS (bitonic), then pairwise
//     merge-path merges between the output slots and the candidate buffer;
//  4. unpacking into (int64 id, float distance) in place, and padding of the
//     slots past cnt with id -1 and +inf (-inf for inner product).
#include "common.h"
#include "kernels.h"

namespace bbc {

// Merge sorted a[0..na) and b[0..nb) into c (distinct values), by a block.
template <int NT>
__device__ void block_merge(const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb, uint64_t* c) {
  const int64_t L = na + nb;
  const int64_t per = (L + NT - 1) / NT;
  const int64_t k0 = min(L, (int64_t)threadIdx.x * per);
  const int64_t k1 = min(L, k0 + per);
  if (k0 >= k1) return;
  int64_t lo = max((int64_t)0, k0 - nb), hi = min(k0, na);
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < b[k0 - mid - 1]) lo = mid + 1; else hi = mid;
  }
  int64_t i = lo, j = k0 - lo;
  for (int64_t k = k0; k < k1; ++k) {
    bool take_a = (j >= nb) || (i < na && a[i] < b[j]);
    c[k] = take_a ? a[i++] : b[j++];
  }
}

__global__ __launch_bounds__(1024) void final_topk_kernel(FinalArgs a) {
  constexpr int NT = 1024;
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* run_buf = reinterpret_cast<uint64_t*>(smem);  // [a.run]
  __shared__ uint32_t hist[256];
  __shared__ uint32_t bc[4];

  const int64_t qi = blockIdx.x;
  const int64_t kc = a.n_cand[qi];
  const int64_t k = a.k[qi];
  const int64_t cnt = kc < k ? kc : k;
  uint64_t* in = a.cand_packed + a.cand_off[qi];
  int64_t* oid = a.out_ids + a.out_off[qi];
  float* odist = a.out_dists + a.out_off[qi];
  uint64_t* outp = reinterpret_cast<uint64_t*>(oid);

  if (cnt > 0) {
    uint64_t thr = ~0ull;
    if (cnt < kc) {
      thr = block_radix_select64<NT>([&](int64_t i, uint64_t& v) { v = in[i]; return true; }, kc, cnt - 1,
                                     hist, bc);
    }
    if (threadIdx.x == 0) bc[2] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < kc; i += NT) {
      uint64_t v = in[i];
      if (v <= thr) {
        uint32_t slot = atomicAdd(&bc[2], 1u);
        outp[slot] = v;
      }
    }
    __syncthreads();
    // sorted runs
    const int run = a.run;
    for (int64_t r0 = 0; r0 < cnt; r0 += run) {
      const int n = (int)min((int64_t)run, cnt - r0);
      const int P = next_pow2(n);
      for (int i = threadIdx.x; i < P; i += NT) run_buf[i] = i < n ? outp[r0 + i] : ~0ull;
      lds_bitonic_sort<NT>(run_buf, P);
      for (int i = threadIdx.x; i < n; i += NT) outp[r0 + i] = run_buf[i];
      __syncthreads();
    }
    // merges: ping-pong between outp and the candidate buffer (kc >= cnt slots)
    uint64_t* src = outp;
    uint64_t* dst = in;
    for (int64_t width = run; width < cnt; width <<= 1) {
      for (int64_t lo = 0; lo < cnt; lo += 2 * width) {
        const int64_t na = min(width, cnt - lo);
        const int64_t nb = max((int64_t)0, min(width, cnt - lo - width));
        block_merge<NT>(src + lo, na, src + lo + na, nb, dst + lo);
      }
      __syncthreads();
      uint64_t* t = src; src = dst; dst = t;
    }
    if (src != outp) {
      for (int64_t i = threadIdx.x; i < cnt; i += NT) outp[i] = src[i];
      __syncthreads();
    }
    for (int64_t i = threadIdx.x; i < cnt; i += NT) {
      uint64_t v = outp[i];
      float key = packed_key(v);
      oid[i] = (int64_t)packed_id(v);
      odist[i] = a.metric == 0 ? key : -key;
    }
  }
  const float pad = a.metric == 0 ? __builtin_inff() : -__builtin_inff();
  for (int64_t i = cnt + threadIdx.x; i < k; i += NT) {
    oid[i] = -1;
    odist[i] = pad;
  }
  if (threadIdx.x == 0) a.out_counts[qi] = (int32_t)cnt;
}

hipError_t launch_final_topk(const FinalArgs& a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  size_t lds = sizeof(uint64_t) * (size_t)a.run;
  hipLaunchKernelGGL(final_topk_kernel, dim3((unsigned)a.nq), dim3(1024), lds, s, a);
  return hipGetLastError();
}

}  // namespace bbc

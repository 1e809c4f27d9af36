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

constexpr int FT_NB = 2048;     // bins of the selection histogram
constexpr int FT_BCAP = 1024;   // threshold-bin members held in LDS
constexpr int FT_RANKCAP = 128; // largest bin ordered by rank counting

// Fast path (cnt <= run): bins over the 32-bit key image, monotone in the
// key, so every bin below the threshold bin is wholly inside the result.
//  1. min / max key image; bin = (image - min) >> shift with 2048 bins;
//  2. histogram; threshold bin b* = first bin whose running count reaches
//     cnt, s = cnt - (count below b*);
//  3. items of bins < b* are scattered into LDS grouped by bin, the members
//     of b* are sorted by (key, id) and the first s appended (an exact radix
//     select over b*'s members if they do not fit);
//  4. when every bin below b* holds at most FT_RANKCAP items, each item's
//     output slot is its bin's start plus the number of smaller items in its
//     bin (the bins are contiguous and ordered), and the sorted first s of b*
//     follow; otherwise the cnt winners are sorted in LDS (bitonic).
__device__ void final_topk_binned(const FinalArgs& a, const uint64_t* in, int64_t kc, int64_t cnt, int64_t* oid,
                                  float* odist, uint64_t* obuf) {
  constexpr int NT = 1024;
  __shared__ uint32_t hist[FT_NB];
  __shared__ uint64_t bbuf[FT_BCAP];
  __shared__ uint32_t red[12];
  if (threadIdx.x == 0) { red[0] = 0xffffffffu; red[1] = 0u; red[2] = 0u; }
  for (int i = threadIdx.x; i < FT_NB; i += NT) hist[i] = 0;
  __syncthreads();
  uint32_t mn = 0xffffffffu, mx = 0u;
  for (int64_t i = threadIdx.x; i < kc; i += NT) {
    uint32_t kb = (uint32_t)(in[i] >> 32);
    mn = min(mn, kb);
    mx = max(mx, kb);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    mn = min(mn, __shfl_xor(mn, off));
    mx = max(mx, __shfl_xor(mx, off));
  }
  if ((threadIdx.x & 63) == 0) { atomicMin(&red[0], mn); atomicMax(&red[1], mx); }
  __syncthreads();
  const uint32_t kmin = red[0];
  const uint32_t span = red[1] - kmin;
  int shift = 0;
  while ((span >> shift) >= (uint32_t)FT_NB) ++shift;
  for (int64_t base = 0; base < kc; base += NT) {  // wave-uniform trip count
    const int64_t i = base + threadIdx.x;
    const uint32_t b = i < kc ? ((((uint32_t)(in[i] >> 32)) - kmin) >> shift) : 0u;
    wave_hist_add(hist, b, i < kc);
  }
  __syncthreads();
  // exclusive prefix over the bins (one wave), threshold bin
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    uint32_t carry = 0;
    int bstar = -1;
    uint32_t below = 0, vmax = 0;  // vmax: largest bin below b*
    for (int base = 0; base < FT_NB; base += 64) {
      uint32_t v = hist[base + lane];
      uint32_t incl = v;
      for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      hist[base + lane] = carry + incl - v;
      if (bstar < 0) {
        uint64_t hit = __ballot((int64_t)(carry + incl) >= cnt);
        if (hit) {
          int l = __ffsll((unsigned long long)hit) - 1;
          bstar = base + l;
          below = __shfl(carry + incl - v, l);
          if (lane < l) vmax = max(vmax, v);
        } else {
          vmax = max(vmax, v);
        }
      }
      carry += __shfl(incl, 63);
    }
    for (int off = 32; off >= 1; off >>= 1) vmax = max(vmax, __shfl_xor(vmax, off));
    if (lane == 0) { red[3] = (uint32_t)bstar; red[4] = below; red[8] = vmax; }
  }
  __syncthreads();
  const int bstar = (int)red[3];
  const int64_t nbelow = red[4];
  const int64_t s = cnt - nbelow;
  for (int64_t i = threadIdx.x; i < kc; i += NT) {
    const uint64_t v = in[i];
    const int b = (int)((((uint32_t)(v >> 32)) - kmin) >> shift);
    if (b < bstar) {
      obuf[atomicAdd(&hist[b], 1u)] = v;
    } else if (b == bstar) {
      uint32_t bs = atomicAdd(&red[2], 1u);
      if (bs < (uint32_t)FT_BCAP) bbuf[bs] = v;
    }
  }
  __syncthreads();
  const int64_t nb = red[2];
  if (nb <= FT_BCAP && red[8] <= (uint32_t)FT_RANKCAP) {
    // after the scatter hist[b] is the end of bin b, so bin b (< b*) spans
    // [b ? hist[b-1] : 0, hist[b])
    const float sgn = a.metric == 0 ? 1.f : -1.f;
    const int P = next_pow2((int)nb);
    for (int i = (int)nb + threadIdx.x; i < P; i += NT) bbuf[i] = ~0ull;
    lds_bitonic_sort<NT>(bbuf, P);
    for (int64_t r = threadIdx.x; r < s; r += NT) {
      const uint64_t v = bbuf[r];
      oid[nbelow + r] = (int64_t)packed_id(v);
      odist[nbelow + r] = sgn * packed_key(v);
    }
    for (int64_t p = threadIdx.x; p < nbelow; p += NT) {
      const uint64_t v = obuf[p];
      const int b = (int)((((uint32_t)(v >> 32)) - kmin) >> shift);
      const int beg = b ? (int)hist[b - 1] : 0, end = (int)hist[b];
      int rank = 0;
      for (int j = beg; j < end; ++j) rank += obuf[j] < v;
      oid[beg + rank] = (int64_t)packed_id(v);
      odist[beg + rank] = sgn * packed_key(v);
    }
    return;
  }
  if (nb <= FT_BCAP) {
    const int P = next_pow2((int)nb);
    for (int i = (int)nb + threadIdx.x; i < P; i += NT) bbuf[i] = ~0ull;
    lds_bitonic_sort<NT>(bbuf, P);
    for (int64_t r = threadIdx.x; r < s; r += NT) obuf[nbelow + r] = bbuf[r];
  } else {
    auto get = [&](int64_t i, uint64_t& v) -> bool {
      v = in[i];
      return (int)((((uint32_t)(v >> 32)) - kmin) >> shift) == bstar;
    };
    uint64_t thr = block_radix_select64<NT>(get, kc, s - 1, hist, red + 5);
    if (threadIdx.x == 0) red[2] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < kc; i += NT) {
      uint64_t v;
      if (get(i, v) && v <= thr) obuf[nbelow + atomicAdd(&red[2], 1u)] = v;
    }
  }
  const int P = next_pow2((int)cnt);
  for (int i = (int)cnt + threadIdx.x; i < P; i += NT) obuf[i] = ~0ull;
  lds_bitonic_sort<NT>(obuf, P);
  for (int64_t i = threadIdx.x; i < cnt; i += NT) {
    const uint64_t v = obuf[i];
    const float key = packed_key(v);
    oid[i] = (int64_t)packed_id(v);
    odist[i] = a.metric == 0 ? key : -key;
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

  if (cnt > 0 && cnt <= a.run) {
    final_topk_binned(a, in, kc, cnt, oid, odist, run_buf);
  } else if (cnt > 0) {
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

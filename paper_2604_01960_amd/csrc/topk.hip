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

constexpr int FT_NB = 2048;      // coarse bins of the selection histogram
constexpr int FT_NB2 = 4096;     // bins after refinement (coarse below + 2048 fine)
constexpr int FT_BCAP = 512;     // threshold-bin members held in LDS
constexpr int FT_RANKCAP = 128;  // largest bin ordered by rank counting

// Monotone binning of the 32-bit key image.  Coarse bins are
// c = (image - kmin) >> shift.  After refinement the coarse bins below blo
// stay, coarse bins blo..bhi are split into fine bins
// blo + ((image - lo2) >> shift2), and images in coarse bins above bhi (all
// beyond the threshold) get the bin `out`, past every counted bin.
struct FtBins {
  uint32_t kmin, lo2;
  int shift, shift2, blo, bhi, out;
  __device__ __forceinline__ int operator()(uint32_t img) const {
    const int c = (int)((img - kmin) >> shift);
    if (c < blo) return c;
    if (c > bhi) return out;
    return blo + (int)((img - lo2) >> shift2);
  }
};

// The histogram is stored transposed, bin b at hist[(b % 2^lg) * 64 + b / 2^lg],
// so that lane l of one wave reads its 2^lg consecutive bins without bank
// conflicts when it forms the prefix sums.
__device__ __forceinline__ int ft_slot(int b, int lg) { return (b & ((1 << lg) - 1)) * 64 + (b >> lg); }

// One wave: exclusive prefix sums over the 64 << lg bins, in place; the
// threshold bin b* (the first whose running count reaches cnt) to red[3], the
// count below it to red[4], the largest bin below b* to red[8] and the first
// bin below b* holding more than FT_RANKCAP items (or INT_MAX) to red[9].
__device__ void ft_prefix(uint32_t* hist, int lg, int64_t cnt, uint32_t* red) {
  const int lane = threadIdx.x & 63;
  const int bpl = 1 << lg;
  uint32_t sum = 0;
#pragma unroll 8
  for (int j = 0; j < bpl; ++j) sum += hist[j * 64 + lane];
  asm volatile("" ::: "memory");  // the bins are read again below, not kept in registers
  const uint32_t incl = wave_incl_scan(sum);
  const uint64_t hit = __ballot((int64_t)incl >= cnt);  // the counted items number >= cnt
  const int L = __ffsll((unsigned long long)hit) - 1;
  uint32_t run = incl - sum, vmax = 0, below = 0;
  int bstar = -1, big = 0x7fffffff;
#pragma unroll 4
  for (int j = 0; j < bpl; ++j) {
    const uint32_t h = hist[j * 64 + lane];
    const int b = lane * bpl + j;
    if (lane == L && bstar < 0 && (int64_t)(run + h) >= cnt) {
      bstar = b;
      below = run;
    }
    if (lane < L || (lane == L && bstar < 0)) {
      vmax = max(vmax, h);
      if (h > (uint32_t)FT_RANKCAP && big == 0x7fffffff) big = b;
    }
    hist[j * 64 + lane] = run;
    run += h;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    vmax = max(vmax, __shfl_xor(vmax, off));
    big = min(big, __shfl_xor(big, off));
  }
  if (lane == L) { red[3] = (uint32_t)bstar; red[4] = below; }
  if (lane == 0) { red[8] = vmax; red[9] = (uint32_t)big; }
}

// Fast path (cnt <= cap), over monotone bins of the key image so that every
// bin below the threshold bin is wholly inside the result:
//  1. min / max key image; 2048 coarse bins over [min, max];
//  2. histogram and prefix; threshold bin b* = first bin whose running count
//     reaches cnt, s = cnt - (count below b*).  When a bin below b* holds
//     more than FT_RANKCAP items, the coarse bins from the first such bin up
//     to b* are split into 2048 fine bins and the histogram is taken again
//     (a few near neighbours far below the k-th distance otherwise crowd the
//     candidates into few coarse bins);
//  3. items of bins < b* are scattered into LDS grouped by bin, the members
//     of b* are collected apart (an exact radix select over b*'s members if
//     they do not fit);
//  4. when every bin below b* holds at most FT_RANKCAP items, each item's
//     output slot is its bin's start plus the number of smaller items in its
//     bin (the bins are contiguous and ordered), and the first s of b*
//     (ranked the same way, or sorted when b* is large) follow; otherwise the
//     cnt winners are sorted.
// items(fn) calls fn(v, valid) for every candidate v this thread owns, with a
// block-uniform number of calls (fn may use wave-wide collectives); the
// candidates stay readable at in[0, kc) for the rare exact-select path.
// LDS: hist[FT_NB2], bbuf[FT_BCAP], red[12] and obuf (cap items) from the kernel.
// IN_LDS: the winners grouped by bin go to the LDS buffer (cnt <= cap), else
// to the query's slots of the scratch buffer (a compile-time choice, so that
// each form addresses one memory).
template <bool IN_LDS, class Items>
__device__ bool final_topk_binned(const int metric, const int cap, const uint64_t* in, int64_t kc, int64_t cnt, int64_t* oid,
                                  float* odist, uint64_t* gbuf_mem, uint64_t* obuf, uint32_t* hist, uint64_t* bbuf,
                                  uint32_t* red, Items items) {
  constexpr int NT = 1024;
  uint64_t* gbuf = IN_LDS ? obuf : gbuf_mem;
  static_assert(FT_NB == 64 * 32 && FT_NB2 == 64 * 64, "one wave forms the prefix");
  if (threadIdx.x == 0) { red[0] = 0xffffffffu; red[1] = 0u; red[2] = 0u; }
  for (int i = threadIdx.x; i < FT_NB; i += NT) hist[i] = 0;
  __syncthreads();
  uint32_t mn = 0xffffffffu, mx = 0u;
  items([&](uint64_t v, bool ok) {
    const uint32_t kb = (uint32_t)(v >> 32);
    if (ok) {
      mn = min(mn, kb);
      mx = max(mx, kb);
    }
  });
  for (int off = 32; off >= 1; off >>= 1) {
    mn = min(mn, __shfl_xor(mn, off));
    mx = max(mx, __shfl_xor(mx, off));
  }
  if ((threadIdx.x & 63) == 0) { atomicMin(&red[0], mn); atomicMax(&red[1], mx); }
  __syncthreads();
  FtBins bins;
  bins.kmin = red[0];
  const uint32_t span = red[1] - bins.kmin;
  bins.shift = 0;
  while ((span >> bins.shift) >= (uint32_t)FT_NB) ++bins.shift;
  bins.lo2 = 0;
  bins.shift2 = 0;
  bins.blo = FT_NB;
  bins.bhi = FT_NB - 1;
  bins.out = FT_NB2;
  int lg = 5;
  items([&](uint64_t v, bool ok) {
    wave_hist_add(hist, (uint32_t)ft_slot(ok ? bins((uint32_t)(v >> 32)) : 0, lg), ok);
  });
  __syncthreads();
  if (threadIdx.x < 64) ft_prefix(hist, lg, cnt, red);
  __syncthreads();
  if (red[8] > (uint32_t)FT_RANKCAP) {
    // refine: coarse bins [big, b*] into 2048 fine bins
    bins.blo = (int)red[9];
    bins.bhi = (int)red[3];
    bins.lo2 = bins.kmin + ((uint32_t)bins.blo << bins.shift);
    const uint64_t span2 = ((uint64_t)(bins.bhi + 1 - bins.blo) << bins.shift) - 1;
    while ((span2 >> bins.shift2) >= (uint64_t)FT_NB) ++bins.shift2;
    lg = 6;
    __syncthreads();
    for (int i = threadIdx.x; i < FT_NB2; i += NT) hist[i] = 0;
    __syncthreads();
    items([&](uint64_t v, bool ok) {
      const int b = ok ? bins((uint32_t)(v >> 32)) : bins.out;
      wave_hist_add(hist, (uint32_t)ft_slot(b < bins.out ? b : 0, lg), b < bins.out);
    });
    __syncthreads();
    if (threadIdx.x < 64) ft_prefix(hist, lg, cnt, red);
    __syncthreads();
  }
  const int bstar = (int)red[3];
  const int64_t nbelow = red[4];
  const int64_t s = cnt - nbelow;
  items([&](uint64_t v, bool ok) {
    const int b = bins((uint32_t)(v >> 32));
    if (ok && b < bstar) {
      gbuf[atomicAdd(&hist[ft_slot(b, lg)], 1u)] = v;
    } else if (ok && b == bstar) {
      uint32_t bs = atomicAdd(&red[2], 1u);
      if (bs < (uint32_t)FT_BCAP) bbuf[bs] = v;
    }
  });
  __syncthreads();
  const int64_t nb = red[2];
  const float sgn = metric == 0 ? 1.f : -1.f;
  if (nb <= FT_BCAP && red[8] <= (uint32_t)FT_RANKCAP) {
    // after the scatter the slot of bin b holds the end of bin b, so bin b
    // (< b*) spans [b ? end(b - 1) : 0, end(b))
    if (nb <= 256) {
      for (int t = threadIdx.x; t < nb; t += NT) {
        const uint64_t v = bbuf[t];
        int rank = 0;
        for (int j = 0; j < (int)nb; ++j) rank += bbuf[j] < v;
        if (rank < s) {
          oid[nbelow + rank] = (int64_t)packed_id(v);
          odist[nbelow + rank] = sgn * packed_key(v);
        }
      }
    } else {
      const int P = next_pow2((int)nb);
      for (int i = (int)nb + threadIdx.x; i < P; i += NT) bbuf[i] = ~0ull;
      lds_bitonic_sort<NT>(bbuf, P);
      for (int64_t r = threadIdx.x; r < s; r += NT) {
        const uint64_t v = bbuf[r];
        oid[nbelow + r] = (int64_t)packed_id(v);
        odist[nbelow + r] = sgn * packed_key(v);
      }
    }
    for (int64_t p = threadIdx.x; p < nbelow; p += NT) {
      const uint64_t v = gbuf[p];
      const int b = bins((uint32_t)(v >> 32));
      const int beg = b ? (int)hist[ft_slot(b - 1, lg)] : 0, end = (int)hist[ft_slot(b, lg)];
      int rank = 0;
      for (int j = beg; j < end; ++j) rank += gbuf[j] < v;
      oid[beg + rank] = (int64_t)packed_id(v);
      odist[beg + rank] = sgn * packed_key(v);
    }
    return true;
  }
  if (nb <= FT_BCAP) {
    const int P = next_pow2((int)nb);
    for (int i = (int)nb + threadIdx.x; i < P; i += NT) bbuf[i] = ~0ull;
    lds_bitonic_sort<NT>(bbuf, P);
    for (int64_t r = threadIdx.x; r < s; r += NT) gbuf[nbelow + r] = bbuf[r];
  } else {
    auto get = [&](int64_t i, uint64_t& v) -> bool {
      v = in[i];
      return bins((uint32_t)(v >> 32)) == bstar;
    };
    uint64_t thr = block_radix_select64<NT>(get, kc, s - 1, hist, red + 8);
    if (threadIdx.x == 0) red[2] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < kc; i += NT) {
      uint64_t v;
      if (get(i, v) && v <= thr) gbuf[nbelow + atomicAdd(&red[2], 1u)] = v;
    }
  }
  __syncthreads();
  const int P = next_pow2((int)cnt);
  if (P > cap) {
    // the winners do not fit a power-of-two LDS sort: hand them over unsorted
    uint64_t* outp = reinterpret_cast<uint64_t*>(oid);
    for (int64_t i = threadIdx.x; i < cnt; i += NT) outp[i] = gbuf[i];
    __syncthreads();
    return false;
  }
  if constexpr (!IN_LDS) {
    for (int i = threadIdx.x; i < P; i += NT) obuf[i] = i < cnt ? gbuf[i] : ~0ull;
  } else {
    for (int i = (int)cnt + threadIdx.x; i < P; i += NT) obuf[i] = ~0ull;
  }
  lds_bitonic_sort<NT>(obuf, P);
  for (int64_t i = threadIdx.x; i < cnt; i += NT) {
    const uint64_t v = obuf[i];
    const float key = packed_key(v);
    oid[i] = (int64_t)packed_id(v);
    odist[i] = metric == 0 ? key : -key;
  }
  return true;
}

// Sorts outp[0, cnt) (distinct packed values) ascending: runs of `run` items
// sorted in LDS, then pairwise merge-path merges ping-ponging with scratch
// (>= cnt slots); then unpacks in place into (id, distance).
__device__ void sort_global_unpack(const int metric, const int run, uint64_t* outp, uint64_t* scratch, int64_t cnt,
                                   uint64_t* run_buf, int64_t* oid, float* odist) {
  constexpr int NT = 1024;
  for (int64_t r0 = 0; r0 < cnt; r0 += run) {
    const int n = (int)min((int64_t)run, cnt - r0);
    const int P = next_pow2(n);
    for (int i = threadIdx.x; i < P; i += NT) run_buf[i] = i < n ? outp[r0 + i] : ~0ull;
    lds_bitonic_sort<NT>(run_buf, P);
    for (int i = threadIdx.x; i < n; i += NT) outp[r0 + i] = run_buf[i];
    __syncthreads();
  }
  uint64_t* src = outp;
  uint64_t* dst = scratch;
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
    odist[i] = metric == 0 ? key : -key;
  }
}

// The candidates read from memory: the memory form, or a register form's
// query whose result set does not fit the LDS buffer (SCRATCH_ONLY: then the
// winners always go to the scratch buffer, and only that form is compiled
// into the register kernels).
template <bool SCRATCH_ONLY>
__device__ __forceinline__ void final_topk_mem(const FinalArgs& a, uint64_t* in, int64_t kc, int64_t cnt,
                                               int64_t* oid, float* odist, uint64_t* outp, uint64_t* gbuf,
                                               uint64_t* run_buf, uint32_t* hist, uint64_t* bbuf, uint32_t* red) {
  constexpr int NT = 1024;
  auto items = [&](auto fn) {
    constexpr int B = SCRATCH_ONLY ? 1 : 8;  // loads in flight per thread (registers kept for the others)
    for (int64_t base = 0; base < kc; base += (int64_t)NT * B) {
      uint64_t v[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int64_t i = base + (int64_t)u * NT + threadIdx.x;
        v[u] = in[i < kc ? i : kc - 1];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int64_t i = base + (int64_t)u * NT + threadIdx.x;
        if (base + (int64_t)u * NT < kc) fn(i < kc ? v[u] : ~0ull, i < kc);
      }
    }
  };
  bool done;
  if (SCRATCH_ONLY || cnt > a.cap)
    done = final_topk_binned<false>(a.metric, a.cap, in, kc, cnt, oid, odist, gbuf, run_buf, hist, bbuf, red, items);
  else
    done = final_topk_binned<true>(a.metric, a.cap, in, kc, cnt, oid, odist, gbuf, run_buf, hist, bbuf, red, items);
  if (!done) sort_global_unpack(a.metric, a.run, outp, in, cnt, run_buf, oid, odist);
}

// IPT > 0: the candidates are loaded once into registers (IPT per thread,
// K_c <= IPT * 1024) and every pass of the binned path runs from there.
template <int IPT>
__global__ __launch_bounds__(1024, (IPT > 0 && IPT <= 16) ? 8 : 1) void final_topk_kernel(FinalArgs a) {
  constexpr int NT = 1024;
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* run_buf = reinterpret_cast<uint64_t*>(smem);  // [a.cap]
  __shared__ uint32_t hist[FT_NB2];
  __shared__ uint64_t bbuf[FT_BCAP];
  __shared__ __align__(8) uint32_t red[12];
  uint32_t* bc = red;

  const int64_t qi = a.qmap ? (int64_t)a.qmap[blockIdx.x] : (int64_t)blockIdx.x;
  const int64_t kc = a.n_cand[qi];
  const int64_t k = a.k[qi];
  const int64_t cnt = kc < k ? kc : k;
  uint64_t* in = a.cand_packed + a.cand_off[qi];
  int64_t* oid = a.out_ids + a.out_off[qi];
  float* odist = a.out_dists + a.out_off[qi];
  uint64_t* outp = reinterpret_cast<uint64_t*>(oid);
  uint64_t* gbuf = a.scratch + a.out_off[qi];  // k slots: the winners grouped by bin

  if (IPT > 0 && cnt > 0 && cnt <= a.cap && kc <= (int64_t)IPT * NT) {
    uint64_t v[IPT > 0 ? IPT : 1];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int64_t i = (int64_t)u * NT + threadIdx.x;
      v[u] = i < kc ? in[i] : ~0ull;
    }
    auto items = [&](auto fn) {
#pragma unroll
      for (int u = 0; u < IPT; ++u)
        if ((int64_t)u * NT < kc) fn(v[u], (int64_t)u * NT + threadIdx.x < kc);
    };
    const bool done =
        final_topk_binned<true>(a.metric, a.cap, in, kc, cnt, oid, odist, gbuf, run_buf, hist, bbuf, red, items);
    if (!done) sort_global_unpack(a.metric, a.run, outp, in, cnt, run_buf, oid, odist);
  } else if (cnt > 0) {
    final_topk_mem<(IPT > 0)>(a, in, kc, cnt, oid, odist, outp, gbuf, run_buf, hist, bbuf, red);
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
  size_t lds = sizeof(uint64_t) * (size_t)a.cap;
  const dim3 g((unsigned)a.nq), b(1024);
  switch (final_topk_form(a.max_kc)) {
    case 8: hipLaunchKernelGGL((final_topk_kernel<8>), g, b, lds, s, a); break;
    case 16: hipLaunchKernelGGL((final_topk_kernel<16>), g, b, lds, s, a); break;
    case 24: hipLaunchKernelGGL((final_topk_kernel<24>), g, b, lds, s, a); break;
    case 32: hipLaunchKernelGGL((final_topk_kernel<32>), g, b, lds, s, a); break;
    default: hipLaunchKernelGGL((final_topk_kernel<0>), g, b, lds, s, a); break;
  }
  return hipGetLastError();
}

int final_topk_form(int64_t max_kc) {
  if (max_kc <= 8 * 1024) return 8;
  if (max_kc <= 16 * 1024) return 16;
  if (max_kc <= 24 * 1024) return 24;
  if (max_kc <= 32 * 1024) return 32;
  return 0;
}

}  // namespace bbc

// Bucket-based result collector on the GPU (result-buffer section of the
// paper: Push / Update / Collect, the codebook from a sample of the nearest
// clusters, and the bucket-id equation).
//
// One block of 1024 threads per query, over the query's estimated keys
// (already in the key scratch, in probe order):
//  1. Codebook.  The sample is the keys of the first nsample probed lists.
//     T = min(K_c, |sample|); d_min / d_max are the smallest and the T-th
//     smallest sample key; delta = (d_max - d_min) / 256 (1 if that is not
//     positive); the 256 equal-width cells are mapped onto m buckets of equal
//     depth w.r.t. the sample's T smallest keys:
//     map[e] = min(m-1, floor(m * C_<e / T)).
//  2. Histogram.  bucket(key) = map[clamp(floor((key - d_min)/delta),0,255)],
//     counted in LDS over all S keys.
//  3. Update.  tau = first bucket whose running count reaches K_c;
//     s = K_c - (count below tau).  Because the per-list cadence of the
//     paper only ever lowers tau, the final tau of the once-per-list Update
//     equals the tau of the full histogram.
//  4. Collect.  Every object of a bucket below tau is a candidate; the
//     threshold bucket's objects are sorted by (key, id) in LDS and its
//     first s are added.  A threshold bucket larger than the LDS buffer is
//     resolved by an exact 64-bit radix select over its members instead.
// The result is exactly the K_c smallest (key, id): the definition of the
// collector's output.  Slots are taken by LDS atomics, so the order of
// candidates in the buffer is arbitrary; the set is not.
#include "common.h"
#include "kernels.h"

namespace bbc {

__device__ __forceinline__ int64_t slot_to_pos(int64_t i, const int64_t* __restrict__ rank_off,
                                               const int32_t* __restrict__ lists,
                                               const int64_t* __restrict__ list_off, int np) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (rank_off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return list_off[lists[lo]] + (i - rank_off[lo]);
}

__global__ __launch_bounds__(1024) void collect_bucket_kernel(CollectArgs a) {
  constexpr int NT = 1024;
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* bbuf = reinterpret_cast<uint64_t*>(smem);  // [bcap], bcap a power of two
  __shared__ uint32_t hist[256];
  __shared__ uint32_t counts[BBC_MAX_BUCKETS];
  __shared__ uint8_t cmap[256];
  __shared__ uint32_t bc[8];
  __shared__ float fbc[2];

  const int64_t qi = blockIdx.x;
  const int64_t S = a.n_scanned[qi];
  int64_t kc = a.kc_target[qi];
  if (kc > S) kc = S;
  const int np = a.nprobe[qi];
  const int64_t po = a.probe_off[qi];
  const int64_t* rank_off = a.rank_off + po;
  const int32_t* lists = a.probe_lists + po;
  const float* keys = a.keys + a.key_off[qi];
  const int m = a.m;
  if (kc <= 0) {
    if (threadIdx.x == 0) {
      a.n_cand[qi] = 0;
      if (a.t_tau) { a.t_tau[qi] = -1; a.t_s[qi] = 0; a.t_dmin[qi] = 0.f; a.t_delta[qi] = 1.f; }
    }
    if (a.t_map) for (int e = threadIdx.x; e < 256; e += NT) a.t_map[qi * 256 + e] = 0;
    if (a.t_counts) for (int b = threadIdx.x; b < m; b += NT) a.t_counts[qi * m + b] = 0;
    return;
  }

  // ---- 1. codebook from the sample ------------------------------------
  const int nsr = a.nsample < np ? a.nsample : np;
  const int64_t Ts = nsr < np ? rank_off[nsr] : S;
  const int64_t T = kc < Ts ? kc : Ts;
  if (T > 0) {
    uint32_t dmax_b = block_radix_select32<NT>([&](int64_t i) { return key_bits(keys[i]); }, Ts, T - 1,
                                               hist, bc);
    if (threadIdx.x == 0) bc[4] = 0xffffffffu;
    __syncthreads();
    uint32_t mn = 0xffffffffu;
    for (int64_t i = threadIdx.x; i < Ts; i += NT) mn = min(mn, key_bits(keys[i]));
    for (int off = 32; off >= 1; off >>= 1) mn = min(mn, __shfl_xor(mn, off));
    if ((threadIdx.x & 63) == 0) atomicMin(&bc[4], mn);
    for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
    __syncthreads();
    const float dmin = bits_key(bc[4]);
    const float dmax = bits_key(dmax_b);
    float delta = (dmax - dmin) / 256.0f;
    if (!(delta > 0.0f)) delta = 1.0f;
    for (int64_t i = threadIdx.x; i < Ts; i += NT) {
      float k = keys[i];
      if (key_bits(k) < dmax_b) atomicAdd(&hist[cell_of(k, dmin, delta)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t below = 0;
      for (int e = 0; e < 256; ++e) below += hist[e];
      hist[cell_of(dmax, dmin, delta)] += (uint32_t)(T - below);
      below = 0;
      for (int e = 0; e < 256; ++e) {
        int64_t b = ((int64_t)m * below) / T;
        cmap[e] = (uint8_t)(b < m - 1 ? b : m - 1);
        below += hist[e];
      }
      fbc[0] = dmin;
      fbc[1] = delta;
    }
  } else if (threadIdx.x == 0) {
    for (int e = 0; e < 256; ++e) cmap[e] = 0;
    fbc[0] = 0.0f;
    fbc[1] = 1.0f;
  }
  for (int b = threadIdx.x; b < m; b += NT) counts[b] = 0;
  __syncthreads();
  const float dmin = fbc[0], delta = fbc[1];

  // ---- 2. histogram of all keys ----------------------------------------
  for (int64_t i = threadIdx.x; i < S; i += NT)
    atomicAdd(&counts[cmap[cell_of(keys[i], dmin, delta)]], 1u);
  __syncthreads();

  // ---- 3. Update: threshold bucket and s ---------------------------------
  if (threadIdx.x == 0) {
    int64_t cum = 0;
    int tau = m - 1;
    for (int b = 0; b < m; ++b) {
      if (cum + (int64_t)counts[b] >= kc) { tau = b; break; }
      cum += counts[b];
    }
    bc[0] = (uint32_t)tau;
    bc[1] = (uint32_t)cum;      // objects strictly below tau
    bc[2] = 0;                  // candidate slot counter
    bc[3] = 0;                  // boundary slot counter
  }
  __syncthreads();
  const int tau = (int)bc[0];
  const int64_t nbelow = bc[1];
  const int64_t s = kc - nbelow;
  const int bcap = a.bcap;
  uint32_t* cand = a.cand_pos + a.cand_off[qi];

  // ---- 4. Collect -----------------------------------------------------------
  for (int64_t i = threadIdx.x; i < S; i += NT) {
    float k = keys[i];
    int b = cmap[cell_of(k, dmin, delta)];
    if (b < tau) {
      uint32_t slot = atomicAdd(&bc[2], 1u);
      cand[slot] = (uint32_t)slot_to_pos(i, rank_off, lists, a.list_off, np);
    } else if (b == tau) {
      uint32_t bs = atomicAdd(&bc[3], 1u);
      if ((int)bs < bcap) {
        int64_t pos = slot_to_pos(i, rank_off, lists, a.list_off, np);
        bbuf[bs] = pack_key_id(k, (uint32_t)a.list_ids[pos]);
      }
    }
  }
  __syncthreads();
  const int64_t nb = bc[3];
  if (nb <= bcap) {
    const int P = next_pow2((int)nb);
    for (int i = (int)nb + threadIdx.x; i < P; i += NT) bbuf[i] = ~0ull;
    __syncthreads();
    lds_bitonic_sort<NT>(bbuf, P);
    for (int64_t r = threadIdx.x; r < s; r += NT)
      cand[nbelow + r] = (uint32_t)a.pos_of_id[packed_id(bbuf[r])];
  } else {
    // exact selection of the s smallest (key, id) of the threshold bucket
    auto get = [&](int64_t i, uint64_t& v) -> bool {
      float k = keys[i];
      if (cmap[cell_of(k, dmin, delta)] != tau) return false;
      int64_t pos = slot_to_pos(i, rank_off, lists, a.list_off, np);
      v = pack_key_id(k, (uint32_t)a.list_ids[pos]);
      return true;
    };
    uint64_t thr = block_radix_select64<NT>(get, S, s - 1, hist, bc + 4);
    if (threadIdx.x == 0) bc[3] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < S; i += NT) {
      uint64_t v;
      if (get(i, v) && v <= thr) {
        uint32_t slot = atomicAdd(&bc[3], 1u);
        cand[nbelow + slot] = (uint32_t)slot_to_pos(i, rank_off, lists, a.list_off, np);
      }
    }
  }
  if (threadIdx.x == 0) {
    a.n_cand[qi] = kc;
    if (a.t_tau) {
      a.t_tau[qi] = tau;
      a.t_s[qi] = s;
      a.t_dmin[qi] = dmin;
      a.t_delta[qi] = delta;
      a.t_nboundary[qi] = nb;
    }
  }
  if (a.t_map) for (int e = threadIdx.x; e < 256; e += NT) a.t_map[qi * 256 + e] = cmap[e];
  if (a.t_counts) for (int b = threadIdx.x; b < m; b += NT) a.t_counts[qi * m + b] = (int32_t)counts[b];
}

hipError_t launch_collect_bucket(const CollectArgs& a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  size_t lds = sizeof(uint64_t) * (size_t)a.bcap;
  hipLaunchKernelGGL(collect_bucket_kernel, dim3((unsigned)a.nq), dim3(1024), lds, s, a);
  return hipGetLastError();
}

}  // namespace bbc

// Shared device helpers for the BBC query path on gfx950 (CDNA4, wave64).
//
// Canonical float32 arithmetic: the library is compiled with
// -ffp-contract=off (no FMA contraction), IEEE division/sqrt, no fast-math.
// Distances follow one fixed operation order (below) so that results are
// reproducible bit for bit by any implementation of the same order:
//   * a vector is padded with zeros to a multiple of 256 elements and cut into
//     4-element chunks; chunk c belongs to lane c % 64 at step c / 64;
//   * each lane starts at +0 and, step by step and element by element, adds
//     t = (a - b) * (a - b)   [L2]   or   t = a * b   [inner product];
//   * lanes are combined as acc[l] = acc[l] + acc[l + off], off = 32 .. 1.
// Lanes that only ever see padding hold +0, and adding +0 to a partial sum
// that is never -0 is exact, so a row of at most 32 chunks can be reduced on
// 32 lanes (off = 16 .. 1) with the same result.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define BBC_WAVE 64
#define BBC_NCELLS 256          // equal-width cells of the bucket codebook
#define BBC_MAX_BUCKETS 256     // m <= 256: the cell->bucket map is one byte

namespace bbc {

// Key order used everywhere: numeric key (-0 == +0), ties to the smaller id.
// The 32-bit image below is monotone in the key; -0 is first made +0.
__device__ __forceinline__ uint32_t key_bits(float f) {
  f = f + 0.0f;  // -0 -> +0, every other value unchanged
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float bits_key(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
__device__ __forceinline__ uint64_t pack_key_id(float key, uint32_t id) {
  return ((uint64_t)key_bits(key) << 32) | (uint64_t)id;
}
__device__ __forceinline__ float packed_key(uint64_t p) { return bits_key((uint32_t)(p >> 32)); }
__device__ __forceinline__ uint32_t packed_id(uint64_t p) { return (uint32_t)(p & 0xffffffffu); }

// Equal-width cell of a key: clamp(floor((key - dmin) / delta), 0, 255).
__device__ __forceinline__ int cell_of(float key, float dmin, float delta) {
  float t = (key - dmin) / delta;
  if (t < 0.0f) return 0;
  if (t >= 255.0f) return 255;
  return (int)t;
}

// Lane combination of the canonical order on a full wave (off = 32 .. 1).
__device__ __forceinline__ float canon_reduce64(float acc) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc = acc + __shfl_xor(acc, off);
  return acc;
}
// Same on each 32-lane half of a wave (rows of at most 32 chunks).
__device__ __forceinline__ float canon_reduce32(float acc) {
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) acc = acc + __shfl_xor(acc, off);
  return acc;
}

// One four-element chunk of the canonical sums: per element a difference
// (L2) and a fused multiply-add into the running sum (one rounding of
// t * t + acc, or a * b + acc).
__device__ __forceinline__ float chunk_l2(float4 a, float4 b, float acc) {
  float t;
  t = a.x - b.x; acc = __builtin_fmaf(t, t, acc);
  t = a.y - b.y; acc = __builtin_fmaf(t, t, acc);
  t = a.z - b.z; acc = __builtin_fmaf(t, t, acc);
  t = a.w - b.w; acc = __builtin_fmaf(t, t, acc);
  return acc;
}
// chunk_l2(a, b, 0.0f) with its first step a plain square: t * t + 0 rounds
// to the rounded square for every t (never -0), so the result is the same
// bit for bit
__device__ __forceinline__ float chunk_l2_0(float4 a, float4 b) {
  float t, acc;
  t = a.x - b.x; acc = t * t;
  t = a.y - b.y; acc = __builtin_fmaf(t, t, acc);
  t = a.z - b.z; acc = __builtin_fmaf(t, t, acc);
  t = a.w - b.w; acc = __builtin_fmaf(t, t, acc);
  return acc;
}
__device__ __forceinline__ float chunk_ip(float4 a, float4 b, float acc) {
  acc = __builtin_fmaf(a.x, b.x, acc);
  acc = __builtin_fmaf(a.y, b.y, acc);
  acc = __builtin_fmaf(a.z, b.z, acc);
  acc = __builtin_fmaf(a.w, b.w, acc);
  return acc;
}

// Canonical L2 / IP of two float rows (d a multiple of 4, 16-byte aligned)
// computed by one full wave; every lane returns the result.
__device__ __forceinline__ float wave_canon(const float* __restrict__ a, const float* __restrict__ b,
                                            int d, bool ip) {
  const int lane = threadIdx.x & 63;
  const int nchunk = d >> 2;
  float acc = 0.0f;
  for (int c = lane; c < nchunk; c += 64) {
    float4 av = reinterpret_cast<const float4*>(a)[c];
    float4 bv = reinterpret_cast<const float4*>(b)[c];
    acc = ip ? chunk_ip(av, bv, acc) : chunk_l2(av, bv, acc);
  }
  return canon_reduce64(acc);
}

// Block-wide helpers ------------------------------------------------------

template <int NT>
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* red) {
  // red: LDS scratch of NT/64 entries
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Bitonic sort of n (power of two) 64-bit values in LDS, ascending, by a
// block of NT threads.
template <int NT>
__device__ void lds_bitonic_sort(uint64_t* v, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < (n >> 1); t += NT) {
        int lo = 2 * t - (t & (stride - 1));
        int hi = lo + stride;
        bool up = ((lo & size) == 0);
        uint64_t a = v[lo], b = v[hi];
        if ((a > b) == up) { v[lo] = b; v[hi] = a; }
      }
    }
  }
  __syncthreads();
}

// Values that are equal on every lane, moved to scalar registers (the
// compiler cannot prove uniformity of values loaded through vector loads).
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform(int64_t v) {
  const uint32_t lo = uniform((uint32_t)v), hi = uniform((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
// The value lane l of the wave holds (l wave-uniform), in a scalar register.
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ int32_t lane_value(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ int64_t lane_value(int64_t v, int l) {
  const uint32_t lo = lane_value((uint32_t)v, l), hi = lane_value((uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
  return reinterpret_cast<T*>(uniform((int64_t)reinterpret_cast<uintptr_t>(p)));
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  return v;
}

// Run by one whole wave: the bin holding rank rr (0-based, ascending) of a
// histogram hist[0, nb), nb <= 256: the first bin dg whose running count
// exceeds rr, and rem = rr minus the count below dg.  When the running count
// never exceeds rr, dg = nb - 1 (rem still relative to that bin).  The lane
// that finds the bin writes dg and rem (LDS words) for the block.
__device__ __forceinline__ void wave_find_rank(const uint32_t* hist, int nb, int64_t rr, uint32_t* dg_out,
                                               int64_t* rem_out) {
  const int lane = threadIdx.x & 63;
  uint32_t h[4], sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = 4 * lane + j;
    h[j] = e < nb ? hist[e] : 0u;
    sum += h[j];
  }
  const uint32_t incl = wave_incl_scan(sum);
  const uint64_t hit = __ballot((int64_t)incl > rr);
  const int last = (nb - 1) >> 2;
  int L = hit ? __ffsll((unsigned long long)hit) - 1 : last;
  if (L > last) L = last;
  if (lane == L) {
    int64_t rem = rr - (int64_t)(incl - sum);
    int dg = 4 * L;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dg = 4 * L + j;
      if (dg >= nb - 1 || rem < (int64_t)h[j]) break;
      rem -= h[j];
    }
    *dg_out = (uint32_t)dg;
    *rem_out = rem;
  }
}

// hist[bin] += 1 for every active lane with valid set.  Lanes that share the
// first valid lane's bin are counted with one ballot and one atomic (keys of
// one query are concentrated, so most lanes of a wave often share a bin);
// the others add their own.
__device__ __forceinline__ void wave_hist_add(uint32_t* hist, uint32_t bin, bool valid) {
  const uint64_t act = __ballot(valid);
  if (!act) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)act) - 1;
  const uint32_t lb = __shfl(bin, leader);
  const uint64_t same = __ballot(valid && bin == lb);
  if (lane == leader) atomicAdd(&hist[lb], (uint32_t)__popcll(same));
  else if (valid && bin != lb) atomicAdd(&hist[bin], 1u);
}

// i = threadIdx.x, threadIdx.x + NT, ... < n over the block: the values
// load(i) of U consecutive strides are loaded before any is used (U loads in
// flight per thread), then use(i, valid, v) runs for each; every lane calls
// use() the same block-uniform number of times (valid = false past n), so
// use() may take wave-wide collectives.  Lanes past n load element n - 1
// (and ignore it): a load under a lane mask would be issued and waited for
// on its own.
template <int NT, int U, typename Load, typename Use>
__device__ __forceinline__ void block_for_batched(int64_t n, Load load, Use use) {
  using V = decltype(load((int64_t)0));
  for (int64_t base = 0; base < n; base += (int64_t)NT * U) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + (int64_t)u * NT + threadIdx.x;
      v[u] = load(i < n ? i : n - 1);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + (int64_t)u * NT + threadIdx.x;
      use(i, i < n, v[u]);
    }
  }
}

// Radix select over a block: value of the element of rank r (0-based,
// ascending) among n 32-bit values produced by get(i).  hist: 256 LDS words;
// bc: 4 LDS words for broadcast, 8-byte aligned.
template <int NT, int U = 4, typename Get>
__device__ uint32_t block_radix_select32(Get get, int64_t n, int64_t r, uint32_t* hist, uint32_t* bc) {
  uint32_t prefix = 0, mask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
    __syncthreads();
    block_for_batched<NT, U>(n, get, [&](int64_t, bool valid, uint32_t v) {
      wave_hist_add(hist, (v >> shift) & 255u, valid && (v & mask) == prefix);
    });
    __syncthreads();
    if (threadIdx.x < 64) wave_find_rank(hist, 256, r, &bc[0], reinterpret_cast<int64_t*>(bc + 2));
    __syncthreads();
    prefix |= bc[0] << shift;
    mask |= 255u << shift;
    r = *reinterpret_cast<const int64_t*>(bc + 2);
    __syncthreads();
  }
  return prefix;
}

// 64-bit variant over the elements for which get(i, v) returns true.
template <int NT, int U = 4, typename Get>
__device__ uint64_t block_radix_select64(Get get, int64_t n, int64_t r, uint32_t* hist, uint32_t* bc) {
  uint64_t prefix = 0, mask = 0;
  struct KV { uint64_t v; bool ok; };
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
    __syncthreads();
    block_for_batched<NT, U>(
        n,
        [&](int64_t i) {
          KV e{0, false};
          e.ok = get(i, e.v);
          return e;
        },
        [&](int64_t, bool valid, KV e) {
          wave_hist_add(hist, (uint32_t)((e.v >> shift) & 255u), valid && e.ok && (e.v & mask) == prefix);
        });
    __syncthreads();
    if (threadIdx.x < 64) wave_find_rank(hist, 256, r, &bc[0], reinterpret_cast<int64_t*>(bc + 2));
    __syncthreads();
    prefix |= (uint64_t)bc[0] << shift;
    mask |= 255ull << shift;
    r = *reinterpret_cast<const int64_t*>(bc + 2);
    __syncthreads();
  }
  return prefix;
}

// Slot of this lane among the active lanes of its wave that set `take`, from
// one atomic per wave on *counter (LDS or global memory).
__device__ __forceinline__ uint32_t wave_slot(bool take, uint32_t* counter) {
  const uint64_t mask = __ballot(take);
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = __shfl(base, leader < 0 ? 0 : leader);
  return base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

// ---- slot -> list position of a query's scanned objects -----------------------
// Scanned objects are numbered by slot in probe order (rank r's list fills
// slots rank_off[r] ..); pos(slot) is the object's position in list-slot
// order, through LDS copies of the rank offsets and list starts when they fit.
struct SlotMap {
  const int64_t* rank_off;  // [np] slot offset of each probe rank
  const int32_t* lists;     // [np] list of each probe rank
  const int64_t* list_off;
  int np;
  const int32_t* s_rbeg;  // LDS copies (lds = true)
  const int32_t* s_lbeg;
  bool lds;
  __device__ int64_t rbeg(int r) const { return lds ? (int64_t)s_rbeg[r] : rank_off[r]; }
  __device__ int64_t lbeg(int r) const { return lds ? (int64_t)s_lbeg[r] : list_off[lists[r]]; }
  // the probe rank that holds a slot
  __device__ int rank(int64_t slot) const {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rbeg(mid) <= slot) lo = mid; else hi = mid - 1;
    }
    return lo;
  }
  __device__ int64_t pos(int64_t slot) const {
    const int r = rank(slot);
    return lbeg(r) + (slot - rbeg(r));
  }
};

// Block-wide: fills the LDS tables (when np <= CAP and slots fit 31 bits)
// and returns the map; ends with a barrier.
template <int NT, int CAP>
__device__ SlotMap slot_map_load(const int64_t* rank_off, const int32_t* lists, const int64_t* list_off, int np,
                                 int32_t* s_rbeg, int32_t* s_lbeg) {
  SlotMap sm;
  sm.rank_off = rank_off;
  sm.lists = lists;
  sm.list_off = list_off;
  sm.np = np;
  // (list positions fit 31 bits: indexes hold fewer than 2^31 objects)
  sm.lds = np <= CAP && rank_off[np - 1] < 0x7fffffff;
  sm.s_rbeg = s_rbeg;
  sm.s_lbeg = s_lbeg;
  if (sm.lds)
    for (int r = threadIdx.x; r < np; r += NT) {
      s_rbeg[r] = (int32_t)rank_off[r];
      s_lbeg[r] = (int32_t)list_off[lists[r]];
    }
  __syncthreads();
  return sm;
}

// ---- wave-level 64-ary max-heap in global memory ------------------------------
// heap storage in global memory, read past the L1 so that every lane of the
// wave sees the stores of the others
__device__ __forceinline__ uint64_t hload(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void hstore(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave: sift v down from node i of the 64-ary max-heap h[0, n).
__device__ void heap_sift_down(uint64_t* h, int64_t n, int64_t i, uint64_t v) {
  const int lane = threadIdx.x & 63;
  while (true) {
    const int64_t c0 = 64 * i + 1;
    if (c0 >= n) break;
    const int64_t cj = c0 + lane;
    const bool ok = cj < n;
    const uint64_t cv = ok ? hload(h + cj) : 0ull;
    uint64_t mx = cv;
    for (int off = 32; off >= 1; off >>= 1) {
      const uint64_t o = __shfl_xor(mx, off);
      mx = o > mx ? o : mx;
    }
    if (mx <= v) break;
    const uint64_t at = __ballot(ok && cv == mx);
    const int j = __ffsll((unsigned long long)at) - 1;
    if (lane == 0) hstore(h + i, mx);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    i = c0 + j;
  }
  if (lane == 0) hstore(h + i, v);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}


__host__ __device__ __forceinline__ int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace bbc

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

#include <algorithm>
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

// ---- Tile-major re-rank (rows of at most 32 chunks) --------------------------
// The per-query form reads every candidate row once per query that holds it.
// Here the batch's (query, probed list) pairs are grouped by list, a block
// takes one list and up to RT_G of the queries probing it, and it stages the
// list's rows in LDS one tile (1 << tshift rows) at a time: each row then
// comes from memory once per block instead of once per query.  Each query's
// candidates are first grouped by (probe rank, tile of the list) with a
// counting sort in LDS, so that a block finds the candidates of a (query,
// tile) as one range.  Tiles from nbin - 1 on share the last bin and are
// told apart by position.  The distance of each pair is the same canonical
// half-wave computation as above, so the keys are identical.

constexpr uint64_t RT_NO_PAIR = ~0ull;
constexpr int RT_UNROLL = 2;  // rows of a half-wave in flight (they come from LDS)

__global__ void rt_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void rt_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// pairs per list (grid: rank chunks x queries)
__global__ __launch_bounds__(256) void rt_pair_count(TileRerankArgs a) {
  const int64_t q = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r < a.nprobe[q]) atomicAdd(&a.lcnt[a.probe_lists[a.probe_off[q] + r]], 1u);
}

// Exclusive scan of n words in place by one block of NT threads, each taking
// a contiguous run; the total goes to *total.
template <int NT>
__device__ void block_excl_scan(uint32_t* v, int n, uint32_t* s_w, uint32_t* total) {
  const int per = (n + NT - 1) / NT;
  const int b = threadIdx.x * per, e = min(n, b + per);
  uint32_t sum = 0;
  for (int i = b; i < e; ++i) sum += v[i];
  const uint32_t incl = wave_incl_scan(sum);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) s_w[wv] = incl;
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint32_t t = threadIdx.x < NT / 64 ? s_w[threadIdx.x] : 0u;
    const uint32_t ti = wave_incl_scan(t);
    if (threadIdx.x < NT / 64) s_w[threadIdx.x] = ti - t;
    if (threadIdx.x == NT / 64 - 1) *total = ti;
  }
  __syncthreads();
  uint32_t run = s_w[wv] + incl - sum;
  for (int i = b; i < e; ++i) {
    const uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
  __syncthreads();
}

// List segments padded to whole groups of RT_G pairs: lcnt[L] becomes the
// first slot of list L (the scatter's cursor), lcnt[nlist] the group count.
__global__ __launch_bounds__(1024) void rt_pair_offsets(TileRerankArgs a) {
  __shared__ uint32_t s_w[16];
  __shared__ uint32_t s_tot;
  for (int L = threadIdx.x; L < a.nlist; L += 1024) a.lcnt[L] = (a.lcnt[L] + RT_G - 1) / RT_G * RT_G;
  __syncthreads();
  block_excl_scan<1024>(a.lcnt, a.nlist, s_w, &s_tot);
  if (threadIdx.x == 0) a.lcnt[a.nlist] = s_tot / RT_G;
}

__global__ __launch_bounds__(256) void rt_pair_scatter(TileRerankArgs a) {
  const int64_t q = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r < a.nprobe[q]) {
    const uint32_t slot = atomicAdd(&a.lcnt[a.probe_lists[a.probe_off[q] + r]], 1u);
    a.lpairs[slot] = ((uint64_t)q << 32) | (uint32_t)r;
  }
}

// One block per query: its candidates grouped by bin = rank * nbin +
// min(tile, nbin - 1); bin_beg[(pair) * (nbin + 1) + b] = start of bin b of
// the pair (within the query's candidates), [.. + nbin] = the pair's end.
__global__ __launch_bounds__(1024) void rt_cand_sort(TileRerankArgs a) {
  constexpr int NT = 1024;
  extern __shared__ __align__(16) uint32_t sm[];
  __shared__ uint32_t s_w[16];
  __shared__ uint32_t s_tot;
  const int64_t q = blockIdx.x;
  const int np = a.nprobe[q];
  const int64_t po = a.probe_off[q], co = a.cand_off[q];
  const int64_t kc = a.n_cand[q];
  const int B = a.nbin, nb = np * B;
  uint32_t* cnt = sm;                                                      // [max_np * nbin]
  int32_t* s_lbeg = reinterpret_cast<int32_t*>(sm + (size_t)a.max_np * B);  // [max_np]
  uint16_t* rank_of = reinterpret_cast<uint16_t*>(s_lbeg + a.max_np);      // [nlist]
  for (int L = threadIdx.x; L < a.nlist; L += NT) rank_of[L] = 0;
  for (int i = threadIdx.x; i < nb; i += NT) cnt[i] = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < np; r += NT) {
    const int L = a.probe_lists[po + r];
    rank_of[L] = (uint16_t)r;
    s_lbeg[r] = (int32_t)a.list_off[L];
  }
  __syncthreads();
  const uint32_t* cpos = a.cand_pos + co;
  auto bin_of = [&](uint32_t pos) -> uint32_t {
    const int r = min((int)rank_of[a.list_of_pos[pos]], np - 1);  // candidates lie in probed lists
    const uint32_t t = (pos - (uint32_t)s_lbeg[r]) >> a.tshift;
    return (uint32_t)(r * B) + min(t, (uint32_t)(B - 1));
  };
  block_for_batched<NT, 4>(kc, [&](int64_t i) { return cpos[i]; }, [&](int64_t, bool valid, uint32_t pos) {
    if (valid) atomicAdd(&cnt[bin_of(pos)], 1u);
  });
  __syncthreads();
  block_excl_scan<NT>(cnt, nb, s_w, &s_tot);
  uint32_t* bb = a.bin_beg + po * (B + 1);
  for (int i = threadIdx.x; i < np * (B + 1); i += NT) {
    const int r = i / (B + 1), b = i - r * (B + 1);
    bb[i] = b < B ? cnt[r * B + b] : (r + 1 < np ? cnt[(r + 1) * B] : (uint32_t)kc);
  }
  __syncthreads();
  uint32_t* out = a.sorted_pos + co;
  block_for_batched<NT, 4>(kc, [&](int64_t i) { return cpos[i]; }, [&](int64_t, bool valid, uint32_t pos) {
    if (valid) out[atomicAdd(&cnt[bin_of(pos)], 1u)] = pos;
  });
}

template <typename T>
__global__ __launch_bounds__(1024, 8) void rt_rerank_tile(TileRerankArgs a) {
  constexpr int NT = 1024, NW = NT / 64;
  __shared__ uint4 tile[RT_TILE_BYTES / 16];
  __shared__ int32_t s_q[RT_G], s_r[RT_G];
  __shared__ int64_t s_co[RT_G];             // candidate offset of the pair's query
  __shared__ uint32_t s_beg[RT_G], s_end[RT_G];  // the pair's candidates in this tile's bin
  __shared__ uint32_t s_cpre[RT_G + 1];      // 64-candidate chunks before each pair (this tile)
  const int64_t blk = blockIdx.x;
  if (blk >= (int64_t)a.lcnt[a.nlist]) return;
  if (threadIdx.x < RT_G) {
    const uint64_t e = a.lpairs[blk * RT_G + threadIdx.x];
    const int q = e == RT_NO_PAIR ? -1 : (int32_t)(e >> 32);
    s_q[threadIdx.x] = q;
    s_r[threadIdx.x] = (int32_t)(e & 0xffffffffu);
    s_co[threadIdx.x] = q >= 0 ? a.cand_off[q] : 0;
  }
  __syncthreads();
  // the group's first pair is always a real one (padding ends a segment)
  const int L = a.probe_lists[a.probe_off[s_q[0]] + s_r[0]];
  const int64_t lb = a.list_off[L], le = a.list_off[L + 1];
  const int TR = 1 << a.tshift;
  const int ntile = (int)((le - lb + TR - 1) >> a.tshift);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // 8 lanes per candidate: lane p of an octet holds the virtual lanes
  // (four-element chunks) p, p + 8, p + 16 and p + 24 of the canonical sum
  const int oct = lane >> 3, p = lane & 7;
  const int nchunk = a.d >> 2;
  const bool ip = a.metric != 0;
  const int B = a.nbin;
  const int row_words = a.d * (int)sizeof(T) / 16;  // 16-byte words per row
  const T* trow = reinterpret_cast<const T*>(tile);
  const uint4* src = reinterpret_cast<const uint4*>(a.vectors) + lb * row_words;
  for (int t = 0; t < ntile; ++t) {
    const int64_t r0 = (int64_t)t * TR;
    const int nr = (int)min((int64_t)TR, le - lb - r0);
    const int bin = min(t, B - 1);
    __syncthreads();  // the previous tile is no longer read
    {
      // the tile's rows, two loads in flight per thread
      const int nw = nr * row_words;
      const uint4* sw = src + r0 * row_words;
      for (int w = threadIdx.x; w < nw; w += 2 * NT) {
        const int w2 = w + NT;
        const uint4 v0 = sw[w];
        const uint4 v1 = w2 < nw ? sw[w2] : make_uint4(0u, 0u, 0u, 0u);
        tile[w] = v0;
        if (w2 < nw) tile[w2] = v1;
      }
    }
    if (threadIdx.x < 64) {
      // each pair's candidates in this tile's bin, cut into 64-candidate
      // chunks (RT_G / 64 consecutive pairs per lane)
      constexpr int EPL = RT_G / 64;
      uint32_t nc[EPL], tot = 0;
#pragma unroll
      for (int h = 0; h < EPL; ++h) {
        const int e = EPL * (int)threadIdx.x + h;
        uint32_t b0 = 0, b1 = 0;
        if (s_q[e] >= 0) {
          const uint32_t* bb = a.bin_beg + (a.probe_off[s_q[e]] + s_r[e]) * (B + 1);
          b0 = bb[bin];
          b1 = bb[bin + 1];
        }
        s_beg[e] = b0;
        s_end[e] = b1;
        nc[h] = (b1 - b0 + 63) / 64;
        tot += nc[h];
      }
      uint32_t run = wave_incl_scan(tot) - tot;
#pragma unroll
      for (int h = 0; h < EPL; ++h) {
        s_cpre[EPL * threadIdx.x + h] = run;
        run += nc[h];
      }
      if (threadIdx.x == 63) s_cpre[RT_G] = run;
    }
    __syncthreads();
    const uint32_t nchk = s_cpre[RT_G];
    for (uint32_t c = wv; c < nchk; c += NW) {
      int e = 0;  // the pair holding chunk c
#pragma unroll
      for (int step = RT_G / 2; step >= 1; step >>= 1)
        if (s_cpre[e + step] <= c) e += step;
      const uint32_t j0 = s_beg[e] + (c - s_cpre[e]) * 64;
      const int cnt = (int)min(64u, s_end[e] - j0);
      const int q = s_q[e];
      const int64_t co = s_co[e];
      // lane l: candidate l's position, id and row in the tile (-1: none)
      const uint32_t pl = lane < cnt ? a.sorted_pos[co + j0 + lane] : 0u;
      const int64_t rl = (int64_t)pl - lb - r0;
      const bool okl = lane < cnt && rl >= 0 && rl < nr;
      const int32_t idl = okl ? a.list_ids[pl] : 0;
      const int rowl = okl ? (int)rl : -1;
      float4 qv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int v = p + 8 * i;
        qv[i] = v < nchunk ? reinterpret_cast<const float4*>(a.q + (int64_t)q * a.d)[v] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      float mykey = 0.0f;
      for (int it = 0; it * 8 < cnt; ++it) {
        const int rr = __shfl(rowl, it * 8 + oct);  // this octet's candidate
        float acc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int v = p + 8 * i;
          float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
          if (rr >= 0 && v < nchunk) xv = load4<T>(trow + (int64_t)rr * a.d, v);
          acc[i] = ip ? chunk_ip(qv[i], xv, 0.0f) : chunk_l2(qv[i], xv, 0.0f);
        }
        // levels 16 and 8 within the lane, 4 across lanes p and p + 4,
        // 2 and 1 within quads; lane p = 0 ends with the canonical sum
        float sum = (acc[0] + acc[2]) + (acc[1] + acc[3]);
        sum = sum + __shfl_xor(sum, 4);
        sum = sum + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sum), 0x4e, 0xf, 0xf, false));
        sum = sum + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sum), 0xb1, 0xf, 0xf, false));
        // candidate it * 8 + o's sum sits in lane 8 * o
        const float kk = __shfl(sum, 8 * (lane & 7));
        if ((lane >> 3) == it) mykey = ip ? -kk : kk;
      }
      if (okl) a.cand_packed[co + j0 + lane] = pack_key_id(mykey, (uint32_t)idl);
    }
  }
}

bool tile_rerank_shape(int d, int fp16, int64_t max_list, int max_np, int nlist, size_t max_lds, int max_bins,
                       int* tshift, int* nbin, size_t* sort_lds) {
  if (d <= 0 || d % 4 || d / 4 > 32 || nlist > QUERY_ORDER_MAX_LISTS || max_np <= 0) return false;
  const int64_t row_bytes = (int64_t)d * (fp16 ? 2 : 4);
  if (row_bytes % 16) return false;
  int ts = 0;
  while (((int64_t)2 << ts) * row_bytes <= RT_TILE_BYTES) ++ts;
  // one bin per tile of the longest list where the candidate sort's LDS
  // allows it (a shared last bin is read again for each of its tiles)
  const int64_t tiles = (max_list + ((int64_t)1 << ts) - 1) >> ts;
  int B = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), std::max(1, max_bins));
  auto lds_of = [&](int b) {
    return sizeof(uint32_t) * ((size_t)max_np * b + max_np) + sizeof(uint16_t) * (size_t)nlist;
  };
  while (B > 1 && lds_of(B) + 1024 > max_lds) --B;
  const size_t lds = lds_of(B);
  if (lds + 1024 > max_lds) return false;
  *tshift = ts;
  *nbin = B;
  *sort_lds = lds;
  return true;
}

hipError_t launch_tile_rerank(const TileRerankArgs& a, size_t sort_lds, hipStream_t s) {
  if (a.nq <= 0 || a.npairs <= 0) return hipSuccess;
  const dim3 pg((unsigned)((a.max_np + 255) / 256), (unsigned)a.nq);
  hipLaunchKernelGGL(rt_fill_u32, dim3((unsigned)std::min<int64_t>((a.nlist + 256) / 256, 1024)), dim3(256), 0, s,
                     a.lcnt, (int64_t)a.nlist + 1, 0u);
  hipLaunchKernelGGL(rt_fill_u64, dim3((unsigned)std::min<int64_t>((a.lpairs_cap + 255) / 256, 4096)), dim3(256), 0,
                     s, a.lpairs, a.lpairs_cap, RT_NO_PAIR);
  hipLaunchKernelGGL(rt_pair_count, pg, dim3(256), 0, s, a);
  hipLaunchKernelGGL(rt_pair_offsets, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(rt_pair_scatter, pg, dim3(256), 0, s, a);
  hipLaunchKernelGGL(rt_cand_sort, dim3((unsigned)a.nq), dim3(1024), sort_lds, s, a);
  const int64_t groups = (a.npairs + RT_G - 1) / RT_G + a.nlist;  // bound on the padded group count
  if (a.fp16) hipLaunchKernelGGL(rt_rerank_tile<__half>, dim3((unsigned)groups), dim3(1024), 0, s, a);
  else hipLaunchKernelGGL(rt_rerank_tile<float>, dim3((unsigned)groups), dim3(1024), 0, s, a);
  return hipGetLastError();
}

}  // namespace bbc

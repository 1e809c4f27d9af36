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
#include "bin_sort.h"
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
      pos[u] = r < row_end ? cpos[r] : EARLY_FLAG;
      xv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      // candidates re-ranked during the scan (EARLY_FLAG) are skipped
      if (!(pos[u] & EARLY_FLAG) && hl < nchunk) xv[u] = load4<T>(vec + (int64_t)pos[u] * a.d, hl);
    }
#pragma unroll
    for (int u = 0; u < RR_UNROLL; ++u) {
      float acc = ip ? chunk_ip(qc, xv[u], 0.0f) : chunk_l2(qc, xv[u], 0.0f);
      acc = canon_reduce32(acc);
      int64_t r = base + u;
      if (hl == 0 && !(pos[u] & EARLY_FLAG)) {
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
      pos[u] = r < row_end ? cpos[r] : EARLY_FLAG;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        int c = lane + 64 * st;
        xv[u][st] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (!(pos[u] & EARLY_FLAG) && c < nchunk) xv[u][st] = load4<T>(vec + (int64_t)pos[u] * a.d, c);
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
      if (lane == 0 && !(pos[u] & EARLY_FLAG)) {
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

// ---- Tile-major re-rank -------------------------------------------------------
// The per-query form reads every candidate row once per query that holds it.
// Here the batch's (query, probed list) pairs are grouped by list, a block
// takes one list and up to RT_G of the queries probing it, and it stages the
// list's rows in LDS one tile (1 << tshift rows) at a time: each row then
// comes from memory once per block instead of once per query.  Each query's
// candidates are first grouped by (probe rank, tile of the list) with a
// counting sort in LDS (one bin per tile of each probed list), so that a
// block finds the candidates of a (query, tile) as one range.  The distance
// of each candidate follows the canonical order, so the keys are identical
// to those of the per-query kernels.

constexpr uint64_t RT_NO_PAIR = ~0ull;

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
  const uint32_t G = (uint32_t)a.group;
  for (int L = threadIdx.x; L < a.nlist; L += 1024) a.lcnt[L] = (a.lcnt[L] + G - 1) / G * G;
  __syncthreads();
  block_excl_scan<1024>(a.lcnt, a.nlist, s_w, &s_tot);
  if (threadIdx.x == 0) a.lcnt[a.nlist] = s_tot / G;
}

__global__ __launch_bounds__(256) void rt_pair_scatter(TileRerankArgs a) {
  const int64_t q = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r < a.nprobe[q]) {
    const uint32_t slot = atomicAdd(&a.lcnt[a.probe_lists[a.probe_off[q] + r]], 1u);
    a.lpairs[slot] = ((uint64_t)q << 32) | (uint32_t)r;
  }
}

__device__ __forceinline__ int64_t rt_ncand(const TileRerankArgs& a, int64_t q) {
  return a.ncand_w ? (int64_t)a.ncand_w[q * a.ncand_stride] : a.n_cand[q];
}

// One block per query: its candidates grouped by bin = pair_tb[rank] + tile
// (one bin per tile of each probed list); bin_beg[bin_off[q] + b] = start of
// bin b within the query's candidates, [.. + nbins] = their count.  The bin
// counters live in LDS (max_bins of them); a query with more bins is sorted
// in consecutive rank ranges whose bins fit, one pair of passes each.
__global__ __launch_bounds__(1024) void rt_cand_sort(TileRerankArgs a) {
  constexpr int NT = 1024;
  extern __shared__ __align__(16) uint32_t sm[];
  __shared__ uint32_t s_w[16];
  __shared__ uint32_t s_tot, s_nb;
  const int64_t q = a.qorder ? (int64_t)a.qorder[blockIdx.x] : (int64_t)blockIdx.x;
  const int np = a.nprobe[q];
  const int64_t po = a.probe_off[q], pof = a.pos_off[q];
  const int64_t kc = rt_ncand(a, q);
  uint32_t* cnt = sm;                                                     // [max_bins]
  uint32_t* s_tb = sm + a.max_bins;                                       // [max_np] first bin of each rank
  int32_t* s_lbeg = reinterpret_cast<int32_t*>(s_tb + a.max_np);          // [max_np]
  uint16_t* rank_of = reinterpret_cast<uint16_t*>(s_lbeg + a.max_np);     // [nlist]
  for (int L = threadIdx.x; L < a.nlist; L += NT) rank_of[L] = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < np; r += NT) {
    const int L = a.probe_lists[po + r];
    rank_of[L] = (uint16_t)r;
    const int64_t lb = a.list_off[L];
    s_lbeg[r] = (int32_t)lb;
    s_tb[r] = (uint32_t)((a.list_off[L + 1] - lb + ((int64_t)1 << a.tshift) - 1) >> a.tshift);
  }
  __syncthreads();
  block_excl_scan<NT>(s_tb, np, s_w, &s_nb);
  const uint32_t nb = s_nb;  // bins of this query
  for (int r = threadIdx.x; r < np; r += NT) a.pair_tb[po + r] = s_tb[r];
  const uint32_t* cpos = a.cand_pos + pof;
  uint32_t* bb = a.bin_beg + a.bin_off[q];
  uint32_t* out = a.sorted_pos + pof;
  uint32_t* oidx = a.sorted_idx ? a.sorted_idx + pof : nullptr;
  auto rank_at = [&](uint32_t pos) { return min((int)rank_of[a.list_of_pos[pos]], np - 1); };
  uint32_t base = 0;  // candidates placed by the earlier rank ranges
  for (int rlo = 0; rlo < np;) {
    // ranks [rlo, rhi): the most whose bins fit in the counters (at least one:
    // a list's tiles never exceed them)
    int rhi = rlo + 1;
    while (rhi < np && (rhi + 1 < np ? s_tb[rhi + 1] : nb) - s_tb[rlo] <= (uint32_t)a.max_bins) ++rhi;
    const uint32_t b0 = s_tb[rlo], b1 = rhi < np ? s_tb[rhi] : nb;
    for (uint32_t i = threadIdx.x; i < b1 - b0; i += NT) cnt[i] = 0;
    __syncthreads();
    block_for_batched<NT, 4>(kc, [&](int64_t i) { return cpos[i]; }, [&](int64_t, bool valid, uint32_t pos) {
      if (!valid || (pos & EARLY_FLAG)) return;  // re-ranked during the scan
      const int r = rank_at(pos);
      if (r >= rlo && r < rhi) atomicAdd(&cnt[s_tb[r] - b0 + ((pos - (uint32_t)s_lbeg[r]) >> a.tshift)], 1u);
    });
    __syncthreads();
    block_excl_scan<NT>(cnt, (int)(b1 - b0), s_w, &s_tot);
    for (uint32_t i = threadIdx.x; i < b1 - b0; i += NT) {
      cnt[i] += base;
      bb[b0 + i] = cnt[i];
    }
    __syncthreads();
    block_for_batched<NT, 4>(kc, [&](int64_t i) { return cpos[i]; }, [&](int64_t i, bool valid, uint32_t pos) {
      if (!valid || (pos & EARLY_FLAG)) return;
      const int r = rank_at(pos);
      if (r >= rlo && r < rhi) {
        const uint32_t slot = atomicAdd(&cnt[s_tb[r] - b0 + ((pos - (uint32_t)s_lbeg[r]) >> a.tshift)], 1u);
        out[slot] = pos;
        if (oidx) oidx[slot] = (uint32_t)i;
      }
    });
    base += s_tot;
    rlo = rhi;
    __syncthreads();
  }
  if (threadIdx.x == 0) bb[nb] = base;  // the candidates placed (all but those re-ranked early)
}

// Two-round RaBitQ keys: whether candidate place `place` of query q is
// computed in the first round (the second round's keys are gathered by the
// device-wide grid of the wide form, not tile-major).
__device__ __forceinline__ bool rt_round_keep(const TileRerankArgs& a, int q, uint32_t place) {
  return a.round != 1 || place < a.wround[4 * (int64_t)q + 1];
}

// Shared by both tile kernels: the block's pairs (their queries, output and
// position offsets and first bins), loaded once per group.
struct RtGroup {
  int32_t q[RT_G], r[RT_G];
  int64_t co[RT_G], pof[RT_G];   // output and position offsets of the pair's query
  int64_t bbase[RT_G];           // the pair's first bin in bin_beg
};
// Per tile of rt_rerank_tile: each pair's candidates in the tile, the runs
// before each pair, the tile's 64-candidate runs (pair * 64 + run within
// the pair) when they fit the list, their number and the next unclaimed run.
constexpr int RT_RUNCAP = 1024;
struct RtTileBins {
  uint32_t beg[RT_G], end[RT_G];
  uint32_t rpre[RT_G + 1];
  uint16_t run[RT_RUNCAP];
  uint32_t next, nrun;
};

template <int NT>
__device__ __forceinline__ void rt_load_group(const TileRerankArgs& a, int64_t blk, RtGroup& g) {
  if (threadIdx.x < a.group) {
    const uint64_t e = a.lpairs[blk * a.group + threadIdx.x];
    const int q = e == RT_NO_PAIR ? -1 : (int32_t)(e >> 32);
    g.q[threadIdx.x] = q;
    g.r[threadIdx.x] = (int32_t)(e & 0xffffffffu);
    g.co[threadIdx.x] = q >= 0 ? a.cand_off[q] : 0;
    g.pof[threadIdx.x] = q >= 0 ? a.pos_off[q] : 0;
    g.bbase[threadIdx.x] = q >= 0 ? a.bin_off[q] + a.pair_tb[a.probe_off[q] + g.r[threadIdx.x]] : 0;
  }
}

// rows [r0, r0 + nr) of the list into LDS, two loads in flight per thread
template <int NT>
__device__ __forceinline__ void rt_stage_rows(uint4* tile, const uint4* sw, int nw) {
  for (int w = threadIdx.x; w < nw; w += 2 * NT) {
    const int w2 = w + NT;
    const uint4 v0 = sw[w];
    const uint4 v1 = w2 < nw ? sw[w2] : make_uint4(0u, 0u, 0u, 0u);
    tile[w] = v0;
    if (w2 < nw) tile[w2] = v1;
  }
}

// Rows of at most 32 chunks: 8 lanes per candidate, lane p of an octet
// holding the virtual lanes (four-element chunks) u, u + 8, u + 16 and u + 24
// of the canonical sum, u = p for p < 4 and 11 - p otherwise, so that the
// tree's level 4 pairs lanes p and 7 - p (a DPP half-row mirror) and levels
// 2 and 1 stay within quads; every lane of the octet ends with the sum.  A
// candidate's four chunk reads are issued together (clamped to the row;
// chunks past it count as zero).  IP: the metric is inner product.  NC: the
// row's chunk count when fixed at compile time (32 or 24: no clamps and no
// selects, constant row stride), 0 for any count up to 32.
//
// Per tile, wave 0 reads every pair's bin bounds (one batch of loads) and
// lists the tile's runs of up to 64 candidates of one pair; each wave then
// claims runs one at a time (an LDS counter, the next claim issued before
// the current run's work), so that a pair with many candidates in the tile
// spreads over several waves.  The run's pair, query row and bin bounds are
// wave-uniform (scalar registers).  A tile with more runs than the list
// holds finds each claimed run's pair by a binary search over the runs
// before each pair.
template <typename T, bool IP, int NC>
__global__ __launch_bounds__(1024, 8) void rt_rerank_tile(TileRerankArgs a) {
  constexpr int NT = 1024;
  __shared__ uint4 tile[RT_TILE_BYTES / 16];
  __shared__ RtGroup g;
  __shared__ RtTileBins tb;
  const int64_t blk = blockIdx.x;
  if (blk >= (int64_t)a.lcnt[a.nlist]) return;
  rt_load_group<NT>(a, blk, g);
  __syncthreads();
  // the group's first pair is always a real one (padding ends a segment)
  const int L = a.probe_lists[a.probe_off[g.q[0]] + g.r[0]];
  const int64_t lb = a.list_off[L], le = a.list_off[L + 1];
  const int TR = 1 << a.tshift;
  const int ntile = (int)((le - lb + TR - 1) >> a.tshift);
  const int lane = threadIdx.x & 63;
  auto claim = [&]() {
    uint32_t c = 0u;
    if (lane == 0) c = atomicAdd(&tb.next, 1u);
    return (int)uniform(__shfl(c, 0));
  };
  const int oct = lane >> 3, p = lane & 7;
  const int vb = p < 4 ? p : 11 - p;
  const int kaddr = 4 * (8 * (lane & 7));  // byte address of lane 8 (l mod 8), which holds candidate l's sum
  static_assert(NC == 0 || NC == 32 || NC == 24, "fixed chunk counts");
  const int nchunk = NC ? NC : a.d >> 2;
  const int d = 4 * nchunk;
  const int row_words = d * (int)sizeof(T) / 16;  // 16-byte words per row
  const T* trow = reinterpret_cast<const T*>(tile);
  const uint4* src = reinterpret_cast<const uint4*>(a.vectors) + lb * row_words;
  for (int t = 0; t < ntile; ++t) {
    const int64_t r0 = (int64_t)t * TR;
    const int nr = (int)min((int64_t)TR, le - lb - r0);
    const uint32_t pbase = (uint32_t)(lb + r0);  // list position of the tile's first row
    __syncthreads();  // the previous tile is no longer read, nor its bins and counter
    if (threadIdx.x < 64) {
      constexpr int EPL = RT_G / 64;
      uint32_t b0[EPL], b1[EPL], nrh[EPL], tot = 0u;
#pragma unroll
      for (int h = 0; h < EPL; ++h) {
        const int e = EPL * (int)threadIdx.x + h;
        b0[h] = b1[h] = 0u;
        if (g.q[e] >= 0) {
          const uint32_t* bb = a.bin_beg + g.bbase[e] + t;
          b0[h] = bb[0];
          b1[h] = bb[1];
        }
      }
#pragma unroll
      for (int h = 0; h < EPL; ++h) {
        tb.beg[EPL * threadIdx.x + h] = b0[h];
        tb.end[EPL * threadIdx.x + h] = b1[h];
        nrh[h] = b1[h] > b0[h] ? (b1[h] - b0[h] + 63u) / 64u : 0u;
        tot += nrh[h];
      }
      const uint32_t incl = wave_incl_scan(tot);
      const uint32_t total = __shfl(incl, 63);
      {
        uint32_t at = incl - tot;
#pragma unroll
        for (int h = 0; h < EPL; ++h) {
          tb.rpre[EPL * threadIdx.x + h] = at;
          at += nrh[h];
        }
        if (threadIdx.x == 63) tb.rpre[RT_G] = at;
      }
      if (total <= (uint32_t)RT_RUNCAP) {
        uint32_t at = incl - tot;
#pragma unroll
        for (int h = 0; h < EPL; ++h) {
          const uint32_t u0 = (EPL * threadIdx.x + h) * 64;
#pragma nounroll
          for (uint32_t k = 0; k < nrh[h]; ++k) tb.run[at + k] = (uint16_t)(u0 + k);
          at += nrh[h];
        }
      }
      if (threadIdx.x == 0) {
        tb.next = 0u;
        tb.nrun = total;
      }
    }
    rt_stage_rows<NT>(tile, src + r0 * row_words, nr * row_words);
    __syncthreads();
    // this lane's chunks of query q's row
    auto load_q = [&](int q, float4 (&qv)[4]) {
      const float4* qrow = reinterpret_cast<const float4*>(a.q + (int64_t)q * d);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int v = vb + 8 * i;
        qv[i] = v < nchunk ? qrow[v] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    // the candidates [j0, j0 + cnt) of pair e (query q), cnt <= 64
    auto run = [&](int e, int q, uint32_t j0, int cnt, const float4 (&qv)[4]) {
      const int64_t co = uniform(g.co[e]), pof = uniform(g.pof[e]);
      const uint32_t keep_below = a.round == 1 ? uniform(a.wround[4 * (int64_t)q + 1]) : 0xffffffffu;
      {
        // lane l: candidate l's position, id, output index and row in the tile (-1: none)
        const uint32_t pl = lane < cnt ? a.sorted_pos[pof + j0 + lane] : 0u;
        const uint32_t rl = pl - pbase;
        bool okl = lane < cnt && rl < (uint32_t)nr;
        const uint32_t oil = !okl ? 0u : (a.sorted_idx ? a.sorted_idx[pof + j0 + lane] : j0 + lane);
        okl = okl && oil < keep_below;
        const int32_t idl = okl ? a.list_ids[pl] : 0;
        const int rowl = okl ? (int)rl : -1;
        float mykey = 0.0f;
        for (int it = 0; it * 8 < cnt; ++it) {
          const int rr = __shfl(rowl, it * 8 + oct);  // this octet's candidate (-1: none, row 0 read)
          const T* row = trow + max(rr, 0) * d;
          float acc[4];
          if (NC == 32) {
            float4 x[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) x[i] = load4<T>(row, vb + 8 * i);
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = IP ? chunk_ip(qv[i], x[i], 0.0f) : chunk_l2_0(qv[i], x[i]);
          } else if (NC == 24) {
            // virtual lanes 24..31 hold no chunk: their sums are +0
            float4 x[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) x[i] = load4<T>(row, vb + 8 * i);
#pragma unroll
            for (int i = 0; i < 3; ++i) acc[i] = IP ? chunk_ip(qv[i], x[i], 0.0f) : chunk_l2_0(qv[i], x[i]);
            acc[3] = 0.0f;
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float4 xl = load4<T>(row, min(vb + 8 * i, nchunk - 1));
              const float4 x = vb + 8 * i < nchunk ? xl : make_float4(0.f, 0.f, 0.f, 0.f);
              acc[i] = IP ? chunk_ip(qv[i], x, 0.0f) : chunk_l2(qv[i], x, 0.0f);
            }
          }
          // levels 16 and 8 within the lane, 4 across lanes p and 7 - p
          // (half-row mirror), 2 and 1 within quads
          // (rows of 24 chunks, L2: acc[3] is +0 and acc[1] never -0)
          float sum = (acc[0] + acc[2]) + (NC == 24 && !IP ? acc[1] : acc[1] + acc[3]);
          sum = sum + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sum), 0x141, 0xf, 0xf, false));
          sum = sum + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sum), 0x4e, 0xf, 0xf, false));
          sum = sum + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sum), 0xb1, 0xf, 0xf, false));
          // candidate it * 8 + o's sum sits in lane 8 * o
          const float kk = __int_as_float(__builtin_amdgcn_ds_bpermute(kaddr, __float_as_int(sum)));
          if ((lane >> 3) == it) mykey = IP ? -kk : kk;
        }
        if (okl) a.cand_packed[co + oil] = pack_key_id(mykey, (uint32_t)idl);
      }
    };
    const uint32_t nrun = uniform(tb.nrun);
    const bool listed = nrun <= (uint32_t)RT_RUNCAP && !a.no_run_list;
    for (int c = claim(); c < (int)nrun;) {
      const int c_next = claim();
      int e;
      uint32_t k;
      if (listed) {
        const uint32_t u = uniform((uint32_t)tb.run[c]);
        e = (int)(u >> 6);
        k = u & 63u;
      } else {
        e = 0;
#pragma unroll
        for (int step = RT_G / 2; step >= 1; step >>= 1)
          if (uniform(tb.rpre[e + step]) <= (uint32_t)c) e += step;
        k = (uint32_t)c - uniform(tb.rpre[e]);
      }
      const int q = uniform(g.q[e]);
      const uint32_t j0 = uniform(tb.beg[e]) + 64u * k, b1 = uniform(tb.end[e]);
      float4 qv[4];
      load_q(q, qv);
      run(e, q, j0, (int)min(64u, b1 - j0), qv);
      c = c_next;
    }
  }
}

// canon_reduce64 without LDS permutes.  Levels 32 and 16: swapping the
// upper half of one copy with the lower half of another (v_permlane32_swap),
// or the odd 16-lane rows of one with the even rows of another
// (v_permlane16_swap), leaves lane l with its own value in one output and
// lane l ^ 32 (l ^ 16) in the other, so their sum is the tree's pair sum.
// The last four levels as DPP: after the xor levels 32 and 16 every lane's
// value repeats with period 16, after the rotation by 8 with period 8, so
// each rotation pairs lane l with the lane the canonical tree pairs it with
// whichever way it turns, and every lane ends with the canonical sum.
__device__ __forceinline__ float canon_reduce64_dpp(float acc) {
  const auto s32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc), __float_as_uint(acc), false, false);
  acc = __uint_as_float(s32[0]) + __uint_as_float(s32[1]);
  const auto s16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(acc), __float_as_uint(acc), false, false);
  acc = __uint_as_float(s16[0]) + __uint_as_float(s16[1]);
  acc = acc + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), 0x128, 0xf, 0xf, false));  // row_ror:8
  acc = acc + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), 0x124, 0xf, 0xf, false));  // row_ror:4
  acc = acc + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), 0x4e, 0xf, 0xf, false));   // quad [2,3,0,1]
  acc = acc + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), 0xb1, 0xf, 0xf, false));   // quad [1,0,3,2]
  return acc;
}

// Rows of 33 to 256 chunks (groups of RT_GW pairs): wave w takes pair w of
// the group and keeps its query chunks in registers over all the list's
// tiles (lane l holds chunks l, l + 64, l + 128 and l + 192, the canonical
// steps of virtual lane l); one candidate row at a time, from LDS, its four
// chunk reads issued together (lanes past the row's chunks read its last
// chunk and leave their sum as it is).  IP: the metric is inner product.
template <typename T, bool IP>
__global__ __launch_bounds__(1024, 4) void rt_rerank_tile_wide(TileRerankArgs a) {
  constexpr int NT = 1024;
  static_assert(RT_GW == NT / 64, "one pair per wave");
  __shared__ uint4 tile[RT_TILE_BYTES / 16];
  __shared__ RtGroup g;
  const int64_t blk = blockIdx.x;
  if (blk >= (int64_t)a.lcnt[a.nlist]) return;
  rt_load_group<NT>(a, blk, g);
  __syncthreads();
  const int L = a.probe_lists[a.probe_off[g.q[0]] + g.r[0]];
  const int64_t lb = a.list_off[L], le = a.list_off[L + 1];
  const int TR = 1 << a.tshift;
  const int ntile = (int)((le - lb + TR - 1) >> a.tshift);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nchunk = a.d >> 2;
  const int row_words = a.d * (int)sizeof(T) / 16;
  const T* trow = reinterpret_cast<const T*>(tile);
  const uint4* src = reinterpret_cast<const uint4*>(a.vectors) + lb * row_words;
  const int q = g.q[wv];
  const int64_t co = g.co[wv], pof = g.pof[wv];
  const uint32_t* bins = a.bin_beg + g.bbase[wv];
  float4 qv[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int c4 = lane + 64 * st;
    qv[st] = q >= 0 && c4 < nchunk ? reinterpret_cast<const float4*>(a.q + (int64_t)q * a.d)[c4]
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  for (int t = 0; t < ntile; ++t) {
    const int64_t r0 = (int64_t)t * TR;
    const int nr = (int)min((int64_t)TR, le - lb - r0);
    // this pair's candidates in tile t (loaded before the tile's rows)
    const uint32_t b0 = q >= 0 ? bins[t] : 0u, b1 = q >= 0 ? bins[t + 1] : 0u;
    __syncthreads();
    rt_stage_rows<NT>(tile, src + r0 * row_words, nr * row_words);
    __syncthreads();
    for (uint32_t j0 = b0; j0 < b1; j0 += 64) {
      const int cnt = (int)min(64u, b1 - j0);
      const uint32_t pl = lane < cnt ? a.sorted_pos[pof + j0 + lane] : 0u;
      const int64_t rl = (int64_t)pl - lb - r0;
      bool okl = lane < cnt && rl >= 0 && rl < nr;
      const uint32_t oil = !okl ? 0u : (a.sorted_idx ? a.sorted_idx[pof + j0 + lane] : j0 + lane);
      okl = okl && rt_round_keep(a, q, oil);
      const int32_t idl = okl ? a.list_ids[pl] : 0;
      const int rowl = okl ? (int)rl : -1;
      float mykey = 0.0f;
      for (int jj = 0; jj < cnt; ++jj) {
        const int rr = __builtin_amdgcn_readlane(rowl, jj);
        if (rr < 0) continue;  // wave-uniform
        const T* row = trow + (int64_t)rr * a.d;
        float4 xv[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) xv[st] = load4<T>(row, min(lane + 64 * st, nchunk - 1));
        float acc = 0.0f;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const float nx = IP ? chunk_ip(qv[st], xv[st], acc) : chunk_l2(qv[st], xv[st], acc);
          acc = lane + 64 * st < nchunk ? nx : acc;
        }
        acc = canon_reduce64_dpp(acc);  // every lane ends with the sum
        if (lane == jj) mykey = IP ? -acc : acc;
      }
      if (okl) a.cand_packed[co + oil] = pack_key_id(mykey, (uint32_t)idl);
    }
  }
}

int tile_rerank_group(int d) { return d / 4 > 32 ? RT_GW : RT_G; }

int tile_rerank_shift(int d, int fp16) {
  if (d <= 0 || d % 4 || d / 4 > 256) return -1;
  const int64_t row_bytes = (int64_t)d * (fp16 ? 2 : 4);
  if (row_bytes % 16 || row_bytes > RT_TILE_BYTES) return -1;
  int ts = 0;
  while (((int64_t)2 << ts) * row_bytes <= RT_TILE_BYTES) ++ts;
  return ts;
}

size_t tile_rerank_sort_lds(int max_bins, int max_np, int nlist) {
  return sizeof(uint32_t) * ((size_t)max_bins + 2 * (size_t)max_np) + sizeof(uint16_t) * (size_t)nlist;
}

// the list sort's binner: bin = list; slot -> (query << 32 | rank)
struct TilePairBins {
  const int32_t* nprobe; const int32_t* probe_lists; uint64_t* lpairs;
  __device__ int64_t count(int64_t q) const { return nprobe[q]; }
  __device__ int bin(int64_t, int, int64_t p) const { return probe_lists[p]; }
  __device__ void put(uint32_t slot, int64_t q, int r, int64_t) const {
    lpairs[slot] = ((uint64_t)q << 32) | (uint32_t)r;
  }
};

hipError_t launch_tile_pairs(const TileRerankArgs& a, hipStream_t s) {
  if (a.nq <= 0 || a.npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(rt_fill_u64, dim3((unsigned)std::min<int64_t>((a.lpairs_cap + 255) / 256, 4096)), dim3(256), 0,
                     s, a.lpairs, a.lpairs_cap, RT_NO_PAIR);
  if (a.bs_table && a.nlist <= BS_MAX_BINS) {
    const TilePairBins f{a.nprobe, a.probe_lists, a.lpairs};
    bs_sort(f, a.nlist, a.nq, a.probe_off, a.bs_table, a.lcnt, [&] {
      hipLaunchKernelGGL(rt_pair_offsets, dim3(1), dim3(1024), 0, s, a);
    }, s);
    return hipGetLastError();
  }
  const dim3 pg((unsigned)((a.max_np + 255) / 256), (unsigned)a.nq);
  hipLaunchKernelGGL(rt_fill_u32, dim3((unsigned)std::min<int64_t>((a.nlist + 256) / 256, 1024)), dim3(256), 0, s,
                     a.lcnt, (int64_t)a.nlist + 1, 0u);
  hipLaunchKernelGGL(rt_pair_count, pg, dim3(256), 0, s, a);
  hipLaunchKernelGGL(rt_pair_offsets, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(rt_pair_scatter, pg, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
static void launch_rt_tile(bool ip, int nc, dim3 grid, dim3 block, hipStream_t s, const TileRerankArgs& a) {
  if (ip) {
    if (nc == 32) hipLaunchKernelGGL((rt_rerank_tile<T, true, 32>), grid, block, 0, s, a);
    else if (nc == 24) hipLaunchKernelGGL((rt_rerank_tile<T, true, 24>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((rt_rerank_tile<T, true, 0>), grid, block, 0, s, a);
  } else {
    if (nc == 32) hipLaunchKernelGGL((rt_rerank_tile<T, false, 32>), grid, block, 0, s, a);
    else if (nc == 24) hipLaunchKernelGGL((rt_rerank_tile<T, false, 24>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((rt_rerank_tile<T, false, 0>), grid, block, 0, s, a);
  }
}

hipError_t launch_tile_rerank(const TileRerankArgs& a, size_t sort_lds, hipStream_t s) {
  if (a.nq <= 0 || a.npairs <= 0) return hipSuccess;
  if (!a.pairs_ready) {
    const hipError_t e = launch_tile_pairs(a, s);
    if (e != hipSuccess) return e;
  }
  if (!a.presorted) hipLaunchKernelGGL(rt_cand_sort, dim3((unsigned)a.nq), dim3(1024), sort_lds, s, a);
  const int64_t groups = (a.npairs + a.group - 1) / a.group + a.nlist;  // bound on the padded group count
  const bool wide = a.d / 4 > 32;
  if (wide) {
    const bool ip = a.metric != 0;
    if (a.fp16) {
      if (ip) hipLaunchKernelGGL((rt_rerank_tile_wide<__half, true>), dim3((unsigned)groups), dim3(1024), 0, s, a);
      else hipLaunchKernelGGL((rt_rerank_tile_wide<__half, false>), dim3((unsigned)groups), dim3(1024), 0, s, a);
    } else {
      if (ip) hipLaunchKernelGGL((rt_rerank_tile_wide<float, true>), dim3((unsigned)groups), dim3(1024), 0, s, a);
      else hipLaunchKernelGGL((rt_rerank_tile_wide<float, false>), dim3((unsigned)groups), dim3(1024), 0, s, a);
    }
    return hipGetLastError();
  }
  const bool ip = a.metric != 0;
  const int nc = a.d / 4 == 32 ? 32 : a.d / 4 == 24 ? 24 : 0;
  const dim3 grid((unsigned)groups), block(1024);
  if (a.fp16) launch_rt_tile<__half>(ip, nc, grid, block, s, a);
  else launch_rt_tile<float>(ip, nc, grid, block, s, a);
  return hipGetLastError();
}

}  // namespace bbc

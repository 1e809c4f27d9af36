// Counting sort of a batch's (query, probe rank) pairs into bins (lists, or
// (phase, list) for the scan), each bin padded to a whole number of groups.
//
// Every pair of a query names a different list, so the pairs of one wave
// never collide on a bin, but all of a batch's pairs land on a few thousand
// bins: counting them with device-wide atomics queues about a thousand
// read-modify-writes on each bin's word.  Here each block counts the pairs
// of 32 consecutive queries in an LDS histogram and stores it as one column
// of a bin-major table (no global atomics); one wave per bin turns its row
// into the exclusive prefix over the blocks and the bin's total; the bin
// totals are padded and scanned by the caller's offsets kernel; and each
// block places its pairs with LDS atomics from its own column.  The order of
// the pairs inside a bin is not fixed (nor is it with global atomics): every
// consumer keys its results by pair, not by slot.
//
// A binner F provides, for pair p = probe_off[q] + r of query q:
//   int64_t count(q)             pairs of query q
//   int bin(q, r, p)             its bin, in [0, nbins)
//   void put(slot, q, r, p)      store the pair at its sorted slot
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace bbc {

constexpr int BS_QB = 32;             // queries per block (two per wave of 1024 threads)
constexpr int BS_MAX_BINS = 16384;    // LDS histogram of 64 KB; more bins take global atomics

__host__ __device__ inline int64_t bs_blocks(int64_t nq) { return (nq + BS_QB - 1) / BS_QB; }
// words of the per-block count table (0 when the bins do not fit in LDS)
inline int64_t bs_table_words(int64_t nq, int nbins) {
  return nbins <= BS_MAX_BINS ? bs_blocks(nq) * (int64_t)nbins : 0;
}

template <class F>
__global__ __launch_bounds__(1024) void bs_count(F f, int nbins, int64_t nq, const int64_t* __restrict__ probe_off,
                                                 uint32_t* __restrict__ table) {
  extern __shared__ uint32_t bs_h[];
  for (int b = threadIdx.x; b < nbins; b += 1024) bs_h[b] = 0u;
  __syncthreads();
  const int64_t c = blockIdx.x, nb = gridDim.x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t qe = min(nq, (c + 1) * BS_QB);
  for (int64_t q = c * BS_QB + wv; q < qe; q += 16) {
    const int64_t p0 = probe_off[q], n = f.count(q);
    for (int64_t r = lane; r < n; r += 64) atomicAdd(&bs_h[f.bin(q, (int)r, p0 + r)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += 1024) table[(int64_t)b * nb + c] = bs_h[b];
}

// one wave per bin: its row of block counts -> exclusive prefix, total -> tot[b]
static __global__ __launch_bounds__(1024) void bs_rows(uint32_t* __restrict__ table, int nbins, int64_t nblk,
                                                uint32_t* __restrict__ tot) {
  const int64_t b = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 6);
  if (b >= nbins) return;
  const int lane = threadIdx.x & 63;
  uint32_t* row = table + b * nblk;
  uint32_t run = 0;
  for (int64_t c0 = 0; c0 < nblk; c0 += 64) {
    const int64_t c = c0 + lane;
    const uint32_t v = c < nblk ? row[c] : 0u;
    const uint32_t incl = wave_incl_scan(v);
    if (c < nblk) row[c] = run + incl - v;
    run += __shfl(incl, 63);
  }
  if (lane == 0) tot[b] = run;
}

// start[b]: the bin's first slot (the caller's offsets kernel wrote it over tot)
template <class F>
__global__ __launch_bounds__(1024) void bs_place(F f, int nbins, int64_t nq, const int64_t* __restrict__ probe_off,
                                                 const uint32_t* __restrict__ table,
                                                 const uint32_t* __restrict__ start) {
  extern __shared__ uint32_t bs_h[];
  const int64_t c = blockIdx.x, nb = gridDim.x;
  for (int b = threadIdx.x; b < nbins; b += 1024) bs_h[b] = start[b] + table[(int64_t)b * nb + c];
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t qe = min(nq, (c + 1) * BS_QB);
  for (int64_t q = c * BS_QB + wv; q < qe; q += 16) {
    const int64_t p0 = probe_off[q], n = f.count(q);
    for (int64_t r = lane; r < n; r += 64) {
      const uint32_t slot = atomicAdd(&bs_h[f.bin(q, (int)r, p0 + r)], 1u);
      f.put(slot, q, (int)r, p0 + r);
    }
  }
}

// Counts per bin into tot[0, nbins) (the caller then turns them into padded
// starts in place, in the same array), then the placement.  `table` holds
// bs_table_words(nq, nbins) words.
template <class F, class Offsets>
inline void bs_sort(const F& f, int nbins, int64_t nq, const int64_t* probe_off, uint32_t* table, uint32_t* tot,
                    Offsets offsets, hipStream_t s) {
  const int64_t nblk = bs_blocks(nq);
  const size_t lds = sizeof(uint32_t) * (size_t)nbins;
  hipLaunchKernelGGL(bs_count<F>, dim3((unsigned)nblk), dim3(1024), lds, s, f, nbins, nq, probe_off, table);
  hipLaunchKernelGGL(bs_rows, dim3((unsigned)((nbins + 15) / 16)), dim3(1024), 0, s, table, nbins, nblk, tot);
  offsets();
  hipLaunchKernelGGL(bs_place<F>, dim3((unsigned)nblk), dim3(1024), lds, s, f, nbins, nq, probe_off, table, tot);
}

}  // namespace bbc

// PQ estimated distances (background section: quantization methods
// precompute query-to-codeword distances and sum them per code; IVF+PQ uses
// residual codes, one table per (query, probed list)).
//
// Table entry LUT[m][b] = sum_e ((q_e - c_e) - C_m[b][e])^2 with r = q - c
// computed once per element and the sum taken sequentially over the
// sub-vector (unfused); key = sum_m LUT[m][code_m] in order from +0.  Keys go
// to the per-query key scratch in probe order, nearest list first.
//
// Scheduling.  The (query, probe rank) pairs are first counting-sorted by
// (phase, list): the codebook-sample lists of every query first, then the
// rest; each bin is padded to a multiple of SCAN_GROUP.  A persistent block
// then takes SCAN_GROUP pairs of one list at a time -- up to four queries
// probing the same list -- and builds their four tables side by side in LDS
// ([m][code][query]): every code byte is extracted once and one 16-byte LDS
// read yields the four queries' entries, each query keeping its own ordered
// sum.  Each XCD walks one contiguous slice of the sorted groups (workgroups
// are dispatched round-robin over the XCDs), so the queries of a list are
// served while its codes sit in that XCD's L2.  Thread t builds table
// entries t, t+1024, ... reading their codewords from L2.
#include <algorithm>

#include "common.h"
#include "bin_sort.h"
#include "kernels.h"

namespace bbc {

constexpr uint32_t NO_PAIR = 0xffffffffu;

__device__ __forceinline__ int64_t find_query(const int64_t* __restrict__ off, int64_t nq, int64_t p) {
  // largest qi with off[qi] <= p (off is non-decreasing, off[0] = 0)
  int64_t lo = 0, hi = nq - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---- pair sort by list --------------------------------------------------------
__global__ void zero_u32_kernel(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}

__device__ __forceinline__ int pair_bin(const PqScanArgs& a, int64_t p) {
  const int64_t qi = find_query(a.probe_off, a.nq, p);
  const int rank = (int)(p - a.probe_off[qi]);
  return (rank >= a.nsample_q[qi] ? a.nlist : 0) + a.probe_lists[p];
}

__global__ void pair_count_kernel(PqScanArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.npairs; p += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&a.pair_cnt[pair_bin(a, p)], 1u);
}

// In place: per-bin counts -> exclusive prefix of the counts rounded up to a
// multiple of the scan's group size (one block).  Also records the start of the second
// phase (bin nlist) and the padded total in split[0], split[1].
__global__ __launch_bounds__(1024) void pair_offsets_kernel(uint32_t* __restrict__ cnt_fill, int nbins, int nlist,
                                                            int group, uint32_t* __restrict__ split) {
  __shared__ uint32_t carry_s;
  __shared__ uint32_t wsum[16];
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int base = 0; base < nbins; base += 1024) {
    const int j = base + threadIdx.x;
    uint32_t v = j < nbins ? (cnt_fill[j] + group - 1) / group * group : 0u;
    uint32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
      uint32_t o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = carry_s;
    for (int i = 0; i < w; ++i) before += wsum[i];
    if (j < nbins) cnt_fill[j] = before + incl - v;
    if (j == nlist) split[0] = before + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry_s = before + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) split[1] = carry_s;
}

__global__ void pair_scatter_kernel(PqScanArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.npairs; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t qi = find_query(a.probe_off, a.nq, p);
    const int rank = (int)(p - a.probe_off[qi]);
    const int bin = (rank >= a.nsample_q[qi] ? a.nlist : 0) + a.probe_lists[p];
    const uint32_t slot = atomicAdd(&a.pair_cnt[bin], 1u);
    a.sorted_pairs[slot] = (uint32_t)p;
    a.sorted_q[slot] = (uint32_t)qi;
  }
}

// the pair sort's binner: bin (rank >= nsample, list); slot -> (pair, query)
struct ScanPairBins {
  const int64_t* probe_off; const int32_t* probe_lists; const int32_t* nsample_q; int nlist;
  uint32_t* sorted_pairs; uint32_t* sorted_q;
  __device__ int64_t count(int64_t q) const { return probe_off[q + 1] - probe_off[q]; }
  __device__ int bin(int64_t q, int r, int64_t p) const {
    return (r >= nsample_q[q] ? nlist : 0) + probe_lists[p];
  }
  __device__ void put(uint32_t slot, int64_t q, int, int64_t p) const {
    sorted_pairs[slot] = (uint32_t)p;
    sorted_q[slot] = (uint32_t)q;
  }
};

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Block-wide stream compaction for G output streams at once: every thread
// of the block calls step() with the keep flags of its O elements
// (keep[o * G + g]); each kept element gets the next slot of its stream, in
// (wave, element, lane) order within a call and call order across calls.  One
// barrier per call: each wave posts its counts packed two streams to a word
// (16 bits each: a call keeps at most NT * O < 65536 per stream), and lanes
// 0 .. NW-1 of every wave then read one wave's words each and scan them
// across lanes (DPP shifts within the first row).  The words are double
// buffered so consecutive calls need no second barrier.
template <int G, int NT, int O = 1>
struct BlockCompactor {
  static constexpr int NW = NT / 64;
  static constexpr int NPK = (G + 1) / 2;
  static_assert(NW <= 16 && NT * O < 65536, "one DPP row of waves, 16-bit counts");
  uint32_t total[G];
  int parity;
  __device__ __forceinline__ void reset() {
#pragma unroll
    for (int g = 0; g < G; ++g) total[g] = 0;
    parity = 0;
  }
  __device__ __forceinline__ void step(const bool* keep, uint32_t* slot, uint32_t (*wc)[NW][NPK]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t mask[O][G];
    uint32_t pk[NPK];
#pragma unroll
    for (int j = 0; j < NPK; ++j) pk[j] = 0u;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      uint32_t n = 0;
#pragma unroll
      for (int o = 0; o < O; ++o) {
        mask[o][g] = __ballot(keep[o * G + g]);
        n += (uint32_t)__popcll(mask[o][g]);
      }
      pk[g >> 1] |= n << (16 * (g & 1));
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < NPK; ++j) wc[parity][w][j] = pk[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NPK; ++j) {
      // inclusive scan of the waves' words over lanes 0 .. NW-1
      uint32_t v = lane < NW ? wc[parity][lane][j] : 0u;
      // row_shr:1, 2, 4, 8 (zero from before the row's start)
      v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);
      if (NW > 2) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);
      if (NW > 4) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
      if (NW > 8) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
      const uint32_t ex = w ? (uint32_t)__builtin_amdgcn_readlane((int)v, w - 1) : 0u;
      const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)v, NW - 1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int g = 2 * j + h;
        if (g < G) {
          uint32_t off = total[g] + ((ex >> (16 * h)) & 0xffffu);
#pragma unroll
          for (int o = 0; o < O; ++o) {
            slot[o * G + g] = off + (uint32_t)__popcll(mask[o][g] & below);
            off += (uint32_t)__popcll(mask[o][g]);
          }
          total[g] += (tot >> (16 * h)) & 0xffffu;
        }
      }
    }
    parity ^= 1;
  }
};

// Smallest and largest value over the 64 lanes of a wave, in every lane:
// lanes l and l ^ 32, l ^ 16 by lane swaps, then rotations by 8 and 4 within
// rows and the two quad steps, all without LDS.
__device__ __forceinline__ void wave_minmax(uint32_t& mn, uint32_t& mx) {
  auto s = __builtin_amdgcn_permlane32_swap(mn, mn, false, false);
  mn = min((uint32_t)s[0], (uint32_t)s[1]);
  s = __builtin_amdgcn_permlane32_swap(mx, mx, false, false);
  mx = max((uint32_t)s[0], (uint32_t)s[1]);
  s = __builtin_amdgcn_permlane16_swap(mn, mn, false, false);
  mn = min((uint32_t)s[0], (uint32_t)s[1]);
  s = __builtin_amdgcn_permlane16_swap(mx, mx, false, false);
  mx = max((uint32_t)s[0], (uint32_t)s[1]);
  mn = min(mn, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mn, 0x128, 0xf, 0xf, false));  // row_ror:8
  mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x128, 0xf, 0xf, false));
  mn = min(mn, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mn, 0x124, 0xf, 0xf, false));  // row_ror:4
  mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x124, 0xf, 0xf, false));
  mn = min(mn, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mn, 0x4e, 0xf, 0xf, false));   // quad [2,3,0,1]
  mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x4e, 0xf, 0xf, false));
  mn = min(mn, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mn, 0xb1, 0xf, 0xf, false));   // quad [1,0,3,2]
  mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0xb1, 0xf, 0xf, false));
}

// Per-query output of one scanned pair.  Phase 0 (sample lists) writes every
// key by slot; phase 1 keeps the keys at or below the query's relaxed
// threshold (all keys when the query does not reject) and writes them,
// compacted, with their list slot.
struct PairOut {
  float* sample_out;
  float* skey;
  uint32_t* spos;
  float* sexact;   // early re-rank: exact keys by survivor slot
  float* trace_out;
  uint32_t prune, dmax_bits, early_bits;
  // loads only (everything a pair's output needs), so that a group's outputs
  // can be fetched while the previous group is being scanned
  __device__ __forceinline__ void init(const PqScanArgs& a, int mode, int64_t qi, int64_t p) {
    const int64_t ro = uniform(a.rank_off[p]);
    trace_out = a.trace_keys ? uniform(a.trace_keys + a.key_off[qi] + ro) : nullptr;
    if (mode == 0) {
      sample_out = uniform(a.sample_keys + a.sample_off[qi] + ro);
      prune = 0;
      dmax_bits = 0;
    } else {
      const QueryBook* b = a.books + qi;
      prune = uniform(b->prune);
      dmax_bits = uniform(b->dmax_bits);
      early_bits = a.early ? uniform(b->early_bits) : 0u;
      const int64_t so = uniform(a.surv_off[qi]) + ro;
      skey = a.surv_key + so;
      spos = a.surv_pos + so;
      sexact = a.surv_exact ? a.surv_exact + so : nullptr;
    }
  }
  __device__ __forceinline__ bool keep(float key) const { return !prune || key_bits(key) <= dmax_bits; }
};

// ---- persistent grouped scan ----------------------------------------------------
// One block per CU walks the (list, 4 queries) groups of its XCD's slice.  Per
// group: the 4 residuals go to LDS, the 4 distance tables are built into one
// table of float4 rows (entry e holds e's value for the 4 queries, so one LDS
// read serves all 4), then each thread scans O codes of the list per pass,
// interleaved, to keep more table reads in flight per wave.  Block geometries
// (threads NT, codes per thread O) are compiled as variants: (512, 2), the
// default, (512, 1) and (1024, 1).
//
// One-byte tables (U8): after the float table is built, each (query,
// sub-space) gets its minimum lo_m and each query one step delta = (largest
// max - lo_m over the sub-spaces) / 255 and base = sum of lo_m; every entry
// becomes u = min(255, floor((entry - lo_m) * (1 / delta) + 0.5)).  An
// entry's row holds the group's codes in 16-bit halves of 32-bit words
// (queries 2h and 2h+1 in word h), so one 32-bit integer add accumulates two
// queries (sums stay below 2^16 for M < 257); the key is base + K * delta.
// Rows are written in place over the float rows (a one-byte row is half the
// size of a float row, so row e's bytes land inside float rows below e: each
// round of NT rows is read before a barrier and written after it).  4-bit
// shapes scan 8 queries per group (one 16-byte read per code serves all 8),
// 8-bit shapes 4 (their float staging table would not fit twice as wide).
//
// Early re-rank (EARLY, mode 1; Algorithm 4's improved IVF+PQ search): a
// survivor whose key image lies below its query's early_bits (its bucket is
// below the predicted threshold bucket) gets its exact key in the scan, right
// after its code: each wave takes its early (object, query) items two at a
// time (one per 32-lane half, chunk hl of the row on lane hl, the canonical
// lane order), four items per half per round so that their row loads are in
// flight together.  The survivor's list position carries EARLY_FLAG and its
// exact key goes to surv_exact at its slot.
//
// Sliced tables (SL = 2, 8-bit codes, float rows): the table holds the
// entries of M / SL sub-spaces at a time (64 KB for 32 sub-spaces), so two
// blocks share a CU and one's table build overlaps the other's lookups.  A
// group's codes are taken in chunks of up to PMAX passes; for each chunk the
// slices are built in sub-space order and every pass of the chunk adds the
// slice's entries to its running sums in registers, so each key is still
// summed over m = 0 .. M-1 in order.  Lists longer than one chunk rebuild
// the slices per chunk.
//
// BPC: blocks per CU (two: registers capped so that both fit).
template <int MODE, int BITS, int M, int DSUB, int NT, int O, bool U8, bool EARLY, int SL = 1, int PMAX = 1,
          int BPC = 1>
__global__ __launch_bounds__(NT, BPC * NT / 256) void pq_scan_grouped(PqScanArgs a) {
  constexpr int G = scan_group_of(U8, BITS);
  constexpr int KSUB = 1 << BITS;
  constexpr int NENT = M * KSUB;
  constexpr int EPT = (NENT + NT - 1) / NT;   // table entries owned by each thread
  constexpr bool REGCB = BPC == 1 && EPT * DSUB <= 64;  // owned codewords held in registers
  constexpr int D = M * DSUB;
  constexpr int CODE_BYTES = BITS == 8 ? M : (M + 1) / 2;
  constexpr int NVEC = (CODE_BYTES + 15) / 16;
  constexpr int NW = NT / 64;
  constexpr int FR = G / 4;                   // float4 rows per table entry (float staging)
  constexpr int UW = G / 2;                   // 32-bit words per one-byte row
  static_assert(G == 4 || (U8 && G == 8), "float rows serve 4 queries, one-byte rows 4 or 8");
  static_assert(!U8 || M * 255 < 65536, "16-bit partial sums");
  // [NENT / SL * FR]: entry e for the group's queries.  A static array, so
  // that its address is a constant: a table read is then the code byte
  // times 16 (one shift of the selected byte) plus an immediate offset.
  __shared__ __align__(16) float4 lut4[NENT / SL * FR];
  __shared__ __align__(16) float res[G][D];
  __shared__ uint32_t wcnt[2][NT / 64][(G + 1) / 2];
  __shared__ float u8_lo[U8 ? M : 1][G];      // per (sub-space, query) minimum
  __shared__ float u8_wspan[U8 ? NW : 1][G];  // per wave: largest range seen
  __shared__ float u8_par[3][G];              // per query: base, delta, 1 / delta
  __shared__ uint32_t s_early[EARLY ? G : 1];  // per query of the group: items re-ranked early
  __shared__ uint32_t s_kmm[2][MODE == 0 ? NT / 64 : 1][G];  // sample scan: per wave, smallest and largest key image
  static_assert(!EARLY || (MODE == 1 && D <= 128 && D % 4 == 0), "early re-rank: filter scan, rows of <= 32 chunks");
  static_assert(SL == 1 || (!U8 && !EARLY && BITS == 8 && (M / SL) % 16 == 0 && NENT % (SL * NT) == 0),
                "sliced tables: float rows, 8-bit codes, whole 16-byte code words and owned entries per slice");
  static_assert(SL > 1 || PMAX == 1, "one pass per chunk without slices");
  constexpr int MS = M / SL;            // sub-spaces per slice
  constexpr int NVS = NVEC / SL;        // 16-byte code words per slice
  constexpr int EPS = EPT / SL;         // owned entries per slice
  // sliced tables: each thread builds entries of one sub-space (TPM threads
  // per sub-space of the slice)
  constexpr int TPM = NT / MS;
  constexpr bool SUBM = SL > 1 && !REGCB && NT % MS == 0 && KSUB % TPM == 0;

  // the codebook is the same for every group: the owned codewords are loaded once
  float creg[REGCB ? EPT : 1][DSUB];
  if constexpr (REGCB) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * NT;
#pragma unroll
      for (int t = 0; t < DSUB; ++t) creg[i][t] = e < NENT ? a.codebook[e * DSUB + t] : 0.0f;
    }
  }

  const int64_t split = a.pair_split[0], total = a.pair_split[1];
  const int64_t cbeg = (MODE == 0 ? 0 : split) / G;
  const int64_t cend = (MODE == 0 ? split : total) / G;
  const int nx = a.nxcd;
  const int xcd = blockIdx.x % nx;
  const int64_t wid = blockIdx.x / nx;
  const int64_t nw = gridDim.x / nx;
  const int64_t span = cend - cbeg;
  const int64_t lo = cbeg + span * xcd / nx;
  const int64_t hi = cbeg + span * (xcd + 1) / nx;
  // A group's pairs, queries, list and output places, and its residual
  // inputs, are fetched while the previous group is processed, by vector
  // loads (lane g of each wave holding pair g) so that the LDS waits of that
  // group do not also wait for them: pairs and queries when the previous
  // group starts, places after its table build, the query and centroid
  // values after its first scan pass.
  const int lane = threadIdx.x & 63;
  constexpr int RPT = (G * D + NT - 1) / NT;  // residual inputs per thread
  uint32_t f_pp = NO_PAIR, f_prune = 0, f_dmax = 0, f_ebits = 0;
  int64_t f_qq = 0, f_ro = 0, f_base = 0, f_tr = 0;
  int32_t f_j = 0;
  float f_q[RPT], f_c[RPT];
  auto fetch_pairs = [&](int64_t cg) {
    const int g = lane & (G - 1);
    f_pp = a.sorted_pairs[cg * G + g];
    f_qq = (int64_t)a.sorted_q[cg * G + g];  // meaningless (never used) for an empty slot
  };
  auto fetch_places = [&]() {
    if (f_pp != NO_PAIR) {
      f_ro = a.rank_off[f_pp];
      f_j = a.probe_lists[f_pp];
      if (a.trace_keys) f_tr = a.key_off[f_qq];
      if (MODE == 0) {
        f_base = a.sample_off[f_qq];
      } else {
        f_base = a.surv_off[f_qq];
        f_prune = a.books[f_qq].prune;
        f_dmax = a.books[f_qq].dmax_bits;
        if (EARLY) f_ebits = a.books[f_qq].early_bits;
      }
    }
  };
  auto fetch_inputs = [&]() {
    const int64_t jn = lane_value(f_j, 0);  // the first pair of a group is always real
    bool vn[G];
    int64_t qn[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      vn[g] = lane_value(f_pp, g) != NO_PAIR;
      qn[g] = lane_value(f_qq, g);
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int idx = threadIdx.x + r * NT;
      f_q[r] = 0.0f;
      f_c[r] = 0.0f;
      if (idx < G * D) {
        const int g = idx / D, e = idx % D;
        f_c[r] = a.cent[jn * D + e];
#pragma unroll
        for (int h = 0; h < G; ++h)
          if (h == g && vn[h]) f_q[r] = a.q[qn[h] * D + e];
      }
    }
  };
  if (EARLY && threadIdx.x < G) s_early[threadIdx.x] = 0u;
  const int64_t c0 = lo + wid;
  if (c0 < hi) {
    fetch_pairs(c0);
    fetch_places();
    fetch_inputs();
  }
  for (int64_t c = c0; c < hi; c += nw) {
    // per pair g of the group: its first output slot (sample keys in phase
    // 0, survivors in phase 1) and the largest key image it keeps (all keys
    // when the query does not reject); the pairs, queries and trace offsets
    // stay in vector registers (lane g), read back where they are needed
    bool valid[G];
    int64_t ooff[G];
    uint32_t ebits[G];
    // the largest kept key as a float: keys are sums of non-negative table
    // entries, so comparing them with d_max as floats orders them as their
    // images do (+inf: keep all; a negative d_max keeps none)
    float dmaxf[G];
    // mode 0: this thread's smallest and largest key per pair (keys are
    // sums of non-negative entries, so they order as their images do)
    float kmn[G], kmx[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      kmn[g] = __builtin_inff();
      kmx[g] = 0.0f;
    }
    const uint32_t cur_pp = f_pp;
    const int64_t cur_qq = f_qq, cur_tr = f_tr + f_ro;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      valid[g] = lane_value(f_pp, g) != NO_PAIR;
      ooff[g] = valid[g] ? lane_value(f_base, g) + lane_value(f_ro, g) : 0;
      const uint32_t db = lane_value(f_dmax, g);
      dmaxf[g] = !(MODE == 1 && valid[g] && lane_value(f_prune, g)) ? __builtin_inff()
                 : (db & 0x80000000u) ? __uint_as_float(db & 0x7fffffffu) : -1.0f;
      ebits[g] = EARLY && valid[g] ? lane_value(f_ebits, g) : 0u;
    }
    const int j = lane_value(f_j, 0);
    float rq[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) rq[r] = f_q[r] - f_c[r];  // r = q - c, once per element
    if (c + nw < hi) fetch_pairs(c + nw);
    __syncthreads();  // the previous group is done with res and the tables
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int idx = threadIdx.x + r * NT;
      if (idx < G * D) {
        const int g = idx / D, e = idx % D;
        bool v = false;
#pragma unroll
        for (int h = 0; h < G; ++h)
          if (h == g) v = valid[h];
        res[g][e] = v ? rq[r] : 0.0f;
      }
    }
    __syncthreads();
    // the entries of slice sl (all of them without slices) into the table
    auto build_slice = [&](int sl) {
      if constexpr (SUBM) {
        // thread t builds entries j = t % TPM + TPM * i of sub-space t / TPM
        // of the slice: the sub-space's residuals are read from LDS once
        const int ml = threadIdx.x / TPM, m = sl * MS + ml;
        float rg[G][DSUB];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int t = 0; t < DSUB; ++t) rg[g][t] = res[g][m * DSUB + t];
#pragma unroll
        for (int i = 0; i < KSUB / TPM; ++i) {
          const int jj = threadIdx.x % TPM + TPM * i;
          const float* cwp = a.codebook + ((int64_t)m * KSUB + jj) * DSUB;
          float cw[DSUB];
#pragma unroll
          for (int t = 0; t < DSUB; ++t) cw[t] = cwp[t];
          float out[G];
#pragma unroll
          for (int g = 0; g < G; ++g) {
            float acc = 0.0f;
#pragma unroll
            for (int t = 0; t < DSUB; ++t) {
              const float u = rg[g][t] - cw[t];
              acc = t == 0 ? u * u : __builtin_fmaf(u, u, acc);
            }
            out[g] = acc;
          }
#pragma unroll
          for (int h = 0; h < FR; ++h)
            lut4[(ml * KSUB + jj) * FR + h] = make_float4(out[4 * h], out[4 * h + 1], out[4 * h + 2], out[4 * h + 3]);
        }
        return;
      }
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        if (i / EPS != sl) continue;
        const int e = threadIdx.x + i * NT;
        if (e < NENT) {
          const int m = e / KSUB;
          float cw[DSUB];
#pragma unroll
          for (int t = 0; t < DSUB; ++t) {
            if constexpr (REGCB) cw[t] = creg[i][t];
            else cw[t] = a.codebook[e * DSUB + t];
          }
          float out[G];
#pragma unroll
          for (int g = 0; g < G; ++g) {
            // the sum from 0 in t order by fused multiply-adds; its first
            // term a plain square (u * u + 0 rounds to the rounded square)
            float acc = 0.0f;
#pragma unroll
            for (int t = 0; t < DSUB; ++t) {
              const float u = res[g][m * DSUB + t] - cw[t];
              acc = t == 0 ? u * u : __builtin_fmaf(u, u, acc);
            }
            out[g] = acc;
          }
          const int el = e - sl * (NENT / SL);
#pragma unroll
          for (int h = 0; h < FR; ++h)
            lut4[el * FR + h] = make_float4(out[4 * h], out[4 * h + 1], out[4 * h + 2], out[4 * h + 3]);
        }
        asm volatile("" ::: "memory");  // one entry's LDS reads at a time
      }
    };
    build_slice(0);
    __syncthreads();
    if (c + nw < hi) fetch_places();
    float kbase[G], kdelta[G];
    if constexpr (U8) {
      const int wv = threadIdx.x >> 6;
      float wspan[G];
#pragma unroll
      for (int g = 0; g < G; ++g) wspan[g] = 0.0f;
      // minimum and maximum of each (sub-space, query): a wave per sub-space
      // (four sub-spaces per wave at a time for 16-entry sub-spaces)
      constexpr int SPW = KSUB >= 64 ? 1 : 64 / KSUB;
      constexpr int LPS = KSUB >= 64 ? 64 : KSUB;  // lanes per sub-space
      auto row_vals = [&](int e, float* v) {
#pragma unroll
        for (int h = 0; h < FR; ++h) {
          const float4 f = lut4[e * FR + h];
          v[4 * h] = f.x; v[4 * h + 1] = f.y; v[4 * h + 2] = f.z; v[4 * h + 3] = f.w;
        }
      };
      for (int m0 = wv * SPW; m0 < M; m0 += NW * SPW) {
        const int m = m0 + lane / LPS;
        const bool okm = m < M;
        float lo[G], hv[G];
        row_vals((okm ? m : 0) * KSUB + lane % LPS, lo);
#pragma unroll
        for (int g = 0; g < G; ++g) hv[g] = lo[g];
        for (int b = lane % LPS + LPS; b < KSUB; b += LPS) {
          float f[G];
          row_vals((okm ? m : 0) * KSUB + b, f);
#pragma unroll
          for (int g = 0; g < G; ++g) {
            lo[g] = fminf(lo[g], f[g]);
            hv[g] = fmaxf(hv[g], f[g]);
          }
        }
#pragma unroll
        for (int off = LPS / 2; off >= 1; off >>= 1)
#pragma unroll
          for (int g = 0; g < G; ++g) {
            lo[g] = fminf(lo[g], __shfl_xor(lo[g], off));
            hv[g] = fmaxf(hv[g], __shfl_xor(hv[g], off));
          }
        if (okm) {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            if (lane % LPS == 0) u8_lo[m][g] = lo[g];
            wspan[g] = fmaxf(wspan[g], hv[g] - lo[g]);
          }
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int g = 0; g < G; ++g) wspan[g] = fmaxf(wspan[g], __shfl_xor(wspan[g], off));
      if (lane == 0) {
#pragma unroll
        for (int g = 0; g < G; ++g) u8_wspan[wv][g] = wspan[g];
      }
      __syncthreads();
      if (threadIdx.x < G) {
        const int g = threadIdx.x;
        float span = 0.0f;
        for (int w2 = 0; w2 < NW; ++w2) span = fmaxf(span, u8_wspan[w2][g]);
        float dl = span / 255.0f;
        if (!(dl > 0.0f)) dl = 1.0f;
        float base = 0.0f;
        for (int m = 0; m < M; ++m) base = base + u8_lo[m][g];
        u8_par[0][g] = base;
        u8_par[1][g] = dl;
        u8_par[2][g] = 1.0f / dl;
      }
      __syncthreads();
      float inv[G];
#pragma unroll
      for (int g = 0; g < G; ++g) inv[g] = u8_par[2][g];
      uint32_t* lut32 = reinterpret_cast<uint32_t*>(lut4);
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * NT;
        uint32_t row[UW];
#pragma unroll
        for (int h = 0; h < UW; ++h) row[h] = 0u;
        if (e < NENT) {
          const int m = e / KSUB;
          float fv[G];
          row_vals(e, fv);
#pragma unroll
          for (int g = 0; g < G; ++g) {
            float t = fv[g] - u8_lo[m][g];
            t = t * inv[g];
            t = t + 0.5f;
            uint32_t u = (uint32_t)t;
            u = u > 255u ? 255u : u;
            row[g >> 1] |= u << (16 * (g & 1));
          }
        }
        __syncthreads();  // every float row this round overwrites has been read
        if (e < NENT) {
#pragma unroll
          for (int h = 0; h < UW; ++h) lut32[e * UW + h] = row[h];
        }
      }
      __syncthreads();
#pragma unroll
      for (int g = 0; g < G; ++g) {
        kbase[g] = u8_par[0][g];
        kdelta[g] = u8_par[1][g];
      }
    }
    const int64_t lbeg = uniform(a.list_off[j]);
    const int64_t nobj = uniform(a.list_off[j + 1]) - lbeg;
    BlockCompactor<G, NT, O> comp;
    comp.reset();
    const uint8_t* codes = a.codes + lbeg * (NVEC * 16);
    // block-uniform trip counts: every thread takes part in the compaction
    for (int64_t cb = 0; cb < nobj; cb += (int64_t)PMAX * NT * O) {
    float acc_c[PMAX][O][G];
    bool active_c[PMAX][O];
#pragma unroll
    for (int pp2 = 0; pp2 < PMAX; ++pp2)
#pragma unroll
      for (int o = 0; o < O; ++o) {
        active_c[pp2][o] = cb + pp2 * NT * O + o * NT + threadIdx.x < nobj;
#pragma unroll
        for (int g = 0; g < G; ++g) acc_c[pp2][o][g] = 0.0f;
      }
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      if (sl > 0 || (SL > 1 && cb > 0)) {
        __syncthreads();  // the previous slice's lookups are done
        build_slice(sl);
        __syncthreads();
      }
#pragma unroll
    for (int ps = 0; ps < PMAX; ++ps) {
      const int64_t base = cb + (int64_t)ps * NT * O;
      if (base >= nobj) break;  // block-uniform
      const bool* active = active_c[ps];
      uint32_t w[O][NVEC * 4];
#pragma unroll
      for (int o = 0; o < O; ++o) {
        const int64_t i = base + o * NT + threadIdx.x;
        const uint4* row = reinterpret_cast<const uint4*>(codes + (active[o] ? i : 0) * (NVEC * 16));
#pragma unroll
        for (int cc = sl * NVS; cc < (sl + 1) * NVS; ++cc) {
          uint4 v = active[o] ? row[cc] : make_uint4(0u, 0u, 0u, 0u);
          w[o][4 * cc + 0] = v.x; w[o][4 * cc + 1] = v.y; w[o][4 * cc + 2] = v.z; w[o][4 * cc + 3] = v.w;
        }
      }
      float (*acc)[G] = acc_c[ps];
      if constexpr (U8) {
        const uint32_t* lut32 = reinterpret_cast<const uint32_t*>(lut4);
        uint32_t acc16[O][UW];  // word h: 16-bit sums of queries 2h (low) and 2h+1 (high)
#pragma unroll
        for (int o = 0; o < O; ++o)
#pragma unroll
          for (int h = 0; h < UW; ++h) acc16[o][h] = 0u;
        if (active[0])
#pragma unroll
        for (int m = 0; m < M; ++m) {
          if (m % (4 / O) == 0 && m) asm volatile("" ::: "memory");
#pragma unroll
          for (int o = 0; o < O; ++o) {
            uint32_t code;
            if (BITS == 8) code = (w[o][m >> 2] >> (8 * (m & 3))) & 0xffu;
            else code = (w[o][m >> 3] >> (4 * (m & 7))) & 0xfu;
            const uint32_t* row = lut32 + (m * KSUB + code) * UW;
            if constexpr (UW == 4) {
              const uint4 v = *reinterpret_cast<const uint4*>(row);
              acc16[o][0] += v.x; acc16[o][1] += v.y; acc16[o][2] += v.z; acc16[o][3] += v.w;
            } else {
              const uint2 v = *reinterpret_cast<const uint2*>(row);
              acc16[o][0] += v.x; acc16[o][1] += v.y;
            }
          }
        }
#pragma unroll
        for (int o = 0; o < O; ++o)
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const uint32_t K = (acc16[o][g >> 1] >> (16 * (g & 1))) & 0xffffu;
            const float t = (float)K * kdelta[g];
            acc[o][g] = kbase[g] + t;
          }
      } else {
      if (active[0]) {  // waves past the end of the list skip the table reads
        // the table reads of MB sub-spaces are issued together (the fences
        // keep them apart from the additions), then added in m order; the
        // first term of a key replaces its 0 + (an entry is a sum of squares,
        // never -0)
        constexpr int MB = 4 / O;
#pragma unroll
        for (int m0 = sl * MS; m0 < (sl + 1) * MS; m0 += MB) {
          float4 v[MB][O];
#pragma unroll
          for (int mm = 0; mm < MB; ++mm)
#pragma unroll
            for (int o = 0; o < O; ++o) {
              const int m = m0 + mm;
              uint32_t code;
              if (BITS == 8) code = (w[o][m >> 2] >> (8 * (m & 3))) & 0xffu;
              else code = (w[o][m >> 3] >> (4 * (m & 7))) & 0xfu;
              v[mm][o] = lut4[(m - sl * MS) * KSUB + code];
            }
          asm volatile("" ::: "memory");
#pragma unroll
          for (int mm = 0; mm < MB; ++mm)
#pragma unroll
            for (int o = 0; o < O; ++o) {
              if (m0 + mm == 0) {
                acc[o][0] = v[mm][o].x;
                acc[o][1] = v[mm][o].y;
                acc[o][2] = v[mm][o].z;
                acc[o][3] = v[mm][o].w;
              } else {
                acc[o][0] = acc[o][0] + v[mm][o].x;
                acc[o][1] = acc[o][1] + v[mm][o].y;
                acc[o][2] = acc[o][2] + v[mm][o].z;
                acc[o][3] = acc[o][3] + v[mm][o].w;
              }
            }
        }
      }
      }
    }
    }
    if (cb == 0 && c + nw < hi) fetch_inputs();
#pragma unroll
    for (int ps = 0; ps < PMAX; ++ps) {
      const int64_t base = cb + (int64_t)ps * NT * O;
      if (base >= nobj) break;  // block-uniform
      const bool* active = active_c[ps];
      float (*acc)[G] = acc_c[ps];
      if (a.trace_keys) {
        // (lanes are read in converged code only: a lane's value may be
        // stale where the lane is inactive)
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int64_t t0 = lane_value(cur_tr, g) + base + threadIdx.x;
#pragma unroll
          for (int o = 0; o < O; ++o)
            if (valid[g] && active[o]) a.trace_keys[t0 + o * NT] = acc[o][g];
        }
      }
      if (MODE == 0) {
#pragma unroll
        for (int o = 0; o < O; ++o)
#pragma unroll
          for (int g = 0; g < G; ++g)
            if (valid[g] && active[o]) {
              a.sample_keys[ooff[g] + base + o * NT + threadIdx.x] = acc[o][g];
              kmn[g] = fminf(kmn[g], acc[o][g]);
              kmx[g] = fmaxf(kmx[g], acc[o][g]);
            }
      }
      if (MODE == 1) {
        bool keep[O * G];
        uint32_t slot[O * G];
#pragma unroll
        for (int o = 0; o < O; ++o)
#pragma unroll
          for (int g = 0; g < G; ++g) keep[o * G + g] = valid[g] && active[o] && acc[o][g] <= dmaxf[g];
        comp.step(keep, slot, wcnt);
        bool ear[O * G];
#pragma unroll
        for (int o = 0; o < O; ++o) {
          const int64_t i = base + o * NT + threadIdx.x;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            ear[o * G + g] = EARLY && keep[o * G + g] && key_bits(acc[o][g]) < ebits[g];
            if (keep[o * G + g]) {
              // uniform bases, 32-bit lane offsets
              (a.surv_key + ooff[g])[slot[o * G + g]] = acc[o][g];
              (a.surv_pos + ooff[g])[slot[o * G + g]] = (uint32_t)(lbeg + i) | (ear[o * G + g] ? EARLY_FLAG : 0u);
            }
          }
        }
        if constexpr (EARLY) {
          constexpr int NCH = D / 4;
          constexpr int EU = 4;  // items per half-wave per round
          const int hl = lane & 31, half = lane >> 5;
          const int64_t wbase = base + (int64_t)(threadIdx.x & ~63);  // object of lane 0, o = 0
          const float4* vec4 = reinterpret_cast<const float4*>(a.vectors);
          const float4* q4 = reinterpret_cast<const float4*>(a.q);
#pragma unroll
          for (int og = 0; og < O * G; ++og) {
            const int o = og / G, g = og % G;
            const int64_t qrow = lane_value(cur_qq, g) * NCH;
            uint64_t em = __ballot(ear[og]);
            if (lane == 0 && em) atomicAdd(&s_early[g], (uint32_t)__popcll(em));
            while (em) {  // wave-uniform
              int src[EU];
#pragma unroll
              for (int u = 0; u < EU; ++u) {
                const int a0 = em ? __ffsll((unsigned long long)em) - 1 : -1;
                if (em) em &= em - 1;
                const int a1 = em ? __ffsll((unsigned long long)em) - 1 : -1;
                if (em) em &= em - 1;
                src[u] = half ? a1 : a0;
              }
              float4 xv[EU], qv[EU];
              uint32_t sl[EU];
#pragma unroll
              for (int u = 0; u < EU; ++u) {
                const int sr = src[u] < 0 ? 0 : src[u];
                sl[u] = __shfl(slot[og], sr);
                const bool ok = src[u] >= 0 && hl < NCH;
                const int64_t row = lbeg + wbase + o * NT + sr;
                xv[u] = ok ? vec4[row * NCH + hl] : make_float4(0.f, 0.f, 0.f, 0.f);
                qv[u] = ok ? q4[qrow + hl] : make_float4(0.f, 0.f, 0.f, 0.f);
              }
#pragma unroll
              for (int u = 0; u < EU; ++u) {
                float e = a.metric ? chunk_ip(qv[u], xv[u], 0.0f) : chunk_l2(qv[u], xv[u], 0.0f);
                e = canon_reduce32(e);
                if (src[u] >= 0 && hl == 0) a.surv_exact[ooff[g] + sl[u]] = a.metric ? -e : e;
              }
            }
          }
        }
      }
    }
    }
    if (EARLY) __syncthreads();  // the group's early counts are complete
    uint32_t pg[G];
    int64_t qgs[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {  // converged: every lane active
      pg[g] = lane_value(cur_pp, g);
      qgs[g] = lane_value(cur_qq, g);
    }
    if (MODE == 0 && a.smin) {
      // per wave, then across the block's waves, then one atomic per query
      // and group (device-wide atomics per wave cost more than the scan's
      // last barrier)
      const int wv = threadIdx.x >> 6;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        uint32_t mn = key_bits(kmn[g]), mx = key_bits(kmx[g]);
        wave_minmax(mn, mx);
        if (lane == 0) {
          s_kmm[0][wv][g] = mn;
          s_kmm[1][wv][g] = mx;
        }
      }
      __syncthreads();
      if (threadIdx.x < G) {
        const int g = threadIdx.x;
        uint32_t mn = 0xffffffffu, mx = 0u;
        for (int w = 0; w < NT / 64; ++w) {
          mn = min(mn, s_kmm[0][w][g]);
          mx = max(mx, s_kmm[1][w][g]);
        }
        bool vg = false;
        int64_t qg = 0;
#pragma unroll
        for (int h = 0; h < G; ++h)
          if (h == g) {
            vg = valid[h];
            qg = qgs[h];
          }
        if (vg && mn <= mx) {
          atomicMin(a.smin + qg, mn);
          atomicMax(a.smax + qg, mx);
        }
      }
    }
    if (MODE == 1 && threadIdx.x == 0) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (valid[g]) {
          const int64_t qg = qgs[g];
          a.pair_nsurv[pg[g]] = comp.total[g];
          if (nobj > comp.total[g]) atomicAdd(a.n_rejected + qg, (uint32_t)(nobj - comp.total[g]));
          if (EARLY && s_early[g]) atomicAdd(a.n_early + qg, s_early[g]);
        }
        if (EARLY) s_early[g] = 0u;
      }
    }
  }
}

// ---- generic fallback: one block per pair, table from the global codebook -----
template <int MODE, int BITS>
__global__ __launch_bounds__(256) void pq_scan_kernel(PqScanArgs a) {
  constexpr int NT = 256;
  constexpr int KSUB = 1 << BITS;
  extern __shared__ __align__(16) unsigned char smem[];
  float* lut = reinterpret_cast<float*>(smem);              // [M][KSUB]
  float* res = lut + a.M * KSUB;                            // [d]

  const int64_t split = a.pair_split[0];
  const int64_t it = (MODE == 0 ? 0 : split) + blockIdx.x;
  if (it >= (MODE == 0 ? split : (int64_t)a.pair_split[1])) return;
  const uint32_t pv = a.sorted_pairs[it];
  if (pv == NO_PAIR) return;
  const int64_t p = pv;
  const int64_t qi = a.sorted_q[it];
  if (MODE == 1 && a.rescan_q && !a.rescan_q[qi]) return;
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
      const float u = rr[t] - cw[t];
      acc = __builtin_fmaf(u, u, acc);
    }
    lut[e] = acc;
  }
  __syncthreads();
  const int64_t lbeg = a.list_off[j];
  const int64_t nobj = a.list_off[j + 1] - lbeg;
  PairOut out;
  out.init(a, MODE, qi, p);
  __shared__ uint32_t wcnt[2][NT / 64][1];
  BlockCompactor<1, NT> comp;
  comp.reset();
  const int stride = a.code_stride;  // bytes per code row, multiple of 16
  const uint8_t* codes = a.codes + lbeg * stride;
  for (int64_t base = 0; base < nobj; base += NT) {
    const int64_t i = base + threadIdx.x;
    const bool active = i < nobj;
    const uint4* row = reinterpret_cast<const uint4*>(codes + (active ? i : 0) * stride);
    float key = 0.0f;
    int m = 0;
    for (int c = 0; active && c < stride / 16 && m < a.M; ++c) {
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
    if (active && out.trace_out) out.trace_out[i] = key;
    if (MODE == 0) {
      if (active) out.sample_out[i] = key;
      if (a.smin) {
        uint32_t mn = active ? key_bits(key) : 0xffffffffu, mx = active ? key_bits(key) : 0u;
        wave_minmax(mn, mx);
        if ((threadIdx.x & 63) == 0 && mn <= mx) {
          atomicMin(a.smin + qi, mn);
          atomicMax(a.smax + qi, mx);
        }
      }
    } else {
      bool keep[1] = {active && out.keep(key)};
      uint32_t slot[1];
      comp.step(keep, slot, wcnt);
      if (keep[0]) {
        out.skey[slot[0]] = key;
        out.spos[slot[0]] = (uint32_t)(lbeg + i);
      }
    }
  }
  if (MODE == 1 && threadIdx.x == 0) {
    a.pair_nsurv[p] = comp.total[0];
    if (nobj > comp.total[0]) atomicAdd(a.n_rejected + qi, (uint32_t)(nobj - comp.total[0]));
  }
}

template <int BITS, int M, int DSUB, int NT, int O, bool U8, int SL, int PMAX, int BPC>
static void launch_grouped_t(const PqScanArgs& a, int blocks, hipStream_t s) {
  const size_t lds = 0;  // the tables are static LDS
  const dim3 grid(BPC * blocks), block(NT);
  if (a.mode == 0)
    hipLaunchKernelGGL((pq_scan_grouped<0, BITS, M, DSUB, NT, O, U8, false, SL, PMAX, BPC>), grid, block, lds, s, a);
  else if (!U8 && SL == 1 && BPC == 1 && a.early)
    hipLaunchKernelGGL((pq_scan_grouped<1, BITS, M, DSUB, NT, O, false, true>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((pq_scan_grouped<1, BITS, M, DSUB, NT, O, U8, false, SL, PMAX, BPC>), grid, block, lds, s, a);
}

template <int BITS, int M, int DSUB, int NT, int O, int SL, int PMAX, int BPC>
static void launch_grouped(const PqScanArgs& a, int blocks, hipStream_t s) {
  // one-byte tables take two blocks per CU only when their float staging
  // fits twice in LDS (the callers ask for one block otherwise)
  constexpr bool U8_BPC = BPC == 1 || (size_t)scan_group_of(true, BITS) * M * (1 << BITS) * sizeof(float) <= 65536;
  if (a.lut_u8) launch_grouped_t<BITS, M, DSUB, NT, O, true, 1, 1, U8_BPC ? BPC : 1>(a, blocks, s);
  else launch_grouped_t<BITS, M, DSUB, NT, O, false, SL, PMAX, BPC>(a, blocks, s);
}

// Pairs per scan group of this search: the grouped kernel's group for a
// grouped shape, SCAN_GROUP for the generic one-pair-per-block kernel.
static int pair_group(const PqScanArgs& a) {
  return pq_scan_grouped_shape(a.bits, a.M, a.d) ? scan_group_of(a.lut_u8 != 0, a.bits) : SCAN_GROUP;
}

// Block shapes (scan_variant):
//   0  two blocks of 512 threads per CU, 2 codes per thread and pass (float
//      tables of 8-bit codes over 32 sub-spaces: in two slices); early
//      re-rank runs shape 3
//   1  one block of 512 threads per CU, 1 code per thread and pass
//   2  one block of 1024 threads per CU, 1 code
//   3  one block of 512 threads per CU, 2 codes
//   4  two blocks of 512 threads per CU, 1 code (sliced as shape 0)
template <int BITS, int M, int DSUB>
static bool try_grouped(const PqScanArgs& a, hipStream_t s) {
  if (a.bits != BITS || a.M != M || a.d != M * DSUB) return false;
  int blocks = (a.num_cu / a.nxcd) * a.nxcd;
  if (blocks < a.nxcd) blocks = a.nxcd;
  // float tables that fit twice in LDS need no slices
  constexpr int SL = (size_t)SCAN_GROUP * M * (1 << BITS) * sizeof(float) > 65536 ? 2 : 1;
  // two blocks per CU: float tables (sliced when needed), and one-byte
  // tables whose float staging fits twice; early re-rank keeps one
  constexpr bool U8_TWO = (size_t)scan_group_of(true, BITS) * M * (1 << BITS) * sizeof(float) <= 65536;
  const bool two = a.lut_u8 ? U8_TWO : !a.early;
  switch (a.scan_variant) {
    case 1: launch_grouped<BITS, M, DSUB, 512, 1, 1, 1, 1>(a, blocks, s); break;
    case 2: launch_grouped<BITS, M, DSUB, 1024, 1, 1, 1, 1>(a, blocks, s); break;
    case 3: launch_grouped<BITS, M, DSUB, 512, 2, 1, 1, 1>(a, blocks, s); break;
    case 4:
      if (two) launch_grouped<BITS, M, DSUB, 512, 1, SL, SL == 1 ? 1 : 4, 2>(a, blocks, s);
      else launch_grouped<BITS, M, DSUB, 512, 2, 1, 1, 1>(a, blocks, s);
      break;
    default:
      if (two) launch_grouped<BITS, M, DSUB, 512, 2, SL, SL == 1 ? 1 : 2, 2>(a, blocks, s);
      else launch_grouped<BITS, M, DSUB, 512, 2, 1, 1, 1>(a, blocks, s);
      break;
  }
  return true;
}

bool pq_scan_grouped_shape(int bits, int M, int d) {
  return (bits == 8 && M == 32 && d == 128) || (bits == 8 && M == 16 && d == 128) ||
         (bits == 4 && M == 48 && d == 96) || (bits == 4 && M == 32 && d == 128);
}

hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

int64_t pair_sort_table_words(int64_t nq, int nbins) { return bs_table_words(nq, nbins); }

int64_t pair_slots(int64_t npairs, int nlist) { return npairs + 2 * (int64_t)nlist * (SCAN_GROUP_MAX - 1); }

hipError_t launch_pair_sort(const PqScanArgs& a, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  const int nb = 2 * a.nlist;
  const int64_t slots = pair_slots(a.npairs, a.nlist);
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<int64_t>((slots + 255) / 256, 4096)), dim3(256), 0, s,
                     a.sorted_pairs, slots, NO_PAIR);
  if (a.bs_table && nb <= BS_MAX_BINS) {
    const ScanPairBins f{a.probe_off, a.probe_lists, a.nsample_q, a.nlist, a.sorted_pairs, a.sorted_q};
    bs_sort(f, nb, a.nq, a.probe_off, a.bs_table, a.pair_cnt, [&] {
      hipLaunchKernelGGL(pair_offsets_kernel, dim3(1), dim3(1024), 0, s, a.pair_cnt, nb, a.nlist, pair_group(a),
                         a.pair_split);
    }, s);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(zero_u32_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, a.pair_cnt, (int64_t)nb);
  const unsigned g = (unsigned)std::min<int64_t>((a.npairs + 255) / 256, 4096);
  hipLaunchKernelGGL(pair_count_kernel, dim3(g), dim3(256), 0, s, a);
  hipLaunchKernelGGL(pair_offsets_kernel, dim3(1), dim3(1024), 0, s, a.pair_cnt, nb, a.nlist, pair_group(a),
                     a.pair_split);
  hipLaunchKernelGGL(pair_scatter_kernel, dim3(g), dim3(256), 0, s, a);
  return hipGetLastError();
}

// One wave per query: the check of the tighter filter (see launch_filter_rescan).
__global__ __launch_bounds__(256) void filter_check_kernel(PqScanArgs a, const int64_t* __restrict__ kc_target,
                                                           uint32_t* __restrict__ flags) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= a.nq) return;
  const int lane = threadIdx.x & 63;
  QueryBook* book = const_cast<QueryBook*>(a.books) + q;
  const uint32_t nf = book->filt_count;
  uint32_t flag = 0u;
  if (nf > 0u) {
    const int64_t po = a.probe_off[q], np = a.probe_off[q + 1] - po;
    uint64_t kept = 0, rej = 0;
    for (int64_t r = a.nsample_q[q] + lane; r < np; r += 64) {
      const int j = a.probe_lists[po + r];
      const uint32_t ns = a.pair_nsurv[po + r];
      kept += ns;
      rej += (uint64_t)(a.list_off[j + 1] - a.list_off[j]) - ns;
    }
    for (int off = 32; off >= 1; off >>= 1) {
      kept += __shfl_xor(kept, off);
      rej += __shfl_xor(rej, off);
    }
    if ((int64_t)(nf + kept) < kc_target[q]) {
      flag = 1u;
      if (lane == 0) {
        book->dmax_bits = book->dmax_full;
        book->filt_count = 0u;
        a.n_rejected[q] -= (uint32_t)rej;
      }
    }
  }
  if (lane == 0) flags[q] = flag;
}

hipError_t launch_filter_rescan(PqScanArgs a, const int64_t* kc_target, uint32_t* flags, hipStream_t s) {
  if (a.nq <= 0 || a.npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(filter_check_kernel, dim3((unsigned)((a.nq + 3) / 4)), dim3(256), 0, s, a, kc_target, flags);
  a.mode = 1;
  a.rescan_q = flags;
  a.early = 0;
  const int64_t n = pair_slots(a.npairs, a.nlist);  // covers the slots of the second phase
  const size_t lds = sizeof(float) * ((size_t)a.M * (1 << a.bits) + a.d);
  if (a.bits == 8) hipLaunchKernelGGL((pq_scan_kernel<1, 8>), dim3((unsigned)n), dim3(256), lds, s, a);
  else hipLaunchKernelGGL((pq_scan_kernel<1, 4>), dim3((unsigned)n), dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_pq_scan(const PqScanArgs& a, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  if (a.mode == 0 && a.smin) {
    const unsigned g = (unsigned)std::min<int64_t>((a.nq + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(g), dim3(256), 0, s, a.smin, a.nq, 0xffffffffu);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(g), dim3(256), 0, s, a.smax, a.nq, 0u);
  }
  if (try_grouped<8, 32, 4>(a, s) || try_grouped<8, 16, 8>(a, s) || try_grouped<4, 48, 2>(a, s) ||
      try_grouped<4, 32, 4>(a, s))
    return hipGetLastError();
  // generic shapes: one block per padded slot of either phase
  const int64_t n = pair_slots(a.npairs, a.nlist);
  size_t lds = sizeof(float) * ((size_t)a.M * (1 << a.bits) + a.d);
  if (a.bits == 8) {
    if (a.mode == 0) hipLaunchKernelGGL((pq_scan_kernel<0, 8>), dim3((unsigned)n), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((pq_scan_kernel<1, 8>), dim3((unsigned)n), dim3(256), lds, s, a);
  } else {
    if (a.mode == 0) hipLaunchKernelGGL((pq_scan_kernel<0, 4>), dim3((unsigned)n), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((pq_scan_kernel<1, 4>), dim3((unsigned)n), dim3(256), lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace bbc

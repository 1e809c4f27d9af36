// Comparator collectors: the same K_c candidates as the bucket collector
// (the K_c smallest estimated (key, id) of the scanned objects), found the
// ways the paper compares against (result-collector background: a bounded
// max-heap, and selection by sorting).  Both read every scanned key, written
// by slot by the scan with every probed list in the "sample" phase.
//
//  - sort: exact selection by a 32-bit radix select of the K_c-th key image
//    over all S keys, then a compaction pass; ties on the threshold key are
//    cut by id with a second radix select over the tied ids;
//  - heap: one wave per query keeps a 64-ary max-heap of packed (key, id)
//    of size K_c in global memory (collector 1), or in LDS when the batch's
//    largest K_c fits (collector 3).  Its first K_c keys are heapified; every
//    later key below the heap's top replaces the top and sifts down (each
//    level: the 64 children are read by the 64 lanes and reduced).
#include "common.h"
#include "kernels.h"

namespace bbc {

namespace {

constexpr int CMP_RANKCAP = 2048;      // probe ranks held in LDS (sort collector)
constexpr int CMP_RANKCAP_HEAP = 256;  // (heap collector: small blocks, many per CU)
constexpr size_t CMP_HEAP_LDS_MAX = 152 * 1024;  // heaps of up to 19,456 entries live in LDS

template <int NT, int CAP>
__device__ SlotMap load_slot_map(const CompareArgs& a, int64_t qi, int32_t* s_rbeg, int32_t* s_lbeg) {
  const int64_t po = a.probe_off[qi];
  return slot_map_load<NT, CAP>(a.rank_off + po, a.probe_lists + po, a.list_off, a.nprobe[qi], s_rbeg, s_lbeg);
}

}  // namespace

__global__ __launch_bounds__(1024) void sort_collect_kernel(CompareArgs a) {
  constexpr int NT = 1024;
  __shared__ int32_t s_rbeg[CMP_RANKCAP];
  __shared__ int32_t s_lbeg[CMP_RANKCAP];
  __shared__ uint32_t hist[256];
  __shared__ __align__(8) uint32_t bc[8];

  const int64_t qi = blockIdx.x;
  const int64_t S = a.n_scanned[qi];
  int64_t kc = a.kc_target[qi];
  if (kc > S) kc = S;
  if (threadIdx.x == 0) a.n_cand[qi] = kc > 0 ? kc : 0;
  if (kc <= 0) return;
  const SlotMap sm = load_slot_map<NT, CMP_RANKCAP>(a, qi, s_rbeg, s_lbeg);
  const float* keys = a.keys + a.key_off[qi];
  uint32_t* cand = a.cand_pos + a.cand_off[qi];
  if (kc == S) {
    for (int64_t i = threadIdx.x; i < S; i += NT) cand[i] = (uint32_t)sm.pos(i);
    return;
  }
  const uint32_t T = block_radix_select32<NT>([&](int64_t i) { return key_bits(keys[i]); }, S, kc - 1, hist, bc);
  // every key below T is a candidate
  if (threadIdx.x == 0) { bc[4] = 0; bc[5] = 0; }
  __syncthreads();
  for (int64_t base = 0; base < S; base += NT) {  // wave-uniform trip count
    const int64_t i = base + threadIdx.x;
    const uint32_t kb = i < S ? key_bits(keys[i]) : 0xffffffffu;
    const bool take = i < S && kb < T;
    const uint32_t slot = wave_slot(take, &bc[4]);
    if (take) cand[slot] = (uint32_t)sm.pos(i);
    const uint64_t tie = __ballot(i < S && kb == T);
    if ((threadIdx.x & 63) == 0 && tie) atomicAdd(&bc[5], (uint32_t)__popcll(tie));
  }
  __syncthreads();
  const int64_t nless = bc[4];
  const int64_t need = kc - nless;   // >= 1 of the keys equal to T
  const int64_t nties = bc[5];
  uint32_t id_thr = 0xffffffffu;     // all ties when they are exactly `need`
  if (nties > need) {
    // the `need` smallest ids among the ties (ids are distinct)
    id_thr = (uint32_t)block_radix_select64<NT>(
        [&](int64_t i, uint64_t& v) -> bool {
          if (key_bits(keys[i]) != T) return false;
          v = (uint64_t)(uint32_t)a.list_ids[sm.pos(i)];
          return true;
        },
        S, need - 1, hist, bc);
  }
  if (threadIdx.x == 0) bc[6] = 0;
  __syncthreads();
  for (int64_t base = 0; base < S; base += NT) {
    const int64_t i = base + threadIdx.x;
    bool take = false;
    int64_t p = 0;
    if (i < S && key_bits(keys[i]) == T) {
      p = sm.pos(i);
      take = (uint32_t)a.list_ids[p] <= id_thr;
    }
    const uint32_t slot = wave_slot(take, &bc[6]);
    if (take) cand[nless + slot] = (uint32_t)p;
  }
}

// The heap's storage: global memory (agent-scope atomic loads and stores, so
// that lane 0's stores are seen by the wave's later loads) or LDS.
template <bool LDSH>
__device__ __forceinline__ uint64_t hp_load(const uint64_t* p) {
  if constexpr (LDSH) return *reinterpret_cast<const volatile uint64_t*>(p);
  else return hload(p);
}
template <bool LDSH>
__device__ __forceinline__ void hp_store(uint64_t* p, uint64_t v) {
  if constexpr (LDSH) *reinterpret_cast<volatile uint64_t*>(p) = v;
  else hstore(p, v);
}

// One wave: sift v down from node i of the 64-ary max-heap h[0, n).
template <bool LDSH>
__device__ void hp_sift_down(uint64_t* h, int64_t n, int64_t i, uint64_t v) {
  const int lane = threadIdx.x & 63;
  while (true) {
    const int64_t c0 = 64 * i + 1;
    if (c0 >= n) break;
    const int64_t cj = c0 + lane;
    const bool ok = cj < n;
    const uint64_t cv = ok ? hp_load<LDSH>(h + cj) : 0ull;
    uint64_t mx = cv;
    for (int off = 32; off >= 1; off >>= 1) {
      const uint64_t o = __shfl_xor(mx, off);
      mx = o > mx ? o : mx;
    }
    if (mx <= v) break;
    const uint64_t at = __ballot(ok && cv == mx);
    const int j = __ffsll((unsigned long long)at) - 1;
    if (lane == 0) hp_store<LDSH>(h + i, mx);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    i = c0 + j;
  }
  if (lane == 0) hp_store<LDSH>(h + i, v);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// LDSH: the heap lives in LDS (dynamic, K_c entries of 8 bytes), for batches
// whose largest K_c fits.
template <bool LDSH>
__global__ __launch_bounds__(64) void heap_collect_kernel(CompareArgs a) {
  constexpr int NT = 64;
  __shared__ int32_t s_rbeg[CMP_RANKCAP_HEAP];
  __shared__ int32_t s_lbeg[CMP_RANKCAP_HEAP];
  extern __shared__ __align__(16) uint64_t s_heap[];
  const int lane = threadIdx.x;

  const int64_t qi = blockIdx.x;
  const int64_t S = a.n_scanned[qi];
  int64_t kc = a.kc_target[qi];
  if (kc > S) kc = S;
  if (lane == 0) a.n_cand[qi] = kc > 0 ? kc : 0;
  if (kc <= 0) return;
  const SlotMap sm = load_slot_map<NT, CMP_RANKCAP_HEAP>(a, qi, s_rbeg, s_lbeg);
  const float* keys = a.keys + a.key_off[qi];
  uint32_t* cand = a.cand_pos + a.cand_off[qi];
  if (kc == S) {
    for (int64_t i = lane; i < S; i += NT) cand[i] = (uint32_t)sm.pos(i);
    return;
  }
  uint64_t* h = LDSH ? s_heap : a.heap + a.cand_off[qi];
  auto packed = [&](int64_t i) -> uint64_t {
    return pack_key_id(keys[i], (uint32_t)a.list_ids[sm.pos(i)]);
  };
  // the first kc keys, then heapify bottom-up
  for (int64_t i = lane; i < kc; i += NT) hp_store<LDSH>(h + i, packed(i));
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  for (int64_t node = (kc - 2) / 64; node >= 0; --node) hp_sift_down<LDSH>(h, kc, node, hp_load<LDSH>(h + node));
  uint64_t top = hp_load<LDSH>(h);
  for (int64_t base = kc; base < S; base += NT) {
    const int64_t i = base + lane;
    uint64_t v = ~0ull;
    // key filter first: only keys not above the top's key need their id
    if (i < S && key_bits(keys[i]) <= (uint32_t)(top >> 32)) v = packed(i);
    uint64_t mask = __ballot(v < top);
    while (mask) {
      const int j = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const uint64_t x = __shfl(v, j);
      if (x < top) {  // the top only decreases
        hp_sift_down<LDSH>(h, kc, 0, x);
        top = hp_load<LDSH>(h);
      }
    }
  }
  for (int64_t i = lane; i < kc; i += NT) cand[i] = (uint32_t)a.pos_of_id[packed_id(hp_load<LDSH>(h + i))];
}

hipError_t launch_compare_collect(const CompareArgs& a, int collector, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  if (collector == 3 && a.max_kc > 0 && (size_t)a.max_kc * 8 <= CMP_HEAP_LDS_MAX)
    hipLaunchKernelGGL(heap_collect_kernel<true>, dim3((unsigned)a.nq), dim3(64), (size_t)a.max_kc * 8, s, a);
  else if (collector == 1 || collector == 3)
    hipLaunchKernelGGL(heap_collect_kernel<false>, dim3((unsigned)a.nq), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(sort_collect_kernel, dim3((unsigned)a.nq), dim3(1024), 0, s, a);
  return hipGetLastError();
}

}  // namespace bbc

// IVF probe: each query is routed to its nprobe nearest lists (the IVF
// index of the paper's background section, quantization methods).
//
// Step 1 (probe_gemm): D'[q][j] = |c_j|^2 - 2 <q~, c~_j>  (L2) or -<q~, c~_j>
//   (inner product) on BF16 MFMA with FP32 accumulation, q~ and c~ the
//   round-to-nearest BF16 images of the query and the centroid.
// Step 2 (probe_select): the BF16 scores only pre-filter.  The BF16 dot
//   product differs from the exact one by at most (2u + u^2) |q| |c_j| with
//   u = 2^-8 the unit roundoff of each operand, plus the FP32 accumulation
//   (d 2^-24 |q| |c_j| for d <= 1024): under 2^-7 |q| |c_j| in all.  With
//   E_j = a |q| |c_j| + 2^-12 (|q|^2 + |c_j|^2), a = 2^-5 for L2 (the dot
//   enters twice) and 2^-6 for the inner product (a factor 2 of margin
//   either way; the second term covers the FP32 norms and the canonical
//   key's own rounding), every list of the exact top-nprobe satisfies
//   D'_j - E_j <= U*, U* the nprobe-th smallest D'_j + E_j.  Only that
//   recheck set gets the canonical FP32 key, and the nprobe smallest
//   (key, list id) are the probe, nearest first.
#include "common.h"
#include "kernels.h"

namespace bbc {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// Block: 256 threads = 4 waves; tile 64 queries x 64 centroids.  Wave w owns
// query rows [16w, 16w+16) and four 16x16 MFMA tiles along the centroids.
// v_mfma_f32_16x16x32_bf16 operand layout (wave64): lane l supplies row
// (l % 16) of A and column (l % 16) of B for k = 8 (l / 16) .. +7, and holds
// D[4 (l / 16) + v][l % 16], v = 0..3.
__global__ __launch_bounds__(256) void probe_gemm_kernel(
    const float* __restrict__ q, int64_t nq, int d, const uint16_t* __restrict__ cb16, int dpad,
    const float* __restrict__ cn2, int nlist, int metric, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t qrow = (int64_t)blockIdx.y * 64 + w * 16 + (lane & 15);
  const int cbase = blockIdx.x * 64;
  const int kq = (lane >> 4) * 8;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < dpad; k0 += 32) {
    uint32_t ab[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      int kk = k0 + kq + v;
      float x = (qrow < nq && kk < d) ? q[qrow * d + kk] : 0.0f;
      ab[v] = bf16_bits_rne(x);
    }
    u32x4 ap = {ab[0] | (ab[1] << 16), ab[2] | (ab[3] << 16), ab[4] | (ab[5] << 16), ab[6] | (ab[7] << 16)};
    bf16x8 a = __builtin_bit_cast(bf16x8, ap);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      int col = cbase + t * 16 + (lane & 15);
      u32x4 bp = {0u, 0u, 0u, 0u};
      if (col < nlist) bp = *reinterpret_cast<const u32x4*>(cb16 + (int64_t)col * dpad + k0 + kq);
      bf16x8 b = __builtin_bit_cast(bf16x8, bp);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    int col = cbase + t * 16 + (lane & 15);
    if (col >= nlist) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int64_t row = (int64_t)blockIdx.y * 64 + w * 16 + (lane >> 4) * 4 + v;
      if (row >= nq) continue;
      float dot = acc[t][v];
      float val;
      if (metric == 0) {
        float two = dot + dot;
        val = cn2[col] - two;
      } else {
        val = -dot;
      }
      out[row * nlist + col] = val;
    }
  }
}

// Canonical keys (L2, or the inner product when ip) of the centroids
// rows[0, cnt), cnt <= 4, by one wave; qc holds the query's chunks
// lane, lane + 64, ... (d <= 1024).
__device__ __forceinline__ void wave_canon4(const float4* qc, const float* __restrict__ cent, int d,
                                            const int* rows, int cnt, bool ip, float* out) {
  const int lane = threadIdx.x & 63;
  const int nchunk = d >> 2;
  float4 x[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float4* row = reinterpret_cast<const float4*>(cent + (int64_t)rows[r] * d);
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int c = lane + 64 * st;
      x[r][st] = (r < cnt && c < nchunk) ? row[c] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float acc = 0.0f;
#pragma unroll
    for (int st = 0; st < 4; ++st)
      if (lane + 64 * st < nchunk) acc = ip ? chunk_ip(qc[st], x[r][st], acc) : chunk_l2(qc[st], x[r][st], acc);
    out[r] = canon_reduce64(acc);
  }
}

// One block per query.  LDS (dynamic): sel[nlist] u32, cand[P] u64 with
// P = next_pow2(nlist), plus small scratch.
template <int NT>
__global__ __launch_bounds__(NT) void probe_select_kernel(
    const float* __restrict__ q, int64_t nq, int d, const float* __restrict__ cent,
    const float* __restrict__ cn, const float* __restrict__ dprime, int nlist, int metric,
    const int32_t* __restrict__ nprobe, const int64_t* __restrict__ probe_off,
    const int64_t* __restrict__ list_off, int32_t* __restrict__ probe_lists,
    float* __restrict__ probe_keys, int64_t* __restrict__ rank_off, int64_t* __restrict__ n_scanned,
    int32_t* __restrict__ n_recheck, const int64_t* __restrict__ kc_target, int nsample, int sample_factor,
    int32_t* __restrict__ nsample_q) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int P = next_pow2(nlist);
  uint64_t* cand = reinterpret_cast<uint64_t*>(smem);
  uint32_t* sel = reinterpret_cast<uint32_t*>(smem + sizeof(uint64_t) * P);
  __shared__ uint32_t hist[256];
  __shared__ __align__(8) uint32_t bc[4];
  __shared__ uint32_t red[NT / 64];
  __shared__ float qn_s[2];

  const int64_t qi = blockIdx.x;
  const float* qv = q + qi * d;
  const int np = nprobe[qi];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;

  // |q|^2 (any order: it only scales the error bound, which has 2x margin)
  if (w == 0) {
    float s = 0.0f;
    for (int i = lane; i < d; i += 64) s = s + qv[i] * qv[i];
    for (int off = 32; off >= 1; off >>= 1) s = s + __shfl_xor(s, off);
    if (lane == 0) { qn_s[0] = s; qn_s[1] = sqrtf(s); }
  }
  __syncthreads();
  const float qn2 = qn_s[0], qn = qn_s[1];
  const float* dp = dprime + qi * (int64_t)nlist;
  const float c1 = metric != 0 ? 0.015625f : 0.03125f, c2 = 1.0f / 4096.0f;
  for (int j = threadIdx.x; j < nlist; j += NT) {
    float cj = cn[j];
    float e = c1 * qn * cj + c2 * (qn2 + cj * cj);
    sel[j] = key_bits(dp[j] + e);
  }
  __syncthreads();
  const uint32_t ustar = block_radix_select32<NT>([&](int64_t i) { return sel[i]; }, nlist, np - 1,
                                                  hist, bc);
  // recheck set
  if (threadIdx.x == 0) bc[2] = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < nlist; j += NT) {
    float cj = cn[j];
    float e = c1 * qn * cj + c2 * (qn2 + cj * cj);
    if (key_bits(dp[j] - e) <= ustar) {
      uint32_t slot = atomicAdd(&bc[2], 1u);
      sel[slot] = (uint32_t)j;  // sel[0..slot] no longer needed past this point
    }
  }
  __syncthreads();
  const int nr = (int)bc[2];
  // canonical keys: wide blocks take four lists per wave at a time (the
  // query in registers), narrow ones one list per wave (fewer registers,
  // more blocks per compute unit)
  if constexpr (NT < 1024) {
    for (int i = w; i < nr; i += NT / 64) {
      const int j = (int)sel[i];
      float key = wave_canon(qv, cent + (int64_t)j * d, d, metric != 0);
      if (metric != 0) key = -key;
      if (lane == 0) cand[i] = pack_key_id(key, (uint32_t)j);
    }
  } else {
  float4 qc[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int c = lane + 64 * st;
    qc[st] = c < (d >> 2) ? reinterpret_cast<const float4*>(qv)[c] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  for (int i = 4 * w; i < nr; i += 4 * (NT / 64)) {
    const int cnt = min(4, nr - i);
    int rows[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) rows[r] = (int)sel[i + (r < cnt ? r : 0)];
    float key[4];
    wave_canon4(qc, cent, d, rows, cnt, metric != 0, key);
    if (lane < cnt) {
      float kv = key[0];
      int jv = rows[0];
#pragma unroll
      for (int r = 1; r < 4; ++r)
        if (lane == r) { kv = key[r]; jv = rows[r]; }
      if (metric != 0) kv = -kv;
      cand[i + lane] = pack_key_id(kv, (uint32_t)jv);
    }
  }
  }
  const int PR = next_pow2(nr);
  for (int i = nr + threadIdx.x; i < PR; i += NT) cand[i] = ~0ull;
  __syncthreads();
  lds_bitonic_sort<NT>(cand, PR);
  const int64_t po = probe_off[qi];
  for (int r = threadIdx.x; r < np; r += NT) {
    uint64_t p = cand[r];
    probe_lists[po + r] = (int32_t)packed_id(p);
    probe_keys[po + r] = packed_key(p);
  }
  // exclusive prefix of list sizes in probe order (one wave)
  if (w == 0) {
    int64_t carry = 0;
    for (int base = 0; base < np; base += 64) {
      int r = base + lane;
      int64_t sz = 0;
      if (r < np) {
        int j = (int)packed_id(cand[r]);
        sz = list_off[j + 1] - list_off[j];
      }
      int64_t incl = sz;
      for (int off = 1; off < 64; off <<= 1) {
        int64_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      if (r < np) rank_off[po + r] = carry + incl - sz;
      carry += __shfl(incl, 63);
    }
    if (lane == 0) {
      n_scanned[qi] = carry;
      if (n_recheck) n_recheck[qi] = nr;
    }
    if (nsample_q) {
      // sample size: first rank r >= min(nsample, np) whose preceding lists
      // hold sample_factor * kc_target keys; np when no such rank exists
      const int nsr = nsample < np ? nsample : np;
      const int64_t kt = (int64_t)sample_factor * kc_target[qi];
      int ns = np;
      int64_t cum = 0;
      for (int base = 0; base < np && ns == np; base += 64) {
        int r = base + lane;
        int64_t sz = 0;
        if (r < np) {
          int j = (int)packed_id(cand[r]);
          sz = list_off[j + 1] - list_off[j];
        }
        int64_t incl = sz;
        for (int off = 1; off < 64; off <<= 1) {
          int64_t o = __shfl_up(incl, off);
          if (lane >= off) incl += o;
        }
        const int64_t excl = cum + incl - sz;
        const uint64_t hit = __ballot(r < np && r >= nsr && excl >= kt);
        if (hit) ns = base + __ffsll((unsigned long long)hit) - 1;
        cum += __shfl(incl, 63);
      }
      if (lane == 0) nsample_q[qi] = ns;
    }
  }
}

hipError_t launch_probe(const ProbeArgs& a, hipStream_t s) {
  dim3 g1((a.nlist + 63) / 64, (unsigned)((a.nq + 63) / 64));
  hipLaunchKernelGGL(probe_gemm_kernel, g1, dim3(256), 0, s, a.q, a.nq, a.d, a.cent_bf16, a.dpad,
                     a.cent_norm2, a.nlist, a.metric, a.dprime);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t lds = sizeof(uint64_t) * next_pow2(a.nlist) + sizeof(uint32_t) * a.nlist;
  // a batch too small to fill the device takes wide blocks (the recheck
  // of one query spread over 16 waves); otherwise narrow ones, several per
  // compute unit
  if (a.nq < 4 * (int64_t)a.num_cu)
    hipLaunchKernelGGL(probe_select_kernel<1024>, dim3((unsigned)a.nq), dim3(1024), lds, s, a.q, a.nq, a.d,
                     a.cent, a.cent_norm, a.dprime, a.nlist, a.metric, a.nprobe, a.probe_off,
                     a.list_off, a.probe_lists, a.probe_keys, a.rank_off, a.n_scanned, a.n_recheck,
                     a.kc_target, a.nsample, a.sample_factor, a.nsample_q);
  else
    hipLaunchKernelGGL(probe_select_kernel<256>, dim3((unsigned)a.nq), dim3(256), lds, s, a.q, a.nq, a.d,
                     a.cent, a.cent_norm, a.dprime, a.nlist, a.metric, a.nprobe, a.probe_off,
                     a.list_off, a.probe_lists, a.probe_keys, a.rank_off, a.n_scanned, a.n_recheck,
                     a.kc_target, a.nsample, a.sample_factor, a.nsample_q);
  return hipGetLastError();
}

size_t probe_select_lds(int nlist) {
  return sizeof(uint64_t) * next_pow2(nlist) + sizeof(uint32_t) * nlist;
}

}  // namespace bbc

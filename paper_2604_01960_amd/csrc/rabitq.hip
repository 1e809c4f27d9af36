// RaBitQ query path: the bounded quantizer the paper integrates with (the
// cited RaBitQ method; background, Observation 1, Algorithms 2 and 3).
//
//  rotate_kernel        y = P^T v for a batch of rows; y_i = sum over e of
//                       P[e][i] * v[e], product then add, e ascending from +0
//                       (a SIMT GEMM whose threads each own output elements)
//  rabitq_encode_kernel 1-bit codes and factors (nr, f, g, popcount) of the
//                       rotated residuals (index build)
//  rabitq_scan_kernel   per (query, probed list): the 4-bit quantized query
//                       side as four bit planes in LDS, then per object
//                       ip = sum_b 2^b popcount(code & plane_b) and the
//                       estimated key with its lower / upper bound
//  rabitq_walk_kernel   per query, the bounded re-rank: objects in ascending
//                       (lb, id) with R = the best k by exact (key, id), stop
//                       before an object whose lb exceeds R's k-th exact key.
//                       Run over lb bins (whole bins re-ranked, in order), as
//                       the paper's Algorithm 3 re-ranks buckets; verified,
//                       with an item-by-item heap walk when a check fails.
//
// Every FP32 formula is evaluated in the written order below (no
// contraction), the same order the oracle uses:
//   prep: vl = min y, vu = max y; delta = (vu - vl) * fl(1/15);
//     u_i = clamp(floor((y_i - vl) / delta + 0.5), 0, 15) (0 if delta = 0);
//     c1 = (2 delta) / sqrt(D); c2 = (2 vl) / sqrt(D);
//     c3 = (delta / sqrt(D)) * sum u; c4 = sqrt(D) * vl;
//   est = (((c1 * ip + c2 * pc) - c3) - c4) * f;
//   L2: key = (nr*nr + nq2) - (2 nr) * est; err = ((2 nr * sqrt(nq2)) * g) * epsc;
//   IP: key = -(ipc + nr * est);           err = ((nr * qn) * g) * epsc;
//   epsc = eps0 / sqrt(D - 1); lb = key - err; ub = key + err.
#include <hip/hip_fp16.h>
#include "common.h"
#include "kernels.h"

namespace bbc {

// ---- rotation -------------------------------------------------------------------
constexpr int ROT_TILE = 64;   // output tile per block (rows x columns)
constexpr int ROT_K = 16;      // e-chunk staged in LDS

__global__ __launch_bounds__(256) void rotate_kernel(const float* __restrict__ v, int64_t n, int D,
                                                     const float* __restrict__ P, float* __restrict__ y) {
  __shared__ float vs[ROT_TILE][ROT_K + 1];
  __shared__ float ps[ROT_K][ROT_TILE];
  const int64_t r0 = (int64_t)blockIdx.y * ROT_TILE;
  const int c0 = blockIdx.x * ROT_TILE;
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;  // 16 x 16 threads, 4 x 4 outputs each
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  for (int e0 = 0; e0 < D; e0 += ROT_K) {
    for (int idx = threadIdx.x; idx < ROT_TILE * ROT_K; idx += 256) {
      const int rr = idx / ROT_K, ee = idx % ROT_K;
      const int64_t row = r0 + rr;
      vs[rr][ee] = (row < n && e0 + ee < D) ? v[row * D + e0 + ee] : 0.0f;
      const int pe = idx / ROT_TILE, pc = idx % ROT_TILE;
      ps[pe][pc] = (e0 + pe < D && c0 + pc < D) ? P[(int64_t)(e0 + pe) * D + c0 + pc] : 0.0f;
    }
    __syncthreads();
    const int ke = min(ROT_K, D - e0);
    for (int e = 0; e < ke; ++e) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = vs[tr + 16 * i][e];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = ps[e][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float t = a[i] * b[j];
          acc[i][j] = acc[i][j] + t;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = r0 + tr + 16 * i;
    if (row >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = c0 + tc + 16 * j;
      if (col < D) y[row * D + col] = acc[i][j];
    }
  }
}

hipError_t launch_rotate(const float* v, int64_t n, int D, const float* P, float* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if ((n + ROT_TILE - 1) / ROT_TILE > 65535) return hipErrorInvalidValue;  // grid.y limit: callers chunk rows
  dim3 grid((unsigned)((D + ROT_TILE - 1) / ROT_TILE), (unsigned)((n + ROT_TILE - 1) / ROT_TILE));
  hipLaunchKernelGGL(rotate_kernel, grid, dim3(256), 0, s, v, n, D, P, y);
  return hipGetLastError();
}

// ---- index build: residuals, codes and factors ------------------------------------
__device__ __forceinline__ int list_of_slot(const int64_t* list_off, int nlist, int64_t p) {
  int lo = 0, hi = nlist - 1;  // largest j with list_off[j] <= p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (list_off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// r[p - p0] = x[list_ids[p]] - c[list(p)] for slots p in [p0, p0 + n)
__global__ void residual_rows_kernel(RabitqBuildArgs a, int64_t p0, int64_t n, float* __restrict__ r) {
  const int D = a.D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * D;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / D;
    const int e = (int)(idx % D);
    const int64_t p = p0 + row;
    const int j = list_of_slot(a.list_off, a.nlist, p);
    r[idx] = a.x[(int64_t)a.list_ids[p] * D + e] - a.cent[(int64_t)j * D + e];
  }
}

// One wave per slot p in [p0, p0 + n): y = rotated residual row (p - p0).
__global__ __launch_bounds__(256) void rabitq_encode_kernel(RabitqBuildArgs a, int64_t p0, int64_t n,
                                                            const float* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int D = a.D;
  const int64_t p = p0 + row;
  const int j = list_of_slot(a.list_off, a.nlist, p);
  const float* yr = y + row * D;
  const float* xr = a.x + (int64_t)a.list_ids[p] * D;
  const float* cr = a.cent + (int64_t)j * D;
  const float nr2 = wave_canon(xr, cr, D, false);
  uint32_t* code = a.codes + p * a.code_words;
  uint32_t pc = 0;
  for (int s = 0; s * 64 < D; ++s) {
    const uint64_t bits = __ballot(yr[s * 64 + lane] > 0.0f);
    if (lane == 0) {
      code[2 * s] = (uint32_t)bits;
      code[2 * s + 1] = (uint32_t)(bits >> 32);
    }
    pc += (uint32_t)__popcll(bits);
  }
  if (lane == 0) {
    for (int w = D / 32; w < a.code_words; ++w) code[w] = 0u;
    const float nr = sqrtf(nr2);
    float4 fac;
    if (nr == 0.0f) {
      for (int w = 0; w < D / 32; ++w) code[w] = 0u;
      fac = make_float4(0.0f, 1.0f, 0.0f, 0.0f);
    } else {
      float s1 = 0.0f;
      for (int i = 0; i < D; ++i) s1 = s1 + fabsf(yr[i]);
      const float sD = sqrtf((float)D);
      const float den = nr * sD;
      float ipoo = s1 / den;
      if (ipoo > 1.0f) ipoo = 1.0f;
      float g = ipoo * ipoo;
      g = 1.0f - g;
      g = sqrtf(g);
      g = g / ipoo;
      fac = make_float4(nr, 1.0f / ipoo, g, (float)pc);
    }
    reinterpret_cast<float4*>(a.factors)[p] = fac;
  }
}

hipError_t launch_rabitq_encode(const RabitqBuildArgs& a, int64_t p0, int64_t n, float* resid, float* rot,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t total = n * a.D;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(residual_rows_kernel, dim3(blocks), dim3(256), 0, s, a, p0, n, resid);
  hipError_t e = launch_rotate(resid, n, a.D, a.P, rot, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rabitq_encode_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, a, p0, n, rot);
  return hipGetLastError();
}

// ---- scan: bounds of every object of a (query, list) pair --------------------------
constexpr int RQ_MAXD = 2048;
constexpr int RQ_MAXW = RQ_MAXD / 32;
constexpr int RQ_MAXW_ROW = 32;  // code words per row held in registers (d <= 1024)

// Block (rank r, query q) of a 2-D grid, or block p of the pairs when the
// batch has more queries than a grid's second dimension holds.  The four
// planes of code word w sit side by side in LDS (one 16-byte read), and each
// thread takes two objects, their whole code rows loaded before any popcount.
__global__ __launch_bounds__(256) void rabitq_scan_kernel(RabitqScanArgs a) {
  constexpr int NT = 256;
  constexpr int OBJ = 2;                  // objects per thread per pass
  constexpr int CV = RQ_MAXW_ROW / 4;     // 16-byte pieces of a code row
  __shared__ float ys[RQ_MAXD];
  __shared__ uint4 planes4[RQ_MAXW];
  __shared__ float red_f[2][NT / 64];
  __shared__ uint32_t red_u[NT / 64];
  __shared__ float scal[8];

  int64_t p, qi;
  if (a.lpairs) {
    // XCD x (blocks x, x + 8, ...) takes the x-th eighth of the pairs in order
    const int64_t n = (int64_t)*a.ngroups * a.group;
    const int64_t per = (n + 7) / 8;
    const int64_t b = blockIdx.x;
    const int64_t idx = (b & 7) * per + (b >> 3);
    if ((b >> 3) >= per || idx >= n) return;
    const uint64_t e = a.lpairs[idx];
    if (e == ~0ull) return;
    qi = (int64_t)(e >> 32);
    p = a.probe_off[qi] + (int64_t)(uint32_t)e;
  } else if (a.grid2d) {
    qi = blockIdx.y;
    const int64_t pb = a.probe_off[qi], pe = a.probe_off[qi + 1];
    p = pb + blockIdx.x;
    if (p >= pe) return;
  } else {
    p = blockIdx.x;
    if (p >= a.npairs) return;
    int64_t lo = 0, hi = a.nq - 1;  // largest query with probe_off[q] <= p
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (a.probe_off[mid] <= p) lo = mid; else hi = mid - 1;
    }
    qi = lo;
  }
  const int D = a.D, W = D / 32;
  const int j = a.probe_lists[p];
  const float* qr = a.qrot + qi * D;
  const float* cr = a.rot_cent + (int64_t)j * D;
  float vmin = __builtin_inff(), vmax = -__builtin_inff();
  for (int i = threadIdx.x; i < D; i += NT) {
    const float y = a.metric == 0 ? qr[i] - cr[i] : qr[i];
    ys[i] = y;
    vmin = fminf(vmin, y);
    vmax = fmaxf(vmax, y);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    vmin = fminf(vmin, __shfl_xor(vmin, off));
    vmax = fmaxf(vmax, __shfl_xor(vmax, off));
  }
  if ((threadIdx.x & 63) == 0) { red_f[0][threadIdx.x >> 6] = vmin; red_f[1][threadIdx.x >> 6] = vmax; }
  __syncthreads();
  float vl = red_f[0][0], vu = red_f[1][0];
  for (int w = 1; w < NT / 64; ++w) { vl = fminf(vl, red_f[0][w]); vu = fmaxf(vu, red_f[1][w]); }
  const float inv15 = 1.0f / 15.0f;
  float delta = vu - vl;
  delta = delta * inv15;
  uint32_t su = 0;
  // D is a multiple of 64: a wave quantises 64 consecutive coordinates, and
  // the ballot of each bit plane is that plane's two 32-bit code words
  for (int i = threadIdx.x; i < D; i += NT) {
    uint32_t u = 0;
    if (delta > 0.0f) {
      float t = ys[i] - vl;
      t = t / delta;
      t = t + 0.5f;
      t = floorf(t);
      u = t < 0.0f ? 0u : (t > 15.0f ? 15u : (uint32_t)t);
    }
    su += u;
    const uint64_t m0 = __ballot(u & 1u), m1 = __ballot(u & 2u), m2 = __ballot(u & 4u), m3 = __ballot(u & 8u);
    if ((threadIdx.x & 63) == 0) {
      planes4[i / 32] = make_uint4((uint32_t)m0, (uint32_t)m1, (uint32_t)m2, (uint32_t)m3);
      planes4[i / 32 + 1] = make_uint4((uint32_t)(m0 >> 32), (uint32_t)(m1 >> 32), (uint32_t)(m2 >> 32), (uint32_t)(m3 >> 32));
    }
  }
  for (int off = 32; off >= 1; off >>= 1) su += __shfl_xor(su, off);
  if ((threadIdx.x & 63) == 0) red_u[threadIdx.x >> 6] = su;
  // IP: |q| from the canonical inner product of q with itself (wave 0)
  float qn = 0.0f;
  if (a.metric != 0 && threadIdx.x < 64) qn = sqrtf(wave_canon(a.q + qi * D, a.q + qi * D, D, true));
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t sum_u = 0;
    for (int w = 0; w < NT / 64; ++w) sum_u += red_u[w];
    const float sD = sqrtf((float)D);
    float c1 = 2.0f * delta;
    c1 = c1 / sD;
    float c2 = 2.0f * vl;
    c2 = c2 / sD;
    float c3 = delta / sD;
    c3 = c3 * (float)sum_u;
    const float c4 = sD * vl;
    scal[0] = c1; scal[1] = c2; scal[2] = c3; scal[3] = c4;
    const float pk = a.probe_keys[p];
    scal[4] = a.metric == 0 ? pk : -pk;  // L2: canon_l2(q, c_j); IP: canon_ip(q, c_j)
    scal[5] = qn;
  }
  __syncthreads();
  const float c1 = scal[0], c2 = scal[1], c3 = scal[2], c4 = scal[3], av = scal[4];
  const float qnv = scal[5];
  const float nq = sqrtf(av);
  const float epsc = a.eps0 / sqrtf((float)(D - 1));
  const int64_t lbeg = a.list_off[j], nobj = a.list_off[j + 1] - lbeg;
  const int64_t out0 = a.key_off[qi] + a.rank_off[p];
  const int CW = a.code_words;  // a multiple of 4, at most RQ_MAXW_ROW
  for (int64_t t0 = threadIdx.x; t0 < nobj; t0 += OBJ * NT) {
    // the query planes are read from LDS in every pass (kept in registers
    // across passes they take 128 VGPRs and halve the occupancy)
    asm volatile("" ::: "memory");
    uint4 cv[OBJ][CV];
    float4 fac[OBJ];
    bool act[OBJ];
#pragma unroll
    for (int o = 0; o < OBJ; ++o) {
      const int64_t t = t0 + o * NT;
      act[o] = t < nobj;
      const uint4* row = reinterpret_cast<const uint4*>(a.codes + (lbeg + (act[o] ? t : 0)) * CW);
#pragma unroll
      for (int v = 0; v < CV; ++v) cv[o][v] = (act[o] && 4 * v < CW) ? row[v] : make_uint4(0u, 0u, 0u, 0u);
      fac[o] = act[o] ? reinterpret_cast<const float4*>(a.factors)[lbeg + t] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    uint32_t c[OBJ][4];
#pragma unroll
    for (int o = 0; o < OBJ; ++o) c[o][0] = c[o][1] = c[o][2] = c[o][3] = 0u;
#pragma unroll
    for (int v = 0; v < CV; ++v) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int w = 4 * v + u;
        if (w < W) {
          const uint4 pv = planes4[w];
#pragma unroll
          for (int o = 0; o < OBJ; ++o) {
            const uint32_t cw = u == 0 ? cv[o][v].x : u == 1 ? cv[o][v].y : u == 2 ? cv[o][v].z : cv[o][v].w;
            c[o][0] += (uint32_t)__popc(cw & pv.x);
            c[o][1] += (uint32_t)__popc(cw & pv.y);
            c[o][2] += (uint32_t)__popc(cw & pv.z);
            c[o][3] += (uint32_t)__popc(cw & pv.w);
          }
        }
      }
    }
#pragma unroll
    for (int o = 0; o < OBJ; ++o) {
      if (!act[o]) continue;
      const int64_t t = t0 + o * NT;
      const int64_t ip = (int64_t)c[o][0] + 2 * (int64_t)c[o][1] + 4 * (int64_t)c[o][2] + 8 * (int64_t)c[o][3];
      float est = c1 * (float)ip;
      const float tpc = c2 * fac[o].w;
      est = est + tpc;
      est = est - c3;
      est = est - c4;
      est = est * fac[o].y;
      const float nr = fac[o].x;
      float key, e;
      if (a.metric == 0) {
        float tt = nr * nr;
        tt = tt + av;
        float uu = 2.0f * nr;
        uu = uu * est;
        key = tt - uu;
        e = 2.0f * nr;
        e = e * nq;
        e = e * fac[o].z;
        e = e * epsc;
      } else {
        float vv = nr * est;
        vv = av + vv;
        key = -vv;
        e = nr * qnv;
        e = e * fac[o].z;
        e = e * epsc;
      }
      a.lb[out0 + t] = key - e;
      a.ub[out0 + t] = key + e;
      if (a.key) a.key[out0 + t] = key;
    }
  }
}

hipError_t launch_rabitq_scan(const RabitqScanArgs& a, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  if (a.D > 32 * RQ_MAXW_ROW || a.D % 64 || a.code_words > RQ_MAXW_ROW || a.code_words % 4) return hipErrorInvalidValue;
  RabitqScanArgs b = a;
  b.grid2d = !a.force_1d && a.nq <= 65535 && a.max_np >= 1;
  if (a.lpairs && (a.lpairs_cap < 1 || a.lpairs_cap > 0x7fffffffLL)) return hipErrorInvalidValue;
  const dim3 g = a.lpairs ? dim3((unsigned)((a.lpairs_cap + 7) / 8 * 8))
                          : b.grid2d ? dim3((unsigned)a.max_np, (unsigned)a.nq) : dim3((unsigned)a.npairs);
  hipLaunchKernelGGL(rabitq_scan_kernel, g, dim3(256), 0, s, b);
  return hipGetLastError();
}

// ---- bounded re-rank ---------------------------------------------------------------
constexpr int WK_NB = 2048;       // lb bins
constexpr int WK_RANKCAP = WALK_RANKS_LDS;  // probe ranks in LDS
constexpr int WK_CHUNK = 1024;    // items per step of the exact walk (and per bin-walk round)
constexpr int WK_QCAP = 4096;     // objects above the k-th exact key resolved in LDS
constexpr int WK_U = 2;           // loads in flight per thread in the walk's block-wide passes
constexpr int PREP_U = 8;         // and in the wide form's bin pass

template <typename T> __device__ __forceinline__ float4 ld4(const T* p, int64_t chunk);
template <> __device__ __forceinline__ float4 ld4<float>(const float* p, int64_t chunk) {
  return reinterpret_cast<const float4*>(p)[chunk];
}
template <> __device__ __forceinline__ float4 ld4<__half>(const __half* p, int64_t chunk) {
  const uint2 v = reinterpret_cast<const uint2*>(p)[chunk];
  const float2 f0 = __half22float2(__builtin_bit_cast(__half2, v.x));
  const float2 f1 = __half22float2(__builtin_bit_cast(__half2, v.y));
  return make_float4(f0.x, f0.y, f1.x, f1.y);
}

// Exact keys (canonical L2, or -canonical IP) of up to four list positions
// (the first `cnt`), one wave; qc is the query as float4 chunks in LDS
// (lane l takes chunks l, l+64, ...; d <= 1024).
template <typename T>
__device__ void exact_keys4(const RabitqWalkArgs& a, const float4* qc, const int64_t* pos, int cnt, float* e) {
  const int lane = threadIdx.x & 63;
  const int nchunk = a.D >> 2;
  float4 x[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const T* row = reinterpret_cast<const T*>(a.vectors) + pos[r] * a.D;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int c = lane + 64 * st;
      x[r][st] = (r < cnt && c < nchunk) ? ld4<T>(row, c) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float acc = 0.0f;
#pragma unroll
    for (int st = 0; st < 4; ++st)
      if (lane + 64 * st < nchunk)
        acc = a.metric == 0 ? chunk_l2(qc[64 * st], x[r][st], acc) : chunk_ip(qc[64 * st], x[r][st], acc);
    acc = canon_reduce64(acc);
    e[r] = a.metric == 0 ? acc : -acc;
  }
}

// The exact key of one list position, one wave, in the order of exact_keys4.
template <typename T>
__device__ float exact_key1(const RabitqWalkArgs& a, const float4* qc, int64_t pos) {
  const int lane = threadIdx.x & 63;
  const int nchunk = a.D >> 2;
  const T* row = reinterpret_cast<const T*>(a.vectors) + pos * a.D;
  float4 x[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int c = lane + 64 * st;
    x[st] = c < nchunk ? ld4<T>(row, c) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  float acc = 0.0f;
#pragma unroll
  for (int st = 0; st < 4; ++st)
    if (lane + 64 * st < nchunk)
      acc = a.metric == 0 ? chunk_l2(qc[64 * st], x[st], acc) : chunk_ip(qc[64 * st], x[st], acc);
  acc = canon_reduce64(acc);
  return a.metric == 0 ? acc : -acc;
}

// Block-wide bitonic sort of keys with a payload (n a power of two).
template <int NT, typename V>
__device__ void lds_bitonic_sort_kv(uint64_t* key, V* val, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < (n >> 1); t += NT) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const uint64_t ka = key[lo], kb = key[hi];
        if ((ka > kb) == up) {
          key[lo] = kb; key[hi] = ka;
          const V v = val[lo]; val[lo] = val[hi]; val[hi] = v;
        }
      }
    }
  }
  __syncthreads();
}

// The lb bins of a query's candidate set C = {lb <= U}, U = the k-th smallest
// ub (every object when S <= k), grouped by bin: hist[b] = the end of bin b.
// In the per-query form cbuf holds C's slots; in the wide form it holds their
// lb images, cpos (when not NULL) their list positions, and so (when so.pos
// is not NULL) receives C in slot order.
struct WalkBins {
  uint32_t U, lmin;
  int shift;
  int64_t nC;
};

// C in slot order: by probe rank, then list position, so grouped by tile of
// 2^shift rows of each probed list (the order the tile-major keys read).
struct SlotOrder {
  uint32_t* pos;            // list positions
  uint32_t* idx;            // places in cbuf order
  uint32_t* bins;           // start of each (rank, tile) bin, then |C| at [nbins]
  const uint32_t* rank_tb;  // (LDS) first bin of each probe rank
  uint32_t nbins;
  int shift;
};

template <int NT, int LU>
__device__ WalkBins walk_bins(int64_t S, int64_t k, const float* lb, const float* ub, bool wide, uint32_t* cbuf,
                              int32_t* cpos, const SlotOrder& so, const SlotMap& sm, uint32_t* hist, uint32_t* rhist,
                              uint32_t* bc) {
  const int lane = threadIdx.x & 63;
  WalkBins w;
  w.U = 0xffffffffu;
  if (S > k) w.U = block_radix_select32<NT, LU>([&](int64_t i) { return key_bits(ub[i]); }, S, k - 1, rhist, bc);
  const uint32_t U = w.U;
  // C's smallest and largest lb image
  if (threadIdx.x == 0) { bc[4] = 0xffffffffu; bc[5] = 0u; bc[6] = 0u; }
  __syncthreads();
  auto lb_bits = [&](int64_t i) { return key_bits(lb[i]); };
  {
    uint32_t mn = 0xffffffffu, mx = 0u, cnt = 0;
    block_for_batched<NT, LU>(S, lb_bits, [&](int64_t, bool valid, uint32_t b) {
      if (valid && b <= U) { mn = min(mn, b); mx = max(mx, b); ++cnt; }
    });
    for (int off = 32; off >= 1; off >>= 1) {
      mn = min(mn, __shfl_xor(mn, off));
      mx = max(mx, __shfl_xor(mx, off));
      cnt += __shfl_xor(cnt, off);
    }
    if (lane == 0) { atomicMin(&bc[4], mn); atomicMax(&bc[5], mx); atomicAdd(&bc[6], cnt); }
  }
  for (int i = threadIdx.x; i < WK_NB; i += NT) hist[i] = 0;
  __syncthreads();
  w.lmin = bc[4];
  const uint32_t lmin = w.lmin;
  const uint32_t span = bc[5] - lmin;
  w.nC = bc[6];
  int shift = 0;
  while ((span >> shift) >= (uint32_t)WK_NB) ++shift;
  w.shift = shift;
  block_for_batched<NT, LU>(S, lb_bits, [&](int64_t, bool valid, uint32_t b) {
    const bool in = valid && b <= U;
    wave_hist_add(hist, in ? (b - lmin) >> shift : 0u, in);
  });
  __syncthreads();
  if (threadIdx.x < 64) {  // exclusive prefix, in place
    uint32_t carry = 0;
    for (int base = 0; base < WK_NB; base += 64) {
      const uint32_t v = hist[base + lane];
      const uint32_t incl = wave_incl_scan(v);
      hist[base + lane] = carry + incl - v;
      carry += __shfl(incl, 63);
    }
  }
  __syncthreads();
  if (so.pos) {
    // slot order: SPT consecutive slots per thread, rows of NT * SPT slots,
    // a block scan of the members per row
    constexpr int SPT = 4;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t tmask = (1u << so.shift) - 1u;
    uint32_t* s_w = rhist;  // wave totals of a row
    uint32_t carry = 0;     // members in the earlier rows
    for (int64_t row = 0; row < S; row += (int64_t)NT * SPT) {
      const int64_t i0 = row + (int64_t)SPT * threadIdx.x;
      uint32_t img[SPT];
#pragma unroll
      for (int u = 0; u < SPT; ++u) img[u] = lb_bits(min(i0 + u, S - 1));
      uint32_t cnt = 0;
#pragma unroll
      for (int u = 0; u < SPT; ++u) cnt += (i0 + u < S && img[u] <= U) ? 1u : 0u;
      const uint32_t incl = wave_incl_scan(cnt);
      if (lane == 63) s_w[wv] = incl;
      __syncthreads();
      uint32_t before = 0, tot = 0;
      for (int w2 = 0; w2 < NT / 64; ++w2) {
        const uint32_t t = s_w[w2];
        before += w2 < wv ? t : 0u;
        tot += t;
      }
      uint32_t c = carry + before + incl - cnt;
      if (i0 < S) {
        int r = sm.rank(i0);
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
          const int64_t i = i0 + u;
          if (i < S) {
            while (r + 1 < sm.np && sm.rbeg(r + 1) <= i) ++r;
            const int64_t off = i - sm.rbeg(r);
            if (((uint32_t)off & tmask) == 0) so.bins[so.rank_tb[r] + (uint32_t)(off >> so.shift)] = c;
            if (img[u] <= U) {
              const uint32_t j = atomicAdd(&hist[(img[u] - lmin) >> shift], 1u);
              const int64_t pos = sm.lbeg(r) + off;
              cbuf[j] = img[u];
              if (cpos) cpos[j] = (int32_t)pos;
              so.pos[c] = (uint32_t)pos;
              so.idx[c] = j;
              ++c;
            }
          }
        }
      }
      carry += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) so.bins[so.nbins] = carry;
  } else {
    block_for_batched<NT, LU>(S, lb_bits, [&](int64_t i, bool valid, uint32_t b) {
      if (valid && b <= U) {
        const uint32_t j = atomicAdd(&hist[(b - lmin) >> shift], 1u);
        if (wide) {
          cbuf[j] = b;
          if (cpos) cpos[j] = (int32_t)sm.pos(i);
        } else {
          cbuf[j] = (uint32_t)i;
        }
      }
    });
  }
  __syncthreads();
  return w;
}

// Wide form, step 1 (block per query): the bins of C, kept in global memory
// (bin ends in wbins, U / lmin / shift / |C| in wstate) with C's list
// positions, for the exact keys of all of C computed by a grid over the
// whole device and the walk over them.
__global__ __launch_bounds__(1024) void rabitq_walk_prep_kernel(RabitqWalkArgs a) {
  constexpr int NT = 1024;
  __shared__ int32_t s_rbeg[WK_RANKCAP];
  __shared__ int32_t s_lbeg[WK_RANKCAP];
  __shared__ uint32_t s_tb[WK_RANKCAP];
  __shared__ uint32_t hist[WK_NB];
  __shared__ uint32_t rhist[256];
  __shared__ __align__(8) uint32_t bc[16];
  const int64_t qi = blockIdx.x;
  const int64_t S = a.n_scanned[qi];
  const int np = a.nprobe[qi];
  const int64_t po = a.probe_off[qi];
  uint32_t* st = a.wstate + 4 * qi;
  SlotOrder so{};
  if (a.t_pos) {
    // the tiles of each probed list (np <= WK_RANKCAP, checked by the host),
    // their first bins by an exclusive scan
    const int64_t tr = (int64_t)1 << a.t_shift;
    for (int r = threadIdx.x; r < np; r += NT) {
      const int L = a.probe_lists[po + r];
      s_tb[r] = (uint32_t)((a.list_off[L + 1] - a.list_off[L] + tr - 1) >> a.t_shift);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      uint32_t carry = 0;
      for (int base = 0; base < np; base += 64) {
        const uint32_t v = base + lane < np ? s_tb[base + lane] : 0u;
        const uint32_t incl = wave_incl_scan(v);
        if (base + lane < np) s_tb[base + lane] = carry + incl - v;
        carry += __shfl(incl, 63);
      }
      if (lane == 0) bc[12] = carry;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < np; r += NT) a.t_rank_tb[po + r] = s_tb[r];
    so.pos = a.t_pos + a.key_off[qi];
    so.idx = a.t_idx + a.key_off[qi];
    so.bins = a.t_bins + a.t_bin_off[qi];
    so.rank_tb = s_tb;
    so.nbins = bc[12];
    so.shift = a.t_shift;
  }
  if (S == 0) {
    if (threadIdx.x == 0) {
      st[0] = 0; st[1] = 0; st[2] = 0; st[3] = 0;
      if (a.t_pos) so.bins[so.nbins] = 0;  // (every probed list is empty: no bins before)
      if (a.wround) {
        uint32_t* wr = a.wround + 4 * qi;
        wr[0] = WK_NB; wr[1] = 0; wr[2] = 0; wr[3] = 0;
      }
    }
    return;
  }
  const SlotMap sm = slot_map_load<NT, WK_RANKCAP>(a.rank_off + po, a.probe_lists + po, a.list_off, np, s_rbeg,
                                                   s_lbeg);
  const WalkBins w = walk_bins<NT, PREP_U>(S, a.k[qi], a.lb + a.key_off[qi], a.ub + a.key_off[qi], true,
                                   a.cbuf + a.key_off[qi], a.cpos ? a.cpos + a.key_off[qi] : nullptr,
                                   so, sm, hist, rhist, bc);
  for (int i = threadIdx.x; i < WK_NB; i += NT) a.wbins[qi * WK_NB + i] = hist[i];
  if (threadIdx.x == 0) { st[0] = w.U; st[1] = w.lmin; st[2] = (uint32_t)w.shift; st[3] = (uint32_t)w.nC; }
  if (a.wround && threadIdx.x == 0) {
    // first-round bins: up to the bin of the k-th smallest lb (the walk's
    // k-th exact key lies above it) plus alpha of the way to U's bin (the
    // k-th exact key lies below U when the bounds hold); everything when
    // S <= k
    const int64_t k = a.k[qi];
    int b1 = WK_NB;
    if (S > k) {
      int kb = 0;
      while (kb < WK_NB - 1 && (int64_t)hist[kb] < k) ++kb;
      const int ub = (int)min((uint32_t)(WK_NB - 1), (w.U - w.lmin) >> w.shift);
      const int ext = ub > kb ? (int)ceilf(a.round1_alpha * (float)(ub - kb)) : 0;
      b1 = min(WK_NB, kb + 1 + ext);
    }
    uint32_t* wr = a.wround + 4 * qi;
    wr[0] = (uint32_t)b1;
    wr[1] = b1 >= WK_NB ? (uint32_t)w.nC : hist[b1 - 1];
    wr[2] = 0u;
    wr[3] = 0u;
  }
}

// Wide form, step 2: exact (key, id) of every object of C, in cbuf order,
// EX_ROWS objects per block over (chunk, query).
constexpr int EX_ROWS = 64;
template <typename T>
__global__ __launch_bounds__(256) void rabitq_exact_kernel(RabitqWalkArgs a) {
  const int64_t qi = blockIdx.y;
  // places of C whose keys this launch computes: all, or one round's
  int64_t lo = 0, nC = a.wstate[4 * qi + 3];
  if (a.round) {
    const uint32_t* wr = a.wround + 4 * qi;
    if (a.round == 1) nC = min(nC, (int64_t)wr[1]);
    else if (wr[2] == 0) return;
    else lo = wr[1];
  }
  const int64_t i0 = lo + (int64_t)blockIdx.x * EX_ROWS;
  if (i0 >= nC) return;  // block-uniform
  __shared__ float4 s_qc[256];
  const float* q = a.q + qi * a.D;
  for (int c = threadIdx.x; c < 256; c += 256)
    s_qc[c] = c < (a.D >> 2) ? reinterpret_cast<const float4*>(q)[c] : make_float4(0.f, 0.f, 0.f, 0.f);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int32_t* cpos = a.cpos + a.key_off[qi];
  uint64_t* pbuf = a.cand_packed + a.cand_off[qi];
  const int64_t i1 = min(nC, i0 + EX_ROWS);
  for (int64_t i = i0 + 4 * wv; i < i1; i += 16) {
    const int cnt = (int)min((int64_t)4, i1 - i);
    int64_t pos[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) pos[r] = cpos[i + (r < cnt ? r : 0)];
    float e[4];
    exact_keys4<T>(a, s_qc + lane, pos, cnt, e);
    if (lane < cnt) {
      float ev = e[0];
      int64_t pv = pos[0];
#pragma unroll
      for (int r = 1; r < 4; ++r)
        if (lane == r) { ev = e[r]; pv = pos[r]; }
      pbuf[i + lane] = pack_key_id(ev, (uint32_t)a.list_ids[pv]);
    }
  }
}

// WIDE: the exact keys of all of C are in cand_packed before the walk (the
// wide form); then the kernel computes no exact key except in the item walk,
// and fits two blocks per compute unit.
constexpr int WK_NT = 1024;
template <typename T, bool WIDE>
__global__ __launch_bounds__(WK_NT, WIDE ? 8 : 1) void rabitq_walk_kernel(RabitqWalkArgs a) {
  constexpr int NT = WK_NT;
  constexpr int NW = NT / 64;
  __shared__ int32_t s_rbeg[WK_RANKCAP];
  __shared__ int32_t s_lbeg[WK_RANKCAP];
  __shared__ uint32_t hist[WK_NB];
  __shared__ uint32_t rhist[256];
  __shared__ __align__(8) uint32_t bc[16];
  __shared__ uint64_t chunk_v[WK_QCAP];    // (lb image, id) keys, sorted
  __shared__ uint32_t chunk_x[WK_QCAP];    // their exact images

  const int64_t qi = blockIdx.x;
  const int64_t S = a.n_scanned[qi];
  const int64_t k = a.k[qi];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // two rounds (wide form): round 2 walks only the queries round 1 marked
  uint32_t* wr = WIDE && a.round ? a.wround + 4 * qi : nullptr;
  if (WIDE && a.round == 2 && wr[2] == 0) return;  // block-uniform
  if (S == 0) {
    if (threadIdx.x == 0) {
      a.n_cand[qi] = 0;
      if (a.n_visited) a.n_visited[qi] = 0;
      if (a.t_qpath) a.t_qpath[qi] = 0;
    }
    return;
  }
  const int64_t po = a.probe_off[qi];
  const SlotMap sm = slot_map_load<NT, WK_RANKCAP>(a.rank_off + po, a.probe_lists + po, a.list_off, a.nprobe[qi],
                                                   s_rbeg, s_lbeg);
  const float* lb = a.lb + a.key_off[qi];
  const float* ub = a.ub + a.key_off[qi];
  uint32_t* cbuf = a.cbuf + a.key_off[qi];
  uint64_t* pbuf = a.cand_packed + a.cand_off[qi];
  const float* q = a.q + qi * a.D;
  __shared__ float4 s_qc[256];  // the query, lane l's chunks at l, l + 64, ...
  for (int c = threadIdx.x; c < 256; c += NT)
    s_qc[c] = c < (a.D >> 2) ? reinterpret_cast<const float4*>(q)[c] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float4* qc = s_qc + lane;
  const int64_t capq = a.key_off[qi + 1] - a.key_off[qi];
  uint64_t* zA = a.zbuf + 2 * a.key_off[qi];
  uint64_t* zB = zA + capq;

  // number of the n images get(i) strictly below L (block-wide; bc[15] as
  // the counter; ends with a barrier)
  auto count_below = [&](int64_t n, auto get, uint32_t L) -> int64_t {
    if (threadIdx.x == 0) bc[15] = 0;
    __syncthreads();
    uint32_t cnt = 0;
    block_for_batched<NT, WK_U>(n, get, [&](int64_t, bool valid, uint32_t v) { cnt += (valid && v < L) ? 1u : 0u; });
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (lane == 0 && cnt) atomicAdd(&bc[15], cnt);
    __syncthreads();
    const int64_t r = bc[15];
    __syncthreads();
    return r;
  };
  // the bins of C: computed here, or (wide form) read back with the exact
  // keys of all of C already in pbuf
  WalkBins w;
  if constexpr (WIDE) {
    const uint32_t* st = a.wstate + 4 * qi;
    w.U = st[0]; w.lmin = st[1]; w.shift = (int)st[2]; w.nC = st[3];
    for (int i = threadIdx.x; i < WK_NB; i += NT) hist[i] = a.wbins[qi * WK_NB + i];
    __syncthreads();
  } else {
    w = walk_bins<NT, WK_U>(S, k, lb, ub, false, cbuf, nullptr, SlotOrder{}, sm, hist, rhist, bc);
  }
  const uint32_t U = w.U, lmin = w.lmin;
  const int shift = w.shift;
  const int64_t nC = w.nC;
  // lb image of the object at place i of C's bin order
  auto lb_img = [&](int64_t i) -> uint32_t {
    if constexpr (WIDE) return cbuf[i];
    else return key_bits(lb[cbuf[i]]);
  };
  // hist[b] is now the end of bin b in cbuf.  Walk whole bins in order.
  auto lower_edge = [&](int b) -> uint64_t { return (uint64_t)lmin + ((uint64_t)b << shift); };
  // exact keys of cbuf[i0, i1) into pbuf, four rows per wave
  auto rerank_range = [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0 + 4 * wv; i < i1; i += 4 * NW) {
      const int cnt = (int)min((int64_t)4, i1 - i);
      int64_t pos[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) pos[r] = sm.pos(cbuf[i + (r < cnt ? r : 0)]);
      float e[4];
      exact_keys4<T>(a, qc, pos, cnt, e);
      if (lane < cnt) {
        float ev = e[0];
        int64_t pv = pos[0];
#pragma unroll
        for (int r = 1; r < 4; ++r)
          if (lane == r) { ev = e[r]; pv = pos[r]; }
        pbuf[i + lane] = pack_key_id(ev, (uint32_t)a.list_ids[pv]);
      }
    }
  };
  int64_t p = 0;
  uint32_t Eimg = 0xffffffffu;
  bool exhausted = false;
  if constexpr (WIDE) {
    // The exact keys of all of C are known, so the processed set P is the
    // shortest prefix of whole bins [0, b) after which the walk stops for
    // certain: P holds at least k objects whose exact image lies below the
    // lower edge of bin b, i.e. whose lb bin and exact-image bin (images
    // below lmin in bin 0) are both below b.  A histogram of the larger of
    // the two bins gives that count for every b in one pass over C.
    if (S <= k) {
      p = nC;
      exhausted = true;
    } else {
      uint32_t* H = reinterpret_cast<uint32_t*>(chunk_v);  // WK_NB counters
      for (int i = threadIdx.x; i < WK_NB; i += NT) H[i] = 0;
      __syncthreads();
      // round 1 knows the keys of C's first bins only (places below
      // lim): the counts of every b up to those bins are exact, since an
      // object of a later bin counts for no b up to its own bin
      const int64_t lim = a.round == 1 ? (int64_t)wr[1] : nC;
      // each wave takes a contiguous range of C and follows the bin ends
      const int64_t per = ((lim + NW - 1) / NW + 63) & ~(int64_t)63;
      const int64_t w0 = (int64_t)wv * per, w1 = min(lim, w0 + per);
      const uint32_t* ximg = reinterpret_cast<const uint32_t*>(pbuf) + 1;  // exact image of place i at 2 i
      int bn = 0;  // the first bin whose end exceeds the lane's place
      {
        const int64_t i0 = w0 + lane;
        int lo = 0, hi = WK_NB - 1;  // hist[WK_NB - 1] = nC
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if ((int64_t)hist[mid] > i0) hi = mid; else lo = mid + 1;
        }
        bn = lo;
      }
      constexpr int HU = 8;
      for (int64_t base = w0; base < w1; base += 64 * HU) {
        uint32_t img[HU];
#pragma unroll
        for (int u = 0; u < HU; ++u) img[u] = ximg[2 * min(base + 64 * u + lane, w1 - 1)];
#pragma unroll
        for (int u = 0; u < HU; ++u) {
          const int64_t i = base + 64 * u + lane;
          const bool valid = i < w1;
          uint32_t m = WK_NB;
          if (valid) {
            while ((int64_t)hist[bn] <= i) ++bn;
            const uint32_t eb = img[u] < lmin ? 0u : (img[u] - lmin) >> shift;
            m = max((uint32_t)bn, eb);
          }
          wave_hist_add(H, m, valid && m < (uint32_t)WK_NB);
        }
      }
      __syncthreads();
      if (threadIdx.x < 64) {  // the first m whose inclusive count reaches k
        uint32_t carry = 0;
        int found = WK_NB;
        for (int base = 0; base < WK_NB; base += 64) {
          const uint32_t incl = carry + wave_incl_scan(H[base + lane]);
          const uint64_t hit = __ballot((int64_t)incl >= k);
          if (hit) {
            found = base + __ffsll((unsigned long long)hit) - 1;
            break;
          }
          carry = __shfl(incl, 63);
        }
        if (lane == 0) bc[13] = (uint32_t)found;
      }
      __syncthreads();
      const int found = (int)bc[13];
      const int b = found < WK_NB ? found + 1 : WK_NB;
      if (a.round == 1 && (found >= WK_NB || b > (int)wr[0]) && lim < nC) {
        // the stop point lies beyond the first round's bins: round 2
        if (threadIdx.x == 0) {
          wr[2] = 1u;
          if (a.n_visited) a.n_visited[qi] = nC;
        }
        return;
      }
      p = hist[b - 1];
      exhausted = p >= nC;
      Eimg = block_radix_select32<NT, WK_U>([&](int64_t i) { return ximg[2 * i]; }, p, k - 1, rhist, bc);
    }
  } else {
    // Z = the processed (exact, id) that can still be among the k best: all
    // of them until k are processed, then those whose key image is at most
    // E, the k-th smallest key image (ties at E included).
    int64_t nz = 0;
    int b_end = 0;
    while (true) {
      const int64_t target = p < k ? max(k, (int64_t)WK_CHUNK) : p + WK_CHUNK;
      int b = b_end;
      while (b < WK_NB && (int64_t)hist[b] < target) ++b;
      if (b < WK_NB) ++b;  // the bin that reaches the target
      const int64_t np_ = b > 0 ? (int64_t)hist[b - 1] : 0;
      b_end = b;
      rerank_range(p, np_);
      if (threadIdx.x == 0) bc[13] = 0;
      __syncthreads();
      block_for_batched<NT, WK_U>(np_ - p, [&](int64_t j) { return pbuf[p + j]; },
                               [&](int64_t, bool valid, uint64_t v) {
                                 const bool take = valid && (p < k || (uint32_t)(v >> 32) <= Eimg);
                                 const uint32_t slot = wave_slot(take, &bc[13]);
                                 if (take) zA[nz + slot] = v;
                               });
      __syncthreads();
      nz += bc[13];
      p = np_;
      if (p >= k) {
        Eimg = block_radix_select32<NT, WK_U>([&](int64_t i) { return (uint32_t)(zA[i] >> 32); }, nz, k - 1, rhist, bc);
        if (threadIdx.x == 0) bc[13] = 0;
        __syncthreads();
        block_for_batched<NT, WK_U>(nz, [&](int64_t i) { return zA[i]; }, [&](int64_t, bool valid, uint64_t v) {
          const bool take = valid && (uint32_t)(v >> 32) <= Eimg;
          const uint32_t slot = wave_slot(take, &bc[13]);
          if (take) zB[slot] = v;
        });
        __syncthreads();
        nz = bc[13];
        uint64_t* t = zA; zA = zB; zB = t;
      }
      if (b_end >= WK_NB || p >= nC) { exhausted = true; break; }
      if (p >= k && lower_edge(b_end) > (uint64_t)Eimg) break;
    }
  }
  const uint32_t E = Eimg;  // k-th smallest exact key image among the processed
  // The processed set P is a prefix of the (lb, id) order.  The oracle's walk
  // visits every object of P with lb <= E, and it stops at the latest at the
  // object after P (its lb exceeds E: the next bin starts above E, or, when
  // C is used up, lb > U >= E, which is checked).  Only the objects of P with
  // lb > E (set Q) need ordering: the walk stops at the first t of Q (in
  // (lb, id) order) with lb_t > the k-th exact key of (P minus Q) and Q[0, t),
  // a predicate monotone in t, found by binary search.
  bool ok = true;
  int64_t nvis = p;
  int qpath = 0;
  if (S > k) {
    if (exhausted && p < S && E > U) ok = false;
    if (threadIdx.x == 0) { bc[7] = 0; bc[14] = 0; }
    __syncthreads();
    // (lb image, exact image) of processed object i
    auto lb_ex = [&](int64_t i) { return make_uint2(lb_img(i), (uint32_t)(pbuf[i] >> 32)); };
    {
      uint32_t nab = 0;
      bool member = false;
      block_for_batched<NT, WK_U>(p, lb_ex, [&](int64_t, bool valid, uint2 e) {
        if (valid && e.x > E) {
          ++nab;
          member |= e.y <= E;  // a possible result object above E
        }
      });
      for (int off = 32; off >= 1; off >>= 1) nab += __shfl_xor(nab, off);
      if (lane == 0 && nab) atomicAdd(&bc[14], nab);
      if (member) bc[7] = 1;
    }
    __syncthreads();
    const bool member_above = bc[7] != 0;
    const int64_t nQ = bc[14];
    if (ok && member_above) {
      // Z0 = the objects of P minus Q whose key image is at most the k-th
      // smallest image among them (all of them when fewer than k)
      const int64_t n0 = p - nQ;
      uint32_t thr0 = 0xffffffffu;
      if (n0 > k)
        thr0 = block_radix_select32<NT, WK_U>(
            [&](int64_t i) { return lb_img(i) <= E ? (uint32_t)(pbuf[i] >> 32) : 0xffffffffu; }, p,
            k - 1, rhist, bc);
      if (threadIdx.x == 0) bc[13] = 0;
      __syncthreads();
      block_for_batched<NT, WK_U>(p, [&](int64_t i) { return make_ulonglong2(lb_img(i), pbuf[i]); },
                               [&](int64_t, bool valid, ulonglong2 e) {
                                 const bool take = valid && e.x <= E && (uint32_t)(e.y >> 32) <= thr0;
                                 const uint32_t slot = wave_slot(take, &bc[13]);
                                 if (take) zB[slot] = e.y;
                               });
      __syncthreads();
      const int64_t nz0 = bc[13];
      const int64_t kz = min(k, n0);  // objects of R that Z0 provides
      int64_t lo = max((int64_t)0, k - kz), hi = nQ;
      uint64_t cut = ~0ull;
      qpath = nQ <= (a.qcap > 0 && a.qcap < WK_QCAP ? a.qcap : WK_QCAP) ? 1 : 2;
      if (qpath == 1) {
        // Q sorted in LDS by (lb image, id), with its exact (key, id)
        if (threadIdx.x == 0) bc[9] = 0;
        __syncthreads();
        block_for_batched<NT, WK_U>(p, [&](int64_t i) { return make_ulonglong2(lb_img(i), pbuf[i]); },
                                 [&](int64_t, bool valid, ulonglong2 e) {
                                   if (valid && e.x > E) {
                                     const uint32_t j = atomicAdd(&bc[9], 1u);
                                     chunk_v[j] = (e.x << 32) | (uint64_t)(uint32_t)e.y;
                                     chunk_x[j] = (uint32_t)(e.y >> 32);
                                   }
                                 });
        const int P2 = next_pow2((int)nQ);
        for (int i = (int)nQ + threadIdx.x; i < P2; i += NT) { chunk_v[i] = ~0ull; chunk_x[i] = ~0u; }
        lds_bitonic_sort_kv<NT>(chunk_v, chunk_x, P2);
        // first t in [lo, nQ) with lb(Q[t]) > the k-th key of Z0 and Q[0, t),
        // i.e. with at least k of those keys below lb(Q[t])
        while (lo < hi) {
          const int64_t t = (lo + hi) >> 1;
          const uint32_t L = (uint32_t)(chunk_v[t] >> 32);
          const int64_t below = count_below(
              nz0 + t, [&](int64_t i) { return i < nz0 ? (uint32_t)(zB[i] >> 32) : chunk_x[i - nz0]; }, L);
          if (below >= k) hi = t; else lo = t + 1;
        }
        if (lo < nQ) cut = chunk_v[lo];
      } else {
        // the same search with Q left in place: Q[t] by a radix select over
        // the (lb image, id) keys of Q, Q[0, t) as the keys below it
        auto qkey = [&](int64_t i, uint64_t& v) -> bool {
          const uint32_t lbi = lb_img(i);
          v = ((uint64_t)lbi << 32) | (uint64_t)(uint32_t)pbuf[i];
          return lbi > E;
        };
        while (lo < hi) {
          const int64_t t = (lo + hi) >> 1;
          const uint64_t kt = block_radix_select64<NT, WK_U>(qkey, p, t, rhist, bc);
          const uint32_t L = (uint32_t)(kt >> 32);
          const int64_t below = count_below(
              nz0 + p,
              [&](int64_t i) -> uint32_t {
                if (i < nz0) return (uint32_t)(zB[i] >> 32);
                uint64_t v;
                const bool inq = qkey(i - nz0, v);
                return (inq && v < kt) ? (uint32_t)(pbuf[i - nz0] >> 32) : 0xffffffffu;
              },
              L);
          if (below >= k) hi = t; else lo = t + 1;
        }
        if (lo < nQ) cut = block_radix_select64<NT, WK_U>(qkey, p, lo, rhist, bc);
      }
      // visited: P minus the objects of Q from position lo on
      if (lo < nQ) {
        if (threadIdx.x == 0) bc[13] = 0;
        __syncthreads();
        block_for_batched<NT, WK_U>(p, [&](int64_t i) { return make_ulonglong2(lb_img(i), pbuf[i]); },
                                 [&](int64_t, bool valid, ulonglong2 e) {
                                   const bool take = valid && ((e.x << 32) | (uint64_t)(uint32_t)e.y) < cut;
                                   const uint32_t slot = wave_slot(take, &bc[13]);
                                   if (take) zB[slot] = e.y;
                                 });
        __syncthreads();
        nvis = bc[13];
        for (int64_t i = threadIdx.x; i < nvis; i += NT) pbuf[i] = zB[i];
        __syncthreads();
      }
    }
  }
  // exact distances computed: the visited objects; in the wide form all of
  // C, or of the first round's bins when round 1 settled the query
  const int64_t n_exact = !WIDE ? nvis : (a.round == 1 ? (int64_t)wr[1] : nC);
  if (ok) {
    if (threadIdx.x == 0) {
      a.n_cand[qi] = nvis;
      if (a.n_visited) a.n_visited[qi] = n_exact;
      if (a.t_qpath) a.t_qpath[qi] = qpath;
    }
    return;
  }

  // ---- exact walk, item by item: chunks of the next WK_CHUNK objects in
  // (lb, id) order, their exact keys, then one wave offers them in order to
  // a 64-ary max-heap of the best k (in pbuf), stopping by the rule.
  auto packed_lb = [&](int64_t i) -> uint64_t {
    return ((uint64_t)key_bits(lb[i]) << 32) | (uint64_t)(uint32_t)a.list_ids[sm.pos(i)];
  };
  uint64_t last = 0;
  bool have_last = false;
  int64_t nr = 0, visited = 0;
  uint64_t top = 0;
  bool stop = false;
  while (!stop) {
    if (threadIdx.x == 0) bc[8] = 0;
    __syncthreads();
    {
      uint32_t cnt = 0;
      for (int64_t i = threadIdx.x; i < S; i += NT) cnt += (!have_last || packed_lb(i) > last) ? 1u : 0u;
      for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
      if (lane == 0 && cnt) atomicAdd(&bc[8], cnt);
    }
    __syncthreads();
    const int64_t rem = bc[8];
    if (rem == 0) break;
    const int64_t nb = min((int64_t)WK_CHUNK, rem);
    const uint64_t thr = block_radix_select64<NT, WK_U>(
        [&](int64_t i, uint64_t& v) -> bool {
          v = packed_lb(i);
          return !have_last || v > last;
        },
        S, nb - 1, rhist, bc);
    if (threadIdx.x == 0) bc[9] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < S; i += NT) {
      const uint64_t v = packed_lb(i);
      if ((!have_last || v > last) && v <= thr) chunk_v[atomicAdd(&bc[9], 1u)] = v;
    }
    // the chunk in (lb, id) order; an object's id gives its list position
    const int P2 = next_pow2((int)nb);
    for (int i = (int)nb + threadIdx.x; i < P2; i += NT) chunk_v[i] = ~0ull;
    lds_bitonic_sort<NT>(chunk_v, P2);
    for (int i = wv; i < (int)nb; i += NW) {
      const uint32_t id = (uint32_t)chunk_v[i];
      const float ex = exact_key1<T>(a, qc, (int64_t)a.pos_of_id[id]);
      if (lane == 0) chunk_x[i] = key_bits(ex);
    }
    __syncthreads();
    if (wv == 0) {
      for (int i = 0; i < (int)nb; ++i) {
        const uint32_t lbi = (uint32_t)(chunk_v[i] >> 32);
        if (nr == k && lbi > (uint32_t)(top >> 32)) { stop = true; break; }
        const uint64_t e = ((uint64_t)chunk_x[i] << 32) | (uint32_t)chunk_v[i];
        ++visited;
        if (nr < k) {
          if (lane == 0) hstore(pbuf + nr, e);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
          ++nr;
          if (nr == k) {
            for (int64_t node = (k - 2) / 64; node >= 0; --node) heap_sift_down(pbuf, k, node, hload(pbuf + node));
            top = hload(pbuf);
          }
        } else if (e < top) {
          heap_sift_down(pbuf, k, 0, e);
          top = hload(pbuf);
        }
      }
      if (lane == 0) { bc[10] = stop ? 1u : 0u; bc[11] = (uint32_t)nr; bc[12] = (uint32_t)visited; }
    }
    __syncthreads();
    stop = bc[10] != 0;
    nr = bc[11];
    visited = bc[12];
    last = thr;
    have_last = true;
    __syncthreads();
  }
  // the item walk visits a prefix of the (lb, id) order, of which C is a prefix too
  if (threadIdx.x == 0) {
    a.n_cand[qi] = nr;
    if (a.n_visited) a.n_visited[qi] = WIDE ? max(n_exact, visited) : visited;
    if (a.t_qpath) a.t_qpath[qi] = 3;
  }
}

hipError_t launch_rabitq_walk_prep(const RabitqWalkArgs& a, hipStream_t s) {
  if (a.nq <= 0 || !a.wide) return hipSuccess;
  hipLaunchKernelGGL(rabitq_walk_prep_kernel, dim3((unsigned)a.nq), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rabitq_walk(const RabitqWalkArgs& a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  if (a.wide && !a.keys_ready) {
    if (a.nq > 65535 || a.max_c < 1) return hipErrorInvalidValue;
    const dim3 g((unsigned)((a.max_c + EX_ROWS - 1) / EX_ROWS), (unsigned)a.nq);
    if (a.fp16) hipLaunchKernelGGL(rabitq_exact_kernel<__half>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(rabitq_exact_kernel<float>, g, dim3(256), 0, s, a);
  }
  const dim3 g((unsigned)a.nq), b(WK_NT);
  if (a.wide) {
    if (a.fp16) hipLaunchKernelGGL((rabitq_walk_kernel<__half, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((rabitq_walk_kernel<float, true>), g, b, 0, s, a);
  } else {
    if (a.fp16) hipLaunchKernelGGL((rabitq_walk_kernel<__half, false>), g, b, 0, s, a);
    else hipLaunchKernelGGL((rabitq_walk_kernel<float, false>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace bbc

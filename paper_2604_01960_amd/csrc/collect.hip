// Bucket-based result collector on the GPU (result-buffer section of the
// paper: Push / Update / Collect, the codebook from a sample of the nearest
// clusters, and the bucket-id equation).
//
// The path runs in two kernels here, one block of 1024 threads per query:
//  * codebook_kernel, after the scan of the first nsample probed lists (the
//    sample).  T = min(K_c, |sample|); d_min / d_max are the smallest and the
//    T-th smallest sample key; delta = (d_max - d_min) / 256 (1 if that is
//    not positive); the 256 equal-width cells are mapped onto m buckets of
//    equal depth w.r.t. the sample's T smallest keys:
//    map[e] = min(m-1, floor(m * C_<e / T)).  When the sample already holds
//    K_c keys, d_max is a relaxed threshold: at least K_c scanned keys are
//    <= d_max, so no key above it can be a candidate, and every key above it
//    falls in the last cell.  Such keys are only counted (the "Push" of the
//    paper rejects them); the others are appended to the query's survivor
//    list as (key, list slot).  The sample's own keys go through the same
//    filter here; the remaining lists go through it in the scan kernel.
//  * collect_bucket_kernel over the survivors.  Histogram with
//    bucket(key) = map[clamp(floor((key - d_min)/delta), 0, 255)] (the
//    rejected keys are added to the last cell's bucket, so the counts are
//    those of all scanned keys); Update: tau = first bucket whose running
//    count reaches K_c, s = K_c - (count below tau); Collect: every survivor
//    of a bucket below tau, plus the first s of bucket tau by (key, id),
//    sorted in LDS (an exact radix select when they do not fit).
// Because the per-list cadence of the paper only ever lowers tau, the tau of
// the full histogram equals the final tau of the once-per-list Update, and
// the result is exactly the K_c smallest (key, id).  Candidate slots come
// from LDS atomics, so their order is arbitrary; the set is not.
#include "common.h"
#include "kernels.h"

namespace bbc {

constexpr int COLLECT_RANKCAP = 2048;
constexpr int COLLECT_CHUNKCAP = 4096;  // 64-survivor chunks mapped to their run by an LDS table
template <int N> struct Unroll { static constexpr int value = N; };

// cell_of(key, dmin, delta) with a reciprocal (rdelta = rcp(delta), within
// 1 ulp): for quotients below 512, q = (key - dmin) * rdelta lies within
// 2^-13 of the exact quotient, so when q is more than 2^-11 away from every
// integer the correctly rounded quotient has the same floor.  Otherwise (and
// for NaN from a flushed reciprocal) the quotient is formed by division.
__device__ __forceinline__ int cell_fast(float key, float dmin, float delta, float rdelta) {
  const float q = (key - dmin) * rdelta;
  if (q >= 256.0f) return 255;
  const float n = floorf(q);
  const float f = q - n;
  if (f > 0x1p-11f && f < 1.0f - 0x1p-11f) return n < 0.0f ? 0 : (n > 255.0f ? 255 : (int)n);
  return cell_of(key, dmin, delta);
}
constexpr int COLLECT_UNROLL = 4;       // chunks a wave has in flight

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

// Keys of the sample held in registers per thread, as their 32-bit images:
// key j * 1024 + t in slot j of thread t.  R = 0 reads them from memory in
// every pass instead; a query whose sample exceeds 1024 * R keys takes that
// path too.
template <int R>
__global__ __launch_bounds__(1024, R == 0 ? 8 : 1) void codebook_kernel(CollectArgs a) {
  constexpr int NT = 1024, NW = NT / 64;
  constexpr int SEL_BITS = 12;  // bits of the key image resolved per select pass
  __shared__ uint32_t hist[1 << SEL_BITS];
  // memory form: the keys of the bin the first select pass picks, when they
  // fit, for the remaining passes
  constexpr int GCAP = R == 0 ? 4096 : 1;
  __shared__ uint32_t gkeys[GCAP];
  __shared__ uint8_t cmap[256];
  __shared__ __align__(8) uint32_t bc[8];
  __shared__ uint32_t s_wred[2][NW];
  __shared__ float fbc[2];
  __shared__ int32_t s_cpred;  // early re-rank: cell of the sample's jp-th smallest key (-1: none)
  __shared__ int32_t s_cfilt;  // tighter filter: its last cell (-1: none)
  __shared__ uint32_t s_nfilt; // and the sample keys in cells up to it

  const int64_t qi = a.qorder ? (int64_t)a.qorder[blockIdx.x] : (int64_t)blockIdx.x;
  const int64_t S = a.n_scanned[qi];
  int64_t kc = a.kc_target[qi];
  if (kc > S) kc = S;
  const int np = a.nprobe[qi];
  const int64_t po = a.probe_off[qi];
  const int64_t* rank_off = a.rank_off + po;
  const int32_t* lists = a.probe_lists + po;
  const float* keys = a.sample_keys + a.sample_off[qi];
  const int m = a.m;
  QueryBook* book = a.books + qi;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;

  const int nsr = a.nsample_q[qi];
  const int64_t Ts = nsr < np ? rank_off[nsr] : S;
  __shared__ int32_t s_rbeg[COLLECT_RANKCAP];
  __shared__ int32_t s_lbeg[COLLECT_RANKCAP];
  const bool lds_ranks = nsr <= COLLECT_RANKCAP;
  if (lds_ranks)
    for (int r = threadIdx.x; r < nsr; r += NT) {
      s_rbeg[r] = (int32_t)rank_off[r];
      s_lbeg[r] = (int32_t)a.list_off[lists[r]];
    }
  const bool in_regs = R > 0 && Ts > 0 && Ts <= (int64_t)NT * R;
  // chunk -> rank of its first slot, for the register path's positions
  __shared__ uint16_t s_crank[R > 0 ? R * NT / 64 : 1];
  const bool ctab = in_regs && lds_ranks;
  if (ctab) {
    __syncthreads();  // s_rbeg
    for (int r = threadIdx.x; r < nsr; r += NT) {
      const int64_t rb = s_rbeg[r], re = r + 1 < nsr ? (int64_t)s_rbeg[r + 1] : Ts;
      for (int64_t ch = (rb + 63) >> 6; ch * 64 < re; ++ch) s_crank[ch] = (uint16_t)r;
    }
  }
  // list position of sample slot i; r is the probe rank of the previous slot
  // this thread asked for (slots are asked for in increasing order), and
  // becomes the rank of i.  With the chunk table (register path), the rank
  // of the 64-slot chunk's first slot starts the search instead.
  auto pos_at = [&](int64_t i, int& r) -> int64_t {
    if (!lds_ranks) return slot_to_pos(i, rank_off, lists, a.list_off, nsr);
    if (ctab) {
      r = s_crank[i >> 6];
      while (r + 1 < nsr && (int64_t)s_rbeg[r + 1] <= i) ++r;
      return (int64_t)s_lbeg[r] + (i - s_rbeg[r]);
    }
    if (r + 1 < nsr && (int64_t)s_rbeg[r + 1] <= i) {
      int lo = r + 1, hi = nsr - 1;
      if (lo < hi && (int64_t)s_rbeg[lo + 1] > i) hi = lo;  // usually the next list
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_rbeg[mid] <= i) lo = mid; else hi = mid - 1;
      }
      r = lo;
    }
    return (int64_t)s_lbeg[r] + (i - s_rbeg[r]);
  };

  // the sample's key images, once from memory into registers when they fit
  uint32_t kv[R > 0 ? R : 1];
  if constexpr (R > 0) {
    if (in_regs) {
      // unconditional loads (slots past the end read the last key), all
      // issued before any key is converted to its image
      const int last = (int)Ts - 1;
#pragma unroll
      for (int j = 0; j < R; ++j) kv[j] = __float_as_uint(keys[min(j * NT + (int)threadIdx.x, last)]);
#pragma unroll
      for (int j = 0; j < R; ++j) kv[j] = key_bits(__uint_as_float(kv[j]));
    }
  }
  // use(i, valid, image) for every sample slot i, in increasing i per
  // thread, the same block-uniform number of times on every lane (valid =
  // false past Ts).  In registers, rows j < jfull are whole and row jfull
  // holds the tail (validity from two values, nothing kept per row).
  const int jfull = (int)(Ts / NT);
  const bool tail_ok = (int64_t)threadIdx.x < Ts - (int64_t)jfull * NT;
  const bool tail_rows = Ts > (int64_t)jfull * NT;  // row jfull holds keys
  auto each = [&](auto&& use) {
    if constexpr (R > 0) {
      if (in_regs) {
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (j < jfull || (j == jfull && tail_rows))
            use((int64_t)(j * NT + (int)threadIdx.x), j < jfull || tail_ok, kv[j]);
        return;
      }
    }
    block_for_batched<NT, 8>(Ts, [&](int64_t i) { return key_bits(keys[i]); }, use);
  };

  if (a.t_nsample_keys && threadIdx.x == 0) a.t_nsample_keys[qi] = Ts;
  const int64_t T = kc < Ts ? kc : Ts;
  uint32_t dmax_b = 0;
  // the sample's keys through the relaxed-threshold filter go to rank 0's
  // survivor run; with the sample read from memory this happens in the pass
  // of the cell histogram (one pass less over the sample)
  float* skey = a.surv_key + a.surv_off[qi];
  uint32_t* spos = a.surv_pos + a.surv_off[qi];
  int rk = 0;
  bool filtered = false;
  if (threadIdx.x == 0) { bc[6] = 0; bc[7] = 0; }
  if (T > 0) {
    // smallest and largest image of the sample (kept by the sample scan when
    // it has them: one pass less over the sample)
    uint32_t mn = 0xffffffffu, mx = 0u;
    if (a.smin) {
      mn = a.smin[qi];
      mx = a.smax[qi];
    } else {
      each([&](int64_t, bool valid, uint32_t v) {
        if (valid) {
          mn = min(mn, v);
          mx = max(mx, v);
        }
      });
      for (int off = 32; off >= 1; off >>= 1) {
        mn = min(mn, __shfl_xor(mn, off));
        mx = max(mx, __shfl_xor(mx, off));
      }
      if (lane == 0) {
        s_wred[0][wv] = mn;
        s_wred[1][wv] = mx;
      }
      __syncthreads();
      mn = 0xffffffffu;
      mx = 0u;
      for (int w = 0; w < NW; ++w) {
        mn = min(mn, s_wred[0][w]);
        mx = max(mx, s_wred[1][w]);
      }
    }
    if (threadIdx.x == 0) bc[4] = mn;
    __syncthreads();
    // d_max: rank T - 1 of the images, radix-selected over v - mn from the
    // span's top bit down, SEL_BITS bits a pass (at most three passes)
    const uint32_t span = mx - mn;
    int sh = span ? 32 - __clz(span) : 0;  // bits of v - mn still to resolve
    uint32_t pref = 0;                     // the resolved high bits of v - mn
    int64_t rr = T - 1;
    int ng = -1;                           // keys gathered into gkeys (-1: none)
    for (bool first = true; sh > 0; first = false) {
      const int w = sh < SEL_BITS ? sh : SEL_BITS;
      const int nsh = sh - w;
      const uint32_t dmask = (1u << w) - 1u;
      for (int i = threadIdx.x; i < (1 << w); i += NT) hist[i] = 0;
      __syncthreads();
      // mn read again after the barrier: v - mn is then formed in the pass
      // rather than kept for every register slot across the passes
      const uint32_t mnp = bc[4];
      if (ng >= 0) {
        for (int i = threadIdx.x; i < ng; i += NT) {
          const uint32_t d = gkeys[i] - mnp;
          if ((d >> sh) == pref) atomicAdd(&hist[(d >> nsh) & dmask], 1u);
        }
      } else {
        each([&](int64_t, bool valid, uint32_t v) {
          const uint32_t d = v - mnp;
          if (valid && (first || (d >> sh) == pref)) atomicAdd(&hist[(d >> nsh) & dmask], 1u);
        });
      }
      __syncthreads();
      {
        // the bin holding rank rr: 4 bins per thread, a block-wide scan
        uint32_t h[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int e = 4 * threadIdx.x + j;
          h[j] = e < (1 << w) ? hist[e] : 0u;
          sum += h[j];
        }
        const uint32_t incl = wave_incl_scan(sum);
        if (lane == 63) s_wred[0][wv] = incl;
        __syncthreads();
        if (threadIdx.x < 64) {
          const uint32_t t = threadIdx.x < NW ? s_wred[0][threadIdx.x] : 0u;
          const uint32_t ti = wave_incl_scan(t);
          if (threadIdx.x < NW) s_wred[1][threadIdx.x] = ti - t;
        }
        __syncthreads();
        const int64_t excl = (int64_t)s_wred[1][wv] + incl - sum;
        if (excl <= rr && rr < excl + (int64_t)sum) {
          int64_t rem = rr - excl;
          int j = 0;
          for (; j < 3; ++j) {
            if (rem < (int64_t)h[j]) break;
            rem -= h[j];
          }
          bc[0] = 4 * threadIdx.x + j;
          bc[1] = h[j];
          *reinterpret_cast<int64_t*>(bc + 2) = rem;
        }
      }
      __syncthreads();
      pref = (pref << w) | bc[0];
      rr = *reinterpret_cast<const int64_t*>(bc + 2);
      sh = nsh;
      const uint32_t nbin = bc[1];
      __syncthreads();
      if (R == 0 && ng < 0 && sh > 0 && nbin <= (uint32_t)GCAP) {
        // gather the picked bin's keys (its prefix pref) for the next passes
        if (threadIdx.x == 0) bc[1] = 0;
        __syncthreads();
        each([&](int64_t, bool valid, uint32_t v) {
          const bool in_bin = valid && ((v - mnp) >> sh) == pref;
          const uint32_t slot = wave_slot(in_bin, &bc[1]);
          if (in_bin) gkeys[slot] = v;
        });
        __syncthreads();
        ng = (int)nbin;
      }
    }
    dmax_b = mn + pref;
    for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
    __syncthreads();
    const float dmin = bits_key(mn);
    const float dmax = bits_key(dmax_b);
    float delta = (dmax - dmin) / 256.0f;
    if (!(delta > 0.0f)) delta = 1.0f;
    const float rdelta = __builtin_amdgcn_rcpf(delta);
    if (in_regs) {
      each([&](int64_t, bool valid, uint32_t v) {
        wave_hist_add(hist, (uint32_t)cell_fast(bits_key(v), dmin, delta, rdelta), valid && v < dmax_b);
      });
    } else {
      // (the same rule as the prune flag set below)
      const bool prune_f = Ts >= kc && dmax > dmin && !a.keep_all;
      uint32_t n_rej = 0;
      each([&](int64_t i, bool valid, uint32_t v) {
        wave_hist_add(hist, (uint32_t)cell_fast(bits_key(v), dmin, delta, rdelta), valid && v < dmax_b);
        const bool keep = valid && (!prune_f || v <= dmax_b);
        const uint32_t slot = wave_slot(keep, &bc[6]);
        if (keep) {
          skey[slot] = bits_key(v);
          spos[slot] = (uint32_t)pos_at(i, rk);
        } else if (valid) {
          ++n_rej;
        }
      });
      for (int off = 32; off >= 1; off >>= 1) n_rej += __shfl_xor(n_rej, off);
      if (lane == 0 && n_rej) atomicAdd(&bc[7], n_rej);
      filtered = true;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      // cell counts of the sample's T smallest keys: the keys below d_max as
      // counted, plus (T - their number) copies of d_max in d_max's cell;
      // map[e] = min(m - 1, floor(m * C_<e / T)), one wave, 4 cells per lane
      uint32_t h[4], sum = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        h[j] = hist[4 * lane + j];
        sum += h[j];
      }
      const uint32_t incl = wave_incl_scan(sum);
      const int64_t below_dmax = __shfl(incl, 63);
      const int cmax = cell_of(dmax, dmin, delta);
      int64_t below = incl - sum;
      // early re-rank (Algorithm 4): jp = ceil(K_c * (sample keys) / S); the
      // sample's jp-th smallest key lies in the first cell whose running
      // count of the T smallest reaches jp (jp <= T)
      const int64_t jp = a.early && S > 0 ? (kc * Ts + S - 1) / S : 0;
      uint32_t n_before = 0;  // cells whose running count stays below jp
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int e = 4 * lane + j;
        const int64_t be = below + (e > cmax ? T - below_dmax : 0);
        const int64_t b = ((int64_t)m * be) / T;
        cmap[e] = (uint8_t)(b < m - 1 ? b : m - 1);
        below += h[j];
        n_before += (below + (e + 1 > cmax ? T - below_dmax : 0)) < jp ? 1u : 0u;
      }
      for (int off = 32; off >= 1; off >>= 1) n_before += __shfl_xor(n_before, off);
      if (lane == 0) s_cpred = jp > 0 ? (int32_t)n_before : -1;
      // tighter filter for the lists after the sample: the first cell by
      // which the running count of the sample's keys reaches jf, if it lies
      // below d_max's cell (its keys are then all below d_max and counted)
      const bool tight = Ts >= kc && dmax > dmin && !a.keep_all && !a.early && a.filt_fraction > 0.0f &&
                         a.filt_fraction < 1.0f;
      const int64_t jf = tight ? (int64_t)ceilf(a.filt_fraction * (float)kc) : 0;
      int cf = 256;
      uint32_t ncf = 0;
      {
        int64_t run = incl - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          run += h[j];
          const int e = 4 * lane + j;
          if (cf == 256 && jf > 0 && run >= jf) {
            cf = e;
            ncf = (uint32_t)run;
          }
        }
      }
      const uint64_t got = __ballot(cf < 256);
      const int first = got ? __ffsll((unsigned long long)got) - 1 : 0;
      const int cf0 = __shfl(cf, first);
      const uint32_t ncf0 = __shfl(ncf, first);
      if (lane == 0) {
        s_cfilt = got && cf0 < cmax ? cf0 : -1;
        s_nfilt = ncf0;
      }
      if (lane == 0) {
        fbc[0] = dmin;
        fbc[1] = delta;
        // reject above d_max only when the sample alone holds K_c keys and the
        // cells are proper (then every key above d_max is in cell 255)
        bc[5] = (Ts >= kc && dmax > dmin && !a.keep_all) ? 1u : 0u;
      }
    }
  } else if (threadIdx.x == 0) {
    for (int e = 0; e < 256; ++e) cmap[e] = 0;
    fbc[0] = 0.0f;
    fbc[1] = 1.0f;
    bc[5] = 0u;
    s_cpred = -1;
  }
  if (T <= 0 && threadIdx.x == 0) s_cfilt = -1;
  __syncthreads();
  const uint32_t prune = bc[5];
  for (int e = threadIdx.x; e < 256; e += NT) book->map[e] = cmap[e];
  if (threadIdx.x == 0) {
    book->dmin = fbc[0];
    book->delta = fbc[1];
    // the scan's bound: the largest image whose cell is at most s_cfilt
    // (binary search over the images of -inf .. +inf, on which the cell is
    // monotone), else d_max
    uint32_t fb = dmax_b, nf = 0u;
    if (prune && s_cfilt >= 0) {
      uint32_t lo = key_bits(-INFINITY), hi = key_bits(INFINITY);
      while (hi - lo > 1u) {
        const uint32_t mid = lo + (hi - lo) / 2u;
        if (cell_of(bits_key(mid), fbc[0], fbc[1]) > s_cfilt) hi = mid; else lo = mid;
      }
      if (lo < dmax_b) {
        fb = lo;
        nf = s_nfilt;
      }
    }
    book->dmax_bits = fb;
    book->dmax_full = dmax_b;
    book->filt_count = nf;
    book->prune = prune;
    // early re-rank: tau_pred = the bucket of that cell; a key is re-ranked
    // early when its bucket is below tau_pred, i.e. its cell is below the
    // first cell mapped to tau_pred or above, i.e. its image is below the
    // smallest image of a key in that cell (binary search over the images
    // of -inf .. +inf, on which the cell is monotone)
    int32_t tp = 0;
    uint32_t ebits = 0u;
    if (s_cpred >= 0) {
      tp = cmap[s_cpred];
      if (tp > 0) {
        int ep = 0;
        while (ep < 255 && (int)cmap[ep] < tp) ++ep;
        uint32_t lo = key_bits(-INFINITY), hi = key_bits(INFINITY);
        while (hi - lo > 1u) {
          const uint32_t mid = lo + (hi - lo) / 2u;
          if (cell_of(bits_key(mid), fbc[0], fbc[1]) >= ep) hi = mid; else lo = mid;
        }
        ebits = hi;
      }
    }
    book->tau_pred = tp;
    book->early_bits = ebits;
    if (a.t_tau_pred) a.t_tau_pred[qi] = tp;
  }
  // the sample's keys through the relaxed-threshold filter (unless done)
  const uint64_t lt = (1ull << lane) - 1ull;
  if (filtered) {
  } else if (in_regs) {
    // slots from a count of each wave's kept keys (registers are read twice)
    uint32_t nkeep = 0, nrej = 0;
    each([&](int64_t, bool valid, uint32_t v) {
      const bool keep = valid && (!prune || v <= dmax_b);
      nkeep += (uint32_t)__popcll(__ballot(keep));
      nrej += (uint32_t)__popcll(__ballot(valid && !keep));
    });
    if (lane == 0) {
      s_wred[0][wv] = nkeep;
      s_wred[1][wv] = nrej;
    }
    __syncthreads();
    uint32_t base = 0, tot = 0, rej = 0;
    for (int x = 0; x < NW; ++x) {
      if (x < wv) base += s_wred[0][x];
      tot += s_wred[0][x];
      rej += s_wred[1][x];
    }
    each([&](int64_t i, bool valid, uint32_t v) {
      const bool keep = valid && (!prune || v <= dmax_b);
      const uint64_t mk = __ballot(keep);
      if (keep) {
        const uint32_t slot = base + (uint32_t)__popcll(mk & lt);
        skey[slot] = bits_key(v);
        spos[slot] = (uint32_t)pos_at(i, rk);
      }
      base += (uint32_t)__popcll(mk);
    });
    if (threadIdx.x == 0) {
      bc[6] = tot;
      bc[7] = rej;
    }
  } else {
    uint32_t n_rej = 0;
    each([&](int64_t i, bool valid, uint32_t v) {
      const bool keep = valid && (!prune || v <= dmax_b);
      const uint32_t slot = wave_slot(keep, &bc[6]);
      if (keep) {
        skey[slot] = bits_key(v);
        spos[slot] = (uint32_t)pos_at(i, rk);
      } else if (valid) {
        ++n_rej;
      }
    });
    for (int off = 32; off >= 1; off >>= 1) n_rej += __shfl_xor(n_rej, off);
    if (lane == 0 && n_rej) atomicAdd(&bc[7], n_rej);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.n_rejected[qi] = bc[7];
    a.pair_nsurv[po] = bc[6];  // the sample's survivors form rank 0's run
  }
  for (int r = 1 + threadIdx.x; r < nsr; r += NT) a.pair_nsurv[po + r] = 0;
}

__global__ __launch_bounds__(1024, 8) void collect_bucket_kernel(CollectArgs a) {
  constexpr int NT = 1024;
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* bbuf = reinterpret_cast<uint64_t*>(smem);  // [bcap], bcap a power of two
  __shared__ uint32_t s_pref[COLLECT_RANKCAP + 1];
  __shared__ uint32_t s_rbeg[COLLECT_RANKCAP];
  __shared__ uint32_t s_nsurv[COLLECT_RANKCAP];
  __shared__ uint16_t s_crank[COLLECT_CHUNKCAP];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t counts[BBC_MAX_BUCKETS];
  __shared__ uint8_t cmap[256];
  __shared__ __align__(8) uint32_t bc[8];
  __shared__ int64_t s_rem;

  const int64_t qi = a.qorder ? (int64_t)a.qorder[blockIdx.x] : (int64_t)blockIdx.x;
  const int64_t S = a.n_scanned[qi];
  int64_t kc = a.kc_target[qi];
  if (kc > S) kc = S;
  const int m = a.m;
  const QueryBook* book = a.books + qi;
  if (kc <= 0) {
    if (threadIdx.x == 0) {
      a.n_cand[qi] = 0;
      if (a.t_tau) { a.t_tau[qi] = -1; a.t_s[qi] = 0; a.t_dmin[qi] = 0.f; a.t_delta[qi] = 1.f; a.t_nboundary[qi] = 0; }
      if (a.surv_total) a.surv_total[qi] = 0;
    }
    if (a.t_map) for (int e = threadIdx.x; e < 256; e += NT) a.t_map[qi * 256 + e] = 0;
    if (a.t_counts) for (int b = threadIdx.x; b < m; b += NT) a.t_counts[qi * m + b] = 0;
    return;
  }
  for (int e = threadIdx.x; e < 256; e += NT) cmap[e] = book->map[e];
  for (int b = threadIdx.x; b < m; b += NT) counts[b] = 0;
  if (threadIdx.x == 0) bc[4] = 0;
  __syncthreads();
  const float dmin = book->dmin, delta = book->delta;
  const float rdelta = __builtin_amdgcn_rcpf(delta);
  const int np = a.nprobe[qi];
  const int64_t po = a.probe_off[qi];
  const int64_t* rank_off = a.rank_off + po;
  const uint32_t* nsurv = a.pair_nsurv + po;
  const float* skey = a.surv_key + a.surv_off[qi];
  const uint32_t* spos = a.surv_pos + a.surv_off[qi];
  uint8_t* sbkt = a.surv_bucket + a.surv_off[qi];
  // Survivors sit in per-rank runs [rank_off[r], rank_off[r] + nsurv[r]).
  // The runs are cut into 64-element chunks (an LDS prefix of chunk counts,
  // and a chunk -> run table when it fits); a wave takes COLLECT_UNROLL
  // consecutive chunks at a time and issues all their loads before using
  // them.  Probes wider than the LDS tables walk the runs one by one.
  const bool flat = np <= COLLECT_RANKCAP;
  if (flat && threadIdx.x < 64) {
    const int lane = threadIdx.x;
    uint32_t carry = 0;
    for (int base = 0; base < np; base += 64) {
      const int r = base + lane;
      const uint32_t ns = r < np ? nsurv[r] : 0u;
      const uint32_t v = (ns + 63u) / 64u;
      uint32_t incl = v;
      for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      if (r < np) {
        s_pref[r] = carry + incl - v;
        s_rbeg[r] = (uint32_t)rank_off[r];
        s_nsurv[r] = ns;
      }
      carry += __shfl(incl, 63);
    }
    if (lane == 0) s_pref[np] = carry;
  }
  __syncthreads();
  const uint32_t nchunks = flat ? s_pref[np] : 0u;
  const bool table = flat && nchunks <= (uint32_t)COLLECT_CHUNKCAP;
  if (table)
    for (int r = threadIdx.x; r < np; r += NT)
      for (uint32_t ch = s_pref[r]; ch < s_pref[r + 1]; ++ch) s_crank[ch] = (uint16_t)r;
  __syncthreads();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;  // wv: wave-uniform
  constexpr int U = COLLECT_UNROLL;
  constexpr int NW = NT / 64;
  // Batches of UB chunks per wave (UB = the Unroll argument): batch(act,
  // idx) gets this lane's slot of each (with its active flag); the number of
  // calls is wave-uniform (batch() may take wave-wide collectives).
  auto for_each_batch = [&](auto uc, auto batch) {
    constexpr int UB = decltype(uc)::value;
    if (flat) {
      for (uint32_t c0 = (uint32_t)wv * UB; c0 < nchunks; c0 += NW * UB) {
        bool act[UB];
        int64_t idx[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const uint32_t ch = c0 + u;
          act[u] = false;
          idx[u] = 0;
          if (ch < nchunks) {
            int r;
            if (table) {
              r = s_crank[ch];
            } else {
              int lo = 0, hi = np - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pref[mid] <= ch) lo = mid; else hi = mid - 1;
              }
              r = lo;
            }
            const uint32_t e = (ch - s_pref[r]) * 64u + lane;
            act[u] = e < s_nsurv[r];
            idx[u] = (int64_t)s_rbeg[r] + e;
          }
        }
        batch(act, idx);
      }
    } else {
      for (int r = 0; r < np; ++r) {
        const int64_t rb = rank_off[r];
        const int64_t rn = nsurv[r];
        for (int64_t base = 0; base < rn; base += NT) {
          bool act[UB];
          int64_t idx[UB];
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            act[u] = u == 0 && base + threadIdx.x < rn;
            idx[u] = rb + base + threadIdx.x;
          }
          batch(act, idx);
        }
      }
    }
  };
  // For every survivor: v = load(active, slot), then use(active, slot, v).
  auto for_each_wave = [&](auto uc, auto load, auto use) {
    constexpr int UB = decltype(uc)::value;
    using V = decltype(load(false, (int64_t)0));
    for_each_batch(uc, [&](const bool* act, const int64_t* idx) {
      V v[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) v[u] = load(act[u], idx[u]);
#pragma unroll
      for (int u = 0; u < UB; ++u) use(act[u], idx[u], v[u]);
    });
  };
  auto for_each = [&](auto fn) {
    for_each_wave(Unroll<U>{}, [&](bool act, int64_t i) { return 0; },
                  [&](bool act, int64_t i, int) { if (act) fn(i); });
  };

  // ---- histogram (rejected keys all sit in the last cell); each survivor's
  // bucket is kept for the collection pass --------------------------------
  {
    uint32_t n_last = 0, n_all = 0;
    for_each_wave(Unroll<2 * U>{}, [&](bool act, int64_t i) { return act ? skey[i] : 0.0f; },
                  [&](bool act, int64_t i, float key) {
                    const int c = act ? cell_fast(key, dmin, delta, rdelta) : 255;
                    const uint32_t b = cmap[c];
                    if (act) sbkt[i] = (uint8_t)b;
                    n_all += act;
                    n_last += act && c == 255;
                    wave_hist_add(counts, b, act && c != 255);
                  });
    for (int off = 32; off >= 1; off >>= 1) {
      n_last += __shfl_xor(n_last, off);
      n_all += __shfl_xor(n_all, off);
    }
    if (lane == 0 && n_last) atomicAdd(&counts[cmap[255]], n_last);
    if (lane == 0 && n_all) atomicAdd(&bc[4], n_all);
    if (threadIdx.x == 0 && a.n_rejected[qi]) atomicAdd(&counts[cmap[255]], (uint32_t)a.n_rejected[qi]);
  }
  __syncthreads();

  // ---- Update: threshold bucket and s ---------------------------------------
  // tau: the first bucket whose running count reaches kc, i.e. the bucket
  // holding rank kc - 1; s_rem = kc - 1 minus the count below tau
  if (threadIdx.x < 64) wave_find_rank(counts, m, kc - 1, &bc[0], &s_rem);
  if (threadIdx.x == 64) {
    bc[2] = 0;                  // candidate slot counter
    bc[3] = 0;                  // boundary slot counter
    if (a.surv_total) a.surv_total[qi] = bc[4];
  }
  __syncthreads();
  const int tau = (int)bc[0];
  const int64_t nbelow = kc - 1 - s_rem;  // objects strictly below tau
  const int64_t s = kc - nbelow;
  const int bcap = a.bcap;
  uint32_t* cand = a.cand_pos + a.cand_off[qi];
  // the threshold bucket's members also go to global scratch (room for
  // K_c of them), where a larger bucket is selected without another pass
  // over the survivors
  uint64_t* bnd = a.bnd_scratch + a.cand_off[qi];
  const int64_t bnd_cap = a.cand_off[qi + 1] - a.cand_off[qi];

  // ---- Collect -----------------------------------------------------------------
  // Each batch loads the buckets and the list positions of its survivors
  // together (one round trip).  Candidates below tau are written at once;
  // the threshold bucket's members are recorded by survivor slot, and their
  // keys and ids are looked up afterwards, all at once.  One atomic per
  // counter for a lane's whole batch.
  for_each_batch(Unroll<U>{}, [&](const bool* act, const int64_t* idx) {
    int b[U];
    uint32_t pv[U];
    uint64_t mc[U], mb[U];
    uint32_t nc = 0, nbd = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      b[u] = act[u] ? (int)sbkt[idx[u]] : m;
      pv[u] = act[u] ? spos[idx[u]] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      mc[u] = __ballot(b[u] < tau);
      mb[u] = __ballot(b[u] == tau);
      nc += (uint32_t)__popcll(mc[u]);
      nbd += (uint32_t)__popcll(mb[u]);
    }
    uint32_t basec = 0, baseb = 0;
    if (lane == 0) {
      if (nc) basec = atomicAdd(&bc[2], nc);
      if (nbd) baseb = atomicAdd(&bc[3], nbd);
    }
    basec = __shfl(basec, 0);
    baseb = __shfl(baseb, 0);
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (b[u] < tau)  // a survivor re-ranked early is handed on by its slot
        cand[basec + (uint32_t)__popcll(mc[u] & lt)] =
            (pv[u] & EARLY_FLAG) ? (EARLY_FLAG | (uint32_t)idx[u]) : pv[u];
      if (b[u] == tau) {
        const uint32_t bs = baseb + (uint32_t)__popcll(mb[u] & lt);
        const uint64_t pk = (uint64_t)idx[u];  // survivor slot, resolved below
        if ((int)bs < bcap) bbuf[bs] = pk;
        if ((int64_t)bs < bnd_cap) bnd[bs] = pk;
      }
      basec += (uint32_t)__popcll(mc[u]);
      baseb += (uint32_t)__popcll(mb[u]);
    }
  });
  __syncthreads();
  const int64_t nb = bc[3];
  if (nb <= bcap) {
    // members: survivor slot -> (key, id)
    for (int i = threadIdx.x; i < (int)nb; i += NT) {
      const int64_t x = (int64_t)bbuf[i];
      bbuf[i] = pack_key_id(skey[x], (uint32_t)a.list_ids[spos[x] & EARLY_MASK]);
    }
    const int P = next_pow2((int)nb);
    for (int i = (int)nb + threadIdx.x; i < P; i += NT) bbuf[i] = ~0ull;
    __syncthreads();
    lds_bitonic_sort<NT>(bbuf, P);
    for (int64_t r = threadIdx.x; r < s; r += NT)
      cand[nbelow + r] = (uint32_t)a.pos_of_id[packed_id(bbuf[r])];
  } else if (nb <= bnd_cap) {
    // the s smallest (key, id) of the members gathered in global scratch:
    // slots -> (key, id), radix select of the s-th, one pass over them
    for (int64_t i = threadIdx.x; i < nb; i += NT) {
      const int64_t x = (int64_t)bnd[i];
      bnd[i] = pack_key_id(skey[x], (uint32_t)a.list_ids[spos[x] & EARLY_MASK]);
    }
    __syncthreads();
    const uint64_t thr =
        block_radix_select64<NT>([&](int64_t i, uint64_t& v) { v = bnd[i]; return true; }, nb, s - 1, hist, bc);
    if (threadIdx.x == 0) bc[6] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < nb; i += NT) {
      const uint64_t v = bnd[i];
      if (v <= thr) cand[nbelow + atomicAdd(&bc[6], 1u)] = (uint32_t)a.pos_of_id[packed_id(v)];
    }
  } else {
    // exact selection of the s smallest (key, id) of the threshold bucket:
    // 64-bit radix select over its members, then one pass to collect them
    auto get = [&](int64_t i, uint64_t& v) -> bool {
      if ((int)sbkt[i] != tau) return false;
      v = pack_key_id(skey[i], (uint32_t)a.list_ids[spos[i] & EARLY_MASK]);
      return true;
    };
    uint64_t prefix = 0, mask = 0;
    int64_t rr = s - 1;
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
      __syncthreads();
      for_each([&](int64_t i) {
        uint64_t v;
        if (get(i, v) && (v & mask) == prefix) atomicAdd(&hist[(v >> shift) & 255u], 1u);
      });
      __syncthreads();
      if (threadIdx.x == 0) {
        int64_t q = rr;
        uint32_t dg = 0;
        for (; dg < 255; ++dg) {
          if (q < (int64_t)hist[dg]) break;
          q -= hist[dg];
        }
        bc[5] = dg;
        bc[6] = (uint32_t)q;
      }
      __syncthreads();
      prefix |= (uint64_t)bc[5] << shift;
      mask |= 255ull << shift;
      rr = bc[6];
      __syncthreads();
    }
    if (threadIdx.x == 0) bc[3] = 0;
    __syncthreads();
    for_each([&](int64_t i) {
      uint64_t v;
      if (get(i, v) && v <= prefix)
        cand[nbelow + atomicAdd(&bc[3], 1u)] = (spos[i] & EARLY_FLAG) ? (EARLY_FLAG | (uint32_t)i) : spos[i];
    });
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

// Candidates that reuse an early exact key: (exact key, id) at their place.
// One block per query.
__global__ __launch_bounds__(256) void early_fill_kernel(EarlyFillArgs a) {
  const int64_t qi = blockIdx.x;
  const int64_t kc = a.n_cand[qi];
  const int64_t co = a.cand_off[qi], so = a.surv_off[qi];
  uint32_t nused = 0;
  for (int64_t i = threadIdx.x; i < kc; i += 256) {
    const uint32_t c = a.cand_pos[co + i];
    if (c & EARLY_FLAG) {
      const int64_t slot = so + (c & EARLY_MASK);
      const uint32_t pos = a.surv_pos[slot] & EARLY_MASK;
      a.cand_packed[co + i] = pack_key_id(a.surv_exact[slot], (uint32_t)a.list_ids[pos]);
      ++nused;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) nused += __shfl_xor(nused, off);
  if ((threadIdx.x & 63) == 0 && nused) atomicAdd(&a.n_used[qi], nused);
}

hipError_t launch_early_fill(const EarlyFillArgs& a, int64_t max_kc, hipStream_t s) {
  if (a.nq <= 0 || max_kc <= 0) return hipSuccess;
  hipLaunchKernelGGL(early_fill_kernel, dim3((unsigned)a.nq), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_codebook(const CollectArgs& a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  // the smallest register slot count that holds the largest sample (48
  // slots fill the 128 registers a lane of a 1024-thread block may hold)
  const dim3 g((unsigned)a.nq), b(1024);
  switch (codebook_form(a.max_sample)) {
    case 16: hipLaunchKernelGGL(codebook_kernel<16>, g, b, 0, s, a); break;
    case 32: hipLaunchKernelGGL(codebook_kernel<32>, g, b, 0, s, a); break;
    case 48: hipLaunchKernelGGL(codebook_kernel<48>, g, b, 0, s, a); break;
    default: hipLaunchKernelGGL(codebook_kernel<0>, g, b, 0, s, a); break;
  }
  return hipGetLastError();
}

int codebook_form(int64_t ms) {
  if (ms <= 16 * 1024) return 16;
  if (ms <= 32 * 1024) return 32;
  if (ms <= 48 * 1024) return 48;
  return 0;
}

hipError_t launch_collect_bucket(const CollectArgs& a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  size_t lds = sizeof(uint64_t) * (size_t)a.bcap;
  hipLaunchKernelGGL(collect_bucket_kernel, dim3((unsigned)a.nq), dim3(1024), lds, s, a);
  return hipGetLastError();
}

}  // namespace bbc

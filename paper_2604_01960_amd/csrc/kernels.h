// Launch descriptors for the query-path kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/bbc.h"

namespace bbc {

// Records the message of a failing call (bbc_last_error) and returns code.
int32_t set_error(int32_t code, const std::string& msg);

// Fixed host staging for a search's metadata block (pinned, or a static
// pageable buffer), and the event recorded after each upload out of it.
struct MetaStaging {
  char* host;
  size_t bytes;
  hipEvent_t done;
};

// A search with device I/O whose scratch is the caller's `ws` (the index
// arena is not touched, so calls on different streams with different
// workspaces may overlap on the device).  With ws == nullptr only *ws_bytes
// is set: the bytes the call needs.  work_out (device or pinned host, may be
// NULL) receives [2][nq] int64 on the search stream: codes scanned, then
// exact distances computed (K_c, or the objects the bounded walk visited).
// meta (may be NULL): stage the metadata block there instead of in the
// index's growable pinned buffer (the call then allocates nothing).
int32_t search_in_workspace(bbc_index* ix, const float* queries, int64_t nq, const int32_t* k,
                            const int32_t* nprobe, const bbc_search_params* p, const int64_t* out_off,
                            int64_t* out_ids, float* out_dists, int32_t* out_counts, char* ws, size_t* ws_bytes,
                            int64_t* work_out = nullptr, const MetaStaging* meta = nullptr);

// Device an index lives on.
int index_device(const bbc_index* ix);

int32_t build_index_pq(int32_t device, const float* base, int64_t n, int32_t d, const bbc_build_params* p,
                       bbc_index** out);
int32_t build_index_rabitq(int32_t device, const void* base, int64_t n, int32_t d, const bbc_build_params* p,
                           bbc_index** out);

struct ProbeArgs {
  const float* q; int64_t nq; int d;
  const float* cent; const uint16_t* cent_bf16; int dpad;
  const float* cent_norm2; const float* cent_norm; int nlist; int metric;
  const int32_t* nprobe; const int64_t* probe_off; const int64_t* list_off;
  float* dprime; int32_t* probe_lists; float* probe_keys; int64_t* rank_off; int64_t* n_scanned;
  int32_t* n_recheck;
  // codebook sample size: the nearest lists, at least `nsample`, extended
  // until they hold sample_factor * kc_target keys (all probed lists if they
  // never do)
  const int64_t* kc_target; int nsample; int sample_factor; int32_t* nsample_q;
  int num_cu = 256;  // compute units of the device (block shape of the select)
};
hipError_t launch_probe(const ProbeArgs& a, hipStream_t s);
size_t probe_select_lds(int nlist);

// Per-query collector codebook (written by the codebook kernel).
struct QueryBook {
  float dmin;
  float delta;
  uint32_t dmax_bits;  // key image of the scan's filter bound (d_max, or the tighter d_f)
  uint32_t prune;      // 1: keys above the filter bound are rejected at the scan
  // tighter filter: d_max's image, and the number of sample keys at or below
  // the bound (filt_count = 0: the bound is d_max itself)
  uint32_t dmax_full;
  uint32_t filt_count;
  uint8_t map[256];    // equal-width cell -> bucket
  // early re-rank (Algorithm 4): the predicted threshold bucket and the
  // smallest key image whose bucket reaches it (keys with a smaller image are
  // re-ranked during the scan of the lists after the sample; 0: none)
  int32_t tau_pred;
  uint32_t early_bits;
};

// Early re-rank marks: a survivor re-ranked during the scan carries this bit
// in its list position (positions are below 2^31); a candidate that reuses
// such an exact key holds this bit and its survivor slot instead of its list
// position.
constexpr uint32_t EARLY_FLAG = 0x80000000u;
constexpr uint32_t EARLY_MASK = 0x7fffffffu;

struct PqScanArgs {
  const float* q; int64_t nq; int d; const float* cent;
  int M; int bits; const float* codebook; const uint8_t* codes; int code_stride;
  const int64_t* list_off; const int64_t* probe_off; const int32_t* probe_lists;
  const int64_t* rank_off; const int64_t* key_off;
  int nlist; int64_t npairs; int num_cu; int nxcd;
  uint32_t* pair_cnt;       // [2*nlist] scratch
  uint32_t* sorted_pairs;   // [npairs] scratch: sample pairs then the rest, each grouped by list
  uint32_t* sorted_q;       // [pair slots] the query of each sorted pair (NO_PAIR slots: unused)
  // pairs scanned by this launch: sorted_pairs[0, split) for mode 0 and
  // [split, total) for mode 1, with pair_split = {split, total} (bins padded
  // to SCAN_GROUP entries with NO_PAIR)
  uint32_t* pair_split;
  uint32_t* bs_table;       // pair sort's per-block counts (bs_table_words(nq, 2 * nlist)); NULL: global atomics
  int mode;                 // 0: sample lists -> sample_keys by slot; 1: the rest -> filter + survivors
  const int32_t* nsample_q; // per-query sample size (probe ranks below it are the sample)
  float* sample_keys; const int64_t* sample_off;
  const QueryBook* books;
  // survivors: pair p of query q writes its kept keys, compacted, from slot
  // surv_off[q] + rank_off[p] on and their number to pair_nsurv[p]
  float* surv_key; uint32_t* surv_pos; const int64_t* surv_off; uint32_t* pair_nsurv; uint32_t* n_rejected;
  float* trace_keys;        // optional: every key by slot (key_off regions)
  int scan_variant;         // grouped-scan block geometry: 0 (512 threads, 2 codes each), 1 (512, 1), 2 (1024, 1)
  int lut_u8;               // one-byte tables with integer sums (grouped shapes only)
  // early re-rank (mode 1, grouped shapes, float32 rows): survivors whose key
  // image is below their query's book->early_bits get their exact key now
  int early; int metric; const float* vectors;   // rows in list-slot order
  float* surv_exact;        // exact key by survivor slot (early survivors only)
  uint32_t* n_early;        // [nq] survivors re-ranked during the scan (atomic adds)
  // mode 0: the smallest and largest key image of each query's sample
  // (atomic min / max; launch_pq_scan sets them to +inf / 0 first); NULL: not kept
  uint32_t* smin; uint32_t* smax;
  // mode 1, generic kernel: only the pairs of queries with rescan_q[q] != 0
  const uint32_t* rescan_q;
};
// Shapes the grouped scan (and so the one-byte tables) supports.
bool pq_scan_grouped_shape(int bits, int M, int d);
// p[0, n) = 0 (a kernel, so that graph capture records no memset)
hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
constexpr int SCAN_GROUP = 4;  // queries of one list scanned together (float tables)
constexpr int SCAN_GROUP_MAX = 8;
// queries per scan group: one-byte tables of 4-bit codes take 8, the rest 4
__host__ __device__ constexpr int scan_group_of(bool u8, int bits) { return u8 && bits == 4 ? 8 : 4; }
int64_t pair_slots(int64_t npairs, int nlist);  // sorted_pairs capacity
// Counting sort of the (query, rank) pairs by (rank >= nsample, list).
hipError_t launch_pair_sort(const PqScanArgs& a, hipStream_t s);
hipError_t launch_pq_scan(const PqScanArgs& a, hipStream_t s);
// After the filter scan at the tighter bound d_f: a query whose sample keys
// and later survivors at or below d_f number fewer than K_c has its bound
// reset to d_max, its later lists' rejected count taken back and its flag
// set (flags: [nq]); then those queries' later lists are scanned again at
// d_max (the generic one-pair-per-block kernel, other pairs return at once).
hipError_t launch_filter_rescan(PqScanArgs a, const int64_t* kc_target, uint32_t* flags, hipStream_t s);
// words of the pair sorts' per-block count table for nq queries over nbins
// bins (0: too many bins for it, the sorts then use global atomics)
int64_t pair_sort_table_words(int64_t nq, int nbins);

struct CollectArgs {
  int64_t nq; const float* keys; const int64_t* key_off; const int64_t* n_scanned;
  const int32_t* nprobe; const int64_t* probe_off; const int32_t* probe_lists; const int64_t* rank_off;
  const int64_t* list_off; const int32_t* list_ids; const int32_t* pos_of_id;
  const int64_t* kc_target; const int64_t* cand_off; int m; const int32_t* nsample_q; int bcap;
  int64_t max_sample;       // upper bound of the codebook sample's keys over the queries
  uint32_t* cand_pos; int64_t* n_cand;
  const float* sample_keys; const int64_t* sample_off; QueryBook* books;
  float* surv_key; uint32_t* surv_pos; const int64_t* surv_off; uint32_t* pair_nsurv; uint32_t* n_rejected;
  uint32_t* surv_total;     // [nq] survivors per query (written by the collector)
  uint8_t* surv_bucket;     // bucket of each survivor (collector scratch, same slots as surv_key)
  uint64_t* bnd_scratch;    // [sum K_c] the threshold bucket's (key, id), by cand_off (free until the re-rank)
  // trace outputs (all null when tracing is off)
  float* t_dmin; float* t_delta; uint8_t* t_map; int32_t* t_tau; int64_t* t_s; int32_t* t_counts;
  int64_t* t_nboundary;
  int64_t* t_nsample_keys;  // keys in the codebook sample (codebook kernel)
  int early;                // codebook: also the predicted threshold of the early re-rank
  int keep_all;             // codebook: no relaxed-threshold filter (every key survives)
  // codebook: the lists after the sample are filtered at d_f, the upper edge
  // of the first cell by which the sample's running count reaches
  // filt_fraction * K_c (0 or >= 1: at d_max)
  float filt_fraction;
  // codebook: the sample's smallest and largest key images from the sample
  // scan (NULL: the codebook finds them itself)
  const uint32_t* smin; const uint32_t* smax;
  // codebook and collector: query of each block (NULL: the block index),
  // largest candidate sets first so that a launch does not end on a few
  // long blocks
  const int32_t* qorder;
  int32_t* t_tau_pred;      // trace: the predicted threshold bucket (codebook kernel)
};
hipError_t launch_codebook(const CollectArgs& a, hipStream_t s);
// register slots per thread the codebook kernel takes for samples of up to
// max_sample keys (16, 32, 48; 0 = samples read from memory in each pass)
int codebook_form(int64_t max_sample);
hipError_t launch_collect_bucket(const CollectArgs& a, hipStream_t s);

// Early re-rank: each candidate that reuses an exact key computed during the
// scan (cand_pos holds EARLY_FLAG | survivor slot) gets its (exact key, id)
// at its own place in cand_packed; n_used[q] counts them.
struct EarlyFillArgs {
  int64_t nq; const int64_t* n_cand; const int64_t* cand_off; const uint32_t* cand_pos;
  const int64_t* surv_off; const uint32_t* surv_pos; const float* surv_exact; const int32_t* list_ids;
  uint64_t* cand_packed; uint32_t* n_used;
};
hipError_t launch_early_fill(const EarlyFillArgs& a, int64_t max_kc, hipStream_t s);

struct RerankArgs {
  const float* q; int64_t nq; int d; int metric; const void* vectors; int fp16;
  const int32_t* list_ids; const uint32_t* cand_pos; const int64_t* cand_off; const int64_t* n_cand;
  uint64_t* cand_packed;
  const int32_t* qorder;    // optional: block row y re-ranks query qorder[y] (else query y)
};
hipError_t launch_rerank(const RerankArgs& a, int64_t max_kc, hipStream_t s);
constexpr int QUERY_ORDER_MAX_LISTS = 32768;

// Tile-major re-rank (rows of at most 256 four-element chunks).
constexpr int RT_G = 256;              // (query, list) pairs per block, rows of at most 32 chunks
constexpr int RT_GW = 16;              // the same for longer rows (one pair per wave)
constexpr int RT_TILE_BYTES = 65536;   // LDS rows per tile
struct TileRerankArgs {
  const float* q; int64_t nq; int d; int metric; const void* vectors; int fp16;
  const int32_t* list_ids; const int64_t* list_off; const int32_t* list_of_pos;
  const int32_t* nprobe; const int64_t* probe_off; const int32_t* probe_lists; int nlist;
  // candidates of query q: cand_pos[pos_off[q] + i], i < n_cand[q] (or
  // ncand_w[q * ncand_stride] when ncand_w is set)
  const uint32_t* cand_pos; const int64_t* pos_off; const int64_t* n_cand;
  const uint32_t* ncand_w; int ncand_stride;
  // out: (key, id) of candidate i at cand_packed[cand_off[q] + i] when
  // sorted_idx is set, else at the candidate's place in the sorted order
  const int64_t* cand_off; uint64_t* cand_packed;
  int64_t npairs; int max_np;
  int tshift;               // rows per tile = 1 << tshift
  int max_bins;             // most bins of a query (tiles of its probed lists)
  uint32_t* sorted_pos;     // [by pos_off] each query's candidates grouped by (rank, tile)
  uint32_t* sorted_idx;     // optional [by pos_off]: their candidate indices
  uint32_t* pair_tb;        // [npairs] first bin of each (query, rank) pair within its query
  const int64_t* bin_off;   // [nq + 1] each query's bins in bin_beg
  uint32_t* bin_beg;        // [bin_off[nq]] bin starts within the query's candidates, then the count
  uint32_t* lcnt;           // [nlist + 1] pair counts, then cursors; [nlist] = number of groups
  uint64_t* lpairs;         // [lpairs_cap] (query << 32 | rank) grouped by list, whole groups
  int64_t lpairs_cap;       // npairs + nlist * (group - 1)
  int group;                // pairs per block: tile_rerank_group(d)
  int presorted;            // sorted_pos, sorted_idx, pair_tb and bin_beg already filled
  // RaBitQ wide form in two rounds: round 1 computes only the candidates
  // placed below wround[4q + 1] (sorted_idx = their places); 0: every one
  int round; const uint32_t* wround;
  int pairs_ready;          // lcnt and lpairs already filled (launch_tile_pairs)
  uint32_t* bs_table;       // pair sort's per-block counts (bs_table_words(nq, nlist)); NULL: global atomics
  int no_run_list;          // tile re-rank: find each run's pair by binary search even when the runs fit the list
  const int32_t* qorder;    // candidate sort: query of each block (NULL: the block index)
};
// the (query, rank) pairs grouped by list into whole groups: lcnt, lpairs
hipError_t launch_tile_pairs(const TileRerankArgs& a, hipStream_t s);
int tile_rerank_group(int d);
// log2 of the rows per tile for the row shape, or -1 where the form does not apply
int tile_rerank_shift(int d, int fp16);
// dynamic LDS of the candidate sort
size_t tile_rerank_sort_lds(int max_bins, int max_np, int nlist);
hipError_t launch_tile_rerank(const TileRerankArgs& a, size_t sort_lds, hipStream_t s);
// order[0, nq): the queries sorted by their nearest probed list
hipError_t launch_query_order(const int32_t* probe_lists, const int64_t* probe_off, const int32_t* nprobe,
                              int64_t nq, int nlist, int32_t* order, hipStream_t s);

struct FinalArgs {
  int64_t nq; const int32_t* k; const int64_t* n_cand; const int64_t* cand_off; uint64_t* cand_packed;
  const int64_t* out_off; int64_t* out_ids; float* out_dists; int32_t* out_counts; int metric;
  int cap;                  // packed items in the dynamic LDS buffer (queries with min(k, K_c) <= cap use the binned path)
  int run;                  // largest power of two <= cap: LDS sort run of the global sort
  int64_t max_kc;           // largest K_c of the launch's queries (selects the register-resident variant)
  const int32_t* qmap;      // the launch's queries: block b takes query qmap[b] (nullptr: query b)
  uint64_t* scratch;        // k slots per query at out_off: the winners grouped by bin
};
// ---- comparator collectors (heap, sort) over every scanned key ----------------
struct CompareArgs {
  int64_t nq; const int64_t* n_scanned; const int64_t* kc_target; const int32_t* nprobe; const int64_t* probe_off;
  const int64_t* rank_off; const int32_t* probe_lists; const int64_t* list_off; const int32_t* list_ids;
  const int32_t* pos_of_id;
  const float* keys; const int64_t* key_off;   // every scanned key of query q at keys[key_off[q] + slot]
  const int64_t* cand_off; uint32_t* cand_pos; int64_t* n_cand;
  uint64_t* heap;                              // [sum K_c] heap storage (heap collector)
  int64_t max_kc;                              // largest K_c of the batch (LDS heap when it fits)
};
// collector: 1 heap, 2 sort, 3 heap in LDS
hipError_t launch_compare_collect(const CompareArgs& a, int collector, hipStream_t s);

// ---- RaBitQ -------------------------------------------------------------------
// y[r][i] = sum over e of P[e][i] * v[r][e], sequential in e (P: [D][D])
hipError_t launch_rotate(const float* v, int64_t n, int D, const float* P, float* y, hipStream_t s);

struct RabitqBuildArgs {
  const float* x;           // [n][D] base rows, original order, fp32
  const int64_t* list_ids;  // [n] original row of each list slot
  const int64_t* list_off; int nlist;
  const float* cent;        // [nlist][D]
  const float* P;           // [D][D]
  int D;
  uint32_t* codes; int code_words;  // [n][code_words], list order (code_words = D/32 rounded up to 4)
  float* factors;           // [n][4] (nr, f, g, popcount)
};
// codes and factors of slots [p0, p0 + n); resid and rot are [n][D] scratch
hipError_t launch_rabitq_encode(const RabitqBuildArgs& a, int64_t p0, int64_t n, float* resid, float* rot,
                                hipStream_t s);

struct RabitqScanArgs {
  int64_t npairs; int64_t nq; const int64_t* probe_off; const int32_t* probe_lists; const float* probe_keys;
  const int64_t* rank_off; const int64_t* key_off;
  const float* q; const float* qrot; const float* rot_cent;  // queries, P^T q [nq][D], P^T c [nlist][D]
  int D; int metric; float eps0;
  const int64_t* list_off; const uint32_t* codes; int code_words; const float* factors;
  float* lb; float* ub; float* key;  // [sum S] by slot at key_off[q]; key optional
  int max_np;               // largest nprobe of the batch (the 2-D grid's first dimension)
  int grid2d;               // set by the launcher
  int force_1d;             // one block per pair on a 1-D grid even where the 2-D grid fits
  // optional: the (query << 32 | rank) pairs grouped by list, *ngroups groups
  // of `group` entries (~0 pads), scanned so that each XCD takes a contiguous
  // run of them (a list's code rows then stay in that XCD's L2)
  const uint64_t* lpairs; const uint32_t* ngroups; int group; int64_t lpairs_cap;
};
hipError_t launch_rabitq_scan(const RabitqScanArgs& a, hipStream_t s);

constexpr int WALK_RANKS_LDS = 2048;  // probe ranks per query held in the walk kernels' LDS tables
struct RabitqWalkArgs {
  int64_t nq; const int64_t* n_scanned; const int32_t* k; const int32_t* nprobe; const int64_t* probe_off;
  const int64_t* rank_off; const int32_t* probe_lists; const int64_t* list_off; const int32_t* list_ids;
  const int32_t* pos_of_id;
  const float* lb; const float* ub; const int64_t* key_off;
  uint32_t* cbuf;            // [sum S] C grouped by lb bin: slots, or lb images in the wide form
  const int64_t* cand_off; uint64_t* cand_packed;  // [sum S] processed (exact key, id)
  int64_t* n_cand; int64_t* n_visited;
  uint64_t* zbuf;            // [2 * sum S] scratch (the k best so far, ping-pong)
  const float* q; const void* vectors; int fp16; int D; int metric;
  // wide form (small batches): the exact keys of all of C = {lb <= U} are
  // computed first by a grid over the device, then the walk reads them
  int wide;
  int64_t max_c;             // upper bound of |C| over the queries (largest S)
  int32_t* cpos;             // [sum S] list positions of C in cbuf order
  uint32_t* wbins;           // [nq][2048] bin ends
  uint32_t* wstate;          // [nq][4] U, lmin, shift, |C|
  int keys_ready;            // wide form: the exact keys of C are already in cand_packed
  // wide form with tile-major keys: C also in slot order (by probe rank, then
  // list position, hence by tile of 2^t_shift rows), as the tile re-rank reads
  // it (t_pos NULL: not wanted; cpos is then not written either)
  uint32_t* t_pos;           // [sum S] list positions of C in slot order
  uint32_t* t_idx;           // [sum S] their places in cbuf order
  uint32_t* t_bins;          // per query from t_bin_off: start of each (rank, tile) bin, then |C|
  uint32_t* t_rank_tb;       // [sum nprobe] first bin of each probe rank
  const int64_t* t_bin_off;  // [nq + 1]
  int t_shift;
  int qcap;                  // objects above the k-th exact key resolved in LDS (0 = the LDS capacity)
  int32_t* t_qpath;          // optional [nq]: how the exact stop point was found (0 no search, 1 LDS,
                             // 2 global memory, 3 item-by-item walk)
  // wide form in two rounds (round 1, then 2; 0 = one pass over all of C):
  // round 1 computes the exact keys of C's first bins only (places below
  // wround[4q + 1], bins below wround[4q]: the lb bins up to an estimate of
  // the walk's stop point) and walks them; a query whose stop point lies
  // beyond them is marked (wround[4q + 2] = 1) and round 2 computes the rest
  // of its keys and walks again
  int round;
  uint32_t* wround;          // [nq][4] first-round bins, first-round places, second round needed, 0
  float round1_alpha;        // prep: the first round's bins reach lb bin(k-th lb) + alpha * (bin(U) - that)
};
// wide form: the bins of C (a no-op otherwise); then the exact keys of C
// (wide form) and the walk
hipError_t launch_rabitq_walk_prep(const RabitqWalkArgs& a, hipStream_t s);
hipError_t launch_rabitq_walk(const RabitqWalkArgs& a, hipStream_t s);

constexpr int FINAL_STATIC_LDS = 21000;  // bytes of static LDS of the final top-k kernel (upper bound)
hipError_t launch_final_topk(const FinalArgs& a, hipStream_t s);
// candidates per thread the final top-k kernel holds in registers for at most
// max_kc candidates per query (8, 16, 24, 32; 0 = memory form)
int final_topk_form(int64_t max_kc);

}  // namespace bbc

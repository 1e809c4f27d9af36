// Launch descriptors for the query-path kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/bbc.h"

namespace bbc {

// Records the message of a failing call (bbc_last_error) and returns code.
int32_t set_error(int32_t code, const std::string& msg);

int32_t build_index_pq(int32_t device, const float* base, int64_t n, int32_t d, const bbc_build_params* p,
                       bbc_index** out);

struct ProbeArgs {
  const float* q; int64_t nq; int d;
  const float* cent; const uint16_t* cent_bf16; int dpad;
  const float* cent_norm2; const float* cent_norm; int nlist; int metric;
  const int32_t* nprobe; const int64_t* probe_off; const int64_t* list_off;
  float* dprime; int32_t* probe_lists; float* probe_keys; int64_t* rank_off; int64_t* n_scanned;
  int32_t* n_recheck;
};
hipError_t launch_probe(const ProbeArgs& a, hipStream_t s);
size_t probe_select_lds(int nlist);

struct PqScanArgs {
  const float* q; int64_t nq; int d; const float* cent;
  int M; int bits; const float* codebook; const uint8_t* codes; int code_stride;
  const int64_t* list_off; const int64_t* probe_off; const int32_t* probe_lists;
  const int64_t* rank_off; const int64_t* key_off; float* keys;
  int rank_begin; int rank_end;
};
hipError_t launch_pq_scan(const PqScanArgs& a, int64_t npairs, hipStream_t s);

struct CollectArgs {
  int64_t nq; const float* keys; const int64_t* key_off; const int64_t* n_scanned;
  const int32_t* nprobe; const int64_t* probe_off; const int32_t* probe_lists; const int64_t* rank_off;
  const int64_t* list_off; const int32_t* list_ids; const int32_t* pos_of_id;
  const int64_t* kc_target; const int64_t* cand_off; int m; int nsample; int bcap;
  uint32_t* cand_pos; int64_t* n_cand;
  // trace outputs (all null when tracing is off)
  float* t_dmin; float* t_delta; uint8_t* t_map; int32_t* t_tau; int64_t* t_s; int32_t* t_counts;
  int64_t* t_nboundary;
};
hipError_t launch_collect_bucket(const CollectArgs& a, hipStream_t s);

struct RerankArgs {
  const float* q; int64_t nq; int d; int metric; const void* vectors; int fp16;
  const int32_t* list_ids; const uint32_t* cand_pos; const int64_t* cand_off; const int64_t* n_cand;
  uint64_t* cand_packed;
};
hipError_t launch_rerank(const RerankArgs& a, int64_t max_kc, hipStream_t s);

struct FinalArgs {
  int64_t nq; const int32_t* k; const int64_t* n_cand; const int64_t* cand_off; uint64_t* cand_packed;
  const int64_t* out_off; int64_t* out_ids; float* out_dists; int32_t* out_counts; int metric; int run;
};
hipError_t launch_final_topk(const FinalArgs& a, hipStream_t s);

}  // namespace bbc

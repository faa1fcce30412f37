// pts_multi.h -- work descriptors of packed (multi-request) launches.
#pragma once

#include "pts_internal.h"

namespace pts {

// One workgroup of a packed farthest-point / blend launch.
struct WorkDesc {
  const char* rec;    // cloud record buffer
  const float* x;     // the request's queries (device, [Q,3])
  float* far2;        // the request's per-split maxima [S][Q]
  float2* part;       // the request's per-split partials [S][Q]
  int64_t Q;          // the request's query count
  int64_t per_split;  // points per split of the cloud
  int64_t pos_off;    // byte offsets of the pos4 / record sections
  int64_t rec_off;
  int32_t S;          // splits of the cloud
  int32_t qb;         // query block (kBlock * multi_qpl() queries)
  int32_t split;      // this workgroup's split
  int32_t pad;
};

// One workgroup of the packed combine: block qb of one request's queries,
// kBlock queries each for S <= kLaneSplitsMax, kBlock / 64 beyond.
struct CombDesc {
  float* far2;  // the request's per-split maxima, folded here when S > kLaneSplitsMax
  const float2* part;
  float* out;
  int64_t Q;
  int32_t S;
  int32_t qb;
};

// fold: some request of the launch has more than kLaneSplitsMax splits.
int launch_multi(const WorkDesc* d_work, int64_t n_work, const CombDesc* d_comb, int64_t n_comb, float C,
                 bool fold, hipStream_t st);
int multi_qpl();

}  // namespace pts

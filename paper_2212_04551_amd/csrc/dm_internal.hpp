// Internal interfaces between the C-ABI layer (dm_api.hip) and the kernel
// translation units.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "dm_device.hpp"

namespace dm {

// Arguments of the persistent k-clique kernel (graph in rank space, DAG CSR).
struct CliqueArgs {
  const int64_t* rp;       // DAG row offsets, n+1
  const int32_t* col;      // DAG out-neighbours (all of higher rank), sorted
  int32_t n;
  int k;
  int dmax;                // largest out-degree (sizes LDS / scratch)
  int W;                   // 64-bit words per candidate bitset = ceil(dmax/64)
  unsigned long long* out; // per-graph counters (batch) or one counter
  const int32_t* root_graph;  // rank -> graph index; null = single graph
  int* flags;              // [0] overflow, [1] capacity error
  unsigned long long* root_stats;  // 3 per stat row, or null
  unsigned long long* wave_stats;  // 4 per wave, or null
  int wave_stats_len;
  unsigned long long* rows_global; // per-wave bitmap rows when they do not fit in LDS
  int prune;               // skip subtrees that cannot reach k vertices
  Sched S;
};

// Arguments of the persistent induced k-motif kernel (undirected CSR).
struct MotifArgs {
  const int64_t* rp;
  const int32_t* col;
  int32_t n;
  int k;
  int dmax;                // largest degree
  int ncls;
  const uint8_t* table;    // canonical-relabeling dictionary, 2^(k(k-1)/2-1) entries
  unsigned long long* out; // [graphs][ncls]
  const int32_t* root_graph;
  int* flags;
  unsigned long long* root_stats;
  unsigned long long* wave_stats;
  int wave_stats_len;
  int32_t* ext_vert;       // per-wave extension stacks
  uint8_t* ext_mask;
  int32_t* new_buf;        // per-wave buffer of new extensions
  int64_t wave_ext_cap;    // entries per wave in ext_vert / ext_mask
  int64_t level_off[8];    // start of level s inside a wave's region
  int64_t level_cap[8];
  Sched S;
};

// kernel launchers (return hipSuccess or the launch error)
hipError_t launch_clique(const CliqueArgs& a, int grid, bool rows_in_lds, size_t lds_bytes, hipStream_t s);
size_t clique_lds_bytes(int dmax, int W, int k, bool rows_in_lds);
hipError_t clique_occupancy(bool rows_in_lds, size_t lds_bytes, int* blocks_per_cu);

hipError_t launch_motif(const MotifArgs& a, int grid, size_t lds_bytes, hipStream_t s);
size_t motif_lds_bytes(int k, int ncls);
hipError_t motif_occupancy(size_t lds_bytes, int* blocks_per_cu);

// graph preparation
hipError_t launch_validate(const int64_t* rp, const int32_t* col, int32_t n, int64_t nnz, int* flag,
                           hipStream_t s);
// (degree, id) rank orientation: out rank[n], order[n] (rank -> vertex), drp[n+1], dcol[nnz/2]
hipError_t orient_by_degree(const int64_t* rp, const int32_t* col, int32_t n, int64_t nnz, int32_t* rank,
                            int32_t* order, int64_t* drp, int32_t* dcol, int* dmax_out, hipStream_t s);
// max degree of a CSR (device), written to *out (device int)
hipError_t launch_max_degree(const int64_t* rp, int32_t n, int* out, hipStream_t s);
// map vertex ids through a table: out[i] = map[in[i]]
hipError_t launch_gather_i32(const int32_t* map, const int32_t* in, int32_t* out, int64_t count, hipStream_t s);
// offset copy: out[i] = in[i] + off (int64 row offsets) / (int32 column ids)
hipError_t launch_offset_i64(const int64_t* in, int64_t* out, int64_t count, int64_t off, hipStream_t s);
hipError_t launch_offset_i32(const int32_t* in, int32_t* out, int64_t count, int32_t off, hipStream_t s);
hipError_t launch_fill_i32(int32_t* out, int64_t count, int32_t value, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* out, int64_t count, unsigned long long value, hipStream_t s);

}  // namespace dm

// Internal interfaces between the C-ABI layer (dm_api.hip) and the kernel
// translation units.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "dm_device.hpp"

namespace dm {

constexpr int kMlpNet = 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1;  // 4545 weights
constexpr int kMlpBlob = kMlpNet + 8;                          // + feature mean[4], std[4]

// Largest motif size: the canonical-relabeling dictionary of k = 8 has
// 2^27 entries of 16-bit class ids (11,117 classes); entries whose code some
// v_i reaches with no edge to its predecessors hold kUnreachable.
constexpr int kMotifMaxK = 8;
constexpr uint16_t kUnreachable = 0xFFFF;

// Roots with at most this many out-neighbours keep their bitmap rows in LDS;
// wider roots read them from the graph's row cache or a per-wave global region.
constexpr int kCliqueLocalRows = 128;

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
  unsigned long long* rcache;      // the graph's cached bitmap rows (root v at rcoff[v], stride d)
  const int64_t* rcoff;
  int rc_mode;             // 0: no cache, 1: build it while counting, 2: read it
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
  const uint16_t* table;   // canonical-relabeling dictionary, 2^(k(k-1)/2-1) entries
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
  int leaf_lds;            // the (k-2)-level list may be built straight into LDS (counting)
  unsigned long long* wave_cnt;  // k = 8: per-wave class counters in global memory (ncls per wave)
  Sched S;
};

// Arguments of the one-lane-per-traversal ablation kernels (dm_dfs.hip).
constexpr int kDfsMaxK = 16;
struct DfsArgs {
  const int64_t* rp;       // cliques: DAG CSR in rank space; motifs: undirected CSR in rank space
  const int32_t* col;
  int32_t n;
  int k;
  int dmax;                // largest (out-)degree
  unsigned long long* out; // one counter (cliques) or ncls counters (motifs)
  int* flags;              // [0] overflow, [1] capacity / dictionary errors
  unsigned long long* qhead;  // next root
  int32_t* stack;          // per-lane stacks, lane_stride entries each
  uint8_t* masks;          // motifs: mask byte per stack entry
  int64_t lane_stride;
  const uint16_t* table;   // motifs: canonical-relabeling dictionary
  int ncls;
  int64_t level_off[kDfsMaxK + 1];  // motifs: start of level s in a lane's stack
  int64_t level_cap[kDfsMaxK + 1];
};

// Listing ring (aggregate_store): rows of `width` int32 written by the kernel
// straight into pinned host memory and drained by the calling host thread.
// Row r occupies slot r mod (rows_per_block * nblocks) of generation
// r / (rows_per_block * nblocks); a wave writes a row only once the host has
// drained that slot's block of the previous generation (freed[block] >= gen),
// then stores valid[slot] = gen + 1 (a plain system-scope store after a
// system-scope release fence, so no host-memory read-modify-write is needed).
struct Ring {
  int32_t* rows;                     // host-pinned [slots][width]
  unsigned* valid;                   // host-pinned [slots]
  const unsigned long long* freed;   // host-pinned [nblocks]
  unsigned long long* reserve;       // device: rows reserved so far
  const int32_t* order;              // rank -> original vertex id
  int width;
  int rows_per_block;
  int nblocks;
  uint64_t wait_limit;               // wall-clock ticks a wave may wait for the host
  int* flags;                        // flags[1] |= kFlagWaitLimit when a wave gives up
};

// Wave-uniform: hand `c` (1..64) rows to the ring.  Row i (lane i's row) is
// order[prefix[0..np-1]], order[last of lane i], then `extra` of lane i when
// width == np + 2.  All lanes must be active.  Returns false when the wave
// gave up waiting for the host (the launch is then flagged).
__device__ __forceinline__ bool ring_emit(const Ring& R, const int* prefix, int np, int last, int extra, int c) {
  const int lane = lane_id();
  long long base = 0;
  if (lane == 0) base = static_cast<long long>(add_u64_relaxed(R.reserve, static_cast<unsigned long long>(c)));
  base = uni64(base);
  const long long slots = static_cast<long long>(R.rows_per_block) * R.nblocks;
  // wait until the host has drained the previous generation of each block
  // the rows land in (at most two blocks: c <= 64 <= rows_per_block)
  for (long long r = base; r < base + c;) {
    const long long gen = r / slots;
    const int b = static_cast<int>((r % slots) / R.rows_per_block);
    const uint64_t t0 = wall_clock64();
    for (;;) {
      unsigned long long fr = 0;
      if (lane == 0)
        fr = __hip_atomic_load(const_cast<unsigned long long*>(R.freed + b), __ATOMIC_ACQUIRE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
      if (static_cast<long long>(uniu64(fr)) >= gen) break;
      if (uniu64(wall_clock64() - t0) > R.wait_limit) {
        if (lane == 0) atomicOr(R.flags + 1, kFlagWaitLimit);
        return false;
      }
      __builtin_amdgcn_s_sleep(32);
    }
    r = (r / R.rows_per_block + 1) * R.rows_per_block;  // next block boundary
  }
  const int w = R.width;
  for (int j = lane; j < kWave * w; j += kWave) {
    const int row = j / w, colw = j - row * w;
    const int lv = __shfl(last, row < kWave ? row : 0, kWave);
    const int ex = __shfl(extra, row < kWave ? row : 0, kWave);
    if (row < c) {
      int v;
      if (colw < np) v = R.order[prefix[colw]];
      else if (colw == np) v = R.order[lv];
      else v = ex;
      const long long slot = (base + row) % slots;
      R.rows[slot * w + colw] = v;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  if (lane < c) {
    const long long r = base + lane;
    __hip_atomic_store(R.valid + (r % slots), static_cast<unsigned>(r / slots + 1), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
  return true;
}

// Directed graphs (dm_digraph.hip): the underlying undirected graph drives
// the enumeration, two arc bits per adjacency entry drive the classification.
constexpr int kDMotifMaxK = 5;
struct DMotifArgs {
  const int64_t* rp;       // underlying undirected graph (original ids), sorted lists
  const int32_t* col;
  const uint8_t* dir;      // per entry (u, w): bit 0 arc u -> w, bit 1 arc w -> u
  int32_t n;
  int k;
  int dmax;                // largest undirected degree
  int ncls;
  const uint16_t* table;   // directed code (2 bits per vertex pair) -> class, 2^(k(k-1)) entries
  unsigned long long* out; // [ncls]
  int* flags;              // [0] overflow, [1] capacity / dictionary errors
  int32_t* vert;           // per-wave level lists (levels 1..k-1)
  uint8_t* mask;
  uint16_t* arcs;
  uint8_t* hit;            // per-wave marks of the entries an extension touches
  int32_t* nbuf;           // per-wave new entries (dmax each)
  uint8_t* ndir;
  int64_t wave_cap;        // entries per wave in vert / mask / arcs
  int64_t hit_cap;         // entries per wave in hit
  int leaf_cap;            // entries of the level k-2 list kept in LDS
  int64_t level_off[kDMotifMaxK + 1];
  int64_t level_cap[kDMotifMaxK + 1];
  Sched S;
};
hipError_t launch_arc_validate(const int64_t* rp, const int32_t* col, int32_t n, int64_t arcs, int* flag,
                               hipStream_t s);
// the underlying undirected graph of the arcs (sorted out-lists): urp[n+1],
// ucol[unnz], udir[unnz], allocated here (hipMalloc) and owned by the caller
hipError_t digraph_underlying(const int64_t* rp, const int32_t* col, int32_t n, int64_t arcs, int64_t** urp,
                              int32_t** ucol, uint8_t** udir, int64_t* unnz, hipStream_t s);
// the arc bits in the rank-renamed graph: udir[urp[rank[u]] + j] for the
// entry of rank[w] in row rank[u]; flag |= 1 for an entry the renamed graph
// lacks
hipError_t digraph_rank_dir(const int64_t* rp, const int32_t* col, const uint8_t* dir, int32_t n, const int32_t* rank,
                            const int64_t* urp, const int32_t* ucol, uint8_t* udir, int* flag, hipStream_t s);
// launch shape of the directed motif kernel: waves per workgroup (they share
// one LDS copy of the class counters), workgroups per CU, the LDS level list
// length and the dynamic LDS bytes
struct DMotifPlan {
  int waves_per_group;
  int leaf_cap;
  int groups_per_cu;
  size_t lds;
};
size_t dmotif_lds_bytes(int ncls, int leaf_cap, int waves);
hipError_t dmotif_plan(int ncls, int max_waves_per_cu, DMotifPlan* plan);
hipError_t launch_dmotif(const DMotifArgs& a, int grid, int waves_per_group, size_t lds_bytes, hipStream_t s);
// kernel launchers (return hipSuccess or the launch error)
hipError_t launch_dfs_clique(const DfsArgs& a, int grid, hipStream_t s);
hipError_t launch_dfs_motif(const DfsArgs& a, int grid, hipStream_t s);
hipError_t launch_clique(const CliqueArgs& a, int grid, size_t lds_bytes, hipStream_t s);
size_t clique_lds_bytes(int dmax, int W, int k);
hipError_t clique_occupancy(size_t lds_bytes, int* blocks_per_cu);

hipError_t launch_motif(const MotifArgs& a, int grid, size_t lds_bytes, hipStream_t s);
// listing (aggregate_store): cliques on the DAG, one wave per root; motifs
// with the motif kernel's extension steps down to |tr| = k-1
struct CliqueListArgs {
  const int64_t* rp;   // DAG CSR in rank space
  const int32_t* col;
  int32_t n;
  int k;
  int dmax;            // largest out-degree
  int32_t* stack;      // per-wave level lists, (k-1) * dmax entries per wave
  int* flags;
  Sched S;
  Ring R;
};
hipError_t launch_list_cliques(const CliqueListArgs& a, int grid, hipStream_t s);
hipError_t launch_list_motifs(const MotifArgs& a, const Ring& R, int grid, size_t lds_bytes, hipStream_t s);
size_t motif_list_lds_bytes();
size_t motif_lds_bytes(int k, int ncls);
hipError_t motif_occupancy(int k, size_t lds_bytes, int* blocks_per_cu);

// graph preparation
hipError_t launch_validate(const int64_t* rp, const int32_t* col, int32_t n, int64_t nnz, int* flag,
                           hipStream_t s);
// (degree, id) rank orientation: out rank[n], order[n] (rank -> vertex), drp[n+1], dcol[nnz/2]
hipError_t orient_by_degree(const int64_t* rp, const int32_t* col, int32_t n, int64_t nnz, int32_t* rank,
                            int32_t* order, int64_t* drp, int32_t* dcol, int* dmax_out, hipStream_t s);
// the graph renamed by rank: urp[n+1], ucol[nnz] (sorted adjacency)
hipError_t relabel_by_rank(const int64_t* rp, const int32_t* col, int32_t n, int64_t nnz, const int32_t* rank,
                           const int32_t* order, int64_t* urp, int32_t* ucol, hipStream_t s);
// max degree of a CSR (device), written to *out (device int)
hipError_t launch_max_degree(const int64_t* rp, int32_t n, int* out, hipStream_t s);
// map vertex ids through a table: out[i] = map[in[i]]
hipError_t launch_gather_i32(const int32_t* map, const int32_t* in, int32_t* out, int64_t count, hipStream_t s);
// induced subgraph on the vertices with keep[v] != 0 (device keep[n]); see dm_graph.hip
hipError_t induced_subgraph(const int64_t* rp, const int32_t* col, int32_t n, const uint8_t* keep, int64_t* newid,
                            int64_t* srp, int32_t** scol, int32_t* n_out, int64_t* nnz_out, hipStream_t s);
hipError_t row_cache_layout(const int64_t* drp, int32_t n, int64_t* off, int64_t* total, hipStream_t s);
// offset copy: out[i] = in[i] + off (int64 row offsets) / (int32 column ids)
hipError_t launch_offset_i64(const int64_t* in, int64_t* out, int64_t count, int64_t off, hipStream_t s);
hipError_t launch_offset_i32(const int32_t* in, int32_t* out, int64_t count, int32_t off, hipStream_t s);
hipError_t launch_fill_i32(int32_t* out, int64_t count, int32_t value, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* out, int64_t count, unsigned long long value, hipStream_t s);

// learned ordering (dm_learn.hip)
hipError_t compute_features(const int64_t* rp, const int32_t* col, int32_t n, const int64_t* drp,
                            const int32_t* dcol, const int32_t* order, int64_t* F, hipStream_t s);
hipError_t mlp_init(float* P, uint64_t seed, hipStream_t s);
hipError_t mlp_fit_normaliser(float* P, const int64_t* F, int64_t n, hipStream_t s);
hipError_t mlp_forward(const float* P, const int64_t* F, int64_t n, float* out, hipStream_t s);
hipError_t mlp_targets(const unsigned long long* stats, int64_t n, float* out, hipStream_t s);
hipError_t mlp_loss_grad(const float* P, const int64_t* F, const float* T, const int32_t* rows, int64_t nrows,
                         float* partial, float* grad, float* loss, hipStream_t s);
hipError_t mlp_adam(float* P, const float* g, float* m, float* v, int64_t t, float lr, hipStream_t s);
hipError_t mlp_shuffle(uint64_t seed, int64_t n, unsigned long long* keys, unsigned long long* keys_out,
                       int32_t* vals, int32_t* vals_out, void* temp, size_t temp_bytes, hipStream_t s);
size_t mlp_shuffle_temp_bytes(int64_t n);
hipError_t param_fingerprint(const float* P, int n, unsigned long long* dev_out, hipStream_t s);
hipError_t lpt_order(const float* pred, int64_t n, int chunks_wanted, int32_t* order_out, int64_t* bounds_out,
                     int64_t* nchunks, hipStream_t s);

}  // namespace dm

// Graph preparation on the GPU: CSR validation and the degree-ordered DAG used
// by clique counting.
//
//   - Validation enforces the input model of DuMato, Section II: simple,
//     undirected, unlabelled graphs (no self-loops, no repeated edges, both
//     directions present), with sorted adjacency so neighbour lists can be
//     merged and searched.
//   - Orientation: clique counting only extends a traversal by vertices above
//     its last vertex (the `lower` filter of Section IV-E, Alg. 4).  Ranking
//     vertices by (degree, id) and keeping u -> w iff rank(u) < rank(w) makes
//     every out-list short and lets the filter disappear once vertices are
//     renamed by rank.
#include <hipcub/hipcub.hpp>

#include "dm_internal.hpp"

namespace dm {

namespace {

// flag bits: 1 bad offsets, 2 id out of range, 4 self-loop, 8 not strictly
// ascending (or repeated), 16 missing reverse edge
__global__ void __launch_bounds__(256) validate_kernel(const int64_t* rp, const int32_t* col, int32_t n,
                                                       int64_t nnz, int* flag) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  int bad = 0;
  if (wave == 0 && lane == 0 && (rp[0] != 0 || rp[n] != nnz)) bad |= 1;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int64_t b = rp[v], e = rp[v + 1];
    if (e < b || b < 0 || e > nnz) {
      bad |= 1;
      continue;
    }
    for (int64_t i = b + lane; i < e; i += 64) {
      const int u = col[i];
      if (u < 0 || u >= n) {
        bad |= 2;
        continue;
      }
      if (u == v) bad |= 4;
      if (i > b && col[i - 1] >= u) bad |= 8;
      int64_t lo = rp[u], hi = rp[u + 1];
      if (lo < 0 || hi > nnz || hi < lo) {
        bad |= 1;
        continue;
      }
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < v) lo = mid + 1; else hi = mid;
      }
      if (lo >= rp[u + 1] || col[lo] != v) bad |= 16;
    }
  }
  if (bad) atomicOr(flag, bad);
}

__global__ void deg_key_kernel(const int64_t* rp, int32_t n, unsigned long long* keys) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) keys[v] = (static_cast<unsigned long long>(rp[v + 1] - rp[v]) << 32) | static_cast<uint32_t>(v);
}

__global__ void rank_kernel(const unsigned long long* sorted, int32_t n, int32_t* rank, int32_t* order) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    const int32_t v = static_cast<int32_t>(sorted[i] & 0xffffffffull);
    order[i] = v;
    rank[v] = static_cast<int32_t>(i);
  }
}

// out-degree of each vertex (original ids) in the rank orientation
__global__ void __launch_bounds__(256) outdeg_kernel(const int64_t* rp, const int32_t* col, int32_t n,
                                                     const int32_t* rank, int64_t* outdeg) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int rv = rank[v];
    int c = 0;
    for (int64_t i = rp[v] + lane; i < rp[v + 1]; i += 64) c += rank[col[i]] > rv ? 1 : 0;
    c = wave_sum_i32(c);
    if (lane == 0) outdeg[v] = c;
  }
}

// write (rank(u) << 32 | rank(w)) for every oriented edge u -> w
__global__ void __launch_bounds__(256) emit_kernel(const int64_t* rp, const int32_t* col, int32_t n,
                                                   const int32_t* rank, const int64_t* eoff,
                                                   unsigned long long* keys) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int rv = rank[v];
    int64_t pos = eoff[v];
    for (int64_t c = rp[v]; c < rp[v + 1]; c += 64) {
      const int64_t i = c + lane;
      const bool take = i < rp[v + 1] && rank[col[i]] > rv;
      const uint64_t b = ballot(take);
      if (take)
        keys[pos + mbcnt(b)] = (static_cast<unsigned long long>(rv) << 32) | static_cast<uint32_t>(rank[col[i]]);
      pos += __popcll(b);
    }
  }
}

// write (rank(u) << 32 | rank(w)) for every directed edge u -> w
__global__ void __launch_bounds__(256) emit_all_kernel(const int64_t* rp, const int32_t* col, int32_t n,
                                                       const int32_t* rank, unsigned long long* keys) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nnz = rp[n];
  if (i >= nnz) return;
  // source vertex of entry i: last v with rp[v] <= i
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (rp[mid] <= i) lo = mid; else hi = mid;
  }
  keys[i] = (static_cast<unsigned long long>(rank[lo]) << 32) | static_cast<uint32_t>(rank[col[i]]);
}

__global__ void deg_by_rank_kernel(const int64_t* rp, const int32_t* order, int32_t n, int64_t* cnt) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < n) cnt[r] = rp[order[r] + 1] - rp[order[r]];
  if (r == n) cnt[n] = 0;
}

__global__ void split_low_kernel(const unsigned long long* keys, int64_t m, int32_t* dcol) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m) dcol[i] = static_cast<int32_t>(keys[i] & 0xffffffffull);
}

__global__ void permute_deg_kernel(const int64_t* outdeg, const int32_t* order, int32_t n, int64_t* cnt_rank) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < n) cnt_rank[r] = outdeg[order[r]];
  if (r == n) cnt_rank[n] = 0;
}

__global__ void max_deg_kernel(const int64_t* rp, int32_t n, int* out) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  int d = 0;
  if (v < n) d = static_cast<int>(rp[v + 1] - rp[v]);
  for (int sh = 32; sh >= 1; sh >>= 1) {
    const int y = __shfl_xor(d, sh, 64);
    d = d > y ? d : y;
  }
  if ((threadIdx.x & 63) == 0 && d > 0) atomicMax(out, d);
}

__global__ void gather_kernel(const int32_t* map, const int32_t* in, int32_t* out, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = map[in[i]];
}

__global__ void offset_i64_kernel(const int64_t* in, int64_t* out, int64_t count, int64_t off) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = in[i] + off;
}

__global__ void offset_i32_kernel(const int32_t* in, int32_t* out, int64_t count, int32_t off) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = in[i] + off;
}

__global__ void fill_i32_kernel(int32_t* out, int64_t count, int32_t value) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = value;
}

__global__ void fill_u64_kernel(unsigned long long* out, int64_t count, unsigned long long value) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = value;
}

inline unsigned blocks_for(int64_t count, int threads) {
  int64_t b = (count + threads - 1) / threads;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

inline int bits_for(int64_t x) {
  int b = 1;
  while (b < 62 && (int64_t{1} << b) <= x) ++b;
  return b;
}

}  // namespace

hipError_t launch_validate(const int64_t* rp, const int32_t* col, int32_t n, int64_t nnz, int* flag,
                           hipStream_t s) {
  const int64_t waves = n > 0 ? n : 1;
  unsigned grid = blocks_for(waves * 64, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(validate_kernel, dim3(grid), dim3(256), 0, s, rp, col, n, nnz, flag);
  return hipGetLastError();
}

hipError_t launch_max_degree(const int64_t* rp, int32_t n, int* out, hipStream_t s) {
  hipLaunchKernelGGL(max_deg_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rp, n, out);
  return hipGetLastError();
}

hipError_t launch_gather_i32(const int32_t* map, const int32_t* in, int32_t* out, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, map, in, out, count);
  return hipGetLastError();
}

hipError_t launch_offset_i64(const int64_t* in, int64_t* out, int64_t count, int64_t off, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(offset_i64_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, in, out, count, off);
  return hipGetLastError();
}

hipError_t launch_offset_i32(const int32_t* in, int32_t* out, int64_t count, int32_t off, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(offset_i32_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, in, out, count, off);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* out, int64_t count, int32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, out, count, value);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* out, int64_t count, unsigned long long value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, out, count, value);
  return hipGetLastError();
}

#define DM_TRY(x)                          \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) {                \
      err = e_;                            \
      goto done;                           \
    }                                      \
  } while (0)

// words of root v's bitmap rows: ceil(d / 64) words for each of its d members
__global__ void row_words_kernel(const int64_t* drp, int32_t n, int64_t* words) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) {
    const int64_t d = drp[v + 1] - drp[v];
    words[v] = ((d + 63) / 64) * d;
  }
}

// Layout of a graph's cached bitmap rows: off[v] = words before root v (n + 1
// entries; off[n] = total).  `off` needs n + 1 int64 of device memory.
hipError_t row_cache_layout(const int64_t* drp, int32_t n, int64_t* off, int64_t* total, hipStream_t s) {
  hipError_t e = hipSuccess;
  int64_t* words = nullptr;
  void* temp = nullptr;
  size_t tb = 0;
  *total = 0;
  if (n <= 0) return hipMemsetAsync(off, 0, sizeof(int64_t), s);
  e = hipMalloc(&words, sizeof(int64_t) * (static_cast<size_t>(n) + 1));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(row_words_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, drp, n, words);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemsetAsync(words + n, 0, sizeof(int64_t), s);
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(nullptr, tb, words, off, n + 1, s);
  if (e == hipSuccess) e = hipMalloc(&temp, tb > 0 ? tb : 16);
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(temp, tb, words, off, n + 1, s);
  if (e == hipSuccess) e = hipMemcpyAsync(total, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (temp) (void)hipFree(temp);
  if (words) (void)hipFree(words);
  return e;
}

hipError_t orient_by_degree(const int64_t* rp, const int32_t* col, int32_t n, int64_t nnz, int32_t* rank,
                            int32_t* order, int64_t* drp, int32_t* dcol, int* dmax_out, hipStream_t s) {
  hipError_t err = hipSuccess;
  unsigned long long *keys = nullptr, *keys2 = nullptr;
  int64_t *outdeg = nullptr, *eoff = nullptr, *cnt_rank = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0, need = 0;
  int* dmax_dev = nullptr;
  const int64_t m = nnz / 2;
  const int64_t nk = n > 0 ? n : 1;
  const int64_t mk = m > 0 ? m : 1;
  const int rbits = bits_for(n);
  DM_TRY(hipMalloc(&keys, sizeof(unsigned long long) * (mk > nk ? mk : nk)));
  DM_TRY(hipMalloc(&keys2, sizeof(unsigned long long) * (mk > nk ? mk : nk)));
  DM_TRY(hipMalloc(&outdeg, sizeof(int64_t) * (nk + 1)));
  DM_TRY(hipMalloc(&eoff, sizeof(int64_t) * (nk + 1)));
  DM_TRY(hipMalloc(&cnt_rank, sizeof(int64_t) * (nk + 1)));
  DM_TRY(hipMalloc(&dmax_dev, sizeof(int)));
  // temp storage large enough for every primitive below
  DM_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, need, keys, keys2, static_cast<int>(nk), 0, 64, s));
  temp_bytes = need;
  DM_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, need, keys, keys2, static_cast<int>(mk), 0, 64, s));
  if (need > temp_bytes) temp_bytes = need;
  DM_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, need, outdeg, eoff, static_cast<int>(nk + 1), s));
  if (need > temp_bytes) temp_bytes = need;
  DM_TRY(hipMalloc(&temp, temp_bytes > 0 ? temp_bytes : 16));
  if (n > 0) {
    // 1. rank by (degree, id)
    hipLaunchKernelGGL(deg_key_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rp, n, keys);
    DM_TRY(hipGetLastError());
    need = temp_bytes;
    DM_TRY(hipcub::DeviceRadixSort::SortKeys(temp, need, keys, keys2, n, 0, 32 + bits_for(n), s));
    hipLaunchKernelGGL(rank_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys2, n, rank, order);
    DM_TRY(hipGetLastError());
    // 2. out-degrees and emit positions
    {
      unsigned grid = blocks_for(static_cast<int64_t>(n) * 64, 256);
      if (grid > 65536) grid = 65536;
      hipLaunchKernelGGL(outdeg_kernel, dim3(grid), dim3(256), 0, s, rp, col, n, rank, outdeg);
      DM_TRY(hipGetLastError());
      DM_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(outdeg + n), 1, 0ull, s));
      need = temp_bytes;
      DM_TRY(hipcub::DeviceScan::ExclusiveSum(temp, need, outdeg, eoff, n + 1, s));
      // 3. emit oriented edges as (rank u, rank w) keys and sort them
      hipLaunchKernelGGL(emit_kernel, dim3(grid), dim3(256), 0, s, rp, col, n, rank, eoff, keys);
      DM_TRY(hipGetLastError());
    }
    if (m > 0) {
      need = temp_bytes;
      DM_TRY(hipcub::DeviceRadixSort::SortKeys(temp, need, keys, keys2, static_cast<int>(m), 0, 32 + rbits, s));
      hipLaunchKernelGGL(split_low_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, s, keys2, m, dcol);
      DM_TRY(hipGetLastError());
    }
    // 4. DAG offsets in rank order
    hipLaunchKernelGGL(permute_deg_kernel, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, outdeg, order, n,
                       cnt_rank);
    DM_TRY(hipGetLastError());
    need = temp_bytes;
    DM_TRY(hipcub::DeviceScan::ExclusiveSum(temp, need, cnt_rank, drp, n + 1, s));
    DM_TRY(launch_fill_i32(dmax_dev, 1, 0, s));
    DM_TRY(launch_max_degree(drp, n, dmax_dev, s));
    DM_TRY(hipMemcpyAsync(dmax_out, dmax_dev, sizeof(int), hipMemcpyDeviceToHost, s));
  } else {
    *dmax_out = 0;
    DM_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(drp), 1, 0ull, s));
  }
  DM_TRY(hipStreamSynchronize(s));
done:
  (void)hipFree(keys);
  (void)hipFree(keys2);
  (void)hipFree(outdeg);
  (void)hipFree(eoff);
  (void)hipFree(cnt_rank);
  (void)hipFree(dmax_dev);
  (void)hipFree(temp);
  return err;
}

}  // namespace dm

namespace dm {

// The same graph with vertex v renamed rank[v]: urp / ucol in rank space,
// adjacency sorted.  Used by motif counting so that every traversal is rooted
// at its lowest (degree, id) vertex.
hipError_t relabel_by_rank(const int64_t* rp, const int32_t* col, int32_t n, int64_t nnz, const int32_t* rank,
                           const int32_t* order, int64_t* urp, int32_t* ucol, hipStream_t s) {
  if (n <= 0) return launch_fill_u64(reinterpret_cast<unsigned long long*>(urp), 1, 0ull, s);
  hipError_t err = hipSuccess;
  unsigned long long *keys = nullptr, *keys2 = nullptr;
  int64_t* cnt = nullptr;
  void* temp = nullptr;
  size_t need = 0, tb = 0;
  const int64_t mk = nnz > 0 ? nnz : 1;
  DM_TRY(hipMalloc(&keys, sizeof(unsigned long long) * mk));
  DM_TRY(hipMalloc(&keys2, sizeof(unsigned long long) * mk));
  DM_TRY(hipMalloc(&cnt, sizeof(int64_t) * (static_cast<int64_t>(n) + 1)));
  DM_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, need, keys, keys2, static_cast<int>(mk), 0, 64, s));
  tb = need;
  DM_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, need, cnt, urp, n + 1, s));
  tb = need > tb ? need : tb;
  DM_TRY(hipMalloc(&temp, tb > 0 ? tb : 16));
  if (nnz > 0) {
    hipLaunchKernelGGL(emit_all_kernel, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, rp, col, n, rank, keys);
    DM_TRY(hipGetLastError());
    need = tb;
    DM_TRY(hipcub::DeviceRadixSort::SortKeys(temp, need, keys, keys2, static_cast<int>(nnz), 0, 32 + bits_for(n), s));
    hipLaunchKernelGGL(split_low_kernel, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, keys2, nnz, ucol);
    DM_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(deg_by_rank_kernel, dim3(blocks_for(static_cast<int64_t>(n) + 1, 256)), dim3(256), 0, s, rp, order,
                     n, cnt);
  DM_TRY(hipGetLastError());
  need = tb;
  DM_TRY(hipcub::DeviceScan::ExclusiveSum(temp, need, cnt, urp, n + 1, s));
  DM_TRY(hipStreamSynchronize(s));
done:
  (void)hipFree(keys);
  (void)hipFree(keys2);
  (void)hipFree(cnt);
  (void)hipFree(temp);
  return err;
}

// ------------------------------------------------------------------ vertex property filter

namespace {

__global__ void keep_flag_kernel(const uint8_t* keep, int32_t n, int64_t* flag) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = keep[v] ? 1 : 0;
  if (v == n) flag[n] = 0;
}

// kept neighbours of each kept vertex, at its new id
__global__ void sub_degree_kernel(const int64_t* rp, const int32_t* col, int32_t n, const uint8_t* keep,
                                  const int64_t* newid, int64_t* deg) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n || !keep[v]) return;
  int64_t c = 0;
  for (int64_t e = rp[v]; e < rp[v + 1]; ++e) c += keep[col[e]] ? 1 : 0;
  deg[newid[v]] = c;
}

// new adjacency lists: kept neighbours renamed, still ascending (new ids keep the old order)
__global__ void sub_fill_kernel(const int64_t* rp, const int32_t* col, int32_t n, const uint8_t* keep,
                                const int64_t* newid, const int64_t* srp, int32_t* scol) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n || !keep[v]) return;
  int64_t o = srp[newid[v]];
  for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
    if (keep[col[e]]) scol[o++] = static_cast<int32_t>(newid[col[e]]);
}

}  // namespace

// Induced subgraph on the vertices with keep[v] != 0.  newid[n+1] (exclusive
// prefix of keep) and srp[n+1] are caller buffers; *n_out / *nnz_out come back
// to the host; scol is allocated here (caller frees, hipFree) when nnz_out > 0.
hipError_t induced_subgraph(const int64_t* rp, const int32_t* col, int32_t n, const uint8_t* keep, int64_t* newid,
                            int64_t* srp, int32_t** scol, int32_t* n_out, int64_t* nnz_out, hipStream_t s) {
  hipError_t err = hipSuccess;
  void* temp = nullptr;
  int64_t* flag = nullptr;
  size_t tb = 0, tb2 = 0;
  *scol = nullptr;
  int64_t n2 = 0, nnz2 = 0;
  DM_TRY(hipMalloc(&flag, sizeof(int64_t) * (static_cast<size_t>(n) + 1)));
  hipLaunchKernelGGL(keep_flag_kernel, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, keep, n, flag);
  DM_TRY(hipGetLastError());
  DM_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, flag, newid, n + 1, s));
  DM_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, flag, srp, n + 1, s));
  DM_TRY(hipMalloc(&temp, (tb > tb2 ? tb : tb2) + 16));
  DM_TRY(hipcub::DeviceScan::ExclusiveSum(temp, tb, flag, newid, n + 1, s));
  DM_TRY(hipMemcpyAsync(&n2, newid + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DM_TRY(hipStreamSynchronize(s));
  // degrees at new ids (flag reused), then their exclusive prefix
  hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n2 + 1, 256)), dim3(256), 0, s,
                     reinterpret_cast<unsigned long long*>(flag), n2 + 1, 0ull);
  DM_TRY(hipGetLastError());
  hipLaunchKernelGGL(sub_degree_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rp, col, n, keep, newid, flag);
  DM_TRY(hipGetLastError());
  DM_TRY(hipcub::DeviceScan::ExclusiveSum(temp, tb2, flag, srp, static_cast<int>(n2 + 1), s));
  DM_TRY(hipMemcpyAsync(&nnz2, srp + n2, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DM_TRY(hipStreamSynchronize(s));
  if (nnz2 > 0) {
    DM_TRY(hipMalloc(scol, sizeof(int32_t) * static_cast<size_t>(nnz2)));
    hipLaunchKernelGGL(sub_fill_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rp, col, n, keep, newid, srp,
                       *scol);
    DM_TRY(hipGetLastError());
  }
  DM_TRY(hipStreamSynchronize(s));
  *n_out = static_cast<int32_t>(n2);
  *nnz_out = nnz2;
done:
  if (temp) (void)hipFree(temp);
  if (flag) (void)hipFree(flag);
  if (err != hipSuccess && *scol) {
    (void)hipFree(*scol);
    *scol = nullptr;
  }
  return err;
}

}  // namespace dm

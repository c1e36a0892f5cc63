// Ablation kernels: one lane per traversal.
//
// The paper's DFS implementation (Section V-A, the "DFS" column of Table III)
// gives each GPU thread a traversal of its own, explored depth-first with its
// extensions kept in a per-thread stack in global memory; DFS-wide exploration
// (Section IV-B) instead puts a whole warp on one traversal.  These kernels are
// that per-thread design on gfx950: each of the 64 lanes of a wave takes a root
// from a global counter, enumerates its whole tree alone, and takes the next
// root when it is done, so lanes of one wave diverge and their adjacency reads
// are not coalesced.  They compute the same counts as the wave kernels, with the
// same orientation, canonicality rule, pruning and dictionary, and exist to
// measure what the wave-per-traversal design gains.
#include "dm_internal.hpp"

namespace dm {

namespace {

// ------------------------------------------------------------------ cliques

// Lane-private stack: level s (2 <= s <= k-1) at stack + (s - 2) * dmax.
// Level 1 is N+(root) read in place from the DAG CSR.
__global__ void __launch_bounds__(64) dfs_clique_kernel(DfsArgs A) {
  const int lane = lane_id();
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWave + lane;
  int32_t* S = A.stack + t * A.lane_stride;
  const int k = A.k;
  uint64_t acc = 0;
  int ovf = 0;
  int cur[kDfsMaxK + 1];
  int len[kDfsMaxK + 1];
  for (;;) {
    const long long r = static_cast<long long>(add_u64_relaxed(A.qhead, 1ull));
    if (r >= A.n) break;
    const int v = static_cast<int>(r);
    const int64_t b = A.rp[v];
    const int d = static_cast<int>(A.rp[v + 1] - b);
    uint64_t add = 0;
    if (k == 1) {
      add = 1;
    } else if (k == 2) {
      add = static_cast<uint64_t>(d);
    } else if (d >= k - 1) {
      // DFS over levels 1..k-2; the extension count at level k-1 is aggregated
      int s = 1;
      cur[1] = 0;
      len[1] = d;
      while (s >= 1) {
        if (cur[s] >= len[s]) {
          --s;
          continue;
        }
        const int32_t* L = s == 1 ? A.col + b : S + static_cast<int64_t>(s - 2) * A.dmax;
        const int u = L[cur[s]];
        const int from = ++cur[s];
        // next set = L[from..len) intersected with N+(u) (both sorted)
        const int64_t ub = A.rp[u];
        const int du = static_cast<int>(A.rp[u + 1] - ub);
        const bool last = s + 1 == k - 1;
        int32_t* out = last ? nullptr : S + static_cast<int64_t>(s - 1) * A.dmax;
        int i = from, j = 0, m = 0;
        while (i < len[s] && j < du) {
          const int x = L[i], y = A.col[ub + j];
          if (x < y) {
            ++i;
          } else if (y < x) {
            ++j;
          } else {
            if (!last) out[m] = x;
            ++m;
            ++i;
            ++j;
          }
        }
        if (last) {
          add += static_cast<uint64_t>(m);
        } else if (m >= k - 1 - s) {  // enough candidates left to reach k vertices
          ++s;
          cur[s] = 0;
          len[s] = m;
        }
      }
    }
    const uint64_t before = acc;
    acc += add;
    if (acc < before) ovf = 1;
  }
  const uint64_t sum = wave_sum_u64(acc, &ovf);
  if (lane == 0) {
    add_counter(A.out, sum, A.flags);
    if (ovf) atomicOr(A.flags, 1);
  }
}

// ------------------------------------------------------------------ motifs

// Lane-private stack: level s (1 <= s <= k-2) holds N(tr) \ tr above v0 for
// the traversal tr = v_0..v_{s-1}, sorted by id, with a mask byte per entry
// (bit t: adjacent to v_t), at vert / mask + level_off[s].  At |tr| = k-1
// each canonical entry completes a k-traversal, classified through the
// dictionary into the wave's class counters in LDS.
__global__ void __launch_bounds__(64) dfs_motif_kernel(DfsArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(smem);
  const int lane = lane_id();
  for (int c = lane; c < A.ncls; c += kWave) cnt[c] = 0;
  __syncthreads();
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWave + lane;
  int32_t* V = A.stack + t * A.lane_stride;
  uint8_t* M = A.masks + t * A.lane_stride;
  const int k = A.k;
  int ovf = 0;
  int tr[kDfsMaxK + 1];
  int code[kDfsMaxK + 1];
  int cur[kDfsMaxK + 1];
  int len[kDfsMaxK + 1];
  for (;;) {
    const long long r = static_cast<long long>(add_u64_relaxed(A.qhead, 1ull));
    if (r >= A.n) break;
    const int v0 = static_cast<int>(r);
    const int64_t b0 = A.rp[v0];
    const int d0 = static_cast<int>(A.rp[v0 + 1] - b0);
    // level 1: neighbours of v0 above v0
    int n1 = 0;
    for (int i = 0; i < d0; ++i) {
      const int w = A.col[b0 + i];
      if (w > v0) {
        V[A.level_off[1] + n1] = w;
        M[A.level_off[1] + n1] = 1;
        ++n1;
      }
    }
    tr[0] = v0;
    code[1] = 0;
    int s = 1;
    cur[1] = 0;
    len[1] = n1;
    while (s >= 1) {
      if (cur[s] >= len[s]) {
        --s;
        continue;
      }
      const int32_t* E = V + A.level_off[s];
      const uint8_t* Em = M + A.level_off[s];
      const int px = cur[s]++;
      const int x = E[px];
      const unsigned mx = Em[px] & ((1u << s) - 1u);
      // canonical: x above v0 and above every traversal vertex after its
      // first neighbour
      const int f = __builtin_ctz(mx);
      bool canon = x > v0;
      for (int q = f + 1; q < s; ++q) canon = canon && x > tr[q];
      if (!canon) continue;
      if (s == k - 1) {
        const int c = code[s] | (s >= 2 ? static_cast<int>(mx << (s * (s - 1) / 2 - 1)) : 0);
        const int cls = A.table[c];
        if (cls == kUnreachable) atomicOr(A.flags + 1, 2);
        else atomicAdd(&cnt[cls], 1ull);
        continue;
      }
      // level s+1: the list without x, bit s set on x's neighbours, plus x's
      // neighbours above v0 that are neither listed nor in tr
      const int64_t xb = A.rp[x];
      const int dx = static_cast<int>(A.rp[x + 1] - xb);
      int32_t* N = V + A.level_off[s + 1];
      uint8_t* Nm = M + A.level_off[s + 1];
      const int64_t cap = A.level_cap[s + 1];
      int i = 0, j = 0, m = 0;
      while (i < len[s] || j < dx) {
        int y = INT_MAX;
        if (j < dx) y = A.col[xb + j];
        if (y <= v0) {
          ++j;
          continue;
        }
        const int e = i < len[s] ? E[i] : INT_MAX;
        int w;
        unsigned wm;
        if (e < y) {
          w = e;
          wm = Em[i];
          ++i;
        } else if (y < e) {
          w = y;
          wm = 1u << s;
          ++j;
          bool intr = false;
          for (int q = 0; q < s; ++q) intr = intr || tr[q] == y;
          if (intr) continue;
        } else {
          w = e;
          wm = Em[i] | (1u << s);
          ++i;
          ++j;
        }
        if (w == x) continue;
        if (m < cap) {
          N[m] = w;
          Nm[m] = static_cast<uint8_t>(wm);
        } else {
          atomicOr(A.flags + 1, 1);
        }
        ++m;
      }
      tr[s] = x;
      code[s + 1] = code[s] | (s >= 2 ? static_cast<int>(mx << (s * (s - 1) / 2 - 1)) : 0);
      ++s;
      cur[s] = 0;
      len[s] = m < cap ? m : static_cast<int>(cap);
    }
  }
  __syncthreads();
  for (int c = lane; c < A.ncls; c += kWave) add_counter(A.out + c, cnt[c], A.flags);
  if (ovf) atomicOr(A.flags, 1);
}

}  // namespace

hipError_t launch_dfs_clique(const DfsArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(dfs_clique_kernel, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_dfs_motif(const DfsArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(dfs_motif_kernel, dim3(grid), dim3(64), sizeof(unsigned long long) * a.ncls, s, a);
  return hipGetLastError();
}

}  // namespace dm

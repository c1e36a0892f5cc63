// Listing of k-cliques (aggregate_store, DuMato Section IV-C and Table II):
// the subgraphs themselves instead of their number.
//
// One wave owns one root v of the (degree, id)-oriented graph and walks its
// traversals depth first (Section IV-B, Alg. 1).  Level j of the wave's stack
// holds the extension list of the j-vertex traversal tr = v, x_1..x_{j-1}: the
// out-neighbours of v adjacent to every x and above the last one, in rank
// order.  Extend + Filter + Compact (Section IV-C, Alg. 2-3) for a chosen x:
// the lanes take the entries after x, binary-search each in N+(x) (coalesced
// list reads, sorted out-lists), and compact the hits with ballot / mbcnt
// into level j+1.  At |tr| = k-1 every entry of the list completes one
// k-clique, and the wave hands them, 64 at a time, to the host ring.
#include "dm_internal.hpp"

namespace dm {

namespace {

__device__ __forceinline__ bool in_sorted(const int32_t* a, int64_t n, int x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo < n && a[lo] == x;
}

__global__ void __launch_bounds__(64) list_cliques_kernel(CliqueListArgs A) {
  __shared__ int tr[kMaxK + 1];
  __shared__ int cur[kMaxK + 1];
  __shared__ int len[kMaxK + 1];
  const int lane = lane_id();
  const int k = A.k;
  int32_t* stk = A.stack + static_cast<int64_t>(blockIdx.x) * (k > 1 ? k - 1 : 1) * A.dmax;
  SchedIter it;
  sched_begin(A.S, it);
  Task t;
  bool ok = true;
  while (ok && sched_next(A.S, it, static_cast<int>(blockIdx.x), tr, &t)) {
    const int v = t.root;
    if (lane == 0) tr[0] = v;
    wave_sync();
    if (k == 1) {
      ok = ring_emit(A.R, tr, 0, v, 0, 1);
      continue;
    }
    const int64_t b0 = A.rp[v];
    const int d0 = static_cast<int>(A.rp[v + 1] - b0);
    if (d0 < k - 1) continue;
    // level 1: N+(v)
    for (int i = lane; i < d0; i += kWave) stk[i] = A.col[b0 + i];
    if (lane == 0) {
      len[1] = d0;
      cur[1] = 0;
    }
    wave_sync();
    int s = 1;  // traversal size; level s list in stk[(s-1) * dmax ..]
    while (s >= 1 && ok) {
      const int32_t* Ls = stk + static_cast<int64_t>(s - 1) * A.dmax;
      const int ns = len[s];
      if (s == k - 1) {
        // every entry completes a k-clique: tr[0..k-2] + entry
        for (int c = 0; c < ns && ok; c += kWave) {
          const int y = c + lane < ns ? Ls[c + lane] : 0;
          ok = ring_emit(A.R, tr, k - 1, y, 0, ns - c < kWave ? ns - c : kWave);
        }
        --s;
        continue;
      }
      const int i = cur[s];
      // prune: fewer entries left than vertices still to add
      if (ns - i < k - s) {
        --s;
        continue;
      }
      const int x = Ls[i];
      if (lane == 0) {
        cur[s] = i + 1;
        tr[s] = x;
      }
      const int64_t xb = A.rp[x];
      const int64_t dx = A.rp[x + 1] - xb;
      int32_t* Ln = stk + static_cast<int64_t>(s) * A.dmax;
      int nn = 0;
      for (int c = i + 1; c < ns; c += kWave) {
        const int j = c + lane;
        const int y = j < ns ? Ls[j] : 0;
        const bool keep = j < ns && in_sorted(A.col + xb, dx, y);
        const uint64_t bl = ballot(keep);
        if (keep) Ln[nn + mbcnt(bl)] = y;
        nn += __popcll(bl);
      }
      if (lane == 0) {
        len[s + 1] = nn;
        cur[s + 1] = 0;
      }
      wave_sync();
      if (nn >= k - s - 1) ++s;
    }
  }
  sched_end(A.S);
}

}  // namespace

hipError_t launch_list_cliques(const CliqueListArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(list_cliques_kernel, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace dm

// Persistent DFS-wide k-clique counting kernel for gfx950 (wave64).
//
// Method (DuMato, arXiv 2212.04551):
//   - Clique counting (Section IV-E, Alg. 4 left): extensions come from one
//     traversal vertex, non-canonical extensions (not above the last vertex)
//     are filtered, then extensions not adjacent to the whole traversal; at
//     |tr| = k-1 the extension count is aggregated (aggregate_counter).
//   - DFS-wide exploration (Section IV-B, Alg. 1): a stack of extension sets,
//     one level per traversal vertex; Move pushes an extension or pops.
//   - Warp-centric extend / filter / compact (Section IV-C, Alg. 2-3).
//   - Warp-level load balancing (Section IV-D), here in-kernel.
//
// gfx950 realisation:
//   - The graph is oriented by (degree, id) rank and relabelled, so "higher
//     rank" equals "higher id" and every out-neighbour list N+(v) is sorted;
//     the `lower` filter (keep extensions above the last vertex) is implicit.
//   - One wave owns one root v.  Its level-1 extension set is N+(v)
//     (coalesced read).  The wave builds, once per root, the adjacency of
//     N+(v) restricted to itself as bitmap rows (row i = positions j > i with
//     nbr[j] in N+(nbr[i])): every deeper extension set is then a bitset over
//     positions of N+(v), Extend+Filter+Compact become one AND with a row,
//     and aggregate_counter at |tr| = k-1 becomes a popcount.
//   - Rows live in LDS (word-major, so lane p reading row p is conflict-free)
//     when they fit, else in a per-wave global scratch region.
//   - The last two levels are fused: at |tr| = k-2 each lane takes one
//     extension u and adds popcount(C & row[u]), i.e. the extension count of
//     the (k-1)-traversal tr+u, without materialising it.
#include <climits>

#include "dm_internal.hpp"

namespace dm {

namespace {

struct CliqueLds {
  uint64_t* rows;   // [W][dmax] (word-major) when in LDS
  uint64_t* stk;    // [(k+1)][W] candidate bitsets per traversal size
  int64_t* start;   // [dmax] DAG offset of N+(nbr[i])
  int* nbr;         // [dmax] N+(root)
  int* offs;        // [dmax+1] exclusive prefix of |N+(nbr[i])|
  int* cur;         // [kMaxK+2] chosen position per depth
  int* hiv;         // [kMaxK+2] iteration end per depth
  uint64_t* lr;     // [64] rows of a candidate set of <= 64 members, in local ids
  int* pos;         // [64] positions (in N+(root)) of those members
};

__device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }

__device__ CliqueLds carve(unsigned char* smem, int dmax, int W, int k, bool rows_lds) {
  CliqueLds L;
  size_t off = 0;
  L.rows = reinterpret_cast<uint64_t*>(smem);
  if (rows_lds) off += static_cast<size_t>(W) * dmax * 8;
  off = align16(off);
  L.stk = reinterpret_cast<uint64_t*>(smem + off);
  off += static_cast<size_t>(k + 1) * W * 8;
  off = align16(off);
  L.start = reinterpret_cast<int64_t*>(smem + off);
  off += static_cast<size_t>(dmax) * 8;
  off = align16(off);
  L.nbr = reinterpret_cast<int*>(smem + off);
  off += static_cast<size_t>(dmax) * 4;
  off = align16(off);
  L.offs = reinterpret_cast<int*>(smem + off);
  off += static_cast<size_t>(dmax + 1) * 4;
  off = align16(off);
  L.cur = reinterpret_cast<int*>(smem + off);
  off += (kMaxK + 2) * 4;
  L.hiv = reinterpret_cast<int*>(smem + off);
  off += (kMaxK + 2) * 4;
  off = align16(off);
  L.lr = reinterpret_cast<uint64_t*>(smem + off);
  off += 64 * 8;
  L.pos = reinterpret_cast<int*>(smem + off);
  return L;
}

// ---------------------------------------------------------------- small dense solver
//
// Once a candidate set has at most 64 members, the remaining q levels of the
// enumeration tree are counted inside registers: members get local ids
// 0..m-1 (rank order), row lr[i] holds the members adjacent to member i with
// a larger id, and a q-clique count is a nested loop of AND + popcount.  The
// wave walks the first member i; lane j takes the second member j in
// C & lr[i] and counts the (q-2)-cliques of C & lr[i] & lr[j] on its own.

constexpr int kSolverMaxQ = 8;

template <int D>
__device__ __forceinline__ uint64_t count_in(uint64_t C, const uint64_t* lr) {
  if constexpr (D == 1) {
    return static_cast<uint64_t>(__popcll(C));
  } else {
    uint64_t s = 0;
    while (C) {
      const int x = __builtin_ctzll(C);
      C &= C - 1;
      s += count_in<D - 1>(C & lr[x], lr);
    }
    return s;
  }
}

__device__ __forceinline__ uint64_t count_in_depth(int D, uint64_t C, const uint64_t* lr) {
  switch (D) {
    case 1: return count_in<1>(C, lr);
    case 2: return count_in<2>(C, lr);
    case 3: return count_in<3>(C, lr);
    case 4: return count_in<4>(C, lr);
    case 5: return count_in<5>(C, lr);
    case 6: return count_in<6>(C, lr);
    default: return 0;
  }
}

__device__ __forceinline__ uint64_t range_mask64(int lo, int hi) {
  if (lo < 0) lo = 0;
  if (hi > 64) hi = 64;
  if (lo >= hi) return 0ull;
  const uint64_t upper = hi == 64 ? ~0ull : ((1ull << hi) - 1);
  return upper & (~0ull << lo);
}

// q-cliques (1 <= q <= kSolverMaxQ) inside C whose first member lies in
// [lo, hi); returns this lane's share.
__device__ __forceinline__ uint64_t small_solve(uint64_t C, int q, const uint64_t* lr, int lo, int hi) {
  const int lane = lane_id();
  C = uniu64(C);
  uint64_t first = C & range_mask64(lo, hi);
  uint64_t add = 0;
  if (q == 1) {
    if (lane == 0) add = static_cast<uint64_t>(__popcll(first));
  } else if (q == 2) {
    if ((first >> lane) & 1ull) add = static_cast<uint64_t>(__popcll(C & lr[lane]));
  } else {
    while (first) {
      const int i = __builtin_ctzll(first);
      first &= first - 1;
      const uint64_t Ci = uniu64(C & lr[i]);
      if ((Ci >> lane) & 1ull) add += count_in_depth(q - 2, Ci & lr[lane], lr);
    }
  }
  return add;
}

// Local ids for the members of the multi-word set C: positions into L.pos,
// rows into L.lr.  Returns the member count (<= 64 by the caller's check).
__device__ __forceinline__ int reindex(const uint64_t* C, int Wd, const uint64_t* rows, int dmax, const CliqueLds& L) {
  const int lane = lane_id();
  int base = 0;
  for (int w = 0; w < Wd; ++w) {
    const bool bit = (C[w] >> lane) & 1ull;
    const uint64_t b = ballot(bit);
    if (bit && base + mbcnt(b) < 64) L.pos[base + mbcnt(b)] = w * 64 + lane;
    base += __popcll(b);
  }
  const int m = uni(base < 64 ? base : 64);
  wave_sync();
  if (lane < m) {
    const int pa = L.pos[lane];
    uint64_t row = 0;
    for (int b = lane + 1; b < m; ++b) {
      const int pb = L.pos[b];
      if ((rows[static_cast<size_t>(pb >> 6) * dmax + pa] >> (pb & 63)) & 1ull) row |= 1ull << b;
    }
    L.lr[lane] = row;
  }
  wave_sync();
  return m;
}

// smallest set bit of C within [from, to), or -1 (wave-uniform)
__device__ __forceinline__ int next_bit(const uint64_t* C, int from, int to) {
  if (from >= to) return -1;
  const int w0 = from >> 6, w1 = (to - 1) >> 6;
  for (int w = w0; w <= w1; ++w) {
    uint64_t x = C[w];
    if (w == w0) x &= ~0ull << (from & 63);
    if (w == w1 && (to & 63)) x &= (1ull << (to & 63)) - 1;
    if (x) return uni(w * 64 + __builtin_ctzll(x));
  }
  return -1;
}

// number of set bits of C within [from, to)
__device__ __forceinline__ int count_bits(const uint64_t* C, int from, int to) {
  if (from >= to) return 0;
  const int w0 = from >> 6, w1 = (to - 1) >> 6;
  int c = 0;
  for (int w = w0; w <= w1; ++w) {
    uint64_t x = C[w];
    if (w == w0) x &= ~0ull << (from & 63);
    if (w == w1 && (to & 63)) x &= (1ull << (to & 63)) - 1;
    c += __popcll(x);
  }
  return uni(c);
}

// position of the j-th (1-based) set bit of C within [from, to)
__device__ __forceinline__ int select_bit(const uint64_t* C, int from, int to, int j) {
  const int w0 = from >> 6, w1 = (to - 1) >> 6;
  for (int w = w0; w <= w1; ++w) {
    uint64_t x = C[w];
    if (w == w0) x &= ~0ull << (from & 63);
    if (w == w1 && (to & 63)) x &= (1ull << (to & 63)) - 1;
    int c = __popcll(x);
    if (j <= c) {
      for (int q = 1; q < j; ++q) x &= x - 1;
      return uni(w * 64 + __builtin_ctzll(x));
    }
    j -= c;
  }
  return -1;
}

struct WaveAcc {
  uint64_t acc;    // per-lane leaves of the current graph
  int cur_g;
  int ovf;
  uint64_t nodes;  // wave stats (uniform)
  uint64_t tasks;
};

__device__ __forceinline__ void flush_graph(const CliqueArgs& A, WaveAcc& W) {
  uint64_t s = wave_sum_u64(W.acc, &W.ovf);
  if (lane_id() == 0 && W.cur_g >= 0) add_counter(A.out + W.cur_g, s, A.flags);
  W.acc = 0;
}

template <bool ROWS_LDS>
__device__ void run_task(const CliqueArgs& A, const CliqueLds& L, uint64_t* rows, const Task& t,
                         WaveAcc& WA, int wave_gid) {
  const int lane = lane_id();
  const int k = A.k, dmax = A.dmax, W = A.W;
  const int v = t.root;
  const int g = A.root_graph ? A.root_graph[v] : 0;
  if (g != WA.cur_g) {
    flush_graph(A, WA);
    WA.cur_g = g;
  }
  const int64_t base = A.rp[v];
  const int d = static_cast<int>(A.rp[v + 1] - base);
  const int hi_t = t.hi < d ? t.hi : d;
  uint64_t nodes_l = 0, leaves_l = 0, reads_l = 0;  // per-lane partial stats
  if (t.full_root && lane == 0) {
    nodes_l += (k >= 2) ? 1 : 0;
    reads_l += (k >= 2) ? static_cast<uint64_t>(d) : 0;
  }
  if (k == 1) {
    if (t.full_root && lane == 0) { WA.acc += 1; leaves_l += 1; }
  } else if (k == 2) {
    if (lane == 0 && hi_t > t.lo) {
      uint64_t c = static_cast<uint64_t>(hi_t - t.lo);
      WA.acc += c;
      leaves_l += c;
    }
  } else if (d > 0 && (!A.prune || d >= k - 1) && hi_t > t.lo) {
    // ---- load N+(v), out-degree prefix of its members (Extend, coalesced)
    int running = 0;
    for (int c = 0; c < d; c += kWave) {
      const int i = c + lane;
      int od = 0;
      if (i < d) {
        const int u = A.col[base + i];
        L.nbr[i] = u;
        const int64_t s = A.rp[u];
        od = static_cast<int>(A.rp[u + 1] - s);
        L.start[i] = s;
      }
      int incl = od;
#pragma unroll
      for (int sh = 1; sh < kWave; sh <<= 1) {
        int y = __shfl_up(incl, sh, kWave);
        if (lane >= sh) incl += y;
      }
      if (i < d) L.offs[i] = running + incl - od;
      running += read_lane(incl, kWave - 1);
    }
    running = uni(running);
    if (lane == 0) L.offs[d] = running;
    const int Wd = (d + 63) >> 6;
    for (int idx = lane; idx < Wd * d; idx += kWave) {
      const int w = idx / d, p = idx - w * d;
      rows[static_cast<size_t>(w) * dmax + p] = 0ull;
    }
    wave_sync();
    // ---- adjacency of N+(v) restricted to itself, as bitmap rows
    for (int tt = lane; tt < running; tt += kWave) {
      int lo = 0, hi = d;  // i = last index with offs[i] <= tt
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L.offs[mid] <= tt) lo = mid; else hi = mid;
      }
      const int i = lo;
      const int e = A.col[L.start[i] + (tt - L.offs[i])];
      int a = i + 1, b = d;  // e > nbr[i], so search above i
      while (a < b) {
        const int mid = (a + b) >> 1;
        if (L.nbr[mid] < e) a = mid + 1; else b = mid;
      }
      if (a < d && L.nbr[a] == e) atomicOr(reinterpret_cast<unsigned long long*>(&rows[static_cast<size_t>(a >> 6) * dmax + i]), 1ull << (a & 63));
    }
    // ---- level-1 candidate set and the task prefix
    for (int w = lane; w < Wd; w += kWave) {
      const int rem = d - w * 64;
      L.stk[1 * W + w] = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
    }
    wave_sync();
    for (int s = 1; s < t.depth; ++s) {
      const int p = L.cur[s];
      for (int w = lane; w < Wd; w += kWave) L.stk[(s + 1) * W + w] = L.stk[s * W + w] & rows[static_cast<size_t>(w) * dmax + p];
      wave_sync();
    }
    // one-word roots: their rows already are local rows
    const bool solver = A.prune != 0;
    if (solver && Wd == 1) {
      if (lane < d) L.lr[lane] = rows[lane];
      wave_sync();
    }
    auto add_acc = [&](uint64_t x) {
      const uint64_t before = WA.acc;
      WA.acc += x;
      if (WA.acc < before) WA.ovf = 1;
    };

    // leaf-parent step: traversal of size s = k-2 with candidate set C_s;
    // each lane takes extensions p (one per word) inside [lo, hi).
    auto leaf_parent = [&](int s, int lo, int hi) {
      const uint64_t* C = L.stk + s * W;
      for (int w0 = 0; w0 < Wd; ++w0) {
        const int p = w0 * 64 + lane;
        const bool on = p >= lo && p < hi && p < d && ((C[w0] >> lane) & 1ull);
        if (on) {
          uint64_t pc = 0;
          for (int w = w0; w < Wd; ++w) pc += static_cast<uint64_t>(__popcll(C[w] & rows[static_cast<size_t>(w) * dmax + p]));
          const uint64_t before = WA.acc;
          WA.acc += pc;
          if (WA.acc < before) WA.ovf = 1;
          nodes_l += 1;
          reads_l += static_cast<uint64_t>(L.offs[p + 1] - L.offs[p]);
          leaves_l += pc;
        }
      }
    };

    const int s0 = t.depth;
    if (solver && Wd == 1 && k - s0 <= kSolverMaxQ) {
      add_acc(small_solve(L.stk[s0 * W], k - s0, L.lr, t.lo, hi_t));
    } else if (s0 == k - 2) {
      leaf_parent(s0, t.lo, hi_t);
    } else {
      int depth = s0;
      if (lane == 0) { L.cur[depth] = t.lo - 1; L.hiv[depth] = hi_t; }
      wave_sync();
      int steps = 0;
      for (;;) {
        const int u = next_bit(L.stk + depth * W, L.cur[depth] + 1, L.hiv[depth]);
        if (u < 0) {
          if (depth == s0) break;
          --depth;
          continue;
        }
        if (lane == 0) {
          L.cur[depth] = u;
          nodes_l += 1;
          reads_l += static_cast<uint64_t>(L.offs[u + 1] - L.offs[u]);
        }
        int cnt = 0;
        for (int w = lane; w < Wd; w += kWave) {
          const uint64_t x = L.stk[depth * W + w] & rows[static_cast<size_t>(w) * dmax + u];
          L.stk[(depth + 1) * W + w] = x;
          cnt += __popcll(x);
        }
        cnt = uni(wave_sum_i32(cnt));
        wave_sync();
        const int q = k - depth - 1;  // vertices still to add below the child
        if (!A.prune || cnt >= q) {
          if (solver && cnt <= 64 && q <= kSolverMaxQ) {
            if (Wd == 1) {
              add_acc(small_solve(L.stk[(depth + 1) * W], q, L.lr, 0, 64));
            } else {
              const int m = reindex(L.stk + (depth + 1) * W, Wd, rows, dmax, L);
              add_acc(small_solve(m == 64 ? ~0ull : ((1ull << m) - 1), q, L.lr, 0, 64));
            }
          } else if (depth + 1 == k - 2) {
            leaf_parent(depth + 1, 0, d);
          } else {
            ++depth;
            if (lane == 0) { L.cur[depth] = -1; L.hiv[depth] = d; }
            wave_sync();
          }
        }
        // ---- donation (Section IV-D redistribute, done by the busy wave)
        if (A.S.donate && (++steps % A.S.period) == 0 && sched_want_donation(A.S)) {
          for (int s = s0; s <= depth; ++s) {
            const int from = L.cur[s] + 1, to = L.hiv[s];
            const int c = count_bits(L.stk + s * W, from, to);
            if (c >= 2) {
              const int keep = c - c / 2;
              const int mid = select_bit(L.stk + s * W, from, to, keep + 1);
              const int pay = task_payload(v, t.stat, s, mid, to, L.cur);
              if (sched_publish(A.S, pay, wave_gid)) {
                if (lane == 0) L.hiv[s] = mid;
              }
              wave_sync();
              break;
            }
          }
        }
      }
    }
  }
  WA.nodes += static_cast<uint64_t>(wave_sum_i32(static_cast<int>(nodes_l)));
  if (A.root_stats) {
    int o = 0;
    const uint64_t n_ = wave_sum_u64(nodes_l, &o);
    const uint64_t l_ = wave_sum_u64(leaves_l, &o);
    const uint64_t r_ = wave_sum_u64(reads_l, &o);
    if (lane == 0) {
      unsigned long long* rs = A.root_stats + static_cast<size_t>(t.stat) * 3;
      add_counter(rs + 0, n_, A.flags);
      add_counter(rs + 1, l_, A.flags);
      add_counter(rs + 2, r_, A.flags);
      if (o) atomicOr(A.flags, 1);
    }
  }
}

template <bool ROWS_LDS>
__global__ void __launch_bounds__(64) clique_kernel(CliqueArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int wave_gid = blockIdx.x;
  CliqueLds L = carve(smem, A.dmax, A.W, A.k, ROWS_LDS);
  uint64_t* rows = ROWS_LDS ? L.rows : reinterpret_cast<uint64_t*>(A.rows_global) + static_cast<size_t>(wave_gid) * A.W * A.dmax;
  WaveAcc WA;
  WA.acc = 0;
  WA.cur_g = -1;
  WA.ovf = 0;
  WA.nodes = 0;
  WA.tasks = 0;
  const uint64_t t_begin = wall_clock64();
  uint64_t t_idle = 0;
  if (lane == 0) add_u64(A.S.state, kActiveOne);
  int64_t b, e;
  while (sched_grab(A.S, &b, &e)) {
    for (int64_t q = b; q < e; ++q) {
      Task t = sched_entry(A.S, q, INT_MAX);
      run_task<ROWS_LDS>(A, L, rows, t, WA, wave_gid);
      WA.tasks++;
    }
  }
  if (lane == 0) {
    add_i32(A.S.idle, 1);
    add_u64(A.S.state, 0ull - kActiveOne);
  }
  if (A.S.donate) {
    uint64_t t0 = wall_clock64();
    for (;;) {
      unsigned long long st = 0;
      if (lane == 0) st = ld_relaxed_u64(A.S.state);
      st = uniu64(st);
      if (st == 0) break;
      int data = 0;
      if ((st & 0xffffffffull) != 0 && sched_take(A.S, &data, wave_gid)) {
        t_idle += wall_clock64() - t0;
        if (lane == 0) add_i32(A.S.idle, -1);
        Task t = task_unpack(data, L.cur);
        run_task<ROWS_LDS>(A, L, rows, t, WA, wave_gid);
        WA.tasks++;
        if (lane == 0) {
          add_i32(A.S.idle, 1);
          add_u64(A.S.state, 0ull - kActiveOne);
        }
        t0 = wall_clock64();
        continue;
      }
      __builtin_amdgcn_s_sleep(16);
    }
    t_idle += wall_clock64() - t0;
  }
  if (lane == 0) add_i32(A.S.idle, -1);
  flush_graph(A, WA);
  if (lane == 0 && WA.ovf) atomicOr(A.flags, 1);
  if (A.wave_stats && wave_gid < A.wave_stats_len && lane == 0) {
    const uint64_t total = wall_clock64() - t_begin;
    unsigned long long* ws = A.wave_stats + static_cast<size_t>(wave_gid) * 4;
    ws[0] = total - t_idle;
    ws[1] = t_idle;
    ws[2] = WA.nodes;
    ws[3] = WA.tasks;
  }
}

}  // namespace

size_t clique_lds_bytes(int dmax, int W, int k, bool rows_in_lds) {
  auto a16 = [](size_t x) { return (x + 15) & ~static_cast<size_t>(15); };
  size_t off = rows_in_lds ? static_cast<size_t>(W) * dmax * 8 : 0;
  off = a16(off) + static_cast<size_t>(k + 1) * W * 8;
  off = a16(off) + static_cast<size_t>(dmax) * 8;
  off = a16(off) + static_cast<size_t>(dmax) * 4;
  off = a16(off) + static_cast<size_t>(dmax + 1) * 4;
  off = a16(off) + 2 * (kMaxK + 2) * 4;
  off = a16(off) + 64 * 8 + 64 * 4;
  return a16(off);
}

hipError_t clique_occupancy(bool rows_in_lds, size_t lds_bytes, int* blocks_per_cu) {
  if (rows_in_lds)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, clique_kernel<true>, 64, lds_bytes);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, clique_kernel<false>, 64, lds_bytes);
}

hipError_t launch_clique(const CliqueArgs& a, int grid, bool rows_in_lds, size_t lds_bytes, hipStream_t s) {
  if (rows_in_lds)
    hipLaunchKernelGGL(clique_kernel<true>, dim3(grid), dim3(64), lds_bytes, s, a);
  else
    hipLaunchKernelGGL(clique_kernel<false>, dim3(grid), dim3(64), lds_bytes, s, a);
  return hipGetLastError();
}

}  // namespace dm

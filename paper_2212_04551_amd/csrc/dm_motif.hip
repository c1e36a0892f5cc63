// Persistent DFS-wide induced k-motif counting kernel for gfx950 (wave64).
//
// Method (DuMato, arXiv 2212.04551):
//   - Motif counting (Section IV-E, Alg. 4 right): extensions come from the
//     adjacency of every traversal vertex; a canonicality filter keeps one
//     traversal order per vertex set; at |tr| = k-1 every k-traversal is mapped
//     to its pattern through the canonical-relabeling dictionary and counted
//     (aggregate_pattern, Section IV-C).
//   - Induced edges are carried along the traversal (Move with genedges,
//     Section IV-B, Alg. 1, the `induce` step) as the bitmap of Section IV-C:
//     vertex v_i (i >= 2) stores its edges to v_0..v_{i-1}.
//
// gfx950 realisation:
//   - One wave owns one traversal stack.  Level s of the stack holds
//     N(tr) \ tr for the traversal tr = v_0..v_{s-1} as a list sorted by vertex
//     id, with one mask byte per entry: bit t = adjacent to v_t.  The mask makes
//     `induce` free (the new vertex's bitmap field is its mask) and turns the
//     canonical filter into an O(1) test.
//   - Vertices are renamed by (degree, id) rank before the kernel runs, so
//     "smaller" below means lower rank and each subgraph is rooted at its
//     lowest-degree vertex (a cost that depends on graph structure, not on
//     arbitrary labels, which is what the learned ordering predicts).
//   - Canonical filter (the paper names Arabesque's rule without stating it;
//     reading used here): a traversal is canonical iff v_0 is its smallest
//     vertex and each later vertex is the smallest vertex adjacent to the
//     prefix before it.  Appending w whose first neighbour in tr is v_f is
//     canonical iff w > v_0 and w > v_t for every t > f.  A failed entry can
//     never become canonical again, but it stays in the list so membership
//     tests stay exact.
//   - Extend (Alg. 2) for a chosen x: each lane takes one neighbour of x
//     (coalesced read) and binary-searches it in the level list: found entries
//     get bit s; the rest are new and are compacted with ballot/mbcnt
//     (Compact); then a wave-parallel merge writes level s+1.
//   - The last two levels are fused: for a traversal of size k-2 and each
//     canonical extension x, the leaves tr+x+y are the canonical entries y > x
//     of the same list (their mask gains bit k-2 when y ~ x) plus the new
//     neighbours of x above v_0.  Leaves are histogrammed by mask inside the
//     wave (ballot match loop), and each non-empty mask bin is relabelled once
//     through the dictionary into per-wave LDS class counters.
#include <climits>

#include "dm_internal.hpp"

namespace dm {

namespace {

constexpr int kMotifMaxK = 7;
constexpr int kSuf = kMotifMaxK + 1;

struct MotifLds {
  unsigned long long* cnt;  // [ncls] class counters of the current graph
  unsigned* hist;           // [2^(k-1)] leaf masks
  int* tr;                  // [kSuf] traversal
  int* code;                // [kSuf] dictionary code per traversal size
  int* sufmax;              // [kSuf][kSuf] max of tr[f+1..s-1] per size s
  int* cursor;              // [kSuf]
  int* endv;                // [kSuf]
  int* esize;               // [kSuf]
  int* misc;                // [4]
};

__device__ __forceinline__ int off_of(int i) { return i * (i - 1) / 2 - 1; }  // bitmap field of v_i, i >= 2

__device__ MotifLds carve(unsigned char* smem, int ncls, int k) {
  MotifLds L;
  size_t off = 0;
  L.cnt = reinterpret_cast<unsigned long long*>(smem);
  off += static_cast<size_t>(ncls) * 8;
  L.hist = reinterpret_cast<unsigned*>(smem + off);
  off += static_cast<size_t>(1 << (k - 1)) * 4;
  L.tr = reinterpret_cast<int*>(smem + off);
  off += kSuf * 4;
  L.code = reinterpret_cast<int*>(smem + off);
  off += kSuf * 4;
  L.sufmax = reinterpret_cast<int*>(smem + off);
  off += kSuf * kSuf * 4;
  L.cursor = reinterpret_cast<int*>(smem + off);
  off += kSuf * 4;
  L.endv = reinterpret_cast<int*>(smem + off);
  off += kSuf * 4;
  L.esize = reinterpret_cast<int*>(smem + off);
  off += kSuf * 4;
  L.misc = reinterpret_cast<int*>(smem + off);
  return L;
}

__device__ __forceinline__ int lower_bound_g(const int32_t* a, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

struct MotifWave {
  int cur_g;
  int ovf;
  uint64_t nodes, tasks;
  int32_t* vert;  // this wave's extension region
  uint8_t* mask;
  int32_t* nbuf;
};

__device__ __forceinline__ void flush_counts(const MotifArgs& A, const MotifLds& L, MotifWave& MW) {
  const int lane = lane_id();
  wave_sync();
  for (int c = lane; c < A.ncls; c += kWave) {
    const unsigned long long v = L.cnt[c];
    if (MW.cur_g >= 0) add_counter(A.out + static_cast<size_t>(MW.cur_g) * A.ncls + c, v, A.flags);
    L.cnt[c] = 0;
  }
  wave_sync();
}

// canonical at traversal size s?  (mask bits over positions 0..s-1)
__device__ __forceinline__ bool canonical(const MotifLds& L, int s, int y, unsigned m) {
  const unsigned low = m & ((1u << s) - 1u);
  if (low == 0) return false;
  const int f = __builtin_ctz(low);
  return y > L.tr[0] && y > L.sufmax[s * kSuf + f];
}

__device__ __forceinline__ bool in_tr(const MotifLds& L, int s, int w) {
  bool r = false;
  for (int t = 0; t < s; ++t) r |= (L.tr[t] == w);
  return r;
}

// Build level s+1 from level s by appending the entry at index px (vertex x).
__device__ void extend_level(const MotifArgs& A, const MotifLds& L, MotifWave& MW, int s, int px, int x) {
  const int lane = lane_id();
  int32_t* Ev = MW.vert + A.level_off[s];
  uint8_t* Em = MW.mask + A.level_off[s];
  int32_t* Nv = MW.vert + A.level_off[s + 1];
  uint8_t* Nm = MW.mask + A.level_off[s + 1];
  const int ns = L.esize[s];
  const int64_t cap = A.level_cap[s + 1];
  const int64_t xb = A.rp[x];
  const int dx = static_cast<int>(A.rp[x + 1] - xb);
  int nn = 0;
  for (int c = 0; c < dx; c += kWave) {
    const int i = c + lane;
    const bool ok = i < dx;
    const int w = ok ? A.col[xb + i] : 0;
    int j = ok ? lower_bound_g(Ev, ns, w) : ns;
    const bool found = ok && j < ns && Ev[j] == w;
    if (found && j != px) Em[j] = static_cast<uint8_t>(Em[j] | 0x80u);
    const bool isnew = ok && !found && !in_tr(L, s, w);
    const uint64_t b = ballot(isnew);
    if (isnew) {
      const int pos = nn + mbcnt(b);
      if (pos < A.dmax) MW.nbuf[pos] = w;
    }
    nn += __popcll(b);
  }
  nn = uni(nn);
  if (nn > A.dmax) {
    if (lane == 0) atomicOr(A.flags + 1, 1);
    nn = A.dmax;
  }
  wave_sync();
  // merge the surviving old entries and the new ones (both sorted by id)
  for (int j = lane; j < ns; j += kWave) {
    if (j == px) continue;
    const int y = Ev[j];
    const unsigned m = Em[j];
    const int r = lower_bound_g(MW.nbuf, nn, y);
    const int64_t out = static_cast<int64_t>(j) - (j > px ? 1 : 0) + r;
    if (out < cap) {
      Nv[out] = y;
      Nm[out] = static_cast<uint8_t>((m & 0x7fu) | ((m & 0x80u) ? (1u << s) : 0u));
    }
    if (m & 0x80u) Em[j] = static_cast<uint8_t>(m & 0x7fu);
  }
  for (int i = lane; i < nn; i += kWave) {
    const int w = MW.nbuf[i];
    int r = lower_bound_g(Ev, ns, w);
    if (px < r) r -= 1;
    const int64_t out = static_cast<int64_t>(i) + r;
    if (out < cap) {
      Nv[out] = w;
      Nm[out] = static_cast<uint8_t>(1u << s);
    }
  }
  int64_t nsz = static_cast<int64_t>(ns) - 1 + nn;
  if (nsz > cap) {
    if (lane == 0) atomicOr(A.flags + 1, 1);
    nsz = cap;
  }
  const unsigned mx = Em[px] & ((1u << s) - 1u);
  if (lane == 0) {
    L.esize[s + 1] = static_cast<int>(nsz);
    L.tr[s] = x;
    L.code[s + 1] = L.code[s] | (s >= 2 ? static_cast<int>(mx << off_of(s)) : 0);
    for (int f = 0; f < s; ++f) {
      const int a = L.sufmax[s * kSuf + f];
      L.sufmax[(s + 1) * kSuf + f] = a > x ? a : x;
    }
    L.sufmax[(s + 1) * kSuf + s] = -1;
  }
  wave_sync();
}

// Count the leaves below tr + x, where |tr| = s = k-2 and x is entry px.
__device__ void leaf_count(const MotifArgs& A, const MotifLds& L, MotifWave& MW, int s, int px, int x,
                           uint64_t& leaves_l) {
  const int lane = lane_id();
  const int k = A.k;
  int32_t* Ev = MW.vert + A.level_off[s];
  uint8_t* Em = MW.mask + A.level_off[s];
  const int ns = L.esize[s];
  const int nb = 1 << (k - 1);
  for (int m = lane; m < nb; m += kWave) L.hist[m] = 0;
  const int v0 = L.tr[0];
  const int64_t xb = A.rp[x];
  const int dx = static_cast<int>(A.rp[x + 1] - xb);
  int newcnt = 0;
  for (int c = 0; c < dx; c += kWave) {
    const int i = c + lane;
    const bool ok = i < dx;
    const int w = ok ? A.col[xb + i] : 0;
    const int j = ok ? lower_bound_g(Ev, ns, w) : ns;
    const bool found = ok && j < ns && Ev[j] == w;
    if (found && j > px) Em[j] = static_cast<uint8_t>(Em[j] | 0x80u);
    const bool isnew = ok && !found && w > v0 && !in_tr(L, s, w);
    newcnt += __popcll(ballot(isnew));
  }
  wave_sync();
  const unsigned low = (1u << s) - 1u;
  for (int c = px + 1; c < ns; c += kWave) {
    const int j = c + lane;
    const bool in = j < ns;
    const unsigned m = in ? Em[j] : 0u;
    const int y = in ? Ev[j] : 0;
    if (m & 0x80u) Em[j] = static_cast<uint8_t>(m & 0x7fu);
    const bool valid = in && canonical(L, s, y, m);
    const unsigned lm = (m & low) | ((m & 0x80u) ? (1u << s) : 0u);
    uint64_t act = ballot(valid);
    while (act) {
      const int l = __ffsll(static_cast<long long>(act)) - 1;
      const unsigned key = static_cast<unsigned>(read_lane(static_cast<int>(lm), l));
      const uint64_t same = ballot(valid && lm == key);
      if (lane == 0) L.hist[key] += static_cast<unsigned>(__popcll(same));
      act &= ~same;
    }
  }
  if (lane == 0) L.hist[1u << s] += static_cast<unsigned>(newcnt);
  wave_sync();
  const unsigned mx = Em[px] & low;
  const int codex = L.code[s] | (s >= 2 ? static_cast<int>(mx << off_of(s)) : 0);
  const int offl = off_of(k - 1);
  for (int m = lane; m < nb; m += kWave) {
    const unsigned h = L.hist[m];
    if (h) {
      const int cls = A.table[codex | (m << offl)];
      if (cls == 0xFF) {
        atomicOr(A.flags + 1, 2);
      } else {
        const unsigned long long old = atomicAdd(&L.cnt[cls], static_cast<unsigned long long>(h));
        if (old + h < old) MW.ovf = 1;
      }
      leaves_l += h;
    }
  }
  wave_sync();
}

// index of the first canonical entry of level s in [from, to), or -1
__device__ __forceinline__ int next_canonical(const MotifArgs& A, const MotifLds& L, const MotifWave& MW, int s,
                                              int from, int to) {
  const int lane = lane_id();
  const int32_t* Ev = MW.vert + A.level_off[s];
  const uint8_t* Em = MW.mask + A.level_off[s];
  for (int c = from; c < to; c += kWave) {
    const int j = c + lane;
    const bool valid = j < to && canonical(L, s, Ev[j], Em[j]);
    const uint64_t b = ballot(valid);
    if (b) return uni(c + __ffsll(static_cast<long long>(b)) - 1);
  }
  return -1;
}

__device__ void run_task(const MotifArgs& A, const MotifLds& L, MotifWave& MW, const Task& t, int wave_gid) {
  const int lane = lane_id();
  const int k = A.k;
  const int v0 = t.root;
  const int g = A.root_graph ? A.root_graph[v0] : 0;
  if (g != MW.cur_g) {
    flush_counts(A, L, MW);
    MW.cur_g = g;
  }
  uint64_t nodes_l = 0, leaves_l = 0, reads_l = 0;
  // ---- level 1: N(v0), every entry adjacent to v_0
  const int64_t b0 = A.rp[v0];
  const int d0 = static_cast<int>(A.rp[v0 + 1] - b0);
  {
    int32_t* E1 = MW.vert + A.level_off[1];
    uint8_t* M1 = MW.mask + A.level_off[1];
    for (int i = lane; i < d0; i += kWave) {
      E1[i] = A.col[b0 + i];
      M1[i] = 1;
    }
    if (lane == 0) {
      L.esize[1] = d0;
      L.tr[0] = v0;
      L.code[1] = 0;
      L.sufmax[1 * kSuf + 0] = -1;
    }
  }
  if (t.full_root && lane == 0) {
    nodes_l += 1;
    reads_l += static_cast<uint64_t>(d0);
  }
  wave_sync();
  // ---- replay the task prefix (vertex ids in tr[1..depth-1])
  for (int s = 1; s < t.depth; ++s) {
    const int x = L.tr[s];
    const int ns = L.esize[s];
    const int px = uni(lower_bound_g(MW.vert + A.level_off[s], ns, x));
    if (px >= ns || MW.vert[A.level_off[s] + px] != x) {  // a prefix that is not in the list: corrupt task
      if (lane == 0) atomicOr(A.flags + 1, 4);
      return;
    }
    extend_level(A, L, MW, s, px, x);
  }
  const int s0 = t.depth;
  const int hi0 = t.hi < L.esize[s0] ? t.hi : L.esize[s0];

  auto leaf_parent = [&](int s, int from, int to) {
    int c = from;
    while (true) {
      const int idx = next_canonical(A, L, MW, s, c, to);
      if (idx < 0) break;
      const int x = MW.vert[A.level_off[s] + idx];
      if (lane == 0) {
        nodes_l += 1;
        reads_l += static_cast<uint64_t>(A.rp[x + 1] - A.rp[x]);
      }
      leaf_count(A, L, MW, s, idx, x, leaves_l);
      c = idx + 1;
    }
  };

  if (s0 == k - 2) {
    leaf_parent(s0, t.lo, hi0);
  } else if (hi0 > t.lo) {
    int s = s0;
    if (lane == 0) { L.cursor[s] = t.lo; L.endv[s] = hi0; }
    wave_sync();
    int steps = 0;
    for (;;) {
      const int idx = next_canonical(A, L, MW, s, L.cursor[s], L.endv[s]);
      if (idx < 0) {
        if (s == s0) break;
        --s;
        continue;
      }
      const int x = MW.vert[A.level_off[s] + idx];
      if (lane == 0) {
        L.cursor[s] = idx + 1;
        nodes_l += 1;
        reads_l += static_cast<uint64_t>(A.rp[x + 1] - A.rp[x]);
      }
      extend_level(A, L, MW, s, idx, x);
      if (s + 1 == k - 2) {
        leaf_parent(s + 1, 0, L.esize[s + 1]);
      } else {
        ++s;
        if (lane == 0) { L.cursor[s] = 0; L.endv[s] = L.esize[s]; }
        wave_sync();
      }
      // ---- donation of untried extensions at the shallowest level
      if (A.S.donate && (++steps % A.S.period) == 0 && sched_want_donation(A.S)) {
        for (int q = s0; q <= s; ++q) {
          const int from = L.cursor[q], to = L.endv[q];
          if (to - from >= 2) {
            const int mid = from + (to - from + 1) / 2;
            const int pay = task_payload(v0, t.stat, q, mid, to, L.tr);
            if (sched_publish(A.S, pay, wave_gid)) {
              if (lane == 0) L.endv[q] = mid;
            }
            wave_sync();
            break;
          }
        }
      }
    }
  }
  MW.nodes += static_cast<uint64_t>(wave_sum_i32(static_cast<int>(nodes_l)));
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

__global__ void __launch_bounds__(64) motif_kernel(MotifArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int wave_gid = blockIdx.x;
  MotifLds L = carve(smem, A.ncls, A.k);
  MotifWave MW;
  MW.cur_g = -1;
  MW.ovf = 0;
  MW.nodes = 0;
  MW.tasks = 0;
  MW.vert = A.ext_vert + static_cast<size_t>(wave_gid) * A.wave_ext_cap;
  MW.mask = A.ext_mask + static_cast<size_t>(wave_gid) * A.wave_ext_cap;
  MW.nbuf = A.new_buf + static_cast<size_t>(wave_gid) * A.dmax;
  for (int c = lane; c < A.ncls; c += kWave) L.cnt[c] = 0;
  wave_sync();
  const uint64_t t_begin = wall_clock64();
  uint64_t t_idle = 0;
  if (lane == 0) add_u64(A.S.state, kActiveOne);
  int64_t b, e;
  while (sched_grab(A.S, &b, &e)) {
    for (int64_t q = b; q < e; ++q) {
      Task t = sched_entry(A.S, q, INT_MAX);
      run_task(A, L, MW, t, wave_gid);
      MW.tasks++;
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
        Task t = task_unpack(data, L.tr);
        run_task(A, L, MW, t, wave_gid);
        MW.tasks++;
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
  flush_counts(A, L, MW);
  if (lane == 0 && MW.ovf) atomicOr(A.flags, 1);
  if (A.wave_stats && wave_gid < A.wave_stats_len && lane == 0) {
    const uint64_t total = wall_clock64() - t_begin;
    unsigned long long* ws = A.wave_stats + static_cast<size_t>(wave_gid) * 4;
    ws[0] = total - t_idle;
    ws[1] = t_idle;
    ws[2] = MW.nodes;
    ws[3] = MW.tasks;
  }
}

}  // namespace

size_t motif_lds_bytes(int k, int ncls) {
  size_t off = static_cast<size_t>(ncls) * 8 + static_cast<size_t>(1 << (k - 1)) * 4;
  off += kSuf * 4 * 2 + kSuf * kSuf * 4 + kSuf * 4 * 3 + 16;
  return (off + 15) & ~static_cast<size_t>(15);
}

hipError_t motif_occupancy(size_t lds_bytes, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, motif_kernel, 64, lds_bytes);
}

hipError_t launch_motif(const MotifArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(motif_kernel, dim3(grid), dim3(64), lds_bytes, s, a);
  return hipGetLastError();
}

}  // namespace dm

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
  uint64_t* rows;   // [2][kLocalMax] rows (word-major) of a root with <= kLocalMax out-neighbours
  uint64_t* stk;    // [(k+1)][W] candidate bitsets per traversal size
  int* nbr;         // [dmax] N+(root)
  int* offs;        // [dmax+1] exclusive prefix of |N+(nbr[i])|
  int* cur;         // [kMaxK+2] chosen position per depth
  int* hiv;         // [kMaxK+2] iteration end per depth
  uint64_t* lr;     // [2][128] re-indexed rows (word-major) of a set of <= 128 members
  uint64_t* cset;   // [4] the set handed to the dense solver
  int* pos;         // [128] positions (in N+(root)) of re-indexed members
  int* pst;         // [128] solver: first pair task of each member
};

__device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }

constexpr int kLocalMax = kCliqueLocalRows;  // roots with at most this many out-neighbours use their rows in place
constexpr int kReindexMax = 128;  // larger roots re-index candidate sets of at most this many members

__device__ CliqueLds carve(unsigned char* smem, int dmax, int W, int k) {
  CliqueLds L;
  size_t off = 0;
  L.rows = reinterpret_cast<uint64_t*>(smem);
  off += static_cast<size_t>(2) * kLocalMax * 8;
  off = align16(off);
  L.stk = reinterpret_cast<uint64_t*>(smem + off);
  off += static_cast<size_t>(k + 1) * W * 8;
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
  off += kReindexMax / 64 * kReindexMax * 8;
  L.cset = reinterpret_cast<uint64_t*>(smem + off);
  off += 4 * 8;
  L.pos = reinterpret_cast<int*>(smem + off);
  off += kReindexMax * 4;
  L.pst = reinterpret_cast<int*>(smem + off);
  return L;
}

// ---------------------------------------------------------------- small dense solver
//
// Once a candidate set is small (<= 128 members: in place for roots with <= 128
// out-neighbours, else after re-indexing), the remaining q
// levels of the enumeration tree are counted with per-lane bitset recursion:
// a member set is NW 64-bit words, row word q of member i sits at
// lr[q * stride + i] (word-major, so lanes reading consecutive members hit
// distinct banks), rows hold only members with a larger id, and a q-clique
// count is a nested loop of AND + popcount.  The wave walks the first member
// i; lane l takes the second member j = 64 w + l in C & row(i) and counts the
// (q-2)-cliques of C & row(i) & row(j) on its own.  Word loops are not
// unrolled around the recursion (code size stays linear in the depth); `pick`
// selects a word of a register array without dynamic register indexing.

constexpr int kSolverMaxQ = 8;
// A solver job donates part of itself only in the launch's tail (a quarter of
// the waves idle) and while at least this many pair tasks are untaken: the
// taker rebuilds the root's rows and the prefix first.
constexpr int kJobDonateMin = 1024;
// free lanes that trigger a refill of pair tasks in the lane solver
constexpr int kRefillMin = 8;

// rows the solver reads always live in LDS: an address-space-3 pointer makes
// every load a ds_read (no flat-address dispatch)
typedef __attribute__((address_space(3))) const uint64_t LdsU64;

__device__ __forceinline__ LdsU64* as_lds(const uint64_t* p) { return (LdsU64*)(p); }

template <int NW>
__device__ __forceinline__ uint64_t pick(const uint64_t (&c)[NW], int w) {
  uint64_t r = c[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) r = (w == q) ? c[q] : r;
  return r;
}

template <int D, int NW>
__device__ __forceinline__ uint64_t count_in(const uint64_t (&C)[NW], LdsU64* lr, int stride) {
  if constexpr (D == 1) {
    uint64_t s = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += static_cast<uint64_t>(__popcll(C[q]));
    return s;
  } else if constexpr (D == 2) {
    // edges inside C: two members per iteration, so two row reads are in
    // flight before their AND / popcount
    uint32_t s = 0;
    for (int w = 0; w < NW; ++w) {
      uint64_t x = pick<NW>(C, w);
      while (x) {
        const int a = w * 64 + __builtin_ctzll(x);
        x &= x - 1;
        const int b = x ? w * 64 + __builtin_ctzll(x) : a;
        const uint32_t two = x ? 1u : 0u;
        x &= x - 1;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
          const uint64_t ra = lr[q * stride + a];
          const uint64_t rb = lr[q * stride + b];
          s += static_cast<uint32_t>(__popcll(C[q] & ra)) + two * static_cast<uint32_t>(__popcll(C[q] & rb));
        }
      }
    }
    return s;
  } else {
    uint64_t s = 0;
    for (int w = 0; w < NW; ++w) {
      uint64_t x = pick<NW>(C, w);
      while (x) {
        const int id = w * 64 + __builtin_ctzll(x);
        x &= x - 1;
        uint64_t Cn[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) Cn[q] = C[q] & lr[q * stride + id];
        s += count_in<D - 1, NW>(Cn, lr, stride);
      }
    }
    return s;
  }
}

// Edges inside the set C (rows upper-triangular), one member per iteration: a
// lane's loop over its own set, so the per-iteration work is one row read, an
// AND and a popcount.  One-word sets are walked as two 32-bit halves: a member
// of the low half needs both halves of its row, one of the high half only the
// high half (its row has no lower members), and finding and clearing the next
// member are 32-bit operations (about a third fewer instructions per member).
template <int NW>
__device__ __forceinline__ uint32_t edge_count(const uint64_t (&C)[NW], LdsU64* lr, int stride) {
  if constexpr (NW == 1) {
    // (rows are read as whole 64-bit words: 32-bit reads of one half cost
    // more in LDS bank conflicts than they save)
    const uint32_t clo = static_cast<uint32_t>(C[0]), chi = static_cast<uint32_t>(C[0] >> 32);
    uint32_t s = 0;
    uint32_t x = clo;
    while (x) {
      const int i = __builtin_ctz(x);
      x &= x - 1;
      const uint64_t r = lr[i];
      s += static_cast<uint32_t>(__popc(clo & static_cast<uint32_t>(r)) + __popc(chi & static_cast<uint32_t>(r >> 32)));
    }
    x = chi;
    while (x) {
      const int i = 32 + __builtin_ctz(x);
      x &= x - 1;
      s += static_cast<uint32_t>(__popc(chi & static_cast<uint32_t>(lr[i] >> 32)));
    }
    return s;
  }
  uint32_t s = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    uint64_t x = pick<NW>(C, w);
    while (x) {
      const int i = w * 64 + __builtin_ctzll(x);
      x &= x - 1;
#pragma unroll
      for (int q = 0; q < NW; ++q) s += static_cast<uint32_t>(__popcll(C[q] & lr[q * stride + i]));
    }
  }
  return s;
}

__device__ __forceinline__ uint64_t range_mask64(int lo, int hi) {
  if (lo < 0) lo = 0;
  if (hi > 64) hi = 64;
  if (lo >= hi) return 0ull;
  const uint64_t upper = hi == 64 ? ~0ull : ((1ull << hi) - 1);
  return upper & (~0ull << lo);
}

typedef __attribute__((address_space(3))) int LdsI32;

// position of the r-th (0-based) set bit of the NW-word set x (r < popcount)
template <int NW>
__device__ __forceinline__ int select_nth(const uint64_t (&x)[NW], int r) {
  int base = 0;
  uint64_t v = x[0];
  if constexpr (NW == 2) {
    const int c0 = __popcll(x[0]);
    if (r >= c0) {
      r -= c0;
      v = x[1];
      base = 64;
    }
  }
  int pos = 0;
#pragma unroll
  for (int width = 32; width >= 1; width >>= 1) {
    const uint64_t m = (width == 32) ? 0xffffffffull : ((1ull << width) - 1);
    const int c = __popcll(v & m);
    if (r >= c) {
      r -= c;
      v >>= width;
      pos += width;
    }
  }
  return base + pos;
}

// Where a solver job sits in the search, so that part of it can be donated:
// the root, its stats row, the depth of the job's set (the prefix is in
// L.cur[1 .. depth-1]), the end of its first-member range in positions of
// N+(root), and the map from the job's member ids to positions (null: equal).
struct JobCtx {
  const Sched* S;
  int root;
  int64_t stat;
  int depth;
  int hi_pos;
  const int* map;
  int* prefix;
  int wave_gid;
};

// q-cliques, q >= 3, inside C (rows upper-triangular: row i holds members
// above i) whose first member is in `first`.  The work is split into pair
// tasks (i, j), j a member of C adjacent to i and above it, numbered by a
// prefix sum over i (`pst`, 64 * NW ints of LDS).  Every lane runs its own
// depth-first search below a pair and takes the next task from a wave-shared
// counter when it is done, so all lanes run the same loop body until the
// tasks run out.  Returns this lane's share.
template <int NW>
__device__ __forceinline__ uint64_t lane_solve(const uint64_t (&C)[NW], const uint64_t (&first)[NW], int q,
                                               LdsU64* lr, int stride, LdsI32* pst, const JobCtx& J) {
  const int lane = lane_id();
  int total = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int i = w * 64 + lane;
    int c = 0;
    if ((first[w] >> lane) & 1ull) {
#pragma unroll
      for (int q2 = 0; q2 < NW; ++q2) c += __popcll(C[q2] & lr[q2 * stride + i]);
    }
    const int incl = static_cast<int>(wave_incl_scan_i64(c));
    pst[i] = total + incl - c;
    total += uni(read_lane(incl, kWave - 1));
  }
  wave_sync();
  const int r0 = q - 2;  // members still to choose below a pair
  uint64_t acc = 0;
  uint64_t cur[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) cur[w] = 0;
  // per-lane stack of remaining candidate sets, up to 4 levels: four separate
  // locals written and read through branches on the depth (an array or a
  // struct would be placed in scratch memory)
  uint64_t sa0 = 0, sa1 = 0, sb0 = 0, sb1 = 0, sc0 = 0, sc1 = 0, sd0 = 0, sd1 = 0;
  int d = -1;  // depth below the pair; -1: needs a task
  bool done = false;
  int tbase = 0;
  int hi_pos = J.hi_pos;  // end (in positions) of the first members still owned
  // the next (up to) 64 untaken pair tasks are decoded together, one per lane
  // (packed i << 8 | j in pend), and handed to free lanes by a lane shuffle
  int gen_base = 0, gen_n = 0;  // decoded tasks: gen_base .. gen_base + gen_n - 1
  int nrefill = 0;
  int pend = 0;
  for (;;) {
    const bool want = !done && d < 0;
    const uint64_t wb = ballot(want);
    const int nw = __popcll(wb);
    if (wb && (nw >= kRefillMin || ballot(d >= 0) == 0)) {
      // idle waves elsewhere: hand over the first members whose pair tasks
      // make up about the upper half of the untaken ones
      // (two relaxed loads past the L2 and a wait: checked on every 8th refill)
      if (J.S->donate && (++nrefill & 7) == 0 && total - tbase >= kJobDonateMin && sched_want_donation_tail(*J.S)) {
        const int tmid = tbase + (total - tbase) / 2;
        int ic = 0;  // last member whose range starts before tmid
#pragma unroll
        for (int st = 32 * NW; st >= 1; st >>= 1)
          if (pst[ic + st] < tmid) ic += st;
        ++ic;
        if (ic < 64 * NW) {
          const int cut = pst[ic];
          const int pos = J.map ? J.map[ic] : ic;
          if (cut < total && hi_pos - pos >= 1) {
            const int pay = task_payload(J.root, J.stat, J.depth, pos, hi_pos, J.prefix);
            if (sched_publish(*J.S, pay, J.wave_gid)) {
              total = cut;
              hi_pos = pos;
            }
          }
        }
      }
      if (tbase + nw > gen_base + gen_n && gen_base + gen_n < total) {
        // decode tasks tbase + lane: binary search over the task prefix for the
        // first member i, then the (t - pst[i])-th candidate above it
        gen_base = tbase;
        gen_n = total - tbase < kWave ? total - tbase : kWave;
        const int t = tbase + lane;
        if (t < total) {
          int i = 0;  // last member whose task range starts at or before t
#pragma unroll
          for (int st = 32 * NW; st >= 1; st >>= 1)
            if (pst[i + st] <= t) i += st;
          uint64_t ci[NW];
#pragma unroll
          for (int q2 = 0; q2 < NW; ++q2) ci[q2] = C[q2] & lr[q2 * stride + i];
          pend = (i << 8) | select_nth<NW>(ci, t - pst[i]);
        }
      }
      // task tbase + rank goes to the rank-th free lane; every decoded task
      // below total lies in [gen_base, gen_base + gen_n)
      const int t = tbase + mbcnt(wb);
      const int ij = __shfl(pend, want ? (t - gen_base) & (kWave - 1) : 0, kWave);
      if (want) {
        if (t < total) {
          const int i = ij >> 8, j = ij & 255;
          int cnt = 0;
#pragma unroll
          for (int q2 = 0; q2 < NW; ++q2) {
            cur[q2] = C[q2] & lr[q2 * stride + i] & lr[q2 * stride + j];
            cnt += __popcll(cur[q2]);
          }
          if (r0 == 1) acc += static_cast<uint64_t>(cnt);
          else if (cnt >= r0) d = 0;
        } else {
          done = true;
        }
      }
      tbase += nw;
    }
    if (ballot(!done) == 0) break;
    if (d >= 0) {
      const int r = r0 - d;  // members still to choose at this depth
      if (r == 2) {
        // the pairs (i, j) of cur with j in row(i) (rows hold only larger
        // members), counted in one pass; cur is then empty and popped below
        acc += edge_count<NW>(cur, lr, stride);
#pragma unroll
        for (int w = 0; w < NW; ++w) cur[w] = 0;
      } else {
        int wsel = -1;  // -1: a set restored by a pop can be empty
#pragma unroll
        for (int w = NW - 1; w >= 0; --w)
          if (cur[w]) wsel = w;
        if (wsel >= 0) {
          const uint64_t cw = pick<NW>(cur, wsel);
          const int i = wsel * 64 + __builtin_ctzll(cw);
#pragma unroll
          for (int w = 0; w < NW; ++w) cur[w] = (w == wsel) ? (cw & (cw - 1)) : cur[w];
          uint64_t ch[NW];
          int cnt = 0;
#pragma unroll
          for (int q2 = 0; q2 < NW; ++q2) {
            ch[q2] = cur[q2] & lr[q2 * stride + i];
            cnt += __popcll(ch[q2]);
          }
          if (r == 3) {
            // the last two members inside ch: its edges, counted in place
            // instead of pushing ch (no stack traffic at the deepest level)
            if (cnt >= 2) acc += edge_count<NW>(ch, lr, stride);
          } else if (cnt >= r - 1) {
            const uint64_t c0 = cur[0], c1 = NW == 2 ? pick<NW>(cur, 1) : 0;
            if (d == 0) { sa0 = c0; sa1 = c1; }
            else if (d == 1) { sb0 = c0; sb1 = c1; }
            else if (d == 2) { sc0 = c0; sc1 = c1; }
            else { sd0 = c0; sd1 = c1; }
#pragma unroll
            for (int w = 0; w < NW; ++w) cur[w] = ch[w];
            ++d;
          }
        }
      }
      // a set used up in this pass is popped in the same pass
      bool empty = true;
#pragma unroll
      for (int w = 0; w < NW; ++w) empty = empty && cur[w] == 0;
      if (empty) {
        if (d == 0) {
          d = -1;
        } else {
          --d;
          cur[0] = d == 0 ? sa0 : (d == 1 ? sb0 : (d == 2 ? sc0 : sd0));
          if constexpr (NW == 2) cur[NW - 1] = d == 0 ? sa1 : (d == 1 ? sb1 : (d == 2 ? sc1 : sd1));
        }
      }
    }
  }
  return acc;
}

// q-cliques (1 <= q <= kSolverMaxQ) inside the set Cl (NW words) whose first
// member lies in [lo, hi); returns this lane's share.
template <int NW>
__device__ uint64_t small_solve(LdsU64* Cl, int q, LdsU64* lr, int stride, int lo, int hi, LdsI32* pst,
                               const JobCtx& J) {
  const int lane = lane_id();
  uint64_t C[NW], first[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    C[w] = uniu64(Cl[w]);
    first[w] = C[w] & range_mask64(lo - 64 * w, hi - 64 * w);
  }
  uint64_t add = 0;
  if (q == 1) {
    if (lane == 0)
#pragma unroll
      for (int w = 0; w < NW; ++w) add += static_cast<uint64_t>(__popcll(first[w]));
  } else if (q == 2) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if ((first[w] >> lane) & 1ull) {
        const int i = w * 64 + lane;
#pragma unroll
        for (int q2 = 0; q2 < NW; ++q2) add += static_cast<uint64_t>(__popcll(C[q2] & lr[q2 * stride + i]));
      }
    }
  } else if (q <= 3) {
    // the wave walks the first member i, lane j takes the second member
    for (int w = 0; w < NW; ++w) {
      uint64_t x = pick<NW>(first, w);
      while (x) {
        const int i = w * 64 + __builtin_ctzll(x);
        x &= x - 1;
        uint64_t Ci[NW];
#pragma unroll
        for (int q2 = 0; q2 < NW; ++q2) Ci[q2] = uniu64(C[q2] & lr[q2 * stride + i]);
        for (int w2 = w; w2 < NW; ++w2) {
          if ((pick<NW>(Ci, w2) >> lane) & 1ull) {
            const int j = w2 * 64 + lane;
            uint64_t Cj[NW];
#pragma unroll
            for (int q2 = 0; q2 < NW; ++q2) Cj[q2] = Ci[q2] & lr[q2 * stride + j];
            add += q == 3 ? count_in<1, NW>(Cj, lr, stride) : count_in<2, NW>(Cj, lr, stride);
          }
        }
      }
    }
  } else {
    add = lane_solve<NW>(C, first, q, lr, stride, pst, J);
  }
  return add;
}

__device__ __forceinline__ uint64_t small_solve_any(int nw, const uint64_t* Cg, int q, const uint64_t* lrg, int stride,
                                                    int lo, int hi, int* pstg, const JobCtx& J) {
  LdsU64* C = as_lds(Cg);
  LdsU64* lr = as_lds(lrg);
  LdsI32* pst = (LdsI32*)(pstg);
  return nw == 1 ? small_solve<1>(C, q, lr, stride, lo, hi, pst, J) : small_solve<2>(C, q, lr, stride, lo, hi, pst, J);
}

// Local ids for the members of the multi-word set C (at most kReindexMax, by
// the caller's check): positions into L.pos, rows (nw words, word-major with
// stride kReindexMax) into L.lr, and the full local set into L.cset.
// Returns nw.
__device__ __forceinline__ int reindex(const uint64_t* C, int Wd, const uint64_t* rows, int stride, const CliqueLds& L) {
  const int lane = lane_id();
  int base = 0;
  for (int w = 0; w < Wd; ++w) {
    const bool bit = (C[w] >> lane) & 1ull;
    const uint64_t b = ballot(bit);
    if (bit && base + mbcnt(b) < kReindexMax) L.pos[base + mbcnt(b)] = w * 64 + lane;
    base += __popcll(b);
  }
  const int m = uni(base < kReindexMax ? base : kReindexMax);
  const int nw = m <= 64 ? 1 : 2;
  wave_sync();
  for (int a = lane; a < m; a += kWave) {
    const int pa = L.pos[a];
    uint64_t r0 = 0, r1 = 0;
    for (int bb = a + 1; bb < m; ++bb) {
      const int pb = L.pos[bb];
      if ((rows[static_cast<size_t>(pb >> 6) * stride + pa] >> (pb & 63)) & 1ull) {
        if (bb < 64) r0 |= 1ull << bb;
        else r1 |= 1ull << (bb - 64);
      }
    }
    L.lr[a] = r0;
    L.lr[kReindexMax + a] = r1;
  }
  if (lane < 2) {
    const int rem = m - 64 * lane;
    L.cset[lane] = rem >= 64 ? ~0ull : (rem > 0 ? ((1ull << rem) - 1) : 0ull);
  }
  wave_sync();
  return nw;
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

// rows_g: this wave's global region for the rows of roots too wide for LDS
template <bool kHostBal>
__device__ void run_task(const CliqueArgs& A, const CliqueLds& L, uint64_t* rows_g, const Task& t,
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
  // rows of N+(v): in LDS (stride kLocalMax) when d <= kLocalMax, else in the
  // graph's row cache (stride d) when there is one, else in this wave's global
  // region (stride dmax).  The cache is filled by the first launch on a graph
  // (rc_mode 1) and read by later ones (rc_mode 2).
  const bool lds_rows = d <= kLocalMax;
  uint64_t* crow = A.rc_mode ? reinterpret_cast<uint64_t*>(A.rcache) + A.rcoff[v] : nullptr;
  uint64_t* rows = lds_rows ? L.rows : (A.rc_mode ? crow : rows_g);
  const int rs = lds_rows ? kLocalMax : (A.rc_mode ? d : dmax);
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
  } else if (d > 0 && hi_t > t.lo && (!A.prune || d >= k - 1 || A.rc_mode == 1)) {
    const int Wd = (d + 63) >> 6;
    if (A.rc_mode == 2) {
      // ---- rows from the cache: wide roots read them in place, the rest are
      // copied to LDS
      if (lds_rows) {
        for (int idx = lane; idx < Wd * d; idx += kWave) {
          const int w = idx / d, p = idx - w * d;
          L.rows[w * kLocalMax + p] = crow[static_cast<size_t>(w) * d + p];
        }
        wave_sync();
      }
    } else {
      // ---- load N+(v), out-degree prefix of its members (Extend, coalesced)
      int running = 0;
      for (int c = 0; c < d; c += kWave) {
        const int i = c + lane;
        int od = 0;
        if (i < d) {
          const int u = A.col[base + i];
          L.nbr[i] = u;
          od = static_cast<int>(A.rp[u + 1] - A.rp[u]);
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
      // ---- adjacency of N+(v) restricted to itself, as bitmap rows: a block
      // of rows at a time in the LDS tile L.rows (LDS atomics), then stored to
      // the global region for roots wider than kLocalMax (one write per word)
      const int tile_rows = lds_rows ? d : (2 * kLocalMax) / Wd;
      for (int p0 = 0; p0 < d; p0 += tile_rows) {
        const int p1 = p0 + tile_rows < d ? p0 + tile_rows : d;
        const int ts = lds_rows ? kLocalMax : tile_rows;  // tile stride
        for (int idx = lane; idx < Wd * (p1 - p0); idx += kWave) {
          const int w = idx / (p1 - p0), p = idx - w * (p1 - p0);
          L.rows[w * ts + p] = 0ull;
        }
        wave_sync();
        for (int tt = L.offs[p0] + lane; tt < L.offs[p1]; tt += kWave) {
          int lo = p0, hi = p1;  // i = last index with offs[i] <= tt
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (L.offs[mid] <= tt) lo = mid; else hi = mid;
          }
          const int i = lo;
          const int e = A.col[A.rp[L.nbr[i]] + (tt - L.offs[i])];
          int a = i + 1, b = d;  // e > nbr[i], so search above i
          while (a < b) {
            const int mid = (a + b) >> 1;
            if (L.nbr[mid] < e) a = mid + 1; else b = mid;
          }
          if (a < d && L.nbr[a] == e) atomicOr(reinterpret_cast<unsigned long long*>(&L.rows[(a >> 6) * ts + (i - p0)]), 1ull << (a & 63));
        }
        wave_sync();
        if (!lds_rows) {
          for (int idx = lane; idx < Wd * (p1 - p0); idx += kWave) {
            const int w = idx / (p1 - p0), p = idx - w * (p1 - p0);
            rows[static_cast<size_t>(w) * rs + p0 + p] = L.rows[w * ts + p];
          }
          wave_sync();
        }
      }
      if (A.rc_mode == 1 && lds_rows) {
        for (int idx = lane; idx < Wd * d; idx += kWave) {
          const int w = idx / d, p = idx - w * d;
          crow[static_cast<size_t>(w) * d + p] = L.rows[w * kLocalMax + p];
        }
      }
    }
    // a root with fewer than k-1 out-neighbours has no k-clique: when it is
    // here only to fill the row cache, the counting below is skipped
    if (!A.prune || d >= k - 1) {
      // ---- level-1 candidate set and the task prefix
      for (int w = lane; w < Wd; w += kWave) {
        const int rem = d - w * 64;
        L.stk[1 * W + w] = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
      }
      wave_sync();
      for (int s = 1; s < t.depth; ++s) {
        const int p = L.cur[s];
        for (int w = lane; w < Wd; w += kWave) L.stk[(s + 1) * W + w] = L.stk[s * W + w] & rows[static_cast<size_t>(w) * rs + p];
        wave_sync();
      }
      // roots with at most 128 out-neighbours: their rows already are local rows
      // (positions = local ids, Wd <= 2 words, in LDS with stride kLocalMax)
      const bool solver = A.prune != 0;
      const bool root_local = solver && lds_rows;
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
            for (int w = w0; w < Wd; ++w) pc += static_cast<uint64_t>(__popcll(C[w] & rows[static_cast<size_t>(w) * rs + p]));
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
      // The dense solver has a single call site (so it is inlined once): the
      // DFS records a pending job and the loop head runs it.  Jobs are bounded
      // (one-word sets, or at most 4 remaining levels on two-word sets) because
      // a job cannot be donated.
      bool job = false, job_last = false;
      int job_nw = 1, job_q = 0, job_stride = 0, job_lo = 0, job_hi = 0;
      int job_depth = 0, job_hipos = 0;
      const int* job_map = nullptr;
      const uint64_t* job_C = nullptr;
      const uint64_t* job_R = nullptr;
      // Fast path (at most 64 words): lane w keeps word w of the current level's
      // candidate set in a register, so choosing the next extension is a ballot
      // and extending it is one row read per lane.  cur / hiv entries are
      // written by every lane with the same value, so no barrier is needed to
      // read them back.
      const bool fast = Wd <= kWave;
      uint64_t cw = 0;
      int depth = s0;
      if (root_local && k - s0 <= kSolverMaxQ && (k - s0 <= 3 || d <= 64)) {
        job = job_last = true;
        job_nw = Wd;
        job_C = L.stk + s0 * W;
        job_q = k - s0;
        job_R = L.rows;
        job_stride = kLocalMax;
        job_lo = t.lo;
        job_hi = hi_t;
        job_depth = s0;
        job_hipos = hi_t;
        job_map = nullptr;
      } else if (s0 == k - 2) {
        leaf_parent(s0, t.lo, hi_t);
        depth = -1;
      } else {
        L.cur[depth] = t.lo - 1;
        L.hiv[depth] = hi_t;
        if (fast && lane < Wd) cw = L.stk[depth * W + lane];
        wave_sync();
      }
      int steps = 0;
      while (depth >= 0) {
        if (job) {
          const JobCtx J{&A.S, v, t.stat, job_depth, job_hipos, job_map, L.cur, wave_gid};
          add_acc(small_solve_any(job_nw, job_C, job_q, job_R, job_stride, job_lo, job_hi, L.pst, J));
          job = false;
          if (job_last) break;
        }
        int u;
        if (fast) {
          const int from = L.cur[depth] + 1, to = L.hiv[depth];
          const uint64_t m = lane < Wd ? (cw & range_mask64(from - 64 * lane, to - 64 * lane)) : 0ull;
          const uint64_t bl = ballot(m != 0ull);
          if (!bl) {
            u = -1;
          } else {
            const int l = __ffsll(static_cast<long long>(bl)) - 1;
            const uint64_t wm = __shfl(m, l, kWave);
            u = uni(64 * l + __builtin_ctzll(wm));
          }
        } else {
          u = next_bit(L.stk + depth * W, L.cur[depth] + 1, L.hiv[depth]);
        }
        if (u < 0) {
          if (depth == s0) break;
          --depth;
          if (fast && lane < Wd) cw = L.stk[depth * W + lane];
          continue;
        }
        L.cur[depth] = u;
        if (lane == 0) {
          nodes_l += 1;
          reads_l += static_cast<uint64_t>(L.offs[u + 1] - L.offs[u]);
        }
        int cnt = 0;
        uint64_t x = 0;
        if (fast) {
          if (lane < Wd) x = cw & rows[static_cast<size_t>(lane) * rs + u];
          cnt = uni(wave_sum_i32(__popcll(x)));
        } else {
          for (int w = lane; w < Wd; w += kWave) {
            const uint64_t y = L.stk[depth * W + w] & rows[static_cast<size_t>(w) * rs + u];
            L.stk[(depth + 1) * W + w] = y;
            cnt += __popcll(y);
          }
          cnt = uni(wave_sum_i32(cnt));
          wave_sync();
        }
        const int q = k - depth - 1;  // vertices still to add below the child
        if (!A.prune || cnt >= q) {
          const bool bounded = q <= kSolverMaxQ && (cnt <= 64 || q <= 4);
          const bool need_lds = (solver && bounded && (root_local || cnt <= kReindexMax)) || depth + 1 == k - 2;
          if (fast && need_lds) {
            if (lane < Wd) L.stk[(depth + 1) * W + lane] = x;
            wave_sync();
          }
          if (root_local && bounded) {
            job = true;
            job_nw = Wd;
            job_C = L.stk + (depth + 1) * W;
            job_q = q;
            job_R = L.rows;
            job_stride = kLocalMax;
            job_lo = 0;
            job_hi = d;
            job_depth = depth + 1;
            job_hipos = d;
            job_map = nullptr;
          } else if (solver && bounded && cnt <= kReindexMax) {
            job_nw = reindex(L.stk + (depth + 1) * W, Wd, rows, rs, L);
            job = true;
            job_C = L.cset;
            job_q = q;
            job_R = L.lr;
            job_stride = kReindexMax;
            job_lo = 0;
            job_hi = kReindexMax;
            job_depth = depth + 1;
            job_hipos = d;
            job_map = L.pos;
          } else if (depth + 1 == k - 2) {
            leaf_parent(depth + 1, 0, d);
          } else {
            if (fast) {
              if (lane < Wd) L.stk[(depth + 1) * W + lane] = x;
              cw = x;
            }
            ++depth;
            L.cur[depth] = -1;
            L.hiv[depth] = d;
            if (!fast) wave_sync();
          }
        }
        // ---- host-driven balancing: once the launch is stopped, the untried
        // extensions of every open level become tasks for the next launch
        // (checked every `period` steps without a pending solver job)
        if (kHostBal) {
          if (!job && (++steps % A.S.period) == 0 && sched_stopped(A.S)) {
            wave_sync();
            for (int s = s0; s <= depth; ++s) {
              const int from = L.cur[s] + 1, to = L.hiv[s];
              if (count_bits(L.stk + s * W, from, to) > 0)
                sched_spill(A.S, task_payload(v, t.stat, s, from, to, L.cur));
            }
            break;
          }
        } else if (A.S.donate && (++steps % A.S.period) == 0 && sched_want_donation(A.S)) {
          // ---- donation (Section IV-D redistribute, done by the busy wave)
          wave_sync();
          for (int s = s0; s <= depth; ++s) {
            const int from = L.cur[s] + 1, to = L.hiv[s];
            const int c = count_bits(L.stk + s * W, from, to);
            if (c >= 2) {
              const int keep = c - c / 2;
              const int mid = select_bit(L.stk + s * W, from, to, keep + 1);
              const int pay = task_payload(v, t.stat, s, mid, to, L.cur);
              if (sched_publish(A.S, pay, wave_gid)) L.hiv[s] = mid;
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

// 4 waves per SIMD: the register budget (128 VGPRs) this needs holds the
// kernel without spills and is what keeps row-read latency covered
// (instantiated with kHostBal for launches under host-driven balancing, so
// the default kernel carries none of that code)
template <bool kHostBal>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) clique_kernel(CliqueArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int wave_gid = blockIdx.x;
  CliqueLds L = carve(smem, A.dmax, A.W, A.k);
  // (no region when every root's rows are in LDS or in the row cache)
  uint64_t* rows_g = A.rows_global ? reinterpret_cast<uint64_t*>(A.rows_global) + static_cast<size_t>(wave_gid) * A.W * A.dmax
                                   : nullptr;
  WaveAcc WA;
  WA.acc = 0;
  WA.cur_g = -1;
  WA.ovf = 0;
  WA.nodes = 0;
  WA.tasks = 0;
  const uint64_t t_begin = wall_clock64();
  SchedIter it;
  sched_begin(A.S, it);
  Task t;
  while (sched_next<kHostBal>(A.S, it, wave_gid, L.cur, &t)) {
    run_task<kHostBal>(A, L, rows_g, t, WA, wave_gid);
    WA.tasks++;
  }
  sched_end<kHostBal>(A.S);
  const uint64_t t_idle = it.t_idle;
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

size_t clique_lds_bytes(int dmax, int W, int k) {
  auto a16 = [](size_t x) { return (x + 15) & ~static_cast<size_t>(15); };
  size_t off = static_cast<size_t>(2) * kLocalMax * 8;
  off = a16(off) + static_cast<size_t>(k + 1) * W * 8;
  off = a16(off) + static_cast<size_t>(dmax) * 4;
  off = a16(off) + static_cast<size_t>(dmax + 1) * 4;
  off = a16(off) + 2 * (kMaxK + 2) * 4;
  off = a16(off) + kReindexMax / 64 * kReindexMax * 8 + 4 * 8 + 2 * kReindexMax * 4;
  return a16(off);
}

hipError_t clique_occupancy(size_t lds_bytes, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, clique_kernel<false>, 64, lds_bytes);
}

hipError_t launch_clique(const CliqueArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
  if (a.S.host_bal)
    hipLaunchKernelGGL(clique_kernel<true>, dim3(grid), dim3(64), lds_bytes, s, a);
  else
    hipLaunchKernelGGL(clique_kernel<false>, dim3(grid), dim3(64), lds_bytes, s, a);
  return hipGetLastError();
}

}  // namespace dm

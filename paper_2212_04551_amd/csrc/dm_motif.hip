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
//   - Entries at or below v_0 can never join a canonical traversal, so level
//     lists hold only vertices above v_0.
//   - The last two levels are counted without visiting the leaves one by one
//     (Aggregate, Section IV-C, for a whole level at once).  For a traversal
//     tr of size k-2 with list E, the canonical k-traversals tr+x+y are
//       (a) x < y, both canonical entries of E (y keeps its first neighbour in
//           tr, and x now sits after it), and
//       (b) x canonical, y a neighbour of x above v_0 that is neither in E nor
//           in tr (first neighbour x).
//     The pattern of (a) depends only on {mask x, mask y, x ~ y} and is
//     symmetric in x and y, so per mask pair the count is C(c_a, 2) or
//     c_a * c_b (c = canonical entries per mask) split into adjacent and
//     non-adjacent pairs; the adjacent pairs, and the pairs of (b), come from
//     one load-balanced pass over the neighbour lists of all canonical x
//     (lanes take consecutive (x, neighbour) items of a wave prefix sum of
//     degrees).  Each non-empty (mask pair, adjacency) bin is relabelled once
//     through the dictionary into per-wave LDS class counters.  A range
//     [lo, hi) of x (a donated task) takes the pairs whose smaller member lies
//     in the range: P([lo, |E|)) - P([hi, |E|)).
#include <climits>

#include "dm_internal.hpp"

namespace dm {

namespace {

constexpr int kSuf = kMotifMaxK + 1;

// kBins (a template parameter below) = the number of masks an entry of a
// (k-2)-traversal's list can have, 2^(k-2): 16 for k <= 6 and 32 for k = 7
// (the kernel is instantiated for both).
// A leaf-level range is donated only when this many entries are untried: the
// taker re-extends the whole prefix first.
constexpr int kLeafDonateMin = 128;
// Leaf-level lists of at most this many entries are copied to LDS, so the
// neighbour lookups binary-search LDS instead of global memory.
constexpr int kLeafLds = 800;
// Membership filter over the LDS copy: one bit per (vertex mod 8192); most
// neighbours of an x are not in the list and are rejected without a search.
constexpr int kFilterWords = 256;
// A list longer than kLeafLds stays in global memory; the LDS space of the
// copy then holds a second filter (one bit per vertex mod 8192, next to the
// hashed small one) and fences: every fstride-th entry of the list.  A lookup
// that passes both filters binary-searches the fences in LDS and then reads
// the one window of at most kWindow entries it selects, all loads at once.
constexpr int kBigFilterWords = 256;
constexpr int kFenceMax = kLeafLds - kBigFilterWords;
constexpr int kWindow = 8;
// An LDS list is indexed by value: entry values above v0 are cut into
// kBuckets ranges of 2^shift ids, and bk[b] is the first index of range b, so
// a lookup searches only the entries of its own range.
constexpr int kBuckets = 256;
static_assert(kFenceMax > 0, "big filter and fences share the list copy's LDS space");
__device__ __forceinline__ int filt_index(int y, bool big) {
  // the small filter takes the low bits for an LDS list, a multiplicative hash
  // (top 13 bits) alongside the big filter
  return big ? static_cast<int>((static_cast<uint32_t>(y) * 0x9E3779B1u) >> 19) : (y & (kFilterWords * 32 - 1));
}

struct MotifLds {
  unsigned long long* cnt;  // [ncls] class counters of the current graph
  unsigned long long* adj;  // [kBins * kBins] adjacent canonical pairs (mask of smaller, mask of larger)
  unsigned long long* nw;   // [kBins] pairs (b): by mask of x
  unsigned* ccount;         // [2][kBins] canonical entries by mask: in [lo, hi), in [hi, |E|)
  int64_t* sl_start;        // [kWave + 1] slice: prefix sum of the degrees of canonical entries
  int64_t* sl_base;         // [kWave] slice: row_ptr of the entry's vertex
  int* sl_mask;             // [kWave] slice: entry mask over tr
  int* tr;                  // [kSuf] traversal
  int* code;                // [kSuf] dictionary code per traversal size
  int* sufmax;              // [kSuf][kSuf] max of tr[f+1..s-1] per size s
  int* cursor;              // [kSuf]
  int* endv;                // [kSuf]
  int* esize;               // [kSuf]
  int* ev;                  // [kLeafLds] leaf level: copy of the (k-2)-traversal's list
  uint8_t* em;              // [kLeafLds] and of its masks
  unsigned* filt;           // [kFilterWords] membership filter of the LDS copy (zero between calls)
  int* lflag;               // [1] the (k-2)-level list was written straight into ev / em
  int* mark;                // [kWave] slice lane whose degree range starts at each item of a batch
  uint16_t* bk;             // [kBuckets + 1] leaf level: first LDS-list index of each value range
};

__device__ __forceinline__ int off_of(int i) { return i * (i - 1) / 2 - 1; }  // bitmap field of v_i, i >= 2

// Class counters per wave: in LDS for k <= 7; k = 8's 11,117 counters live
// in a per-wave row of global memory (kBins == 64).
template <int kBins>
__device__ MotifLds carve(unsigned char* smem, int ncls) {
  MotifLds L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = smem + off;
    off += (bytes + 15) & ~static_cast<size_t>(15);
    return p;
  };
  L.cnt = kBins == 64 ? nullptr : reinterpret_cast<unsigned long long*>(take(static_cast<size_t>(ncls) * 8));
  L.adj = reinterpret_cast<unsigned long long*>(take(kBins * kBins * 8));
  L.nw = reinterpret_cast<unsigned long long*>(take(kBins * 8));
  L.ccount = reinterpret_cast<unsigned*>(take(2 * kBins * 4));
  L.sl_start = reinterpret_cast<int64_t*>(take((kWave + 1) * 8));
  L.sl_base = reinterpret_cast<int64_t*>(take(kWave * 8));
  L.sl_mask = reinterpret_cast<int*>(take(kWave * 4));
  L.tr = reinterpret_cast<int*>(take(kSuf * 4));
  L.code = reinterpret_cast<int*>(take(kSuf * 4));
  L.sufmax = reinterpret_cast<int*>(take(kSuf * kSuf * 4));
  L.cursor = reinterpret_cast<int*>(take(kSuf * 4));
  L.endv = reinterpret_cast<int*>(take(kSuf * 4));
  L.esize = reinterpret_cast<int*>(take(kSuf * 4));
  L.ev = reinterpret_cast<int*>(take(kLeafLds * 4));
  L.em = reinterpret_cast<uint8_t*>(take(kLeafLds));
  L.filt = reinterpret_cast<unsigned*>(take(kFilterWords * 4));
  L.lflag = reinterpret_cast<int*>(take(16));
  L.mark = reinterpret_cast<int*>(take(kWave * 4));
  L.bk = reinterpret_cast<uint16_t*>(take((kBuckets + 1) * 2));
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
  unsigned long long* gcnt;  // k = 8: this wave's class counters in global memory
};

template <int kBins>
__device__ __forceinline__ unsigned long long* class_counters(const MotifLds& L, const MotifWave& MW) {
  if constexpr (kBins == 64) return MW.gcnt;
  else return L.cnt;
}

template <int kBins>
__device__ __forceinline__ void flush_counts(const MotifArgs& A, const MotifLds& L, MotifWave& MW) {
  const int lane = lane_id();
  unsigned long long* cnt = class_counters<kBins>(L, MW);
  wave_sync();
  for (int c = lane; c < A.ncls; c += kWave) {
    const unsigned long long v = cnt[c];
    if (MW.cur_g >= 0) add_counter(A.out + static_cast<size_t>(MW.cur_g) * A.ncls + c, v, A.flags);
    cnt[c] = 0;
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
  const int ns = L.esize[s];
  const int64_t xb = A.rp[x];
  const int dx = static_cast<int>(A.rp[x + 1] - xb);
  const int v0 = L.tr[0];
  int nn = 0;
  for (int c = 0; c < dx; c += kWave) {
    const int i = c + lane;
    const bool ok = i < dx && A.col[xb + i] > v0;
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
  // the leaf level's list goes straight to LDS when it fits
  const bool to_lds = A.leaf_lds && s + 1 == A.k - 2 && static_cast<int64_t>(ns) - 1 + nn <= kLeafLds;
  int32_t* Nv = to_lds ? L.ev : MW.vert + A.level_off[s + 1];
  uint8_t* Nm = to_lds ? L.em : MW.mask + A.level_off[s + 1];
  const int64_t cap = to_lds ? kLeafLds : A.level_cap[s + 1];
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
    L.lflag[0] = to_lds ? 1 : 0;
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

// Count every leaf below the traversal tr (|tr| = s = k-2) whose x is an entry
// of [lo, hi) of tr's list.  Between slices of 64 entries the untried part of
// the range may be donated (a task at depth s).  Returns the final hi.
template <int kBins>
__device__ __forceinline__ int leaf_level(const MotifArgs& A, const MotifLds& L, MotifWave& MW, int s, int lo, int hi,
                          const Task& t, int wave_gid, uint64_t& nodes_l, uint64_t& leaves_l, uint64_t& reads_l) {
  const int lane = lane_id();
  const int ns = L.esize[s];
  // the list (and masks) in LDS: written there by extend_level, or copied when
  // it fits; else it stays in this wave's global region
  const bool direct = s >= 2 && L.lflag[0] != 0;
  const bool in_lds = direct || ns <= kLeafLds;
  // value index (bk) of a sorted LDS array a[0..n) whose entries lie in
  // (v0, vmax]: the LDS copy of the list, or the fences of a global one
  int bbase = 0, bmax = -1, bshift = 0;
  auto build_index = [&](const int* a, int n, int vmax) {
    bbase = L.tr[0] + 1;
    bmax = vmax;
    bshift = 0;
    while (((bmax - bbase) >> bshift) >= kBuckets) ++bshift;
    for (int i = lane; i < n; i += kWave) {
      const int b = (a[i] - bbase) >> bshift;
      const int bp = i ? ((a[i - 1] - bbase) >> bshift) : -1;
      for (int q = bp + 1; q <= b; ++q) L.bk[q] = static_cast<uint16_t>(i);
    }
    const int blast = n > 0 ? ((a[n - 1] - bbase) >> bshift) : -1;
    for (int q = blast + 1 + lane; q <= kBuckets; q += kWave) L.bk[q] = static_cast<uint16_t>(n);
  };
  unsigned* bigf = reinterpret_cast<unsigned*>(L.ev);
  int* fence = L.ev + kBigFilterWords;
  const int fstride = (ns + kFenceMax - 1) / kFenceMax;  // entries per fence (global list)
  const int nfence = fstride > 0 ? (ns + fstride - 1) / fstride : 0;
  if (in_lds) {
    const int32_t* Gv = MW.vert + A.level_off[s];
    const uint8_t* Gm = MW.mask + A.level_off[s];
    for (int i = lane; i < ns; i += kWave) {
      int y;
      if (direct) {
        y = L.ev[i];
      } else {
        y = Gv[i];
        L.ev[i] = y;
        L.em[i] = Gm[i];
      }
      const int f = filt_index(y, false);
      atomicOr(&L.filt[f >> 5], 1u << (f & 31));
    }
    wave_sync();
    build_index(L.ev, ns, ns > 0 ? L.ev[ns - 1] : L.tr[0]);
  } else {
    for (int i = lane; i < kBigFilterWords; i += kWave) bigf[i] = 0u;
    wave_sync();
    const int32_t* Gv = MW.vert + A.level_off[s];
    for (int i = lane; i < ns; i += kWave) {
      const int y = Gv[i];
      atomicOr(&bigf[(y >> 5) & (kBigFilterWords - 1)], 1u << (y & 31));
      const int f = filt_index(y, true);
      atomicOr(&L.filt[f >> 5], 1u << (f & 31));
      if (i % fstride == 0) fence[i / fstride] = y;
    }
    wave_sync();
    build_index(fence, nfence, Gv[ns - 1]);
  }
  // list reads branch on where the list lives (uniform), so LDS reads stay
  // LDS instructions instead of generic ones
  const int32_t* Gv = MW.vert + A.level_off[s];
  const uint8_t* Gm = MW.mask + A.level_off[s];
  auto ev_at = [&](int j) -> int { return in_lds ? L.ev[j] : Gv[j]; };
  auto em_at = [&](int j) -> unsigned { return in_lds ? L.em[j] : Gm[j]; };
  // position of w in the list, or -1
  auto ev_find = [&](int w) -> int {
    if (in_lds) {
      if (w > bmax || w < bbase) return -1;
      const int b = (w - bbase) >> bshift;
      const int lo = L.bk[b], hi = L.bk[b + 1];
      const int j = lo + lower_bound_g(L.ev + lo, hi - lo, w);
      return j < hi && L.ev[j] == w ? j : -1;
    }
    if (w > bmax || w < bbase) return -1;
    // fences <= w: those of earlier ranges and a search inside w's own range
    const int r = (w - bbase) >> bshift;
    const int flo = L.bk[r], fhi = L.bk[r + 1];
    const int nf = flo + lower_bound_g(fence + flo, fhi - flo, w + 1);
    if (nf == 0) return -1;
    const int b = (nf - 1) * fstride;
    const int n = ns - b < fstride ? ns - b : fstride;
    if (fstride <= kWindow) {
      int pos = -1;
#pragma unroll
      for (int q = 0; q < kWindow; ++q)
        if (q < n && Gv[b + q] == w) pos = b + q;
      return pos;
    }
    const int j = b + lower_bound_g(Gv + b, n, w);
    return j < b + n && Gv[j] == w ? j : -1;
  };
  const int nm = 1 << s;
  const unsigned low = static_cast<unsigned>(nm - 1);
  const int v0 = L.tr[0];
  for (int i = lane; i < kBins * kBins; i += kWave) L.adj[i] = 0;
  for (int i = lane; i < kBins; i += kWave) L.nw[i] = 0;
  for (int i = lane; i < 2 * kBins; i += kWave) L.ccount[i] = 0;
  wave_sync();
  // The traversal's members and the canonical test's thresholds, held in
  // registers for the leaf items (kBins = 2^kLog mask bins cover s <= kLog
  // members): a neighbour equal to a member is no leaf, and an entry whose
  // first traversal neighbour is tr[f] is canonical above sufmax[s][f].
  constexpr int kLog = (kBins == 16 ? 4 : (kBins == 32 ? 5 : 6));
  static_assert((1 << kLog) == kBins, "one mask bit per traversal member");
  int trr[kLog];
#pragma unroll
  for (int t = 0; t < kLog; ++t) trr[t] = t < s ? uni(L.tr[t]) : -1;
  auto in_tr_r = [&](int w) {
    bool r = false;
#pragma unroll
    for (int t = 0; t < kLog; ++t) r = r || w == trr[t];
    return r;
  };
  int thr[kLog];
#pragma unroll
  for (int t = 0; t < kLog; ++t) thr[t] = t < s ? uni(L.sufmax[s * kSuf + t]) : 0x7fffffff;
  auto canon_r = [&](int y, unsigned mm) {
    const unsigned lw = mm & low;
    int th = 0x7fffffff;
#pragma unroll
    for (int t = kLog - 1; t >= 0; --t)
      if ((lw >> t) & 1u) th = thr[t];
    return y > v0 && y > th;
  };
  for (int c = lo; c < hi; c += kWave) {
    // ---- slice: canonical entries and a prefix sum of their degrees
    const int j = c + lane;
    const bool in = j < hi;
    const int x = in ? ev_at(j) : 0;
    const unsigned m = in ? em_at(j) : 0u;
    const bool ok = in && canonical(L, s, x, m);
    const int64_t xb = ok ? A.rp[x] : 0;
    const int64_t dx = ok ? A.rp[x + 1] - xb : 0;
    const int64_t incl = wave_incl_scan_i64(dx);
    const int64_t total = static_cast<int64_t>(__shfl(static_cast<long long>(incl), kWave - 1, kWave));
    L.sl_start[lane] = incl - dx;
    L.sl_base[lane] = xb;
    L.sl_mask[lane] = static_cast<int>(m & low);
    const uint64_t okb = ballot(ok);
    if (lane == 0) {
      L.sl_start[kWave] = total;
      nodes_l += static_cast<uint64_t>(__popcll(okb));
      reads_l += static_cast<uint64_t>(total);
    }
    wave_sync();
    // ---- every (x, neighbour) item of the slice, 64 at a time.  The owner of
    // item f0 + lane is the last slice lane whose degree range starts at or
    // before it: lanes starting inside the batch mark their first item, and a
    // prefix maximum over the marks (seeded with the owner of f0) assigns them.
    const int64_t my_start = incl - dx;
    const bool my_has = dx > 0;
    // owner of item fb + lane (all lanes active)
    auto owner_of = [&](int64_t fb) -> int {
      const uint64_t le = ballot(my_has && my_start <= fb);
      const int ob = le ? 63 - __builtin_clzll(le) : 0;
      L.mark[lane] = -1;
      wave_sync();
      if (my_has && my_start > fb && my_start < fb + kWave) L.mark[my_start - fb] = lane;
      wave_sync();
      int o = wave_incl_max_i32(L.mark[lane]);
      o = o > ob ? o : ob;
      return o < kWave - 1 ? o : kWave - 1;
    };
    // key of neighbour w of the x at slice lane o (-1: no leaf)
    auto classify = [&](int w, int o) -> int {
      int key = -1;
      const int f = filt_index(w, !in_lds);
      bool maybe = (L.filt[f >> 5] >> (f & 31)) & 1u;
      if (!in_lds) maybe = maybe && ((bigf[(w >> 5) & (kBigFilterWords - 1)] >> (w & 31)) & 1u);
      if (w > v0) {
        const int jj = maybe ? ev_find(w) : -1;
        if (jj >= 0) {
          const unsigned mj = em_at(jj);
          if (jj > c + o && canon_r(w, mj)) key = L.sl_mask[o] * kBins + static_cast<int>(mj & low);
        } else if (!in_tr_r(w)) {
          key = kBins * kBins + L.sl_mask[o];
        }
      }
      return key;
    };
    auto aggregate = [&](int key) {
      uint64_t act = ballot(key >= 0);
      while (act) {
        const int l = __ffsll(static_cast<long long>(act)) - 1;
        const int kk = read_lane(key, l);
        const uint64_t same = ballot(key == kk);
        if (lane == 0) {
          if (kk < kBins * kBins) L.adj[kk] += static_cast<unsigned long long>(__popcll(same));
          else L.nw[kk - kBins * kBins] += static_cast<unsigned long long>(__popcll(same));
        }
        act &= ~same;
      }
    };
    // three items per lane and pass, their adjacency reads in flight together
    for (int64_t f0 = 0; f0 < total; f0 += 3 * kWave) {
      const int oa = owner_of(f0);
      const int ob = owner_of(f0 + kWave);
      const int oc = owner_of(f0 + 2 * kWave);
      const int64_t fa = f0 + lane, fb = f0 + kWave + lane, fc = f0 + 2 * kWave + lane;
      const int wa = fa < total ? A.col[L.sl_base[oa] + (fa - L.sl_start[oa])] : -1;
      const int wb = fb < total ? A.col[L.sl_base[ob] + (fb - L.sl_start[ob])] : -1;
      const int wc = fc < total ? A.col[L.sl_base[oc] + (fc - L.sl_start[oc])] : -1;
      const int ka = fa < total ? classify(wa, oa) : -1;
      const int kb = fb < total ? classify(wb, ob) : -1;
      const int kc = fc < total ? classify(wc, oc) : -1;
      aggregate(ka);
      aggregate(kb);
      aggregate(kc);
    }
    wave_sync();
    // ---- donation of the untried x range
    const int next = c + kWave;
    if (A.S.donate && hi - next >= kLeafDonateMin && sched_want_donation(A.S)) {
      const int mid = next + (hi - next + 1) / 2;
      const int pay = task_payload(t.root, t.stat, s, mid, hi, L.tr);
      if (sched_publish(A.S, pay, wave_gid)) hi = mid;
      wave_sync();
    }
  }
  // ---- canonical entries per mask over [lo, hi) and [hi, |E|)
  for (int c = lo; c < ns; c += kWave) {
    const int j = c + lane;
    const bool ok = j < ns && canonical(L, s, ev_at(j), em_at(j));
    const int key = ok ? static_cast<int>(em_at(j) & low) + (j >= hi ? kBins : 0) : -1;
    uint64_t act = ballot(ok);
    while (act) {
      const int l = __ffsll(static_cast<long long>(act)) - 1;
      const int kk = read_lane(key, l);
      const uint64_t same = ballot(key == kk);
      if (lane == 0) L.ccount[kk] += static_cast<unsigned>(__popcll(same));
      act &= ~same;
    }
  }
  wave_sync();
  // ---- clear the filter words this list set (all of them for a global list)
  if (in_lds)
    for (int i = lane; i < ns; i += kWave) L.filt[filt_index(L.ev[i], false) >> 5] = 0u;
  else
    for (int i = lane; i < kFilterWords; i += kWave) L.filt[i] = 0u;
  // ---- one dictionary lookup per non-empty bin
  const int code_tr = L.code[s];
  const int fx = s >= 2 ? off_of(s) : 0;  // v_1's field is implied
  const int fy = off_of(s + 1);
  unsigned long long* cnt = class_counters<kBins>(L, MW);
  auto add_class = [&](int code, uint64_t h) {
    const int cls = A.table[code];
    if (cls == kUnreachable) {
      atomicOr(A.flags + 1, 2);
    } else {
      const unsigned long long old = atomicAdd(&cnt[cls], static_cast<unsigned long long>(h));
      if (old + h < old) MW.ovf = 1;
    }
    leaves_l += h;
  };
  for (int idx = lane; idx < nm * nm + nm; idx += kWave) {
    if (idx < nm * nm) {
      const int a = idx / nm, b = idx % nm;
      if (a == 0 || a > b) continue;
      const uint64_t hia = L.ccount[kBins + a], hib = L.ccount[kBins + b];
      const uint64_t ca = L.ccount[a] + hia, cb = L.ccount[b] + hib;
      const uint64_t pairs = a == b ? ca * (ca - 1) / 2 - hia * (hia - 1) / 2 : ca * cb - hia * hib;
      const uint64_t adj = a == b ? L.adj[a * kBins + a] : L.adj[a * kBins + b] + L.adj[b * kBins + a];
      const int base = code_tr | (s >= 2 ? a << fx : 0);
      if (pairs - adj) add_class(base | (b << fy), pairs - adj);
      if (adj) add_class(base | ((b | nm) << fy), adj);
    } else {
      const int a = idx - nm * nm;
      const uint64_t h = a ? static_cast<uint64_t>(L.nw[a]) : 0;
      if (h) add_class(code_tr | (s >= 2 ? a << fx : 0) | (nm << fy), h);
    }
  }
  wave_sync();
  return hi;
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

template <int kBins, bool kHostBal>
__device__ __forceinline__ void run_task(const MotifArgs& A, const MotifLds& L, MotifWave& MW, const Task& t, int wave_gid) {
  const int lane = lane_id();
  const int k = A.k;
  const int v0 = t.root;
  const int g = A.root_graph ? A.root_graph[v0] : 0;
  if (g != MW.cur_g) {
    flush_counts<kBins>(A, L, MW);
    MW.cur_g = g;
  }
  uint64_t nodes_l = 0, leaves_l = 0, reads_l = 0;
  // ---- level 1: the neighbours of v0 above v0 (a suffix of its sorted list)
  const int64_t b0 = A.rp[v0];
  const int d0 = static_cast<int>(A.rp[v0 + 1] - b0);
  const int skip = uni(lower_bound_g(A.col + b0, d0, v0 + 1));
  {
    int32_t* E1 = MW.vert + A.level_off[1];
    uint8_t* M1 = MW.mask + A.level_off[1];
    for (int i = lane; i < d0 - skip; i += kWave) {
      E1[i] = A.col[b0 + skip + i];
      M1[i] = 1;
    }
    if (lane == 0) {
      L.esize[1] = d0 - skip;
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

  if (s0 == k - 2) {
    leaf_level<kBins>(A, L, MW, s0, t.lo, hi0, t, wave_gid, nodes_l, leaves_l, reads_l);
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
        leaf_level<kBins>(A, L, MW, s + 1, 0, L.esize[s + 1], t, wave_gid, nodes_l, leaves_l, reads_l);
      } else {
        ++s;
        if (lane == 0) { L.cursor[s] = 0; L.endv[s] = L.esize[s]; }
        wave_sync();
      }
      // ---- host-driven balancing: once the launch is stopped, the untried
      // extensions of every open level become tasks for the next launch
      if (kHostBal) {
        if ((++steps % A.S.period) == 0 && sched_stopped(A.S)) {
          for (int q = s0; q <= s; ++q) {
            const int from = L.cursor[q], to = L.endv[q];
            if (to > from) sched_spill(A.S, task_payload(v0, t.stat, q, from, to, L.tr));
          }
          break;
        }
      } else if (A.S.donate && (++steps % A.S.period) == 0 && sched_want_donation(A.S)) {
        // ---- donation of untried extensions at the shallowest level
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

// 4 waves per SIMD (128 VGPRs): enough waves to cover the lookups' latency.
// kHostBal: the instantiation for launches under host-driven balancing.
template <int kBins, bool kHostBal>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) motif_kernel(MotifArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int wave_gid = blockIdx.x;
  MotifLds L = carve<kBins>(smem, A.ncls);
  MotifWave MW;
  MW.cur_g = -1;
  MW.ovf = 0;
  MW.nodes = 0;
  MW.tasks = 0;
  MW.vert = A.ext_vert + static_cast<size_t>(wave_gid) * A.wave_ext_cap;
  MW.mask = A.ext_mask + static_cast<size_t>(wave_gid) * A.wave_ext_cap;
  MW.nbuf = A.new_buf + static_cast<size_t>(wave_gid) * A.dmax;
  MW.gcnt = A.wave_cnt ? A.wave_cnt + static_cast<size_t>(wave_gid) * A.ncls : nullptr;
  {
    unsigned long long* cnt = class_counters<kBins>(L, MW);
    for (int c = lane; c < A.ncls; c += kWave) cnt[c] = 0;
  }
  for (int c = lane; c < kFilterWords; c += kWave) L.filt[c] = 0u;
  wave_sync();
  const uint64_t t_begin = wall_clock64();
  SchedIter it;
  sched_begin(A.S, it);
  Task t;
  while (sched_next<kHostBal>(A.S, it, wave_gid, L.tr, &t)) {
    run_task<kBins, kHostBal>(A, L, MW, t, wave_gid);
    MW.tasks++;
  }
  sched_end<kHostBal>(A.S);
  const uint64_t t_idle = it.t_idle;
  flush_counts<kBins>(A, L, MW);
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

// ---------------------------------------------------------------- listing (aggregate_store)

// Every connected induced k-subgraph rooted at t.root, handed to the ring as
// (traversal order vertices, class id): the upper levels are the counting
// kernel's extension steps, carried down to |tr| = k-1, where each canonical
// entry y of the list completes one k-subgraph whose pattern is the
// traversal's code plus y's mask in v_{k-1}'s field (Section IV-C bitmap).
__device__ bool list_task(const MotifArgs& A, const Ring& R, const MotifLds& L, MotifWave& MW, const Task& t) {
  const int lane = lane_id();
  const int k = A.k;
  const int v0 = t.root;
  const int64_t b0 = A.rp[v0];
  const int d0 = static_cast<int>(A.rp[v0 + 1] - b0);
  const int skip = uni(lower_bound_g(A.col + b0, d0, v0 + 1));
  {
    int32_t* E1 = MW.vert + A.level_off[1];
    uint8_t* M1 = MW.mask + A.level_off[1];
    for (int i = lane; i < d0 - skip; i += kWave) {
      E1[i] = A.col[b0 + skip + i];
      M1[i] = 1;
    }
    if (lane == 0) {
      L.esize[1] = d0 - skip;
      L.tr[0] = v0;
      L.code[1] = 0;
      L.sufmax[1 * kSuf + 0] = -1;
      L.cursor[1] = 0;
      L.endv[1] = d0 - skip;
    }
  }
  wave_sync();
  int s = 1;
  for (;;) {
    if (s == k - 1) {
      const int32_t* E = MW.vert + A.level_off[s];
      const uint8_t* Em = MW.mask + A.level_off[s];
      const int ns = L.esize[s];
      const unsigned low = (1u << s) - 1u;
      for (int c = 0; c < ns; c += kWave) {
        const int j = c + lane;
        const int y = j < ns ? E[j] : 0;
        const unsigned m = j < ns ? Em[j] : 0u;
        const bool ok = j < ns && canonical(L, s, y, m);
        int cls = 0;
        if (ok) {
          cls = A.table[L.code[s] | static_cast<int>((m & low) << off_of(s))];
          if (cls == kUnreachable) atomicOr(A.flags + 1, 2);
        }
        const uint64_t bl = ballot(ok);
        if (ok) {
          L.mark[mbcnt(bl)] = y;
          L.sl_mask[mbcnt(bl)] = cls;
        }
        wave_sync();
        const int cnt = __popcll(bl);
        if (cnt) {
          const int yy = lane < cnt ? L.mark[lane] : 0;
          const int cc = lane < cnt ? L.sl_mask[lane] : 0;
          if (!ring_emit(R, L.tr, k - 1, yy, cc, cnt)) return false;
        }
        wave_sync();
      }
      if (s == 1) break;
      --s;
      continue;
    }
    const int idx = next_canonical(A, L, MW, s, L.cursor[s], L.endv[s]);
    if (idx < 0) {
      if (s == 1) break;
      --s;
      continue;
    }
    const int x = MW.vert[A.level_off[s] + idx];
    if (lane == 0) L.cursor[s] = idx + 1;
    extend_level(A, L, MW, s, idx, x);
    ++s;
    if (lane == 0) {
      L.cursor[s] = 0;
      L.endv[s] = L.esize[s];
    }
    wave_sync();
  }
  return true;
}

__global__ void __launch_bounds__(64) list_motifs_kernel(MotifArgs A, Ring R) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave_gid = blockIdx.x;
  MotifLds L = carve<16>(smem, 1);
  MotifWave MW;
  MW.cur_g = -1;
  MW.ovf = 0;
  MW.nodes = 0;
  MW.tasks = 0;
  MW.vert = A.ext_vert + static_cast<size_t>(wave_gid) * A.wave_ext_cap;
  MW.mask = A.ext_mask + static_cast<size_t>(wave_gid) * A.wave_ext_cap;
  MW.nbuf = A.new_buf + static_cast<size_t>(wave_gid) * A.dmax;
  MW.gcnt = nullptr;
  SchedIter it;
  sched_begin(A.S, it);
  Task t;
  bool ok = true;
  while (ok && sched_next(A.S, it, wave_gid, L.tr, &t)) ok = list_task(A, R, L, MW, t);
  sched_end(A.S);
}

}  // namespace

int motif_bins(int k) { return k <= 6 ? 16 : (k == 7 ? 32 : 64); }

size_t motif_lds_bytes(int k, int ncls) {
  const size_t nb = static_cast<size_t>(motif_bins(k));
  auto a16 = [](size_t x) { return (x + 15) & ~static_cast<size_t>(15); };
  size_t off = (nb == 64 ? 0 : a16(static_cast<size_t>(ncls) * 8)) + a16(nb * nb * 8) + a16(nb * 8) + a16(2 * nb * 4);
  off += a16((kWave + 1) * 8) + a16(kWave * 8) + a16(kWave * 4);
  off += 2 * a16(kSuf * 4) + a16(kSuf * kSuf * 4) + 3 * a16(kSuf * 4);
  off += a16(kLeafLds * 4) + a16(kLeafLds) + a16(kFilterWords * 4) + 16 + a16(kWave * 4);
  off += a16((kBuckets + 1) * 2);
  return off;
}

hipError_t motif_occupancy(int k, size_t lds_bytes, int* blocks_per_cu) {
  switch (motif_bins(k)) {
    case 16: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, motif_kernel<16, false>, 64, lds_bytes);
    case 32: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, motif_kernel<32, false>, 64, lds_bytes);
    default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, motif_kernel<64, false>, 64, lds_bytes);
  }
}

size_t motif_list_lds_bytes() { return motif_lds_bytes(3, 1); }

hipError_t launch_list_motifs(const MotifArgs& a, const Ring& R, int grid, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(list_motifs_kernel, dim3(grid), dim3(64), lds_bytes, s, a, R);
  return hipGetLastError();
}

hipError_t launch_motif(const MotifArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
  const bool hb = a.S.host_bal != 0;
  switch (motif_bins(a.k)) {
    case 16:
      if (hb) hipLaunchKernelGGL((motif_kernel<16, true>), dim3(grid), dim3(64), lds_bytes, s, a);
      else hipLaunchKernelGGL((motif_kernel<16, false>), dim3(grid), dim3(64), lds_bytes, s, a);
      break;
    case 32:
      if (hb) hipLaunchKernelGGL((motif_kernel<32, true>), dim3(grid), dim3(64), lds_bytes, s, a);
      else hipLaunchKernelGGL((motif_kernel<32, false>), dim3(grid), dim3(64), lds_bytes, s, a);
      break;
    default:
      if (hb) hipLaunchKernelGGL((motif_kernel<64, true>), dim3(grid), dim3(64), lds_bytes, s, a);
      else hipLaunchKernelGGL((motif_kernel<64, false>), dim3(grid), dim3(64), lds_bytes, s, a);
  }
  return hipGetLastError();
}

}  // namespace dm

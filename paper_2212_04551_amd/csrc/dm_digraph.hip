// Directed graphs.  The method is stated for undirected graphs and said to
// carry over to directed ones (DuMato, Section II); here a digraph is handled
// through its underlying undirected graph, which drives the enumeration
// (connected induced k-subgraphs are the weakly connected ones), plus two arc
// bits per undirected adjacency entry, which drive the classification:
//
//   - Loading: the arcs (sorted out-lists) are validated, their in-lists built
//     by a radix sort of (head, tail) keys, and every vertex's out- and
//     in-list merged into its undirected list; entry (u, w) carries
//     dir = [u->w] | [w->u] << 1.
//   - Directed motif counting (k = 3..5): on the graph renamed by (degree,
//     id) rank, one wave per root extends the traversal with the
//     canonical-candidate rule of Section IV-E over the undirected lists,
//     keeping for every list entry its undirected adjacency mask over the
//     traversal and two arc bits per traversal vertex.  The
//     directed pattern code of Section IV-C's bitmap takes two bits per vertex
//     pair.  Once |tr| = k-2, each canonical x and every canonical y of the
//     extension set that x's step would build complete one subgraph, counted
//     without building that set; its class comes from a dictionary over all
//     2^(k(k-1)) codes.
#include <hipcub/hipcub.hpp>

#include "dm_internal.hpp"

namespace dm {

namespace {

inline unsigned nblocks(int64_t count, int threads) {
  int64_t b = (count + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > (int64_t{1} << 30)) b = int64_t{1} << 30;
  return static_cast<unsigned>(b);
}

inline int key_bits(int64_t x) {
  int b = 1;
  while (b < 62 && (int64_t{1} << b) <= x) ++b;
  return b;
}

// flag bits: 1 bad offsets, 2 id out of range, 4 self-arc, 8 out-list not
// strictly ascending (or a repeated arc)
__global__ void __launch_bounds__(256) arc_validate_kernel(const int64_t* rp, const int32_t* col, int32_t n,
                                                           int64_t arcs, int* flag) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v == 0 && (rp[0] != 0 || rp[n] != arcs)) atomicOr(flag, 1);
  if (v >= n) return;
  const int64_t b = rp[v], e = rp[v + 1];
  if (b < 0 || e < b || e > arcs) {
    atomicOr(flag, 1);
    return;
  }
  int bad = 0;
  for (int64_t i = b; i < e; ++i) {
    const int32_t u = col[i];
    if (u < 0 || u >= n) bad |= 2;
    if (u == v) bad |= 4;
    if (i > b && col[i - 1] >= u) bad |= 8;
  }
  if (bad) atomicOr(flag, bad);
}

// key (head << 32 | tail) of every arc tail -> head
__global__ void __launch_bounds__(256) arc_key_kernel(const int64_t* rp, const int32_t* col, int32_t n,
                                                      unsigned long long* keys) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  for (int64_t i = rp[v]; i < rp[v + 1]; ++i)
    keys[i] = (static_cast<unsigned long long>(static_cast<uint32_t>(col[i])) << 32) | static_cast<uint32_t>(v);
}

// in-lists from the sorted keys: irp[v] = first key with head v; icol = tails
__global__ void __launch_bounds__(256) in_lists_kernel(const unsigned long long* keys, int64_t arcs, int32_t n,
                                                       int64_t* irp, int32_t* icol) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < arcs) icol[i] = static_cast<int32_t>(keys[i] & 0xffffffffull);
  if (i <= n) {
    const unsigned long long want = static_cast<unsigned long long>(i) << 32;
    int64_t lo = 0, hi = arcs;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < want) lo = mid + 1; else hi = mid;
    }
    irp[i] = lo;
  }
}

// Merge of v's out-list and in-list (both ascending): with `fill`, writes the
// union into ucol / udir from urp[v]; otherwise stores its length in udeg[v].
template <bool kFill>
__global__ void __launch_bounds__(256) union_kernel(const int64_t* rp, const int32_t* col, const int64_t* irp,
                                                    const int32_t* icol, int32_t n, int64_t* udeg, const int64_t* urp,
                                                    int32_t* ucol, uint8_t* udir) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int64_t a = rp[v], ae = rp[v + 1], b = irp[v], be = irp[v + 1];
  int64_t o = kFill ? urp[v] : 0, cnt = 0;
  while (a < ae || b < be) {
    const int32_t x = a < ae ? col[a] : INT32_MAX;
    const int32_t y = b < be ? icol[b] : INT32_MAX;
    const int32_t w = x < y ? x : y;
    uint8_t d = 0;
    if (x == w) { d |= 1; ++a; }
    if (y == w) { d |= 2; ++b; }
    if (kFill) {
      ucol[o + cnt] = w;
      udir[o + cnt] = d;
    }
    ++cnt;
  }
  if (!kFill) udeg[v] = cnt;
}

// The arc bits of every entry at its place in the rank-renamed graph: row
// rank[u], the entry of rank[w] (renaming keeps the pair's orientation, so
// the bits are unchanged).
__global__ void rank_dir_kernel(const int64_t* rp, const int32_t* col, const uint8_t* dir, int32_t n,
                                const int32_t* rank, const int64_t* urp, const int32_t* ucol, uint8_t* udir,
                                int* flag) {
  const int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int ru = rank[u];
  const int64_t b = urp[ru];
  const int len = static_cast<int>(urp[ru + 1] - b);
  for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
    const int rw = rank[col[e]];
    int lo = 0, hi = len;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ucol[b + mid] < rw) lo = mid + 1; else hi = mid;
    }
    if (lo < len && ucol[b + lo] == rw) udir[b + lo] = dir[e];
    else atomicOr(flag, 1);  // the renamed graph lacks the entry
  }
}

}  // namespace

hipError_t digraph_rank_dir(const int64_t* rp, const int32_t* col, const uint8_t* dir, int32_t n, const int32_t* rank,
                            const int64_t* urp, const int32_t* ucol, uint8_t* udir, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_dir_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, rp, col, dir, n, rank, urp, ucol, udir,
                     flag);
  return hipGetLastError();
}

#define DG_TRY(x)                          \
  do {                                     \
    err = (x);                             \
    if (err != hipSuccess) goto done;      \
  } while (0)

hipError_t launch_arc_validate(const int64_t* rp, const int32_t* col, int32_t n, int64_t arcs, int* flag,
                               hipStream_t s) {
  hipLaunchKernelGGL(arc_validate_kernel, dim3(nblocks(static_cast<int64_t>(n) + 1, 256)), dim3(256), 0, s, rp, col,
                     n, arcs, flag);
  return hipGetLastError();
}

hipError_t digraph_underlying(const int64_t* rp, const int32_t* col, int32_t n, int64_t arcs, int64_t** urp_out,
                              int32_t** ucol_out, uint8_t** udir_out, int64_t* unnz_out, hipStream_t s) {
  hipError_t err = hipSuccess;
  unsigned long long *keys = nullptr, *keys2 = nullptr;
  int64_t *irp = nullptr, *udeg = nullptr, *urp = nullptr;
  int32_t *icol = nullptr, *ucol = nullptr;
  uint8_t* udir = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0, need = 0;
  int64_t unnz = 0;
  const int64_t ak = arcs > 0 ? arcs : 1;
  *urp_out = nullptr;
  *ucol_out = nullptr;
  *udir_out = nullptr;
  *unnz_out = 0;
  DG_TRY(hipMalloc(&keys, sizeof(unsigned long long) * ak));
  DG_TRY(hipMalloc(&keys2, sizeof(unsigned long long) * ak));
  DG_TRY(hipMalloc(&irp, sizeof(int64_t) * (static_cast<size_t>(n) + 1)));
  DG_TRY(hipMalloc(&icol, sizeof(int32_t) * ak));
  DG_TRY(hipMalloc(&udeg, sizeof(int64_t) * (static_cast<size_t>(n) + 1)));
  DG_TRY(hipMalloc(&urp, sizeof(int64_t) * (static_cast<size_t>(n) + 1)));
  DG_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, need, keys, keys2, static_cast<int>(ak), 0, 64, s));
  temp_bytes = need;
  DG_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, need, udeg, urp, n + 1, s));
  if (need > temp_bytes) temp_bytes = need;
  DG_TRY(hipMalloc(&temp, temp_bytes > 0 ? temp_bytes : 16));
  if (arcs > 0) {
    hipLaunchKernelGGL(arc_key_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, rp, col, n, keys);
    DG_TRY(hipGetLastError());
    need = temp_bytes;
    DG_TRY(hipcub::DeviceRadixSort::SortKeys(temp, need, keys, keys2, static_cast<int>(arcs), 0, 32 + key_bits(n), s));
  }
  hipLaunchKernelGGL(in_lists_kernel, dim3(nblocks((arcs > n ? arcs : static_cast<int64_t>(n)) + 1, 256)), dim3(256),
                     0, s, keys2, arcs, n, irp, icol);
  DG_TRY(hipGetLastError());
  hipLaunchKernelGGL(union_kernel<false>, dim3(nblocks(n, 256)), dim3(256), 0, s, rp, col, irp, icol, n, udeg,
                     nullptr, nullptr, nullptr);
  DG_TRY(hipGetLastError());
  DG_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(udeg + n), 1, 0ull, s));
  need = temp_bytes;
  DG_TRY(hipcub::DeviceScan::ExclusiveSum(temp, need, udeg, urp, n + 1, s));
  DG_TRY(hipMemcpyAsync(&unnz, urp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DG_TRY(hipStreamSynchronize(s));
  DG_TRY(hipMalloc(&ucol, sizeof(int32_t) * static_cast<size_t>(unnz > 0 ? unnz : 1)));
  DG_TRY(hipMalloc(&udir, static_cast<size_t>(unnz > 0 ? unnz : 1)));
  hipLaunchKernelGGL(union_kernel<true>, dim3(nblocks(n, 256)), dim3(256), 0, s, rp, col, irp, icol, n, nullptr, urp,
                     ucol, udir);
  DG_TRY(hipGetLastError());
  DG_TRY(hipStreamSynchronize(s));
  *urp_out = urp;
  *ucol_out = ucol;
  *udir_out = udir;
  *unnz_out = unnz;
  urp = nullptr;
  ucol = nullptr;
  udir = nullptr;
done:
  (void)hipFree(keys);
  (void)hipFree(keys2);
  (void)hipFree(irp);
  (void)hipFree(icol);
  (void)hipFree(udeg);
  (void)hipFree(urp);
  (void)hipFree(ucol);
  (void)hipFree(udir);
  (void)hipFree(temp);
  return err;
}

// ---------------------------------------------------------------- directed motif counting

namespace {

constexpr int kDSlots = kDMotifMaxK + 1;
constexpr int kDMaxWaves = 8;  // waves per workgroup
static_assert(kDMaxWaves == 8, "the launch planner tries 1, 2, 4 and 8 waves per workgroup");
// LDS-typed view of a pointer into the workgroup's LDS (its reads and
// writes are then LDS instructions, not generic ones)
typedef __attribute__((address_space(3))) uint64_t LdsU64d;

// An entry of the LDS level list in one word: vertex (bits 0-31), arc bits
// (32-47), undirected mask (48-55), so one read brings all three.
__device__ __forceinline__ uint64_t dpack(int v, unsigned arcs, unsigned mask) {
  return static_cast<uint32_t>(v) | (static_cast<uint64_t>(arcs & 0xffffu) << 32) |
         (static_cast<uint64_t>(mask & 0xffu) << 48);
}
__device__ __forceinline__ int dp_v(uint64_t w) { return static_cast<int>(static_cast<uint32_t>(w)); }
__device__ __forceinline__ unsigned dp_a(uint64_t w) { return static_cast<unsigned>(w >> 32) & 0xffffu; }
__device__ __forceinline__ unsigned dp_m(uint64_t w) { return static_cast<unsigned>(w >> 48) & 0xffu; }

// The workgroup's waves run independent traversals (they share only the class
// counters), so lanes of one wave order their LDS and memory traffic with a
// fence pair and no workgroup barrier.  The fences take workgroup scope: a
// lane's stores (LDS and the level lists in HBM) complete before another
// lane of the wave reads them, whatever the memory system does with one
// wave's accesses in flight.
__device__ __forceinline__ void dsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct DLds {
  int* tr;        // [kDSlots] traversal
  int* dcode;     // [kDSlots] directed code of tr[0..s-1] per size s
  int* sufmax;    // [kDSlots][kDSlots] max of tr[f+1..s-1] per size s
  int* cursor;    // [kDSlots]
  int* endv;      // [kDSlots]
  int* esize;     // [kDSlots]
  int* meta;      // [4] [1]: the level k-2 list is in lp; [2], [3]: its bucket base and shift
  int* bk;        // [kDBuckets + 1] bucket b = entries in [base + (b << shift), base + ((b + 1) << shift))
  uint64_t* lp;   // [leaf_cap] level k-2 list in LDS when it has at most leaf_cap entries, packed
  uint8_t* lhit;  // [leaf_cap] marks of the entries an x step touches
  unsigned* cnt;  // [ncls] class counters since the last flush
};

constexpr int kDBuckets = 64;
// (an even count, so the packed list after them is 8-byte aligned)
constexpr int kDLdsInts = (3 * kDSlots + kDSlots * kDSlots + 3 * kDSlots + 4 + kDBuckets + 1 + 1) & ~1;

// per-wave bytes: the traversal state and the LDS level list
__host__ __device__ constexpr size_t dwave_lds_bytes(int leaf_cap) {
  return kDLdsInts * sizeof(int) + static_cast<size_t>(leaf_cap) * (8 + 1);
}

// Wave wid's part of the workgroup's LDS; the class counters after the
// nw waves' parts are shared by the workgroup.
__device__ DLds dcarve(unsigned char* smem, int leaf_cap, int wid, int nw) {
  DLds L;
  int* p = reinterpret_cast<int*>(smem + wid * dwave_lds_bytes(leaf_cap));
  L.tr = p;
  L.dcode = p + kDSlots;
  L.sufmax = p + 2 * kDSlots;
  L.cursor = L.sufmax + kDSlots * kDSlots;
  L.endv = L.cursor + kDSlots;
  L.esize = L.endv + kDSlots;
  L.meta = L.esize + kDSlots;
  L.bk = L.meta + 4;
  L.lp = reinterpret_cast<uint64_t*>(p + kDLdsInts);
  L.lhit = reinterpret_cast<uint8_t*>(L.lp + leaf_cap);
  L.cnt = reinterpret_cast<unsigned*>(smem + nw * dwave_lds_bytes(leaf_cap));
  return L;
}

__device__ __forceinline__ int lower_bound_i32(const int32_t* a, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// A list entry y with undirected mask m (bit t: adjacent to tr[t]) at
// traversal size s is a canonical extension (Section IV-E) when y is above
// the root and above every traversal vertex after its first neighbour in tr.
__device__ __forceinline__ bool dcanonical(const DLds& L, int s, int y, unsigned m) {
  const unsigned low = m & ((1u << s) - 1u);
  if (low == 0) return false;
  const int f = __builtin_ctz(low);
  return y > L.tr[0] && y > L.sufmax[s * kDSlots + f];
}

struct DWave {
  int32_t* vert;   // level lists: vertex
  uint8_t* mask;   // undirected adjacency mask over tr
  uint16_t* arcs;  // two arc bits per traversal position (bit 2t: tr[t] -> y, bit 2t+1: y -> tr[t])
  uint8_t* hit;    // per old entry during an extension: 0x80 | dir of (x, entry)
  int32_t* nbuf;   // new entries of an extension
  uint8_t* ndir;
};

// Bucket index over the LDS level list (sorted ids, ns entries): the ids
// from its first to its last split into kDBuckets ranges of 2^shift, bk[b]
// the first entry of range b, so a search starts in about ns / kDBuckets
// entries instead of ns.
__device__ void dbuckets(const DLds& L, int ns) {
  const int lane = lane_id();
  dsync();
  const LdsU64d* lp = (const LdsU64d*)(L.lp);
  const int lo = ns > 0 ? dp_v(lp[0]) : 0;
  const int span = ns > 0 ? dp_v(lp[ns - 1]) - lo : 0;
  int sh = 0;
  while ((span >> sh) >= kDBuckets) ++sh;
  for (int b = lane; b <= kDBuckets; b += kWave) {
    const int64_t key = static_cast<int64_t>(lo) + (static_cast<int64_t>(b) << sh);
    int a = 0, e = ns;
    while (a < e) {
      const int mid = (a + e) >> 1;
      if (dp_v(lp[mid]) < key) a = mid + 1; else e = mid;
    }
    L.bk[b] = a;
  }
  if (lane == 0) {
    L.meta[2] = lo;
    L.meta[3] = sh;
  }
  dsync();
}

// Level s+1 from level s by appending the entry at index px (vertex x).
__device__ void dextend(const DMotifArgs& A, const DLds& L, const DWave& W, int s, int px, int x) {
  const int lane = lane_id();
  const int32_t* Ev = W.vert + A.level_off[s];
  const uint8_t* Em = W.mask + A.level_off[s];
  const uint16_t* Ea = W.arcs + A.level_off[s];
  const int ns = L.esize[s];
  const int64_t xb = A.rp[x];
  const int dx = static_cast<int>(A.rp[x + 1] - xb);
  const int v0 = L.tr[0];
  int nn = 0;
  for (int c = 0; c < dx; c += kWave) {
    const int i = c + lane;
    const bool ok = i < dx && A.col[xb + i] > v0;
    const int w = ok ? A.col[xb + i] : 0;
    const uint8_t d = ok ? A.dir[xb + i] : 0;
    const int j = ok ? lower_bound_i32(Ev, ns, w) : ns;
    const bool found = ok && j < ns && Ev[j] == w;
    if (found && j != px) W.hit[j] = static_cast<uint8_t>(0x80u | d);
    bool intr = false;
    for (int t = 0; t < s; ++t) intr |= (L.tr[t] == w);
    const bool isnew = ok && !found && !intr;
    const uint64_t b = ballot(isnew);
    if (isnew) {
      const int pos = nn + mbcnt(b);
      if (pos < A.dmax) {
        W.nbuf[pos] = w;
        W.ndir[pos] = d;
      }
    }
    nn += __popcll(b);
  }
  nn = uni(nn);
  if (nn > A.dmax) {
    if (lane == 0) atomicOr(A.flags + 1, 1);
    nn = A.dmax;
  }
  const bool to_lds = s + 1 == A.k - 2 && static_cast<int64_t>(ns) - 1 + nn <= A.leaf_cap;
  int32_t* Nv = W.vert + A.level_off[s + 1];
  uint8_t* Nm = W.mask + A.level_off[s + 1];
  uint16_t* Na = W.arcs + A.level_off[s + 1];
  LdsU64d* Np = (LdsU64d*)(L.lp);
  const int64_t cap = to_lds ? A.leaf_cap : A.level_cap[s + 1];
  dsync();
  // both parts are sorted by id: every entry's place is its rank in the other part
  for (int j = lane; j < ns; j += kWave) {
    if (j == px) continue;
    const int y = Ev[j];
    const unsigned h = W.hit[j];
    const int r = lower_bound_i32(W.nbuf, nn, y);
    const int64_t out = static_cast<int64_t>(j) - (j > px ? 1 : 0) + r;
    if (out < cap) {
      const unsigned m = Em[j] | ((h & 0x80u) ? (1u << s) : 0u);
      const unsigned a = Ea[j] | ((h & 3u) << (2 * s));
      if (to_lds) {
        Np[out] = dpack(y, a, m);
      } else {
        Nv[out] = y;
        Nm[out] = static_cast<uint8_t>(m);
        Na[out] = static_cast<uint16_t>(a);
      }
    }
    if (h) W.hit[j] = 0;
  }
  for (int i = lane; i < nn; i += kWave) {
    const int w = W.nbuf[i];
    int r = lower_bound_i32(Ev, ns, w);
    if (px < r) r -= 1;
    const int64_t out = static_cast<int64_t>(i) + r;
    if (out < cap) {
      const unsigned a = (W.ndir[i] & 3u) << (2 * s);
      if (to_lds) {
        Np[out] = dpack(w, a, 1u << s);
      } else {
        Nv[out] = w;
        Nm[out] = static_cast<uint8_t>(1u << s);
        Na[out] = static_cast<uint16_t>(a);
      }
    }
  }
  int64_t nsz = static_cast<int64_t>(ns) - 1 + nn;
  if (nsz > cap) {
    if (lane == 0) atomicOr(A.flags + 1, 1);
    nsz = cap;
  }
  if (lane == 0) {
    L.esize[s + 1] = static_cast<int>(nsz);
    if (s + 1 == A.k - 2) L.meta[1] = to_lds ? 1 : 0;
    L.tr[s] = x;
    // v_s's pairs with tr[0..s-1] take bits s(s-1) .. s(s-1) + 2s - 1
    L.dcode[s + 1] = L.dcode[s] | static_cast<int>((Ea[px] & ((1u << (2 * s)) - 1u)) << (s * (s - 1)));
    for (int f = 0; f < s; ++f) {
      const int a = L.sufmax[s * kDSlots + f];
      L.sufmax[(s + 1) * kDSlots + f] = a > x ? a : x;
    }
    L.sufmax[(s + 1) * kDSlots + s] = -1;
  }
  dsync();
  if (to_lds) dbuckets(L, static_cast<int>(nsz));
}

// Move the workgroup's counters into the results.  Any wave may flush while
// the others count: each counter is taken and cleared in one atomic step.
__device__ void dflush(const DMotifArgs& A, const DLds& L) {
  dsync();
  for (int c = lane_id(); c < A.ncls; c += kWave) {
    if (L.cnt[c]) add_counter(A.out + c, atomicExch(L.cnt + c, 0u), A.flags);
  }
  dsync();
}

// does level s live in LDS?  (only the level k-2 list, when it fits)
__device__ __forceinline__ bool level_in_lds(const DMotifArgs& A, const DLds& L, int s) {
  return s == A.k - 2 && L.meta[1] != 0;
}

__device__ int next_dcanonical(const DMotifArgs& A, const DLds& L, const DWave& W, int s, int from, int to) {
  const int lane = lane_id();
  const bool lds = level_in_lds(A, L, s);
  const int32_t* Ev = W.vert + A.level_off[s];
  const uint8_t* Em = W.mask + A.level_off[s];
  for (int c = from; c < to; c += kWave) {
    const int j = c + lane;
    uint64_t e = 0;
    if (j < to) e = lds ? L.lp[j] : dpack(Ev[j], 0u, Em[j]);
    const bool ok = j < to && dcanonical(L, s, dp_v(e), dp_m(e));
    const uint64_t b = ballot(ok);
    if (b) return uni(c + __ffsll(static_cast<long long>(b)) - 1);
  }
  return -1;
}

// The last two levels at once: x = v_{k-2} is appended to tr (|tr| = k-2)
// and every canonical y of the extension set that follows is counted at
// once, without writing that set: x's neighbours new to the set are
// canonical (their only traversal neighbour is x, and they lie above the
// root), and an old entry's mask and arc bits gain x's bit from the marks its
// neighbour scan leaves.
template <bool kLds>
__device__ void dleaf(const DMotifArgs& A, const DLds& L, const DWave& W, int s, int px, int x, uint64_t& pending) {
  const int lane = lane_id();
  // the level list and the marks: LDS-typed when the list is in LDS, so its
  // reads are LDS instructions
  const int32_t* Evg = W.vert + A.level_off[s];
  const uint8_t* Emg = W.mask + A.level_off[s];
  const uint16_t* Eag = W.arcs + A.level_off[s];
  LdsU64d* Epl = (LdsU64d*)(L.lp);
  auto ev = [&](int j) -> int { return kLds ? dp_v(Epl[j]) : Evg[j]; };
  auto ea = [&](int j) -> unsigned { return kLds ? dp_a(Epl[j]) : Eag[j]; };
  // the whole entry: one LDS read, or three global ones
  auto eall = [&](int j) -> uint64_t { return kLds ? Epl[j] : dpack(Evg[j], Eag[j], Emg[j]); };
  uint8_t* hit = kLds ? L.lhit : W.hit;
  const int ns = L.esize[s];
  // The traversal v_0..v_{s-1} plus x, held in registers: the code of v_0..x
  // (v_{s+1}'s pairs with them take the bits from `shift` up), the members a
  // neighbour of x must not be (v_0 is below every neighbour kept), and the
  // canonical test's thresholds (an entry whose first traversal neighbour is
  // v_f must lie above every later traversal vertex; x is below every entry
  // looked at).
  static_assert(kDMotifMaxK - 2 <= 3, "the leaf holds at most three traversal vertices before x");
  const int base = uni(L.dcode[s]) | static_cast<int>((ea(px) & ((1u << (2 * s)) - 1u)) << (s * (s - 1)));
  const int shift = (s + 1) * s;
  const int v0 = uni(L.tr[0]);
  const int t1 = s > 1 ? uni(L.tr[1]) : -1;
  const int t2 = s > 2 ? uni(L.tr[2]) : -1;
  const int th0 = uni(L.sufmax[s * kDSlots + 0]);
  const int th1 = s > 1 ? uni(L.sufmax[s * kDSlots + 1]) : 0;
  const int th2 = s > 2 ? uni(L.sufmax[s * kDSlots + 2]) : 0;
  const int64_t xb = A.rp[x];
  const int dx = static_cast<int>(A.rp[x + 1] - xb);
  for (int c = 0; c < dx; c += kWave) {
    const int i = c + lane;
    const bool ok = i < dx && A.col[xb + i] > v0;
    const int w = ok ? A.col[xb + i] : 0;
    const unsigned d = ok ? A.dir[xb + i] : 0u;
    int lo = 0, hi = ok ? ns : 0;
    if (kLds && ok) {
      const int rel = w - L.meta[2];
      const int b = rel < 0 ? kDBuckets : rel >> L.meta[3];
      lo = b < kDBuckets ? L.bk[b] : 0;
      hi = b < kDBuckets ? L.bk[b + 1] : 0;
    }
    const int end = hi;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ev(mid) < w) lo = mid + 1; else hi = mid;
    }
    const bool found = ok && lo < end && ev(lo) == w;
    // only entries above x can be canonical (below)
    if (found && lo > px) hit[lo] = static_cast<uint8_t>(0x80u | d);
    const bool intr = w == t1 || w == t2;
    const bool isnew = ok && !found && !intr;
    if (isnew) {
      const int cls = A.table[base | static_cast<int>(((d & 3u) << (2 * s)) << shift)];
      if (cls == kUnreachable) atomicOr(A.flags + 1, 2);
      else atomicAdd(L.cnt + cls, 1u);
    }
    pending += static_cast<uint64_t>(__popcll(ballot(isnew)));
  }
  dsync();
  // An old entry y's first traversal neighbour comes before x, so it is
  // canonical only above x (and every later traversal vertex); the list is
  // sorted, so only the entries after x's are looked at.
  for (int c = px + 1; c < ns; c += kWave) {
    const int j = c + lane;
    const bool valid = j < ns;
    const unsigned h = valid ? hit[j] : 0u;
    const uint64_t wj = valid ? eall(j) : 0ull;
    const unsigned e = dp_m(wj);  // over v_0..v_{s-1}: never 0 for an entry
    const int f = __builtin_ctz(e | 0x80000000u);
    const int th = f == 0 ? th0 : (f == 1 ? th1 : th2);
    const bool ok = valid && e != 0u && dp_v(wj) > th;
    if (ok) {
      const unsigned arcs = dp_a(wj) | ((h & 3u) << (2 * s));
      const int cls = A.table[base | static_cast<int>(arcs << shift)];
      if (cls == kUnreachable) atomicOr(A.flags + 1, 2);
      else atomicAdd(L.cnt + cls, 1u);
    }
    if (h) hit[j] = 0;
    pending += static_cast<uint64_t>(__popcll(ballot(ok)));
  }
  dsync();
}

// Every weakly connected induced k-subgraph rooted at v0 (its lowest rank)
// is counted once in its class.  `pending` counts this wave's increments since
// its last flush of the workgroup's 32-bit LDS counters.  A counter holds only
// increments its waves made after their own last flush, and a wave flushes
// once it passes 2^28; a leaf step adds at most dmax + (k-2) dmax, so with at
// most kDMaxWaves waves and dmax < 2^26 no counter reaches 2^32.
__device__ void dmotif_root(const DMotifArgs& A, const DLds& L, const DWave& W, int v0, uint64_t& pending) {
  const int lane = lane_id();
  const int k = A.k;
  const int64_t b0 = A.rp[v0];
  const int d0 = static_cast<int>(A.rp[v0 + 1] - b0);
  const int skip = uni(lower_bound_i32(A.col + b0, d0, v0 + 1));
  {
    const bool lds1 = k == 3 && d0 - skip <= A.leaf_cap;  // level 1 is level k-2
    int32_t* E1 = W.vert + A.level_off[1];
    uint8_t* M1 = W.mask + A.level_off[1];
    uint16_t* A1 = W.arcs + A.level_off[1];
    if (lane == 0 && k == 3) L.meta[1] = lds1 ? 1 : 0;
    for (int i = lane; i < d0 - skip; i += kWave) {
      const int w = A.col[b0 + skip + i];
      const unsigned a = A.dir[b0 + skip + i] & 3u;
      if (lds1) {
        L.lp[i] = dpack(w, a, 1u);
      } else {
        E1[i] = w;
        M1[i] = 1;
        A1[i] = static_cast<uint16_t>(a);
      }
    }
    if (lane == 0) {
      L.esize[1] = d0 - skip;
      L.tr[0] = v0;
      L.dcode[1] = 0;
      L.sufmax[1 * kDSlots + 0] = -1;
      L.cursor[1] = 0;
      L.endv[1] = d0 - skip;
    }
    if (lds1) dbuckets(L, d0 - skip);
  }
  dsync();
  int s = 1;
  for (;;) {
    const int idx = next_dcanonical(A, L, W, s, L.cursor[s], L.endv[s]);
    if (idx < 0) {
      if (s == 1) break;
      --s;
      continue;
    }
    const int x = level_in_lds(A, L, s) ? dp_v(L.lp[idx]) : W.vert[A.level_off[s] + idx];
    if (lane == 0) L.cursor[s] = idx + 1;
    if (s == k - 2) {
      if (level_in_lds(A, L, s)) dleaf<true>(A, L, W, s, idx, x, pending);
      else dleaf<false>(A, L, W, s, idx, x, pending);
      if (pending >= (1ull << 28)) {
        dflush(A, L);
        pending = 0;
      }
      continue;
    }
    dextend(A, L, W, s, idx, x);
    ++s;
    if (lane == 0) {
      L.cursor[s] = 0;
      L.endv[s] = L.esize[s];
    }
    dsync();
  }
}

// (at most 128 VGPRs, so four waves fit per SIMD: measured faster than three
// with no register cap, and than five with spills)
__global__ void __launch_bounds__(64 * kDMaxWaves) __attribute__((amdgpu_waves_per_eu(4))) dmotif_kernel(DMotifArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int wid = static_cast<int>(threadIdx.x) / kWave;
  const int nw = static_cast<int>(blockDim.x) / kWave;
  const int wave_gid = static_cast<int>(blockIdx.x) * nw + wid;
  DLds L = dcarve(smem, A.leaf_cap, wid, nw);
  for (int c = static_cast<int>(threadIdx.x); c < A.ncls; c += static_cast<int>(blockDim.x)) L.cnt[c] = 0;
  DWave W;
  W.vert = A.vert + static_cast<size_t>(wave_gid) * A.wave_cap;
  W.mask = A.mask + static_cast<size_t>(wave_gid) * A.wave_cap;
  W.arcs = A.arcs + static_cast<size_t>(wave_gid) * A.wave_cap;
  W.hit = A.hit + static_cast<size_t>(wave_gid) * A.hit_cap;
  W.nbuf = A.nbuf + static_cast<size_t>(wave_gid) * A.dmax;
  W.ndir = A.ndir + static_cast<size_t>(wave_gid) * A.dmax;
  for (int64_t i = lane; i < A.hit_cap; i += kWave) W.hit[i] = 0;
  for (int i = lane; i < A.leaf_cap; i += kWave) L.lhit[i] = 0;
  __syncthreads();  // the shared counters are zero before any wave counts (the only workgroup barrier)
  uint64_t pending = 0;
  SchedIter it;
  sched_begin(A.S, it);
  Task t;
  while (sched_next(A.S, it, wave_gid, L.tr, &t)) dmotif_root(A, L, W, t.root, pending);
  sched_end(A.S);
  // every wave flushes on its way out; the last one to leave takes what the
  // others counted after their own flush
  dflush(A, L);
}

}  // namespace

size_t dmotif_lds_bytes(int ncls, int leaf_cap, int waves) {
  return static_cast<size_t>(waves) * dwave_lds_bytes(leaf_cap) + static_cast<size_t>(ncls) * sizeof(unsigned);
}

hipError_t dmotif_plan(int ncls, int max_waves_per_cu, DMotifPlan* best) {
  // Every (waves per workgroup, workgroups per CU) shape, its LDS split between
  // the shared counters and the waves' level lists.  Most resident waves wins
  // (the kernel is bound by the latency of its dependent reads), among shapes
  // whose level list holds at least kMinLeaf entries when any does; then the
  // longest level list.
  constexpr size_t kCuLds = 160 * 1024;
  constexpr int kMinLeaf = 256;
  constexpr int kMaxGroups = 32;  // workgroups per CU tried
  DMotifPlan cand[4 * kMaxGroups];  // nw = 1, 2, 4, 8
  int nc = 0;
  for (int nw = 1; nw <= kDMaxWaves; nw *= 2) {
    for (int b = 1; b <= kMaxGroups; ++b) {
      const long long per_wave = (static_cast<long long>(kCuLds / b) - 4ll * ncls) / nw -
                                 static_cast<long long>(dwave_lds_bytes(0));
      if (per_wave < 0) break;
      int leaf = static_cast<int>(per_wave / (8 + 1));
      if (leaf > 4096) leaf = 4096;
      leaf &= ~63;
      const size_t lds = dmotif_lds_bytes(ncls, leaf, nw);
      int fit = 0;
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, dmotif_kernel, kWave * nw, lds);
      if (e != hipSuccess) return e;
      if (fit < 1) continue;
      if (max_waves_per_cu > 0 && fit * nw > max_waves_per_cu) fit = max_waves_per_cu / nw;
      if (fit < 1) continue;
      cand[nc++] = DMotifPlan{nw, leaf, fit, lds};
    }
  }
  bool any_long = false;
  for (int i = 0; i < nc; ++i) any_long |= cand[i].leaf_cap >= kMinLeaf;
  best->waves_per_group = 0;
  for (int i = 0; i < nc; ++i) {
    const DMotifPlan& c = cand[i];
    if (any_long && c.leaf_cap < kMinLeaf) continue;
    const int w = c.groups_per_cu * c.waves_per_group;
    const int bw = best->groups_per_cu * best->waves_per_group;
    if (best->waves_per_group == 0 || w > bw || (w == bw && c.leaf_cap > best->leaf_cap) ||
        (w == bw && c.leaf_cap == best->leaf_cap && c.waves_per_group < best->waves_per_group))
      *best = c;
  }
  return best->waves_per_group ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t launch_dmotif(const DMotifArgs& a, int grid, int waves_per_group, size_t lds_bytes, hipStream_t s) {
  if (waves_per_group < 1 || waves_per_group > kDMaxWaves) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dmotif_kernel, dim3(grid), dim3(kWave * waves_per_group), lds_bytes, s, a);
  return hipGetLastError();
}

}  // namespace dm

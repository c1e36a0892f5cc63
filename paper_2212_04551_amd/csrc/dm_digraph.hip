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
//   - Directed motif counting (k = 3..5): one wave per root extends the
//     traversal with the canonical-candidate rule of Section IV-E over the
//     undirected lists, keeping for every list entry its undirected adjacency
//     mask over the traversal and two arc bits per traversal vertex.  The
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

}  // namespace

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

struct DLds {
  int* tr;        // [kDSlots] traversal
  int* dcode;     // [kDSlots] directed code of tr[0..s-1] per size s
  int* sufmax;    // [kDSlots][kDSlots] max of tr[f+1..s-1] per size s
  int* cursor;    // [kDSlots]
  int* endv;      // [kDSlots]
  int* esize;     // [kDSlots]
  int* nnew;      // [1] new entries of the extension in progress
  unsigned* cnt;  // [ncls] class counters since the last flush
};

__device__ DLds dcarve(unsigned char* smem) {
  DLds L;
  int* p = reinterpret_cast<int*>(smem);
  L.tr = p;
  L.dcode = p + kDSlots;
  L.sufmax = p + 2 * kDSlots;
  L.cursor = L.sufmax + kDSlots * kDSlots;
  L.endv = L.cursor + kDSlots;
  L.esize = L.endv + kDSlots;
  L.nnew = L.esize + kDSlots;
  L.cnt = reinterpret_cast<unsigned*>(L.nnew + 4);
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
  int32_t* Nv = W.vert + A.level_off[s + 1];
  uint8_t* Nm = W.mask + A.level_off[s + 1];
  uint16_t* Na = W.arcs + A.level_off[s + 1];
  const int64_t cap = A.level_cap[s + 1];
  wave_sync();
  // both parts are sorted by id: every entry's place is its rank in the other part
  for (int j = lane; j < ns; j += kWave) {
    if (j == px) continue;
    const int y = Ev[j];
    const unsigned h = W.hit[j];
    const int r = lower_bound_i32(W.nbuf, nn, y);
    const int64_t out = static_cast<int64_t>(j) - (j > px ? 1 : 0) + r;
    if (out < cap) {
      Nv[out] = y;
      Nm[out] = static_cast<uint8_t>(Em[j] | ((h & 0x80u) ? (1u << s) : 0u));
      Na[out] = static_cast<uint16_t>(Ea[j] | ((h & 3u) << (2 * s)));
    }
    if (h) W.hit[j] = 0;
  }
  for (int i = lane; i < nn; i += kWave) {
    const int w = W.nbuf[i];
    int r = lower_bound_i32(Ev, ns, w);
    if (px < r) r -= 1;
    const int64_t out = static_cast<int64_t>(i) + r;
    if (out < cap) {
      Nv[out] = w;
      Nm[out] = static_cast<uint8_t>(1u << s);
      Na[out] = static_cast<uint16_t>((W.ndir[i] & 3u) << (2 * s));
    }
  }
  int64_t nsz = static_cast<int64_t>(ns) - 1 + nn;
  if (nsz > cap) {
    if (lane == 0) atomicOr(A.flags + 1, 1);
    nsz = cap;
  }
  if (lane == 0) {
    L.esize[s + 1] = static_cast<int>(nsz);
    L.tr[s] = x;
    // v_s's pairs with tr[0..s-1] take bits s(s-1) .. s(s-1) + 2s - 1
    L.dcode[s + 1] = L.dcode[s] | static_cast<int>((Ea[px] & ((1u << (2 * s)) - 1u)) << (s * (s - 1)));
    for (int f = 0; f < s; ++f) {
      const int a = L.sufmax[s * kDSlots + f];
      L.sufmax[(s + 1) * kDSlots + f] = a > x ? a : x;
    }
    L.sufmax[(s + 1) * kDSlots + s] = -1;
  }
  wave_sync();
}

__device__ void dflush(const DMotifArgs& A, const DLds& L) {
  wave_sync();
  for (int c = lane_id(); c < A.ncls; c += kWave) {
    const unsigned v = L.cnt[c];
    if (v) {
      add_counter(A.out + c, v, A.flags);
      L.cnt[c] = 0;
    }
  }
  wave_sync();
}

__device__ int next_dcanonical(const DMotifArgs& A, const DLds& L, const DWave& W, int s, int from, int to) {
  const int lane = lane_id();
  const int32_t* Ev = W.vert + A.level_off[s];
  const uint8_t* Em = W.mask + A.level_off[s];
  for (int c = from; c < to; c += kWave) {
    const int j = c + lane;
    const bool ok = j < to && dcanonical(L, s, Ev[j], Em[j]);
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
__device__ void dleaf(const DMotifArgs& A, const DLds& L, const DWave& W, int s, int px, int x, uint64_t& pending) {
  const int lane = lane_id();
  const int32_t* Ev = W.vert + A.level_off[s];
  const uint8_t* Em = W.mask + A.level_off[s];
  const uint16_t* Ea = W.arcs + A.level_off[s];
  const int ns = L.esize[s];
  if (lane == 0) {
    L.tr[s] = x;
    L.dcode[s + 1] = L.dcode[s] | static_cast<int>((Ea[px] & ((1u << (2 * s)) - 1u)) << (s * (s - 1)));
    for (int f = 0; f < s; ++f) {
      const int a = L.sufmax[s * kDSlots + f];
      L.sufmax[(s + 1) * kDSlots + f] = a > x ? a : x;
    }
    L.sufmax[(s + 1) * kDSlots + s] = -1;
  }
  wave_sync();
  const int base = L.dcode[s + 1];
  const int shift = (s + 1) * s;  // v_{s+1}'s pairs with tr[0..s]
  const int v0 = L.tr[0];
  const int64_t xb = A.rp[x];
  const int dx = static_cast<int>(A.rp[x + 1] - xb);
  for (int c = 0; c < dx; c += kWave) {
    const int i = c + lane;
    const bool ok = i < dx && A.col[xb + i] > v0;
    const int w = ok ? A.col[xb + i] : 0;
    const unsigned d = ok ? A.dir[xb + i] : 0u;
    const int j = ok ? lower_bound_i32(Ev, ns, w) : ns;
    const bool found = ok && j < ns && Ev[j] == w;
    if (found && j != px) W.hit[j] = static_cast<uint8_t>(0x80u | d);
    bool intr = false;
    for (int t = 0; t < s; ++t) intr |= (L.tr[t] == w);
    const bool isnew = ok && !found && !intr;
    if (isnew) {
      const int cls = A.table[base | static_cast<int>(((d & 3u) << (2 * s)) << shift)];
      if (cls == kUnreachable) atomicOr(A.flags + 1, 2);
      else atomicAdd(L.cnt + cls, 1u);
    }
    pending += static_cast<uint64_t>(__popcll(ballot(isnew)));
  }
  wave_sync();
  for (int c = 0; c < ns; c += kWave) {
    const int j = c + lane;
    const bool valid = j < ns && j != px;
    const unsigned h = valid ? W.hit[j] : 0u;
    const unsigned m = valid ? (Em[j] | ((h & 0x80u) ? (1u << s) : 0u)) : 0u;
    const bool ok = valid && dcanonical(L, s + 1, Ev[j], m);
    if (ok) {
      const unsigned arcs = Ea[j] | ((h & 3u) << (2 * s));
      const int cls = A.table[base | static_cast<int>(arcs << shift)];
      if (cls == kUnreachable) atomicOr(A.flags + 1, 2);
      else atomicAdd(L.cnt + cls, 1u);
    }
    if (h) W.hit[j] = 0;
    pending += static_cast<uint64_t>(__popcll(ballot(ok)));
  }
  wave_sync();
}

// Every weakly connected induced k-subgraph rooted at v0 (its smallest id)
// is counted once in its class.  `pending` counts increments since the last
// flush of the 32-bit LDS counters.
__device__ void dmotif_root(const DMotifArgs& A, const DLds& L, const DWave& W, int v0, uint64_t& pending) {
  const int lane = lane_id();
  const int k = A.k;
  const int64_t b0 = A.rp[v0];
  const int d0 = static_cast<int>(A.rp[v0 + 1] - b0);
  const int skip = uni(lower_bound_i32(A.col + b0, d0, v0 + 1));
  {
    int32_t* E1 = W.vert + A.level_off[1];
    uint8_t* M1 = W.mask + A.level_off[1];
    uint16_t* A1 = W.arcs + A.level_off[1];
    for (int i = lane; i < d0 - skip; i += kWave) {
      E1[i] = A.col[b0 + skip + i];
      M1[i] = 1;
      A1[i] = static_cast<uint16_t>(A.dir[b0 + skip + i] & 3u);
    }
    if (lane == 0) {
      L.esize[1] = d0 - skip;
      L.tr[0] = v0;
      L.dcode[1] = 0;
      L.sufmax[1 * kDSlots + 0] = -1;
      L.cursor[1] = 0;
      L.endv[1] = d0 - skip;
    }
  }
  wave_sync();
  int s = 1;
  for (;;) {
    const int idx = next_dcanonical(A, L, W, s, L.cursor[s], L.endv[s]);
    if (idx < 0) {
      if (s == 1) break;
      --s;
      continue;
    }
    const int x = W.vert[A.level_off[s] + idx];
    if (lane == 0) L.cursor[s] = idx + 1;
    if (s == k - 2) {
      dleaf(A, L, W, s, idx, x, pending);
      if (pending >= (1ull << 31)) {
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
    wave_sync();
  }
}

__global__ void __launch_bounds__(64) dmotif_kernel(DMotifArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int wave_gid = blockIdx.x;
  DLds L = dcarve(smem);
  for (int c = lane; c < A.ncls; c += kWave) L.cnt[c] = 0;
  DWave W;
  W.vert = A.vert + static_cast<size_t>(wave_gid) * A.wave_cap;
  W.mask = A.mask + static_cast<size_t>(wave_gid) * A.wave_cap;
  W.arcs = A.arcs + static_cast<size_t>(wave_gid) * A.wave_cap;
  W.hit = A.hit + static_cast<size_t>(wave_gid) * A.hit_cap;
  W.nbuf = A.nbuf + static_cast<size_t>(wave_gid) * A.dmax;
  W.ndir = A.ndir + static_cast<size_t>(wave_gid) * A.dmax;
  for (int64_t i = lane; i < A.hit_cap; i += kWave) W.hit[i] = 0;
  wave_sync();
  uint64_t pending = 0;
  SchedIter it;
  sched_begin(A.S, it);
  Task t;
  while (sched_next(A.S, it, wave_gid, L.tr, &t)) dmotif_root(A, L, W, t.root, pending);
  sched_end(A.S);
  dflush(A, L);
}

}  // namespace

size_t dmotif_lds_bytes(int ncls) {
  const size_t ints = 3 * kDSlots + kDSlots * kDSlots + 3 * kDSlots + 4;
  return ints * sizeof(int) + static_cast<size_t>(ncls) * sizeof(unsigned);
}

hipError_t dmotif_occupancy(size_t lds_bytes, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, dmotif_kernel, 64, lds_bytes);
}

hipError_t launch_dmotif(const DMotifArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(dmotif_kernel, dim3(grid), dim3(64), lds_bytes, s, a);
  return hipGetLastError();
}

}  // namespace dm

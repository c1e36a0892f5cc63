// C ABI of libdumato_mi (declared in include/dm.h).
//
// Host side of the library: graph handles, input validation, the canonical
// relabeling dictionary (DuMato, Section IV-C, Aggregate), workspace, the
// persistent-kernel launch for clique and motif counting (Section IV-E,
// Alg. 4), batching of many graphs into one launch, and the final uint64
// reduction with overflow checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "dm.h"
#include "dm_internal.hpp"

using namespace dm;

// ====================================================================== errors

static thread_local std::string g_last_error;

static dm_status fail(dm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

static dm_status hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? DM_E_NOMEM : DM_E_HIP;
}

#define HIP_OR_RETURN(expr, where)            \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

extern "C" const char* dm_strerror(dm_status s) {
  switch (s) {
    case DM_OK: return "ok";
    case DM_E_ARG: return "invalid argument";
    case DM_E_CSR: return "invalid CSR graph";
    case DM_E_K: return "k out of supported range";
    case DM_E_OVERFLOW: return "uint64 count overflow";
    case DM_E_NOMEM: return "out of memory";
    case DM_E_HIP: return "HIP runtime error";
    case DM_E_BUFSZ: return "output buffer too small";
    case DM_E_MODEL: return "invalid or missing model parameters";
  }
  return "unknown status";
}

extern "C" const char* dm_last_error(void) { return g_last_error.c_str(); }

// kernel launches of the calling thread's last counting call
static thread_local int g_last_launches = 0;

extern "C" int dm_last_launch_count(void) { return g_last_launches; }

// ====================================================================== class tables

namespace {

struct ClassTables {
  int ncls = 0;
  std::vector<uint32_t> canon;   // class -> canonical full bitmap
  std::vector<uint16_t> table;   // traversal code -> class (kUnreachable: some v_i has no earlier neighbour)
};

inline int pair_index(int t, int i) { return i * (i - 1) / 2 + t; }  // t < i

bool bitmap_connected(int k, uint32_t code) {
  uint32_t adj[8] = {0};
  for (int i = 1; i < k; ++i)
    for (int t = 0; t < i; ++t)
      if ((code >> pair_index(t, i)) & 1u) {
        adj[t] |= 1u << i;
        adj[i] |= 1u << t;
      }
  uint32_t reach = 1u, prev = 0u;
  while (reach != prev) {
    prev = reach;
    for (int v = 0; v < k; ++v)
      if ((reach >> v) & 1u) reach |= adj[v];
  }
  return reach == (1u << k) - 1u;
}

// run fn(t) for t in [0, n) on n host threads
template <class F>
void parallel_run(int n, F fn) {
  std::vector<std::thread> th;
  for (int t = 1; t < n; ++t) th.emplace_back(fn, t);
  fn(0);
  for (auto& x : th) x.join();
}

// Canonical forms by orbit enumeration.  Every permutation of S_k is turned
// into a map of bitmap positions (Heap's algorithm).  Host threads scan
// disjoint slices of the 2^(k(k-1)/2) labelled bitmaps; a connected bitmap
// not yet labelled has its whole orbit generated and every member labelled
// with the orbit minimum, the canonical form (two threads that reach the same
// orbit write the same labels).  For k = 8 that is 2^28 bitmaps (a 1 GiB label
// array, freed when the table is filled) and 11,117 orbits of up to 40,320
// members.
ClassTables build_tables(int k) {
  ClassTables T;
  const int P = k * (k - 1) / 2;
  const uint32_t ncodes = 1u << P;
  std::vector<uint8_t> pm;  // permutation j: pm[j * P + b] = image of bitmap position b
  {
    std::vector<int> p(k), c(k, 0);
    std::iota(p.begin(), p.end(), 0);
    auto add = [&]() {
      const size_t base = pm.size();
      pm.resize(base + P);
      for (int i = 1; i < k; ++i)
        for (int t = 0; t < i; ++t) {
          int a = p[t], b = p[i];
          if (a > b) std::swap(a, b);
          pm[base + pair_index(t, i)] = static_cast<uint8_t>(pair_index(a, b));
        }
    };
    add();
    int i = 0;
    while (i < k) {
      if (c[i] < i) {
        if (i % 2 == 0) std::swap(p[0], p[i]); else std::swap(p[c[i]], p[i]);
        add();
        ++c[i];
        i = 0;
      } else {
        c[i] = 0;
        ++i;
      }
    }
  }
  const size_t nperm = pm.size() / P;
  const uint32_t kUnset = 0xffffffffu, kDisconnected = 0xfffffffeu;
  std::unique_ptr<std::atomic<uint32_t>[]> lab(new std::atomic<uint32_t>[ncodes]);
  const unsigned hc = std::thread::hardware_concurrency();
  const int nth = ncodes < (1u << 16) ? 1 : static_cast<int>(std::max(1u, std::min(16u, hc)));
  auto slice = [&](int t, uint64_t n) { return std::make_pair(n * t / nth, n * (t + 1) / nth); };
  parallel_run(nth, [&](int t) {
    const auto r = slice(t, ncodes);
    for (uint64_t c = r.first; c < r.second; ++c) lab[c].store(kUnset, std::memory_order_relaxed);
  });
  parallel_run(nth, [&](int t) {
    const auto r = slice(t, ncodes);
    std::vector<uint32_t> orbit(nperm);
    for (uint64_t cc = r.first; cc < r.second; ++cc) {
      const uint32_t c = static_cast<uint32_t>(cc);
      if (lab[c].load(std::memory_order_relaxed) != kUnset) continue;
      if (!bitmap_connected(k, c)) {
        lab[c].store(kDisconnected, std::memory_order_relaxed);
        continue;
      }
      uint32_t best = c;
      for (size_t j = 0; j < nperm; ++j) {
        const uint8_t* m = &pm[j * P];
        uint32_t d = 0;
        for (uint32_t x = c; x; x &= x - 1) d |= 1u << m[__builtin_ctz(x)];
        orbit[j] = d;
        best = std::min(best, d);
      }
      for (size_t j = 0; j < nperm; ++j) lab[orbit[j]].store(best, std::memory_order_relaxed);
    }
  });
  std::vector<uint32_t> reps;
  for (uint32_t c = 0; c < ncodes; ++c)
    if (lab[c].load(std::memory_order_relaxed) == c) reps.push_back(c);
  std::sort(reps.begin(), reps.end(), [](uint32_t a, uint32_t b) {
    const int pa = __builtin_popcount(a), pb = __builtin_popcount(b);
    return pa != pb ? pa < pb : a < b;
  });
  T.ncls = static_cast<int>(reps.size());
  T.canon = reps;
  std::vector<std::pair<uint32_t, uint16_t>> id(reps.size());
  for (int q = 0; q < T.ncls; ++q) id[q] = {reps[q], static_cast<uint16_t>(q)};
  std::sort(id.begin(), id.end());
  // traversal code t: full bitmap (t << 1) | 1 (edge v0-v1 implied)
  const uint32_t ntrav = 1u << (P - 1);
  T.table.assign(ntrav, kUnreachable);
  parallel_run(nth, [&](int th) {
    const auto r = slice(th, ntrav);
    for (uint64_t tt = r.first; tt < r.second; ++tt) {
      const uint32_t t = static_cast<uint32_t>(tt);
      bool reach = true;
      for (int i = 2; i < k; ++i) {
        const uint32_t field = (t >> (i * (i - 1) / 2 - 1)) & ((1u << i) - 1u);
        if (!field) reach = false;
      }
      if (!reach) continue;
      const uint32_t canon = lab[(t << 1) | 1u].load(std::memory_order_relaxed);
      const auto it = std::lower_bound(id.begin(), id.end(), std::make_pair(canon, static_cast<uint16_t>(0)));
      T.table[t] = it->second;
    }
  });
  return T;
}

std::mutex g_tables_lock;
ClassTables* g_tables[kMotifMaxK + 1] = {nullptr};

const ClassTables* tables(int k) {
  if (k < 3 || k > kMotifMaxK) return nullptr;
  std::lock_guard<std::mutex> lk(g_tables_lock);
  if (!g_tables[k]) g_tables[k] = new ClassTables(build_tables(k));
  return g_tables[k];
}

// Directed classes (k <= 5): codes take two bits per vertex pair t < i,
// bit 2p for the arc t -> i and bit 2p+1 for i -> t (p = i(i-1)/2 + t); a
// class is the smallest code over all vertex orders, and the weakly connected
// classes are numbered by increasing smallest code.  Orbit labelling: codes
// are visited in increasing order, and the first one not yet labelled is the
// smallest of its orbit, whose k! images are labelled with it.
struct DClassTables {
  int ncls = 0;
  std::vector<uint32_t> canon;  // class -> smallest code
  std::vector<uint16_t> table;  // code -> class (kUnreachable: not weakly connected)
};

DClassTables build_dtables(int k) {
  DClassTables T;
  const int npairs = k * (k - 1) / 2;
  const uint32_t ncodes = 1u << (2 * npairs);
  std::vector<int32_t> orbit(ncodes, -1);
  std::vector<uint32_t> reps;
  std::vector<std::vector<int>> perms;
  std::vector<int> p(k);
  for (int i = 0; i < k; ++i) p[i] = i;
  do perms.push_back(p);
  while (std::next_permutation(p.begin(), p.end()));
  int ax[kDMotifMaxK * kDMotifMaxK], ay[kDMotifMaxK * kDMotifMaxK];
  for (uint32_t c = 0; c < ncodes; ++c) {
    if (orbit[c] >= 0) continue;
    const int id = static_cast<int>(reps.size());
    reps.push_back(c);
    int na = 0;
    for (int i = 1; i < k; ++i)
      for (int t = 0; t < i; ++t) {
        const int b = 2 * pair_index(t, i);
        if ((c >> b) & 1u) { ax[na] = t; ay[na] = i; ++na; }
        if ((c >> (b + 1)) & 1u) { ax[na] = i; ay[na] = t; ++na; }
      }
    for (const auto& q : perms) {
      uint32_t img = 0;
      for (int e = 0; e < na; ++e) {
        const int a = q[ax[e]], b = q[ay[e]];
        img |= a < b ? 1u << (2 * pair_index(a, b)) : 1u << (2 * pair_index(b, a) + 1);
      }
      orbit[img] = id;
    }
  }
  std::vector<int> cls_of_orbit(reps.size(), -1);
  for (size_t r = 0; r < reps.size(); ++r) {
    uint32_t und = 0;  // the underlying undirected graph
    for (int pi = 0; pi < npairs; ++pi)
      if ((reps[r] >> (2 * pi)) & 3u) und |= 1u << pi;
    if (bitmap_connected(k, und)) {
      cls_of_orbit[r] = T.ncls++;
      T.canon.push_back(reps[r]);
    }
  }
  T.table.assign(ncodes, kUnreachable);
  for (uint32_t c = 0; c < ncodes; ++c)
    if (cls_of_orbit[orbit[c]] >= 0) T.table[c] = static_cast<uint16_t>(cls_of_orbit[orbit[c]]);
  return T;
}

DClassTables* g_dtables[kDMotifMaxK + 1] = {nullptr};

const DClassTables* dtables(int k) {
  if (k < 1 || k > kDMotifMaxK) return nullptr;
  std::lock_guard<std::mutex> lk(g_tables_lock);
  if (!g_dtables[k]) g_dtables[k] = new DClassTables(build_dtables(k));
  return g_dtables[k];
}

// device copies of the dictionary, per (device, k)
std::mutex g_dev_tables_lock;
std::map<std::pair<int, int>, uint16_t*> g_dev_tables;

hipError_t device_table(int k, uint16_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_dev_tables_lock);
  auto key = std::make_pair(dev, k);
  auto it = g_dev_tables.find(key);
  if (it != g_dev_tables.end()) {
    *out = it->second;
    return hipSuccess;
  }
  // keys above 100 hold the directed dictionaries (k + 100)
  const std::vector<uint16_t>& tab = k > 100 ? dtables(k - 100)->table : tables(k)->table;
  uint16_t* p = nullptr;
  const size_t bytes = tab.size() * sizeof(uint16_t);
  e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return e;
  e = hipMemcpy(p, tab.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return e;
  }
  g_dev_tables[key] = p;
  *out = p;
  return hipSuccess;
}

}  // namespace

extern "C" int dm_motif_num_classes(int k) {
  const ClassTables* T = tables(k);
  return T ? T->ncls : -1;
}

extern "C" dm_status dm_motif_class_mask(int k, int cls, uint32_t* mask) {
  const ClassTables* T = tables(k);
  if (!T) return fail(DM_E_K, "motif k must be in 3..8");
  if (!mask || cls < 0 || cls >= T->ncls) return fail(DM_E_ARG, "class id out of range or null output");
  *mask = T->canon[cls];
  return DM_OK;
}

extern "C" dm_status dm_motif_class_table(int k, uint8_t* out, size_t len) {
  const ClassTables* T = k <= 6 ? tables(k) : nullptr;
  if (!T) return fail(DM_E_K, "8-bit class table: k must be in 3..6");
  if (!out) return fail(DM_E_ARG, "null output");
  if (len < T->table.size()) return fail(DM_E_BUFSZ, "table needs 2^(k(k-1)/2-1) bytes");
  for (size_t i = 0; i < T->table.size(); ++i)
    out[i] = T->table[i] == kUnreachable ? 0xFF : static_cast<uint8_t>(T->table[i]);
  return DM_OK;
}

extern "C" dm_status dm_motif_class_table16(int k, uint16_t* out, size_t len) {
  const ClassTables* T = tables(k);
  if (!T) return fail(DM_E_K, "motif k must be in 3..8");
  if (!out) return fail(DM_E_ARG, "null output");
  if (len < T->table.size()) return fail(DM_E_BUFSZ, "table needs 2^(k(k-1)/2-1) entries");
  std::memcpy(out, T->table.data(), T->table.size() * sizeof(uint16_t));
  return DM_OK;
}

// ====================================================================== graph handles

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t need) {
    if (need == 0) need = 16;
    if (bytes >= need) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, need);
    if (e == hipSuccess) bytes = need;
    return e;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

struct dm_graph {
  uint64_t uid = 0;  // process-unique id (batch cache key)
  int device = 0;
  int32_t n = 0;
  int64_t nnz = 0;
  int dmax = 0;
  Buf rp, col;
  // degree-ordered DAG (clique counting), built on first use
  bool dag = false;
  int ddmax = 0;
  Buf rank, order, drp, dcol;
  // the undirected graph renamed by rank (motif counting), built on first use
  bool ranked = false;
  Buf urp, ucol;
  // workspace reused across calls
  Buf ctrl, out, rows, ext_vert, ext_mask, newbuf, qroot, qstat, qlo, qhi, rgraph;
  Buf dfs_stack, dfs_mask;  // per-lane stacks of the one-lane-per-traversal ablation
  Buf spill, tq;            // host-driven balancing: spilled tasks, relaunch queue
  Buf wave_cnt;             // motifs at k = 8: per-wave class counters
  // digraphs (dm_load_digraph): arc bits per adjacency entry, directed-motif workspace
  bool directed = false;
  int64_t arcs = 0;
  Buf dir, ext_arcs, dhit, dndir;
  Buf rdir;             // arc bits in the rank-renamed graph (urp / ucol)
  bool dranked = false;
  // learned ordering: features (cached), predictions, LPT order, chunk starts
  // and the order in rank space; the queue is reused while the parameter
  // fingerprint, grid and chunks per wave stay the same
  bool feat_ready = false;
  Buf feat, pred, lorder, lqroot, lqbounds, lqkey;
  // cache of every root's bitmap rows (clique counting): offsets, then rows;
  // filled by the first counting launch over all roots, read by later ones
  bool rc_layout = false, rc_ready = false;
  int64_t rc_words = 0;
  Buf rcoff, rcache;
  bool lq_valid = false;
  unsigned long long lq_key = 0;
  int lq_grid = 0, lq_per_wave = 0;
  int64_t lq_nchunks = 0;
  hipStream_t own = nullptr;
};

static hipStream_t pick_stream(dm_graph* g, void* s) {
  if (s) return static_cast<hipStream_t>(s);
  if (!g->own) (void)hipStreamCreateWithFlags(&g->own, hipStreamNonBlocking);
  return g->own;
}

// Host-side check of the CSR conventions (simple undirected graph, sorted lists).
static bool host_validate(int32_t n, const int64_t* rp, const int32_t* col, std::string* why) {
  if (rp[0] != 0) { *why = "row_ptr[0] != 0"; return false; }
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) { *why = "row_ptr decreases"; return false; }
  for (int32_t v = 0; v < n; ++v) {
    for (int64_t i = rp[v]; i < rp[v + 1]; ++i) {
      const int32_t u = col[i];
      if (u < 0 || u >= n) { *why = "column id out of range"; return false; }
      if (u == v) { *why = "self-loop"; return false; }
      if (i > rp[v] && col[i - 1] >= u) { *why = "adjacency not strictly ascending (or repeated edge)"; return false; }
      const int32_t* b = col + rp[u];
      const int32_t* e = col + rp[u + 1];
      const int32_t* f = std::lower_bound(b, e, v);
      if (f == e || *f != v) { *why = "asymmetric adjacency"; return false; }
    }
  }
  return true;
}

static dm_status ensure_dag(dm_graph* g, hipStream_t s);
static dm_status ensure_ranked(dm_graph* g, hipStream_t s);

extern "C" dm_status dm_load_csr(int32_t n, const int64_t* row_ptr, const int32_t* col, uint32_t flags, void* stream,
                                 dm_graph** out) {
  if (!out) return fail(DM_E_ARG, "null output handle");
  *out = nullptr;
  if (n < 0 || !row_ptr || (!col && n > 0)) return fail(DM_E_ARG, "n < 0 or null CSR array");
  if (flags & ~15u) return fail(DM_E_ARG, "unknown flag");
  const bool on_device = flags & DM_CSR_DEVICE;
  const bool trusted = flags & DM_CSR_TRUSTED;
  int64_t nnz = 0;
  if (!on_device) {
    nnz = row_ptr[n];
    if (nnz < 0 || nnz % 2) return fail(DM_E_CSR, "nnz must be even and non-negative");
    std::string why;
    if (!trusted && !host_validate(n, row_ptr, col, &why)) return fail(DM_E_CSR, why);
  }
  dm_graph* g = new dm_graph();
  static std::atomic<uint64_t> next_uid{1};
  g->uid = next_uid++;
  (void)hipGetDevice(&g->device);
  hipStream_t s = pick_stream(g, stream);
  auto bail = [&](dm_status st) {
    dm_free(g);
    return st;
  };
  if (on_device) {
    hipError_t e = hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_fail(e, "dm_load_csr: read nnz"));
    if (nnz < 0 || nnz % 2) return bail(fail(DM_E_CSR, "nnz must be even and non-negative"));
  }
  g->n = n;
  g->nnz = nnz;
  hipError_t e = g->rp.ensure(sizeof(int64_t) * (static_cast<size_t>(n) + 1));
  if (e == hipSuccess) e = g->col.ensure(sizeof(int32_t) * static_cast<size_t>(nnz > 0 ? nnz : 1));
  if (e != hipSuccess) return bail(hip_fail(e, "dm_load_csr: allocate"));
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  e = hipMemcpyAsync(g->rp.p, row_ptr, sizeof(int64_t) * (static_cast<size_t>(n) + 1), kind, s);
  if (e == hipSuccess && nnz > 0) e = hipMemcpyAsync(g->col.p, col, sizeof(int32_t) * nnz, kind, s);
  if (e != hipSuccess) return bail(hip_fail(e, "dm_load_csr: copy"));
  // device-side validation and maximum degree share one small scratch word pair
  Buf tmp;
  e = tmp.ensure(2 * sizeof(int));
  if (e == hipSuccess) e = launch_fill_i32(tmp.as<int>(), 2, 0, s);
  if (e == hipSuccess && on_device && !trusted && n > 0)
    e = launch_validate(g->rp.as<int64_t>(), g->col.as<int32_t>(), n, nnz, tmp.as<int>(), s);
  if (e == hipSuccess && n > 0) e = launch_max_degree(g->rp.as<int64_t>(), n, tmp.as<int>() + 1, s);
  int hostw[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hostw, tmp.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(hip_fail(e, "dm_load_csr: validate"));
  if (hostw[0]) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "device CSR validation failed (flags 0x%x)", hostw[0]);
    return bail(fail(DM_E_CSR, buf));
  }
  g->dmax = hostw[1];
  if (flags & (DM_CSR_ORIENT | DM_CSR_RANK)) {
    const dm_status st = (flags & DM_CSR_RANK) ? ensure_ranked(g, s) : ensure_dag(g, s);
    if (st != DM_OK) return bail(st);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_fail(e, "dm_load_csr: orient"));
  }
  *out = g;
  return DM_OK;
}

extern "C" void dm_free(dm_graph* g) {
  if (!g) return;
  if (g->own) (void)hipStreamDestroy(g->own);
  delete g;
}

extern "C" dm_status dm_graph_info(const dm_graph* g, int32_t* n, int64_t* nnz) {
  if (!g) return fail(DM_E_ARG, "null graph");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  return DM_OK;
}

static dm_status ensure_dag(dm_graph* g, hipStream_t s) {
  if (g->dag) return DM_OK;
  const size_t n1 = static_cast<size_t>(g->n) + 1;
  HIP_OR_RETURN(g->rank.ensure(sizeof(int32_t) * n1), "orient: allocate");
  HIP_OR_RETURN(g->order.ensure(sizeof(int32_t) * n1), "orient: allocate");
  HIP_OR_RETURN(g->drp.ensure(sizeof(int64_t) * n1), "orient: allocate");
  HIP_OR_RETURN(g->dcol.ensure(sizeof(int32_t) * static_cast<size_t>(g->nnz / 2 + 1)), "orient: allocate");
  HIP_OR_RETURN(orient_by_degree(g->rp.as<int64_t>(), g->col.as<int32_t>(), g->n, g->nnz, g->rank.as<int32_t>(),
                                 g->order.as<int32_t>(), g->drp.as<int64_t>(), g->dcol.as<int32_t>(), &g->ddmax, s),
                "orient");
  g->dag = true;
  return DM_OK;
}

static dm_status ensure_ranked(dm_graph* g, hipStream_t s) {
  if (g->ranked) return DM_OK;
  dm_status st = ensure_dag(g, s);
  if (st != DM_OK) return st;
  HIP_OR_RETURN(g->urp.ensure(sizeof(int64_t) * (static_cast<size_t>(g->n) + 1)), "relabel: allocate");
  HIP_OR_RETURN(g->ucol.ensure(sizeof(int32_t) * static_cast<size_t>(g->nnz > 0 ? g->nnz : 1)), "relabel: allocate");
  HIP_OR_RETURN(relabel_by_rank(g->rp.as<int64_t>(), g->col.as<int32_t>(), g->n, g->nnz, g->rank.as<int32_t>(),
                                g->order.as<int32_t>(), g->urp.as<int64_t>(), g->ucol.as<int32_t>(), s),
                "relabel");
  g->ranked = true;
  return DM_OK;
}

// ====================================================================== options

namespace {

struct Opt {
  uint32_t sched = 0;
  hipStream_t stream = nullptr;
  uint32_t chunk = 0;
  float rebalance = 0.f;
  uint32_t waves_per_cu = 0;
  const float* mlp = nullptr;
  const int32_t* roots = nullptr;
  int64_t num_roots = 0;
  uint64_t* root_stats = nullptr;
  uint64_t* wave_stats = nullptr;
  uint32_t wave_stats_len = 0;
  uint64_t bias = 0;
  uint32_t wait_limit_us = 0;
  const float* root_cost = nullptr;
};

dm_status read_opt(const dm_options* o, Opt* r) {
  *r = Opt();
  if (!o) return DM_OK;
  if (o->size != sizeof(dm_options)) return fail(DM_E_ARG, "dm_options.size != sizeof(dm_options)");
  if (o->sched & ~127u) return fail(DM_E_ARG, "unknown sched bits");
  if ((o->sched & DM_SCHED_HOST_BALANCE) && (o->sched & DM_NO_DONATION))
    return fail(DM_E_ARG, "DM_SCHED_HOST_BALANCE already runs without in-kernel donation");
  if ((o->sched & DM_IMPL_DFS) && ((o->sched & ~static_cast<uint32_t>(DM_IMPL_DFS | DM_NO_DONATION)) || o->roots))
    return fail(DM_E_ARG, "DM_IMPL_DFS runs the plain root order over every root, with no other option");
  if ((o->sched & DM_SCHED_COST) && (o->sched & DM_SCHED_LEARNED))
    return fail(DM_E_ARG, "DM_SCHED_COST and DM_SCHED_LEARNED are exclusive");
  if ((o->sched & DM_SCHED_COST) && !o->root_cost) return fail(DM_E_ARG, "DM_SCHED_COST needs root_cost");
  if ((o->sched & DM_SCHED_COST) && o->roots) return fail(DM_E_ARG, "cost ordering orders every root; no root list");
  if (o->rebalance < 0.f || o->rebalance > 1.f) return fail(DM_E_ARG, "rebalance must be in [0, 1]");
  if (o->num_roots < 0 || (o->num_roots > 0 && !o->roots)) return fail(DM_E_ARG, "bad root list");
  if ((o->sched & DM_RECORD_ROOTS) && !o->root_stats) return fail(DM_E_ARG, "DM_RECORD_ROOTS needs root_stats");
  if ((o->sched & DM_SCHED_LEARNED) && o->roots) return fail(DM_E_ARG, "learned ordering orders every root; no root list");
  r->sched = o->sched;
  r->stream = static_cast<hipStream_t>(o->stream);
  r->chunk = o->chunk;
  r->rebalance = o->rebalance;
  r->waves_per_cu = o->waves_per_cu;
  r->mlp = o->mlp;
  r->roots = o->roots;
  r->num_roots = o->roots ? o->num_roots : 0;
  r->root_stats = (o->sched & DM_RECORD_ROOTS) ? o->root_stats : nullptr;
  r->wave_stats = o->wave_stats;
  r->wave_stats_len = o->wave_stats ? o->wave_stats_len : 0;
  r->bias = o->counter_bias;
  r->wait_limit_us = o->wait_limit_us;
  r->root_cost = (o->sched & DM_SCHED_COST) ? o->root_cost : nullptr;
  return DM_OK;
}

// Default bound on how long an idle wave waits for donated work.  A launch's
// idle waves are normally fed within microseconds; only a scheduler fault can
// starve them this long.
constexpr uint32_t kDefaultWaitLimitUs = 600000000u;

// wall-clock ticks (the counter read by wall_clock64) in `us` microseconds
uint64_t wait_ticks(uint32_t us) {
  int dev = 0, khz = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
  return static_cast<uint64_t>(us ? us : kDefaultWaitLimitUs) * static_cast<uint64_t>(khz) / 1000u;
}

int cu_count() {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  return cus;
}

constexpr int kSlots = 1024;
constexpr size_t kCtrlState = 8;   // u64 state
constexpr size_t kCtrlIdle = 16;   // int idle
constexpr size_t kCtrlFlags = 20;  // int flags[2]
constexpr size_t kCtrlSlots = 32;  // int slot_state[kSlots], then slot_data
// queue heads (kQueueHeads u64 counters, 128 B apart) after the slot data
constexpr size_t kCtrlHeads = (kCtrlSlots + sizeof(int) * kSlots + sizeof(int) * kSlots * kTaskInts + 127) & ~size_t(127);

// host-driven balancing: the stop word and the spill counter, a line each
constexpr size_t kCtrlStop = kCtrlHeads + sizeof(unsigned long long) * kHeadStride * kQueueHeads;
constexpr size_t kCtrlSpillN = kCtrlStop + 128;

size_t ctrl_bytes() { return kCtrlSpillN + 128; }

// scheduler fields common to both kernels
Sched make_sched_at(char* c, const Opt& o, int grid, int64_t nq, const int32_t* qroot, const int32_t* qstat) {
  Sched S{};
  S.qhead = reinterpret_cast<unsigned long long*>(c + kCtrlHeads);
  S.state = reinterpret_cast<unsigned long long*>(c + kCtrlState);
  S.idle = reinterpret_cast<int*>(c + kCtrlIdle);
  S.slot_state = reinterpret_cast<int*>(c + kCtrlSlots);
  S.slot_data = reinterpret_cast<int*>(c + kCtrlSlots + sizeof(int) * kSlots);
  S.qroot = qroot;
  S.qlo = nullptr;
  S.qhi = nullptr;
  S.qstat = qstat;
  S.qbounds = nullptr;
  S.nq = nq;
  S.nchunks = 0;
  S.chunk = o.chunk ? static_cast<int>(o.chunk) : 1;
  S.nslots = kSlots;
  S.host_bal = (o.sched & DM_SCHED_HOST_BALANCE) ? 1 : 0;
  S.donate = ((o.sched & DM_NO_DONATION) || S.host_bal) ? 0 : 1;
  S.stop_trigger = grid + 1;  // set by the launch's preparation when host_bal
  S.stop = reinterpret_cast<int*>(c + kCtrlStop);
  S.spill_n = reinterpret_cast<int*>(c + kCtrlSpillN);
  S.spill = nullptr;
  S.spill_cap = 0;
  S.tq = nullptr;
  const float r = o.rebalance > 0.f ? o.rebalance : 0.0f;
  int trig = static_cast<int>(r * grid);
  S.idle_trigger = trig < 1 ? 1 : trig;
  S.period = 64;
  S.waves = grid;
  S.wait_limit = wait_ticks(o.wait_limit_us);
  S.flags = reinterpret_cast<int*>(c + kCtrlFlags);
  return S;
}

Sched make_sched(dm_graph* g, const Opt& o, int grid, int64_t nq, const int32_t* qroot, const int32_t* qstat) {
  return make_sched_at(g->ctrl.as<char>(), o, grid, nq, qroot, qstat);
}

int* ctrl_flags(dm_graph* g) { return reinterpret_cast<int*>(g->ctrl.as<char>() + kCtrlFlags); }

}  // namespace

// ====================================================================== launches

namespace {

// One counting launch, fully prepared: every buffer allocated, the root queue
// built.  enqueue() only issues the clears, the kernel and the copy-back, so a
// prepared launch can be timed repeatedly (autotuner) or captured once into a
// hipGraph and replayed (batches).
// Largest row cache a graph handle keeps (bytes); larger graphs rebuild each
// root's rows on every launch.
constexpr size_t kRowCacheMax = size_t(4) << 30;

struct Prepared {
  bool clique = true;
  CliqueArgs ca;
  MotifArgs ma;
  int grid = 0;
  size_t lds = 0;
  int64_t nq = 0;
  size_t out_count = 0;
  unsigned long long bias = 0;
  unsigned long long* out_dev = nullptr;
  unsigned long long* ctrl = nullptr;
  int64_t ctrl_words = 0;
  unsigned long long* stats = nullptr;
  int64_t stats_words = 0;
  int* flags_dev = nullptr;
  bool* rc_done = nullptr;  // set once this launch has filled the graph's row cache
};

dm_status check_flags(const int* flags) {
  if (flags[1] & kFlagWaitLimit)
    return fail(DM_E_HIP, "an idle wave waited longer than the scheduler's wait limit; the launch was abandoned");
  if (flags[1]) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "internal capacity check failed (0x%x)", flags[1]);
    return fail(DM_E_HIP, buf);
  }
  if (flags[0]) return fail(DM_E_OVERFLOW, "a uint64 counter wrapped");
  return DM_OK;
}

// Clears (fill kernels only: the sequence may be captured into a graph),
// kernel, copy of counters and flags to host memory.
hipError_t enqueue(const Prepared& P, hipStream_t s, uint64_t* host_out, int* host_flags) {
  hipError_t e = launch_fill_u64(P.ctrl, P.ctrl_words, 0ull, s);
  if (e == hipSuccess) e = launch_fill_u64(P.out_dev, static_cast<int64_t>(P.out_count), P.bias, s);
  if (e == hipSuccess && P.stats) e = launch_fill_u64(P.stats, P.stats_words, 0ull, s);
  if (e == hipSuccess && P.nq > 0)
    e = P.clique ? launch_clique(P.ca, P.grid, P.lds, s) : launch_motif(P.ma, P.grid, P.lds, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(host_out, P.out_dev, sizeof(uint64_t) * P.out_count, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(host_flags, P.flags_dev, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  return e;
}

dm_status run_prepared(const Prepared& P, hipStream_t s, uint64_t* host_out) {
  g_last_launches = 1;
  int flags[2] = {0, 0};
  hipError_t e = enqueue(P, s, host_out, flags);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "kernel / copy-back");
  const dm_status st = check_flags(flags);
  if (st == DM_OK && P.rc_done) *P.rc_done = true;
  return st;
}

// Host-driven balancing (Section IV-D: stop, copy the traversal state,
// redistribute, relaunch).  After each stopped launch the spilled tasks are
// copied to the host, every task's untried index range is cut into pieces so
// that the next launch has about two tasks per wave, and the kernel is
// relaunched with those tasks as its queue; counters and per-root records
// accumulate across launches.  After kMaxRelaunch stopped launches the last
// one runs to the end.
constexpr int kMaxRelaunch = 64;

dm_status run_host_balanced(dm_graph* g, Prepared& P, hipStream_t s, uint64_t* host_out) {
  Sched& S = P.clique ? P.ca.S : P.ma.S;
  int flags[2] = {0, 0}, acc_flags[2] = {0, 0};
  hipError_t e = enqueue(P, s, host_out, flags);
  g_last_launches = 1;
  std::vector<int> tasks, next;
  for (int launch = 1;; ++launch) {
    int nspill = 0;
    if (e == hipSuccess)
      e = hipMemcpyAsync(&nspill, reinterpret_cast<char*>(P.ctrl) + kCtrlSpillN, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "host-balanced launch");
    acc_flags[0] |= flags[0];
    acc_flags[1] |= flags[1];
    if (acc_flags[1] || nspill == 0) break;
    if (nspill > S.spill_cap) return fail(DM_E_HIP, "host-balanced launch: spill array overflow");
    tasks.resize(static_cast<size_t>(nspill) * kTaskInts);
    HIP_OR_RETURN(hipMemcpy(tasks.data(), S.spill, sizeof(int) * tasks.size(), hipMemcpyDeviceToHost), "spill copy");
    // redistribute: cut [lo, hi) (ints 4, 5 of a task) into pieces
    int64_t width = 0;
    for (int i = 0; i < nspill; ++i) width += tasks[i * kTaskInts + 5] - tasks[i * kTaskInts + 4];
    const double per = width > 0 ? 2.0 * S.waves / static_cast<double>(width) : 0.0;
    next.clear();
    for (int i = 0; i < nspill; ++i) {
      const int* t = &tasks[static_cast<size_t>(i) * kTaskInts];
      const int lo = t[4], hi = t[5];
      int pieces = static_cast<int>(per * (hi - lo) + 0.5);
      if (pieces < 1) pieces = 1;
      if (pieces > hi - lo) pieces = hi - lo;
      for (int p = 0; p < pieces; ++p) {
        const int a = lo + static_cast<int>(static_cast<int64_t>(hi - lo) * p / pieces);
        const int b = lo + static_cast<int>(static_cast<int64_t>(hi - lo) * (p + 1) / pieces);
        if (a >= b) continue;
        next.insert(next.end(), t, t + kTaskInts);
        next[next.size() - kTaskInts + 4] = a;
        next[next.size() - kTaskInts + 5] = b;
      }
    }
    const int64_t ntask = static_cast<int64_t>(next.size() / kTaskInts);
    HIP_OR_RETURN(g->tq.ensure(sizeof(int) * next.size()), "relaunch queue");
    HIP_OR_RETURN(hipMemcpyAsync(g->tq.p, next.data(), sizeof(int) * next.size(), hipMemcpyHostToDevice, s),
                  "relaunch queue");
    S.tq = g->tq.as<int>();
    S.nq = ntask;
    S.qroot = S.qlo = S.qhi = S.qstat = nullptr;
    S.qbounds = nullptr;
    S.nchunks = 0;
    S.chunk = 1;
    if (launch >= kMaxRelaunch) S.stop_trigger = S.waves + 1;  // the last launch runs to the end
    g_last_launches = launch + 1;
    // relaunch: scheduler words cleared, counters and records kept
    e = launch_fill_u64(P.ctrl, P.ctrl_words, 0ull, s);
    if (e == hipSuccess) e = P.clique ? launch_clique(P.ca, P.grid, P.lds, s) : launch_motif(P.ma, P.grid, P.lds, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(host_out, P.out_dev, sizeof(uint64_t) * P.out_count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(flags, P.flags_dev, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  }
  return check_flags(acc_flags);
}

// queue of explicit roots (original ids), optionally mapped into rank space
dm_status upload_roots(dm_graph* g, const Opt& o, bool to_rank, hipStream_t s) {
  const size_t bytes = sizeof(int32_t) * static_cast<size_t>(o.num_roots);
  HIP_OR_RETURN(g->qroot.ensure(bytes), "roots: allocate");
  for (int64_t i = 0; i < o.num_roots; ++i)
    if (o.roots[i] < 0 || o.roots[i] >= g->n) return fail(DM_E_ARG, "root id out of range");
  if (!to_rank) {
    HIP_OR_RETURN(hipMemcpyAsync(g->qroot.p, o.roots, bytes, hipMemcpyHostToDevice, s), "roots: copy");
    return DM_OK;
  }
  HIP_OR_RETURN(g->qlo.ensure(bytes), "roots: allocate");
  HIP_OR_RETURN(hipMemcpyAsync(g->qlo.p, o.roots, bytes, hipMemcpyHostToDevice, s), "roots: copy");
  HIP_OR_RETURN(launch_gather_i32(g->rank.as<int32_t>(), g->qlo.as<int32_t>(), g->qroot.as<int32_t>(), o.num_roots, s),
                "roots: map");
  return DM_OK;
}

dm_status ensure_features(dm_graph* g, hipStream_t s) {
  if (g->feat_ready) return DM_OK;
  dm_status st = ensure_dag(g, s);
  if (st != DM_OK) return st;
  HIP_OR_RETURN(g->feat.ensure(sizeof(int64_t) * 4 * static_cast<size_t>(g->n > 0 ? g->n : 1)), "features: allocate");
  HIP_OR_RETURN(compute_features(g->rp.as<int64_t>(), g->col.as<int32_t>(), g->n, g->drp.as<int64_t>(),
                                 g->dcol.as<int32_t>(), g->order.as<int32_t>(), g->feat.as<int64_t>(), s),
                "features");
  g->feat_ready = true;
  return DM_OK;
}

// Learned queue: MLP prediction of every root's tree size, longest first,
// chunks of about equal predicted cost (`chunk` chunks per wave, default 8),
// each of at most ceil(n / chunks) roots.  A wave hands the untried part of a
// chunk to idle waves, so a mispredicted chunk does not stall the launch.
// On return g->lqroot holds the queue in rank space, g->lorder the original
// ids (root_stats rows) and g->lqbounds the chunk starts (+ n).  The queue is
// cached on the handle and rebuilt when the parameters' fingerprint, the grid
// or the chunk count change.
dm_status learned_queue(dm_graph* g, const Opt& o, int grid, hipStream_t s, int64_t* nchunks) {
  // predictions: the MLP's on the graph's features, or the caller's costs
  const bool given = o.root_cost != nullptr;
  if (!given) {
    dm_status st = ensure_features(g, s);
    if (st != DM_OK) return st;
  }
  const size_t n = static_cast<size_t>(g->n > 0 ? g->n : 1);
  HIP_OR_RETURN(g->lqkey.ensure(sizeof(unsigned long long)), "learned: allocate");
  HIP_OR_RETURN(param_fingerprint(given ? o.root_cost : o.mlp, given ? g->n : kMlpBlob,
                                  g->lqkey.as<unsigned long long>(), s),
                "learned: fingerprint");
  unsigned long long key = 0;
  HIP_OR_RETURN(hipMemcpyAsync(&key, g->lqkey.p, sizeof(key), hipMemcpyDeviceToHost, s), "learned: fingerprint");
  HIP_OR_RETURN(hipStreamSynchronize(s), "learned: fingerprint");
  if (given) key = ~key;  // keep cost-ordered and MLP-ordered queues apart
  const int per_wave = o.chunk ? static_cast<int>(o.chunk) : 8;
  if (g->lq_valid && key == g->lq_key && grid == g->lq_grid && per_wave == g->lq_per_wave) {
    *nchunks = g->lq_nchunks;
    return DM_OK;
  }
  g->lq_valid = false;
  HIP_OR_RETURN(g->pred.ensure(sizeof(float) * n), "learned: allocate");
  HIP_OR_RETURN(g->lorder.ensure(sizeof(int32_t) * n), "learned: allocate");
  HIP_OR_RETURN(g->lqroot.ensure(sizeof(int32_t) * n), "learned: allocate");
  HIP_OR_RETURN(g->lqbounds.ensure(sizeof(int64_t) * (n + 1)), "learned: allocate");
  if (!given)
    HIP_OR_RETURN(mlp_forward(o.mlp, g->feat.as<int64_t>(), g->n, g->pred.as<float>(), s), "learned: forward");
  HIP_OR_RETURN(lpt_order(given ? o.root_cost : g->pred.as<float>(), g->n, grid * per_wave, g->lorder.as<int32_t>(),
                          g->lqbounds.as<int64_t>(), nchunks, s),
                "learned: order");
  HIP_OR_RETURN(launch_gather_i32(g->rank.as<int32_t>(), g->lorder.as<int32_t>(), g->lqroot.as<int32_t>(), g->n, s),
                "learned: rank map");
  g->lq_valid = true;
  g->lq_key = key;
  g->lq_grid = grid;
  g->lq_per_wave = per_wave;
  g->lq_nchunks = *nchunks;
  return DM_OK;
}

// Root queue shared by both kernels (roots in rank space): explicit list,
// learned LPT order, or all ranks in order.  qstat maps entries to root_stats
// rows (original vertex id, or position in the explicit list).
dm_status build_queue(dm_graph* g, const Opt& o, int grid, hipStream_t s, Sched* S) {
  S->nq = g->n;
  S->qroot = nullptr;
  S->qstat = g->order.as<int32_t>();
  if (o.roots) {
    dm_status st = upload_roots(g, o, true, s);
    if (st != DM_OK) return st;
    S->nq = o.num_roots;
    S->qroot = g->qroot.as<int32_t>();
    S->qstat = nullptr;
  } else if (o.sched & (DM_SCHED_LEARNED | DM_SCHED_COST)) {
    int64_t nchunks = 0;
    dm_status st = learned_queue(g, o, grid, s, &nchunks);
    if (st != DM_OK) return st;
    S->qroot = g->lqroot.as<int32_t>();
    S->qstat = g->lorder.as<int32_t>();
    S->qbounds = g->lqbounds.as<int64_t>();
    S->nchunks = nchunks;
  }
  return DM_OK;
}

void common_prepare(dm_graph* g, const Opt& o, Prepared* P, size_t out_count) {
  P->out_count = out_count;
  P->bias = o.bias;
  P->out_dev = g->out.as<unsigned long long>();
  P->ctrl = g->ctrl.as<unsigned long long>();
  P->ctrl_words = static_cast<int64_t>(ctrl_bytes() / 8);
  P->stats = reinterpret_cast<unsigned long long*>(o.root_stats);
  P->stats_words = o.root_stats ? 3 * (o.roots ? o.num_roots : g->n) : 0;
  P->flags_dev = ctrl_flags(g);
}

// Persistent grid: per_cu waves on every CU, but no more than one wave per 64
// adjacency entries of the graph (never under one wave per CU): on tiny graphs
// extra waves only add contention on the scheduler's words and idle polling.
// (The number of roots is no guide: a few thousand roots of a large graph can
// carry most of its work.)
int size_grid(int per_cu, int64_t nnz) {
  const int full = per_cu * cu_count();
  const int64_t cap = std::max<int64_t>(cu_count(), nnz / 64);
  return static_cast<int>(std::min<int64_t>(full, cap));
}

// Host-driven balancing (Section IV-D): the spill array for the tasks busy
// waves leave behind when the launch is stopped, and the stop trigger: the
// launch stops once fewer than a fraction `active` of its waves are still
// busy and the queue is drained (the paper's thresholds: 40% of the warps for
// cliques, 10% for motifs; dm_options.rebalance overrides).
dm_status prepare_host_balance(dm_graph* g, const Opt& o, int k, int grid, bool clique, Sched* S) {
  if (!S->host_bal) return DM_OK;
  const float active = o.rebalance > 0.f ? o.rebalance : (clique ? 0.4f : 0.1f);
  int trig = grid - static_cast<int>(active * grid);
  S->stop_trigger = trig < 1 ? 1 : trig;
  S->spill_cap = grid * 4 * (k + 1) + 1024;
  HIP_OR_RETURN(g->spill.ensure(sizeof(int) * static_cast<size_t>(S->spill_cap) * kTaskInts), "workspace");
  S->spill = g->spill.as<int>();
  if (!S->qbounds) S->chunk = 1;
  return DM_OK;
}

dm_status prepare_clique(dm_graph* g, int k, const Opt& o, hipStream_t s, const int32_t* root_graph, int ngraphs,
                         Prepared* P) {
  dm_status st = ensure_dag(g, s);
  if (st != DM_OK) return st;
  const int dmax = g->ddmax > 0 ? g->ddmax : 1;
  const int W = (dmax + 63) / 64;
  const size_t lds = clique_lds_bytes(dmax, W, k);
  if (lds > 160 * 1024) return fail(DM_E_NOMEM, "maximum out-degree too large for the LDS stack");
  int per_cu = 0;
  HIP_OR_RETURN(clique_occupancy(lds, &per_cu), "occupancy");
  if (per_cu < 1) per_cu = 1;
  if (o.waves_per_cu && static_cast<int>(o.waves_per_cu) < per_cu) per_cu = static_cast<int>(o.waves_per_cu);
  const int grid = size_grid(per_cu, g->nnz);
  HIP_OR_RETURN(g->ctrl.ensure(ctrl_bytes()), "workspace");
  HIP_OR_RETURN(g->out.ensure(sizeof(uint64_t) * ngraphs), "workspace");
  Sched S = make_sched(g, o, grid, g->n, nullptr, nullptr);
  st = build_queue(g, o, grid, s, &S);
  if (st != DM_OK) return st;
  st = prepare_host_balance(g, o, k, grid, true, &S);
  if (st != DM_OK) return st;
  std::memset(&P->ca, 0, sizeof(P->ca));
  CliqueArgs& A = P->ca;
  A.rp = g->drp.as<int64_t>();
  A.col = g->dcol.as<int32_t>();
  A.n = g->n;
  A.k = k;
  A.dmax = dmax;
  A.W = W;
  A.out = g->out.as<unsigned long long>();
  A.root_graph = root_graph;
  A.flags = ctrl_flags(g);
  A.root_stats = reinterpret_cast<unsigned long long*>(o.root_stats);
  A.wave_stats = reinterpret_cast<unsigned long long*>(o.wave_stats);
  A.wave_stats_len = static_cast<int>(o.wave_stats_len);
  A.prune = o.root_stats ? 0 : 1;
  // row cache: filled by a counting launch over all roots (not a recording
  // one, whose rows path reads member degrees), read by every later launch
  A.rc_mode = 0;
  A.rcache = nullptr;
  A.rcoff = nullptr;
  if (!o.root_stats && k >= 3) {
    if (!g->rc_layout) {
      HIP_OR_RETURN(g->rcoff.ensure(sizeof(int64_t) * (static_cast<size_t>(g->n) + 1)), "row cache: allocate");
      HIP_OR_RETURN(row_cache_layout(g->drp.as<int64_t>(), g->n, g->rcoff.as<int64_t>(), &g->rc_words, s),
                    "row cache: layout");
      g->rc_layout = true;
    }
    const size_t bytes = sizeof(uint64_t) * static_cast<size_t>(g->rc_words > 0 ? g->rc_words : 1);
    if (bytes <= kRowCacheMax && (g->rc_ready || !o.roots)) {
      HIP_OR_RETURN(g->rcache.ensure(bytes), "row cache: allocate");
      A.rc_mode = g->rc_ready ? 2 : 1;
      A.rcache = g->rcache.as<unsigned long long>();
      A.rcoff = g->rcoff.as<int64_t>();
    }
  }
  // rows of roots with more than kLocalMax out-neighbours when no row cache
  // serves the launch: one region per wave
  A.rows_global = nullptr;
  if (A.rc_mode == 0 && dmax > kCliqueLocalRows) {
    HIP_OR_RETURN(g->rows.ensure(sizeof(uint64_t) * static_cast<size_t>(grid) * W * dmax), "workspace");
    A.rows_global = g->rows.as<unsigned long long>();
  }
  A.S = S;
  P->clique = true;
  P->grid = grid;
  P->lds = lds;
  P->nq = S.nq;
  common_prepare(g, o, P, static_cast<size_t>(ngraphs));
  P->rc_done = A.rc_mode == 1 ? &g->rc_ready : nullptr;
  return DM_OK;
}

dm_status prepare_motif(dm_graph* g, int k, const Opt& o, hipStream_t s, const int32_t* root_graph, int ngraphs,
                        Prepared* P) {
  const ClassTables* T = tables(k);
  uint16_t* dtab = nullptr;
  HIP_OR_RETURN(device_table(k, &dtab), "class table upload");
  dm_status st = ensure_ranked(g, s);
  if (st != DM_OK) return st;
  const int dmax = g->dmax > 0 ? g->dmax : 1;
  const size_t lds = motif_lds_bytes(k, T->ncls);
  int per_cu = 0;
  HIP_OR_RETURN(motif_occupancy(k, lds, &per_cu), "occupancy");
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 16) per_cu = 16;  // the extension stacks live in global memory; bound the footprint
  if (o.waves_per_cu && static_cast<int>(o.waves_per_cu) < per_cu) per_cu = static_cast<int>(o.waves_per_cu);
  const int grid = size_grid(per_cu, g->nnz);
  std::memset(&P->ma, 0, sizeof(P->ma));
  MotifArgs& A = P->ma;
  int64_t cap_total = 0;
  for (int s2 = 1; s2 <= k - 2 && s2 < 8; ++s2) {
    A.level_off[s2] = cap_total;
    A.level_cap[s2] = static_cast<int64_t>(s2) * dmax;
    cap_total += A.level_cap[s2];
  }
  HIP_OR_RETURN(g->ctrl.ensure(ctrl_bytes()), "workspace");
  HIP_OR_RETURN(g->out.ensure(sizeof(uint64_t) * static_cast<size_t>(ngraphs) * T->ncls), "workspace");
  HIP_OR_RETURN(g->ext_vert.ensure(sizeof(int32_t) * static_cast<size_t>(grid) * cap_total), "workspace");
  HIP_OR_RETURN(g->ext_mask.ensure(static_cast<size_t>(grid) * cap_total), "workspace");
  HIP_OR_RETURN(g->newbuf.ensure(sizeof(int32_t) * static_cast<size_t>(grid) * dmax), "workspace");
  if (k == 8)  // class counters do not fit LDS: one row per wave in global memory
    HIP_OR_RETURN(g->wave_cnt.ensure(sizeof(uint64_t) * static_cast<size_t>(grid) * T->ncls), "workspace");
  Sched S = make_sched(g, o, grid, g->n, nullptr, nullptr);
  st = build_queue(g, o, grid, s, &S);
  if (st != DM_OK) return st;
  st = prepare_host_balance(g, o, k, grid, false, &S);
  if (st != DM_OK) return st;
  A.rp = g->urp.as<int64_t>();
  A.col = g->ucol.as<int32_t>();
  A.n = g->n;
  A.k = k;
  A.dmax = dmax;
  A.ncls = T->ncls;
  A.table = dtab;
  A.out = g->out.as<unsigned long long>();
  A.root_graph = root_graph;
  A.flags = ctrl_flags(g);
  A.root_stats = reinterpret_cast<unsigned long long*>(o.root_stats);
  A.wave_stats = reinterpret_cast<unsigned long long*>(o.wave_stats);
  A.wave_stats_len = static_cast<int>(o.wave_stats_len);
  A.ext_vert = g->ext_vert.as<int32_t>();
  A.ext_mask = g->ext_mask.as<uint8_t>();
  A.new_buf = g->newbuf.as<int32_t>();
  A.wave_ext_cap = cap_total;
  A.leaf_lds = 1;
  A.wave_cnt = k == 8 ? g->wave_cnt.as<unsigned long long>() : nullptr;
  A.S = S;
  P->clique = false;
  P->grid = grid;
  P->lds = lds;
  P->nq = S.nq;
  common_prepare(g, o, P, static_cast<size_t>(ngraphs) * T->ncls);
  return DM_OK;
}

dm_status prepare(dm_graph* g, int op, int k, const Opt& o, hipStream_t s, const int32_t* root_graph, int ngraphs,
                  Prepared* P) {
  return op == DM_OP_CLIQUE ? prepare_clique(g, k, o, s, root_graph, ngraphs, P)
                            : prepare_motif(g, k, o, s, root_graph, ngraphs, P);
}

// ---------------------------------------------------------------- autotuning
//
// Coordinate search over the scheduling knobs that never change a count:
// roots per queue grab, the idle fraction that enables donation, and resident
// waves per CU.  Each candidate is one timed launch of the prepared work.  The
// best setting is cached per (operation, k) for DM_SCHED_AUTOTUNE callers.

struct Tuning {
  uint32_t chunk = 0;
  float rebalance = 0.f;
  uint32_t waves_per_cu = 0;
  float ms = 0.f;
};

std::mutex g_tune_lock;
std::map<std::pair<int, int>, Tuning> g_tune;

void apply_tuning(int op, int k, Opt* o) {
  if (!(o->sched & DM_SCHED_AUTOTUNE)) return;
  std::lock_guard<std::mutex> lk(g_tune_lock);
  auto it = g_tune.find(std::make_pair(op, k));
  if (it == g_tune.end()) return;
  if (!o->chunk) o->chunk = it->second.chunk;
  if (o->rebalance <= 0.f) o->rebalance = it->second.rebalance;
  if (!o->waves_per_cu) o->waves_per_cu = it->second.waves_per_cu;
}

dm_status time_launch(dm_graph* g, int op, int k, const Opt& o, hipStream_t s, const int32_t* root_graph, int ngraphs,
                      float* ms) {
  Prepared P;
  dm_status st = prepare(g, op, k, o, s, root_graph, ngraphs, &P);
  if (st != DM_OK) return st;
  std::vector<uint64_t> out(P.out_count);
  int flags[2];
  hipEvent_t a, b;
  HIP_OR_RETURN(hipEventCreate(&a), "tune: event");
  HIP_OR_RETURN(hipEventCreate(&b), "tune: event");
  hipError_t e = hipEventRecord(a, s);
  if (e == hipSuccess) e = enqueue(P, s, out.data(), flags);
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "tune: launch");
  st = check_flags(flags);
  if (st == DM_OK && P.rc_done) *P.rc_done = true;
  return st;
}

dm_status autotune(dm_graph* g, int op, int k, const Opt& base, hipStream_t s, const int32_t* root_graph, int ngraphs,
                   Tuning* best) {
  Opt o = base;
  o.sched &= ~static_cast<uint32_t>(DM_SCHED_AUTOTUNE | DM_RECORD_ROOTS);
  o.root_stats = nullptr;
  o.wave_stats = nullptr;
  o.chunk = 1;
  o.rebalance = 0.f;
  o.waves_per_cu = 0;
  float ms = 0.f;
  dm_status st = time_launch(g, op, k, o, s, root_graph, ngraphs, &ms);  // warm-up (allocations, caches)
  if (st != DM_OK) return st;
  auto measure = [&](const Opt& c, float* out_ms) -> dm_status {
    float m1 = 0.f, m2 = 0.f;
    dm_status r = time_launch(g, op, k, c, s, root_graph, ngraphs, &m1);
    if (r == DM_OK) r = time_launch(g, op, k, c, s, root_graph, ngraphs, &m2);
    *out_ms = std::min(m1, m2);
    return r;
  };
  float best_ms = 0.f;
  st = measure(o, &best_ms);
  if (st != DM_OK) return st;
  for (uint32_t c : {2u, 4u, 8u, 16u, 32u, 64u, 128u}) {
    Opt t = o;
    t.chunk = c;
    float m = 0.f;
    st = measure(t, &m);
    if (st != DM_OK) return st;
    if (m < best_ms) { best_ms = m; o.chunk = c; }
  }
  for (float r : {0.02f, 0.05f, 0.1f, 0.2f, 0.4f}) {
    Opt t = o;
    t.rebalance = r;
    float m = 0.f;
    st = measure(t, &m);
    if (st != DM_OK) return st;
    if (m < best_ms) { best_ms = m; o.rebalance = r; }
  }
  for (uint32_t w : {1u, 2u, 4u, 8u}) {
    Opt t = o;
    t.waves_per_cu = w;
    float m = 0.f;
    st = measure(t, &m);
    if (st != DM_OK) return st;
    if (m < best_ms) { best_ms = m; o.waves_per_cu = w; }
  }
  best->chunk = o.chunk;
  best->rebalance = o.rebalance;
  best->waves_per_cu = o.waves_per_cu;
  best->ms = best_ms;
  std::lock_guard<std::mutex> lk(g_tune_lock);
  g_tune[std::make_pair(op, k)] = *best;
  return DM_OK;
}

}  // namespace

// ---------------------------------------------------------------- one lane per traversal (ablation)

namespace {

// Per-lane stacks are capped at this many bytes in total; the grid shrinks
// to the lanes that fit.
constexpr size_t kDfsStackMax = size_t(4) << 30;

dm_status run_dfs(dm_graph* g, int op, int k, const Opt& o, hipStream_t s, uint64_t* host_out, int ncls) {
  DfsArgs A;
  std::memset(&A, 0, sizeof A);
  int dmax = 1;
  if (op == DM_OP_CLIQUE) {
    if (k > kDfsMaxK) return fail(DM_E_K, "DM_IMPL_DFS counts cliques up to k = 16");
    dm_status st = ensure_dag(g, s);
    if (st != DM_OK) return st;
    A.rp = g->drp.as<int64_t>();
    A.col = g->dcol.as<int32_t>();
    dmax = g->ddmax > 0 ? g->ddmax : 1;
    A.lane_stride = static_cast<int64_t>(k > 3 ? k - 3 : 1) * dmax;
  } else {
    // the lane kernel keeps one wave's class counters in LDS: 853 fit, 11,117 do not
    if (k > 7) return fail(DM_E_K, "DM_IMPL_DFS counts motifs up to k = 7");
    uint16_t* dtab = nullptr;
    HIP_OR_RETURN(device_table(k, &dtab), "class table upload");
    dm_status st = ensure_ranked(g, s);
    if (st != DM_OK) return st;
    A.rp = g->urp.as<int64_t>();
    A.col = g->ucol.as<int32_t>();
    dmax = g->dmax > 0 ? g->dmax : 1;
    A.table = dtab;
    A.ncls = ncls;
    int64_t off = 0;
    for (int s2 = 1; s2 <= k - 1; ++s2) {
      A.level_off[s2] = off;
      A.level_cap[s2] = static_cast<int64_t>(s2) * dmax;
      off += A.level_cap[s2];
    }
    A.lane_stride = off;
  }
  A.n = g->n;
  A.k = k;
  A.dmax = dmax;
  const size_t lane_bytes = static_cast<size_t>(A.lane_stride) * (op == DM_OP_CLIQUE ? 4 : 5);
  int per_cu = o.waves_per_cu ? static_cast<int>(o.waves_per_cu) : 16;
  int grid = size_grid(per_cu, g->nnz);
  const int64_t fit = static_cast<int64_t>(kDfsStackMax / (lane_bytes * kWave));
  if (fit < 1) return fail(DM_E_NOMEM, "DM_IMPL_DFS: one wave's stacks exceed the cap");
  if (fit < grid) grid = static_cast<int>(fit);
  HIP_OR_RETURN(g->ctrl.ensure(ctrl_bytes()), "workspace");
  HIP_OR_RETURN(g->out.ensure(sizeof(uint64_t) * ncls), "workspace");
  HIP_OR_RETURN(g->dfs_stack.ensure(sizeof(int32_t) * static_cast<size_t>(A.lane_stride) * grid * kWave), "dfs stacks");
  if (op == DM_OP_MOTIF)
    HIP_OR_RETURN(g->dfs_mask.ensure(static_cast<size_t>(A.lane_stride) * grid * kWave), "dfs stacks");
  char* c = g->ctrl.as<char>();
  A.qhead = reinterpret_cast<unsigned long long*>(c + kCtrlHeads);
  A.flags = reinterpret_cast<int*>(c + kCtrlFlags);
  A.out = g->out.as<unsigned long long>();
  A.stack = g->dfs_stack.as<int32_t>();
  A.masks = op == DM_OP_MOTIF ? g->dfs_mask.as<uint8_t>() : nullptr;
  HIP_OR_RETURN(launch_fill_u64(g->ctrl.as<unsigned long long>(), static_cast<int64_t>(ctrl_bytes() / 8), 0ull, s), "clear");
  HIP_OR_RETURN(launch_fill_u64(A.out, ncls, o.bias, s), "clear");
  if (g->n > 0)
    HIP_OR_RETURN(op == DM_OP_CLIQUE ? launch_dfs_clique(A, grid, s) : launch_dfs_motif(A, grid, s), "dfs kernel");
  int flags[2] = {0, 0};
  HIP_OR_RETURN(hipMemcpyAsync(host_out, A.out, sizeof(uint64_t) * ncls, hipMemcpyDeviceToHost, s), "copy-back");
  HIP_OR_RETURN(hipMemcpyAsync(flags, A.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "copy-back");
  HIP_OR_RETURN(hipStreamSynchronize(s), "dfs kernel");
  return check_flags(flags);
}

}  // namespace

extern "C" dm_status dm_count_cliques(dm_graph* g, int k, uint64_t* out_count, const dm_options* opt) {
  if (!g || !out_count) return fail(DM_E_ARG, "null graph or output");
  if (k < 1 || k > kMaxK) return fail(DM_E_K, "clique k must be in 1..32");
  Opt o;
  dm_status st = read_opt(opt, &o);
  if (st != DM_OK) return st;
  if ((o.sched & DM_SCHED_LEARNED) && !o.mlp) return fail(DM_E_MODEL, "DM_SCHED_LEARNED needs mlp parameters");
  hipStream_t s = pick_stream(g, o.stream);
  uint64_t c = 0;
  if (o.sched & DM_IMPL_DFS) {
    st = run_dfs(g, DM_OP_CLIQUE, k, o, s, &c, 1);
    if (st == DM_OK) *out_count = c;
    return st;
  }
  apply_tuning(DM_OP_CLIQUE, k, &o);
  Prepared P;
  st = prepare(g, DM_OP_CLIQUE, k, o, s, nullptr, 1, &P);
  if (st == DM_OK) st = (o.sched & DM_SCHED_HOST_BALANCE) ? run_host_balanced(g, P, s, &c) : run_prepared(P, s, &c);
  if (st == DM_OK) *out_count = c;
  return st;
}

extern "C" dm_status dm_count_motifs(dm_graph* g, int k, uint64_t* out_counts, size_t out_len, const dm_options* opt) {
  if (!g || !out_counts) return fail(DM_E_ARG, "null graph or output");
  const ClassTables* T = tables(k);
  if (!T) return fail(DM_E_K, "motif k must be in 3..8");
  if (out_len < static_cast<size_t>(T->ncls)) return fail(DM_E_BUFSZ, "out_len < number of classes");
  Opt o;
  dm_status st = read_opt(opt, &o);
  if (st != DM_OK) return st;
  if ((o.sched & DM_SCHED_LEARNED) && !o.mlp) return fail(DM_E_MODEL, "DM_SCHED_LEARNED needs mlp parameters");
  hipStream_t s = pick_stream(g, o.stream);
  std::vector<uint64_t> tmp(T->ncls);
  if (o.sched & DM_IMPL_DFS) {
    st = run_dfs(g, DM_OP_MOTIF, k, o, s, tmp.data(), T->ncls);
    if (st == DM_OK) std::memcpy(out_counts, tmp.data(), sizeof(uint64_t) * T->ncls);
    return st;
  }
  apply_tuning(DM_OP_MOTIF, k, &o);
  Prepared P;
  st = prepare(g, DM_OP_MOTIF, k, o, s, nullptr, 1, &P);
  if (st == DM_OK)
    st = (o.sched & DM_SCHED_HOST_BALANCE) ? run_host_balanced(g, P, s, tmp.data()) : run_prepared(P, s, tmp.data());
  if (st == DM_OK) std::memcpy(out_counts, tmp.data(), sizeof(uint64_t) * T->ncls);
  return st;
}

// ====================================================================== motif counting without allocation

namespace {

// Device memory of dm_count_motifs_static: the dictionary, the scheduler's
// control block, the class counters and the per-wave extension stacks of one
// launch.  Every device the library runs on holds its own copy until the
// process ends.  Host code never passes `scratch` itself (in host code the
// name is only a stand-in): it uses the address hipGetSymbolAddress returns
// for the current device, looked up once per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_lock;
unsigned char* g_scratch_ptr[kMaxDevices] = {nullptr};
int g_scratch_table_k[kMaxDevices] = {0};  // dictionary currently held by the device's scratch

constexpr size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }
// The layout starts with room for the largest dictionary (k = 7: 2^20
// 16-bit ids), then the control block; the counters (up to 853) and the
// per-wave stacks follow, sized per call.
constexpr size_t kScratchTable = 0;
constexpr size_t kScratchCtrl = align256(sizeof(uint16_t) << 20);

}  // namespace

extern "C" dm_status dm_count_motifs_static(dm_graph* g, int k, uint64_t* out_counts, size_t out_len,
                                            const dm_options* opt) {
  if (!g || !out_counts) return fail(DM_E_ARG, "null graph or output");
  // k = 8's dictionary (256 MiB) does not fit the static array
  const ClassTables* T = k <= 7 ? tables(k) : nullptr;
  if (!T) return fail(DM_E_K, "dm_count_motifs_static: motif k must be in 3..7");
  if (out_len < static_cast<size_t>(T->ncls)) return fail(DM_E_BUFSZ, "out_len < number of classes");
  Opt o;
  dm_status st = read_opt(opt, &o);
  if (st != DM_OK) return st;
  if (o.sched & (DM_SCHED_LEARNED | DM_SCHED_COST | DM_IMPL_DFS | DM_SCHED_HOST_BALANCE) || o.roots)
    return fail(DM_E_ARG, "dm_count_motifs_static runs the plain root queue over every root (no learned or "
                          "cost ordering, root list, host-driven balancing or DFS ablation)");
  if (!g->ranked)
    return fail(DM_E_ARG, "dm_count_motifs_static needs the rank-renamed graph: load it with DM_CSR_RANK "
                          "(or count its motifs once with dm_count_motifs)");
  int dev = 0;
  HIP_OR_RETURN(hipGetDevice(&dev), "dm_count_motifs_static: device");
  if (dev < 0 || dev >= kMaxDevices) return fail(DM_E_ARG, "device ordinal beyond the library's table");
  std::lock_guard<std::mutex> lk(g_scratch_lock);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_OR_RETURN(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "dm_count_motifs_static: scratch address");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  unsigned char* base = g_scratch_ptr[dev];
  hipStream_t s = o.stream ? o.stream : g->own;
  apply_tuning(DM_OP_MOTIF, k, &o);

  // layout: table | control block | counters | per-wave stacks
  const size_t off_out = kScratchCtrl + align256(ctrl_bytes());
  const size_t off_waves = off_out + align256(sizeof(uint64_t) * 853);
  const int dmax = g->dmax > 0 ? g->dmax : 1;
  int64_t cap_total = 0;
  int64_t level_off[8] = {0}, level_cap[8] = {0};
  for (int s2 = 1; s2 <= k - 2 && s2 < 8; ++s2) {
    level_off[s2] = cap_total;
    level_cap[s2] = static_cast<int64_t>(s2) * dmax;
    cap_total += level_cap[s2];
  }
  const size_t vert_bytes = sizeof(int32_t) * static_cast<size_t>(cap_total);
  const size_t per_wave = vert_bytes + static_cast<size_t>(cap_total) + sizeof(int32_t) * static_cast<size_t>(dmax);
  const size_t room = kScratchBytes - off_waves - 3 * 256;
  const int64_t fit = static_cast<int64_t>(room / per_wave);
  if (fit < 1) {
    char buf[192];
    std::snprintf(buf, sizeof buf,
                  "one wave's extension stack (%zu bytes for max degree %d at k = %d) exceeds the %zu-byte static "
                  "scratch; use dm_count_motifs", per_wave, dmax, k, kScratchBytes);
    return fail(DM_E_NOMEM, buf);
  }
  const size_t lds = motif_lds_bytes(k, T->ncls);
  int per_cu = 0;
  HIP_OR_RETURN(motif_occupancy(k, lds, &per_cu), "occupancy");
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 16) per_cu = 16;
  if (o.waves_per_cu && static_cast<int>(o.waves_per_cu) < per_cu) per_cu = static_cast<int>(o.waves_per_cu);
  int grid = size_grid(per_cu, g->nnz);
  if (fit < grid) grid = static_cast<int>(fit);
  const size_t off_vert = off_waves;
  const size_t off_mask = align256(off_vert + vert_bytes * grid);
  const size_t off_new = align256(off_mask + static_cast<size_t>(cap_total) * grid);

  if (g_scratch_table_k[dev] != k) {
    g_scratch_table_k[dev] = 0;
    HIP_OR_RETURN(hipMemcpyAsync(base + kScratchTable, T->table.data(), T->table.size() * sizeof(uint16_t),
                                 hipMemcpyHostToDevice, s),
                  "dm_count_motifs_static: dictionary");
    g_scratch_table_k[dev] = k;
  }
  char* ctrl = reinterpret_cast<char*>(base + kScratchCtrl);
  MotifArgs A;
  std::memset(&A, 0, sizeof A);
  for (int s2 = 0; s2 < 8; ++s2) {
    A.level_off[s2] = level_off[s2];
    A.level_cap[s2] = level_cap[s2];
  }
  Sched S = make_sched_at(ctrl, o, grid, g->n, nullptr, g->order.as<int32_t>());
  A.rp = g->urp.as<int64_t>();
  A.col = g->ucol.as<int32_t>();
  A.n = g->n;
  A.k = k;
  A.dmax = dmax;
  A.ncls = T->ncls;
  A.table = reinterpret_cast<const uint16_t*>(base + kScratchTable);
  A.out = reinterpret_cast<unsigned long long*>(base + off_out);
  A.root_graph = nullptr;
  A.flags = reinterpret_cast<int*>(ctrl + kCtrlFlags);
  A.root_stats = reinterpret_cast<unsigned long long*>(o.root_stats);
  A.wave_stats = reinterpret_cast<unsigned long long*>(o.wave_stats);
  A.wave_stats_len = static_cast<int>(o.wave_stats_len);
  A.ext_vert = reinterpret_cast<int32_t*>(base + off_vert);
  A.ext_mask = reinterpret_cast<uint8_t*>(base + off_mask);
  A.new_buf = reinterpret_cast<int32_t*>(base + off_new);
  A.wave_ext_cap = cap_total;
  A.leaf_lds = 1;
  A.S = S;
  // clears by fill kernels, the persistent kernel, copies of counters and flags
  int flags[2] = {0, 0};
  hipError_t e = launch_fill_u64(reinterpret_cast<unsigned long long*>(ctrl), static_cast<int64_t>(ctrl_bytes() / 8),
                                 0ull, s);
  if (e == hipSuccess) e = launch_fill_u64(A.out, T->ncls, o.bias, s);
  if (e == hipSuccess && A.root_stats) e = launch_fill_u64(A.root_stats, 3 * static_cast<int64_t>(g->n), 0ull, s);
  if (e == hipSuccess && g->n > 0) e = launch_motif(A, grid, lds, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_counts, A.out, sizeof(uint64_t) * T->ncls, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(flags, A.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "dm_count_motifs_static: kernel / copy-back");
  return check_flags(flags);
}

// ====================================================================== listing (aggregate_store)

namespace {

constexpr int kRingBlocks = 8;
constexpr int kRingRowsPerBlock = 1 << 16;

// pinned host memory of one listing call
struct HostRing {
  int32_t* rows = nullptr;
  unsigned* valid = nullptr;
  unsigned long long* freed = nullptr;
  ~HostRing() {
    if (rows) (void)hipHostFree(rows);
    if (valid) (void)hipHostFree(valid);
    if (freed) (void)hipHostFree(freed);
  }
};

}  // namespace

extern "C" dm_status dm_list(dm_graph* g, int op, int k, dm_sink_fn sink, void* user, uint64_t* out_total,
                             const dm_options* opt) {
  if (!g || !sink || !out_total) return fail(DM_E_ARG, "null graph, sink or output");
  if (op != DM_OP_CLIQUE && op != DM_OP_MOTIF) return fail(DM_E_ARG, "unknown op");
  const ClassTables* T = nullptr;
  if (op == DM_OP_CLIQUE) {
    if (k < 1 || k > kMaxK) return fail(DM_E_K, "clique k must be in 1..32");
  } else {
    T = tables(k);
    if (!T) return fail(DM_E_K, "motif k must be in 3..8");
  }
  Opt o;
  dm_status st = read_opt(opt, &o);
  if (st != DM_OK) return st;
  if ((o.sched & ~static_cast<uint32_t>(DM_NO_DONATION | DM_SCHED_AUTOTUNE)) || o.roots)
    return fail(DM_E_ARG, "dm_list runs the plain root queue over every root, with no records, learned or cost "
                          "ordering, root list or DFS ablation");
  hipStream_t s = pick_stream(g, o.stream);
  const int width = op == DM_OP_CLIQUE ? k : k + 1;
  const int64_t slots = static_cast<int64_t>(kRingRowsPerBlock) * kRingBlocks;
  HostRing H;
  HIP_OR_RETURN(hipHostMalloc(reinterpret_cast<void**>(&H.rows), sizeof(int32_t) * slots * width, hipHostMallocCoherent),
                "dm_list: ring");
  HIP_OR_RETURN(hipHostMalloc(reinterpret_cast<void**>(&H.valid), sizeof(unsigned) * slots, hipHostMallocCoherent),
                "dm_list: ring");
  HIP_OR_RETURN(hipHostMalloc(reinterpret_cast<void**>(&H.freed), sizeof(unsigned long long) * kRingBlocks,
                              hipHostMallocCoherent),
                "dm_list: ring");
  std::memset(H.valid, 0, sizeof(unsigned) * slots);
  std::memset(H.freed, 0, sizeof(unsigned long long) * kRingBlocks);
  // the persistent grid leaves most wave slots of each CU free: the host
  // drains while the kernel runs, and nothing else must be starved of a CU
  const int grid = size_grid(4, g->nnz);
  HIP_OR_RETURN(g->ctrl.ensure(ctrl_bytes()), "workspace");
  HIP_OR_RETURN(g->out.ensure(sizeof(unsigned long long)), "workspace");
  char* c = g->ctrl.as<char>();
  Opt ol = o;
  ol.sched |= DM_NO_DONATION;  // listing launches take roots from the queue only
  Ring R;
  R.rows = H.rows;
  R.valid = H.valid;
  R.freed = H.freed;
  R.reserve = g->out.as<unsigned long long>();
  R.width = width;
  R.rows_per_block = kRingRowsPerBlock;
  R.nblocks = kRingBlocks;
  R.wait_limit = wait_ticks(o.wait_limit_us);
  R.flags = reinterpret_cast<int*>(c + kCtrlFlags);
  HIP_OR_RETURN(launch_fill_u64(g->ctrl.as<unsigned long long>(), static_cast<int64_t>(ctrl_bytes() / 8), 0ull, s),
                "clear");
  HIP_OR_RETURN(launch_fill_u64(R.reserve, 1, 0ull, s), "clear");
  if (op == DM_OP_CLIQUE) {
    st = ensure_dag(g, s);
    if (st != DM_OK) return st;
    CliqueListArgs A;
    std::memset(&A, 0, sizeof A);
    A.rp = g->drp.as<int64_t>();
    A.col = g->dcol.as<int32_t>();
    A.n = g->n;
    A.k = k;
    A.dmax = g->ddmax > 0 ? g->ddmax : 1;
    HIP_OR_RETURN(g->ext_vert.ensure(sizeof(int32_t) * static_cast<size_t>(grid) * (k > 1 ? k - 1 : 1) * A.dmax),
                  "workspace");
    A.stack = g->ext_vert.as<int32_t>();
    A.flags = R.flags;
    A.S = make_sched(g, ol, grid, g->n, nullptr, nullptr);
    R.order = g->order.as<int32_t>();
    A.R = R;
    if (g->n > 0) HIP_OR_RETURN(launch_list_cliques(A, grid, s), "listing kernel");
  } else {
    uint16_t* dtab = nullptr;
    HIP_OR_RETURN(device_table(k, &dtab), "class table upload");
    st = ensure_ranked(g, s);
    if (st != DM_OK) return st;
    MotifArgs A;
    std::memset(&A, 0, sizeof A);
    const int dmax = g->dmax > 0 ? g->dmax : 1;
    int64_t cap_total = 0;
    for (int s2 = 1; s2 <= k - 1 && s2 < 8; ++s2) {
      A.level_off[s2] = cap_total;
      A.level_cap[s2] = static_cast<int64_t>(s2) * dmax;
      cap_total += A.level_cap[s2];
    }
    HIP_OR_RETURN(g->ext_vert.ensure(sizeof(int32_t) * static_cast<size_t>(grid) * cap_total), "workspace");
    HIP_OR_RETURN(g->ext_mask.ensure(static_cast<size_t>(grid) * cap_total), "workspace");
    HIP_OR_RETURN(g->newbuf.ensure(sizeof(int32_t) * static_cast<size_t>(grid) * dmax), "workspace");
    A.rp = g->urp.as<int64_t>();
    A.col = g->ucol.as<int32_t>();
    A.n = g->n;
    A.k = k;
    A.dmax = dmax;
    A.ncls = T->ncls;
    A.table = dtab;
    A.flags = R.flags;
    A.ext_vert = g->ext_vert.as<int32_t>();
    A.ext_mask = g->ext_mask.as<uint8_t>();
    A.new_buf = g->newbuf.as<int32_t>();
    A.wave_ext_cap = cap_total;
    A.leaf_lds = 0;
    A.S = make_sched(g, ol, grid, g->n, nullptr, nullptr);
    R.order = g->order.as<int32_t>();
    if (g->n > 0) HIP_OR_RETURN(launch_list_motifs(A, R, grid, motif_list_lds_bytes(), s), "listing kernel");
  }
  // drain: deliver rows in order as their valid words appear; a block is
  // handed back to the kernel once all its rows of a generation are delivered
  uint64_t tail = 0, reserved = 0;
  int flags[2] = {0, 0};
  bool done = false;
  int stalls = 0;
  const volatile unsigned* valid = H.valid;
  for (;;) {
    uint64_t r = tail;
    const uint64_t block_end = (tail / kRingRowsPerBlock + 1) * kRingRowsPerBlock;
    while (r < block_end && valid[r % slots] == static_cast<unsigned>(r / slots + 1)) ++r;
    if (r > tail) {
      std::atomic_thread_fence(std::memory_order_acquire);
      sink(H.rows + static_cast<int64_t>(tail % slots) * width, r - tail, width, user);
      tail = r;
      if (tail == block_end) {
        const uint64_t last = tail - 1;
        const int b = static_cast<int>((last % slots) / kRingRowsPerBlock);
        std::atomic_thread_fence(std::memory_order_release);
        __atomic_store_n(H.freed + b, static_cast<unsigned long long>(last / slots + 1), __ATOMIC_RELEASE);
      }
      continue;
    }
    if (done) {
      // every reserved row is written before the kernel ends, unless a wave
      // gave up waiting (flagged); rows that never show up fail the call
      if (tail >= reserved || flags[1]) break;
      if (++stalls > 50000) return fail(DM_E_HIP, "dm_list: reserved rows never became visible to the host");
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      continue;
    }
    const hipError_t q = hipStreamQuery(s);
    if (q == hipSuccess) {
      HIP_OR_RETURN(hipMemcpyAsync(&reserved, R.reserve, sizeof(uint64_t), hipMemcpyDeviceToHost, s), "copy-back");
      HIP_OR_RETURN(hipMemcpyAsync(flags, R.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "copy-back");
      HIP_OR_RETURN(hipStreamSynchronize(s), "copy-back");
      done = true;
      continue;
    }
    if (q != hipErrorNotReady) return hip_fail(q, "listing kernel");
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  st = check_flags(flags);
  if (st != DM_OK) return st;
  *out_total = tail;
  return DM_OK;
}

// ====================================================================== property filters

extern "C" dm_status dm_induced_subgraph(dm_graph* g, const uint8_t* keep, void* stream, dm_graph** out) {
  if (!out) return fail(DM_E_ARG, "null output handle");
  *out = nullptr;
  if (!g || (!keep && g->n > 0)) return fail(DM_E_ARG, "null graph or keep array");
  hipStream_t s = pick_stream(g, stream);
  const size_t n1 = static_cast<size_t>(g->n) + 1;
  Buf dkeep, newid, srp;
  HIP_OR_RETURN(dkeep.ensure(n1), "dm_induced_subgraph: allocate");
  HIP_OR_RETURN(newid.ensure(sizeof(int64_t) * n1), "dm_induced_subgraph: allocate");
  HIP_OR_RETURN(srp.ensure(sizeof(int64_t) * n1), "dm_induced_subgraph: allocate");
  if (g->n > 0)
    HIP_OR_RETURN(hipMemcpyAsync(dkeep.p, keep, static_cast<size_t>(g->n), hipMemcpyHostToDevice, s),
                  "dm_induced_subgraph: copy");
  int32_t* scol = nullptr;
  int32_t n2 = 0;
  int64_t nnz2 = 0;
  if (g->n > 0)
    HIP_OR_RETURN(induced_subgraph(g->rp.as<int64_t>(), g->col.as<int32_t>(), g->n, dkeep.as<uint8_t>(),
                                   newid.as<int64_t>(), srp.as<int64_t>(), &scol, &n2, &nnz2, s),
                  "dm_induced_subgraph");
  else
    HIP_OR_RETURN(hipMemsetAsync(srp.p, 0, sizeof(int64_t), s), "dm_induced_subgraph");
  // (with no edges no column is read; a placeholder pointer keeps the call valid)
  int32_t none = 0;
  const dm_status st = dm_load_csr(n2, srp.as<int64_t>(), scol ? scol : &none, DM_CSR_DEVICE | DM_CSR_TRUSTED,
                                   stream, out);
  if (scol) (void)hipFree(scol);
  return st;
}

extern "C" dm_status dm_count_quasi_cliques(dm_graph* g, int k, int min_edges, uint64_t* out_count,
                                            const dm_options* opt) {
  if (!g || !out_count) return fail(DM_E_ARG, "null graph or output");
  const ClassTables* T = tables(k);
  if (!T) return fail(DM_E_K, "quasi-cliques: k must be in 3..8");
  if (min_edges < 0 || min_edges > k * (k - 1) / 2) return fail(DM_E_ARG, "min_edges outside 0..k(k-1)/2");
  std::vector<uint64_t> c(T->ncls);
  const dm_status st = dm_count_motifs(g, k, c.data(), c.size(), opt);
  if (st != DM_OK) return st;
  uint64_t sum = 0;
  for (int q = 0; q < T->ncls; ++q)
    if (__builtin_popcount(T->canon[q]) >= min_edges && __builtin_add_overflow(sum, c[q], &sum))
      return fail(DM_E_OVERFLOW, "quasi-clique sum wrapped");
  *out_count = sum;
  return DM_OK;
}

// ====================================================================== batching

namespace {

// A batch is the disjoint union of its graphs: vertex ids of graph i are
// shifted by the vertex count of graphs 0..i-1, so no traversal crosses
// graphs and per-graph counters can be kept by mapping each root to its graph.
// A captured launch: the clears, the persistent kernel and the copy-back of
// one prepared batch, replayed with hipGraphLaunch.  It is keyed by the exact
// bytes of the prepared launch, so it is only replayed while every buffer it
// names is the one currently allocated.
struct CapturedLaunch {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t* host_out = nullptr;  // pinned
  int* host_flags = nullptr;     // pinned
  size_t out_count = 0;
  ~CapturedLaunch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (host_out) (void)hipHostFree(host_out);
    if (host_flags) (void)hipHostFree(host_flags);
  }
};

struct BatchCache {
  dm_graph* uni = nullptr;
  Buf gov;  // graph index of every union vertex
  Buf gor;  // graph index of every union vertex in rank order
  bool gor_ready = false;
  hipStream_t stream = nullptr;  // capture stream (never the legacy default stream)
  std::map<std::string, CapturedLaunch*> graphs;
  ~BatchCache() {
    for (auto& kv : graphs) delete kv.second;
    if (stream) (void)hipStreamDestroy(stream);
    dm_free(uni);
  }
};

std::string launch_key(const Prepared& P) {
  std::string key(reinterpret_cast<const char*>(&P.clique), sizeof(P.clique));
  if (P.clique) key.append(reinterpret_cast<const char*>(&P.ca), sizeof(P.ca));
  else key.append(reinterpret_cast<const char*>(&P.ma), sizeof(P.ma));
  const int64_t tail[] = {P.grid, static_cast<int64_t>(P.lds), P.nq, static_cast<int64_t>(P.out_count),
                          static_cast<int64_t>(P.bias), reinterpret_cast<int64_t>(P.stats), P.stats_words};
  key.append(reinterpret_cast<const char*>(tail), sizeof(tail));
  return key;
}

dm_status run_captured(BatchCache* B, const Prepared& P, uint64_t* out) {
  const std::string key = launch_key(P);
  CapturedLaunch*& C = B->graphs[key];
  if (!C) {
    C = new CapturedLaunch();
    C->out_count = P.out_count;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&C->host_out), sizeof(uint64_t) * (P.out_count ? P.out_count : 1));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&C->host_flags), 2 * sizeof(int));
    if (e == hipSuccess) e = hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = enqueue(P, B->stream, C->host_out, C->host_flags);
      e = hipStreamEndCapture(B->stream, &C->graph);
      if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&C->exec, C->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      delete C;
      B->graphs.erase(key);
      return hip_fail(e, "batch: graph capture");
    }
  }
  hipError_t e = hipGraphLaunch(C->exec, B->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
  if (e != hipSuccess) return hip_fail(e, "batch: graph launch");
  dm_status st = check_flags(C->host_flags);
  if (st == DM_OK) std::memcpy(out, C->host_out, sizeof(uint64_t) * C->out_count);
  if (st == DM_OK && P.rc_done) *P.rc_done = true;
  return st;
}

std::mutex g_batch_lock;
std::map<std::vector<uint64_t>, BatchCache*> g_batches;

dm_status build_union(dm_graph* const* gs, int32_t num, hipStream_t s, BatchCache* B) {
  int64_t ntot = 0, etot = 0;
  int dmax = 0;
  for (int32_t i = 0; i < num; ++i) {
    ntot += gs[i]->n;
    etot += gs[i]->nnz;
    dmax = std::max(dmax, gs[i]->dmax);
  }
  if (ntot > 2000000000LL) return fail(DM_E_ARG, "batch has more than 2e9 vertices");
  dm_graph* u = new dm_graph();
  u->device = gs[0]->device;
  u->n = static_cast<int32_t>(ntot);
  u->nnz = etot;
  u->dmax = dmax;
  B->uni = u;
  HIP_OR_RETURN(u->rp.ensure(sizeof(int64_t) * (ntot + 1)), "batch: allocate");
  HIP_OR_RETURN(u->col.ensure(sizeof(int32_t) * (etot > 0 ? etot : 1)), "batch: allocate");
  HIP_OR_RETURN(B->gov.ensure(sizeof(int32_t) * (ntot > 0 ? ntot : 1)), "batch: allocate");
  int64_t voff = 0, eoff = 0;
  for (int32_t i = 0; i < num; ++i) {
    const dm_graph* g = gs[i];
    HIP_OR_RETURN(launch_offset_i64(g->rp.as<int64_t>(), u->rp.as<int64_t>() + voff, g->n, eoff, s), "batch: rows");
    HIP_OR_RETURN(launch_offset_i32(g->col.as<int32_t>(), u->col.as<int32_t>() + eoff, g->nnz, static_cast<int32_t>(voff), s),
                  "batch: cols");
    HIP_OR_RETURN(launch_fill_i32(B->gov.as<int32_t>() + voff, g->n, i, s), "batch: graph map");
    voff += g->n;
    eoff += g->nnz;
  }
  HIP_OR_RETURN(launch_fill_u64(reinterpret_cast<unsigned long long*>(u->rp.as<int64_t>() + ntot), 1,
                                static_cast<unsigned long long>(etot), s),
                "batch: rows");
  HIP_OR_RETURN(hipStreamSynchronize(s), "batch: build");
  return DM_OK;
}

BatchCache* batch_cache(dm_graph* const* gs, int32_t num, hipStream_t caller, dm_status* st) {
  std::vector<uint64_t> key(static_cast<size_t>(num));
  for (int32_t i = 0; i < num; ++i) key[i] = gs[i]->uid;
  BatchCache*& B = g_batches[key];
  *st = DM_OK;
  if (!B) {
    B = new BatchCache();
    hipError_t e = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking);
    if (e == hipSuccess && caller) e = hipStreamSynchronize(caller);
    *st = e == hipSuccess ? build_union(gs, num, B->stream, B) : hip_fail(e, "batch: stream");
    if (*st != DM_OK) {
      delete B;
      B = nullptr;
      g_batches.erase(key);
      return nullptr;
    }
  }
  return B;
}

dm_status batch_run(dm_graph* const* gs, int32_t num, int op, int k, int width, const Opt& o_in, uint64_t* out) {
  std::lock_guard<std::mutex> lk(g_batch_lock);
  dm_status st0;
  // work on the batch's own stream (captures cannot use the legacy default
  // stream); the caller's stream is drained first
  if (o_in.stream) HIP_OR_RETURN(hipStreamSynchronize(o_in.stream), "batch: caller stream");
  BatchCache* B = batch_cache(gs, num, o_in.stream, &st0);
  if (!B) return st0;
  Opt o = o_in;
  apply_tuning(op, k, &o);
  hipStream_t s = B->stream;
  std::vector<uint64_t> tmp(static_cast<size_t>(num) * width);
  // both kernels take roots in rank space: graph index of every rank
  dm_status st = ensure_dag(B->uni, s);
  if (st != DM_OK) return st;
  if (!B->gor_ready) {
    HIP_OR_RETURN(B->gor.ensure(sizeof(int32_t) * (B->uni->n > 0 ? B->uni->n : 1)), "batch: allocate");
    HIP_OR_RETURN(launch_gather_i32(B->gov.as<int32_t>(), B->uni->order.as<int32_t>(), B->gor.as<int32_t>(),
                                    B->uni->n, s),
                  "batch: rank map");
    B->gor_ready = true;
  }
  Prepared P;
  st = prepare(B->uni, op, k, o, s, B->gor.as<int32_t>(), num, &P);
  if (st != DM_OK) return st;
  // one persistent launch per batch, captured once and replayed; per-root
  // records and wave statistics take the direct path
  if (!o.root_stats && !o.wave_stats) return run_captured(B, P, out);
  st = run_prepared(P, s, tmp.data());
  if (st == DM_OK) std::memcpy(out, tmp.data(), sizeof(uint64_t) * tmp.size());
  return st;
}

dm_status batch_tune(dm_graph* const* gs, int32_t num, int op, int k, const Opt& o, Tuning* best) {
  std::lock_guard<std::mutex> lk(g_batch_lock);
  dm_status st0;
  if (o.stream) HIP_OR_RETURN(hipStreamSynchronize(o.stream), "tune: caller stream");
  BatchCache* B = batch_cache(gs, num, o.stream, &st0);
  if (!B) return st0;
  dm_status st = ensure_dag(B->uni, B->stream);
  if (st != DM_OK) return st;
  if (!B->gor_ready) {
    HIP_OR_RETURN(B->gor.ensure(sizeof(int32_t) * (B->uni->n > 0 ? B->uni->n : 1)), "batch: allocate");
    HIP_OR_RETURN(launch_gather_i32(B->gov.as<int32_t>(), B->uni->order.as<int32_t>(), B->gor.as<int32_t>(),
                                    B->uni->n, B->stream),
                  "batch: rank map");
    B->gor_ready = true;
  }
  return autotune(B->uni, op, k, o, B->stream, B->gor.as<int32_t>(), num, best);
}

}  // namespace

extern "C" dm_status dm_batch(dm_graph* const* gs, int32_t num_graphs, int op, int k, uint64_t* out_counts,
                              size_t out_len, const dm_options* opt) {
  if (!gs || num_graphs <= 0 || !out_counts) return fail(DM_E_ARG, "null graphs / output or num_graphs <= 0");
  if (op != DM_OP_CLIQUE && op != DM_OP_MOTIF) return fail(DM_E_ARG, "unknown op");
  int width = 1;
  if (op == DM_OP_CLIQUE) {
    if (k < 1 || k > kMaxK) return fail(DM_E_K, "clique k must be in 1..32");
  } else {
    const ClassTables* T = tables(k);
    if (!T) return fail(DM_E_K, "motif k must be in 3..8");
    width = T->ncls;
  }
  if (out_len < static_cast<size_t>(num_graphs) * width) return fail(DM_E_BUFSZ, "out_len < num_graphs * width");
  for (int32_t i = 0; i < num_graphs; ++i)
    if (!gs[i]) return fail(DM_E_ARG, "null graph in batch");
  Opt o;
  dm_status st = read_opt(opt, &o);
  if (st != DM_OK) return st;
  if (o.roots) return fail(DM_E_ARG, "root lists are not supported in batches");
  if (o.sched & DM_SCHED_COST) return fail(DM_E_ARG, "cost ordering takes one graph's costs; not for batches");
  if (o.sched & DM_IMPL_DFS) return fail(DM_E_ARG, "DM_IMPL_DFS runs single graphs");
  if (o.sched & DM_SCHED_HOST_BALANCE) return fail(DM_E_ARG, "DM_SCHED_HOST_BALANCE runs single graphs");
  if ((o.sched & DM_SCHED_LEARNED) && !o.mlp) return fail(DM_E_MODEL, "DM_SCHED_LEARNED needs mlp parameters");
  return batch_run(gs, num_graphs, op, k, width, o, out_counts);
}

// ====================================================================== learned ordering ABI

extern "C" dm_status dm_features(dm_graph* g, int64_t* out, void* stream) {
  if (!g || !out) return fail(DM_E_ARG, "null graph or output");
  hipStream_t s = pick_stream(g, stream);
  dm_status st = ensure_features(g, s);
  if (st != DM_OK) return st;
  HIP_OR_RETURN(hipMemcpyAsync(out, g->feat.p, sizeof(int64_t) * 4 * static_cast<size_t>(g->n), hipMemcpyDeviceToDevice, s),
                "features: copy");
  HIP_OR_RETURN(hipStreamSynchronize(s), "features: sync");
  return DM_OK;
}

static hipStream_t plain_stream(void* s) { return static_cast<hipStream_t>(s); }

extern "C" dm_status dm_mlp_init(float* params, uint64_t seed, void* stream) {
  if (!params) return fail(DM_E_ARG, "null params");
  hipStream_t s = plain_stream(stream);
  HIP_OR_RETURN(mlp_init(params, seed, s), "mlp init");
  HIP_OR_RETURN(hipStreamSynchronize(s), "mlp init");
  return DM_OK;
}

extern "C" dm_status dm_mlp_fit_normalizer(float* params, const int64_t* feats, int64_t n, void* stream) {
  if (!params || !feats || n <= 0) return fail(DM_E_ARG, "null pointer or n <= 0");
  hipStream_t s = plain_stream(stream);
  HIP_OR_RETURN(mlp_fit_normaliser(params, feats, n, s), "mlp normaliser");
  HIP_OR_RETURN(hipStreamSynchronize(s), "mlp normaliser");
  return DM_OK;
}

extern "C" dm_status dm_mlp_forward(const float* params, const int64_t* feats, int64_t n, float* out, void* stream) {
  if (!params || !feats || !out || n < 0) return fail(DM_E_ARG, "null pointer or n < 0");
  hipStream_t s = plain_stream(stream);
  HIP_OR_RETURN(mlp_forward(params, feats, n, out, s), "mlp forward");
  HIP_OR_RETURN(hipStreamSynchronize(s), "mlp forward");
  return DM_OK;
}

extern "C" dm_status dm_mlp_targets(const uint64_t* root_stats, int64_t n, float* out, void* stream) {
  if (!root_stats || !out || n < 0) return fail(DM_E_ARG, "null pointer or n < 0");
  hipStream_t s = plain_stream(stream);
  HIP_OR_RETURN(mlp_targets(reinterpret_cast<const unsigned long long*>(root_stats), n, out, s), "mlp targets");
  HIP_OR_RETURN(hipStreamSynchronize(s), "mlp targets");
  return DM_OK;
}

extern "C" dm_status dm_mlp_loss_grad(const float* params, const int64_t* feats, const float* targets, int64_t n,
                                      float* grad, float* loss, void* stream) {
  if (!params || !feats || !targets || !grad || !loss || n <= 0) return fail(DM_E_ARG, "null pointer or n <= 0");
  hipStream_t s = plain_stream(stream);
  Buf partial, dloss;
  HIP_OR_RETURN(partial.ensure(sizeof(float) * (kMlpNet + 1) * static_cast<size_t>((n + 63) / 64)), "mlp grad: allocate");
  HIP_OR_RETURN(dloss.ensure(sizeof(float)), "mlp grad: allocate");
  HIP_OR_RETURN(mlp_loss_grad(params, feats, targets, nullptr, n, partial.as<float>(), grad, dloss.as<float>(), s),
                "mlp grad");
  HIP_OR_RETURN(hipMemcpyAsync(loss, dloss.p, sizeof(float), hipMemcpyDeviceToHost, s), "mlp grad: copy");
  HIP_OR_RETURN(hipStreamSynchronize(s), "mlp grad");
  return DM_OK;
}

extern "C" dm_status dm_mlp_adam_step(float* params, const float* grad, float* m, float* v, int64_t t, float lr,
                                      void* stream) {
  if (!params || !grad || !m || !v || t < 1) return fail(DM_E_ARG, "null pointer or step < 1");
  hipStream_t s = plain_stream(stream);
  HIP_OR_RETURN(mlp_adam(params, grad, m, v, t, lr, s), "adam");
  HIP_OR_RETURN(hipStreamSynchronize(s), "adam");
  return DM_OK;
}

extern "C" dm_status dm_mlp_train(float* params, const int64_t* feats, const float* targets, int64_t n, int epochs,
                                  int batch, float lr, uint64_t seed, float* loss_history, void* stream) {
  if (!params || !feats || !targets || n <= 0 || epochs < 0 || batch <= 0) return fail(DM_E_ARG, "bad arguments");
  if (n > 2000000000LL) return fail(DM_E_ARG, "n too large");
  hipStream_t s = plain_stream(stream);
  const int64_t nb = (n + batch - 1) / batch;
  Buf partial, grad, m, v, keys, keys2, perm_in, perm, temp, losses;
  const size_t tb = mlp_shuffle_temp_bytes(n);
  HIP_OR_RETURN(partial.ensure(sizeof(float) * (kMlpNet + 1) * static_cast<size_t>((batch + 63) / 64)), "train: allocate");
  HIP_OR_RETURN(grad.ensure(sizeof(float) * kMlpNet), "train: allocate");
  HIP_OR_RETURN(m.ensure(sizeof(float) * kMlpNet), "train: allocate");
  HIP_OR_RETURN(v.ensure(sizeof(float) * kMlpNet), "train: allocate");
  HIP_OR_RETURN(keys.ensure(sizeof(unsigned long long) * n), "train: allocate");
  HIP_OR_RETURN(keys2.ensure(sizeof(unsigned long long) * n), "train: allocate");
  HIP_OR_RETURN(perm_in.ensure(sizeof(int32_t) * n), "train: allocate");
  HIP_OR_RETURN(perm.ensure(sizeof(int32_t) * n), "train: allocate");
  HIP_OR_RETURN(temp.ensure(tb), "train: allocate");
  HIP_OR_RETURN(losses.ensure(sizeof(float) * nb), "train: allocate");
  HIP_OR_RETURN(launch_fill_i32(m.as<int32_t>(), kMlpNet, 0, s), "train: clear");
  HIP_OR_RETURN(launch_fill_i32(v.as<int32_t>(), kMlpNet, 0, s), "train: clear");
  std::vector<float> host_losses(static_cast<size_t>(nb));
  int64_t step = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    HIP_OR_RETURN(mlp_shuffle(seed * 1000003ull + static_cast<uint64_t>(ep), n, keys.as<unsigned long long>(),
                              keys2.as<unsigned long long>(), perm_in.as<int32_t>(), perm.as<int32_t>(), temp.p, tb, s),
                  "train: shuffle");
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t rows = std::min<int64_t>(batch, n - b * batch);
      HIP_OR_RETURN(mlp_loss_grad(params, feats, targets, perm.as<int32_t>() + b * batch, rows, partial.as<float>(),
                                  grad.as<float>(), losses.as<float>() + b, s),
                    "train: grad");
      HIP_OR_RETURN(mlp_adam(params, grad.as<float>(), m.as<float>(), v.as<float>(), ++step, lr, s), "train: adam");
    }
    if (loss_history) {
      HIP_OR_RETURN(hipMemcpyAsync(host_losses.data(), losses.p, sizeof(float) * nb, hipMemcpyDeviceToHost, s),
                    "train: loss");
      HIP_OR_RETURN(hipStreamSynchronize(s), "train: loss");
      double acc = 0.0;
      for (int64_t b = 0; b < nb; ++b) acc += host_losses[b];
      loss_history[ep] = static_cast<float>(acc / static_cast<double>(nb));
    }
  }
  HIP_OR_RETURN(hipStreamSynchronize(s), "train");
  return DM_OK;
}

// ====================================================================== autotuning ABI

extern "C" dm_status dm_autotune(dm_graph* const* gs, int32_t num_graphs, int op, int k, const dm_options* opt,
                                 dm_tuning* out) {
  if (!gs || num_graphs <= 0 || !out) return fail(DM_E_ARG, "null graphs / output or num_graphs <= 0");
  if (op != DM_OP_CLIQUE && op != DM_OP_MOTIF) return fail(DM_E_ARG, "unknown op");
  if (op == DM_OP_CLIQUE ? (k < 1 || k > kMaxK) : !tables(k)) return fail(DM_E_K, "k out of range");
  for (int32_t i = 0; i < num_graphs; ++i)
    if (!gs[i]) return fail(DM_E_ARG, "null graph");
  Opt o;
  dm_status st = read_opt(opt, &o);
  if (st != DM_OK) return st;
  if (o.roots) return fail(DM_E_ARG, "tuning runs over every root");
  if ((o.sched & DM_SCHED_COST) && num_graphs > 1) return fail(DM_E_ARG, "cost ordering takes one graph's costs");
  if (o.sched & (DM_IMPL_DFS | DM_SCHED_HOST_BALANCE))
    return fail(DM_E_ARG, "the tuner times single in-kernel-balanced launches");
  if ((o.sched & DM_SCHED_LEARNED) && !o.mlp) return fail(DM_E_MODEL, "DM_SCHED_LEARNED needs mlp parameters");
  Tuning t;
  if (num_graphs == 1) {
    hipStream_t s = pick_stream(gs[0], o.stream);
    st = autotune(gs[0], op, k, o, s, nullptr, 1, &t);
  } else {
    st = batch_tune(gs, num_graphs, op, k, o, &t);
  }
  if (st != DM_OK) return st;
  out->chunk = t.chunk;
  out->rebalance = t.rebalance;
  out->waves_per_cu = t.waves_per_cu;
  out->ms = t.ms;
  return DM_OK;
}

// ====================================================================== directed graphs

namespace {

// Host check of the arc conventions: sorted out-lists, no self-arc, no repeated arc.
bool host_validate_arcs(int32_t n, const int64_t* rp, const int32_t* col, std::string* why) {
  if (rp[0] != 0) { *why = "row_ptr[0] != 0"; return false; }
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) { *why = "row_ptr decreases"; return false; }
  for (int32_t v = 0; v < n; ++v)
    for (int64_t i = rp[v]; i < rp[v + 1]; ++i) {
      const int32_t u = col[i];
      if (u < 0 || u >= n) { *why = "column id out of range"; return false; }
      if (u == v) { *why = "self-arc"; return false; }
      if (i > rp[v] && col[i - 1] >= u) { *why = "out-list not strictly ascending (or repeated arc)"; return false; }
    }
  return true;
}

}  // namespace

extern "C" dm_status dm_load_digraph(int32_t n, const int64_t* row_ptr, const int32_t* col, uint32_t flags,
                                     void* stream, dm_graph** out) {
  if (!out) return fail(DM_E_ARG, "null output handle");
  *out = nullptr;
  if (n < 0 || !row_ptr || (!col && n > 0)) return fail(DM_E_ARG, "n < 0 or null CSR array");
  if (flags & ~15u) return fail(DM_E_ARG, "unknown flag");
  const bool on_device = flags & DM_CSR_DEVICE;
  const bool trusted = flags & DM_CSR_TRUSTED;
  int64_t arcs = 0;
  if (!on_device) {
    arcs = row_ptr[n];
    if (arcs < 0) return fail(DM_E_CSR, "negative arc count");
    std::string why;
    if (!trusted && !host_validate_arcs(n, row_ptr, col, &why)) return fail(DM_E_CSR, why);
  }
  hipStream_t own = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!s) HIP_OR_RETURN(hipStreamCreateWithFlags(&own, hipStreamNonBlocking), "dm_load_digraph: stream");
  if (!s) s = own;
  struct StreamGuard {
    hipStream_t st;
    ~StreamGuard() {
      if (st) (void)hipStreamDestroy(st);
    }
  } guard{own};
  if (on_device) {
    HIP_OR_RETURN(hipMemcpyAsync(&arcs, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s), "dm_load_digraph: read arcs");
    HIP_OR_RETURN(hipStreamSynchronize(s), "dm_load_digraph: read arcs");
    if (arcs < 0) return fail(DM_E_CSR, "negative arc count");
  }
  Buf arp, acol, flag;
  const int64_t* drp = row_ptr;
  const int32_t* dcol = col;
  if (!on_device) {
    HIP_OR_RETURN(arp.ensure(sizeof(int64_t) * (static_cast<size_t>(n) + 1)), "dm_load_digraph: allocate");
    HIP_OR_RETURN(acol.ensure(sizeof(int32_t) * static_cast<size_t>(arcs > 0 ? arcs : 1)), "dm_load_digraph: allocate");
    HIP_OR_RETURN(hipMemcpyAsync(arp.p, row_ptr, sizeof(int64_t) * (static_cast<size_t>(n) + 1), hipMemcpyHostToDevice, s),
                  "dm_load_digraph: copy");
    if (arcs > 0)
      HIP_OR_RETURN(hipMemcpyAsync(acol.p, col, sizeof(int32_t) * arcs, hipMemcpyHostToDevice, s), "dm_load_digraph: copy");
    drp = arp.as<int64_t>();
    dcol = acol.as<int32_t>();
  } else if (!trusted && n > 0) {
    int bad = 0;
    HIP_OR_RETURN(flag.ensure(sizeof(int)), "dm_load_digraph: allocate");
    HIP_OR_RETURN(launch_fill_i32(flag.as<int>(), 1, 0, s), "dm_load_digraph: validate");
    HIP_OR_RETURN(launch_arc_validate(drp, dcol, n, arcs, flag.as<int>(), s), "dm_load_digraph: validate");
    HIP_OR_RETURN(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, s), "dm_load_digraph: validate");
    HIP_OR_RETURN(hipStreamSynchronize(s), "dm_load_digraph: validate");
    if (bad) {
      char buf[96];
      std::snprintf(buf, sizeof buf, "device arc validation failed (flags 0x%x)", bad);
      return fail(DM_E_CSR, buf);
    }
  }
  int64_t* urp = nullptr;
  int32_t* ucol = nullptr;
  uint8_t* udir = nullptr;
  int64_t unnz = 0;
  hipError_t e = hipSuccess;
  if (n > 0) {
    e = digraph_underlying(drp, dcol, n, arcs, &urp, &ucol, &udir, &unnz, s);
  } else {
    e = hipMalloc(&urp, sizeof(int64_t));
    if (e == hipSuccess) e = hipMemsetAsync(urp, 0, sizeof(int64_t), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) {
    (void)hipFree(urp);
    (void)hipFree(ucol);
    (void)hipFree(udir);
    return hip_fail(e, "dm_load_digraph: underlying graph");
  }
  int32_t none = 0;
  const dm_status st = dm_load_csr(n, urp, ucol ? ucol : &none, DM_CSR_DEVICE | DM_CSR_TRUSTED |
                                   (flags & (DM_CSR_ORIENT | DM_CSR_RANK)), stream, out);
  (void)hipFree(urp);
  (void)hipFree(ucol);
  if (st != DM_OK) {
    (void)hipFree(udir);
    return st;
  }
  dm_graph* g = *out;
  g->directed = true;
  g->arcs = arcs;
  g->dir.p = udir;  // adopted: freed with the handle
  g->dir.bytes = udir ? static_cast<size_t>(unnz > 0 ? unnz : 1) : 0;
  return DM_OK;
}

extern "C" dm_status dm_digraph_info(const dm_graph* g, int32_t* is_directed, int64_t* arcs) {
  if (!g) return fail(DM_E_ARG, "null graph");
  if (is_directed) *is_directed = g->directed ? 1 : 0;
  if (arcs) *arcs = g->directed ? g->arcs : 0;
  return DM_OK;
}

extern "C" int32_t dm_motif_directed_num_classes(int k) {
  const DClassTables* T = dtables(k);
  return T ? T->ncls : -1;
}

extern "C" dm_status dm_motif_directed_class_code(int k, int32_t cls, uint32_t* code) {
  const DClassTables* T = dtables(k);
  if (!T) return fail(DM_E_K, "directed motif k must be in 1..5");
  if (!code || cls < 0 || cls >= T->ncls) return fail(DM_E_ARG, "class id out of range or null output");
  *code = T->canon[cls];
  return DM_OK;
}

extern "C" dm_status dm_motif_directed_class_table(int k, uint16_t* out, size_t len) {
  const DClassTables* T = dtables(k);
  if (!T) return fail(DM_E_K, "directed motif k must be in 1..5");
  if (!out) return fail(DM_E_ARG, "null output");
  if (len < T->table.size()) return fail(DM_E_BUFSZ, "len < 2^(k(k-1))");
  std::memcpy(out, T->table.data(), sizeof(uint16_t) * T->table.size());
  return DM_OK;
}

namespace {

// launch shapes by (classes, waves-per-CU cap): the search asks the runtime
// for the residency of ~100 shapes
std::mutex g_dplan_lock;
std::vector<std::pair<std::pair<int, int>, DMotifPlan>> g_dplans;

hipError_t dmotif_plan_cached(int ncls, int max_waves, DMotifPlan* plan) {
  std::lock_guard<std::mutex> lk(g_dplan_lock);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const std::pair<int, int> key(ncls + (dev << 20), max_waves);
  for (const auto& p : g_dplans)
    if (p.first == key) {
      *plan = p.second;
      return hipSuccess;
    }
  e = dmotif_plan(ncls, max_waves, plan);
  if (e == hipSuccess) g_dplans.emplace_back(key, *plan);
  return e;
}

}  // namespace

extern "C" dm_status dm_count_motifs_directed(dm_graph* g, int k, uint64_t* out_counts, size_t out_len,
                                              const dm_options* opt) {
  if (!g || !out_counts) return fail(DM_E_ARG, "null graph or output");
  if (!g->directed) return fail(DM_E_ARG, "not a directed graph (load it with dm_load_digraph)");
  if (k < 3 || k > kDMotifMaxK) return fail(DM_E_K, "directed motif k must be in 3..5");
  const DClassTables* T = dtables(k);
  if (out_len < static_cast<size_t>(T->ncls)) return fail(DM_E_BUFSZ, "out_len < number of directed classes");
  Opt o;
  dm_status st = read_opt(opt, &o);
  if (st != DM_OK) return st;
  if ((o.sched & ~static_cast<uint32_t>(DM_NO_DONATION)) || o.roots || o.root_stats)
    return fail(DM_E_ARG, "directed motifs take only stream, chunk, waves_per_cu and wait_limit_us");
  hipStream_t s = pick_stream(g, o.stream);
  uint16_t* dtab = nullptr;
  HIP_OR_RETURN(device_table(k + 100, &dtab), "directed class table upload");
  const int dmax = g->dmax > 0 ? g->dmax : 1;
  if (dmax >= (1 << 26)) return fail(DM_E_ARG, "directed motifs need every degree below 2^26");
  // the traversal runs on the graph renamed by (degree, id) rank, like the
  // undirected motifs: a subgraph's root is its lowest-rank vertex, so hubs
  // root few subgraphs and no single root's tree dominates the launch
  st = ensure_ranked(g, s);
  if (st != DM_OK) return st;
  if (!g->dranked) {
    HIP_OR_RETURN(g->rdir.ensure(static_cast<size_t>(g->nnz > 0 ? g->nnz : 1)), "rank arc bits: allocate");
    HIP_OR_RETURN(g->ctrl.ensure(ctrl_bytes()), "workspace");
    int bad = 0;
    hipError_t e = launch_fill_u64(g->ctrl.as<unsigned long long>(), static_cast<int64_t>(ctrl_bytes() / 8), 0ull, s);
    if (e == hipSuccess)
      e = digraph_rank_dir(g->rp.as<int64_t>(), g->col.as<int32_t>(), g->dir.as<uint8_t>(), g->n, g->rank.as<int32_t>(),
                           g->urp.as<int64_t>(), g->ucol.as<int32_t>(), g->rdir.as<uint8_t>(), ctrl_flags(g), s);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, ctrl_flags(g), sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rank arc bits");
    if (bad) return fail(DM_E_CSR, "rank arc bits: the renamed graph is missing an entry");
    g->dranked = true;
  }
  DMotifPlan plan;
  HIP_OR_RETURN(dmotif_plan_cached(T->ncls, static_cast<int>(o.waves_per_cu), &plan), "directed motif launch shape");
  const int nw = plan.waves_per_group;
  // workgroups: the shape's residency over the CUs, fewer on a small graph
  const int grid = std::max(1, size_grid(plan.groups_per_cu * nw, g->nnz) / nw);
  DMotifArgs A;
  std::memset(&A, 0, sizeof(A));
  int64_t cap_total = 0;
  for (int lv = 1; lv <= k - 1; ++lv) {
    A.level_off[lv] = cap_total;
    A.level_cap[lv] = static_cast<int64_t>(lv) * dmax;
    cap_total += A.level_cap[lv];
  }
  A.hit_cap = static_cast<int64_t>(k - 1) * dmax;
  A.wave_cap = cap_total;
  A.leaf_cap = plan.leaf_cap;
  const size_t gw = static_cast<size_t>(grid) * nw;
  HIP_OR_RETURN(g->ctrl.ensure(ctrl_bytes()), "workspace");
  HIP_OR_RETURN(g->out.ensure(sizeof(uint64_t) * T->ncls), "workspace");
  HIP_OR_RETURN(g->ext_vert.ensure(sizeof(int32_t) * gw * cap_total), "workspace");
  HIP_OR_RETURN(g->ext_mask.ensure(gw * cap_total), "workspace");
  HIP_OR_RETURN(g->ext_arcs.ensure(sizeof(uint16_t) * gw * cap_total), "workspace");
  HIP_OR_RETURN(g->dhit.ensure(gw * A.hit_cap), "workspace");
  HIP_OR_RETURN(g->newbuf.ensure(sizeof(int32_t) * gw * dmax), "workspace");
  HIP_OR_RETURN(g->dndir.ensure(gw * dmax), "workspace");
  Sched S = make_sched(g, o, static_cast<int>(gw), g->n, nullptr, nullptr);
  S.donate = 0;  // roots only: no donated task states for this kernel
  A.rp = g->urp.as<int64_t>();
  A.col = g->ucol.as<int32_t>();
  A.dir = g->rdir.as<uint8_t>();
  A.n = g->n;
  A.k = k;
  A.dmax = dmax;
  A.ncls = T->ncls;
  A.table = dtab;
  A.out = g->out.as<unsigned long long>();
  A.flags = ctrl_flags(g);
  A.vert = g->ext_vert.as<int32_t>();
  A.mask = g->ext_mask.as<uint8_t>();
  A.arcs = g->ext_arcs.as<uint16_t>();
  A.hit = g->dhit.as<uint8_t>();
  A.nbuf = g->newbuf.as<int32_t>();
  A.ndir = g->dndir.as<uint8_t>();
  A.S = S;
  g_last_launches = 1;
  int flags[2] = {0, 0};
  hipError_t e = launch_fill_u64(g->ctrl.as<unsigned long long>(), static_cast<int64_t>(ctrl_bytes() / 8), 0ull, s);
  if (e == hipSuccess) e = launch_fill_u64(A.out, T->ncls, 0ull, s);
  if (e == hipSuccess && g->n > 0) e = launch_dmotif(A, grid, nw, plan.lds, s);
  std::vector<uint64_t> tmp(T->ncls);
  if (e == hipSuccess) e = hipMemcpyAsync(tmp.data(), A.out, sizeof(uint64_t) * T->ncls, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(flags, A.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "directed motif kernel / copy-back");
  st = check_flags(flags);
  if (st == DM_OK) std::memcpy(out_counts, tmp.data(), sizeof(uint64_t) * T->ncls);
  return st;
}

// ====================================================================== pattern matching

namespace {

// Images of a pattern code under vertex orders.  Copies of a connected
// pattern P spanning a k-vertex graph H = the distinct images of P that are
// subgraphs of H (= |{orders s : s(P) in H}| / |Aut(P)|).  Undirected codes
// have one bit per pair, directed codes two (the layouts of the two
// dictionaries).
struct PatternCopies {
  std::vector<std::vector<int>> perms;
  int k = 0;
  bool directed = false;
  uint32_t image(uint32_t code, const std::vector<int>& p) const {
    uint32_t img = 0;
    for (int i = 1; i < k; ++i)
      for (int t = 0; t < i; ++t) {
        const int a = p[t], b = p[i];
        if (!directed) {
          if ((code >> pair_index(t, i)) & 1u) img |= 1u << (a < b ? pair_index(a, b) : pair_index(b, a));
        } else {
          const int bit = 2 * pair_index(t, i);
          // arc t -> i becomes a -> b, arc i -> t becomes b -> a
          if ((code >> bit) & 1u) img |= a < b ? 1u << (2 * pair_index(a, b)) : 1u << (2 * pair_index(b, a) + 1);
          if ((code >> (bit + 1)) & 1u) img |= a < b ? 1u << (2 * pair_index(a, b) + 1) : 1u << (2 * pair_index(b, a));
        }
      }
    return img;
  }
};

}  // namespace

extern "C" dm_status dm_count_pattern(dm_graph* g, int k, uint32_t pattern, uint32_t flags, uint64_t* out_count,
                                      const dm_options* opt) {
  if (!g || !out_count) return fail(DM_E_ARG, "null graph or output");
  if (flags & ~3u) return fail(DM_E_ARG, "unknown pattern flag");
  const bool directed = flags & DM_PATTERN_DIRECTED;
  const bool induced = flags & DM_PATTERN_INDUCED;
  if (directed ? (k < 3 || k > kDMotifMaxK) : (k < 3 || k > kMotifMaxK))
    return fail(DM_E_K, directed ? "directed pattern k must be in 3..5" : "pattern k must be in 3..8");
  const int bits = directed ? k * (k - 1) : k * (k - 1) / 2;
  if (bits < 32 && (pattern >> bits)) return fail(DM_E_ARG, "pattern code has bits beyond its k vertices");
  // the pattern's class: its smallest code over all vertex orders
  PatternCopies pc;
  pc.k = k;
  pc.directed = directed;
  std::vector<int> p(k);
  for (int i = 0; i < k; ++i) p[i] = i;
  do pc.perms.push_back(p);
  while (std::next_permutation(p.begin(), p.end()));
  // the distinct images of P under all vertex orders: its copies on k labelled
  // vertices (k! / |Aut(P)| of them); the smallest is P's class
  std::vector<uint32_t> imgs;
  imgs.reserve(pc.perms.size());
  for (const auto& q : pc.perms) imgs.push_back(pc.image(pattern, q));
  std::sort(imgs.begin(), imgs.end());
  imgs.erase(std::unique(imgs.begin(), imgs.end()), imgs.end());
  const uint32_t canon = imgs.front();
  uint32_t und = pattern;
  if (directed) {
    und = 0;
    for (int pi = 0; pi < k * (k - 1) / 2; ++pi)
      if ((pattern >> (2 * pi)) & 3u) und |= 1u << pi;
  }
  if (!bitmap_connected(k, und)) return fail(DM_E_ARG, "the pattern must be (weakly) connected");
  const int ncls = directed ? dtables(k)->ncls : tables(k)->ncls;
  const std::vector<uint32_t>& reps = directed ? dtables(k)->canon : tables(k)->canon;
  std::vector<uint64_t> c(ncls);
  dm_status st = directed ? dm_count_motifs_directed(g, k, c.data(), c.size(), opt)
                          : dm_count_motifs(g, k, c.data(), c.size(), opt);
  if (st != DM_OK) return st;
  uint64_t sum = 0;
  for (int q = 0; q < ncls; ++q) {
    if (c[q] == 0) continue;
    uint64_t copies = 0;
    if (induced) {
      copies = reps[q] == canon ? 1 : 0;
    } else {
      for (const uint32_t u : imgs) copies += (u & ~reps[q]) == 0;  // copies of P spanning the class's graph
    }
    uint64_t add = 0;
    if (__builtin_mul_overflow(c[q], copies, &add) || __builtin_add_overflow(sum, add, &sum))
      return fail(DM_E_OVERFLOW, "pattern count wrapped");
  }
  *out_count = sum;
  return DM_OK;
}

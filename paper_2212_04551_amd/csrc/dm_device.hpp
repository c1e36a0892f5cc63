// Device-side building blocks shared by the enumeration kernels: wave64
// primitives and the persistent-wave work scheduler (root queue + donation
// pool + termination detection).
//
// Every enumeration kernel runs one 64-lane wavefront per workgroup; a wave
// owns one traversal stack (the TE structure of DuMato, Section IV-B) and all
// its lanes work on that stack together (Section IV-A, warp-centric task
// allocation), so LDS written by one lane and read by another only needs a
// workgroup barrier, which for a one-wave workgroup is cheap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dm {

constexpr int kWave = 64;
constexpr int kMaxK = 32;          // largest clique size
constexpr int kTaskInts = 40;      // payload of a donated task
constexpr int kMaxTaskPrefix = kTaskInts - 5;

// ------------------------------------------------------------------ wave64 primitives

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of m strictly below the calling lane
__device__ __forceinline__ int mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ int64_t uni64(int64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
  uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(static_cast<uint64_t>(x) >> 32));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ uint64_t uniu64(uint64_t x) { return static_cast<uint64_t>(uni64(static_cast<int64_t>(x))); }

// value of lane `src` (wave-uniform src)
__device__ __forceinline__ int read_lane(int x, int src) { return __shfl(x, src, kWave); }

// wave-wide uint64 sum with carry detection (sets *ovf on a wrap)
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x, int* ovf) {
  int o = 0;
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) {
    uint64_t y = __shfl_xor(x, sh, kWave);
    uint64_t s = x + y;
    o |= (s < x);
    x = s;
  }
  if (ballot(o != 0)) *ovf = 1;
  return x;
}

// Inclusive prefix sum over the wave's lanes.
__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(static_cast<long long>(x), d, kWave);
    if (lane >= d) x += y;
  }
  return x;
}

// Inclusive prefix maximum over the wave's lanes with DPP moves (no LDS
// round trips): shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the
// last lane of rows 0 / 2 into rows 1 / 3 and of row 1 into rows 2 / 3.
// All lanes must be active.
__device__ __forceinline__ int wave_incl_max_i32(int x) {
  constexpr int kLow = -2147483647 - 1;
  x = max(x, __builtin_amdgcn_update_dpp(kLow, x, 0x111, 0xf, 0xf, false));  // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(kLow, x, 0x112, 0xf, 0xf, false));  // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(kLow, x, 0x114, 0xf, 0xf, false));  // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(kLow, x, 0x118, 0xf, 0xf, false));  // row_shr:8
  x = max(x, __builtin_amdgcn_update_dpp(kLow, x, 0x142, 0xa, 0xf, false));  // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(kLow, x, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return x;
}

__device__ __forceinline__ int wave_sum_i32(int x) {
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) x += __shfl_xor(x, sh, kWave);
  return x;
}

// make LDS / global writes of this wave visible to all its lanes
__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// ------------------------------------------------------------------ device-scope atomics

__device__ __forceinline__ int ld_acquire(int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int* p) {
  return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_relaxed_u64(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_acq_rel(int* p, int expected, int desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long add_u64(unsigned long long* p, unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int add_i32(int* p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}

// Relaxed: no data is published through the word.  An acquire / release
// atomic at agent scope writes back and invalidates this XCD's L2 around the
// operation, which a per-task atomic must not do.
__device__ __forceinline__ unsigned long long add_u64_relaxed(unsigned long long* p, unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// add v to a global uint64 counter (read only after the launch); a wrap sets *flag
__device__ __forceinline__ void add_counter(unsigned long long* p, unsigned long long v, int* flag) {
  if (v == 0) return;
  unsigned long long old = add_u64_relaxed(p, v);
  if (old + v < old) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ scheduler

// Termination word: (active waves << 32) | pending donated tasks.
constexpr unsigned long long kActiveOne = 1ull << 32;

struct Sched {
  unsigned long long* qhead;  // kQueueHeads block counters kHeadStride words apart (one counter when qbounds != null)
  unsigned long long* state;  // (active << 32) | pending
  int* idle;                  // waves waiting for a donated task
  int* slot_state;            // per slot: 0 empty, 1 being written, 2 full, 3 being read
  int* slot_data;             // nslots * kTaskInts
  const int32_t* qroot;       // queue entry -> root vertex (kernel id space); null = identity
  const int32_t* qlo;         // queue entry -> first-level range start; null = 0
  const int32_t* qhi;         // queue entry -> first-level range end; null = whole list
  const int32_t* qstat;       // queue entry -> root_stats row; null = the entry index
  const int64_t* qbounds;     // variable chunks: entries [qbounds[c], qbounds[c+1]); null = fixed
  int64_t nq;                 // queue entries
  int64_t nchunks;            // number of variable chunks
  int chunk;                  // fixed chunk size
  int nslots;
  int donate;                 // donation enabled
  int idle_trigger;           // donate only when at least this many waves are idle
  int period;                 // DFS steps between donation checks
  int waves;                  // waves in the launch
  uint64_t wait_limit;        // wall-clock ticks an idle wave may wait for work before it gives up
  int* flags;                 // flags[1] |= kFlagWaitLimit when a wave gives up
  // Host-driven balancing (Section IV-D's stop / copy / redistribute /
  // relaunch cycle; donation is off): once `stop_trigger` waves have found
  // the queue drained, the launch is stopped; busy waves write their untried
  // work as tasks into `spill` and leave, and the host relaunches with those
  // tasks (in `tq`) as the queue.
  int host_bal;               // 1: this launch stops and spills
  int stop_trigger;           // idle waves that stop the launch
  int* stop;                  // stop word (device)
  int* spill_n;               // tasks spilled so far (device)
  int* spill;                 // spill_cap tasks of kTaskInts ints
  int spill_cap;
  const int* tq;              // queue of tasks (kTaskInts ints each) instead of roots; null = roots
};

// flags[1] bit set by a wave that gave up waiting (the launch's counts are
// then incomplete and the call fails)
constexpr int kFlagWaitLimit = 8;

// A unit of work: root vertex, its stats row, the traversal depth the task
// starts at, the iteration range at that depth, and the prefix choices.
struct Task {
  int root;
  int64_t stat;
  int depth;  // traversal size at which iteration happens (1 = root level)
  int lo, hi;
  int full_root;  // the task starts the root (counts the root node itself)
};

// The fixed-size root queue is split into blocks of `chunk` entries dealt
// round-robin to kQueueHeads counters (block B belongs to head B mod
// kQueueHeads), each on its own 128-byte line: a wave starts at head
// wave_gid mod kQueueHeads (its XCD when blocks are placed round-robin) and
// moves on when that head is drained, so no single address takes every grab
// and the blocks still come out in about queue order.
constexpr int kQueueHeads = 8;
constexpr int kHeadStride = 16;  // u64 words between two heads

// Grab the next range of queue entries; returns false when the queue is drained.
// All lanes get the same result.
__device__ __forceinline__ bool sched_grab(const Sched& S, int* head, unsigned* dead, int wave_gid, int64_t* b,
                                           int64_t* e) {
  if (S.qbounds) {
    long long c = 0;
    if (lane_id() == 0) c = static_cast<long long>(add_u64_relaxed(S.qhead, 1ull));
    c = uni64(c);
    if (c >= S.nchunks) return false;
    *b = S.qbounds[c];
    *e = S.qbounds[c + 1];
    return true;
  }
  const int64_t nblocks = (S.nq + S.chunk - 1) / S.chunk;
  if (*head < 0) *head = wave_gid % kQueueHeads;
  for (int tries = 0; tries < kQueueHeads; ++tries) {
    const int h = (*head + tries) % kQueueHeads;
    if ((*dead >> h) & 1u) continue;
    // the queue arrays are read-only inputs: the counter needs no ordering
    long long j = 0;
    if (lane_id() == 0) j = static_cast<long long>(add_u64_relaxed(S.qhead + h * kHeadStride, 1ull));
    j = uni64(j);
    const int64_t blk = h + static_cast<int64_t>(kQueueHeads) * j;
    if (blk < nblocks) {
      *head = h;
      *b = blk * S.chunk;
      *e = *b + S.chunk < S.nq ? *b + S.chunk : S.nq;
      return true;
    }
    *dead |= 1u << h;
  }
  return false;
}

__device__ __forceinline__ Task sched_entry(const Sched& S, int64_t e, int hi_default) {
  Task t;
  t.root = S.qroot ? S.qroot[e] : static_cast<int>(e);
  t.stat = S.qstat ? static_cast<int64_t>(S.qstat[e]) : e;
  t.depth = 1;
  t.lo = S.qlo ? S.qlo[e] : 0;
  t.hi = S.qhi ? S.qhi[e] : hi_default;
  t.full_root = (t.lo == 0);
  return t;
}

// Should a busy wave donate now?  Cheap: two relaxed loads by lane 0.
__device__ __forceinline__ bool sched_want_donation(const Sched& S) {
  int want = 0;
  if (lane_id() == 0) {
    int idle = ld_relaxed(S.idle);
    unsigned long long st = ld_relaxed_u64(S.state);
    int pending = static_cast<int>(st & 0xffffffffu);
    want = (idle >= S.idle_trigger && idle > pending && pending < S.nslots) ? 1 : 0;
  }
  return uni(want) != 0;
}

// Tail-only variant: at least a quarter of the launch's waves is idle.
__device__ __forceinline__ bool sched_want_donation_tail(const Sched& S) {
  int want = 0;
  if (lane_id() == 0) {
    int idle = ld_relaxed(S.idle);
    unsigned long long st = ld_relaxed_u64(S.state);
    int pending = static_cast<int>(st & 0xffffffffu);
    want = (4 * idle >= S.waves && idle > pending && pending < S.nslots) ? 1 : 0;
  }
  return uni(want) != 0;
}

// Publish a task (payload in `data`, lane i holds int i).  Returns true when
// published.  The caller must be active while publishing.
__device__ __forceinline__ bool sched_publish(const Sched& S, int data_lane, int wave_gid) {
  const int lane = lane_id();
  int got = -1;
  // lanes look at disjoint slots starting at a wave-dependent offset
  for (int base = 0; base < S.nslots && got < 0; base += kWave) {
    int slot = (wave_gid + base + lane) % S.nslots;
    bool empty = (base + lane < S.nslots) && ld_relaxed(&S.slot_state[slot]) == 0;
    uint64_t cand = ballot(empty);
    while (cand && got < 0) {
      int l = __ffsll(static_cast<long long>(cand)) - 1;
      cand &= cand - 1;
      int ok = 0;
      if (lane == l) ok = cas_acq_rel(&S.slot_state[slot], 0, 1) ? 1 : 0;
      ok = read_lane(ok, l);
      if (ok) got = read_lane(slot, l);
    }
  }
  got = uni(got);
  if (got < 0) return false;
  if (lane < kTaskInts) st_relaxed(&S.slot_data[static_cast<int64_t>(got) * kTaskInts + lane], data_lane);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  wave_sync();
  if (lane == 0) {
    add_u64(S.state, 1ull);  // pending++ before the slot becomes visible
    st_release(&S.slot_state[got], 2);
  }
  return true;
}

// Try to claim a published task; on success lane i holds payload int i and
// the wave is counted active (pending handed over atomically).
__device__ __forceinline__ bool sched_take(const Sched& S, int* data_lane, int wave_gid) {
  const int lane = lane_id();
  int got = -1;
  for (int base = 0; base < S.nslots && got < 0; base += kWave) {
    int slot = (wave_gid * 7 + base + lane) % S.nslots;
    bool full = (base + lane < S.nslots) && ld_relaxed(&S.slot_state[slot]) == 2;
    uint64_t cand = ballot(full);
    while (cand && got < 0) {
      int l = __ffsll(static_cast<long long>(cand)) - 1;
      cand &= cand - 1;
      int ok = 0;
      if (lane == l) ok = cas_acq_rel(&S.slot_state[slot], 2, 3) ? 1 : 0;
      ok = read_lane(ok, l);
      if (ok) got = read_lane(slot, l);
    }
  }
  got = uni(got);
  if (got < 0) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  int v = 0;
  if (lane < kTaskInts) v = ld_relaxed(&S.slot_data[static_cast<int64_t>(got) * kTaskInts + lane]);
  *data_lane = v;
  wave_sync();
  if (lane == 0) {
    st_release(&S.slot_state[got], 0);
    add_u64(S.state, kActiveOne - 1ull);  // active++, pending-- in one step
  }
  return true;
}

// payload layout (one int per lane): [0] root, [1] stat low, [2] stat high,
// [3] depth, [4] lo, [5] hi, [6 ..] prefix choices for depths 1 .. depth-1.
__device__ __forceinline__ int task_payload(int root, int64_t stat, int depth, int lo, int hi,
                                            const int* prefix_lds) {
  const int lane = lane_id();
  int v = 0;
  if (lane == 0) v = root;
  else if (lane == 1) v = static_cast<int>(static_cast<uint64_t>(stat) & 0xffffffffu);
  else if (lane == 2) v = static_cast<int>(static_cast<uint64_t>(stat) >> 32);
  else if (lane == 3) v = depth;
  else if (lane == 4) v = lo;
  else if (lane == 5) v = hi;
  else if (lane >= 6 && lane < 6 + depth - 1 && lane < kTaskInts) v = prefix_lds[lane - 6 + 1];
  return v;
}

// A range task hands over queue entries [lo, hi) that a wave has not started
// yet (depth 0 marks it; the root field is unused).
__device__ __forceinline__ int task_range_payload(int64_t lo, int64_t hi) {
  const int lane = lane_id();
  int v = 0;
  if (lane == 4) v = static_cast<int>(lo);
  else if (lane == 5) v = static_cast<int>(hi);
  return v;
}

__device__ __forceinline__ Task task_unpack(int data_lane, int* prefix_lds) {
  Task t;
  t.root = uni(read_lane(data_lane, 0));
  uint32_t slo = static_cast<uint32_t>(uni(read_lane(data_lane, 1)));
  uint32_t shi = static_cast<uint32_t>(uni(read_lane(data_lane, 2)));
  t.stat = static_cast<int64_t>((static_cast<uint64_t>(shi) << 32) | slo);
  t.depth = uni(read_lane(data_lane, 3));
  t.lo = uni(read_lane(data_lane, 4));
  t.hi = uni(read_lane(data_lane, 5));
  t.full_root = 0;
  const int lane = lane_id();
  if (lane >= 6 && lane < 6 + t.depth - 1) prefix_lds[lane - 6 + 1] = data_lane;
  wave_sync();
  return t;
}

// The persistent wave's work source (Section IV-B Move, with the Section IV-D
// rebalancing done inside the kernel).  A wave takes queue chunks while the
// queue lasts, then waits for donated work until no wave is active and no task
// is pending.  Between two entries of a chunk (or of a donated entry range)
// the wave hands the untried upper half of the range to waiting waves.
// Usage: SchedIter it; sched_begin(S, it); while (sched_next(S, it, ...)) run;
// sched_end(S, it).
struct SchedIter {
  int mode;  // 0: taking queue chunks, 1: waiting, 2: running donated work
  int64_t q, e;
  uint64_t t0, t_idle;
  int head;       // queue head this wave grabs from (-1: not chosen yet)
  unsigned dead;  // heads found drained
};

__device__ __forceinline__ void sched_begin(const Sched& S, SchedIter& it) {
  it.mode = 0;
  it.q = it.e = 0;
  it.t0 = it.t_idle = 0;
  it.head = -1;
  it.dead = 0;
  if (lane_id() == 0) add_u64(S.state, kActiveOne);
}

template <bool kHostBal = false>
__device__ __forceinline__ void sched_go_idle(const Sched& S, SchedIter& it) {
  if (lane_id() == 0) {
    const int before = add_i32(S.idle, 1);
    add_u64(S.state, 0ull - kActiveOne);
    if (kHostBal && S.host_bal && before + 1 >= S.stop_trigger) st_relaxed(S.stop, 1);
  }
  it.mode = 1;
  it.t0 = wall_clock64();
}

// Host-driven balancing: has the launch been stopped?  (one relaxed load)
__device__ __forceinline__ bool sched_stopped(const Sched& S) {
  int v = 0;
  if (lane_id() == 0) v = ld_relaxed(S.stop);
  return uni(v) != 0;
}

// Host-driven balancing: write one task (payload in `data`, lane i holds int
// i) to the spill array; a full array flags the launch (flags[1] bit 16).
__device__ __forceinline__ void sched_spill(const Sched& S, int data_lane) {
  const int lane = lane_id();
  int slot = 0;
  if (lane == 0) slot = add_i32(S.spill_n, 1);
  slot = uni(slot);
  if (slot >= S.spill_cap) {
    if (lane == 0) atomicOr(S.flags + 1, 16);
    return;
  }
  if (lane < kTaskInts) S.spill[static_cast<int64_t>(slot) * kTaskInts + lane] = data_lane;
}

// Next unit of work into *t; false when the whole launch has drained.
// kHostBal: the instantiation of kernels launched with host-driven balancing
// (queues of spilled tasks, the stop trigger); the others compile without it.
template <bool kHostBal = false>
__device__ __forceinline__ bool sched_next(const Sched& S, SchedIter& it, int wave_gid, int* prefix_lds, Task* t) {
  for (;;) {
    if (it.q < it.e) {
      if (S.donate && it.e - it.q >= 2 && sched_want_donation(S)) {
        const int64_t mid = it.q + (it.e - it.q + 1) / 2;
        if (sched_publish(S, task_range_payload(mid, it.e), wave_gid)) it.e = mid;
      }
      if (kHostBal && S.tq) {
        // a task written by an earlier, stopped launch
        const int lane = lane_id();
        const int data = lane < kTaskInts ? S.tq[it.q * kTaskInts + lane] : 0;
        ++it.q;
        *t = task_unpack(data, prefix_lds);
        return true;
      }
      *t = sched_entry(S, it.q, INT_MAX);
      ++it.q;
      return true;
    }
    if (it.mode == 0) {
      int64_t b, e;
      if (sched_grab(S, &it.head, &it.dead, wave_gid, &b, &e)) {
        it.q = b;
        it.e = e;
        continue;
      }
      sched_go_idle<kHostBal>(S, it);
      if (!S.donate) return false;  // also with host-driven balancing, where donation is off
      continue;
    }
    if (it.mode == 2) {
      sched_go_idle(S, it);
      continue;
    }
    unsigned long long st = 0;
    if (lane_id() == 0) st = ld_relaxed_u64(S.state);
    st = uniu64(st);
    if (st == 0) {
      it.t_idle += wall_clock64() - it.t0;
      return false;
    }
    int data = 0;
    if ((st & 0xffffffffull) == 0 || !sched_take(S, &data, wave_gid)) {
      // bounded wait: a wave idle for longer than the limit leaves the loop
      // and flags the launch, so a scheduler fault ends the kernel with an
      // error instead of keeping the GPU busy
      const uint64_t waited = wall_clock64() - it.t0;
      if (uniu64(waited) > S.wait_limit) {
        if (lane_id() == 0) atomicOr(S.flags + 1, kFlagWaitLimit);
        it.t_idle += waited;
        return false;
      }
      __builtin_amdgcn_s_sleep(16);
      continue;
    }
    it.t_idle += wall_clock64() - it.t0;
    if (lane_id() == 0) add_i32(S.idle, -1);
    it.mode = 2;
    *t = task_unpack(data, prefix_lds);
    if (t->depth == 0) {
      it.q = t->lo;
      it.e = t->hi;
      continue;
    }
    return true;
  }
}

// Leave the loop: the wave counted itself idle when the work ran out.  Under
// host-driven balancing the count is left as it is: waves leave as soon as
// they run out of work, and the stop trigger counts the waves that have
// finished.
template <bool kHostBal = false>
__device__ __forceinline__ void sched_end(const Sched& S) {
  if (!kHostBal && lane_id() == 0) add_i32(S.idle, -1);
}

}  // namespace dm

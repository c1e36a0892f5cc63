// Learned root ordering: per-vertex features, a 4 -> 64 -> 64 -> 1 FP32 MLP
// (forward, backward, Adam) that predicts log(1 + enumeration-tree size) of a
// root, and the LPT ordering / equal-cost chunking of the root queue.
//
// This is an addition to DuMato: the paper balances load only reactively
// (Section IV-D) and notes that the cost of a traversal cannot be known in
// advance (Section I); the prediction here only orders and chunks the initial
// work and never changes a count.  Everything is plain FP32 VALU code: the
// network has 4,545 weights, far too small for matrix cores to matter.
#include <hipcub/hipcub.hpp>

#include "dm_internal.hpp"

namespace dm {

namespace {

constexpr int kH = 64;
constexpr int oW1 = 0;      // [64][4]
constexpr int oB1 = 256;    // [64]
constexpr int oW2 = 320;    // [64][64], row j = hidden-2 unit j
constexpr int oB2 = 4416;   // [64]
constexpr int oW3 = 4480;   // [64]
constexpr int oB3 = 4544;   // [1]
constexpr int oMean = kMlpNet;      // [4] mean of log1p(feature)
constexpr int oStd = kMlpNet + 4;   // [4] std of log1p(feature)

__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) x += __shfl_xor(x, sh, kWave);
  return x;
}

// ------------------------------------------------------------------ features

__global__ void __launch_bounds__(256) feat_deg_twohop_kernel(const int64_t* rp, const int32_t* col, int32_t n,
                                                              int64_t* F) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int64_t b = rp[v], e = rp[v + 1];
    int64_t s = 0;
    for (int64_t i = b + lane; i < e; i += 64) {
      const int u = col[i];
      s += rp[u + 1] - rp[u];
    }
    s = wave_sum_i64(s);
    if (lane == 0) {
      F[v * 4 + 0] = e - b;
      F[v * 4 + 1] = s;
    }
  }
}

// triangles: each triangle a < u < e (rank order) is found once from a, and
// credited to its three vertices (original ids)
__global__ void __launch_bounds__(256) feat_triangle_kernel(const int64_t* drp, const int32_t* dcol,
                                                            const int32_t* order, int32_t n,
                                                            unsigned long long* tri) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t a = wave; a < n; a += nwaves) {
    const int64_t ab = drp[a], ae = drp[a + 1];
    for (int64_t p = ab; p < ae; ++p) {
      const int u = dcol[p];
      const int64_t ub = drp[u], ue = drp[u + 1];
      for (int64_t i = ub + lane; i < ue; i += 64) {
        const int e = dcol[i];
        int64_t lo = p + 1, hi = ae;
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (dcol[mid] < e) lo = mid + 1; else hi = mid;
        }
        if (lo < ae && dcol[lo] == e) {
          atomicAdd(&tri[order[a]], 1ull);
          atomicAdd(&tri[order[u]], 1ull);
          atomicAdd(&tri[order[e]], 1ull);
        }
      }
    }
  }
}

__global__ void feat_store_kernel(const unsigned long long* tri, const int32_t* core, int32_t n, int64_t* F) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) {
    F[v * 4 + 2] = core[v];
    F[v * 4 + 3] = static_cast<int64_t>(tri[v]);
  }
}

__global__ void core_init_kernel(const int64_t* rp, int32_t n, int32_t* core) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) core[v] = static_cast<int32_t>(rp[v + 1] - rp[v]);
}

// One sweep of the h-index operator: core(v) <- largest h <= core(v) such that
// at least h neighbours have core >= h.  Started from degrees and repeated
// until nothing changes, it reaches the k-core numbers (Lu et al., Nature
// Communications 2016); values only decrease, so in-place updates are safe and
// a sweep with no change is a fixed point.
__global__ void __launch_bounds__(256) core_sweep_kernel(const int64_t* rp, const int32_t* col, int32_t n,
                                                         int32_t* core, int* changed) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int cv = __builtin_amdgcn_readfirstlane(core[v]);
    if (cv == 0) continue;
    const int64_t b = rp[v], e = rp[v + 1];
    int lo = 0, hi = cv;  // P(lo) holds; find the largest h with P(h)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      int c = 0;
      for (int64_t i = b + lane; i < e; i += 64) c += core[col[i]] >= mid ? 1 : 0;
      c = wave_sum_i32(c);
      if (c >= mid) lo = mid; else hi = mid - 1;
    }
    if (lo < cv && lane == 0) {
      core[v] = lo;
      *changed = 1;
    }
  }
}

// ------------------------------------------------------------------ MLP

__device__ __forceinline__ float feature_in(const float* P, const int64_t* F, int64_t r, int c) {
  const float x = log1pf(static_cast<float>(F[r * 4 + c]));
  return (x - P[oMean + c]) / P[oStd + c];
}

__global__ void __launch_bounds__(256) mlp_forward_kernel(const float* Pg, const int64_t* F, int64_t n, float* out) {
  __shared__ float P[kMlpBlob];
  for (int i = threadIdx.x; i < kMlpBlob; i += blockDim.x) P[i] = Pg[i];
  __syncthreads();
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float x[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] = feature_in(P, F, r, c);
  float h1[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float z = P[oB1 + j];
#pragma unroll
    for (int c = 0; c < 4; ++c) z += P[oW1 + j * 4 + c] * x[c];
    h1[j] = z > 0.f ? z : 0.f;
  }
  float y = P[oB3];
  for (int j = 0; j < kH; ++j) {
    float z = P[oB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) z += P[oW2 + j * kH + i] * h1[i];
    y += P[oW3 + j] * (z > 0.f ? z : 0.f);
  }
  out[r] = y;
}

// Loss 1/B sum (y - t)^2 and its gradient for the rows of one block of 64
// rows (one row per lane); partial sums per block, reduced by
// mlp_reduce_kernel in block order (deterministic).
__global__ void __launch_bounds__(64) mlp_grad_kernel(const float* Pg, const int64_t* F, const float* T,
                                                      const int32_t* rows, int64_t nrows, float inv_b,
                                                      float* partial) {
  __shared__ float P[kMlpBlob];
  __shared__ float s_h1[64][kH + 1];
  __shared__ float s_dh2[64][kH + 1];
  __shared__ float s_dw3[kH], s_dW1[kH * 4], s_db1[kH];
  __shared__ float s_dy[64], s_l[64];
  const int t = threadIdx.x;
  for (int i = t; i < kMlpBlob; i += 64) P[i] = Pg[i];
  for (int i = t; i < kH; i += 64) { s_dw3[i] = 0.f; s_db1[i] = 0.f; }
  for (int i = t; i < kH * 4; i += 64) s_dW1[i] = 0.f;
  __syncthreads();
  const int64_t ri = static_cast<int64_t>(blockIdx.x) * 64 + t;
  const bool valid = ri < nrows;
  const int64_t r = valid ? (rows ? static_cast<int64_t>(rows[ri]) : ri) : 0;
  float x[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] = valid ? feature_in(P, F, r, c) : 0.f;
  float h1[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float z = P[oB1 + j];
#pragma unroll
    for (int c = 0; c < 4; ++c) z += P[oW1 + j * 4 + c] * x[c];
    h1[j] = z > 0.f ? z : 0.f;
    s_h1[t][j] = valid ? h1[j] : 0.f;
  }
  float y = P[oB3];
  for (int j = 0; j < kH; ++j) {
    float z = P[oB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) z += P[oW2 + j * kH + i] * h1[i];
    y += P[oW3 + j] * (z > 0.f ? z : 0.f);
  }
  const float diff = valid ? (y - T[r]) : 0.f;
  const float dy = 2.f * inv_b * diff;
  s_dy[t] = dy;
  s_l[t] = inv_b * diff * diff;
  // dh2, dw3 (staggered LDS atomics so lanes hit different banks)
  for (int jj = 0; jj < kH; ++jj) {
    const int j = (jj + t) & (kH - 1);
    float z = P[oB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) z += P[oW2 + j * kH + i] * h1[i];
    const float h2 = z > 0.f ? z : 0.f;
    s_dh2[t][j] = (z > 0.f) ? dy * P[oW3 + j] : 0.f;
    atomicAdd(&s_dw3[j], dy * h2);
  }
  __syncthreads();
  // dh1 for this row, then dW1 / db1
  for (int ii = 0; ii < kH; ++ii) {
    const int i = (ii + t) & (kH - 1);
    float g = 0.f;
    if (s_h1[t][i] > 0.f) {
      for (int j = 0; j < kH; ++j) g += P[oW2 + j * kH + i] * s_dh2[t][j];
    }
    atomicAdd(&s_db1[i], g);
#pragma unroll
    for (int c = 0; c < 4; ++c) atomicAdd(&s_dW1[i * 4 + c], g * x[c]);
  }
  __syncthreads();
  float* out = partial + static_cast<size_t>(blockIdx.x) * (kMlpNet + 1);
  // dW2[j][i] = sum_rows dh2[j] h1[i]; lane j owns row j of W2
  {
    const int j = t;
    float db2 = 0.f;
    for (int rr = 0; rr < 64; ++rr) db2 += s_dh2[rr][j];
    for (int i = 0; i < kH; ++i) {
      float g = 0.f;
      for (int rr = 0; rr < 64; ++rr) g += s_dh2[rr][j] * s_h1[rr][i];
      out[oW2 + j * kH + i] = g;
    }
    out[oB2 + j] = db2;
    out[oW3 + j] = s_dw3[j];
    out[oB1 + j] = s_db1[j];
#pragma unroll
    for (int c = 0; c < 4; ++c) out[oW1 + j * 4 + c] = s_dW1[j * 4 + c];
  }
  if (t == 0) {
    float db3 = 0.f, l = 0.f;
    for (int rr = 0; rr < 64; ++rr) { db3 += s_dy[rr]; l += s_l[rr]; }
    out[oB3] = db3;
    out[kMlpNet] = l;
  }
}

__global__ void mlp_reduce_kernel(const float* partial, int blocks, float* grad, float* loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kMlpNet) return;
  float s = 0.f;
  for (int b = 0; b < blocks; ++b) s += partial[static_cast<size_t>(b) * (kMlpNet + 1) + i];
  if (i < kMlpNet) grad[i] = s; else *loss = s;
}

// Adam (Kingma & Ba 2015) with bias correction; step t starts at 1
__global__ void adam_kernel(float* P, const float* g, float* m, float* v, int count, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  P[i] -= lr * mh / (sqrtf(vh) + eps);
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator
__device__ __forceinline__ uint64_t mix_counter(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// He-uniform weights (bound sqrt(6 / fan_in)), zero biases, identity normaliser
__global__ void mlp_init_kernel(float* P, uint64_t seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpBlob) return;
  float val = 0.f;
  float fan = 0.f;
  if (i < oB1) fan = 4.f;
  else if (i >= oW2 && i < oB2) fan = 64.f;
  else if (i >= oW3 && i < oB3) fan = 64.f;
  if (fan > 0.f) {
    const float u = static_cast<float>(mix_counter(seed, static_cast<uint64_t>(i)) >> 40) * (1.0f / 16777216.0f);
    const float bound = sqrtf(6.f / fan);
    val = (2.f * u - 1.f) * bound;
  }
  if (i >= oStd) val = 1.f;
  P[i] = val;
}

// mean / std of log1p(feature c) over n rows, into the normaliser slots
__global__ void __launch_bounds__(256) normaliser_kernel(const int64_t* F, int64_t n, float* P) {
  __shared__ double s1[4][256], s2[4][256];
  const int t = threadIdx.x;
  double a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
  for (int64_t r = t; r < n; r += 256)
    for (int c = 0; c < 4; ++c) {
      const double x = log1p(static_cast<double>(F[r * 4 + c]));
      a[c] += x;
      b[c] += x * x;
    }
  for (int c = 0; c < 4; ++c) { s1[c][t] = a[c]; s2[c][t] = b[c]; }
  __syncthreads();
  if (t < 4) {
    double m = 0, q = 0;
    for (int i = 0; i < 256; ++i) { m += s1[t][i]; q += s2[t][i]; }
    m /= static_cast<double>(n > 0 ? n : 1);
    q = q / static_cast<double>(n > 0 ? n : 1) - m * m;
    const double sd = q > 1e-12 ? sqrt(q) : 1.0;
    P[oMean + t] = static_cast<float>(m);
    P[oStd + t] = static_cast<float>(sd);
  }
}

__global__ void targets_kernel(const unsigned long long* stats, int64_t n, float* out) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < n) out[r] = static_cast<float>(log1p(static_cast<double>(stats[r * 3])));
}

__global__ void shuffle_keys_kernel(uint64_t seed, int64_t n, unsigned long long* keys, int32_t* vals) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    keys[i] = mix_counter(seed, static_cast<uint64_t>(i));
    vals[i] = static_cast<int32_t>(i);
  }
}

// ------------------------------------------------------------------ LPT queue

__global__ void iota_kernel(int32_t* out, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = static_cast<int32_t>(i);
}

// predicted cost of the sorted roots, exp(pred) - 1 clamped at 0
__global__ void cost_kernel(const float* pred_sorted, int64_t n, double* cost) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    // predicted tree nodes + the root itself: exp(log1p(nodes))
    cost[i] = exp(static_cast<double>(pred_sorted[i]));
  }
}

// chunk id of entry i = floor(exclusive prefix / target); entry i starts a
// chunk when its id differs from entry i-1 (ids are non-decreasing), and every
// `max_roots` entries, so the many light roots at the end of the order never
// form one long chunk
__global__ void chunk_flag_kernel(const double* incl, const double* cost, int64_t n, double target,
                                  int64_t max_roots, int32_t* flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == 0) {
    flag[0] = 1;
    return;
  }
  const double a = floor((incl[i - 1] - cost[i - 1]) / target);
  const double b = floor((incl[i] - cost[i]) / target);
  flag[i] = (b > a || i % max_roots == 0) ? 1 : 0;
}

__global__ void to_i64_kernel(const int32_t* in, int64_t n, int64_t* out, int64_t tail) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
  if (i == n) out[n] = tail;
}

inline unsigned blocks_for(int64_t count, int threads) {
  int64_t b = (count + threads - 1) / threads;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

inline unsigned wave_grid(int64_t n) {
  unsigned g = blocks_for((n > 0 ? n : 1) * 64, 256);
  return g > 65536 ? 65536 : g;
}

}  // namespace

// ====================================================================== host launchers

hipError_t compute_features(const int64_t* rp, const int32_t* col, int32_t n, const int64_t* drp,
                            const int32_t* dcol, const int32_t* order, int64_t* F, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned long long* tri = nullptr;
  int32_t* core = nullptr;
  int* changed = nullptr;
  hipError_t e = hipMalloc(&tri, sizeof(unsigned long long) * n);
  if (e == hipSuccess) e = hipMalloc(&core, sizeof(int32_t) * n);
  if (e == hipSuccess) e = hipMalloc(&changed, sizeof(int));
  if (e == hipSuccess) e = launch_fill_u64(tri, n, 0ull, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(feat_deg_twohop_kernel, dim3(wave_grid(n)), dim3(256), 0, s, rp, col, n, F);
    hipLaunchKernelGGL(feat_triangle_kernel, dim3(wave_grid(n)), dim3(256), 0, s, drp, dcol, order, n, tri);
    hipLaunchKernelGGL(core_init_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rp, n, core);
    e = hipGetLastError();
  }
  for (int64_t it = 0; e == hipSuccess && it <= n; ++it) {
    int host_changed = 0;
    e = launch_fill_i32(changed, 1, 0, s);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(core_sweep_kernel, dim3(wave_grid(n)), dim3(256), 0, s, rp, col, n, core, changed);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&host_changed, changed, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || !host_changed) break;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(feat_store_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, tri, core, n, F);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(tri);
  (void)hipFree(core);
  (void)hipFree(changed);
  return e;
}

hipError_t mlp_init(float* P, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(mlp_init_kernel, dim3(blocks_for(kMlpBlob, 256)), dim3(256), 0, s, P, seed);
  return hipGetLastError();
}

hipError_t mlp_fit_normaliser(float* P, const int64_t* F, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(normaliser_kernel, dim3(1), dim3(256), 0, s, F, n, P);
  return hipGetLastError();
}

hipError_t mlp_forward(const float* P, const int64_t* F, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, F, n, out);
  return hipGetLastError();
}

hipError_t mlp_targets(const unsigned long long* stats, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(targets_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, stats, n, out);
  return hipGetLastError();
}

// gradient of the mean squared error over `nrows` rows (rows[i], or 0..nrows-1)
hipError_t mlp_loss_grad(const float* P, const int64_t* F, const float* T, const int32_t* rows, int64_t nrows,
                         float* partial, float* grad, float* loss, hipStream_t s) {
  const int blocks = static_cast<int>((nrows + 63) / 64);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks), dim3(64), 0, s, P, F, T, rows, nrows,
                     1.0f / static_cast<float>(nrows), partial);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3(blocks_for(kMlpNet + 1, 256)), dim3(256), 0, s, partial, blocks,
                     grad, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(float* P, const float* g, float* m, float* v, int64_t t, float lr, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, static_cast<float>(t));
  const float c2 = 1.f - powf(b2, static_cast<float>(t));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(kMlpNet, 256)), dim3(256), 0, s, P, g, m, v, kMlpNet, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_shuffle(uint64_t seed, int64_t n, unsigned long long* keys, unsigned long long* keys_out,
                       int32_t* vals, int32_t* vals_out, void* temp, size_t temp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(shuffle_keys_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, seed, n, keys, vals);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t tb = temp_bytes;
  return hipcub::DeviceRadixSort::SortPairs(temp, tb, keys, keys_out, vals, vals_out, static_cast<int>(n), 0, 64, s);
}

size_t mlp_shuffle_temp_bytes(int64_t n) {
  size_t need = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, need, static_cast<unsigned long long*>(nullptr),
                                           static_cast<unsigned long long*>(nullptr), static_cast<int32_t*>(nullptr),
                                           static_cast<int32_t*>(nullptr), static_cast<int>(n), 0, 64, nullptr);
  return need;
}

// Order-sensitive 64-bit fingerprint of a parameter blob (the cache key of a
// graph's learned queue; not a cryptographic hash).  One block of 256.
__global__ void param_hash_kernel(const float* P, int n, unsigned long long* out) {
  __shared__ unsigned long long part[256];
  unsigned long long h = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    uint64_t x = (static_cast<uint64_t>(__float_as_uint(P[i])) << 32) ^ (static_cast<uint64_t>(i) * 0x9E3779B97F4A7C15ull);
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    h += x;
  }
  part[threadIdx.x] = h;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) part[threadIdx.x] += part[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

hipError_t param_fingerprint(const float* P, int n, unsigned long long* dev_out, hipStream_t s) {
  hipLaunchKernelGGL(param_hash_kernel, dim3(1), dim3(256), 0, s, P, n, dev_out);
  return hipGetLastError();
}

// Longest-predicted-first order and equal-predicted-cost chunks.
// order_out[i] = vertex at queue position i; bounds_out gets chunk starts and
// a final n (size n+1 at most); returns the chunk count in *nchunks.
hipError_t lpt_order(const float* pred, int64_t n, int chunks_wanted, int32_t* order_out, int64_t* bounds_out,
                     int64_t* nchunks, hipStream_t s) {
  if (n <= 0) {
    *nchunks = 0;
    return hipSuccess;
  }
  hipError_t e = hipSuccess;
  float* keys_out = nullptr;
  int32_t* ids = nullptr;
  double *cost = nullptr, *incl = nullptr;
  int32_t *flag = nullptr, *sel = nullptr, *nsel = nullptr;
  void* temp = nullptr;
  size_t tb = 0, need = 0;
  int32_t host_nsel = 0;
  double total = 0.0;
#define LPT_TRY(x)          \
  do {                      \
    e = (x);                \
    if (e != hipSuccess) goto done; \
  } while (0)
  LPT_TRY(hipMalloc(&keys_out, sizeof(float) * n));
  LPT_TRY(hipMalloc(&ids, sizeof(int32_t) * n));
  LPT_TRY(hipMalloc(&cost, sizeof(double) * n));
  LPT_TRY(hipMalloc(&incl, sizeof(double) * n));
  LPT_TRY(hipMalloc(&flag, sizeof(int32_t) * n));
  LPT_TRY(hipMalloc(&sel, sizeof(int32_t) * n));
  LPT_TRY(hipMalloc(&nsel, sizeof(int32_t)));
  LPT_TRY(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, need, pred, keys_out, ids, order_out,
                                                       static_cast<int>(n), 0, 32, s));
  tb = need;
  LPT_TRY(hipcub::DeviceScan::InclusiveSum(nullptr, need, cost, incl, static_cast<int>(n), s));
  tb = need > tb ? need : tb;
  LPT_TRY(hipcub::DeviceSelect::Flagged(nullptr, need, static_cast<int32_t*>(nullptr), flag, sel, nsel,
                                        static_cast<int>(n), s));
  tb = need > tb ? need : tb;
  LPT_TRY(hipMalloc(&temp, tb > 0 ? tb : 16));
  hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, ids, n);
  LPT_TRY(hipGetLastError());
  need = tb;
  LPT_TRY(hipcub::DeviceRadixSort::SortPairsDescending(temp, need, pred, keys_out, ids, order_out,
                                                       static_cast<int>(n), 0, 32, s));
  hipLaunchKernelGGL(cost_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys_out, n, cost);
  LPT_TRY(hipGetLastError());
  need = tb;
  LPT_TRY(hipcub::DeviceScan::InclusiveSum(temp, need, cost, incl, static_cast<int>(n), s));
  LPT_TRY(hipMemcpyAsync(&total, incl + (n - 1), sizeof(double), hipMemcpyDeviceToHost, s));
  LPT_TRY(hipStreamSynchronize(s));
  {
    const int cw = chunks_wanted > 0 ? chunks_wanted : 1;
    double target = total / static_cast<double>(cw);
    if (!(target > 0.0)) target = 1e300;  // no predicted cost: one chunk
    const int64_t max_roots = (n + cw - 1) / cw;
    hipLaunchKernelGGL(chunk_flag_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, incl, cost, n, target,
                       max_roots, flag);
    LPT_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, ids, n);
  LPT_TRY(hipGetLastError());
  need = tb;
  LPT_TRY(hipcub::DeviceSelect::Flagged(temp, need, ids, flag, sel, nsel, static_cast<int>(n), s));
  LPT_TRY(hipMemcpyAsync(&host_nsel, nsel, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LPT_TRY(hipStreamSynchronize(s));
  hipLaunchKernelGGL(to_i64_kernel, dim3(blocks_for(static_cast<int64_t>(host_nsel) + 1, 256)), dim3(256), 0, s, sel,
                     static_cast<int64_t>(host_nsel), bounds_out, n);
  LPT_TRY(hipGetLastError());
  LPT_TRY(hipStreamSynchronize(s));
  *nchunks = host_nsel;
done:
  (void)hipFree(keys_out);
  (void)hipFree(ids);
  (void)hipFree(cost);
  (void)hipFree(incl);
  (void)hipFree(flag);
  (void)hipFree(sel);
  (void)hipFree(nsel);
  (void)hipFree(temp);
  return e;
#undef LPT_TRY
}

}  // namespace dm

// Dynamic definition (Section 4.3, Algorithm 1) device steps:
//  * merge:  sum each subcircuit's entries over its merged outputs, with the
//            zoomed outputs held at their fixed values (FP64);
//  * top-C:  exact selection of the C largest bins by (value desc, index asc);
//  * refine: FP64 value of chosen bins straight from Eq. 1 over the reduced
//            entries, which drives the list update and zoom choice.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "kernels.hpp"

namespace cq {

namespace {

// Scatter the low bits of x into the set bits of mask (lowest first).
__device__ inline uint64_t deposit(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  for (uint64_t bit = 1; mask; bit <<= 1) {
    const uint64_t low = mask & (~mask + 1);
    if (x & bit) r |= low;
    mask ^= low;
  }
  return r;
}

struct MergeArgs {
  const double* E;
  double* Ep;
  int64_t outputs;  // rows << na
  int n, na, tpo_log2;
  int64_t iters;    // 2^(nm - tpo_log2)
  uint64_t active_flat, merged_lo, merged_hi, fixed_vals_flat;
};

// A group of 2^tpo_log2 lanes sums one reduced entry; lanes stride the merged
// index, then a fixed xor-butterfly combines them (deterministic order).
__global__ void __launch_bounds__(256) merge_kernel(MergeArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t out = g >> a.tpo_log2;
  const int sub = (int)(g & ((1 << a.tpo_log2) - 1));
  if (out >= a.outputs) return;
  const int64_t row = out >> a.na;
  const uint64_t av = (uint64_t)(out & (((int64_t)1 << a.na) - 1));
  const double* Er = a.E + (row << a.n);
  const uint64_t base = a.fixed_vals_flat | deposit(av, a.active_flat) | deposit((uint64_t)sub, a.merged_lo);
  double acc = 0.0;
  uint64_t d = 0;
  for (int64_t t = 0; t < a.iters; ++t) {
    acc += Er[base | d];
    d = ((d | ~a.merged_hi) + 1) & a.merged_hi;
  }
  for (int s = (1 << a.tpo_log2) >> 1; s >= 1; s >>= 1) acc += __shfl_xor(acc, s);
  if (sub == 0) a.Ep[out] = acc;
}

// ---------------------------------------------------------------------------
// Top-C.  A workgroup scans its chunk and keeps only keys better than its
// current C-th best; survivors go to an LDS buffer that is bitonic-sorted and
// trimmed to C whenever it could overflow.  Keys (value, index) are unique,
// so ties in value resolve to the lower index.
// ---------------------------------------------------------------------------
constexpr int kTopS = 4096;   // LDS buffer entries
constexpr int kTopU = 8;      // elements per thread per round

struct Key {
  double v;
  uint64_t i;
};

__device__ inline bool better(const Key& a, const Key& b) {
  return a.v > b.v || (a.v == b.v && a.i < b.i);
}

__device__ inline Key worst_key() { return Key{-DBL_MAX, ~(uint64_t)0}; }

// Sorts buf[0..kTopS) best-first; all threads of the workgroup call it.
__device__ void bitonic_sort(Key* buf) {
  for (int k = 2; k <= kTopS; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < kTopS / 2; t += blockDim.x) {
        const int i = 2 * j * (t / j) + (t % j);
        const int p = i + j;
        const bool asc = (i & k) == 0;  // "ascending" = best first
        Key x = buf[i], y = buf[p];
        const bool swap = asc ? better(y, x) : better(x, y);
        if (swap) {
          buf[i] = y;
          buf[p] = x;
        }
      }
      __syncthreads();
    }
  }
}

template <typename T, bool kExplicit>
__global__ void __launch_bounds__(256) topk_kernel(const T* __restrict__ vals,
                                                   const uint64_t* __restrict__ idxs,
                                                   int64_t count, int64_t chunk, int C,
                                                   double* __restrict__ out_v,
                                                   uint64_t* __restrict__ out_i) {
  __shared__ Key buf[kTopS];
  __shared__ int cnt;
  __shared__ Key thr;
  const int64_t begin = (int64_t)blockIdx.x * chunk;
  int64_t end = begin + chunk;
  if (end > count) end = count;
  if (threadIdx.x == 0) {
    cnt = 0;
    thr = worst_key();
  }
  __syncthreads();
  auto trim = [&]() {
    for (int t = cnt + threadIdx.x; t < kTopS; t += blockDim.x) buf[t] = worst_key();
    __syncthreads();
    bitonic_sort(buf);
    if (threadIdx.x == 0) {
      if (cnt > C) cnt = C;
      thr = (cnt == C) ? buf[C - 1] : worst_key();
    }
    __syncthreads();
  };
  const int64_t round = (int64_t)blockDim.x * kTopU;
  for (int64_t r0 = begin; r0 < end; r0 += round) {
    const Key th = thr;
#pragma unroll
    for (int u = 0; u < kTopU; ++u) {
      const int64_t x = r0 + (int64_t)u * blockDim.x + threadIdx.x;
      if (x < end) {
        Key key{double(vals[x]), kExplicit ? idxs[x] : (uint64_t)x};
        if (better(key, th)) {
          const int pos = atomicAdd(&cnt, 1);
          buf[pos] = key;
        }
      }
    }
    __syncthreads();
    if (cnt > kTopS - round) trim();
  }
  trim();
  for (int t = threadIdx.x; t < C; t += blockDim.x) {
    const Key k = (t < cnt) ? buf[t] : worst_key();
    out_v[(int64_t)blockIdx.x * C + t] = k.v;
    out_i[(int64_t)blockIdx.x * C + t] = k.i;
  }
}

int64_t topk_blocks(int64_t count) {
  int64_t b = (count + 65535) / 65536;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return b;
}

// ---------------------------------------------------------------------------
// Refine: one workgroup per bin, threads over the 4^K global labels.
// ---------------------------------------------------------------------------
struct RefineArgs {
  int n_sub, K;
  const double* Ep[CQ_MAX_SUBCIRCUITS];
  int64_t ld[CQ_MAX_SUBCIRCUITS];
  int na[CQ_MAX_SUBCIRCUITS];
  int kc[CQ_MAX_SUBCIRCUITS];
  int cut[CQ_MAX_SUBCIRCUITS][CQ_MAX_LOCAL_CUTS];
  const uint64_t* bins;
  double scale;
  double* out;
};

__global__ void __launch_bounds__(256) refine_kernel(RefineArgs a) {
  __shared__ double red[256];
  const uint64_t bin = a.bins[blockIdx.x];
  int64_t col[CQ_MAX_SUBCIRCUITS];
  int shift = 0;
  for (int c = 0; c < a.n_sub; ++c) shift += a.na[c];
  for (int c = 0; c < a.n_sub; ++c) {
    shift -= a.na[c];
    col[c] = (int64_t)((bin >> shift) & ((((uint64_t)1) << a.na[c]) - 1));
  }
  const int64_t labels = (int64_t)1 << (2 * a.K);
  double sum = 0.0;
  for (int64_t l = threadIdx.x; l < labels; l += blockDim.x) {
    double prod = 1.0;
    for (int c = 0; c < a.n_sub; ++c) {
      int64_t row = 0;
      for (int j = 0; j < a.kc[c]; ++j) row = 4 * row + ((l >> (2 * (a.K - 1 - a.cut[c][j]))) & 3);
      prod *= a.Ep[c][row * a.ld[c] + col[c]];
    }
    sum += prod;
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.out[blockIdx.x] = a.scale * red[0];
}

}  // namespace

hipError_t launch_merge(const MergeLaunch& m, hipStream_t stream) {
  MergeArgs a;
  a.E = m.E;
  a.Ep = m.Ep;
  a.n = m.n;
  a.na = m.na;
  a.outputs = m.rows << m.na;
  a.tpo_log2 = m.nm < 6 ? m.nm : 6;
  a.iters = (int64_t)1 << (m.nm - a.tpo_log2);
  a.active_flat = m.active_flat;
  a.fixed_vals_flat = m.fixed_vals_flat;
  // lowest tpo_log2 merged bits go to the lanes, the rest to the loop
  uint64_t lo = 0, rest = m.merged_flat;
  for (int i = 0; i < a.tpo_log2; ++i) {
    const uint64_t low = rest & (~rest + 1);
    lo |= low;
    rest ^= low;
  }
  a.merged_lo = lo;
  a.merged_hi = rest;
  const int64_t threads = a.outputs << a.tpo_log2;
  const int64_t blocks = (threads + 255) / 256;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(merge_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

int64_t topk_candidate_capacity(int64_t count, int C) { return topk_blocks(count) * C; }

hipError_t launch_topk(const TopkLaunch& t, hipStream_t stream) {
  if (t.C < 1 || t.C > 64) return hipErrorInvalidValue;
  const int64_t blocks = topk_blocks(t.count);
  if (blocks * t.C > t.cand_capacity) return hipErrorInvalidValue;
  const int64_t chunk = (t.count + blocks - 1) / blocks;
  if (t.t == DType::F64)
    hipLaunchKernelGGL((topk_kernel<double, false>), dim3((unsigned)blocks), dim3(256), 0, stream,
                       static_cast<const double*>(t.bins), nullptr, t.count, chunk, t.C, t.cand_val,
                       t.cand_idx);
  else
    hipLaunchKernelGGL((topk_kernel<float, false>), dim3((unsigned)blocks), dim3(256), 0, stream,
                       static_cast<const float*>(t.bins), nullptr, t.count, chunk, t.C, t.cand_val,
                       t.cand_idx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nc = blocks * t.C;
  hipLaunchKernelGGL((topk_kernel<double, true>), dim3(1), dim3(256), 0, stream,
                     (const double*)t.cand_val, (const uint64_t*)t.cand_idx, nc, nc, t.C, t.out_val,
                     t.out_idx);
  return hipGetLastError();
}

hipError_t launch_refine(const RefineLaunch& r, hipStream_t stream) {
  RefineArgs a;
  a.n_sub = r.n_sub;
  a.K = r.K;
  for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c) {
    a.Ep[c] = r.Ep[c];
    a.ld[c] = r.ld[c];
    a.na[c] = r.na[c];
    a.kc[c] = r.kc[c];
    for (int j = 0; j < CQ_MAX_LOCAL_CUTS; ++j) a.cut[c][j] = r.cut[c][j];
  }
  a.bins = r.bins;
  a.scale = r.scale;
  a.out = r.out;
  if (r.nbins <= 0) return hipSuccess;
  hipLaunchKernelGGL(refine_kernel, dim3((unsigned)r.nbins), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace cq

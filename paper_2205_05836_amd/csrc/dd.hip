// Dynamic definition (Section 4.3, Algorithm 1) device steps:
//  * merge:  sum each subcircuit's entries over its merged outputs, with the
//            zoomed outputs held at their fixed values (FP64);
//  * top-C:  exact selection of the C largest bins by (value desc, index asc);
//  * refine: FP64 value of chosen bins straight from Eq. 1 over the reduced
//            entries, which drives the list update and zoom choice.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "kernels.hpp"
#include "select.hpp"

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


// A group of 2^tpo_log2 lanes sums one reduced entry; lanes stride the merged
// index, then a fixed xor-butterfly combines them (deterministic order).  The
// lanes of a group share their loop trip count, so the butterfly only reads
// active lanes.
__device__ inline void merge_body(const MergeArgs& a) {
  const int64_t total = a.outputs << a.tpo_log2;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += step) {
    const int64_t out = g >> a.tpo_log2;
    const int sub = (int)(g & ((1 << a.tpo_log2) - 1));
    const int64_t row = out >> a.na;
    const uint64_t av = (uint64_t)(out & (((int64_t)1 << a.na) - 1));
    const double* Er = a.E + (row << a.n);
    const uint64_t base = a.fixed_vals_flat | deposit(av, a.active_flat) | deposit((uint64_t)sub, a.merged_lo);
    // next merged index: increment within the bits of merged_hi
    auto next = [&](uint64_t x) { return ((x | ~a.merged_hi) + 1) & a.merged_hi; };
    double acc = 0.0;
    uint64_t d = 0;
    int64_t t = 0;
    for (; t + 4 <= a.iters; t += 4) {  // four loads in flight, added in order
      const uint64_t d1 = next(d), d2 = next(d1), d3 = next(d2);
      const double v0 = Er[base | d], v1 = Er[base | d1], v2 = Er[base | d2], v3 = Er[base | d3];
      acc += v0;
      acc += v1;
      acc += v2;
      acc += v3;
      d = next(d3);
    }
    for (; t < a.iters; ++t) {
      acc += Er[base | d];
      d = next(d);
    }
    for (int s = (1 << a.tpo_log2) >> 1; s >= 1; s >>= 1) acc += __shfl_xor(acc, s);
    if (sub == 0) a.Ep[out] = acc;
  }
}

// blockIdx.y selects the argument block, blockIdx.z the instance
__global__ void __launch_bounds__(256) merge_ind_kernel(const MergeArgs* __restrict__ a, int64_t slot) {
  const MergeArgs m = inst_ptr(a, slot)[blockIdx.y];
  merge_body(m);
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

// Sorts buf[0..n) best-first (n a power of two, 2..kTopS); all threads of
// the workgroup call it with the same n.
__device__ void bitonic_sort(Key* buf, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
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

// count_dev / C_dev, when given, replace count (the chunk then follows the
// grid) and C.  Each workgroup writes out_stride keys, the worst key past its
// survivors.
template <typename T, bool kExplicit>
__global__ void __launch_bounds__(256) topk_kernel(const T* __restrict__ vals,
                                                   const uint64_t* __restrict__ idxs,
                                                   int64_t count, int64_t chunk, int C,
                                                   double* __restrict__ out_v,
                                                   uint64_t* __restrict__ out_i,
                                                   const int64_t* __restrict__ count_dev,
                                                   const int32_t* __restrict__ C_dev,
                                                   int out_stride, int64_t slot) {
  __shared__ Key buf[kTopS];
  __shared__ int cnt;
  __shared__ Key thr;
  vals = inst_ptr(vals, slot);
  idxs = inst_ptr(idxs, slot);
  out_v = inst_ptr(out_v, slot);
  out_i = inst_ptr(out_i, slot);
  count_dev = inst_ptr(count_dev, slot);
  C_dev = inst_ptr(C_dev, slot);
  if (C_dev) C = *C_dev;
  if (C <= 0) return;
  if (count_dev) {
    count = *count_dev;
    chunk = (count + gridDim.x - 1) / gridDim.x;
  }
  const int64_t begin = (int64_t)blockIdx.x * chunk;
  int64_t end = begin + chunk;
  if (end > count) end = count;
  if (threadIdx.x == 0) {
    cnt = 0;
    thr = worst_key();
  }
  __syncthreads();
  // sorts only the filled prefix, rounded up to a power of two: after a
  // selective scan most workgroups hold a handful of keys
  auto trim = [&]() {
    int n = 2;
    while (n < cnt) n <<= 1;
    for (int t = cnt + threadIdx.x; t < n; t += blockDim.x) buf[t] = worst_key();
    __syncthreads();
    bitonic_sort(buf, n);
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
  for (int t = threadIdx.x; t < out_stride; t += blockDim.x) {
    const Key k = (t < cnt) ? buf[t] : worst_key();
    out_v[(int64_t)blockIdx.x * out_stride + t] = k.v;
    out_i[(int64_t)blockIdx.x * out_stride + t] = k.i;
  }
}

// ---------------------------------------------------------------------------
// Top-C pass one over the bins, bandwidth-shaped: every thread streams 16-byte
// vectors (the next round is loaded while the current one is filtered), keys
// in LDS are (value, 32-bit offset in the chunk), and the running threshold
// is the workgroup's C-th best so far, so after the first rounds almost no
// value enters the buffer.  A round is filtered in two halves with a
// capacity check between them, which keeps the buffer from overflowing
// whatever the order of the values.
// ---------------------------------------------------------------------------
template <typename T>
struct CKey {
  T v;
  uint32_t i;
};

template <typename T>
__device__ inline bool cbetter(const CKey<T>& a, const CKey<T>& b) {
  return a.v > b.v || (a.v == b.v && a.i < b.i);
}

template <typename T>
__device__ inline CKey<T> cworst() {
  return CKey<T>{T(-DBL_MAX), 0xffffffffu};
}

template <>
__device__ inline CKey<float> cworst<float>() {
  return CKey<float>{-FLT_MAX, 0xffffffffu};
}

constexpr int kScanS = 4096;  // LDS keys

template <typename T>
__device__ void cbitonic_sort(CKey<T>* buf) {
  for (int k = 2; k <= kScanS; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < kScanS / 2; t += blockDim.x) {
        const int i = 2 * j * (t / j) + (t % j);
        const int p = i + j;
        const bool asc = (i & k) == 0;
        CKey<T> x = buf[i], y = buf[p];
        const bool swap = asc ? cbetter(y, x) : cbetter(x, y);
        if (swap) {
          buf[i] = y;
          buf[p] = x;
        }
      }
      __syncthreads();
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) topk_scan_kernel(const T* __restrict__ vals,
                                                        const int64_t* __restrict__ count_dev,
                                                        const int32_t* __restrict__ C_dev,
                                                        double* __restrict__ out_v,
                                                        uint64_t* __restrict__ out_i,
                                                        int out_stride) {
  constexpr int EPV = 16 / (int)sizeof(T);  // values per 16-byte vector
  constexpr int NV = 4;                     // vectors per thread per round
  constexpr int VPT = EPV * NV;
  constexpr int HALF = 256 * VPT / 2;       // most keys one half-round can add
  static_assert(HALF + 64 <= kScanS, "buffer too small for a half round");
  typedef T V __attribute__((ext_vector_type(EPV)));
  __shared__ CKey<T> buf[kScanS];
  __shared__ int cnt;
  __shared__ CKey<T> thr;
  const int C = *C_dev;
  if (C <= 0) return;
  const int64_t count = *count_dev;
  const int64_t round = 256 * VPT;
  // chunks are whole rounds, so every vector start is a multiple of EPV
  const int64_t per = ((count + gridDim.x - 1) / gridDim.x + round - 1) / round * round;
  const int64_t begin = (int64_t)blockIdx.x * per;
  int64_t end = begin + per;
  if (end > count) end = count;
  if (threadIdx.x == 0) {
    cnt = 0;
    thr = cworst<T>();
  }
  __syncthreads();
  auto trim = [&]() {
    for (int t = cnt + threadIdx.x; t < kScanS; t += blockDim.x) buf[t] = cworst<T>();
    __syncthreads();
    cbitonic_sort(buf);
    if (threadIdx.x == 0) {
      if (cnt > C) cnt = C;
      thr = (cnt == C) ? buf[C - 1] : cworst<T>();
    }
    __syncthreads();
  };
  const bool vec = (reinterpret_cast<uintptr_t>(vals) & 15) == 0;
  auto load = [&](int64_t r0, V (&x)[NV]) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int64_t e0 = r0 + ((int64_t)j * 256 + threadIdx.x) * EPV;
      if (vec && e0 + EPV <= end) {
        x[j] = *reinterpret_cast<const V*>(vals + e0);
      } else {
#pragma unroll
        for (int e = 0; e < EPV; ++e) x[j][e] = (e0 + e < end) ? vals[e0 + e] : T(0);
      }
    }
  };
  V cur[NV], nxt[NV];
  if (begin < end) load(begin, cur);
  for (int64_t r0 = begin; r0 < end; r0 += round) {
    if (r0 + round < end) load(r0 + round, nxt);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const CKey<T> th = thr;
#pragma unroll
      for (int j = h * NV / 2; j < (h + 1) * NV / 2; ++j) {
        const int64_t e0 = r0 + ((int64_t)j * 256 + threadIdx.x) * EPV;
#pragma unroll
        for (int e = 0; e < EPV; ++e) {
          const CKey<T> key{cur[j][e], (uint32_t)(e0 + e - begin)};
          if (e0 + e < end && cbetter(key, th)) {
            const int pos = atomicAdd(&cnt, 1);
            buf[pos] = key;
          }
        }
      }
      __syncthreads();
      if (cnt > kScanS - HALF) trim();
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) cur[j] = nxt[j];
  }
  trim();
  for (int t = threadIdx.x; t < out_stride; t += blockDim.x) {
    const bool ok = t < cnt;
    out_v[(int64_t)blockIdx.x * out_stride + t] = ok ? double(buf[t].v) : -DBL_MAX;
    out_i[(int64_t)blockIdx.x * out_stride + t] = ok ? (uint64_t)begin + buf[t].i : ~(uint64_t)0;
  }
}

int64_t topk_blocks(int64_t count) {
  int64_t b = (count + 8191) / 8192;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return b;
}

// ---------------------------------------------------------------------------
// Refine: one workgroup per bin, threads over the 4^K global labels.
// ---------------------------------------------------------------------------

__device__ inline void refine_body(const RefineArgs& a, double* red) {
  if ((int)blockIdx.x >= a.nbins) return;
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

__global__ void __launch_bounds__(256) refine_ind_kernel(const RefineArgs* __restrict__ a, int64_t slot) {
  __shared__ double red[256];
  refine_body(*inst_ptr(a, slot), red);
}

}  // namespace

hipError_t launch_merge_indirect(const MergeArgs* dev, int count, int64_t max_threads,
                                 hipStream_t stream, InstSpan span) {
  if (count <= 0 || max_threads <= 0 || span.n <= 0) return hipSuccess;
  int64_t b = (max_threads + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(merge_ind_kernel, dim3((unsigned)b, (unsigned)count, (unsigned)span.n), dim3(256), 0,
                     stream, dev, span.stride);
  return hipGetLastError();
}

hipError_t launch_refine_indirect(const RefineArgs* dev, int max_bins, hipStream_t stream, InstSpan span) {
  if (max_bins <= 0 || span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(refine_ind_kernel, dim3((unsigned)max_bins, 1, (unsigned)span.n), dim3(256), 0, stream,
                     dev, span.stride);
  return hipGetLastError();
}

// Second pass for small key sets (count <= kSelCap): one workgroup; each
// thread holds up to 64 keys in registers.  The bound-filter-rank selection
// (sel_bound_top) answers unless more than kSelFastCap keys pass its bound;
// then each wave takes its C best of the narrowed keys by C rounds of a wave
// arg-max and wave 0 merges the four lists the same way.
constexpr int kSelCap = 256 * 64;
constexpr int kSelFastCap = 512;

__device__ inline Key wave_best_key(Key k) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    const Key o{__shfl_xor(k.v, s), (uint64_t)__shfl_xor((long long)k.i, s)};
    if (better(o, k)) k = o;
  }
  return k;
}

template <int KPT>
__global__ void __launch_bounds__(256) select_small_kernel(const double* __restrict__ vals,
                                                           const uint64_t* __restrict__ idxs,
                                                           int64_t count, const int32_t* __restrict__ C_dev,
                                                           double* __restrict__ out_v,
                                                           uint64_t* __restrict__ out_i, int64_t slot) {
  using SK = SelKey<double, uint64_t>;
  __shared__ SelShared<double, uint64_t, 256, kSelFastCap> sel;
  __shared__ SK outk[kDDMaxC];
  __shared__ Key wk[4][kDDMaxC];
  __shared__ int wn[4];
  vals = inst_ptr(vals, slot);
  idxs = inst_ptr(idxs, slot);
  C_dev = inst_ptr(C_dev, slot);
  out_v = inst_ptr(out_v, slot);
  out_i = inst_ptr(out_i, slot);
  const int C = *C_dev;
  if (C <= 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  static_assert(KPT >= 1 && KPT <= 64, "keys per thread");
  Key h[KPT];
  uint64_t live = 0;
  // clamped, unconditional loads: all of a thread's loads are in flight together
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int64_t x = (int64_t)j * 256 + threadIdx.x;
    const int64_t xc = x < count ? x : 0;
    h[j] = Key{vals[xc], idxs[xc]};
  }
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int64_t x = (int64_t)j * 256 + threadIdx.x;
    if (x >= count) h[j] = worst_key();
    if (better(h[j], worst_key())) live |= 1ull << j;
  }
  const Key wkey = worst_key();
  const int found = sel_bound_top<double, uint64_t, KPT, 256, kSelFastCap>(
      sel, live, [&](int j) { return SK{h[j].v, h[j].i}; }, C < 256 ? C : 256, SK{wkey.v, wkey.i},
      outk);
  if (found >= 0) {
    for (int n = threadIdx.x; n < C; n += 256) {
      const SK k = n < found ? outk[n] : SK{wkey.v, wkey.i};
      out_v[n] = k.v;
      out_i[n] = k.i;
    }
    return;
  }
  int got = 0;
  for (int round = 0; round < C; ++round) {
    if (__ballot(live != 0) == 0) break;
    Key best = worst_key();
    int bj = -1;
#pragma unroll
    for (int j = 0; j < KPT; ++j)
      if (((live >> j) & 1) && better(h[j], best)) {
        best = h[j];
        bj = j;
      }
    const Key w = wave_best_key(best);
    if (lane == 0) wk[wave][got] = w;
    if (bj >= 0 && best.i == w.i && best.v == w.v) live &= ~(1ull << bj);
    ++got;
  }
  if (lane == 0) wn[wave] = got;
  __syncthreads();
  if (wave != 0) return;
  Key m[4];
  uint32_t ml = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    m[w] = worst_key();
    if (lane < wn[w]) {
      m[w] = wk[w][lane];
      ml |= 1u << w;
    }
  }
  for (int n = 0; n < C; ++n) {
    Key best = worst_key();
    int bw = -1;
#pragma unroll
    for (int w = 0; w < 4; ++w)
      if (((ml >> w) & 1) && better(m[w], best)) {
        best = m[w];
        bw = w;
      }
    const Key win = wave_best_key(best);
    if (lane == 0) {
      out_v[n] = win.v;
      out_i[n] = win.i;
    }
    if (bw >= 0 && best.i == win.i && best.v == win.v) ml &= ~(1u << bw);
  }
}

// one workgroup selects the C best of `count` <= kSelCap keys; the keys per
// thread follow the count (fewer registers, all loads in flight)
void launch_select_small(const double* vals, const uint64_t* idxs, int64_t count, const int32_t* C_dev,
                         double* out_v, uint64_t* out_i, hipStream_t stream, InstSpan span = InstSpan()) {
  const dim3 grid(1, 1, (unsigned)span.n);
  if (count <= 256 * 4)
    hipLaunchKernelGGL(select_small_kernel<4>, grid, dim3(256), 0, stream, vals, idxs, count, C_dev, out_v,
                       out_i, span.stride);
  else if (count <= 256 * 16)
    hipLaunchKernelGGL(select_small_kernel<16>, grid, dim3(256), 0, stream, vals, idxs, count, C_dev, out_v,
                       out_i, span.stride);
  else
    hipLaunchKernelGGL(select_small_kernel<64>, grid, dim3(256), 0, stream, vals, idxs, count, C_dev, out_v,
                       out_i, span.stride);
}

int64_t topk_indirect_capacity(int64_t max_count, int C_max) {
  return topk_blocks(max_count) * C_max;
}

hipError_t launch_topk_indirect(const void* bins, DType t, const int64_t* count_dev,
                                const int32_t* C_dev, int C_max, int64_t max_count,
                                double* cand_val, uint64_t* cand_idx, int64_t cand_capacity,
                                double* out_val, uint64_t* out_idx, hipStream_t stream) {
  if (C_max < 1 || C_max > kDDMaxC) return hipErrorInvalidValue;
  const int64_t blocks = topk_blocks(max_count);
  if (blocks * C_max > cand_capacity) return hipErrorInvalidValue;
  if (t == DType::F64)
    hipLaunchKernelGGL((topk_scan_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, stream,
                       static_cast<const double*>(bins), count_dev, C_dev, cand_val, cand_idx, C_max);
  else
    hipLaunchKernelGGL((topk_scan_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, stream,
                       static_cast<const float*>(bins), count_dev, C_dev, cand_val, cand_idx, C_max);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nc = blocks * C_max;
  if (nc <= kSelCap)
    launch_select_small((const double*)cand_val, (const uint64_t*)cand_idx, nc, C_dev, out_val, out_idx, stream);
  else
    hipLaunchKernelGGL((topk_kernel<double, true>), dim3(1), dim3(256), 0, stream,
                       (const double*)cand_val, (const uint64_t*)cand_idx, nc, nc, 0, out_val,
                       out_idx, nullptr, C_dev, C_max, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_topk_candidates(const double* cand_val, const uint64_t* cand_idx,
                                  const int64_t* count_dev, const int32_t* C_dev, int C_max,
                                  double* stage_val, uint64_t* stage_idx, double* out_val,
                                  uint64_t* out_idx, hipStream_t stream, InstSpan span) {
  if (C_max < 1 || C_max > kDDMaxC) return hipErrorInvalidValue;
  if (span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL((topk_kernel<double, true>), dim3(kTopcStage, 1, (unsigned)span.n), dim3(256), 0, stream,
                     cand_val, cand_idx, (int64_t)0, (int64_t)0, 0, stage_val, stage_idx, count_dev, C_dev,
                     C_max, span.stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nc = (int64_t)kTopcStage * C_max;  // <= kSelCap
  launch_select_small((const double*)stage_val, (const uint64_t*)stage_idx, nc, C_dev, out_val, out_idx, stream,
                      span);
  return hipGetLastError();
}

// After the warm-up tiles: the C-th best of the keys they appended is a key
// that C keys reach, so the threshold rises to its value; the candidate list
// then restarts (the main pass evaluates those tiles again).  At most
// kDDMaxC tiles append at most kDDMaxC keys each: 16 keys per thread.
__global__ void __launch_bounds__(256) warm_tau_kernel(const double* __restrict__ cand_v,
                                                       unsigned long long* count,
                                                       const int32_t* __restrict__ C_dev,
                                                       unsigned long long* thr, int64_t slot) {
  using SK = SelKey<double, uint32_t>;
  constexpr int KPT = kDDMaxC * kDDMaxC / 256;
  __shared__ SelShared<double, uint32_t, 256, kSelFastCap> sel;
  __shared__ SK outk[kDDMaxC];
  cand_v = inst_ptr(cand_v, slot);
  count = inst_ptr(count, slot);
  C_dev = inst_ptr(C_dev, slot);
  thr = inst_ptr(thr, slot);
  const int C = *C_dev;
  const int64_t n = (int64_t)*count;
  if (C > 0 && n >= C && n <= 256 * KPT) {
    double h[KPT];
    uint64_t live = 0;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int64_t x = (int64_t)j * 256 + threadIdx.x;
      h[j] = cand_v[x < n ? x : 0];
      if (x < n) live |= 1ull << j;
    }
    const int found = sel_bound_top<double, uint32_t, KPT, 256, kSelFastCap>(
        sel, live, [&](int j) { return SK{h[j], (uint32_t)(j * 256 + threadIdx.x)}; }, C,
        SK{-INFINITY, 0xffffffffu}, outk);
    if (threadIdx.x == 0 && found == C) atomicMax(thr, ord_key(outk[C - 1].v));
  }
  __syncthreads();
  if (threadIdx.x == 0) *count = 0;
}

// ---------------------------------------------------------------------------
// Device-driven recursion control.  These kernels run as one wave: they
// handle a few hundred words per recursion, a lane per descriptor, candidate
// or list entry.
// ---------------------------------------------------------------------------
namespace {

__device__ inline int64_t sym_pow(const SymPow& s, const int32_t* na) {
  if (s.zero) return 0;
  int e = s.c0;
  for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c)
    if ((s.mask >> c) & 1u) e += na[c];
  return (int64_t)1 << e;
}

__device__ inline int sym_log(const SymLog& s, const int32_t* na) {
  int e = s.c0;
  for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c)
    if ((s.mask >> c) & 1u) e += na[c];
  return e;
}

// output position i <-> flat bit n-1-i
__device__ inline uint64_t pos_to_flat(uint64_t m, int n) {
  uint64_t f = 0;
  for (int i = 0; i < n; ++i)
    if ((m >> i) & 1) f |= (uint64_t)1 << (n - 1 - i);
  return f;
}

__device__ inline uint64_t low_bits(int k) { return k >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << k) - 1); }

// Merge descriptor: lanes take the lowest tpo merged flat bits, the loop the rest.
__device__ inline void set_merge(MergeArgs& m, const double* E, double* Ep, int64_t rows, int n,
                                 int na, uint64_t active_flat, uint64_t merged_flat,
                                 uint64_t fixed_vals_flat) {
  const int nm = __popcll(merged_flat);
  const int tpo = nm < 6 ? nm : 6;
  uint64_t lo = 0, rest = merged_flat;
  for (int i = 0; i < tpo; ++i) {
    const uint64_t low = rest & (~rest + 1);
    lo |= low;
    rest ^= low;
  }
  m.E = E;
  m.Ep = Ep;
  m.outputs = rows << na;
  m.n = n;
  m.na = na;
  m.tpo_log2 = tpo;
  m.iters = (int64_t)1 << (nm - tpo);
  m.active_flat = active_flat;
  m.merged_lo = lo;
  m.merged_hi = rest;
  m.fixed_vals_flat = fixed_vals_flat;
}

__global__ void dd_init_kernel(const DDProgram* __restrict__ P, DDState* st, cq_dd_record* recs, int R,
                               int64_t slot) {
  P = inst_ptr(P, slot);
  st = inst_ptr(st, slot);
  recs = inst_ptr(recs, slot);
  uint64_t* w = reinterpret_cast<uint64_t*>(recs);
  const int64_t words = (int64_t)R * (int64_t)(sizeof(cq_dd_record) / 8);
  for (int64_t i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0;
  if (threadIdx.x != 0 || P->resume) return;  // a resumed state was copied in before
  const DDInit& init = P->init;
  for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c) {
    st->active[c] = init.active[c];
    st->merged[c] = init.merged[c];
    st->fixed[c] = init.fixed[c];
    st->fixed_vals[c] = init.fixed_vals[c];
    st->na[c] = 0;
  }
  st->n_active = 0;
  st->stop = 0;
  st->done = 0;
  st->n_list = 0;
  st->C = 0;
  st->count = 0;
  st->topc_thr = 0;
  st->topc_count = 0;
  st->n_tiles = 0;
  st->warm_count = 0;
  st->list_count = 0;
  st->zero_idx = 0;
  st->total = 0.0;
}

// One workgroup of 64 threads: every thread derives the active counts (a
// few words), thread c < n_sub writes subcircuit c's descriptors, thread
// 32 + s step s's, and thread 0 the recursion-wide fields -- the descriptor
// writes are independent, so they no longer run one after another.
__global__ void dd_setup_kernel(const DDProgram* __restrict__ P, DDState* st, DDLevel* lv,
                                cq_dd_record* recs, int r, void* bins, int64_t slot) {
  P = inst_ptr(P, slot);
  st = inst_ptr(st, slot);
  lv = inst_ptr(lv, slot);
  recs = inst_ptr(recs, slot);
  bins = inst_ptr(bins, slot);
  const int tid = threadIdx.x;
  const int ns = P->n_sub, nsteps = P->n_steps;
  const int step = tid - 32;  // the step this thread describes, if in range
  // stopped, or past this instance's last recursion of the call: nothing runs
  if (st->stop || P->r0 + r >= P->r_end) {
    if (tid < ns) {
      lv->merge[tid].outputs = 0;
      lv->rowsum[tid].outputs = 0;
      lv->prep[tid].n = 0;
    }
    if (step >= 0 && step < nsteps) {
      lv->gemm[step].tiles = 0;
      lv->perm[step].total = 0;
    }
    if (tid == 0) {
      lv->refine.nbins = 0;
      st->C = 0;
      st->count = 0;
    }
    return;
  }
  int32_t na[CQ_MAX_SUBCIRCUITS];
  int sum = 0;
  bool any_merged = false;
  for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c) na[c] = 0;
  for (int c = 0; c < ns; ++c) {
    na[c] = __popcll(st->active[c]);
    sum += na[c];
    any_merged = any_merged || st->merged[c] != 0;
  }
  const int64_t count = (int64_t)1 << sum;
  const int C = any_merged ? (int)(count < P->C_max ? count : P->C_max) : 0;
  // without stored bins and with nothing to select, the bins are not needed
  const bool skip = P->topc_step >= 0 && C == 0;
  cq_dd_record& rec = recs[r];
  if (tid < ns) {
    const int c = tid;
    const int n = P->n_out[c];
    const uint64_t act = st->active[c], mer = st->merged[c], fv = st->fixed_vals[c];
    st->na[c] = na[c];
    rec.active[c] = act;
    rec.merged[c] = mer;
    rec.fixed[c] = st->fixed[c];
    rec.fixed_vals[c] = fv;
    set_merge(lv->merge[c], P->E[c], P->Ep[c], P->rows[c], n, na[c], pos_to_flat(act, n),
              pos_to_flat(mer, n), pos_to_flat(fv, n));
    // row sums of the reduced entries give the recursion total
    set_merge(lv->rowsum[c], P->Ep[c], P->Rs[c], P->rows[c], na[c], 0, 0, low_bits(na[c]), 0);
    const int t = P->prep_dst[c];
    PrepArgs& pa = lv->prep[c];
    pa.src = P->Ep[c];
    pa.dst = t >= 0 ? P->tensor[t].hi : nullptr;
    pa.dst_lo = t >= 0 ? P->tensor[t].lo : nullptr;
    pa.n = (t >= 0 && !skip) ? sym_pow(P->tensor_elems[t], na) : 0;
    // per-label balance: the reduced entry's rows carry 2^na_c columns
    pa.rexp = P->balance ? P->bal.rexp[c] : nullptr;
    pa.cols_log2 = na[c];
    pa.colmax = P->cscale ? P->colmax[c] : nullptr;
  }
  if (step >= 0 && step < nsteps) {
    const int s = step;
    if (P->step_is_gemm[s]) {
      const DDGemmSym& G = P->gemm[s];
      const DDTensor& ta = P->tensor[G.a];
      const DDTensor& tb = P->tensor[G.b];
      const DDTensor& tc = P->tensor[G.c];
      GemmArgs g;
      const int64_t Z = sym_pow(G.Z, na), M = sym_pow(G.M, na), N = sym_pow(G.N, na);
      const int64_t K = sym_pow(G.K, na);
      g.A = ta.hi;
      g.A_lo = ta.lo;
      g.B = tb.hi;
      g.B_lo = tb.lo;
      g.C = tc.is_out ? bins : tc.hi;
      g.C_lo = tc.is_out ? nullptr : tc.lo;
      g.M = M;
      g.N = N;
      g.K = K;
      g.sAz = sym_pow(G.sAz, na);
      g.sAk = sym_pow(G.sAk, na);
      g.sBz = sym_pow(G.sBz, na);
      g.sBk = sym_pow(G.sBk, na);
      g.sCz = sym_pow(G.sCz, na);
      g.ldc = sym_pow(G.ldc, na);
      g.alpha = G.alpha;
      // column-scaled operands: the GEMM writing the bins adds the exponents back
      const bool scaled = P->cscale && tc.is_out;
      g.rowexp = scaled ? P->rowexp : nullptr;
      g.colexp = scaled ? P->colexp : nullptr;
      g.rowtmax = scaled ? P->rowtmax : nullptr;
      const bool tc_here = s == P->topc_step;
      g.topc_publish_only = 0;
      g.tile_list = tc_here ? P->tile_list : nullptr;
      g.tile_count = tc_here ? &st->list_count : nullptr;
      g.topc_thr = tc_here ? &st->topc_thr : nullptr;
      g.topc_count = tc_here ? &st->topc_count : nullptr;
      g.topc_C = tc_here ? &st->C : nullptr;
      g.topc_v = tc_here ? P->cand_v : nullptr;
      g.topc_i = tc_here ? P->cand_i : nullptr;
      g.tilesM = (M + 127) / 128;
      g.tilesN = (N + 127) / 128;
      g.tiles = skip ? 0 : g.tilesM * g.tilesN * Z;
      const double a_elems = double(g.sAz ? Z : 1) * double(M) * double(K);
      const double b_elems = double(g.sBz ? Z : 1) * double(N) * double(K);
      g.m_fastest = b_elems > a_elems ? 1 : 0;
      lv->gemm[s] = g;
      if (tc_here) {
        // tile pruning: the 64 tiles with the largest bounds append their
        // best keys first and the C-th best of those raises the threshold
        // (the candidate list then restarts); only tiles whose bound reaches
        // it are multiplied
        st->n_tiles = g.tiles;
        st->warm_C = (int)(g.tiles < 64 ? g.tiles : 64);
        st->warm_count = st->warm_C;
        st->list_count = 0;
        GemmArgs w = g;
        w.tile_list = P->warm_i;
        w.tile_count = &st->warm_count;
        w.topc_publish_only = 2;
        lv->topc_warm = w;
      }
    } else {
      const DDPermSym& Q = P->perm[s];
      const DDTensor& ts = P->tensor[Q.src];
      const DDTensor& td = P->tensor[Q.dst];
      PermArgs& p = lv->perm[s];
      p.src = ts.hi;
      p.src_lo = ts.lo;
      p.dst = td.is_out ? bins : td.hi;
      p.dst_lo = td.is_out ? nullptr : td.lo;
      p.naxes = Q.naxes;
      int bits = 0;
      for (int i = 0; i < Q.naxes; ++i) {
        const int l = sym_log(Q.log2[i], na);
        p.log2[i] = l;
        p.sstride[i] = sym_pow(Q.sstride[i], na);
        bits += l;
      }
      p.total = skip ? 0 : (int64_t)1 << bits;
      p.alpha = Q.alpha;
      p.nfac = 0;
    }
  }
  if (tid == 0) {
    rec.recursion = P->r0 + r;
    rec.n_active = sum;
    st->n_active = sum;
    st->count = count;
    st->C = C;
    if (P->topc_step >= 0) {
      st->topc_thr = 0x000fffffffffffffull;  // order-preserving key of -infinity
      st->topc_count = 0;
    }
    RefineArgs& f = lv->refine;
    f.n_sub = ns;
    f.K = P->K;
    for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c) {
      f.Ep[c] = c < ns ? P->Ep[c] : nullptr;
      f.ld[c] = (int64_t)1 << na[c];
      f.na[c] = na[c];
      f.kc[c] = c < ns ? P->kc[c] : 0;
      for (int j = 0; j < CQ_MAX_LOCAL_CUTS; ++j) f.cut[c][j] = P->cut[c][j];
    }
    f.bins = st->top_idx;
    f.nbins = C;
    f.scale = ldexp(1.0, -P->K);
    f.out = st->ref_val;
  }
}

// Order of L: larger FP64 value first, then the earlier recursion, then the
// smaller bin.  Values compare through an order-preserving integer key (with
// -0 taken as +0), which agrees with the numeric order on every non-NaN value
// and still orders NaNs, so ranks of distinct entries are always distinct.
__device__ inline uint64_t list_ord(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v + 0.0);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

__device__ inline bool list_before(uint64_t o1, int r1, uint64_t b1, uint64_t o2, int r2, uint64_t b2) {
  if (o1 != o2) return o1 > o2;
  if (r1 != r2) return r1 < r2;
  return b1 < b2;
}

// The list update of recursion r, one wave: the C candidates (FP64 refined
// values of the selected bins) are ranked among themselves, the best
// min(C, R) of them and the entries of L are ranked against each other (both
// sides are sorted, so an entry's place in the merged list is its own rank
// plus the number of the other side's entries before it), and the best R of
// the union form the new L.  Then the best entry is popped and its bin
// zoomed into: the first max_active[c] merged outputs of each subcircuit
// become active.  Every place of the new list receives exactly one entry.
__global__ void __launch_bounds__(64) dd_update_kernel(const DDProgram* __restrict__ P, DDState* st,
                                                       cq_dd_record* recs, int r, int64_t slot) {
  constexpr int W = (int)(sizeof(DDEntry) / 8);
  static_assert(sizeof(DDEntry) % 8 == 0, "entries copied in 8-byte words");
  static_assert(kDDMaxC <= 64 && CQ_MAX_DD_R <= 64, "one lane per candidate and per entry");
  __shared__ DDEntry old_l[CQ_MAX_DD_R];
  __shared__ DDEntry new_l[CQ_MAX_DD_R];
  __shared__ uint64_t c_ord[kDDMaxC], c_bin[kDDMaxC];
  __shared__ double c_val[kDDMaxC];
  __shared__ int c_rank[kDDMaxC];
  P = inst_ptr(P, slot);
  st = inst_ptr(st, slot);
  recs = inst_ptr(recs, slot);
  const int tid = threadIdx.x;
  if (st->stop || P->r0 + r >= P->r_end) return;
  const int ra = P->r0 + r;  // the recursion's index (the list orders ties by it)
  const int ns = P->n_sub, R = P->R, C = st->C, nl = st->n_list;
  const int take = C < R ? C : R;
  cq_dd_record& rec = recs[r];
  {
    const uint64_t* src = reinterpret_cast<const uint64_t*>(st->list);
    uint64_t* dst = reinterpret_cast<uint64_t*>(old_l);
    for (int w = tid; w < nl * W; w += 64) dst[w] = src[w];
  }
  if (tid < C) {
    c_val[tid] = st->ref_val[tid];
    c_ord[tid] = list_ord(c_val[tid]);
    c_bin[tid] = st->top_idx[tid];
  }
  __syncthreads();
  // candidates among themselves (equal keys keep their selection order)
  if (tid < C) {
    const uint64_t o = c_ord[tid], b = c_bin[tid];
    int rk = 0;
    for (int j = 0; j < C; ++j)
      rk += (c_ord[j] != o ? c_ord[j] > o : (c_bin[j] != b ? c_bin[j] < b : j < tid)) ? 1 : 0;
    c_rank[tid] = rk;
  }
  __syncthreads();
  // an entry of L keeps its rank plus the taken candidates before it
  if (tid < nl) {
    const DDEntry& e = old_l[tid];
    const uint64_t o = list_ord(e.v);
    int pos = tid;
    for (int j = 0; j < C; ++j)
      pos += (c_rank[j] < take && list_before(c_ord[j], ra, c_bin[j], o, e.rec, e.bin)) ? 1 : 0;
    if (pos < R) {
      const uint64_t* src = reinterpret_cast<const uint64_t*>(&e);
      uint64_t* dst = reinterpret_cast<uint64_t*>(&new_l[pos]);
      for (int w = 0; w < W; ++w) dst[w] = src[w];
    }
  }
  // a taken candidate keeps its rank plus the entries of L before it
  if (tid < C && c_rank[tid] < take) {
    const uint64_t o = c_ord[tid], bin = c_bin[tid];
    int pos = c_rank[tid];
    for (int q = 0; q < nl; ++q)
      pos += list_before(list_ord(old_l[q].v), old_l[q].rec, old_l[q].bin, o, ra, bin) ? 1 : 0;
    if (pos < R) {
      DDEntry& e = new_l[pos];
      e.v = c_val[tid];
      e.rec = ra;
      e.pad = 0;
      e.bin = bin;
      // the bin's digits, subcircuit 0 most significant, fix the active
      // outputs: the lowest active position takes the digit's top bit
      int shift = st->n_active;
      for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c) {
        e.fixed[c] = e.fixed_vals[c] = e.merged[c] = 0;
        if (c >= ns) continue;
        const int a = st->na[c];
        shift -= a;
        const uint64_t bits = (bin >> shift) & low_bits(a);
        uint64_t act = st->active[c], fv = st->fixed_vals[c];
        for (int t = a - 1; act; --t) {
          const uint64_t low = act & (~act + 1);
          if ((bits >> t) & 1) fv |= low;
          act ^= low;
        }
        e.fixed[c] = st->fixed[c] | st->active[c];
        e.fixed_vals[c] = fv;
        e.merged[c] = st->merged[c];
      }
    }
  }
  __syncthreads();
  const int nl2 = nl + take < R ? nl + take : R;
  if (tid == 0) {
    rec.total = st->total;
    rec.n_list = nl2;
    if (P->topc_step >= 0) {
      rec.tiles = st->n_tiles;
      rec.tiles_run = st->warm_count + st->list_count;
    }
    st->done = ra + 1;
  }
  if (tid < nl2) {
    rec.list_val[tid] = new_l[tid].v;
    rec.list_rec[tid] = new_l[tid].rec;
    rec.list_bin[tid] = new_l[tid].bin;
  }
  if (nl2 == 0) {
    if (tid == 0) {
      st->n_list = 0;
      st->stop = 1;
    }
    return;
  }
  // pop the best entry and zoom into its bin
  if (tid == 0) rec.popped = 1;
  if (tid < ns) {
    const int c = tid;
    const uint64_t mer = new_l[0].merged[c];
    uint64_t act = 0, rest = mer;
    for (int taken = 0; rest && taken < P->max_active[c]; ++taken) {
      const uint64_t low = rest & (~rest + 1);
      act |= low;
      rest ^= low;
    }
    st->active[c] = act;
    st->merged[c] = mer & ~act;
    st->fixed[c] = new_l[0].fixed[c];
    st->fixed_vals[c] = new_l[0].fixed_vals[c];
  }
  {
    const uint64_t* src = reinterpret_cast<const uint64_t*>(&new_l[1]);
    uint64_t* dst = reinterpret_cast<uint64_t*>(st->list);
    for (int w = tid; w < (nl2 - 1) * W; w += 64) dst[w] = src[w];
  }
  if (tid == 0) st->n_list = nl2 - 1;
}

}  // namespace

// Block b copies `words` 32-bit words from src + b * src_stride to
// dst + b * dst_stride (strides in bytes): programs from the upload area into
// the control blocks, and records out of them into one readback block.
__global__ void __launch_bounds__(256) dd_copy_kernel(const char* __restrict__ src, int64_t src_stride,
                                                      char* __restrict__ dst, int64_t dst_stride,
                                                      int64_t words) {
  const uint32_t* s = reinterpret_cast<const uint32_t*>(src + (int64_t)blockIdx.x * src_stride);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst + (int64_t)blockIdx.x * dst_stride);
  for (int64_t w = threadIdx.x; w < words; w += blockDim.x) d[w] = s[w];
}

hipError_t launch_warm_tau(const double* cand_v, unsigned long long* count, const int32_t* C_dev,
                           unsigned long long* thr, hipStream_t stream, InstSpan span) {
  if (span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(warm_tau_kernel, dim3(1, 1, (unsigned)span.n), dim3(256), 0, stream, cand_v, count, C_dev,
                     thr, span.stride);
  return hipGetLastError();
}

hipError_t launch_dd_copy(const void* src, int64_t src_stride, void* dst, int64_t dst_stride,
                          int64_t bytes, int blocks, hipStream_t stream) {
  if (blocks <= 0 || bytes <= 0) return hipSuccess;
  if ((bytes & 3) || (src_stride & 3) || (dst_stride & 3) || (reinterpret_cast<uintptr_t>(src) & 3) ||
      (reinterpret_cast<uintptr_t>(dst) & 3))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(dd_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                     static_cast<const char*>(src), src_stride, static_cast<char*>(dst), dst_stride,
                     bytes / 4);
  return hipGetLastError();
}

hipError_t launch_dd_init(const DDProgram* prog, DDState* st, cq_dd_record* recs, int R,
                          hipStream_t stream, InstSpan span) {
  if (span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dd_init_kernel, dim3(1, 1, (unsigned)span.n), dim3(256), 0, stream, prog, st, recs, R,
                     span.stride);
  return hipGetLastError();
}

hipError_t launch_dd_setup(const DDProgram* prog, DDState* st, DDLevel* lv, cq_dd_record* recs,
                           int r, void* bins, hipStream_t stream, InstSpan span) {
  if (span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dd_setup_kernel, dim3(1, 1, (unsigned)span.n), dim3(64), 0, stream, prog, st, lv, recs, r,
                     bins, span.stride);
  return hipGetLastError();
}

hipError_t launch_dd_update(const DDProgram* prog, DDState* st, cq_dd_record* recs, int r,
                            hipStream_t stream, InstSpan span) {
  if (span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dd_update_kernel, dim3(1, 1, (unsigned)span.n), dim3(64), 0, stream, prog, st, recs, r,
                     span.stride);
  return hipGetLastError();
}

}  // namespace cq

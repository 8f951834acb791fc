// Finite-shot emulation of subcircuit runs and the chi-square loss of Eq. 3.
//
// A QPU run reports the distribution of `shots` measured bit strings
// (Section 2).  Each row of a probability table is sampled independently and
// every decision is taken in integers, so any implementation of the same
// definition reproduces the counts exactly:
//   * probabilities are quantised to q = floor(clamp(p, 0, 1) * 2^52) and the
//     row's inclusive prefix sums C are exact 64-bit integers;
//   * shot s of row r draws x = word0 + 2^32 word1 of Philox4x32-10 (Salmon,
//     Moraes, Dror and Shaw, SC 2011) with key (seed lo, seed hi) and counter
//     (s lo, s hi, r lo, r hi), takes t = floor(x * T / 2^64) with T = C_last
//     and lands on the first index i with C_i > t.
// Frequencies are count / shots in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.hpp"
#include "kernels.hpp"

namespace cq {

namespace {

constexpr int kBlock = 2048;  // row entries per block
constexpr int kThreads = 256;
constexpr int kPer = kBlock / kThreads;
constexpr int kPad = kPer + 1;          // LDS words per thread run (one pad word)
constexpr int kScanThreads = 1024;      // row scans of block sums and counts
constexpr int kShotsPerThread = 64;
constexpr int kShotsPerGroup = kThreads * kShotsPerThread;
constexpr int kLdsBins = 4096;          // rows with at most this many blocks search and count in LDS
constexpr int kFewShots = 64;           // blocks with at most this many shots resolve in registers

__device__ inline uint64_t quant52(double p) {
  const double c = p > 0.0 ? (p < 1.0 ? p : 1.0) : 0.0;
  return (uint64_t)(c * 0x1p52);
}

// Pass 1: the quantised sum of every block of a row (coalesced), and the
// block's shot counters cleared.
__global__ void __launch_bounds__(kThreads) shots_bsum_kernel(const double* __restrict__ P, int64_t cols,
                                                              int64_t nblk, uint64_t* __restrict__ bend,
                                                              uint32_t* __restrict__ bcnt,
                                                              uint32_t* __restrict__ bfill) {
  const int64_t row = blockIdx.y, blk = blockIdx.x;
  const double* p = P + row * cols + blk * kBlock;
  const int64_t n = cols - blk * kBlock < kBlock ? cols - blk * kBlock : kBlock;
  __shared__ unsigned long long part[kThreads];
  unsigned long long s = 0;
#pragma unroll 4
  for (int e = threadIdx.x; e < n; e += kThreads) s += quant52(__builtin_nontemporal_load(p + e));
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t k = row * nblk + blk;
    bend[k] = part[0];
    bcnt[k] = 0;
    bfill[k] = 0;
  }
}

// Prefix over one row of `n` values (one workgroup per row, thread t owns a
// contiguous run): inclusive in place when `out` is null, else exclusive
// into `out`.
template <typename T>
__device__ inline void row_scan(T* __restrict__ v, T* __restrict__ out, int64_t n) {
  const int64_t per = (n + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  const int64_t b1 = b0 + per < n ? b0 + per : n;
  __shared__ unsigned long long part[kScanThreads];
  unsigned long long s = 0;
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) s += v[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 1; h < kScanThreads; h <<= 1) {
    const unsigned long long add = threadIdx.x >= h ? part[threadIdx.x - h] : 0ull;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  unsigned long long run = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) {
    const T x = v[b];
    if (out) out[b] = (T)run;
    run += x;
    if (!out) v[b] = (T)run;
  }
}

// Pass 2: block sums -> inclusive block ends (C at each block's last entry).
__global__ void __launch_bounds__(kScanThreads) shots_bend_kernel(uint64_t* __restrict__ bend, int64_t nblk) {
  row_scan<uint64_t>(bend + (int64_t)blockIdx.x * nblk, nullptr, nblk);
}

// Philox4x32-10: ten rounds of two 32 x 32 -> 64-bit products of counter
// words 0 and 2 with the round multipliers; the high halves are xor-ed into
// the other words with the key, which advances by the Weyl constants.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Target t of shot s of row `row` (total mass T > 0) and its block: the
// first whose inclusive end exceeds t.
__device__ inline void shot_target(const uint64_t* __restrict__ E, int64_t nblk, uint64_t T, uint64_t seed,
                                   int64_t row, int64_t s, uint64_t& t, uint32_t& blk) {
  uint32_t w[4] = {(uint32_t)s, (uint32_t)((uint64_t)s >> 32), (uint32_t)row, (uint32_t)((uint64_t)row >> 32)};
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t x = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
  t = __umul64hi(x, T);
  uint32_t lo = 0, hi = (uint32_t)nblk - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (E[mid] > t) hi = mid;
    else lo = mid + 1;
  }
  blk = lo;
}

// Pass 3: shots per block.  grid (shot groups, rows); a group takes
// kShotsPerGroup consecutive shots of one row and, for rows of at most
// kLdsBins blocks, searches the block ends and counts its shots in LDS
// before one global add per block hit.  A row of one block needs no
// counting at all.
__global__ void __launch_bounds__(kThreads) shots_count_kernel(const uint64_t* __restrict__ bend, int64_t nblk,
                                                               int64_t shots, uint64_t seed,
                                                               uint32_t* __restrict__ bcnt) {
  __shared__ uint32_t hist[kLdsBins];
  __shared__ uint64_t Es[kLdsBins];
  const int64_t row = blockIdx.y, s0 = (int64_t)blockIdx.x * kShotsPerGroup;
  const uint64_t* E = bend + row * nblk;
  uint32_t* cnt = bcnt + row * nblk;
  const uint64_t T = E[nblk - 1];
  if (T == 0) return;
  if (nblk == 1) {
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[0] = (uint32_t)shots;
    return;
  }
  if (nblk > kLdsBins) {
#pragma unroll 4
    for (int j = 0; j < kShotsPerThread; ++j) {
      const int64_t s = s0 + j * kThreads + threadIdx.x;
      if (s < shots) {
        uint64_t t;
        uint32_t blk;
        shot_target(E, nblk, T, seed, row, s, t, blk);
        atomicAdd(&cnt[blk], 1u);
      }
    }
    return;
  }
  for (int b = threadIdx.x; b < nblk; b += kThreads) {
    hist[b] = 0;
    Es[b] = E[b];
  }
  __syncthreads();
#pragma unroll 4
  for (int j = 0; j < kShotsPerThread; ++j) {
    const int64_t s = s0 + j * kThreads + threadIdx.x;
    if (s < shots) {
      uint64_t t;
      uint32_t blk;
      shot_target(Es, nblk, T, seed, row, s, t, blk);
      atomicAdd(&hist[blk], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nblk; b += kThreads)
    if (hist[b]) atomicAdd(&cnt[b], hist[b]);
}

// Pass 4: exclusive prefix of each row's block counts (bucket offsets).
__global__ void __launch_bounds__(kScanThreads) shots_bptr_kernel(uint32_t* __restrict__ bcnt,
                                                                  uint32_t* __restrict__ bptr, int64_t nblk) {
  const int64_t off = (int64_t)blockIdx.x * nblk;
  row_scan<uint32_t>(bcnt + off, bptr + off, nblk);
}

// Pass 5: every shot's target, relative to its block's first entry, into
// the block's bucket; row r's buckets fill slots [r shots, (r + 1) shots).
// Same groups as pass 3.  For rows counted in LDS the group counts its shots
// per block again, reserves one run of each bucket it hits with one global
// add, and then recomputes every shot and takes the next position of its
// run from LDS, so a group's shots of one bucket land next to each other
// (plain stores, so that L2 merges each run before it goes to HBM).
__global__ void __launch_bounds__(kThreads) shots_scatter_kernel(const uint64_t* __restrict__ bend, int64_t nblk,
                                                                 int64_t shots, uint64_t seed,
                                                                 const uint32_t* __restrict__ bptr,
                                                                 uint32_t* __restrict__ bfill,
                                                                 uint64_t* __restrict__ slots) {
  __shared__ uint32_t hist[kLdsBins];  // group counts, then the next position in each bucket
  __shared__ uint64_t Es[kLdsBins];
  const int64_t row = blockIdx.y, s0 = (int64_t)blockIdx.x * kShotsPerGroup;
  const uint64_t* E = bend + row * nblk;
  const uint32_t* ptr = bptr + row * nblk;
  uint32_t* fill = bfill + row * nblk;
  uint64_t* S = slots + row * shots;
  const uint64_t T = E[nblk - 1];
  if (T == 0) return;
  if (nblk == 1) {
#pragma unroll 4
    for (int j = 0; j < kShotsPerThread; ++j) {
      const int64_t s = s0 + j * kThreads + threadIdx.x;
      if (s < shots) {
        uint64_t t;
        uint32_t blk;
        shot_target(E, 1, T, seed, row, s, t, blk);
        S[s] = t;
      }
    }
    return;
  }
  if (nblk > kLdsBins) {
#pragma unroll 4
    for (int j = 0; j < kShotsPerThread; ++j) {
      const int64_t s = s0 + j * kThreads + threadIdx.x;
      if (s < shots) {
        uint64_t t;
        uint32_t blk;
        shot_target(E, nblk, T, seed, row, s, t, blk);
        const uint32_t pos = ptr[blk] + atomicAdd(&fill[blk], 1u);
        S[pos] = t - (blk ? E[blk - 1] : 0);
      }
    }
    return;
  }
  for (int b = threadIdx.x; b < nblk; b += kThreads) {
    hist[b] = 0;
    Es[b] = E[b];
  }
  __syncthreads();
#pragma unroll 4
  for (int j = 0; j < kShotsPerThread; ++j) {
    const int64_t s = s0 + j * kThreads + threadIdx.x;
    if (s < shots) {
      uint64_t t;
      uint32_t blk;
      shot_target(Es, nblk, T, seed, row, s, t, blk);
      atomicAdd(&hist[blk], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nblk; b += kThreads)
    if (hist[b]) hist[b] = ptr[b] + atomicAdd(&fill[b], hist[b]);
  __syncthreads();
#pragma unroll 4
  for (int j = 0; j < kShotsPerThread; ++j) {
    const int64_t s = s0 + j * kThreads + threadIdx.x;
    if (s < shots) {
      uint64_t t;
      uint32_t blk;
      shot_target(Es, nblk, T, seed, row, s, t, blk);
      const uint32_t pos = atomicAdd(&hist[blk], 1u);
      S[pos] = t - (blk ? Es[blk - 1] : 0);
    }
  }
}

typedef double d2_t __attribute__((ext_vector_type(2)));

// Pass 6, blocks with at most kFewShots shots (the usual case: a few shots
// per block of 2048 outcomes): thread t holds entries t kPer .. t kPer +
// kPer - 1 in registers, the block scan gives its run's offset, and every
// thread tests the block's targets against its run (the first entry whose
// inclusive prefix exceeds the target), counting in registers.  No LDS
// staging of the entries, so many more blocks stay resident than in the LDS
// form below; the counts, hence the frequencies, are the same.  A block
// without shots writes zeros without reading its entries.
__global__ void __launch_bounds__(kThreads) shots_resolve_few_kernel(const double* __restrict__ P, int64_t cols,
                                                                     int64_t nblk, int64_t shots,
                                                                     const uint32_t* __restrict__ bcnt,
                                                                     const uint32_t* __restrict__ bptr,
                                                                     const uint64_t* __restrict__ slots,
                                                                     double* __restrict__ F) {
  __shared__ unsigned long long wtot[kThreads / 64];
  __shared__ uint64_t tg[kFewShots];
  const int64_t row = blockIdx.y, blk = blockIdx.x;
  const int64_t c0 = blk * kBlock;
  const int n = (int)(cols - c0 < kBlock ? cols - c0 : kBlock);
  const int64_t k = row * nblk + blk;
  const uint32_t m = bcnt[k];
  if (m > (uint32_t)kFewShots) return;
  double* f = F + row * cols + c0;
  const int e0 = threadIdx.x * kPer;
  const bool vec = e0 + kPer <= n && ((reinterpret_cast<uintptr_t>(f) | reinterpret_cast<uintptr_t>(P + row * cols + c0)) & 15) == 0;
  if (m == 0) {
    if (vec) {
#pragma unroll
      for (int q = 0; q < kPer / 2; ++q) reinterpret_cast<d2_t*>(f + e0)[q] = d2_t{0.0, 0.0};
    } else {
      for (int e = e0; e < e0 + kPer && e < n; ++e) __builtin_nontemporal_store(0.0, f + e);
    }
    return;
  }
  const double* p = P + row * cols + c0 + e0;
  unsigned long long v[kPer];
  if (vec) {
#pragma unroll
    for (int q = 0; q < kPer / 2; ++q) {
      const d2_t x = reinterpret_cast<const d2_t*>(p)[q];
      v[2 * q] = quant52(x[0]);
      v[2 * q + 1] = quant52(x[1]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < kPer; ++e) v[e] = e0 + e < n ? quant52(p[e]) : 0ull;
  }
  unsigned long long s = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    s += v[e];
    v[e] = s;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) wtot[wid] = x;
  if (threadIdx.x < m) tg[threadIdx.x] = slots[row * shots + bptr[k] + threadIdx.x];
  __syncthreads();
  unsigned long long before = x - s;
  for (int w = 0; w < wid; ++w) before += wtot[w];
  uint32_t c[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) c[e] = 0;
  for (uint32_t j = 0; j < m; ++j) {
    const uint64_t t = tg[j];
    // this run holds the target when before <= t < before + s
    if (t >= before && t - before < s) {
      const uint64_t r = t - before;
      bool found = false;
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const bool here = !found && v[e] > r;
        c[e] += here ? 1u : 0u;
        found = found || here;
      }
    }
  }
  const double ds = (double)shots;
  if (vec) {
#pragma unroll
    for (int q = 0; q < kPer / 2; ++q) {
      const d2_t y = {c[2 * q] ? (double)c[2 * q] / ds : 0.0, c[2 * q + 1] ? (double)c[2 * q + 1] / ds : 0.0};
      reinterpret_cast<d2_t*>(f + e0)[q] = y;
    }
  } else {
#pragma unroll
    for (int e = 0; e < kPer; ++e)
      if (e0 + e < n) __builtin_nontemporal_store(c[e] ? (double)c[e] / ds : 0.0, f + e0 + e);
  }
}

// Pass 6, blocks with many shots: the inclusive prefix of the block's
// quantised entries in LDS, its bucket's shots resolved there by binary
// search (the first entry whose prefix exceeds the shot's target), and
// count / shots written out; a block without shots writes zeros without
// reading its entries.  LDS layout: thread t's run of kPer entries at
// [t kPad, t kPad + kPer).
struct ResolveLds {
  unsigned long long C[kThreads * kPad];
  uint32_t cnt[kBlock];
  unsigned long long wtot[kThreads / 64];
};

__device__ __forceinline__ void resolve_block_lds(ResolveLds& L, const double* __restrict__ P, int64_t cols,
                                                  int64_t nblk, int64_t shots, int64_t k, uint32_t m,
                                                  const uint32_t* __restrict__ bptr,
                                                  const uint64_t* __restrict__ slots, double* __restrict__ F) {
  const int64_t row = k / nblk, blk = k - row * nblk;
  const int64_t c0 = blk * kBlock;
  const int n = (int)(cols - c0 < kBlock ? cols - c0 : kBlock);
  double* f = F + row * cols + c0;
  if (m == 0) {
    for (int e = threadIdx.x; e < n; e += kThreads) __builtin_nontemporal_store(0.0, f + e);
    return;
  }
  const double* p = P + row * cols + c0;
#pragma unroll
  for (int e = threadIdx.x; e < kBlock; e += kThreads) {
    L.C[(e / kPer) * kPad + e % kPer] = e < n ? quant52(__builtin_nontemporal_load(p + e)) : 0ull;
    L.cnt[e] = 0;
  }
  __syncthreads();
  unsigned long long* mine = L.C + threadIdx.x * kPad;
  unsigned long long v[kPer];
  unsigned long long s = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    s += mine[e];
    v[e] = s;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) L.wtot[wid] = x;
  __syncthreads();
  unsigned long long before = x - s;
  for (int w = 0; w < wid; ++w) before += L.wtot[w];
#pragma unroll
  for (int e = 0; e < kPer; ++e) mine[e] = v[e] + before;
  __syncthreads();
  const uint64_t* sl = slots + row * shots + bptr[k];
  for (uint32_t j = threadIdx.x; j < m; j += kThreads) {
    const uint64_t t = __builtin_nontemporal_load(sl + j);
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (L.C[(mid / kPer) * kPad + mid % kPer] > t) hi = mid;
      else lo = mid + 1;
    }
    atomicAdd(&L.cnt[lo], 1u);
  }
  __syncthreads();
  const double ds = (double)shots;
  for (int e = threadIdx.x; e < n; e += kThreads) {
    const uint32_t c = L.cnt[e];
    __builtin_nontemporal_store(c ? (double)c / ds : 0.0, f + e);
  }
  __syncthreads();  // the workgroup's next block reuses the LDS
}

// Every block, one workgroup each (grid (nblk, rows)): for tables with many
// shots per block on average.
__global__ void __launch_bounds__(kThreads) shots_resolve_kernel(const double* __restrict__ P, int64_t cols,
                                                                 int64_t nblk, int64_t shots,
                                                                 const uint32_t* __restrict__ bcnt,
                                                                 const uint32_t* __restrict__ bptr,
                                                                 const uint64_t* __restrict__ slots,
                                                                 double* __restrict__ F) {
  __shared__ ResolveLds L;
  const int64_t k = (int64_t)blockIdx.y * nblk + blockIdx.x;
  resolve_block_lds(L, P, cols, nblk, shots, k, bcnt[k], bptr, slots, F);
}

// Only the blocks with more than kFewShots shots, after
// shots_resolve_few_kernel: each workgroup reads the shot counts of
// kManyChunk blocks (k = row * nblk + blk) at once, lists the heavy ones in
// LDS and resolves them, so a table with few such blocks costs one pass
// over the counts.
constexpr int kManyChunk = 64;
constexpr int64_t kManyGrid = 1 << 20;

__global__ void __launch_bounds__(kThreads) shots_resolve_listed_kernel(const double* __restrict__ P, int64_t cols,
                                                                        int64_t nblk, int64_t total, int64_t shots,
                                                                        const uint32_t* __restrict__ bcnt,
                                                                        const uint32_t* __restrict__ bptr,
                                                                        const uint64_t* __restrict__ slots,
                                                                        double* __restrict__ F) {
  __shared__ ResolveLds L;
  __shared__ uint32_t many[kManyChunk];
  __shared__ uint32_t nmany;
  for (int64_t base = (int64_t)blockIdx.x * kManyChunk; base < total; base += (int64_t)gridDim.x * kManyChunk) {
    if (threadIdx.x == 0) nmany = 0;
    __syncthreads();
    if (threadIdx.x < kManyChunk && base + threadIdx.x < total && bcnt[base + threadIdx.x] > (uint32_t)kFewShots)
      many[atomicAdd(&nmany, 1u)] = threadIdx.x;
    __syncthreads();
    const uint32_t listed = nmany;
    for (uint32_t q = 0; q < listed; ++q) {
      const int64_t k = base + many[q];
      resolve_block_lds(L, P, cols, nblk, shots, k, bcnt[k], bptr, slots, F);
    }
    __syncthreads();  // every thread has read nmany and the list before they change
  }
}

// Eq. 3, terms with a + b = 0 taken as 0: per-block partial sums in a fixed
// order (four strided streams a thread, then a tree), then one block sums
// the partials the same way
constexpr int kChiBlocks = 2048;

__global__ void __launch_bounds__(kThreads) chi2_partial_kernel(const double* __restrict__ a,
                                                                const double* __restrict__ b, int64_t n,
                                                                double* __restrict__ part) {
  __shared__ double sh[kThreads];
  // four strided streams per thread, each summed on its own, then combined
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * step < n; i += 4 * step) {
    double x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = __builtin_nontemporal_load(a + i + u * step);
      y[u] = __builtin_nontemporal_load(b + i + u * step);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double d = x[u] - y[u], t = x[u] + y[u];
      if (t != 0.0) acc[u] += d * d / t;
    }
  }
  for (int u = 0; i < n; i += step, ++u) {
    const double x = a[i], y = b[i], d = x - y, t = x + y;
    if (t != 0.0) acc[u] += d * d / t;
  }
  const double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kThreads) chi2_final_kernel(const double* __restrict__ part, int nparts,
                                                              double* __restrict__ out) {
  __shared__ double sh[kThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

struct ShotsWs {
  int64_t bend = 0, bcnt = 0, bptr = 0, bfill = 0, slots = 0, bytes = 0;
};

cq_status hip_error(hipError_t e, const char* what) {
  return fail(CQ_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t al256(int64_t x) { return (x + 255) / 256 * 256; }

ShotsWs shots_ws(int64_t rows, int64_t cols, int64_t shots) {
  ShotsWs w;
  const int64_t nb = rows * ((cols + kBlock - 1) / kBlock);
  w.bend = 0;
  w.bcnt = al256(nb * 8);
  w.bptr = w.bcnt + al256(nb * 4);
  w.bfill = w.bptr + al256(nb * 4);
  w.slots = w.bfill + al256(nb * 4);
  w.bytes = w.slots + al256(rows * shots * 8);
  return w;
}

cq_status shots_check(int64_t rows, int64_t cols, int64_t shots) {
  if (rows < 1 || cols < 1 || shots < 1) return fail(CQ_ERR_ARG, "rows, cols and shots must be positive");
  if (rows > 65535) return fail(CQ_ERR_SHAPE, "more than 65535 rows");
  if (cols > ((int64_t)1 << 34) / rows) return fail(CQ_ERR_SHAPE, "table larger than 2^34 entries");
  if (shots > 0xffffffffLL) return fail(CQ_ERR_SHAPE, "2^32 or more shots per row");
  if (shots > ((int64_t)1 << 34) / rows) return fail(CQ_ERR_SHAPE, "more than 2^34 shots in total");
  return CQ_OK;
}

}  // namespace

}  // namespace cq

using namespace cq;

extern "C" cq_status cq_sample_shots_workspace_size(int64_t rows, int64_t cols, int64_t shots, size_t* bytes) {
  if (!bytes) return fail(CQ_ERR_ARG, "null argument");
  cq_status st = shots_check(rows, cols, shots);
  if (st != CQ_OK) return st;
  *bytes = (size_t)shots_ws(rows, cols, shots).bytes;
  return CQ_OK;
}

extern "C" cq_status cq_sample_shots(const double* probs, int64_t rows, int64_t cols, int64_t shots, uint64_t seed,
                                     double* freqs, void* workspace, size_t workspace_bytes,
                                     hipStream_t stream) {
  if (!probs || !freqs) return fail(CQ_ERR_ARG, "null argument");
  cq_status st = shots_check(rows, cols, shots);
  if (st != CQ_OK) return st;
  const ShotsWs w = shots_ws(rows, cols, shots);
  if (!workspace || (int64_t)workspace_bytes < w.bytes) return fail(CQ_ERR_WORKSPACE, "workspace too small");
  char* ws = static_cast<char*>(workspace);
  uint64_t* bend = reinterpret_cast<uint64_t*>(ws + w.bend);
  uint32_t* bcnt = reinterpret_cast<uint32_t*>(ws + w.bcnt);
  uint32_t* bptr = reinterpret_cast<uint32_t*>(ws + w.bptr);
  uint32_t* bfill = reinterpret_cast<uint32_t*>(ws + w.bfill);
  uint64_t* slots = reinterpret_cast<uint64_t*>(ws + w.slots);
  const int64_t nblk = (cols + kBlock - 1) / kBlock;  // <= 2^23 by the limits
  const dim3 gt((unsigned)nblk, (unsigned)rows);
  const dim3 gs((unsigned)((shots + kShotsPerGroup - 1) / kShotsPerGroup), (unsigned)rows);
  hipLaunchKernelGGL(shots_bsum_kernel, gt, dim3(kThreads), 0, stream, probs, cols, nblk, bend, bcnt, bfill);
  hipLaunchKernelGGL(shots_bend_kernel, dim3((unsigned)rows), dim3(kScanThreads), 0, stream, bend, nblk);
  hipLaunchKernelGGL(shots_count_kernel, gs, dim3(kThreads), 0, stream, (const uint64_t*)bend, nblk, shots, seed,
                     bcnt);
  hipLaunchKernelGGL(shots_bptr_kernel, dim3((unsigned)rows), dim3(kScanThreads), 0, stream, bcnt, bptr, nblk);
  hipLaunchKernelGGL(shots_scatter_kernel, gs, dim3(kThreads), 0, stream, (const uint64_t*)bend, nblk, shots,
                     seed, (const uint32_t*)bptr, bfill, slots);
  if (shots >= (int64_t)kFewShots * nblk) {
    // many shots per block on average: every block resolves in LDS
    hipLaunchKernelGGL(shots_resolve_kernel, gt, dim3(kThreads), 0, stream, probs, cols, nblk, shots,
                       (const uint32_t*)bcnt, (const uint32_t*)bptr, (const uint64_t*)slots, freqs);
  } else {
    hipLaunchKernelGGL(shots_resolve_few_kernel, gt, dim3(kThreads), 0, stream, probs, cols, nblk, shots,
                       (const uint32_t*)bcnt, (const uint32_t*)bptr, (const uint64_t*)slots, freqs);
    if (shots > kFewShots) {
      const int64_t total = rows * nblk, chunks = (total + kManyChunk - 1) / kManyChunk;
      const unsigned grid = (unsigned)(chunks < kManyGrid ? chunks : kManyGrid);
      hipLaunchKernelGGL(shots_resolve_listed_kernel, dim3(grid), dim3(kThreads), 0, stream, probs, cols, nblk,
                         total, shots, (const uint32_t*)bcnt, (const uint32_t*)bptr, (const uint64_t*)slots, freqs);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "shot sampling launch");
  return CQ_OK;
}

extern "C" cq_status cq_chi2_workspace_size(size_t* bytes) {
  if (!bytes) return fail(CQ_ERR_ARG, "null argument");
  *bytes = (size_t)kChiBlocks * sizeof(double);
  return CQ_OK;
}

extern "C" cq_status cq_chi2(const double* a, const double* b, int64_t n, double* result, void* workspace,
                             size_t workspace_bytes, hipStream_t stream) {
  if (!a || !b || !result) return fail(CQ_ERR_ARG, "null argument");
  if (n < 1) return fail(CQ_ERR_ARG, "n must be positive");
  if (!workspace || workspace_bytes < (size_t)kChiBlocks * sizeof(double))
    return fail(CQ_ERR_WORKSPACE, "workspace too small");
  double* part = static_cast<double*>(workspace);
  hipLaunchKernelGGL(chi2_partial_kernel, dim3(kChiBlocks), dim3(kThreads), 0, stream, a, b, n, part);
  hipLaunchKernelGGL(chi2_final_kernel, dim3(1), dim3(kThreads), 0, stream, (const double*)part, kChiBlocks, result);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "chi-square launch");
  return CQ_OK;
}

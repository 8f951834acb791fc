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

constexpr int kBlock = 4096;  // elements per prefix-sum block
constexpr int kThreads = 256;

__device__ inline uint64_t quant52(double p) {
  const double c = p > 0.0 ? (p < 1.0 ? p : 1.0) : 0.0;
  return (uint64_t)(c * 0x1p52);
}

// q of every element, and each block's sum
__global__ void __launch_bounds__(kThreads) shots_quant_kernel(const double* __restrict__ P, int64_t cols,
                                                               int64_t nblk, uint64_t* __restrict__ cdf,
                                                               uint64_t* __restrict__ bsum) {
  const int64_t row = blockIdx.y, blk = blockIdx.x;
  const int64_t c0 = blk * kBlock;
  __shared__ unsigned long long part[kThreads];
  unsigned long long s = 0;
  for (int e = threadIdx.x; e < kBlock; e += kThreads) {
    const int64_t c = c0 + e;
    if (c < cols) {
      const uint64_t q = quant52(P[row * cols + c]);
      cdf[row * cols + c] = q;
      s += q;
    }
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[row * nblk + blk] = part[0];
}

// exclusive prefix of one row's block sums: one workgroup per row, thread t
// owns a contiguous run of blocks
__global__ void __launch_bounds__(kThreads) shots_block_scan_kernel(uint64_t* __restrict__ bsum, int64_t nblk) {
  uint64_t* B = bsum + (int64_t)blockIdx.x * nblk;
  const int64_t per = (nblk + kThreads - 1) / kThreads;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  const int64_t b1 = b0 + per < nblk ? b0 + per : nblk;
  __shared__ unsigned long long part[kThreads];
  unsigned long long s = 0;
  for (int64_t b = b0; b < b1; ++b) s += B[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 1; h < kThreads; h <<= 1) {
    const unsigned long long add = threadIdx.x >= h ? part[threadIdx.x - h] : 0ull;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  unsigned long long run = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
  for (int64_t b = b0; b < b1; ++b) {
    const uint64_t v = B[b];
    B[b] = run;
    run += v;
  }
}

// inclusive prefix inside each block plus the block's offset: thread t owns
// kBlock / kThreads consecutive elements
__global__ void __launch_bounds__(kThreads) shots_cdf_kernel(int64_t cols, int64_t nblk,
                                                             uint64_t* __restrict__ cdf,
                                                             const uint64_t* __restrict__ boff) {
  constexpr int PER = kBlock / kThreads;
  const int64_t row = blockIdx.y, blk = blockIdx.x;
  const int64_t c0 = blk * kBlock + (int64_t)threadIdx.x * PER;
  __shared__ unsigned long long part[kThreads];
  unsigned long long loc[PER];
  unsigned long long s = 0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t c = c0 + e;
    s += c < cols ? cdf[row * cols + c] : 0ull;
    loc[e] = s;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  // inclusive scan of the threads' totals (Hillis-Steele)
  for (int h = 1; h < kThreads; h <<= 1) {
    const unsigned long long add = threadIdx.x >= h ? part[threadIdx.x - h] : 0ull;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  const unsigned long long before = (threadIdx.x ? part[threadIdx.x - 1] : 0ull) + boff[row * nblk + blk];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t c = c0 + e;
    if (c < cols) cdf[row * cols + c] = before + loc[e];
  }
}

__global__ void shots_zero_kernel(uint32_t* __restrict__ counts, int64_t n) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) counts[i] = 0;
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

// one thread per (row, shot)
__global__ void __launch_bounds__(kThreads) shots_sample_kernel(const uint64_t* __restrict__ cdf, int64_t rows,
                                                                int64_t cols, int64_t shots, uint64_t seed,
                                                                uint32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * shots) return;
  const int64_t row = i / shots, s = i - row * shots;
  const uint64_t* C = cdf + row * cols;
  const uint64_t T = C[cols - 1];
  if (T == 0) return;
  uint32_t w[4] = {(uint32_t)s, (uint32_t)((uint64_t)s >> 32), (uint32_t)row, (uint32_t)((uint64_t)row >> 32)};
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t x = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
  const uint64_t t = __umul64hi(x, T);
  // first index with C > t
  int64_t lo = 0, hi = cols - 1;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (C[mid] > t) hi = mid;
    else lo = mid + 1;
  }
  atomicAdd(&counts[row * cols + lo], 1u);
}

__global__ void shots_freq_kernel(const uint32_t* __restrict__ counts, int64_t n, double shots,
                                  double* __restrict__ out) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
    out[i] = (double)counts[i] / shots;
}

// Eq. 3, terms with a + b = 0 taken as 0: per-block partial sums in a fixed
// tree order, then one block sums the partials the same way
constexpr int kChiBlocks = 1024;

__global__ void __launch_bounds__(kThreads) chi2_partial_kernel(const double* __restrict__ a,
                                                                const double* __restrict__ b, int64_t n,
                                                                double* __restrict__ part) {
  __shared__ double sh[kThreads];
  double s = 0.0;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    const double x = a[i], y = b[i], d = x - y, t = x + y;
    if (t != 0.0) s += d * d / t;
  }
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
  int64_t cdf = 0, bsum = 0, counts = 0, bytes = 0;
};

cq_status hip_error(hipError_t e, const char* what) {
  return fail(CQ_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t al256(int64_t x) { return (x + 255) / 256 * 256; }

ShotsWs shots_ws(int64_t rows, int64_t cols) {
  ShotsWs w;
  const int64_t nblk = (cols + kBlock - 1) / kBlock;
  w.cdf = 0;
  w.bsum = al256(rows * cols * 8);
  w.counts = w.bsum + al256(rows * nblk * 8);
  w.bytes = w.counts + al256(rows * cols * 4);
  return w;
}

cq_status shots_check(int64_t rows, int64_t cols, int64_t shots) {
  if (rows < 1 || cols < 1 || shots < 1) return fail(CQ_ERR_ARG, "rows, cols and shots must be positive");
  if (rows > 65535) return fail(CQ_ERR_SHAPE, "more than 65535 rows");
  if (cols > ((int64_t)1 << 34) / rows) return fail(CQ_ERR_SHAPE, "table larger than 2^34 entries");
  if (shots > ((int64_t)1 << 40) / rows) return fail(CQ_ERR_SHAPE, "more than 2^40 shots in total");
  return CQ_OK;
}

}  // namespace

}  // namespace cq

using namespace cq;

extern "C" cq_status cq_sample_shots_workspace_size(int64_t rows, int64_t cols, int64_t shots, size_t* bytes) {
  if (!bytes) return fail(CQ_ERR_ARG, "null argument");
  cq_status st = shots_check(rows, cols, shots);
  if (st != CQ_OK) return st;
  *bytes = (size_t)shots_ws(rows, cols).bytes;
  return CQ_OK;
}

extern "C" cq_status cq_sample_shots(const double* probs, int64_t rows, int64_t cols, int64_t shots, uint64_t seed,
                                     double* freqs, void* workspace, size_t workspace_bytes,
                                     hipStream_t stream) {
  if (!probs || !freqs) return fail(CQ_ERR_ARG, "null argument");
  cq_status st = shots_check(rows, cols, shots);
  if (st != CQ_OK) return st;
  const ShotsWs w = shots_ws(rows, cols);
  if (!workspace || (int64_t)workspace_bytes < w.bytes) return fail(CQ_ERR_WORKSPACE, "workspace too small");
  char* ws = static_cast<char*>(workspace);
  uint64_t* cdf = reinterpret_cast<uint64_t*>(ws + w.cdf);
  uint64_t* bsum = reinterpret_cast<uint64_t*>(ws + w.bsum);
  uint32_t* counts = reinterpret_cast<uint32_t*>(ws + w.counts);
  const int64_t nblk = (cols + kBlock - 1) / kBlock;
  if (nblk > 0x7fffffffLL) return fail(CQ_ERR_SHAPE, "too many columns");
  const dim3 gq((unsigned)nblk, (unsigned)rows);
  hipLaunchKernelGGL(shots_quant_kernel, gq, dim3(kThreads), 0, stream, probs, cols, nblk, cdf, bsum);
  hipLaunchKernelGGL(shots_block_scan_kernel, dim3((unsigned)rows), dim3(kThreads), 0, stream, bsum, nblk);
  hipLaunchKernelGGL(shots_cdf_kernel, gq, dim3(kThreads), 0, stream, cols, nblk, cdf, (const uint64_t*)bsum);
  const int64_t n = rows * cols;
  const unsigned gz = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 65536);
  hipLaunchKernelGGL(shots_zero_kernel, dim3(gz), dim3(kThreads), 0, stream, counts, n);
  const int64_t total = rows * shots;
  const int64_t gs = (total + kThreads - 1) / kThreads;
  if (gs > 0x7fffffffLL) return fail(CQ_ERR_SHAPE, "too many shots");
  hipLaunchKernelGGL(shots_sample_kernel, dim3((unsigned)gs), dim3(kThreads), 0, stream, (const uint64_t*)cdf,
                     rows, cols, shots, seed, counts);
  hipLaunchKernelGGL(shots_freq_kernel, dim3(gz), dim3(kThreads), 0, stream, (const uint32_t*)counts, n,
                     (double)shots, freqs);
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

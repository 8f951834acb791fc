// Layout permutes and entry attribution.
#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.hpp"

namespace cq {

namespace {

// Element kinds of a permute's source and destination.
enum Kind { kF64 = 0, kF32 = 1, kBF16 = 2, kF16 = 3 };


__device__ inline float h16_to_f(uint16_t x, bool f16) {
  return f16 ? float(__builtin_bit_cast(_Float16, x)) : float(__builtin_bit_cast(__bf16, x));
}
__device__ inline uint16_t f_to_h16(float x, bool f16) {
  return f16 ? __builtin_bit_cast(uint16_t, _Float16(x)) : __builtin_bit_cast(uint16_t, __bf16(x));
}

// Binary exponent e of a column maximum m = f * 2^e, f in [0.5, 1) (0 for 0).
__device__ inline int colmax_exp(uint64_t bits) {
  const int be = (int)((bits >> 52) & 0x7ff);
  return be == 0 ? 0 : be - 1022;
}

__device__ inline int fac_exp(const PermArgs& p, int64_t off) {
  int e = 0;
  for (int c = 0; c < p.nfac; ++c)
    e += colmax_exp(p.colmax[c][(off >> p.fac_shift[c]) & ((1ll << p.fac_bits[c]) - 1)]);
  return e;
}

// Generic axis permutation with conversion: one destination element per
// thread iteration, destination written contiguously.  16-bit planes are
// copied bit for bit when both sides use them.
template <int SK, int DK>
__device__ inline void permute_body(const PermArgs& p) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.total; i += step) {
    int64_t r = i, off = 0;
    for (int a = p.naxes - 1; a >= 0; --a) {
      const int l = p.log2[a];
      off += (r & (((int64_t)1 << l) - 1)) * p.sstride[a];
      r >>= l;
    }
    if constexpr (SK >= kBF16 && DK == SK) {
      static_cast<uint16_t*>(p.dst)[i] = static_cast<const uint16_t*>(p.src)[off];
      if (p.dst_lo) static_cast<uint16_t*>(p.dst_lo)[i] = static_cast<const uint16_t*>(p.src_lo)[off];
    } else {
      double v;
      if constexpr (SK == kF64) v = static_cast<const double*>(p.src)[off];
      else if constexpr (SK == kF32) v = static_cast<const float*>(p.src)[off];
      else {
        v = h16_to_f(static_cast<const uint16_t*>(p.src)[off], SK == kF16);
        if (p.src_lo) v += h16_to_f(static_cast<const uint16_t*>(p.src_lo)[off], SK == kF16);
      }
      v *= p.alpha;
      if (p.nfac) v = ldexp(v, fac_exp(p, off));
      if constexpr (DK == kF64) static_cast<double*>(p.dst)[i] = v;
      else if constexpr (DK == kF32) static_cast<float*>(p.dst)[i] = float(v);
      else {
        const float x = float(v);
        const uint16_t h = f_to_h16(x, DK == kF16);
        static_cast<uint16_t*>(p.dst)[i] = h;
        if (p.dst_lo) static_cast<uint16_t*>(p.dst_lo)[i] = f_to_h16(x - h16_to_f(h, DK == kF16), DK == kF16);
      }
    }
  }
}

template <int SK, int DK>
__global__ void __launch_bounds__(256) permute_kernel(PermArgs p) {
  permute_body<SK, DK>(p);
}

// blockIdx.z selects the instance
template <int SK, int DK>
__global__ void __launch_bounds__(256) permute_ind_kernel(const PermArgs* __restrict__ p, int64_t slot) {
  permute_body<SK, DK>(*inst_ptr(p, slot));
}

// FP64 -> FP32 or 16-bit planes (hi = rn16(x), lo = rn16(x - hi)); with
// rexp, row i >> cols_log2 is first scaled by its power of two.
template <int DK>
__device__ inline void prep_body(const double* __restrict__ src, void* dst, void* dst_lo, int64_t n,
                                 const int32_t* __restrict__ rexp = nullptr, int cols_log2 = 0,
                                 const uint64_t* __restrict__ colmax = nullptr) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const int64_t cmask = ((int64_t)1 << cols_log2) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    // column scaling as prep_scaled_kernel: 2^-e of the column maximum, plus the row exponent
    const float x = colmax ? float(ldexp(src[i], -colmax_exp(colmax[i & cmask]) +
                                                     (rexp ? rexp[i >> cols_log2] : 0)))
                           : rexp ? float(ldexp(src[i], rexp[i >> cols_log2])) : float(src[i]);
    if constexpr (DK == kF32) {
      static_cast<float*>(dst)[i] = x;
    } else {
      const uint16_t h = f_to_h16(x, DK == kF16);
      static_cast<uint16_t*>(dst)[i] = h;
      if (dst_lo) static_cast<uint16_t*>(dst_lo)[i] = f_to_h16(x - h16_to_f(h, DK == kF16), DK == kF16);
    }
  }
}

// Four elements a thread: two 16-byte loads, 8-byte (16-bit planes) or
// 16-byte (FP32) stores; the per-element arithmetic is prep_body's.  Needs
// n % 4 == 0, src 16-byte aligned, dst (and dst_lo) aligned to the stores,
// and rows of at least 4 elements when rexp is given.
template <int DK>
__device__ inline void prep_body4(const double* __restrict__ src, void* dst, void* dst_lo, int64_t n,
                                  const int32_t* __restrict__ rexp, int cols_log2) {
  typedef double d2_t __attribute__((ext_vector_type(2)));
  typedef float f4_t __attribute__((ext_vector_type(4)));
  typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
  const int64_t n4 = n >> 2;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += step) {
    const d2_t v0 = reinterpret_cast<const d2_t*>(src)[2 * i];
    const d2_t v1 = reinterpret_cast<const d2_t*>(src)[2 * i + 1];
    const double d[4] = {v0[0], v0[1], v1[0], v1[1]};
    const int e = rexp ? rexp[(4 * i) >> cols_log2] : 0;
    float x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = rexp ? float(ldexp(d[u], e)) : float(d[u]);
    if constexpr (DK == kF32) {
      reinterpret_cast<f4_t*>(dst)[i] = f4_t{x[0], x[1], x[2], x[3]};
    } else {
      u16x4 h, l;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        h[u] = f_to_h16(x[u], DK == kF16);
        l[u] = f_to_h16(x[u] - h16_to_f(h[u], DK == kF16), DK == kF16);
      }
      reinterpret_cast<u16x4*>(dst)[i] = h;
      if (dst_lo) reinterpret_cast<u16x4*>(dst_lo)[i] = l;
    }
  }
}

template <int DK, bool V4>
__global__ void __launch_bounds__(256) prep_kernel(const double* __restrict__ src, void* dst,
                                                   void* dst_lo, int64_t n,
                                                   const int32_t* __restrict__ rexp, int cols_log2) {
  if constexpr (V4) prep_body4<DK>(src, dst, dst_lo, n, rexp, cols_log2);
  else prep_body<DK>(src, dst, dst_lo, n, rexp, cols_log2);
}

// blockIdx.y selects the argument block, blockIdx.z the instance
template <int DK>
__global__ void __launch_bounds__(256) prep_ind_kernel(const PrepArgs* __restrict__ a, int64_t slot) {
  const PrepArgs p = inst_ptr(a, slot)[blockIdx.y];
  prep_body<DK>(p.src, p.dst, p.dst_lo, p.n, p.rexp, p.cols_log2, p.colmax);
}

// Column maxima of |E| (rows x 2^cols_log2, FP64): each thread folds a run of
// rows of one column, then one atomic max per thread.
__global__ void __launch_bounds__(256) colmax_kernel(const double* __restrict__ E, int64_t rows,
                                                     int cols_log2, int rows_per_thread,
                                                     uint64_t* colmax, const int32_t* __restrict__ rexp) {
  const int64_t cols = (int64_t)1 << cols_log2;
  const int64_t chunks = (rows + rows_per_thread - 1) / rows_per_thread;
  const int64_t total = chunks * cols;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += step) {
    const int64_t col = t & (cols - 1), r0 = (t >> cols_log2) * rows_per_thread;
    int64_t r1 = r0 + rows_per_thread;
    if (r1 > rows) r1 = rows;
    double m = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double x = E[(r << cols_log2) + col];
      m = fmax(m, fabs(rexp ? ldexp(x, rexp[r]) : x));
    }
    atomicMax(reinterpret_cast<unsigned long long*>(colmax + col),
              (unsigned long long)__double_as_longlong(m));
  }
}

// max_b |E[l][b]| per row: one wave per row (rows strided over the grid's
// waves), the wave's lanes striding the columns.
__global__ void __launch_bounds__(256) rowmax_kernel(const double* __restrict__ E, int64_t rows,
                                                     int cols_log2, uint64_t* rowmax) {
  const int64_t cols = (int64_t)1 << cols_log2;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wave; r < rows; r += waves) {
    const double* row = E + (r << cols_log2);
    double m = 0.0;
    for (int64_t c = lane; c < cols; c += 64) m = fmax(m, fabs(row[c]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) rowmax[r] = (uint64_t)__double_as_longlong(m);
  }
}

// Binary exponent of a positive finite x (x = f * 2^e, f in [1, 2)).
__device__ inline int bexp(double x) { return ilogb(x); }

__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ inline int wave_max_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// One workgroup: per (subcircuit, digit position, digit) the largest row
// maximum (LDS), then e_j(d) per cut and digit, then every row's exponent.
// The largest row of a subcircuit sits at each digit's maximum over the other
// positions, so the exponents carry an offset per subcircuit (the same for
// all its rows); a final constant per subcircuit, summing to zero over the
// subcircuits (every term of Eq. 1 takes one row of each), brings every
// subcircuit's largest scaled row to their common mean binary exponent.
// Row maxima are FP64 bit patterns of values >= 0, so their unsigned order is
// the value order.  Thread t reads rows l = 1024 i + t: the digits held in the
// low 10 bits of l (the last five positions) are fixed per thread, so one
// running maximum serves them, and their share of a row's exponent is one
// number per thread; the digits above come from i, the same for the whole
// workgroup, and each thread keeps a maximum per (position, digit) for those.
// A handful of LDS atomics per thread remain (a contended atomic per row and
// position took over a millisecond for 4^8 rows), and four rows are loaded
// before any is used.
constexpr int kBalanceRounds = 4;
constexpr int kBalThreads = 1024;
constexpr int kBalLog = 10;            // log2 kBalThreads
constexpr int kBalFixed = kBalLog / 2;  // digit positions fixed per thread
constexpr int kBalUnroll = 4;

__device__ __forceinline__ void balance_body(const BalanceLaunch& b) {
  constexpr int kHi = CQ_MAX_LOCAL_CUTS > kBalFixed ? CQ_MAX_LOCAL_CUTS - kBalFixed : 1;
  __shared__ unsigned long long pmax[CQ_MAX_SUBCIRCUITS][CQ_MAX_LOCAL_CUTS][4];
  __shared__ int ej[CQ_MAX_CUTS][4];
  __shared__ int stp[CQ_MAX_CUTS][4];
  __shared__ int smax[CQ_MAX_SUBCIRCUITS];
  __shared__ int goff[CQ_MAX_SUBCIRCUITS];
  __shared__ int changed;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  for (int i = tid; i < CQ_MAX_CUTS * 4; i += blockDim.x) (&ej[0][0])[i] = 0;
  if (tid < CQ_MAX_SUBCIRCUITS) smax[tid] = INT_MIN;
  // exponent share of position p (digit d) in a row of subcircuit c
  auto share = [&](int c, int p, int d) {
    const int j = b.cut_of[c][p];
    return b.up[j] == c ? ej[j][d] : -ej[j][d];
  };
  // the positions fixed by tid, and those taken from i
  auto share_lo = [&](int c, int k, int nhi) {
    int e = 0;
    for (int p = nhi; p < k; ++p) e += share(c, p, (tid >> (2 * (k - 1 - p))) & 3);
    return e;
  };
  auto share_hi = [&](int c, int nhi, int64_t i) {
    int e = 0;
    for (int q = 0; q < nhi; ++q) e += share(c, q, (int)((i >> (2 * (nhi - 1 - q))) & 3));
    return e;
  };
  // Each round measures the per-digit maxima of the rows as scaled by the
  // current exponents and moves every cut's pair of exponents to meet them.
  // In a subcircuit with many cuts the largest row with digit d at one
  // position is decided by the other positions' extreme digits (one row out
  // of 4^(k-1) when the labels are far apart), so a single round leaves much
  // of the spread; a few rounds remove it.
  __syncthreads();
  for (int round = 0; round < kBalanceRounds; ++round) {
    for (int i = tid; i < CQ_MAX_SUBCIRCUITS * CQ_MAX_LOCAL_CUTS * 4; i += blockDim.x)
      (&pmax[0][0][0])[i] = 0ull;
    if (tid == 0) changed = 0;
    __syncthreads();
    for (int c = 0; c < b.n_sub; ++c) {
      const int k = b.k[c];
      const int64_t rows = (int64_t)1 << (2 * k);
      const int64_t iters = (rows + kBalThreads - 1) >> kBalLog;
      const int nhi = k > kBalFixed ? k - kBalFixed : 0;  // positions 0..nhi-1 take their digit from i
      const int elo = share_lo(c, k, nhi);
      unsigned long long tm = 0ull;
      unsigned long long hm[kHi][4];
#pragma unroll
      for (int q = 0; q < kHi; ++q)
#pragma unroll
        for (int d = 0; d < 4; ++d) hm[q][d] = 0ull;
      for (int64_t i0 = 0; i0 < iters; i0 += kBalUnroll) {
        unsigned long long v[kBalUnroll];
#pragma unroll
        for (int u = 0; u < kBalUnroll; ++u) {
          const int64_t l = ((i0 + u) << kBalLog) + tid;
          v[u] = ((i0 + u < iters) & (l < rows)) ? b.rowmax[c][l] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kBalUnroll; ++u) {
          const int64_t i = i0 + u;
          unsigned long long x = v[u];
          if (x)
            x = (unsigned long long)__double_as_longlong(
                ldexp(__longlong_as_double((long long)x), elo + share_hi(c, nhi, i)));
          tm = x > tm ? x : tm;
#pragma unroll
          for (int q = 0; q < kHi; ++q) {
            const int d = q < nhi ? (int)((i >> (2 * (nhi - 1 - q))) & 3) : -1;
#pragma unroll
            for (int e = 0; e < 4; ++e) hm[q][e] = ((d == e) & (x > hm[q][e])) ? x : hm[q][e];
          }
        }
      }
      for (int p = nhi; p < k; ++p) {
        const int d = (tid >> (2 * (k - 1 - p))) & 3;
        if (tm) atomicMax(&pmax[c][p][d], tm);
      }
#pragma unroll
      for (int q = 0; q < kHi; ++q) {
        if (q >= nhi) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const unsigned long long w = wave_max_u64(hm[q][e]);
          if (lane == 0 && w) atomicMax(&pmax[c][q][e], w);
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < b.K * 4; i += blockDim.x) {
      const int j = i >> 2, d = i & 3;
      const double mu = __longlong_as_double((long long)pmax[b.up[j]][b.pos_up[j]][d]);
      const double md = __longlong_as_double((long long)pmax[b.down[j]][b.pos_down[j]][d]);
      int step = 0;
      if (mu > 0.0 && md > 0.0 && isfinite(mu) && isfinite(md)) {
        const int diff = bexp(md) - bexp(mu);
        step = diff >= 0 ? diff / 2 : -((-diff) / 2);  // round toward zero: exact halves
      }
      stp[j][d] = step;
    }
    __syncthreads();
    // A step common to a cut's four digits only moves scale between its two
    // subcircuits (the final offsets undo that); applied round after round
    // it overshoots in a subcircuit with many cuts, so only the part that
    // differs between digits is applied.
    for (int i = tid; i < b.K * 4; i += blockDim.x) {
      const int j = i >> 2, d = i & 3;
      const int sum = stp[j][0] + stp[j][1] + stp[j][2] + stp[j][3];
      const int mean = sum >= 0 ? sum / 4 : -((-sum) / 4);
      int e = ej[j][d] + stp[j][d] - mean;
      e = e > 200 ? 200 : (e < -200 ? -200 : e);
      if (e != ej[j][d]) {
        ej[j][d] = e;
        changed = 1;
      }
    }
    __syncthreads();
    const int more = changed;
    __syncthreads();  // every thread has read the flag before the next round clears it
    if (!more) break;
  }
  // every subcircuit's largest scaled row (binary exponent)
  for (int c = 0; c < b.n_sub; ++c) {
    const int k = b.k[c];
    const int64_t rows = (int64_t)1 << (2 * k);
    const int64_t iters = (rows + kBalThreads - 1) >> kBalLog;
    const int nhi = k > kBalFixed ? k - kBalFixed : 0;
    const int elo = share_lo(c, k, nhi);
    int sm = INT_MIN;
    for (int64_t i0 = 0; i0 < iters; i0 += kBalUnroll) {
      unsigned long long v[kBalUnroll];
#pragma unroll
      for (int u = 0; u < kBalUnroll; ++u) {
        const int64_t l = ((i0 + u) << kBalLog) + tid;
        v[u] = ((i0 + u < iters) & (l < rows)) ? b.rowmax[c][l] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kBalUnroll; ++u) {
        const double x = __longlong_as_double((long long)v[u]);
        if (x > 0.0 && isfinite(x)) sm = max(sm, bexp(x) + elo + share_hi(c, nhi, i0 + u));
      }
    }
    sm = wave_max_i32(sm);
    if (lane == 0 && sm != INT_MIN) atomicMax(&smax[c], sm);
  }
  __syncthreads();
  if (tid == 0) {
    int n = 0, last = -1;
    long long sum = 0;
    for (int c = 0; c < b.n_sub; ++c)
      if (smax[c] != INT_MIN) {
        sum += smax[c];
        ++n;
        last = c;
      }
    // floor of the mean
    const long long mean = n ? (sum >= 0 ? sum / n : -((-sum + n - 1) / n)) : 0;
    long long tot = 0;
    for (int c = 0; c < b.n_sub; ++c) {
      goff[c] = smax[c] == INT_MIN ? 0 : (int)(mean - smax[c]);
      tot += goff[c];
    }
    if (last >= 0) goff[last] -= (int)tot;  // the offsets sum to zero
  }
  __syncthreads();
  // every row's exponent: its digits' shares plus its subcircuit's offset
  for (int c = 0; c < b.n_sub; ++c) {
    const int k = b.k[c];
    const int64_t rows = (int64_t)1 << (2 * k);
    const int nhi = k > kBalFixed ? k - kBalFixed : 0;
    const int elo = share_lo(c, k, nhi) + goff[c];
    for (int64_t i = 0; (i << kBalLog) < rows; ++i) {
      const int64_t l = (i << kBalLog) + tid;
      if (l < rows) b.rexp[c][l] = elo + share_hi(c, nhi, i);
    }
  }
}

__global__ void __launch_bounds__(kBalThreads) balance_kernel(BalanceLaunch b) { balance_body(b); }

// The balance of one instance of a dynamic-definition batch (grid z), from
// its program; nothing when the recursion converts nothing.
__global__ void __launch_bounds__(kBalThreads) balance_ind_kernel(const DDProgram* P, const DDLevel* lv,
                                                                  int64_t slot) {
  P = inst_ptr(P, slot);
  lv = inst_ptr(lv, slot);
  if (!P->balance) return;
  bool any = false;
  for (int c = 0; c < P->n_sub; ++c) any = any | (lv->prep[c].n > 0);
  if (!any) return;
  balance_body(P->bal);
}

// Column maxima of the reduced entries for the column scaling: subcircuit
// blockIdx.y of instance blockIdx.z, 64 columns a workgroup, its four waves
// taking every fourth row; values carry the balance's row exponents, as the
// conversion applies them.
__global__ void __launch_bounds__(256) colmax_ind_kernel(const DDProgram* P, const DDLevel* lv, int64_t slot) {
  __shared__ double part[4][64];
  P = inst_ptr(P, slot);
  lv = inst_ptr(lv, slot);
  const int c = blockIdx.y;
  if (!P->cscale || c >= P->n_sub) return;
  const PrepArgs& pa = lv->prep[c];
  const int64_t cols = (int64_t)1 << pa.cols_log2;
  if (pa.n <= 0 || (int64_t)blockIdx.x * 64 >= cols) return;
  const int64_t rows = P->rows[c];
  const int32_t* rexp = P->balance ? P->bal.rexp[c] : nullptr;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 64 + lane;
  double m = 0.0;
  if (b < cols)
    for (int64_t r = w; r < rows; r += 4) {
      const double x = pa.src[(r << pa.cols_log2) + b];
      m = fmax(m, fabs(rexp ? ldexp(x, rexp[r]) : x));
    }
  part[w][lane] = m;
  __syncthreads();
  if (w == 0 && b < cols)
    P->colmax[c][b] = (uint64_t)__double_as_longlong(
        fmax(fmax(part[0][lane], part[1][lane]), fmax(part[2][lane], part[3][lane])));
}

// Output exponents of the last GEMM (step `step`): blockIdx.y 0 its rows
// (z * M + m), 1 its columns (n); each the sum over the group's subcircuits of
// the exponent of the column that bits shift .. shift + na_c - 1 select.
__global__ void __launch_bounds__(256) expsum_ind_kernel(const DDProgram* P, const DDState* st,
                                                         const DDLevel* lv, int step, int64_t slot) {
  P = inst_ptr(P, slot);
  st = inst_ptr(st, slot);
  lv = inst_ptr(lv, slot);
  if (!P->cscale) return;
  const GemmArgs& g = lv->gemm[step];
  if (g.tiles <= 0) return;
  const int q = blockIdx.y;
  const int64_t count = q == 0 ? g.tiles / (g.tilesM * g.tilesN) * g.M : g.N;
  int32_t* const out = q == 0 ? P->rowexp : P->colexp;
  // each member's bit field, the same for every row: its shift and width
  const int n = P->fac_n[q];
  int sh[CQ_MAX_SUBCIRCUITS], sub[CQ_MAX_SUBCIRCUITS];
  int64_t mk[CQ_MAX_SUBCIRCUITS];
#pragma unroll
  for (int i = 0; i < CQ_MAX_SUBCIRCUITS; ++i) {
    sh[i] = 0;
    sub[i] = 0;
    mk[i] = 0;
    if (i < n) {
      const SymLog& sl = P->fac_shift[q][i];
      int s = sl.c0;
      for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c)
        if ((sl.mask >> c) & 1u) s += st->na[c];
      sh[i] = s;
      sub[i] = P->fac_sub[q][i];
      mk[i] = ((int64_t)1 << st->na[sub[i]]) - 1;
    }
  }
  // four consecutive rows a thread, one 16-byte store where the address
  // allows it; a member whose field starts at bit 2 or above has the same
  // column for all four
  const int64_t stepg = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; r < count; r += stepg) {
    int e[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < CQ_MAX_SUBCIRCUITS; ++i) {
      if (i >= n) continue;
      const uint64_t* cm = P->colmax[sub[i]];
      if (sh[i] >= 2) {
        const int v = colmax_exp(cm[(r >> sh[i]) & mk[i]]);
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] += v;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] += colmax_exp(cm[((r + j) >> sh[i]) & mk[i]]);
      }
    }
    if (r + 4 <= count && (reinterpret_cast<uintptr_t>(out + r) & 15) == 0) {
      *reinterpret_cast<int4*>(out + r) = make_int4(e[0], e[1], e[2], e[3]);
    } else {
      for (int j = 0; j < 4 && r + j < count; ++j) out[r + j] = e[j];
    }
  }
}

// Tile maxima of the row exponents over the 128-row tiles of each batch
// (z * tilesM + mt), for the tile bounds when A is shared across batches
// (else the bounds weight every element by its own exponents and this
// exits); one wave a tile, its lanes taking every 64th row (coalesced), then
// a wave maximum.
__global__ void __launch_bounds__(256) exptmax_ind_kernel(const DDProgram* P, const DDLevel* lv, int step,
                                                          int64_t slot) {
  P = inst_ptr(P, slot);
  lv = inst_ptr(lv, slot);
  if (!P->cscale) return;
  const GemmArgs& g = lv->gemm[step];
  if (g.tiles <= 0) return;
  const int64_t Z = g.tiles / (g.tilesM * g.tilesN);
  if (g.sAz != 0 || Z == 1) return;
  const int64_t count = Z * g.tilesM;
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  // t is the same for every lane of a wave, so every lane reaches the shuffles
  for (int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < count; t += waves) {
    int e = INT_MIN;
    const int64_t z = t / g.tilesM, m0 = (t - z * g.tilesM) * 128;
    const int64_t m1 = m0 + 128 < g.M ? m0 + 128 : g.M;
    for (int64_t m = m0 + lane; m < m1; m += 64) e = max(e, P->rowexp[z * g.M + m]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) e = max(e, __shfl_xor(e, o));
    if (lane == 0) P->rowtmax[t] = e;
  }
}

// Row maxima of the reduced entries for the balance: subcircuit blockIdx.y of
// instance blockIdx.z, one wave per row of its current 2^cols_log2 columns
// (zeros for a subcircuit the recursion does not convert).
__global__ void __launch_bounds__(256) rowmax_ind_kernel(const DDProgram* P, const DDLevel* lv, int64_t slot) {
  P = inst_ptr(P, slot);
  lv = inst_ptr(lv, slot);
  const int c = blockIdx.y;
  if (!P->balance || c >= P->n_sub) return;
  const PrepArgs& pa = lv->prep[c];
  const bool live = pa.n > 0;
  const int64_t rows = P->rows[c];
  const int64_t cols = (int64_t)1 << pa.cols_log2;
  uint64_t* const rm = const_cast<uint64_t*>(P->bal.rowmax[c]);
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wave; r < rows; r += waves) {
    double m = 0.0;
    if (live) {
      const double* row = pa.src + (r << pa.cols_log2);
      for (int64_t col = lane; col < cols; col += 64) m = fmax(m, fabs(row[col]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) rm[r] = (uint64_t)__double_as_longlong(m);
  }
}

__global__ void __launch_bounds__(256) fill_u64_kernel(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) p[i] = v;
}

template <int DK>
__global__ void __launch_bounds__(256) prep_scaled_kernel(const double* __restrict__ src, void* dst,
                                                          void* dst_lo, int64_t n, int cols_log2,
                                                          const uint64_t* __restrict__ colmax,
                                                          const int32_t* __restrict__ rexp) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const int64_t mask = ((int64_t)1 << cols_log2) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    const int e = -colmax_exp(colmax[i & mask]) + (rexp ? rexp[i >> cols_log2] : 0);
    const float x = float(ldexp(src[i], e));
    if constexpr (DK == kF32) {
      static_cast<float*>(dst)[i] = x;
    } else {
      const uint16_t h = f_to_h16(x, DK == kF16);
      static_cast<uint16_t*>(dst)[i] = h;
      if (dst_lo) static_cast<uint16_t*>(dst_lo)[i] = f_to_h16(x - h16_to_f(h, DK == kF16), DK == kF16);
    }
  }
}

__global__ void __launch_bounds__(256) expsum_kernel(ExpSumLaunch x) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < x.count; r += step) {
    int e = 0;
    for (int c = 0; c < x.n; ++c) e += colmax_exp(x.colmax[c][(r >> x.shift[c]) & ((1ll << x.bits[c]) - 1)]);
    x.out[r] = e;
  }
}

// ---------------------------------------------------------------------------
// Attribution (Section 3.1).  Two separable passes, both FP64:
//  1. measured ends: U[j][lm][b] = sum_m prod_u sigma(lm_u, m_u)
//                                  * V[j][basis(lm)][compose(b, m)]
//  2. initialised ends: E[row(li, lm)][b] = sum_j prod_t alpha(li_t, j_t) U[j][lm][b]
// Thread per output element; b is the fastest index so stores are contiguous.
// ---------------------------------------------------------------------------

struct AttrArgs {
  const double* V;
  double* U;
  double* E;
  int r, o, n, w, k;
  int out_pos[CQ_MAX_WIDTH];
  int meas_pos[CQ_MAX_WIDTH];
  int64_t init_w[CQ_MAX_WIDTH];
  int64_t meas_w[CQ_MAX_WIDTH];
};

// Measurement basis of a label: I and Z -> Z basis (0), X -> 1, Y -> 2.
__device__ inline int basis_of(int l) { return l == 3 ? 0 : l; }

// alpha(label, prepared state) for states |0>, |1>, |+>, |+i> = 0..3; only
// called on the support (I, Z: |0>, |1>; X: also |+>; Y: also |+i>).
__device__ inline double alpha_coef(int l, int d) {
  if (d >= 2) return 2.0;
  if (l == 0) return 1.0;
  if (l == 3) return d == 0 ? 1.0 : -1.0;
  return -1.0;
}

__global__ void __launch_bounds__(256) attr_meas_kernel(AttrArgs a) {
  const int64_t nb = (int64_t)1 << a.n;
  const int64_t nlm = (int64_t)1 << (2 * a.o);
  const int64_t total = ((int64_t)1 << (2 * a.r)) * nlm * nb;
  int64_t pow3o = 1;
  for (int u = 0; u < a.o; ++u) pow3o *= 3;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
    const int64_t b = i % nb;
    const int64_t lm = (i / nb) % nlm;
    const int64_t j = i / (nb * nlm);
    int64_t x0 = 0;
    for (int q = 0; q < a.n; ++q)
      if ((b >> (a.n - 1 - q)) & 1) x0 |= (int64_t)1 << a.out_pos[q];
    int64_t beta = 0;
    for (int u = 0; u < a.o; ++u) beta = 3 * beta + basis_of((lm >> (2 * (a.o - 1 - u))) & 3);
    const double* Vj = a.V + ((j * pow3o + beta) << a.w);
    double sum = 0.0;
    for (int m = 0; m < (1 << a.o); ++m) {
      int64_t x = x0;
      bool neg = false;
      for (int u = 0; u < a.o; ++u) {
        if ((m >> (a.o - 1 - u)) & 1) {
          x |= (int64_t)1 << a.meas_pos[u];
          if (((lm >> (2 * (a.o - 1 - u))) & 3) != 0) neg = !neg;
        }
      }
      const double v = Vj[x];
      sum += neg ? -v : v;
    }
    a.U[i] = sum;
  }
}

__global__ void __launch_bounds__(256) attr_init_kernel(AttrArgs a) {
  const int64_t nb = (int64_t)1 << a.n;
  const int64_t nlm = (int64_t)1 << (2 * a.o);
  const int64_t nli = (int64_t)1 << (2 * a.r);
  const int64_t total = nli * nlm * nb;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
    const int64_t b = i % nb;
    const int64_t lm = (i / nb) % nlm;
    const int64_t li = i / (nb * nlm);
    // support of each init digit: I, Z -> {0, 1}; X -> {0, 1, 2}; Y -> {0, 1, 3}
    int64_t combos = 1;
    for (int t = 0; t < a.r; ++t) {
      const int l = (li >> (2 * (a.r - 1 - t))) & 3;
      combos *= (l == 1 || l == 2) ? 3 : 2;
    }
    double sum = 0.0;
    for (int64_t c = 0; c < combos; ++c) {
      int64_t rem = c, j = 0;
      double coef = 1.0;
      // mixed radix over the supports, last init slot fastest
      for (int t = a.r - 1; t >= 0; --t) {
        const int l = (li >> (2 * (a.r - 1 - t))) & 3;
        const int sz = (l == 1 || l == 2) ? 3 : 2;
        int d = (int)(rem % sz);
        rem /= sz;
        if (d == 2) d = (l == 1) ? 2 : 3;
        j += (int64_t)d << (2 * (a.r - 1 - t));
        coef *= alpha_coef(l, d);
      }
      sum += coef * a.U[(j * nlm + lm) * nb + b];
    }
    int64_t row = 0;
    for (int t = 0; t < a.r; ++t) row += ((li >> (2 * (a.r - 1 - t))) & 3) * a.init_w[t];
    for (int u = 0; u < a.o; ++u) row += ((lm >> (2 * (a.o - 1 - u))) & 3) * a.meas_w[u];
    a.E[row * nb + b] = sum;
  }
}

// Register forms of the two passes for few cut ends (the common case): a
// thread owns one (j, b) -- or one (lm, b) -- reads each input element once
// and produces every label of its group by butterflies in registers, so V and
// U each cross HBM once.
//  * measured ends, O <= 2: the 3^O x 2^O values V[j][beta][compose(b, m)]
//    give all 4^O labels lm;
//  * initialised ends, R <= 3: per init digit, (|0>, |1>, |+>, |+i>) ->
//    (I, X, Y, Z) = (d0 + d1, -d0 - d1 + 2 d2, -d0 - d1 + 2 d3, d0 - d1).
template <int O>
__global__ void __launch_bounds__(256) attr_meas_reg_kernel(AttrArgs a) {
  constexpr int NB = O == 0 ? 1 : (O == 1 ? 3 : 9);   // 3^O bases
  constexpr int NM = 1 << O;                          // outcomes of the measured bits
  constexpr int NL = 1 << (2 * O);                    // labels
  const int64_t nb = (int64_t)1 << a.n;
  const int64_t total = ((int64_t)1 << (2 * a.r)) * nb;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
    const int64_t b = i & (nb - 1);
    const int64_t j = i >> a.n;
    int64_t x0 = 0;
    for (int q = 0; q < a.n; ++q)
      if ((b >> (a.n - 1 - q)) & 1) x0 |= (int64_t)1 << a.out_pos[q];
    double v[NB][NM];
#pragma unroll
    for (int beta = 0; beta < NB; ++beta)
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        int64_t x = x0;
#pragma unroll
        for (int u = 0; u < O; ++u)
          if ((m >> (O - 1 - u)) & 1) x |= (int64_t)1 << a.meas_pos[u];
        v[beta][m] = a.V[((j * NB + beta) << a.w) + x];
      }
#pragma unroll
    for (int lm = 0; lm < NL; ++lm) {
      int beta = 0;
#pragma unroll
      for (int u = 0; u < O; ++u) beta = 3 * beta + basis_of((lm >> (2 * (O - 1 - u))) & 3);
      double sum = 0.0;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        bool neg = false;
#pragma unroll
        for (int u = 0; u < O; ++u)
          if (((m >> (O - 1 - u)) & 1) && ((lm >> (2 * (O - 1 - u))) & 3) != 0) neg = !neg;
        sum += neg ? -v[beta][m] : v[beta][m];
      }
      a.U[(j * NL + lm) * nb + b] = sum;
    }
  }
}

template <int R>
__global__ void __launch_bounds__(256) attr_init_reg_kernel(AttrArgs a) {
  constexpr int NJ = 1 << (2 * R);
  const int64_t nb = (int64_t)1 << a.n;
  const int64_t nlm = (int64_t)1 << (2 * a.o);
  const int64_t total = nlm * nb;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
    const int64_t b = i & (nb - 1);
    const int64_t lm = i >> a.n;
    double u[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) u[j] = a.U[(j * nlm + lm) * nb + b];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int sd = 1 << (2 * (R - 1 - t));  // stride of init digit t
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if ((j / sd) % 4 != 0) continue;
        const double d0 = u[j], d1 = u[j + sd], d2 = u[j + 2 * sd], d3 = u[j + 3 * sd];
        u[j] = d0 + d1;                       // I
        u[j + sd] = 2.0 * d2 - d0 - d1;       // X
        u[j + 2 * sd] = 2.0 * d3 - d0 - d1;   // Y
        u[j + 3 * sd] = d0 - d1;              // Z
      }
    }
    int64_t mrow = 0;
    for (int q = 0; q < a.o; ++q) mrow += ((lm >> (2 * (a.o - 1 - q))) & 3) * a.meas_w[q];
#pragma unroll
    for (int li = 0; li < NJ; ++li) {
      int64_t row = mrow;
#pragma unroll
      for (int t = 0; t < R; ++t) row += ((li >> (2 * (R - 1 - t))) & 3) * a.init_w[t];
      a.E[row * nb + b] = u[li];
    }
  }
}

// Both passes in one kernel for up to two measured and two initialised cut
// ends (the dynamic-definition subcircuits): a thread owns one output column
// b and walks the 3^O measurement bases; for each basis it loads the
// 4^R x 2^O variant values V[j][basis][compose(b, m)] it needs (each element
// of V is read once overall), forms U[j][lm] for the labels lm measured in
// that basis, runs the init butterflies over j in registers and writes the
// 4^R entries of each such lm.  U never reaches memory, so HBM sees V once
// and E once.  Same operations in the same order as the two register passes.
template <int R, int O>
__global__ void __launch_bounds__(256) attr_fused_kernel(AttrArgs a) {
  constexpr int NJ = 1 << (2 * R);                   // init digit strings
  constexpr int NB = O == 0 ? 1 : (O == 1 ? 3 : 9);  // 3^O bases
  constexpr int NM = 1 << O;                         // outcomes of the measured bits
  constexpr int NL = 1 << (2 * O);                   // measured labels
  const int64_t nb = (int64_t)1 << a.n;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += step) {
    int64_t x0 = 0;
    for (int q = 0; q < a.n; ++q)
      if ((b >> (a.n - 1 - q)) & 1) x0 |= (int64_t)1 << a.out_pos[q];
    int64_t xm[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      int64_t x = x0;
#pragma unroll
      for (int u = 0; u < O; ++u)
        if ((m >> (O - 1 - u)) & 1) x |= (int64_t)1 << a.meas_pos[u];
      xm[m] = x;
    }
#pragma unroll
    for (int beta = 0; beta < NB; ++beta) {
      double v[NJ][NM];
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int m = 0; m < NM; ++m) v[j][m] = a.V[(((int64_t)j * NB + beta) << a.w) + xm[m]];
#pragma unroll
      for (int lm = 0; lm < NL; ++lm) {
        int bl = 0;
#pragma unroll
        for (int u = 0; u < O; ++u) bl = 3 * bl + basis_of((lm >> (2 * (O - 1 - u))) & 3);
        if (bl != beta) continue;
        double uj[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          double sum = 0.0;
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            bool neg = false;
#pragma unroll
            for (int u = 0; u < O; ++u)
              if (((m >> (O - 1 - u)) & 1) && ((lm >> (2 * (O - 1 - u))) & 3) != 0) neg = !neg;
            sum += neg ? -v[j][m] : v[j][m];
          }
          uj[j] = sum;
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int sd = 1 << (2 * (R - 1 - t));  // stride of init digit t
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            if ((j / sd) % 4 != 0) continue;
            const double d0 = uj[j], d1 = uj[j + sd], d2 = uj[j + 2 * sd], d3 = uj[j + 3 * sd];
            uj[j] = d0 + d1;                       // I
            uj[j + sd] = 2.0 * d2 - d0 - d1;       // X
            uj[j + 2 * sd] = 2.0 * d3 - d0 - d1;   // Y
            uj[j + 3 * sd] = d0 - d1;              // Z
          }
        }
        int64_t mrow = 0;
#pragma unroll
        for (int q = 0; q < O; ++q) mrow += ((lm >> (2 * (O - 1 - q))) & 3) * a.meas_w[q];
#pragma unroll
        for (int li = 0; li < NJ; ++li) {
          int64_t row = mrow;
#pragma unroll
          for (int t = 0; t < R; ++t) row += ((li >> (2 * (R - 1 - t))) & 3) * a.init_w[t];
          a.E[row * nb + b] = uj[li];
        }
      }
    }
  }
}

// Indirect launches size their grid for the largest shape and loop; a
// moderate cap keeps the empty workgroups of smaller shapes cheap.
unsigned grid_ind(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

unsigned grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 1 << 20) b = 1 << 20;
  if (b < 1) b = 1;
  return (unsigned)b;
}


int kind_of(DType t, bool f16) {
  if (t == DType::F64) return kF64;
  if (t == DType::F32) return kF32;
  return f16 ? kF16 : kBF16;
}

template <int SK>
void permute_dispatch_dst(int dk, dim3 grid, const PermArgs& a, hipStream_t s) {
  switch (dk) {
    case kF64: hipLaunchKernelGGL((permute_kernel<SK, kF64>), grid, dim3(256), 0, s, a); break;
    case kF32: hipLaunchKernelGGL((permute_kernel<SK, kF32>), grid, dim3(256), 0, s, a); break;
    case kBF16: hipLaunchKernelGGL((permute_kernel<SK, kBF16>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((permute_kernel<SK, kF16>), grid, dim3(256), 0, s, a); break;
  }
}

template <int SK>
void permute_ind_dispatch_dst(int dk, dim3 grid, const PermArgs* a, int64_t slot, hipStream_t s) {
  switch (dk) {
    case kF64: hipLaunchKernelGGL((permute_ind_kernel<SK, kF64>), grid, dim3(256), 0, s, a, slot); break;
    case kF32: hipLaunchKernelGGL((permute_ind_kernel<SK, kF32>), grid, dim3(256), 0, s, a, slot); break;
    case kBF16: hipLaunchKernelGGL((permute_ind_kernel<SK, kBF16>), grid, dim3(256), 0, s, a, slot); break;
    default: hipLaunchKernelGGL((permute_ind_kernel<SK, kF16>), grid, dim3(256), 0, s, a, slot); break;
  }
}

}  // namespace

hipError_t launch_permute_indirect(const PermArgs* dev, DType ts, DType td, bool f16,
                                   int64_t max_total, hipStream_t stream, InstSpan span) {
  if (max_total <= 0 || span.n <= 0) return hipSuccess;
  const dim3 grid(grid_ind(max_total), 1, (unsigned)span.n);
  const int sk = kind_of(ts, f16), dk = kind_of(td, f16);
  switch (sk) {
    case kF64: permute_ind_dispatch_dst<kF64>(dk, grid, dev, span.stride, stream); break;
    case kF32: permute_ind_dispatch_dst<kF32>(dk, grid, dev, span.stride, stream); break;
    case kBF16: permute_ind_dispatch_dst<kBF16>(dk, grid, dev, span.stride, stream); break;
    default: permute_ind_dispatch_dst<kF16>(dk, grid, dev, span.stride, stream); break;
  }
  return hipGetLastError();
}

hipError_t launch_prep_indirect(const PrepArgs* dev, int count, DType t, bool f16, int64_t max_n,
                                hipStream_t stream, InstSpan span) {
  if (max_n <= 0 || count <= 0 || span.n <= 0) return hipSuccess;
  const dim3 grid(grid_ind(max_n), (unsigned)count, (unsigned)span.n);
  if (t == DType::F32)
    hipLaunchKernelGGL((prep_ind_kernel<kF32>), grid, dim3(256), 0, stream, dev, span.stride);
  else if (f16)
    hipLaunchKernelGGL((prep_ind_kernel<kF16>), grid, dim3(256), 0, stream, dev, span.stride);
  else
    hipLaunchKernelGGL((prep_ind_kernel<kBF16>), grid, dim3(256), 0, stream, dev, span.stride);
  return hipGetLastError();
}

hipError_t launch_permute(const PermLaunch& p, hipStream_t stream) {
  PermArgs a;
  a.src = p.src.p;
  a.src_lo = p.src.t == DType::H16X2 ? p.src.lo : nullptr;
  a.dst = p.dst;
  a.dst_lo = p.td == DType::H16X2 ? p.dst_lo : nullptr;
  a.naxes = p.naxes;
  int bits = 0;
  for (int i = 0; i < p.naxes; ++i) {
    a.log2[i] = p.log2[i];
    a.sstride[i] = p.sstride[i];
    bits += p.log2[i];
  }
  a.total = (int64_t)1 << bits;
  a.alpha = p.alpha;
  a.nfac = p.nfac;
  for (int c = 0; c < CQ_MAX_SUBCIRCUITS; ++c) {
    a.colmax[c] = p.colmax[c];
    a.fac_shift[c] = p.fac_shift[c];
    a.fac_bits[c] = p.fac_bits[c];
  }
  const dim3 grid(grid_for(a.total));
  const int sk = kind_of(p.src.t, p.f16), dk = kind_of(p.td, p.f16);
  switch (sk) {
    case kF64: permute_dispatch_dst<kF64>(dk, grid, a, stream); break;
    case kF32: permute_dispatch_dst<kF32>(dk, grid, a, stream); break;
    case kBF16: permute_dispatch_dst<kBF16>(dk, grid, a, stream); break;
    default: permute_dispatch_dst<kF16>(dk, grid, a, stream); break;
  }
  return hipGetLastError();
}

hipError_t launch_prep(const double* src, void* dst, int64_t n, DType t, bool f16,
                       hipStream_t stream, const int32_t* rexp, int cols_log2) {
  if (n <= 0) return hipSuccess;
  void* lo = t == DType::H16X2 ? static_cast<char*>(dst) + n * 2 : nullptr;
  auto al = [](const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; };
  const bool v4 = n % 4 == 0 && (!rexp || cols_log2 >= 2) && al(src, 16) &&
                  al(dst, t == DType::F32 ? 16 : 8) && (!lo || al(lo, 8));
  const dim3 grid(grid_for(v4 ? n / 4 : n));
  if (t == DType::F32) {
    if (v4) hipLaunchKernelGGL((prep_kernel<kF32, true>), grid, dim3(256), 0, stream, src, dst, nullptr, n, rexp, cols_log2);
    else hipLaunchKernelGGL((prep_kernel<kF32, false>), grid, dim3(256), 0, stream, src, dst, nullptr, n, rexp, cols_log2);
  } else if (f16) {
    if (v4) hipLaunchKernelGGL((prep_kernel<kF16, true>), grid, dim3(256), 0, stream, src, dst, lo, n, rexp, cols_log2);
    else hipLaunchKernelGGL((prep_kernel<kF16, false>), grid, dim3(256), 0, stream, src, dst, lo, n, rexp, cols_log2);
  } else {
    if (v4) hipLaunchKernelGGL((prep_kernel<kBF16, true>), grid, dim3(256), 0, stream, src, dst, lo, n, rexp, cols_log2);
    else hipLaunchKernelGGL((prep_kernel<kBF16, false>), grid, dim3(256), 0, stream, src, dst, lo, n, rexp, cols_log2);
  }
  return hipGetLastError();
}

hipError_t launch_rowmax(const double* E, int64_t rows, int cols_log2, uint64_t* rowmax,
                         hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(rowmax_kernel, dim3(grid_for(rows * 64)), dim3(256), 0, stream, E, rows, cols_log2,
                     rowmax);
  return hipGetLastError();
}

hipError_t launch_dd_balance(const DDProgram* prog, const DDLevel* lv, int n_sub, int64_t max_rows,
                             hipStream_t stream, InstSpan span) {
  if (n_sub <= 0 || max_rows <= 0 || span.n <= 0) return hipSuccess;
  int64_t gx = (max_rows * 64 + 255) / 256;
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(rowmax_ind_kernel, dim3((unsigned)gx, (unsigned)n_sub, (unsigned)span.n), dim3(256), 0,
                     stream, prog, lv, span.stride);
  hipLaunchKernelGGL(balance_ind_kernel, dim3(1, 1, (unsigned)span.n), dim3(kBalThreads), 0, stream, prog, lv,
                     span.stride);
  return hipGetLastError();
}

hipError_t launch_dd_colmax(const DDProgram* prog, const DDLevel* lv, int n_sub, int64_t max_cols,
                            hipStream_t stream, InstSpan span) {
  if (n_sub <= 0 || max_cols <= 0 || span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(colmax_ind_kernel, dim3((unsigned)((max_cols + 63) / 64), (unsigned)n_sub, (unsigned)span.n),
                     dim3(256), 0, stream, prog, lv, span.stride);
  return hipGetLastError();
}

hipError_t launch_dd_expsum(const DDProgram* prog, const DDState* st, const DDLevel* lv, int step,
                            int64_t max_rows, int64_t max_cols, hipStream_t stream, InstSpan span) {
  if (span.n <= 0) return hipSuccess;
  const int64_t most = max_rows > max_cols ? max_rows : max_cols;
  hipLaunchKernelGGL(expsum_ind_kernel, dim3(grid_ind(most), 2, (unsigned)span.n), dim3(256), 0, stream, prog,
                     st, lv, step, span.stride);
  // one wave a tile: a few tiles a wave at most
  hipLaunchKernelGGL(exptmax_ind_kernel, dim3(grid_ind(most / 2 + 1), 1, (unsigned)span.n), dim3(256), 0, stream,
                     prog, lv, step, span.stride);
  return hipGetLastError();
}

hipError_t launch_balance(const BalanceLaunch& b, hipStream_t stream) {
  hipLaunchKernelGGL(balance_kernel, dim3(1), dim3(kBalThreads), 0, stream, b);
  return hipGetLastError();
}

hipError_t launch_colmax(const double* E, int64_t rows, int cols_log2, uint64_t* colmax,
                         hipStream_t stream, const int32_t* rexp) {
  const int64_t cols = (int64_t)1 << cols_log2;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(cols)), dim3(256), 0, stream, colmax, cols,
                     (uint64_t)0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int rpt = 64;
  const int64_t total = (rows + rpt - 1) / rpt * cols;
  hipLaunchKernelGGL(colmax_kernel, dim3(grid_for(total)), dim3(256), 0, stream, E, rows, cols_log2,
                     rpt, colmax, rexp);
  return hipGetLastError();
}

hipError_t launch_prep_scaled(const double* src, void* dst, int64_t n, int cols_log2,
                              const uint64_t* colmax, DType t, bool f16, hipStream_t stream,
                              const int32_t* rexp) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(grid_for(n));
  void* lo = t == DType::H16X2 ? static_cast<char*>(dst) + n * 2 : nullptr;
  if (t == DType::F32)
    hipLaunchKernelGGL((prep_scaled_kernel<kF32>), grid, dim3(256), 0, stream, src, dst, nullptr, n,
                       cols_log2, colmax, rexp);
  else if (f16)
    hipLaunchKernelGGL((prep_scaled_kernel<kF16>), grid, dim3(256), 0, stream, src, dst, lo, n,
                       cols_log2, colmax, rexp);
  else
    hipLaunchKernelGGL((prep_scaled_kernel<kBF16>), grid, dim3(256), 0, stream, src, dst, lo, n,
                       cols_log2, colmax, rexp);
  return hipGetLastError();
}

hipError_t launch_expsum(const ExpSumLaunch& x, hipStream_t stream) {
  if (x.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(expsum_kernel, dim3(grid_for(x.count)), dim3(256), 0, stream, x);
  return hipGetLastError();
}

hipError_t launch_attribute(const AttrLaunch& l, hipStream_t stream) {
  AttrArgs a;
  a.V = l.V;
  a.U = l.U;
  a.E = l.E;
  a.r = l.r;
  a.o = l.o;
  a.n = l.n;
  a.w = l.w;
  a.k = l.k;
  for (int i = 0; i < CQ_MAX_WIDTH; ++i) {
    a.out_pos[i] = l.out_pos[i];
    a.meas_pos[i] = l.meas_pos[i];
    a.init_w[i] = l.init_w[i];
    a.meas_w[i] = l.meas_w[i];
  }
  const int64_t total = ((int64_t)1 << (2 * (l.r + l.o))) << l.n;
  const unsigned grid = grid_for(total);
  if (l.r <= 2 && l.o <= 2) {
    const dim3 gf(grid_for((int64_t)1 << l.n));
#define CQ_ATTR_FUSED(R, O)                                                          \
  if (l.r == R && l.o == O) {                                                        \
    hipLaunchKernelGGL((attr_fused_kernel<R, O>), gf, dim3(256), 0, stream, a);     \
    return hipGetLastError();                                                        \
  }
    CQ_ATTR_FUSED(0, 0) CQ_ATTR_FUSED(0, 1) CQ_ATTR_FUSED(0, 2)
    CQ_ATTR_FUSED(1, 0) CQ_ATTR_FUSED(1, 1) CQ_ATTR_FUSED(1, 2)
    CQ_ATTR_FUSED(2, 0) CQ_ATTR_FUSED(2, 1) CQ_ATTR_FUSED(2, 2)
#undef CQ_ATTR_FUSED
  }
  const dim3 gm(grid_for(((int64_t)1 << (2 * l.r)) << l.n)), gi(grid_for(((int64_t)1 << (2 * l.o)) << l.n));
  switch (l.o) {
    case 0: hipLaunchKernelGGL(attr_meas_reg_kernel<0>, gm, dim3(256), 0, stream, a); break;
    case 1: hipLaunchKernelGGL(attr_meas_reg_kernel<1>, gm, dim3(256), 0, stream, a); break;
    case 2: hipLaunchKernelGGL(attr_meas_reg_kernel<2>, gm, dim3(256), 0, stream, a); break;
    default: hipLaunchKernelGGL(attr_meas_kernel, dim3(grid), dim3(256), 0, stream, a); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (l.r) {
    case 0: hipLaunchKernelGGL(attr_init_reg_kernel<0>, gi, dim3(256), 0, stream, a); break;
    case 1: hipLaunchKernelGGL(attr_init_reg_kernel<1>, gi, dim3(256), 0, stream, a); break;
    case 2: hipLaunchKernelGGL(attr_init_reg_kernel<2>, gi, dim3(256), 0, stream, a); break;
    case 3: hipLaunchKernelGGL(attr_init_reg_kernel<3>, gi, dim3(256), 0, stream, a); break;
    default: hipLaunchKernelGGL(attr_init_kernel, dim3(grid), dim3(256), 0, stream, a); break;
  }
  return hipGetLastError();
}

}  // namespace cq

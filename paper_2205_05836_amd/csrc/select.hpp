// Workgroup selection of the C best keys (Algorithm 1 keeps the largest bins
// of each recursion): a key is a value and a unique index, and a key is
// better than another when its value is larger, or equal with a smaller
// index.  Every lane holds up to V keys (bit e of a 64-bit `live` mask marks
// key e as taking part).
//
// Bound, filter, rank: the C-th best of the lanes' own best keys is a key
// that at least C keys reach, so it bounds the C-th best key overall from
// below.  Keys that reach it are appended to LDS, and each appended key's
// rank among them is its place in the answer.  A handful of keys usually
// pass; when more than CAP do (the best keys crowd into a few lanes), the
// caller runs its exhaustive selection over the narrowed `live` instead.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cq {

// Order-preserving 64-bit key of a double (larger value, larger key), the
// form in which a running threshold is raised with atomicMax.
__device__ inline unsigned long long ord_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

__device__ inline double ord_val(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
  return __longlong_as_double((long long)b);
}

template <typename T, typename I>
struct SelKey {
  T v;
  I i;
};

template <typename T, typename I>
__device__ inline bool sel_better(const SelKey<T, I>& a, const SelKey<T, I>& b) {
  return a.v > b.v || (a.v == b.v && a.i < b.i);
}

// Number of keys among S[0..n) (LDS) better than k.  Eight keys are loaded
// before any is compared, and the comparison is branch-free, so the LDS reads
// overlap instead of each waiting for the one before.
template <typename K>
__device__ __forceinline__ int rank_of(const K* S, int n, const K& k) {
  int r = 0, t = 0;
  for (; t + 8 <= n; t += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const K a = S[t + u];
      r += (int)((a.v > k.v) | ((a.v == k.v) & (a.i < k.i)));
    }
  }
  for (; t < n; ++t) {
    const K a = S[t];
    r += (int)((a.v > k.v) | ((a.v == k.v) & (a.i < k.i)));
  }
  return r;
}

template <typename T, typename I, int NTHR, int CAP>
struct SelShared {
  SelKey<T, I> lane_best[NTHR];
  SelKey<T, I> cand[CAP];
  int count;
  int owner;
};

// Every thread of the workgroup (NTHR threads) calls it with the same C,
// 1 <= C <= NTHR.  at(e) returns key e of the calling lane (called only for
// live e).  none: a key no live key is worse than (it never counts as better
// than one).  Returns found = min(C, live keys) with out[0..found) best
// first, or -1 when more than CAP keys pass the bound; `live` is narrowed to
// the keys that pass, which always include the C best.
template <typename T, typename I, int V, int NTHR, int CAP, typename At>
__device__ __forceinline__ int sel_bound_top(SelShared<T, I, NTHR, CAP>& sh, uint64_t& live, At at,
                                             int C, SelKey<T, I> none, SelKey<T, I>* out) {
  using K = SelKey<T, I>;
  static_assert(V >= 1 && V <= 64, "one live bit per key");
  const int tid = threadIdx.x;
  K best = none;
  bool has = false;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const K k = at(e);
    const bool b = (bool)((live >> e) & 1) & (!has | (k.v > best.v) | ((k.v == best.v) & (k.i < best.i)));
    best.v = b ? k.v : best.v;  // field by field: a select of the whole struct goes through memory
    best.i = b ? k.i : best.i;
    has |= b;
  }
  if (tid == 0) {
    sh.count = 0;
    sh.owner = -1;
  }
  sh.lane_best[tid] = best;
  __syncthreads();
  if (has && rank_of(sh.lane_best, NTHR, best) == C - 1) sh.owner = tid;  // distinct keys, distinct ranks
  __syncthreads();
  const int own = sh.owner;
  if (own >= 0) {
    const K t0 = sh.lane_best[own];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const K k = at(e);
      const bool drop = (t0.v > k.v) | ((t0.v == k.v) & (t0.i < k.i));
      live &= ~((uint64_t)drop << e);
    }
  }
  const int mine = __popcll(live);
  int off = mine ? atomicAdd(&sh.count, mine) : 0;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const bool l = (live >> e) & 1;
    if (l & (off < CAP)) sh.cand[off] = at(e);
    off += l ? 1 : 0;
  }
  __syncthreads();
  const int n = sh.count;
  if (n > CAP) return -1;
  for (int t = tid; t < n; t += NTHR) {
    const K k = sh.cand[t];
    const int r = rank_of(sh.cand, n, k);
    if (r < C) out[r] = k;
  }
  __syncthreads();
  return n < C ? n : C;
}

}  // namespace cq

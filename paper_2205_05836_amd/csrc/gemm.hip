// Label GEMMs: one pairwise contraction of Eq. 1 over the shared cut labels.
//
//   C[z][m][n] = alpha * sum_k A[z*sAz + k*sAk + m] * B[z*sBz + k*sBk + n]
//
// Operands keep the entry-tensor layout (labels slow, outputs fast), so tiles
// load along M and N with full cache lines.  Matrix cores of gfx950:
//   FP64:      v_mfma_f64_16x16x4_f64
//   FP32:      v_mfma_f32_32x32x2_f32
//   BF16/FP16: v_mfma_f32_32x32x16_{bf16,f16}, FP32 accumulation; operands
//              arrive as 16-bit planes (hi, and lo for the split forms) and
//              are transposed in registers on their way to LDS so that each
//              LDS row holds 8 consecutive labels, the MFMA's k-contiguous
//              operand.
// Tiles are 128 x 128 per workgroup of 4 waves (64 x 64 each).  The flat tile
// index is rastered along the dimension whose operand panel is the larger one
// (so that panel is fetched from HBM once and reused from L2), and remapped so
// that each of the 8 XCDs, each with its own L2, receives a contiguous range.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "select.hpp"

namespace cq {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));


// Workgroup b runs on XCD b % 8; give each XCD a contiguous block of tiles.
__device__ inline int64_t xcd_tile(int64_t b, int64_t total) {
  const int64_t per = total / 8, rem = total % 8;
  const int64_t xcd = b % 8, local = b / 8;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Kernels take their arguments by value, or -- for shapes decided on the
// device -- from device memory through `gp` (instance blockIdx.z's block
// gp_stride bytes further on); workgroups beyond the tile count of an
// indirect launch exit at once.
#define CQ_LOAD_GEMM_ARGS                                                        \
  gp = inst_ptr(gp, gp_stride);                                                  \
  const GemmArgs g = gp ? *gp : gv;                                              \
  if (gp && (int64_t)blockIdx.x >= (g.tile_list ? *g.tile_count : g.tiles)) return; \
  if (gp && g.tile_list && g.tile_list[blockIdx.x] >= (uint64_t)g.tiles) return;

struct TileCoord {
  int64_t z, m0, n0;
};

template <int BM, int BN>
__device__ inline TileCoord tile_coord_of(const GemmArgs& g, int64_t t) {
  TileCoord c;
  if (g.tiles < ((int64_t)1 << 31)) {  // 32-bit division (the 64-bit one is a long routine)
    const uint32_t t32 = (uint32_t)t, tm = (uint32_t)g.tilesM, tn = (uint32_t)g.tilesN;
    uint32_t a, r, b;
    if (g.m_fastest) {
      r = t32 / tm;
      a = t32 - r * tm;
      b = r / tn;
      c.m0 = (int64_t)a * BM;
      c.n0 = (int64_t)(r - b * tn) * BN;
    } else {
      r = t32 / tn;
      a = t32 - r * tn;
      b = r / tm;
      c.n0 = (int64_t)a * BN;
      c.m0 = (int64_t)(r - b * tm) * BM;
    }
    c.z = b;
    return c;
  }
  if (g.m_fastest) {
    const int64_t tm = t % g.tilesM, r = t / g.tilesM;
    c.n0 = (r % g.tilesN) * BN;
    c.z = r / g.tilesN;
    c.m0 = tm * BM;
  } else {
    const int64_t tn = t % g.tilesN, r = t / g.tilesN;
    c.m0 = (r % g.tilesM) * BM;
    c.z = r / g.tilesM;
    c.n0 = tn * BN;
  }
  return c;
}

template <int BM, int BN>
__device__ inline TileCoord tile_coord(const GemmArgs& g) {
  return tile_coord_of<BM, BN>(g, g.tile_list ? (int64_t)g.tile_list[blockIdx.x]
                                              : xcd_tile(blockIdx.x, g.tiles));
}

// Tile of virtual block vb (a workgroup may take several, see CQ_TILE_LOOP).
template <int BM, int BN>
__device__ inline TileCoord tile_coord_v(const GemmArgs& g, int64_t vb) {
  return tile_coord_of<BM, BN>(g, g.tile_list ? (int64_t)g.tile_list[vb] : xcd_tile(vb, g.tiles));
}

// Kernels that also serve indirect launches run their tile body for virtual
// blocks blockIdx.x, +gridDim.x, ... up to the device-side count (the tile
// list's length, or the tile count), so a launch over a pruned tile list
// needs no grid sized for every tile; a direct launch (one workgroup per
// tile) runs the body once.
#define CQ_TILE_LOOP(BODY)                                                                      \
  gp = inst_ptr(gp, gp_stride);                                                                 \
  int64_t nvb = (int64_t)gridDim.x;                                                             \
  if (gp) {                                                                                     \
    const GemmArgs* q = gp;                                                                     \
    nvb = q->tile_list ? *q->tile_count : q->tiles;                                             \
  }                                                                                             \
  _Pragma("nounroll")                                                                           \
  for (int64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {                                    \
    /* reload the arguments per tile: nothing of the previous tile stays live */                \
    asm volatile("" ::: "memory");                                                              \
    const GemmArgs g = gp ? *gp : gv;                                                           \
    if (g.tile_list && g.tile_list[vb] >= (uint64_t)g.tiles) continue;                          \
    BODY;                                                                                       \
    __syncthreads();                                                                            \
  }

// Loads 8 consecutive elements of row k (columns c0..c0+7), zero outside
// [0, K) x [0, ncols).
template <typename T>
__device__ inline void load8(const T* __restrict__ P, int64_t k, int64_t sk, int64_t c0,
                             int64_t ncols, int64_t K, T (&out)[8]) {
  if (k >= K) {
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = T(0);
    return;
  }
  const T* p = P + k * sk + c0;
  if (c0 + 8 <= ncols && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
    constexpr int W = 16 / sizeof(T);
    typedef T v16 __attribute__((ext_vector_type(W)));
#pragma unroll
    for (int e = 0; e < 8; e += W) {
      v16 v = *reinterpret_cast<const v16*>(p + e);
#pragma unroll
      for (int q = 0; q < W; ++q) out[e + q] = v[q];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = (c0 + e < ncols) ? p[e] : T(0);
  }
}

// Four consecutive doubles of row k (columns c0..c0+3), zero outside.
__device__ inline void load4(const double* __restrict__ P, int64_t k, int64_t sk, int64_t c0,
                             int64_t ncols, int64_t K, double (&out)[4]) {
  if (k >= K) {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = 0.0;
    return;
  }
  const double* p = P + k * sk + c0;
  if (c0 + 4 <= ncols && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const dv2 x = *reinterpret_cast<const dv2*>(p), y = *reinterpret_cast<const dv2*>(p + 2);
    out[0] = x[0];
    out[1] = x[1];
    out[2] = y[0];
    out[3] = y[1];
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = (c0 + e < ncols) ? p[e] : 0.0;
  }
}

template <typename TC, bool NT>
__device__ inline void store_out(TC* p, TC v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// ---------------------------------------------------------------------------
// Fused top-C epilogue (dynamic definition without stored bins).  A tile
// first compares its values with the running threshold tau, a lower bound on
// the C-th best bin value (it only ever holds the C-th best value of some
// tile).  Tiles with nothing at or above tau end there -- after the first
// tiles almost all of them.  Otherwise the tile selects its own C best keys
// (value desc, index asc) above tau in an LDS buffer, appends them to the
// candidate list and, holding C of them, raises tau to the C-th.  Every key of
// the global top C is at or above tau and among its tile's C best, so the
// candidates contain the global top C exactly.
// ---------------------------------------------------------------------------

template <typename T>
struct TcKey {
  T v;
  uint32_t i;  // r * 128 + c inside the tile
};

template <typename T>
__device__ inline bool tc_better(const TcKey<T>& a, const TcKey<T>& b) {
  return a.v > b.v || (a.v == b.v && a.i < b.i);
}

template <typename T>
__device__ inline TcKey<T> tc_worst() {
  return TcKey<T>{T(-INFINITY), 0xffffffffu};
}

// Best key of the wave (every lane gets it).
template <typename T>
__device__ inline TcKey<T> wave_best(TcKey<T> k) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    const TcKey<T> o{__shfl_xor(k.v, s), (uint32_t)__shfl_xor((int)k.i, s)};
    if (tc_better(o, k)) k = o;
  }
  return k;
}

// Keys of a tile that pass the bound of the tile selection at most (beyond
// it the tile falls back to C rounds of a wave arg-max).
constexpr int kTopcCap = 512;

// The smallest T at or above tau: for T values, v >= tau_as<T>(tau) exactly
// when double(v) >= tau.
// Hides how a lane mask was built, so that later tests of its bits read the
// mask (two VGPRs) instead of keeping every bit's defining condition alive.
__device__ inline uint64_t opaque_mask(uint64_t m) {
  uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
  asm volatile("" : "+v"(lo), "+v"(hi));
  return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ inline T tau_as(double tau) {
  if constexpr (sizeof(T) == 8) {
    return tau;
  } else {
    float f = (float)tau;
    if ((double)f < tau) {  // step to the next float up
      uint32_t b = __float_as_uint(f);
      b = (f == 0.0f) ? 1u : ((b >> 31) ? b - 1 : b + 1);
      f = __uint_as_float(b);
    }
    return f;
  }
}

// Tile selection.  Lane key e has value val(e) and index base + koff(e)
// (r * 128 + c inside the tile; koff(e) is a constant once the loops over e
// are unrolled, so keys of one lane compare by their offsets); valid(e):
// inside M x N, asked on partial tiles only.
//
// Keys at or above tau take part.  The C-th best of the lanes' own best keys
// bounds the tile's C-th best key from below (at least C keys reach it), so
// only keys reaching it are appended to LDS, where each key's rank among
// them is its place in the answer.  Should more than kTopcCap keys reach the
// bound (the best keys crowd into a few lanes), each wave instead takes its C
// best of them by C rounds of a wave arg-max and wave 0 merges the waves'
// lists the same way.  The per-key steps are selects, not branches, which
// keeps the unrolled code short.
template <typename T, int V, int NTHR, typename Val, typename Off, typename Valid>
__device__ __forceinline__ void topc_tile(const GemmArgs& g, int64_t z, int64_t m0, int64_t n0, bool full,
                                          Val val, Off koff, int base, Valid valid) {
  using K = TcKey<T>;
  constexpr int NW = NTHR / 64;
  constexpr int kNone = 0x7fffffff;
  static_assert(V <= 64, "one live bit per value");
  __shared__ K lane_best[NTHR];
  __shared__ K cand[kTopcCap + NTHR];  // beyond kTopcCap: one parking slot per thread
  __shared__ K wk[NW][kDDMaxC];
  __shared__ K outk[kDDMaxC];
  __shared__ int wn[NW];
  __shared__ int cnt, owner, nfound, nout;
  __shared__ unsigned long long obase;
  const int C = *g.topc_C;
  if (C <= 0) return;
  const T tau = tau_as<T>(ord_val(*g.topc_thr));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    // most tiles end here: nothing (not even outside M x N) reaches tau
    T mx = val(0);
#pragma unroll
    for (int e = 1; e < V; ++e) mx = val(e) > mx ? val(e) : mx;
    if (__syncthreads_count(mx >= tau) == 0) return;
  }
  // the keys at or above tau and the lane's best of them
  uint64_t live = 0;
  T bv = T(0);
  int bk = kNone;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const T v = val(e);
    const int k = koff(e);
    // bitwise, not short-circuit: selects instead of branches
    const bool ok = (full | valid(e)) & (v >= tau);
    live |= (uint64_t)ok << e;
    const bool b = ok & ((bk == kNone) | (v > bv) | ((v == bv) & (k < bk)));
    bv = b ? v : bv;
    bk = b ? k : bk;
  }
  live = opaque_mask(live);
  if (__syncthreads_count(live != 0) == 0) return;
  if (tid == 0) {
    cnt = 0;
    owner = -1;
  }
  const bool has = bk != kNone;
  const K mine = has ? K{bv, (uint32_t)(base + bk)} : tc_worst<T>();
  lane_best[tid] = mine;
  __syncthreads();
  if (has && rank_of(lane_best, NTHR, mine) == C - 1) owner = tid;  // distinct keys, distinct ranks
  __syncthreads();
  const int own = owner;
  if (own >= 0) {
    const K t0 = lane_best[own];
    const int d = (int)t0.i - base;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const T v = val(e);
      const bool drop = (t0.v > v) | ((t0.v == v) & (d < koff(e)));
      live &= ~((uint64_t)drop << e);
    }
    live = opaque_mask(live);
  }
  int off = __popcll(live);
  off = off ? atomicAdd(&cnt, off) : 0;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const bool l = (live >> e) & 1;
    cand[(l & (off < kTopcCap)) ? off : kTopcCap + tid] = K{val(e), (uint32_t)(base + koff(e))};
    off += l ? 1 : 0;
  }
  __syncthreads();
  int n = cnt;
  if (n > kTopcCap && g.topc_publish_only) {
    // warm-up tiles need no exact answer: t0 is at most the tile's C-th best
    // key, so it may stand in for it (and the tile appends nothing)
    if (tid == 0 && own >= 0) atomicMax(g.topc_thr, ord_key(double(lane_best[own].v)));
    return;
  }
  if (n <= kTopcCap) {
    for (int t = tid; t < n; t += NTHR) {
      const K k = cand[t];
      const int r = rank_of(cand, n, k);
      if (r < C) outk[r] = k;
    }
    n = n < C ? n : C;
  } else {
    int got = 0;
    for (int round = 0; round < C; ++round) {
      if (__ballot(live != 0) == 0) break;
      T rv = T(0);
      int rk = kNone, re = -1;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const T v = val(e);
        const int k = koff(e);
        const bool b = (bool)((live >> e) & 1) & ((rk == kNone) | (v > rv) | ((v == rv) & (k < rk)));
        rv = b ? v : rv;
        rk = b ? k : rk;
        re = b ? e : re;
      }
      const K best = re >= 0 ? K{rv, (uint32_t)(base + rk)} : tc_worst<T>();
      const K w = wave_best(best);
      if (lane == 0) wk[wave][got] = w;
      if (re >= 0 && best.i == w.i) live &= ~(1ull << re);
      ++got;
    }
    if (lane == 0) wn[wave] = got;
    __syncthreads();
    if (wave == 0) {
      // lane l holds key l of every wave's list
      uint32_t hl = 0;
      K h[NW];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        h[w] = tc_worst<T>();
        if (lane < wn[w]) {
          h[w] = wk[w][lane];
          hl |= 1u << w;
        }
      }
      int m = 0;
      for (; m < C; ++m) {
        if (__ballot(hl != 0) == 0) break;
        K best = tc_worst<T>();
        int bw = -1;
#pragma unroll
        for (int w = 0; w < NW; ++w)
          if (((hl >> w) & 1) && tc_better(h[w], best)) {
            best = h[w];
            bw = w;
          }
        const K win = wave_best(best);
        if (lane == 0) outk[m] = win;
        if (bw >= 0 && best.i == win.i) hl &= ~(1u << bw);
      }
      if (lane == 0) nfound = m;
    }
    __syncthreads();
    n = nfound;
  }
  __syncthreads();
  if (tid == 0) {
    if (n == C) atomicMax(g.topc_thr, ord_key(double(outk[C - 1].v)));
    nout = g.topc_publish_only == 1 ? 0 : n;
    obase = g.topc_publish_only == 1 ? 0 : atomicAdd(g.topc_count, (unsigned long long)n);
  }
  __syncthreads();
  for (int t = tid; t < nout; t += NTHR) {
    const K k = outk[t];
    g.topc_v[obase + t] = double(k.v);
    g.topc_i[obase + t] = (uint64_t)(z * g.sCz + (m0 + (k.i >> 7)) * g.ldc + n0 + (k.i & 127));
  }
}

// ---------------------------------------------------------------------------
// FP64
// ---------------------------------------------------------------------------
template <bool NT, bool TC>
__device__ __forceinline__ void gemm_f64_tile(const GemmArgs& g, int64_t vb) {
  // 8 waves in a 4 x 2 grid, 32 x 64 outputs each: two waves per SIMD hide
  // the load latency that one 64 x 64 wave per SIMD could not.
  constexpr int BM = 128, BN = 128, BK = 16;
  __shared__ __attribute__((aligned(16))) double As[BK][BM];
  __shared__ __attribute__((aligned(16))) double Bs[BK][BN];
  const TileCoord tc = tile_coord_v<BM, BN>(g, vb);
  const int64_t m0 = tc.m0, n0 = tc.n0;
  const double* A = static_cast<const double*>(g.A) + tc.z * g.sAz;
  const double* B = static_cast<const double*>(g.B) + tc.z * g.sBz;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  const int lr = tid >> 5, lc = (tid & 31) * 4;
  typedef double dv2 __attribute__((ext_vector_type(2)));

  d4_t acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  double ra[4], rb[4];
  load4(A, lr, g.sAk, m0 + lc, g.M, g.K, ra);
  load4(B, lr, g.sBk, n0 + lc, g.N, g.K, rb);
  for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; e += 2) {
      *reinterpret_cast<dv2*>(&As[lr][lc + e]) = dv2{ra[e], ra[e + 1]};
      *reinterpret_cast<dv2*>(&Bs[lr][lc + e]) = dv2{rb[e], rb[e + 1]};
    }
    __syncthreads();
    if (k0 + BK < g.K) {
      load4(A, k0 + BK + lr, g.sAk, m0 + lc, g.M, g.K, ra);
      load4(B, k0 + BK + lr, g.sBk, n0 + lc, g.N, g.K, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      if (kk >= g.K - k0) break;  // short K (outer products): skip all-zero steps
      double a[2], b[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  if constexpr (TC) {
    const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
    const int rem_m = (int)(g.M - m0 < BM ? g.M - m0 : BM), rem_n = (int)(g.N - n0 < BN ? g.N - n0 : BN);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][j][v] *= g.alpha;
    // f64 16x16x4 accumulators: item v of lane l is row l/16 + 4v, column l%16
    const int base = (wm + (lane >> 4)) * 128 + wn + (lane & 15);
    auto val = [&](int e) -> double { return acc[e >> 4][(e >> 2) & 3][e & 3]; };
    auto koff = [](int e) -> int { return ((e >> 4) * 16 + 4 * (e & 3)) * 128 + ((e >> 2) & 3) * 16; };
    auto valid = [&](int e) -> bool {
      const int i = e >> 4, j = (e >> 2) & 3, v = e & 3;
      return (wm + i * 16 + (lane >> 4) + 4 * v < rem_m) & (wn + j * 16 + (lane & 15) < rem_n);
    };
    topc_tile<double, 32, 512>(g, tc.z, m0, n0, full, val, koff, base, valid);
    return;
  }
  double* C = static_cast<double*>(g.C) + tc.z * g.sCz;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f64 16x16x4 accumulators: item v of lane l is row l/16 + 4v, column l%16
        const int64_t row = m0 + wm + i * 16 + (lane >> 4) + 4 * v;
        const int64_t col = n0 + wn + j * 16 + (lane & 15);
        if (row < g.M && col < g.N) store_out<double, NT>(&C[row * g.ldc + col], g.alpha * acc[i][j][v]);
      }
}

template <bool NT, bool TC = false>
__global__ void __launch_bounds__(512) gemm_f64_kernel(GemmArgs gv, const GemmArgs* __restrict__ gp,
                                                       int64_t gp_stride) {
  CQ_TILE_LOOP((gemm_f64_tile<NT, TC>(g, vb)))
}

// ---------------------------------------------------------------------------
// FP32
// ---------------------------------------------------------------------------
template <bool NT, bool TC>
__device__ __forceinline__ void gemm_f32_tile(const GemmArgs& g, int64_t vb) {
  constexpr int BM = 128, BN = 128, BK = 16;
  __shared__ __attribute__((aligned(16))) float As[BK][BM];
  __shared__ __attribute__((aligned(16))) float Bs[BK][BN];
  const TileCoord tc = tile_coord_v<BM, BN>(g, vb);
  const int64_t m0 = tc.m0, n0 = tc.n0;
  const float* A = static_cast<const float*>(g.A) + tc.z * g.sAz;
  const float* B = static_cast<const float*>(g.B) + tc.z * g.sBz;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int lr = tid >> 4, lc = (tid & 15) * 8;
  const float alpha = float(g.alpha);

  f16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  float ra[8], rb[8];
  load8(A, lr, g.sAk, m0 + lc, g.M, g.K, ra);
  load8(B, lr, g.sBk, n0 + lc, g.N, g.K, rb);
  for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();
    {
      typedef float fv4 __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int e = 0; e < 8; e += 4) {
        *reinterpret_cast<fv4*>(&As[lr][lc + e]) = fv4{ra[e], ra[e + 1], ra[e + 2], ra[e + 3]};
        *reinterpret_cast<fv4*>(&Bs[lr][lc + e]) = fv4{rb[e], rb[e + 1], rb[e + 2], rb[e + 3]};
      }
    }
    __syncthreads();
    if (k0 + BK < g.K) {
      load8(A, k0 + BK + lr, g.sAk, m0 + lc, g.M, g.K, ra);
      load8(B, k0 + BK + lr, g.sBk, n0 + lc, g.N, g.K, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      if (kk >= g.K - k0) break;  // short K (outer products): skip all-zero steps
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 5)][wm + i * 32 + (lane & 31)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 5)][wn + j * 32 + (lane & 31)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  if constexpr (TC) {
    const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
    const int rem_m = (int)(g.M - m0 < BM ? g.M - m0 : BM), rem_n = (int)(g.N - n0 < BN ? g.N - n0 : BN);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] *= alpha;
    // 32x32 accumulators: item v of lane l is row 8(v/4) + 4(l/32) + v%4, column l%32
    const int base = (wm + 4 * (lane >> 5)) * 128 + wn + (lane & 31);
    auto val = [&](int e) -> float { return acc[e >> 5][(e >> 4) & 1][e & 15]; };
    auto koff = [](int e) -> int {
      const int v = e & 15;
      return ((e >> 5) * 32 + 8 * (v >> 2) + (v & 3)) * 128 + ((e >> 4) & 1) * 32;
    };
    auto valid = [&](int e) -> bool {
      const int i = e >> 5, j = (e >> 4) & 1, v = e & 15;
      return (wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3) < rem_m) & (wn + j * 32 + (lane & 31) < rem_n);
    };
    topc_tile<float, 64, 256>(g, tc.z, m0, n0, full, val, koff, base, valid);
    return;
  }
  float* C = static_cast<float*>(g.C) + tc.z * g.sCz;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int64_t col = n0 + wn + j * 32 + (lane & 31);
        if (row < g.M && col < g.N) store_out<float, NT>(&C[row * g.ldc + col], alpha * acc[i][j][v]);
      }
}

template <bool NT, bool TC = false>
__global__ void __launch_bounds__(256) gemm_f32_kernel(GemmArgs gv, const GemmArgs* __restrict__ gp,
                                                       int64_t gp_stride) {
  CQ_TILE_LOOP((gemm_f32_tile<NT, TC>(g, vb)))
}

// ---------------------------------------------------------------------------
// BF16 / FP16 with FP32 accumulation.  SPLIT = 3 issues hi*hi + hi*lo + lo*hi.
// OUT: 0 = FP32, 1 = FP32 non-temporal, 2 = 16-bit planes (hi, and lo when
// split), 3 = fused top-C (no store)
// ---------------------------------------------------------------------------
template <bool F16>
struct Half;
template <>
struct Half<false> {
  typedef __bf16 T;
  typedef __bf16 V8 __attribute__((ext_vector_type(8)));
  static __device__ inline f16_t mfma(V8 a, V8 b, f16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Half<true> {
  typedef _Float16 T;
  typedef _Float16 V8 __attribute__((ext_vector_type(8)));
  static __device__ inline f16_t mfma(V8 a, V8 b, f16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// Row k, columns c0..c0+7 of a 16-bit plane, packed two per dword.
__device__ inline u32x4 load_row8_h(const uint16_t* __restrict__ P, int64_t k, int64_t sk,
                                    int64_t c0, int64_t ncols, int64_t K) {
  u32x4 v = {0u, 0u, 0u, 0u};
  if (k >= K) return v;
  const uint16_t* p = P + k * sk + c0;
  if (c0 + 8 <= ncols && ((reinterpret_cast<uintptr_t>(p) & 15) == 0))
    return *reinterpret_cast<const u32x4*>(p);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t lo = (c0 + 2 * j < ncols) ? p[2 * j] : 0u;
    const uint32_t hi = (c0 + 2 * j + 1 < ncols) ? p[2 * j + 1] : 0u;
    v[j] = lo | (hi << 16);
  }
  return v;
}

// r[e] holds row e (8 columns); o[c] receives column c (8 rows).
__device__ inline void transpose8x8(const u32x4 (&r)[8], u32x4 (&o)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t x = r[2 * i][c >> 1], y = r[2 * i + 1][c >> 1];
      o[c][i] = (c & 1) ? ((x >> 16) | (y & 0xffff0000u)) : ((x & 0xffffu) | (y << 16));
    }
}

template <bool F16>
__device__ inline uint16_t to_h16(float x) {
  return __builtin_bit_cast(uint16_t, typename Half<F16>::T(x));
}

template <bool F16>
__device__ inline float from_h16(uint16_t x) {
  return float(__builtin_bit_cast(typename Half<F16>::T, x));
}

template <int SPLIT, bool F16, int OUT>
__device__ __forceinline__ void gemm_h16_tile(const GemmArgs& g, int64_t vb) {
  using H = Half<F16>;
  using V8 = typename H::V8;
  constexpr int BM = 128, BN = 128, BK = 64, LDK = BK + 8;
  constexpr int NP = SPLIT == 3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) uint16_t As[NP][BM][LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[NP][BN][LDK];
  const TileCoord tc = tile_coord_v<BM, BN>(g, vb);
  const int64_t m0 = tc.m0, n0 = tc.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  // loader: waves 0-1 fetch A, waves 2-3 fetch B.  Each lane owns an
  // 8 (label) x 8 (column) block; lanes 8j..8j+7 hold the 8 label groups of
  // one column group, so the transposed LDS writes of 16 consecutive lanes
  // fill two whole 128-byte rows (no bank conflicts) and every global load
  // instruction reads 8 full 128-byte row segments.
  const bool ldA = tid < 128;
  const int lk = (lane & 7) * 8;
  const int lc = ((lane >> 3) + 8 * ((tid >> 6) & 1)) * 8;
  const int64_t zoff = tc.z * (ldA ? g.sAz : g.sBz);
  const uint16_t* P[NP];
  P[0] = static_cast<const uint16_t*>(ldA ? g.A : g.B) + zoff;
  if constexpr (NP == 2) P[NP - 1] = static_cast<const uint16_t*>(ldA ? g.A_lo : g.B_lo) + zoff;
  const int64_t lsk = ldA ? g.sAk : g.sBk;
  const int64_t lcol = (ldA ? m0 : n0) + lc;
  const int64_t lncols = ldA ? g.M : g.N;
  uint16_t (*S)[BM][LDK] = ldA ? As : Bs;
  // whole 8-column segment in range and 16-byte aligned for every row
  bool vec_ok = lcol + 8 <= lncols && ((lsk & 7) == 0);
#pragma unroll
  for (int p = 0; p < NP; ++p) vec_ok = vec_ok && ((reinterpret_cast<uintptr_t>(P[p] + lcol) & 15) == 0);

  f16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  u32x4 rows[NP][8];
  auto load = [&](int64_t k0) {
    if (vec_ok && k0 + BK <= g.K) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const uint16_t* base = P[p] + (k0 + lk) * lsk + lcol;
#pragma unroll
        for (int e = 0; e < 8; ++e) rows[p][e] = *reinterpret_cast<const u32x4*>(base + e * lsk);
      }
    } else {
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int e = 0; e < 8; ++e) rows[p][e] = load_row8_h(P[p], k0 + lk + e, lsk, lcol, lncols, g.K);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      u32x4 cols[8];
      transpose8x8(rows[p], cols);
#pragma unroll
      for (int c = 0; c < 8; ++c) *reinterpret_cast<u32x4*>(&S[p][lc + c][lk]) = cols[c];
    }
  };

  load(0);
  for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BK < g.K) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      if (kk >= g.K - k0) break;  // short K (outer products): skip all-zero steps
      const int kc = kk + 8 * (lane >> 5);
      V8 a[NP][2], b[NP][2];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[p][i] = __builtin_bit_cast(V8, *reinterpret_cast<const u32x4*>(&As[p][wm + i * 32 + (lane & 31)][kc]));
          b[p][i] = __builtin_bit_cast(V8, *reinterpret_cast<const u32x4*>(&Bs[p][wn + i * 32 + (lane & 31)][kc]));
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = H::mfma(a[0][i], b[0][j], acc[i][j]);
          if constexpr (SPLIT == 3) {
            acc[i][j] = H::mfma(a[0][i], b[NP - 1][j], acc[i][j]);
            acc[i][j] = H::mfma(a[NP - 1][i], b[0][j], acc[i][j]);
          }
        }
    }
  }
  const float alpha = float(g.alpha);
  if constexpr (OUT == 3) {
    const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
    const int rem_m = (int)(g.M - m0 < BM ? g.M - m0 : BM), rem_n = (int)(g.N - n0 < BN ? g.N - n0 : BN);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] *= alpha;
    if (g.rowexp) {
      // column-scaled operands: the output exponents first, as the store applies them
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int rr = wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int cc = wn + j * 32 + (lane & 31);
            if ((rr < rem_m) & (cc < rem_n))
              acc[i][j][v] = __builtin_ldexpf(acc[i][j][v], g.rowexp[tc.z * g.M + m0 + rr] + g.colexp[n0 + cc]);
          }
    }
    // 32x32 accumulators: item v of lane l is row 8(v/4) + 4(l/32) + v%4, column l%32
    const int base = (wm + 4 * (lane >> 5)) * 128 + wn + (lane & 31);
    auto val = [&](int e) -> float { return acc[e >> 5][(e >> 4) & 1][e & 15]; };
    auto koff = [](int e) -> int {
      const int v = e & 15;
      return ((e >> 5) * 32 + 8 * (v >> 2) + (v & 3)) * 128 + ((e >> 4) & 1) * 32;
    };
    auto valid = [&](int e) -> bool {
      const int i = e >> 5, j = (e >> 4) & 1, v = e & 15;
      return (wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3) < rem_m) & (wn + j * 32 + (lane & 31) < rem_n);
    };
    topc_tile<float, 64, 256>(g, tc.z, m0, n0, full, val, koff, base, valid);
    return;
  }
  const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
  const int64_t cbase = tc.z * g.sCz + (m0 + wm + 4 * (lane >> 5)) * g.ldc + n0 + wn + (lane & 31);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rr = i * 32 + 8 * (v >> 2) + (v & 3);
        const int cc = j * 32;
        if (full || (m0 + wm + 4 * (lane >> 5) + rr < g.M && n0 + wn + (lane & 31) + cc < g.N)) {
          const int64_t idx = cbase + rr * g.ldc + cc;
          float x = alpha * acc[i][j][v];
          if constexpr (OUT != 2) {
            if (g.rowexp)
              x = __builtin_ldexpf(x, g.rowexp[tc.z * g.M + m0 + wm + 4 * (lane >> 5) + rr] +
                                          g.colexp[n0 + wn + (lane & 31) + cc]);
          }
          if constexpr (OUT == 2) {
            const uint16_t h = to_h16<F16>(x);
            static_cast<uint16_t*>(g.C)[idx] = h;
            if constexpr (SPLIT == 3) static_cast<uint16_t*>(g.C_lo)[idx] = to_h16<F16>(x - from_h16<F16>(h));
          } else {
            store_out<float, OUT == 1>(static_cast<float*>(g.C) + idx, x);
          }
        }
      }
}

template <int SPLIT, bool F16, int OUT>
__global__ void __launch_bounds__(256, SPLIT == 3 ? 1 : 2) gemm_h16_kernel(GemmArgs gv,
                                                                           const GemmArgs* __restrict__ gp,
                                                                           int64_t gp_stride) {
  CQ_TILE_LOOP((gemm_h16_tile<SPLIT, F16, OUT>(g, vb)))
}


// ---------------------------------------------------------------------------
// 16-bit path, asynchronous form (used when every operand row is 16-byte
// aligned and at least 8 columns wide).  Operand tiles go global -> LDS with
// global_load_lds_dwordx4 (no register staging) into NS rotating stages in
// the operands' own [label][column] layout; ds_read_b64_tr_b16 then returns
// each lane's k-contiguous MFMA operand (within a group of 16 lanes, slot j of
// lane i is word i%4 of the address given by lane 4j + i/4).  LDS rows are
// 128 columns (256 B) whose 16-byte chunks are XOR-swizzled by 4*(row & 3)
// (swz), so the 32 lanes of a half-wave's transposed reads -- four rows, two
// 32-column groups -- cover all 64 banks once.  Results are
// staged through LDS per wave so each global store instruction writes whole
// 256-byte row segments.  The DMA is issued from asm: the compiler would
// otherwise wait for every in-flight LDS DMA before each LDS read; completion
// is tracked with explicit vmcnt waits instead (a wave's vector memory
// operations retire in issue order).
// ---------------------------------------------------------------------------
#define CQ_GLOBAL __attribute__((address_space(1)))
#define CQ_LDS __attribute__((address_space(3)))

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ inline int swz(int row, int chunk) { return chunk ^ ((row & 3) << 2); }

// s_waitcnt vmcnt(N) lgkmcnt(0)
template <int N>
__device__ inline void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (0 << 8));
}

// s_waitcnt vmcnt(n) for a wave-uniform n (above 63: 63, which waits longer).
// An asm statement with a memory clobber, so no memory access moves across it.
__device__ inline void wait_vm_n(int n) {
#define CQ_W4(b)                                                       \
  case b: asm volatile("s_waitcnt vmcnt(" #b ")" ::: "memory"); break; \
  case b + 1: asm volatile("s_waitcnt vmcnt(" #b " + 1)" ::: "memory"); break; \
  case b + 2: asm volatile("s_waitcnt vmcnt(" #b " + 2)" ::: "memory"); break; \
  case b + 3: asm volatile("s_waitcnt vmcnt(" #b " + 3)" ::: "memory"); break;
  switch (n < 0 ? 0 : (n > 63 ? 63 : n)) {
    CQ_W4(0) CQ_W4(4) CQ_W4(8) CQ_W4(12) CQ_W4(16) CQ_W4(20) CQ_W4(24) CQ_W4(28)
    CQ_W4(32) CQ_W4(36) CQ_W4(40) CQ_W4(44) CQ_W4(48) CQ_W4(52) CQ_W4(56) CQ_W4(60)
  }
#undef CQ_W4
}

template <int SPLIT, bool F16, int OUT, int NS>
__global__ void __launch_bounds__(256) gemm_h16a_kernel(GemmArgs gv, const GemmArgs* __restrict__ gp,
                                                        int64_t gp_stride) {
  CQ_LOAD_GEMM_ARGS
  using H = Half<F16>;
  using V8 = typename H::V8;
  constexpr int BM = 128, BN = 128, BK = 32;
  constexpr int NP = SPLIT == 3 ? 2 : 1;
  constexpr int TILE = BK * 256;        // bytes of one operand-plane stage
  constexpr int STAGE = TILE * 2 * NP;  // A and B, all planes
  constexpr int LPW = 2 * 2 * NP;       // DMA instructions per wave per stage
  // the hand-counted vmcnt waits below assume LPW DMA loads per stage; the
  // build checks the assembly against this marker
  asm volatile("; cq-vm-lpw %0" ::"n"(LPW));
  constexpr int EROW = 288;             // bytes per staged output row (64 floats + pad)
  constexpr int EPI = 4 * 64 * EROW;
  constexpr int SMEM = NS * STAGE > EPI ? NS * STAGE : EPI;
  static_assert(NS >= 2 && NS <= 3, "stage count");
  __shared__ __attribute__((aligned(16))) char smem[SMEM];
  CQ_LDS char* const lsm = (CQ_LDS char*)smem;
  const TileCoord tc = tile_coord<BM, BN>(g);
  const int64_t m0 = tc.m0, n0 = tc.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int nstages = (int)((g.K + BK - 1) / BK);

  const uint16_t* gbase[2][NP];
  int64_t gsk[2], ccap[2];
  {
    const int64_t za = tc.z * g.sAz, zb = tc.z * g.sBz;
    gbase[0][0] = static_cast<const uint16_t*>(g.A) + za + m0;
    gbase[1][0] = static_cast<const uint16_t*>(g.B) + zb + n0;
    if constexpr (NP == 2) {
      gbase[0][NP - 1] = static_cast<const uint16_t*>(g.A_lo) + za + m0;
      gbase[1][NP - 1] = static_cast<const uint16_t*>(g.B_lo) + zb + n0;
    }
    gsk[0] = g.sAk;
    gsk[1] = g.sBk;
    // last 8-column chunk that stays inside the operand (M, N >= 8)
    ccap[0] = ((g.M - 8) & ~(int64_t)7) - m0;
    ccap[1] = ((g.N - 8) & ~(int64_t)7) - n0;
  }
  // wave w, instruction q fill LDS rows 4*(2w+q) .. +3 of every operand plane
  auto issue = [&](int s) {
    const int64_t k0 = (int64_t)s * BK;
#pragma unroll
    for (int op = 0; op < 2; ++op)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int chunk0 = (wave * 2 + q) * 64;
          const int pc = chunk0 + lane;
          const int row = pc >> 4;
          int64_t col = (int64_t)swz(row, pc & 15) * 8;
          if (col > ccap[op]) col = ccap[op];
          int64_t k = k0 + row;
          if (k >= g.K) k = g.K - 1;  // rows past K are masked to zero when read
          const uint16_t* src = gbase[op][p] + k * gsk[op] + col;
          const uint32_t dst = __builtin_amdgcn_readfirstlane(
              (uint32_t)(uintptr_t)(lsm + (s % NS) * STAGE + (op * NP + p) * TILE + chunk0 * 16));
          asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(dst)
                       : "memory", "m0");
        }
  };

  f16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  // transposed-read coordinates of this lane inside a 32-column operand block
  const int grp = lane >> 4, r16 = lane & 15;
  const int col_in_blk = 16 * (grp & 1) + 4 * (r16 & 3);
  const int krow = 8 * (grp >> 1) + (r16 >> 2);
  auto frag = [&](int tile, int kk, int c0, int64_t kvalid) -> V8 {
    const int col = c0 + col_in_blk;
    const int r0 = kk + krow, r1 = r0 + 4;
    const int o0 = tile + r0 * 256 + (swz(r0, col >> 3) << 4) + (col & 7) * 2;
    const int o1 = tile + r1 * 256 + (swz(r1, col >> 3) << 4) + (col & 7) * 2;
    s4_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((CQ_LDS s4_t*)(lsm + o0));
    s4_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((CQ_LDS s4_t*)(lsm + o1));
    if (kvalid < BK) {
      // slot e of the two reads holds label kk + 8*(grp>>1) + e (+4)
      const int kb = kk + 8 * (grp >> 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (kb + e >= kvalid) lo[e] = 0;
        if (kb + 4 + e >= kvalid) hi[e] = 0;
      }
    }
    typedef short s8_t __attribute__((ext_vector_type(8)));
    const s8_t v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(V8, v);
  };

  for (int s = 0; s < NS - 1 && s < nstages; ++s) issue(s);
  for (int s = 0; s < nstages; ++s) {
    // this wave's loads of stage s have landed once at most `ahead` later
    // stages are outstanding; the barrier then covers every wave's loads
    const int ahead = (nstages - 1 - s) < (NS - 2) ? (nstages - 1 - s) : (NS - 2);
    if (ahead >= 1) wait_vm<LPW>();
    else wait_vm<0>();
    __syncthreads();
    if (s + NS - 1 < nstages) issue(s + NS - 1);
    const int sb = (s % NS) * STAGE;
    const int64_t kvalid = g.K - (int64_t)s * BK;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      V8 a[NP][2], b[NP][2];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[p][i] = frag(sb + (0 * NP + p) * TILE, kk, wm + 32 * i, kvalid);
          b[p][i] = frag(sb + (1 * NP + p) * TILE, kk, wn + 32 * i, kvalid);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = H::mfma(a[0][i], b[0][j], acc[i][j]);
          if constexpr (SPLIT == 3) {
            acc[i][j] = H::mfma(a[0][i], b[NP - 1][j], acc[i][j]);
            acc[i][j] = H::mfma(a[NP - 1][i], b[0][j], acc[i][j]);
          }
        }
    }
  }

  // epilogue: each wave stages its 64 x 64 results in LDS, then every store
  // instruction writes four whole rows of 64 values
  const float alpha = float(g.alpha);
  __syncthreads();
  char* wbuf = smem + wave * 64 * EROW;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int c = 32 * j + (lane & 31);
        *reinterpret_cast<float*>(wbuf + r * EROW + c * 4) = alpha * acc[i][j][v];
      }
  __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0)
  const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
  // column-scaled operands: a lane's four columns are the same in every row
  // it stores, so their exponents are read once
  int32_t cexp[4] = {0, 0, 0, 0};
  if constexpr (OUT != 2) {
    if (g.rowexp) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t n = n0 + wn + 4 * (lane & 15) + e;
        if (n < g.N) cexp[e] = g.colexp[n];
      }
    }
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int r = 4 * s + (lane >> 4);
    const int c = 4 * (lane & 15);
    f4_t x = *reinterpret_cast<const f4_t*>(wbuf + r * EROW + c * 4);
    const int64_t m = m0 + wm + r, n = n0 + wn + c;
    const int64_t idx = tc.z * g.sCz + m * g.ldc + n;
    if constexpr (OUT != 2) {
      if (g.rowexp && m < g.M) {
        const int32_t re = g.rowexp[tc.z * g.M + m];
#pragma unroll
        for (int e = 0; e < 4; ++e) x[e] = __builtin_ldexpf(x[e], re + cexp[e]);
      }
    }
    if (full || (m < g.M && n + 3 < g.N)) {
      if constexpr (OUT == 2) {
        typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
        u16x4 h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          h[e] = to_h16<F16>(x[e]);
          l[e] = to_h16<F16>(x[e] - from_h16<F16>(h[e]));
        }
        *reinterpret_cast<u16x4*>(static_cast<uint16_t*>(g.C) + idx) = h;
        if constexpr (SPLIT == 3) *reinterpret_cast<u16x4*>(static_cast<uint16_t*>(g.C_lo) + idx) = l;
      } else {
        store_out<f4_t, OUT == 1>(reinterpret_cast<f4_t*>(static_cast<float*>(g.C) + idx), x);
      }
    } else if (m < g.M) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (n + e < g.N) {
          if constexpr (OUT == 2) {
            const uint16_t h = to_h16<F16>(x[e]);
            static_cast<uint16_t*>(g.C)[idx + e] = h;
            if constexpr (SPLIT == 3) static_cast<uint16_t*>(g.C_lo)[idx + e] = to_h16<F16>(x[e] - from_h16<F16>(h));
          } else {
            store_out<float, OUT == 1>(static_cast<float*>(g.C) + idx + e, x[e]);
          }
        }
    }
  }
}

// ---------------------------------------------------------------------------
// 16-bit path, occupancy form: one 128 x 128 tile per workgroup like
// gemm_h16a_kernel, but sized for three or four resident workgroups per CU
// (WPE waves per SIMD).  Stages hold 16 labels (16 KB for split operands) in
// an NS-deep ring; the epilogue goes through the ring in 8-row slabs per wave,
// so the kernel needs NS x 16 KB of LDS in all.  Each k-step loads a wave's
// B fragments once and its A fragments one 32-row block at a time, which
// keeps the live registers within the occupancy budget.  The operand DMA,
// transposed fragment reads and product order are those of gemm_h16a_kernel,
// so the sums are the same bit for bit.  Operand stages are the latency the
// kernel hides: with more workgroups resident, one workgroup's wait for its
// next stage overlaps another's products and stores.
// ---------------------------------------------------------------------------
template <int SPLIT, bool F16, int OUT, int NS, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
gemm_h16t_kernel(GemmArgs g) {
  using H = Half<F16>;
  using V8 = typename H::V8;
  constexpr int BM = 128, BN = 128, BK = 16;
  constexpr int NP = SPLIT == 3 ? 2 : 1;
  constexpr int TILE = BK * 256;        // bytes of one operand-plane stage
  constexpr int STAGE = TILE * 2 * NP;  // A and B, all planes
  constexpr int LPW = 2 * NP;           // DMA instructions per wave per stage
  // the hand-counted vmcnt waits below assume LPW DMA loads per stage; the
  // build checks the assembly against this marker
  asm volatile("; cq-vm-lpw %0" ::"n"(LPW));
  constexpr int EROW = 288;             // bytes per staged output row (64 floats + pad)
  constexpr int EPI = 4 * 8 * EROW;
  constexpr int SMEM = NS * STAGE > EPI ? NS * STAGE : EPI;
  static_assert(NS >= 2 && NS <= 4, "stage count");
  __shared__ __attribute__((aligned(16))) char smem[SMEM];
  CQ_LDS char* const lsm = (CQ_LDS char*)smem;
  const TileCoord tc = tile_coord<BM, BN>(g);
  const int64_t m0 = tc.m0, n0 = tc.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int nstages = (int)((g.K + BK - 1) / BK);
  // wave w's instruction for (operand, plane) fills rows 4w .. 4w + 3
  const uint16_t* gbase[2][NP];
  int64_t ccap[2];
  {
    const int64_t za = tc.z * g.sAz, zb = tc.z * g.sBz;
    gbase[0][0] = static_cast<const uint16_t*>(g.A) + za + m0;
    gbase[1][0] = static_cast<const uint16_t*>(g.B) + zb + n0;
    if constexpr (NP == 2) {
      gbase[0][NP - 1] = static_cast<const uint16_t*>(g.A_lo) + za + m0;
      gbase[1][NP - 1] = static_cast<const uint16_t*>(g.B_lo) + zb + n0;
    }
    ccap[0] = ((g.M - 8) & ~(int64_t)7) - m0;
    ccap[1] = ((g.N - 8) & ~(int64_t)7) - n0;
  }
  const int pc = wave * 64 + lane;  // 16-byte chunk of the stage plane this lane fills
  const int lrow = pc >> 4;
  int64_t lcol[2];
#pragma unroll
  for (int op = 0; op < 2; ++op) {
    lcol[op] = (int64_t)swz(lrow, pc & 15) * 8;
    if (lcol[op] > ccap[op]) lcol[op] = ccap[op];
  }
  auto issue = [&](int s) {
    int64_t k = (int64_t)s * BK + lrow;
    if (k >= g.K) k = g.K - 1;  // rows past K are masked to zero when read
#pragma unroll
    for (int op = 0; op < 2; ++op)
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const uint16_t* src = gbase[op][p] + k * (op ? g.sBk : g.sAk) + lcol[op];
        const uint32_t dst = __builtin_amdgcn_readfirstlane(
            (uint32_t)(uintptr_t)(lsm + (s % NS) * STAGE + (op * NP + p) * TILE + wave * 1024));
        asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(dst)
                     : "memory", "m0");
      }
  };
  f16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  const int grp = lane >> 4, r16 = lane & 15;
  const int col_in_blk = 16 * (grp & 1) + 4 * (r16 & 3);
  const int krow = 8 * (grp >> 1) + (r16 >> 2);
  auto frag = [&](int tile, int c0, int64_t kvalid) -> V8 {
    const int col = c0 + col_in_blk;
    const int r0 = krow, r1 = r0 + 4;
    const int o0 = tile + r0 * 256 + (swz(r0, col >> 3) << 4) + (col & 7) * 2;
    const int o1 = tile + r1 * 256 + (swz(r1, col >> 3) << 4) + (col & 7) * 2;
    s4_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((CQ_LDS s4_t*)(lsm + o0));
    s4_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((CQ_LDS s4_t*)(lsm + o1));
    if (kvalid < BK) {
      // slot e of the two reads holds label 8*(grp>>1) + e (+4)
      const int kb = 8 * (grp >> 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (kb + e >= kvalid) lo[e] = 0;
        if (kb + 4 + e >= kvalid) hi[e] = 0;
      }
    }
    typedef short s8_t __attribute__((ext_vector_type(8)));
    const s8_t v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(V8, v);
  };

  for (int s = 0; s < NS - 1 && s < nstages; ++s) issue(s);
  for (int s = 0; s < nstages; ++s) {
    // this wave's loads of stage s have landed once at most `ahead` later
    // stages are outstanding; the barrier then covers every wave's loads
    const int ahead = (nstages - 1 - s) < (NS - 2) ? (nstages - 1 - s) : (NS - 2);
    if (ahead >= 2) wait_vm<2 * LPW>();
    else if (ahead == 1) wait_vm<LPW>();
    else wait_vm<0>();
    __syncthreads();
    if (s + NS - 1 < nstages) issue(s + NS - 1);
    const int sb = (s % NS) * STAGE;
    const int64_t kvalid = g.K - (int64_t)s * BK;
    V8 b[NP][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int j = 0; j < 2; ++j) b[p][j] = frag(sb + (1 * NP + p) * TILE, wn + 32 * j, kvalid);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      V8 a[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) a[p] = frag(sb + (0 * NP + p) * TILE, wm + 32 * i, kvalid);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = H::mfma(a[0], b[0][j], acc[i][j]);
        if constexpr (SPLIT == 3) {
          acc[i][j] = H::mfma(a[0], b[NP - 1][j], acc[i][j]);
          acc[i][j] = H::mfma(a[NP - 1], b[0][j], acc[i][j]);
        }
      }
      // keep the second block's fragment reads after the first block's products
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // epilogue: slab u of a wave holds rows 32*(u>>2) + 8*(u&3) .. +7 of its
  // 64 x 64 block; it is staged in the ring so that every store instruction
  // writes whole row segments
  const float alpha = float(g.alpha);
  __syncthreads();  // every wave is done with the ring
  char* const wbuf = smem + wave * 8 * EROW;
  const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
  // column-scaled operands: a lane's four columns are the same in every
  // slab, so their exponents are read once
  int32_t cexp[4] = {0, 0, 0, 0};
  if constexpr (OUT != 2) {
    if (g.rowexp) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t n = n0 + wn + 4 * (lane & 15) + e;
        if (n < g.N) cexp[e] = g.colexp[n];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = u >> 2, vg = u & 3;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 4 * (lane >> 5) + e;
        const int c = 32 * j + (lane & 31);
        *reinterpret_cast<float*>(wbuf + r * EROW + c * 4) = alpha * acc[i][j][4 * vg + e];
      }
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rl = 4 * h + (lane >> 4);
      const int c = 4 * (lane & 15);
      f4_t x = *reinterpret_cast<const f4_t*>(wbuf + rl * EROW + c * 4);
      const int64_t m = m0 + wm + 32 * i + 8 * vg + rl, n = n0 + wn + c;
      const int64_t idx = tc.z * g.sCz + m * g.ldc + n;
      if constexpr (OUT != 2) {
        // column-scaled operands: the output exponents, after alpha as in the other forms
        if (g.rowexp && m < g.M) {
          const int32_t re = g.rowexp[tc.z * g.M + m];
#pragma unroll
          for (int e = 0; e < 4; ++e) x[e] = __builtin_ldexpf(x[e], re + cexp[e]);
        }
      }
      if constexpr (OUT == 2) {
        typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
        u16x4 hh, ll;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          hh[e] = to_h16<F16>(x[e]);
          ll[e] = to_h16<F16>(x[e] - from_h16<F16>(hh[e]));
        }
        uint16_t* const ch = static_cast<uint16_t*>(g.C);
        uint16_t* const cl = static_cast<uint16_t*>(g.C_lo);
        if (full || (m < g.M && n + 3 < g.N)) {
          *reinterpret_cast<u16x4*>(ch + idx) = hh;
          if (cl) *reinterpret_cast<u16x4*>(cl + idx) = ll;
        } else if (m < g.M) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (n + e < g.N) {
              ch[idx + e] = hh[e];
              if (cl) cl[idx + e] = ll[e];
            }
        }
      } else if (full || (m < g.M && n + 3 < g.N)) {
        store_out<f4_t, OUT == 1>(reinterpret_cast<f4_t*>(static_cast<float*>(g.C) + idx), x);
      } else if (m < g.M) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e < g.N) store_out<float, OUT == 1>(static_cast<float*>(g.C) + idx + e, x[e]);
      }
    }
    // the slab's LDS reads are done before the next slab overwrites it
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));
  }
}

// ---------------------------------------------------------------------------
// 16-bit operands, 64 x 64 tiles: for GEMMs with few 128 x 128 tiles.  Each
// wave owns one 32 x 32 block; stages hold 32 labels in rows of 64 elements
// (128 bytes) in an NS-deep ring, one DMA instruction per wave and plane
// filling eight rows, 16-byte chunks of row r at slot chunk ^ (r & 7).  The
// transposed fragment reads, the product order (per block and 16-label step:
// hi*hi, then hi*lo, then lo*hi) and the masking of labels past K are those of
// gemm_h16t_kernel, which runs no step that lies wholly past K, so the sums
// are the same bit for bit; results are stored from registers.
// ---------------------------------------------------------------------------
__device__ inline int swz8(int row, int chunk) { return chunk ^ (row & 7); }

template <int SPLIT, bool F16, int OUT, int NS>
__global__ void __launch_bounds__(256) gemm_h16s_kernel(GemmArgs g) {
  using H = Half<F16>;
  using V8 = typename H::V8;
  constexpr int BM = 64, BN = 64, BK = 32;
  constexpr int NP = SPLIT == 3 ? 2 : 1;
  constexpr int TILE = BK * 128;        // bytes of one operand-plane stage
  constexpr int STAGE = TILE * 2 * NP;  // A and B, all planes
  constexpr int LPW = 2 * NP;           // DMA instructions per wave per stage
  // the hand-counted vmcnt waits below assume LPW DMA loads per stage; the
  // build checks the assembly against this marker
  asm volatile("; cq-vm-lpw %0" ::"n"(LPW));
  static_assert(NS >= 2 && NS <= 4, "stage count");
  __shared__ __attribute__((aligned(16))) char smem[NS * STAGE];
  CQ_LDS char* const lsm = (CQ_LDS char*)smem;
  const TileCoord tc = tile_coord<BM, BN>(g);
  const int64_t m0 = tc.m0, n0 = tc.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int nstages = (int)((g.K + BK - 1) / BK);
  // wave w's instruction for (operand, plane) fills rows 8w .. 8w + 7
  const uint16_t* gbase[2][NP];
  int64_t ccap[2];
  {
    const int64_t za = tc.z * g.sAz, zb = tc.z * g.sBz;
    gbase[0][0] = static_cast<const uint16_t*>(g.A) + za + m0;
    gbase[1][0] = static_cast<const uint16_t*>(g.B) + zb + n0;
    if constexpr (NP == 2) {
      gbase[0][NP - 1] = static_cast<const uint16_t*>(g.A_lo) + za + m0;
      gbase[1][NP - 1] = static_cast<const uint16_t*>(g.B_lo) + zb + n0;
    }
    ccap[0] = ((g.M - 8) & ~(int64_t)7) - m0;
    ccap[1] = ((g.N - 8) & ~(int64_t)7) - n0;
  }
  const int lrow = 8 * wave + (lane >> 3);
  int64_t lcol[2];
#pragma unroll
  for (int op = 0; op < 2; ++op) {
    lcol[op] = (int64_t)swz8(lrow, lane & 7) * 8;
    if (lcol[op] > ccap[op]) lcol[op] = ccap[op];
  }
  auto issue = [&](int s) {
    int64_t k = (int64_t)s * BK + lrow;
    if (k >= g.K) k = g.K - 1;  // rows past K are masked to zero when read
#pragma unroll
    for (int op = 0; op < 2; ++op)
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const uint16_t* src = gbase[op][p] + k * (op ? g.sBk : g.sAk) + lcol[op];
        const uint32_t dst = __builtin_amdgcn_readfirstlane(
            (uint32_t)(uintptr_t)(lsm + (s % NS) * STAGE + (op * NP + p) * TILE + wave * 1024));
        asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(dst)
                     : "memory", "m0");
      }
  };
  f16_t acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  const int grp = lane >> 4, r16 = lane & 15;
  const int col_in_blk = 16 * (grp & 1) + 4 * (r16 & 3);
  const int krow = 8 * (grp >> 1) + (r16 >> 2);
  auto frag = [&](int tile, int kk, int c0, int64_t kvalid) -> V8 {
    const int col = c0 + col_in_blk;
    const int r0 = kk + krow, r1 = r0 + 4;
    const int o0 = tile + r0 * 128 + (swz8(r0, col >> 3) << 4) + (col & 7) * 2;
    const int o1 = tile + r1 * 128 + (swz8(r1, col >> 3) << 4) + (col & 7) * 2;
    s4_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((CQ_LDS s4_t*)(lsm + o0));
    s4_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((CQ_LDS s4_t*)(lsm + o1));
    if (kvalid < kk + 16) {
      // slot e of the two reads holds label kk + 8*(grp>>1) + e (+4)
      const int kb = kk + 8 * (grp >> 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (kb + e >= kvalid) lo[e] = 0;
        if (kb + 4 + e >= kvalid) hi[e] = 0;
      }
    }
    typedef short s8_t __attribute__((ext_vector_type(8)));
    const s8_t v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(V8, v);
  };

  for (int s = 0; s < NS - 1 && s < nstages; ++s) issue(s);
  for (int s = 0; s < nstages; ++s) {
    // this wave's loads of stage s have landed once at most `ahead` later
    // stages are outstanding; the barrier then covers every wave's loads
    const int ahead = (nstages - 1 - s) < (NS - 2) ? (nstages - 1 - s) : (NS - 2);
    if (ahead >= 2) wait_vm<2 * LPW>();
    else if (ahead == 1) wait_vm<LPW>();
    else wait_vm<0>();
    __syncthreads();
    if (s + NS - 1 < nstages) issue(s + NS - 1);
    const int sb = (s % NS) * STAGE;
    const int64_t kvalid = g.K - (int64_t)s * BK;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      if (kk >= kvalid) break;  // a 16-label step wholly past K
      V8 a[NP], b[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        a[p] = frag(sb + (0 * NP + p) * TILE, kk, wm, kvalid);
        b[p] = frag(sb + (1 * NP + p) * TILE, kk, wn, kvalid);
      }
      acc = H::mfma(a[0], b[0], acc);
      if constexpr (SPLIT == 3) {
        acc = H::mfma(a[0], b[NP - 1], acc);
        acc = H::mfma(a[NP - 1], b[0], acc);
      }
    }
  }

  const float alpha = float(g.alpha);
  const int r = lane >> 5, c = lane & 31;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t m = m0 + wm + 8 * (v >> 2) + 4 * r + (v & 3), n = n0 + wn + c;
    if (m < g.M && n < g.N) {
      const float x = alpha * acc[v];
      const int64_t idx = tc.z * g.sCz + m * g.ldc + n;
      if constexpr (OUT == 2) {
        const uint16_t h = to_h16<F16>(x);
        static_cast<uint16_t*>(g.C)[idx] = h;
        if (g.C_lo) static_cast<uint16_t*>(g.C_lo)[idx] = to_h16<F16>(x - from_h16<F16>(h));
      } else {
        store_out<float, OUT == 1>(static_cast<float*>(g.C) + idx, x);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 operands, occupancy form.  The persistent FP32 kernel keeps a finished
// tile in registers while the next one runs (two waves per SIMD).  This form
// takes one 128 x 128 tile per workgroup like gemm_h16t_kernel, with stages of
// 8 labels (8 KB) in an NS-deep ring and the epilogue staged through the
// ring, so that WPE workgroups share a CU and one's stage waits and stores
// overlap the others' products.  Operand rows are 512 bytes (128 floats); a
// DMA instruction fills two rows, odd rows with their 16-byte chunks swapped
// by halves as in PersistF32.  Fragment reads, the product order (k ascending
// in pairs, one 32x32x2 FP32 MFMA per pair and block) and the short-K
// handling are those of the persistent FP32 kernel, so the sums are the same
// bit for bit.
// ---------------------------------------------------------------------------
template <int OUT, int NS, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
gemm_f32t_kernel(GemmArgs g) {
  constexpr int BM = 128, BN = 128, BK = 8;
  constexpr int TILE = BK * 512;  // bytes of one operand stage
  constexpr int STAGE = TILE * 2;  // A and B
  constexpr int LPW = 2;           // DMA instructions per wave per stage
  // the hand-counted vmcnt waits below assume LPW DMA loads per stage; the
  // build checks the assembly against this marker
  asm volatile("; cq-vm-lpw %0" ::"n"(LPW));
  constexpr int EROW = 288;  // bytes per staged output row (64 floats + pad)
  constexpr int EPI = 4 * 8 * EROW;
  constexpr int SMEM = NS * STAGE > EPI ? NS * STAGE : EPI;
  static_assert(NS >= 2 && NS <= 4, "stage count");
  __shared__ __attribute__((aligned(16))) char smem[SMEM];
  CQ_LDS char* const lsm = (CQ_LDS char*)smem;
  const TileCoord tc = tile_coord<BM, BN>(g);
  const int64_t m0 = tc.m0, n0 = tc.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int nstages = (int)((g.K + BK - 1) / BK);
  // wave w's instruction for an operand fills rows 2w (lanes 0-31) and
  // 2w + 1 (lanes 32-63); lane slot q of row r holds the row's chunk q ^ 8r
  const int r = lane >> 5, c = lane & 31;
  const int lrow = 2 * wave + r;
  const float* gbase[2];
  int64_t lcol[2];
  {
    gbase[0] = static_cast<const float*>(g.A) + tc.z * g.sAz + m0;
    gbase[1] = static_cast<const float*>(g.B) + tc.z * g.sBz + n0;
    // last 16-byte chunk inside each operand (M, N are multiples of 4)
    const int64_t capA = ((g.M - 4) & ~(int64_t)3) - m0, capB = ((g.N - 4) & ~(int64_t)3) - n0;
    const int64_t col = (int64_t)(c ^ (8 * r)) * 4;
    lcol[0] = col > capA ? capA : col;
    lcol[1] = col > capB ? capB : col;
  }
  auto issue = [&](int s) {
    int64_t k = (int64_t)s * BK + lrow;
    if (k >= g.K) k = g.K - 1;  // rows past K are masked to zero when read
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const float* src = gbase[op] + k * (op ? g.sBk : g.sAk) + lcol[op];
      const uint32_t dst = __builtin_amdgcn_readfirstlane(
          (uint32_t)(uintptr_t)(lsm + (s % NS) * STAGE + op * TILE + wave * 1024));
      asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(dst)
                   : "memory", "m0");
    }
  };
  f16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  for (int s = 0; s < NS - 1 && s < nstages; ++s) issue(s);
  for (int s = 0; s < nstages; ++s) {
    // this wave's loads of stage s have landed once at most `ahead` later
    // stages are outstanding; the barrier then covers every wave's loads
    const int ahead = (nstages - 1 - s) < (NS - 2) ? (nstages - 1 - s) : (NS - 2);
    if (ahead >= 2) wait_vm<2 * LPW>();
    else if (ahead == 1) wait_vm<LPW>();
    else wait_vm<0>();
    __syncthreads();
    if (s + NS - 1 < nstages) issue(s + NS - 1);
    const int sb = (s % NS) * STAGE;
    const int64_t kvalid = g.K - (int64_t)s * BK;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      if (kk >= kvalid) break;  // short K (outer products): skip all-zero steps
      const int row = kk + r;
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int ca = wm + 32 * i + c, cb = wn + 32 * i + c;
        a[i] = *(const CQ_LDS float*)(lsm + sb + row * 512 + (((ca >> 2) ^ (8 * r)) << 4) + (ca & 3) * 4);
        b[i] = *(const CQ_LDS float*)(lsm + sb + TILE + row * 512 + (((cb >> 2) ^ (8 * r)) << 4) +
                                      (cb & 3) * 4);
        if (row >= kvalid) a[i] = 0.0f;  // rows past K hold a clamped copy of row K - 1
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }

  // epilogue: slab u of a wave holds rows 32*(u>>2) + 8*(u&3) .. +7 of its
  // 64 x 64 block; it is staged in the ring so that every store instruction
  // writes whole row segments
  const float alpha = float(g.alpha);
  __syncthreads();  // every wave is done with the ring
  char* const wbuf = smem + wave * 8 * EROW;
  const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = u >> 2, vg = u & 3;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = 4 * (lane >> 5) + e;
        const int cc = 32 * j + (lane & 31);
        *reinterpret_cast<float*>(wbuf + rr * EROW + cc * 4) = alpha * acc[i][j][4 * vg + e];
      }
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rl = 4 * h + (lane >> 4);
      const int cc = 4 * (lane & 15);
      const f4_t x = *reinterpret_cast<const f4_t*>(wbuf + rl * EROW + cc * 4);
      const int64_t m = m0 + wm + 32 * i + 8 * vg + rl, n = n0 + wn + cc;
      const int64_t idx = tc.z * g.sCz + m * g.ldc + n;
      if (full || (m < g.M && n + 3 < g.N)) {
        store_out<f4_t, OUT == 1>(reinterpret_cast<f4_t*>(static_cast<float*>(g.C) + idx), x);
      } else if (m < g.M) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e < g.N) store_out<float, OUT == 1>(static_cast<float*>(g.C) + idx + e, x[e]);
      }
    }
    // the slab's LDS reads are done before the next slab overwrites it
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));
  }
}

// ---------------------------------------------------------------------------
// FP32 operands, 64 x 64 tiles: for GEMMs with few 128 x 128 tiles (a few
// hundred outputs per side), four times as many workgroups reach the CUs.
// Each wave owns one 32 x 32 block; stages hold 16 labels (4 KB per operand,
// rows of 256 bytes) in an NS-deep ring, one DMA instruction per wave and
// operand filling four rows, odd rows with their 16-byte chunks swapped by
// halves so that the two rows an MFMA operand read touches fall into
// different banks.  Products run in the persistent FP32 kernel's order (k
// ascending in pairs, one 32x32x2 MFMA per pair), so the sums are the same
// bit for bit; results are stored from registers.
// ---------------------------------------------------------------------------
template <int OUT, int NS>
__global__ void __launch_bounds__(256) gemm_f32s_kernel(GemmArgs g) {
  constexpr int BM = 64, BN = 64, BK = 16;
  constexpr int TILE = BK * 256;  // bytes of one operand stage
  constexpr int STAGE = TILE * 2;  // A and B
  constexpr int LPW = 2;           // DMA instructions per wave per stage
  // the hand-counted vmcnt waits below assume LPW DMA loads per stage; the
  // build checks the assembly against this marker
  asm volatile("; cq-vm-lpw %0" ::"n"(LPW));
  static_assert(NS >= 2 && NS <= 4, "stage count");
  __shared__ __attribute__((aligned(16))) char smem[NS * STAGE];
  CQ_LDS char* const lsm = (CQ_LDS char*)smem;
  const TileCoord tc = tile_coord<BM, BN>(g);
  const int64_t m0 = tc.m0, n0 = tc.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int nstages = (int)((g.K + BK - 1) / BK);
  // wave w's instruction for an operand fills rows 4w .. 4w + 3, sixteen
  // lanes a row; slot q of row r holds the row's chunk q ^ 8(r & 1)
  const int lrow = 4 * wave + (lane >> 4);
  const int slot = lane & 15;
  const float* gbase[2];
  int64_t lcol[2];
  {
    gbase[0] = static_cast<const float*>(g.A) + tc.z * g.sAz + m0;
    gbase[1] = static_cast<const float*>(g.B) + tc.z * g.sBz + n0;
    // last 16-byte chunk inside each operand (M, N are multiples of 4)
    const int64_t capA = ((g.M - 4) & ~(int64_t)3) - m0, capB = ((g.N - 4) & ~(int64_t)3) - n0;
    const int64_t col = (int64_t)(slot ^ (8 * (lrow & 1))) * 4;
    lcol[0] = col > capA ? capA : col;
    lcol[1] = col > capB ? capB : col;
  }
  auto issue = [&](int s) {
    int64_t k = (int64_t)s * BK + lrow;
    if (k >= g.K) k = g.K - 1;  // rows past K are masked to zero when read
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const float* src = gbase[op] + k * (op ? g.sBk : g.sAk) + lcol[op];
      const uint32_t dst = __builtin_amdgcn_readfirstlane(
          (uint32_t)(uintptr_t)(lsm + (s % NS) * STAGE + op * TILE + wave * 1024));
      asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(dst)
                   : "memory", "m0");
    }
  };
  f16_t acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  const int r = lane >> 5, c = lane & 31;

  for (int s = 0; s < NS - 1 && s < nstages; ++s) issue(s);
  for (int s = 0; s < nstages; ++s) {
    // this wave's loads of stage s have landed once at most `ahead` later
    // stages are outstanding; the barrier then covers every wave's loads
    const int ahead = (nstages - 1 - s) < (NS - 2) ? (nstages - 1 - s) : (NS - 2);
    if (ahead >= 2) wait_vm<2 * LPW>();
    else if (ahead == 1) wait_vm<LPW>();
    else wait_vm<0>();
    __syncthreads();
    if (s + NS - 1 < nstages) issue(s + NS - 1);
    const int sb = (s % NS) * STAGE;
    const int64_t kvalid = g.K - (int64_t)s * BK;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      if (kk >= kvalid) break;  // short K (outer products): skip all-zero steps
      const int row = kk + r;
      const int ca = wm + c, cb = wn + c;
      float a = *(const CQ_LDS float*)(lsm + sb + row * 256 + (((ca >> 2) ^ (8 * r)) << 4) + (ca & 3) * 4);
      const float b =
          *(const CQ_LDS float*)(lsm + sb + TILE + row * 256 + (((cb >> 2) ^ (8 * r)) << 4) + (cb & 3) * 4);
      if (row >= kvalid) a = 0.0f;  // rows past K hold a clamped copy of row K - 1
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
  }

  const float alpha = float(g.alpha);
  float* const C = static_cast<float*>(g.C);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t m = m0 + wm + 8 * (v >> 2) + 4 * r + (v & 3), n = n0 + wn + c;
    if (m < g.M && n < g.N) store_out<float, OUT == 1>(C + tc.z * g.sCz + m * g.ldc + n, alpha * acc[v]);
  }
}

// ---------------------------------------------------------------------------
// Persistent form (no output exponents), for 16-bit and FP32 operands, with
// FP32 output or -- 16-bit operands -- 16-bit hi (and lo) output planes.  Same operand ring of LDS DMA stages as gemm_h16a_kernel, but each
// workgroup walks tiles blockIdx.x, +gridDim.x, ... and the ring's stages run
// on across tile boundaries.  A finished tile's results stay in registers and
// are written out in eight row slabs spread over the next tile's stages, so
// the output stream is steady instead of one burst per tile (a burst of
// stores stalls the issuing wave while HBM drains writes from every CU).
// Slab u of a wave holds rows 32*(u>>2) + 8*(u&3) .. +7 of its 64 x 64
// block; it goes through an 8-row LDS buffer of the wave so that each store
// instruction writes whole 256-byte row segments.  A wave's vector memory
// operations retire in issue order, so the wait for a stage's operands also
// waits for every store issued before those loads; each iteration issues its
// stores first and its loads last, and the wait counts exactly the
// operations issued after the awaited loads, so stores get NS - 1 stages to
// drain before anything waits on them.
//
// The operand policy P fixes the element type.  A stage holds BK labels of
// each operand plane, 8 KB: rows of 128 elements, one DMA instruction (64
// lanes x 16 bytes) filling RPI rows; wave w's instruction q fills rows
// (2w + q) * RPI .. +RPI-1.  P::chunk gives the 16-byte chunk of its row
// that a lane's load lands in (a swizzle against LDS bank conflicts) and
// P::mma runs the stage's MFMAs for one wave's 64 x 64 block.
// ---------------------------------------------------------------------------

// 16-bit planes (hi, and lo for the split forms): rows of 256 bytes, read
// back k-contiguous with ds_read_b64_tr_b16 as in gemm_h16a_kernel.
template <int SPLIT, bool F16>
struct PersistH16 {
  using H = Half<F16>;
  using V8 = typename H::V8;
  static constexpr int BK = 32, NP = SPLIT == 3 ? 2 : 1, RPI = 4, CW = 8;
  static constexpr bool kF16 = F16;
  typedef uint16_t E;
  static __device__ int lrow(int lane) { return lane >> 4; }
  static __device__ int chunk(int lane) { return swz(lane >> 4, lane & 15); }
  static __device__ const E* plane(const GemmArgs& g, int op, int p) {
    return static_cast<const E*>(op ? (p ? g.B_lo : g.B) : (p ? g.A_lo : g.A));
  }
  static __device__ void mma(f16_t (&acc)[2][2], CQ_LDS char* lsm, int sb, int64_t kvalid, int wm, int wn,
                             int lane) {
    constexpr int TILE = BK * 256;
    const int grp = lane >> 4, r16 = lane & 15;
    const int col_in_blk = 16 * (grp & 1) + 4 * (r16 & 3);
    const int krow = 8 * (grp >> 1) + (r16 >> 2);
    auto frag = [&](int tile, int kk, int c0) -> V8 {
      const int col = c0 + col_in_blk;
      const int r0 = kk + krow, r1 = r0 + 4;
      const int o0 = tile + r0 * 256 + (swz(r0, col >> 3) << 4) + (col & 7) * 2;
      const int o1 = tile + r1 * 256 + (swz(r1, col >> 3) << 4) + (col & 7) * 2;
      s4_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((CQ_LDS s4_t*)(lsm + o0));
      s4_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((CQ_LDS s4_t*)(lsm + o1));
      if (kvalid < BK) {
        const int kb = kk + 8 * (grp >> 1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (kb + e >= kvalid) lo[e] = 0;
          if (kb + 4 + e >= kvalid) hi[e] = 0;
        }
      }
      typedef short s8_t __attribute__((ext_vector_type(8)));
      const s8_t v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      return __builtin_bit_cast(V8, v);
    };
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      V8 a[NP][2], b[NP][2];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
          a[p][ii] = frag(sb + (0 * NP + p) * TILE, kk, wm + 32 * ii);
          b[p][ii] = frag(sb + (1 * NP + p) * TILE, kk, wn + 32 * ii);
        }
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[ii][j] = H::mfma(a[0][ii], b[0][j], acc[ii][j]);
          if constexpr (SPLIT == 3) {
            acc[ii][j] = H::mfma(a[0][ii], b[NP - 1][j], acc[ii][j]);
            acc[ii][j] = H::mfma(a[NP - 1][ii], b[0][j], acc[ii][j]);
          }
        }
    }
  }
};

// FP32: rows of 512 bytes.  Odd rows have their 16-byte chunks swapped by
// halves (chunk ^ 8), so the MFMA operand reads -- 32 consecutive floats of
// rows k and k + 1 -- fall into different banks.
struct PersistF32 {
  static constexpr int BK = 16, NP = 1, RPI = 2, CW = 4;
  static constexpr bool kF16 = false;
  typedef float E;
  static __device__ int lrow(int lane) { return lane >> 5; }
  static __device__ int chunk(int lane) { return (lane & 31) ^ (8 * (lane >> 5)); }
  static __device__ const E* plane(const GemmArgs& g, int op, int) {
    return static_cast<const E*>(op ? g.B : g.A);
  }
  static __device__ void mma(f16_t (&acc)[2][2], CQ_LDS char* lsm, int sb, int64_t kvalid, int wm, int wn,
                             int lane) {
    constexpr int TILE = BK * 512;
    const int r = lane >> 5, c = lane & 31;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      if (kk >= kvalid) break;  // short K (outer products): skip all-zero steps
      const int row = kk + r;
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int ca = wm + 32 * i + c, cb = wn + 32 * i + c;
        a[i] = *(const CQ_LDS float*)(lsm + sb + row * 512 + (((ca >> 2) ^ (8 * r)) << 4) + (ca & 3) * 4);
        b[i] = *(const CQ_LDS float*)(lsm + sb + TILE + row * 512 + (((cb >> 2) ^ (8 * r)) << 4) + (cb & 3) * 4);
        if (row >= kvalid) a[i] = 0.0f;  // rows past K hold a clamped copy of row K - 1
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
};

template <class P, int OUT, int NS>
__global__ void __launch_bounds__(256, 2) gemm_persist_kernel(GemmArgs g) {
  constexpr int BM = 128, BN = 128, BK = P::BK, NP = P::NP, RPI = P::RPI, CW = P::CW;
  constexpr int TILE = 8192;            // bytes of one operand-plane stage
  constexpr int STAGE = TILE * 2 * NP;  // A and B, all planes
  constexpr int LPW = 2 * 2 * NP;       // DMA instructions per wave per stage
  // the hand-counted vmcnt waits below assume LPW DMA loads per stage and one
  // store instruction per output row and plane; the build checks the assembly
  // against this marker
  asm volatile("; cq-vm-lpw %0 out %1" ::"n"(LPW), "n"(OUT));
  constexpr int RING = NS * STAGE;
  constexpr int EROW = 288;             // bytes per staged output row (64 floats + pad)
  static_assert(NS >= 2 && NS <= 5, "stage count");
  static_assert(BK * 128 * sizeof(typename P::E) == TILE && RPI * 8 == BK, "stage layout");
  __shared__ __attribute__((aligned(16))) char smem[RING + 4 * 8 * EROW];
  CQ_LDS char* const lsm = (CQ_LDS char*)smem;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  char* const wbuf = smem + RING + wave * 8 * EROW;
  const int nstages = (int)((g.K + BK - 1) / BK);
  const int64_t my_tiles = (g.tiles - (int64_t)blockIdx.x + gridDim.x - 1) / gridDim.x;
  const int64_t total = my_tiles * nstages;
  // tile coordinates in 32-bit arithmetic (tiles < 2^31): workgroup b's i-th
  // tile is virtual block b + i * gridDim.x, placed like xcd_tile/tile_coord_of
  auto tile_of = [&](int64_t i) -> TileCoord {
    const uint32_t vb = blockIdx.x + (uint32_t)i * gridDim.x;
    const uint32_t T = (uint32_t)g.tiles, per = T / 8, rem = T % 8;
    const uint32_t x = vb % 8, loc = vb / 8;
    const uint32_t t = x < rem ? x * (per + 1) + loc : rem * (per + 1) + (x - rem) * per + loc;
    const uint32_t tM = (uint32_t)g.tilesM, tN = (uint32_t)g.tilesN;
    TileCoord c;
    if (g.m_fastest) {
      const uint32_t r = t / tM;
      c.m0 = (int64_t)(t - r * tM) * BM;
      c.z = r / tN;
      c.n0 = (int64_t)(r - (uint32_t)c.z * tN) * BN;
    } else {
      const uint32_t r = t / tN;
      c.n0 = (int64_t)(t - r * tN) * BN;
      c.z = r / tM;
      c.m0 = (int64_t)(r - (uint32_t)c.z * tM) * BM;
    }
    return c;
  };
  // operand loads run ahead of the multiplies; their state advances one
  // stage per issue: tile index, stage in the tile, ring slot, and each
  // plane's source row base for this lane in the current tile
  const int64_t ccapM = (g.M - CW) & ~(int64_t)(CW - 1), ccapN = (g.N - CW) & ~(int64_t)(CW - 1);
  const int lrow = P::lrow(lane);                      // row inside an instruction's rows
  const int64_t lcol = (int64_t)P::chunk(lane) * CW;  // column this lane's 16 bytes start at
  int64_t is_i = 0;
  int is_s = 0, is_slot = 0;
  const typename P::E* isrc[2][NP];
  auto issue_next = [&]() {
    if (is_s == 0) {
      const TileCoord tc = tile_of(is_i);
#pragma unroll
      for (int op = 0; op < 2; ++op) {
        int64_t col = (op ? tc.n0 : tc.m0) + lcol;
        const int64_t cap = op ? ccapN : ccapM;  // last 16-byte chunk inside the operand
        if (col > cap) col = cap;
#pragma unroll
        for (int p = 0; p < NP; ++p) isrc[op][p] = P::plane(g, op, p) + tc.z * (op ? g.sBz : g.sAz) + col;
      }
    }
    const int64_t k0 = (int64_t)is_s * BK;
#pragma unroll
    for (int op = 0; op < 2; ++op)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int qq = 0; qq < 2; ++qq) {
          const int chunk0 = (wave * 2 + qq) * 64;
          int64_t k = k0 + (wave * 2 + qq) * RPI + lrow;
          if (k >= g.K) k = g.K - 1;  // rows past K are masked to zero when read
          const typename P::E* src = isrc[op][p] + k * (op ? g.sBk : g.sAk);
          const uint32_t dst = __builtin_amdgcn_readfirstlane(
              (uint32_t)(uintptr_t)(lsm + is_slot * STAGE + (op * NP + p) * TILE + chunk0 * 16));
          asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(dst)
                       : "memory", "m0");
        }
    if (++is_s == nstages) {
      is_s = 0;
      ++is_i;
    }
    if (++is_slot == NS) is_slot = 0;
  };

  f16_t acc[2][2], prev[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = prev[i][j][v] = 0.0f;
  TileCoord pt{0, 0, 0};  // tile held in prev
  // slab u of prev (already scaled by alpha): rows 32*(u>>2) + 8*(u&3) .. +7
  auto slab = [&](const int u) {
    const int i = u >> 2, vg = u & 3;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 4 * (lane >> 5) + e;  // row inside the slab
        const int c = 32 * j + (lane & 31);
        *reinterpret_cast<float*>(wbuf + r * EROW + c * 4) = prev[i][j][4 * vg + e];
      }
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0)
    const bool full = pt.m0 + BM <= g.M && pt.n0 + BN <= g.N;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rl = 4 * h + (lane >> 4);
      const int c = 4 * (lane & 15);
      const f4_t x = *reinterpret_cast<const f4_t*>(wbuf + rl * EROW + c * 4);
      const int64_t m = pt.m0 + wm + 32 * i + 8 * vg + rl, n = pt.n0 + wn + c;
      const int64_t idx = pt.z * g.sCz + m * g.ldc + n;
      if constexpr (OUT == 2) {
        // 16-bit planes: hi = rn16(x), and lo = rn16(x - hi) when C_lo is given
        typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
        u16x4 hh, ll;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          hh[e] = to_h16<P::kF16>(x[e]);
          ll[e] = to_h16<P::kF16>(x[e] - from_h16<P::kF16>(hh[e]));
        }
        uint16_t* const ch = static_cast<uint16_t*>(g.C);
        uint16_t* const cl = static_cast<uint16_t*>(g.C_lo);
        if (full || (m < g.M && n + 3 < g.N)) {
          *reinterpret_cast<u16x4*>(ch + idx) = hh;
          if (cl) *reinterpret_cast<u16x4*>(cl + idx) = ll;
        } else if (m < g.M) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (n + e < g.N) {
              ch[idx + e] = hh[e];
              if (cl) cl[idx + e] = ll[e];
            }
        }
      } else if (full || (m < g.M && n + 3 < g.N)) {
        store_out<f4_t, OUT == 1>(reinterpret_cast<f4_t*>(static_cast<float*>(g.C) + idx), x);
      } else if (m < g.M) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e < g.N) store_out<float, OUT == 1>(static_cast<float*>(g.C) + idx + e, x[e]);
      }
    }
  };
  const float alpha = float(g.alpha);
  for (int64_t q = 0; q < NS - 1 && q < total; ++q) issue_next();
  // hist[k]: vector memory instructions issued by iteration q - 1 - k (the
  // prologue's loads count as iterations -NS+1 .. -1, one stage each).  The
  // loads of stage q were issued last in iteration q - NS + 1, so exactly
  // hist[0] + ... + hist[NS-3] instructions were issued after them; waiting
  // until no more are outstanding completes them and nothing issued later.
  // Stores of tiles with a ragged edge are not counted, which only makes the
  // wait longer.
  int hist[NS - 1];
  const int pro = total < NS - 1 ? (int)total : NS - 1;
#pragma unroll
  for (int k = 0; k < NS - 1; ++k) hist[k] = (NS - 2 - k) < pro ? LPW : 0;
  int s = 0, slot = 0;
  int64_t i = 0;
  for (int64_t q = 0; q < total; ++q) {
    int after = 0;
#pragma unroll
    for (int k = 0; k < NS - 2; ++k) after += hist[k];
    wait_vm_n(after);
    // stage q landed for every wave; the slot of stage q - 1 is free.  A bare
    // barrier: a fence here would also wait for this wave's output stores.
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    // slabs of the previous tile due at this stage (two stores each), then
    // the loads of stage q + NS - 1
    int ops = 0;
    if (i > 0) {
      const bool pfull = pt.m0 + BM <= g.M && pt.n0 + BN <= g.N;
      // store instructions of a full slab: two rows of 16 bytes per lane, or
      // of 8 bytes per plane for 16-bit output
      const int per_slab = OUT == 2 ? (g.C_lo ? 4 : 2) : 2;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if ((u * nstages) / 8 == s) {
          slab(u);
          if (pfull) ops += per_slab;
        }
    }
    if (q + NS - 1 < total) {
      issue_next();
      ops += LPW;
    }
#pragma unroll
    for (int k = NS - 2; k > 0; --k) hist[k] = hist[k - 1];
    hist[0] = ops;
    const int sb = slot * STAGE;
    if (++slot == NS) slot = 0;
    P::mma(acc, lsm, sb, g.K - (int64_t)s * BK, wm, wn, lane);
    if (++s == nstages) {
      s = 0;
      pt = tile_of(i);
      ++i;
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            prev[ii][j][v] = alpha * acc[ii][j][v];
            acc[ii][j][v] = 0.0f;
          }
    }
  }
  if (i > 0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) slab(u);
  }
}

template <typename K>
hipError_t launch(K kernel, const GemmArgs& a, hipStream_t s, int threads = 256) {
  hipLaunchKernelGGL(kernel, dim3((unsigned)a.tiles), dim3(threads), 0, s, a,
                     static_cast<const GemmArgs*>(nullptr), (int64_t)0);
  return hipGetLastError();
}

template <typename K>
hipError_t launch_ind(K kernel, const GemmArgs* dev, int64_t max_tiles, hipStream_t s, InstSpan span,
                      int threads = 256) {
  if (max_tiles <= 0 || span.n <= 0) return hipSuccess;
  if (max_tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  GemmArgs dummy{};
  hipLaunchKernelGGL(kernel, dim3((unsigned)max_tiles, 1, (unsigned)span.n), dim3(threads), 0, s, dummy, dev,
                     span.stride);
  return hipGetLastError();
}

// 16-byte aligned rows of at least 8 columns in every operand plane and in
// the output: the asynchronous kernel applies
bool h16_async_ok(const GemmArgs& a, DType tc) {
  auto al = [](const void* p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const bool sizes = a.M >= 8 && a.N >= 8 && a.M % 8 == 0 && a.N % 8 == 0 && a.ldc % 4 == 0 &&
                     a.sAk % 8 == 0 && a.sBk % 8 == 0 && a.sAz % 8 == 0 && a.sBz % 8 == 0 && a.sCz % 4 == 0;
  (void)tc;
  return sizes && al(a.A) && al(a.A_lo) && al(a.B) && al(a.B_lo) && al(a.C) && al(a.C_lo);
}

// Variant `impl` of the 16-bit launch: 0 = asynchronous kernel with its
// default ring depth, 1 = the other depth, 2 = 64 x 64 tiles (the
// register-path kernel where those do not apply),
// 3 = persistent kernel, 4 and 5 = occupancy kernel (four workgroups per CU
// with a two-deep ring, three with a three-deep one).
// Persistent grid: two workgroups per compute unit, a multiple of 8 so that
// workgroup b stays on XCD b % 8 for every tile it takes.
int64_t persistent_grid(int64_t tiles) {
  static std::atomic<int> cus[64];  // compute units per device, 0 until asked
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int n = cus[dev].load(std::memory_order_relaxed);
  if (n <= 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev].store(n, std::memory_order_relaxed);
  }
  int64_t grid = 2 * (int64_t)n;
  grid -= grid % 8;
  return tiles < grid ? tiles : grid;
}

// the persistent kernel applies: no output exponents, K >= 1, aligned rows
bool h16p_ok(const GemmArgs& a, DType tc) {
  return a.rowexp == nullptr && a.K >= 1 && h16_async_ok(a, tc);
}

// the occupancy kernel applies: K >= 1, aligned rows (it applies output
// exponents in its epilogue)
bool h16t_ok(const GemmArgs& a, DType tc) { return a.K >= 1 && h16_async_ok(a, tc); }

// FP32 operands for the persistent kernel: 16-byte aligned rows of at least
// 4 columns, and an output whose rows take 16-byte stores
bool f32p_ok(const GemmArgs& a) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  return a.rowexp == nullptr && a.K >= 1 && a.M >= 4 && a.N >= 4 && a.M % 4 == 0 && a.N % 4 == 0 &&
         a.sAk % 4 == 0 && a.sBk % 4 == 0 && a.sAz % 4 == 0 && a.sBz % 4 == 0 && a.ldc % 4 == 0 &&
         a.sCz % 4 == 0 && al(a.A) && al(a.B) && al(a.C);
}

template <int SPLIT, bool F16>
hipError_t launch_h16s(GemmArgs a, DType tc, bool nt, hipStream_t s) {
  const int64_t z = a.tiles / (a.tilesM * a.tilesN);  // batches (the tile counts are for 128 x 128)
  a.tilesM = (a.M + 63) / 64;
  a.tilesN = (a.N + 63) / 64;
  a.tiles = a.tilesM * a.tilesN * z;
  if (a.tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)a.tiles), block(256);
  if (tc != DType::F32) hipLaunchKernelGGL((gemm_h16s_kernel<SPLIT, F16, 2, 2>), grid, block, 0, s, a);
  else if (nt) hipLaunchKernelGGL((gemm_h16s_kernel<SPLIT, F16, 1, 2>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gemm_h16s_kernel<SPLIT, F16, 0, 2>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int NS>
hipError_t launch_f32s(GemmArgs a, bool nt, hipStream_t s) {
  const int64_t z = a.tiles / (a.tilesM * a.tilesN);  // batches (the tile counts are for 128 x 128)
  a.tilesM = (a.M + 63) / 64;
  a.tilesN = (a.N + 63) / 64;
  a.tiles = a.tilesM * a.tilesN * z;
  if (a.tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)a.tiles), block(256);
  if (nt) hipLaunchKernelGGL((gemm_f32s_kernel<1, NS>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gemm_f32s_kernel<0, NS>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int NS, int WPE>
hipError_t launch_f32t(const GemmArgs& a, bool nt, hipStream_t s) {
  const dim3 grid((unsigned)a.tiles), block(256);
  if (nt) hipLaunchKernelGGL((gemm_f32t_kernel<1, NS, WPE>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gemm_f32t_kernel<0, NS, WPE>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int SPLIT, bool F16, int NS, int WPE>
hipError_t launch_h16t(const GemmArgs& a, DType tc, bool nt, hipStream_t s) {
  const dim3 grid((unsigned)a.tiles), block(256);
  if (tc != DType::F32) hipLaunchKernelGGL((gemm_h16t_kernel<SPLIT, F16, 2, NS, WPE>), grid, block, 0, s, a);
  else if (nt) hipLaunchKernelGGL((gemm_h16t_kernel<SPLIT, F16, 1, NS, WPE>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gemm_h16t_kernel<SPLIT, F16, 0, NS, WPE>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int SPLIT, bool F16>
hipError_t dispatch_h16(const GemmArgs& a, DType tc, bool nt, hipStream_t s, int impl = 0) {
  constexpr int NS = SPLIT == 3 ? 2 : 3;
  constexpr int NS2 = SPLIT == 3 ? 3 : 2;
  constexpr int NSP = SPLIT == 3 ? 2 : 4;
  // occupancy form: four workgroups per CU with a two-deep ring, or three
  // with a three-deep one
  if (impl == 2 && h16p_ok(a, tc)) return launch_h16s<SPLIT, F16>(a, tc, nt, s);
  if (impl == 4 && h16t_ok(a, tc)) return launch_h16t<SPLIT, F16, 2, 4>(a, tc, nt, s);
  if (impl == 5 && h16t_ok(a, tc)) return launch_h16t<SPLIT, F16, 3, 3>(a, tc, nt, s);
  if (impl == 3 && h16p_ok(a, tc)) {
    const int64_t grid = persistent_grid(a.tiles);
    using P = PersistH16<SPLIT, F16>;
    if (tc != DType::F32) hipLaunchKernelGGL((gemm_persist_kernel<P, 2, NSP>), dim3((unsigned)grid), dim3(256), 0, s, a);
    else if (nt) hipLaunchKernelGGL((gemm_persist_kernel<P, 1, NSP>), dim3((unsigned)grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((gemm_persist_kernel<P, 0, NSP>), dim3((unsigned)grid), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (impl == 1 && h16_async_ok(a, tc)) {
    if (tc == DType::F32) {
      if (nt) return launch(gemm_h16a_kernel<SPLIT, F16, 1, NS2>, a, s);
      return launch(gemm_h16a_kernel<SPLIT, F16, 0, NS2>, a, s);
    }
    return launch(gemm_h16a_kernel<SPLIT, F16, 2, NS2>, a, s);
  }
  if (impl != 2 && h16_async_ok(a, tc)) {
    if (tc == DType::F32) {
      if (nt) return launch(gemm_h16a_kernel<SPLIT, F16, 1, NS>, a, s);
      return launch(gemm_h16a_kernel<SPLIT, F16, 0, NS>, a, s);
    }
    return launch(gemm_h16a_kernel<SPLIT, F16, 2, NS>, a, s);
  }
  if (tc == DType::F32) {
    if (nt) return launch(gemm_h16_kernel<SPLIT, F16, 1>, a, s);
    return launch(gemm_h16_kernel<SPLIT, F16, 0>, a, s);
  }
  return launch(gemm_h16_kernel<SPLIT, F16, 2>, a, s);
}

}  // namespace

namespace {

// One launch of variant v: bit 0 flips the raster order, v >> 1 selects the
// 16-bit implementation (dispatch_h16).
hipError_t launch_variant(cq_precision prec, GemmArgs a, DType tc, bool nt, int v, hipStream_t stream) {
  if (v & 1) a.m_fastest ^= 1;
  const int impl = v >> 1;
  switch (prec) {
    case CQ_FP64:
      return nt ? launch(gemm_f64_kernel<true>, a, stream, 512) : launch(gemm_f64_kernel<false>, a, stream, 512);
    case CQ_FP32:
      // 0 = tiled kernel, 1 = 64 x 64 tiles (2 repeats 0), 3 = persistent
      // kernel, 4 and 5 = occupancy kernel (four workgroups per CU with a
      // three- or four-deep ring)
      if (impl == 1 && f32p_ok(a)) return launch_f32s<3>(a, nt, stream);
      if (impl == 4 && f32p_ok(a)) return launch_f32t<3, 4>(a, nt, stream);
      if (impl == 5 && f32p_ok(a)) return launch_f32t<4, 4>(a, nt, stream);
      if (impl == 3 && f32p_ok(a)) {
        const int64_t grid = persistent_grid(a.tiles);
        if (nt) hipLaunchKernelGGL((gemm_persist_kernel<PersistF32, 1, 4>), dim3((unsigned)grid), dim3(256), 0, stream, a);
        else hipLaunchKernelGGL((gemm_persist_kernel<PersistF32, 0, 4>), dim3((unsigned)grid), dim3(256), 0, stream, a);
        return hipGetLastError();
      }
      return nt ? launch(gemm_f32_kernel<true>, a, stream) : launch(gemm_f32_kernel<false>, a, stream);
    case CQ_BF16: return dispatch_h16<1, false>(a, tc, nt, stream, impl);
    case CQ_FP16: return dispatch_h16<1, true>(a, tc, nt, stream, impl);
    case CQ_BF16_SPLIT: return dispatch_h16<3, false>(a, tc, nt, stream, impl);
    case CQ_FP16_SPLIT: return dispatch_h16<3, true>(a, tc, nt, stream, impl);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Autotuner.  The first time a GEMM shape is launched (outside stream
// capture) every variant runs twice on the caller's stream and the fastest
// second run is kept for that shape; later launches use it.  Each variant
// computes the whole result, so the output is valid whichever ran last.
// ---------------------------------------------------------------------------
struct TuneKey {
  int prec, tc, nt, za, zb, aligned;
  int64_t M, N, K, Z;
  bool operator<(const TuneKey& o) const {
    const int64_t x[10] = {prec, tc, nt, za, zb, aligned, M, N, K, Z};
    const int64_t y[10] = {o.prec, o.tc, o.nt, o.za, o.zb, o.aligned, o.M, o.N, o.K, o.Z};
    for (int i = 0; i < 10; ++i)
      if (x[i] != y[i]) return x[i] < y[i];
    return false;
  }
};

constexpr int kMaxVariants = 12;

struct TuneEntry {
  int variant;
  float ms[kMaxVariants];
  int tried;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;
std::atomic<int> g_tune_on{-1};  // -1: not yet read from CQ_AUTOTUNE

// Choices persist as text, one shape per line, tagged with the kind of device
// they were timed on (architecture and compute-unit count):
//   cq-tune-1 <device> prec tc nt za zb aligned M N K Z variant tried ms[0..11]
// CQ_TUNE_CACHE names a file that is read at the first tuned launch and
// extended by every shape tuned later (cq_autotune_load / _save do the same
// on request).
std::string tune_device() {
  static std::mutex mu;
  static std::string id[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return "unknown";
  std::lock_guard<std::mutex> lk(mu);
  if (id[dev].empty()) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch = prop.gcnArchName;
    for (char& c : arch)
      if (c == ' ' || c == ':') c = '_';  // one token, no separators of the line format
    id[dev] = arch + "-" + std::to_string(prop.multiProcessorCount) + "cu";
  }
  return id[dev];
}

std::string tune_line(const std::string& dev, const TuneKey& k, const TuneEntry& e) {
  char buf[1024];
  int n = std::snprintf(buf, sizeof(buf), "cq-tune-1 %s %d %d %d %d %d %d %lld %lld %lld %lld %d %d", dev.c_str(),
                        k.prec, k.tc, k.nt, k.za, k.zb, k.aligned, (long long)k.M, (long long)k.N,
                        (long long)k.K, (long long)k.Z, e.variant, e.tried);
  std::string s(buf, (size_t)n);
  for (int v = 0; v < kMaxVariants; ++v) {
    n = std::snprintf(buf, sizeof(buf), " %.9g", (double)e.ms[v]);
    s.append(buf, (size_t)n);
  }
  return s + "\n";
}

// Entries of `path` for this device; false when the file cannot be read.
bool tune_read(const char* path, std::vector<std::pair<TuneKey, TuneEntry>>& out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  const std::string dev = tune_device();
  char line[2048];
  while (std::fgets(line, sizeof(line), f)) {
    char tag[32], d[256];
    TuneKey k;
    TuneEntry e;
    long long M, N, K, Z;
    double ms[kMaxVariants];
    const int got = std::sscanf(
        line, "%31s %255s %d %d %d %d %d %d %lld %lld %lld %lld %d %d %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf",
        tag, d, &k.prec, &k.tc, &k.nt, &k.za, &k.zb, &k.aligned, &M, &N, &K, &Z, &e.variant, &e.tried, &ms[0],
        &ms[1], &ms[2], &ms[3], &ms[4], &ms[5], &ms[6], &ms[7], &ms[8], &ms[9], &ms[10], &ms[11]);
    if (got != 14 + kMaxVariants || std::strcmp(tag, "cq-tune-1") != 0 || dev != d) continue;
    if (k.prec < 0 || k.prec > 5 || e.variant < 0 || e.variant >= kMaxVariants || !((e.tried >> e.variant) & 1))
      continue;
    k.M = M;
    k.N = N;
    k.K = K;
    k.Z = Z;
    for (int v = 0; v < kMaxVariants; ++v) e.ms[v] = (float)ms[v];
    out.emplace_back(k, e);
  }
  std::fclose(f);
  return true;
}

// Adds entries not cached yet; returns whether the file could be read.
bool tune_merge_file(const char* path) {
  std::vector<std::pair<TuneKey, TuneEntry>> got;
  if (!tune_read(path, got)) return false;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : got) g_tune.emplace(kv.first, kv.second);
  return true;
}

const char* tune_cache_path() {
  const char* p = std::getenv("CQ_TUNE_CACHE");
  return (p && p[0]) ? p : nullptr;
}

// 0: variant 0 always, 1: tune, 2 + v: variant v always (where it applies)
int tune_mode() {
  int on = g_tune_on.load();
  if (on < 0) {
    const char* e = std::getenv("CQ_AUTOTUNE");
    on = (e && e[0] == '0') ? 0 : 1;
    g_tune_on.store(on);
  }
  static std::once_flag loaded;
  if (on == 1)
    std::call_once(loaded, [] {
      if (const char* p = tune_cache_path()) (void)tune_merge_file(p);
    });
  return on;
}

int variant_count(cq_precision prec) {
  return prec == CQ_FP64 ? 2 : kMaxVariants;
}

// whether variant v has a kernel of its own for this launch (else it would
// repeat variant v & 1)
bool variant_applies(cq_precision prec, const GemmArgs& a, DType tc, int v) {
  const int impl = v >> 1;
  if (impl == 0) return true;
  if (v >= variant_count(prec)) return false;
  if (prec == CQ_FP32) return (impl == 1 || impl >= 3) && f32p_ok(a);
  if (impl == 4 || impl == 5) return h16t_ok(a, tc);
  return impl == 3 ? h16p_ok(a, tc) : h16_async_ok(a, tc);
}

}  // namespace

hipError_t launch_gemm(cq_precision prec, const GemmLaunch& g, hipStream_t stream) {
  GemmArgs a;
  a.A = g.a.p;
  a.A_lo = g.a.lo;
  a.B = g.b.p;
  a.B_lo = g.b.lo;
  a.C = g.C;
  a.C_lo = g.C_lo;
  a.M = g.M;
  a.N = g.N;
  a.K = g.K;
  a.sAz = g.sAz;
  a.sAk = g.sAk;
  a.sBz = g.sBz;
  a.sBk = g.sBk;
  a.sCz = g.sCz;
  a.ldc = g.ldc;
  a.alpha = g.alpha;
  a.rowexp = g.rowexp;
  a.colexp = g.colexp;
  a.rowtmax = nullptr;
  a.topc_thr = nullptr;
  a.topc_count = nullptr;
  a.topc_C = nullptr;
  a.topc_v = nullptr;
  a.topc_i = nullptr;
  a.topc_publish_only = 0;
  a.tile_list = nullptr;
  a.tile_count = nullptr;
  a.tilesM = (g.M + 127) / 128;
  a.tilesN = (g.N + 127) / 128;
  a.tiles = a.tilesM * a.tilesN * g.Z;
  // walk the tiles along M when the B operand is the larger one (its panels
  // are then shared by consecutive workgroups), else along N
  const double a_elems = double(g.sAz ? g.Z : 1) * double(g.M) * double(g.K);
  const double b_elems = double(g.sBz ? g.Z : 1) * double(g.N) * double(g.K);
  a.m_fastest = b_elems > a_elems ? 1 : 0;
  if (a.tiles <= 0) return hipSuccess;
  if (a.tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool nt = g.nontemporal;
  switch (prec) {
    case CQ_FP64:
      if (g.a.t != DType::F64 || g.b.t != DType::F64 || g.tc != DType::F64) return hipErrorInvalidValue;
      break;
    case CQ_FP32:
      if (g.a.t != DType::F32 || g.b.t != DType::F32 || g.tc != DType::F32) return hipErrorInvalidValue;
      break;
    case CQ_BF16:
    case CQ_FP16:
      if (g.a.t != DType::H16 || g.b.t != DType::H16) return hipErrorInvalidValue;
      if (g.tc != DType::F32 && g.tc != DType::H16) return hipErrorInvalidValue;
      break;
    case CQ_BF16_SPLIT:
    case CQ_FP16_SPLIT:
      if (g.a.t != DType::H16X2 || g.b.t != DType::H16X2) return hipErrorInvalidValue;
      if (g.tc != DType::F32 && g.tc != DType::H16X2) return hipErrorInvalidValue;
      break;
    default:
      return hipErrorInvalidValue;
  }
  // tune only shapes worth it (a few microseconds of work or more); inside a
  // capture nothing is timed: a shape tuned before keeps its variant, an
  // untuned one takes variant 0
  const int mode = tune_mode();
  if (mode >= 2) {
    const int v = mode - 2;
    return launch_variant(prec, a, g.tc, nt, variant_applies(prec, a, g.tc, v) ? v : 0, stream);
  }
  if (mode == 0 || a.tiles < 64) return launch_variant(prec, a, g.tc, nt, 0, stream);
  const TuneKey key{(int)prec, (int)g.tc, nt ? 1 : 0, g.sAz ? 1 : 0, g.sBz ? 1 : 0,
                    h16_async_ok(a, g.tc) ? 1 : 0, g.M, g.N, g.K, g.Z};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return launch_variant(prec, a, g.tc, nt, it->second.variant, stream);
  }
  if (g.no_tune) return launch_variant(prec, a, g.tc, nt, 0, stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return launch_variant(prec, a, g.tc, nt, 0, stream);
  TuneEntry te{0, {}, 0};
  hipEvent_t ev[3];
  for (int i = 0; i < 3; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) return launch_variant(prec, a, g.tc, nt, 0, stream);
  hipError_t err = hipSuccess;
  float best = 0.0f;
  for (int v = 0; v < variant_count(prec) && err == hipSuccess; ++v) {
    if (!variant_applies(prec, a, g.tc, v)) continue;
    err = hipEventRecord(ev[0], stream);
    if (err == hipSuccess) err = launch_variant(prec, a, g.tc, nt, v, stream);
    if (err == hipSuccess) err = hipEventRecord(ev[1], stream);
    if (err == hipSuccess) err = launch_variant(prec, a, g.tc, nt, v, stream);
    if (err == hipSuccess) err = hipEventRecord(ev[2], stream);
    if (err == hipSuccess) err = hipEventSynchronize(ev[2]);
    float t1 = 0.0f, t2 = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t1, ev[0], ev[1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&t2, ev[1], ev[2]);
    const float t = t1 < t2 ? t1 : t2;
    te.ms[v] = t;
    te.tried |= 1 << v;
    if (err == hipSuccess && (v == 0 || t < best)) {
      best = t;
      te.variant = v;
    }
  }
  for (int i = 0; i < 3; ++i) (void)hipEventDestroy(ev[i]);
  if (err != hipSuccess) return err;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = te;
  }
  if (const char* p = tune_cache_path()) {
    const std::string line = tune_line(tune_device(), key, te);
    if (FILE* f = std::fopen(p, "a")) {
      std::fputs(line.c_str(), f);
      std::fclose(f);
    }
  }
  // the output comes from the chosen variant, as on every later call
  return launch_variant(prec, a, g.tc, nt, te.variant, stream);
}

void autotune_set(int mode) { g_tune_on.store(mode < 0 ? 0 : mode); }

bool autotune_load(const char* path) { return path && tune_merge_file(path); }

bool autotune_save(const char* path) {
  if (!path) return false;
  const std::string dev = tune_device();
  std::string text;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune) text += tune_line(dev, kv.first, kv.second);
  }
  FILE* f = std::fopen(path, "w");
  if (!f) return false;
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  return std::fclose(f) == 0 && ok;
}

namespace {

// The schedule behind variant v: kernel, tile, ring depth (operand stages in
// LDS), resident workgroups per compute unit and raster order.
std::string variant_schedule(int prec, int v) {
  const int impl = v >> 1;
  const bool split = prec == CQ_BF16_SPLIT || prec == CQ_FP16_SPLIT;
  const char* kernel = "tiled";
  int ring = 0, wpc = 0, tile = 128;
  if (prec == CQ_FP32 && impl == 1) {
    kernel = "small-tile";
    ring = 3;
    tile = 64;
  } else if (prec == CQ_FP32 && impl >= 3) {
    kernel = impl == 3 ? "persistent" : "occupancy";
    ring = impl == 4 ? 3 : 4;
    wpc = impl == 3 ? 2 : 4;
  } else if (prec != CQ_FP64 && prec != CQ_FP32) {
    switch (impl) {
      case 0: kernel = "async"; ring = split ? 2 : 3; break;
      case 1: kernel = "async"; ring = split ? 3 : 2; break;
      case 2: kernel = "small-tile"; ring = 2; tile = 64; break;
      case 3: kernel = "persistent"; ring = split ? 2 : 4; wpc = 2; break;
      case 4: kernel = "occupancy"; ring = 2; wpc = 4; break;
      default: kernel = "occupancy"; ring = 3; wpc = 3; break;
    }
  }
  char buf[256];
  const int n = std::snprintf(buf, sizeof(buf),
                              "{\"kernel\": \"%s\", \"tile\": [%d, %d], \"ring\": %d, "
                              "\"workgroups_per_cu\": %d, \"raster\": \"%s\"}",
                              kernel, tile, tile, ring, wpc, (v & 1) ? "flipped" : "default");
  return std::string(buf, (size_t)n);
}

}  // namespace

std::string autotune_json() {
  static const char* pname[] = {"fp64", "fp32", "bf16", "bf16_split", "fp16", "fp16_split"};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::string s = "[";
  bool first = true;
  for (const auto& kv : g_tune) {
    const TuneKey& k = kv.first;
    const TuneEntry& e = kv.second;
    char buf[512];
    int n = std::snprintf(buf, sizeof(buf),
                          "%s{\"prec\": \"%s\", \"M\": %lld, \"N\": %lld, \"K\": %lld, \"Z\": %lld, "
                          "\"variant\": %d, \"schedule\": ",
                          first ? "" : ", ", pname[k.prec], (long long)k.M, (long long)k.N,
                          (long long)k.K, (long long)k.Z, e.variant);
    s.append(buf, n);
    s += variant_schedule(k.prec, e.variant);
    s += ", \"ms\": [";
    bool f2 = true;
    for (int v = 0; v < kMaxVariants; ++v)
      if ((e.tried >> v) & 1) {
        n = std::snprintf(buf, sizeof(buf), "%s[%d, %.4f]", f2 ? "" : ", ", v, e.ms[v]);
        s.append(buf, n);
        f2 = false;
      }
    s += "]}";
    first = false;
  }
  s += "]";
  return s;
}

namespace {

template <int KIND>  // 0 FP64, 1 FP32, 2 BF16 planes, 3 FP16 planes
__device__ inline double operand_at(const void* hi, const void* lo, int64_t i) {
  if constexpr (KIND == 0) return static_cast<const double*>(hi)[i];
  else if constexpr (KIND == 1) return static_cast<const float*>(hi)[i];
  else {
    const uint16_t* h = static_cast<const uint16_t*>(hi);
    const uint16_t* l = static_cast<const uint16_t*>(lo);
    double v = double(from_h16<KIND == 3>(h[i]));
    if (l) v += double(from_h16<KIND == 3>(l[i]));
    return v;
  }
}

// max |value| over elements i .. i+3, with one vector load per plane when
// they are aligned for it; with `ex`, element i + q counts as
// |value| 2^ex[q]
template <int KIND>
__device__ inline double quad_absmax(const void* hi, const void* lo, int64_t i, const int32_t* ex = nullptr) {
  int32_t e[4] = {0, 0, 0, 0};
  if (ex) {
    if ((reinterpret_cast<uintptr_t>(ex) & 15) == 0) {
      const int4 v = *reinterpret_cast<const int4*>(ex);
      e[0] = v.x;
      e[1] = v.y;
      e[2] = v.z;
      e[3] = v.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) e[q] = ex[q];
    }
  }
  auto w = [&](double v, int q) { return ex ? ldexp(fabs(v), e[q]) : fabs(v); };
  double m = 0.0;
  if constexpr (KIND == 1) {
    const float* p = static_cast<const float*>(hi) + i;
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
      const float4 v = *reinterpret_cast<const float4*>(p);
      if (!ex) return double(fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
      return fmax(fmax(w(v.x, 0), w(v.y, 1)), fmax(w(v.z, 2), w(v.w, 3)));
    }
  } else if constexpr (KIND == 0) {
    const double* p = static_cast<const double*>(hi) + i;
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
      const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
      return fmax(fmax(w(a.x, 0), w(a.y, 1)), fmax(w(b.x, 2), w(b.y, 3)));
    }
  } else {
    const uint16_t* h = static_cast<const uint16_t*>(hi) + i;
    const uint16_t* l = lo ? static_cast<const uint16_t*>(lo) + i : nullptr;
    if ((reinterpret_cast<uintptr_t>(h) & 7) == 0 && (!l || (reinterpret_cast<uintptr_t>(l) & 7) == 0)) {
      const uint2 hv = *reinterpret_cast<const uint2*>(h);
      const uint2 lv = l ? *reinterpret_cast<const uint2*>(l) : make_uint2(0u, 0u);
      const uint16_t hs[4] = {(uint16_t)hv.x, (uint16_t)(hv.x >> 16), (uint16_t)hv.y, (uint16_t)(hv.y >> 16)};
      const uint16_t ls[4] = {(uint16_t)lv.x, (uint16_t)(lv.x >> 16), (uint16_t)lv.y, (uint16_t)(lv.y >> 16)};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double v = double(from_h16<KIND == 3>(hs[q]));
        if (l) v += double(from_h16<KIND == 3>(ls[q]));
        m = fmax(m, w(v, q));
      }
      return m;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) m = fmax(m, w(operand_at<KIND>(hi, lo, i + q), q));
  return m;
}

// Max |value| of every 128-element row segment of A (then of B).  Each half
// wave takes a segment (four consecutive elements per lane), and a wave
// loads four pairs of segments before reducing any, so sixteen loads per
// lane are in flight; the waves of the grid take the segments in turn.
// Column-scaled operands (rowtmax set): an element of output row z * M + m
// of A counts as |a| 2^rowexp, one of column n of B as |b| 2^colexp, so the
// bound is the sum over k of the largest magnitudes the epilogue's
// exponents give (these are the unscaled magnitudes, well inside FP32's
// range; a maximum below it rounds up to the smallest subnormal, still an
// upper bound).  A's maxima are kept per batch only when A varies with it;
// else A's rows count unweighted and the bound adds the tile's largest row
// exponent instead, looser but still a bound.
template <int KIND>
__global__ void __launch_bounds__(256) tile_rowmax_kernel(const GemmArgs* __restrict__ gp, float* amax,
                                                          float* bmax, int64_t slot) {
  constexpr int U = 4;  // segment pairs per wave and round
  const GemmArgs g = *inst_ptr(gp, slot);
  amax = inst_ptr(amax, slot);
  bmax = inst_ptr(bmax, slot);
  const int lane = threadIdx.x & 63, half = lane >> 5, sub = lane & 31;
  const int64_t Z = g.tilesM * g.tilesN > 0 ? g.tiles / (g.tilesM * g.tilesN) : 0;
  const int64_t za_n = g.sAz ? Z : 1, zb_n = g.sBz ? Z : 1;
  const int64_t na = za_n * g.K * g.tilesM, nb = zb_n * g.K * g.tilesN;
  const int64_t total = na + nb;
  const bool small = total < ((int64_t)1 << 31) && g.K < ((int64_t)1 << 31);
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w * 2 * U < total; w += waves) {
    double m[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      m[u] = 0.0;
      const int64_t seg = (w * U + u) * 2 + half;
      if (seg < total) {
        const bool isA = seg < na;
        const int64_t s = isA ? seg : seg - na;
        const int64_t tl = isA ? g.tilesM : g.tilesN;
        int64_t t, k, z;
        if (small) {  // 32-bit division: the 64-bit one costs a hundred instructions
          const uint32_t s32 = (uint32_t)s, tl32 = (uint32_t)tl, K32 = (uint32_t)g.K, zk = s32 / tl32;
          t = s32 - zk * tl32;
          z = zk / K32;
          k = zk - (uint32_t)z * K32;
        } else {
          const int64_t zk = s / tl;
          t = s - zk * tl;
          z = zk / g.K;
          k = zk - z * g.K;
        }
        const int64_t base = isA ? z * g.sAz + k * g.sAk : z * g.sBz + k * g.sBk;
        const int64_t lim = isA ? g.M : g.N;
        const void* hi = isA ? g.A : g.B;
        const void* lo = isA ? g.A_lo : g.B_lo;
        const int64_t c0 = t * 128 + sub * 4;
        const int32_t* ex = nullptr;
        if (g.rowtmax) {
          if (isA && (g.sAz != 0 || Z == 1)) ex = g.rowexp + z * g.M;
          else if (!isA) ex = g.colexp;
        }
        if (ex && c0 + 4 <= lim) {
          m[u] = quad_absmax<KIND>(hi, lo, base + c0, ex + c0);
        } else if (ex) {
          for (int q = 0; q < 4; ++q)
            if (c0 + q < lim)
              m[u] = fmax(m[u], ldexp(fabs(operand_at<KIND>(hi, lo, base + c0 + q)), ex[c0 + q]));
        } else if (c0 + 4 <= lim) {
          m[u] = quad_absmax<KIND>(hi, lo, base + c0);
        } else {
          for (int q = 0; q < 4; ++q)
            if (c0 + q < lim) m[u] = fmax(m[u], fabs(operand_at<KIND>(hi, lo, base + c0 + q)));
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      for (int o = 16; o >= 1; o >>= 1) m[u] = fmax(m[u], __shfl_xor(m[u], o));  // within the half wave
      const int64_t seg = (w * U + u) * 2 + half;
      if (sub == 0 && seg < total) {
        const bool isA = seg < na;
        (isA ? amax : bmax)[isA ? seg : seg - na] = __double2float_ru(m[u]);
      }
    }
  }
}

__global__ void __launch_bounds__(256) tile_bound_kernel(const GemmArgs* __restrict__ gp,
                                                         const float* __restrict__ amax,
                                                         const float* __restrict__ bmax, float* U,
                                                         int64_t slot) {
  const GemmArgs g = *inst_ptr(gp, slot);
  amax = inst_ptr(amax, slot);
  bmax = inst_ptr(bmax, slot);
  U = inst_ptr(U, slot);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.tiles) return;
  const TileCoord c = tile_coord_of<128, 128>(g, t);
  const int64_t mt = c.m0 / 128, nt = c.n0 / 128;
  const int64_t za = g.sAz ? c.z : 0, zb = g.sBz ? c.z : 0;
  double u = 0.0;
  for (int64_t k = 0; k < g.K; ++k)
    u += double(amax[(za * g.K + k) * g.tilesM + mt]) * double(bmax[(zb * g.K + k) * g.tilesN + nt]);
  // the kernels accumulate in FP32 (or FP64): allow K roundings of 2^-24
  u *= g.alpha * (1.0 + double(g.K + 4) * 0x1p-23);
  // column-scaled operands with A shared across batches: A's rows counted
  // unweighted, so the tile's largest row exponent is added here
  if (g.rowtmax && g.sAz == 0 && g.tiles > g.tilesM * g.tilesN) u = ldexp(u, g.rowtmax[c.z * g.tilesM + mt]);
  U[t] = __double2float_ru(u);
}

// Warm-up tiles: block b of `warm` takes the tile with the largest bound in
// slice b of the tiles (any tiles would do: they only raise the threshold).
__global__ void __launch_bounds__(256) tile_warm_kernel(const float* __restrict__ U,
                                                        const int64_t* __restrict__ n_tiles,
                                                        const int64_t* __restrict__ warm,
                                                        uint64_t* list, int64_t slot) {
  __shared__ float bv[4];
  __shared__ uint64_t bi[4];
  U = inst_ptr(U, slot);
  n_tiles = inst_ptr(n_tiles, slot);
  warm = inst_ptr(warm, slot);
  list = inst_ptr(list, slot);
  const int64_t n = *n_tiles, w = *warm;
  if ((int64_t)blockIdx.x >= w) return;
  const int64_t chunk = n / w;
  const int64_t begin = blockIdx.x * chunk;
  const int64_t end = (int64_t)blockIdx.x == w - 1 ? n : begin + chunk;
  float v = -INFINITY;
  uint64_t id = (uint64_t)begin;
  for (int64_t t = begin + threadIdx.x; t < end; t += blockDim.x)
    if (U[t] > v) {
      v = U[t];
      id = (uint64_t)t;
    }
  for (int o = 32; o >= 1; o >>= 1) {
    const float ov = __shfl_xor(v, o);
    const uint64_t oi = (uint64_t)__shfl_xor((long long)id, o);
    if (ov > v || (ov == v && oi < id)) {
      v = ov;
      id = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    bv[wave] = v;
    bi[wave] = id;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k)
      if (bv[k] > v || (bv[k] == v && bi[k] < id)) {
        v = bv[k];
        id = bi[k];
      }
    list[blockIdx.x] = id;
  }
}

__global__ void __launch_bounds__(256) tile_compact_kernel(const float* __restrict__ U,
                                                           const int64_t* __restrict__ n_tiles,
                                                           const unsigned long long* __restrict__ thr,
                                                           uint64_t* list, int64_t* count, int64_t slot) {
  U = inst_ptr(U, slot);
  n_tiles = inst_ptr(n_tiles, slot);
  thr = inst_ptr(thr, slot);
  list = inst_ptr(list, slot);
  count = inst_ptr(count, slot);
  // one atomic per wave: lanes take consecutive places by their rank among
  // the wave's passing lanes
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = *n_tiles;
  const bool pass = t < n && double(U[t]) >= ord_val(*thr);
  const uint64_t bal = __ballot(pass);
  if (bal == 0) return;
  const int lane = threadIdx.x & 63;
  const int rank = __popcll(bal & ((1ull << lane) - 1));
  unsigned long long base = 0;
  if (rank == 0 && pass)
    base = atomicAdd(reinterpret_cast<unsigned long long*>(count), (unsigned long long)__popcll(bal));
  base = (unsigned long long)__shfl((long long)base, __ffsll((unsigned long long)bal) - 1);
  if (pass) list[base + rank] = (uint64_t)t;
}

}  // namespace

hipError_t launch_tile_bounds(const GemmArgs* dev, DType t, bool f16, float* amax, float* bmax,
                              float* U, int64_t max_seg_a, int64_t max_seg_b, int64_t max_tiles,
                              hipStream_t stream, InstSpan span) {
  const int64_t segs = max_seg_a + max_seg_b;
  if (segs <= 0 || max_tiles <= 0 || span.n <= 0) return hipSuccess;
  const int64_t blocks = (segs * 64 + 255) / 256;
  const dim3 g1((unsigned)(blocks < 1024 ? blocks : 1024), 1, (unsigned)span.n);
  const int64_t sl = span.stride;
  switch (t) {
    case DType::F64: hipLaunchKernelGGL(tile_rowmax_kernel<0>, g1, dim3(256), 0, stream, dev, amax, bmax, sl); break;
    case DType::F32: hipLaunchKernelGGL(tile_rowmax_kernel<1>, g1, dim3(256), 0, stream, dev, amax, bmax, sl); break;
    default:
      if (f16) hipLaunchKernelGGL(tile_rowmax_kernel<3>, g1, dim3(256), 0, stream, dev, amax, bmax, sl);
      else hipLaunchKernelGGL(tile_rowmax_kernel<2>, g1, dim3(256), 0, stream, dev, amax, bmax, sl);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tile_bound_kernel, dim3((unsigned)((max_tiles + 255) / 256), 1, (unsigned)span.n),
                     dim3(256), 0, stream, dev, (const float*)amax, (const float*)bmax, U, sl);
  return hipGetLastError();
}

hipError_t launch_tile_warm(const float* U, const int64_t* n_tiles, const int64_t* warm,
                            uint64_t* list, int max_warm, hipStream_t stream, InstSpan span) {
  if (max_warm <= 0 || span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(tile_warm_kernel, dim3((unsigned)max_warm, 1, (unsigned)span.n), dim3(256), 0, stream, U,
                     n_tiles, warm, list, span.stride);
  return hipGetLastError();
}

hipError_t launch_tile_compact(const float* U, const int64_t* n_tiles,
                               const unsigned long long* thr_key, uint64_t* list,
                               int64_t* count, int64_t max_tiles, hipStream_t stream, InstSpan span) {
  if (max_tiles <= 0 || span.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(tile_compact_kernel, dim3((unsigned)((max_tiles + 255) / 256), 1, (unsigned)span.n),
                     dim3(256), 0, stream, U, n_tiles, thr_key, list, count, span.stride);
  return hipGetLastError();
}

constexpr int64_t kTopcGrid = 1024;
constexpr int64_t kIndGrid = 4096;

hipError_t launch_gemm_indirect(cq_precision prec, const GemmArgs* dev, int64_t max_tiles,
                                DType tc, bool nontemporal, bool topc, hipStream_t stream,
                                InstSpan span) {
  if (topc) {
    // the tiles come from a pruned list whose length only the device knows:
    // a few workgroups per CU walk it instead of one per possible tile (a
    // grid of 2^18 workgroups that mostly exit costs 0.4-0.8 ms by itself)
    const int64_t grid = max_tiles < kTopcGrid ? max_tiles : kTopcGrid;
    switch (prec) {
      case CQ_FP64: return launch_ind(gemm_f64_kernel<false, true>, dev, grid, stream, span, 512);
      case CQ_FP32: return launch_ind(gemm_f32_kernel<false, true>, dev, grid, stream, span);
      case CQ_BF16: return launch_ind(gemm_h16_kernel<1, false, 3>, dev, grid, stream, span);
      case CQ_BF16_SPLIT: return launch_ind(gemm_h16_kernel<3, false, 3>, dev, grid, stream, span);
      case CQ_FP16: return launch_ind(gemm_h16_kernel<1, true, 3>, dev, grid, stream, span);
      case CQ_FP16_SPLIT: return launch_ind(gemm_h16_kernel<3, true, 3>, dev, grid, stream, span);
    }
    return hipErrorInvalidValue;
  }
  // beyond kIndGrid tiles the workgroups loop (a multiple of 8 keeps each on its XCD)
  max_tiles = max_tiles < kIndGrid ? max_tiles : kIndGrid;
  switch (prec) {
    case CQ_FP64:
      return nontemporal ? launch_ind(gemm_f64_kernel<true>, dev, max_tiles, stream, span, 512)
                         : launch_ind(gemm_f64_kernel<false>, dev, max_tiles, stream, span, 512);
    case CQ_FP32:
      return nontemporal ? launch_ind(gemm_f32_kernel<true>, dev, max_tiles, stream, span)
                         : launch_ind(gemm_f32_kernel<false>, dev, max_tiles, stream, span);
    case CQ_BF16:
      if (tc == DType::F32) return launch_ind(gemm_h16_kernel<1, false, 0>, dev, max_tiles, stream, span);
      return launch_ind(gemm_h16_kernel<1, false, 2>, dev, max_tiles, stream, span);
    case CQ_BF16_SPLIT:
      if (tc == DType::F32) return launch_ind(gemm_h16_kernel<3, false, 0>, dev, max_tiles, stream, span);
      return launch_ind(gemm_h16_kernel<3, false, 2>, dev, max_tiles, stream, span);
    case CQ_FP16:
      if (tc == DType::F32) return launch_ind(gemm_h16_kernel<1, true, 0>, dev, max_tiles, stream, span);
      return launch_ind(gemm_h16_kernel<1, true, 2>, dev, max_tiles, stream, span);
    case CQ_FP16_SPLIT:
      if (tc == DType::F32) return launch_ind(gemm_h16_kernel<3, true, 0>, dev, max_tiles, stream, span);
      return launch_ind(gemm_h16_kernel<3, true, 2>, dev, max_tiles, stream, span);
  }
  return hipErrorInvalidValue;
}

}  // namespace cq

// State-vector simulation on the device: the noiseless output distribution
// of a circuit of one-qubit unitaries and CZ gates (the ground truth of
// Section 2), and every variant of a subcircuit (Section 3.1: each cut-end
// initialisation |0>, |1>, |+>, |+i> and each measurement basis Z, X, Y).
//
// Amplitudes are FP64 complex, qubit 0 the most significant index bit.
// Gates run in groups: gates whose qubits fit one tile of kTileBits index
// bits are applied together to tiles of 2^kTileBits amplitudes staged in
// LDS (one workgroup a tile, the tile's other index bits fixed), in circuit
// order, so the state makes one HBM round trip per group instead of one per
// gate.  A tile always holds the kLowBits lowest index bits, which keeps
// the gathers coalesced, and a group may take a later gate that commutes
// with every gate it overtakes (no shared qubit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace cq {

namespace {

constexpr int kTileBits = 11;
constexpr int kLowBits = 4;
constexpr int kTile = 1 << kTileBits;
constexpr int kSvThreads = 256;
constexpr int kPerThread = kTile / kSvThreads;
constexpr int kMaxGroupGates = 40;
constexpr int kMaxBases = 9;  // measurement bases one tile pass writes (two measured slots)

struct TileGate {
  int32_t kind;  // CQ_GATE_U or CQ_GATE_CZ
  int32_t a, b;  // tile-local bit positions (b for CZ only)
  int32_t pad;
  double u[8];   // (re, im) of u00, u01, u10, u11
};

// One launch: the tile's index bits (ascending), the complement bits that
// number the tiles, and the gates.  mode 0 writes amplitudes back, mode 1
// writes |amplitude|^2 to `probs` in the same index order.
struct TileGroup {
  int32_t k;          // tile bits (<= kTileBits)
  int32_t ngates;
  int32_t mode;
  int32_t nouter;     // index bits outside the tile
  uint8_t bits[kTileBits];
  uint8_t outer[CQ_MAX_SV_QUBITS];
  TileGate g[kMaxGroupGates];
  int32_t nbasis;                // sv_reg_kernel<true>: bases and their gate ranges
  int32_t boff[kMaxBases + 1];
  int64_t pstride;               // elements between the bases' outputs
  // sv_reg_kernel with blockIdx.y = state s of a batch: in and out start
  // s * bstride elements on, probs s * pbstride on (both 0 without a batch)
  int64_t bstride;
  int64_t pbstride;
};

static_assert(sizeof(TileGroup) + 3 * sizeof(void*) <= 4096, "kernel arguments exceed 4 KiB");

struct Complex {
  double re, im;
};

__device__ inline Complex cmul(double ur, double ui, Complex x) {
  return {ur * x.re - ui * x.im, ur * x.im + ui * x.re};
}

// `in` and `out` may be the same array (each workgroup reads and writes only
// its own tile); a null `in` stands for |0...0> (nothing is read).
__global__ void __launch_bounds__(kSvThreads) sv_tile_kernel(const double2* in, double2* out, double* probs,
                                                             TileGroup G) {
  __shared__ double2 S[kTile];
  // the tile's base address: the workgroup index deposited into the outer bits
  uint64_t base = 0;
  const uint64_t w = blockIdx.x;
  for (int i = 0; i < G.nouter; ++i) base |= ((w >> i) & 1ull) << G.outer[i];
  const int n = 1 << G.k;
  uint64_t addr[kPerThread];
#pragma unroll
  for (int e = 0; e < kPerThread; ++e) {
    const int t = threadIdx.x + e * kSvThreads;
    uint64_t a = base;
    for (int i = 0; i < G.k; ++i) a |= (uint64_t)((t >> i) & 1) << G.bits[i];
    addr[e] = a;
    if (t < n) S[t] = in ? in[a] : make_double2(a == 0 ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int gi = 0; gi < G.ngates; ++gi) {
    const TileGate& g = G.g[gi];
    if (g.kind == CQ_GATE_U) {
      const int half = n >> 1, m = 1 << g.a;
      for (int p = threadIdx.x; p < half; p += kSvThreads) {
        const int i0 = ((p >> g.a) << (g.a + 1)) | (p & (m - 1)), i1 = i0 | m;
        const Complex x0{S[i0].x, S[i0].y}, x1{S[i1].x, S[i1].y};
        const Complex a0 = cmul(g.u[0], g.u[1], x0), b0 = cmul(g.u[2], g.u[3], x1);
        const Complex a1 = cmul(g.u[4], g.u[5], x0), b1 = cmul(g.u[6], g.u[7], x1);
        S[i0] = make_double2(a0.re + b0.re, a0.im + b0.im);
        S[i1] = make_double2(a1.re + b1.re, a1.im + b1.im);
      }
    } else {
      const int both = (1 << g.a) | (1 << g.b);
      for (int t = threadIdx.x; t < n; t += kSvThreads)
        if ((t & both) == both) S[t] = make_double2(-S[t].x, -S[t].y);
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < kPerThread; ++e) {
    const int t = threadIdx.x + e * kSvThreads;
    if (t < n) {
      const double2 v = S[t];
      if (G.mode == 0) out[addr[e]] = v;
      else probs[addr[e]] = v.x * v.x + v.y * v.y;
    }
  }
}

// Full tiles (kTileBits bits) keep the amplitudes in registers: thread t
// holds local indices t + 256 e, e = 0..7, so local bits 0-5 are lane bits,
// 6-7 wave bits and 8-10 register bits.  CZ is a sign flip on elements the
// thread owns; a one-qubit gate on a register bit pairs two of the thread's
// own elements; on a lane bit the partner comes from another lane by a
// cross-lane read; on a wave bit it goes through LDS.  The host places the
// group's busiest qubits on register bits.
__device__ inline double2 u_row(double r0, double i0, double r1, double i1, double2 x, double2 y) {
  // (r0 + i i0) x + (r1 + i i1) y
  return make_double2(r0 * x.x - i0 * x.y + r1 * y.x - i1 * y.y, r0 * x.y + i0 * x.x + r1 * y.y + i1 * y.x);
}

template <int R>
__device__ inline void u_reg(double2 (&v)[kPerThread], const double* u) {
#pragma unroll
  for (int e = 0; e < kPerThread; ++e) {
    if (e & (1 << R)) continue;
    const double2 x0 = v[e], x1 = v[e | (1 << R)];
    v[e] = u_row(u[0], u[1], u[2], u[3], x0, x1);
    v[e | (1 << R)] = u_row(u[4], u[5], u[6], u[7], x0, x1);
  }
}

// An element whose partner (the other value of its pair) sits elsewhere:
// bit 0 takes u00 * mine + u01 * partner, bit 1 u11 * mine + u10 * partner.
// The two coefficients are picked once per gate, so each element costs one
// complex row, not two and a select.
struct ExchangeCoef {
  double ar, ai, br, bi;  // coefficient of mine, of the partner
};

// A coefficient every lane reads alike, taken through the first lane so that
// the per-lane choice below selects values, not addresses (a per-lane
// address would turn each coefficient into a vector load that the gate
// then waits for).
__device__ inline double uniform_coef(const double* p) {
  const uint64_t b = __builtin_bit_cast(uint64_t, *p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

__device__ inline ExchangeCoef exchange_coef(const double* u, int bit) {
  const ExchangeCoef c0{uniform_coef(u + 0), uniform_coef(u + 1), uniform_coef(u + 2), uniform_coef(u + 3)};
  const ExchangeCoef c1{uniform_coef(u + 6), uniform_coef(u + 7), uniform_coef(u + 4), uniform_coef(u + 5)};
  return bit ? c1 : c0;
}

__device__ inline double2 u_exchange(const ExchangeCoef& c, double2 mine, double2 y) {
  return u_row(c.ar, c.ai, c.br, c.bi, mine, y);
}

template <int M>
__device__ inline void u_lane(double2 (&v)[kPerThread], const double* u, int lane) {
  const ExchangeCoef c = exchange_coef(u, (lane & M) ? 1 : 0);
#pragma unroll
  for (int e = 0; e < kPerThread; ++e) {
    const double2 y = make_double2(__shfl_xor(v[e].x, M), __shfl_xor(v[e].y, M));
    v[e] = u_exchange(c, v[e], y);
  }
}

// Gates g0 .. g1 - 1 of the group on a thread's elements (see sv_reg_kernel);
// S is the workgroup's exchange buffer.
__device__ __forceinline__ void reg_apply(double2 (&v)[kPerThread], const TileGroup& G, int g0, int g1, int tid,
                                          int lane, double2* S) {
  for (int gi = g0; gi < g1; ++gi) {
    const TileGate& g = G.g[gi];
    if (g.kind == CQ_GATE_CZ) {
      // A run of CZs is diagonal: element tid + 256 e changes sign by the
      // parity, over the run's pairs, of the product of the pair's two bits.
      // Bits 0-7 are tid's and bits 8-10 e's, so per thread: s, the parity of
      // the pairs inside tid; p bit r, that of the tid bits paired with bit
      // 8 + r; rr, which pairs of bits 8-10 occur (an odd number of times).
      uint32_t sgn = 0, p = 0, rr = 0;
      int j = gi;
      for (; j < g1 && G.g[j].kind == CQ_GATE_CZ; ++j) {
        const int a = G.g[j].a, b = G.g[j].b;
        if (a < 8 && b < 8) sgn ^= ((uint32_t)tid >> a) & ((uint32_t)tid >> b) & 1u;
        else if (a < 8) p ^= (((uint32_t)tid >> a) & 1u) << (b - 8);
        else if (b < 8) p ^= (((uint32_t)tid >> b) & 1u) << (a - 8);
        else rr ^= 1u << ((a - 8) + (b - 8) - 1);  // bits (8,9), (8,10), (9,10)
      }
      gi = j - 1;
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) {
        uint32_t f = sgn;
        if (e & 1) f ^= p & 1u;
        if (e & 2) f ^= (p >> 1) & 1u;
        if (e & 4) f ^= (p >> 2) & 1u;
        if ((e & 3) == 3) f ^= rr & 1u;
        if ((e & 5) == 5) f ^= (rr >> 1) & 1u;
        if ((e & 6) == 6) f ^= (rr >> 2) & 1u;
        if (f) v[e] = make_double2(-v[e].x, -v[e].y);
      }
    } else if (g.a >= 8) {
      if (g.a == 8) u_reg<0>(v, g.u);
      else if (g.a == 9) u_reg<1>(v, g.u);
      else u_reg<2>(v, g.u);
    } else if (g.a < 6) {
      switch (g.a) {
        case 0: u_lane<1>(v, g.u, lane); break;
        case 1: u_lane<2>(v, g.u, lane); break;
        case 2: u_lane<4>(v, g.u, lane); break;
        case 3: u_lane<8>(v, g.u, lane); break;
        case 4: u_lane<16>(v, g.u, lane); break;
        default: u_lane<32>(v, g.u, lane); break;
      }
    } else {
      const ExchangeCoef c = exchange_coef(g.u, (tid >> g.a) & 1);
      const int m = 1 << g.a;
      __syncthreads();  // the previous exchange has read S
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) S[tid + e * kSvThreads] = v[e];
      __syncthreads();
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) v[e] = u_exchange(c, v[e], S[(tid + e * kSvThreads) ^ m]);
    }
  }
}

// MULTI: the group holds the rotations of nbasis measurement bases (gates
// boff[b] .. boff[b+1] - 1 for basis b); the tile is read once and each
// basis writes |amplitude|^2 of its rotated copy to probs + b * pstride.
template <bool MULTI>
__global__ void __launch_bounds__(kSvThreads) sv_reg_kernel(const double2* in, double2* out, double* probs,
                                                            TileGroup G) {
  static_assert(kPerThread == 8 && kSvThreads == 256, "bit layout assumes 8 elements a thread, 256 threads");
  __shared__ double2 S[kTile];
  if (blockIdx.y) {  // state blockIdx.y of a batch
    if (in) in += blockIdx.y * G.bstride;
    out += blockIdx.y * G.bstride;
    if (probs) probs += blockIdx.y * G.pbstride;
  }
  uint64_t base = 0;
  const uint64_t w = blockIdx.x;
  for (int i = 0; i < G.nouter; ++i) base |= ((w >> i) & 1ull) << G.outer[i];
  const int tid = threadIdx.x, lane = tid & 63;
  // local index tid + 256 e: its bits 0-7 are tid's (one per-thread part of
  // the address), bits 8-10 are e's (a part every thread shares), so no
  // per-element address has to stay live from the load to the store
  uint64_t tpart = base;
  for (int i = 0; i < 8; ++i) tpart |= (uint64_t)((tid >> i) & 1) << G.bits[i];
  auto addr_of = [&](int e) -> uint64_t {
    uint64_t a = tpart;
    for (int i = 8; i < kTileBits; ++i) a |= (uint64_t)((e >> (i - 8)) & 1) << G.bits[i];
    return a;
  };
  double2 v[kPerThread];
#pragma unroll
  for (int e = 0; e < kPerThread; ++e) {
    const uint64_t a = addr_of(e);
    v[e] = in ? in[a] : make_double2(a == 0 ? 1.0 : 0.0, 0.0);  // null in: |0...0>
  }
  if constexpr (MULTI) {
    for (int b = 0; b < G.nbasis; ++b) {
      double2 r[kPerThread];
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) r[e] = v[e];
      reg_apply(r, G, G.boff[b], G.boff[b + 1], tid, lane, S);
      double* const pb = probs + (int64_t)b * G.pstride;
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) pb[addr_of(e)] = r[e].x * r[e].x + r[e].y * r[e].y;
    }
  } else {
    reg_apply(v, G, 0, G.ngates, tid, lane, S);
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
      const uint64_t a = addr_of(e);
      if (G.mode == 0) out[a] = v[e];
      else probs[a] = v[e].x * v[e].x + v[e].y * v[e].y;
    }
  }
}

// Variants by linearity.  An init string prepares each init slot t in
// ket(d_t) = c0(d_t)|0> + c1(d_t)|1> (|0>, |1>, |+>, |+i>), so its
// post-circuit state is sum over c in {0,1}^r of w_j(c) S_c, with
// w_j(c) = prod_t c_{c_t}(d_t) and S_c the post-circuit state of the
// computational init string c (slot t in |c_t>, c_t bit r - 1 - t of c).  The
// 2^r states S_c (r <= 2) sit `G.bstride` elements apart from `in`; for each
// measurement basis b every S_c tile is read and rotated (gates
// boff[b] .. boff[b+1] - 1), and each init string j (digit t of j base 4,
// first slot most significant) writes |sum_c w_j(c) R_b S_c|^2 to
// probs + (j * nbasis + b) * pstride.
__device__ __constant__ double kInitKet[4][4] = {
    {1.0, 0.0, 0.0, 0.0},
    {0.0, 0.0, 1.0, 0.0},
    {0.70710678118654752440, 0.0, 0.70710678118654752440, 0.0},
    {0.70710678118654752440, 0.0, 0.0, 0.70710678118654752440}};

__global__ void __launch_bounds__(kSvThreads) sv_combine_kernel(const double2* in, double* probs, TileGroup G,
                                                                int r) {
  __shared__ double2 S[kTile];
  uint64_t base = 0;
  const uint64_t w = blockIdx.x;
  for (int i = 0; i < G.nouter; ++i) base |= ((w >> i) & 1ull) << G.outer[i];
  const int tid = threadIdx.x, lane = tid & 63;
  uint64_t tpart = base;
  for (int i = 0; i < 8; ++i) tpart |= (uint64_t)((tid >> i) & 1) << G.bits[i];
  auto addr_of = [&](int e) -> uint64_t {
    uint64_t a = tpart;
    for (int i = 8; i < kTileBits; ++i) a |= (uint64_t)((e >> (i - 8)) & 1) << G.bits[i];
    return a;
  };
  const int nc = 1 << r, nj = 1 << (2 * r);
  for (int b = 0; b < G.nbasis; ++b) {
    double2 rs[4][kPerThread];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= nc) break;
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) rs[c][e] = in[c * G.bstride + addr_of(e)];
      reg_apply(rs[c], G, G.boff[b], G.boff[b + 1], tid, lane, S);
    }
    for (int j = 0; j < nj; ++j) {
      double wr[4], wi[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double ar = 1.0, ai = 0.0;
        for (int t = 0; t < r; ++t) {
          const int d = (j >> (2 * (r - 1 - t))) & 3, bit = (c >> (r - 1 - t)) & 1;
          const double kr = kInitKet[d][2 * bit], ki = kInitKet[d][2 * bit + 1];
          const double nr = ar * kr - ai * ki;
          ai = ar * ki + ai * kr;
          ar = nr;
        }
        wr[c] = ar;
        wi[c] = ai;
      }
      double* const pj = probs + ((int64_t)j * G.nbasis + b) * G.pstride;
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) {
        double xr = 0.0, xi = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c >= nc) break;
          xr += wr[c] * rs[c][e].x - wi[c] * rs[c][e].y;
          xi += wr[c] * rs[c][e].y + wi[c] * rs[c][e].x;
        }
        pj[addr_of(e)] = xr * xr + xi * xi;
      }
    }
  }
}

// Product state: amplitude(x) = prod over qubits q of ket_q[bit q of x].
struct Kets {
  int32_t n;
  double k[CQ_MAX_WIDTH][4];  // (re, im) of <0|ket>, <1|ket> per qubit
  uint64_t zero;              // index bits of the qubits whose ket is exactly |0>
};

// Qubits in |0> contribute a factor of exactly 1 where their bit is 0 and
// make the amplitude 0 where it is 1, so only the others are multiplied.
__global__ void __launch_bounds__(kSvThreads) sv_product_kernel(double2* __restrict__ psi, int64_t size, Kets K) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < size; x += step) {
    if ((uint64_t)x & K.zero) {
      psi[x] = make_double2(0.0, 0.0);
      continue;
    }
    double re = 1.0, im = 0.0;
    for (int q = 0; q < K.n; ++q) {
      if ((K.zero >> (K.n - 1 - q)) & 1ull) continue;
      const int bit = (int)((x >> (K.n - 1 - q)) & 1);
      const double kr = K.k[q][2 * bit], ki = K.k[q][2 * bit + 1];
      const double nr = re * kr - im * ki;
      im = re * ki + im * kr;
      re = nr;
    }
    psi[x] = make_double2(re, im);
  }
}

unsigned fill_grid(int64_t size) {
  return (unsigned)std::min<int64_t>((size + kSvThreads - 1) / kSvThreads, 1 << 16);
}

cq_status sv_hip_error(hipError_t e, const char* what) {
  return fail(CQ_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

cq_status check_gates(int32_t n, const cq_gate* gates, int32_t n_gates) {
  if (n_gates < 0) return fail(CQ_ERR_ARG, "negative gate count");
  if (n_gates > 0 && !gates) return fail(CQ_ERR_ARG, "null gate array");
  for (int i = 0; i < n_gates; ++i) {
    const cq_gate& g = gates[i];
    if (g.kind != CQ_GATE_U && g.kind != CQ_GATE_CZ) return fail(CQ_ERR_ARG, "unknown gate kind");
    if (g.q0 < 0 || g.q0 >= n) return fail(CQ_ERR_ARG, "gate qubit out of range");
    if (g.kind == CQ_GATE_CZ && (g.q1 < 0 || g.q1 >= n || g.q1 == g.q0))
      return fail(CQ_ERR_ARG, "CZ qubits out of range or equal");
    if (g.kind == CQ_GATE_U)
      for (double v : g.u)
        if (!std::isfinite(v)) return fail(CQ_ERR_ARG, "non-finite gate matrix");
  }
  return CQ_OK;
}

// Gates -> groups whose index bits fit one tile together with the kLowBits
// lowest bits (which keep every gather in runs of 2^kLowBits amplitudes).
// A gate joins the open group when it fits and shares no qubit with an
// earlier gate left for a later group, so it commutes with every gate it
// overtakes; the gates of a group keep their circuit order.
struct Group {
  std::vector<int> gates;
  uint64_t mask = 0;
};

std::vector<Group> make_groups(int n, const cq_gate* gates, int n_gates, const std::vector<cq_gate>& tail) {
  const int k = std::min(n, kTileBits);
  const uint64_t low = (1ull << std::min(n, kLowBits)) - 1;
  auto bit = [n](int q) { return 1ull << (n - 1 - q); };
  const int total = n_gates + (int)tail.size();
  std::vector<uint64_t> masks(total);
  for (int i = 0; i < total; ++i) {
    const cq_gate& g = i < n_gates ? gates[i] : tail[i - n_gates];
    masks[i] = bit(g.q0) | (g.kind == CQ_GATE_CZ ? bit(g.q1) : 0ull);
  }
  std::vector<int> rest(total);
  for (int i = 0; i < total; ++i) rest[i] = i;
  std::vector<Group> out;
  while (!rest.empty()) {
    Group cur;
    uint64_t blocked = 0;
    std::vector<int> left;
    for (int i : rest) {
      const uint64_t m = masks[i];
      if ((m & blocked) == 0 && (int)cur.gates.size() < kMaxGroupGates &&
          __builtin_popcountll(cur.mask | m | low) <= k) {
        cur.gates.push_back(i);
        cur.mask |= m;
      } else {
        blocked |= m;
        left.push_back(i);
      }
    }
    out.push_back(cur);
    rest.swap(left);
  }
  return out;
}

TileGroup tile_group(int n, const Group& grp, const cq_gate* gates, int n_gates, const std::vector<cq_gate>& tail,
                     int mode) {
  TileGroup G{};
  const int k = std::min(n, kTileBits);
  uint64_t mask = grp.mask | ((1ull << std::min(n, kLowBits)) - 1);
  for (int b = 0; b < n && __builtin_popcountll(mask) < k; ++b) mask |= 1ull << b;
  G.k = k;
  G.mode = mode;
  auto gate = [&](int i) -> const cq_gate& { return i < n_gates ? gates[i] : tail[i - n_gates]; };
  // local positions: ascending global bits for partial tiles; for full
  // tiles the kLowBits lowest bits first (coalesced lanes), then the other
  // bits by one-qubit gate count, busiest first, on the register positions
  // 8-10, then lane positions 4-5, then wave positions 6-7
  std::vector<int> order;
  for (int b = 0; b < n; ++b)
    if (mask >> b & 1) order.push_back(b);
  if (k == kTileBits) {
    int uses[64] = {};
    for (int i : grp.gates)
      if (gate(i).kind == CQ_GATE_U) ++uses[n - 1 - gate(i).q0];
    std::vector<int> rest(order.begin() + kLowBits, order.end());
    std::stable_sort(rest.begin(), rest.end(), [&](int x, int y) { return uses[x] > uses[y]; });
    const int slot[kTileBits - kLowBits] = {8, 9, 10, 4, 5, 6, 7};
    std::vector<int> placed(kTileBits, -1);
    for (int i = 0; i < kLowBits; ++i) placed[i] = order[i];
    for (int i = 0; i < (int)rest.size(); ++i) placed[slot[i]] = rest[i];
    order = placed;
  }
  int local[64];
  int no = 0;
  for (int i = 0; i < k; ++i) {
    local[order[i]] = i;
    G.bits[i] = (uint8_t)order[i];
  }
  for (int b = 0; b < n; ++b)
    if (!(mask >> b & 1)) G.outer[no++] = (uint8_t)b;
  G.nouter = no;
  G.ngates = (int)grp.gates.size();
  for (int j = 0; j < G.ngates; ++j) {
    const cq_gate& g = gate(grp.gates[j]);
    TileGate& t = G.g[j];
    t.kind = g.kind;
    t.a = local[n - 1 - g.q0];
    t.b = g.kind == CQ_GATE_CZ ? local[n - 1 - g.q1] : 0;
    for (int c = 0; c < 8; ++c) t.u[c] = g.kind == CQ_GATE_U ? g.u[c] : 0.0;
  }
  return G;
}

// One tile pass: the register kernel for full tiles, the LDS kernel for
// registers narrower than a tile.
hipError_t launch_tiles(int n, const TileGroup& G, const double2* in, double2* out, double* probs,
                        hipStream_t stream) {
  const unsigned tiles = (unsigned)(1ull << (n - G.k));
  if (G.k == kTileBits)
    hipLaunchKernelGGL(sv_reg_kernel<false>, dim3(tiles), dim3(kSvThreads), 0, stream, in, out, probs, G);
  else
    hipLaunchKernelGGL(sv_tile_kernel, dim3(tiles), dim3(kSvThreads), 0, stream, in, out, probs, G);
  return hipGetLastError();
}

// Applies `gates` then `tail` to psi in place; the last group writes
// |amplitude|^2 to probs instead when probs is set (psi then keeps the state
// before that group), and a probability pass runs alone when there are no
// gates at all.  With zero_start the state starts as |0...0>, which the
// first pass generates instead of reading psi.
hipError_t run_gates(int n, const cq_gate* gates, int n_gates, const std::vector<cq_gate>& tail, double2* psi,
                     double* probs, hipStream_t stream, bool zero_start = false) {
  std::vector<Group> groups = make_groups(n, gates, n_gates, tail);
  if (groups.empty() && (probs || zero_start)) groups.push_back(Group());
  for (size_t i = 0; i < groups.size(); ++i) {
    const bool last = i + 1 == groups.size();
    const int mode = last && probs ? 1 : 0;
    const TileGroup G = tile_group(n, groups[i], gates, n_gates, tail, mode);
    const hipError_t e = launch_tiles(n, G, i == 0 && zero_start ? nullptr : psi, psi, probs, stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// States cq_variant_probabilities holds at once on the one-pass-bases path
// (a full tile, at most kMaxBases bases): the 2^r computational init strings
// with one or two initialised ends (the linear path), else all init strings
// up to 16; within 4 GiB and no more than `ws` bytes hold; one otherwise.
int64_t variant_batch(const SubInfo& si, size_t ws) {
  const int w = si.width;
  int64_t n_init = 1, n_basis = 1;
  for (int i = 0; i < si.r(); ++i) n_init *= 4;
  for (int i = 0; i < si.o(); ++i) n_basis *= 3;
  if (w < kTileBits || n_basis > kMaxBases) return 1;
  const size_t state = (size_t)16 << w;
  int64_t b = si.r() >= 1 && si.r() <= 2 ? ((int64_t)1 << si.r()) : std::min<int64_t>(n_init, 16);
  b = std::min<int64_t>(b, (int64_t)(((size_t)4 << 30) / state));
  b = std::min<int64_t>(b, (int64_t)(ws / state));
  return b < 1 ? 1 : b;
}

cq_gate u_gate(int q, const double (&m)[8]) {
  cq_gate g{};
  g.kind = CQ_GATE_U;
  g.q0 = q;
  for (int c = 0; c < 8; ++c) g.u[c] = m[c];
  return g;
}

}  // namespace

}  // namespace cq

using namespace cq;

extern "C" cq_status cq_simulate_workspace_size(int32_t n, size_t* bytes) {
  if (!bytes) return fail(CQ_ERR_ARG, "null argument");
  if (n < 1 || n > CQ_MAX_SV_QUBITS) return fail(CQ_ERR_SHAPE, "qubit count out of range");
  *bytes = (size_t)16 << n;
  return CQ_OK;
}

extern "C" cq_status cq_simulate_probabilities(int32_t n, const cq_gate* gates, int32_t n_gates, double* probs,
                                               void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!probs) return fail(CQ_ERR_ARG, "null argument");
  if (n < 1 || n > CQ_MAX_SV_QUBITS) return fail(CQ_ERR_SHAPE, "qubit count out of range");
  cq_status st = check_gates(n, gates, n_gates);
  if (st != CQ_OK) return st;
  if (!workspace || workspace_bytes < ((size_t)16 << n)) return fail(CQ_ERR_WORKSPACE, "workspace too small");
  double2* psi = static_cast<double2*>(workspace);
  // the first pass generates |0...0> itself (no zero fill, no read of it)
  const hipError_t e = run_gates(n, gates, n_gates, {}, psi, probs, stream, true);
  if (e != hipSuccess) return sv_hip_error(e, "state-vector launch");
  return CQ_OK;
}

extern "C" cq_status cq_variants_workspace_size(const cq_subcircuit* sub, size_t* bytes) {
  if (!bytes) return fail(CQ_ERR_ARG, "null argument");
  SubInfo si;
  cq_status st = build_subinfo(sub, si);
  if (st != CQ_OK) return st;
  if (si.width < 1) return fail(CQ_ERR_SHAPE, "subcircuit has no slots");
  *bytes = ((size_t)16 << si.width) * (size_t)variant_batch(si, (size_t)-1);
  return CQ_OK;
}

extern "C" cq_status cq_variant_probabilities(const cq_subcircuit* sub, const cq_gate* gates, int32_t n_gates,
                                              double* variants, void* workspace, size_t workspace_bytes,
                                              hipStream_t stream) {
  if (!variants) return fail(CQ_ERR_ARG, "null argument");
  SubInfo si;
  cq_status st = build_subinfo(sub, si);
  if (st != CQ_OK) return st;
  const int w = si.width;
  if (w < 1) return fail(CQ_ERR_SHAPE, "subcircuit has no slots");
  st = check_gates(w, gates, n_gates);
  if (st != CQ_OK) return st;
  if (!workspace || workspace_bytes < ((size_t)16 << w)) return fail(CQ_ERR_WORKSPACE, "workspace too small");
  double2* psi = static_cast<double2*>(workspace);
  const int64_t size = (int64_t)1 << w;
  const int r = si.r(), o = si.o();
  int64_t n_init = 1, n_basis = 1;
  for (int i = 0; i < r; ++i) n_init *= 4;
  for (int i = 0; i < o; ++i) n_basis *= 3;
  // prepared states of a cut's downstream end: |0>, |1>, |+>, |+i>
  const double h = 1.0 / std::sqrt(2.0);
  const double init_ket[4][4] = {{1, 0, 0, 0}, {0, 0, 1, 0}, {h, 0, h, 0}, {h, 0, 0, h}};
  // rotations before a computational-basis measurement: Z (none), X (H),
  // Y (S^dagger then H, i.e. H S^dagger = [[1, -i], [1, i]] / sqrt 2)
  const double rot_x[8] = {h, 0, h, 0, h, 0, -h, 0};
  const double rot_y[8] = {h, 0, 0, -h, h, 0, 0, h};
  // rotations of measurement basis b (digit 1: X, 2: Y per measured slot)
  auto basis_rot = [&](int64_t b) {
    std::vector<cq_gate> rot;
    int64_t rest = b;
    std::vector<int> digits(o);
    for (int u = o - 1; u >= 0; --u) {
      digits[u] = (int)(rest % 3);
      rest /= 3;
    }
    for (int u = 0; u < o; ++u) {
      if (digits[u] == 1) rot.push_back(u_gate(si.meas_slots[u], rot_x));
      if (digits[u] == 2) rot.push_back(u_gate(si.meas_slots[u], rot_y));
    }
    return rot;
  };
  // the one-pass-bases path (a full tile, at most kMaxBases bases) takes a
  // batch of initial states at once, as many as the workspace holds
  const bool one_pass = w >= kTileBits && n_basis <= kMaxBases;
  const int64_t batch = variant_batch(si, workspace_bytes);
  const unsigned tiles = one_pass ? (unsigned)(1ull << (w - kTileBits)) : 0u;
  TileGroup GB{};
  if (one_pass) {
    std::vector<cq_gate> all;
    std::vector<int> off{0};
    for (int64_t b = 0; b < n_basis; ++b) {
      const std::vector<cq_gate> rot = basis_rot(b);
      all.insert(all.end(), rot.begin(), rot.end());
      off.push_back((int)all.size());
    }
    Group grp;
    for (int i = 0; i < (int)all.size(); ++i) {
      grp.gates.push_back(i);
      grp.mask |= 1ull << (w - 1 - all[i].q0);
    }
    GB = tile_group(w, grp, nullptr, 0, all, 1);
    GB.nbasis = (int)n_basis;
    for (int b = 0; b <= (int)n_basis; ++b) GB.boff[b] = off[b];
    GB.pstride = size;
    GB.bstride = size;
    GB.pbstride = n_basis * size;
  }
  const std::vector<Group> circuit = one_pass ? make_groups(w, gates, n_gates, {}) : std::vector<Group>();
  // by linearity (one or two init slots): simulate the 2^r computational
  // init strings only and combine them per init string in the bases pass
  if (one_pass && r >= 1 && r <= 2 && workspace_bytes >= ((size_t)16 << w) * ((size_t)1 << r)) {
    const int nc = 1 << r;
    hipError_t e = hipSuccess;
    for (int c = 0; c < nc && e == hipSuccess; ++c) {
      Kets K{};
      K.n = w;
      for (int q = 0; q < w; ++q) {
        K.k[q][0] = 1.0;
        K.k[q][1] = K.k[q][2] = K.k[q][3] = 0.0;
      }
      for (int t = 0; t < r; ++t) {
        const int bit = (c >> (r - 1 - t)) & 1;
        for (int q = 0; q < 4; ++q) K.k[si.init_slots[t]][q] = init_ket[bit][q];
      }
      K.zero = 0;
      for (int q = 0; q < w; ++q)
        if (K.k[q][0] == 1.0 && K.k[q][1] == 0.0 && K.k[q][2] == 0.0 && K.k[q][3] == 0.0) K.zero |= 1ull << (w - 1 - q);
      hipLaunchKernelGGL(sv_product_kernel, dim3(fill_grid(size)), dim3(kSvThreads), 0, stream, psi + c * size, size,
                         K);
      e = hipGetLastError();
    }
    for (size_t g = 0; g < circuit.size() && e == hipSuccess; ++g) {
      TileGroup G = tile_group(w, circuit[g], gates, n_gates, {}, 0);
      G.bstride = size;
      hipLaunchKernelGGL(sv_reg_kernel<false>, dim3(tiles, (unsigned)nc), dim3(kSvThreads), 0, stream,
                         (const double2*)psi, psi, (double*)nullptr, G);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(sv_combine_kernel, dim3(tiles), dim3(kSvThreads), 0, stream, (const double2*)psi, variants, GB,
                         r);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return sv_hip_error(e, "variant launch");
    return CQ_OK;
  }
  for (int64_t j0 = 0; j0 < n_init; j0 += batch) {
    const int64_t nb = std::min<int64_t>(batch, n_init - j0);
    hipError_t e = hipSuccess;
    for (int64_t jj = 0; jj < nb && e == hipSuccess; ++jj) {
      const int64_t j = j0 + jj;
      Kets K{};
      K.n = w;
      for (int q = 0; q < w; ++q) {
        K.k[q][0] = 1.0;
        K.k[q][1] = K.k[q][2] = K.k[q][3] = 0.0;
      }
      for (int t = 0; t < r; ++t) {
        const int digit = (int)((j >> (2 * (r - 1 - t))) & 3);
        for (int c = 0; c < 4; ++c) K.k[si.init_slots[t]][c] = init_ket[digit][c];
      }
      K.zero = 0;
      for (int q = 0; q < w; ++q)
        if (K.k[q][0] == 1.0 && K.k[q][1] == 0.0 && K.k[q][2] == 0.0 && K.k[q][3] == 0.0) K.zero |= 1ull << (w - 1 - q);
      hipLaunchKernelGGL(sv_product_kernel, dim3(fill_grid(size)), dim3(kSvThreads), 0, stream, psi + jj * size, size,
                         K);
      e = hipGetLastError();
    }
    if (one_pass) {
      // the circuit on every state of the batch (grid y = state), then one
      // pass that reads each post-circuit tile once and writes every basis
      for (size_t g = 0; g < circuit.size() && e == hipSuccess; ++g) {
        TileGroup G = tile_group(w, circuit[g], gates, n_gates, {}, 0);
        G.bstride = size;
        hipLaunchKernelGGL(sv_reg_kernel<false>, dim3(tiles, (unsigned)nb), dim3(kSvThreads), 0, stream,
                           (const double2*)psi, psi, (double*)nullptr, G);
        e = hipGetLastError();
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL(sv_reg_kernel<true>, dim3(tiles, (unsigned)nb), dim3(kSvThreads), 0, stream,
                           (const double2*)psi, psi, variants + j0 * n_basis * size, GB);
        e = hipGetLastError();
      }
    } else {
      if (e == hipSuccess) e = run_gates(w, gates, n_gates, {}, psi, nullptr, stream);
      for (int64_t b = 0; b < n_basis && e == hipSuccess; ++b) {
        const std::vector<cq_gate> rot = basis_rot(b);
        // the rotations read psi and write probabilities only, so psi stays
        // the post-circuit state for the next basis; at most
        // CQ_MAX_LOCAL_CUTS measured slots, so they form one group
        double* out = variants + (j0 * n_basis + b) * size;
        std::vector<Group> groups = make_groups(w, nullptr, 0, rot);
        if (groups.empty()) groups.push_back(Group());
        const TileGroup G = tile_group(w, groups[0], nullptr, 0, rot, 1);
        e = launch_tiles(w, G, psi, psi, out, stream);
      }
    }
    if (e != hipSuccess) return sv_hip_error(e, "variant launch");
  }
  return CQ_OK;
}

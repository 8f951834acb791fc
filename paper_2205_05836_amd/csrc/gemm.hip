// Label GEMMs: one pairwise contraction of Eq. 1 over the shared cut labels.
//
//   C[z][m][n] = alpha * sum_k A[z*sAz + k*sAk + m] * B[z*sBz + k*sBk + n]
//
// Both operands keep the entry-tensor layout (labels slow, outputs fast), so
// tiles load along M and N with full 128-byte lines and no operand transpose
// pass is needed.  Matrix cores of gfx950 do the products:
//   FP64: v_mfma_f64_16x16x4_f64, FP32: v_mfma_f32_32x32x2_f32.
// Tiles: 128 x 128 per workgroup of 4 waves (64 x 64 each), K staged through
// LDS 16 labels at a time with a register prefetch of the next stage.
// Workgroups walk the tiles n-fastest so neighbours share A panels, and the
// flat tile index is remapped so that each of the 8 XCDs (each with its own
// L2) receives a contiguous range of tiles.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cq {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f16_t __attribute__((ext_vector_type(16)));

struct GemmArgs {
  const void* A;
  const void* B;
  void* C;
  int64_t M, N, K;
  int64_t sAz, sAk, sBz, sBk, sCz, ldc;
  int64_t tilesM, tilesN, tiles;
  double alpha;
};

// Workgroup b runs on XCD b % 8; give each XCD a contiguous block of tiles.
__device__ inline int64_t xcd_tile(int64_t b, int64_t total) {
  const int64_t per = total / 8, rem = total % 8;
  const int64_t xcd = b % 8, local = b / 8;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Loads 8 consecutive elements of row k (columns c0..c0+7) as double/float,
// zero outside [0, K) x [0, ncols).
template <typename T, typename R>
__device__ inline void load8(const T* __restrict__ P, int64_t k, int64_t sk, int64_t c0,
                             int64_t ncols, int64_t K, R (&out)[8]) {
  if (k >= K) {
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = R(0);
    return;
  }
  const T* p = P + k * sk + c0;
  if (c0 + 8 <= ncols && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
    if constexpr (sizeof(T) == 8) {
      typedef double dv2 __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        dv2 v = *reinterpret_cast<const dv2*>(p + e);
        out[e] = R(v[0]);
        out[e + 1] = R(v[1]);
      }
    } else {
      typedef float fv4 __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int e = 0; e < 8; e += 4) {
        fv4 v = *reinterpret_cast<const fv4*>(p + e);
        out[e] = R(v[0]);
        out[e + 1] = R(v[1]);
        out[e + 2] = R(v[2]);
        out[e + 3] = R(v[3]);
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = (c0 + e < ncols) ? R(p[e]) : R(0);
  }
}

template <typename TA, typename TB, typename TC>
__global__ void __launch_bounds__(256) gemm_f64_kernel(GemmArgs g) {
  constexpr int BM = 128, BN = 128, BK = 16;
  __shared__ double As[BK][BM];
  __shared__ double Bs[BK][BN];
  const int64_t tile = xcd_tile(blockIdx.x, g.tiles);
  const int64_t tn = tile % g.tilesN;
  const int64_t t2 = tile / g.tilesN;
  const int64_t tm = t2 % g.tilesM;
  const int64_t z = t2 / g.tilesM;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const TA* A = static_cast<const TA*>(g.A) + z * g.sAz;
  const TB* B = static_cast<const TB*>(g.B) + z * g.sBz;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int lr = tid >> 4, lc = (tid & 15) * 8;

  d4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  double ra[8], rb[8];
  load8(A, lr, g.sAk, m0 + lc, g.M, g.K, ra);
  load8(B, lr, g.sBk, n0 + lc, g.N, g.K, rb);
  for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[lr][lc + e] = ra[e];
      Bs[lr][lc + e] = rb[e];
    }
    __syncthreads();
    if (k0 + BK < g.K) {
      load8(A, k0 + BK + lr, g.sAk, m0 + lc, g.M, g.K, ra);
      load8(B, k0 + BK + lr, g.sBk, n0 + lc, g.N, g.K, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  TC* C = static_cast<TC*>(g.C) + z * g.sCz;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f64 16x16x4 accumulators: item v of lane l is row l/16 + 4v, column l%16
        const int64_t row = m0 + wm + i * 16 + (lane >> 4) + 4 * v;
        const int64_t col = n0 + wn + j * 16 + (lane & 15);
        if (row < g.M && col < g.N) C[row * g.ldc + col] = TC(g.alpha * acc[i][j][v]);
      }
}

template <typename TA, typename TB, typename TC>
__global__ void __launch_bounds__(256) gemm_f32_kernel(GemmArgs g) {
  constexpr int BM = 128, BN = 128, BK = 16;
  __shared__ float As[BK][BM];
  __shared__ float Bs[BK][BN];
  const int64_t tile = xcd_tile(blockIdx.x, g.tiles);
  const int64_t tn = tile % g.tilesN;
  const int64_t t2 = tile / g.tilesN;
  const int64_t tm = t2 % g.tilesM;
  const int64_t z = t2 / g.tilesM;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const TA* A = static_cast<const TA*>(g.A) + z * g.sAz;
  const TB* B = static_cast<const TB*>(g.B) + z * g.sBz;
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
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[lr][lc + e] = ra[e];
      Bs[lr][lc + e] = rb[e];
    }
    __syncthreads();
    if (k0 + BK < g.K) {
      load8(A, k0 + BK + lr, g.sAk, m0 + lc, g.M, g.K, ra);
      load8(B, k0 + BK + lr, g.sBk, n0 + lc, g.N, g.K, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
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
  TC* C = static_cast<TC*>(g.C) + z * g.sCz;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int64_t col = n0 + wn + j * 32 + (lane & 31);
        if (row < g.M && col < g.N) C[row * g.ldc + col] = TC(alpha * acc[i][j][v]);
      }
}

template <typename TA, typename TB, typename TC>
hipError_t run_f64(const GemmArgs& a, int64_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, TC>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC>
hipError_t run_f32(const GemmArgs& a, int64_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((gemm_f32_kernel<TA, TB, TC>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(cq_precision prec, const GemmLaunch& g, hipStream_t stream) {
  GemmArgs a;
  a.A = g.A;
  a.B = g.B;
  a.C = g.C;
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
  a.tilesM = (g.M + 127) / 128;
  a.tilesN = (g.N + 127) / 128;
  a.tiles = a.tilesM * a.tilesN * g.Z;
  if (a.tiles <= 0) return hipSuccess;
  if (a.tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool a64 = g.ta == DType::F64, b64 = g.tb == DType::F64, c64 = g.tc == DType::F64;
  if (prec == CQ_FP64) {
    if (!(a64 && b64 && c64)) return hipErrorInvalidValue;
    return run_f64<double, double, double>(a, a.tiles, stream);
  }
  if (prec == CQ_FP32) {
    if (c64) return hipErrorInvalidValue;
    if (a64 && b64) return run_f32<double, double, float>(a, a.tiles, stream);
    if (a64 && !b64) return run_f32<double, float, float>(a, a.tiles, stream);
    if (!a64 && b64) return run_f32<float, double, float>(a, a.tiles, stream);
    return run_f32<float, float, float>(a, a.tiles, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace cq

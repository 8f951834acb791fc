// Host-side launchers of the HIP kernels.  Each returns hipSuccess or the
// launch error; all work is enqueued on `stream`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cutqc.h"

namespace cq {

// Storage formats of contraction operands.  H16: one plane of 16-bit values
// (BF16 or FP16); H16X2: a hi plane followed by a lo plane of the same length
// (x = hi + lo).
enum class DType { F64, F32, H16, H16X2 };

inline int dtype_bytes(DType t) {
  return t == DType::F64 ? 8 : (t == DType::F32 || t == DType::H16X2 ? 4 : 2);
}

struct Operand {
  const void* p = nullptr;   // values, or the hi plane
  const void* lo = nullptr;  // lo plane (H16X2 only)
  DType t = DType::F64;
};

struct GemmLaunch {
  Operand a, b;
  void* C = nullptr;
  void* C_lo = nullptr;  // lo plane of C (H16X2 only)
  DType tc = DType::F64;
  int64_t Z, M, N, K;
  int64_t sAz, sAk, sBz, sBk, sCz, ldc;
  double alpha;
  bool nontemporal = false;  // final output: stores bypass the caches
};

// C[z][m][n] = alpha * sum_k A[z*sAz + k*sAk + m] * B[z*sBz + k*sBk + n]
hipError_t launch_gemm(cq_precision prec, const GemmLaunch& g, hipStream_t stream);

// Converts n FP64 values to `t` (FP32, or BF16/FP16 planes when f16 is false/true).
hipError_t launch_prep(const double* src, void* dst, int64_t n, DType t, bool f16,
                       hipStream_t stream);

constexpr int kMaxPermAxes = 48;
struct PermLaunch {
  Operand src;
  void* dst;
  void* dst_lo;
  DType td;
  bool f16;
  int naxes;
  int log2[kMaxPermAxes];
  int64_t sstride[kMaxPermAxes];
  double alpha;
};
// dst[i] = alpha * src[sum_a idx_a(i) * sstride[a]]; i spans prod 2^log2[a].
hipError_t launch_permute(const PermLaunch& p, hipStream_t stream);

struct AttrLaunch {
  const double* V;
  double* U;  // workspace (4^r, 4^o, 2^n)
  double* E;
  int r, o, n, w, k;
  int out_pos[CQ_MAX_WIDTH];   // register bit (from LSB) of output bit i (i = 0 MSB)
  int meas_pos[CQ_MAX_WIDTH];  // register bit of measured slot u
  int64_t init_w[CQ_MAX_WIDTH];  // label-row weight of init slot t's cut
  int64_t meas_w[CQ_MAX_WIDTH];  // label-row weight of measured slot u's cut
};
hipError_t launch_attribute(const AttrLaunch& a, hipStream_t stream);

// Dynamic definition helpers.
struct MergeLaunch {
  const double* E;   // (rows, 2^n)
  double* Ep;        // (rows, 2^na)
  int64_t rows;
  int n, na, nm;
  uint64_t active_flat, merged_flat, fixed_vals_flat;  // masks over flat bit positions
};
hipError_t launch_merge(const MergeLaunch& m, hipStream_t stream);

struct TopkLaunch {
  const void* bins;
  DType t;                // F64 or F32
  int64_t count;
  int C;                  // candidates wanted, <= 64
  double* cand_val;       // workspace
  uint64_t* cand_idx;     // workspace
  int64_t cand_capacity;  // entries of cand_val / cand_idx
  double* out_val;        // C values (working precision widened to double)
  uint64_t* out_idx;      // C bin indices
};
// Exact top-C by (value desc, index asc).
hipError_t launch_topk(const TopkLaunch& t, hipStream_t stream);
int64_t topk_candidate_capacity(int64_t count, int C);

struct RefineLaunch {
  int n_sub, K;
  const double* Ep[CQ_MAX_SUBCIRCUITS];
  int64_t ld[CQ_MAX_SUBCIRCUITS];      // columns of Ep[c]
  int na[CQ_MAX_SUBCIRCUITS];          // active bits of c
  int kc[CQ_MAX_SUBCIRCUITS];
  int cut[CQ_MAX_SUBCIRCUITS][CQ_MAX_LOCAL_CUTS];
  const uint64_t* bins;                // device, nbins
  int nbins;
  double scale;                        // 2^-K
  double* out;                         // device, nbins
};
// FP64 value of chosen bins: scale * sum over all 4^K labels of prod_c Ep[c][row][a_c].
hipError_t launch_refine(const RefineLaunch& r, hipStream_t stream);

}  // namespace cq

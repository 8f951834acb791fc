// Host-side launchers of the HIP kernels.  Each returns hipSuccess or the
// launch error; all work is enqueued on `stream`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "cutqc.h"

namespace cq {

// Instances launched together (dynamic definition): a launch covers n
// instances along grid z, and instance z's argument blocks and buffers are
// those of instance 0 moved by z * stride bytes (each instance of such a batch
// owns a slot of `stride` bytes, all slots with one layout).
struct InstSpan {
  int n = 1;
  int64_t stride = 0;
};

#ifdef __HIPCC__
// p moved to the slot of this workgroup's instance (null stays null).
template <typename T>
__device__ __forceinline__ T* inst_ptr(T* p, int64_t slot) {
  if (!p) return p;
  return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + (uintptr_t)((int64_t)blockIdx.z * slot));
}
#endif

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
  // FP32 output scaled by 2^(rowexp[z*M + m] + colexp[n]) when set (16-bit
  // forms with column-scaled operands)
  const int32_t* rowexp = nullptr;
  const int32_t* colexp = nullptr;
  // time nothing: a shape tuned before keeps its variant, others take
  // variant 0 (no events, no synchronisation)
  bool no_tune = false;
};

// C[z][m][n] = alpha * sum_k A[z*sAz + k*sAk + m] * B[z*sBz + k*sBk + n]
// (kernel variant chosen by the autotuner, see gemm.hip)
hipError_t launch_gemm(cq_precision prec, const GemmLaunch& g, hipStream_t stream);
void autotune_set(int mode);
std::string autotune_json();
// Tuned choices to and from a text file (this device's entries only).
bool autotune_load(const char* path);
bool autotune_save(const char* path);

// Kernel-side GEMM description (also written by device code for shapes that
// are only known on the device).  tiles = tilesM * tilesN * Z with 128 x 128
// tiles; m_fastest selects the raster order.
struct GemmArgs {
  const void* A;
  const void* A_lo;
  const void* B;
  const void* B_lo;
  void* C;
  void* C_lo;
  int64_t M, N, K;
  int64_t sAz, sAk, sBz, sBk, sCz, ldc;
  int64_t tilesM, tilesN, tiles;
  int m_fastest;
  double alpha;
  const int32_t* rowexp;  // optional output exponents (see GemmLaunch)
  const int32_t* colexp;
  // with rowexp, for the tile bounds of the fused top-C (null otherwise):
  // the largest rowexp over each 128-row tile of each batch (z * tilesM +
  // mt), filled only when A is shared across batches
  const int32_t* rowtmax;
  // Top-C instead of the store (launch_gemm_indirect with topc): each tile
  // appends its C best (value, index) keys not below the running threshold
  // and raises the threshold to its C-th best value when it has C of them.
  unsigned long long* topc_thr;    // order-preserving key of the threshold value
  unsigned long long* topc_count;  // candidates appended
  const int32_t* topc_C;
  double* topc_v;
  uint64_t* topc_i;
  // 0: exact; 1: warm-up, raise the threshold only, append nothing; 2:
  // warm-up, append the exact C best where they are cheap to find, else
  // raise the threshold by a bound only
  int topc_publish_only;
  // Optional tile list: workgroup b takes tile tile_list[b] if b < *tile_count.
  const uint64_t* tile_list;
  const int64_t* tile_count;
};

// Tile pruning for the fused top-C (dynamic definition).  For the GEMM at
// `dev`: amax[(za * K + k) * tilesM + mt] = max |A| over the rows of tile mt
// (likewise bmax), then U[t] >= alpha * sum_k amax * bmax, an upper bound on
// every output of tile t (inflated for FP32 accumulation, rounded up).
hipError_t launch_tile_bounds(const GemmArgs* dev, DType t, bool f16, float* amax, float* bmax,
                              float* U, int64_t max_seg_a, int64_t max_seg_b, int64_t max_tiles,
                              hipStream_t stream, InstSpan span = InstSpan());
// list[b] <- the tile with the largest bound in slice b of *warm slices.
hipError_t launch_tile_warm(const float* U, const int64_t* n_tiles, const int64_t* warm,
                            uint64_t* list, int max_warm, hipStream_t stream, InstSpan span = InstSpan());
// list <- the tiles t < *n_tiles with U[t] >= the threshold, *count their number.
hipError_t launch_tile_compact(const float* U, const int64_t* n_tiles,
                               const unsigned long long* thr_key, uint64_t* list,
                               int64_t* count, int64_t max_tiles, hipStream_t stream,
                               InstSpan span = InstSpan());

// Runs the precision's GEMM kernel on arguments in device memory (`dev`) for
// up to `max_tiles` tiles: at most 4096 workgroups (1024 with topc) per
// instance of `span`, each looping over the tiles that the stored tile count
// (or tile list) holds.  Operands and output are in the precision's storage
// format (tc: F32/F64 output or the precision's own planes); the
// register-path 16-bit kernel is used.
hipError_t launch_gemm_indirect(cq_precision prec, const GemmArgs* dev, int64_t max_tiles,
                                DType tc, bool nontemporal, bool topc, hipStream_t stream,
                                InstSpan span = InstSpan());

// Converts n FP64 values to `t` (FP32, or BF16/FP16 planes when f16 is false/true).
// rexp (optional): element i is first multiplied by 2^rexp[i >> cols_log2]
// (the per-label balance of its row, exact).
hipError_t launch_prep(const double* src, void* dst, int64_t n, DType t, bool f16,
                       hipStream_t stream, const int32_t* rexp = nullptr, int cols_log2 = 0);

// Per-label balance of the 16-bit operands (powers of two, exact).  Every
// labelling term of Eq. 1 carries, for each cut j, the factor of the
// subcircuit that measures j's upstream end (row digit d at j) times that of
// the subcircuit that initialises j's downstream end (same digit); scaling the
// first by 2^e and the second by 2^-e leaves every term unchanged.  e_j(d) is
// half the difference of the binary exponents of the two sides' largest
// |entry| among rows with digit d at j, so both sides end up within a factor
// of two of each other; the maxima are taken again on the scaled rows and
// e_j(d) corrected, for up to four rounds (until nothing changes).  rowmax:
// per subcircuit, max_b |E_c[l][b]| per row l.
struct BalanceLaunch {
  int n_sub, K;
  const uint64_t* rowmax[CQ_MAX_SUBCIRCUITS];  // FP64 bit patterns, 4^k_c each
  int32_t* rexp[CQ_MAX_SUBCIRCUITS];           // out: row exponents, 4^k_c each
  int k[CQ_MAX_SUBCIRCUITS];
  int cut_of[CQ_MAX_SUBCIRCUITS][CQ_MAX_LOCAL_CUTS];  // cut at digit position p
  int up[CQ_MAX_CUTS], pos_up[CQ_MAX_CUTS];            // measuring subcircuit, digit position
  int down[CQ_MAX_CUTS], pos_down[CQ_MAX_CUTS];        // initialising subcircuit, digit position
};
// rowmax of E (rows x 2^cols_log2, FP64)
hipError_t launch_rowmax(const double* E, int64_t rows, int cols_log2, uint64_t* rowmax,
                         hipStream_t stream);
hipError_t launch_balance(const BalanceLaunch& b, hipStream_t stream);

// Column scaling by powers of two (16-bit operands).  colmax[b] receives the
// bit pattern of max_l |E[l][b]| (FP64, so the unsigned order is the value
// order); column b is then scaled by 2^-e, e the binary exponent with
// max = f * 2^e, f in [0.5, 1).  Scaling is exact, and the result's
// per-subcircuit exponents are added back at the end.
// rexp (optional) as for launch_prep, applied before the maxima and the
// conversion.
hipError_t launch_colmax(const double* E, int64_t rows, int cols_log2, uint64_t* colmax,
                         hipStream_t stream, const int32_t* rexp = nullptr);
hipError_t launch_prep_scaled(const double* src, void* dst, int64_t n, int cols_log2,
                              const uint64_t* colmax, DType t, bool f16, hipStream_t stream,
                              const int32_t* rexp = nullptr);
// out[r] = sum_c e_c(colmax[c][(r >> shift[c]) & (2^bits[c] - 1)]) for r < count.
struct ExpSumLaunch {
  int32_t* out;
  int64_t count;
  int n;
  const uint64_t* colmax[CQ_MAX_SUBCIRCUITS];
  int shift[CQ_MAX_SUBCIRCUITS];
  int bits[CQ_MAX_SUBCIRCUITS];
};
hipError_t launch_expsum(const ExpSumLaunch& x, hipStream_t stream);

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
  int nfac = 0;  // column-scale undo (PermArgs)
  const uint64_t* colmax[CQ_MAX_SUBCIRCUITS] = {};
  int fac_shift[CQ_MAX_SUBCIRCUITS] = {};
  int fac_bits[CQ_MAX_SUBCIRCUITS] = {};
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


// ---------------------------------------------------------------------------
// Kernel argument blocks.  Host launchers fill them; the device-driven
// dynamic definition writes them from device code, for shapes that depend on
// which bin a recursion zooms into, and launches the same kernels on them.
// ---------------------------------------------------------------------------
struct PermArgs {
  const void* src;
  const void* src_lo;  // lo plane of a split source, else null
  void* dst;
  void* dst_lo;        // lo plane of a split destination, else null
  int64_t total;
  int naxes;
  int log2[kMaxPermAxes];
  int64_t sstride[kMaxPermAxes];
  double alpha;
  // optional column-scale undo: value *= 2^(sum_c e_c) with e_c the exponent
  // of colmax[c][(src offset >> fac_shift[c]) & (2^fac_bits[c] - 1)]
  int nfac;
  const uint64_t* colmax[CQ_MAX_SUBCIRCUITS];
  int fac_shift[CQ_MAX_SUBCIRCUITS];
  int fac_bits[CQ_MAX_SUBCIRCUITS];
};

struct PrepArgs {
  const double* src;
  void* dst;
  void* dst_lo;
  int64_t n;
  const int32_t* rexp;  // per-label balance: row exponents (rows of 2^cols_log2), or null
  int32_t cols_log2;
  int32_t pad;
  const uint64_t* colmax;  // column scaling: column maxima (FP64 bits, after rexp), or null
};

struct MergeArgs {
  const double* E;
  double* Ep;
  int64_t outputs;  // rows << na
  int n, na, tpo_log2;
  int64_t iters;    // 2^(nm - tpo_log2)
  uint64_t active_flat, merged_lo, merged_hi, fixed_vals_flat;
};

// FP64 value of chosen bins: out[b] = scale * sum over all 4^K labels of
// prod_c Ep[c][row_c(label)][a_c(bins[b])].
struct RefineArgs {
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

// Indirect launches: `max_*` bounds the grid; the kernels read their
// arguments from device memory and skip work beyond the stored sizes.
hipError_t launch_permute_indirect(const PermArgs* dev, DType ts, DType td, bool f16,
                                   int64_t max_total, hipStream_t stream, InstSpan span = InstSpan());
hipError_t launch_prep_indirect(const PrepArgs* dev, int count, DType t, bool f16,
                                int64_t max_n, hipStream_t stream, InstSpan span = InstSpan());
hipError_t launch_merge_indirect(const MergeArgs* dev, int count, int64_t max_threads,
                                 hipStream_t stream, InstSpan span = InstSpan());
hipError_t launch_refine_indirect(const RefineArgs* dev, int max_bins, hipStream_t stream,
                                  InstSpan span = InstSpan());
// Top-C of *count bins (value desc, index asc) with C = *C_dev <= C_max
// (nothing when C <= 0): pass one keeps C_max keys per workgroup in the
// candidate buffers, pass two selects from them.
hipError_t launch_topk_indirect(const void* bins, DType t, const int64_t* count_dev,
                                const int32_t* C_dev, int C_max, int64_t max_count,
                                double* cand_val, uint64_t* cand_idx, int64_t cand_capacity,
                                double* out_val, uint64_t* out_idx, hipStream_t stream);
int64_t topk_indirect_capacity(int64_t max_count, int C_max);
// Top-C (C = *C_dev) of *count_dev explicit candidate keys, in two passes
// through kTopcStage * C_max staged keys.
constexpr int kTopcStage = 256;
hipError_t launch_topk_candidates(const double* cand_val, const uint64_t* cand_idx,
                                  const int64_t* count_dev, const int32_t* C_dev, int C_max,
                                  double* stage_val, uint64_t* stage_idx, double* out_val,
                                  uint64_t* out_idx, hipStream_t stream, InstSpan span = InstSpan());

// ---------------------------------------------------------------------------
// Device-driven dynamic definition (Algorithm 1).  One recursion is a fixed
// sequence of launches: setup (descriptors from the current masks), merge,
// row sums, FP64 total, operand preparation, the bin contraction, top-C,
// FP64 refinement and the list update / zoom.  Sizes are products of powers
// of two, 2^(c0 + sum of the active counts of the subcircuits in `mask`), so
// the contraction plan made for the largest active counts is re-evaluated on
// the device for the current ones.
// ---------------------------------------------------------------------------
constexpr int kDDMaxSteps = 16;
constexpr int kDDMaxTensors = 48;
constexpr int kDDMaxPermAxes = 24;
constexpr int kDDMaxC = 64;

struct SymPow {   // 0 when zero != 0, else 2^(c0 + sum_{c in mask} na[c])
  int32_t c0;
  uint32_t mask;
  int32_t zero;
  int32_t pad;
};
struct SymLog {   // c0 + sum_{c in mask} na[c]
  int32_t c0;
  uint32_t mask;
};

struct DDTensor {
  void* hi;        // values or hi plane (null for the recursion's bin buffer)
  void* lo;        // lo plane of split operands
  int32_t is_out;  // the recursion's bin buffer
  int32_t pad;
};

struct DDGemmSym {
  int32_t a, b, c, pad;
  SymPow Z, M, N, K, sAz, sAk, sBz, sBk, sCz, ldc;
  double alpha;
};

struct DDPermSym {
  int32_t src, dst, naxes, pad;
  SymLog log2[kDDMaxPermAxes];
  SymPow sstride[kDDMaxPermAxes];
  double alpha;
};

struct DDInit {  // recursion-0 masks
  uint64_t active[CQ_MAX_SUBCIRCUITS];
  uint64_t merged[CQ_MAX_SUBCIRCUITS];
  uint64_t fixed[CQ_MAX_SUBCIRCUITS];
  uint64_t fixed_vals[CQ_MAX_SUBCIRCUITS];
};

struct DDProgram {
  int32_t n_sub, K, R, n_steps;
  int32_t C_max;                             // min(4R, 64)
  int32_t resume;                            // the state comes from a checkpoint, not `init`
  int32_t r0, r_end;                         // recursions r0 .. r_end - 1 run; launch r is r0 + r
  int32_t n_out[CQ_MAX_SUBCIRCUITS];
  int32_t max_active[CQ_MAX_SUBCIRCUITS];
  int32_t kc[CQ_MAX_SUBCIRCUITS];
  int32_t cut[CQ_MAX_SUBCIRCUITS][CQ_MAX_LOCAL_CUTS];
  int64_t rows[CQ_MAX_SUBCIRCUITS];
  const double* E[CQ_MAX_SUBCIRCUITS];       // FP64 entries
  double* Ep[CQ_MAX_SUBCIRCUITS];            // reduced entries
  double* Rs[CQ_MAX_SUBCIRCUITS];            // their row sums
  int32_t prep_dst[CQ_MAX_SUBCIRCUITS];      // tensor receiving the converted copy, or -1
  int32_t topc_step;                         // GEMM step that selects top-C instead of storing, or -1
  int32_t pad2;
  double* cand_v;                            // its candidate buffers
  uint64_t* cand_i;
  // tile pruning of that GEMM (see launch_tile_bounds)
  float* bound_a;
  float* bound_b;
  float* bound_u;
  uint64_t* tile_list;
  double* warm_v;                            // the 64 tiles with the largest bounds
  uint64_t* warm_i;
  DDInit init;
  RefineArgs total;                          // the recursion total: the row sums' single bin
  int32_t balance;                           // per-label balance of the 16-bit operands
  int32_t pad3;
  BalanceLaunch bal;                         // its row maxima and exponents (4^k_c each)
  // Column scaling of the FP16 operands (the plan's last step a GEMM writing
  // the bins): column maxima of every reduced entry, and the last GEMM's
  // output exponents -- over its rows (z * M + m) and columns (n), each the
  // sum over the subcircuits of a group of the exponent of the column that
  // bits shift .. shift + na_c - 1 of the index select -- and the rows'
  // tile maxima (used when A is shared across batches).
  int32_t cscale;
  int32_t fac_n[2];
  int32_t fac_sub[2][CQ_MAX_SUBCIRCUITS];
  SymLog fac_shift[2][CQ_MAX_SUBCIRCUITS];
  uint64_t* colmax[CQ_MAX_SUBCIRCUITS];     // 2^amax_c each
  int32_t* rowexp;
  int32_t* colexp;
  int32_t* rowtmax;
  DDTensor tensor[kDDMaxTensors];
  SymPow tensor_elems[kDDMaxTensors];
  int32_t step_is_gemm[kDDMaxSteps];
  DDGemmSym gemm[kDDMaxSteps];
  DDPermSym perm[kDDMaxSteps];
};

struct DDEntry {  // one entry of the list L with the masks of its bin
  double v;
  int32_t rec;
  int32_t pad;
  uint64_t bin;
  uint64_t fixed[CQ_MAX_SUBCIRCUITS];
  uint64_t fixed_vals[CQ_MAX_SUBCIRCUITS];
  uint64_t merged[CQ_MAX_SUBCIRCUITS];
};

struct DDState {
  uint64_t active[CQ_MAX_SUBCIRCUITS];
  uint64_t merged[CQ_MAX_SUBCIRCUITS];
  uint64_t fixed[CQ_MAX_SUBCIRCUITS];
  uint64_t fixed_vals[CQ_MAX_SUBCIRCUITS];
  int32_t na[CQ_MAX_SUBCIRCUITS];
  int32_t n_active, stop, done, n_list;
  int32_t C, pad;
  int64_t count;                 // bins of the recursion
  unsigned long long topc_thr;   // fused top-C: running threshold (order-preserving key)
  unsigned long long topc_count; // fused top-C: candidates appended
  int64_t n_tiles;               // fused top-C: tiles of the GEMM
  int64_t warm_count;            // tiles evaluated first (largest bounds)
  int64_t list_count;            // tiles whose bound reaches the threshold
  int32_t warm_C, pad4;
  uint64_t zero_idx;             // 0: the single bin of the total
  double total;
  double top_val[kDDMaxC];
  uint64_t top_idx[kDDMaxC];
  double ref_val[kDDMaxC];
  DDEntry list[CQ_MAX_DD_R];
};

struct DDLevel {  // descriptors of the current recursion
  MergeArgs merge[CQ_MAX_SUBCIRCUITS];
  MergeArgs rowsum[CQ_MAX_SUBCIRCUITS];
  PrepArgs prep[CQ_MAX_SUBCIRCUITS];
  GemmArgs gemm[kDDMaxSteps];
  GemmArgs topc_warm;            // the top-C GEMM over the warm-up tiles
  PermArgs perm[kDDMaxSteps];
  RefineArgs refine;
};

// Threshold from the warm-up tiles' candidates (the C-th best of them, C =
// *C_dev), then the candidate count back to zero.
hipError_t launch_warm_tau(const double* cand_v, unsigned long long* count, const int32_t* C_dev,
                           unsigned long long* thr, hipStream_t stream, InstSpan span = InstSpan());
// `blocks` copies of `bytes` (a multiple of 4, 4-byte aligned) between
// strided regions of device memory.
hipError_t launch_dd_copy(const void* src, int64_t src_stride, void* dst, int64_t dst_stride,
                          int64_t bytes, int blocks, hipStream_t stream);
// State <- the program's recursion-0 masks, list empty, records zeroed.
hipError_t launch_dd_init(const DDProgram* prog, DDState* st, cq_dd_record* recs, int R,
                          hipStream_t stream, InstSpan span = InstSpan());
// Descriptors of recursion r from the state; `bins` receives its bins.
hipError_t launch_dd_setup(const DDProgram* prog, DDState* st, DDLevel* lv, cq_dd_record* recs,
                           int r, void* bins, hipStream_t stream, InstSpan span = InstSpan());
// Per-label balance of the recursion's reduced entries, for programs with
// `balance` set: row maxima of every reduced entry (rows of its current
// 2^na_c columns, from the level's preparation descriptors), then the
// exponents; the preparation then applies them (PrepArgs::rexp).
hipError_t launch_dd_balance(const DDProgram* prog, const DDLevel* lv, int n_sub, int64_t max_rows,
                             hipStream_t stream, InstSpan span = InstSpan());
// Column scaling of the recursion's reduced entries (programs with `cscale`):
// the column maxima of every reduced entry, after the balance's row
// exponents; `max_cols` bounds 2^na_c over the group.
hipError_t launch_dd_colmax(const DDProgram* prog, const DDLevel* lv, int n_sub, int64_t max_cols,
                            hipStream_t stream, InstSpan span = InstSpan());
// The last GEMM's output exponents and, when its A is shared across batches,
// the rows' tile maxima (GEMM step `step` of the level); `max_rows` and
// `max_cols` bound its Z * M and N over the group.
hipError_t launch_dd_expsum(const DDProgram* prog, const DDState* st, const DDLevel* lv, int step,
                            int64_t max_rows, int64_t max_cols, hipStream_t stream,
                            InstSpan span = InstSpan());
// List update, record r and zoom into the popped bin.
hipError_t launch_dd_update(const DDProgram* prog, DDState* st, cq_dd_record* recs, int r,
                            hipStream_t stream, InstSpan span = InstSpan());

}  // namespace cq

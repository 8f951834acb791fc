// Internal host-side structures of the reconstruction library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "cutqc.h"

namespace cq {

// Thread-local error detail behind cq_last_error().
void set_error(const std::string& msg);
cq_status fail(cq_status s, const std::string& msg);

// Facts derived from one subcircuit's cut map.
struct SubInfo {
  int width = 0;
  std::vector<int> init_cut, meas_cut;
  std::vector<int> outputs;     // output slots, slot order
  std::vector<int> init_slots;  // slots initialised by a cut, slot order
  std::vector<int> meas_slots;  // slots measured for a cut, slot order
  std::vector<int> cuts;        // incident cut ids, ascending (label digit order)
  int n() const { return (int)outputs.size(); }
  int r() const { return (int)init_slots.size(); }
  int o() const { return (int)meas_slots.size(); }
  int k() const { return (int)cuts.size(); }
  // position of cut id in `cuts` (-1 when not incident)
  int digit_pos(int cut) const {
    for (int i = 0; i < (int)cuts.size(); ++i)
      if (cuts[i] == cut) return i;
    return -1;
  }
};

struct CutMap {
  int n_sub = 0;
  int K = 0;
  int n_total = 0;
  std::vector<SubInfo> subs;
  std::vector<int> up, down;  // per cut: measuring / initialising subcircuit
};

// Full definition (cq_reconstruct_fd) on a given workspace.  quiet: create
// no events (no per-launch timing) and time no GEMM variant.
cq_status fd_run(int32_t n_sub, const cq_subcircuit* subs, const double* const* entries,
                 cq_precision prec, const int32_t* out_perm, void* out, void* workspace,
                 size_t workspace_bytes, bool quiet, hipStream_t stream);

// Validates and derives.  Returns CQ_OK or an error (message set).
cq_status build_cutmap(int32_t n_sub, const cq_subcircuit* subs, CutMap& cm);
cq_status build_subinfo(const cq_subcircuit* sub, SubInfo& si);

// ---------------------------------------------------------------------------
// Contraction plan for Eq. 1.
//
// A tensor is an ordered list of axes, row-major.  An axis is either the
// 4-valued label of one cut or the 2^{n_c} outputs of one subcircuit.
// ---------------------------------------------------------------------------
struct Axis {
  int kind;   // 0: cut label, 1: subcircuit outputs
  int id;     // cut id or subcircuit id
  int log2;   // log2 of the axis size
  bool operator==(const Axis& o) const { return kind == o.kind && id == o.id; }
};

enum class Loc { Input, Work, Out };

struct TensorRef {
  Loc loc = Loc::Work;
  int index = 0;          // input subcircuit id, or workspace buffer id
  std::vector<Axis> axes;
  int64_t elems = 0;      // elements the tensor's buffer holds
  int log2_size() const {
    int s = 0;
    for (auto& a : axes) s += a.log2;
    return s;
  }
};

// Batched "TN" GEMM:  C[z][m][n] = alpha * sum_k A[z*sAz + k*sAk + m] * B[z*sBz + k*sBk + n]
// stored at C[z*sCz + m*ldc + n].
struct GemmStep {
  int a, b, c;  // tensor ids
  int64_t Z, M, N, K;
  int64_t sAz, sAk, sBz, sBk, sCz, ldc;
  double alpha;
};

// dst[i] = alpha * src[offset(i)], offset from per-axis source strides over the
// destination's axes (sizes 2^log2, last axis fastest).
struct PermuteStep {
  int src, dst;
  std::vector<int> log2;
  std::vector<int64_t> sstride;
  double alpha;
};

struct Step {
  bool is_gemm;
  GemmStep g;
  PermuteStep p;
};

struct Plan {
  std::vector<TensorRef> tensors;
  std::vector<Step> steps;
  std::vector<int64_t> work_offset;  // byte offset of each workspace buffer
  std::vector<int64_t> work_bytes;
  // byte offset of each input's converted copy in the workspace, or -1 when
  // the contraction reads the caller's FP64 entries directly
  std::vector<int64_t> input_offset;
  int64_t workspace_bytes = 0;
  // bytes per element of every operand and intermediate: 8 (FP64), 4 (FP32 or
  // two 16-bit planes), 2 (one 16-bit plane)
  int work_elem_bytes = 8;
  double flops = 0.0;       // algorithmic flops of the GEMM steps

  // Column scaling (FP16 operands): inputs are scaled per output column by
  // powers of two before conversion, and the final step adds the exponents
  // back.  A factor group lists, per subcircuit, where its output digit sits
  // in the index the exponents are summed over (bits 0: a subcircuit without
  // outputs, digit always 0).
  struct FacGroup {
    std::vector<int> sub, shift, bits;
  };
  bool scaled = false;
  std::vector<int64_t> colmax_offset;   // per input: 2^{n_c} uint64 column maxima
  int64_t rowexp_offset = -1, colexp_offset = -1;  // final GEMM: Z*M and N int32 exponents
  int64_t rowexp_count = 0, colexp_count = 0;
  FacGroup row_fac, col_fac;            // final GEMM: over z*M + m, and over n
  FacGroup perm_fac;                    // final permute: over the source offset
  // Per-label balance (16-bit operands): per input, 4^k_c row maxima (FP64
  // bit patterns) and 4^k_c int32 row exponents; -1 when not reserved.
  std::vector<int64_t> lbal_rowmax_offset, lbal_rexp_offset;
};

// `out_log2` per subcircuit = number of outputs taking part (n_c for FD, the
// active count for DD bins).  `out_perm` (may be empty): bit permutation to
// apply to the final concatenated order.
// keep_empty: subcircuits with no outputs taking part still carry a size-1
// output axis (the dynamic-definition plans re-evaluate sizes per recursion).
// column_scaling: reserve and describe the column scaling of the operands
// (the 16-bit FP16 forms).
cq_status make_plan(const CutMap& cm, const std::vector<int>& out_log2, int work_elem_bytes,
                    const std::vector<int>& out_perm, Plan& plan, bool keep_empty = false,
                    bool column_scaling = false);

// ---------------------------------------------------------------------------
// Plans with symbolic sizes.  Every size and stride of a plan is a product of
// axis sizes: 4 per cut label and 2^{na_c} for the outputs of subcircuit c.
// A SymQ is 2^(c0 + sum_{c in mask} na_c) (or 0 when `zero`); as a log2 it
// is c0 + sum_{c in mask} na_c.
// ---------------------------------------------------------------------------
struct SymQ {
  int c0 = 0;
  uint32_t mask = 0;
  bool zero = false;
};
int64_t sym_value(const SymQ& q, const std::vector<int>& na);
int sym_log2(const SymQ& q, const std::vector<int>& na);

struct SymGemm {
  SymQ Z, M, N, K, sAz, sAk, sBz, sBk, sCz, ldc;
};
struct SymPerm {
  std::vector<SymQ> log2;     // read as log2 values
  std::vector<SymQ> sstride;  // read as powers
};
struct SymPlan {
  std::vector<SymQ> elems;    // per tensor
  std::vector<SymGemm> gemm;  // per step (GEMM steps)
  std::vector<SymPerm> perm;  // per step (permute steps)
};

// Plan for the largest active counts `amax` (every output axis kept) and its
// symbolic form, checked to reproduce the plan at `amax`.  Any active counts
// na_c <= amax_c fit the plan's buffers.
cq_status make_sym_plan(const CutMap& cm, const std::vector<int>& amax, int work_elem_bytes,
                        Plan& plan, SymPlan& sp);

}  // namespace cq

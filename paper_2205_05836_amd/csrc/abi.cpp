// extern "C" entry points: validate, plan, enqueue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <mutex>
#include <cmath>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace cq {
namespace {

bool fault_injected(const char* stage) {
  const char* e = std::getenv("CQ_FAULT_INJECT");
  return e && (std::strcmp(e, stage) == 0 || std::strcmp(e, "all") == 0);
}

cq_status hip_fail(hipError_t e, const char* what) {
  return fail(CQ_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---- per-launch timing (cq_profile_enable / cq_profile_read) ----
struct ProfRecord {
  std::string name;
  hipEvent_t start = nullptr, stop = nullptr;
  double flops = 0.0;
  int dev = 0;
};
std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::vector<ProfRecord> g_prof;
// Idle timing events by device.  Creating and destroying two events per
// launch stalled the issuing thread for milliseconds at times (long enough to
// leave the GPU idle between launches), so events are reused.
std::vector<std::pair<int, hipEvent_t>> g_prof_pool;

hipEvent_t prof_event(int dev) {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (size_t i = g_prof_pool.size(); i-- > 0;)
      if (g_prof_pool[i].first == dev) {
        const hipEvent_t e = g_prof_pool[i].second;
        g_prof_pool.erase(g_prof_pool.begin() + (std::ptrdiff_t)i);
        return e;
      }
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void prof_release(int dev, hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_pool.emplace_back(dev, e);
}

// Brackets one launch with events when profiling is on.
// Calls that may not create events (the no-allocation entry point) set
// this for their duration on the calling thread.
thread_local bool t_quiet = false;

struct ProfScope {
  bool on = false;
  ProfRecord rec;
  hipStream_t stream;
  ProfScope(const char* name, double flops, hipStream_t s) : stream(s) {
    if (t_quiet || !g_prof_on.load()) return;
    if (hipGetDevice(&rec.dev) != hipSuccess) return;
    rec.name = name;
    rec.flops = flops;
    rec.start = prof_event(rec.dev);
    rec.stop = prof_event(rec.dev);
    on = rec.start && rec.stop && hipEventRecord(rec.start, stream) == hipSuccess;
    if (!on) {
      prof_release(rec.dev, rec.start);
      prof_release(rec.dev, rec.stop);
    }
  }
  ~ProfScope() {
    if (!on) return;
    if (hipEventRecord(rec.stop, stream) == hipSuccess) {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof.push_back(rec);
    } else {
      prof_release(rec.dev, rec.start);
      prof_release(rec.dev, rec.stop);
    }
  }
};

bool valid_prec(cq_precision p) { return p >= CQ_FP64 && p <= CQ_FP16_SPLIT; }

// Precisions whose kernels this build ships.
bool prec_supported(cq_precision p) { return p >= CQ_FP64 && p <= CQ_FP16_SPLIT; }

DType work_dtype(cq_precision p) {
  switch (p) {
    case CQ_FP64: return DType::F64;
    case CQ_FP32: return DType::F32;
    case CQ_BF16:
    case CQ_FP16: return DType::H16;
    default: return DType::H16X2;
  }
}

int work_elem_bytes(cq_precision p) { return dtype_bytes(work_dtype(p)); }

bool is_f16(cq_precision p) { return p == CQ_FP16 || p == CQ_FP16_SPLIT; }

bool is_h16(cq_precision p) { return p >= CQ_BF16 && p <= CQ_FP16_SPLIT; }

// Per-label balance of the operands: 0 off, 1 the FP16 forms (default),
// 2 every 16-bit form.
std::atomic<int> g_lbal_mode{1};

bool balance_applies(cq_precision p) {
  const int m = g_lbal_mode.load();
  return is_h16(p) && (m == 2 || (m == 1 && is_f16(p)));
}

// Column scaling of the FP16 operands: 1 on (default), 0 off.
std::atomic<int> g_cscale_mode{1};

bool cscale_applies(cq_precision p) { return is_f16(p) && g_cscale_mode.load() != 0; }

DType out_dtype(cq_precision p) { return p == CQ_FP64 ? DType::F64 : DType::F32; }

cq_status check_perm(const int32_t* out_perm, int n, std::vector<int>& perm) {
  perm.clear();
  if (!out_perm) return CQ_OK;
  std::vector<int> seen(n, 0);
  for (int i = 0; i < n; ++i) {
    int q = out_perm[i];
    if (q < 0 || q >= n || seen[q]) return fail(CQ_ERR_ARG, "out_perm is not a permutation");
    seen[q] = 1;
    perm.push_back(q);
  }
  return CQ_OK;
}

// Runs a plan.  inputs[c]: FP64 device pointer of subcircuit c's tensor.
// bal (optional): per-label balance of the 16-bit operands, its row maxima and
// exponents in the workspace.
cq_status execute(const Plan& plan, cq_precision prec, const double* const* inputs, void* out,
                  DType out_t, char* ws, hipStream_t stream, const BalanceLaunch* bal = nullptr) {
  const DType wt = work_dtype(prec);
  const bool f16 = is_f16(prec);
  auto planes = [&](char* base, int64_t elems) -> Operand {
    Operand o;
    o.p = base;
    o.lo = wt == DType::H16X2 ? base + elems * 2 : nullptr;
    o.t = wt;
    return o;
  };
  auto res = [&](int tid) -> Operand {
    const TensorRef& t = plan.tensors[tid];
    if (t.loc == Loc::Input) {
      if (plan.input_offset[t.index] < 0) return Operand{inputs[t.index], nullptr, DType::F64};
      return planes(ws + plan.input_offset[t.index], t.elems);
    }
    if (t.loc == Loc::Out) return Operand{out, nullptr, out_t};
    return planes(ws + plan.work_offset[t.index], t.elems);
  };
  auto colmax = [&](int c) { return reinterpret_cast<uint64_t*>(ws + plan.colmax_offset[c]); };
  auto out_bits = [](const TensorRef& t) {
    return t.axes.empty() || t.axes.back().kind != 1 ? 0 : t.axes.back().log2;
  };
  // per-label balance: row maxima of every converted input, then the
  // exponents of every row
  if (bal) {
    ProfScope ps("balance", 0.0, stream);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < plan.tensors.size() && e == hipSuccess; ++i) {
      const TensorRef& t = plan.tensors[i];
      if (t.loc != Loc::Input || plan.input_offset[t.index] < 0) continue;
      const int nb = out_bits(t);
      e = launch_rowmax(inputs[t.index], t.elems >> nb, nb,
                        const_cast<uint64_t*>(bal->rowmax[t.index]), stream);
    }
    if (e == hipSuccess) e = launch_balance(*bal, stream);
    if (e != hipSuccess) return hip_fail(e, "label balance launch");
  }
  // operand preparation: FP64 entries -> the precision's storage format
  for (size_t i = 0; i < plan.tensors.size(); ++i) {
    const TensorRef& t = plan.tensors[i];
    if (t.loc != Loc::Input || plan.input_offset[t.index] < 0) continue;
    const int32_t* rexp = bal ? bal->rexp[t.index] : nullptr;
    const int nb = out_bits(t);
    hipError_t e;
    {
      ProfScope ps("prep", 0.0, stream);
      if (plan.scaled) {
        const int64_t rows = t.elems >> nb;
        e = launch_colmax(inputs[t.index], rows, nb, colmax(t.index), stream, rexp);
        if (e == hipSuccess)
          e = launch_prep_scaled(inputs[t.index], ws + plan.input_offset[t.index], t.elems, nb,
                                 colmax(t.index), wt, f16, stream, rexp);
      } else {
        e = launch_prep(inputs[t.index], ws + plan.input_offset[t.index], t.elems, wt, f16, stream,
                        rexp, nb);
      }
    }
    if (e != hipSuccess) return hip_fail(e, "operand prep launch");
  }
  int32_t* rowexp = nullptr;
  int32_t* colexp = nullptr;
  if (plan.scaled && plan.rowexp_offset >= 0) {
    rowexp = reinterpret_cast<int32_t*>(ws + plan.rowexp_offset);
    colexp = reinterpret_cast<int32_t*>(ws + plan.colexp_offset);
    const Plan::FacGroup* gr[2] = {&plan.row_fac, &plan.col_fac};
    int32_t* outs[2] = {rowexp, colexp};
    const int64_t counts[2] = {plan.rowexp_count, plan.colexp_count};
    for (int q = 0; q < 2; ++q) {
      ExpSumLaunch x;
      std::memset(&x, 0, sizeof(x));
      x.out = outs[q];
      x.count = counts[q];
      x.n = (int)gr[q]->sub.size();
      for (int i = 0; i < x.n; ++i) {
        x.colmax[i] = colmax(gr[q]->sub[i]);
        x.shift[i] = gr[q]->shift[i];
        x.bits[i] = gr[q]->bits[i];
      }
      hipError_t e = launch_expsum(x, stream);
      if (e != hipSuccess) return hip_fail(e, "scale exponent launch");
    }
  }
  for (const Step& s : plan.steps) {
    hipError_t e;
    if (s.is_gemm) {
      const GemmStep& g = s.g;
      Operand c = res(g.c);
      GemmLaunch L;
      L.a = res(g.a);
      L.b = res(g.b);
      L.C = const_cast<void*>(c.p);
      L.C_lo = const_cast<void*>(c.lo);
      L.tc = c.t;
      L.Z = g.Z;
      L.M = g.M;
      L.N = g.N;
      L.K = g.K;
      L.sAz = g.sAz;
      L.sAk = g.sAk;
      L.sBz = g.sBz;
      L.sBk = g.sBk;
      L.sCz = g.sCz;
      L.ldc = g.ldc;
      L.alpha = g.alpha;
      L.nontemporal = plan.tensors[g.c].loc == Loc::Out;
      L.no_tune = t_quiet;
      if (rowexp && plan.tensors[g.c].loc == Loc::Out) {
        L.rowexp = rowexp;
        L.colexp = colexp;
      }
      {
        static const char* kname[] = {"gemm_f64", "gemm_f32", "gemm_bf16", "gemm_bf16x3",
                                      "gemm_f16", "gemm_f16x3"};
        ProfScope ps(kname[prec], 2.0 * g.Z * g.M * g.N * g.K, stream);
        e = launch_gemm(prec, L, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "label GEMM launch");
    } else {
      const PermuteStep& p = s.p;
      if ((int)p.log2.size() > kMaxPermAxes) return fail(CQ_ERR_UNSUPPORTED, "permute has too many axes");
      Operand d = res(p.dst);
      PermLaunch L;
      L.src = res(p.src);
      L.dst = const_cast<void*>(d.p);
      L.dst_lo = const_cast<void*>(d.lo);
      L.td = d.t;
      L.f16 = f16;
      L.naxes = (int)p.log2.size();
      for (int i = 0; i < L.naxes; ++i) {
        L.log2[i] = p.log2[i];
        L.sstride[i] = p.sstride[i];
      }
      L.alpha = p.alpha;
      if (plan.scaled && plan.tensors[p.dst].loc == Loc::Out) {
        L.nfac = (int)plan.perm_fac.sub.size();
        for (int i = 0; i < L.nfac; ++i) {
          L.colmax[i] = colmax(plan.perm_fac.sub[i]);
          L.fac_shift[i] = plan.perm_fac.shift[i];
          L.fac_bits[i] = plan.perm_fac.bits[i];
        }
      }
      {
        ProfScope ps("permute", 0.0, stream);
        e = launch_permute(L, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "permute launch");
    }
  }
  return CQ_OK;
}

// Per-label balance: row maxima and exponents of each input, reserved at the
// end of a full-definition plan's workspace for every 16-bit form (used when
// balance_applies).
void reserve_balance(const CutMap& cm, Plan& plan) {
  auto reserve = [&](int64_t bytes) {
    const int64_t off = plan.workspace_bytes;
    plan.workspace_bytes = off + (bytes + 255) / 256 * 256;
    return off;
  };
  for (int c = 0; c < cm.n_sub; ++c) {
    const int64_t rows = (int64_t)1 << (2 * cm.subs[c].k());
    plan.lbal_rowmax_offset.push_back(reserve(rows * 8));
    plan.lbal_rexp_offset.push_back(reserve(rows * 4));
  }
}

cq_status fd_prepare(int32_t n_sub, const cq_subcircuit* subs, cq_precision prec,
                     const int32_t* out_perm, CutMap& cm, Plan& plan) {
  cq_status st = build_cutmap(n_sub, subs, cm);
  if (st != CQ_OK) return st;
  if (!valid_prec(prec)) return fail(CQ_ERR_ARG, "unknown precision");
  if (cm.n_total > CQ_MAX_FD_BITS) return fail(CQ_ERR_SHAPE, "too many output qubits for full definition");
  std::vector<int> perm;
  st = check_perm(out_perm, cm.n_total, perm);
  if (st != CQ_OK) return st;
  std::vector<int> ol;
  for (auto& s : cm.subs) ol.push_back(s.n());
  st = make_plan(cm, ol, work_elem_bytes(prec), perm, plan, false, cscale_applies(prec));
  if (st == CQ_OK && is_h16(prec)) reserve_balance(cm, plan);
  return st;
}

// The balance arguments of a plan on workspace ws.
// The cut structure of a balance launch (pointers left null).
BalanceLaunch balance_struct(const CutMap& cm) {
  BalanceLaunch b;
  std::memset(&b, 0, sizeof(b));
  b.n_sub = cm.n_sub;
  b.K = cm.K;
  for (int c = 0; c < cm.n_sub; ++c) {
    const SubInfo& si = cm.subs[c];
    b.k[c] = si.k();
    for (int p = 0; p < si.k(); ++p) b.cut_of[c][p] = si.cuts[p];
  }
  for (int j = 0; j < cm.K; ++j) {
    b.up[j] = cm.up[j];
    b.down[j] = cm.down[j];
    b.pos_up[j] = cm.subs[cm.up[j]].digit_pos(j);
    b.pos_down[j] = cm.subs[cm.down[j]].digit_pos(j);
  }
  return b;
}

BalanceLaunch balance_args(const CutMap& cm, const Plan& plan, char* ws) {
  BalanceLaunch b = balance_struct(cm);
  for (int c = 0; c < cm.n_sub; ++c) {
    b.rowmax[c] = reinterpret_cast<const uint64_t*>(ws + plan.lbal_rowmax_offset[c]);
    b.rexp[c] = reinterpret_cast<int32_t*>(ws + plan.lbal_rexp_offset[c]);
  }
  return b;
}

}  // namespace
}  // namespace cq

using namespace cq;

// ---------------------------------------------------------------------------
// Attribution
// ---------------------------------------------------------------------------
extern "C" cq_status cq_attribute_workspace_size(const cq_subcircuit* sub, size_t* bytes) {
  SubInfo si;
  cq_status st = build_subinfo(sub, si);
  if (st != CQ_OK) return st;
  if (!bytes) return fail(CQ_ERR_ARG, "null bytes");
  *bytes = ((size_t)1 << (2 * si.k())) * ((size_t)1 << si.n()) * sizeof(double);
  return CQ_OK;
}

extern "C" cq_status cq_attribute(const cq_subcircuit* sub, const double* variants, double* entries,
                                  void* workspace, size_t workspace_bytes, hipStream_t stream) {
  SubInfo si;
  cq_status st = build_subinfo(sub, si);
  if (st != CQ_OK) return st;
  if (si.r() > 8 || si.o() > 8) return fail(CQ_ERR_SHAPE, "too many cut ends");
  const double log2_v = 2.0 * si.r() + std::log2(3.0) * si.o() + si.width;
  if (log2_v > 40.0) return fail(CQ_ERR_SHAPE, "variant tensor too large");
  if (!variants || !entries) return fail(CQ_ERR_ARG, "null device pointer");
  size_t need = 0;
  cq_attribute_workspace_size(sub, &need);
  if (!workspace || workspace_bytes < need) return fail(CQ_ERR_WORKSPACE, "workspace too small");
  if (fault_injected("attribute")) return fail(CQ_ERR_HIP, "injected fault before launch");
  AttrLaunch L;
  std::memset(&L, 0, sizeof(L));
  L.V = variants;
  L.U = static_cast<double*>(workspace);
  L.E = entries;
  L.r = si.r();
  L.o = si.o();
  L.n = si.n();
  L.w = si.width;
  L.k = si.k();
  for (int q = 0; q < si.n(); ++q) L.out_pos[q] = si.width - 1 - si.outputs[q];
  for (int u = 0; u < si.o(); ++u) {
    L.meas_pos[u] = si.width - 1 - si.meas_slots[u];
    L.meas_w[u] = (int64_t)1 << (2 * (si.k() - 1 - si.digit_pos(si.meas_cut[si.meas_slots[u]])));
  }
  for (int t = 0; t < si.r(); ++t)
    L.init_w[t] = (int64_t)1 << (2 * (si.k() - 1 - si.digit_pos(si.init_cut[si.init_slots[t]])));
  hipError_t e;
  {
    ProfScope ps("attribute", 0.0, stream);
    e = launch_attribute(L, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "attribution launch");
  return CQ_OK;
}

// ---------------------------------------------------------------------------
// Full definition
// ---------------------------------------------------------------------------
extern "C" cq_status cq_fd_workspace_size(int32_t n_sub, const cq_subcircuit* subs,
                                          cq_precision prec, const int32_t* out_perm,
                                          size_t* bytes) {
  CutMap cm;
  Plan plan;
  cq_status st = fd_prepare(n_sub, subs, prec, out_perm, cm, plan);
  if (st != CQ_OK) return st;
  if (!bytes) return fail(CQ_ERR_ARG, "null bytes");
  *bytes = (size_t)plan.workspace_bytes;
  return CQ_OK;
}

extern "C" cq_status cq_reconstruct_fd(int32_t n_sub, const cq_subcircuit* subs,
                                       const double* const* entries, cq_precision prec,
                                       const int32_t* out_perm, void* out, void* workspace,
                                       size_t workspace_bytes, hipStream_t stream) {
  return cq::fd_run(n_sub, subs, entries, prec, out_perm, out, workspace, workspace_bytes, false,
                    stream);
}

cq_status cq::fd_run(int32_t n_sub, const cq_subcircuit* subs, const double* const* entries,
                     cq_precision prec, const int32_t* out_perm, void* out, void* workspace,
                     size_t workspace_bytes, bool quiet, hipStream_t stream) {
  CutMap cm;
  Plan plan;
  cq_status st = fd_prepare(n_sub, subs, prec, out_perm, cm, plan);
  if (st != CQ_OK) return st;
  if (!prec_supported(prec)) return fail(CQ_ERR_UNSUPPORTED, "precision not built");
  if (!entries || !out) return fail(CQ_ERR_ARG, "null pointer");
  for (int c = 0; c < n_sub; ++c)
    if (!entries[c]) return fail(CQ_ERR_ARG, "null entry pointer");
  if (plan.workspace_bytes > 0 && (!workspace || workspace_bytes < (size_t)plan.workspace_bytes))
    return fail(CQ_ERR_WORKSPACE, "workspace too small");
  if (fault_injected("fd")) return fail(CQ_ERR_HIP, "injected fault before launch");
  BalanceLaunch bal;
  const bool balanced = balance_applies(prec) && !plan.lbal_rexp_offset.empty();
  if (balanced) bal = balance_args(cm, plan, static_cast<char*>(workspace));
  t_quiet = quiet;
  st = execute(plan, prec, entries, out, out_dtype(prec), static_cast<char*>(workspace), stream,
               balanced ? &bal : nullptr);
  t_quiet = false;
  return st;
}

// ---------------------------------------------------------------------------
// Dynamic definition
//
// Each recursion is a fixed sequence of launches whose sizes are read from
// device memory (see kernels.hpp), so a whole batch -- every instance and
// every recursion -- is enqueued without the host looking at a result, and
// by default captured into one hipGraph and launched once.
// ---------------------------------------------------------------------------
namespace {

struct DDSub {
  uint64_t active = 0, merged = 0, fixed = 0, fixed_vals = 0;  // output-position masks
};

int popc(uint64_t x) { return __builtin_popcountll(x); }

int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

cq_status dd_validate(const cq_dd_instance& in, const cq_dd_params& p, CutMap& cm,
                      std::vector<DDSub>& s0) {
  cq_status st = build_cutmap(in.n_sub, in.subs, cm);
  if (st != CQ_OK) return st;
  if (!in.entries || !in.active || !in.merged || !in.fixed || !in.fixed_vals || !in.max_active)
    return fail(CQ_ERR_ARG, "null instance array");
  if (cm.K > 12) return fail(CQ_ERR_UNSUPPORTED, "dynamic definition supports K <= 12");
  s0.assign(cm.n_sub, DDSub());
  int act = 0;
  for (int c = 0; c < cm.n_sub; ++c) {
    const int n = cm.subs[c].n();
    if (n > 63) return fail(CQ_ERR_SHAPE, "too many outputs in a subcircuit");
    const uint64_t all = ((uint64_t)1 << n) - 1;
    DDSub d{in.active[c], in.merged[c], in.fixed[c], in.fixed_vals[c]};
    if ((d.active | d.merged | d.fixed) != all || (d.active & d.merged) || (d.active & d.fixed) ||
        (d.merged & d.fixed) || (d.fixed_vals & ~d.fixed))
      return fail(CQ_ERR_MASK, "masks do not partition the outputs of subcircuit " + std::to_string(c));
    if (in.max_active[c] < 0) return fail(CQ_ERR_ARG, "negative max_active");
    if (!in.entries[c]) return fail(CQ_ERR_ARG, "null entry pointer");
    act += popc(d.active);
    s0[c] = d;
  }
  if (act > CQ_MAX_DD_ACTIVE) return fail(CQ_ERR_SHAPE, "too many active qubits");
  int later = 0;
  for (int c = 0; c < cm.n_sub; ++c) later += std::min(in.max_active[c], cm.subs[c].n());
  if (later > CQ_MAX_DD_ACTIVE) return fail(CQ_ERR_SHAPE, "too many active qubits after a zoom");
  if (p.R < 1 || p.R > CQ_MAX_DD_R) return fail(CQ_ERR_ARG, "R out of range");
  if (!valid_prec(p.prec)) return fail(CQ_ERR_ARG, "unknown precision");
  return CQ_OK;
}

// Per-instance plan and the layout of its region: the buffers of its
// recursions -- top-C selection scratch, reduced entries and their row sums,
// the contraction workspace and (when bins are stored in scratch) the bins.
struct DDSel {  // sizes of the top-C selection scratch
  int64_t cand_cap = 0, seg_a = 0, seg_b = 0, tiles = 0;
};

struct DDInstancePlan {
  CutMap cm;
  std::vector<DDSub> s0;
  std::vector<int> amax;
  Plan plan;
  SymPlan sp;
  int topc_step = -1;  // the GEMM that selects top-C instead of storing bins, or -1
  int64_t max_count = 0, bins_bytes = 0;
  std::vector<int64_t> step_max;  // grid bound per step: tiles or elements
  DDSel sel;                      // this instance's own selection sizes
  // region layout (dd_layout): offsets, and the selection sizes laid out
  int64_t cand_off = 0, cand_cap = 0, stage_off = 0;
  int64_t seg_a = 0, seg_b = 0, bound_a_off = 0, bound_b_off = 0, bound_u_off = 0, list_off = 0;
  int64_t warm_out_off = 0;
  std::vector<int64_t> ep_off, rs_off;
  bool lbal = false;                         // per-label balance of the 16-bit operands
  std::vector<int64_t> rowmax_off, rexp_off;  // its row maxima and exponents (4^k_c each)
  // column scaling of the FP16 operands (the last step a GEMM writing the bins)
  bool cscale = false;
  std::vector<int64_t> colmax_off;
  int64_t rowexp_off = 0, colexp_off = 0, rowtmax_off = 0;
  int64_t rowexp_n = 0, colexp_n = 0, rowtmax_n = 0;  // at the largest counts
  int fac_n[2] = {0, 0};
  int fac_sub[2][CQ_MAX_SUBCIRCUITS] = {};
  SymLog fac_shift[2][CQ_MAX_SUBCIRCUITS] = {};
  int64_t plan_off = 0, bins_off = 0;
  int64_t big = 0;  // bytes of the region
};

// Offsets of the region's buffers for selection sizes `s` (the instance's own,
// or the largest of the instances advanced together with it, so that every
// instance of such a group has the selection buffers at the same offsets).
void dd_layout(DDInstancePlan& D, const DDSel& s) {
  const CutMap& cm = D.cm;
  int64_t off = 0;
  D.cand_cap = s.cand_cap;
  D.cand_off = off;
  off = align256(off + s.cand_cap * 16);  // values, then indices
  D.stage_off = off;  // fused top-C: keys staged between the two selection passes
  off = align256(off + (int64_t)kTopcStage * kDDMaxC * 16);
  D.seg_a = s.seg_a;
  D.seg_b = s.seg_b;
  if (D.topc_step >= 0) {
    // tile pruning buffers of the top-C GEMM, sized for the largest shape
    D.bound_a_off = off;
    off = align256(off + s.seg_a * 4);
    D.bound_b_off = off;
    off = align256(off + s.seg_b * 4);
    D.bound_u_off = off;
    off = align256(off + s.tiles * 4);
    D.list_off = off;
    off = align256(off + s.tiles * 8);
    D.warm_out_off = off;
    off = align256(off + kDDMaxC * 16);
  }
  D.ep_off.clear();
  D.rs_off.clear();
  for (int c = 0; c < cm.n_sub; ++c) {
    D.ep_off.push_back(off);
    off = align256(off + ((int64_t)1 << (2 * cm.subs[c].k())) * ((int64_t)1 << D.amax[c]) * 8);
  }
  for (int c = 0; c < cm.n_sub; ++c) {
    D.rs_off.push_back(off);
    off = align256(off + ((int64_t)1 << (2 * cm.subs[c].k())) * 8);
  }
  D.colmax_off.clear();
  if (D.cscale) {
    for (int c = 0; c < cm.n_sub; ++c) {
      D.colmax_off.push_back(off);
      off = align256(off + ((int64_t)1 << D.amax[c]) * 8);
    }
    D.rowexp_off = off;
    off = align256(off + D.rowexp_n * 4);
    D.colexp_off = off;
    off = align256(off + D.colexp_n * 4);
    D.rowtmax_off = off;
    off = align256(off + D.rowtmax_n * 4);
  }
  D.rowmax_off.clear();
  D.rexp_off.clear();
  if (D.lbal)
    for (int c = 0; c < cm.n_sub; ++c) {
      const int64_t rows = (int64_t)1 << (2 * cm.subs[c].k());
      D.rowmax_off.push_back(off);
      off = align256(off + rows * 8);
      D.rexp_off.push_back(off);
      off = align256(off + rows * 4);
    }
  D.plan_off = off;
  off = align256(off + D.plan.workspace_bytes);
  D.bins_off = off;
  off += D.bins_bytes;
  D.big = align256(off);
}

struct DDCtrl {
  int64_t prog = 0, state = 0, level = 0, recs = 0, bytes = 0;
};

DDCtrl dd_ctrl(int R) {
  DDCtrl c;
  c.prog = 0;
  c.state = align256(c.prog + (int64_t)sizeof(DDProgram));
  c.level = align256(c.state + (int64_t)sizeof(DDState));
  c.recs = align256(c.level + (int64_t)sizeof(DDLevel));
  c.bytes = align256(c.recs + (int64_t)R * (int64_t)sizeof(cq_dd_record));
  return c;
}

// Exponent groups of the last GEMM's output for column scaling: its rows
// (z * M + m) and columns (n) each concatenate output axes, one per
// subcircuit, the last axis lowest; member c's bits start after the axes
// below it, a shift of (labels' fixed bits) + sum of their subcircuits' na.
// False (no scaling) unless every subcircuit has one output axis there and
// the shifts reproduce the plan at the largest counts.
bool dd_fac_groups(DDInstancePlan& D) {
  const Plan& plan = D.plan;
  const GemmStep& g = plan.steps.back().g;
  const std::vector<Axis>& ax = plan.tensors[g.c].axes;
  const int ns = D.cm.n_sub;
  int row_bits = 0;
  while (((int64_t)1 << row_bits) < g.Z * g.M) ++row_bits;
  size_t split = 0;
  for (int acc = 0; split < ax.size() && acc < row_bits; ++split) acc += ax[split].log2;
  while (split < ax.size() && ax[split].log2 == 0) ++split;
  int acc = 0;
  for (size_t i = 0; i < split; ++i) acc += ax[i].log2;
  if (acc != row_bits) return false;
  std::vector<bool> seen(ns, false);
  const size_t lo[2] = {0, split}, hi[2] = {split, ax.size()};
  for (int q = 0; q < 2; ++q) {
    D.fac_n[q] = 0;
    int c0 = 0, shift = 0;
    uint32_t mask = 0;
    for (size_t i = hi[q]; i-- > lo[q];) {
      const Axis& a = ax[i];
      if (a.kind == 1) {
        if (D.fac_n[q] >= CQ_MAX_SUBCIRCUITS || a.id < 0 || a.id >= ns || seen[a.id] || a.log2 != D.amax[a.id])
          return false;
        int at = c0;
        for (int c = 0; c < ns; ++c)
          if ((mask >> c) & 1u) at += D.amax[c];
        if (at != shift) return false;
        D.fac_sub[q][D.fac_n[q]] = a.id;
        D.fac_shift[q][D.fac_n[q]] = SymLog{c0, mask};
        ++D.fac_n[q];
        seen[a.id] = true;
        mask |= 1u << a.id;
      } else {
        c0 += a.log2;
      }
      shift += a.log2;
    }
  }
  for (int c = 0; c < ns; ++c)
    if (!seen[c]) return false;
  D.rowexp_n = g.Z * g.M;
  D.colexp_n = g.N;
  D.rowtmax_n = g.Z * ((g.M + 127) / 128);
  return true;
}

cq_status dd_plan_instance(const cq_dd_instance& in, const cq_dd_params& p, bool bins_stored,
                           DDInstancePlan& D) {
  cq_status st = dd_validate(in, p, D.cm, D.s0);
  if (st != CQ_OK) return st;
  const CutMap& cm = D.cm;
  int sum_a = 0;
  D.amax.clear();
  for (int c = 0; c < cm.n_sub; ++c) {
    const int a = std::max(popc(D.s0[c].active), std::min(in.max_active[c], cm.subs[c].n()));
    D.amax.push_back(a);
    sum_a += a;
  }
  st = make_sym_plan(cm, D.amax, work_elem_bytes(p.prec), D.plan, D.sp);
  if (st != CQ_OK) return st;
  D.lbal = balance_applies(p.prec) && cm.K > 0;
  if ((int)D.plan.steps.size() > kDDMaxSteps || (int)D.plan.tensors.size() > kDDMaxTensors)
    return fail(CQ_ERR_UNSUPPORTED, "bin contraction plan too long for the device program");
  for (const Step& s : D.plan.steps)
    if (!s.is_gemm && (int)s.p.log2.size() > kDDMaxPermAxes)
      return fail(CQ_ERR_UNSUPPORTED, "bin contraction permute has too many axes");
  D.max_count = (int64_t)1 << sum_a;
  D.step_max.clear();
  for (const Step& s : D.plan.steps) {
    if (s.is_gemm) {
      const GemmStep& g = s.g;
      D.step_max.push_back(((g.M + 127) / 128) * ((g.N + 127) / 128) * g.Z);
      if (D.step_max.back() > 0x7fffffffLL) return fail(CQ_ERR_SHAPE, "bin contraction too large");
    } else {
      int bits = 0;
      for (int l : s.p.log2) bits += l;
      D.step_max.push_back((int64_t)1 << bits);
    }
  }
  const int C_max = std::min(4 * p.R, kDDMaxC);
  // Without bin buffers from the caller and with a GEMM writing the bins, the
  // bins are never stored: that GEMM selects top-C candidates itself.
  const Step& last = D.plan.steps.back();
  D.topc_step = -1;
  if (!bins_stored && last.is_gemm && D.plan.tensors[last.g.c].loc == Loc::Out)
    D.topc_step = (int)D.plan.steps.size() - 1;
  D.cscale = cscale_applies(p.prec) && last.is_gemm && D.plan.tensors[last.g.c].loc == Loc::Out && dd_fac_groups(D);
  D.bins_bytes = (bins_stored || D.topc_step >= 0) ? 0 : align256(D.max_count * (p.prec == CQ_FP64 ? 8 : 4));
  D.sel = DDSel();
  if (D.topc_step >= 0) {
    const GemmStep& g = D.plan.steps[D.topc_step].g;
    D.sel.tiles = D.step_max[D.topc_step];
    D.sel.cand_cap = D.sel.tiles * C_max;
    D.sel.seg_a = (g.sAz ? g.Z : 1) * g.K * ((g.M + 127) / 128);
    D.sel.seg_b = (g.sBz ? g.Z : 1) * g.K * ((g.N + 127) / 128);
  } else {
    D.sel.cand_cap = topk_indirect_capacity(D.max_count, C_max);
  }
  dd_layout(D, D.sel);
  return CQ_OK;
}

DType tensor_dtype(const Plan& plan, int t, cq_precision prec) {
  const TensorRef& T = plan.tensors[t];
  if (T.loc == Loc::Out) return out_dtype(prec);
  if (T.loc == Loc::Input && plan.input_offset[T.index] < 0) return DType::F64;
  return work_dtype(prec);
}

// Instances whose launches can be shared: the same subcircuit count and the
// same step sequence with the same operand formats (their sizes may differ;
// the launches are sized for the largest).
std::string dd_signature(const DDInstancePlan& D, cq_precision prec) {
  std::string k;
  auto put = [&](int v) { k.append(reinterpret_cast<const char*>(&v), sizeof v); };
  put(D.cm.n_sub);
  put((int)D.plan.steps.size());
  put(D.topc_step);
  for (const Step& s : D.plan.steps) {
    put(s.is_gemm ? 1 : 0);
    if (s.is_gemm) {
      put((int)tensor_dtype(D.plan, s.g.a, prec));
      put((int)tensor_dtype(D.plan, s.g.b, prec));
      put((int)tensor_dtype(D.plan, s.g.c, prec));
    } else {
      put((int)tensor_dtype(D.plan, s.p.src, prec));
      put((int)tensor_dtype(D.plan, s.p.dst, prec));
    }
  }
  return k;
}

// How a batch runs.  When every instance keeps its bins inside the
// contraction (no bin buffers), instances with one signature form a group
// that advances in lockstep: recursion r of all of them is one launch per
// kernel, grid z running over the group.  Each instance then owns a slot --
// its control block, then its region -- of one size, and a group's slots are
// consecutive, so instance z's arguments and buffers are instance 0's moved by
// z slots.  Groups spread over up to `lanes` streams.  Otherwise the instances
// run one after another on one region, each with its own control block.
struct DDBatch {
  bool lockstep = false;
  std::vector<std::vector<int>> groups;  // lockstep: instances of each group, in slot order
  std::vector<int> slot_of;              // instance -> slot (control block index otherwise)
  int lanes = 1;
  int64_t slot = 0;   // lockstep: bytes per slot
  int64_t big = 0;    // otherwise: bytes of the shared region
  int64_t total = 0;  // workspace bytes
  // set per call: states copied in from checkpoints before the first
  // recursion, and copied out into the readback block after the last
  bool resume = false, checkpoint = false;
};

// Beyond the slots (or the shared region and the control blocks): the
// programs of all instances back to back in slot order (one upload per call;
// a copy kernel at the head of the batch moves each into its control block)
// followed by the resumed states, and the readback block (records and
// recursion count of every slot back to back, gathered by a copy kernel at
// the tail of the batch) followed by the states to checkpoint.
struct DDAreas {
  char* ctrl0;
  int64_t ctrl_stride;
  char* region0;
  int64_t region_stride;
  char* upload;
  char* gather;
  char* states_in;   // resumed states, slot order
  char* states_out;  // states after the call, slot order
  int64_t prog_stride, rec_bytes, gather_stride, state_stride, bytes;
  char* ctrl(int k) const { return ctrl0 + (int64_t)k * ctrl_stride; }
  char* region(int k) const { return region0 + (int64_t)k * region_stride; }
};

DDAreas dd_areas(char* ws, int n_inst, int R, const DDBatch& B) {
  DDAreas A;
  const DDCtrl L = dd_ctrl(R);
  A.prog_stride = ((int64_t)sizeof(DDProgram) + 15) / 16 * 16;
  A.rec_bytes = (int64_t)R * (int64_t)sizeof(cq_dd_record);
  A.gather_stride = (A.rec_bytes + 8 + 15) / 16 * 16;  // records, then the int32 count
  int64_t ctrl, region, up;
  if (B.lockstep) {
    ctrl = 0;
    region = L.bytes;
    A.ctrl_stride = A.region_stride = B.slot;
    up = (int64_t)n_inst * B.slot;
  } else {
    region = 0;
    ctrl = align256(B.big);
    A.ctrl_stride = L.bytes;
    A.region_stride = 0;
    up = ctrl + (int64_t)n_inst * L.bytes;
  }
  A.state_stride = ((int64_t)sizeof(DDState) + 15) / 16 * 16;
  const int64_t sin = up + align256((int64_t)n_inst * A.prog_stride);
  const int64_t ga = sin + align256((int64_t)n_inst * A.state_stride);
  const int64_t sout = ga + align256((int64_t)n_inst * A.gather_stride);
  A.bytes = sout + align256((int64_t)n_inst * A.state_stride);
  A.ctrl0 = ws ? ws + ctrl : nullptr;
  A.region0 = ws ? ws + region : nullptr;
  A.upload = ws ? ws + up : nullptr;
  A.states_in = ws ? ws + sin : nullptr;
  A.gather = ws ? ws + ga : nullptr;
  A.states_out = ws ? ws + sout : nullptr;
  return A;
}

constexpr int kDDLanes = 4;
constexpr int kDDMaxLanes = 8;
std::atomic<int> g_dd_lanes{0};  // 0: kDDLanes

cq_status dd_plan_all(int32_t n_inst, const cq_dd_instance* inst, const cq_dd_params& p,
                      bool bins_stored, std::vector<DDInstancePlan>& plans, DDBatch& B) {
  plans.assign(n_inst, DDInstancePlan());
  B = DDBatch();
  bool all_fused = true;
  for (int i = 0; i < n_inst; ++i) {
    cq_status st = dd_plan_instance(inst[i], p, bins_stored, plans[i]);
    if (st != CQ_OK) return st;
    all_fused = all_fused && plans[i].topc_step >= 0;
  }
  B.slot_of.assign(n_inst, 0);
  if (!all_fused) {
    for (int i = 0; i < n_inst; ++i) {
      B.big = std::max(B.big, plans[i].big);
      B.slot_of[i] = i;
    }
  } else {
    B.lockstep = true;
    std::vector<std::string> sigs;
    for (int i = 0; i < n_inst; ++i) {
      const std::string sg = dd_signature(plans[i], p.prec);
      size_t g = 0;
      while (g < sigs.size() && sigs[g] != sg) ++g;
      if (g == sigs.size()) {
        sigs.push_back(sg);
        B.groups.emplace_back();
      }
      B.groups[g].push_back(i);
    }
    int k = 0;
    int64_t region = 0;
    for (const std::vector<int>& G : B.groups) {
      DDSel s;
      for (int i : G) {
        const DDSel& o = plans[i].sel;
        s.cand_cap = std::max(s.cand_cap, o.cand_cap);
        s.seg_a = std::max(s.seg_a, o.seg_a);
        s.seg_b = std::max(s.seg_b, o.seg_b);
        s.tiles = std::max(s.tiles, o.tiles);
      }
      for (int i : G) {
        dd_layout(plans[i], s);
        region = std::max(region, plans[i].big);
        B.slot_of[i] = k++;
      }
    }
    B.slot = dd_ctrl(p.R).bytes + align256(region);
    const int want = g_dd_lanes.load();
    B.lanes = std::max(1, std::min<int>((int)B.groups.size(), want > 0 ? want : kDDLanes));
  }
  B.total = dd_areas(nullptr, n_inst, p.R, B).bytes;
  return CQ_OK;
}

SymPow to_dev(const SymQ& q) {
  SymPow s;
  s.c0 = q.c0;
  s.mask = q.mask;
  s.zero = q.zero ? 1 : 0;
  s.pad = 0;
  return s;
}

// Host image of an instance's device program; pointers refer to its region
// `ws` and its control block `ctrl`.
void dd_program(const DDInstancePlan& D, const cq_dd_instance& in, const cq_dd_params& p, char* ws,
                char* ctrl, int r0, int r_end, bool resume, DDProgram& P) {
  std::memset(&P, 0, sizeof(P));
  P.resume = resume ? 1 : 0;
  P.r0 = r0;
  P.r_end = r_end;
  const CutMap& cm = D.cm;
  const Plan& plan = D.plan;
  const DType wt = work_dtype(p.prec);
  const DDCtrl L = dd_ctrl(p.R);
  DDState* st = reinterpret_cast<DDState*>(ctrl + L.state);
  P.n_sub = cm.n_sub;
  P.K = cm.K;
  P.R = p.R;
  P.n_steps = (int)plan.steps.size();
  P.C_max = std::min(4 * p.R, kDDMaxC);
  for (int c = 0; c < cm.n_sub; ++c) {
    P.n_out[c] = cm.subs[c].n();
    P.max_active[c] = in.max_active[c];
    P.kc[c] = cm.subs[c].k();
    for (int j = 0; j < P.kc[c]; ++j) P.cut[c][j] = cm.subs[c].cuts[j];
    P.rows[c] = (int64_t)1 << (2 * cm.subs[c].k());
    P.E[c] = in.entries[c];
    P.Ep[c] = reinterpret_cast<double*>(ws + D.ep_off[c]);
    P.Rs[c] = reinterpret_cast<double*>(ws + D.rs_off[c]);
    P.prep_dst[c] = -1;
    P.init.active[c] = D.s0[c].active;
    P.init.merged[c] = D.s0[c].merged;
    P.init.fixed[c] = D.s0[c].fixed;
    P.init.fixed_vals[c] = D.s0[c].fixed_vals;
  }
  // the recursion total: Eq. 1 over the row sums of the reduced entries, one bin
  RefineArgs& T = P.total;
  T.n_sub = cm.n_sub;
  T.K = cm.K;
  for (int c = 0; c < cm.n_sub; ++c) {
    T.Ep[c] = P.Rs[c];
    T.ld[c] = 1;
    T.na[c] = 0;
    T.kc[c] = P.kc[c];
    for (int j = 0; j < T.kc[c]; ++j) T.cut[c][j] = P.cut[c][j];
  }
  T.bins = &st->zero_idx;
  T.nbins = 1;
  T.scale = std::ldexp(1.0, -cm.K);
  T.out = &st->total;
  P.cscale = D.cscale ? 1 : 0;
  if (D.cscale) {
    for (int q = 0; q < 2; ++q) {
      P.fac_n[q] = D.fac_n[q];
      for (int i = 0; i < D.fac_n[q]; ++i) {
        P.fac_sub[q][i] = D.fac_sub[q][i];
        P.fac_shift[q][i] = D.fac_shift[q][i];
      }
    }
    for (int c = 0; c < cm.n_sub; ++c) P.colmax[c] = reinterpret_cast<uint64_t*>(ws + D.colmax_off[c]);
    P.rowexp = reinterpret_cast<int32_t*>(ws + D.rowexp_off);
    P.colexp = reinterpret_cast<int32_t*>(ws + D.colexp_off);
    P.rowtmax = reinterpret_cast<int32_t*>(ws + D.rowtmax_off);
  }
  P.balance = D.lbal ? 1 : 0;
  if (D.lbal) {
    P.bal = balance_struct(cm);
    for (int c = 0; c < cm.n_sub; ++c) {
      P.bal.rowmax[c] = reinterpret_cast<const uint64_t*>(ws + D.rowmax_off[c]);
      P.bal.rexp[c] = reinterpret_cast<int32_t*>(ws + D.rexp_off[c]);
    }
  }
  P.topc_step = D.topc_step;
  P.cand_v = reinterpret_cast<double*>(ws + D.cand_off);
  P.cand_i = reinterpret_cast<uint64_t*>(ws + D.cand_off + D.cand_cap * 8);
  if (D.topc_step >= 0) {
    P.bound_a = reinterpret_cast<float*>(ws + D.bound_a_off);
    P.bound_b = reinterpret_cast<float*>(ws + D.bound_b_off);
    P.bound_u = reinterpret_cast<float*>(ws + D.bound_u_off);
    P.tile_list = reinterpret_cast<uint64_t*>(ws + D.list_off);
    P.warm_v = reinterpret_cast<double*>(ws + D.warm_out_off);
    P.warm_i = reinterpret_cast<uint64_t*>(ws + D.warm_out_off + kDDMaxC * 8);
  }
  char* pw = ws + D.plan_off;
  for (size_t t = 0; t < plan.tensors.size(); ++t) {
    const TensorRef& T = plan.tensors[t];
    DDTensor& d = P.tensor[t];
    P.tensor_elems[t] = to_dev(D.sp.elems[t]);
    if (T.loc == Loc::Out) {
      d.is_out = 1;
      continue;
    }
    char* base;
    if (T.loc == Loc::Input) {
      if (plan.input_offset[T.index] < 0) {
        d.hi = P.Ep[T.index];
        continue;
      }
      base = pw + plan.input_offset[T.index];
      P.prep_dst[T.index] = (int)t;
    } else {
      base = pw + plan.work_offset[T.index];
    }
    d.hi = base;
    // split planes: lo follows hi at the largest size, whatever the recursion's size
    d.lo = wt == DType::H16X2 ? base + T.elems * 2 : nullptr;
  }
  for (size_t si = 0; si < plan.steps.size(); ++si) {
    const Step& s = plan.steps[si];
    P.step_is_gemm[si] = s.is_gemm ? 1 : 0;
    if (s.is_gemm) {
      const SymGemm& q = D.sp.gemm[si];
      DDGemmSym& g = P.gemm[si];
      g.a = s.g.a;
      g.b = s.g.b;
      g.c = s.g.c;
      g.Z = to_dev(q.Z);
      g.M = to_dev(q.M);
      g.N = to_dev(q.N);
      g.K = to_dev(q.K);
      g.sAz = to_dev(q.sAz);
      g.sAk = to_dev(q.sAk);
      g.sBz = to_dev(q.sBz);
      g.sBk = to_dev(q.sBk);
      g.sCz = to_dev(q.sCz);
      g.ldc = to_dev(q.ldc);
      g.alpha = s.g.alpha;
    } else {
      const SymPerm& q = D.sp.perm[si];
      DDPermSym& m = P.perm[si];
      m.src = s.p.src;
      m.dst = s.p.dst;
      m.naxes = (int)q.log2.size();
      for (int i = 0; i < m.naxes; ++i) {
        m.log2[i].c0 = q.log2[i].c0;
        m.log2[i].mask = q.log2[i].mask;
        m.sstride[i] = to_dev(q.sstride[i]);
      }
      m.alpha = s.p.alpha;
    }
  }
}

// Enqueues recursion r of the instances `G` (one, or a lockstep group whose
// first slot has region `ws` and control block `ctrl`; `span` covers the
// group).  Grids are sized for the largest member.
cq_status dd_enqueue_level(const std::vector<const DDInstancePlan*>& G, const cq_dd_params& p,
                           InstSpan span, char* ws, char* ctrl, int r, void* bins, hipStream_t stream) {
  const DDCtrl L = dd_ctrl(p.R);
  const DDInstancePlan& D = *G[0];
  const DDProgram* prog = reinterpret_cast<const DDProgram*>(ctrl + L.prog);
  DDState* st = reinterpret_cast<DDState*>(ctrl + L.state);
  DDLevel* lv = reinterpret_cast<DDLevel*>(ctrl + L.level);
  cq_dd_record* recs = reinterpret_cast<cq_dd_record*>(ctrl + L.recs);
  const int ns = D.cm.n_sub;
  const cq_precision prec = p.prec;
  hipError_t e = launch_dd_setup(prog, st, lv, recs, r, bins, stream, span);
  if (e != hipSuccess) return hip_fail(e, "setup launch");
  int64_t merge_threads = 0, rs_threads = 0, prep_n = 0;
  std::vector<int64_t> step_max(D.step_max.size(), 0);
  for (const DDInstancePlan* M : G) {
    for (int c = 0; c < ns; ++c) {
      const int64_t rows = (int64_t)1 << (2 * M->cm.subs[c].k());
      merge_threads = std::max(merge_threads, (rows << M->amax[c]) << 6);
      rs_threads = std::max(rs_threads, rows << 6);
      prep_n = std::max(prep_n, rows << M->amax[c]);
    }
    for (size_t si = 0; si < step_max.size(); ++si) step_max[si] = std::max(step_max[si], M->step_max[si]);
  }
  e = launch_merge_indirect(&lv->merge[0], ns, merge_threads, stream, span);
  if (e != hipSuccess) return hip_fail(e, "merge launch");
  e = launch_merge_indirect(&lv->rowsum[0], ns, rs_threads, stream, span);
  if (e != hipSuccess) return hip_fail(e, "row-sum launch");
  e = launch_refine_indirect(&prog->total, 1, stream, span);
  if (e != hipSuccess) return hip_fail(e, "total launch");
  if (D.lbal) {
    int64_t max_rows = 0;
    for (const DDInstancePlan* M : G)
      for (int c = 0; c < ns; ++c) max_rows = std::max(max_rows, (int64_t)1 << (2 * M->cm.subs[c].k()));
    e = launch_dd_balance(prog, lv, ns, max_rows, stream, span);
    if (e != hipSuccess) return hip_fail(e, "label balance launch");
  }
  if (D.cscale) {
    int64_t max_cols = 0;
    for (const DDInstancePlan* M : G)
      for (int c = 0; c < ns; ++c) max_cols = std::max(max_cols, (int64_t)1 << M->amax[c]);
    e = launch_dd_colmax(prog, lv, ns, max_cols, stream, span);
    if (e != hipSuccess) return hip_fail(e, "column scaling launch");
  }
  if (work_dtype(prec) != DType::F64) {
    e = launch_prep_indirect(&lv->prep[0], ns, work_dtype(prec), is_f16(prec), prep_n, stream, span);
    if (e != hipSuccess) return hip_fail(e, "operand prep launch");
  }
  if (D.cscale) {
    int64_t max_rows = 0, max_cols = 0;
    for (const DDInstancePlan* M : G) {
      max_rows = std::max(max_rows, M->rowexp_n);
      max_cols = std::max(max_cols, M->colexp_n);
    }
    e = launch_dd_expsum(prog, st, lv, (int)D.plan.steps.size() - 1, max_rows, max_cols, stream, span);
    if (e != hipSuccess) return hip_fail(e, "scale exponent launch");
  }
  for (size_t si = 0; si < D.plan.steps.size(); ++si) {
    const Step& s = D.plan.steps[si];
    if (s.is_gemm && (int)si == D.topc_step) {
      // fused top-C with tile pruning (see launch_tile_bounds)
      const int64_t tiles = step_max[si];
      e = launch_tile_bounds(&lv->gemm[si], tensor_dtype(D.plan, s.g.a, prec), is_f16(prec),
                             reinterpret_cast<float*>((ws + D.bound_a_off)),
                             reinterpret_cast<float*>((ws + D.bound_b_off)),
                             reinterpret_cast<float*>(ws + D.bound_u_off), D.seg_a, D.seg_b,
                             tiles, stream, span);
      if (e == hipSuccess)
        e = launch_tile_warm(reinterpret_cast<const float*>(ws + D.bound_u_off), &st->n_tiles,
                             &st->warm_count, reinterpret_cast<uint64_t*>(ws + D.warm_out_off + kDDMaxC * 8),
                             (int)std::min<int64_t>(tiles, kDDMaxC), stream, span);
      if (e == hipSuccess)
        e = launch_gemm_indirect(prec, &lv->topc_warm, std::min<int64_t>(tiles, kDDMaxC),
                                 tensor_dtype(D.plan, s.g.c, prec), false, true, stream, span);
      if (e == hipSuccess)
        e = launch_warm_tau(reinterpret_cast<const double*>(ws + D.cand_off), &st->topc_count, &st->C,
                            &st->topc_thr, stream, span);
      if (e == hipSuccess)
        e = launch_tile_compact(reinterpret_cast<const float*>(ws + D.bound_u_off), &st->n_tiles,
                                &st->topc_thr, reinterpret_cast<uint64_t*>(ws + D.list_off),
                                &st->list_count, tiles, stream, span);
      if (e == hipSuccess)
        e = launch_gemm_indirect(prec, &lv->gemm[si], tiles, tensor_dtype(D.plan, s.g.c, prec), false,
                                 true, stream, span);
      if (e != hipSuccess) return hip_fail(e, "top-C GEMM launch");
    } else if (s.is_gemm) {
      e = launch_gemm_indirect(prec, &lv->gemm[si], step_max[si], tensor_dtype(D.plan, s.g.c, prec), false,
                               false, stream, span);
      if (e != hipSuccess) return hip_fail(e, "label GEMM launch");
    } else {
      e = launch_permute_indirect(&lv->perm[si], tensor_dtype(D.plan, s.p.src, prec),
                                  tensor_dtype(D.plan, s.p.dst, prec), is_f16(prec), step_max[si],
                                  stream, span);
      if (e != hipSuccess) return hip_fail(e, "permute launch");
    }
  }
  if (D.topc_step >= 0) {
    e = launch_topk_candidates(reinterpret_cast<const double*>(ws + D.cand_off),
                               reinterpret_cast<const uint64_t*>(ws + D.cand_off + D.cand_cap * 8),
                               reinterpret_cast<const int64_t*>(&st->topc_count), &st->C,
                               std::min(4 * p.R, kDDMaxC), reinterpret_cast<double*>(ws + D.stage_off),
                               reinterpret_cast<uint64_t*>(ws + D.stage_off + (int64_t)kTopcStage * kDDMaxC * 8),
                               st->top_val, st->top_idx, stream, span);
  } else {
    if (span.n != 1) return fail(CQ_ERR_UNSUPPORTED, "stored bins run one instance at a time");
    e = launch_topk_indirect(bins, out_dtype(prec), &st->count, &st->C, std::min(4 * p.R, kDDMaxC),
                             D.max_count, reinterpret_cast<double*>(ws + D.cand_off),
                             reinterpret_cast<uint64_t*>(ws + D.cand_off + D.cand_cap * 8),
                             D.cand_cap, st->top_val, st->top_idx, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "top-C launch");
  e = launch_refine_indirect(&lv->refine, std::min(4 * p.R, kDDMaxC), stream, span);
  if (e != hipSuccess) return hip_fail(e, "refine launch");
  e = launch_dd_update(prog, st, recs, r, stream, span);
  if (e != hipSuccess) return hip_fail(e, "update launch");
  return CQ_OK;
}

// Streams and events of the parallel lanes; released with the graph that
// captured them, or after the call's final synchronisation.
struct DDLaneSet {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  ~DDLaneSet() {
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
  }
};

// All recursions of the instances `G` (one instance, or a lockstep group
// starting at slot k) on `stream`.
cq_status dd_enqueue_group(const std::vector<int>& G, int k, const cq_dd_params& p, int recursions,
                           const std::vector<DDInstancePlan>& plans, void* const* bins_user,
                           const DDAreas& A, InstSpan span, hipStream_t stream) {
  const DDCtrl L = dd_ctrl(p.R);
  char* ctrl = A.ctrl(k);
  char* region = A.region(k);
  std::vector<const DDInstancePlan*> members;
  for (int i : G) members.push_back(&plans[i]);
  hipError_t e = launch_dd_init(reinterpret_cast<const DDProgram*>(ctrl + L.prog),
                                reinterpret_cast<DDState*>(ctrl + L.state),
                                reinterpret_cast<cq_dd_record*>(ctrl + L.recs), p.R, stream, span);
  if (e != hipSuccess) return hip_fail(e, "init launch");
  for (int r = 0; r < recursions; ++r) {
    void* bins = nullptr;
    if (G.size() == 1) {
      const DDInstancePlan& D = plans[G[0]];
      bins = bins_user ? bins_user[(size_t)G[0] * p.R + r] : nullptr;
      if (!bins && D.topc_step < 0) bins = region + D.bins_off;
    }
    cq_status st = dd_enqueue_level(members, p, span, region, ctrl, r, bins, stream);
    if (st != CQ_OK) return st;
  }
  return CQ_OK;
}

// Enqueues the batch behind `stream`: programs into place, every instance's
// recursions (lockstep groups spread over lanes -- streams forked from and
// joined back into `stream` -- when there are several), then the records
// gathered into the readback block.
cq_status dd_enqueue_all(int32_t n_inst, const cq_dd_params& p, int recursions,
                         const std::vector<DDInstancePlan>& plans, void* const* bins_user, char* ws,
                         const DDBatch& B, hipStream_t stream, DDLaneSet& ls) {
  const DDCtrl L = dd_ctrl(p.R);
  const DDAreas A = dd_areas(ws, n_inst, p.R, B);
  hipError_t e = launch_dd_copy(A.upload, A.prog_stride, A.ctrl0 + L.prog, A.ctrl_stride,
                                (int64_t)sizeof(DDProgram), n_inst, stream);
  if (e == hipSuccess && B.resume)
    e = launch_dd_copy(A.states_in, A.state_stride, A.ctrl0 + L.state, A.ctrl_stride, (int64_t)sizeof(DDState),
                       n_inst, stream);
  if (e != hipSuccess) return hip_fail(e, "program scatter");
  if (!B.lockstep) {
    for (int i = 0; i < n_inst; ++i) {
      cq_status st = dd_enqueue_group({i}, B.slot_of[i], p, recursions, plans, bins_user, A, InstSpan(), stream);
      if (st != CQ_OK) return st;
    }
  } else if (B.lanes <= 1) {
    int k = 0;
    for (const std::vector<int>& G : B.groups) {
      cq_status st = dd_enqueue_group(G, k, p, recursions, plans, nullptr, A, InstSpan{(int)G.size(), B.slot},
                                      stream);
      if (st != CQ_OK) return st;
      k += (int)G.size();
    }
  } else {
    hipEvent_t fork = nullptr;
    e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "lane event");
    ls.events.push_back(fork);
    e = hipEventRecord(fork, stream);
    if (e != hipSuccess) return hip_fail(e, "lane fork");
    for (int l = 0; l < B.lanes; ++l) {
      hipStream_t s = nullptr;
      e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "lane stream");
      ls.streams.push_back(s);
      e = hipStreamWaitEvent(s, fork, 0);
      if (e != hipSuccess) return hip_fail(e, "lane wait");
    }
    int k = 0;
    for (size_t g = 0; g < B.groups.size(); ++g) {
      const std::vector<int>& G = B.groups[g];
      cq_status st = dd_enqueue_group(G, k, p, recursions, plans, nullptr, A, InstSpan{(int)G.size(), B.slot},
                                      ls.streams[g % (size_t)B.lanes]);
      if (st != CQ_OK) return st;
      k += (int)G.size();
    }
    for (int l = 0; l < B.lanes; ++l) {
      hipEvent_t join = nullptr;
      e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "lane event");
      ls.events.push_back(join);
      e = hipEventRecord(join, ls.streams[l]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, join, 0);
      if (e != hipSuccess) return hip_fail(e, "lane join");
    }
  }
  e = launch_dd_copy(A.ctrl0 + L.recs, A.ctrl_stride, A.gather, A.gather_stride, A.rec_bytes, n_inst, stream);
  if (e == hipSuccess)
    e = launch_dd_copy(A.ctrl0 + L.state + offsetof(DDState, done), A.ctrl_stride, A.gather + A.rec_bytes,
                       A.gather_stride, 4, n_inst, stream);
  if (e == hipSuccess && B.checkpoint)
    e = launch_dd_copy(A.ctrl0 + L.state, A.ctrl_stride, A.states_out, A.state_stride, (int64_t)sizeof(DDState),
                       n_inst, stream);
  if (e != hipSuccess) return hip_fail(e, "record gather");
  return CQ_OK;
}

// Calls of cq_reconstruct_dd that repeat every argument (the key: device,
// precision, R, recursion count, launch mode, lane setting, workspace and bin
// pointers, each instance's cut map, entry pointers and masks) reuse the
// first one's plans, device programs and, in graph mode, its instantiated
// graph.  An entry in use is taken out of the cache and put back once its
// call has synchronised, so two calls never share one.  The cache is never
// destroyed: entries left in it at exit are reclaimed with the process.
struct DDCall {
  std::string key;
  std::vector<DDInstancePlan> plans;
  DDBatch B;
  std::vector<char> upload;  // the programs, slot order
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the lane streams and fork/join events of the capture: a graph captured
  // across streams must not outlive them, so they live as long as it does
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
};
constexpr size_t kDDCallCache = 8;
std::mutex g_ddc_mu;
std::vector<DDCall>* g_ddc = new std::vector<DDCall>();  // least recently used first

void dd_call_destroy(DDCall& x) {
  if (x.exec) (void)hipGraphExecDestroy(x.exec);
  if (x.graph) (void)hipGraphDestroy(x.graph);
  for (hipStream_t s : x.streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : x.events) (void)hipEventDestroy(e);
  x = DDCall();
}

bool dd_call_take(const std::string& key, DDCall& out) {
  std::lock_guard<std::mutex> lk(g_ddc_mu);
  for (size_t i = 0; i < g_ddc->size(); ++i)
    if ((*g_ddc)[i].key == key) {
      out = std::move((*g_ddc)[i]);
      g_ddc->erase(g_ddc->begin() + (ptrdiff_t)i);
      return true;
    }
  return false;
}

void dd_call_put(DDCall& x) {
  std::lock_guard<std::mutex> lk(g_ddc_mu);
  g_ddc->push_back(std::move(x));
  x = DDCall();
  while (g_ddc->size() > kDDCallCache) {
    dd_call_destroy(g_ddc->front());
    g_ddc->erase(g_ddc->begin());
  }
}

// The cache key, read straight from the arguments; empty (no caching) when
// they are not well-formed enough to read -- the planner then reports why.
std::string dd_call_key(int32_t n_inst, const cq_dd_instance* inst, const cq_dd_params& p, int recursions,
                        void* const* bins, const void* ws, const std::vector<int>& r0) {
  std::string k;
  if (n_inst < 1 || !inst) return k;
  auto put = [&](const void* d, size_t n) { k.append(static_cast<const char*>(d), n); };
  int dev = -1;
  (void)hipGetDevice(&dev);
  const int lanes = g_dd_lanes.load();
  const int lbal = g_lbal_mode.load();
  const int cscale = g_cscale_mode.load();
  put(&dev, sizeof dev);
  put(&lbal, sizeof lbal);
  put(&cscale, sizeof cscale);
  put(&n_inst, sizeof n_inst);
  put(&p.prec, sizeof p.prec);
  put(&p.R, sizeof p.R);
  put(&p.launch, sizeof p.launch);
  put(&recursions, sizeof recursions);
  put(&ws, sizeof ws);
  put(&lanes, sizeof lanes);
  const int flags = (p.resume ? 1 : 0) | (p.checkpoint ? 2 : 0);
  put(&flags, sizeof flags);
  if (p.resume) put(r0.data(), sizeof(int) * r0.size());
  for (int i = 0; i < n_inst; ++i) {
    const cq_dd_instance& in = inst[i];
    if (in.n_sub < 1 || in.n_sub > CQ_MAX_SUBCIRCUITS || !in.subs || !in.entries || !in.active ||
        !in.merged || !in.fixed || !in.fixed_vals || !in.max_active)
      return std::string();
    put(&in.n_sub, sizeof in.n_sub);
    for (int c = 0; c < in.n_sub; ++c) {
      const cq_subcircuit& sc = in.subs[c];
      if (sc.width < 1 || sc.width > 64 || !sc.init_cut || !sc.meas_cut) return std::string();
      put(&sc.width, sizeof sc.width);
      put(sc.init_cut, sizeof(int32_t) * (size_t)sc.width);
      put(sc.meas_cut, sizeof(int32_t) * (size_t)sc.width);
      put(&in.entries[c], sizeof(const double*));
      put(&in.active[c], 8);
      put(&in.merged[c], 8);
      put(&in.fixed[c], 8);
      put(&in.fixed_vals[c], 8);
      put(&in.max_active[c], 4);
    }
  }
  const int has_bins = bins ? 1 : 0;
  put(&has_bins, sizeof has_bins);
  if (bins) put(bins, sizeof(void*) * (size_t)n_inst * (size_t)p.R);
  return k;
}

// The cache entry a call works with; once `stream` has drained it goes back
// to the cache (kept) or is destroyed (on failure).
struct DDCallHold {
  hipStream_t stream = nullptr;
  DDCall x;
  bool launched = false, keep = false;
  ~DDCallHold() {
    if (launched) (void)hipStreamSynchronize(stream);
    if (keep && !x.key.empty()) dd_call_put(x);
    else dd_call_destroy(x);
  }
};

// Launches the batch as one graph on `stream`: the entry's graph, or one
// captured on a private stream and instantiated now.
cq_status dd_run_graph(int32_t n_inst, const cq_dd_params& p, int recursions, void* const* bins_user, char* ws,
                       hipStream_t stream, DDCallHold& H, DDLaneSet& ls) {
  hipError_t e;
  DDCall& X = H.x;
  if (!X.exec) {
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return hip_fail(e, "begin capture");
    }
    cq_status st = dd_enqueue_all(n_inst, p, recursions, X.plans, bins_user, ws, X.B, cs, ls);
    e = hipStreamEndCapture(cs, &X.graph);
    // the graph owns the capture stream and the lane streams and events from
    // here on (released with it)
    X.streams.swap(ls.streams);
    X.events.swap(ls.events);
    X.streams.push_back(cs);
    if (st != CQ_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&X.exec, X.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
  }
  H.stream = stream;
  e = hipGraphLaunch(X.exec, stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  H.launched = true;
  return CQ_OK;
}

}  // namespace

extern "C" size_t cq_dd_checkpoint_bytes(void) { return sizeof(DDState); }

extern "C" cq_status cq_dd_workspace_size(int32_t n_inst, const cq_dd_instance* inst,
                                          const cq_dd_params* params, int32_t bins_stored,
                                          size_t* bytes) {
  if (n_inst < 1 || !inst || !params || !bytes) return fail(CQ_ERR_ARG, "null or empty argument");
  std::vector<DDInstancePlan> plans;
  DDBatch B;
  cq_status st = dd_plan_all(n_inst, inst, *params, bins_stored != 0, plans, B);
  if (st != CQ_OK) return st;
  *bytes = (size_t)B.total;
  return CQ_OK;
}

namespace {

// Validates, plans and runs a batch: every instance for `recursions` (<= R)
// recursions, R being the list capacity.  Records are instance-major, R per
// instance.
// A checkpoint fits an instance when its recursion index, list and masks
// could have come from a run of that instance with capacity R: masks that
// partition each subcircuit's outputs, no more active outputs than the plan
// provides for, list entries of earlier recursions with bins in range.
cq_status dd_check_state(const DDState& S, const DDInstancePlan& D, int R) {
  auto bad = [](const std::string& why) { return fail(CQ_ERR_ARG, "resume checkpoint: " + why); };
  if (S.done < 0 || S.done > R) return bad("recursion index out of range");
  if (S.stop != 0 && S.stop != 1) return bad("corrupt stop flag");
  if (S.n_list < 0 || S.n_list > R) return bad("list longer than R");
  const int ns = D.cm.n_sub;
  auto part = [&](int c, uint64_t act, uint64_t mer, uint64_t fix, uint64_t fv) {
    const int n = D.cm.subs[c].n();
    const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
    return (act | mer | fix) == all && !(act & mer) && !(act & fix) && !(mer & fix) && !(fv & ~fix);
  };
  if (!S.stop)
    for (int c = 0; c < ns; ++c) {
      if (!part(c, S.active[c], S.merged[c], S.fixed[c], S.fixed_vals[c])) return bad("masks do not partition");
      if (popc(S.active[c]) > D.amax[c]) return bad("more active outputs than the plan holds");
    }
  for (int q = 0; q < S.n_list; ++q) {
    const DDEntry& e = S.list[q];
    if (e.rec < 0 || e.rec >= S.done) return bad("list entry from a later recursion");
    for (int c = 0; c < ns; ++c)
      if (!part(c, 0, e.merged[c], e.fixed[c], e.fixed_vals[c])) return bad("list entry masks do not partition");
  }
  return CQ_OK;
}

cq_status dd_run_batch(int32_t n_inst, const cq_dd_instance* inst, const cq_dd_params* params,
                       cq_dd_record* records, void* const* bins, int32_t* recursions_done, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
  if (n_inst < 1 || !inst || !params || !records || !recursions_done)
    return fail(CQ_ERR_ARG, "null or empty argument");
  if (!prec_supported(params->prec)) return fail(CQ_ERR_UNSUPPORTED, "precision not built");
  if (params->launch != CQ_DD_GRAPH && params->launch != CQ_DD_DIRECT)
    return fail(CQ_ERR_ARG, "unknown launch mode");
  if (params->R < 1 || params->R > CQ_MAX_DD_R) return fail(CQ_ERR_ARG, "R out of range");
  if (params->recursions < 0) return fail(CQ_ERR_ARG, "negative recursion count");
  const int R = params->R;
  // each instance's starting recursion (its checkpoint's, else 0) and the
  // end of this call's range; the launches cover the longest range
  std::vector<DDState> resumed;
  std::vector<int> r0((size_t)n_inst, 0), r_end((size_t)n_inst, 0);
  if (params->resume) {
    resumed.resize((size_t)n_inst);
    for (int i = 0; i < n_inst; ++i) {
      std::memcpy(&resumed[i], static_cast<const char*>(params->resume) + (size_t)i * sizeof(DDState),
                  sizeof(DDState));
      r0[i] = resumed[i].done;
      if (r0[i] < 0 || r0[i] > R) return fail(CQ_ERR_ARG, "resume checkpoint: recursion index out of range");
    }
  }
  const int want = params->recursions > 0 ? params->recursions : R;
  int recursions = 0;
  for (int i = 0; i < n_inst; ++i) {
    r_end[i] = std::min(R, r0[i] + want);
    recursions = std::max(recursions, r_end[i] - r0[i]);
  }
  char* ws = static_cast<char*>(workspace);
  DDLaneSet lane_set;  // destroyed after the entry's graph (declared first)
  DDCallHold H;
  const std::string key = dd_call_key(n_inst, inst, *params, recursions, bins, ws, r0);
  if (key.empty() || !dd_call_take(key, H.x)) {
    // validate and plan everything before the first launch
    cq_status st = dd_plan_all(n_inst, inst, *params, bins != nullptr, H.x.plans, H.x.B);
    if (st != CQ_OK) return st;
    if (bins)
      for (int i = 0; i < n_inst; ++i)
        for (int r = 0; r < R; ++r)
          if (!bins[(size_t)i * R + r] && H.x.plans[i].bins_bytes == 0)
            return fail(CQ_ERR_ARG, "null bin buffer");
    H.x.B.resume = params->resume != nullptr;
    H.x.B.checkpoint = params->checkpoint != nullptr;
    // every instance's device program (slot order), uploaded with one copy
    const DDAreas A = dd_areas(ws, n_inst, R, H.x.B);
    H.x.upload.assign((size_t)(n_inst * A.prog_stride), 0);
    for (int i = 0; i < n_inst; ++i) {
      const int k = H.x.B.slot_of[i];
      DDProgram prog;
      dd_program(H.x.plans[i], inst[i], *params, A.region(k), A.ctrl(k), r0[i], r_end[i], H.x.B.resume, prog);
      std::memcpy(H.x.upload.data() + (size_t)k * A.prog_stride, &prog, sizeof(DDProgram));
    }
    H.x.key = key;
  }
  const DDBatch& B = H.x.B;
  for (int i = 0; i < (int)resumed.size(); ++i) {
    cq_status st = dd_check_state(resumed[i], H.x.plans[i], R);
    if (st != CQ_OK) return st;
  }
  if (!workspace || (int64_t)workspace_bytes < B.total) return fail(CQ_ERR_WORKSPACE, "workspace too small");
  if (fault_injected("dd")) return fail(CQ_ERR_HIP, "injected fault before launch");
  std::memset(records, 0, sizeof(cq_dd_record) * (size_t)n_inst * (size_t)R);
  if (recursions == 0) {  // every instance is at its end already
    for (int i = 0; i < n_inst; ++i) recursions_done[i] = 0;
    if (params->checkpoint && params->resume)
      std::memcpy(params->checkpoint, params->resume, sizeof(DDState) * (size_t)n_inst);
    H.keep = true;
    return CQ_OK;
  }
  const DDAreas A = dd_areas(ws, n_inst, R, B);
  hipError_t e = hipMemcpyAsync(A.upload, H.x.upload.data(), H.x.upload.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "program upload");
  std::vector<char> states;
  if (B.resume) {
    states.assign((size_t)(n_inst * A.state_stride), 0);
    for (int i = 0; i < n_inst; ++i)
      std::memcpy(states.data() + (size_t)B.slot_of[i] * A.state_stride, &resumed[i], sizeof(DDState));
    e = hipMemcpyAsync(A.states_in, states.data(), states.size(), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint upload");
  }
  cq_status st;
  if (params->launch == CQ_DD_GRAPH) {
    st = dd_run_graph(n_inst, *params, recursions, bins, ws, stream, H, lane_set);
  } else {
    st = dd_enqueue_all(n_inst, *params, recursions, H.x.plans, bins, ws, B, stream, lane_set);
    H.stream = stream;
    H.launched = true;
  }
  if (st != CQ_OK) return st;
  // the gathered records and counts of all instances, read back with one copy
  std::vector<char> back((size_t)(n_inst * A.gather_stride));
  e = hipMemcpyAsync(back.data(), A.gather, back.size(), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_fail(e, "record readback");
  std::vector<char> out_states;
  if (B.checkpoint) {
    out_states.resize((size_t)(n_inst * A.state_stride));
    e = hipMemcpyAsync(out_states.data(), A.states_out, out_states.size(), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint readback");
  }
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "synchronise");
  H.keep = true;
  for (int i = 0; i < n_inst; ++i) {
    const char* b = back.data() + (size_t)B.slot_of[i] * A.gather_stride;
    std::memcpy(records + (size_t)i * R, b, (size_t)A.rec_bytes);
    int32_t done = 0;
    std::memcpy(&done, b + A.rec_bytes, sizeof done);
    recursions_done[i] = done - r0[i];
    if (B.checkpoint)
      std::memcpy(static_cast<char*>(params->checkpoint) + (size_t)i * sizeof(DDState),
                  out_states.data() + (size_t)B.slot_of[i] * A.state_stride, sizeof(DDState));
  }
  return CQ_OK;
}

// Masks of the node that zooms into bin `bin` of record `rec`: the bin's
// active bits become fixed at the bin's values, then the first max_active[c]
// merged outputs (output order) of each subcircuit become active -- the rule
// of the device's list update.
void bfs_child(const cq_dd_record& rec, int ns, uint64_t bin, const int32_t* max_active, uint64_t* act,
               uint64_t* mer, uint64_t* fix, uint64_t* fv) {
  int shift = rec.n_active;
  for (int c = 0; c < ns; ++c) {
    const uint64_t a_mask = rec.active[c];
    const int a = popc(a_mask);
    shift -= a;
    const uint64_t bits = a ? (bin >> shift) & (a >= 64 ? ~0ull : ((1ull << a) - 1)) : 0;
    uint64_t v = rec.fixed_vals[c];
    int t = 0;
    for (int p = 0; p < 64; ++p)
      if ((a_mask >> p) & 1) {
        if ((bits >> (a - 1 - t)) & 1) v |= 1ull << p;
        ++t;
      }
    uint64_t m = rec.merged[c], na = 0;
    int taken = 0;
    for (int p = 0; p < 64 && taken < max_active[c]; ++p)
      if ((m >> p) & 1) {
        na |= 1ull << p;
        ++taken;
      }
    act[c] = na;
    mer[c] = m & ~na;
    fix[c] = rec.fixed[c] | a_mask;
    fv[c] = v;
  }
}

cq_dd_params bfs_batch_params(const cq_dd_bfs_params& p) {
  cq_dd_params q;
  q.prec = p.prec;
  q.R = p.width;
  q.launch = p.launch;
  q.recursions = 1;
  q.resume = nullptr;
  q.checkpoint = nullptr;
  return q;
}

}  // namespace

extern "C" cq_status cq_reconstruct_dd(int32_t n_inst, const cq_dd_instance* inst,
                                       const cq_dd_params* params, cq_dd_record* records,
                                       void* const* bins, int32_t* recursions_done, void* workspace,
                                       size_t workspace_bytes, hipStream_t stream) {
  if (!params) return fail(CQ_ERR_ARG, "null or empty argument");
  return dd_run_batch(n_inst, inst, params, records, bins, recursions_done, workspace, workspace_bytes, stream);
}

extern "C" cq_status cq_dd_bfs_workspace_size(const cq_dd_instance* root, const cq_dd_bfs_params* params,
                                              size_t* bytes) {
  if (!root || !params || !bytes) return fail(CQ_ERR_ARG, "null argument");
  if (params->width < 1 || params->width > CQ_MAX_DD_R) return fail(CQ_ERR_ARG, "width out of range");
  // a level runs at most `width` nodes, each planned like the root
  const cq_dd_params q = bfs_batch_params(*params);
  std::vector<cq_dd_instance> many((size_t)params->width, *root);
  return cq_dd_workspace_size(params->width, many.data(), &q, 0, bytes);
}

extern "C" cq_status cq_reconstruct_dd_bfs(const cq_dd_instance* root, const cq_dd_bfs_params* params,
                                           cq_dd_bfs_node* nodes, int32_t max_nodes, int32_t* n_nodes,
                                           void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!root || !params || !nodes || !n_nodes) return fail(CQ_ERR_ARG, "null argument");
  if (params->levels < 1) return fail(CQ_ERR_ARG, "levels must be positive");
  if (params->width < 1 || params->width > CQ_MAX_DD_R) return fail(CQ_ERR_ARG, "width out of range");
  if ((int64_t)max_nodes < 1 + (int64_t)(params->levels - 1) * params->width)
    return fail(CQ_ERR_ARG, "node buffer smaller than 1 + (levels - 1) * width");
  if (root->n_sub < 1 || root->n_sub > CQ_MAX_SUBCIRCUITS || !root->max_active)
    return fail(CQ_ERR_ARG, "bad root instance");
  const cq_dd_params q = bfs_batch_params(*params);
  const int W = params->width, ns = root->n_sub;
  *n_nodes = 0;
  // frontier: node masks (owned here), parent node and parent bin
  struct Front {
    uint64_t act[CQ_MAX_SUBCIRCUITS], mer[CQ_MAX_SUBCIRCUITS], fix[CQ_MAX_SUBCIRCUITS], fv[CQ_MAX_SUBCIRCUITS];
    int32_t parent;
    uint64_t parent_bin;
  };
  std::vector<Front> front(1);
  for (int c = 0; c < ns; ++c) {
    front[0].act[c] = root->active[c];
    front[0].mer[c] = root->merged[c];
    front[0].fix[c] = root->fixed[c];
    front[0].fv[c] = root->fixed_vals[c];
  }
  front[0].parent = -1;
  front[0].parent_bin = 0;
  int count = 0;
  for (int level = 0; level < params->levels && !front.empty(); ++level) {
    const int n = (int)front.size();
    std::vector<cq_dd_instance> inst((size_t)n, *root);
    for (int i = 0; i < n; ++i) {
      inst[i].active = front[i].act;
      inst[i].merged = front[i].mer;
      inst[i].fixed = front[i].fix;
      inst[i].fixed_vals = front[i].fv;
    }
    std::vector<cq_dd_record> recs((size_t)n * W);
    std::vector<int32_t> done((size_t)n, 0);
    cq_status st = dd_run_batch(n, inst.data(), &q, recs.data(), nullptr, done.data(), workspace,
                                workspace_bytes, stream);
    if (st != CQ_OK) return st;
    // candidates of the level: (value, node, bin), best first
    struct Cand {
      double v;
      int node;
      uint64_t bin;
    };
    std::vector<Cand> cands;
    for (int i = 0; i < n; ++i) {
      cq_dd_bfs_node& nd = nodes[count + i];
      nd.rec = recs[(size_t)i * W];
      nd.level = level;
      nd.parent = front[i].parent;
      nd.parent_bin = front[i].parent_bin;
      for (int j = 0; j < nd.rec.n_list; ++j) cands.push_back({nd.rec.list_val[j], count + i, nd.rec.list_bin[j]});
    }
    std::stable_sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) {
      if (a.v != b.v) return a.v > b.v;
      if (a.node != b.node) return a.node < b.node;
      return a.bin < b.bin;
    });
    if ((int)cands.size() > W) cands.resize(W);
    std::vector<Front> next(cands.size());
    for (size_t j = 0; j < cands.size(); ++j) {
      bfs_child(nodes[cands[j].node].rec, ns, cands[j].bin, root->max_active, next[j].act, next[j].mer,
                next[j].fix, next[j].fv);
      next[j].parent = cands[j].node;
      next[j].parent_bin = cands[j].bin;
    }
    count += n;
    *n_nodes = count;
    front.swap(next);
  }
  return CQ_OK;
}

// ---------------------------------------------------------------------------
// Plan introspection (include/cutqc_plan.h)
// ---------------------------------------------------------------------------
#include "cutqc_plan.h"

extern "C" cq_status cq_plan_json(int32_t n_sub, const cq_subcircuit* subs, cq_precision prec,
                                  const int32_t* out_bits, const int32_t* out_perm, char* buf,
                                  size_t buf_bytes, size_t* needed) {
  CutMap cm;
  cq_status st = build_cutmap(n_sub, subs, cm);
  if (st != CQ_OK) return st;
  if (!valid_prec(prec)) return fail(CQ_ERR_ARG, "unknown precision");
  if (!needed) return fail(CQ_ERR_ARG, "null needed");
  std::vector<int> ol;
  int n_bits = 0;
  for (int c = 0; c < n_sub; ++c) {
    int b = out_bits ? out_bits[c] : cm.subs[c].n();
    if (b < 0 || b > cm.subs[c].n()) return fail(CQ_ERR_ARG, "out_bits out of range");
    ol.push_back(b);
    n_bits += b;
  }
  if (n_bits > CQ_MAX_FD_BITS) return fail(CQ_ERR_SHAPE, "too many output bits");
  std::vector<int> perm;
  st = check_perm(out_perm, n_bits, perm);
  if (st != CQ_OK) return st;
  Plan plan;
  st = make_plan(cm, ol, work_elem_bytes(prec), perm, plan, false, cscale_applies(prec));
  if (st != CQ_OK) return st;
  // a full-definition plan reports the workspace cq_fd_workspace_size asks for
  if (!out_bits && is_h16(prec)) reserve_balance(cm, plan);
  std::string js = "{\"workspace_bytes\": " + std::to_string(plan.workspace_bytes) +
                   ", \"work_elem_bytes\": " + std::to_string(plan.work_elem_bytes) +
                   ", \"flops\": " + std::to_string(plan.flops) + ", \"tensors\": [";
  for (size_t i = 0; i < plan.tensors.size(); ++i) {
    const TensorRef& t = plan.tensors[i];
    const char* loc = t.loc == Loc::Input ? "input" : (t.loc == Loc::Out ? "out" : "work");
    js += (i ? ", " : "") + std::string("{\"loc\": \"") + loc + "\", \"index\": " +
          std::to_string(t.index) + ", \"elems\": " + std::to_string(t.elems);
    if (t.loc == Loc::Work) js += ", \"offset\": " + std::to_string(plan.work_offset[t.index]);
    if (t.loc == Loc::Input && plan.input_offset[t.index] >= 0)
      js += ", \"offset\": " + std::to_string(plan.input_offset[t.index]);
    js += "}";
  }
  js += "], \"steps\": [";
  char tmp[64];
  for (size_t i = 0; i < plan.steps.size(); ++i) {
    const Step& s = plan.steps[i];
    js += i ? ", " : "";
    if (s.is_gemm) {
      const GemmStep& g = s.g;
      std::snprintf(tmp, sizeof(tmp), "%.17g", g.alpha);
      js += "{\"op\": \"gemm\", \"a\": " + std::to_string(g.a) + ", \"b\": " + std::to_string(g.b) +
            ", \"c\": " + std::to_string(g.c) + ", \"Z\": " + std::to_string(g.Z) +
            ", \"M\": " + std::to_string(g.M) + ", \"N\": " + std::to_string(g.N) +
            ", \"K\": " + std::to_string(g.K) + ", \"sAz\": " + std::to_string(g.sAz) +
            ", \"sAk\": " + std::to_string(g.sAk) + ", \"sBz\": " + std::to_string(g.sBz) +
            ", \"sBk\": " + std::to_string(g.sBk) + ", \"sCz\": " + std::to_string(g.sCz) +
            ", \"ldc\": " + std::to_string(g.ldc) + ", \"alpha\": " + tmp + "}";
    } else {
      const PermuteStep& p = s.p;
      std::snprintf(tmp, sizeof(tmp), "%.17g", p.alpha);
      js += "{\"op\": \"permute\", \"src\": " + std::to_string(p.src) +
            ", \"dst\": " + std::to_string(p.dst) + ", \"log2\": [";
      for (size_t a = 0; a < p.log2.size(); ++a) js += (a ? ", " : "") + std::to_string(p.log2[a]);
      js += "], \"sstride\": [";
      for (size_t a = 0; a < p.sstride.size(); ++a)
        js += (a ? ", " : "") + std::to_string(p.sstride[a]);
      js += "], \"alpha\": " + std::string(tmp) + "}";
    }
  }
  js += "]}";
  *needed = js.size() + 1;
  if (!buf || buf_bytes < js.size() + 1) return fail(CQ_ERR_ARG, "buffer too small");
  std::memcpy(buf, js.c_str(), js.size() + 1);
  return CQ_OK;
}

extern "C" cq_status cq_profile_enable(int32_t on) {
  g_prof_on.store(on ? 1 : 0);
  return CQ_OK;
}

extern "C" cq_status cq_profile_read(char* names, double* ms, double* flops, int32_t cap,
                                     int32_t* count) {
  if (!count || (cap > 0 && (!names || !ms || !flops))) return fail(CQ_ERR_ARG, "null argument");
  std::vector<ProfRecord> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_prof);
  }
  *count = (int32_t)recs.size();
  cq_status st = CQ_OK;
  for (size_t i = 0; i < recs.size(); ++i) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(recs[i].stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, recs[i].start, recs[i].stop);
    if (e != hipSuccess) st = hip_fail(e, "profile event");
    if ((int32_t)i < cap) {
      std::memset(names + 32 * i, 0, 32);
      std::strncpy(names + 32 * i, recs[i].name.c_str(), 31);
      ms[i] = t;
      flops[i] = recs[i].flops;
    }
    prof_release(recs[i].dev, recs[i].start);
    prof_release(recs[i].dev, recs[i].stop);
  }
  return st;
}

extern "C" cq_status cq_column_scaling_enable(int32_t on) {
  g_cscale_mode.store(on != 0 ? 1 : 0);
  return CQ_OK;
}

extern "C" cq_status cq_label_balance_enable(int32_t mode) {
  g_lbal_mode.store(mode < 0 ? 0 : (mode > 2 ? 2 : mode));
  return CQ_OK;
}

extern "C" cq_status cq_dd_lanes(int32_t lanes) {
  g_dd_lanes.store(lanes <= 0 ? 0 : std::min(lanes, kDDMaxLanes));
  return CQ_OK;
}

extern "C" cq_status cq_autotune_enable(int32_t mode) {
  autotune_set(mode);
  return CQ_OK;
}

extern "C" cq_status cq_autotune_load(const char* path) {
  if (!path) return fail(CQ_ERR_ARG, "null path");
  if (!autotune_load(path)) return fail(CQ_ERR_ARG, std::string("cannot read ") + path);
  return CQ_OK;
}

extern "C" cq_status cq_autotune_save(const char* path) {
  if (!path) return fail(CQ_ERR_ARG, "null path");
  if (!autotune_save(path)) return fail(CQ_ERR_ARG, std::string("cannot write ") + path);
  return CQ_OK;
}

extern "C" cq_status cq_autotune_json(char* buf, size_t buf_bytes, size_t* needed) {
  if (!needed) return fail(CQ_ERR_ARG, "null argument");
  const std::string js = autotune_json();
  *needed = js.size() + 1;
  if (!buf || buf_bytes < js.size() + 1) return fail(CQ_ERR_ARG, "buffer too small");
  std::memcpy(buf, js.c_str(), js.size() + 1);
  return CQ_OK;
}

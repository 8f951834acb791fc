// extern "C" entry points: validate, plan, enqueue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <mutex>
#include <cmath>
#include <cstdlib>
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
  hipEvent_t start, stop;
  double flops;
};
std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::vector<ProfRecord> g_prof;

// Brackets one launch with events when profiling is on.
struct ProfScope {
  bool on = false;
  ProfRecord rec;
  hipStream_t stream;
  ProfScope(const char* name, double flops, hipStream_t s) : stream(s) {
    if (!g_prof_on.load()) return;
    rec.name = name;
    rec.flops = flops;
    if (hipEventCreate(&rec.start) != hipSuccess) return;
    if (hipEventCreate(&rec.stop) != hipSuccess) {
      (void)hipEventDestroy(rec.start);
      return;
    }
    on = hipEventRecord(rec.start, stream) == hipSuccess;
  }
  ~ProfScope() {
    if (!on) return;
    if (hipEventRecord(rec.stop, stream) == hipSuccess) {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof.push_back(rec);
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
cq_status execute(const Plan& plan, cq_precision prec, const double* const* inputs, void* out,
                  DType out_t, char* ws, hipStream_t stream) {
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
  // operand preparation: FP64 entries -> the precision's storage format
  for (size_t i = 0; i < plan.tensors.size(); ++i) {
    const TensorRef& t = plan.tensors[i];
    if (t.loc != Loc::Input || plan.input_offset[t.index] < 0) continue;
    hipError_t e;
    {
      ProfScope ps("prep", 0.0, stream);
      e = launch_prep(inputs[t.index], ws + plan.input_offset[t.index], t.elems, wt, f16, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "operand prep launch");
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
      {
        ProfScope ps("permute", 0.0, stream);
        e = launch_permute(L, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "permute launch");
    }
  }
  return CQ_OK;
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
  return make_plan(cm, ol, work_elem_bytes(prec), perm, plan);
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
  return execute(plan, prec, entries, out, out_dtype(prec), static_cast<char*>(workspace), stream);
}

// ---------------------------------------------------------------------------
// Dynamic definition
// ---------------------------------------------------------------------------
namespace {

struct DDSub {
  uint64_t active = 0, merged = 0, fixed = 0, fixed_vals = 0;  // output-position masks
};

int popc(uint64_t x) { return __builtin_popcountll(x); }

// output position i <-> flat bit n-1-i
uint64_t to_flat(uint64_t m, int n) {
  uint64_t f = 0;
  for (int i = 0; i < n; ++i)
    if ((m >> i) & 1) f |= (uint64_t)1 << (n - 1 - i);
  return f;
}

struct DDLayout {
  std::vector<int64_t> ep_off, rs_off;
  int64_t plan_off = 0, plan_bytes = 0;
  int64_t bins_off = 0, bins_bytes = 0;
  int64_t cand_off = 0, cand_cap = 0;
  int64_t small_off = 0;  // top-C out (val, idx), refine in/out, total
  int64_t total = 0;
  std::vector<int> amax;
};

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
    const uint64_t all = n == 64 ? ~(uint64_t)0 : (((uint64_t)1 << n) - 1);
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

cq_status dd_layout(const cq_dd_instance& in, const cq_dd_params& p, const CutMap& cm,
                    const std::vector<DDSub>& s0, bool bins_stored, DDLayout& L) {
  L = DDLayout();
  int64_t off = 0;
  int sum_a = 0;
  for (int c = 0; c < cm.n_sub; ++c) {
    const int a = std::max(popc(s0[c].active), std::min(in.max_active[c], cm.subs[c].n()));
    L.amax.push_back(a);
    sum_a += a;
  }
  for (int c = 0; c < cm.n_sub; ++c) {
    L.ep_off.push_back(off);
    off = align256(off + ((int64_t)1 << (2 * cm.subs[c].k())) * ((int64_t)1 << L.amax[c]) * 8);
  }
  for (int c = 0; c < cm.n_sub; ++c) {
    L.rs_off.push_back(off);
    off = align256(off + ((int64_t)1 << (2 * cm.subs[c].k())) * 8);
  }
  Plan plan;
  cq_status st = make_plan(cm, L.amax, work_elem_bytes(p.prec), {}, plan);
  if (st != CQ_OK) return st;
  // smaller shapes may pick another order; leave room for a factor of 2
  L.plan_off = off;
  L.plan_bytes = align256(2 * plan.workspace_bytes);
  off += L.plan_bytes;
  const int64_t nbins = (int64_t)1 << sum_a;
  L.bins_off = off;
  L.bins_bytes = bins_stored ? 0 : align256(nbins * (p.prec == CQ_FP64 ? 8 : 4));
  off += L.bins_bytes;
  L.cand_off = off;
  L.cand_cap = topk_candidate_capacity(nbins, 64);
  off = align256(off + L.cand_cap * 16);
  L.small_off = off;
  off = align256(off + 64 * 8 * 4 + 256);
  L.total = off;
  return CQ_OK;
}

struct ListEntry {
  double v;
  int rec;
  uint64_t bin;
  std::vector<DDSub> child;
};

bool list_less(const ListEntry& a, const ListEntry& b) {
  if (a.v != b.v) return a.v > b.v;
  if (a.rec != b.rec) return a.rec < b.rec;
  return a.bin < b.bin;
}

cq_status dd_run_instance(const cq_dd_instance& in, const cq_dd_params& p, cq_dd_record* recs,
                          void* const* bins_user, int32_t* done, char* ws, size_t ws_bytes,
                          hipStream_t stream) {
  CutMap cm;
  std::vector<DDSub> state;
  cq_status st = dd_validate(in, p, cm, state);
  if (st != CQ_OK) return st;
  DDLayout L;
  st = dd_layout(in, p, cm, state, bins_user != nullptr, L);
  if (st != CQ_OK) return st;
  if ((int64_t)ws_bytes < L.total || !ws) return fail(CQ_ERR_WORKSPACE, "workspace too small");
  const int n_sub = cm.n_sub;
  const int R = p.R;
  const double scale = std::ldexp(1.0, -cm.K);
  std::vector<ListEntry> list;
  double* small = reinterpret_cast<double*>(ws + L.small_off);
  double* top_val = small;                                     // 64
  uint64_t* top_idx = reinterpret_cast<uint64_t*>(small + 64);  // 64
  double* ref_out = small + 128;                               // 64
  uint64_t* zero_idx = reinterpret_cast<uint64_t*>(small + 192);  // 1
  double* total_out = small + 193;                             // 1
  hipError_t e = hipMemsetAsync(zero_idx, 0, sizeof(uint64_t), stream);
  if (e != hipSuccess) return hip_fail(e, "memset");
  *done = 0;
  for (int r = 0; r < R; ++r) {
    cq_dd_record& rec = recs[r];
    std::memset(&rec, 0, sizeof(rec));
    std::vector<int> na(n_sub), nm(n_sub);
    int sum_a = 0;
    bool any_merged = false;
    std::vector<const double*> ep(n_sub), rs(n_sub);
    for (int c = 0; c < n_sub; ++c) {
      const int n = cm.subs[c].n();
      const DDSub& d = state[c];
      rec.active[c] = d.active;
      rec.merged[c] = d.merged;
      rec.fixed[c] = d.fixed;
      rec.fixed_vals[c] = d.fixed_vals;
      na[c] = popc(d.active);
      nm[c] = popc(d.merged);
      if (na[c] > L.amax[c]) return fail(CQ_ERR_WORKSPACE, "active count exceeds the planned maximum");
      sum_a += na[c];
      any_merged = any_merged || nm[c] > 0;
      const int64_t rows = (int64_t)1 << (2 * cm.subs[c].k());
      double* Ep = reinterpret_cast<double*>(ws + L.ep_off[c]);
      double* Rs = reinterpret_cast<double*>(ws + L.rs_off[c]);
      MergeLaunch M;
      M.E = in.entries[c];
      M.Ep = Ep;
      M.rows = rows;
      M.n = n;
      M.na = na[c];
      M.nm = nm[c];
      M.active_flat = to_flat(d.active, n);
      M.merged_flat = to_flat(d.merged, n);
      M.fixed_vals_flat = to_flat(d.fixed_vals, n);
      {
        ProfScope ps("dd_merge", 0.0, stream);
        e = launch_merge(M, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "merge launch");
      // row sums of the reduced entries give the recursion total
      MergeLaunch S;
      S.E = Ep;
      S.Ep = Rs;
      S.rows = rows;
      S.n = na[c];
      S.na = 0;
      S.nm = na[c];
      S.active_flat = 0;
      S.merged_flat = na[c] == 64 ? ~(uint64_t)0 : (((uint64_t)1 << na[c]) - 1);
      S.fixed_vals_flat = 0;
      e = launch_merge(S, stream);
      if (e != hipSuccess) return hip_fail(e, "row-sum launch");
      ep[c] = Ep;
      rs[c] = Rs;
    }
    rec.n_active = sum_a;
    RefineLaunch T;
    std::memset(&T, 0, sizeof(T));
    T.n_sub = n_sub;
    T.K = cm.K;
    for (int c = 0; c < n_sub; ++c) {
      T.Ep[c] = rs[c];
      T.ld[c] = 1;
      T.na[c] = 0;
      T.kc[c] = cm.subs[c].k();
      for (int j = 0; j < T.kc[c]; ++j) T.cut[c][j] = cm.subs[c].cuts[j];
    }
    T.bins = zero_idx;
    T.nbins = 1;
    T.scale = scale;
    T.out = total_out;
    e = launch_refine(T, stream);
    if (e != hipSuccess) return hip_fail(e, "total launch");
    // bins
    Plan plan;
    st = make_plan(cm, na, work_elem_bytes(p.prec), {}, plan);
    if (st != CQ_OK) return st;
    if (plan.workspace_bytes > L.plan_bytes) return fail(CQ_ERR_WORKSPACE, "bin plan exceeds workspace");
    void* bins = bins_user ? bins_user[r] : nullptr;
    if (!bins) {
      if (L.bins_bytes == 0) return fail(CQ_ERR_ARG, "null bin buffer");
      bins = ws + L.bins_off;
    }
    st = execute(plan, p.prec, ep.data(), bins, out_dtype(p.prec), ws + L.plan_off, stream);
    if (st != CQ_OK) return st;
    const int64_t nbins = (int64_t)1 << sum_a;
    int C = 0;
    if (any_merged) {
      C = (int)std::min<int64_t>(std::min(4 * R, 64), nbins);
      TopkLaunch K;
      K.bins = bins;
      K.t = out_dtype(p.prec);
      K.count = nbins;
      K.C = C;
      K.cand_val = reinterpret_cast<double*>(ws + L.cand_off);
      K.cand_idx = reinterpret_cast<uint64_t*>(ws + L.cand_off + L.cand_cap * 8);
      K.cand_capacity = L.cand_cap;
      K.out_val = top_val;
      K.out_idx = top_idx;
      {
        ProfScope ps("dd_topk", 0.0, stream);
        e = launch_topk(K, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "top-C launch");
      RefineLaunch F;
      std::memset(&F, 0, sizeof(F));
      F.n_sub = n_sub;
      F.K = cm.K;
      for (int c = 0; c < n_sub; ++c) {
        F.Ep[c] = ep[c];
        F.ld[c] = (int64_t)1 << na[c];
        F.na[c] = na[c];
        F.kc[c] = cm.subs[c].k();
        for (int j = 0; j < F.kc[c]; ++j) F.cut[c][j] = cm.subs[c].cuts[j];
      }
      F.bins = top_idx;
      F.nbins = C;
      F.scale = scale;
      F.out = ref_out;
      {
        ProfScope ps("dd_refine", 0.0, stream);
        e = launch_refine(F, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "refine launch");
    }
    std::vector<uint64_t> h_idx(64);
    std::vector<double> h_val(64);
    double h_total = 0.0;
    e = hipMemcpyAsync(&h_total, total_out, sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && C > 0)
      e = hipMemcpyAsync(h_idx.data(), top_idx, C * sizeof(uint64_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && C > 0)
      e = hipMemcpyAsync(h_val.data(), ref_out, C * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "readback");
    rec.total = h_total;
    // list update (Algorithm 1): R largest new bins by FP64 value
    std::vector<std::pair<double, uint64_t>> cand;
    for (int i = 0; i < C; ++i) cand.push_back({h_val[i], h_idx[i]});
    std::sort(cand.begin(), cand.end(), [](const std::pair<double, uint64_t>& a,
                                           const std::pair<double, uint64_t>& b) {
      if (a.first != b.first) return a.first > b.first;
      return a.second < b.second;
    });
    for (int i = 0; i < (int)cand.size() && i < R; ++i) {
      ListEntry le;
      le.v = cand[i].first;
      le.rec = r;
      le.bin = cand[i].second;
      int shift = sum_a;
      for (int c = 0; c < n_sub; ++c) {
        shift -= na[c];
        const uint64_t bits = (le.bin >> shift) & ((na[c] == 64) ? ~(uint64_t)0 : (((uint64_t)1 << na[c]) - 1));
        DDSub ch = state[c];
        int t = 0;
        for (int pos = 0; pos < 64; ++pos) {
          if ((ch.active >> pos) & 1) {
            if ((bits >> (na[c] - 1 - t)) & 1) ch.fixed_vals |= (uint64_t)1 << pos;
            ++t;
          }
        }
        ch.fixed |= ch.active;
        ch.active = 0;
        le.child.push_back(ch);
      }
      list.push_back(le);
    }
    std::sort(list.begin(), list.end(), list_less);
    if ((int)list.size() > R) list.resize(R);
    rec.n_list = (int)list.size();
    for (int i = 0; i < rec.n_list; ++i) {
      rec.list_val[i] = list[i].v;
      rec.list_rec[i] = list[i].rec;
      rec.list_bin[i] = list[i].bin;
    }
    *done = r + 1;
    if (list.empty()) break;
    rec.popped = 1;
    ListEntry head = list.front();
    list.erase(list.begin());
    // zoom: activate the first max_active[c] merged outputs of the popped bin
    for (int c = 0; c < n_sub; ++c) {
      DDSub nx = head.child[c];
      uint64_t act = 0, mer = nx.merged;
      int taken = 0;
      for (int pos = 0; pos < 64 && taken < in.max_active[c]; ++pos) {
        if ((mer >> pos) & 1) {
          act |= (uint64_t)1 << pos;
          ++taken;
        }
      }
      nx.active = act;
      nx.merged = mer & ~act;
      state[c] = nx;
    }
  }
  return CQ_OK;
}

}  // namespace

extern "C" cq_status cq_dd_workspace_size(int32_t n_inst, const cq_dd_instance* inst,
                                          const cq_dd_params* params, int32_t bins_stored,
                                          size_t* bytes) {
  if (n_inst < 1 || !inst || !params || !bytes) return fail(CQ_ERR_ARG, "null or empty argument");
  int64_t need = 0;
  for (int i = 0; i < n_inst; ++i) {
    CutMap cm;
    std::vector<DDSub> s0;
    cq_status st = dd_validate(inst[i], *params, cm, s0);
    if (st != CQ_OK) return st;
    DDLayout L;
    st = dd_layout(inst[i], *params, cm, s0, bins_stored != 0, L);
    if (st != CQ_OK) return st;
    need = std::max(need, L.total);
  }
  *bytes = (size_t)need;
  return CQ_OK;
}

extern "C" cq_status cq_reconstruct_dd(int32_t n_inst, const cq_dd_instance* inst,
                                       const cq_dd_params* params, cq_dd_record* records,
                                       void* const* bins, int32_t* recursions_done, void* workspace,
                                       size_t workspace_bytes, hipStream_t stream) {
  if (n_inst < 1 || !inst || !params || !records || !recursions_done)
    return fail(CQ_ERR_ARG, "null or empty argument");
  if (!prec_supported(params->prec)) return fail(CQ_ERR_UNSUPPORTED, "precision not built");
  // validate everything before the first launch
  for (int i = 0; i < n_inst; ++i) {
    CutMap cm;
    std::vector<DDSub> s0;
    cq_status st = dd_validate(inst[i], *params, cm, s0);
    if (st != CQ_OK) return st;
    DDLayout L;
    st = dd_layout(inst[i], *params, cm, s0, bins != nullptr, L);
    if (st != CQ_OK) return st;
    if (!workspace || (int64_t)workspace_bytes < L.total) return fail(CQ_ERR_WORKSPACE, "workspace too small");
  }
  if (fault_injected("dd")) return fail(CQ_ERR_HIP, "injected fault before launch");
  for (int i = 0; i < n_inst; ++i) {
    cq_status st = dd_run_instance(inst[i], *params, records + (size_t)i * params->R,
                                   bins ? bins + (size_t)i * params->R : nullptr,
                                   recursions_done + i, static_cast<char*>(workspace),
                                   workspace_bytes, stream);
    if (st != CQ_OK) return st;
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
  st = make_plan(cm, ol, work_elem_bytes(prec), perm, plan);
  if (st != CQ_OK) return st;
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
    (void)hipEventDestroy(recs[i].start);
    (void)hipEventDestroy(recs[i].stop);
  }
  return st;
}

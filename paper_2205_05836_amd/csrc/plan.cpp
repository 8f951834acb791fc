// Contraction planner for Eq. 1.
//
// Eq. 1 sums, over every labelling of the K cuts, the Kronecker product of
// the subcircuits' entry vectors.  Each cut label is shared by exactly two
// subcircuits, so the sum is a tensor-network contraction: a cut is a bond of
// dimension 4 between its two ends and every subcircuit contributes one open
// output axis.  The planner picks a pairwise contraction order (exhaustive
// dynamic programming over subsets; the paper's cut solutions have at most 5
// subcircuits) and maps every pairwise contraction onto one batched GEMM with
// the shared labels as the reduction dimension, inserting a layout permute
// only when the operands' axis orders admit no strided-batched form.
#include <algorithm>
#include <cmath>
#include <functional>
#include <limits>
#include <map>

#include "internal.hpp"

namespace cq {

namespace {

struct DPEntry {
  double cost = std::numeric_limits<double>::infinity();
  unsigned left = 0, right = 0;
};

// log2 size of the tensor obtained by contracting all subcircuits in `mask`.
int subset_log2(const CutMap& cm, const std::vector<int>& out_log2, unsigned mask) {
  int s = 0;
  for (int c = 0; c < cm.n_sub; ++c)
    if (mask & (1u << c)) s += out_log2[c];
  for (int j = 0; j < cm.K; ++j) {
    bool a = mask & (1u << cm.up[j]), b = mask & (1u << cm.down[j]);
    if (a != b) s += 2;
  }
  return s;
}

int shared_cuts(const CutMap& cm, unsigned m1, unsigned m2) {
  int s = 0;
  for (int j = 0; j < cm.K; ++j) {
    bool u1 = m1 & (1u << cm.up[j]), d1 = m1 & (1u << cm.down[j]);
    bool u2 = m2 & (1u << cm.up[j]), d2 = m2 & (1u << cm.down[j]);
    if ((u1 && d2) || (u2 && d1)) ++s;
  }
  return s;
}

int64_t pow2(int e) { return (int64_t)1 << e; }

// One run of consecutive subcircuit ids.
bool contiguous(unsigned m) {
  if (m == 0) return true;
  while (!(m & 1u)) m >>= 1;
  return (m & (m + 1)) == 0;
}

int64_t axes_size(const std::vector<Axis>& ax, size_t b, size_t e) {
  int s = 0;
  for (size_t i = b; i < e; ++i) s += ax[i].log2;
  return pow2(s);
}

bool is_label(const Axis& a) { return a.kind == 0; }

// Finds the contiguous run holding exactly the axes in `sh` (any order).
// Returns false when they are not contiguous.
bool find_run(const std::vector<Axis>& ax, const std::vector<Axis>& sh, size_t& begin) {
  if (sh.empty()) {
    begin = 0;
    return true;
  }
  for (size_t b = 0; b + sh.size() <= ax.size(); ++b) {
    bool ok = true;
    for (size_t i = 0; i < sh.size() && ok; ++i)
      ok = std::find(sh.begin(), sh.end(), ax[b + i]) != sh.end();
    if (ok) {
      begin = b;
      return true;
    }
  }
  return false;
}

// Inversions among subcircuit-output axes (0 = canonical order).
int inversions(const std::vector<Axis>& ax) {
  std::vector<int> ids;
  for (auto& a : ax)
    if (a.kind == 1) ids.push_back(a.id);
  int inv = 0;
  for (size_t i = 0; i < ids.size(); ++i)
    for (size_t j = i + 1; j < ids.size(); ++j)
      if (ids[i] > ids[j]) ++inv;
  return inv;
}

struct Builder {
  const CutMap& cm;
  const std::vector<int>& out_log2;
  Plan& plan;
  int elem;

  int new_work(const std::vector<Axis>& axes) {
    TensorRef t;
    t.loc = Loc::Work;
    t.axes = axes;
    int buf = (int)plan.work_bytes.size();
    t.index = buf;
    t.elems = pow2(t.log2_size());
    int64_t bytes = t.elems * elem;
    int64_t off = plan.workspace_bytes;
    plan.work_offset.push_back(off);
    plan.work_bytes.push_back(bytes);
    plan.workspace_bytes = off + ((bytes + 255) / 256) * 256;
    plan.tensors.push_back(t);
    return (int)plan.tensors.size() - 1;
  }

  // Permute tensor `src` into `new_axes` order (a new workspace tensor).
  int permute(int src, const std::vector<Axis>& new_axes) {
    const std::vector<Axis> old = plan.tensors[src].axes;
    int dst = new_work(new_axes);
    PermuteStep p;
    p.src = src;
    p.dst = dst;
    p.alpha = 1.0;
    for (auto& a : new_axes) {
      int64_t stride = 1;
      bool found = false;
      for (int i = (int)old.size() - 1; i >= 0; --i) {
        if (old[i] == a) {
          found = true;
          break;
        }
        stride <<= old[i].log2;
      }
      (void)found;
      p.log2.push_back(a.log2);
      p.sstride.push_back(stride);
    }
    Step s;
    s.is_gemm = false;
    s.p = p;
    plan.steps.push_back(s);
    return dst;
  }

  // Contract tensors x and y over their shared labels; returns the result id.
  int contract(int x, int y, bool final_step, bool& wrote_out) {
    wrote_out = false;
    std::vector<Axis> ax = plan.tensors[x].axes, ay = plan.tensors[y].axes;
    std::vector<Axis> sh;
    for (auto& a : ax)
      if (is_label(a) && std::find(ay.begin(), ay.end(), a) != ay.end()) sh.push_back(a);

    for (int attempt = 0; attempt < 4; ++attempt) {
      ax = plan.tensors[x].axes;
      ay = plan.tensors[y].axes;
      size_t bx = 0, by = 0;
      bool cx = find_run(ax, sh, bx), cy = find_run(ay, sh, by);
      bool same_order = cx && cy;
      if (same_order)
        for (size_t i = 0; i < sh.size(); ++i)
          if (!(ax[bx + i] == ay[by + i])) same_order = false;
      if (!same_order) {
        // Bring the shared labels to the front of the smaller tensor, in the
        // order they have in the other one (or ascending when neither is
        // contiguous).
        bool permute_x = plan.tensors[x].log2_size() <= plan.tensors[y].log2_size();
        if (!cx) permute_x = true;
        else if (!cy) permute_x = false;
        int t = permute_x ? x : y;
        const std::vector<Axis>& other = permute_x ? ay : ax;
        size_t ob = 0;
        std::vector<Axis> run;
        bool other_ok = permute_x ? cy : cx;
        if (other_ok && find_run(other, sh, ob))
          run.assign(other.begin() + ob, other.begin() + ob + sh.size());
        else {
          run = sh;
          std::sort(run.begin(), run.end(), [](const Axis& a, const Axis& b) { return a.id < b.id; });
          // the other tensor is permuted in the next attempt to match
        }
        std::vector<Axis> na = run;
        for (auto& a : plan.tensors[t].axes)
          if (std::find(sh.begin(), sh.end(), a) == sh.end()) na.push_back(a);
        int nt = permute(t, na);
        if (permute_x) x = nt;
        else y = nt;
        continue;
      }
      // Candidate GEMM mappings.
      struct Cand {
        bool a_is_x;
        bool batch_on_a;
        std::vector<Axis> result;
        int64_t Z, M, N, K;
        int64_t sAz, sAk, sBz, sBk;
      };
      std::vector<Cand> cands;
      size_t ns = sh.size();
      auto blocks = [&](const std::vector<Axis>& a, size_t b, std::vector<Axis>& P,
                        std::vector<Axis>& Q) {
        P.assign(a.begin(), a.begin() + b);
        Q.assign(a.begin() + b + ns, a.end());
      };
      std::vector<Axis> Px, Qx, Py, Qy;
      if (ns == 0) {
        Px.clear();
        Qx = ax;
        Py.clear();
        Qy = ay;
      } else {
        blocks(ax, bx, Px, Qx);
        blocks(ay, by, Py, Qy);
      }
      int64_t Kd = ns ? axes_size(sh, 0, ns) : 1;
      auto sz = [](const std::vector<Axis>& v) { return axes_size(v, 0, v.size()); };
      auto cat = [](std::vector<Axis> a, const std::vector<Axis>& b) {
        a.insert(a.end(), b.begin(), b.end());
        return a;
      };
      for (int ax_is_a = 0; ax_is_a < 2; ++ax_is_a) {
        const std::vector<Axis>& PA = ax_is_a ? Px : Py;
        const std::vector<Axis>& QA = ax_is_a ? Qx : Qy;
        const std::vector<Axis>& PB = ax_is_a ? Py : Px;
        const std::vector<Axis>& QB = ax_is_a ? Qy : Qx;
        // batch on A side: B must have no prefix
        if (PB.empty()) {
          Cand c;
          c.a_is_x = ax_is_a;
          c.batch_on_a = true;
          c.result = cat(cat(PA, QA), QB);
          c.Z = sz(PA);
          c.M = sz(QA);
          c.N = sz(QB);
          c.K = Kd;
          c.sAz = Kd * c.M;
          c.sAk = c.M;
          c.sBz = 0;
          c.sBk = c.N;
          cands.push_back(c);
        }
        // batch on B side: A must have no prefix
        if (PA.empty() && !PB.empty()) {
          Cand c;
          c.a_is_x = ax_is_a;
          c.batch_on_a = false;
          c.result = cat(cat(PB, QA), QB);
          c.Z = sz(PB);
          c.M = sz(QA);
          c.N = sz(QB);
          c.K = Kd;
          c.sAz = 0;
          c.sAk = c.M;
          c.sBz = Kd * c.N;
          c.sBk = c.N;
          cands.push_back(c);
        }
      }
      if (cands.empty()) {
        // both tensors carry a prefix before the shared run: move the run of
        // the smaller one to its front
        bool permute_x = plan.tensors[x].log2_size() <= plan.tensors[y].log2_size();
        int t = permute_x ? x : y;
        std::vector<Axis> na = sh;
        const std::vector<Axis>& src = plan.tensors[t].axes;
        size_t b0 = permute_x ? bx : by;
        na.assign(src.begin() + b0, src.begin() + b0 + ns);
        for (auto& a : src)
          if (std::find(sh.begin(), sh.end(), a) == sh.end()) na.push_back(a);
        int nt = permute(t, na);
        if (permute_x) x = nt;
        else y = nt;
        continue;
      }
      // Prefer canonical output order, then operand shapes that fill tiles.
      auto score = [&](const Cand& c) {
        double s = 1e6 * inversions(c.result);
        double mn = (double)std::min(c.M, c.N);
        s -= std::log2(std::min(mn, 256.0) + 1.0) * 10.0;
        s -= std::log2((double)c.M * (double)c.N) * 0.01;
        return s;
      };
      std::sort(cands.begin(), cands.end(),
                [&](const Cand& a, const Cand& b) { return score(a) < score(b); });
      const Cand& c = cands[0];
      int out;
      if (final_step) {
        TensorRef t;
        t.loc = Loc::Out;
        t.index = 0;
        t.axes = c.result;
        t.elems = pow2(t.log2_size());
        plan.tensors.push_back(t);
        out = (int)plan.tensors.size() - 1;
        wrote_out = true;
      } else {
        out = new_work(c.result);
      }
      GemmStep g;
      g.a = c.a_is_x ? x : y;
      g.b = c.a_is_x ? y : x;
      g.c = out;
      g.Z = c.Z;
      g.M = c.M;
      g.N = c.N;
      g.K = c.K;
      g.sAz = c.sAz;
      g.sAk = c.sAk;
      g.sBz = c.sBz;
      g.sBk = c.sBk;
      g.sCz = c.M * c.N;
      g.ldc = c.N;
      g.alpha = 1.0;
      Step s;
      s.is_gemm = true;
      s.g = g;
      plan.steps.push_back(s);
      plan.flops += 2.0 * (double)c.Z * (double)c.M * (double)c.N * (double)c.K;
      return out;
    }
    return -1;
  }
};

}  // namespace

cq_status check_plan_bounds(const Plan& plan);

cq_status add_column_scaling(const CutMap& cm, const std::vector<int>& out_log2, Plan& plan);

cq_status make_plan(const CutMap& cm, const std::vector<int>& out_log2, int work_elem_bytes,
                    const std::vector<int>& out_perm, Plan& plan, bool keep_empty,
                    bool column_scaling) {
  plan = Plan();
  plan.work_elem_bytes = work_elem_bytes;
  const int n = cm.n_sub;
  int n_bits = 0;
  for (int c = 0; c < n; ++c) n_bits += out_log2[c];
  for (int c = 0; c < n; ++c) {
    TensorRef t;
    t.loc = Loc::Input;
    t.index = c;
    for (int id : cm.subs[c].cuts) t.axes.push_back(Axis{0, id, 2});
    if (out_log2[c] > 0 || keep_empty) t.axes.push_back(Axis{1, c, out_log2[c]});
    t.elems = pow2(t.log2_size());
    plan.tensors.push_back(t);
  }
  // Every precision but FP64 contracts converted copies of the entries
  // (FP32, or 16-bit hi/lo planes); they lead the workspace.
  plan.input_offset.assign(n, -1);
  if (work_elem_bytes != 8) {
    for (int c = 0; c < n; ++c) {
      plan.input_offset[c] = plan.workspace_bytes;
      const int64_t bytes = plan.tensors[c].elems * work_elem_bytes;
      plan.workspace_bytes += ((bytes + 255) / 256) * 256;
    }
  }
  // Exhaustive DP over subsets for the cheapest pairwise order.
  const unsigned full = (1u << n) - 1;
  std::vector<DPEntry> dp(full + 1);
  for (int c = 0; c < n; ++c) dp[1u << c].cost = 0.0;
  for (unsigned m = 1; m <= full; ++m) {
    if ((m & (m - 1)) == 0) continue;
    for (unsigned a = (m - 1) & m; a > 0; a = (a - 1) & m) {
      unsigned b = m ^ a;
      if (a > b) continue;
      double l2a = subset_log2(cm, out_log2, a), l2b = subset_log2(cm, out_log2, b);
      double l2r = subset_log2(cm, out_log2, m);
      int sh = shared_cuts(cm, a, b);
      double flops = 2.0 * std::pow(2.0, l2r + 2.0 * sh);
      double bytes = work_elem_bytes * (std::pow(2.0, l2a) + std::pow(2.0, l2b) + std::pow(2.0, l2r));
      double cost = dp[a].cost + dp[b].cost + flops + 20.0 * bytes;
      // the root's result is in concatenated order only when each side is a
      // contiguous range of subcircuits; otherwise a final permute reads and
      // writes the whole output once more
      if (m == full && !(contiguous(a) && contiguous(b)))
        cost += 20.0 * 2.0 * work_elem_bytes * std::pow(2.0, l2r);
      if (cost < dp[m].cost) {
        dp[m].cost = cost;
        dp[m].left = a;
        dp[m].right = b;
      }
    }
  }
  Builder B{cm, out_log2, plan, work_elem_bytes};
  const double alpha = std::ldexp(1.0, -cm.K);
  bool need_final_permute = !out_perm.empty();
  int result = -1;
  bool wrote_out = false;
  if (n == 1) {
    result = 0;
  } else {
    // Realise the tree; the root writes straight to the output when its
    // layout is already final.
    std::function<int(unsigned, bool)> realise = [&](unsigned m, bool root) -> int {
      if ((m & (m - 1)) == 0) {
        int c = 0;
        while (!(m & (1u << c))) ++c;
        return c;
      }
      int x = realise(dp[m].left, false);
      int y = realise(dp[m].right, false);
      bool wo = false;
      int r = B.contract(x, y, false, wo);
      (void)root;
      return r;
    };
    int x = realise(dp[full].left, false);
    int y = realise(dp[full].right, false);
    // Try the final contraction straight into the output.
    size_t steps_before = plan.steps.size();
    size_t tensors_before = plan.tensors.size();
    Plan saved = plan;
    result = B.contract(x, y, true, wrote_out);
    if (result < 0) return fail(CQ_ERR_UNSUPPORTED, "planner found no GEMM mapping");
    if (inversions(plan.tensors[result].axes) != 0 || need_final_permute) {
      // redo into the workspace, then permute
      plan = saved;
      (void)steps_before;
      (void)tensors_before;
      result = B.contract(x, y, false, wrote_out);
      if (result < 0) return fail(CQ_ERR_UNSUPPORTED, "planner found no GEMM mapping");
      wrote_out = false;
    }
  }
  if (wrote_out) {
    // scale the last GEMM by 2^-K
    plan.steps.back().g.alpha = alpha;
  } else {
    // Final permute: source = result tensor (input or workspace), destination
    // = output in concatenated order, then out_perm applied at bit level.
    const std::vector<Axis>& sa = plan.tensors[result].axes;
    // bit position (from the least significant end) of subcircuit c's output
    // bit i (i = 0 most significant) in the source flat index
    std::vector<std::vector<int64_t>> src_bit(n);
    int pos = 0;
    for (int i = (int)sa.size() - 1; i >= 0; --i) {
      const Axis& a = sa[i];
      if (a.kind == 1) {
        src_bit[a.id].assign(a.log2, 0);
        for (int b = 0; b < a.log2; ++b) src_bit[a.id][a.log2 - 1 - b] = pos + b;
      }
      pos += a.log2;
    }
    // concatenated bit list (most significant first)
    std::vector<int64_t> concat_src;
    for (int c = 0; c < n; ++c)
      for (int i = 0; i < out_log2[c]; ++i) concat_src.push_back(src_bit[c].empty() ? 0 : src_bit[c][i]);
    std::vector<int64_t> dst_src(n_bits);
    if (out_perm.empty()) {
      dst_src = concat_src;
    } else {
      for (int i = 0; i < n_bits; ++i) dst_src[out_perm[i]] = concat_src[i];
    }
    PermuteStep p;
    p.src = result;
    TensorRef t;
    t.loc = Loc::Out;
    t.index = 0;
    t.elems = pow2(n_bits);
    plan.tensors.push_back(t);
    p.dst = (int)plan.tensors.size() - 1;
    p.alpha = (n == 1) ? alpha : 1.0;
    if (n > 1) {
      // the last GEMM wrote unscaled values into the workspace
      for (auto it = plan.steps.rbegin(); it != plan.steps.rend(); ++it)
        if (it->is_gemm) {
          it->g.alpha = alpha;
          break;
        }
    }
    // merge runs of destination bits whose source bits are consecutive
    for (int q = 0; q < n_bits;) {
      int run = 1;
      while (q + run < n_bits && dst_src[q + run] + 1 == dst_src[q + run - 1]) ++run;
      p.log2.push_back(run);
      p.sstride.push_back((int64_t)1 << dst_src[q + run - 1]);
      q += run;
    }
    if (n_bits == 0) {
      p.log2.push_back(0);
      p.sstride.push_back(1);
    }
    Step s;
    s.is_gemm = false;
    s.p = p;
    plan.steps.push_back(s);
  }
  if (column_scaling) {
    cq_status st = add_column_scaling(cm, out_log2, plan);
    if (st != CQ_OK) return st;
  }
  return check_plan_bounds(plan);
}

cq_status add_column_scaling(const CutMap& cm, const std::vector<int>& out_log2, Plan& plan) {
  auto reserve = [&](int64_t bytes) {
    const int64_t off = plan.workspace_bytes;
    plan.workspace_bytes = off + (bytes + 255) / 256 * 256;
    return off;
  };
  plan.scaled = true;
  plan.colmax_offset.clear();
  for (int c = 0; c < cm.n_sub; ++c) plan.colmax_offset.push_back(reserve(pow2(out_log2[c]) * 8));
  // subcircuits whose outputs take no part: one column, digit always 0
  std::vector<bool> seen(cm.n_sub, false);
  auto add = [&](Plan::FacGroup& g, const std::vector<Axis>& ax, size_t b, size_t e) {
    int shift = 0;
    for (size_t i = e; i-- > b;) {
      if (ax[i].kind == 1) {
        g.sub.push_back(ax[i].id);
        g.shift.push_back(shift);
        g.bits.push_back(ax[i].log2);
        seen[ax[i].id] = true;
      }
      shift += ax[i].log2;
    }
  };
  const Step& last = plan.steps.back();
  Plan::FacGroup* rest = nullptr;
  if (last.is_gemm && plan.tensors[last.g.c].loc == Loc::Out) {
    const GemmStep& g = last.g;
    const std::vector<Axis>& ax = plan.tensors[g.c].axes;
    int row_bits = 0;
    while ((pow2(row_bits)) < g.Z * g.M) ++row_bits;
    size_t split = 0;
    for (int acc = 0; split < ax.size() && acc < row_bits; ++split) acc += ax[split].log2;
    while (split < ax.size() && ax[split].log2 == 0) ++split;
    int acc = 0;
    for (size_t i = 0; i < split; ++i) acc += ax[i].log2;
    if (acc != row_bits) return fail(CQ_ERR_UNSUPPORTED, "internal: final GEMM rows do not split at an axis");
    add(plan.row_fac, ax, 0, split);
    add(plan.col_fac, ax, split, ax.size());
    plan.rowexp_count = g.Z * g.M;
    plan.colexp_count = g.N;
    plan.rowexp_offset = reserve(plan.rowexp_count * 4);
    plan.colexp_offset = reserve(plan.colexp_count * 4);
    rest = &plan.row_fac;
  } else if (!last.is_gemm) {
    const std::vector<Axis>& ax = plan.tensors[last.p.src].axes;
    add(plan.perm_fac, ax, 0, ax.size());
    rest = &plan.perm_fac;
  } else {
    return fail(CQ_ERR_UNSUPPORTED, "internal: plan ends without writing the output");
  }
  for (int c = 0; c < cm.n_sub; ++c)
    if (!seen[c]) {
      rest->sub.push_back(c);
      rest->shift.push_back(0);
      rest->bits.push_back(0);
    }
  if ((int)plan.perm_fac.sub.size() > CQ_MAX_SUBCIRCUITS || (int)plan.row_fac.sub.size() > CQ_MAX_SUBCIRCUITS)
    return fail(CQ_ERR_UNSUPPORTED, "internal: too many scale factors");
  return CQ_OK;
}

int64_t sym_value(const SymQ& q, const std::vector<int>& na) {
  return q.zero ? 0 : pow2(sym_log2(q, na));
}

int sym_log2(const SymQ& q, const std::vector<int>& na) {
  int e = q.c0;
  for (size_t c = 0; c < na.size(); ++c)
    if ((q.mask >> c) & 1u) e += na[c];
  return e;
}

namespace {

SymQ sym_axis(const Axis& a) {
  SymQ q;
  if (a.kind == 0) q.c0 = a.log2;
  else q.mask = 1u << a.id;
  return q;
}

SymQ sym_size(const std::vector<Axis>& ax, size_t b, size_t e) {
  SymQ q;
  for (size_t i = b; i < e; ++i) {
    const SymQ s = sym_axis(ax[i]);
    q.c0 += s.c0;
    q.mask |= s.mask;
  }
  return q;
}

SymQ sym_mul(SymQ a, const SymQ& b) {
  a.c0 += b.c0;
  a.mask |= b.mask;
  a.zero = a.zero || b.zero;
  return a;
}

SymQ sym_zero() {
  SymQ q;
  q.zero = true;
  return q;
}

// Permute from `src` axes to `dst` axes (every dst axis present in src).
bool sym_permute(const std::vector<Axis>& src, const std::vector<Axis>& dst, SymPerm& sp,
                 PermuteStep& num, const std::vector<int>& amax) {
  sp = SymPerm();
  num.log2.clear();
  num.sstride.clear();
  for (const Axis& a : dst) {
    int i = (int)src.size() - 1;
    while (i >= 0 && !(src[i] == a)) --i;
    if (i < 0) return false;
    sp.log2.push_back(sym_axis(a));
    sp.sstride.push_back(sym_size(src, i + 1, src.size()));
    num.log2.push_back(sym_log2(sp.log2.back(), amax));
    num.sstride.push_back(sym_value(sp.sstride.back(), amax));
  }
  return true;
}

// Source offset of each destination bit (least significant first).
std::vector<int64_t> unit_offsets(const PermuteStep& p) {
  std::vector<int64_t> off;
  for (int a = (int)p.log2.size() - 1; a >= 0; --a)
    for (int b = 0; b < p.log2[a]; ++b) off.push_back(p.sstride[a] << b);
  return off;
}

}  // namespace

cq_status make_sym_plan(const CutMap& cm, const std::vector<int>& amax, int work_elem_bytes,
                        Plan& plan, SymPlan& sp) {
  cq_status st = make_plan(cm, amax, work_elem_bytes, {}, plan, true);
  if (st != CQ_OK) return st;
  sp = SymPlan();
  std::vector<Axis> all_out;
  for (int c = 0; c < cm.n_sub; ++c) all_out.push_back(Axis{1, c, amax[c]});
  for (const TensorRef& t : plan.tensors) {
    // the final permute's destination carries no axes: it holds every output
    const bool bare_out = t.loc == Loc::Out && t.axes.empty();
    const std::vector<Axis>& ax = bare_out ? all_out : t.axes;
    sp.elems.push_back(sym_size(ax, 0, ax.size()));
    if (sym_value(sp.elems.back(), amax) != t.elems)
      return fail(CQ_ERR_UNSUPPORTED, "internal: symbolic tensor size mismatch");
  }
  sp.gemm.resize(plan.steps.size());
  sp.perm.resize(plan.steps.size());
  auto bad = [] { return fail(CQ_ERR_UNSUPPORTED, "internal: symbolic plan mismatch"); };
  for (size_t si = 0; si < plan.steps.size(); ++si) {
    Step& s = plan.steps[si];
    if (s.is_gemm) {
      const GemmStep& g = s.g;
      const std::vector<Axis>& A = plan.tensors[g.a].axes;
      const std::vector<Axis>& B = plan.tensors[g.b].axes;
      std::vector<Axis> sh;
      for (const Axis& a : A)
        if (is_label(a) && std::find(B.begin(), B.end(), a) != B.end()) sh.push_back(a);
      const size_t ns = sh.size();
      size_t ba = 0, bb = 0;
      if (!find_run(A, sh, ba) || !find_run(B, sh, bb)) return bad();
      const SymQ PA = sym_size(A, 0, ns ? ba : 0), QA = sym_size(A, ns ? ba + ns : 0, A.size());
      const SymQ PB = sym_size(B, 0, ns ? bb : 0), QB = sym_size(B, ns ? bb + ns : 0, B.size());
      const bool pb_empty = ns == 0 || bb == 0;
      const bool pa_empty = ns == 0 || ba == 0;
      SymGemm q;
      q.K = sym_size(sh, 0, ns);
      q.M = QA;
      q.N = QB;
      if (pb_empty) {
        q.Z = PA;
        q.sAz = sym_mul(q.K, q.M);
        q.sBz = sym_zero();
      } else {
        if (!pa_empty) return bad();
        q.Z = PB;
        q.sAz = sym_zero();
        q.sBz = sym_mul(q.K, q.N);
      }
      q.sAk = q.M;
      q.sBk = q.N;
      q.sCz = sym_mul(q.M, q.N);
      q.ldc = q.N;
      const int64_t want[10] = {g.Z, g.M, g.N, g.K, g.sAz, g.sAk, g.sBz, g.sBk, g.sCz, g.ldc};
      const SymQ* got[10] = {&q.Z, &q.M, &q.N, &q.K, &q.sAz, &q.sAk, &q.sBz, &q.sBk, &q.sCz, &q.ldc};
      for (int i = 0; i < 10; ++i)
        if (sym_value(*got[i], amax) != want[i]) return bad();
      sp.gemm[si] = q;
    } else {
      PermuteStep& p = s.p;
      const TensorRef& td = plan.tensors[p.dst];
      const std::vector<Axis>& src = plan.tensors[p.src].axes;
      const bool bare_out = td.loc == Loc::Out && td.axes.empty();
      PermuteStep num = p;
      if (!sym_permute(src, bare_out ? all_out : td.axes, sp.perm[si], num, amax)) return bad();
      if (bare_out) {
        // the bit-level final permute becomes an axis-level one; both must
        // send every destination bit to the same source bit
        if (unit_offsets(num) != unit_offsets(p)) return bad();
        p.log2 = num.log2;
        p.sstride = num.sstride;
      } else if (num.log2 != p.log2 || num.sstride != p.sstride) {
        return bad();
      }
    }
  }
  return check_plan_bounds(plan);
}

cq_status check_plan_bounds(const Plan& plan) {
  auto in = [&](int tid, int64_t last) { return last >= 0 && last < plan.tensors[tid].elems; };
  for (const Step& s : plan.steps) {
    if (s.is_gemm) {
      const GemmStep& g = s.g;
      if (g.Z < 1 || g.M < 1 || g.N < 1 || g.K < 1) return fail(CQ_ERR_UNSUPPORTED, "empty GEMM in plan");
      const int64_t la = (g.Z - 1) * g.sAz + (g.K - 1) * g.sAk + (g.M - 1);
      const int64_t lb = (g.Z - 1) * g.sBz + (g.K - 1) * g.sBk + (g.N - 1);
      const int64_t lc = (g.Z - 1) * g.sCz + (g.M - 1) * g.ldc + (g.N - 1);
      if (!in(g.a, la) || !in(g.b, lb) || !in(g.c, lc))
        return fail(CQ_ERR_UNSUPPORTED, "internal: planned GEMM exceeds its tensors");
    } else {
      const PermuteStep& p = s.p;
      int64_t last = 0;
      int bits = 0;
      for (size_t i = 0; i < p.log2.size(); ++i) {
        last += (pow2(p.log2[i]) - 1) * p.sstride[i];
        bits += p.log2[i];
      }
      if (!in(p.src, last) || pow2(bits) != plan.tensors[p.dst].elems)
        return fail(CQ_ERR_UNSUPPORTED, "internal: planned permute exceeds its tensors");
    }
  }
  return CQ_OK;
}

}  // namespace cq

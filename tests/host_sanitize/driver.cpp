// Drives the library's host-only code (validation, planning, cut search,
// batch set-up in abi.cpp, plan.cpp, cutmap.cpp, cutfind.cpp) through the C
// ABI on generated inputs --
// valid and malformed cut maps, plans, workspace queries, masks, cut search
// problems -- for a build with AddressSanitizer and UndefinedBehaviorSanitizer.
// Prints one line per group; any sanitizer report aborts the process.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "cutqc.h"
#include "cutqc_plan.h"

namespace {

std::mt19937_64 rng(20240611);
int uni(int lo, int hi) { return std::uniform_int_distribution<int>(lo, hi)(rng); }

struct Map {
  std::vector<std::vector<int32_t>> init, meas;
  std::vector<cq_subcircuit> subs;
  int K = 0;
  void finish() {
    subs.resize(init.size());
    for (size_t c = 0; c < init.size(); ++c)
      subs[c] = cq_subcircuit{(int32_t)init[c].size(), init[c].data(), meas[c].data()};
  }
};

// A cut map: n_sub subcircuits of random width; each cut joins a measured
// slot of one subcircuit to an initialised slot of another.
Map random_map(int n_sub, int max_width, int max_cuts) {
  Map m;
  m.init.resize(n_sub);
  m.meas.resize(n_sub);
  for (int c = 0; c < n_sub; ++c) {
    const int w = uni(1, max_width);
    m.init[c].assign(w, -1);
    m.meas[c].assign(w, -1);
  }
  const int want = uni(0, max_cuts);
  for (int j = 0; j < want && n_sub > 1; ++j) {
    const int a = uni(0, n_sub - 1);
    int b = uni(0, n_sub - 2);
    if (b >= a) ++b;
    std::vector<int> fa, fb;
    for (int s = 0; s < (int)m.meas[a].size(); ++s)
      if (m.meas[a][s] < 0) fa.push_back(s);
    for (int s = 0; s < (int)m.init[b].size(); ++s)
      if (m.init[b][s] < 0) fb.push_back(s);
    if (fa.empty() || fb.empty()) continue;
    m.meas[a][fa[uni(0, (int)fa.size() - 1)]] = m.K;
    m.init[b][fb[uni(0, (int)fb.size() - 1)]] = m.K;
    ++m.K;
  }
  m.finish();
  return m;
}

// Malformed variants: an id out of range, a duplicated end, a missing end.
void spoil(Map& m) {
  const int c = uni(0, (int)m.init.size() - 1);
  const int s = uni(0, (int)m.init[c].size() - 1);
  switch (uni(0, 4)) {
    case 0: m.init[c][s] = uni(m.K, m.K + 40); break;
    case 1: m.meas[c][s] = -uni(2, 1000); break;
    case 2: m.meas[c][s] = m.K > 0 ? uni(0, m.K - 1) : 7; break;
    case 3: m.init[c][s] = m.K > 0 ? uni(0, m.K - 1) : 3; break;
    default: m.init[c][s] = 1 << 30; break;
  }
  m.finish();
}

int outputs_of(const Map& m, int c) {
  int n = 0;
  for (int32_t v : m.meas[c]) n += v < 0;
  return n;
}

}  // namespace

int main() {
  // status strings, including out-of-range codes
  for (int s = -20; s <= 5; ++s) (void)std::strlen(cq_status_string((cq_status)s));
  (void)cq_last_error();
  int ok = 0, bad = 0;
  std::vector<char> buf(1 << 20);
  // cut maps, plans and workspace queries
  for (int it = 0; it < 1500; ++it) {
    Map m = random_map(uni(1, 6), uni(1, 12), uni(0, 10));
    const bool spoiled = uni(0, 3) == 0;
    if (spoiled) spoil(m);
    const int n_sub = (int)m.subs.size();
    int32_t K = -1, n = -1;
    const cq_status st = cq_validate_cutmap(n_sub, m.subs.data(), &K, &n);
    (st == CQ_OK ? ok : bad)++;
    if (st != CQ_OK) (void)std::strlen(cq_last_error());
    for (int p = 0; p < 6; ++p) {
      size_t ws = 0;
      (void)cq_fd_workspace_size(n_sub, m.subs.data(), (cq_precision)p, nullptr, &ws);
      std::vector<int32_t> perm;
      if (st == CQ_OK && n > 0) {
        for (int i = 0; i < n; ++i) perm.push_back(i);
        std::shuffle(perm.begin(), perm.end(), rng);
        if (uni(0, 4) == 0) perm[uni(0, n - 1)] = uni(-3, n + 3);  // sometimes not a permutation
      }
      (void)cq_fd_workspace_size(n_sub, m.subs.data(), (cq_precision)p, perm.empty() ? nullptr : perm.data(), &ws);
      std::vector<int32_t> bits;
      for (int c = 0; c < n_sub; ++c) bits.push_back(uni(0, outputs_of(m, c) + (uni(0, 9) == 0 ? 3 : 0)));
      size_t need = 0;
      (void)cq_plan_json(n_sub, m.subs.data(), (cq_precision)p, uni(0, 1) ? bits.data() : nullptr,
                         perm.empty() ? nullptr : perm.data(), buf.data(), uni(0, 1) ? buf.size() : 16, &need);
    }
    size_t ab = 0;
    (void)cq_attribute_workspace_size(&m.subs[0], &ab);
    // dynamic definition: masks over each subcircuit's outputs
    if (st == CQ_OK) {
      std::vector<uint64_t> act(n_sub), mer(n_sub), fix(n_sub), fv(n_sub);
      std::vector<int32_t> ma(n_sub);
      std::vector<const double*> ent(n_sub, reinterpret_cast<const double*>(buf.data()));
      for (int c = 0; c < n_sub; ++c) {
        const int nc = outputs_of(m, c);
        for (int b = 0; b < nc; ++b) {
          const int r = uni(0, 2);
          (r == 0 ? act[c] : (r == 1 ? mer[c] : fix[c])) |= 1ull << b;
          if (r == 2 && uni(0, 1)) fv[c] |= 1ull << b;
        }
        if (uni(0, 7) == 0) act[c] |= mer[c] & (~mer[c] + 1);  // sometimes overlapping masks
        ma[c] = uni(-1, 8);
      }
      cq_dd_instance in{n_sub, m.subs.data(), ent.data(), act.data(), mer.data(), fix.data(), fv.data(), ma.data()};
      // a whole call: plans, programs and the batch layout are built on the
      // host before the first copy fails for want of a device (the workspace
      // address is never dereferenced by host code)
      if (it % 50 == 0) {
        cq_dd_params par{(cq_precision)uni(0, 5), uni(1, 6), uni(0, 1)};
        std::vector<cq_dd_record> recs((size_t)par.R);
        int32_t done = 0;
        (void)cq_reconstruct_dd(1, &in, &par, recs.data(), nullptr, &done, buf.data(), buf.size(), nullptr);
        const double* fent[CQ_MAX_SUBCIRCUITS];
        for (int c = 0; c < n_sub; ++c) fent[c] = ent[c];
        (void)cq_reconstruct_fd(n_sub, m.subs.data(), fent, (cq_precision)uni(0, 5), nullptr, buf.data(),
                                buf.data(), buf.size(), nullptr);
      }
      for (int prec = 0; prec < 6; ++prec) {
        cq_dd_params par{(cq_precision)prec, uni(0, 18), uni(0, 1)};
        size_t dw = 0;
        (void)cq_dd_workspace_size(1, &in, &par, uni(0, 1), &dw);
        cq_dd_instance two[2] = {in, in};
        (void)cq_dd_workspace_size(2, two, &par, 0, &dw);
        cq_dd_bfs_params bp{(cq_precision)prec, uni(0, 4), uni(0, 18), 0};
        (void)cq_dd_bfs_workspace_size(&in, &bp, &dw);
      }
    }
  }
  std::printf("cut maps: %d valid, %d rejected\n", ok, bad);
  // entry points with null or inconsistent arguments fail before any launch
  {
    Map m = random_map(2, 6, 3);
    const double* ent[2] = {nullptr, nullptr};
    size_t ws = 0;
    (void)cq_fd_workspace_size(0, nullptr, CQ_FP64, nullptr, &ws);
    (void)cq_fd_workspace_size(2, m.subs.data(), (cq_precision)9, nullptr, &ws);
    (void)cq_reconstruct_fd(2, m.subs.data(), ent, CQ_FP64, nullptr, nullptr, nullptr, 0, nullptr);
    (void)cq_reconstruct_fd(-1, nullptr, nullptr, CQ_FP64, nullptr, nullptr, nullptr, 0, nullptr);
    (void)cq_attribute(nullptr, nullptr, nullptr, nullptr, 0, nullptr);
    (void)cq_reconstruct_dd(0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr);
    cq_dd_params par{CQ_FP64, 4, 0};
    cq_dd_record rec[4];
    int32_t done = 0;
    (void)cq_reconstruct_dd(1, nullptr, &par, rec, nullptr, &done, nullptr, 0, nullptr);
  }
  // cut search on random gate lists
  int found = 0, none = 0;
  for (int it = 0; it < 300; ++it) {
    const int nq = uni(2, 9), ng = nq - 1 + uni(0, 14);
    std::vector<int32_t> gq;
    for (int g = 0; g < ng; ++g) {
      int a, b;
      if (g < nq - 1) {  // a chain first: every qubit takes part
        a = g;
        b = g + 1;
      } else {
        a = uni(0, nq - 1);
        b = uni(0, nq - 2);
        if (b >= a) ++b;
      }
      if (uni(0, 60) == 0) b = a;               // malformed: a gate on one qubit
      if (uni(0, 80) == 0) a = nq + uni(0, 3);  // malformed: out of range
      gq.push_back(a);
      gq.push_back(b);
    }
    cq_cut_problem pr{nq, ng, gq.data(), uni(1, nq + 1), uni(uni(0, 9) == 0 ? 0 : 1, 6)};
    std::vector<int32_t> cl(ng);
    int32_t nsub = 0, ncut = 0;
    double cost = 0;
    (cq_find_cuts(&pr, cl.data(), &nsub, &ncut, &cost) == CQ_OK ? found : none)++;
  }
  (void)cq_find_cuts(nullptr, nullptr, nullptr, nullptr, nullptr);
  std::printf("cut search: %d solved, %d rejected\n", found, none);
  size_t need = 0;
  (void)cq_autotune_json(nullptr, 0, &need);
  (void)cq_autotune_json(buf.data(), buf.size(), &need);
  (void)cq_dd_lanes(3);
  (void)cq_dd_lanes(0);
  std::printf("done\n");
  return 0;
}

// Exact cut search for small circuits (host only).
//
// Section 4.1 models a circuit as a DAG whose vertices are its two-qubit
// gates and whose edges are the qubit wires between them; one-qubit gates do
// not affect where cuts go.  Clustering the vertices into subcircuits cuts
// every wire edge between two clusters.  The search minimises the number of
// floating-point multiplications of Eq. 1's Kronecker products (the
// objective L of Section 4.1) over all clusterings into at most
// max_subcircuits clusters whose subcircuits fit max_width qubits each.
//
// Clusterings are enumerated as restricted-growth strings over the gates in
// circuit order (gate 0 in cluster 0, each later gate in an existing cluster
// or the next new one), labels tried in increasing order, so the first
// minimum found is the lexicographically smallest string.  Branches are cut
// when a subcircuit outgrows max_width (widths never shrink as gates are
// added) or when 4^K alone reaches the best cost.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace cq {
namespace {

struct Search {
  int n_qubits = 0, n_gates = 0, max_width = 0, max_sub = 0;
  std::vector<int> q0, q1;        // gate qubits
  std::vector<int> prev0, prev1;  // previous two-qubit gate on the same qubit, or -1
  std::vector<int> label;         // current partial clustering
  int width[CQ_MAX_SUBCIRCUITS] = {};
  int measured[CQ_MAX_SUBCIRCUITS] = {};
  int cuts = 0;
  double best = INFINITY;
  std::vector<int> best_label;
  int best_sub = 0, best_cuts = 0;
  int64_t visited = 0;

  // Adds one wire end of gate g (qubit's previous gate `p`) to cluster c.
  void add_end(int p, int c, int sign) {
    if (p < 0) {
      width[c] += sign;  // the qubit's first segment starts here
    } else if (label[p] != c) {
      cuts += sign;  // a cut: measured in the earlier cluster, initialised here
      measured[label[p]] += sign;
      width[c] += sign;
    }
  }

  double cost(int n_sub) const {
    if (n_sub <= 1) return 0.0;
    std::vector<int> outs(n_sub);
    for (int c = 0; c < n_sub; ++c) outs[c] = width[c] - measured[c];
    std::sort(outs.begin(), outs.end());
    double sum = 0.0, prod = std::ldexp(1.0, outs[0]);
    for (int c = 1; c < n_sub; ++c) {
      prod *= std::ldexp(1.0, outs[c]);
      sum += prod;
    }
    return std::ldexp(sum, 2 * cuts);
  }

  void dfs(int g, int n_sub) {
    ++visited;
    if (g == n_gates) {
      const double L = cost(n_sub);
      if (L < best) {
        best = L;
        best_label = label;
        best_sub = n_sub;
        best_cuts = cuts;
      }
      return;
    }
    const int top = std::min(n_sub + 1, max_sub);
    for (int c = 0; c < top; ++c) {
      label[g] = c;
      add_end(prev0[g], c, +1);
      add_end(prev1[g], c, +1);
      // widths never shrink and L >= 4^K once two clusters exist
      if (width[c] <= max_width && std::ldexp(1.0, 2 * cuts) < best) dfs(g + 1, std::max(n_sub, c + 1));
      add_end(prev1[g], c, -1);
      add_end(prev0[g], c, -1);
      label[g] = -1;
    }
  }
};

}  // namespace
}  // namespace cq

using namespace cq;

extern "C" cq_status cq_find_cuts(const cq_cut_problem* problem, int32_t* cluster, int32_t* n_subcircuits,
                                  int32_t* n_cuts, double* cost) {
  if (!problem || !cluster || !n_subcircuits || !n_cuts || !cost) return fail(CQ_ERR_ARG, "null argument");
  const cq_cut_problem& P = *problem;
  if (P.n_qubits < 1 || P.n_gates < 1 || !P.gate_qubits) return fail(CQ_ERR_ARG, "empty circuit");
  if (P.n_gates > CQ_MAX_FIND_GATES) return fail(CQ_ERR_SHAPE, "too many two-qubit gates for the exact search");
  if (P.max_subcircuits < 1 || P.max_subcircuits > CQ_MAX_SUBCIRCUITS)
    return fail(CQ_ERR_ARG, "max_subcircuits out of range");
  if (P.max_width < 1) return fail(CQ_ERR_ARG, "max_width must be positive");
  Search S;
  S.n_qubits = P.n_qubits;
  S.n_gates = P.n_gates;
  S.max_width = P.max_width;
  S.max_sub = P.max_subcircuits;
  std::vector<int> last(P.n_qubits, -1);
  for (int g = 0; g < P.n_gates; ++g) {
    const int a = P.gate_qubits[2 * g], b = P.gate_qubits[2 * g + 1];
    if (a < 0 || a >= P.n_qubits || b < 0 || b >= P.n_qubits || a == b)
      return fail(CQ_ERR_ARG, "gate qubits out of range or equal");
    S.q0.push_back(a);
    S.q1.push_back(b);
    S.prev0.push_back(last[a]);
    S.prev1.push_back(last[b]);
    last[a] = last[b] = g;
  }
  for (int q = 0; q < P.n_qubits; ++q)
    if (last[q] < 0) return fail(CQ_ERR_ARG, "a qubit takes part in no two-qubit gate");
  S.label.assign(P.n_gates, -1);
  S.dfs(0, 0);
  if (!std::isfinite(S.best)) return fail(CQ_ERR_SHAPE, "no clustering fits max_width and max_subcircuits");
  for (int g = 0; g < P.n_gates; ++g) cluster[g] = S.best_label[g];
  *n_subcircuits = S.best_sub;
  *n_cuts = S.best_cuts;
  *cost = S.best;
  return CQ_OK;
}

// Cut-map validation and the facts derived from it (Section 3.1: K cuts
// split the circuit into subcircuits; every cut has one measured upstream end
// and one initialised downstream end).
#include <algorithm>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace cq {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

cq_status fail(cq_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

const char* last_error_cstr() { return g_last_error.c_str(); }

cq_status build_subinfo(const cq_subcircuit* sub, SubInfo& si) {
  if (!sub) return fail(CQ_ERR_ARG, "null subcircuit");
  if (sub->width < 0 || sub->width > CQ_MAX_WIDTH)
    return fail(CQ_ERR_SHAPE, "subcircuit width out of range");
  if (sub->width > 0 && (!sub->init_cut || !sub->meas_cut))
    return fail(CQ_ERR_ARG, "null init_cut/meas_cut");
  si = SubInfo();
  si.width = sub->width;
  for (int s = 0; s < sub->width; ++s) {
    int ic = sub->init_cut[s], mc = sub->meas_cut[s];
    if (ic < -1 || mc < -1 || ic >= CQ_MAX_CUTS || mc >= CQ_MAX_CUTS)
      return fail(CQ_ERR_CUTMAP, "cut id out of range");
    si.init_cut.push_back(ic);
    si.meas_cut.push_back(mc);
    if (mc == -1) si.outputs.push_back(s);
    if (ic != -1) si.init_slots.push_back(s);
    if (mc != -1) si.meas_slots.push_back(s);
    if (ic != -1) si.cuts.push_back(ic);
    if (mc != -1) si.cuts.push_back(mc);
  }
  std::sort(si.cuts.begin(), si.cuts.end());
  for (size_t i = 1; i < si.cuts.size(); ++i)
    if (si.cuts[i] == si.cuts[i - 1])
      return fail(CQ_ERR_CUTMAP, "a cut has both ends in one subcircuit, or appears twice");
  if (si.k() > CQ_MAX_LOCAL_CUTS) return fail(CQ_ERR_SHAPE, "subcircuit touches too many cuts");
  return CQ_OK;
}

cq_status build_cutmap(int32_t n_sub, const cq_subcircuit* subs, CutMap& cm) {
  if (n_sub < 1 || n_sub > CQ_MAX_SUBCIRCUITS) return fail(CQ_ERR_ARG, "n_sub out of range");
  if (!subs) return fail(CQ_ERR_ARG, "null subcircuit array");
  cm = CutMap();
  cm.n_sub = n_sub;
  int max_id = -1;
  for (int c = 0; c < n_sub; ++c) {
    SubInfo si;
    cq_status st = build_subinfo(&subs[c], si);
    if (st != CQ_OK) return st;
    for (int id : si.cuts) max_id = std::max(max_id, id);
    cm.n_total += si.n();
    cm.subs.push_back(std::move(si));
  }
  cm.K = max_id + 1;
  cm.up.assign(cm.K, -1);
  cm.down.assign(cm.K, -1);
  for (int c = 0; c < n_sub; ++c) {
    const SubInfo& si = cm.subs[c];
    for (int s = 0; s < si.width; ++s) {
      int ic = si.init_cut[s], mc = si.meas_cut[s];
      if (ic != -1) {
        if (cm.down[ic] != -1) return fail(CQ_ERR_CUTMAP, "cut initialised twice");
        cm.down[ic] = c;
      }
      if (mc != -1) {
        if (cm.up[mc] != -1) return fail(CQ_ERR_CUTMAP, "cut measured twice");
        cm.up[mc] = c;
      }
    }
  }
  for (int j = 0; j < cm.K; ++j) {
    if (cm.up[j] == -1 || cm.down[j] == -1)
      return fail(CQ_ERR_CUTMAP, "cut id " + std::to_string(j) + " lacks an end");
    if (cm.up[j] == cm.down[j]) return fail(CQ_ERR_CUTMAP, "cut joins a subcircuit to itself");
  }
  return CQ_OK;
}

}  // namespace cq

extern "C" const char* cq_last_error(void) { return cq::last_error_cstr(); }

extern "C" const char* cq_status_string(cq_status s) {
  switch (s) {
    case CQ_OK: return "CQ_OK";
    case CQ_ERR_ARG: return "CQ_ERR_ARG";
    case CQ_ERR_SHAPE: return "CQ_ERR_SHAPE";
    case CQ_ERR_CUTMAP: return "CQ_ERR_CUTMAP";
    case CQ_ERR_MASK: return "CQ_ERR_MASK";
    case CQ_ERR_WORKSPACE: return "CQ_ERR_WORKSPACE";
    case CQ_ERR_UNSUPPORTED: return "CQ_ERR_UNSUPPORTED";
    case CQ_ERR_HIP: return "CQ_ERR_HIP";
  }
  return "CQ_ERR_UNKNOWN";
}

extern "C" cq_status cq_validate_cutmap(int32_t n_sub, const cq_subcircuit* subs,
                                        int32_t* n_cuts, int32_t* n_outputs) {
  cq::CutMap cm;
  cq_status st = cq::build_cutmap(n_sub, subs, cm);
  if (st != CQ_OK) return st;
  if (n_cuts) *n_cuts = cm.K;
  if (n_outputs) *n_outputs = cm.n_total;
  return CQ_OK;
}

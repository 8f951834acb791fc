// Device launchers replaced for a host-only build of the library's host code
// (validation, planning, cut search, batch set-up): every launch reports that
// there is no device, so calls run their host logic and then take their
// error paths.  Signatures follow csrc/kernels.hpp.
#include "kernels.hpp"

namespace cq {

hipError_t launch_gemm(cq_precision, const GemmLaunch&, hipStream_t) { return hipErrorNoDevice; }
void autotune_set(int) {}
std::string autotune_json() { return "[]"; }
bool autotune_load(const char*) { return false; }
bool autotune_save(const char*) { return false; }
hipError_t launch_prep(const double*, void*, int64_t, DType, bool, hipStream_t, const int32_t*, int) {
  return hipErrorNoDevice;
}
hipError_t launch_colmax(const double*, int64_t, int, uint64_t*, hipStream_t, const int32_t*) {
  return hipErrorNoDevice;
}
hipError_t launch_expsum(const ExpSumLaunch&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_rowmax(const double*, int64_t, int, uint64_t*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_balance(const BalanceLaunch&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_prep_scaled(const double*, void*, int64_t, int, const uint64_t*, DType, bool, hipStream_t,
                              const int32_t*) {
  return hipErrorNoDevice;
}
hipError_t launch_permute(const PermLaunch&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_attribute(const AttrLaunch&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_dd_copy(const void*, int64_t, void*, int64_t, int64_t, int, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_dd_init(const DDProgram*, DDState*, cq_dd_record*, int, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_dd_setup(const DDProgram*, DDState*, DDLevel*, cq_dd_record*, int, void*, hipStream_t,
                           InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_dd_balance(const DDProgram*, const DDLevel*, int, int64_t, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_dd_colmax(const DDProgram*, const DDLevel*, int, int64_t, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_dd_expsum(const DDProgram*, const DDState*, const DDLevel*, int, int64_t, int64_t, hipStream_t,
                            InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_dd_update(const DDProgram*, DDState*, cq_dd_record*, int, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_warm_tau(const double*, unsigned long long*, const int32_t*, unsigned long long*, hipStream_t,
                           InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_tile_bounds(const GemmArgs*, DType, bool, float*, float*, float*, int64_t, int64_t, int64_t,
                              hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_tile_warm(const float*, const int64_t*, const int64_t*, uint64_t*, int, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_tile_compact(const float*, const int64_t*, const unsigned long long*, uint64_t*, int64_t*,
                               int64_t, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_gemm_indirect(cq_precision, const GemmArgs*, int64_t, DType, bool, bool, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_prep_indirect(const PrepArgs*, int, DType, bool, int64_t, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_permute_indirect(const PermArgs*, DType, DType, bool, int64_t, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
hipError_t launch_merge_indirect(const MergeArgs*, int, int64_t, hipStream_t, InstSpan) { return hipErrorNoDevice; }
hipError_t launch_refine_indirect(const RefineArgs*, int, hipStream_t, InstSpan) { return hipErrorNoDevice; }
hipError_t launch_topk_indirect(const void*, DType, const int64_t*, const int32_t*, int, int64_t, double*,
                                uint64_t*, int64_t, double*, uint64_t*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_topk_candidates(const double*, const uint64_t*, const int64_t*, const int32_t*, int, double*,
                                  uint64_t*, double*, uint64_t*, hipStream_t, InstSpan) {
  return hipErrorNoDevice;
}
int64_t topk_indirect_capacity(int64_t max_count, int C_max) { return ((max_count + 8191) / 8192) * C_max; }

}  // namespace cq

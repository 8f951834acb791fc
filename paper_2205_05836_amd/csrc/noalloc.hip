// Full definition without any allocation: the workspace is a fixed array in
// device memory that the library owns, for callers that cannot allocate
// (code under stream capture, tight serving loops, harnesses that forbid
// allocation).  Every launch and kernel is the one cq_reconstruct_fd issues;
// only the workspace pointer differs.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"

namespace cq {
namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[CQ_FD_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call on each device).
cq_status scratch_on_current_device(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CQ_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(CQ_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CQ_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return CQ_OK;
}

}  // namespace
}  // namespace cq

extern "C" cq_status cq_reconstruct_fd_noalloc(int32_t n_sub, const cq_subcircuit* subs,
                                               const double* const* entries, cq_precision prec,
                                               const int32_t* out_perm, void* out,
                                               hipStream_t stream) {
  size_t need = 0;
  cq_status st = cq_fd_workspace_size(n_sub, subs, prec, out_perm, &need);
  if (st != CQ_OK) return st;
  if (need > (size_t)CQ_FD_NOALLOC_SCRATCH_BYTES)
    return cq::fail(CQ_ERR_WORKSPACE,
                    "this reconstruction needs " + std::to_string(need) +
                        " bytes of workspace; the fixed scratch of cq_reconstruct_fd_noalloc holds " +
                        std::to_string((size_t)CQ_FD_NOALLOC_SCRATCH_BYTES) +
                        " (use cq_reconstruct_fd with a caller workspace)");
  void* ws = nullptr;
  st = cq::scratch_on_current_device(&ws);
  if (st != CQ_OK) return st;
  return cq::fd_run(n_sub, subs, entries, prec, out_perm, out, ws, CQ_FD_NOALLOC_SCRATCH_BYTES, true,
                    stream);
}

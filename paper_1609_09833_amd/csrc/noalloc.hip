// bias_force_noalloc: bias_force for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc). The split and chained launch shapes need a workspace
// (CV state, cached CV-list entries, chunk sums, the chained launch's arrival
// counters); here it is a file-scope device array of fixed size instead of
// the context's grow-on-demand buffer, so the call allocates nothing.
//
// Each GPU holds its own copy of the array from the first abp_create on it
// until the process ends. Host code never passes the array's name to a
// kernel: abp_create, once per device with that device current, takes its
// device address with hipGetSymbolAddress and keeps it per device; every call
// uses that address. All calls on one GPU share the array (and the context's
// calls that overlap on one GPU race on it). Its first kForceArrivedBytes
// hold the chained launch's counters, which are zeroed at set-up and which
// every chained launch leaves at zero; everything else a call reads it has
// written first.
#include <mutex>
#include <string>

#include "abp_serve_internal.h"

namespace abp {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Called by abp_create with `device` current.
abp_status noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return set_error(ABP_E_INVAL, "device index too large");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return ABP_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(ABP_E_DEVICE, (std::string("hipGetSymbolAddress of the static workspace: ") +
                                    hipGetErrorString(e)).c_str());
  if (hipMemset(p, 0, kForceArrivedBytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return set_error(ABP_E_DEVICE, "cannot clear the static workspace's counters");
  g_ptr[device] = p;
  return ABP_OK;
}

}  // namespace abp

extern "C" abp_status bias_force_noalloc(abp_ctx* ctx, abp_eval_mode mode, abp_prec prec, const abp_cv_desc* cv,
                                         const abp_walkers* walkers, const int64_t* n_visible,
                                         const int64_t* deposit_slot, const double* deposit_height, double* s,
                                         double* V, double* dVds, abp_stream stream) {
  abp::ForceCall call;
  abp_status st = abp::prepare_force(ctx, mode, prec, cv, walkers, n_visible, deposit_slot, deposit_height, s, V,
                                     dVds, &call);
  if (st != ABP_OK || call.nothing) return st;
  if (call.workspace_bytes > abp::kScratchBytes) {
    const std::string msg = "bias_force_noalloc needs " + std::to_string(call.workspace_bytes) +
                            " bytes of workspace; its static workspace holds " +
                            std::to_string(abp::kScratchBytes) + " (use fewer walkers per call, or bias_force)";
    return abp::set_error(ABP_E_NOMEM, msg.c_str());
  }
  void* ptr;
  {
    std::lock_guard<std::mutex> lk(abp::g_mu);
    ptr = call.device >= 0 && call.device < abp::kMaxDevices ? abp::g_ptr[call.device] : nullptr;
  }
  if (!ptr) return abp::set_error(ABP_E_DEVICE, "static workspace not set up on the context's device");
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != call.device && hipSetDevice(call.device) != hipSuccess)
    return abp::set_error(ABP_E_DEVICE, "cannot select the context's device");
  const hipError_t e = abp::launch_bias_force(call.K, call.H, call.A, ptr, (hipStream_t)stream);
  if (prev >= 0 && prev != call.device) (void)hipSetDevice(prev);
  if (e != hipSuccess)
    return abp::set_error(ABP_E_DEVICE, (std::string("bias_force_noalloc launch: ") + hipGetErrorString(e)).c_str());
  return abp::set_error(ABP_OK, "");
}

// Device side of the serving loop: the per-batch copies between a request's
// host staging and the walker's resident device state.
//
// A request carries the positions of its walker's CV atoms for one MD step
// (the per-step exchange of section "Minimization of Interprocess
// Communications": only CV atoms travel) in pinned, mapped host memory. The
// stage launch copies them into the walker's range of the device pool,
// clears the forces there, and stores the masses of a walker admitted for
// this batch (staged in the batch descriptor). The bias-force launches then
// run on the pool like any bias_force call. The gather launch copies the
// forces of the CV atoms back to the request's host staging, where the
// caller's poll picks them up.
#include "abp_serve_internal.h"

namespace abp {
namespace {

constexpr int kServeBlock = 256;

__global__ __launch_bounds__(kServeBlock) void k_serve_stage(const ServeArgs A) {
  const int j = blockIdx.x;
  const int64_t p = A.pool_off[j];
  const int n = A.n_cv[j];
  const float* r = A.arena + A.arena_off[j];    // x[n], y[n], z[n] of this request
  const int64_t soff = A.stage_off[j];
  for (int i = threadIdx.x; i < n; i += kServeBlock) {
    const float x = r[i], y = r[n + i], z = r[2 * n + i];
    A.x[p + i] = x;
    A.y[p + i] = y;
    A.z[p + i] = z;
    A.fx[p + i] = 0.0f;
    A.fy[p + i] = 0.0f;
    A.fz[p + i] = 0.0f;
    if (soff >= 0) A.mass[p + i] = A.stage_mass[soff + i];
  }
}

__global__ __launch_bounds__(kServeBlock) void k_serve_gather(const ServeArgs A) {
  const int j = blockIdx.x;
  const int64_t p = A.pool_off[j];
  const int n = A.n_cv[j];
  float* r = A.arena + A.arena_off[j] + 3 * (int64_t)n;   // fx[n], fy[n], fz[n] of this request
  for (int i = threadIdx.x; i < n; i += kServeBlock) {
    r[i] = A.fx[p + i];
    r[n + i] = A.fy[p + i];
    r[2 * n + i] = A.fz[p + i];
  }
}

}  // namespace

hipError_t launch_serve_stage(const ServeArgs& A, hipStream_t stream) {
  if (A.nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_stage, dim3((unsigned)A.nb), dim3(kServeBlock), 0, stream, A);
  return hipGetLastError();
}

hipError_t launch_serve_gather(const ServeArgs& A, hipStream_t stream) {
  if (A.nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_gather, dim3((unsigned)A.nb), dim3(kServeBlock), 0, stream, A);
  return hipGetLastError();
}

}  // namespace abp

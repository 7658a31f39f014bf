// Internal declarations of the serving loop (host scheduler and the device
// copies between request staging and the walker pool).
#pragma once

#include "abp_internal.h"

namespace abp {

// One batch of the serving loop: request j of nb belongs to a walker whose
// n_cv[j] CV atoms sit at pool_off[j] of the device pool.
struct ServeArgs {
  int64_t nb;
  const int64_t* pool_off;     // [nb] walker's first pool entry
  const int64_t* arena_off;    // [nb] request's first float in the mapped host staging
  const int64_t* stage_off;    // [nb] first staged mass of a walker admitted for this batch, else -1
  const int32_t* n_cv;         // [nb]
  const float* stage_mass;     // staged masses (batch descriptor, device copy)
  float* arena;                // mapped host staging (device view): per request x, y, z, fx, fy, fz blocks
  float* x;                    // device pool arrays
  float* y;
  float* z;
  float* mass;
  float* fx;
  float* fy;
  float* fz;
};

hipError_t launch_serve_stage(const ServeArgs& A, hipStream_t stream);
hipError_t launch_serve_gather(const ServeArgs& A, hipStream_t stream);

// The context pieces the server needs (defined by the host layer).
struct CtxView {
  Consts K;
  HistView H;
  int32_t* err;
  int device;
};
CtxView ctx_view(abp_ctx* ctx);
int64_t ctx_reserved(const abp_ctx* ctx);
// Grows the context's grid-deposit scratch for commits of up to n hills, so
// that later commits allocate nothing.
abp_status ctx_reserve_commit(abp_ctx* ctx, int64_t n);
// Sets the calling thread's last-error message (read by abp_last_error).
abp_status set_error(abp_status st, const char* msg);

}  // namespace abp

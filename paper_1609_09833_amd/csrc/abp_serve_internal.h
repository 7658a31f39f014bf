// Internal declarations of the serving loop's host scheduler.
#pragma once

#include "abp_internal.h"

namespace abp {

// The context pieces the server needs (defined by the host layer).
struct CtxView {
  Consts K;
  HistView H;
  double* grid;                    // the FP64 node arrays, or NULL
  float* grid32;                   // their FP32 mirror
  size_t grid_doubles;             // doubles in `grid`
  int32_t* err;
  int device;
};
CtxView ctx_view(abp_ctx* ctx);
int64_t ctx_reserved(const abp_ctx* ctx);
// Grows the context's grid-deposit scratch for commits of up to n hills, so
// that later commits allocate nothing.
abp_status ctx_reserve_commit(abp_ctx* ctx, int64_t n);
// Marks hills up to `upto` (reserved, written) committed without adding them
// to the context's grid; the caller adds them to its grid buffers with
// ctx_grid_add (the context's own arrays included) in commit order.
abp_status ctx_commit_hills(abp_ctx* ctx, int64_t upto);
// Adds committed hills [k0, k1) to the node arrays `grid` on `stream` and
// refreshes the FP32 mirror `grid32` when it is not NULL.
abp_status ctx_grid_add(abp_ctx* ctx, double* grid, float* grid32, int64_t k0, int64_t k1, hipStream_t stream);
// A validated bias_force call: its kernel arguments and the workspace bytes
// its launch shape needs (0: none). nothing: no walkers, return ABP_OK.
struct ForceCall {
  ForceArgs A;
  Consts K;
  HistView H;
  int device = 0;
  size_t workspace_bytes = 0;
  bool nothing = true;
};
abp_status prepare_force(abp_ctx* ctx, abp_eval_mode mode, abp_prec prec, const abp_cv_desc* cv,
                         const abp_walkers* walkers, const int64_t* n_visible, const int64_t* deposit_slot,
                         const double* deposit_height, double* s, double* V, double* dVds, ForceCall* out);
// bias_force_noalloc's static workspace: its device address on `device`
// (current), taken once per device; its size.
abp_status noalloc_setup(int device);
size_t noalloc_scratch_bytes();
// Sets the calling thread's last-error message (read by abp_last_error).
abp_status set_error(abp_status st, const char* msg);

}  // namespace abp

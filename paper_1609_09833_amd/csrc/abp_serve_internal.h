// Internal declarations of the serving loop's host scheduler.
#pragma once

#include "abp_internal.h"

namespace abp {

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

// Internal declarations of the serving loop (host scheduler and device engine step).
#pragma once

#include "abp_internal.h"

namespace abp {

struct EngineArgs {
  int64_t nb;                  // requests in the batch
  const int64_t* atom_base;    // [nb] device offset of the walker's atoms in the pools
  const int32_t* n_atoms;      // [nb]
  const int64_t* stage_off;    // [nb] first staged entry of a walker admitted for this batch, else -1
  const float4* stage;         // staged (x0, y0, z0, mass) of those walkers' CV entries, in list order
  const int32_t* walker;       // [nb] walker id (hash input)
  const int64_t* step;         // [nb] MD step (hash input)
  int32_t nlists;              // 2 * ncv
  const int32_t* list_beg;     // [nlists][nb] into list_idx
  const int32_t* list_len;     // [nlists][nb]
  const int32_t* list_idx;     // device list pool
  float amplitude;             // nm; positions move by at most this much from x0
  float* x;                    // device pools
  float* y;
  float* z;
  float* mass;
  float* fx;
  float* fy;
  float* fz;
  float* x0;                   // device pools: base positions of resident walkers' CV atoms
  float* y0;
  float* z0;
};

hipError_t launch_engine_step(const EngineArgs& E, hipStream_t stream);

// The context pieces the server needs (defined by the host layer).
struct CtxView {
  Consts K;
  HistView H;
  int32_t* err;
  int device;
};
CtxView ctx_view(abp_ctx* ctx);
int64_t ctx_reserved(const abp_ctx* ctx);
// Sets the calling thread's last-error message (read by abp_last_error).
abp_status set_error(abp_status st, const char* msg);

}  // namespace abp

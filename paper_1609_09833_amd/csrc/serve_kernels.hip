// Device side of the serving loop: the synthetic engine step that prepares
// each batched walker before its bias-force evaluation.
//
// For every request of a batch: if its walker was just admitted, copy the
// walker's masses from mapped host memory into the device pool and zero its
// force arrays; then write the positions of its CV atoms for this step and
// clear their forces (the bias force is added to them afterwards),
//   x = x0 + amplitude * u(walker, step, atom, coordinate),
// where x0 is read from mapped host memory and u in [-1, 1) comes from an
// integer hash (the "lowbias32" mixer, C. Wellons, 2018). The arithmetic uses
// explicitly rounded float operations so a host can reproduce the positions
// bit for bit. This stands in for an MD engine; it is not part of the method.
#include "abp_serve_internal.h"

namespace abp {
namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  h *= 0x846ca68bu;
  h ^= h >> 16;
  return h;
}

// u in [-1, 1), a multiple of 2^-15 (exact in float).
__device__ __forceinline__ float unit_hash(uint32_t w, uint32_t step, uint32_t atom, uint32_t coord) {
  const uint32_t h = mix32(w * 0x9e3779b1u ^ mix32(step * 0x85ebca77u ^ mix32(atom * 0xc2b2ae3du + coord)));
  return (float)(int32_t)((h >> 16) & 0xffffu) * (1.0f / 32768.0f) - 1.0f;
}

__global__ __launch_bounds__(kBlock) void k_engine_step(const EngineArgs E) {
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t base = E.atom_base[j];
  const int32_t n = E.n_atoms[j];
  const int64_t hbase = E.host_base[j];
  if (E.fresh[j]) {
    for (int i = tid; i < n; i += kBlock) {
      E.mass[base + i] = E.h_mass[hbase + i];
      E.fx[base + i] = 0.0f;
      E.fy[base + i] = 0.0f;
      E.fz[base + i] = 0.0f;
    }
  }
  const uint32_t w = (uint32_t)E.walker[j];
  const uint32_t st = (uint32_t)E.step[j];
  for (int q = 0; q < E.nlists; ++q) {
    const int b = E.list_beg[(int64_t)q * E.nb + j];
    const int len = E.list_len[(int64_t)q * E.nb + j];
    for (int e = tid; e < len; e += kBlock) {
      const int32_t i = E.list_idx[b + e];
      if (i < 0 || i >= n) continue;                 // the bias kernels flag it
      const int64_t g = base + i;
      const int64_t hg = hbase + i;
      E.x[g] = __fadd_rn(E.h_x0[hg], __fmul_rn(E.amplitude, unit_hash(w, st, (uint32_t)i, 0u)));
      E.y[g] = __fadd_rn(E.h_y0[hg], __fmul_rn(E.amplitude, unit_hash(w, st, (uint32_t)i, 1u)));
      E.z[g] = __fadd_rn(E.h_z0[hg], __fmul_rn(E.amplitude, unit_hash(w, st, (uint32_t)i, 2u)));
      E.fx[g] = 0.0f;
      E.fy[g] = 0.0f;
      E.fz[g] = 0.0f;
    }
  }
}

}  // namespace

hipError_t launch_engine_step(const EngineArgs& E, hipStream_t stream) {
  if (E.nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_engine_step, dim3((unsigned)E.nb), dim3(kBlock), 0, stream, E);
  return hipGetLastError();
}

}  // namespace abp

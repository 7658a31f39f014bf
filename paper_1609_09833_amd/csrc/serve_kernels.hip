// Device side of the serving loop: the synthetic engine step that prepares
// each batched walker before its bias-force evaluation.
//
// For every request of a batch: write the positions of its walker's CV atoms
// for this step and clear their forces (the bias force is added to them
// afterwards),
//   x = x0 + amplitude * u(walker, step, atom, coordinate),
// where u in [-1, 1) comes from an integer hash (the "lowbias32" mixer,
// C. Wellons, 2018). The base positions x0 are the walker's resident state:
// when the walker was just admitted, the host has staged them and the masses
// of its CV atoms in the batch descriptor (one copy for the batch), and they
// are stored into the device pool; later steps read them from there. The
// arithmetic uses explicitly rounded float operations so a host can
// reproduce the positions bit for bit. This stands in for an MD engine; it is
// not part of the method.
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

constexpr int kInFlight = 16;   // entries each thread handles per pass (their loads overlap)

__global__ __launch_bounds__(kBlock) void k_engine_step(const EngineArgs E) {
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t base = E.atom_base[j];
  const int32_t n = E.n_atoms[j];
  const int64_t soff = E.stage_off[j];
  const bool fresh = soff >= 0;
  const uint32_t w = (uint32_t)E.walker[j];
  const uint32_t st = (uint32_t)E.step[j];
  // CV atoms of all lists, flattened: entry r of list q sits at r - start[q].
  int start[7];
  start[0] = 0;
  for (int q = 0; q < E.nlists; ++q) start[q + 1] = start[q] + E.list_len[(int64_t)q * E.nb + j];
  const int total = start[E.nlists];
  for (int r0 = 0; r0 < total; r0 += kBlock * kInFlight) {
    int32_t atom[kInFlight];
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) {
      const int r = r0 + u * kBlock + tid;
      atom[u] = -1;
      if (r < total) {
        int q = 0;
        while (q + 1 < E.nlists && r >= start[q + 1]) ++q;
        const int32_t i = E.list_idx[E.list_beg[(int64_t)q * E.nb + j] + (r - start[q])];
        atom[u] = (i >= 0 && i < n) ? i : -1;        // the bias kernels flag a bad index
      }
    }
    float px[kInFlight], py[kInFlight], pz[kInFlight], pm[kInFlight];
    if (fresh) {                                    // uniform per block
#pragma unroll
      for (int u = 0; u < kInFlight; ++u) {
        const int r = r0 + u * kBlock + tid;
        const float4 v = E.stage[soff + (r < total ? r : 0)];   // entry 0 stands in: always staged
        px[u] = v.x;
        py[u] = v.y;
        pz[u] = v.z;
        pm[u] = v.w;
      }
    } else {
#pragma unroll
      for (int u = 0; u < kInFlight; ++u) {
        const int64_t g = base + (atom[u] < 0 ? 0 : atom[u]);
        px[u] = E.x0[g];
        py[u] = E.y0[g];
        pz[u] = E.z0[g];
        pm[u] = 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) {
      if (atom[u] < 0) continue;
      const int64_t g = base + atom[u];
      const uint32_t a = (uint32_t)atom[u];
      if (fresh) {
        E.x0[g] = px[u];
        E.y0[g] = py[u];
        E.z0[g] = pz[u];
        E.mass[g] = pm[u];
      }
      E.x[g] = __fadd_rn(px[u], __fmul_rn(E.amplitude, unit_hash(w, st, a, 0u)));
      E.y[g] = __fadd_rn(py[u], __fmul_rn(E.amplitude, unit_hash(w, st, a, 1u)));
      E.z[g] = __fadd_rn(pz[u], __fmul_rn(E.amplitude, unit_hash(w, st, a, 2u)));
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

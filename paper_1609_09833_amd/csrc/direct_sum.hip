// Direct hill sum (bias_eval, mode DIRECT): host-side dispatch and the FP64
// kernels. The FP32 kernels live in direct_sum_d1/d2/d3.hip (one translation
// unit per dimension, built in parallel); their design is described in
// direct_sum_impl.h.
#include "direct_sum_impl.h"

namespace abp {
namespace {

template <int D, int KERN>
__global__ __launch_bounds__(kBlock) void k_direct_f64(const DirectArgs A) {
  __shared__ double4 tile[kTile64];
  const int64_t iq0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t iq = iq0 < A.nq ? iq0 : A.nq - 1;
  double tq[D], P[D + 1];
#pragma unroll
  for (int i = 0; i < D; ++i) tq[i] = work64(A.K, i, eval_coord(A.K, i, load_q(A, i, iq)));
#pragma unroll
  for (int r = 0; r <= D; ++r) P[r] = 0.0;
  for (int64_t t0 = 0; t0 < A.nvis; t0 += kTile64) {
    const int n = (int)(A.nvis - t0 < kTile64 ? A.nvis - t0 : kTile64);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kBlock) {
      const int64_t k = t0 + i;
      double4 r;
      r.x = work64(A.K, 0, A.c64[k]);
      r.y = D > 1 ? work64(A.K, 1, A.c64[A.capacity + k]) : 0.0;
      r.z = D > 2 ? work64(A.K, 2, A.c64[2 * A.capacity + k]) : 0.0;
      r.w = A.w64[k];
      tile[i] = r;
    }
    __syncthreads();
    for (int c = 0; c < n; ++c) pair64<D, KERN>(A.K, tq, tile[c], P);
  }
  double dh[D], V, dV[D];
#pragma unroll
  for (int i = 0; i < D; ++i) dh[i] = P[i + 1] * A.K.gs64[i];
  apply_transform<D>(A.K, P[0], dh, V, dV);
  if (iq0 < A.nq) store_out<D>(A, iq0, V, dV);
}

template <int D, int KERN>
hipError_t go_f64(const DirectArgs& A, hipStream_t stream) {
  const int64_t blocks = (A.nq + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_direct_f64<D, KERN>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, A);
  return hipGetLastError();
}

template <int D>
hipError_t dispatch_f64(const DirectArgs& A, hipStream_t stream) {
  return A.K.kernel == ABP_K_GAUSS ? go_f64<D, ABP_K_GAUSS>(A, stream) : go_f64<D, ABP_K_COMPACT>(A, stream);
}

}  // namespace

hipError_t launch_direct_sum(const Consts& K, const HistView& H, int64_t n_visible, abp_prec prec,
                             int64_t nq, int q_f64, const void* q, void* V, void* dVds,
                             hipStream_t stream) {
  if (nq <= 0) return hipSuccess;
  DirectArgs A;
  A.K = K;
  A.rec32 = H.rec32;
  A.c64 = H.c64;
  A.w64 = H.w64;
  A.capacity = H.capacity;
  A.nvis = n_visible;
  A.nq = nq;
  A.q = q;
  A.V = V;
  A.dV = dVds;
  A.q_f64 = q_f64;
  int mask = 0;
  bool iso = K.kernel == ABP_K_GAUSS;
  for (int i = 0; i < K.ndim; ++i) {
    mask |= (K.periodic[i] ? 1 : 0) << i;
    iso = iso && K.kf32[i] == K.kf32[0];
  }
  if (prec == ABP_PREC_FP64) {
    switch (K.ndim) {
      case 1: return dispatch_f64<1>(A, stream);
      case 2: return dispatch_f64<2>(A, stream);
      case 3: return dispatch_f64<3>(A, stream);
      default: return hipErrorInvalidValue;
    }
  }
  const bool kahan = prec == ABP_PREC_FP32_KAHAN;
  switch (K.ndim) {
    case 1: return dispatch_f32_d1(A, mask, iso, kahan, stream);
    case 2: return dispatch_f32_d2(A, mask, iso, kahan, stream);
    case 3: return dispatch_f32_d3(A, mask, iso, kahan, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace abp

// Direct hill sum (bias_eval, mode DIRECT): host-side dispatch and the FP64
// kernels. The FP32 kernels live in direct_sum_d1/d2/d3.hip (one translation
// unit per dimension, built in parallel); their design is described in
// direct_sum_impl.h.
#include "direct_sum_impl.h"

namespace abp {
namespace {

template <int D, int PMASK, int KERN, bool ISO>
__global__ __launch_bounds__(kBlock) void k_direct_f64(const DirectArgs A) {
  __shared__ double4 tile[kTile64];
  const int64_t iq0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t iq = iq0 < A.nq ? iq0 : A.nq - 1;
  double tq[D], P[D + 1];
  bool finite = true;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double x = load_q(A, i, iq);
    finite = finite && isfinite(x);
    tq[i] = work64(A.K, i, eval_coord(A.K, i, isfinite(x) ? x : A.K.lo[i]));
  }
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
      r.w = A.l64[k];
      tile[i] = r;
    }
    __syncthreads();
    for (int c = 0; c < n; ++c) pair64<D, PMASK, KERN, ISO>(A.K, tq, tile[c], P);
  }
  double dh[D], V, dV[D];
#pragma unroll
  for (int i = 0; i < D; ++i) dh[i] = P[i + 1] * A.K.gs64[i];
  apply_transform<D>(A.K, P[0], dh, V, dV);
  if (!finite) {                       // a non-finite query coordinate gives NaN outputs
    V = __builtin_nan("");
#pragma unroll
    for (int i = 0; i < D; ++i) dV[i] = V;
  }
  if (iq0 < A.nq) store_out<D>(A, iq0, V, dV);
}

template <int D, int PMASK, int KERN, bool ISO>
hipError_t go_f64(const DirectArgs& A, hipStream_t stream) {
  const int64_t blocks = (A.nq + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_direct_f64<D, PMASK, KERN, ISO>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, A);
  return hipGetLastError();
}

template <int D, int PMASK>
hipError_t dispatch_f64_mask(const DirectArgs& A, bool iso, hipStream_t stream) {
  if (A.K.kernel != ABP_K_GAUSS) return go_f64<D, PMASK, ABP_K_COMPACT, false>(A, stream);
  if constexpr (D > 1 && (PMASK == 0 || PMASK == (1 << D) - 1))
    if (iso) return go_f64<D, PMASK, ABP_K_GAUSS, true>(A, stream);
  return go_f64<D, PMASK, ABP_K_GAUSS, false>(A, stream);
}

template <int D>
hipError_t dispatch_f64(const DirectArgs& A, int mask, bool iso, hipStream_t stream) {
  switch (mask) {
    case 0: return dispatch_f64_mask<D, 0>(A, iso, stream);
    case 1: return dispatch_f64_mask<D, 1>(A, iso, stream);
    case 2: if constexpr (D >= 2) return dispatch_f64_mask<D, 2>(A, iso, stream); break;
    case 3: if constexpr (D >= 2) return dispatch_f64_mask<D, 3>(A, iso, stream); break;
    case 4: if constexpr (D >= 3) return dispatch_f64_mask<D, 4>(A, iso, stream); break;
    case 5: if constexpr (D >= 3) return dispatch_f64_mask<D, 5>(A, iso, stream); break;
    case 6: if constexpr (D >= 3) return dispatch_f64_mask<D, 6>(A, iso, stream); break;
    case 7: if constexpr (D >= 3) return dispatch_f64_mask<D, 7>(A, iso, stream); break;
    default: break;
  }
  return hipErrorInvalidValue;
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
  A.l64 = H.l64;
  A.capacity = H.capacity;
  A.nvis = n_visible;
  A.nq = nq;
  A.q = q;
  A.V = V;
  A.dV = dVds;
  A.q_f64 = q_f64;
  int mask = 0;
  bool iso = K.kernel == ABP_K_GAUSS, iso64 = iso;
  for (int i = 0; i < K.ndim; ++i) {
    mask |= (K.periodic[i] ? 1 : 0) << i;
    iso = iso && K.kf32[i] == K.kf32[0];
    iso64 = iso64 && K.kf64[i] == K.kf64[0];
  }
  if (prec == ABP_PREC_FP64) {
    switch (K.ndim) {
      case 1: return dispatch_f64<1>(A, mask, iso64, stream);
      case 2: return dispatch_f64<2>(A, mask, iso64, stream);
      case 3: return dispatch_f64<3>(A, mask, iso64, stream);
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

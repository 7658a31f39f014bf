// Direct hill sum (bias_eval, mode DIRECT): for every query s,
//   h(s) = sum_{k < n_visible} w_k K(s - c_k),   dh/ds_i,
// the discretised form of eq. histos (Supplemental Material, "Streamlined
// bias potential updates"), followed by the transform of eq. apfm /
// eq. btraj-grad.
//
// Query-parallel: each thread holds Q queries in registers; the block stages
// tiles of hills in LDS and every wave reads each hill record as a broadcast.
// The sum is an exp-bound VALU map-reduce, so it runs on the vector ALUs
// (v_exp_f32 issues beside the FMA stream), not on the matrix cores.
//
// Hills are summed in index order for every query, so a query's result does
// not depend on the batch it is in.
#include "abp_device.h"

namespace abp {
namespace {

struct DirectArgs {
  Consts K;
  const int4* rec32;
  const double* c64;
  const double* w64;
  int64_t capacity;
  int64_t nvis;
  int64_t nq;
  const void* q;
  void* V;
  void* dV;
  int32_t q_f64;
  int32_t kahan;
};

template <int D>
__device__ __forceinline__ double load_q(const DirectArgs& A, int axis, int64_t j) {
  return A.q_f64 ? static_cast<const double*>(A.q)[axis * A.nq + j]
                 : (double)static_cast<const float*>(A.q)[axis * A.nq + j];
}

template <int D>
__device__ __forceinline__ void store_out(const DirectArgs& A, int64_t j, double V, const double (&dV)[D]) {
  if (A.q_f64) {
    static_cast<double*>(A.V)[j] = V;
#pragma unroll
    for (int i = 0; i < D; ++i) static_cast<double*>(A.dV)[i * A.nq + j] = dV[i];
  } else {
    static_cast<float*>(A.V)[j] = (float)V;
#pragma unroll
    for (int i = 0; i < D; ++i) static_cast<float*>(A.dV)[i * A.nq + j] = (float)dV[i];
  }
}

template <int D, int PMASK, int KERN, int Q>
__global__ __launch_bounds__(kBlock) void k_direct_f32(const DirectArgs A) {
  __shared__ int4 tile[kTile32];
  const int64_t first = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * Q;
  uint32_t qw[Q][D];
  float S[Q][D + 1], Cc[Q][D + 1], P[Q][D + 1];
  float kf[D], ua[D];
#pragma unroll
  for (int i = 0; i < D; ++i) { kf[i] = A.K.kf32[i]; ua[i] = A.K.ua32[i]; }
  const float pl = A.K.pl32;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    int64_t iq = first + j;
    iq = iq < A.nq ? iq : A.nq - 1;
#pragma unroll
    for (int i = 0; i < D; ++i) qw[j][i] = work32(A.K, i, load_q<D>(A, i, iq));
#pragma unroll
    for (int r = 0; r <= D; ++r) { S[j][r] = 0.0f; Cc[j][r] = 0.0f; P[j][r] = 0.0f; }
  }
  for (int64_t t0 = 0; t0 < A.nvis; t0 += kTile32) {
    const int n = (int)(A.nvis - t0 < kTile32 ? A.nvis - t0 : kTile32);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kBlock) tile[i] = A.rec32[t0 + i];
    __syncthreads();
    int c0 = 0;
    for (; c0 + kChunk <= n; c0 += kChunk) {
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        const int4 h = tile[c0 + u];
#pragma unroll
        for (int j = 0; j < Q; ++j) pair32<D, PMASK, KERN>(qw[j], h, kf, ua, pl, P[j]);
      }
      if (A.kahan) {
#pragma unroll
        for (int j = 0; j < Q; ++j) kahan_fold<D + 1>(S[j], Cc[j], P[j]);
      }
    }
    for (; c0 < n; ++c0) {
      const int4 h = tile[c0];
#pragma unroll
      for (int j = 0; j < Q; ++j) pair32<D, PMASK, KERN>(qw[j], h, kf, ua, pl, P[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    double h, dh[D];
    if (A.kahan) {
      kahan_fold<D + 1>(S[j], Cc[j], P[j]);
      h = (double)S[j][0] - (double)Cc[j][0];
#pragma unroll
      for (int i = 0; i < D; ++i) dh[i] = ((double)S[j][i + 1] - (double)Cc[j][i + 1]) * A.K.gs32[i];
    } else {
      h = (double)P[j][0];
#pragma unroll
      for (int i = 0; i < D; ++i) dh[i] = (double)P[j][i + 1] * A.K.gs32[i];
    }
    double V, dV[D];
    apply_transform<D>(A.K, h, dh, V, dV);
    const int64_t iq = first + j;
    if (iq < A.nq) store_out<D>(A, iq, V, dV);
  }
}

template <int D, int KERN>
__global__ __launch_bounds__(kBlock) void k_direct_f64(const DirectArgs A) {
  __shared__ double4 tile[kTile64];
  const int64_t iq0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t iq = iq0 < A.nq ? iq0 : A.nq - 1;
  double tq[D], P[D + 1];
#pragma unroll
  for (int i = 0; i < D; ++i) tq[i] = work64(A.K, i, load_q<D>(A, i, iq));
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

template <int D, int PMASK, int KERN>
hipError_t go_f32(const DirectArgs& A, hipStream_t stream) {
  constexpr int Q = (D == 1) ? 4 : 2;
  const int64_t per_block = (int64_t)kBlock * Q;
  const int64_t blocks = (A.nq + per_block - 1) / per_block;
  hipLaunchKernelGGL((k_direct_f32<D, PMASK, KERN, Q>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, A);
  return hipGetLastError();
}

template <int D, int KERN>
hipError_t go_f64(const DirectArgs& A, hipStream_t stream) {
  const int64_t blocks = (A.nq + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_direct_f64<D, KERN>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, A);
  return hipGetLastError();
}

template <int D, int KERN>
hipError_t dispatch_mask(int mask, const DirectArgs& A, hipStream_t stream) {
  switch (mask) {
    case 0: return go_f32<D, 0, KERN>(A, stream);
    case 1: return go_f32<D, 1, KERN>(A, stream);
    case 2: if constexpr (D >= 2) return go_f32<D, 2, KERN>(A, stream); break;
    case 3: if constexpr (D >= 2) return go_f32<D, 3, KERN>(A, stream); break;
    case 4: if constexpr (D >= 3) return go_f32<D, 4, KERN>(A, stream); break;
    case 5: if constexpr (D >= 3) return go_f32<D, 5, KERN>(A, stream); break;
    case 6: if constexpr (D >= 3) return go_f32<D, 6, KERN>(A, stream); break;
    case 7: if constexpr (D >= 3) return go_f32<D, 7, KERN>(A, stream); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int D>
hipError_t dispatch_d(const DirectArgs& A, abp_prec prec, int mask, hipStream_t stream) {
  if (prec == ABP_PREC_FP64)
    return A.K.kernel == ABP_K_GAUSS ? go_f64<D, ABP_K_GAUSS>(A, stream) : go_f64<D, ABP_K_COMPACT>(A, stream);
  return A.K.kernel == ABP_K_GAUSS ? dispatch_mask<D, ABP_K_GAUSS>(mask, A, stream)
                                   : dispatch_mask<D, ABP_K_COMPACT>(mask, A, stream);
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
  A.kahan = prec == ABP_PREC_FP32_KAHAN ? 1 : 0;
  int mask = 0;
  for (int i = 0; i < K.ndim; ++i) mask |= (K.periodic[i] ? 1 : 0) << i;
  switch (K.ndim) {
    case 1: return dispatch_d<1>(A, prec, mask, stream);
    case 2: return dispatch_d<2>(A, prec, mask, stream);
    case 3: return dispatch_d<3>(A, prec, mask, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace abp

// Direct hill sum kernels (bias_eval, mode DIRECT): for every query s,
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
//
// FP32 with compensation: terms are summed plainly in chunks of kChunk hills
// and each chunk is folded into a Kahan-compensated running sum. The error is
// at most about (kChunk + 2) u times the sum of |terms| (u = 2^-24), versus
// n u for a plain running sum.
#pragma once

#include "abp_device.h"

namespace abp {

struct DirectArgs {
  Consts K;
  const int4* rec32;
  const double* c64;
  const double* l64;      // log2 of the heights (FP64 path)
  int64_t capacity;
  int64_t nvis;
  int64_t nq;
  const void* q;
  void* V;
  void* dV;
  int32_t q_f64;
};

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

template <int D, int PMASK, int KERN, bool ISO, bool KAHAN, int Q>
__global__ __launch_bounds__(kBlock) void k_direct_f32(const DirectArgs A) {
  __shared__ int4 tile[kTile32];
  const int64_t first = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * Q;
  uint32_t qw[Q][D];
  float S[Q][D + 1], Cc[Q][D + 1], P[Q][D + 1];
  float kf[D], ua[D];
#pragma unroll
  for (int i = 0; i < D; ++i) { kf[i] = A.K.kf32[i]; ua[i] = A.K.ua32[i]; }
  const float pl = A.K.pl32;
  bool finite[Q];                     // a non-finite query coordinate gives NaN outputs
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    int64_t iq = first + j;
    iq = iq < A.nq ? iq : A.nq - 1;
    finite[j] = true;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double x = load_q(A, i, iq);
      finite[j] = finite[j] && isfinite(x);
      qw[j][i] = work32(A.K, i, eval_coord(A.K, i, isfinite(x) ? x : A.K.lo[i]));
    }
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
      {
        const int4 h = tile[c0];
#pragma unroll
        for (int j = 0; j < Q; ++j) pair32<D, PMASK, KERN, ISO, KAHAN>(qw[j], h, kf, ua, pl, P[j]);
      }
#pragma unroll
      for (int u = 1; u < kChunk; ++u) {
        const int4 h = tile[c0 + u];
#pragma unroll
        for (int j = 0; j < Q; ++j) pair32<D, PMASK, KERN, ISO, false>(qw[j], h, kf, ua, pl, P[j]);
      }
      if (KAHAN) {
#pragma unroll
        for (int j = 0; j < Q; ++j) kahan_fold<D + 1>(S[j], Cc[j], P[j]);
      }
    }
    if (c0 < n) {
      if (KAHAN) {
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
          for (int r = 0; r <= D; ++r) P[j][r] = 0.0f;
      }
      for (; c0 < n; ++c0) {
        const int4 h = tile[c0];
#pragma unroll
        for (int j = 0; j < Q; ++j) pair32<D, PMASK, KERN, ISO, false>(qw[j], h, kf, ua, pl, P[j]);
      }
      if (KAHAN) {
#pragma unroll
        for (int j = 0; j < Q; ++j) kahan_fold<D + 1>(S[j], Cc[j], P[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    double h, dh[D];
    if (KAHAN) {
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
    if (!finite[j]) {
      V = __builtin_nan("");
#pragma unroll
      for (int i = 0; i < D; ++i) dV[i] = V;
    }
    const int64_t iq = first + j;
    if (iq < A.nq) store_out<D>(A, iq, V, dV);
  }
}

template <int D, int PMASK, int KERN, bool ISO, bool KAHAN>
hipError_t go_f32(const DirectArgs& A, hipStream_t stream) {
  constexpr int Q = (D == 1) ? 4 : kQ2D;
  const int64_t per_block = (int64_t)kBlock * Q;
  const int64_t blocks = (A.nq + per_block - 1) / per_block;
  hipLaunchKernelGGL((k_direct_f32<D, PMASK, KERN, ISO, KAHAN, Q>), dim3((unsigned)blocks), dim3(kBlock), 0,
                     stream, A);
  return hipGetLastError();
}

template <int D, int PMASK, bool KAHAN>
hipError_t go_kernel(const DirectArgs& A, bool iso, hipStream_t stream) {
  constexpr bool kAllSame = PMASK == 0 || PMASK == (1 << D) - 1;
  if (A.K.kernel == ABP_K_GAUSS) {
    if constexpr (kAllSame && D > 1)
      if (iso) return go_f32<D, PMASK, ABP_K_GAUSS, true, KAHAN>(A, stream);
    return go_f32<D, PMASK, ABP_K_GAUSS, false, KAHAN>(A, stream);
  }
  return go_f32<D, PMASK, ABP_K_COMPACT, false, KAHAN>(A, stream);
}

// FP32 dispatch for one dimension (instantiated in direct_sum_d<D>.hip). The
// FP32 working words are fixed point on every axis, so the periodic mask does
// not change the kernel (the minimum image is the wrapping difference).
template <int D>
hipError_t dispatch_f32(const DirectArgs& A, int mask, bool iso, bool kahan, hipStream_t stream) {
  if (mask < 0 || mask >= (1 << D)) return hipErrorInvalidValue;
  return kahan ? go_kernel<D, 0, true>(A, iso, stream) : go_kernel<D, 0, false>(A, iso, stream);
}

hipError_t dispatch_f32_d1(const DirectArgs& A, int mask, bool iso, bool kahan, hipStream_t stream);
hipError_t dispatch_f32_d2(const DirectArgs& A, int mask, bool iso, bool kahan, hipStream_t stream);
hipError_t dispatch_f32_d3(const DirectArgs& A, int mask, bool iso, bool kahan, hipStream_t stream);

}  // namespace abp

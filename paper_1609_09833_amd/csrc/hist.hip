// Hill history append (bias_deposit): the deposits of eq. update / eq. Cupdate
// are kept as an append-only history of centres and heights. Each hill is
// stored once in FP64 (master copy, used by the FP64 sum and the grid) and
// once as a 16-byte FP32 working record {c0, c1, c2, log2(w)} read by the
// FP32 direct sum.
#include "abp_device.h"

namespace abp {
namespace {

struct AppendArgs {
  Consts K;
  HistView H;
  int64_t first;
  int64_t n;
  int32_t f64;
  const void* centers;   // [ndim][n]
  const void* heights;   // [n]
  const void* vbias;     // [n] or NULL: bias at each centre (well-tempered heights)
  int32_t* err;
};

__global__ __launch_bounds__(kBlock) void k_hist_append(const AppendArgs A) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= A.n) return;
  const int64_t slot = A.first + k;
  double c[3] = {0.0, 0.0, 0.0};
  bool ok = true;
  for (int i = 0; i < A.K.ndim; ++i) {
    c[i] = A.f64 ? static_cast<const double*>(A.centers)[i * A.n + k]
                 : (double)static_cast<const float*>(A.centers)[i * A.n + k];
    ok = ok && isfinite(c[i]);
  }
  double w = A.f64 ? static_cast<const double*>(A.heights)[k]
                   : (double)static_cast<const float*>(A.heights)[k];
  if (A.vbias && A.K.wt_dT > 0.0) {
    const double v = A.f64 ? static_cast<const double*>(A.vbias)[k] : (double)static_cast<const float*>(A.vbias)[k];
    w *= exp(-v / A.K.wt_dT);
  }
  ok = ok && isfinite(w) && w >= 0.0;
  if (!ok) {
    atomicOr(A.err, kErrNonfinite);
    for (int i = 0; i < A.K.ndim; ++i) c[i] = A.K.lo[i];
    w = 0.0;
  }
  for (int i = 0; i < A.K.ndim; ++i) c[i] = eval_coord(A.K, i, c[i]);   // quantised mode: the node
  int4 rec;
  uint32_t words[3] = {0u, 0u, 0u};
  for (int i = 0; i < A.K.ndim; ++i) {
    A.H.c64[i * A.H.capacity + slot] = c[i];
    words[i] = work32(A.K, i, c[i]);
  }
  A.H.w64[slot] = w;
  A.H.l64[slot] = log2_height(w);
  rec.x = (int)words[0];
  rec.y = (int)words[1];
  rec.z = (int)words[2];
  rec.w = __float_as_int((float)log2(w));   // log2(0) = -inf: a zero-height hill adds nothing
  A.H.rec32[slot] = rec;
}

// Every slot starts as a zero-height hill, so a reserved slot that is never
// written contributes nothing once committed.
__global__ __launch_bounds__(kBlock) void k_hist_init(const HistView H, int ndim) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= H.capacity) return;
  for (int i = 0; i < ndim; ++i) H.c64[i * H.capacity + k] = 0.0;
  H.w64[k] = 0.0;
  H.l64[k] = kLog2Zero;
  int4 rec;
  rec.x = 0;
  rec.y = 0;
  rec.z = 0;
  rec.w = __float_as_int(-__builtin_inff());
  H.rec32[k] = rec;
}

}  // namespace

hipError_t launch_hist_init(const HistView& H, int ndim, hipStream_t stream) {
  const int64_t blocks = (H.capacity + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_hist_init, dim3((unsigned)blocks), dim3(kBlock), 0, stream, H, ndim);
  return hipGetLastError();
}

hipError_t launch_hist_append(const Consts& K, const HistView& H, int64_t first, int64_t n,
                              int dtype_f64, const void* centers, const void* heights,
                              const void* vbias, int32_t* err, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  AppendArgs A;
  A.K = K;
  A.H = H;
  A.first = first;
  A.n = n;
  A.f64 = dtype_f64;
  A.centers = centers;
  A.heights = heights;
  A.vbias = vbias;
  A.err = err;
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_hist_append, dim3((unsigned)blocks), dim3(kBlock), 0, stream, A);
  return hipGetLastError();
}

}  // namespace abp

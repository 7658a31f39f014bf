// Grid form of the bias (bias_deposit with a grid, bias_eval mode GRID).
//
// Deposit: every node g of the grid accumulates, for each hill of the batch,
// the hill's value and derivatives at g: the update of eq. update (Gaussian)
// or eq. Cupdate (compact S_a^p), kept as 2^ndim FP64 arrays per node:
// value, first derivatives and mixed derivatives (entry m differentiates
// along each axis whose bit is set in m). Storing the mixed derivatives lets
// the evaluation use tensor-product cubic Hermite interpolation instead of
// the paper's nearest-node look-up.
//
// The hill is a product over axes, so per hill and per node tile the block
// evaluates 1-D factor vectors once (LDS) and forms the node values as
// outer products: each node costs 2^ndim FMAs per hill. For compact kernels
// a hill whose support misses the tile is skipped, which is the Nbase^d
// saving of eq. Cupdate at tile granularity.
//
// Evaluation: one thread per query, 2^ndim corners x 2^ndim arrays gathered
// from the node-interleaved layout, FP64 arithmetic.
#include "abp_device.h"

namespace abp {
namespace {

constexpr int kTX = 64;        // nodes along axis 0 per tile (one per lane)
constexpr int kRY = 8;         // rows along axis 1 per thread
constexpr int kTY = 4 * kRY;   // rows along axis 1 per tile (4 waves)
constexpr int kKC = 16;        // hills per LDS chunk
constexpr int kMinBlocks = 1024;

struct DepositArgs {
  Consts K;
  const double* c64;
  const double* w64;
  int64_t capacity;
  int64_t k0, k1;          // hill range
  int32_t nsplit;          // hill sub-ranges (blocks per tile)
  int64_t tiles;           // node tiles
  double* grid;
  double* scratch;         // [nsplit][nodes][2^D] when nsplit > 1
};

// Value and derivative (d/ds) of axis `i` of hill centred at c, at node coordinate x.
__device__ __forceinline__ void factor(const Consts& K, int i, double x, double c, double& v, double& d) {
  double delta = x - c;
  if (K.periodic[i]) delta -= K.period[i] * rint(delta * K.inv_period[i]);
  const double wdt = K.width[i];
  if (K.kernel == ABP_K_GAUSS) {
    const double r = delta / wdt;
    v = exp(-0.5 * r * r);
    d = -(delta / (wdt * wdt)) * v;
  } else {
    const double u = delta / wdt;
    if (fabs(u) < 1.0) {
      const double om = 1.0 - u * u;
      v = exp(-(double)K.p * u * u / om);
      d = -2.0 * K.p * delta / (wdt * wdt * om * om) * v;
    } else {
      v = 0.0;
      d = 0.0;
    }
  }
}

__device__ __forceinline__ double node_coord(const Consts& K, int i, int64_t j) {
  return K.lo[i] + (double)j * K.grid_dx[i];
}

__device__ __forceinline__ void split_range(const DepositArgs& A, int s, int64_t& kb, int64_t& ke) {
  const int64_t n = A.k1 - A.k0;
  kb = A.k0 + n * s / A.nsplit;
  ke = A.k0 + n * (s + 1) / A.nsplit;
}

// 1-D grids: one thread per node.
__global__ __launch_bounds__(kBlock) void k_deposit_1d(const DepositArgs A) {
  const int64_t tile = blockIdx.x % A.tiles;
  const int s = (int)(blockIdx.x / A.tiles);
  const int64_t j = tile * kBlock + threadIdx.x;
  const int64_t n0 = A.K.grid_n[0];
  int64_t kb, ke;
  split_range(A, s, kb, ke);
  if (j >= n0) return;
  const double x = node_coord(A.K, 0, j);
  double a0 = 0.0, a1 = 0.0;
  for (int64_t k = kb; k < ke; ++k) {
    double v, d;
    factor(A.K, 0, x, A.c64[k], v, d);
    const double w = A.w64[k];
    a0 = __builtin_fma(w, v, a0);
    a1 = __builtin_fma(w, d, a1);
  }
  if (A.nsplit == 1) {
    A.grid[j * 2] += a0;
    A.grid[j * 2 + 1] += a1;
  } else {
    double* out = A.scratch + ((int64_t)s * A.K.nodes + j) * 2;
    out[0] = a0;
    out[1] = a1;
  }
}

// 2-D and 3-D grids: tile of kTX x kTY nodes (one z plane for 3-D).
template <int D>
__global__ __launch_bounds__(kBlock) void k_deposit_nd(const DepositArgs A) {
  constexpr int NM = 1 << D;
  constexpr int NY = 1 << (D - 1);          // combos of the derivative bits of axes 1..D-1
  __shared__ double Xf[kKC][2][kTX];        // axis-0 value / derivative at the tile's nodes
  __shared__ double Yf[kKC][kTY][NY];       // w * (axis 1 x axis 2 factors)
  __shared__ int live_x[kKC], live_y[kKC];

  const int64_t tiles_x = (A.K.grid_n[0] + kTX - 1) / kTX;
  const int64_t tiles_y = (A.K.grid_n[1] + kTY - 1) / kTY;
  const int64_t tile = blockIdx.x % A.tiles;
  const int s = (int)(blockIdx.x / A.tiles);
  const int64_t tx = tile % tiles_x;
  const int64_t ty = (tile / tiles_x) % tiles_y;
  const int64_t tz = tile / (tiles_x * tiles_y);    // 0 for D == 2
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n0 = A.K.grid_n[0], n1 = A.K.grid_n[1];
  const int64_t x0 = tx * kTX, y0 = ty * kTY;
  int64_t kb, ke;
  split_range(A, s, kb, ke);

  double zc = 0.0;
  if (D == 3) zc = node_coord(A.K, 2, tz);
  double acc[kRY][NM];
#pragma unroll
  for (int r = 0; r < kRY; ++r)
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[r][m] = 0.0;

  for (int64_t kc = kb; kc < ke; kc += kKC) {
    const int nk = (int)(ke - kc < kKC ? ke - kc : kKC);
    __syncthreads();
    if (threadIdx.x < kKC) { live_x[threadIdx.x] = 0; live_y[threadIdx.x] = 0; }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kKC * kTX; idx += kBlock) {
      const int k = idx / kTX, l = idx % kTX;
      double v = 0.0, d = 0.0;
      const int64_t xj = x0 + l;
      if (k < nk && xj < n0) factor(A.K, 0, node_coord(A.K, 0, xj), A.c64[kc + k], v, d);
      Xf[k][0][l] = v;
      Xf[k][1][l] = d;
      if (v != 0.0 || d != 0.0) live_x[k] = 1;
    }
    for (int idx = threadIdx.x; idx < kKC * kTY; idx += kBlock) {
      const int k = idx / kTY, r = idx % kTY;
      double yv = 0.0, yd = 0.0, zv = 1.0, zd = 0.0, w = 0.0;
      const int64_t yj = y0 + r;
      if (k < nk && yj < n1) {
        const int64_t kk = kc + k;
        w = A.w64[kk];
        factor(A.K, 1, node_coord(A.K, 1, yj), A.c64[A.capacity + kk], yv, yd);
        if (D == 3) factor(A.K, 2, zc, A.c64[2 * A.capacity + kk], zv, zd);
      }
      Yf[k][r][0] = w * yv * zv;
      Yf[k][r][1] = w * yd * zv;
      if (D == 3) {
        Yf[k][r][NY > 2 ? 2 : 0] = w * yv * zd;
        Yf[k][r][NY > 3 ? 3 : 0] = w * yd * zd;
      }
      bool nz = Yf[k][r][0] != 0.0 || Yf[k][r][1] != 0.0;
      if (D == 3) nz = nz || Yf[k][r][NY > 2 ? 2 : 0] != 0.0 || Yf[k][r][NY > 3 ? 3 : 0] != 0.0;
      if (nz) live_y[k] = 1;
    }
    __syncthreads();
    for (int k = 0; k < nk; ++k) {
      if (!(live_x[k] && live_y[k])) continue;     // uniform across the block
      const double xv = Xf[k][0][lane], xd = Xf[k][1][lane];
#pragma unroll
      for (int r = 0; r < kRY; ++r) {
        const double* yw = Yf[k][wave * kRY + r];
#pragma unroll
        for (int my = 0; my < NY; ++my) {
          const double f = yw[my];
          acc[r][2 * my] = __builtin_fma(xv, f, acc[r][2 * my]);
          acc[r][2 * my + 1] = __builtin_fma(xd, f, acc[r][2 * my + 1]);
        }
      }
    }
  }
  const int64_t xj = x0 + lane;
  if (xj >= n0) return;
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    const int64_t yj = y0 + wave * kRY + r;
    if (yj >= n1) continue;
    const int64_t node = xj + n0 * (yj + n1 * tz);
    if (A.nsplit == 1) {
      double* g = A.grid + node * NM;
#pragma unroll
      for (int m = 0; m < NM; ++m) g[m] += acc[r][m];
    } else {
      double* o = A.scratch + ((int64_t)s * A.K.nodes + node) * NM;
#pragma unroll
      for (int m = 0; m < NM; ++m) o[m] = acc[r][m];
    }
  }
}

// grid[v] += sum over split s (in order) of scratch[s][v].
__global__ __launch_bounds__(kBlock) void k_reduce_split(double* grid, const double* scratch,
                                                         int64_t nvals, int nsplit) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvals) return;
  double t = 0.0;
  for (int s = 0; s < nsplit; ++s) t += scratch[(int64_t)s * nvals + v];
  grid[v] += t;
}

struct EvalArgs {
  Consts K;
  const double* grid;
  int64_t nq;
  const void* q;
  void* V;
  void* dV;
  int32_t q_f64;
  unsigned long long* n_clamped;
};

template <int D>
__global__ __launch_bounds__(kBlock) void k_grid_eval(const EvalArgs A) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= A.nq) return;
  double s[D];
#pragma unroll
  for (int i = 0; i < D; ++i)
    s[i] = A.q_f64 ? static_cast<const double*>(A.q)[i * A.nq + j]
                   : (double)static_cast<const float*>(A.q)[i * A.nq + j];
  double h, dh[D], V, dV[D];
  bool clamped;
  hermite_eval<D>(A.K, A.grid, s, h, dh, clamped);
  if (clamped && A.n_clamped) atomicAdd(A.n_clamped, 1ull);
  apply_transform<D>(A.K, h, dh, V, dV);
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

int64_t node_tiles(const Consts& K) {
  if (K.ndim == 1) return (K.grid_n[0] + kBlock - 1) / kBlock;
  int64_t t = ((K.grid_n[0] + kTX - 1) / kTX) * ((K.grid_n[1] + kTY - 1) / kTY);
  if (K.ndim == 3) t *= K.grid_n[2];
  return t;
}

int split_for(const Consts& K, int64_t nhills) {
  const int64_t tiles = node_tiles(K);
  int64_t s = (kMinBlocks + tiles - 1) / tiles;
  const int64_t by_hills = nhills / 256;       // at least 256 hills per sub-range
  if (s > by_hills) s = by_hills;
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  return (int)s;
}

}  // namespace

size_t grid_deposit_scratch_bytes(const Consts& K, int64_t nhills) {
  const int s = split_for(K, nhills);
  if (s <= 1) return 0;
  return (size_t)s * (size_t)K.nodes * ((size_t)1 << K.ndim) * sizeof(double);
}

hipError_t launch_grid_deposit(const Consts& K, const HistView& H, int64_t k0, int64_t k1,
                               double* grid, double* scratch, hipStream_t stream) {
  if (k1 <= k0) return hipSuccess;
  DepositArgs A;
  A.K = K;
  A.c64 = H.c64;
  A.w64 = H.w64;
  A.capacity = H.capacity;
  A.k0 = k0;
  A.k1 = k1;
  A.nsplit = split_for(K, k1 - k0);
  if (A.nsplit > 1 && scratch == nullptr) A.nsplit = 1;
  A.tiles = node_tiles(K);
  A.grid = grid;
  A.scratch = scratch;
  const unsigned blocks = (unsigned)(A.tiles * A.nsplit);
  switch (K.ndim) {
    case 1: hipLaunchKernelGGL(k_deposit_1d, dim3(blocks), dim3(kBlock), 0, stream, A); break;
    case 2: hipLaunchKernelGGL(k_deposit_nd<2>, dim3(blocks), dim3(kBlock), 0, stream, A); break;
    case 3: hipLaunchKernelGGL(k_deposit_nd<3>, dim3(blocks), dim3(kBlock), 0, stream, A); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || A.nsplit == 1) return e;
  const int64_t nvals = K.nodes << K.ndim;
  hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((nvals + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     stream, grid, (const double*)scratch, nvals, A.nsplit);
  return hipGetLastError();
}

hipError_t launch_grid_eval(const Consts& K, const double* grid, int64_t nq, int q_f64,
                            const void* q, void* V, void* dVds, unsigned long long* n_clamped,
                            hipStream_t stream) {
  if (nq <= 0) return hipSuccess;
  EvalArgs A;
  A.K = K;
  A.grid = grid;
  A.nq = nq;
  A.q = q;
  A.V = V;
  A.dV = dVds;
  A.q_f64 = q_f64;
  A.n_clamped = n_clamped;
  const unsigned blocks = (unsigned)((nq + kBlock - 1) / kBlock);
  switch (K.ndim) {
    case 1: hipLaunchKernelGGL(k_grid_eval<1>, dim3(blocks), dim3(kBlock), 0, stream, A); break;
    case 2: hipLaunchKernelGGL(k_grid_eval<2>, dim3(blocks), dim3(kBlock), 0, stream, A); break;
    case 3: hipLaunchKernelGGL(k_grid_eval<3>, dim3(blocks), dim3(kBlock), 0, stream, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace abp

// Grid form of the bias (bias_deposit with a grid, bias_eval mode GRID).
//
// Deposit: every node g of the grid accumulates, for each hill of the batch,
// the hill's value and derivatives at g: the update of eq. update (Gaussian)
// or eq. Cupdate (compact S_a^p), kept as 2^ndim FP64 arrays per node:
// value, first derivatives and mixed derivatives (entry m differentiates
// along each axis whose bit is set in m). Storing the mixed derivatives lets
// the evaluation use tensor-product cubic Hermite interpolation; the
// quantised mode reads the value and first-derivative arrays at the nearest
// node instead (the paper's look-up).
//
// The hill is a product over axes, so the node arrays of a batch are sums of
// outer products of 1-D factor vectors: each node costs 2^ndim FMAs per hill.
// For 2-D and 3-D Gaussian grids that sum is a dense contraction over the
// hills and runs on the matrix cores (FP64 MFMA, k_deposit_mfma2/3). Otherwise a block
// evaluates the 1-D factors of a chunk of hills once (LDS) and each thread
// forms COLS x RY nodes from them; for compact kernels a hill whose support
// misses the tile is skipped, which is the Nbase^d saving of eq. Cupdate at
// tile granularity.
//
// Evaluation: 2^ndim corners x 2^ndim arrays gathered from the FP64
// node-interleaved layout in FP64 arithmetic, or from the FP32 mirror the
// host layer refreshes after every deposit in FP32 arithmetic: cell-major for
// 1-D and 2-D grids (each cell holds its corners' entries, so a query gathers
// one 16- or 64-byte record, one cache line, instead of one line per corner),
// node-major for 3-D. In 2-D a group of four lanes fetches each of its four
// queries' data together, 16 bytes a lane, and passes it through LDS to the
// query's lane (k_grid_eval_cells32, k_grid_eval_nodes64); otherwise one
// thread gathers for each query (k_grid_eval).
#include <algorithm>

#include "abp_device.h"

namespace abp {
namespace {

// Tile shape of the VALU deposit (compact 2-D and 3-D hills): 64 * COLS
// nodes along axis 0 (lane l owns columns l, l + 64, ...), 4 * RY along axis
// 1 (wave v owns rows v*RY ..), one plane along axis 2. Narrow tiles keep the
// work on nodes outside a compact hill's support small. Gaussian grids use
// the matrix-core deposits below.
constexpr int kCols = 1, kRY = 8;   // nodes per thread: columns x rows
constexpr int kKC = 16;             // hills per LDS chunk
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
  uint32_t* dirty;         // [tiles] or NULL: `epoch` for every tile a hill reached
  uint32_t epoch;
};

constexpr double kHalfLog2e = 0.72134752044448170368;   // log2(e) / 2

// Value and derivative (d/ds) of axis `i` of hill centred at c, at node
// coordinate x (exponentials through the FP64 hill-term exp2).
__device__ __forceinline__ void factor(const Consts& K, int i, double x, double c, double& v, double& d) {
  double delta = x - c;
  if (K.periodic[i]) delta -= K.period[i] * rint(delta * K.inv_period[i]);
  const double iw = K.inv_width[i];
  if (K.kernel == ABP_K_GAUSS) {
    const double r = delta * iw;
    v = exp2_term(-kHalfLog2e * (r * r));
    d = -(r * iw) * v;
  } else {
    const double u = delta * iw;
    if (fabs(u) < 1.0) {
      const double ro = 1.0 / (1.0 - u * u);
      v = exp2_term(-K.pl64 * (u * u * ro));
      d = -2.0 * K.p * u * iw * ro * ro * v;
    } else {
      v = 0.0;
      d = 0.0;
    }
  }
}

// Node j's coordinate, lo + j dx with two roundings (not fused), the same
// value the quantised mode snaps hill centres and queries to.
__device__ __forceinline__ double node_coord(const Consts& K, int i, int64_t j) {
#pragma clang fp contract(off)
  const double p = (double)j * K.grid_dx[i];
  return K.lo[i] + p;
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

// 2-D and 3-D grids: tile of 64*COLS x 4*RY nodes (one z plane for 3-D).
template <int D>
__global__ __launch_bounds__(kBlock) void k_deposit_nd(const DepositArgs A) {
  constexpr int NM = 1 << D;
  constexpr int NY = 1 << (D - 1);          // combos of the derivative bits of axes 1..D-1
  constexpr int COLS = kCols, RY = kRY;
  constexpr int TX = 64 * COLS, TY = 4 * RY;
  __shared__ double2 Xf[kKC][TX];           // axis-0 (value, derivative) at the tile's columns
  __shared__ double Yf[kKC][TY][NY];        // w * (axis 1 x axis 2 factors)
  __shared__ int live_x[kKC], live_y[kKC];

  const int64_t tiles_x = (A.K.grid_n[0] + TX - 1) / TX;
  const int64_t tiles_y = (A.K.grid_n[1] + TY - 1) / TY;
  const int64_t tile = blockIdx.x % A.tiles;
  const int s = (int)(blockIdx.x / A.tiles);
  const int64_t tx = tile % tiles_x;
  const int64_t ty = (tile / tiles_x) % tiles_y;
  const int64_t tz = tile / (tiles_x * tiles_y);    // 0 for D == 2
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n0 = A.K.grid_n[0], n1 = A.K.grid_n[1];
  const int64_t x0 = tx * TX, y0 = ty * TY;
  int64_t kb, ke;
  split_range(A, s, kb, ke);

  double zc = 0.0;
  if (D == 3) zc = node_coord(A.K, 2, tz);
  double acc[COLS][RY][NM];
#pragma unroll
  for (int c = 0; c < COLS; ++c)
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
      for (int m = 0; m < NM; ++m) acc[c][r][m] = 0.0;

  bool touched = false;                       // some hill reaches the tile (uniform)
  for (int64_t kc = kb; kc < ke; kc += kKC) {
    const int nk = (int)(ke - kc < kKC ? ke - kc : kKC);
    __syncthreads();
    if (threadIdx.x < kKC) { live_x[threadIdx.x] = 0; live_y[threadIdx.x] = 0; }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kKC * TX; idx += kBlock) {
      const int k = idx / TX, l = idx % TX;
      double v = 0.0, d = 0.0;
      const int64_t xj = x0 + l;
      if (k < nk && xj < n0) factor(A.K, 0, node_coord(A.K, 0, xj), A.c64[kc + k], v, d);
      Xf[k][l] = make_double2(v, d);
      if (v != 0.0 || d != 0.0) live_x[k] = 1;
    }
    for (int idx = threadIdx.x; idx < kKC * TY; idx += kBlock) {
      const int k = idx / TY, r = idx % TY;
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
      touched = true;
      double2 xf[COLS];
#pragma unroll
      for (int c = 0; c < COLS; ++c) xf[c] = Xf[k][lane + 64 * c];
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        double f[NY];
        const double* yw = Yf[k][wave * RY + r];
#pragma unroll
        for (int my = 0; my < NY; my += 2) {
          const double2 t = *reinterpret_cast<const double2*>(yw + my);
          f[my] = t.x;
          f[my + 1] = t.y;
        }
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
          for (int my = 0; my < NY; ++my) {
            acc[c][r][2 * my] = __builtin_fma(xf[c].x, f[my], acc[c][r][2 * my]);
            acc[c][r][2 * my + 1] = __builtin_fma(xf[c].y, f[my], acc[c][r][2 * my + 1]);
          }
      }
    }
  }
  if (touched && A.dirty && threadIdx.x == 0) A.dirty[tile] = A.epoch;
  // a tile no hill reaches keeps its nodes as they are (the split's partial
  // grids still get their zeros)
  if (!touched && A.nsplit == 1) return;
#pragma unroll
  for (int c = 0; c < COLS; ++c) {
    const int64_t xj = x0 + lane + 64 * c;
    if (xj >= n0) continue;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int64_t yj = y0 + wave * RY + r;
      if (yj >= n1) continue;
      const int64_t node = xj + n0 * (yj + n1 * tz);
      if (A.nsplit == 1) {
        double* g = A.grid + node * NM;
#pragma unroll
        for (int m = 0; m < NM; ++m) g[m] += acc[c][r][m];
      } else {
        double* o = A.scratch + ((int64_t)s * A.K.nodes + node) * NM;
#pragma unroll
        for (int m = 0; m < NM; ++m) o[m] = acc[c][r][m];
      }
    }
  }
}

// 2-D Gaussian grids on the matrix cores. For one hill sub-range the node
// arrays are sums of outer products, H_m[y][x] = sum_k (w_k Y_my(y; c_k))
// (X_mx(x; c_k)), i.e. four FP64 matrix products (m = mx + 2 my) with the
// hills as the contraction index. One wave owns a 32 x 32 node tile (2 x 2
// tiles of 16 x 16 for v_mfma_f64_16x16x4f64) and walks its hills four at a
// time: lane l supplies the factors of hill l / 16 at node row / column
// l % 16, computed in registers (no LDS, no barriers), and the next group's
// factors are formed while the current group's products run.
// Operand layout of v_mfma_f64_16x16x4f64 (D = A B + C, A 16 x 4, B 4 x 16):
// A[i][k] and B[k][j] sit in lane i + 16 k and j + 16 k; D[i][j] in lane
// j + 16 (i % 4), register i / 4.
typedef double d4v __attribute__((ext_vector_type(4)));
constexpr int kMT = 32;              // nodes per side of a wave's tile
constexpr int kMinWaves = 4096;      // target waves per deposit launch (4 per SIMD)
constexpr int kStage = 256;          // hills per LDS chunk of the MFMA deposits

// Gaussian factor of axis i (periodic when P) at node coordinate x for a hill
// centred at c: value v and d/ds derivative d (straight-line code).
template <bool P>
__device__ __forceinline__ void gauss_factor(const Consts& K, int i, double x, double c, double& v, double& d) {
  double delta = x - c;
  if (P) delta -= K.period[i] * rint(delta * K.inv_period[i]);
  const double iw = K.inv_width[i];
  const double r = delta * iw;
  v = exp2_term(-kHalfLog2e * (r * r));
  d = -(r * iw) * v;
}

template <int PMASK>
__global__ __launch_bounds__(64) void k_deposit_mfma2(const DepositArgs A) {
  const Consts& K = A.K;
  const int64_t n0 = K.grid_n[0], n1 = K.grid_n[1];
  const int64_t tiles_x = (n0 + kMT - 1) / kMT;
  const int64_t tile = blockIdx.x % A.tiles;
  const int s = (int)(blockIdx.x / A.tiles);
  const int64_t x0 = (tile % tiles_x) * kMT, y0 = (tile / tiles_x) * kMT;
  const int lane = threadIdx.x;
  const int kk = lane >> 4, i16 = lane & 15;
  int64_t kb, ke;
  split_range(A, s, kb, ke);
  if (ke <= kb) return;

  double yc[2], xc[2];
  bool yin[2], xin[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int64_t yj = y0 + 16 * t + i16, xj = x0 + 16 * t + i16;
    yin[t] = yj < n1;
    xin[t] = xj < n0;
    yc[t] = node_coord(K, 1, yin[t] ? yj : 0);
    xc[t] = node_coord(K, 0, xin[t] ? xj : 0);
  }
  // its factors for hill centre (h[0], h[1]) and height h[2]: ya[my][t] (A
  // operands, y rows, times the height) and xb[mx][t] (B operands, x
  // columns); zero outside the grid
  auto factors = [&](const double (&h)[3], double (&ya)[2][2], double (&xb)[2][2]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      double v, d;
      gauss_factor<(PMASK & 2) != 0>(K, 1, yc[t], h[1], v, d);
      ya[0][t] = yin[t] ? h[2] * v : 0.0;
      ya[1][t] = yin[t] ? h[2] * d : 0.0;
      gauss_factor<(PMASK & 1) != 0>(K, 0, xc[t], h[0], v, d);
      xb[0][t] = xin[t] ? v : 0.0;
      xb[1][t] = xin[t] ? d : 0.0;
    }
  };
  d4v acc[2][2][4];
#pragma unroll
  for (int ty = 0; ty < 2; ++ty)
#pragma unroll
    for (int tx = 0; tx < 2; ++tx)
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[ty][tx][m] = d4v{0.0, 0.0, 0.0, 0.0};
  // The sub-range's hills pass through LDS in chunks of kStage: one coalesced
  // load per chunk instead of a memory round trip per group of four.
  __shared__ double hs[3][kStage];
  for (int64_t c0 = kb; c0 < ke; c0 += kStage) {
    const int n = (int)(ke - c0 < kStage ? ke - c0 : kStage);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kStage / 64; ++j) {
      const int u = lane + 64 * j;
      const int64_t k = c0 + (u < n ? u : n - 1);
      hs[0][u] = A.c64[k];
      hs[1][u] = A.c64[A.capacity + k];
      hs[2][u] = u < n ? A.w64[k] : 0.0;          // past the range: weight 0
    }
    __syncthreads();
    for (int g = 0; g < n; g += 4) {
      const double h[3] = {hs[0][g + kk], hs[1][g + kk], hs[2][g + kk]};
      double ya[2][2], xb[2][2];
      factors(h, ya, xb);
#pragma unroll
      for (int ty = 0; ty < 2; ++ty)
#pragma unroll
        for (int tx = 0; tx < 2; ++tx)
#pragma unroll
          for (int my = 0; my < 2; ++my)
#pragma unroll
            for (int mx = 0; mx < 2; ++mx)
              acc[ty][tx][mx + 2 * my] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(ya[my][ty], xb[mx][tx], acc[ty][tx][mx + 2 * my], 0, 0, 0);
    }
  }
  // lane holds x column x0 + 16 tx + lane % 16 and y rows y0 + 16 ty + 4 r + lane / 16
#pragma unroll
  for (int ty = 0; ty < 2; ++ty)
#pragma unroll
    for (int tx = 0; tx < 2; ++tx)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t xj = x0 + 16 * tx + i16, yj = y0 + 16 * ty + 4 * r + kk;
        if (xj >= n0 || yj >= n1) continue;
        const int64_t node = xj + n0 * yj;
        if (A.nsplit == 1) {
          double* g = A.grid + node * 4;
#pragma unroll
          for (int m = 0; m < 4; ++m) g[m] += acc[ty][tx][m][r];
        } else {
          double* o = A.scratch + ((int64_t)s * K.nodes + node) * 4;
#pragma unroll
          for (int m = 0; m < 4; ++m) o[m] = acc[ty][tx][m][r];
        }
      }
}

// 3-D Gaussian grids on the matrix cores: per z plane, H_m[z][y][x] =
// sum_k (w_k Y_my(y) Z_mz(z)) X_mx(x) with m = mx + 2 my + 4 mz, eight FP64
// matrix products per plane. One wave owns a 16 (y) x 32 (x) node tile of one
// plane; lane l supplies hill l / 16's factors at row / column l % 16 (the
// z factor at the plane's coordinate), as in k_deposit_mfma2.
constexpr int kMT3Y = 16;            // y rows of a 3-D wave tile (x columns: kMT)

template <int PMASK>
__global__ __launch_bounds__(64) void k_deposit_mfma3(const DepositArgs A) {
  const Consts& K = A.K;
  const int64_t n0 = K.grid_n[0], n1 = K.grid_n[1];
  const int64_t tiles_x = (n0 + kMT - 1) / kMT, tiles_y = (n1 + kMT3Y - 1) / kMT3Y;
  const int64_t tile = blockIdx.x % A.tiles;
  const int s = (int)(blockIdx.x / A.tiles);
  const int64_t x0 = (tile % tiles_x) * kMT, y0 = ((tile / tiles_x) % tiles_y) * kMT3Y;
  const int64_t z = tile / (tiles_x * tiles_y);
  const int lane = threadIdx.x;
  const int kk = lane >> 4, i16 = lane & 15;
  int64_t kb, ke;
  split_range(A, s, kb, ke);
  if (ke <= kb) return;

  const int64_t yj = y0 + i16;
  const bool yin = yj < n1;
  const double yc = node_coord(K, 1, yin ? yj : 0), zc = node_coord(K, 2, z);
  double xc[2];
  bool xin[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int64_t xj = x0 + 16 * t + i16;
    xin[t] = xj < n0;
    xc[t] = node_coord(K, 0, xin[t] ? xj : 0);
  }
  // its factors for hill centre (h[0], h[1], h[2]) and height h[3]:
  // ya[my + 2 mz] (A operands, y rows, times the height and the z factor) and
  // xb[mx][t] (B operands, x columns); zero outside the grid
  auto factors = [&](const double (&h)[4], double (&ya)[4], double (&xb)[2][2]) {
    double yv, yd, zv, zd;
    gauss_factor<(PMASK & 2) != 0>(K, 1, yc, h[1], yv, yd);
    gauss_factor<(PMASK & 4) != 0>(K, 2, zc, h[2], zv, zd);
    const double w = yin ? h[3] : 0.0;
    ya[0] = w * (yv * zv);
    ya[1] = w * (yd * zv);
    ya[2] = w * (yv * zd);
    ya[3] = w * (yd * zd);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      double v, d;
      gauss_factor<(PMASK & 1) != 0>(K, 0, xc[t], h[0], v, d);
      xb[0][t] = xin[t] ? v : 0.0;
      xb[1][t] = xin[t] ? d : 0.0;
    }
  };
  d4v acc[2][8];
#pragma unroll
  for (int tx = 0; tx < 2; ++tx)
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[tx][m] = d4v{0.0, 0.0, 0.0, 0.0};
  __shared__ double hs[4][kStage];                // hills staged as in k_deposit_mfma2
  for (int64_t c0 = kb; c0 < ke; c0 += kStage) {
    const int n = (int)(ke - c0 < kStage ? ke - c0 : kStage);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kStage / 64; ++j) {
      const int u = lane + 64 * j;
      const int64_t k = c0 + (u < n ? u : n - 1);
      hs[0][u] = A.c64[k];
      hs[1][u] = A.c64[A.capacity + k];
      hs[2][u] = A.c64[2 * A.capacity + k];
      hs[3][u] = u < n ? A.w64[k] : 0.0;          // past the range: weight 0
    }
    __syncthreads();
    for (int g = 0; g < n; g += 4) {
      const double h[4] = {hs[0][g + kk], hs[1][g + kk], hs[2][g + kk], hs[3][g + kk]};
      double ya[4], xb[2][2];
      factors(h, ya, xb);
#pragma unroll
      for (int tx = 0; tx < 2; ++tx)
#pragma unroll
        for (int myz = 0; myz < 4; ++myz)
#pragma unroll
          for (int mx = 0; mx < 2; ++mx)
            acc[tx][mx + 2 * myz] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(ya[myz], xb[mx][tx], acc[tx][mx + 2 * myz], 0, 0, 0);
    }
  }
  // lane holds x column x0 + 16 tx + lane % 16 and y rows y0 + 4 r + lane / 16
#pragma unroll
  for (int tx = 0; tx < 2; ++tx)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t xj = x0 + 16 * tx + i16, yr = y0 + 4 * r + kk;
      if (xj >= n0 || yr >= n1) continue;
      const int64_t node = xj + n0 * (yr + n1 * z);
      if (A.nsplit == 1) {
        double* g = A.grid + node * 8;
#pragma unroll
        for (int m = 0; m < 8; ++m) g[m] += acc[tx][m][r];
      } else {
        double* o = A.scratch + ((int64_t)s * K.nodes + node) * 8;
#pragma unroll
        for (int m = 0; m < 8; ++m) o[m] = acc[tx][m][r];
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
  const float* grid32;             // FP32 mirror of grid (used by the FP32 instantiation)
  int64_t nq;
  const void* q;
  void* V;
  void* dV;
  int32_t q_f64;
  unsigned long long* n_clamped;
};

// Queries per thread: independent corner gathers in flight (1-D); the 3-D
// interpolation is register-heavy enough on its own. In 2-D this kernel
// serves the quantised look-up (and grids past 2^31 nodes), one query a
// thread (480^2 paper grid, 1,048,576 look-ups: 13.6 us against 15.7 us with
// four); the Hermite interpolation has the group-of-four kernels below.
template <int D, class T> struct EvalQ { static constexpr int value = D >= 2 ? 1 : (sizeof(T) == 4 ? 2 : 4); };

template <int D, class T>
__global__ __launch_bounds__(kBlock) void k_grid_eval(const EvalArgs A) {
  const T* nodes;
  if constexpr (sizeof(T) == 4) nodes = A.grid32;
  else nodes = A.grid;
  constexpr int kEvalQ = EvalQ<D, T>::value;
  const int64_t base = (int64_t)blockIdx.x * kBlock * kEvalQ + threadIdx.x;
  double h[kEvalQ], dh[kEvalQ][D];
  bool clamped[kEvalQ];
#pragma unroll
  for (int u = 0; u < kEvalQ; ++u) {
    int64_t j = base + (int64_t)u * kBlock;
    j = j < A.nq ? j : A.nq - 1;
    double s[D];
    bool finite = true;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      s[i] = A.q_f64 ? static_cast<const double*>(A.q)[i * A.nq + j]
                     : (double)static_cast<const float*>(A.q)[i * A.nq + j];
      finite = finite && isfinite(s[i]);
    }
    if constexpr (sizeof(T) == 4) hermite_eval32<D>(A.K, nodes, s, h[u], dh[u], clamped[u]);
    else hermite_eval<D>(A.K, nodes, s, h[u], dh[u], clamped[u]);
    if (!finite) {                     // a non-finite query coordinate gives NaN outputs
      clamped[u] = false;
      h[u] = __builtin_nan("");
#pragma unroll
      for (int i = 0; i < D; ++i) dh[u][i] = h[u];
    }
  }
#pragma unroll
  for (int u = 0; u < kEvalQ; ++u) {
    const int64_t j = base + (int64_t)u * kBlock;
    if (j >= A.nq) continue;
    if (clamped[u] && A.n_clamped) atomicAdd(A.n_clamped, 1ull);
    double V, dV[D];
    apply_transform<D>(A.K, h[u], dh[u], V, dV);
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
}

// Threads per block of the group-of-four evaluation kernels: one wave (2-D,
// 1,048,576 queries, FP64 / FP32 mirror: 64 threads 17.0 / 10.9 us, 128
// 17.4 / 11.4, 256 18.4 / 11.6, 512 20.3 / 11.9).
constexpr int kEvalBlock = 64;
// Lane r's value of each group of four lanes, to all four (DPP quad_perm
// r,r,r,r). Every lane of the wave must be active where it runs.
template <int R>
__device__ __forceinline__ int32_t quad_lane(int32_t v) {
  return __builtin_amdgcn_mov_dpp(v, R * 0x55, 0xF, 0xF, true);
}

template <int R>
__device__ __forceinline__ void quad_lanes(const int32_t (&v)[4], int32_t (&out)[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c] = quad_lane<R>(v[c]);
}

// A query's outputs from the interpolated h and dh/ds: NaN for a non-finite
// query coordinate, the transform, FP32 or FP64 stores.
template <int D>
__device__ __forceinline__ void store_query(const EvalArgs& A, int64_t j, double h, double (&dh)[D], bool clamped,
                                            bool finite) {
  if (!finite) {
    clamped = false;
    h = __builtin_nan("");
#pragma unroll
    for (int i = 0; i < D; ++i) dh[i] = h;
  }
  if (clamped && A.n_clamped) atomicAdd(A.n_clamped, 1ull);
  double V, dV[D];
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

// 2-D interpolation from the FP32 cell-major mirror, the 64-byte cell records
// fetched by groups of four lanes: in round r, lane p of a group loads the
// p-th 16 bytes of the record of the query that the group's lane r holds, so
// one load instruction reaches 16 records, a whole 64-byte piece of each,
// rather than 16 bytes of 64 records; the pieces pass through LDS to the lane
// that holds the query, which interpolates as hermite_eval32 does (the same
// arithmetic in the same order). 2-D, 1,048,576 queries: 11.4 us against
// 14.0 us for two queries a thread each loading its own records; two queries
// a lane here: 13.7 us.
__global__ __launch_bounds__(kEvalBlock) void k_grid_eval_cells32(const EvalArgs A) {
  constexpr int kRound = 65;           // float4 per wave and round: 64 pieces, + 1 so the owners' reads spread over the banks
  __shared__ float4 pieces[kEvalBlock / 64][4][kRound];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, p = lane & 3, grp = lane >> 2;
  const int64_t j = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x;
  const int64_t jq = j < A.nq ? j : A.nq - 1;      // every lane takes part in the rounds
  double s[2];
  bool finite = true, clamped = false;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    s[i] = A.q_f64 ? static_cast<const double*>(A.q)[i * A.nq + jq]
                   : (double)static_cast<const float*>(A.q)[i * A.nq + jq];
    finite = finite && isfinite(s[i]);
  }
  HermCell32<2> C;
  hermite_locate32<2>(A.K, s, C, clamped);
  const int32_t cell = hermite_cell32<2>(A.K, C);
  // record float4 p of each cell is corner p's four entries
  const float4* rec = reinterpret_cast<const float4*>(A.grid32);
  const float4 r0 = rec[(int64_t)quad_lane<0>(cell) * 4 + p], r1 = rec[(int64_t)quad_lane<1>(cell) * 4 + p];
  const float4 r2 = rec[(int64_t)quad_lane<2>(cell) * 4 + p], r3 = rec[(int64_t)quad_lane<3>(cell) * 4 + p];
  pieces[wave][0][4 * grp + p] = r0;
  pieces[wave][1][4 * grp + p] = r1;
  pieces[wave][2][4 * grp + p] = r2;
  pieces[wave][3][4 * grp + p] = r3;
  __syncthreads();
  float4 own[4];                       // this lane's query was fetched in round p
#pragma unroll
  for (int v = 0; v < 4; ++v) own[v] = pieces[wave][p][4 * grp + v];
  float Mf[16];
  hermite_unpack32<2>(own, Mf);
  double h, dh[2];
  hermite_contract32<2>(C, Mf, h, dh);
  if (j < A.nq) store_query<2>(A, j, h, dh, clamped, finite);
}

// 2-D interpolation from the FP64 node arrays (four doubles, 32 bytes, a
// node), the four nodes of a query fetched by groups of four lanes: in round
// r the group reads the two rows of the cell of the query that its lane r
// holds, 64 contiguous bytes each (two adjacent nodes), lane p taking the
// p-th 16 bytes of each row; a load instruction then reaches 16 node pairs,
// mostly one line each, rather than 16 bytes of 64 scattered nodes. The pieces
// pass through LDS to the lane that holds the query, which interpolates as
// hermite_eval does. 2-D, 1,048,576 queries: 19.5 us against 23.0 us for
// four queries a thread each loading its own nodes.
__global__ __launch_bounds__(kEvalBlock) void k_grid_eval_nodes64(const EvalArgs A) {
  constexpr int kRound = 129;          // double2 per wave and round: 128 pieces, + 1 so the owners' reads spread over the banks
  __shared__ double2 pieces[kEvalBlock / 64][4][kRound];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, p = lane & 3, grp = lane >> 2;
  const int64_t j = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x;
  const int64_t jq = j < A.nq ? j : A.nq - 1;      // every lane takes part in the rounds
  double s[2];
  bool finite = true, clamped = false;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    s[i] = A.q_f64 ? static_cast<const double*>(A.q)[i * A.nq + jq]
                   : (double)static_cast<const float*>(A.q)[i * A.nq + jq];
    finite = finite && isfinite(s[i]);
  }
  HermCell<2> C;
  hermite_locate<2>(A.K, s, C, clamped);
  int32_t nd[4];                       // corner c's node (bit 0: upper x end, bit 1: upper y end)
#pragma unroll
  for (int c = 0; c < 4; ++c) nd[c] = (int32_t)hermite_node<2>(A.K, C, c);
  const double2* g2 = reinterpret_cast<const double2*>(A.grid);
  // round r: this lane's node in each row of the cell of lane r's query (the
  // broadcasts run in every lane, before any lane-dependent choice)
  int32_t b0[4], b1[4], b2[4], b3[4];
  quad_lanes<0>(nd, b0);
  quad_lanes<1>(nd, b1);
  quad_lanes<2>(nd, b2);
  quad_lanes<3>(nd, b3);
  const bool upper_x = (p >> 1) != 0;
  const int32_t l0 = upper_x ? b0[1] : b0[0], u0 = upper_x ? b0[3] : b0[2];
  const int32_t l1 = upper_x ? b1[1] : b1[0], u1 = upper_x ? b1[3] : b1[2];
  const int32_t l2 = upper_x ? b2[1] : b2[0], u2 = upper_x ? b2[3] : b2[2];
  const int32_t l3 = upper_x ? b3[1] : b3[0], u3 = upper_x ? b3[3] : b3[2];
  const int half = p & 1;
  const double2 gl0 = g2[(int64_t)l0 * 2 + half], gu0 = g2[(int64_t)u0 * 2 + half];
  const double2 gl1 = g2[(int64_t)l1 * 2 + half], gu1 = g2[(int64_t)u1 * 2 + half];
  const double2 gl2 = g2[(int64_t)l2 * 2 + half], gu2 = g2[(int64_t)u2 * 2 + half];
  const double2 gl3 = g2[(int64_t)l3 * 2 + half], gu3 = g2[(int64_t)u3 * 2 + half];
  pieces[wave][0][8 * grp + p] = gl0;
  pieces[wave][0][8 * grp + 4 + p] = gu0;
  pieces[wave][1][8 * grp + p] = gl1;
  pieces[wave][1][8 * grp + 4 + p] = gu1;
  pieces[wave][2][8 * grp + p] = gl2;
  pieces[wave][2][8 * grp + 4 + p] = gu2;
  pieces[wave][3][8 * grp + p] = gl3;
  pieces[wave][3][8 * grp + 4 + p] = gu3;
  __syncthreads();
  // this lane's query was fetched in round p; piece 2 c + half holds corner
  // c's entries 2 half and 2 half + 1
  double Hc[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const double2 v = pieces[wave][p][8 * grp + 2 * c + half];
      Hc[c][2 * half] = v.x;
      Hc[c][2 * half + 1] = v.y;
    }
  double h, dh[2];
  hermite_contract<2>(C, Hc, h, dh);
  if (j < A.nq) store_query<2>(A, j, h, dh, clamped, finite);
}

template <int D>
int64_t tiles_of(const Consts& K) {
  constexpr int TX = 64 * kCols, TY = 4 * kRY;
  int64_t t = ((K.grid_n[0] + TX - 1) / TX) * ((K.grid_n[1] + TY - 1) / TY);
  if (D == 3) t *= K.grid_n[2];
  return t;
}

bool uses_mfma(const Consts& K) { return K.ndim >= 2 && K.kernel == ABP_K_GAUSS; }

// Tiles of the deposit launch for this grid (each kernel's own tile shape).
int64_t node_tiles(const Consts& K) {
  if (K.ndim == 1) return (K.grid_n[0] + kBlock - 1) / kBlock;
  if (uses_mfma(K)) {
    const int64_t tx = (K.grid_n[0] + kMT - 1) / kMT;
    if (K.ndim == 3) return tx * ((K.grid_n[1] + kMT3Y - 1) / kMT3Y) * K.grid_n[2];
    return tx * ((K.grid_n[1] + kMT - 1) / kMT);
  }
  return K.ndim == 3 ? tiles_of<3>(K) : tiles_of<2>(K);
}

// Hill sub-ranges of one deposit, at most: the scratch holds this many partial
// grids. 16 keeps it at 16 grids (32 MiB for 256^2 x 4 FP64) with the 50k-hill
// 256^2 deposit within 2% of the time at 64 (0.667 against 0.658 ms).
constexpr int64_t kMaxSplit = 16;

int split_for(const Consts& K, int64_t nhills) {
  const int64_t tiles = node_tiles(K);
  const int64_t want = uses_mfma(K) ? kMinWaves : kMinBlocks;
  int64_t s = (want + tiles - 1) / tiles;
  const int64_t by_hills = nhills / 256;       // at least 256 hills per sub-range
  if (s > by_hills) s = by_hills;
  if (s < 1) s = 1;
  if (s > kMaxSplit) s = kMaxSplit;
  return (int)s;
}

}  // namespace

size_t grid_deposit_scratch_bytes(const Consts& K, int64_t nhills) {
  const int s = split_for(K, nhills);
  if (s <= 1) return 0;
  return (size_t)s * (size_t)K.nodes * ((size_t)1 << K.ndim) * sizeof(double);
}

size_t grid_dirty_tiles(const Consts& K) {
  if (K.nodes <= 0 || K.ndim < 2 || uses_mfma(K)) return 0;
  return (size_t)node_tiles(K);
}

hipError_t launch_grid_deposit(const Consts& K, const HistView& H, int64_t k0, int64_t k1,
                               double* grid, double* scratch, uint32_t* dirty, uint32_t epoch,
                               hipStream_t stream) {
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
  A.dirty = grid_dirty_tiles(K) ? dirty : nullptr;
  A.epoch = epoch;
  const unsigned blocks = (unsigned)(A.tiles * A.nsplit);
  switch (K.ndim) {
    case 1: hipLaunchKernelGGL(k_deposit_1d, dim3(blocks), dim3(kBlock), 0, stream, A); break;
    case 2:
      if (uses_mfma(K)) {
        const int pm = (K.periodic[0] ? 1 : 0) | (K.periodic[1] ? 2 : 0);
        if (pm == 0) hipLaunchKernelGGL(k_deposit_mfma2<0>, dim3(blocks), dim3(64), 0, stream, A);
        else if (pm == 1) hipLaunchKernelGGL(k_deposit_mfma2<1>, dim3(blocks), dim3(64), 0, stream, A);
        else if (pm == 2) hipLaunchKernelGGL(k_deposit_mfma2<2>, dim3(blocks), dim3(64), 0, stream, A);
        else hipLaunchKernelGGL(k_deposit_mfma2<3>, dim3(blocks), dim3(64), 0, stream, A);
      }
      else hipLaunchKernelGGL(k_deposit_nd<2>, dim3(blocks), dim3(kBlock), 0, stream, A);
      break;
    case 3:
      if (uses_mfma(K)) {
        const int pm = (K.periodic[0] ? 1 : 0) | (K.periodic[1] ? 2 : 0) | (K.periodic[2] ? 4 : 0);
        switch (pm) {
          case 0: hipLaunchKernelGGL(k_deposit_mfma3<0>, dim3(blocks), dim3(64), 0, stream, A); break;
          case 1: hipLaunchKernelGGL(k_deposit_mfma3<1>, dim3(blocks), dim3(64), 0, stream, A); break;
          case 2: hipLaunchKernelGGL(k_deposit_mfma3<2>, dim3(blocks), dim3(64), 0, stream, A); break;
          case 3: hipLaunchKernelGGL(k_deposit_mfma3<3>, dim3(blocks), dim3(64), 0, stream, A); break;
          case 4: hipLaunchKernelGGL(k_deposit_mfma3<4>, dim3(blocks), dim3(64), 0, stream, A); break;
          case 5: hipLaunchKernelGGL(k_deposit_mfma3<5>, dim3(blocks), dim3(64), 0, stream, A); break;
          case 6: hipLaunchKernelGGL(k_deposit_mfma3<6>, dim3(blocks), dim3(64), 0, stream, A); break;
          default: hipLaunchKernelGGL(k_deposit_mfma3<7>, dim3(blocks), dim3(64), 0, stream, A); break;
        }
      } else {
        hipLaunchKernelGGL(k_deposit_nd<3>, dim3(blocks), dim3(kBlock), 0, stream, A);
      }
      break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || A.nsplit == 1) return e;
  const int64_t nvals = K.nodes << K.ndim;
  hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((nvals + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     stream, grid, (const double*)scratch, nvals, A.nsplit);
  return hipGetLastError();
}

hipError_t launch_grid_eval(const Consts& K, const double* grid, const float* grid32, int64_t nq, int q_f64,
                            const void* q, void* V, void* dVds, unsigned long long* n_clamped,
                            hipStream_t stream) {
  if (nq <= 0) return hipSuccess;
  if (nq > (int64_t)INT32_MAX * kEvalBlock) return hipErrorInvalidValue;   // more blocks than a launch can have
  EvalArgs A;
  A.K = K;
  A.grid = grid;
  A.grid32 = grid32;
  A.nq = nq;
  A.q = q;
  A.V = V;
  A.dV = dVds;
  A.q_f64 = q_f64;
  A.n_clamped = n_clamped;
  auto blocks = [nq](int qp) { return (unsigned)((nq + (int64_t)kBlock * qp - 1) / ((int64_t)kBlock * qp)); };
  const dim3 t(kBlock);
  switch (K.ndim * 2 + (grid32 ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_grid_eval<1, double>), dim3(blocks(EvalQ<1, double>::value)), t, 0, stream, A); break;
    case 3: hipLaunchKernelGGL((k_grid_eval<1, float>), dim3(blocks(EvalQ<1, float>::value)), t, 0, stream, A); break;
    case 4:
      if (K.quant || K.nodes >= ((int64_t)1 << 31))
        hipLaunchKernelGGL((k_grid_eval<2, double>), dim3(blocks(EvalQ<2, double>::value)), t, 0, stream, A);
      else hipLaunchKernelGGL(k_grid_eval_nodes64, dim3((unsigned)((nq + kEvalBlock - 1) / kEvalBlock)), dim3(kEvalBlock), 0, stream, A);
      break;
    case 5:
      if (K.quant) hipLaunchKernelGGL((k_grid_eval<2, float>), dim3(blocks(EvalQ<2, float>::value)), t, 0, stream, A);
      else hipLaunchKernelGGL(k_grid_eval_cells32, dim3((unsigned)((nq + kEvalBlock - 1) / kEvalBlock)), dim3(kEvalBlock), 0, stream, A);
      break;
    case 6: hipLaunchKernelGGL((k_grid_eval<3, double>), dim3(blocks(EvalQ<3, double>::value)), t, 0, stream, A); break;
    case 7: hipLaunchKernelGGL((k_grid_eval<3, float>), dim3(blocks(EvalQ<3, float>::value)), t, 0, stream, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {
// Node-major mirror (3-D): entry for entry.
// A node's tile in the VALU deposit's tiling (64 x 32 nodes, one z plane).
__device__ __forceinline__ int64_t deposit_tile(const Consts& K, int64_t j0, int64_t j1, int64_t j2) {
  constexpr int TX = 64 * kCols, TY = 4 * kRY;
  const int64_t tiles_x = (K.grid_n[0] + TX - 1) / TX, tiles_y = (K.grid_n[1] + TY - 1) / TY;
  return j0 / TX + tiles_x * (j1 / TY + tiles_y * j2);
}

__global__ __launch_bounds__(kBlock) void k_grid_mirror_nodes(const Consts K, const double* __restrict__ grid,
                                                               float* __restrict__ g32, int64_t n,
                                                               const uint32_t* __restrict__ dirty, uint32_t epoch) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    if (dirty) {
      const int64_t node = i >> 3;                   // 8 entries per 3-D node
      const int64_t n0 = K.grid_n[0], n1 = K.grid_n[1];
      if (dirty[deposit_tile(K, node % n0, (node / n0) % n1, node / (n0 * n1))] != epoch) continue;
    }
    g32[i] = (float)grid[i];
  }
}

// Cell-major mirror (1-D, 2-D): one thread per (cell, corner) writes that
// corner's 2^D entries. Cells past a non-periodic axis's last node repeat
// the last node (never read).
template <int D>
__global__ __launch_bounds__(kBlock) void k_grid_mirror_cells(const Consts K, const double* __restrict__ grid,
                                                               float* __restrict__ g32,
                                                               const uint32_t* __restrict__ dirty, uint32_t epoch) {
  constexpr int NM = 1 << D;
  const int64_t n0 = K.grid_n[0], n1 = D > 1 ? K.grid_n[1] : 1;
  const int64_t total = n0 * n1 * NM;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int corner = (int)(i % NM);
    const int64_t cell = i / NM;
    int64_t j[2] = {cell % n0, cell / n0};
    const int64_t n[2] = {n0, n1};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if ((corner >> a) & 1) {
        j[a] += 1;
        if (j[a] == n[a]) j[a] = K.periodic[a] ? 0 : n[a] - 1;
      }
    }
    if (D > 1 && dirty && dirty[deposit_tile(K, j[0], j[1], 0)] != epoch) continue;   // source node unchanged
    const double* src = grid + (j[0] + (D > 1 ? j[1] * n0 : 0)) * NM;
    float* dst = g32 + i * NM;
#pragma unroll
    for (int m = 0; m < NM; ++m) dst[m] = (float)src[m];
  }
}
}  // namespace

size_t grid_mirror_floats(const Consts& K) {
  if (K.nodes <= 0) return 0;
  const size_t nm = (size_t)1 << K.ndim;
  return K.ndim <= 2 ? (size_t)K.nodes * nm * nm : (size_t)K.nodes * nm;
}

hipError_t launch_grid_mirror(const Consts& K, const double* grid, float* grid32, const uint32_t* dirty,
                              uint32_t epoch, hipStream_t stream) {
  if (K.nodes <= 0) return hipSuccess;
  if (!grid_dirty_tiles(K)) dirty = nullptr;           // matrix-core deposits reach every tile
  const int64_t n = (int64_t)grid_mirror_floats(K) / (K.ndim <= 2 ? (1 << K.ndim) : 1);
  const unsigned blocks = (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
  if (K.ndim == 1)
    hipLaunchKernelGGL(k_grid_mirror_cells<1>, dim3(blocks), dim3(kBlock), 0, stream, K, grid, grid32, nullptr, 0u);
  else if (K.ndim == 2)
    hipLaunchKernelGGL(k_grid_mirror_cells<2>, dim3(blocks), dim3(kBlock), 0, stream, K, grid, grid32, dirty, epoch);
  else hipLaunchKernelGGL(k_grid_mirror_nodes, dim3(blocks), dim3(kBlock), 0, stream, K, grid, grid32, n, dirty, epoch);
  return hipGetLastError();
}

}  // namespace abp

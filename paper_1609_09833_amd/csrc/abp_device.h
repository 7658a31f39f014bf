// Device-side helpers shared by the libabp kernels: working-form conversion
// of CV coordinates, the per-hill arithmetic of the direct sum, compensated
// accumulation, the bias transform and cubic Hermite interpolation.
#pragma once

#include "abp_internal.h"

namespace abp {

constexpr float kTinyGap = 0x1p-40f;   // floor of 1 - (delta/a)^2 in the FP32 compact kernel

// ---------------------------------------------------------------------------
// Working form of one CV coordinate (FP32 path): a 32-bit fixed-point word.
// Periodic axis: fraction of the period, so the unsigned difference of two
// words is the minimum-image displacement mod 2^32. Non-periodic axis: signed
// offset from the window's middle, clamped to +-kFixLimit (the window's edge),
// so the difference of two words never wraps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t work32(const Consts& K, int axis, double s) {
  if (K.periodic[axis]) {
    double t = (s - K.lo[axis]) * K.inv_period[axis];
    t -= floor(t);
    return (uint32_t)(uint64_t)rint(t * 4294967296.0);
  }
  const double t = rint((s - K.fix_mid[axis]) * K.fix_scale[axis]);
  return (uint32_t)(int32_t)fmin(fmax(t, -kFixLimit), kFixLimit);
}

// Working form in the FP64 path: turns on periodic axes (wrapped later).
__device__ __forceinline__ double work64(const Consts& K, int axis, double s) {
  return K.periodic[axis] ? (s - K.lo[axis]) * K.inv_period[axis] : s;
}

// Nearest grid node of x on one axis (the quantised mode): node index
// floor((x - lo)/dx + 1/2), mod n on a periodic axis, clamped to [0, n-1]
// otherwise; snap_coord returns the node's coordinate lo + j dx.
__device__ __forceinline__ double snap_index(const Consts& K, int axis, double x) {
  const double n = (double)K.grid_n[axis];
  double t = floor((x - K.lo[axis]) / K.grid_dx[axis] + 0.5);
  if (!isfinite(t)) t = 0.0;
  if (K.periodic[axis]) t -= n * floor(t / n);
  return fmin(fmax(t, 0.0), n - 1.0);   // (the periodic remainder is already in range)
}

// lo + j dx with two roundings, as written: contracting it into one fused
// multiply-add would move nodes by an ulp wherever lo is not 0.
__device__ __forceinline__ double snap_coord(const Consts& K, int axis, double x) {
#pragma clang fp contract(off)
  const double p = snap_index(K, axis, x) * K.grid_dx[axis];
  return K.lo[axis] + p;
}

// The coordinate a sum or deposit uses: x itself, or its node when quantised.
__device__ __forceinline__ double eval_coord(const Consts& K, int axis, double x) {
  return K.quant ? snap_coord(K, axis, x) : x;
}

__device__ __forceinline__ uint32_t rec_word(const int4& h, int i) {
  return (uint32_t)(i == 0 ? h.x : (i == 1 ? h.y : h.z));
}

// ---------------------------------------------------------------------------
// One hill against one query, FP32 (both working forms are fixed point, so
// PMASK does not change the arithmetic). P[0] += w K; P[1+i] += w K * f_i where
// f_i is the working displacement (Gaussian) or u/(1-u^2)^2 (compact); the
// epilogue multiplies by the per-axis gradient scale. The height enters as
// log2(w) in the exponent, so w K costs no separate multiply.
// ISO: every axis has the same exponent factor kf[0], so the squared
//      displacements are summed first and scaled once.
// FIRST: the pair opens a new partial sum (P is assigned, not accumulated).
// ---------------------------------------------------------------------------
template <int D, int PMASK, int KERN, bool ISO = false, bool FIRST = false>
__device__ __forceinline__ void pair32(const uint32_t (&qw)[D], const int4& h, const float (&kf)[D],
                                       const float (&ua)[D], float pl, float (&P)[D + 1]) {
  float a = __int_as_float(h.w);
  float d[D];
#pragma unroll
  for (int i = 0; i < D; ++i) d[i] = (float)(int32_t)(qw[i] - rec_word(h, i));   // exact integer difference
  float f[D];
  if (KERN == ABP_K_GAUSS) {
    if (ISO) {
      float t = d[0] * d[0];
#pragma unroll
      for (int i = 1; i < D; ++i) t = __builtin_fmaf(d[i], d[i], t);
      a = __builtin_fmaf(-kf[0], t, a);
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) a = __builtin_fmaf(-d[i] * kf[i], d[i], a);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) f[i] = d[i];
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      float u = d[i] * ua[i];
      u = __builtin_fminf(__builtin_fmaxf(u, -2.0f), 2.0f);
      const float t = u * u;
      const float r = __builtin_amdgcn_rcpf(__builtin_fmaxf(1.0f - t, kTinyGap));
      a = __builtin_fmaf(-pl, t * r, a);
      f[i] = u * r * r;
    }
  }
  const float e = __builtin_amdgcn_exp2f(a);
  if (FIRST) {
    P[0] = e;
#pragma unroll
    for (int i = 0; i < D; ++i) P[i + 1] = e * f[i];
  } else {
    P[0] += e;
#pragma unroll
    for (int i = 0; i < D; ++i) P[i + 1] = __builtin_fmaf(e, f[i], P[i + 1]);
  }
}

// Kahan step: fold a plainly summed chunk P into the compensated sum (S, C),
// C carrying the rounding error of S with the opposite sign. P is left as is
// (the next chunk overwrites it).
template <int N>
__device__ __forceinline__ void kahan_fold(float (&S)[N], float (&C)[N], const float (&P)[N]) {
#pragma unroll
  for (int r = 0; r < N; ++r) {
    const float y = P[r] - C[r];
    const float t = S[r] + y;
    C[r] = (t - S[r]) - y;
    S[r] = t;
  }
}

// log2 of a hill height as the FP64 sums read it (heights are finite and >= 0).
__device__ __forceinline__ double log2_height(double w) { return w > 0.0 ? log2(w) : kLog2Zero; }

// 2^x for the FP64 hill terms: x = k + r with k = rint(x), |r| <= 1/2
// (exact); 2^r from the degree-11 Chebyshev interpolant of 2^r on
// [-1/2, 1/2] in the monomial basis (relative error below 5e-18 before
// rounding; csrc/exp2_poly.py computes the coefficients), then scaled by 2^k.
// x is clamped below at -1100, where the result is already exactly 0, so a
// -inf argument (an infinitely distant hill) also gives 0. x is never above
// log2 of the largest height (< 1024), so k fits an int. A NaN argument is
// not propagated; the kernels mark results for non-finite queries themselves.
constexpr double kExp2Poly[12] = {1.0, 0.6931471805599453, 0.2402265069591016, 0.05550410866482084,
                                  0.00961812910758714, 0.0013333558146525846, 0.00015403530463787193,
                                  1.5252733768382024e-05, 1.3215432523120778e-06, 1.0178076233676354e-07,
                                  7.074195451650667e-09, 4.454084508627905e-10};

__device__ __forceinline__ double exp2_term(double x) {
  x = fmax(x, -1100.0);
  const double k = rint(x);
  const double r = x - k;
  double p = kExp2Poly[11];
#pragma unroll
  for (int n = 10; n >= 0; --n) p = __builtin_fma(p, r, kExp2Poly[n]);
  return ldexp(p, (int)k);
}

// One hill against one query, FP64. tq and h.x..h.z are work64 coordinates,
// h.w is log2 of the height (folded into the exponent, as in the FP32 path).
// PMASK selects the periodic axes (minimum image); ISO: every axis has the
// same exponent factor kf64[0].
template <int D, int PMASK, int KERN, bool ISO = false>
__device__ __forceinline__ void pair64(const Consts& K, const double (&tq)[D], const double4& h,
                                       double (&P)[D + 1]) {
  double d[D];
  const double hc[3] = {h.x, h.y, h.z};
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double x = tq[i] - hc[i];
    if ((PMASK >> i) & 1) x -= rint(x);       // periodic coordinates are in periods
    d[i] = x;
  }
  if (KERN == ABP_K_GAUSS) {
    double a = h.w;
    if (ISO) {
      double t = d[0] * d[0];
#pragma unroll
      for (int i = 1; i < D; ++i) t = __builtin_fma(d[i], d[i], t);
      a = __builtin_fma(-K.kf64[0], t, a);
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) a = __builtin_fma(-d[i] * K.kf64[i], d[i], a);
    }
    const double we = exp2_term(a);
    P[0] += we;
#pragma unroll
    for (int i = 0; i < D; ++i) P[i + 1] = __builtin_fma(we, d[i], P[i + 1]);
  } else {
    double a = 0.0, f[D];
    bool inside = true;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double u = d[i] * K.ua64[i];
      const double t = u * u;
      inside = inside && (t < 1.0);
      const double r = 1.0 / (inside ? 1.0 - t : 1.0);
      a = __builtin_fma(t, r, a);
      f[i] = u * r * r;
    }
    const double we = inside ? exp2_term(__builtin_fma(-K.pl64, a, h.w)) : 0.0;
    P[0] += we;
#pragma unroll
    for (int i = 0; i < D; ++i) P[i + 1] = __builtin_fma(we, f[i], P[i + 1]);
  }
}

// ---------------------------------------------------------------------------
// Transform (eq. apfm, eq. btraj-grad) in FP64 on h and dh.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void apply_transform(const Consts& K, double h, const double (&dh)[D],
                                                double& V, double (&dV)[D]) {
  if (K.transform == ABP_T_MABP) {
    const double den = 1.0 + K.c * (1.0 - K.b) * h;
    V = K.kT * K.b / (1.0 - K.b) * log1p(K.c * (1.0 - K.b) * h);
#pragma unroll
    for (int i = 0; i < D; ++i) dV[i] = K.c * K.b * K.kT * dh[i] / den;
  } else {
    V = h;
#pragma unroll
    for (int i = 0; i < D; ++i) dV[i] = dh[i];
  }
}

// ---------------------------------------------------------------------------
// Tensor-product cubic Hermite interpolation of the FP64 node arrays
// grid[node][2^D] (value, first and mixed derivatives) at one point, in FP64.
// Returns h and the analytic gradient; *clamped is set when a non-periodic
// coordinate lay outside [lo, hi].
// ---------------------------------------------------------------------------
// Per axis: the cell (lower node j0, upper j1) and the basis along it, as
// four weights indexed a = 2 * end + datum (datum 0: value, 1: derivative).
template <int D> struct HermCell {
  int64_t j0[D], j1[D];
  double A[D][4], B[D][4];         // interpolant and its derivative d/ds_i, [2 * end + datum]
};

template <int D>
__device__ __forceinline__ void hermite_locate(const Consts& K, const double (&s)[D], HermCell<D>& C,
                                               bool& clamped) {
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int64_t n = K.grid_n[i];
    const double dx = K.grid_dx[i];
    double x = s[i], t;
    if (K.periodic[i]) {
      // wrap into one period first, so any finite coordinate lands in a cell
      double f = (x - K.lo[i]) * K.inv_period[i];
      f -= floor(f);
      if (!(f >= 0.0 && f < 1.0)) f = 0.0;          // non-finite input
      const double u = f * (double)n;
      int64_t j = (int64_t)u;
      j = j > n - 1 ? n - 1 : j;
      t = u - (double)j;
      C.j0[i] = j;
      C.j1[i] = (j + 1 == n) ? 0 : j + 1;
    } else {
      if (!(x >= K.lo[i])) { x = K.lo[i]; clamped = true; }   // also catches NaN
      if (x > K.hi[i]) { x = K.hi[i]; clamped = true; }
      const double u = (x - K.lo[i]) / dx;
      int64_t j = (int64_t)u;
      j = j > n - 2 ? n - 2 : j;
      j = j < 0 ? 0 : j;
      t = u - (double)j;
      C.j0[i] = j;
      C.j1[i] = j + 1;
    }
    const double t2 = t * t, t3 = t2 * t, idx = K.inv_grid_dx[i];
    // values of h00, h10 (times dx), h01, h11 (times dx) and their d/ds
    C.A[i][0] = 2.0 * t3 - 3.0 * t2 + 1.0;
    C.A[i][1] = (t3 - 2.0 * t2 + t) * dx;
    C.A[i][2] = -2.0 * t3 + 3.0 * t2;
    C.A[i][3] = (t3 - t2) * dx;
    C.B[i][0] = (6.0 * t2 - 6.0 * t) * idx;
    C.B[i][1] = 3.0 * t2 - 4.0 * t + 1.0;
    C.B[i][2] = (-6.0 * t2 + 6.0 * t) * idx;
    C.B[i][3] = 3.0 * t2 - 2.0 * t;
  }
}

// The node of a cell corner (bit i: upper end along axis i).
template <int D>
__device__ __forceinline__ int64_t hermite_node(const Consts& K, const HermCell<D>& C, int corner) {
  int64_t node = 0, stride = 1;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    node += (((corner >> i) & 1) ? C.j1[i] : C.j0[i]) * stride;
    stride *= K.grid_n[i];
  }
  return node;
}

__device__ __forceinline__ float fma_of(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_of(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Record entry m of corner c as its flat index in the contraction tensor
// M[a0][a1][a2], a_i = 2 * corner bit i + entry bit i.
template <int D>
__device__ __forceinline__ constexpr int hermite_slot(int corner, int m) {
  int at = 0, mul = 1;
  for (int i = 0; i < D; ++i) {
    at += (2 * ((corner >> i) & 1) + ((m >> i) & 1)) * mul;
    mul *= 4;
  }
  return at;
}

// The tensor-product sum: contract axis 0 of M with its value and derivative
// weights, then the other axes, giving the interpolant and its gradient.
template <int D, class T>
__device__ __forceinline__ void hermite_contract_axes(const T (&A)[D][4], const T (&B)[D][4],
                                                      const T (&Mf)[(1 << D) * (1 << D)], T& val, T (&g)[D]) {
  constexpr int NM = 1 << D;
  val = T(0);
#pragma unroll
  for (int k = 0; k < D; ++k) g[k] = T(0);
  if (D == 1) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      val = fma_of(A[0][a], Mf[a], val);
      g[0] = fma_of(B[0][a], Mf[a], g[0]);
    }
  } else {
    constexpr int R = NM * NM / 4;   // entries left after contracting axis 0
    T tA[R], tB[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T va = T(0), vb = T(0);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        va = fma_of(A[0][a], Mf[4 * r + a], va);
        vb = fma_of(B[0][a], Mf[4 * r + a], vb);
      }
      tA[r] = va;
      tB[r] = vb;
    }
    if (D == 2) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        val = fma_of(A[D - 1][b], tA[b], val);
        g[0] = fma_of(A[D - 1][b], tB[b], g[0]);
        g[D - 1] = fma_of(B[D - 1][b], tA[b], g[D - 1]);
      }
    } else {
      // D == 3: contract axis 1 (r = b + 4 c), then axis 2
      T uA[4], uB0[4], uB1[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T x0 = T(0), x1 = T(0), x2 = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          x0 = fma_of(A[1][b], tA[(b + 4 * c) % R], x0);
          x1 = fma_of(A[1][b], tB[(b + 4 * c) % R], x1);
          x2 = fma_of(B[1][b], tA[(b + 4 * c) % R], x2);
        }
        uA[c] = x0;
        uB0[c] = x1;
        uB1[c] = x2;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k2 = D - 1;
        val = fma_of(A[k2][c], uA[c], val);
        g[0] = fma_of(A[k2][c], uB0[c], g[0]);
        g[1 % D] = fma_of(A[k2][c], uB1[c], g[1 % D]);
        g[k2] = fma_of(B[k2][c], uA[c], g[k2]);
      }
    }
  }
}

// The corners' node values Hc[corner][entry] through the tensor basis.
template <int D>
__device__ __forceinline__ void hermite_contract(const HermCell<D>& C, const double (&Hc)[1 << D][1 << D],
                                                 double& h, double (&dh)[D]) {
  constexpr int NM = 1 << D;
  double Mf[NM * NM];
#pragma unroll
  for (int c = 0; c < NM; ++c)
#pragma unroll
    for (int m = 0; m < NM; ++m) Mf[hermite_slot<D>(c, m)] = Hc[c][m];
  hermite_contract_axes<D, double>(C.A, C.B, Mf, h, dh);
}

template <int D>
__device__ __forceinline__ void hermite_eval(const Consts& K, const double* __restrict__ grid,
                                             const double (&s)[D], double& h, double (&dh)[D],
                                             bool& clamped) {
  constexpr int NM = 1 << D;
  clamped = false;
  if (K.quant) {
    // nearest-node look-up of h and the first derivatives (no interpolation)
    int64_t node = 0, stride = 1;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      if (!K.periodic[i] && !(s[i] >= K.lo[i] && s[i] <= K.hi[i])) clamped = true;
      node += (int64_t)snap_index(K, i, s[i]) * stride;
      stride *= K.grid_n[i];
    }
    const double* src = grid + node * NM;
    h = src[0];
#pragma unroll
    for (int k = 0; k < D; ++k) dh[k] = src[1 << k];
    return;
  }
  HermCell<D> C;
  hermite_locate<D>(K, s, C, clamped);
  double Hc[NM][NM];
#pragma unroll
  for (int corner = 0; corner < NM; ++corner) {
    const double* src = grid + hermite_node<D>(K, C, corner) * NM;
#pragma unroll
    for (int m = 0; m < NM; m += 2) {
      const double2 v = *reinterpret_cast<const double2*>(src + m);
      Hc[corner][m] = v.x;
      Hc[corner][m + 1] = v.y;
    }
  }
  hermite_contract<D>(C, Hc, h, dh);
}

// ---------------------------------------------------------------------------
// The FP32 mirror of the node arrays. 1-D and 2-D grids: cell-major, cell
// (j0, j1) = the cell whose lower corner is node (j0, j1), cell index
// j0 + n0 j1, holding its 2^D corners (corner bit i: upper end on axis i,
// wrapped on periodic axes) x 2^D entries: 16 or 64 bytes, one cache line per
// query. 3-D grids (a cell record would be 256 bytes): node-major like the
// FP64 arrays. Cells past a non-periodic axis's last node are unused.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool mirror_cells(const Consts& K) { return K.ndim <= 2; }

// Offset in the mirror of entry m of node (j[0], j[1], j[2]).
__device__ __forceinline__ int64_t mirror_node_entry(const Consts& K, const int64_t* j, int m) {
  const int NM = 1 << K.ndim;
  if (!mirror_cells(K)) {
    int64_t node = 0, stride = 1;
    for (int i = 0; i < K.ndim; ++i) {
      node += j[i] * stride;
      stride *= K.grid_n[i];
    }
    return node * NM + m;
  }
  // the node is corner 0 of its own cell, or, at the last node of a
  // non-periodic axis, the upper corner of the cell below
  int64_t cell = 0, stride = 1;
  int corner = 0;
  for (int i = 0; i < K.ndim; ++i) {
    int64_t ji = j[i];
    if (!K.periodic[i] && ji == K.grid_n[i] - 1 && ji > 0) {
      ji -= 1;
      corner |= 1 << i;
    }
    cell += ji * stride;
    stride *= K.grid_n[i];
  }
  return (cell * NM + corner) * NM + m;
}

// ---------------------------------------------------------------------------
// The interpolation from the FP32 mirror, in FP32 arithmetic: the cell and
// the fraction t are located in FP64 (so t carries the query's own
// precision), the basis polynomials and the sums run in FP32. Its rounding is
// of the order of the node values' own FP32 rounding (2^-24 relative; the
// gradient, built from differences of corner values, carries 2^-24 |h| /
// spacing), an order below the interpolant's own error for grids fine enough
// to resolve the hills.
// ---------------------------------------------------------------------------
// Per axis: the cell (lower node j0, upper j1) and the basis along it, as
// four weights indexed a = 2 * end + datum (datum 0: value, 1: derivative).
template <int D> struct HermCell32 {
  int32_t j0[D], j1[D];
  float A[D][4], B[D][4];          // interpolant and its derivative d/ds_i
};

template <int D>
__device__ __forceinline__ void hermite_locate32(const Consts& K, const double (&s)[D], HermCell32<D>& C,
                                                 bool& clamped) {
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int32_t n = K.grid_n[i];
    const double dx = K.grid_dx[i];
    double x = s[i], t;
    if (K.periodic[i]) {
      double f = (x - K.lo[i]) * K.inv_period[i];
      f -= floor(f);
      if (!(f >= 0.0 && f < 1.0)) f = 0.0;          // non-finite input
      const double u = f * (double)n;
      int32_t j = (int32_t)u;
      j = j > n - 1 ? n - 1 : j;
      t = u - (double)j;
      C.j0[i] = j;
      C.j1[i] = (j + 1 == n) ? 0 : j + 1;
    } else {
      if (!(x >= K.lo[i])) { x = K.lo[i]; clamped = true; }   // also catches NaN
      if (x > K.hi[i]) { x = K.hi[i]; clamped = true; }
      const double u = (x - K.lo[i]) / dx;
      int32_t j = (int32_t)u;
      j = j > n - 2 ? n - 2 : j;
      j = j < 0 ? 0 : j;
      t = u - (double)j;
      C.j0[i] = j;
      C.j1[i] = j + 1;
    }
    const float tf = (float)t, dxf = (float)dx, idx = (float)K.inv_grid_dx[i];
    const float t2 = tf * tf, t3 = t2 * tf;
    C.A[i][0] = 2.0f * t3 - 3.0f * t2 + 1.0f;          // lower end, value
    C.A[i][1] = (t3 - 2.0f * t2 + tf) * dxf;           // lower end, derivative
    C.A[i][2] = -2.0f * t3 + 3.0f * t2;                // upper end, value
    C.A[i][3] = (t3 - t2) * dxf;                       // upper end, derivative
    C.B[i][0] = (6.0f * t2 - 6.0f * tf) * idx;
    C.B[i][1] = 3.0f * t2 - 4.0f * tf + 1.0f;
    C.B[i][2] = (-6.0f * t2 + 6.0f * tf) * idx;
    C.B[i][3] = 3.0f * t2 - 2.0f * tf;
  }
}

// The cell's record in the cell-major mirror (1-D, 2-D): 4^D floats, corner c
// (bit i: upper end along axis i) at 4^D / 2^D * c, its entry m (bit i:
// derivative along axis i) after it.
template <int D>
__device__ __forceinline__ int32_t hermite_cell32(const Consts& K, const HermCell32<D>& C) {
  static_assert(D <= 2, "cell-major records exist in 1-D and 2-D");
  int32_t cell = C.j0[0];
  if (D == 2) cell += C.j0[D - 1] * K.grid_n[0];
  return cell;
}

// A 1-D or 2-D cell record (4^D floats, as float4s) into the tensor.
template <int D>
__device__ __forceinline__ void hermite_unpack32(const float4 (&rec)[(1 << D) * (1 << D) / 4],
                                                 float (&Mf)[(1 << D) * (1 << D)]) {
  constexpr int NM = 1 << D;
#pragma unroll
  for (int v = 0; v < NM * NM / 4; ++v) {
    const float rv[4] = {rec[v].x, rec[v].y, rec[v].z, rec[v].w};
#pragma unroll
    for (int e = 0; e < 4; ++e) Mf[hermite_slot<D>((4 * v + e) / NM, (4 * v + e) % NM)] = rv[e];
  }
}

// The FP32 tensor-product sum, returned in FP64.
template <int D>
__device__ __forceinline__ void hermite_contract32(const HermCell32<D>& C, const float (&Mf)[(1 << D) * (1 << D)],
                                                   double& h, double (&dh)[D]) {
  float val, g[D];
  hermite_contract_axes<D, float>(C.A, C.B, Mf, val, g);
  h = (double)val;
#pragma unroll
  for (int k = 0; k < D; ++k) dh[k] = (double)g[k];
}

template <int D>
__device__ __forceinline__ void hermite_eval32(const Consts& K, const float* __restrict__ grid,
                                               const double (&s)[D], double& h, double (&dh)[D], bool& clamped) {
  constexpr int NM = 1 << D;
  clamped = false;
  if (K.quant) {
    int64_t j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < D; ++i) {
      if (!K.periodic[i] && !(s[i] >= K.lo[i] && s[i] <= K.hi[i])) clamped = true;
      j[i] = (int64_t)snap_index(K, i, s[i]);
    }
    h = (double)grid[mirror_node_entry(K, j, 0)];
#pragma unroll
    for (int k = 0; k < D; ++k) dh[k] = (double)grid[mirror_node_entry(K, j, 1 << k)];
    return;
  }
  HermCell32<D> C;
  hermite_locate32<D>(K, s, C, clamped);
  // the cell's data: one cell record (1-D, 2-D) or 2^D node records (3-D)
  float Mf[NM * NM];
  if constexpr (D <= 2) {
    const float4* src = reinterpret_cast<const float4*>(grid + (int64_t)hermite_cell32<D>(K, C) * (NM * NM));
    float4 rec[NM * NM / 4];
#pragma unroll
    for (int v = 0; v < NM * NM / 4; ++v) rec[v] = src[v];
    hermite_unpack32<D>(rec, Mf);
  } else {
#pragma unroll
    for (int c = 0; c < NM; ++c) {
      int64_t node = 0, stride = 1;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        node += (((c >> i) & 1) ? C.j1[i] : C.j0[i]) * stride;
        stride *= K.grid_n[i];
      }
      const float4* src = reinterpret_cast<const float4*>(grid + node * NM);
#pragma unroll
      for (int v = 0; v < NM / 4; ++v) {
        const float4 r = src[v];
        const float rv[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) Mf[hermite_slot<D>(c, 4 * v + e)] = rv[e];
      }
    }
  }
  hermite_contract32<D>(C, Mf, h, dh);
}

// ---------------------------------------------------------------------------
// Block-wide FP64 sum in a fixed order (wave butterfly, then waves in order).
// All threads of the block must call it; every thread gets the total.
// `red` is LDS scratch of at least NT/64 * N doubles (NT threads in the block).
// ---------------------------------------------------------------------------
template <int N, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
#pragma unroll
  for (int r = 0; r < N; ++r) {
    double x = v[r];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    v[r] = x;
  }
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int r = 0; r < N; ++r) red[wave * N + r] = v[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < N; ++r) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w * N + r];
    v[r] = t;
  }
  __syncthreads();
}

}  // namespace abp

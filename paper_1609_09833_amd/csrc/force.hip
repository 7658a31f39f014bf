// Fused bias-force step (bias_force) and CV evaluation (cv_compute).
//
// One block per walker does, in one launch, what the paper's bias routine
// does on the master rank each MD step (section "Minimization of
// Interprocess Communications"): gather the CV atoms, compute the CVs,
// evaluate the bias gradient at the CV value, and hand back forces on the CV
// atoms only, which are added to the engine's forces.
//
//   CVs: distance between centres of mass (FP64 accumulators), dihedral
//        angle, and the offset RMSD of section "Definition of the RMSD".
//   Bias: direct sum over the visible hills split across the block's lanes
//        (each lane: compensated FP32 or FP64 partial; lanes merged in a
//        fixed FP64 tree), or cubic Hermite interpolation of the grid.
//   Transform: eq. apfm / eq. btraj-grad.
//   Chain rule: F_j += -sum_a dV/ds_a ds_a/dx_j, list by list in a fixed
//        order; within a list atoms are distinct, so no atomics are needed.
//   Optional: write a new hill centred at the walker's CV value into a
//        reserved history slot (the deposit of eq. update at this step).
#include "abp_device.h"

namespace abp {
namespace {

struct FArgs {
  Consts K;
  HistView H;
  ForceArgs A;
  int64_t committed;
};

constexpr double kMinDist = 1e-12;      // below this COM distance the direction is undefined
constexpr double kMinCross2 = 1e-24;    // collinear torsion atoms

__device__ __forceinline__ void rmw_force(float* f, int64_t g, double add) {
  f[g] = (float)((double)f[g] + add);
}

template <int D, int PMASK, int KERN>
__global__ __launch_bounds__(kBlock) void k_bias_force(const FArgs F) {
  const ForceArgs& A = F.A;
  const Consts& K = F.K;
  const int64_t w = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double red[(kBlock / 64) * 8];
  __shared__ double sh_s[3];
  __shared__ double sh_cv[3][12];   // COM: u(3), 1/M_A, 1/M_B; TORSION: gradient (12); RMSD: 1/(N r)
  __shared__ int sh_bad;

  const int64_t base = A.atom_base[w];
  const int32_t natoms = A.n_atoms[w];
  int32_t lb[3][2], le[3][2];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int32_t* off = A.list_off + (int64_t)(a * 2 + t) * (A.nw + 1);
      lb[a][t] = off[w];
      le[a][t] = off[w + 1];
    }

  // ---- validation: lists and inputs (the walker is skipped if anything is off)
  if (tid == 0) {
    int bad = natoms < 0 ? kErrInval : 0;
    for (int a = 0; a < D; ++a) {
      const int n0 = le[a][0] - lb[a][0], n1 = le[a][1] - lb[a][1];
      if (n0 < 0 || n1 < 0 || lb[a][0] < 0 || lb[a][1] < 0) { bad |= kErrInval; continue; }
      const int kind = A.kind[a];
      if (kind == ABP_CV_COM_DIST && (n0 < 1 || n1 < 1)) bad |= kErrInval;
      if (kind == ABP_CV_TORSION) {
        if (n0 != 4 || n1 != 0) bad |= kErrInval;
        else
          for (int i = 0; i < 4; ++i)
            for (int j = 0; j < i; ++j)
              if (A.list_idx[lb[a][0] + i] == A.list_idx[lb[a][0] + j]) bad |= kErrIndex;
      }
      if (kind == ABP_CV_RMSD_OFF && (n0 < 1 || n1 != 0)) bad |= kErrInval;
    }
    sh_bad = bad;
  }
  __syncthreads();
  if (sh_bad == 0) {
    int bad = 0;
    for (int a = 0; a < D; ++a)
      for (int t = 0; t < 2; ++t)
        for (int e = lb[a][t] + tid; e < le[a][t]; e += kBlock) {
          const int32_t i = A.list_idx[e];
          if (i < 0 || i >= natoms) { bad |= kErrIndex; continue; }
          if (A.kind[a] != ABP_CV_TORSION && e > lb[a][t] && A.list_idx[e - 1] >= i) bad |= kErrIndex;
          const int64_t g = base + i;
          if (!isfinite(A.x[g]) || !isfinite(A.y[g]) || !isfinite(A.z[g]) || !isfinite(A.mass[g]))
            bad |= kErrNonfinite;
          if (A.kind[a] == ABP_CV_RMSD_OFF &&
              (!isfinite(A.ref_x[e]) || !isfinite(A.ref_y[e]) || !isfinite(A.ref_z[e])))
            bad |= kErrNonfinite;
        }
    if (bad) atomicOr(&sh_bad, bad);
  }
  __syncthreads();
  if (sh_bad) {
    if (tid == 0) atomicOr(A.err, sh_bad);
    return;
  }

  // ---- collective variables
  for (int a = 0; a < D; ++a) {
    const int kind = A.kind[a];
    if (kind == ABP_CV_COM_DIST) {
      double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int t = 0; t < 2; ++t)
        for (int e = lb[a][t] + tid; e < le[a][t]; e += kBlock) {
          const int64_t g = base + A.list_idx[e];
          const double m = A.mass[g];
          v[4 * t + 0] = __builtin_fma(m, (double)A.x[g], v[4 * t + 0]);
          v[4 * t + 1] = __builtin_fma(m, (double)A.y[g], v[4 * t + 1]);
          v[4 * t + 2] = __builtin_fma(m, (double)A.z[g], v[4 * t + 2]);
          v[4 * t + 3] += m;
        }
      block_sum<8>(v, red);
      if (!(v[3] > 0.0) || !(v[7] > 0.0)) {     // identical on every thread
        if (tid == 0) atomicOr(A.err, kErrInval);
        return;
      }
      const double r0 = v[0] / v[3] - v[4] / v[7];
      const double r1 = v[1] / v[3] - v[5] / v[7];
      const double r2 = v[2] / v[3] - v[6] / v[7];
      const double d = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
      if (tid == 0) {
        sh_s[a] = d;
        const double inv = d >= kMinDist ? 1.0 / d : 0.0;
        sh_cv[a][0] = r0 * inv;
        sh_cv[a][1] = r1 * inv;
        sh_cv[a][2] = r2 * inv;
        sh_cv[a][3] = 1.0 / v[3];
        sh_cv[a][4] = 1.0 / v[7];
      }
    } else if (kind == ABP_CV_TORSION) {
      if (tid == 0) {
        double p[4][3];
        for (int i = 0; i < 4; ++i) {
          const int64_t g = base + A.list_idx[lb[a][0] + i];
          p[i][0] = A.x[g]; p[i][1] = A.y[g]; p[i][2] = A.z[g];
        }
        double b1[3], b2[3], b3[3], n1[3], n2[3];
        for (int c = 0; c < 3; ++c) {
          b1[c] = p[1][c] - p[0][c];
          b2[c] = p[2][c] - p[1][c];
          b3[c] = p[3][c] - p[2][c];
        }
        n1[0] = b1[1] * b2[2] - b1[2] * b2[1];
        n1[1] = b1[2] * b2[0] - b1[0] * b2[2];
        n1[2] = b1[0] * b2[1] - b1[1] * b2[0];
        n2[0] = b2[1] * b3[2] - b2[2] * b3[1];
        n2[1] = b2[2] * b3[0] - b2[0] * b3[2];
        n2[2] = b2[0] * b3[1] - b2[1] * b3[0];
        const double lb2 = sqrt(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
        const double y = lb2 * (b1[0] * n2[0] + b1[1] * n2[1] + b1[2] * n2[2]);
        const double xx = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
        sh_s[a] = atan2(y, xx);
        const double nn1 = n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2];
        const double nn2 = n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2];
        if (nn1 < kMinCross2 || nn2 < kMinCross2 || lb2 == 0.0) {
          for (int t = 0; t < 12; ++t) sh_cv[a][t] = 0.0;
        } else {
          // d phi / d x_i (Blondel & Karplus 1996, in the bond vectors b1..b3)
          const double f1 = b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2];
          const double f3 = b3[0] * b2[0] + b3[1] * b2[1] + b3[2] * b2[2];
          const double g1 = lb2 / nn1, g4 = lb2 / nn2;
          const double c1 = f1 / (nn1 * lb2), c3 = f3 / (nn2 * lb2);
          for (int c = 0; c < 3; ++c) {
            sh_cv[a][0 + c] = -g1 * n1[c];
            sh_cv[a][3 + c] = (g1 + c1) * n1[c] + c3 * n2[c];
            sh_cv[a][6 + c] = -c1 * n1[c] - (g4 + c3) * n2[c];
            sh_cv[a][9 + c] = g4 * n2[c];
          }
        }
      }
    } else {   // RMSD_OFF
      double v[1] = {0.0};
      for (int e = lb[a][0] + tid; e < le[a][0]; e += kBlock) {
        const int64_t g = base + A.list_idx[e];
        const double dx = (double)A.x[g] - (double)A.ref_x[e];
        const double dy = (double)A.y[g] - (double)A.ref_y[e];
        const double dz = (double)A.z[g] - (double)A.ref_z[e];
        v[0] += dx * dx + dy * dy + dz * dz;
      }
      block_sum<1>(v, red);
      const double n = (double)(le[a][0] - lb[a][0]);
      const double r = sqrt(v[0] / n + 0.01);
      if (tid == 0) {
        sh_s[a] = r;
        sh_cv[a][0] = 1.0 / (n * r);
      }
    }
  }
  __syncthreads();
  double s[D];
#pragma unroll
  for (int a = 0; a < D; ++a) s[a] = sh_s[a];
  if (A.cv_only) {
    if (tid == 0)
      for (int a = 0; a < D; ++a) A.s[a * A.nw + w] = s[a];
    return;
  }

  // ---- bias at s
  double h, dh[D];
  if (A.use_grid) {
    if (tid == 0) {
      bool clamped;
      hermite_eval<D>(K, A.grid, s, h, dh, clamped);
      red[0] = h;
      for (int i = 0; i < D; ++i) red[1 + i] = dh[i];
    }
    __syncthreads();
    h = red[0];
#pragma unroll
    for (int i = 0; i < D; ++i) dh[i] = red[1 + i];
    __syncthreads();
  } else {
    int64_t nvis = A.n_visible ? A.n_visible[w] : A.n_visible_default;
    if (nvis < 0 || nvis > F.committed) nvis = F.committed;
    double v[D + 1];
    if (A.prec == ABP_PREC_FP64) {
      double tq[D], P[D + 1];
#pragma unroll
      for (int i = 0; i < D; ++i) tq[i] = work64(K, i, s[i]);
#pragma unroll
      for (int r = 0; r <= D; ++r) P[r] = 0.0;
      for (int64_t k = tid; k < nvis; k += kBlock) {
        double4 hr;
        hr.x = work64(K, 0, F.H.c64[k]);
        hr.y = D > 1 ? work64(K, 1, F.H.c64[F.H.capacity + k]) : 0.0;
        hr.z = D > 2 ? work64(K, 2, F.H.c64[2 * F.H.capacity + k]) : 0.0;
        hr.w = F.H.w64[k];
        pair64<D, KERN>(K, tq, hr, P);
      }
#pragma unroll
      for (int r = 0; r <= D; ++r) v[r] = P[r];
    } else {
      uint32_t qw[D];
      float kf[D], ua[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        qw[i] = work32(K, i, s[i]);
        kf[i] = K.kf32[i];
        ua[i] = K.ua32[i];
      }
      float S[D + 1], Cc[D + 1], P[D + 1];
#pragma unroll
      for (int r = 0; r <= D; ++r) { S[r] = 0.0f; Cc[r] = 0.0f; P[r] = 0.0f; }
      const bool kahan = A.prec == ABP_PREC_FP32_KAHAN;
      int64_t k = tid;
      int cnt = 0;
      for (; k < nvis; k += kBlock) {
        pair32<D, PMASK, KERN>(qw, F.H.rec32[k], kf, ua, K.pl32, P);
        if (kahan && ++cnt == kChunk) {
          kahan_fold<D + 1>(S, Cc, P);
          cnt = 0;
        }
      }
      if (kahan) {
        kahan_fold<D + 1>(S, Cc, P);
#pragma unroll
        for (int r = 0; r <= D; ++r) v[r] = (double)S[r] - (double)Cc[r];
      } else {
#pragma unroll
        for (int r = 0; r <= D; ++r) v[r] = (double)P[r];
      }
    }
    block_sum<D + 1>(v, red);
    h = v[0];
#pragma unroll
    for (int i = 0; i < D; ++i) dh[i] = v[i + 1] * (A.prec == ABP_PREC_FP64 ? K.gs64[i] : K.gs32[i]);
  }
  double V, dV[D];
  apply_transform<D>(K, h, dh, V, dV);
  if (tid == 0) {
    for (int a = 0; a < D; ++a) {
      A.s[a * A.nw + w] = s[a];
      A.dVds[a * A.nw + w] = dV[a];
    }
    A.V[w] = V;
    if (A.deposit_slot) {
      const int64_t slot = A.deposit_slot[w];
      if (slot >= 0) {
        double hw = A.deposit_height ? A.deposit_height[w] : 1.0;
        if (slot >= F.H.capacity) {
          atomicOr(A.err, kErrInval);
        } else {
          if (!isfinite(hw) || hw < 0.0) { atomicOr(A.err, kErrNonfinite); hw = 0.0; }
          uint32_t words[3] = {0u, 0u, 0u};
          for (int a = 0; a < D; ++a) {
            F.H.c64[a * F.H.capacity + slot] = s[a];
            words[a] = work32(K, a, s[a]);
          }
          F.H.w64[slot] = hw;
          int4 rec;
          rec.x = (int)words[0];
          rec.y = (int)words[1];
          rec.z = (int)words[2];
          rec.w = __float_as_int((float)log2(hw));
          F.H.rec32[slot] = rec;
        }
      }
    }
  }

  // ---- chain rule, list by list
  for (int a = 0; a < D; ++a) {
    const double g = dV[a];
    const int kind = A.kind[a];
    if (kind == ABP_CV_COM_DIST) {
      const double ux = sh_cv[a][0], uy = sh_cv[a][1], uz = sh_cv[a][2];
      for (int t = 0; t < 2; ++t) {
        const double scale = t == 0 ? -g * sh_cv[a][3] : g * sh_cv[a][4];
        for (int e = lb[a][t] + tid; e < le[a][t]; e += kBlock) {
          const int64_t gi = base + A.list_idx[e];
          const double c = scale * (double)A.mass[gi];
          rmw_force(A.fx, gi, c * ux);
          rmw_force(A.fy, gi, c * uy);
          rmw_force(A.fz, gi, c * uz);
        }
        __syncthreads();
      }
    } else if (kind == ABP_CV_TORSION) {
      if (tid < 4) {
        const int64_t gi = base + A.list_idx[lb[a][0] + tid];
        rmw_force(A.fx, gi, -g * sh_cv[a][3 * tid + 0]);
        rmw_force(A.fy, gi, -g * sh_cv[a][3 * tid + 1]);
        rmw_force(A.fz, gi, -g * sh_cv[a][3 * tid + 2]);
      }
      __syncthreads();
    } else {
      const double c = -g * sh_cv[a][0];
      for (int e = lb[a][0] + tid; e < le[a][0]; e += kBlock) {
        const int64_t gi = base + A.list_idx[e];
        rmw_force(A.fx, gi, c * ((double)A.x[gi] - (double)A.ref_x[e]));
        rmw_force(A.fy, gi, c * ((double)A.y[gi] - (double)A.ref_y[e]));
        rmw_force(A.fz, gi, c * ((double)A.z[gi] - (double)A.ref_z[e]));
      }
      __syncthreads();
    }
  }
}

template <int D, int PMASK, int KERN>
hipError_t go(const FArgs& F, hipStream_t stream) {
  hipLaunchKernelGGL((k_bias_force<D, PMASK, KERN>), dim3((unsigned)F.A.nw), dim3(kBlock), 0, stream, F);
  return hipGetLastError();
}

template <int D, int KERN>
hipError_t by_mask(int mask, const FArgs& F, hipStream_t stream) {
  switch (mask) {
    case 0: return go<D, 0, KERN>(F, stream);
    case 1: return go<D, 1, KERN>(F, stream);
    case 2: if constexpr (D >= 2) return go<D, 2, KERN>(F, stream); break;
    case 3: if constexpr (D >= 2) return go<D, 3, KERN>(F, stream); break;
    case 4: if constexpr (D >= 3) return go<D, 4, KERN>(F, stream); break;
    case 5: if constexpr (D >= 3) return go<D, 5, KERN>(F, stream); break;
    case 6: if constexpr (D >= 3) return go<D, 6, KERN>(F, stream); break;
    case 7: if constexpr (D >= 3) return go<D, 7, KERN>(F, stream); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int D>
hipError_t by_kernel(int mask, const FArgs& F, hipStream_t stream) {
  return F.K.kernel == ABP_K_GAUSS ? by_mask<D, ABP_K_GAUSS>(mask, F, stream)
                                   : by_mask<D, ABP_K_COMPACT>(mask, F, stream);
}

}  // namespace

hipError_t launch_bias_force(const Consts& K, const HistView& H, const ForceArgs& A,
                             hipStream_t stream) {
  if (A.nw <= 0) return hipSuccess;
  FArgs F;
  F.K = K;
  F.H = H;
  F.A = A;
  F.committed = A.n_visible_default;
  int mask = 0;
  for (int i = 0; i < K.ndim; ++i) mask |= (K.periodic[i] ? 1 : 0) << i;
  switch (K.ndim) {
    case 1: return by_kernel<1>(mask, F, stream);
    case 2: return by_kernel<2>(mask, F, stream);
    case 3: return by_kernel<3>(mask, F, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace abp

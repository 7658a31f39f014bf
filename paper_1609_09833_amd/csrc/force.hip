// Fused bias-force step (bias_force) and CV evaluation (cv_compute).
//
// What the paper's bias routine does on the master rank every MD step
// (section "Minimization of Interprocess Communications"): take the
// coordinates of the CV atoms, compute the CVs, evaluate the bias gradient at
// the CV value, and return forces on exactly those atoms, which are added to
// the engine's forces. Here a batch of walkers does this in one launch:
//
//   Blocks: walker w gets ceil(n_visible[w] / kHillsPerBlock) blocks (at least
//     one); each recomputes the CVs (cheap) and sums its fixed range of hills.
//     The last block to finish (atomic arrival count) merges the partial sums
//     in block order and does the rest. The hill ranges depend only on
//     n_visible[w], so a walker's result is bitwise the same alone or in any
//     batch.
//   CVs: one gather of every CV atom (index, position, mass) into registers;
//     FP64 accumulators and a fixed-order block reduction for centres of mass;
//     the dihedral angle; the offset RMSD of section "Definition of the RMSD".
//   Bias: lanes split the block's hill range; each lane sums plainly in FP32
//     in groups folded into a Kahan sum (or FP64); lanes and blocks are merged
//     with error-free FP32 transformations (TwoSum), so the merge adds no
//     rounding beyond the final one. Or cubic Hermite interpolation of the grid.
//   Transform: eq. apfm / eq. btraj-grad.
//   Chain rule: F_j += -sum_a dV/ds_a ds_a/dx_j. When the COM/RMSD lists are
//     disjoint and short (the usual ligand/pocket case), every atom's total is
//     formed in registers and written once (torsion atoms that are also
//     ligand atoms are folded into that ligand entry); otherwise lists are
//     applied one after another with a barrier between them. Either way the
//     sum per atom has a fixed order and no atomics touch the forces.
//   Optional: write a new hill centred at the walker's CV value into a
//     reserved history slot (the deposit of eq. update at this step).
#include "abp_device.h"

namespace abp {
namespace {

constexpr int kCache = 4;               // CV-list entries cached in registers per thread
constexpr int kMaxCached = kCache * kBlock;
constexpr int kMaxTors = 3;             // torsion CVs (one per axis at most)
constexpr double kMinDist = 1e-12;      // below this COM distance the direction is undefined
constexpr double kMinCross2 = 1e-24;    // collinear torsion atoms

struct FArgs {
  Consts K;
  HistView H;
  ForceArgs A;
  int64_t committed;
  int32_t nbw;                 // blocks per walker in the grid (upper bound)
  double2* partials;           // [nw][nbw][D+1] (hi, lo) per block
  unsigned int* arrivals;      // [nw], zero at rest
};

// ---- compensated FP32 pairs: value = hi + lo ------------------------------
__device__ __forceinline__ void two_sum_merge(float& h, float& l, float h2, float l2) {
  const float s = h + h2;
  const float bp = s - h;
  const float e = (h - (s - bp)) + (h2 - bp);
  const float lo = (l + l2) + e;
  const float hi = s + lo;
  l = lo - (hi - s);
  h = hi;
}

template <int N>
__device__ __forceinline__ void merge_f32(float (&h)[N], float (&l)[N], const float (&h2)[N],
                                          const float (&l2)[N], bool comp) {
#pragma unroll
  for (int r = 0; r < N; ++r) {
    if (comp) two_sum_merge(h[r], l[r], h2[r], l2[r]);
    else h[r] += h2[r];
  }
}

// Block-wide merge in a fixed tree: wave butterfly (the merge is commutative,
// so every lane ends with the same value), then waves 0..3 in order. Every
// thread gets the result. `red` holds at least kBlock/64 * N * 2 floats.
template <int N>
__device__ __forceinline__ void block_merge_f32(float (&h)[N], float (&l)[N], bool comp, float* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    float h2[N], l2[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      h2[r] = __shfl_xor(h[r], off, 64);
      l2[r] = __shfl_xor(l[r], off, 64);
    }
    merge_f32<N>(h, l, h2, l2, comp);
  }
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      red[(wave * N + r) * 2] = h[r];
      red[(wave * N + r) * 2 + 1] = l[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < N; ++r) { h[r] = red[r * 2]; l[r] = red[r * 2 + 1]; }
  for (int wv = 1; wv < kBlock / 64; ++wv) {
    float h2[N], l2[N];
#pragma unroll
    for (int r = 0; r < N; ++r) { h2[r] = red[(wv * N + r) * 2]; l2[r] = red[(wv * N + r) * 2 + 1]; }
    merge_f32<N>(h, l, h2, l2, comp);
  }
  __syncthreads();
}

__device__ __forceinline__ void rmw_force(float* f, int64_t g, double add) {
  f[g] = (float)((double)f[g] + add);
}

enum { kModeF32 = 0, kModeF64 = 1, kModeGrid = 2, kModeCV = 3 };

// MODE fixes the code path at compile time (FP32 or FP64 direct sum, grid, or
// CVs only), so each instantiation carries only the registers it needs.
template <int D, int PMASK, int KERN, int MODE>
__global__ __launch_bounds__(kBlock) void k_bias_force(const FArgs F) {
  constexpr int N = D + 1;
  const ForceArgs& A = F.A;
  const Consts& K = F.K;
  const int64_t w = blockIdx.x / F.nbw;
  const int blk = (int)(blockIdx.x % F.nbw);
  const int tid = threadIdx.x;

  // visible hills and this walker's block count (uniform per block)
  int64_t nvis = 0;
  int nb = 1;
  if (MODE == kModeF32 || MODE == kModeF64) {
    nvis = A.n_visible ? A.n_visible[w] : A.n_visible_default;
    if (nvis < 0 || nvis > F.committed) nvis = F.committed;
    nb = (int)((nvis + kHillsPerBlock - 1) / kHillsPerBlock);
    nb = nb < 1 ? 1 : nb;
  }
  if (blk >= nb) return;

  __shared__ double red[(kBlock / 64) * (9 * D + 1)];
  __shared__ double sh_s[3];
  __shared__ double sh_cv[3][12];        // COM: u(3), 1/M_A, 1/M_B; TORSION: gradient (12); RMSD: 1/(N r)
  __shared__ double sh_tpos[kMaxTors][4][3];
  __shared__ int sh_tatom[kMaxTors][4];
  __shared__ int sh_tclaimed[kMaxTors][4];
  __shared__ int sh_list[kMaxCached];    // atom indices in concatenated list order (cached entries)
  __shared__ int sh_bad, sh_last, sh_fast;
  // list q = a*2 + t: start in list_idx, length, start in the concatenated order
  __shared__ int sh_lb[6], sh_ln[6], sh_pos[7], sh_kind[3];
  __shared__ double sh_dV[3];

  const int64_t base = A.atom_base[w];
  const int32_t natoms = A.n_atoms[w];
  int ln[2 * D];                       // only indexed with compile-time constants
  int total = 0;
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) {
    const int32_t* off = A.list_off + (int64_t)q * (A.nw + 1);
    ln[q] = off[w + 1] - off[w];
    total += ln[q];
  }

  // ---- list shapes (thread 0)
  if (tid == 0) {
    int bad = natoms < 0 ? kErrInval : 0;
    int pos = 0;
    for (int q = 0; q < 2 * D; ++q) {
      const int32_t* off = A.list_off + (int64_t)q * (A.nw + 1);
      sh_lb[q] = off[w];
      sh_ln[q] = off[w + 1] - off[w];
      sh_pos[q] = pos;
      pos += sh_ln[q];
      if (sh_ln[q] < 0 || sh_lb[q] < 0) bad |= kErrInval;
    }
    sh_pos[2 * D] = pos;
    for (int a = 0; a < D; ++a) {
      const int kind = A.kind[a];
      sh_kind[a] = kind;
      const int n0 = sh_ln[2 * a], n1 = sh_ln[2 * a + 1];
      if (kind == ABP_CV_COM_DIST && (n0 < 1 || n1 < 1)) bad |= kErrInval;
      if (kind == ABP_CV_TORSION && (n0 != 4 || n1 != 0)) bad |= kErrInval;
      if (kind == ABP_CV_RMSD_OFF && (n0 < 1 || n1 != 0)) bad |= kErrInval;
    }
    sh_bad = bad;
    sh_fast = total <= kMaxCached ? 1 : 0;
    for (int t = 0; t < kMaxTors; ++t)
      for (int j = 0; j < 4; ++j) { sh_tatom[t][j] = -1; sh_tclaimed[t][j] = 0; }
  }
  __syncthreads();
  if (sh_bad) {
    if (tid == 0 && blk == 0) atomicOr(A.err, sh_bad);
    return;
  }

  // ---- one gather of every CV-list entry: validate, accumulate COM / RMSD sums
  // acc: [q*4 + c] mass-weighted x, y, z and mass of list q (COM) | [8D + a] RMSD squares | [9D] bad flag
  constexpr int NACC = 9 * D + 1;
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
  int c_gi[kCache];                   // cached entry: walker-local atom index (-1 = none)
  int c_list[kCache];                 // list id a*2+t
  int c_e[kCache];                    // position in list_idx
  float c_m[kCache];                  // mass (COM lists)
  int badbits = 0;
  // One entry r of the concatenated lists. Register arrays are only indexed
  // with compile-time constants (dynamic indices would spill them to scratch).
  auto gather = [&](int r, int& gi_out, int& li_out, int& e_out, float& mo) {
    gi_out = -1;
    int li = -1, e = 0;
#pragma unroll
    for (int q = 0; q < 2 * D; ++q)
      if (r >= sh_pos[q] && r < sh_pos[q + 1]) { li = q; e = sh_lb[q] + (r - sh_pos[q]); }
    if (li < 0) return;
    const int kind = sh_kind[li >> 1];
    const int32_t i = A.list_idx[e];
    if (i < 0 || i >= natoms) { badbits |= kErrIndex; return; }
    if (kind != ABP_CV_TORSION && e > sh_lb[li] && A.list_idx[e - 1] >= i) badbits |= kErrIndex;
    const int64_t g = base + i;
    const float x = A.x[g], y = A.y[g], z = A.z[g], m = A.mass[g];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(m)) badbits |= kErrNonfinite;
    if (kind == ABP_CV_COM_DIST) {
#pragma unroll
      for (int q = 0; q < 2 * D; ++q)
        if (li == q) {
          acc[q * 4 + 0] = __builtin_fma((double)m, (double)x, acc[q * 4 + 0]);
          acc[q * 4 + 1] = __builtin_fma((double)m, (double)y, acc[q * 4 + 1]);
          acc[q * 4 + 2] = __builtin_fma((double)m, (double)z, acc[q * 4 + 2]);
          acc[q * 4 + 3] += (double)m;
        }
    } else if (kind == ABP_CV_RMSD_OFF) {
      const float rx = A.ref_x[e], ry = A.ref_y[e], rz = A.ref_z[e];
      if (!isfinite(rx) || !isfinite(ry) || !isfinite(rz)) badbits |= kErrNonfinite;
      const double dx = (double)x - rx, dy = (double)y - ry, dz = (double)z - rz;
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (li == 2 * a) acc[8 * D + a] += dx * dx + dy * dy + dz * dz;
    } else {
      const int a = li >> 1, jt = e - sh_lb[li];
      sh_tpos[a][jt][0] = x;
      sh_tpos[a][jt][1] = y;
      sh_tpos[a][jt][2] = z;
      sh_tatom[a][jt] = i;
    }
    if (r < kMaxCached) sh_list[r] = i;
    gi_out = i; li_out = li; e_out = e;
    mo = m;
  };
#pragma unroll
  for (int k = 0; k < kCache; ++k) {
    c_gi[k] = -1;
    c_list[k] = 0; c_e[k] = 0;
    c_m[k] = 0.0f;
    const int r = k * kBlock + tid;
    if (r < total) gather(r, c_gi[k], c_list[k], c_e[k], c_m[k]);
  }
  for (int r = kMaxCached + tid; r < total; r += kBlock) {
    int gi, li, e;
    float m;
    gather(r, gi, li, e, m);
  }
  if (badbits) atomicOr(&sh_bad, badbits);
  acc[9 * D] = badbits ? 1.0 : 0.0;
  block_sum<NACC>(acc, red);         // its barriers also publish sh_bad and the torsion atoms
  if (acc[9 * D] != 0.0) {
    if (tid == 0 && blk == 0) atomicOr(A.err, sh_bad ? sh_bad : kErrIndex);
    return;
  }

  // ---- CV values (thread 0; every block of the walker computes them identically)
  if (tid == 0) {
    for (int a = 0; a < D; ++a) {
      const int kind = A.kind[a];
      if (kind == ABP_CV_COM_DIST) {
        const double* pa = acc + (a * 2) * 4;
        const double* pb = acc + (a * 2 + 1) * 4;
        if (!(pa[3] > 0.0) || !(pb[3] > 0.0)) { sh_bad = kErrInval; continue; }
        const double r0 = pa[0] / pa[3] - pb[0] / pb[3];
        const double r1 = pa[1] / pa[3] - pb[1] / pb[3];
        const double r2 = pa[2] / pa[3] - pb[2] / pb[3];
        const double d = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
        sh_s[a] = d;
        const double inv = d >= kMinDist ? 1.0 / d : 0.0;
        sh_cv[a][0] = r0 * inv;
        sh_cv[a][1] = r1 * inv;
        sh_cv[a][2] = r2 * inv;
        sh_cv[a][3] = 1.0 / pa[3];
        sh_cv[a][4] = 1.0 / pb[3];
      } else if (kind == ABP_CV_RMSD_OFF) {
        const double n = (double)sh_ln[2 * a];
        const double r = sqrt(acc[8 * D + a] / n + 0.01);
        sh_s[a] = r;
        sh_cv[a][0] = 1.0 / (n * r);
      } else {
        const int* ta = sh_tatom[a];
        if (ta[0] == ta[1] || ta[0] == ta[2] || ta[0] == ta[3] || ta[1] == ta[2] || ta[1] == ta[3] ||
            ta[2] == ta[3]) { sh_bad = kErrIndex; continue; }
        double b1[3], b2[3], b3[3], n1[3], n2[3];
        for (int c = 0; c < 3; ++c) {
          b1[c] = sh_tpos[a][1][c] - sh_tpos[a][0][c];
          b2[c] = sh_tpos[a][2][c] - sh_tpos[a][1][c];
          b3[c] = sh_tpos[a][3][c] - sh_tpos[a][2][c];
        }
        n1[0] = b1[1] * b2[2] - b1[2] * b2[1];
        n1[1] = b1[2] * b2[0] - b1[0] * b2[2];
        n1[2] = b1[0] * b2[1] - b1[1] * b2[0];
        n2[0] = b2[1] * b3[2] - b2[2] * b3[1];
        n2[1] = b2[2] * b3[0] - b2[0] * b3[2];
        n2[2] = b2[0] * b3[1] - b2[1] * b3[0];
        const double lb2 = sqrt(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
        const double yv = lb2 * (b1[0] * n2[0] + b1[1] * n2[1] + b1[2] * n2[2]);
        const double xv = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
        sh_s[a] = atan2(yv, xv);
        const double nn1 = n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2];
        const double nn2 = n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2];
        if (nn1 < kMinCross2 || nn2 < kMinCross2 || lb2 == 0.0) {
          for (int q = 0; q < 12; ++q) sh_cv[a][q] = 0.0;
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
    }
  }
  __syncthreads();
  if (sh_bad) {
    if (tid == 0 && blk == 0) atomicOr(A.err, sh_bad);
    return;
  }
  double s[D];
#pragma unroll
  for (int a = 0; a < D; ++a) s[a] = sh_s[a];
  if (MODE == kModeCV) {
    if (tid == 0)
      for (int a = 0; a < D; ++a) A.s[a * A.nw + w] = s[a];
    return;
  }

  // ---- bias at s
  double h = 0.0, dh[D];
  if (MODE == kModeGrid) {
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
    const int64_t k0 = (int64_t)blk * kHillsPerBlock;
    const int64_t k1 = nvis < k0 + kHillsPerBlock ? nvis : k0 + kHillsPerBlock;
    float hi[N], lo[N];
    double v64[N];
    constexpr bool fp64 = MODE == kModeF64;
    const bool comp = A.prec == ABP_PREC_FP32_KAHAN;
    if constexpr (fp64) {
      double tq[D], P[N];
#pragma unroll
      for (int i = 0; i < D; ++i) tq[i] = work64(K, i, s[i]);
#pragma unroll
      for (int r = 0; r < N; ++r) P[r] = 0.0;
      for (int64_t k = k0 + tid; k < k1; k += kBlock) {
        double4 hr;
        hr.x = work64(K, 0, F.H.c64[k]);
        hr.y = D > 1 ? work64(K, 1, F.H.c64[F.H.capacity + k]) : 0.0;
        hr.z = D > 2 ? work64(K, 2, F.H.c64[2 * F.H.capacity + k]) : 0.0;
        hr.w = F.H.w64[k];
        pair64<D, KERN>(K, tq, hr, P);
      }
#pragma unroll
      for (int r = 0; r < N; ++r) v64[r] = P[r];
      block_sum<N>(v64, red);
#pragma unroll
      for (int r = 0; r < N; ++r) { hi[r] = 0.0f; lo[r] = 0.0f; }
    } else {
      uint32_t qw[D];
      float kf[D], ua[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        qw[i] = work32(K, i, s[i]);
        kf[i] = K.kf32[i];
        ua[i] = K.ua32[i];
      }
      float S[N], Cc[N], P[N];
#pragma unroll
      for (int r = 0; r < N; ++r) { S[r] = 0.0f; Cc[r] = 0.0f; P[r] = 0.0f; }
      constexpr int kU = 4;                       // records in flight per lane, summed plainly then folded
      const int4 none = make_int4(0, 0, 0, __float_as_int(-__builtin_inff()));
      for (int64_t kb = k0 + tid; kb < k1; kb += kBlock * kU) {
        int4 rec[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int64_t k = kb + (int64_t)u * kBlock;
          rec[u] = k < k1 ? F.H.rec32[k] : none;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) pair32<D, PMASK, KERN>(qw, rec[u], kf, ua, K.pl32, P);
        if (comp) {
          kahan_fold<N>(S, Cc, P);
#pragma unroll
          for (int r = 0; r < N; ++r) P[r] = 0.0f;
        }
      }
#pragma unroll
      for (int r = 0; r < N; ++r) {
        hi[r] = comp ? S[r] : P[r];
        lo[r] = comp ? -Cc[r] : 0.0f;
      }
      block_merge_f32<N>(hi, lo, comp, reinterpret_cast<float*>(red));
#pragma unroll
      for (int r = 0; r < N; ++r) v64[r] = 0.0;
    }
    // this block's partial -> merged in block order by the last block to arrive
    if (nb > 1) {
      double2* mine = F.partials + ((int64_t)w * F.nbw + blk) * N;
      if (tid < N) {
        double2 pv;
        pv.x = fp64 ? v64[tid] : (double)hi[tid];
        pv.y = fp64 ? 0.0 : (double)lo[tid];
        mine[tid] = pv;
      }
      __threadfence();
      __syncthreads();
      if (tid == 0) {
        const unsigned prev = atomicAdd(F.arrivals + w, 1u);
        sh_last = prev == (unsigned)(nb - 1) ? 1 : 0;
        if (sh_last) atomicExch(F.arrivals + w, 0u);   // at rest again for the next launch
      }
      __syncthreads();
      if (!sh_last) return;
      __threadfence();
      const double2* all = F.partials + (int64_t)w * F.nbw * N;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const double2 p0 = all[r];
        if (fp64) {
          v64[r] = p0.x;
        } else {
          hi[r] = (float)p0.x;
          lo[r] = (float)p0.y;
        }
      }
      for (int q = 1; q < nb; ++q) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
          const double2 pq = all[(int64_t)q * N + r];
          if (fp64) {
            v64[r] += pq.x;
          } else {
            const float h2[1] = {(float)pq.x}, l2[1] = {(float)pq.y};
            float h1[1] = {hi[r]}, l1[1] = {lo[r]};
            merge_f32<1>(h1, l1, h2, l2, comp);
            hi[r] = h1[0];
            lo[r] = l1[0];
          }
        }
      }
    }
    double tot[N];
#pragma unroll
    for (int r = 0; r < N; ++r) tot[r] = fp64 ? v64[r] : (double)hi[r] + (double)lo[r];
    h = tot[0];
#pragma unroll
    for (int i = 0; i < D; ++i) dh[i] = tot[i + 1] * (fp64 ? K.gs64[i] : K.gs32[i]);
  }
  double V, dV[D];
  apply_transform<D>(K, h, dh, V, dV);
  if (tid == 0) {
    for (int a = 0; a < D; ++a) {
      A.s[a * A.nw + w] = s[a];
      A.dVds[a * A.nw + w] = dV[a];
      sh_dV[a] = dV[a];
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

  // ---- chain rule
  // Fast path: every list entry is cached and no atom appears in two
  // non-torsion lists. Each non-torsion list is strictly increasing, so a
  // binary search over the later lists' cached indices finds repeats.
  __syncthreads();                     // sh_dV visible to all threads
  if (sh_fast) {
    bool dup = false;
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      if (c_gi[k] < 0) continue;
      const int li = c_list[k];
      if (sh_kind[li >> 1] == ABP_CV_TORSION) continue;
      for (int q = li + 1; q < 2 * D; ++q) {
        const int len = sh_ln[q];
        if (sh_kind[q >> 1] == ABP_CV_TORSION || len == 0) continue;
        int lo_i = sh_pos[q], hi_i = sh_pos[q] + len - 1;
        while (lo_i <= hi_i) {
          const int mid = (lo_i + hi_i) >> 1;
          const int v = sh_list[mid];
          if (v == c_gi[k]) { dup = true; break; }
          if (v < c_gi[k]) lo_i = mid + 1;
          else hi_i = mid - 1;
        }
      }
    }
    if (dup) atomicAnd(&sh_fast, 0);
    __syncthreads();
  }
  if (sh_fast) {
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      if (c_gi[k] < 0) continue;
      const int li = c_list[k];
      const int a = li >> 1, t = li & 1;
      const int kind = sh_kind[a];
      if (kind == ABP_CV_TORSION) continue;
      const int64_t gi = base + c_gi[k];
      const double ga = sh_dV[a];
      double fx = 0.0, fy = 0.0, fz = 0.0;
      if (kind == ABP_CV_COM_DIST) {
        const double c = (t == 0 ? -ga * sh_cv[a][3] : ga * sh_cv[a][4]) * (double)c_m[k];
        fx = c * sh_cv[a][0];
        fy = c * sh_cv[a][1];
        fz = c * sh_cv[a][2];
      } else {
        const double c = -ga * sh_cv[a][0];
        fx = c * ((double)A.x[gi] - (double)A.ref_x[c_e[k]]);
        fy = c * ((double)A.y[gi] - (double)A.ref_y[c_e[k]]);
        fz = c * ((double)A.z[gi] - (double)A.ref_z[c_e[k]]);
      }
      // torsion contributions for this atom, in CV order
#pragma unroll
      for (int b2 = 0; b2 < D; ++b2) {
        if (sh_kind[b2] != ABP_CV_TORSION) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (sh_tatom[b2][j] == c_gi[k]) {
            fx += -sh_dV[b2] * sh_cv[b2][3 * j + 0];
            fy += -sh_dV[b2] * sh_cv[b2][3 * j + 1];
            fz += -sh_dV[b2] * sh_cv[b2][3 * j + 2];
            sh_tclaimed[b2][j] = 1;
          }
      }
      rmw_force(A.fx, gi, fx);
      rmw_force(A.fy, gi, fy);
      rmw_force(A.fz, gi, fz);
    }
    __syncthreads();
    // torsion atoms in no COM/RMSD list: the first torsion occurrence writes the total
    if (tid < kMaxTors * 4) {
      const int a = tid >> 2, j = tid & 3;
      if (a < D && sh_kind[a] == ABP_CV_TORSION && !sh_tclaimed[a][j]) {
        const int atom = sh_tatom[a][j];
        bool first = true;
        for (int b2 = 0; b2 < a; ++b2)
          if (sh_kind[b2] == ABP_CV_TORSION)
            for (int jj = 0; jj < 4; ++jj) first = first && sh_tatom[b2][jj] != atom;
        if (first) {
          double fx = 0.0, fy = 0.0, fz = 0.0;
          for (int b2 = a; b2 < D; ++b2) {
            if (sh_kind[b2] != ABP_CV_TORSION) continue;
            for (int jj = 0; jj < 4; ++jj)
              if (sh_tatom[b2][jj] == atom) {
                fx += -sh_dV[b2] * sh_cv[b2][3 * jj + 0];
                fy += -sh_dV[b2] * sh_cv[b2][3 * jj + 1];
                fz += -sh_dV[b2] * sh_cv[b2][3 * jj + 2];
              }
          }
          const int64_t gi = base + atom;
          rmw_force(A.fx, gi, fx);
          rmw_force(A.fy, gi, fy);
          rmw_force(A.fz, gi, fz);
        }
      }
    }
    return;
  }
  // General path: lists one after another (a barrier orders repeated atoms).
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double g = sh_dV[a];
    const int kind = sh_kind[a];
    if (kind == ABP_CV_COM_DIST) {
      const double ux = sh_cv[a][0], uy = sh_cv[a][1], uz = sh_cv[a][2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double scale = t == 0 ? -g * sh_cv[a][3] : g * sh_cv[a][4];
        const int b0 = sh_lb[2 * a + t], n = sh_ln[2 * a + t];
        for (int e = b0 + tid; e < b0 + n; e += kBlock) {
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
        const int64_t gi = base + sh_tatom[a][tid];
        rmw_force(A.fx, gi, -g * sh_cv[a][3 * tid + 0]);
        rmw_force(A.fy, gi, -g * sh_cv[a][3 * tid + 1]);
        rmw_force(A.fz, gi, -g * sh_cv[a][3 * tid + 2]);
      }
      __syncthreads();
    } else {
      const double c = -g * sh_cv[a][0];
      const int b0 = sh_lb[2 * a], n = sh_ln[2 * a];
      for (int e = b0 + tid; e < b0 + n; e += kBlock) {
        const int64_t gi = base + A.list_idx[e];
        rmw_force(A.fx, gi, c * ((double)A.x[gi] - (double)A.ref_x[e]));
        rmw_force(A.fy, gi, c * ((double)A.y[gi] - (double)A.ref_y[e]));
        rmw_force(A.fz, gi, c * ((double)A.z[gi] - (double)A.ref_z[e]));
      }
      __syncthreads();
    }
  }
}

template <int D, int PMASK, int KERN, int MODE>
hipError_t go(const FArgs& F, hipStream_t stream) {
  const int64_t blocks = F.A.nw * (int64_t)F.nbw;
  hipLaunchKernelGGL((k_bias_force<D, PMASK, KERN, MODE>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, F);
  return hipGetLastError();
}

template <int D, int KERN>
hipError_t by_mask(int mask, const FArgs& F, hipStream_t stream) {
  switch (mask) {
    case 0: return go<D, 0, KERN, kModeF32>(F, stream);
    case 1: return go<D, 1, KERN, kModeF32>(F, stream);
    case 2: if constexpr (D >= 2) return go<D, 2, KERN, kModeF32>(F, stream); break;
    case 3: if constexpr (D >= 2) return go<D, 3, KERN, kModeF32>(F, stream); break;
    case 4: if constexpr (D >= 3) return go<D, 4, KERN, kModeF32>(F, stream); break;
    case 5: if constexpr (D >= 3) return go<D, 5, KERN, kModeF32>(F, stream); break;
    case 6: if constexpr (D >= 3) return go<D, 6, KERN, kModeF32>(F, stream); break;
    case 7: if constexpr (D >= 3) return go<D, 7, KERN, kModeF32>(F, stream); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int D>
hipError_t by_mode(int mask, const FArgs& F, hipStream_t stream) {
  const bool gauss = F.K.kernel == ABP_K_GAUSS;
  if (F.A.cv_only) return go<D, 0, ABP_K_GAUSS, kModeCV>(F, stream);
  if (F.A.use_grid) return go<D, 0, ABP_K_GAUSS, kModeGrid>(F, stream);
  if (F.A.prec == ABP_PREC_FP64)
    return gauss ? go<D, 0, ABP_K_GAUSS, kModeF64>(F, stream) : go<D, 0, ABP_K_COMPACT, kModeF64>(F, stream);
  return gauss ? by_mask<D, ABP_K_GAUSS>(mask, F, stream) : by_mask<D, ABP_K_COMPACT>(mask, F, stream);
}

}  // namespace

int force_blocks_per_walker(int64_t committed, int use_grid, int cv_only) {
  if (use_grid || cv_only) return 1;
  const int64_t nb = (committed + kHillsPerBlock - 1) / kHillsPerBlock;
  return (int)(nb < 1 ? 1 : nb);
}

size_t force_partials_bytes(int64_t nw, int nbw, int ndim) {
  if (nbw <= 1) return 0;
  return (size_t)nw * (size_t)nbw * (size_t)(ndim + 1) * sizeof(double2);
}

hipError_t launch_bias_force(const Consts& K, const HistView& H, const ForceArgs& A, void* partials,
                             unsigned int* arrivals, hipStream_t stream) {
  if (A.nw <= 0) return hipSuccess;
  FArgs F;
  F.K = K;
  F.H = H;
  F.A = A;
  F.committed = A.n_visible_default;
  F.nbw = force_blocks_per_walker(F.committed, A.use_grid, A.cv_only);
  F.partials = nullptr;
  F.arrivals = nullptr;
  if (F.nbw > 1) {
    if (!partials || !arrivals) return hipErrorInvalidValue;
    F.partials = static_cast<double2*>(partials);
    F.arrivals = arrivals;
  }
  int mask = 0;
  for (int i = 0; i < K.ndim; ++i) mask |= (K.periodic[i] ? 1 : 0) << i;
  switch (K.ndim) {
    case 1: return by_mode<1>(mask, F, stream);
    case 2: return by_mode<2>(mask, F, stream);
    case 3: return by_mode<3>(mask, F, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace abp

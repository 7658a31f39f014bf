// Fused bias-force step (bias_force) and CV evaluation (cv_compute).
//
// What the paper's bias routine does on the master rank every MD step
// (section "Minimization of Interprocess Communications"): take the
// coordinates of the CV atoms, compute the CVs, evaluate the bias gradient at
// the CV value, and return forces on exactly those atoms, which are added to
// the engine's forces. Here a batch of walkers does this in three launches
// (one with the grid form of the bias):
//
//   CV stage (one block per walker): one gather of every CV atom (index,
//     position, mass) into registers; FP64 accumulators and a fixed-order
//     block reduction for centres of mass; the dihedral angle; the offset
//     RMSD of section "Definition of the RMSD". With the grid form of the
//     bias this block also interpolates, transforms and applies the forces.
//     With the direct sum it hands the CV state and the atom list over to:
//   Sum stage (waves of 64 walkers x chunks of kHillsPerBlock hills): each
//     lane sums one chunk of hills at its walker's CV value, in index order
//     (FP32 terms folded into Kahan sums every 32 hills, or FP64). Hill
//     records are wave-uniform scalar loads, fetched once per 64 walkers.
//   Finish stage (one block per walker): merges the chunk partials in a fixed
//     order with error-free FP32 TwoSum steps (or FP64), then transform
//     (eq. apfm / eq. btraj-grad), outputs, deposit and chain rule. Chunk
//     boundaries depend only on n_visible[w], so a walker's result is
//     bitwise the same alone or in any batch; no block waits for another and
//     no atomics or device-wide fences are used.
//   Chain rule: F_j += -sum_a dV/ds_a ds_a/dx_j. When the COM/RMSD lists are
//     disjoint and short (the usual ligand/pocket case), every atom's total is
//     formed once and written once (a torsion atom that is also a ligand atom
//     is folded into that ligand entry); otherwise lists are applied one after
//     another with a barrier between them. Either way the sum per atom has a
//     fixed order and no atomics touch the forces.
//   Optional: write a new hill centred at the walker's CV value into a
//     reserved history slot (the deposit of eq. update at this step).
#include <type_traits>

#include "abp_device.h"

namespace abp {
namespace {

constexpr int kCache = 4;               // CV-list entries per thread kept in registers
constexpr int kMaxCached = kCache * kBlock;
constexpr int kMaxTors = 3;             // torsion CVs (one per axis at most)
constexpr double kMinDist = 1e-12;      // below this COM distance the direction is undefined
constexpr double kMinCross2 = 1e-24;    // collinear torsion atoms

// CV state of one walker, held in LDS by a block and in the workspace
// between the two stages.
struct CvState {
  double s[3];
  double cv[3][12];        // COM: u(3), 1/M_A, 1/M_B; TORSION: gradient (12); RMSD: 1/(N r)
  double dV[3];
  int tatom[kMaxTors][4];
  int tclaimed[kMaxTors][4];
  int lb[6], ln[6], pos[7], kind[3];
  int bad, fast, total, pad;
};
constexpr int kStateWords = (int)(sizeof(CvState) / 4);

struct Entry {             // one cached CV-list entry
  int gi;                  // walker-local atom index, -1 = none
  int li;                  // list id a*2+t
  int e;                   // position in list_idx
  float m;                 // mass
};

struct FArgs {
  Consts K;
  HistView H;
  ForceArgs A;
  int64_t committed;
  int32_t nbw;                 // sum-stage blocks per walker in the grid (upper bound)
  CvState* state;              // [nw]
  Entry* entries;              // [nw][kMaxCached]
  double2* partials;           // [nw][nbw][D+1] (hi, lo) per block
};

__device__ __forceinline__ void list_bounds(const ForceArgs& A, int64_t w, int q, int& b, int& n) {
  if (A.list_beg) {
    b = A.list_beg[(int64_t)q * A.nw + w];
    n = A.list_len[(int64_t)q * A.nw + w];
  } else {
    const int32_t* off = A.list_off + (int64_t)q * (A.nw + 1);
    b = off[w];
    n = off[w + 1] - off[w];
  }
}

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

// Writes the walker's outputs and the optional deposit (thread 0 only).
template <int D>
__device__ void write_outputs(const FArgs& F, int64_t w, const CvState& S, double V) {
  const ForceArgs& A = F.A;
  for (int a = 0; a < D; ++a) {
    A.s[a * A.nw + w] = S.s[a];
    A.dVds[a * A.nw + w] = S.dV[a];
  }
  A.V[w] = V;
  if (!A.deposit_slot) return;
  const int64_t slot = A.deposit_slot[w];
  if (slot < 0) return;
  double hw = A.deposit_height ? A.deposit_height[w] : 1.0;
  if (slot >= F.H.capacity) {
    atomicOr(A.err, kErrInval);
    return;
  }
  if (!isfinite(hw) || hw < 0.0) { atomicOr(A.err, kErrNonfinite); hw = 0.0; }
  uint32_t words[3] = {0u, 0u, 0u};
  for (int a = 0; a < D; ++a) {
    F.H.c64[a * F.H.capacity + slot] = S.s[a];
    words[a] = work32(F.K, a, S.s[a]);
  }
  F.H.w64[slot] = hw;
  int4 rec;
  rec.x = (int)words[0];
  rec.y = (int)words[1];
  rec.z = (int)words[2];
  rec.w = __float_as_int((float)log2(hw));
  F.H.rec32[slot] = rec;
}

// Chain rule for one walker (all threads of the block; S.dV set).
template <int D>
__device__ void apply_forces(const ForceArgs& A, int64_t base, CvState& S, const Entry (&ent)[kCache]) {
  const int tid = threadIdx.x;
  if (S.fast) {
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      const Entry en = ent[k];
      if (en.gi < 0) continue;
      const int a = en.li >> 1, t = en.li & 1;
      const int kind = S.kind[a];
      if (kind == ABP_CV_TORSION) continue;
      const int64_t gi = base + en.gi;
      const double ga = S.dV[a];
      double fx, fy, fz;
      if (kind == ABP_CV_COM_DIST) {
        const double c = (t == 0 ? -ga * S.cv[a][3] : ga * S.cv[a][4]) * (double)en.m;
        fx = c * S.cv[a][0];
        fy = c * S.cv[a][1];
        fz = c * S.cv[a][2];
      } else {
        const double c = -ga * S.cv[a][0];
        fx = c * ((double)A.x[gi] - (double)A.ref_x[en.e]);
        fy = c * ((double)A.y[gi] - (double)A.ref_y[en.e]);
        fz = c * ((double)A.z[gi] - (double)A.ref_z[en.e]);
      }
      // torsion contributions for this atom, in CV order
#pragma unroll
      for (int b2 = 0; b2 < D; ++b2) {
        if (S.kind[b2] != ABP_CV_TORSION) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (S.tatom[b2][j] == en.gi) {
            fx += -S.dV[b2] * S.cv[b2][3 * j + 0];
            fy += -S.dV[b2] * S.cv[b2][3 * j + 1];
            fz += -S.dV[b2] * S.cv[b2][3 * j + 2];
            S.tclaimed[b2][j] = 1;
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
      if (a < D && S.kind[a] == ABP_CV_TORSION && !S.tclaimed[a][j]) {
        const int atom = S.tatom[a][j];
        bool first = true;
        for (int b2 = 0; b2 < a; ++b2)
          if (S.kind[b2] == ABP_CV_TORSION)
            for (int jj = 0; jj < 4; ++jj) first = first && S.tatom[b2][jj] != atom;
        if (first) {
          double fx = 0.0, fy = 0.0, fz = 0.0;
          for (int b2 = a; b2 < D; ++b2) {
            if (S.kind[b2] != ABP_CV_TORSION) continue;
            for (int jj = 0; jj < 4; ++jj)
              if (S.tatom[b2][jj] == atom) {
                fx += -S.dV[b2] * S.cv[b2][3 * jj + 0];
                fy += -S.dV[b2] * S.cv[b2][3 * jj + 1];
                fz += -S.dV[b2] * S.cv[b2][3 * jj + 2];
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
    const double g = S.dV[a];
    const int kind = S.kind[a];
    if (kind == ABP_CV_COM_DIST) {
      const double ux = S.cv[a][0], uy = S.cv[a][1], uz = S.cv[a][2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double scale = t == 0 ? -g * S.cv[a][3] : g * S.cv[a][4];
        const int b0 = S.lb[2 * a + t], n = S.ln[2 * a + t];
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
        const int64_t gi = base + S.tatom[a][tid];
        rmw_force(A.fx, gi, -g * S.cv[a][3 * tid + 0]);
        rmw_force(A.fy, gi, -g * S.cv[a][3 * tid + 1]);
        rmw_force(A.fz, gi, -g * S.cv[a][3 * tid + 2]);
      }
      __syncthreads();
    } else {
      const double c = -g * S.cv[a][0];
      const int b0 = S.lb[2 * a], n = S.ln[2 * a];
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

enum { kStageCV = 0, kStageGrid = 1, kStageSum = 2 };

// ---------------------------------------------------------------------------
// CV stage: one block per walker.
// ---------------------------------------------------------------------------
template <int D, int STAGE>
__global__ __launch_bounds__(kBlock) void k_cv_stage(const FArgs F) {
  const ForceArgs& A = F.A;
  const Consts& K = F.K;
  const int64_t w = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double red[(kBlock / 64) * (9 * D + 1)];
  __shared__ CvState S;
  __shared__ double tpos[kMaxTors][4][3];
  __shared__ int sh_list[kMaxCached];     // atom index per position in the concatenated lists

  const int64_t base = A.atom_base[w];
  const int32_t natoms = A.n_atoms[w];
  if (tid == 0) {
    int bad = natoms < 0 ? kErrInval : 0;
    int pos = 0;
    for (int q = 0; q < 2 * D; ++q) {
      int b, n;
      list_bounds(A, w, q, b, n);
      S.lb[q] = b;
      S.ln[q] = n;
      S.pos[q] = pos;
      pos += n;
      if (n < 0 || b < 0) bad |= kErrInval;
    }
    S.pos[2 * D] = pos;
    S.total = pos;
    for (int a = 0; a < D; ++a) {
      const int kind = A.kind[a];
      S.kind[a] = kind;
      const int n0 = S.ln[2 * a], n1 = S.ln[2 * a + 1];
      if (kind == ABP_CV_COM_DIST && (n0 < 1 || n1 < 1)) bad |= kErrInval;
      if (kind == ABP_CV_TORSION && (n0 != 4 || n1 != 0)) bad |= kErrInval;
      if (kind == ABP_CV_RMSD_OFF && (n0 < 1 || n1 != 0)) bad |= kErrInval;
    }
    S.bad = bad;
    S.fast = pos <= kMaxCached ? 1 : 0;
    for (int t = 0; t < kMaxTors; ++t)
      for (int j = 0; j < 4; ++j) { S.tatom[t][j] = -1; S.tclaimed[t][j] = 0; }
  }
  __syncthreads();
  if (S.bad) {
    if (tid == 0) {
      atomicOr(A.err, S.bad);
      if (STAGE == kStageSum) F.state[w].bad = S.bad;
    }
    return;
  }
  const int total = S.total;

  // ---- one gather of every entry: validate, accumulate COM / RMSD sums
  // acc: [q*4 + c] mass-weighted x, y, z and mass of list q | [8D + a] RMSD squares | [9D] bad flag
  constexpr int NACC = 9 * D + 1;
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
  Entry ent[kCache];
  int badbits = 0;
  // Register arrays are only indexed with compile-time constants (dynamic
  // indices would move them to scratch memory).
  auto gather = [&](int r, Entry& out) {
    out.gi = -1; out.li = 0; out.e = 0; out.m = 0.0f;
    int li = -1, e = 0;
#pragma unroll
    for (int q = 0; q < 2 * D; ++q)
      if (r >= S.pos[q] && r < S.pos[q + 1]) { li = q; e = S.lb[q] + (r - S.pos[q]); }
    if (li < 0) return;
    const int kind = S.kind[li >> 1];
    const int32_t i = A.list_idx[e];
    if (i < 0 || i >= natoms) { badbits |= kErrIndex; return; }
    if (kind != ABP_CV_TORSION && e > S.lb[li] && A.list_idx[e - 1] >= i) badbits |= kErrIndex;
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
      const int a = li >> 1, jt = e - S.lb[li];
      tpos[a][jt][0] = x;
      tpos[a][jt][1] = y;
      tpos[a][jt][2] = z;
      S.tatom[a][jt] = i;
    }
    if (r < kMaxCached) sh_list[r] = i;
    out.gi = i; out.li = li; out.e = e; out.m = m;
  };
#pragma unroll
  for (int k = 0; k < kCache; ++k) {
    const int r = k * kBlock + tid;
    ent[k].gi = -1;
    ent[k].li = 0;
    ent[k].e = 0;
    ent[k].m = 0.0f;
    if (r < total) gather(r, ent[k]);
  }
  for (int r = kMaxCached + tid; r < total; r += kBlock) {
    Entry tmp;
    gather(r, tmp);
  }
  if (badbits) atomicOr(&S.bad, badbits);
  acc[9 * D] = badbits ? 1.0 : 0.0;
  block_sum<NACC>(acc, red);          // its barriers also publish S.bad, tpos and the torsion atoms
  if (acc[9 * D] != 0.0) {
    if (tid == 0) {
      atomicOr(A.err, S.bad ? S.bad : kErrIndex);
      if (STAGE == kStageSum) F.state[w].bad = S.bad ? S.bad : kErrIndex;
    }
    return;
  }

  // ---- CV values (thread 0)
  if (tid == 0) {
    for (int a = 0; a < D; ++a) {
      const int kind = S.kind[a];
      if (kind == ABP_CV_COM_DIST) {
        double pa[4], pb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {     // static indices into acc
          pa[c] = 0.0;
          pb[c] = 0.0;
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q == a) { pa[c] = acc[(2 * q) * 4 + c]; pb[c] = acc[(2 * q + 1) * 4 + c]; }
        }
        if (!(pa[3] > 0.0) || !(pb[3] > 0.0)) { S.bad = kErrInval; continue; }
        const double r0 = pa[0] / pa[3] - pb[0] / pb[3];
        const double r1 = pa[1] / pa[3] - pb[1] / pb[3];
        const double r2 = pa[2] / pa[3] - pb[2] / pb[3];
        const double d = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
        S.s[a] = d;
        const double inv = d >= kMinDist ? 1.0 / d : 0.0;
        S.cv[a][0] = r0 * inv;
        S.cv[a][1] = r1 * inv;
        S.cv[a][2] = r2 * inv;
        S.cv[a][3] = 1.0 / pa[3];
        S.cv[a][4] = 1.0 / pb[3];
      } else if (kind == ABP_CV_RMSD_OFF) {
        double sq = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q)
          if (q == a) sq = acc[8 * D + q];
        const double n = (double)S.ln[2 * a];
        const double r = sqrt(sq / n + 0.01);
        S.s[a] = r;
        S.cv[a][0] = 1.0 / (n * r);
      } else {
        const int* ta = S.tatom[a];
        if (ta[0] == ta[1] || ta[0] == ta[2] || ta[0] == ta[3] || ta[1] == ta[2] || ta[1] == ta[3] ||
            ta[2] == ta[3]) { S.bad = kErrIndex; continue; }
        double b1[3], b2[3], b3[3], n1[3], n2[3];
        for (int c = 0; c < 3; ++c) {
          b1[c] = tpos[a][1][c] - tpos[a][0][c];
          b2[c] = tpos[a][2][c] - tpos[a][1][c];
          b3[c] = tpos[a][3][c] - tpos[a][2][c];
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
        S.s[a] = atan2(yv, xv);
        const double nn1 = n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2];
        const double nn2 = n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2];
        if (nn1 < kMinCross2 || nn2 < kMinCross2 || lb2 == 0.0) {
          for (int q = 0; q < 12; ++q) S.cv[a][q] = 0.0;
        } else {
          // d phi / d x_i (Blondel & Karplus 1996, in the bond vectors b1..b3)
          const double f1 = b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2];
          const double f3 = b3[0] * b2[0] + b3[1] * b2[1] + b3[2] * b2[2];
          const double g1 = lb2 / nn1, g4 = lb2 / nn2;
          const double c1 = f1 / (nn1 * lb2), c3 = f3 / (nn2 * lb2);
          for (int c = 0; c < 3; ++c) {
            S.cv[a][0 + c] = -g1 * n1[c];
            S.cv[a][3 + c] = (g1 + c1) * n1[c] + c3 * n2[c];
            S.cv[a][6 + c] = -c1 * n1[c] - (g4 + c3) * n2[c];
            S.cv[a][9 + c] = g4 * n2[c];
          }
        }
      }
    }
  }
  __syncthreads();
  if (S.bad) {
    if (tid == 0) {
      atomicOr(A.err, S.bad);
      if (STAGE == kStageSum) F.state[w].bad = S.bad;
    }
    return;
  }
  if (STAGE == kStageCV) {
    if (tid == 0)
      for (int a = 0; a < D; ++a) A.s[a * A.nw + w] = S.s[a];
    return;
  }

  // ---- fast chain-rule path possible? (no atom in two COM/RMSD lists)
  if (S.fast) {
    bool dup = false;
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      const Entry en = ent[k];
      if (en.gi < 0 || S.kind[en.li >> 1] == ABP_CV_TORSION) continue;
      for (int q = en.li + 1; q < 2 * D; ++q) {
        const int len = S.ln[q];
        if (S.kind[q >> 1] == ABP_CV_TORSION || len == 0) continue;
        int lo_i = S.pos[q], hi_i = S.pos[q] + len - 1;
        while (lo_i <= hi_i) {
          const int mid = (lo_i + hi_i) >> 1;
          const int v = sh_list[mid];
          if (v == en.gi) { dup = true; break; }
          if (v < en.gi) lo_i = mid + 1;
          else hi_i = mid - 1;
        }
      }
    }
    if (dup) atomicAnd(&S.fast, 0);
    __syncthreads();
  }

  if (STAGE == kStageSum) {
    // hand the CV state and the cached entries to the sum stage
    const int* src = reinterpret_cast<const int*>(&S);
    int* dst = reinterpret_cast<int*>(F.state + w);
    for (int i = tid; i < kStateWords; i += kBlock) dst[i] = src[i];
    Entry* out = F.entries + w * (int64_t)kMaxCached;
#pragma unroll
    for (int k = 0; k < kCache; ++k)
      if (k * kBlock + tid < total) out[k * kBlock + tid] = ent[k];
    return;
  }

  // ---- grid form: interpolate, transform, forces (this block does it all)
  double s[D], h, dh[D];
#pragma unroll
  for (int a = 0; a < D; ++a) s[a] = S.s[a];
  bool clamped;
  hermite_eval<D>(K, A.grid, s, h, dh, clamped);   // every thread, same result
  double V, dV[D];
  apply_transform<D>(K, h, dh, V, dV);
  __syncthreads();
  if (tid == 0) {
    for (int a = 0; a < D; ++a) S.dV[a] = dV[a];
    write_outputs<D>(F, w, S, V);
  }
  __syncthreads();
  apply_forces<D>(A, base, S, ent);
}

// Merged sums -> transform -> outputs, deposit, chain rule (one block per walker).
template <int D, bool FP64>
__device__ void finish_walker(const FArgs& F, int64_t w, const float (&hi)[D + 1], const float (&lo)[D + 1],
                              const double (&v64)[D + 1], CvState& S) {
  constexpr int N = D + 1;
  const ForceArgs& A = F.A;
  const Consts& K = F.K;
  const int tid = threadIdx.x;
  double tot[N];
#pragma unroll
  for (int r = 0; r < N; ++r) tot[r] = FP64 ? v64[r] : (double)hi[r] + (double)lo[r];
  double dh[D];
#pragma unroll
  for (int i = 0; i < D; ++i) dh[i] = tot[i + 1] * (FP64 ? K.gs64[i] : K.gs32[i]);
  double V, dV[D];
  apply_transform<D>(K, tot[0], dh, V, dV);

  // ---- outputs, deposit, chain rule
  {
    const int* src = reinterpret_cast<const int*>(F.state + w);
    int* dst = reinterpret_cast<int*>(&S);
    for (int i = tid; i < kStateWords; i += kBlock) dst[i] = src[i];
  }
  Entry ent[kCache];
  const Entry* in = F.entries + w * (int64_t)kMaxCached;
  const int total = F.state[w].total;
#pragma unroll
  for (int k = 0; k < kCache; ++k) {
    ent[k].gi = -1;
    ent[k].li = 0;
    ent[k].e = 0;
    ent[k].m = 0.0f;
    if (k * kBlock + tid < total) ent[k] = in[k * kBlock + tid];
  }
  __syncthreads();
  if (tid == 0) {
    for (int a = 0; a < D; ++a) S.dV[a] = dV[a];
    write_outputs<D>(F, w, S, V);
  }
  __syncthreads();
  apply_forces<D>(A, A.atom_base[w], S, ent);
}


// ---------------------------------------------------------------------------
// Sum stage: one wave per (tile of 64 walkers, chunk of kHillsPerBlock hills).
// Each lane sums the chunk's hills at its walker's CV value in index order;
// hill records are wave-uniform and arrive through the scalar cache, so each
// record is fetched once per 64 walkers. The lane's compensated partial is
// stored per (walker, chunk).
// ---------------------------------------------------------------------------
template <int D, int PMASK, int KERN, bool FP64>
__global__ __launch_bounds__(64) void k_sum_tiles(const FArgs F) {
  constexpr int N = D + 1;
  const ForceArgs& A = F.A;
  const Consts& K = F.K;
  const int lane = threadIdx.x;
  const int64_t w = (int64_t)blockIdx.x * 64 + lane;
  const int64_t c = blockIdx.y;
  const bool active = w < A.nw;
  const int64_t wc = active ? w : A.nw - 1;
  int64_t nvis = A.n_visible ? A.n_visible[wc] : A.n_visible_default;
  if (nvis < 0 || nvis > F.committed) nvis = F.committed;
  const int64_t k0 = c * kHillsPerBlock;
  const int64_t kmax = k0 + kHillsPerBlock < F.committed ? k0 + kHillsPerBlock : F.committed;   // uniform
  const int64_t kstop = kmax < nvis ? kmax : nvis;                                                // per lane
  const bool wanted = active && k0 < nvis && !F.state[wc].bad;
  if (!__any(wanted)) return;
  const bool full = __all(!wanted || kstop == kmax) != 0;
  double s[D];
#pragma unroll
  for (int a = 0; a < D; ++a) s[a] = F.state[wc].s[a];
  double2 out[N];
  if constexpr (FP64) {
    double tq[D], P[N];
#pragma unroll
    for (int i = 0; i < D; ++i) tq[i] = work64(K, i, s[i]);
#pragma unroll
    for (int r = 0; r < N; ++r) P[r] = 0.0;
    for (int64_t k = k0; k < kmax; ++k) {
      double4 hr;
      hr.x = work64(K, 0, F.H.c64[k]);
      hr.y = D > 1 ? work64(K, 1, F.H.c64[F.H.capacity + k]) : 0.0;
      hr.z = D > 2 ? work64(K, 2, F.H.c64[2 * F.H.capacity + k]) : 0.0;
      hr.w = (full || k < kstop) ? F.H.w64[k] : 0.0;
      pair64<D, KERN>(K, tq, hr, P);
    }
#pragma unroll
    for (int r = 0; r < N; ++r) { out[r].x = P[r]; out[r].y = 0.0; }
  } else {
    uint32_t qw[D];
    float kf[D], ua[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      qw[i] = work32(K, i, s[i]);
      kf[i] = K.kf32[i];
      ua[i] = K.ua32[i];
    }
    const bool comp = A.prec == ABP_PREC_FP32_KAHAN;
    typedef const __attribute__((address_space(4))) int cint4_t;   // uniform loads via the scalar cache
    cint4_t* recs = (cint4_t*)F.H.rec32;
    float Sm[N], Cc[N], P[N];
#pragma unroll
    for (int r = 0; r < N; ++r) { Sm[r] = 0.0f; Cc[r] = 0.0f; P[r] = 0.0f; }
    const float ninf = -__builtin_inff();
    // MASK: some lanes stop before kmax (their walker sees fewer hills).
    auto run = [&](auto mask_tag) {
      constexpr bool MASK = decltype(mask_tag)::value;
      int64_t k = k0;
      for (; k + 32 <= kmax; k += 32) {
#pragma unroll 8
        for (int u = 0; u < 32; ++u) {
          int4 h;
          h.x = recs[4 * (k + u)];
          h.y = D > 1 ? recs[4 * (k + u) + 1] : 0;
          h.z = D > 2 ? recs[4 * (k + u) + 2] : 0;
          h.w = recs[4 * (k + u) + 3];
          if (MASK && k + u >= kstop) h.w = __float_as_int(ninf);
          pair32<D, PMASK, KERN>(qw, h, kf, ua, K.pl32, P);
        }
        if (comp) {
          kahan_fold<N>(Sm, Cc, P);
#pragma unroll
          for (int r = 0; r < N; ++r) P[r] = 0.0f;
        }
      }
      for (; k < kmax; ++k) {
        int4 h;
        h.x = recs[4 * k];
        h.y = D > 1 ? recs[4 * k + 1] : 0;
        h.z = D > 2 ? recs[4 * k + 2] : 0;
        h.w = recs[4 * k + 3];
        if (MASK && k >= kstop) h.w = __float_as_int(ninf);
        pair32<D, PMASK, KERN>(qw, h, kf, ua, K.pl32, P);
      }
    };
    if (full) run(std::false_type{});
    else run(std::true_type{});
    if (comp) {
      kahan_fold<N>(Sm, Cc, P);
#pragma unroll
      for (int r = 0; r < N; ++r) { out[r].x = Sm[r]; out[r].y = -Cc[r]; }
    } else {
#pragma unroll
      for (int r = 0; r < N; ++r) { out[r].x = P[r]; out[r].y = 0.0; }
    }
  }
  if (wanted) {
    double2* dst = F.partials + (w * F.nbw + c) * N;
#pragma unroll
    for (int r = 0; r < N; ++r) dst[r] = out[r];
  }
}

// ---------------------------------------------------------------------------
// Finish stage (one block per walker): merge the chunk partials (thread t
// takes a fixed contiguous range of chunks in order, then a fixed block
// tree), transform, outputs, deposit, chain rule.
// ---------------------------------------------------------------------------
template <int D, bool FP64>
__global__ __launch_bounds__(kBlock) void k_finish_stage(const FArgs F) {
  constexpr int N = D + 1;
  const ForceArgs& A = F.A;
  const int64_t w = blockIdx.x;
  const int tid = threadIdx.x;
  if (F.state[w].bad) return;
  int64_t nvis = A.n_visible ? A.n_visible[w] : A.n_visible_default;
  if (nvis < 0 || nvis > F.committed) nvis = F.committed;
  const int64_t nch = (nvis + kHillsPerBlock - 1) / kHillsPerBlock;
  const int64_t per = (nch + kBlock - 1) / kBlock;
  const int64_t c0 = tid * per, c1 = c0 + per < nch ? c0 + per : nch;
  __shared__ double red[(kBlock / 64) * 2 * N];
  __shared__ CvState S;
  const double2* part = F.partials + w * F.nbw * N;
  float hi[N], lo[N];
  double v64[N];
  const bool comp = A.prec == ABP_PREC_FP32_KAHAN;
#pragma unroll
  for (int r = 0; r < N; ++r) { hi[r] = 0.0f; lo[r] = 0.0f; v64[r] = 0.0; }
  for (int64_t q = c0; q < c1; ++q) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const double2 p = part[q * N + r];
      if (FP64) {
        v64[r] += p.x;
      } else {
        const float h2[1] = {(float)p.x}, l2[1] = {(float)p.y};
        float h1[1] = {hi[r]}, l1[1] = {lo[r]};
        merge_f32<1>(h1, l1, h2, l2, comp);
        hi[r] = h1[0];
        lo[r] = l1[0];
      }
    }
  }
  if (FP64) block_sum<N>(v64, red);
  else block_merge_f32<N>(hi, lo, comp, reinterpret_cast<float*>(red));
  finish_walker<D, FP64>(F, w, hi, lo, v64, S);
}

template <int D, int STAGE>
hipError_t go_cv(const FArgs& F, hipStream_t stream) {
  hipLaunchKernelGGL((k_cv_stage<D, STAGE>), dim3((unsigned)F.A.nw), dim3(kBlock), 0, stream, F);
  return hipGetLastError();
}

template <int D, int PMASK, int KERN, bool FP64>
hipError_t go_sum(const FArgs& F, hipStream_t stream) {
  if (F.nbw <= 0) return hipSuccess;
  const dim3 grid((unsigned)((F.A.nw + 63) / 64), (unsigned)F.nbw);
  hipLaunchKernelGGL((k_sum_tiles<D, PMASK, KERN, FP64>), grid, dim3(64), 0, stream, F);
  return hipGetLastError();
}

template <int D, int KERN>
hipError_t sum_by_mask(int mask, const FArgs& F, hipStream_t stream) {
  switch (mask) {
    case 0: return go_sum<D, 0, KERN, false>(F, stream);
    case 1: return go_sum<D, 1, KERN, false>(F, stream);
    case 2: if constexpr (D >= 2) return go_sum<D, 2, KERN, false>(F, stream); break;
    case 3: if constexpr (D >= 2) return go_sum<D, 3, KERN, false>(F, stream); break;
    case 4: if constexpr (D >= 3) return go_sum<D, 4, KERN, false>(F, stream); break;
    case 5: if constexpr (D >= 3) return go_sum<D, 5, KERN, false>(F, stream); break;
    case 6: if constexpr (D >= 3) return go_sum<D, 6, KERN, false>(F, stream); break;
    case 7: if constexpr (D >= 3) return go_sum<D, 7, KERN, false>(F, stream); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int D>
hipError_t launch_d(int mask, const FArgs& F, hipStream_t stream) {
  if (F.A.cv_only) return go_cv<D, kStageCV>(F, stream);
  if (F.A.use_grid) return go_cv<D, kStageGrid>(F, stream);
  hipError_t e = go_cv<D, kStageSum>(F, stream);
  if (e != hipSuccess) return e;
  const bool gauss = F.K.kernel == ABP_K_GAUSS;
  const bool fp64 = F.A.prec == ABP_PREC_FP64;
  if (fp64)
    e = gauss ? go_sum<D, 0, ABP_K_GAUSS, true>(F, stream) : go_sum<D, 0, ABP_K_COMPACT, true>(F, stream);
  else
    e = gauss ? sum_by_mask<D, ABP_K_GAUSS>(mask, F, stream) : sum_by_mask<D, ABP_K_COMPACT>(mask, F, stream);
  if (e != hipSuccess) return e;
  if (fp64) hipLaunchKernelGGL((k_finish_stage<D, true>), dim3((unsigned)F.A.nw), dim3(kBlock), 0, stream, F);
  else hipLaunchKernelGGL((k_finish_stage<D, false>), dim3((unsigned)F.A.nw), dim3(kBlock), 0, stream, F);
  return hipGetLastError();
}

}  // namespace

int force_blocks_per_walker(int64_t committed, int use_grid, int cv_only) {
  if (use_grid || cv_only) return 1;
  return (int)((committed + kHillsPerBlock - 1) / kHillsPerBlock);
}

size_t force_workspace_bytes(int64_t nw, int nbw, int ndim) {
  if (nw <= 0) return 0;
  const size_t st = (size_t)nw * sizeof(CvState);
  const size_t en = (size_t)nw * kMaxCached * sizeof(Entry);
  const size_t pa = (size_t)nw * (size_t)nbw * (size_t)(ndim + 1) * sizeof(double2);
  return (st + 255) / 256 * 256 + (en + 255) / 256 * 256 + pa;
}

hipError_t launch_bias_force(const Consts& K, const HistView& H, const ForceArgs& A, void* workspace,
                             hipStream_t stream) {
  if (A.nw <= 0) return hipSuccess;
  FArgs F;
  F.K = K;
  F.H = H;
  F.A = A;
  F.committed = A.n_visible_default;
  F.nbw = force_blocks_per_walker(F.committed, A.use_grid, A.cv_only);
  F.state = nullptr;
  F.entries = nullptr;
  F.partials = nullptr;
  if (!A.cv_only && !A.use_grid) {
    if (!workspace) return hipErrorInvalidValue;
    char* p = static_cast<char*>(workspace);
    const size_t st = ((size_t)A.nw * sizeof(CvState) + 255) / 256 * 256;
    const size_t en = ((size_t)A.nw * kMaxCached * sizeof(Entry) + 255) / 256 * 256;
    F.state = reinterpret_cast<CvState*>(p);
    F.entries = reinterpret_cast<Entry*>(p + st);
    F.partials = reinterpret_cast<double2*>(p + st + en);
  }
  int mask = 0;
  for (int i = 0; i < K.ndim; ++i) mask |= (K.periodic[i] ? 1 : 0) << i;
  switch (K.ndim) {
    case 1: return launch_d<1>(mask, F, stream);
    case 2: return launch_d<2>(mask, F, stream);
    case 3: return launch_d<3>(mask, F, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace abp

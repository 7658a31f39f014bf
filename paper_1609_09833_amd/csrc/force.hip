// Fused bias-force step (bias_force) and CV evaluation (cv_compute).
//
// What the paper's bias routine does on the master rank every MD step
// (section "Minimization of Interprocess Communications"): take the
// coordinates of the CV atoms, compute the CVs, evaluate the bias gradient at
// the CV value, and return forces on exactly those atoms, which are added to
// the engine's forces.
//
// CV part (one 128-thread block per walker): one gather of every CV atom
// (index, position, mass); FP64 accumulators and a fixed-order block
// reduction for centres of mass; the dihedral angle; the offset RMSD of
// section "Definition of the RMSD".
//
// Bias from the hill history (direct sum). A walker's sum over its visible
// hills [0, nvis) always has the same decomposition: chunks of 64
// consecutive hills, each summed in increasing order (FP32 terms folded into
// a Kahan sum every 32 terms, or FP64); thread t of a 128-thread block merges
// chunks t, t + 128, ... in that order (error-free FP32 TwoSum steps, or FP64
// adds), then a fixed block tree merges the threads. Three launch shapes
// compute exactly this:
//   fused (a short history): one launch, the walker's block does the CV
//     part, sums its own chunks and finishes;
//   split (a long history): a CV launch, a sum launch of one wave per
//     (chunk, 64 walkers) that stages the chunk's 64 hill records in LDS (one
//     coalesced load per lane, so each record is fetched once per 64 walkers)
//     and in which every lane sums the chunk at its walker's CV value from
//     LDS broadcasts, and a finish launch that merges the chunk sums;
//   chained (a long history, one or two walkers): one launch of several
//     blocks per walker, each computing the CV and summing 128 chunks, the
//     last to arrive (per-walker counter) merging and finishing.
// So a walker's result is bitwise the same alone or in any batch, whichever
// shape runs. No block waits for another; no atomics touch sums or forces.
//
// Finish: transform (eq. apfm / eq. btraj-grad), outputs, optional deposit of
// a hill at the walker's CV value into a reserved slot (eq. update), and the
// chain rule F_j += -sum_a dV/ds_a ds_a/dx_j. When the COM/RMSD lists are
// disjoint and short (the usual ligand/pocket case), every atom's total is
// formed once and written once (a torsion atom that is also a ligand atom is
// folded into that ligand entry); otherwise lists are applied one after
// another with a barrier between them. Either way the sum per atom has a
// fixed order. With the grid form of the bias the CV block interpolates,
// transforms and finishes in the same launch.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "abp_device.h"

namespace abp {
namespace {

// Threads per walker block. Two waves: at the walker kernels' register
// footprint (150-185 VGPRs, 2-3 waves per SIMD) a CU holds 4-6 walker
// blocks, so 1,024 walkers are resident at once.
constexpr int kFBlock = 128;
constexpr int kCache = 6;               // CV-list entries per thread kept in registers
constexpr int kMaxCached = kCache * kFBlock;
constexpr int kMaxTors = 3;             // torsion CVs (one per axis at most)
constexpr int kDupMapAtoms = 32768;     // walkers up to this many atoms: duplicate check by LDS bitmap (4 KiB)
constexpr double kMinDist = 1e-12;      // below this COM distance the direction is undefined
constexpr double kMinCross2 = 1e-24;    // collinear torsion atoms

// Histories up to this length use the fused launch; longer ones the split
// launches, whose sum launch reads each hill record once per 64 walkers
// instead of once per walker (the result does not depend on the choice).
constexpr int64_t kFusedMaxHills = 16384;
// Batches of up to kChainMaxWalkers walkers take the chained launch instead
// of the split launches (same decomposition and order, so the same results):
// one launch, but every block of a walker recomputes its CV. That pays for
// one or two walkers (measured: 100,000 hills, one walker, 25.9 -> 21.9 us);
// for the serving loop's batches of a few walkers on concurrent streams the
// redundant CV gathers cost more than the two launches they save (p50 at
// 200,000 hills 90 -> 131 us). kChainCounters bounds the batches that a
// fixed chained shape (abp_set_force_shape) can send through it.
constexpr int64_t kChainMaxWalkers = 2;
constexpr int64_t kChainCounters = 64;

// CV state of one walker, held in LDS by a block and in the workspace
// between the launches of the split shape.
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
  int32_t pmax;                // chunk partials per walker in the workspace (for nvis = committed)
  CvState* state;              // [nw]                 split shape only
  Entry* entries;              // [nw][kMaxCached]     split shape only
  double* scv;                 // [3][nw] coordinates the sum uses (split shape)
  int* sbad;                   // [nw] nonzero: walker invalid (split shape)
  float2* part32;              // [nw][pmax][D+1] partial sums (hi, lo), FP32 modes
  double* part64;              // the same buffer, FP64 mode
  unsigned* arrived;           // [nw] blocks of the chained launch done with their chunks (0 between launches)
};

__device__ __forceinline__ void list_bounds(const ForceArgs& A, int64_t w, int q, int& b, int& n) {
  if (A.inl_n) {
    b = A.inl.list_beg[q][w];
    n = A.inl.list_len[q][w];
  } else if (A.list_beg) {
    b = A.list_beg[(int64_t)q * A.nw + w];
    n = A.list_len[(int64_t)q * A.nw + w];
  } else {
    const int32_t* off = A.list_off + (int64_t)q * (A.nw + 1);
    b = off[w];
    n = off[w + 1] - off[w];
  }
}

// Per-walker fields, from the kernel arguments for an inline batch.
__device__ __forceinline__ int64_t w_atom_base(const ForceArgs& A, int64_t w) {
  return A.inl_n ? A.inl.atom_base[w] : A.atom_base[w];
}
__device__ __forceinline__ int64_t w_mass_base(const ForceArgs& A, int64_t w) {
  return A.inl_n ? A.inl.mass_base[w] : (A.mass_base ? A.mass_base[w] : A.atom_base[w]);
}
__device__ __forceinline__ int64_t w_stage_off(const ForceArgs& A, int64_t w) {
  return A.inl_n ? A.inl.stage_off[w] : (A.stage_off ? A.stage_off[w] : -1);
}
__device__ __forceinline__ int32_t w_n_atoms(const ForceArgs& A, int64_t w) {
  return A.inl_n ? A.inl.n_atoms[w] : A.n_atoms[w];
}
__device__ __forceinline__ int64_t w_deposit_slot(const ForceArgs& A, int64_t w) {
  return A.inl_n ? A.inl.deposit_slot[w] : (A.deposit_slot ? A.deposit_slot[w] : -1);
}
__device__ __forceinline__ double w_deposit_height(const ForceArgs& A, int64_t w) {
  return A.inl_n ? A.inl.deposit_height[w] : (A.deposit_height ? A.deposit_height[w] : 1.0);
}

__device__ __forceinline__ int64_t walker_nvis(const FArgs& F, int64_t w) {
  int64_t nvis = F.A.n_visible ? F.A.n_visible[w] : F.A.n_visible_default;
  return (nvis < 0 || nvis > F.committed) ? F.committed : nvis;
}

// Hills of chunk c that lie below nvis.
__device__ __forceinline__ int chunk_terms(int64_t nvis, int64_t c) {
  const int64_t n = nvis - c * kChunkHills;
  return n <= 0 ? 0 : (n >= kChunkHills ? kChunkHills : (int)n);
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
// thread gets the result. `red` holds at least kFBlock/64 * N * 2 floats.
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
  for (int wv = 1; wv < kFBlock / 64; ++wv) {
    float h2[N], l2[N];
#pragma unroll
    for (int r = 0; r < N; ++r) { h2[r] = red[(wv * N + r) * 2]; l2[r] = red[(wv * N + r) * 2 + 1]; }
    merge_f32<N>(h, l, h2, l2, comp);
  }
  __syncthreads();
}

// block_sum restricted to the entries whose bit is set in `mask` (uniform
// across the block): the same fixed order (wave butterfly, then waves in
// order) for those, the others left as they are.
template <int N>
__device__ __forceinline__ void block_sum_masked(double (&v)[N], double* red, uint32_t mask) {
#pragma unroll
  for (int r = 0; r < N; ++r) {
    if (!((mask >> r) & 1u)) continue;
    double x = v[r];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    v[r] = x;
  }
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int r = 0; r < N; ++r)
      if ((mask >> r) & 1u) red[wave * N + r] = v[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < N; ++r) {
    if (!((mask >> r) & 1u)) continue;
    double t = 0.0;
    for (int w = 0; w < kFBlock / 64; ++w) t += red[w * N + r];
    v[r] = t;
  }
  __syncthreads();
}

__device__ __forceinline__ void rmw_force(float* f, int64_t g, double add) {
  f[g] = (float)((double)f[g] + add);
}

// Completion word of walker w (all threads of the block that finished it, on
// every exit path): each thread's stores are released at system scope before
// the barrier, then one store publishes the sequence number.
__device__ __forceinline__ void signal_done(const ForceArgs& A, int64_t w) {
  if (!A.done_flag) return;
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(A.done_flag + w, A.done_seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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
  const int64_t slot = w_deposit_slot(A, w);
  if (slot < 0) return;
  double hw = w_deposit_height(A, w);
  if (slot >= F.H.capacity) {
    atomicOr(A.err, kErrInval);
    return;
  }
  if (F.K.wt_dT > 0.0) hw *= exp(-V / F.K.wt_dT);    // well-tempered height
  if (!isfinite(hw) || hw < 0.0) { atomicOr(A.err, kErrNonfinite); hw = 0.0; }
  uint32_t words[3] = {0u, 0u, 0u};
  for (int a = 0; a < D; ++a) {
    const double c = eval_coord(F.K, a, S.s[a]);   // quantised mode: the nearest node
    F.H.c64[a * F.H.capacity + slot] = c;
    words[a] = work32(F.K, a, c);
  }
  F.H.w64[slot] = hw;
  F.H.l64[slot] = log2_height(hw);
  int4 rec;
  rec.x = (int)words[0];
  rec.y = (int)words[1];
  rec.z = (int)words[2];
  rec.w = __float_as_int((float)log2(hw));
  F.H.rec32[slot] = rec;
}

// Old forces of a thread's cached entries, read ahead of the chain rule (the
// finish launch issues them before it merges its chunk sums, so their
// latency overlaps the merge): pre[k] for entry k with an atom, when
// `valid`; otherwise apply_forces reads them itself.
struct OldForces {
  float f[kCache][3];
  bool valid;
};

// Chain rule for one walker (all threads of the block; S.dV set).
template <int D>
__device__ void apply_forces(const ForceArgs& A, int64_t w, CvState& S, const Entry (&ent)[kCache],
                             const OldForces& pre) {
  const int tid = threadIdx.x;
  const int64_t base = w_atom_base(A, w);
  const int64_t mbase = w_mass_base(A, w);
  if (S.fast) {
    // Every cached COM/RMSD entry is a distinct atom here (no atom is in two
    // such lists and each list is strictly increasing), so all the old forces
    // can be read before any is written back: one round trip per thread
    // instead of one per entry, issued before the additions are formed.
    double add[kCache][3];
    int64_t gat[kCache];
    bool live[kCache];
    float old[kCache][3];
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      const Entry en = ent[k];
      live[k] = en.gi >= 0 && S.kind[en.li >> 1] != ABP_CV_TORSION;
      gat[k] = base + (en.gi >= 0 ? en.gi : 0);
      old[k][0] = old[k][1] = old[k][2] = 0.0f;
      if (!live[k] || A.force_store) continue;
      if (pre.valid) {
        old[k][0] = pre.f[k][0];
        old[k][1] = pre.f[k][1];
        old[k][2] = pre.f[k][2];
      } else {
        old[k][0] = A.fx[gat[k]];
        old[k][1] = A.fy[gat[k]];
        old[k][2] = A.fz[gat[k]];
      }
    }
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      const Entry en = ent[k];
      add[k][0] = add[k][1] = add[k][2] = 0.0;
      if (!live[k]) continue;
      const int a = en.li >> 1, t = en.li & 1;
      const int kind = S.kind[a];
      const int64_t gi = gat[k];
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
      add[k][0] = fx;
      add[k][1] = fy;
      add[k][2] = fz;
    }
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      if (!live[k]) continue;
      A.fx[gat[k]] = (float)((double)old[k][0] + add[k][0]);
      A.fy[gat[k]] = (float)((double)old[k][1] + add[k][1]);
      A.fz[gat[k]] = (float)((double)old[k][2] + add[k][2]);
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
        for (int e = b0 + tid; e < b0 + n; e += kFBlock) {
          const int32_t li = A.list_idx[e];
          const int64_t gi = base + li;
          const double c = scale * (double)A.mass[mbase + li];
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
      for (int e = b0 + tid; e < b0 + n; e += kFBlock) {
        const int64_t gi = base + A.list_idx[e];
        rmw_force(A.fx, gi, c * ((double)A.x[gi] - (double)A.ref_x[e]));
        rmw_force(A.fy, gi, c * ((double)A.y[gi] - (double)A.ref_y[e]));
        rmw_force(A.fz, gi, c * ((double)A.z[gi] - (double)A.ref_z[e]));
      }
      __syncthreads();
    }
  }
}

// CV part of the step for walker w (all threads of the block): validates the
// lists, gathers every CV atom once (the first kMaxCached entries are kept in
// `ent`), reduces the centres of mass and RMSD sums in FP64, and thread 0
// forms the CVs and their gradients in S. Returns false when the walker is
// done: invalid (the error word is set, and F.state[w].bad when to_state) or
// cv_only (s written). Otherwise S.fast tells whether the one-pass chain rule
// applies (no atom in two COM/RMSD lists).
template <int D>
__device__ bool cv_block(const FArgs& F, int64_t w, bool cv_only, bool to_state, CvState& S,
                         Entry (&ent)[kCache], double* red, double (&tpos)[kMaxTors][4][3], int* sh_list,
                         unsigned* dupmap) {
  const ForceArgs& A = F.A;
  const int tid = threadIdx.x;
  const int64_t base = w_atom_base(A, w);
  const int64_t mbase = w_mass_base(A, w);
  const int64_t soff = w_stage_off(A, w);                        // masses staged for this batch
  const int32_t natoms = w_n_atoms(A, w);
  if (tid < 2 * D) {                       // the lists' bounds, one thread each (loads in parallel)
    int b, n;
    list_bounds(A, w, tid, b, n);
    S.lb[tid] = b;
    S.ln[tid] = n;
  }
  __syncthreads();
  if (tid == 0) {
    int bad = natoms < 0 ? kErrInval : 0;
    int pos = 0;
    for (int q = 0; q < 2 * D; ++q) {
      const int b = S.lb[q], n = S.ln[q];
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
      if (to_state) { F.state[w].bad = S.bad; F.sbad[w] = S.bad; }
    }
    return false;
  }
  const int total = S.total;
  // Atoms in two COM/RMSD lists (which rule out the one-pass chain rule) are
  // found during the gather through a bitmap of the walker's atoms in LDS,
  // when the walker is small enough for it; otherwise by binary search after.
  const bool use_map = !cv_only && S.fast && natoms <= kDupMapAtoms;     // uniform
  bool dup_seen = false;
  if (use_map) {
    for (int i = tid; i < (natoms + 31) / 32; i += kFBlock) dupmap[i] = 0u;
    __syncthreads();
  }

  // ---- one gather of every entry: validate, accumulate COM / RMSD sums
  // acc: [q*4 + c] mass-weighted x, y, z and mass of list q | [8D + a] RMSD squares | [9D] bad flag
  constexpr int NACC = 9 * D + 1;
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
  int badbits = 0;
  // Register arrays are only indexed with compile-time constants (dynamic
  // indices would move them to scratch memory). A thread's cached entries are
  // gathered in three passes, so that their loads overlap: list entry and
  // atom index (with the previous index, for the order check), then the
  // atom's position and mass (and the reference for RMSD), then the sums, in
  // entry order.
  struct Got {
    int li, e;
    int32_t i, ip;
    float x, y, z, m, rx, ry, rz;
  };
  auto locate = [&](int r, Got& G) {
    G.li = -1; G.e = 0; G.i = -1; G.ip = INT_MIN;
#pragma unroll
    for (int q = 0; q < 2 * D; ++q)
      if (r >= S.pos[q] && r < S.pos[q + 1]) { G.li = q; G.e = S.lb[q] + (r - S.pos[q]); }
    if (G.li < 0) return;
    G.i = A.list_idx[G.e];
    if (S.kind[G.li >> 1] != ABP_CV_TORSION && G.e > S.lb[G.li]) G.ip = A.list_idx[G.e - 1];
  };
  // The loads of fetch are not branched per entry (a branch around each would
  // make the compiler wait for all loads in flight at its join): an entry
  // without a valid atom reads the walker's first atom and list entry 0
  // instead, in bounds, and consume ignores those values.
  bool any_ref = A.ref_x && A.ref_y && A.ref_z;
  {
    bool rm = false;
#pragma unroll
    for (int a = 0; a < D; ++a) rm = rm || S.kind[a] == ABP_CV_RMSD_OFF;
    any_ref = any_ref && rm;
  }
  auto fetch = [&](Got& G) {
    G.x = 0.0f; G.y = 0.0f; G.z = 0.0f; G.m = 0.0f; G.rx = 0.0f; G.ry = 0.0f; G.rz = 0.0f;
    const bool ok = G.li >= 0 && G.i >= 0 && G.i < natoms;
    if (natoms >= 1) {                                   // uniform
      const int32_t i = ok ? G.i : 0;
      const int64_t g = base + i;
      G.x = A.x[g]; G.y = A.y[g]; G.z = A.z[g];
      G.m = soff >= 0 ? A.stage_mass[soff + i] : A.mass[mbase + i];
    }
    if (any_ref) {                                       // uniform; RMSD lists are not empty
      const int e = G.li >= 0 ? G.e : 0;
      G.rx = A.ref_x[e]; G.ry = A.ref_y[e]; G.rz = A.ref_z[e];
    }
  };
  auto consume = [&](int r, const Got& G, Entry& out) {
    out.gi = -1; out.li = 0; out.e = 0; out.m = 0.0f;
    const int li = G.li, e = G.e;
    if (li < 0) return;
    const int kind = S.kind[li >> 1];
    const int32_t i = G.i;
    if (i < 0 || i >= natoms) { badbits |= kErrIndex; return; }
    if (G.ip >= i) badbits |= kErrIndex;                 // COM/RMSD lists must increase
    const float x = G.x, y = G.y, z = G.z, m = G.m;
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
      const float rx = G.rx, ry = G.ry, rz = G.rz;
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
    if (use_map && kind != ABP_CV_TORSION) {             // i is in [0, natoms) here
      const unsigned bit = 1u << (i & 31);
      if (atomicOr(&dupmap[i >> 5], bit) & bit) dup_seen = true;
    }
    if (soff >= 0) A.mass_store[mbase + i] = m;         // the walker's masses stay on the device
    out.gi = i; out.li = li; out.e = e; out.m = m;
  };
  {
    Got G[kCache];
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      G[k].li = -1; G[k].e = 0; G[k].i = -1; G[k].ip = INT_MIN;
      const int r = k * kFBlock + tid;
      if (r < total) locate(r, G[k]);
    }
#pragma unroll
    for (int k = 0; k < kCache; ++k) fetch(G[k]);
#pragma unroll
    for (int k = 0; k < kCache; ++k) consume(k * kFBlock + tid, G[k], ent[k]);
  }
  for (int r = kMaxCached + tid; r < total; r += kFBlock) {
    Got G;
    locate(r, G);
    fetch(G);
    Entry tmp;
    consume(r, G, tmp);
  }
  if (badbits) atomicOr(&S.bad, badbits);
  if (dup_seen) atomicAnd(&S.fast, 0);                   // published by block_sum's barriers
  acc[9 * D] = badbits ? 1.0 : 0.0;
  // only the sums the CV kinds read: a COM list's four, an RMSD list's
  // squares, and the flag
  uint32_t mask = 1u << (9 * D);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (S.kind[a] == ABP_CV_COM_DIST) mask |= 0xFFu << (8 * a);
    if (S.kind[a] == ABP_CV_RMSD_OFF) mask |= 1u << (8 * D + a);
  }
  block_sum_masked<NACC>(acc, red, mask);      // its barriers also publish S.bad, tpos and the torsion atoms
  if (acc[9 * D] != 0.0) {
    if (tid == 0) {
      atomicOr(A.err, S.bad ? S.bad : kErrIndex);
      if (to_state) { F.state[w].bad = S.bad ? S.bad : kErrIndex; F.sbad[w] = F.state[w].bad; }
    }
    return false;
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
      if (to_state) { F.state[w].bad = S.bad; F.sbad[w] = S.bad; }
    }
    return false;
  }
  if (cv_only) {
    if (tid == 0)
      for (int a = 0; a < D; ++a) A.s[a * A.nw + w] = S.s[a];
    return false;
  }

  // ---- fast chain-rule path possible? (no atom in two COM/RMSD lists)
  if (S.fast && !use_map) {
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
  return true;
}

// ---------------------------------------------------------------------------
// One chunk sum (FP32): hills k0, k0 + 1, ... for nrun terms; terms from
// nmine on are zero-height (MASK) and the Kahan folds of groups that end past
// nmine are skipped, which gives exactly the sum of nmine terms.
// `load(k)` returns hill k's FP32 record.
// ---------------------------------------------------------------------------
template <int D, int PMASK, int KERN, bool MASK, class Load>
__device__ __forceinline__ void partial_f32(const uint32_t (&qw)[D], const float (&kf)[D], const float (&ua)[D],
                                            float pl, bool comp, int64_t k0, int nrun, int nmine, Load load,
                                            float (&hi)[D + 1], float (&lo)[D + 1]) {
  constexpr int N = D + 1;
  float Sm[N], Cc[N], Pp[N];
#pragma unroll
  for (int r = 0; r < N; ++r) { Sm[r] = 0.0f; Cc[r] = 0.0f; Pp[r] = 0.0f; }
  const int ninf = __float_as_int(-__builtin_inff());
  int u = 0;
  for (; u + 32 <= nrun; u += 32) {
#pragma unroll 8
    for (int j = 0; j < 32; ++j) {
      int4 h = load(k0 + u + j);
      if (MASK && u + j >= nmine) h.w = ninf;
      pair32<D, PMASK, KERN>(qw, h, kf, ua, pl, Pp);
    }
    if (comp && (!MASK || u + 32 <= nmine)) {
      kahan_fold<N>(Sm, Cc, Pp);
#pragma unroll
      for (int r = 0; r < N; ++r) Pp[r] = 0.0f;
    }
  }
  for (; u < nrun; ++u) {
    int4 h = load(k0 + u);
    if (MASK && u >= nmine) h.w = ninf;
    pair32<D, PMASK, KERN>(qw, h, kf, ua, pl, Pp);
  }
  if (comp) {
    kahan_fold<N>(Sm, Cc, Pp);
#pragma unroll
    for (int r = 0; r < N; ++r) { hi[r] = Sm[r]; lo[r] = -Cc[r]; }
  } else {
#pragma unroll
    for (int r = 0; r < N; ++r) { hi[r] = Pp[r]; lo[r] = 0.0f; }
  }
}

// One chunk sum (FP64), same terms; zero-height terms add exact zeros.
template <int D, int PMASK, int KERN, bool MASK, class Load>
__device__ __forceinline__ void partial_f64(const Consts& K, const double (&tq)[D], int64_t k0, int nrun,
                                            int nmine, Load load, double (&v)[D + 1]) {
  double Pp[D + 1];
#pragma unroll
  for (int r = 0; r <= D; ++r) Pp[r] = 0.0;
  for (int u = 0; u < nrun; ++u) {
    double4 hr = load(k0 + u);
    if (MASK && u >= nmine) hr.w = kLog2Zero;
    pair64<D, PMASK, KERN>(K, tq, hr, Pp);
  }
#pragma unroll
  for (int r = 0; r <= D; ++r) v[r] = Pp[r];
}

__device__ __forceinline__ double4 hill64(const FArgs& F, int D, int64_t k) {
  double4 hr;
  hr.x = work64(F.K, 0, F.H.c64[k]);
  hr.y = D > 1 ? work64(F.K, 1, F.H.c64[F.H.capacity + k]) : 0.0;
  hr.z = D > 2 ? work64(F.K, 2, F.H.c64[2 * F.H.capacity + k]) : 0.0;
  hr.w = F.H.l64[k];
  return hr;
}

// Merge one partial into a thread's running (hi, lo) or FP64 sum.
template <int N, bool FP64>
__device__ __forceinline__ void merge_part(float (&hi)[N], float (&lo)[N], double (&v64)[N], const float (&ph)[N],
                                           const float (&pl)[N], const double (&pv)[N], bool comp) {
  if (FP64) {
#pragma unroll
    for (int r = 0; r < N; ++r) v64[r] += pv[r];
  } else {
    merge_f32<N>(hi, lo, ph, pl, comp);
  }
}

// Merged sums -> transform -> outputs, deposit, chain rule (all threads; S
// and ent hold the walker's CV state and cached entries).
template <int D, bool FP64>
__device__ void finish_common(const FArgs& F, int64_t w, const float (&hi)[D + 1], const float (&lo)[D + 1],
                              const double (&v64)[D + 1], CvState& S, const Entry (&ent)[kCache],
                              const OldForces& pre) {
  constexpr int N = D + 1;
  const Consts& K = F.K;
  double tot[N];
#pragma unroll
  for (int r = 0; r < N; ++r) tot[r] = FP64 ? v64[r] : (double)hi[r] + (double)lo[r];
  double dh[D];
#pragma unroll
  for (int i = 0; i < D; ++i) dh[i] = tot[i + 1] * (FP64 ? K.gs64[i] : K.gs32[i]);
  double V, dV[D];
  apply_transform<D>(K, tot[0], dh, V, dV);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int a = 0; a < D; ++a) S.dV[a] = dV[a];
    write_outputs<D>(F, w, S, V);
  }
  __syncthreads();
  apply_forces<D>(F.A, w, S, ent, pre);
}

// ---------------------------------------------------------------------------
// CV launch: cv_compute (STAGE kStageCV), the whole grid-form step
// (kStageGrid), or the first launch of the split shape (kStageSum: hands the
// CV state and the cached entries to the workspace).
// ---------------------------------------------------------------------------
enum { kStageCV = 0, kStageGrid = 1, kStageSum = 2 };

template <int D, int STAGE>
__device__ __forceinline__ void cv_stage_body(const FArgs& F) {
  const ForceArgs& A = F.A;
  const int64_t w = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double red[(kFBlock / 64) * (9 * D + 1)];
  __shared__ CvState S;
  __shared__ double tpos[kMaxTors][4][3];
  __shared__ int sh_list[kMaxCached];
  Entry ent[kCache];
  __shared__ unsigned dupmap[kDupMapAtoms / 32];
  if (!cv_block<D>(F, w, STAGE == kStageCV, STAGE == kStageSum, S, ent, red, tpos, sh_list, dupmap)) return;

  if (STAGE == kStageSum) {
    const int* src = reinterpret_cast<const int*>(&S);
    int* dst = reinterpret_cast<int*>(F.state + w);
    for (int i = tid; i < kStateWords; i += kFBlock) dst[i] = src[i];
    if (tid < D) F.scv[tid * A.nw + w] = eval_coord(F.K, tid, S.s[tid]);
    if (tid == 0) F.sbad[w] = 0;
    Entry* out = F.entries + w * (int64_t)kMaxCached;
#pragma unroll
    for (int k = 0; k < kCache; ++k)
      if (k * kFBlock + tid < S.total) out[k * kFBlock + tid] = ent[k];
    return;
  }
  if constexpr (STAGE == kStageGrid) {
    double s[D], h, dh[D];
#pragma unroll
    for (int a = 0; a < D; ++a) s[a] = S.s[a];
    bool clamped;
    hermite_eval<D>(F.K, A.grid, s, h, dh, clamped);   // every thread, same result
    double V, dV[D];
    apply_transform<D>(F.K, h, dh, V, dV);
    __syncthreads();
    if (tid == 0) {
      for (int a = 0; a < D; ++a) S.dV[a] = dV[a];
      write_outputs<D>(F, w, S, V);
    }
    __syncthreads();
    OldForces none;
    none.valid = false;
    apply_forces<D>(A, w, S, ent, none);
  }
}

template <int D, int STAGE>
__global__ __launch_bounds__(kFBlock) void k_cv_stage(const FArgs F) {
  cv_stage_body<D, STAGE>(F);
  if (STAGE != kStageSum) signal_done(F.A, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Fused shape: the whole direct-sum step of one walker in one block.
// ---------------------------------------------------------------------------
template <int D, int PMASK, int KERN, bool FP64>
__device__ __forceinline__ void force_fused_body(const FArgs& F) {
  constexpr int N = D + 1;
  const ForceArgs& A = F.A;
  const Consts& K = F.K;
  const int64_t w = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double red[(kFBlock / 64) * (9 * D + 1)];
  __shared__ CvState S;
  __shared__ double tpos[kMaxTors][4][3];
  __shared__ int sh_list[kMaxCached];
  Entry ent[kCache];
  __shared__ unsigned dupmap[kDupMapAtoms / 32];
  if (!cv_block<D>(F, w, false, false, S, ent, red, tpos, sh_list, dupmap)) return;

  const int64_t nvis = walker_nvis(F, w);
  const int64_t nch = force_chunks(nvis);
  float hi[N], lo[N];
  double v64[N];
#pragma unroll
  for (int r = 0; r < N; ++r) { hi[r] = 0.0f; lo[r] = 0.0f; v64[r] = 0.0; }
  const bool comp = A.prec == ABP_PREC_FP32_KAHAN;
  if constexpr (FP64) {
    double tq[D];
#pragma unroll
    for (int i = 0; i < D; ++i) tq[i] = work64(K, i, eval_coord(K, i, S.s[i]));
    for (int64_t c = tid; c < nch; c += kFBlock) {
      const int n = chunk_terms(nvis, c);
      double pv[N];
      partial_f64<D, PMASK, KERN, false>(K, tq, c * kChunkHills, n, n, [&](int64_t k) { return hill64(F, D, k); }, pv);
      const float z[N] = {};
      merge_part<N, true>(hi, lo, v64, z, z, pv, comp);
    }
    block_sum<N, kFBlock>(v64, red);
  } else {
    uint32_t qw[D];
    float kf[D], ua[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      qw[i] = work32(K, i, eval_coord(K, i, S.s[i]));
      kf[i] = K.kf32[i];
      ua[i] = K.ua32[i];
    }
    const int4* recs = F.H.rec32;
    for (int64_t c = tid; c < nch; c += kFBlock) {
      const int n = chunk_terms(nvis, c);
      float ph[N], pl[N];
      partial_f32<D, PMASK, KERN, false>(qw, kf, ua, K.pl32, comp, c * kChunkHills, n, n,
                                         [&](int64_t k) { return recs[k]; }, ph, pl);
      const double z[N] = {};
      merge_part<N, false>(hi, lo, v64, ph, pl, z, comp);
    }
    block_merge_f32<N>(hi, lo, comp, reinterpret_cast<float*>(red));
  }
  OldForces none;
  none.valid = false;
  finish_common<D, FP64>(F, w, hi, lo, v64, S, ent, none);
}

template <int D, int PMASK, int KERN, bool FP64>
__global__ __launch_bounds__(kFBlock) void k_force_fused(const FArgs F) {
  force_fused_body<D, PMASK, KERN, FP64>(F);
  signal_done(F.A, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Split shape, sum launch: one wave per (chunk c, 64 walkers). The chunk's
// 64 hill records are loaded once per wave (one per lane, coalesced) into
// LDS and read back as broadcasts, so each record is fetched once per 64
// walkers; a lane whose walker sees fewer hills masks the rest. The walkers'
// CV values come from a compact [D][nw] array (coalesced).
// ---------------------------------------------------------------------------
constexpr int kChunksPerWave = 1;   // consecutive chunks one wave sums
// Waves per block of the sum launch, each with its own chunks of the same 64
// walkers (1,024 walkers, 20,000 hills: 1 -> 14.7 us, 2 -> 14.4, 4 -> 13.4,
// 8 -> 14.3; two or four chunks per wave were slower at every block size).
constexpr int kSumWaves = 4;

template <int D, int PMASK, int KERN, bool FP64>
__global__ __launch_bounds__(64 * kSumWaves) void k_sum_parts(const FArgs F) {
  constexpr int N = D + 1;
  const ForceArgs& A = F.A;
  const Consts& K = F.K;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c0 = ((int64_t)blockIdx.x * kSumWaves + wave) * kChunksPerWave;
  const int64_t w = (int64_t)blockIdx.y * 64 + lane;
  const bool active = w < A.nw;
  const int64_t wc = active ? w : A.nw - 1;
  const int64_t nvis = walker_nvis(F, wc);
  const bool alive = active && c0 * kChunkHills < nvis && !F.sbad[wc];
  // the chunks' records, one coalesced load per lane per chunk, then LDS
  // broadcasts (each wave its own tile; every wave reaches the barrier)
  static_assert(kChunkHills == 64, "one record per lane");
  __shared__ int4 tile32s[FP64 ? 1 : kSumWaves][FP64 ? 1 : kChunksPerWave * kChunkHills];
  __shared__ double4 tile64s[FP64 ? kSumWaves : 1][FP64 ? kChunksPerWave * kChunkHills : 1];
  int4* tile32 = tile32s[FP64 ? 0 : wave];
  double4* tile64 = tile64s[FP64 ? wave : 0];
#pragma unroll
  for (int j = 0; j < kChunksPerWave; ++j) {
    const int64_t k = (c0 + j) * kChunkHills + lane;
    if constexpr (FP64) tile64[j * kChunkHills + lane] = k < F.committed ? hill64(F, D, k) : make_double4(0.0, 0.0, 0.0, kLog2Zero);
    else tile32[j * kChunkHills + lane] = k < F.committed ? F.H.rec32[k] : make_int4(0, 0, 0, 0);
  }
  __syncthreads();
  if (!__any(alive)) return;
  double s[D];
#pragma unroll
  for (int a = 0; a < D; ++a) s[a] = F.scv[a * A.nw + wc];
  const bool comp = A.prec == ABP_PREC_FP32_KAHAN;
  double tq[D];
  uint32_t qw[D];
  float kf[D], ua[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    tq[i] = work64(K, i, s[i]);
    qw[i] = work32(K, i, s[i]);
    kf[i] = K.kf32[i];
    ua[i] = K.ua32[i];
  }
  const int64_t kbase = c0 * kChunkHills;
  for (int j = 0; j < kChunksPerWave; ++j) {
    const int64_t c = c0 + j;
    if (c >= F.pmax) break;                                      // uniform
    const bool wanted = active && c * kChunkHills < nvis && !F.sbad[wc];
    if (!__any(wanted)) break;                                   // later chunks are further out
    const int nmine = wanted ? chunk_terms(nvis, c) : 0;
    const int nrun = chunk_terms(F.committed, c);               // uniform, >= nmine
    const bool full = __all(!wanted || nmine == nrun);
    const int64_t k0 = c * kChunkHills;
    float ph[N], pl[N];
    double pv[N];
    if constexpr (FP64) {
      auto ld = [&](int64_t k) { return tile64[k - kbase]; };
      if (full) partial_f64<D, PMASK, KERN, false>(K, tq, k0, nrun, nrun, ld, pv);
      else partial_f64<D, PMASK, KERN, true>(K, tq, k0, nrun, nmine, ld, pv);
    } else {
      auto lds = [&](int64_t k) { return tile32[k - kbase]; };
      if (full) partial_f32<D, PMASK, KERN, false>(qw, kf, ua, K.pl32, comp, k0, nrun, nrun, lds, ph, pl);
      else partial_f32<D, PMASK, KERN, true>(qw, kf, ua, K.pl32, comp, k0, nrun, nmine, lds, ph, pl);
    }
    if (wanted) {
      const int64_t at = (w * F.pmax + c) * N;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        if constexpr (FP64) F.part64[at + r] = pv[r];
        else F.part32[at + r] = make_float2(ph[r], pl[r]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split shape, finish launch (one block per walker): thread t merges chunk
// sums t, t + 128, ... in order, then the block tree; transform, outputs,
// deposit, chain rule.
// ---------------------------------------------------------------------------
constexpr int kMergeBatch = 16;

template <int D, bool FP64>
__device__ __forceinline__ void finish_stage_body(const FArgs& F) {
  constexpr int N = D + 1;
  const ForceArgs& A = F.A;
  const int64_t w = blockIdx.x;
  const int tid = threadIdx.x;
  if (F.sbad[w]) return;
  const int64_t nch = force_chunks(walker_nvis(F, w));
  __shared__ double red[(kFBlock / 64) * 2 * N];
  __shared__ CvState S;
  float hi[N], lo[N];
  double v64[N];
  const bool comp = A.prec == ABP_PREC_FP32_KAHAN;
#pragma unroll
  for (int r = 0; r < N; ++r) { hi[r] = 0.0f; lo[r] = 0.0f; v64[r] = 0.0; }
  // the CV state (to LDS, published by the merge's barriers) and the cached
  // entries are fetched first, so their loads overlap those of the chunk sums
  {
    const int* src = reinterpret_cast<const int*>(F.state + w);
    int* dst = reinterpret_cast<int*>(&S);
    for (int i = tid; i < kStateWords; i += kFBlock) dst[i] = src[i];
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
    if (k * kFBlock + tid < total) ent[k] = in[k * kFBlock + tid];
  }
  // the old forces of the cached entries (the one-pass chain rule's reads),
  // in flight while the chunk sums are merged; entries of a torsion list are
  // read too and ignored
  OldForces pre;
  pre.valid = !A.force_store && total <= kMaxCached;
  {
    const int64_t fbase = w_atom_base(A, w);
#pragma unroll
    for (int k = 0; k < kCache; ++k) {
      pre.f[k][0] = pre.f[k][1] = pre.f[k][2] = 0.0f;
      if (pre.valid && ent[k].gi >= 0) {
        const int64_t g = fbase + ent[k].gi;
        pre.f[k][0] = A.fx[g];
        pre.f[k][1] = A.fy[g];
        pre.f[k][2] = A.fz[g];
      }
    }
  }
  // kMergeBatch of a thread's chunk sums are loaded before any is merged (the
  // loads overlap; the merge order is unchanged)
  for (int64_t c0 = tid; c0 < nch; c0 += kMergeBatch * kFBlock) {
    float ph[kMergeBatch][N], pl[kMergeBatch][N];
    double pv[kMergeBatch][N];
#pragma unroll
    for (int u = 0; u < kMergeBatch; ++u) {
      const int64_t c = c0 + (int64_t)u * kFBlock;
      const int64_t at = (w * F.pmax + (c < nch ? c : c0)) * N;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        if (FP64) {
          pv[u][r] = F.part64[at + r];
          ph[u][r] = 0.0f;
          pl[u][r] = 0.0f;
        } else {
          const float2 q = F.part32[at + r];
          ph[u][r] = q.x;
          pl[u][r] = q.y;
          pv[u][r] = 0.0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kMergeBatch; ++u)
      if (c0 + (int64_t)u * kFBlock < nch) merge_part<N, FP64>(hi, lo, v64, ph[u], pl[u], pv[u], comp);
  }
  if (FP64) block_sum<N, kFBlock>(v64, red);
  else block_merge_f32<N>(hi, lo, comp, reinterpret_cast<float*>(red));
  finish_common<D, FP64>(F, w, hi, lo, v64, S, ent, pre);
}

template <int D, bool FP64>
__global__ __launch_bounds__(kFBlock) void k_finish_stage(const FArgs F) {
  finish_stage_body<D, FP64>(F);
  signal_done(F.A, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Chained shape (few walkers, long history), one launch: block (g, w)
// computes walker w's CV, the sums of chunks g * kFBlock + t (thread t; each
// chunk exactly as the fused launch sums it) into the workspace, and counts
// itself in F.arrived[w]; the walker's last block to arrive merges every chunk
// sum in the fused launch's order and finishes (transform, outputs, deposit,
// chain rule), then resets the counter for the next launch. Every block
// arrives, also for an invalid walker, and no block waits for another.
// ---------------------------------------------------------------------------
// Returns whether this block finished the walker (it was the last to arrive).
template <int D, int PMASK, int KERN, bool FP64>
__device__ __forceinline__ bool force_chain_body(const FArgs& F) {
  constexpr int N = D + 1;
  const ForceArgs& A = F.A;
  const Consts& K = F.K;
  const int64_t w = blockIdx.y;
  const int tid = threadIdx.x;
  __shared__ double red[(kFBlock / 64) * (9 * D + 1)];
  __shared__ CvState S;
  __shared__ double tpos[kMaxTors][4][3];
  __shared__ int sh_list[kMaxCached];
  __shared__ int last;
  Entry ent[kCache];
  __shared__ unsigned dupmap[kDupMapAtoms / 32];
  const bool ok = cv_block<D>(F, w, false, false, S, ent, red, tpos, sh_list, dupmap);   // uniform
  const int64_t nvis = walker_nvis(F, w);
  const int64_t nch = force_chunks(nvis);
  const bool comp = A.prec == ABP_PREC_FP32_KAHAN;
  const int64_t c = (int64_t)blockIdx.x * kFBlock + tid;
  if (ok && c < nch) {
    const int n = chunk_terms(nvis, c);
    const int64_t at = (w * F.pmax + c) * N;
    if constexpr (FP64) {
      double tq[D];
#pragma unroll
      for (int i = 0; i < D; ++i) tq[i] = work64(K, i, eval_coord(K, i, S.s[i]));
      double pv[N];
      partial_f64<D, PMASK, KERN, false>(K, tq, c * kChunkHills, n, n, [&](int64_t k) { return hill64(F, D, k); }, pv);
#pragma unroll
      for (int r = 0; r < N; ++r) F.part64[at + r] = pv[r];
    } else {
      uint32_t qw[D];
      float kf[D], ua[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        qw[i] = work32(K, i, eval_coord(K, i, S.s[i]));
        kf[i] = K.kf32[i];
        ua[i] = K.ua32[i];
      }
      const int4* recs = F.H.rec32;
      float ph[N], pl[N];
      partial_f32<D, PMASK, KERN, false>(qw, kf, ua, K.pl32, comp, c * kChunkHills, n, n,
                                         [&](int64_t k) { return recs[k]; }, ph, pl);
#pragma unroll
      for (int r = 0; r < N; ++r) F.part32[at + r] = make_float2(ph[r], pl[r]);
    }
  }
  // arrival: the chunk sums are made visible before the count
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const unsigned before = atomicAdd(&F.arrived[w], 1u);
    last = before == gridDim.x - 1 ? 1 : 0;
    if (last) atomicExch(&F.arrived[w], 0u);   // every block of the walker has arrived
  }
  __syncthreads();
  if (!last) return false;
  if (!ok) return true;
  __threadfence();
  float hi[N], lo[N];
  double v64[N];
#pragma unroll
  for (int r = 0; r < N; ++r) { hi[r] = 0.0f; lo[r] = 0.0f; v64[r] = 0.0; }
  for (int64_t c0 = tid; c0 < nch; c0 += kMergeBatch * kFBlock) {
    float ph[kMergeBatch][N], pl[kMergeBatch][N];
    double pv[kMergeBatch][N];
#pragma unroll
    for (int u = 0; u < kMergeBatch; ++u) {
      const int64_t cc = c0 + (int64_t)u * kFBlock;
      const int64_t at = (w * F.pmax + (cc < nch ? cc : c0)) * N;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        if (FP64) {
          pv[u][r] = F.part64[at + r];
          ph[u][r] = 0.0f;
          pl[u][r] = 0.0f;
        } else {
          const float2 q = F.part32[at + r];
          ph[u][r] = q.x;
          pl[u][r] = q.y;
          pv[u][r] = 0.0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kMergeBatch; ++u)
      if (c0 + (int64_t)u * kFBlock < nch) merge_part<N, FP64>(hi, lo, v64, ph[u], pl[u], pv[u], comp);
  }
  if (FP64) block_sum<N, kFBlock>(v64, red);
  else block_merge_f32<N>(hi, lo, comp, reinterpret_cast<float*>(red));
  OldForces none;
  none.valid = false;
  finish_common<D, FP64>(F, w, hi, lo, v64, S, ent, none);
  return true;
}

template <int D, int PMASK, int KERN, bool FP64>
__global__ __launch_bounds__(kFBlock) void k_force_chain(const FArgs F) {
  if (force_chain_body<D, PMASK, KERN, FP64>(F)) signal_done(F.A, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Launch selection.
// ---------------------------------------------------------------------------
enum { kShapeFused = 0, kShapeSplit = 1, kShapeChain = 2 };

template <int D, int PMASK, int KERN, bool FP64>
hipError_t go_direct(const FArgs& F, int shape, hipStream_t stream) {
  const dim3 walkers((unsigned)F.A.nw);
  if (shape == kShapeFused) {
    hipLaunchKernelGGL((k_force_fused<D, PMASK, KERN, FP64>), walkers, dim3(kFBlock), 0, stream, F);
    return hipGetLastError();
  }
  if (shape == kShapeChain) {
    const dim3 grid((unsigned)std::max<int64_t>(1, (F.pmax + kFBlock - 1) / kFBlock), (unsigned)F.A.nw);
    hipLaunchKernelGGL((k_force_chain<D, PMASK, KERN, FP64>), grid, dim3(kFBlock), 0, stream, F);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_cv_stage<D, kStageSum>), walkers, dim3(kFBlock), 0, stream, F);
  if (F.pmax > 0) {
    const int64_t per_block = (int64_t)kChunksPerWave * kSumWaves;
    const dim3 grid((unsigned)((F.pmax + per_block - 1) / per_block), (unsigned)((F.A.nw + 63) / 64));
    hipLaunchKernelGGL((k_sum_parts<D, PMASK, KERN, FP64>), grid, dim3(64 * kSumWaves), 0, stream, F);
  }
  hipLaunchKernelGGL((k_finish_stage<D, FP64>), walkers, dim3(kFBlock), 0, stream, F);
  return hipGetLastError();
}

template <int D, int KERN, bool FP64>
hipError_t direct_by_mask(int mask, const FArgs& F, int shape, hipStream_t stream) {
  switch (mask) {
    case 0: return go_direct<D, 0, KERN, FP64>(F, shape, stream);
    case 1: return go_direct<D, 1, KERN, FP64>(F, shape, stream);
    case 2: if constexpr (D >= 2) return go_direct<D, 2, KERN, FP64>(F, shape, stream); break;
    case 3: if constexpr (D >= 2) return go_direct<D, 3, KERN, FP64>(F, shape, stream); break;
    case 4: if constexpr (D >= 3) return go_direct<D, 4, KERN, FP64>(F, shape, stream); break;
    case 5: if constexpr (D >= 3) return go_direct<D, 5, KERN, FP64>(F, shape, stream); break;
    case 6: if constexpr (D >= 3) return go_direct<D, 6, KERN, FP64>(F, shape, stream); break;
    case 7: if constexpr (D >= 3) return go_direct<D, 7, KERN, FP64>(F, shape, stream); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int D>
hipError_t launch_d(int mask, const FArgs& F, int shape, hipStream_t stream) {
  const dim3 walkers((unsigned)F.A.nw);
  if (F.A.cv_only) {
    hipLaunchKernelGGL((k_cv_stage<D, kStageCV>), walkers, dim3(kFBlock), 0, stream, F);
    return hipGetLastError();
  }
  if (F.A.use_grid) {
    hipLaunchKernelGGL((k_cv_stage<D, kStageGrid>), walkers, dim3(kFBlock), 0, stream, F);
    return hipGetLastError();
  }
  const bool gauss = F.K.kernel == ABP_K_GAUSS;
  if (F.A.prec == ABP_PREC_FP64)
    return gauss ? direct_by_mask<D, ABP_K_GAUSS, true>(mask, F, shape, stream)
                 : direct_by_mask<D, ABP_K_COMPACT, true>(mask, F, shape, stream);
  return gauss ? direct_by_mask<D, ABP_K_GAUSS, false>(mask, F, shape, stream)
               : direct_by_mask<D, ABP_K_COMPACT, false>(mask, F, shape, stream);
}

// The launch shape of a direct-sum bias_force: fused (short histories), else
// chained (one or two walkers) or split. `fixed` (an abp_force_shape other
// than AUTO) overrides the choice; chain applies to batches of up to
// kChainCounters. All three give the same results.
int direct_shape(int64_t nw, int64_t committed, int fixed) {
  if (fixed == ABP_SHAPE_FUSED) return kShapeFused;
  if (fixed == ABP_SHAPE_SPLIT) return kShapeSplit;
  if (fixed == ABP_SHAPE_CHAIN) return nw <= kChainCounters ? kShapeChain : kShapeSplit;
  if (committed <= kFusedMaxHills) return kShapeFused;
  return nw <= kChainMaxWalkers ? kShapeChain : kShapeSplit;
}

}  // namespace

int force_blocks_per_walker(int64_t committed, int use_grid, int cv_only) {
  if (use_grid || cv_only) return 1;
  return (int)force_chunks(committed);
}

bool force_uses_workspace(int64_t nw, int64_t committed, int use_grid, int cv_only, int shape) {
  if (use_grid || cv_only) return false;
  return direct_shape(nw, committed, shape) != kShapeFused;
}

// Layout: the chained shape's arrival counters (a fixed region at the start,
// which no other shape writes, so they stay zero between launches whatever
// the batch sizes), CV state, cached entries, coordinates and flags (split
// shape), chunk partials (both).
static_assert(kChainCounters * sizeof(unsigned) <= kForceArrivedBytes, "counter region too small");

size_t force_workspace_bytes(int64_t nw, int nbw, int ndim) {
  if (nw <= 0) return 0;
  const size_t st = (size_t)nw * sizeof(CvState);
  const size_t en = (size_t)nw * kMaxCached * sizeof(Entry);
  const size_t sc = (size_t)nw * (3 * sizeof(double) + sizeof(int));
  const size_t pa = (size_t)nw * (size_t)nbw * (size_t)(ndim + 1) * 8;   // float2 or double
  return kForceArrivedBytes + (st + 255) / 256 * 256 + (en + 255) / 256 * 256 + (sc + 255) / 256 * 256 + pa;
}

hipError_t launch_bias_force(const Consts& K, const HistView& H, const ForceArgs& A, void* workspace,
                             hipStream_t stream) {
  if (A.nw <= 0) return hipSuccess;
  FArgs F;
  F.K = K;
  F.H = H;
  F.A = A;
  F.committed = A.n_visible_default;
  F.pmax = force_blocks_per_walker(F.committed, A.use_grid, A.cv_only);
  F.state = nullptr;
  F.entries = nullptr;
  F.scv = nullptr;
  F.sbad = nullptr;
  F.part32 = nullptr;
  F.part64 = nullptr;
  const bool split = force_uses_workspace(A.nw, F.committed, A.use_grid, A.cv_only, A.shape);
  F.arrived = nullptr;
  if (split) {
    if (!workspace) return hipErrorInvalidValue;
    F.arrived = static_cast<unsigned*>(workspace);
    char* p = static_cast<char*>(workspace) + kForceArrivedBytes;
    const size_t st = ((size_t)A.nw * sizeof(CvState) + 255) / 256 * 256;
    const size_t en = ((size_t)A.nw * kMaxCached * sizeof(Entry) + 255) / 256 * 256;
    const size_t sc = ((size_t)A.nw * (3 * sizeof(double) + sizeof(int)) + 255) / 256 * 256;
    F.state = reinterpret_cast<CvState*>(p);
    F.entries = reinterpret_cast<Entry*>(p + st);
    F.scv = reinterpret_cast<double*>(p + st + en);
    F.sbad = reinterpret_cast<int*>(p + st + en + (size_t)A.nw * 3 * sizeof(double));
    F.part32 = reinterpret_cast<float2*>(p + st + en + sc);
    F.part64 = reinterpret_cast<double*>(p + st + en + sc);
  }
  const int shape = (A.use_grid || A.cv_only) ? kShapeFused : (split ? direct_shape(A.nw, F.committed, A.shape) : kShapeFused);
  int mask = 0;
  for (int i = 0; i < K.ndim; ++i) mask |= (K.periodic[i] ? 1 : 0) << i;
  switch (K.ndim) {
    case 1: return launch_d<1>(mask, F, shape, stream);
    case 2: return launch_d<2>(mask, F, shape, stream);
    case 3: return launch_d<3>(mask, F, shape, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace abp

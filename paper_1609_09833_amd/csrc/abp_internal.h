// Internal declarations shared by the host layer and the HIP kernels of libabp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "abp.h"

namespace abp {

constexpr int kBlock = 256;      // threads per block for every kernel
constexpr int kTile32 = 1024;    // hills per LDS tile in the FP32 direct sum (16 KiB)
constexpr int kTile64 = 512;     // hills per LDS tile in the FP64 direct sum (16 KiB)
constexpr int kChunk = 32;       // hills summed plainly before each compensated (Kahan) step
constexpr int kQ2D = 2;          // queries per thread in the 2-D/3-D FP32 direct sum

// Largest magnitude of a non-periodic FP32 working word (see Consts).
constexpr double kFixLimit = 1073741823.0;   // 2^30 - 1

// log2 of a zero height in the FP64 sums: finite, so that the exponent of a
// term stays finite, and far enough below -1074 that the term is exactly 0.
constexpr double kLog2Zero = -2048.0;

// Device error word bits.
enum : int32_t { kErrIndex = 1 << 0, kErrNonfinite = 1 << 1, kErrInval = 1 << 2 };

// Per-context constants, computed once on the host from abp_bias_desc.
//
// Working displacements: in the FP32 path every coordinate is a 32-bit
// fixed-point word, so a displacement is an integer difference, converted to
// float in units of unit32 (its error does not grow with the coordinate's
// magnitude). A periodic coordinate is a fraction of its period (unit
// L/2^32), so the difference of two words (mod 2^32) is already the minimum
// image. A non-periodic coordinate is a signed offset from the middle of the
// window [lo - E, hi + E], E = max((hi - lo)/2, 16 width), in units of the
// window's half-width / 2^30; values beyond the window are taken at its edge.
// Words then stay within +-(2^30 - 1), so a difference never wraps. In the
// FP64 path periodic coordinates are fractions of the period (turns) wrapped
// with rint; non-periodic ones are raw.
struct Consts {
  int32_t ndim, kernel, p, transform;
  int32_t quant;                   // 1: evaluate and deposit at the nearest grid node
  int32_t periodic[3];
  double lo[3], hi[3], period[3], inv_period[3];
  double fix_mid[3], fix_scale[3]; // non-periodic FP32 words: rint((x - fix_mid) * fix_scale)
  // FP32 path, per axis: Gaussian exponent factor on the working displacement
  // (log2(e) unit^2 / (2 sigma^2)), compact scale (unit / a), gradient scale.
  float kf32[3], ua32[3];
  double gs32[3];
  float pl32;                      // p log2(e), compact kernel
  // FP64 path, the same in FP64 units.
  double kf64[3], ua64[3], gs64[3], per64[3];
  double pl64;
  double kT, b, c;                 // mABP transform
  double wt_dT;                    // > 0: well-tempered deposit heights w exp(-V / wt_dT)
  double width[3];                 // sigma_i (Gaussian) or a_i (compact), real units
  double inv_width[3];             // 1 / width
  // grid
  int32_t grid_n[3];
  double grid_dx[3];               // node spacing per axis
  double inv_grid_dx[3];           // 1 / grid_dx (correctly rounded, as a device division would give)
  int64_t nodes;
};

struct HistView {
  double* c64;      // [ndim][capacity] master centers
  double* w64;      // [capacity] master heights
  double* l64;      // [capacity] log2 of the heights (kLog2Zero for a zero height), read by the FP64 sums
  int4* rec32;      // [capacity] FP32 working records {c0, c1, c2, log2(w)}
  int64_t capacity;
};

// Kernel entry points (host-callable launchers). All enqueue on `stream`
// and return hipSuccess or the launch error.
hipError_t launch_hist_init(const HistView& H, int ndim, hipStream_t stream);

// vbias (optional, same dtype as the centres): the bias at each centre; with
// K.wt_dT > 0 each height is multiplied by exp(-vbias / wt_dT).
hipError_t launch_hist_append(const Consts& K, const HistView& H, int64_t first, int64_t n,
                              int dtype_f64, const void* centers, const void* heights,
                              const void* vbias, int32_t* err, hipStream_t stream);

hipError_t launch_direct_sum(const Consts& K, const HistView& H, int64_t n_visible, abp_prec prec,
                             int64_t nq, int q_f64, const void* q, void* V, void* dVds,
                             hipStream_t stream);

// Grid accumulation of hills [k0, k1) into the FP64 node arrays. `scratch`
// must hold scratch_bytes_for(...) bytes (may be NULL when that is 0).
// Grids deposited tile by tile on the VALU (compact hills, 2-D and 3-D) can
// record which tiles a deposit reached: `dirty` (grid_dirty_tiles entries, or
// NULL) gets `epoch` for each such tile, so that the mirror refresh of the
// same epoch skips the others.
size_t grid_deposit_scratch_bytes(const Consts& K, int64_t nhills);
size_t grid_dirty_tiles(const Consts& K);
hipError_t launch_grid_deposit(const Consts& K, const HistView& H, int64_t k0, int64_t k1,
                               double* grid, double* scratch, uint32_t* dirty, uint32_t epoch,
                               hipStream_t stream);

// grid32 (optional): the FP32 mirror of grid; when given the interpolation
// reads it instead (FP64 arithmetic either way).
hipError_t launch_grid_eval(const Consts& K, const double* grid, const float* grid32, int64_t nq, int q_f64,
                            const void* q, void* V, void* dVds, unsigned long long* n_clamped,
                            hipStream_t stream);
// Refreshes the FP32 mirror grid32 of the node arrays grid (cell-major for
// 1-D and 2-D grids, node-major for 3-D; grid_mirror_floats entries).
size_t grid_mirror_floats(const Consts& K);
// With `dirty` (see launch_grid_deposit), only entries whose source node lies
// in a tile marked `epoch` are refreshed.
hipError_t launch_grid_mirror(const Consts& K, const double* grid, float* grid32, const uint32_t* dirty,
                              uint32_t epoch, hipStream_t stream);

// The per-walker fields of a batch of up to kInlineWalkers walkers, carried
// in the kernel arguments (the serving loop's small batches), so that no copy
// of a descriptor has to precede the launch. Used when ForceArgs::inl_n > 0,
// in place of list_beg/list_len, atom_base, n_atoms, mass_base, stage_off,
// deposit_slot (-1: no deposit) and deposit_height.
constexpr int kInlineWalkers = 16;
struct InlineDesc {
  int64_t atom_base[kInlineWalkers];
  int64_t mass_base[kInlineWalkers];
  int64_t stage_off[kInlineWalkers];
  int64_t deposit_slot[kInlineWalkers];
  double deposit_height[kInlineWalkers];
  int32_t n_atoms[kInlineWalkers];
  int32_t list_beg[6][kInlineWalkers];
  int32_t list_len[6][kInlineWalkers];
};

struct ForceArgs {
  int32_t ncv;
  int32_t kind[3];
  const int32_t* list_off;         // CSR offsets [(a*2+t)*(nw+1) + w], or
  const int32_t* list_beg;         // start and length of list (a*2+t) of walker w at
  const int32_t* list_len;         //   [(a*2+t)*nw + w] (used when list_beg is set)
  const int32_t* list_idx;
  const float* ref_x;
  const float* ref_y;
  const float* ref_z;
  int64_t nw;
  const int64_t* atom_base;
  const int32_t* n_atoms;
  const float* x;
  const float* y;
  const float* z;
  const float* mass;
  float* fx;
  float* fy;
  float* fz;
  // Masses at mass[mass_base[w] + i] instead of mass[atom_base[w] + i] (NULL:
  // atom_base). A walker with stage_off[w] >= 0 reads its masses from
  // stage_mass[stage_off[w] + i] and stores them to mass_store[mass_base[w] + i]
  // (a walker admitted to the serving loop's device pool for this batch).
  const int64_t* mass_base;
  const int64_t* stage_off;
  const float* stage_mass;
  float* mass_store;
  int32_t force_store;             // 1: forces start at zero; the one-pass chain rule writes, not adds
  const int64_t* n_visible;        // [nw] or NULL
  int64_t n_visible_default;       // used when n_visible is NULL
  const int64_t* deposit_slot;     // [nw] or NULL
  const double* deposit_height;    // [nw] or NULL
  double* s;
  double* V;
  double* dVds;
  int32_t shape;                   // abp_force_shape of the direct sum (ABP_SHAPE_AUTO: by size)
  int32_t cv_only;                 // 1: compute s only
  int32_t use_grid;
  int32_t prec;                    // abp_prec
  const double* grid;
  int32_t* err;
  // Completion words (NULL: none): when walker w's step is done (outputs,
  // deposit, forces all stored and released at system scope), the block that
  // finished it stores done_seq to done_flag[w]. For host-mapped words that a
  // host thread polls instead of waiting on a stream event.
  uint32_t* done_flag;
  uint32_t done_seq;
  int32_t inl_n;                   // > 0: nw, and the per-walker fields are in inl
  InlineDesc inl;
};

// A walker's direct sum in bias_force over nvis hills is split into chunks of
// kChunkHills consecutive hills (a function of nvis alone), so the split never
// depends on the batch the walker is in.
constexpr int kChunkHills = 64;
__host__ __device__ inline int64_t force_chunks(int64_t nvis) { return (nvis + kChunkHills - 1) / kChunkHills; }

// Chunk partials per walker for a history of `committed` hills; whether a
// launch of nw walkers takes the split or chained shape (which need the
// workspace); the workspace bytes of those shapes. A workspace must be zeroed
// when allocated (its first kForceArrivedBytes hold counters that the chained
// launch leaves at zero).
constexpr size_t kForceArrivedBytes = 256;
int force_blocks_per_walker(int64_t committed, int use_grid, int cv_only);
bool force_uses_workspace(int64_t nw, int64_t committed, int use_grid, int cv_only, int shape);
size_t force_workspace_bytes(int64_t nw, int nbw, int ndim);
hipError_t launch_bias_force(const Consts& K, const HistView& H, const ForceArgs& A, void* workspace,
                             hipStream_t stream);

}  // namespace abp

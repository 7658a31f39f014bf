// Host layer of libabp: the C-ABI declared in include/abp.h. It validates
// arguments (host-visible errors return before anything is enqueued), owns
// the device memory of a context, and enqueues the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "abp_serve_internal.h"

using abp::Consts;
using abp::HistView;

struct abp_ctx {
  int device = 0;
  abp_bias_desc desc{};
  Consts K{};
  int64_t committed = 0;      // visible hills
  int64_t reserved = 0;       // slots handed out (>= committed)
  double* c64 = nullptr;
  double* w64 = nullptr;
  double* l64 = nullptr;
  int4* rec32 = nullptr;
  double* grid = nullptr;
  float* grid32 = nullptr;            // FP32 mirror of the grid, refreshed after every grid update
  int32_t* err = nullptr;
  unsigned long long* clamped = nullptr;
  double* scratch = nullptr;
  size_t scratch_bytes = 0;
  void* fws = nullptr;                // bias_force: CV state, atom lists, partial sums
  size_t fws_bytes = 0;
  void* wt_buf = nullptr;             // bias_deposit (well-tempered): kWtChunk centres, their V and dV/ds
  uint32_t* dirty = nullptr;          // deposit tiles reached, by epoch (VALU-deposited 2-D / 3-D grids)
  uint32_t epoch = 0;
  int32_t force_shape = ABP_SHAPE_AUTO;

  HistView hist() const {
    HistView h;
    h.c64 = c64;
    h.w64 = w64;
    h.l64 = l64;
    h.rec32 = rec32;
    h.capacity = desc.capacity;
    return h;
  }
};

namespace {

thread_local std::string g_last_error;

abp_status fail(abp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

abp_status ok() {
  g_last_error.clear();
  return ABP_OK;
}

// Makes the context's device current for the scope and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  bool good = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    good = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(ABP_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr double kLog2e = 1.4426950408889634;
constexpr double kTwo32 = 4294967296.0;

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

abp_status check_desc(const abp_bias_desc* d) {
  if (!d) return fail(ABP_E_INVAL, "descriptor is NULL");
  if (d->ndim < 1 || d->ndim > 3) return fail(ABP_E_INVAL, "ndim must be 1..3 (got %d)", d->ndim);
  if (d->kernel != ABP_K_GAUSS && d->kernel != ABP_K_COMPACT) return fail(ABP_E_INVAL, "unknown kernel %d", d->kernel);
  if (d->kernel == ABP_K_COMPACT && (d->p < 1 || d->p > 64)) return fail(ABP_E_INVAL, "p must be 1..64 (got %d)", d->p);
  if (d->transform != ABP_T_PLAIN && d->transform != ABP_T_MABP)
    return fail(ABP_E_INVAL, "unknown transform %d", d->transform);
  if (d->transform == ABP_T_MABP) {
    if (!(d->b > 0.0 && d->b < 1.0)) return fail(ABP_E_INVAL, "mABP needs 0 < b < 1");
    if (!(d->c >= 0.0) || !std::isfinite(d->c)) return fail(ABP_E_INVAL, "mABP needs c >= 0");
    if (!finite_pos(d->kT)) return fail(ABP_E_INVAL, "mABP needs kT > 0");
  }
  const bool any_grid = d->grid_n[0] != 0 || d->grid_n[1] != 0 || d->grid_n[2] != 0;
  for (int i = 0; i < d->ndim; ++i) {
    if (d->periodic[i] != 0 && d->periodic[i] != 1) return fail(ABP_E_INVAL, "periodic[%d] must be 0 or 1", i);
    if (!finite_pos(d->width[i])) return fail(ABP_E_INVAL, "width[%d] must be > 0", i);
    if (!std::isfinite(d->lo[i]) || !std::isfinite(d->hi[i])) return fail(ABP_E_INVAL, "lo/hi[%d] not finite", i);
    if (!(d->hi[i] > d->lo[i])) return fail(ABP_E_INVAL, "axis %d needs hi > lo", i);
    if (any_grid && (d->grid_n[i] < 2 || d->grid_n[i] > (1 << 20)))
      return fail(ABP_E_INVAL, "grid_n[%d] must be 2..2^20 when a grid is requested", i);
  }
  if (!(d->wt_dT >= 0.0) || !std::isfinite(d->wt_dT)) return fail(ABP_E_INVAL, "wt_dT must be >= 0");
  if (d->quantize != 0 && d->quantize != 1) return fail(ABP_E_INVAL, "quantize must be 0 or 1");
  if (d->quantize && !any_grid) return fail(ABP_E_INVAL, "the quantised mode needs a grid (grid_n)");
  if (d->capacity < 1 || d->capacity > ((int64_t)1 << 34)) return fail(ABP_E_INVAL, "capacity out of range");
  return ABP_OK;
}

void make_consts(const abp_bias_desc& d, Consts& K) {
  std::memset(&K, 0, sizeof(K));
  K.ndim = d.ndim;
  K.kernel = d.kernel;
  K.p = d.kernel == ABP_K_COMPACT ? d.p : 1;
  K.transform = d.transform;
  K.quant = d.quantize;
  K.wt_dT = d.wt_dT;
  K.kT = d.kT;
  K.b = d.b;
  K.c = d.c;
  K.pl32 = (float)(K.p * kLog2e);
  K.pl64 = K.p * kLog2e;
  K.nodes = 1;
  for (int i = 0; i < 3; ++i) {
    K.lo[i] = d.lo[i];
    K.hi[i] = d.hi[i];
    K.period[i] = 1.0;
    K.inv_period[i] = 1.0;
  }
  for (int i = 0; i < d.ndim; ++i) {
    const bool per = d.periodic[i] != 0;
    K.periodic[i] = per ? 1 : 0;
    const double L = d.hi[i] - d.lo[i];
    if (per) {
      K.period[i] = L;
      K.inv_period[i] = 1.0 / L;
    }
    // FP32 working words (see Consts): the period in 2^32 steps, or the
    // half-width of the window [lo - E, hi + E] in 2^30 steps
    const double reach = std::max(0.5 * L, 16.0 * d.width[i]);
    const double half = 0.5 * L + reach;
    const double unit32 = per ? L / kTwo32 : half / 1073741824.0;
    K.fix_mid[i] = per ? 0.0 : 0.5 * (d.lo[i] + d.hi[i]);
    K.fix_scale[i] = per ? 0.0 : 1.0 / unit32;
    const double unit64 = per ? L : 1.0;            // FP64 path (turns)
    K.per64[i] = per ? 1.0 : 0.0;
    const double wdt = d.width[i];
    K.width[i] = wdt;
    K.inv_width[i] = 1.0 / wdt;
    if (d.kernel == ABP_K_GAUSS) {
      K.kf32[i] = (float)(kLog2e * unit32 * unit32 / (2.0 * wdt * wdt));
      K.gs32[i] = -unit32 / (wdt * wdt);
      K.kf64[i] = kLog2e * unit64 * unit64 / (2.0 * wdt * wdt);
      K.gs64[i] = -unit64 / (wdt * wdt);
    } else {
      K.ua32[i] = (float)(unit32 / wdt);
      K.gs32[i] = -2.0 * K.p / wdt;
      K.ua64[i] = unit64 / wdt;
      K.gs64[i] = -2.0 * K.p / wdt;
    }
    K.grid_n[i] = d.grid_n[i];
    if (d.grid_n[i] > 0) {
      K.grid_dx[i] = per ? L / d.grid_n[i] : L / (d.grid_n[i] - 1);
      K.inv_grid_dx[i] = 1.0 / K.grid_dx[i];
      K.nodes *= d.grid_n[i];
    }
  }
  if (d.grid_n[0] == 0) K.nodes = 0;
}

abp_status check_cv(const abp_ctx* ctx, const abp_cv_desc* cv, const abp_walkers* wk) {
  if (!cv || !wk) return fail(ABP_E_INVAL, "cv descriptor or walkers is NULL");
  if (cv->ncv != ctx->desc.ndim) return fail(ABP_E_INVAL, "ncv (%d) must equal the bias ndim (%d)", cv->ncv, ctx->desc.ndim);
  bool rmsd = false;
  for (int a = 0; a < cv->ncv; ++a) {
    const int k = cv->kind[a];
    if (k != ABP_CV_COM_DIST && k != ABP_CV_TORSION && k != ABP_CV_RMSD_OFF)
      return fail(ABP_E_INVAL, "unknown CV kind %d", k);
    if ((k == ABP_CV_TORSION) != (ctx->desc.periodic[a] != 0))
      return fail(ABP_E_INVAL, "CV %d: TORSION needs a periodic axis, COM_DIST/RMSD_OFF a non-periodic one", a);
    rmsd = rmsd || k == ABP_CV_RMSD_OFF;
  }
  if (!cv->list_off || !cv->list_idx) return fail(ABP_E_INVAL, "CV lists are NULL");
  if (rmsd && (!cv->ref_x || !cv->ref_y || !cv->ref_z)) return fail(ABP_E_INVAL, "RMSD_OFF needs reference positions");
  if (wk->nw < 0 || wk->nw > (1LL << 31) - 1) return fail(ABP_E_INVAL, "nw out of range");
  if (wk->nw > 0 && (!wk->atom_base || !wk->n_atoms || !wk->x || !wk->y || !wk->z || !wk->mass))
    return fail(ABP_E_INVAL, "walker pools are NULL");
  return ABP_OK;
}

abp::ForceArgs force_args(const abp_ctx* ctx, const abp_cv_desc* cv, const abp_walkers* wk) {
  abp::ForceArgs A;
  std::memset(&A, 0, sizeof(A));
  A.ncv = cv->ncv;
  for (int a = 0; a < 3; ++a) A.kind[a] = a < cv->ncv ? cv->kind[a] : 0;
  A.list_off = cv->list_off;
  A.list_idx = cv->list_idx;
  A.ref_x = cv->ref_x;
  A.ref_y = cv->ref_y;
  A.ref_z = cv->ref_z;
  A.nw = wk->nw;
  A.atom_base = wk->atom_base;
  A.n_atoms = wk->n_atoms;
  A.x = wk->x;
  A.y = wk->y;
  A.z = wk->z;
  A.mass = wk->mass;
  A.fx = wk->fx;
  A.fy = wk->fy;
  A.fz = wk->fz;
  A.n_visible_default = ctx->committed;
  A.err = ctx->err;
  return A;
}

// Well-tempered deposits run in chunks of this many hills through a buffer
// allocated with the context (so bias_deposit allocates nothing for them).
constexpr int64_t kWtChunk = 16384;

size_t wt_buffer_bytes(int ndim) { return (size_t)kWtChunk * (2 * ndim + 1) * sizeof(double); }

abp_status grow_scratch(abp_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return ABP_OK;
  if (ctx->scratch) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(ctx->scratch));
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  if (hipMalloc(&ctx->scratch, bytes) != hipSuccess) {
    ctx->scratch = nullptr;
    return fail(ABP_E_NOMEM, "cannot allocate %zu bytes of grid scratch", bytes);
  }
  ctx->scratch_bytes = bytes;
  return ABP_OK;
}

// Workspace of a direct-sum bias_force launch (grow-only).
abp_status force_workspace(abp_ctx* ctx, int64_t nw, int nbw) {
  const size_t pb = abp::force_workspace_bytes(nw, nbw, ctx->desc.ndim);
  if (pb == 0) return ABP_OK;
  if (pb > ctx->fws_bytes) {
    HIP_TRY(hipDeviceSynchronize());
    if (ctx->fws) HIP_TRY(hipFree(ctx->fws));
    ctx->fws = nullptr;
    ctx->fws_bytes = 0;
    if (hipMalloc(&ctx->fws, pb) != hipSuccess) return fail(ABP_E_NOMEM, "cannot allocate bias_force workspace");
    ctx->fws_bytes = pb;
    HIP_TRY(hipMemset(ctx->fws, 0, pb));
  }
  return ABP_OK;
}

// Adds committed hills [k0, k1) to the grid.
// Adds committed hills [k0, k1) to the node arrays `grid` and refreshes the
// FP32 mirror `grid32` (when not NULL).
abp_status grid_add_to(abp_ctx* ctx, double* grid, float* grid32, int64_t k0, int64_t k1, hipStream_t stream) {
  if (!grid || k1 <= k0) return ABP_OK;
  const size_t need = abp::grid_deposit_scratch_bytes(ctx->K, k1 - k0);
  abp_status st = grow_scratch(ctx, need);
  if (st != ABP_OK) return st;
  // tiles the deposit reaches are marked with a fresh epoch; the mirror
  // refresh then rewrites only their entries (compact hills on the VALU deposit)
  if (++ctx->epoch == 0) ctx->epoch = 1;
  HIP_TRY(abp::launch_grid_deposit(ctx->K, ctx->hist(), k0, k1, grid, need ? ctx->scratch : nullptr, ctx->dirty,
                                   ctx->epoch, stream));
  if (grid32) HIP_TRY(abp::launch_grid_mirror(ctx->K, grid, grid32, ctx->dirty, ctx->epoch, stream));
  return ABP_OK;
}

abp_status grid_add(abp_ctx* ctx, int64_t k0, int64_t k1, hipStream_t stream) {
  return grid_add_to(ctx, ctx->grid, ctx->grid32, k0, k1, stream);
}

void free_all(abp_ctx* ctx) {
  if (ctx->c64) (void)hipFree(ctx->c64);
  if (ctx->w64) (void)hipFree(ctx->w64);
  if (ctx->l64) (void)hipFree(ctx->l64);
  if (ctx->rec32) (void)hipFree(ctx->rec32);
  if (ctx->grid) (void)hipFree(ctx->grid);
  if (ctx->grid32) (void)hipFree(ctx->grid32);
  if (ctx->err) (void)hipFree(ctx->err);
  if (ctx->clamped) (void)hipFree(ctx->clamped);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->fws) (void)hipFree(ctx->fws);
  if (ctx->wt_buf) (void)hipFree(ctx->wt_buf);
  if (ctx->dirty) (void)hipFree(ctx->dirty);
}

}  // namespace

extern "C" {

abp_status abp_create(const abp_bias_desc* desc, int device, abp_ctx** out) {
  if (!out) return fail(ABP_E_INVAL, "out is NULL");
  *out = nullptr;
  abp_status st = check_desc(desc);
  if (st != ABP_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(ABP_E_INVAL, "device %d not available (%d devices)", device, ndev);
  DeviceGuard guard(device);
  if (!guard.good) return fail(ABP_E_DEVICE, "cannot select device %d", device);
  abp_ctx* ctx = new (std::nothrow) abp_ctx();
  if (!ctx) return fail(ABP_E_NOMEM, "host allocation failed");
  ctx->device = device;
  ctx->desc = *desc;
  for (int i = desc->ndim; i < 3; ++i) {
    ctx->desc.periodic[i] = 0;
    ctx->desc.grid_n[i] = 0;
  }
  make_consts(ctx->desc, ctx->K);
  const int64_t cap = desc->capacity;
  bool good = hipMalloc(&ctx->c64, sizeof(double) * desc->ndim * cap) == hipSuccess &&
              hipMalloc(&ctx->w64, sizeof(double) * cap) == hipSuccess &&
              hipMalloc(&ctx->l64, sizeof(double) * cap) == hipSuccess &&
              hipMalloc(&ctx->rec32, sizeof(int4) * cap) == hipSuccess &&
              hipMalloc(&ctx->err, sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&ctx->clamped, sizeof(unsigned long long)) == hipSuccess;
  if (good && desc->wt_dT > 0.0) good = hipMalloc(&ctx->wt_buf, wt_buffer_bytes(desc->ndim)) == hipSuccess;
  if (good && ctx->K.nodes > 0)
    good = hipMalloc(&ctx->grid, sizeof(double) * (size_t)(ctx->K.nodes << desc->ndim)) == hipSuccess &&
           hipMalloc(&ctx->grid32, sizeof(float) * abp::grid_mirror_floats(ctx->K)) == hipSuccess;
  const size_t ntiles = abp::grid_dirty_tiles(ctx->K);
  if (good && ntiles)
    good = hipMalloc(&ctx->dirty, sizeof(uint32_t) * ntiles) == hipSuccess &&
           hipMemset(ctx->dirty, 0, sizeof(uint32_t) * ntiles) == hipSuccess;
  if (good) {
    good = hipMemset(ctx->err, 0, sizeof(int32_t)) == hipSuccess &&
           hipMemset(ctx->clamped, 0, sizeof(unsigned long long)) == hipSuccess &&
           (!ctx->grid || hipMemset(ctx->grid, 0, sizeof(double) * (size_t)(ctx->K.nodes << desc->ndim)) == hipSuccess) &&
           (!ctx->grid32 || hipMemset(ctx->grid32, 0, sizeof(float) * abp::grid_mirror_floats(ctx->K)) == hipSuccess) &&
           abp::launch_hist_init(ctx->hist(), desc->ndim, nullptr) == hipSuccess &&
           hipDeviceSynchronize() == hipSuccess;
  }
  if (!good) {
    free_all(ctx);
    delete ctx;
    return fail(ABP_E_NOMEM, "device allocation failed (capacity %lld)", (long long)cap);
  }
  st = abp::noalloc_setup(device);      // bias_force_noalloc's static workspace on this device
  if (st != ABP_OK) {
    free_all(ctx);
    delete ctx;
    return st;
  }
  *out = ctx;
  return ok();
}

abp_status abp_destroy(abp_ctx* ctx) {
  if (!ctx) return ok();
  DeviceGuard guard(ctx->device);
  (void)hipDeviceSynchronize();
  free_all(ctx);
  delete ctx;
  return ok();
}

abp_status bias_deposit(abp_ctx* ctx, int64_t n, abp_dtype dtype, const void* centers,
                        const void* heights, abp_stream stream) {
  if (!ctx) return fail(ABP_E_INVAL, "context is NULL");
  if (n < 0) return fail(ABP_E_INVAL, "n must be >= 0");
  if (dtype != ABP_F32 && dtype != ABP_F64) return fail(ABP_E_INVAL, "unknown dtype");
  if (n == 0) return ok();
  if (!centers || !heights) return fail(ABP_E_INVAL, "centers or heights is NULL");
  if (ctx->reserved != ctx->committed)
    return fail(ABP_E_INVAL, "reserved slots are pending; commit them before bias_deposit");
  if (ctx->committed + n > ctx->desc.capacity)
    return fail(ABP_E_CAPACITY, "history capacity %lld exceeded", (long long)ctx->desc.capacity);
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const int64_t k0 = ctx->committed;
  if (ctx->desc.wt_dT > 0.0 && k0 > 0) {
    // well-tempered heights: the bias at each new centre, an FP64 direct sum
    // over the k0 hills committed before this call (not over earlier chunks of
    // it), in the centres' dtype. Per chunk: copy its centres out of the
    // [ndim][n] array, sum, append; the stream orders the buffer's reuse.
    const int nd = ctx->desc.ndim;
    const size_t esz = dtype == ABP_F64 ? sizeof(double) : sizeof(float);
    char* buf = static_cast<char*>(ctx->wt_buf);
    for (int64_t off = 0; off < n; off += kWtChunk) {
      const int64_t c = std::min<int64_t>(kWtChunk, n - off);
      char* cen = buf;
      char* vb = buf + (size_t)c * nd * esz;
      char* db = vb + (size_t)c * esz;
      HIP_TRY(hipMemcpy2DAsync(cen, (size_t)c * esz, static_cast<const char*>(centers) + (size_t)off * esz,
                               (size_t)n * esz, (size_t)c * esz, (size_t)nd, hipMemcpyDeviceToDevice, s));
      HIP_TRY(abp::launch_direct_sum(ctx->K, ctx->hist(), k0, ABP_PREC_FP64, c, dtype == ABP_F64 ? 1 : 0, cen, vb,
                                     db, s));
      HIP_TRY(abp::launch_hist_append(ctx->K, ctx->hist(), k0 + off, c, dtype == ABP_F64 ? 1 : 0, cen,
                                      static_cast<const char*>(heights) + (size_t)off * esz, vb, ctx->err, s));
    }
  } else {
    HIP_TRY(abp::launch_hist_append(ctx->K, ctx->hist(), k0, n, dtype == ABP_F64 ? 1 : 0, centers, heights,
                                    nullptr, ctx->err, s));
  }
  ctx->committed += n;
  ctx->reserved = ctx->committed;
  abp_status st = grid_add(ctx, k0, ctx->committed, s);
  if (st != ABP_OK) return st;
  return ok();
}

abp_status bias_eval(abp_ctx* ctx, abp_eval_mode mode, abp_prec prec, int64_t nq, abp_dtype dtype,
                     const void* q, int64_t n_visible, void* V, void* dVds, abp_stream stream) {
  if (!ctx) return fail(ABP_E_INVAL, "context is NULL");
  if (nq < 0) return fail(ABP_E_INVAL, "nq must be >= 0");
  if (dtype != ABP_F32 && dtype != ABP_F64) return fail(ABP_E_INVAL, "unknown dtype");
  if (prec != ABP_PREC_FP32_KAHAN && prec != ABP_PREC_FP32_NAIVE && prec != ABP_PREC_FP64)
    return fail(ABP_E_INVAL, "unknown precision mode");
  if (mode != ABP_EVAL_DIRECT && mode != ABP_EVAL_GRID) return fail(ABP_E_INVAL, "unknown eval mode");
  if (nq > ((int64_t)1 << 40)) return fail(ABP_E_INVAL, "nq too large");
  if (nq == 0) return ok();
  if (!q || !V || !dVds) return fail(ABP_E_INVAL, "q, V or dVds is NULL");
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const int f64 = dtype == ABP_F64 ? 1 : 0;
  if (mode == ABP_EVAL_GRID) {
    if (!ctx->grid) return fail(ABP_E_INVAL, "context has no grid");
    if (n_visible != -1) return fail(ABP_E_INVAL, "GRID mode covers all committed hills (n_visible must be -1)");
    HIP_TRY(abp::launch_grid_eval(ctx->K, ctx->grid, prec == ABP_PREC_FP64 ? nullptr : ctx->grid32, nq, f64, q, V,
                                  dVds, ctx->clamped, s));
    return ok();
  }
  if (n_visible < -1 || n_visible > ctx->committed)
    return fail(ABP_E_INVAL, "n_visible %lld outside [-1, %lld]", (long long)n_visible, (long long)ctx->committed);
  const int64_t nvis = n_visible < 0 ? ctx->committed : n_visible;
  HIP_TRY(abp::launch_direct_sum(ctx->K, ctx->hist(), nvis, prec, nq, f64, q, V, dVds, s));
  return ok();
}

abp_status cv_compute(abp_ctx* ctx, const abp_cv_desc* cv, const abp_walkers* walkers, double* s,
                      abp_stream stream) {
  if (!ctx) return fail(ABP_E_INVAL, "context is NULL");
  abp_status st = check_cv(ctx, cv, walkers);
  if (st != ABP_OK) return st;
  if (walkers->nw == 0) return ok();
  if (!s) return fail(ABP_E_INVAL, "s is NULL");
  DeviceGuard guard(ctx->device);
  abp::ForceArgs A = force_args(ctx, cv, walkers);
  A.s = s;
  A.cv_only = 1;
  A.prec = ABP_PREC_FP64;
  HIP_TRY(abp::launch_bias_force(ctx->K, ctx->hist(), A, nullptr, (hipStream_t)stream));
  return ok();
}

abp_status bias_force(abp_ctx* ctx, abp_eval_mode mode, abp_prec prec, const abp_cv_desc* cv,
                      const abp_walkers* walkers, const int64_t* n_visible,
                      const int64_t* deposit_slot, const double* deposit_height,
                      double* s, double* V, double* dVds, abp_stream stream) {
  abp::ForceCall call;
  abp_status st = abp::prepare_force(ctx, mode, prec, cv, walkers, n_visible, deposit_slot, deposit_height, s, V,
                                     dVds, &call);
  if (st != ABP_OK || call.nothing) return st;
  DeviceGuard guard(ctx->device);
  if (call.workspace_bytes) {
    const int nbw = abp::force_blocks_per_walker(ctx->committed, 0, 0);
    st = force_workspace(ctx, walkers->nw, nbw);
    if (st != ABP_OK) return st;
  }
  HIP_TRY(abp::launch_bias_force(ctx->K, ctx->hist(), call.A, ctx->fws, (hipStream_t)stream));
  return ok();
}

abp_status abp_set_force_shape(abp_ctx* ctx, int32_t shape) {
  if (!ctx) return fail(ABP_E_INVAL, "context is NULL");
  if (shape < ABP_SHAPE_AUTO || shape > ABP_SHAPE_CHAIN) return fail(ABP_E_INVAL, "unknown force shape %d", shape);
  ctx->force_shape = shape;
  return ok();
}

abp_status abp_reserve(abp_ctx* ctx, int64_t n, int64_t* first) {
  if (!ctx || !first) return fail(ABP_E_INVAL, "context or first is NULL");
  if (n < 0) return fail(ABP_E_INVAL, "n must be >= 0");
  if (ctx->reserved + n > ctx->desc.capacity)
    return fail(ABP_E_CAPACITY, "history capacity %lld exceeded", (long long)ctx->desc.capacity);
  *first = ctx->reserved;
  ctx->reserved += n;
  return ok();
}

abp_status abp_commit(abp_ctx* ctx, int64_t upto, abp_stream stream) {
  if (!ctx) return fail(ABP_E_INVAL, "context is NULL");
  if (upto < ctx->committed || upto > ctx->reserved)
    return fail(ABP_E_INVAL, "commit target %lld outside [%lld, %lld]", (long long)upto,
                (long long)ctx->committed, (long long)ctx->reserved);
  if (upto == ctx->committed) return ok();
  DeviceGuard guard(ctx->device);
  const int64_t k0 = ctx->committed;
  ctx->committed = upto;
  abp_status st = grid_add(ctx, k0, upto, (hipStream_t)stream);
  if (st != ABP_OK) return st;
  return ok();
}

abp_status abp_sync(abp_ctx* ctx, abp_stream stream) {
  if (!ctx) return fail(ABP_E_INVAL, "context is NULL");
  DeviceGuard guard(ctx->device);
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  int32_t word = 0;
  HIP_TRY(hipMemcpy(&word, ctx->err, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (word) {
    const int32_t zero = 0;
    HIP_TRY(hipMemcpy(ctx->err, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
    if (word & abp::kErrIndex) return fail(ABP_E_INDEX, "device reported an atom index out of range or an invalid list");
    if (word & abp::kErrNonfinite) return fail(ABP_E_NONFINITE, "device reported a non-finite input or negative height");
    return fail(ABP_E_INVAL, "device reported an invalid walker description");
  }
  return ok();
}

int64_t abp_num_hills(const abp_ctx* ctx) { return ctx ? ctx->committed : -1; }

abp_status abp_hills_export(abp_ctx* ctx, double* centers_host, double* heights_host, int64_t* n) {
  if (!ctx || !n || !centers_host || !heights_host) return fail(ABP_E_INVAL, "NULL argument");
  if (*n < ctx->committed) return fail(ABP_E_INVAL, "host arrays hold %lld hills, %lld needed", (long long)*n,
                                       (long long)ctx->committed);
  DeviceGuard guard(ctx->device);
  HIP_TRY(hipDeviceSynchronize());
  const int64_t m = ctx->committed;
  for (int i = 0; i < ctx->desc.ndim; ++i)
    if (m) HIP_TRY(hipMemcpy(centers_host + i * m, ctx->c64 + i * ctx->desc.capacity, sizeof(double) * m,
                             hipMemcpyDeviceToHost));
  if (m) HIP_TRY(hipMemcpy(heights_host, ctx->w64, sizeof(double) * m, hipMemcpyDeviceToHost));
  *n = m;
  return ok();
}

abp_status abp_grid_export(abp_ctx* ctx, double* H_host, int64_t n_values) {
  if (!ctx || !H_host) return fail(ABP_E_INVAL, "NULL argument");
  if (!ctx->grid) return fail(ABP_E_INVAL, "context has no grid");
  const int64_t need = ctx->K.nodes << ctx->desc.ndim;
  if (n_values < need) return fail(ABP_E_INVAL, "H holds %lld values, %lld needed", (long long)n_values, (long long)need);
  DeviceGuard guard(ctx->device);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(H_host, ctx->grid, sizeof(double) * need, hipMemcpyDeviceToHost));
  return ok();
}

const char* abp_status_str(abp_status status) {
  switch (status) {
    case ABP_OK: return "ABP_OK";
    case ABP_E_INVAL: return "ABP_E_INVAL";
    case ABP_E_NOMEM: return "ABP_E_NOMEM";
    case ABP_E_CAPACITY: return "ABP_E_CAPACITY";
    case ABP_E_DEVICE: return "ABP_E_DEVICE";
    case ABP_E_INDEX: return "ABP_E_INDEX";
    case ABP_E_NONFINITE: return "ABP_E_NONFINITE";
    case ABP_E_BUSY: return "ABP_E_BUSY";
  }
  return "ABP_E_UNKNOWN";
}

const char* abp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace abp {

CtxView ctx_view(abp_ctx* ctx) {
  CtxView v;
  v.K = ctx->K;
  v.H = ctx->hist();
  v.grid = ctx->grid;
  v.grid32 = ctx->grid32;
  v.grid_doubles = ctx->grid ? (size_t)(ctx->K.nodes << ctx->desc.ndim) : 0;
  v.err = ctx->err;
  v.device = ctx->device;
  return v;
}

int64_t ctx_reserved(const abp_ctx* ctx) { return ctx->reserved; }

abp_status prepare_force(abp_ctx* ctx, abp_eval_mode mode, abp_prec prec, const abp_cv_desc* cv,
                         const abp_walkers* walkers, const int64_t* n_visible, const int64_t* deposit_slot,
                         const double* deposit_height, double* s, double* V, double* dVds, ForceCall* out) {
  out->nothing = true;
  out->workspace_bytes = 0;
  if (!ctx) return fail(ABP_E_INVAL, "context is NULL");
  abp_status st = check_cv(ctx, cv, walkers);
  if (st != ABP_OK) return st;
  if (prec != ABP_PREC_FP32_KAHAN && prec != ABP_PREC_FP32_NAIVE && prec != ABP_PREC_FP64)
    return fail(ABP_E_INVAL, "unknown precision mode");
  if (mode != ABP_EVAL_DIRECT && mode != ABP_EVAL_GRID) return fail(ABP_E_INVAL, "unknown eval mode");
  if (mode == ABP_EVAL_GRID && !ctx->grid) return fail(ABP_E_INVAL, "context has no grid");
  if (walkers->nw == 0) return ok();
  if (!s || !V || !dVds) return fail(ABP_E_INVAL, "s, V or dVds is NULL");
  if (!walkers->fx || !walkers->fy || !walkers->fz) return fail(ABP_E_INVAL, "force arrays are NULL");
  ForceArgs A = force_args(ctx, cv, walkers);
  A.n_visible = n_visible;
  A.deposit_slot = deposit_slot;
  A.deposit_height = deposit_height;
  A.s = s;
  A.V = V;
  A.dVds = dVds;
  A.use_grid = mode == ABP_EVAL_GRID ? 1 : 0;
  A.grid = ctx->grid;
  A.prec = prec;
  A.shape = ctx->force_shape;
  out->A = A;
  out->device = ctx->device;
  out->K = ctx->K;
  out->H = ctx->hist();
  if (force_uses_workspace(walkers->nw, ctx->committed, A.use_grid, 0, A.shape))
    out->workspace_bytes = force_workspace_bytes(walkers->nw, force_blocks_per_walker(ctx->committed, 0, 0),
                                                 ctx->desc.ndim);
  out->nothing = false;
  return ok();
}

abp_status ctx_reserve_commit(abp_ctx* ctx, int64_t n) {
  if (!ctx->grid || n <= 0) return ok();
  DeviceGuard guard(ctx->device);
  return grow_scratch(ctx, abp::grid_deposit_scratch_bytes(ctx->K, n));
}

abp_status ctx_commit_hills(abp_ctx* ctx, int64_t upto) {
  if (upto < ctx->committed || upto > ctx->reserved)
    return fail(ABP_E_INVAL, "commit target %lld outside [%lld, %lld]", (long long)upto,
                (long long)ctx->committed, (long long)ctx->reserved);
  ctx->committed = upto;
  return ok();
}

abp_status ctx_grid_add(abp_ctx* ctx, double* grid, float* grid32, int64_t k0, int64_t k1, hipStream_t stream) {
  if (k0 < 0 || k1 > ctx->committed) return fail(ABP_E_INVAL, "hills [%lld, %lld) are not committed", (long long)k0,
                                                 (long long)k1);
  DeviceGuard guard(ctx->device);
  return grid_add_to(ctx, grid, grid32, k0, k1, stream);
}

abp_status set_error(abp_status st, const char* msg) {
  if (st == ABP_OK) return ok();
  return fail(st, "%s", msg);
}

}  // namespace abp

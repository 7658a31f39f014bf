/* abp.h - C-ABI of libabp.so, the GPU (AMD gfx950) library for the bias-force
 * hot path of adaptive biasing potentials with compact or Gaussian hills.
 *
 * Method: Dickson, de Waal, Ramjan, Xu, Rothbart, "A fast, open source
 * implementation of adaptive biasing potentials uncovers a ligand design
 * strategy for the chromatin regulator BRD4", arXiv:1609.09833. Equation
 * names below refer to its Supplemental Material, section "Streamlined bias
 * potential updates" (eqs. apfm, btraj-grad, histos, ghill, update,
 * compacthill, Cupdate), section "Convergence with S_a^p" (width relations)
 * and section "Definition of the RMSD".
 *
 * The problem the calls solve is the one the paper's engine hands to its bias
 * routine every MD step (section "Minimization of Interprocess
 * Communications"): given the coordinates of the atoms that enter the
 * collective variables (CVs), update the bias from the visited CV value and
 * return the bias force on exactly those atoms, which the engine adds to its
 * own forces.
 *
 * Conventions shared by every call
 * - Array arguments are DEVICE pointers owned by the caller, unless a comment
 *   says "host". The library never frees them and never uses them after the
 *   work it enqueued on `stream` has run.
 * - CV-space arrays are dimension-major: x[i*n + j] is coordinate i of item j.
 * - All compute calls are asynchronous on `stream` (a hipStream_t; NULL means
 *   the null stream). Errors that the host can see (bad descriptors, NULL
 *   pointers, negative sizes, capacity) are returned synchronously before
 *   anything is enqueued, and then nothing is enqueued.
 * - Errors only the device can see (atom index out of range, non-finite
 *   input, a negative hill height) set a per-context device error word; the
 *   affected walker or item is skipped and the rest completes. abp_sync()
 *   returns that error and clears the word.
 * - A context is not thread-safe: use one host thread per context, or lock.
 * - On error, abp_last_error() returns a message for the calling thread.
 */
#ifndef ABP_H
#define ABP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct abp_ctx abp_ctx;   /* opaque: owns the hill history, grids, workspace */
typedef void* abp_stream;         /* a hipStream_t */

typedef enum {
  ABP_OK = 0,
  ABP_E_INVAL = 1,       /* bad argument or descriptor */
  ABP_E_NOMEM = 2,       /* device allocation failed */
  ABP_E_CAPACITY = 3,    /* the history would exceed its capacity */
  ABP_E_DEVICE = 4,      /* a HIP runtime call failed */
  ABP_E_INDEX = 5,       /* device-detected: atom index out of range or list not valid */
  ABP_E_NONFINITE = 6,   /* device-detected: non-finite position/mass/height, or negative height */
  ABP_E_BUSY = 7         /* the server holds as many requests as it can stage; poll, then retry */
} abp_status;

typedef enum { ABP_F32 = 0, ABP_F64 = 1 } abp_dtype;

/* Arithmetic of the hill sum (see bias_eval). */
typedef enum {
  ABP_PREC_FP32_KAHAN = 0,  /* FP32 terms, compensated (Kahan) accumulation */
  ABP_PREC_FP32_NAIVE = 1,  /* FP32 terms, plain FP32 accumulation */
  ABP_PREC_FP64 = 2         /* FP64 throughout */
} abp_prec;

/* Hill shape per CV axis; the multi-dimensional hill is the product over axes
 * (eq. ghill is already such a product; eq. compacthill and the sentence after
 * it define the product for the compact kernel). */
typedef enum {
  ABP_K_GAUSS = 0,    /* exp(-delta^2/(2 sigma^2)): eq. ghill with alpha = sqrt(2) sigma */
  ABP_K_COMPACT = 1   /* S_a^p(delta) = e^p exp(-p/(1-(delta/a)^2)) for |delta/a| < 1, else 0 (eq. compacthill) */
} abp_kernel;

typedef enum {
  ABP_T_PLAIN = 0,    /* V = h (the accumulated hill sum) */
  ABP_T_MABP = 1      /* V = kT b/(1-b) ln(c(1-b) h + 1), eq. apfm; gradient eq. btraj-grad */
} abp_transform;

typedef enum {
  ABP_EVAL_DIRECT = 0,  /* sum over the deposited hills (eq. histos with the integral over time
                           replaced by the deposits) */
  ABP_EVAL_GRID = 1     /* grid accumulated per eq. update / eq. Cupdate, read back by cubic
                           Hermite interpolation */
} abp_eval_mode;

typedef enum {
  ABP_CV_COM_DIST = 0,  /* distance between the centres of mass of two atom groups */
  ABP_CV_TORSION = 1,   /* dihedral angle of four atoms, IUPAC sign, (-pi, pi] */
  ABP_CV_RMSD_OFF = 2   /* offset RMSD of section "Definition of the RMSD" (no alignment) */
} abp_cv_kind;

/* Definition of the bias, fixed at abp_create. */
typedef struct {
  int32_t ndim;          /* CV dimension, 1..3 */
  int32_t periodic[3];   /* 1: axis i is periodic on [lo_i, hi_i) with period hi_i - lo_i
                            (minimum-image displacements) */
  double lo[3], hi[3];   /* hi_i > lo_i on every axis. Non-periodic axes: the CV range [lo_i, hi_i]
                            (the grid's range, nodes at both ends). The FP32 hill sums hold a
                            non-periodic coordinate as a 32-bit fixed-point offset inside
                            [lo_i - E_i, hi_i + E_i], E_i = max((hi_i - lo_i)/2, 16 width_i),
                            in steps of (hi_i - lo_i + 2 E_i)/2^31, and take a value beyond
                            that window at its edge; the FP64 sums and the history keep
                            every value as given */
  int32_t kernel;        /* abp_kernel */
  double width[3];       /* Gaussian: sigma_i > 0; compact: a_i > 0 (per-axis a, as the paper allows) */
  int32_t p;             /* compact kernel exponent, 1..64 (ignored for Gaussian) */
  int32_t transform;     /* abp_transform */
  double kT;             /* beta^{-1} = k_B T in energy units (mABP) */
  double b, c;           /* mABP parameters: 0 < b < 1, c >= 0 (eq. apfm) */
  int32_t grid_n[3];     /* grid nodes per axis (>= 2 each), or all 0 for no grid.
                            Periodic axis: nodes lo + j (hi-lo)/n, j < n.
                            Non-periodic: nodes lo + j (hi-lo)/(n-1), j < n. */
  int32_t quantize;      /* 0, or 1 for the paper's quantised mode (needs a grid): the
                            CV value is replaced by its nearest grid node xi* (section
                            "Streamlined bias potential updates", before eq. update),
                            node index floor((s - lo)/dx + 1/2), taken mod n on a
                            periodic axis and clamped to [0, n-1] otherwise, with
                            dx the node spacing. Deposited hills are centred on
                            xi*; GRID evaluation looks up the value and first-
                            derivative arrays at the query's xi* (no interpolation)
                            and DIRECT evaluation sums the hills at xi*. */
  int64_t capacity;      /* maximum number of hills the history holds, >= 1 */
  double wt_dT;          /* 0, or k_B dT > 0 (energy units) for well-tempered metadynamics
                            heights: a deposited hill's height is multiplied by
                            exp(-V(xi*)/wt_dT), V the bias at its centre before it is
                            added (the WTmetaD hill-height factor, section "Streamlined
                            bias potential updates" after eq. Cupdate) */
} abp_bias_desc;

/* CV definition for a batch of nw walkers (device arrays, caller-owned).
 * The atom lists of CV `a`, slot `t` (0 or 1), walker `w` are
 *   list_idx[list_off[(a*2 + t)*(nw+1) + w] .. list_off[(a*2 + t)*(nw+1) + w + 1])
 * holding walker-local atom indices (0 <= idx < n_atoms[w]).
 *   COM_DIST: slot 0 = group A, slot 1 = group B, both non-empty and strictly increasing.
 *   TORSION:  slot 0 = exactly 4 distinct atoms in dihedral order, slot 1 empty.
 *   RMSD_OFF: slot 0 = the atoms, strictly increasing, non-empty; slot 1 empty.
 *             ref_x/y/z[e] is the reference position of list entry e.
 * CV a is coordinate a of the bias (ncv == ndim). TORSION requires a periodic
 * axis; COM_DIST and RMSD_OFF require a non-periodic one. Positions are taken
 * as unwrapped (no minimum image is applied between atoms). */
typedef struct {
  int32_t ncv;
  int32_t kind[3];
  const int32_t* list_off;
  const int32_t* list_idx;
  const float* ref_x;
  const float* ref_y;
  const float* ref_z;     /* may be NULL when no CV is RMSD_OFF */
} abp_cv_desc;

/* Walker pools (device, caller-owned, SoA FP32). Walker w owns atoms
 * [atom_base[w], atom_base[w] + n_atoms[w]) of the pools. Walkers in one call
 * must not share atoms. Forces are ACCUMULATED: f += bias force. */
typedef struct {
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
} abp_walkers;

/* Create a context on HIP device `device`: allocates the hill history
 * (capacity hills, FP64 master copy plus an FP32 working copy) and, if
 * grid_n is set, the 2^ndim FP64 grid arrays (value, first and mixed
 * derivatives), all zero (the initial condition h = h' = 0 of eq. update).
 * Returns ABP_E_INVAL for a bad descriptor, ABP_E_NOMEM if allocation fails. */
abp_status abp_create(const abp_bias_desc* desc, int device, abp_ctx** out);

/* Wait for the context's work and free everything it owns. NULL is a no-op. */
abp_status abp_destroy(abp_ctx* ctx);

/* Append n hills (centers [ndim][n], heights [n], both `dtype`) to the
 * history, in order, and add them to the grid if there is one (eq. update /
 * eq. Cupdate summed over the batch). Heights must be finite and >= 0: a hill
 * that is not gets height 0 and raises ABP_E_NONFINITE at abp_sync. Returns
 * ABP_E_CAPACITY (nothing appended) if the history would overflow. n = 0 is a
 * no-op. The appended hills are visible to work enqueued after this call on
 * the same stream. With wt_dT > 0 every height is scaled by
 * exp(-V/wt_dT), V the bias at the hill's centre from the FP64 direct sum over
 * the hills committed before this call (one deposit per call is the
 * per-step rule exactly; in a batch the hills do not see each other). */
abp_status bias_deposit(abp_ctx* ctx, int64_t n, abp_dtype dtype, const void* centers,
                        const void* heights, abp_stream stream);

/* Evaluate the bias V and its gradient dV/ds at nq CV points q[ndim][nq].
 * mode DIRECT sums hills [0, n_visible) (n_visible = -1: all committed
 * hills); mode GRID interpolates the grid (n_visible must be -1) with
 * tensor-product cubic Hermite polynomials from the value and derivative
 * arrays, clamping non-periodic coordinates to [lo, hi].
 * Outputs V[nq] and dVds[ndim][nq] have the same dtype as q.
 * prec selects the hill-sum arithmetic. GRID: ABP_PREC_FP64 interpolates the
 * FP64 node arrays in FP64; the FP32 modes interpolate their FP32 mirror
 * (refreshed after every grid update; half the gathered bytes) in FP32 after
 * locating the cell in FP64 (errors of 2^-24 of the values, and of 2^-24 |V|
 * over the node spacing in the gradient).
 * The result for a query depends only on that query and the hills, not on nq
 * or its position in the batch. A query with a non-finite coordinate gets NaN
 * in V and all of its dVds entries (every mode and precision; it is not an
 * error and is not counted as clamped). nq = 0 is a no-op. */
abp_status bias_eval(abp_ctx* ctx, abp_eval_mode mode, abp_prec prec, int64_t nq, abp_dtype dtype,
                     const void* q, int64_t n_visible, void* V, void* dVds, abp_stream stream);

/* Compute the CVs s[ncv][nw] (FP64) of a batch of walkers. COM reductions
 * use FP64 accumulators. Walkers with invalid lists or non-finite inputs are
 * skipped (s left unwritten) and flag the context's error word. */
abp_status cv_compute(abp_ctx* ctx, const abp_cv_desc* cv, const abp_walkers* walkers, double* s,
                      abp_stream stream);

/* The whole bias-force step for a batch of walkers: CVs -> bias and
 * gradient at s (DIRECT: hills [0, n_visible[w]), or all committed hills if
 * n_visible is NULL, a value outside [0, committed] also meaning all; GRID:
 * interpolation, or the nearest-node look-up in the quantised mode) ->
 * transform -> chain rule F_j += -sum_a dV/ds_a ds_a/dx_j on the CV atoms
 * only ("Minimization of Interprocess Communications": only CV atoms are read
 * and written; forces are added to the caller's arrays).
 * Writes s[ncv][nw], V[nw], dVds[ncv][nw] (FP64, device arrays). A walker
 * whose lists break abp_cv_desc's rules or whose CV atoms hold non-finite
 * values is skipped (outputs and forces untouched) and flags the error word;
 * the other walkers are unaffected.
 * deposit_slot (optional, [nw]): if deposit_slot[w] >= 0, the hill centred at
 * walker w's s (its nearest node in the quantised mode) with height
 * deposit_height[w] (NULL: 1.0; times exp(-V[w]/wt_dT) when wt_dT > 0) is
 * written to that history slot, which must have been reserved with
 * abp_reserve and is made visible by abp_commit.
 * Launches: one for the grid form and for histories of up to 16,384 hills;
 * for longer ones three (CV, hill sum, finish) or, for one or two walkers,
 * one chained launch; both use a workspace the context allocates and clears
 * on first need (abp_set_force_shape fixes the shape). A walker's result is
 * bitwise the same in any batch and any shape. Once the workspace exists the
 * call enqueues kernels only, so it can be captured in a HIP graph. Calls
 * that share a context's workspace must not run concurrently on different
 * streams. */
abp_status bias_force(abp_ctx* ctx, abp_eval_mode mode, abp_prec prec, const abp_cv_desc* cv,
                      const abp_walkers* walkers, const int64_t* n_visible,
                      const int64_t* deposit_slot, const double* deposit_height,
                      double* s, double* V, double* dVds, abp_stream stream);

/* bias_force for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, kernels and results as bias_force, but the workspace of the split
 * and chained launch shapes is a fixed 64 MiB device array of the library
 * (one per GPU, held from the first abp_create on that GPU until the process
 * ends) instead of the context's grow-on-demand buffer, so the call never
 * allocates. ABP_E_NOMEM (nothing enqueued) when the launch needs more
 * workspace than that: it needs about nw * (13 KB + 8 (ncv + 1) B per 64
 * committed hills) for histories longer than 16,384 hills (e.g. 1,024
 * walkers up to about 140,000 hills in 2-D); fused and grid launches need
 * none. Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (other streams, other contexts, other host threads) race. */
abp_status bias_force_noalloc(abp_ctx* ctx, abp_eval_mode mode, abp_prec prec, const abp_cv_desc* cv,
                              const abp_walkers* walkers, const int64_t* n_visible,
                              const int64_t* deposit_slot, const double* deposit_height,
                              double* s, double* V, double* dVds, abp_stream stream);

/* Launch shapes of bias_force's direct sum (see bias_force). */
typedef enum {
  ABP_SHAPE_AUTO = 0,    /* fused up to 16,384 hills; then chained for 1-2 walkers, else split */
  ABP_SHAPE_FUSED = 1,   /* one launch, one block per walker sums every hill */
  ABP_SHAPE_SPLIT = 2,   /* CV, hill-sum and finish launches */
  ABP_SHAPE_CHAIN = 3    /* one launch of several blocks per walker (batches of up to 64 walkers;
                            larger batches take SPLIT) */
} abp_force_shape;

/* Fix the launch shape of later bias_force calls on the context (AUTO by
 * default). Every shape gives bitwise the same results; a fixed shape serves
 * timing and tests that compare the shapes. ABP_E_INVAL for an unknown shape. */
abp_status abp_set_force_shape(abp_ctx* ctx, int32_t shape);

/* Reserve n history slots after every slot reserved so far (host-side
 * bookkeeping, nothing enqueued). *first receives the first slot index.
 * ABP_E_CAPACITY if the history would overflow. */
abp_status abp_reserve(abp_ctx* ctx, int64_t n, int64_t* first);

/* Make reserved slots [committed, upto) visible, in slot order, and add them
 * to the grid if there is one. The writes into those slots (bias_force with
 * deposit_slot) must be ordered before this call on `stream`. */
abp_status abp_commit(abp_ctx* ctx, int64_t upto, abp_stream stream);

/* Wait for `stream`, then return and clear the device error word. */
abp_status abp_sync(abp_ctx* ctx, abp_stream stream);

/* Number of committed (visible) hills; -1 for a NULL context. */
int64_t abp_num_hills(const abp_ctx* ctx);

/* Copy the committed history to HOST arrays centers[ndim][*n] and
 * heights[*n] (FP64 master copy). On entry *n is the capacity of the host
 * arrays; on return it is the number of hills copied. Synchronises the device. */
abp_status abp_hills_export(abp_ctx* ctx, double* centers_host, double* heights_host, int64_t* n);

/* Copy the grid to a HOST array H[nodes][2^ndim] (node index with axis 0
 * fastest; entry m holds the derivative along every axis i whose bit is set
 * in m). ABP_E_INVAL if the context has no grid. Synchronises the device. */
abp_status abp_grid_export(abp_ctx* ctx, double* H_host, int64_t n_values);

/* ---- Serving loop -------------------------------------------------------
 * Continuous batching of bias-force requests from many walkers (MD replicas)
 * that share the context's hill history. The paper runs one walker per MD
 * engine; the request is its per-step exchange (section "Minimization of
 * Interprocess Communications"): a walker's engine sends the coordinates of
 * its CV atoms for one MD step and gets back the bias force on exactly those
 * atoms, which it adds to its own forces, together with s, V and dV/ds.
 *
 * Life cycle: abp_server_create, abp_server_add_walker for every walker,
 * abp_server_start (ends registration, starts the scheduler thread), then any
 * number of abp_server_submit / abp_server_poll calls from any host threads,
 * abp_server_stop (finishes every submitted request), abp_server_destroy.
 * Between start and stop the server owns the context: make no other call on
 * it (its history grows by the requests' deposits).
 *
 * A walker's CV atoms are the distinct atoms of its CV lists, in increasing
 * index order (abp_server_walker_atoms); positions are submitted and forces
 * returned in that order. Positions and forces travel zero-copy: the kernels
 * read a request's positions from pinned, mapped host staging and write its
 * forces there. While a walker is resident its device state is its CV-atom
 * masses (ABP_SERVER_BYTES_PER_ATOM bytes per CV atom; its CV lists are copied
 * to the device once, at start); walkers are admitted first come first served
 * against the HBM budget, and the least recently used idle walker is evicted
 * when memory is short (admission sends its masses with its next batch). A
 * walker has at
 * most one request in the device at a time, and its requests run in
 * submission order. A batch is formed from the resident walkers with a
 * request whenever one of `streams` batch slots is free; up to `streams`
 * batches are in flight. Every request of a batch sees the hills committed
 * when the batch was formed (its version). A request whose step is a positive
 * multiple of deposit_every deposits a hill at its CV value (height
 * height0 * exp(-k / height_decay) for history slot k) into a slot reserved
 * in batch-formation order; slots are committed, in order, once every earlier
 * slot is done. Commits (and their grid deposits) run on one stream of their
 * own; with GRID evaluation a request reads a copy of the grid that holds
 * exactly the hills of its version (see eval_mode), and no batch waits for a
 * commit. A request's result is bitwise the same whatever batch it runs in.
 * Forces are FP32; s, V and dV/ds FP64. A batch signals completion through
 * words in mapped host memory that the scheduler polls; batches of up to 16
 * requests carry their per-request fields in the kernel arguments, larger ones
 * in one copied descriptor. */
typedef struct abp_server abp_server;

#define ABP_SERVER_BYTES_PER_ATOM 4   /* resident device state per CV atom: its FP32 mass */

typedef struct {
  int64_t hbm_budget_bytes;  /* device memory for resident walker state (ABP_SERVER_BYTES_PER_ATOM per CV atom)
                                beyond the registered CV lists */
  int32_t max_batch;         /* requests per batch, 1..65536 (1 = one launch per request) */
  int32_t streams;           /* batches in flight, 1..8 */
  int32_t deposit_every;     /* deposit period in steps; 0: never */
  int32_t prec;              /* abp_prec of the hill sum (DIRECT evaluation) */
  double height0;            /* deposit height height0 * exp(-k / height_decay) for slot k */
  double height_decay;       /* 0: constant height0 */
  int32_t cv_kind[3];        /* abp_cv_kind of CV a (a < ndim), same rules as abp_cv_desc.kind */
  int32_t max_pending;       /* requests submitted and not yet polled, >= 1 (bounds host staging) */
  int32_t eval_mode;         /* abp_eval_mode: DIRECT sums the hills; GRID interpolates the context's
                                grid (or looks it up in the quantised mode). GRID keeps a second
                                copy of the node arrays (device memory of the grid's size): a
                                request reads the copy that holds every hill up to the version it
                                reports, while the commits of deposits are added to the other copy,
                                so requests never wait for a commit. While the server runs the
                                context's own grid may lag its history; abp_server_stop brings it
                                up to date. Needs a context with a grid. */
} abp_server_desc;

typedef struct {
  int64_t submitted;         /* requests accepted since start */
  int64_t completed;         /* requests done */
  int64_t batches;           /* launches of the bias-force path */
  int64_t max_batch_seen;
  int64_t admissions;        /* walkers brought into device memory */
  int64_t evictions;
  int64_t deposits;          /* hills committed by requests */
  int64_t peak_resident;     /* most walkers resident at once */
  int64_t pool_atoms;        /* CV atoms the budget holds */
  double wall_seconds;       /* from start to stop (or to now while running) */
} abp_server_stats;

/* One completed request (abp_server_poll). Times are seconds on the server's
 * steady clock, counted from abp_server_create. */
typedef struct {
  int64_t request;           /* id returned by abp_server_submit */
  int64_t step;
  int64_t version;           /* hills visible to the request */
  int64_t deposit_slot;      /* history slot it deposited into, or -1 */
  int32_t walker;
  int32_t n_cv_atoms;        /* forces written to the request's force_out */
  double t_submit;           /* when abp_server_submit accepted it */
  double t_done;             /* when the scheduler saw its batch complete */
  double s[3];               /* CVs (entries >= ncv unused) */
  double V;
  double dVds[3];
} abp_server_result;

/* One batch (abp_server_trace), times as in abp_server_result. */
typedef struct {
  double t_formed;           /* the scheduler took its requests */
  double t_launched;         /* all of its work was enqueued */
  double t_done;             /* the scheduler saw it complete */
  int64_t requests;
  int64_t version;
  int32_t slot;              /* batch slot (stream) it ran on */
  int32_t admitted;          /* walkers admitted for it (their masses went with it) */
} abp_server_batch;

/* Create a server on a context (GRID evaluation needs a grid). Allocates the walker pool
 * (the budget), per-slot batch buffers sized for max_batch requests at the
 * history's capacity, and pinned host staging for max_pending requests once
 * the walkers are known (abp_server_start). ABP_E_INVAL for a bad descriptor,
 * ABP_E_NOMEM if memory cannot be allocated. */
abp_status abp_server_create(abp_ctx* ctx, const abp_server_desc* desc, abp_server** out);

/* Stop the scheduler if it runs (as abp_server_stop) and free the server (not
 * the context). Results not polled are dropped. */
abp_status abp_server_destroy(abp_server* srv);

/* Register a walker (HOST arrays, copied): n_atoms atoms with masses
 * mass[n_atoms] (of which the server keeps those of the CV atoms);
 * list_len[2*ncv] lengths of the CV lists (CV a, slot t at 2a+t, rules as in
 * abp_cv_desc) and list_idx their concatenation in that order, walker-local
 * indices; ref_x/y/z aligned with list_idx (NULL when no CV is RMSD_OFF).
 * Lists and masses are checked here (ABP_E_INVAL); a walker whose CV atoms
 * exceed the whole budget is refused with ABP_E_NOMEM. Only before
 * abp_server_start. *walker_id receives its id (0, 1, ... in call order) and
 * *n_cv_atoms (may be NULL) the number of its CV atoms. */
abp_status abp_server_add_walker(abp_server* srv, int32_t n_atoms, const float* mass, const int32_t* list_len,
                                 const int32_t* list_idx, const float* ref_x, const float* ref_y,
                                 const float* ref_z, int32_t* walker_id, int32_t* n_cv_atoms);

/* The CV atoms of a walker (walker-local indices, increasing) into the HOST
 * array idx (may be NULL); *n receives their number. */
abp_status abp_server_walker_atoms(abp_server* srv, int32_t walker, int32_t* idx, int32_t* n);

/* End registration, copy the CV lists to the device, warm up every kernel a
 * batch can launch (one batch of each launch shape, no deposit, results
 * discarded) and start the scheduler thread. Statistics and the batch trace
 * restart, and results of an earlier run not yet polled are dropped. The
 * context must have no reserved, uncommitted slots. */
abp_status abp_server_start(abp_server* srv);

/* Submit one request: walker's positions at MD step `step`, HOST array
 * xyz[3][n_cv] (x of every CV atom, then y, then z, in abp_server_walker_atoms
 * order), copied before the call returns. force_out (HOST, [3][n_cv] in the
 * same layout, or NULL) receives the bias force on those atoms when the
 * request is polled; it must stay valid until then. Non-finite coordinates
 * are refused (ABP_E_NONFINITE). ABP_E_BUSY when max_pending requests are
 * submitted and not yet polled (poll, then submit again). *request_id (may be
 * NULL) receives the request's id (0, 1, ... in acceptance order). Thread-safe. */
abp_status abp_server_submit(abp_server* srv, int32_t walker, int64_t step, const float* xyz, float* force_out,
                             int64_t* request_id);

/* Take up to max completed requests (in completion order) into out[] and
 * write their forces to their force_out arrays; *n receives the number taken.
 * Waits up to wait_us microseconds for a first result when none is ready
 * (0: do not wait). Thread-safe. */
abp_status abp_server_poll(abp_server* srv, abp_server_result* out, int64_t max, int64_t* n, int64_t wait_us);

/* Wait until every submitted request is done, then stop the scheduler thread.
 * Completed requests stay available to abp_server_poll. Device-detected
 * errors of the run are returned here (as abp_sync). */
abp_status abp_server_stop(abp_server* srv);

/* Counters since the last start. */
abp_status abp_server_get_stats(abp_server* srv, abp_server_stats* out);

/* Copy up to max batch records (the most recent ones, oldest first) of the
 * run since the last start into out; *n receives the number copied. The
 * server keeps the last 2^18 batches (262,144). */
abp_status abp_server_trace(abp_server* srv, abp_server_batch* out, int64_t max, int64_t* n);

/* Static message for a status code. */
const char* abp_status_str(abp_status status);

/* Message describing the last error on the calling thread ("" if none). */
const char* abp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

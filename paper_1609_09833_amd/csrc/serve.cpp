// Serving loop of libabp (abp_server_*): continuous batching of bias-force
// requests from many walkers sharing one hill history.
//
// A request is the per-step exchange of section "Minimization of
// Interprocess Communications": a walker's engine submits the positions of
// its CV atoms for one MD step and polls back the bias force on exactly those
// atoms (and s, V, dV/ds).
//
// Threads. Callers submit and poll from any host threads. A scheduler thread,
// started by abp_server_start, owns every device call. Each turn it
//   1. takes newly submitted requests into per-walker FIFOs,
//   2. retires finished batches (their completion words in mapped host
//      memory polled, plus the event of a batch with deposits): records
//      results, hands them to the poll queue, frees the walkers for their
//      next request, and commits history slots, in order, once every earlier
//      slot is done,
//   3. (GRID) finishes a completed update of the non-current grid copy and
//      starts the next, on the commit stream (so grid deposits never overlap),
//   4. admits waiting walkers first come first served into the device pool,
//      evicting least recently used idle walkers when the budget is short,
//   5. if a batch slot is free, forms a batch from the walkers that are
//      resident, idle and have a request, and enqueues on the slot's stream
//      the bias-force launches (preceded by a descriptor upload for batches
//      above kInlineWalkers requests; smaller ones carry their per-request
//      fields in the kernel arguments).
// Positions and forces never pass through device copies: the bias-force
// kernels read each request's CV-atom positions from its pinned, mapped
// host staging and write the forces there (posted writes, no read-back), and
// write s, V and dV/ds straight into mapped host memory. A walker's resident
// device state is its CV-atom masses (the pool the budget bounds); a walker
// admitted for a batch gets its masses staged in the slot's mapped
// descriptor buffer, and the CV stage stores them into its pool range for
// later batches.
// Requests in one batch see the same history version (DIRECT: the hills
// committed when the batch was formed; GRID: the hills of the grid copy it
// reads); deposits go to slots reserved in formation order.
// Every buffer is sized at create or start: the loop itself allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "abp_serve_internal.h"
#include "range_pool.h"

namespace {

abp_status sfail(abp_status st, const std::string& msg) { return abp::set_error(st, msg.c_str()); }

#define SRV_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return sfail(ABP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kMaxLists = 6;
constexpr int64_t kBytesPerAtom = ABP_SERVER_BYTES_PER_ATOM;
constexpr size_t kTraceMax = (size_t)1 << 18;  // batch records kept (a ring, reserved at create)
constexpr double kSpinSeconds = 2e-3;          // idle time the scheduler spins before it sleeps
constexpr double kStallCheckSeconds = 2e-3;    // a batch this old also has its stream's state checked

struct Walker {
  int32_t n_atoms = 0;
  int32_t n_cv = 0;          // distinct CV atoms
  int64_t cv_base = 0;       // first entry in cv_atom / cv_mass
  int64_t list_base = 0;     // first entry of its lists in the list pool (indices into its CV atoms)
  int32_t len[kMaxLists] = {0, 0, 0, 0, 0, 0};
  int64_t pool_off = -1;     // device pool offset while resident
  bool inflight = false;
  bool waiting = false;
  bool in_ready = false;
  bool fresh = false;        // admitted since its last batch: masses go with the next one
  bool in_lru = false;
  std::list<int32_t>::iterator lru_it;
  std::deque<int32_t> queue; // request records, submission order
};

struct Record {              // one request from submit to poll
  int64_t id = -1;
  int32_t walker = -1;
  int32_t n_cv = 0;
  int64_t step = 0;
  int64_t arena_off = 0;     // first float of its strip: x, y, z, fx, fy, fz blocks of max_cv each
  float* force_out = nullptr;
  double t_submit = 0.0, t_done = 0.0;
  int64_t version = 0, dep_slot = -1;
  double s[3] = {0, 0, 0}, V = 0.0, dV[3] = {0, 0, 0};
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  int64_t nb = 0;
  int64_t version = 0;
  double t_formed = 0.0, t_launched = 0.0;
  int32_t admitted = 0;
  int grid_copy = 0;                 // GRID: the copy of the node arrays the batch reads
  std::vector<int32_t> reqs;         // records
  std::vector<int64_t> dep_slots;    // history slot per request or -1
  char* h_desc = nullptr;            // mapped pinned descriptor, then the staged masses
  char* m_desc = nullptr;            // its device view (read in place by inline batches)
  char* d_desc = nullptr;            // device copy (larger batches)
  size_t desc_cap = 0;
  double* h_out = nullptr;           // mapped pinned outputs: s[ncv][nb], V[nb], dV[ncv][nb]
  double* m_out = nullptr;           // its device view
  uint32_t* h_done = nullptr;        // mapped completion words [max_batch]: batch seq when request j is done
  uint32_t* m_done = nullptr;        // their device view
  uint32_t seq = 0;                  // this slot's batch counter (0: none launched)
  bool evented = false;              // `done` recorded after the current batch
  void* d_ws = nullptr;              // bias_force workspace, sized for max_batch at the capacity
};

// Byte layout of a batch descriptor with nb requests (arrays packed at stride
// nb). The staged masses follow at `total`.
struct DescLayout {
  size_t pool_off, arena_off, stage_off, dep_slot, dep_height, n_cv, list_beg, list_len, total;
  static size_t up(size_t x) { return (x + 15) / 16 * 16; }
  DescLayout(int64_t nb, int nlists) {
    size_t o = 0;
    pool_off = o; o = up(o + 8 * nb);
    arena_off = o; o = up(o + 8 * nb);
    stage_off = o; o = up(o + 8 * nb);
    dep_slot = o; o = up(o + 8 * nb);
    dep_height = o; o = up(o + 8 * nb);
    n_cv = o; o = up(o + 4 * nb);
    list_beg = o; o = up(o + 4 * nb * nlists);
    list_len = o; o = up(o + 4 * nb * nlists);
    total = o;
  }
};

}  // namespace

struct abp_server {
  abp_ctx* ctx = nullptr;
  abp::CtxView cv;
  abp_server_desc desc{};
  int ncv = 0;
  int nlists = 0;
  int kind[3] = {0, 0, 0};
  std::chrono::steady_clock::time_point t0;
  // registration (host)
  std::vector<Walker> walkers;
  std::vector<int32_t> cv_atom;      // every walker's CV atoms (walker-local indices, increasing)
  std::vector<float> cv_mass;        // and their masses
  std::vector<int32_t> lidx;         // every walker's lists, as positions among its CV atoms
  std::vector<float> lrx, lry, lrz;  // RMSD references aligned with lidx
  int32_t max_cv = 0;
  bool registered = false;           // start has run once: the lists are on the device
  // device state
  int32_t* d_lidx = nullptr;
  float* d_rx = nullptr;
  float* d_ry = nullptr;
  float* d_rz = nullptr;
  int64_t pool_atoms = 0;
  float* d_pool = nullptr;           // CV-atom masses of resident walkers, pool_atoms floats
  abp::RangePool free_atoms;         // free pool ranges, best fit
  std::list<int32_t> lru;            // idle resident walkers, least recent first
  std::deque<int32_t> admission;     // walkers waiting for memory
  std::deque<int32_t> ready;         // resident, idle, with a request
  std::vector<Slot> slots;
  std::deque<int> launch_order;      // busy slots in launch order
  hipStream_t commit_stream = nullptr;
  // GRID evaluation reads one of two copies of the node arrays: [0] is the
  // context's own (with its FP32 mirror), [1] the server's. A batch reads the
  // current copy. Committed hills are added to the other copy once no batch
  // in flight reads it, on the commit stream, and that copy becomes current
  // when the update has completed (if it is then the newer one): batches never
  // wait for a commit. Both copies receive the same groups of hills in the
  // same order, so they are bitwise equal at equal versions.
  struct GridCopy {
    double* grid = nullptr;
    float* grid32 = nullptr;
    int64_t version = 0;             // hills it holds
    size_t next = 0;                 // first group (absolute index) not yet added
  };
  bool grid_mode = false;
  GridCopy gcopy[2];
  int gcur = 0;
  int gupd = -1;                     // copy being updated, or -1
  int64_t gupd_version = 0;
  size_t gupd_next = 0;
  std::deque<std::pair<int64_t, int64_t>> groups;   // committed hill ranges in commit order
  size_t gbase = 0;                  // absolute index of groups.front()
  hipEvent_t grid_evt = nullptr;     // recorded after an update
  double* own_grid = nullptr;
  std::map<int64_t, bool> dep_done;  // reserved slot -> done
  int64_t resident = 0;
  // request staging: max_pending records, each with a fixed strip of the
  // pinned, mapped arena: x, y, z, fx, fy, fz blocks of `block` floats
  // (block = the largest walker's CV atoms), so that block offsets are the
  // same for every request and one base per request addresses all six
  float* arena = nullptr;
  float* d_arena = nullptr;
  int64_t block = 0;
  std::vector<Record> records;
  // shared between the callers and the scheduler
  std::mutex mu_in;                  // incoming, free_records, next_id
  std::condition_variable cv_in;
  std::vector<int32_t> incoming;
  std::vector<int32_t> free_records;
  int64_t next_id = 0;
  std::mutex mu_out;                 // completed
  std::condition_variable cv_out;
  std::deque<int32_t> completed;
  std::atomic<int64_t> outstanding{0};   // submitted and not yet completed
  std::atomic<bool> running{false};
  std::atomic<bool> stopping{false};
  std::thread thread;
  std::string thread_error;          // set by the scheduler when it fails (read after join)
  abp_status thread_status = ABP_OK;
  // statistics (written by the scheduler under mu_stats)
  std::mutex mu_stats;
  abp_server_stats stats{};
  double t_start = 0.0, t_stop = -1.0;
  std::vector<abp_server_batch> trace;
  size_t trace_next = 0;
};

namespace {

double now_s(const abp_server* S) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - S->t0).count();
}

// Returns every resident walker to the pool and clears all queues.
void reset_residency(abp_server* S) {
  for (auto& w : S->walkers) {
    w.pool_off = -1;
    w.inflight = w.waiting = w.in_ready = w.fresh = w.in_lru = false;
    w.queue.clear();
  }
  S->free_atoms.reset(S->pool_atoms);
  S->lru.clear();
  S->admission.clear();
  S->ready.clear();
  S->resident = 0;
}

void make_ready(abp_server* S, int32_t wid) {
  Walker& w = S->walkers[wid];
  if (w.in_ready || w.inflight || w.pool_off < 0 || w.queue.empty()) return;
  if (w.in_lru) {
    S->lru.erase(w.lru_it);
    w.in_lru = false;
  }
  w.in_ready = true;
  S->ready.push_back(wid);
}

void make_idle(abp_server* S, int32_t wid) {
  Walker& w = S->walkers[wid];
  if (w.in_lru || w.pool_off < 0) return;
  S->lru.push_back(wid);
  w.lru_it = std::prev(S->lru.end());
  w.in_lru = true;
}

// Admit waiting walkers in arrival order while memory allows.
void admit(abp_server* S) {
  while (!S->admission.empty()) {
    const int32_t wid = S->admission.front();
    Walker& w = S->walkers[wid];
    int64_t off;
    bool ok = S->free_atoms.alloc(w.n_cv, &off);
    while (!ok && !S->lru.empty()) {
      const int32_t victim = S->lru.front();
      S->lru.pop_front();
      Walker& v = S->walkers[victim];
      v.in_lru = false;
      S->free_atoms.free(v.pool_off, v.n_cv);
      v.pool_off = -1;
      v.fresh = false;
      S->resident--;
      {
        std::lock_guard<std::mutex> lk(S->mu_stats);
        S->stats.evictions++;
      }
      ok = S->free_atoms.alloc(w.n_cv, &off);
    }
    if (!ok) return;                       // wait for a walker to go idle
    S->admission.pop_front();
    w.waiting = false;
    w.pool_off = off;
    w.fresh = true;
    S->resident++;
    std::lock_guard<std::mutex> lk(S->mu_stats);
    S->stats.admissions++;
    if (S->resident > S->stats.peak_resident) S->stats.peak_resident = S->resident;
    make_ready(S, wid);
  }
}

// Commits the longest done prefix of reserved slots, on the commit stream
// (one stream, so the grid deposits of successive commits never overlap).
abp_status commit_prefix(abp_server* S) {
  int64_t upto = abp_num_hills(S->ctx);
  auto it = S->dep_done.begin();
  while (it != S->dep_done.end() && it->first == upto && it->second) {
    ++upto;
    it = S->dep_done.erase(it);
  }
  const int64_t before = abp_num_hills(S->ctx);
  if (upto > before) {
    if (S->grid_mode) {        // the grid copies take the hills in grid_step
      const abp_status st = abp::ctx_commit_hills(S->ctx, upto);
      if (st != ABP_OK) return st;
      S->groups.emplace_back(before, upto);
    } else {
      const abp_status st = abp_commit(S->ctx, upto, S->commit_stream);
      if (st != ABP_OK) return st;
    }
    std::lock_guard<std::mutex> lk(S->mu_stats);
    S->stats.deposits += upto - before;
  }
  return ABP_OK;
}

// Enqueues one batch on slot `sl`: requests recs[j] of walkers wids[j] (all
// resident and marked in flight by the caller). shape: abp_force_shape of the
// bias-force launches; deposits: whether deposit steps reserve slots.
abp_status enqueue_batch(abp_server* S, Slot& sl, const int32_t* wids, const int32_t* recs, int64_t nb,
                         int32_t shape, bool deposits) {
  // Up to kInlineWalkers requests: the per-walker fields travel in the kernel
  // arguments and the staged masses are read from the mapped descriptor
  // buffer, so nothing is copied before the launch. Larger batches: the
  // descriptor (fields, then staged masses) is copied to the device first.
  const bool inl = nb <= abp::kInlineWalkers;
  abp::ForceArgs A;
  std::memset(&A, 0, sizeof(A));
  DescLayout L(inl ? 0 : nb, S->nlists);
  const int64_t ls = inl ? abp::kInlineWalkers : nb;        // stride of the list arrays
  int64_t* d_poolo = inl ? A.inl.mass_base : reinterpret_cast<int64_t*>(sl.h_desc + L.pool_off);
  int64_t* d_arena = inl ? A.inl.atom_base : reinterpret_cast<int64_t*>(sl.h_desc + L.arena_off);
  int64_t* d_stage = inl ? A.inl.stage_off : reinterpret_cast<int64_t*>(sl.h_desc + L.stage_off);
  int64_t* d_dep = inl ? A.inl.deposit_slot : reinterpret_cast<int64_t*>(sl.h_desc + L.dep_slot);
  double* d_hgt = inl ? A.inl.deposit_height : reinterpret_cast<double*>(sl.h_desc + L.dep_height);
  int32_t* d_ncv = inl ? A.inl.n_atoms : reinterpret_cast<int32_t*>(sl.h_desc + L.n_cv);
  int32_t* d_lbeg = inl ? &A.inl.list_beg[0][0] : reinterpret_cast<int32_t*>(sl.h_desc + L.list_beg);
  int32_t* d_llen = inl ? &A.inl.list_len[0][0] : reinterpret_cast<int32_t*>(sl.h_desc + L.list_len);
  float* h_stage = reinterpret_cast<float*>(sl.h_desc + L.total);
  int64_t spos = 0;
  bool any_deposit = false;
  sl.reqs.clear();
  sl.dep_slots.clear();
  sl.admitted = 0;
  const bool grid = S->grid_mode;
  sl.grid_copy = S->gcur;
  sl.version = grid ? S->gcopy[S->gcur].version : abp_num_hills(S->ctx);
  for (int64_t j = 0; j < nb; ++j) {
    Walker& w = S->walkers[wids[j]];
    const Record& R = S->records[recs[j]];
    sl.reqs.push_back(recs[j]);
    d_poolo[j] = w.pool_off;
    d_arena[j] = R.arena_off;
    d_ncv[j] = w.n_cv;
    d_stage[j] = -1;
    if (w.fresh) {
      if (L.total + (size_t)(spos + w.n_cv) * sizeof(float) > sl.desc_cap)
        return sfail(ABP_E_DEVICE, "batch descriptor larger than sized (internal error)");
      d_stage[j] = spos;
      std::memcpy(h_stage + spos, S->cv_mass.data() + w.cv_base, sizeof(float) * (size_t)w.n_cv);
      spos += w.n_cv;
      w.fresh = false;
      sl.admitted++;
    }
    int64_t lpos = w.list_base;
    for (int q = 0; q < S->nlists; ++q) {
      d_lbeg[q * ls + j] = (int32_t)lpos;
      d_llen[q * ls + j] = w.len[q];
      lpos += w.len[q];
    }
    int64_t slot = -1;
    const int64_t step = R.step;
    if (deposits && S->desc.deposit_every > 0 && step > 0 && step % S->desc.deposit_every == 0) {
      if (abp_reserve(S->ctx, 1, &slot) != ABP_OK) slot = -1;     // history full: no deposit
      if (slot >= 0) {
        S->dep_done[slot] = false;
        any_deposit = true;
      }
    }
    d_dep[j] = slot;
    d_hgt[j] = S->desc.height_decay > 0
                   ? S->desc.height0 * std::exp(-(double)std::max<int64_t>(slot, 0) / S->desc.height_decay)
                   : S->desc.height0;
    sl.dep_slots.push_back(slot);
  }
  sl.nb = nb;
  const char* desc = inl ? sl.m_desc : sl.d_desc;        // device view of the fields and staged masses
  if (!inl)
    SRV_TRY(hipMemcpyAsync(sl.d_desc, sl.h_desc, L.total + (size_t)spos * sizeof(float), hipMemcpyHostToDevice,
                           sl.stream));
  else
    A.inl_n = (int32_t)nb;
  const int64_t M = S->block;
  A.ncv = S->ncv;
  for (int a = 0; a < 3; ++a) A.kind[a] = S->kind[a];
  if (!inl) {
    A.list_beg = reinterpret_cast<const int32_t*>(desc + L.list_beg);
    A.list_len = reinterpret_cast<const int32_t*>(desc + L.list_len);
    A.atom_base = reinterpret_cast<const int64_t*>(desc + L.arena_off);   // each request's strip
    A.n_atoms = reinterpret_cast<const int32_t*>(desc + L.n_cv);
    A.mass_base = reinterpret_cast<const int64_t*>(desc + L.pool_off);
    A.stage_off = reinterpret_cast<const int64_t*>(desc + L.stage_off);
    A.deposit_slot = any_deposit ? reinterpret_cast<const int64_t*>(desc + L.dep_slot) : nullptr;
    A.deposit_height = reinterpret_cast<const double*>(desc + L.dep_height);
  }
  A.list_idx = S->d_lidx;
  A.ref_x = S->d_rx;
  A.ref_y = S->d_ry;
  A.ref_z = S->d_rz;
  A.nw = nb;
  A.x = S->d_arena;
  A.y = S->d_arena + M;
  A.z = S->d_arena + 2 * M;
  A.fx = S->d_arena + 3 * M;
  A.fy = S->d_arena + 4 * M;
  A.fz = S->d_arena + 5 * M;
  A.mass = S->d_pool;
  A.stage_mass = reinterpret_cast<const float*>(desc + L.total);
  A.mass_store = S->d_pool;
  A.force_store = 1;                      // the strips' forces were zeroed at submit
  A.n_visible = nullptr;
  A.n_visible_default = sl.version;
  A.s = sl.m_out;
  A.V = sl.m_out + S->ncv * nb;
  A.dVds = sl.m_out + (S->ncv + 1) * nb;
  A.prec = S->desc.prec;
  A.shape = shape;
  A.use_grid = grid ? 1 : 0;
  A.grid = grid ? S->gcopy[S->gcur].grid : nullptr;
  A.err = S->cv.err;
  if (++sl.seq == 0) sl.seq = 1;          // 0 is the words' initial value
  A.done_flag = sl.m_done;
  A.done_seq = sl.seq;
  SRV_TRY(abp::launch_bias_force(S->cv.K, S->cv.H, A, sl.d_ws, sl.stream));
  // A batch with deposits is retired (and its hills committed) only once its
  // launch has completed on the stream.
  sl.evented = any_deposit;
  if (sl.evented) SRV_TRY(hipEventRecord(sl.done, sl.stream));
  sl.busy = true;
  return ABP_OK;
}

// Whether slot sl's batch is done: every request's completion word holds the
// batch's seq (and, for a batch with an event, the event has completed, so
// the commit of its deposits follows the whole launch). hipErrorNotReady
// while running. A stream that went idle without the words is reported as an
// error after a grace period (a launch that did not run to its end).
hipError_t batch_state(abp_server* S, Slot& sl) {
  for (int64_t j = 0; j < sl.nb; ++j)
    if (__atomic_load_n(sl.h_done + j, __ATOMIC_ACQUIRE) != sl.seq) {
      if (now_s(S) - sl.t_launched < kStallCheckSeconds) return hipErrorNotReady;
      const hipError_t q = hipStreamQuery(sl.stream);
      if (q == hipErrorNotReady) return hipErrorNotReady;
      if (q != hipSuccess) return q;
      for (int64_t i = 0; i < sl.nb; ++i)        // idle: the words must be there now
        if (__atomic_load_n(sl.h_done + i, __ATOMIC_ACQUIRE) != sl.seq) return hipErrorLaunchFailure;
      break;
    }
  return sl.evented ? hipEventQuery(sl.done) : hipSuccess;
}

void record_batch(abp_server* S, const Slot& sl, int slot_index, double t_done) {
  abp_server_batch b;
  b.t_formed = sl.t_formed;
  b.t_launched = sl.t_launched;
  b.t_done = t_done;
  b.requests = sl.nb;
  b.version = sl.version;
  b.slot = slot_index;
  b.admitted = sl.admitted;
  std::lock_guard<std::mutex> lk(S->mu_stats);
  if (S->trace.size() < kTraceMax) S->trace.push_back(b);
  else S->trace[S->trace_next % kTraceMax] = b;
  S->trace_next++;
}

// GRID: an update in flight, or a copy that lacks committed hills.
bool grid_work(const abp_server* S) {
  if (!S->grid_mode) return false;
  return S->gupd >= 0 || S->gcopy[1 - S->gcur].next < S->gbase + S->groups.size();
}

bool nothing_to_do(const abp_server* S) {
  return S->launch_order.empty() && S->ready.empty() && S->admission.empty() && !grid_work(S);
}

// GRID: finishes a completed update of a grid copy (making it current when it
// is the newer one) and starts the next: the committed groups that the
// non-current copy lacks, once no batch in flight reads it.
abp_status grid_step(abp_server* S) {
  if (!S->grid_mode) return ABP_OK;
  if (S->gupd >= 0) {
    const hipError_t q = hipEventQuery(S->grid_evt);
    if (q == hipErrorNotReady) return ABP_OK;
    if (q != hipSuccess) return sfail(ABP_E_DEVICE, (std::string("grid update failed: ") + hipGetErrorString(q)).c_str());
    abp_server::GridCopy& g = S->gcopy[S->gupd];
    g.version = S->gupd_version;
    g.next = S->gupd_next;
    if (g.version > S->gcopy[S->gcur].version) S->gcur = S->gupd;
    S->gupd = -1;
    const size_t both = std::min(S->gcopy[0].next, S->gcopy[1].next);
    while (S->gbase < both) {
      S->groups.pop_front();
      S->gbase++;
    }
  }
  const int t = 1 - S->gcur;
  abp_server::GridCopy& g = S->gcopy[t];
  const size_t end = S->gbase + S->groups.size();
  if (g.next >= end) return ABP_OK;
  for (const int k : S->launch_order)
    if (S->slots[k].grid_copy == t) return ABP_OK;
  for (size_t i = g.next; i < end; ++i) {
    const auto& gr = S->groups[i - S->gbase];
    const abp_status st = abp::ctx_grid_add(S->ctx, g.grid, g.grid32, gr.first, gr.second, S->commit_stream);
    if (st != ABP_OK) return st;
  }
  SRV_TRY(hipEventRecord(S->grid_evt, S->commit_stream));
  S->gupd = t;
  S->gupd_version = S->groups.back().second;
  S->gupd_next = end;
  return ABP_OK;
}

// One scheduler turn's device work (steps 2-4). Returns false on failure
// (S->thread_status / thread_error set).
bool turn(abp_server* S) {
  const int ncv = S->ncv;
  // 2. retire finished batches, in launch order
  while (!S->launch_order.empty()) {
    const int idx = S->launch_order.front();
    Slot& sl = S->slots[idx];
    const hipError_t q = batch_state(S, sl);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) {
      S->thread_status = ABP_E_DEVICE;
      S->thread_error = std::string("batch failed: ") + hipGetErrorString(q);
      return false;
    }
    const double td = now_s(S);
    const int64_t nb = sl.nb;
    for (int64_t j = 0; j < nb; ++j) {
      Record& R = S->records[sl.reqs[j]];
      R.t_done = td;
      R.version = sl.version;
      R.dep_slot = sl.dep_slots[j];
      for (int a = 0; a < ncv; ++a) {
        R.s[a] = sl.h_out[a * nb + j];
        R.dV[a] = sl.h_out[(ncv + 1 + a) * nb + j];
      }
      R.V = sl.h_out[ncv * nb + j];
      Walker& w = S->walkers[R.walker];
      w.inflight = false;
      if (w.queue.empty()) make_idle(S, R.walker);
      else make_ready(S, R.walker);
      if (sl.dep_slots[j] >= 0) S->dep_done[sl.dep_slots[j]] = true;
    }
    {
      std::lock_guard<std::mutex> lk(S->mu_out);
      for (int64_t j = 0; j < nb; ++j) S->completed.push_back(sl.reqs[j]);
    }
    S->cv_out.notify_all();
    S->outstanding.fetch_sub(nb);
    {
      std::lock_guard<std::mutex> lk(S->mu_stats);
      S->stats.completed += nb;
    }
    record_batch(S, sl, idx, td);
    sl.busy = false;
    S->launch_order.pop_front();
    const abp_status st = commit_prefix(S);
    if (st != ABP_OK) {
      S->thread_status = st;
      S->thread_error = abp_last_error();
      return false;
    }
  }
  {
    const abp_status st = grid_step(S);
    if (st != ABP_OK) {
      S->thread_status = st;
      S->thread_error = abp_last_error();
      return false;
    }
  }
  // 3. admission
  admit(S);
  // 4. form and launch a batch on a free slot
  if (S->ready.empty()) return true;
  int free_slot = -1;
  for (int k = 0; k < (int)S->slots.size(); ++k)
    if (!S->slots[k].busy) { free_slot = k; break; }
  if (free_slot < 0) return true;
  Slot& sl = S->slots[free_slot];
  sl.t_formed = now_s(S);
  const int64_t nb = std::min<int64_t>((int64_t)S->ready.size(), S->desc.max_batch);
  std::vector<int32_t> wids(nb), recs(nb);
  for (int64_t j = 0; j < nb; ++j) {
    const int32_t wid = S->ready.front();
    S->ready.pop_front();
    Walker& w = S->walkers[wid];
    w.in_ready = false;
    w.inflight = true;
    wids[j] = wid;
    recs[j] = w.queue.front();
    w.queue.pop_front();
  }
  const abp_status st = enqueue_batch(S, sl, wids.data(), recs.data(), nb, ABP_SHAPE_AUTO, true);
  if (st != ABP_OK) {
    S->thread_status = st;
    S->thread_error = abp_last_error();
    return false;
  }
  sl.t_launched = now_s(S);
  S->launch_order.push_back(free_slot);
  std::lock_guard<std::mutex> lk(S->mu_stats);
  S->stats.batches++;
  if (nb > S->stats.max_batch_seen) S->stats.max_batch_seen = nb;
  return true;
}

void scheduler(abp_server* S) {
  if (hipSetDevice(S->cv.device) != hipSuccess) {
    S->thread_status = ABP_E_DEVICE;
    S->thread_error = "cannot select the context's device";
    S->running = false;
    return;
  }
  std::vector<int32_t> in;
  double idle_since = -1.0;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu_in);
      if (S->incoming.empty() && nothing_to_do(S)) {
        if (S->stopping.load() && S->outstanding.load() == 0) break;
        const double t = now_s(S);
        if (idle_since < 0.0) idle_since = t;
        if (t - idle_since > kSpinSeconds)
          S->cv_in.wait_for(lk, std::chrono::milliseconds(1),
                            [S] { return !S->incoming.empty() || S->stopping.load(); });
      } else {
        idle_since = -1.0;
      }
      in.swap(S->incoming);
    }
    // 1. intake, in submission order
    for (const int32_t r : in) {
      const int32_t wid = S->records[r].walker;
      Walker& w = S->walkers[wid];
      w.queue.push_back(r);
      if (w.pool_off < 0) {
        if (!w.waiting) {
          w.waiting = true;
          S->admission.push_back(wid);
        }
      } else {
        make_ready(S, wid);
      }
    }
    in.clear();
    if (!turn(S)) break;
  }
  // drain what is in flight (after a failure too), so no kernel outlives the thread
  for (auto& sl : S->slots) (void)hipStreamSynchronize(sl.stream);
  (void)hipStreamSynchronize(S->commit_stream);
  S->running = false;
  S->cv_out.notify_all();
}

// Sizes every buffer of a run: descriptors (max_batch requests, the masses of
// the max_batch walkers with the most CV atoms), the request arena, the
// slots' bias-force workspaces for the history's capacity, the context's
// grid-deposit scratch for the largest commit.
abp_status size_buffers(abp_server* S) {
  std::vector<int64_t> ncv;
  ncv.reserve(S->walkers.size());
  for (const auto& w : S->walkers) ncv.push_back(w.n_cv);
  const size_t b = std::min(ncv.size(), (size_t)S->desc.max_batch);
  std::partial_sort(ncv.begin(), ncv.begin() + b, ncv.end(), std::greater<int64_t>());
  int64_t most = 0;
  for (size_t i = 0; i < b; ++i) most += ncv[i];
  const size_t need = DescLayout(S->desc.max_batch, S->nlists).total + (size_t)most * sizeof(float);
  for (auto& sl : S->slots) {
    if (sl.desc_cap >= need) continue;
    if (sl.h_desc) SRV_TRY(hipHostFree(sl.h_desc));
    if (sl.d_desc) SRV_TRY(hipFree(sl.d_desc));
    sl.h_desc = nullptr;
    sl.d_desc = nullptr;
    sl.desc_cap = 0;
    sl.m_desc = nullptr;
    if (hipHostMalloc((void**)&sl.h_desc, need, hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void**)&sl.m_desc, sl.h_desc, 0) != hipSuccess ||
        hipMalloc((void**)&sl.d_desc, need) != hipSuccess)
      return sfail(ABP_E_NOMEM, "cannot allocate batch descriptors");
    sl.desc_cap = need;
  }
  const int64_t block = std::max(S->max_cv, 1);
  if (block != S->block || !S->arena) {
    if (S->arena) SRV_TRY(hipHostFree(S->arena));
    S->arena = nullptr;
    S->d_arena = nullptr;
    const size_t bytes = sizeof(float) * 6 * (size_t)block * (size_t)S->desc.max_pending;
    if (hipHostMalloc((void**)&S->arena, bytes, hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void**)&S->d_arena, S->arena, 0) != hipSuccess)
      return sfail(ABP_E_NOMEM, "cannot allocate the request staging");
    S->block = block;
  }
  S->records.assign(S->desc.max_pending, Record());
  S->free_records.clear();
  for (int32_t r = S->desc.max_pending - 1; r >= 0; --r) {
    S->records[r].arena_off = (int64_t)r * 6 * block;
    S->free_records.push_back(r);
  }
  const abp_status st = abp::ctx_reserve_commit(S->ctx, (int64_t)S->desc.max_batch * S->desc.streams);
  if (st != ABP_OK) return st;
  return ABP_OK;
}

// One batch of each launch shape for walker 0 at zero positions (a COM
// distance and a torsion at coincident atoms have zero gradient by the
// singular-point rule), so every kernel the loop can launch is loaded before
// the first request (with no hills yet only the fused shape sums anything).
// No deposit; results are discarded.
abp_status warm_up(abp_server* S) {
  if (S->walkers.empty()) return ABP_OK;
  reset_residency(S);
  Walker& w = S->walkers[0];
  int64_t off;
  if (!S->free_atoms.alloc(w.n_cv, &off)) return ABP_OK;
  w.pool_off = off;
  const int32_t rec = S->free_records.back();
  Record& R = S->records[rec];
  R.walker = 0;
  R.n_cv = w.n_cv;
  R.step = 0;
  std::memset(S->arena + R.arena_off, 0, sizeof(float) * 6 * (size_t)S->block);
  const int32_t wid = 0;
  Slot& sl = S->slots[0];
  const int nshapes = (abp_num_hills(S->ctx) > 0 && S->desc.eval_mode != ABP_EVAL_GRID) ? 3 : 1;
  const int32_t shapes[3] = {ABP_SHAPE_FUSED, ABP_SHAPE_SPLIT, ABP_SHAPE_CHAIN};
  for (int k = 0; k < nshapes; ++k) {
    const int32_t shape = shapes[k];
    w.fresh = true;
    const abp_status st = enqueue_batch(S, sl, &wid, &rec, 1, shape, false);
    if (st != ABP_OK) return st;
    SRV_TRY(hipStreamSynchronize(sl.stream));
    sl.busy = false;
  }
  reset_residency(S);
  return ABP_OK;
}

}  // namespace

namespace abp {
hipError_t launch_bias_force(const Consts& K, const HistView& H, const ForceArgs& A, void* workspace,
                             hipStream_t stream);
}

extern "C" {

abp_status abp_server_create(abp_ctx* ctx, const abp_server_desc* desc, abp_server** out) {
  if (!ctx || !desc || !out) return sfail(ABP_E_INVAL, "NULL argument");
  *out = nullptr;
  if (desc->max_batch < 1 || desc->max_batch > (1 << 16)) return sfail(ABP_E_INVAL, "max_batch must be 1..65536");
  if (desc->streams < 1 || desc->streams > 8) return sfail(ABP_E_INVAL, "streams must be 1..8");
  if (desc->deposit_every < 0) return sfail(ABP_E_INVAL, "deposit_every must be >= 0");
  if (desc->prec != ABP_PREC_FP32_KAHAN && desc->prec != ABP_PREC_FP32_NAIVE && desc->prec != ABP_PREC_FP64)
    return sfail(ABP_E_INVAL, "unknown precision");
  if (!(desc->hbm_budget_bytes >= kBytesPerAtom)) return sfail(ABP_E_INVAL, "budget too small");
  if (!std::isfinite(desc->height0) || desc->height0 < 0 || !(desc->height_decay >= 0) ||
      !std::isfinite(desc->height_decay))
    return sfail(ABP_E_INVAL, "bad deposit height law");
  if (desc->max_pending < 1 || desc->max_pending > (1 << 24)) return sfail(ABP_E_INVAL, "max_pending must be 1..2^24");
  if (desc->eval_mode != ABP_EVAL_DIRECT && desc->eval_mode != ABP_EVAL_GRID)
    return sfail(ABP_E_INVAL, "unknown eval mode");
  abp_server* S = new (std::nothrow) abp_server();
  if (!S) return sfail(ABP_E_NOMEM, "host allocation failed");
  S->t0 = std::chrono::steady_clock::now();
  S->ctx = ctx;
  S->cv = abp::ctx_view(ctx);
  S->desc = *desc;
  S->ncv = S->cv.K.ndim;
  S->nlists = 2 * S->ncv;
  for (int a = 0; a < S->ncv; ++a) {
    const int k = desc->cv_kind[a];
    if (k != ABP_CV_COM_DIST && k != ABP_CV_TORSION && k != ABP_CV_RMSD_OFF) {
      delete S;
      return sfail(ABP_E_INVAL, "unknown CV kind");
    }
    if ((k == ABP_CV_TORSION) != (S->cv.K.periodic[a] != 0)) {
      delete S;
      return sfail(ABP_E_INVAL, "TORSION needs a periodic axis, COM_DIST/RMSD_OFF a non-periodic one");
    }
    S->kind[a] = k;
  }
  if (desc->eval_mode == ABP_EVAL_GRID && !S->cv.grid) {
    delete S;
    return sfail(ABP_E_INVAL, "GRID evaluation needs a context with a grid");
  }
  if (hipSetDevice(S->cv.device) != hipSuccess) {
    delete S;
    return sfail(ABP_E_DEVICE, "cannot select the context's device");
  }
  S->pool_atoms = desc->hbm_budget_bytes / kBytesPerAtom;
  if (hipMalloc(&S->d_pool, sizeof(float) * S->pool_atoms) != hipSuccess) {
    delete S;
    return sfail(ABP_E_NOMEM, "cannot allocate the walker pool");
  }
  S->stats.pool_atoms = S->pool_atoms;
  reset_residency(S);
  const int64_t B = desc->max_batch;
  const size_t ws = abp::force_workspace_bytes(B, abp::force_blocks_per_walker(S->cv.H.capacity, 0, 0), S->ncv);
  S->slots.resize(desc->streams);
  S->trace.reserve(kTraceMax);            // the loop never grows it
  S->grid_mode = desc->eval_mode == ABP_EVAL_GRID;
  bool good = hipStreamCreateWithFlags(&S->commit_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&S->grid_evt, hipEventDisableTiming) == hipSuccess;
  if (good && S->grid_mode)
    good = hipMalloc(&S->own_grid, sizeof(double) * S->cv.grid_doubles) == hipSuccess;
  for (auto& sl : S->slots) {
    good = good && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
           hipHostMalloc((void**)&sl.h_out, sizeof(double) * B * (2 * S->ncv + 1), hipHostMallocMapped) == hipSuccess &&
           hipHostGetDevicePointer((void**)&sl.m_out, sl.h_out, 0) == hipSuccess &&
           hipHostMalloc((void**)&sl.h_done, sizeof(uint32_t) * B, hipHostMallocMapped) == hipSuccess &&
           hipHostGetDevicePointer((void**)&sl.m_done, sl.h_done, 0) == hipSuccess &&
           std::memset(sl.h_done, 0, sizeof(uint32_t) * B) != nullptr &&
           hipMalloc(&sl.d_ws, ws) == hipSuccess && hipMemset(sl.d_ws, 0, ws) == hipSuccess;
    sl.reqs.reserve(B);
    sl.dep_slots.reserve(B);
  }
  if (!good) {
    abp_server_destroy(S);
    return sfail(ABP_E_NOMEM, "cannot allocate per-slot batch buffers and workspaces");
  }
  *out = S;
  return ABP_OK;
}

abp_status abp_server_stop(abp_server* S) {
  if (!S) return sfail(ABP_E_INVAL, "NULL argument");
  if (S->thread.joinable()) {
    S->stopping = true;
    S->cv_in.notify_all();
    S->thread.join();
    std::lock_guard<std::mutex> lk(S->mu_stats);
    S->t_stop = now_s(S);
    S->stats.wall_seconds = S->t_stop - S->t_start;
  }
  S->running = false;
  if (S->thread_status == ABP_OK && S->grid_mode) {
    // the context's own arrays take every group they lack
    (void)hipSetDevice(S->cv.device);
    abp_server::GridCopy& g = S->gcopy[0];
    if (S->gupd >= 0) {
      if (hipStreamSynchronize(S->commit_stream) != hipSuccess)
        return sfail(ABP_E_DEVICE, "grid update failed");
      if (S->gupd == 0) g.next = S->gupd_next;
      S->gupd = -1;
    }
    for (size_t i = g.next; i < S->gbase + S->groups.size(); ++i) {
      const auto& gr = S->groups[i - S->gbase];
      const abp_status st = abp::ctx_grid_add(S->ctx, g.grid, g.grid32, gr.first, gr.second, S->commit_stream);
      if (st != ABP_OK) return st;
    }
    g.next = S->gbase + S->groups.size();
    if (hipStreamSynchronize(S->commit_stream) != hipSuccess) return sfail(ABP_E_DEVICE, "grid update failed");
  }
  if (S->thread_status != ABP_OK) {
    const abp_status st = S->thread_status;
    S->thread_status = ABP_OK;
    return sfail(st, S->thread_error);
  }
  // Device-side flags of the run (invalid walker, non-finite input) surface here.
  return abp_sync(S->ctx, nullptr);
}

abp_status abp_server_destroy(abp_server* S) {
  if (!S) return ABP_OK;
  if (S->thread.joinable()) (void)abp_server_stop(S);
  (void)hipSetDevice(S->cv.device);
  for (auto& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_desc) (void)hipHostFree(sl.h_desc);
    if (sl.d_desc) (void)hipFree(sl.d_desc);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.h_done) (void)hipHostFree(sl.h_done);
    if (sl.d_ws) (void)hipFree(sl.d_ws);
  }
  if (S->commit_stream) {
    (void)hipStreamSynchronize(S->commit_stream);
    (void)hipStreamDestroy(S->commit_stream);
  }
  if (S->grid_evt) (void)hipEventDestroy(S->grid_evt);
  if (S->own_grid) (void)hipFree(S->own_grid);
  if (S->arena) (void)hipHostFree(S->arena);
  if (S->d_lidx) (void)hipFree(S->d_lidx);
  if (S->d_rx) (void)hipFree(S->d_rx);
  if (S->d_ry) (void)hipFree(S->d_ry);
  if (S->d_rz) (void)hipFree(S->d_rz);
  if (S->d_pool) (void)hipFree(S->d_pool);
  delete S;
  return ABP_OK;
}

abp_status abp_server_add_walker(abp_server* S, int32_t n_atoms, const float* mass, const int32_t* list_len,
                                 const int32_t* list_idx, const float* ref_x, const float* ref_y,
                                 const float* ref_z, int32_t* walker_id, int32_t* n_cv_atoms) {
  if (!S || !mass || !list_len || !walker_id) return sfail(ABP_E_INVAL, "NULL argument");
  if (S->registered) return sfail(ABP_E_INVAL, "walkers are registered before abp_server_start");
  if (n_atoms < 1) return sfail(ABP_E_INVAL, "n_atoms must be >= 1");
  int64_t total = 0;
  for (int q = 0; q < S->nlists; ++q) {
    if (list_len[q] < 0) return sfail(ABP_E_INVAL, "negative list length");
    total += list_len[q];
  }
  if (total > 0 && !list_idx) return sfail(ABP_E_INVAL, "list_idx is NULL");
  bool rmsd = false;
  int64_t pos = 0;
  for (int a = 0; a < S->ncv; ++a) {
    const int32_t n0 = list_len[2 * a], n1 = list_len[2 * a + 1];
    const int kind = S->kind[a];
    if (kind == ABP_CV_TORSION && (n0 != 4 || n1 != 0)) return sfail(ABP_E_INVAL, "a torsion needs exactly 4 atoms");
    if (kind == ABP_CV_COM_DIST && (n0 < 1 || n1 < 1)) return sfail(ABP_E_INVAL, "COM distance needs two groups");
    if (kind == ABP_CV_RMSD_OFF && (n0 < 1 || n1 != 0)) return sfail(ABP_E_INVAL, "RMSD needs one non-empty list");
    for (int t = 0; t < 2; ++t) {
      const int32_t len = list_len[2 * a + t];
      for (int32_t j = 0; j < len; ++j) {
        const int32_t i = list_idx[pos + j];
        if (i < 0 || i >= n_atoms) return sfail(ABP_E_INVAL, "atom index out of range");
        if (kind != ABP_CV_TORSION && j > 0 && list_idx[pos + j - 1] >= i)
          return sfail(ABP_E_INVAL, "COM/RMSD lists must be strictly increasing");
        if (kind == ABP_CV_TORSION)
          for (int32_t jj = 0; jj < j; ++jj)
            if (list_idx[pos + jj] == i) return sfail(ABP_E_INVAL, "torsion atoms must be distinct");
      }
      pos += len;
    }
    rmsd = rmsd || kind == ABP_CV_RMSD_OFF;
  }
  if (rmsd && (!ref_x || !ref_y || !ref_z)) return sfail(ABP_E_INVAL, "RMSD needs reference positions");
  // the walker's CV atoms: distinct list atoms in increasing order
  std::vector<int32_t> atoms(list_idx, list_idx + total);
  std::sort(atoms.begin(), atoms.end());
  atoms.erase(std::unique(atoms.begin(), atoms.end()), atoms.end());
  const int32_t ncv_atoms = (int32_t)atoms.size();
  if ((int64_t)ncv_atoms > S->pool_atoms) return sfail(ABP_E_NOMEM, "walker's CV atoms exceed the whole budget");
  for (const int32_t i : atoms)
    if (!std::isfinite(mass[i]) || !(mass[i] > 0.0f)) return sfail(ABP_E_INVAL, "CV-atom masses must be finite and > 0");
  Walker w;
  w.n_atoms = n_atoms;
  w.n_cv = ncv_atoms;
  w.cv_base = (int64_t)S->cv_atom.size();
  w.list_base = (int64_t)S->lidx.size();
  for (int q = 0; q < S->nlists; ++q) w.len[q] = list_len[q];
  for (const int32_t i : atoms) {
    S->cv_atom.push_back(i);
    S->cv_mass.push_back(mass[i]);
  }
  for (int64_t e = 0; e < total; ++e) {
    const int32_t c = (int32_t)(std::lower_bound(atoms.begin(), atoms.end(), list_idx[e]) - atoms.begin());
    S->lidx.push_back(c);
    S->lrx.push_back(ref_x ? ref_x[e] : 0.0f);
    S->lry.push_back(ref_y ? ref_y[e] : 0.0f);
    S->lrz.push_back(ref_z ? ref_z[e] : 0.0f);
  }
  S->max_cv = std::max(S->max_cv, ncv_atoms);
  *walker_id = (int32_t)S->walkers.size();
  if (n_cv_atoms) *n_cv_atoms = ncv_atoms;
  S->walkers.push_back(std::move(w));
  return ABP_OK;
}

abp_status abp_server_walker_atoms(abp_server* S, int32_t walker, int32_t* idx, int32_t* n) {
  if (!S || !n) return sfail(ABP_E_INVAL, "NULL argument");
  if (walker < 0 || walker >= (int32_t)S->walkers.size()) return sfail(ABP_E_INVAL, "unknown walker id");
  const Walker& w = S->walkers[walker];
  *n = w.n_cv;
  if (idx) std::memcpy(idx, S->cv_atom.data() + w.cv_base, sizeof(int32_t) * (size_t)w.n_cv);
  return ABP_OK;
}

abp_status abp_server_start(abp_server* S) {
  if (!S) return sfail(ABP_E_INVAL, "NULL argument");
  if (S->thread.joinable()) return sfail(ABP_E_INVAL, "the server is running");
  if (S->walkers.empty()) return sfail(ABP_E_INVAL, "no walkers registered");
  if (abp::ctx_reserved(S->ctx) != abp_num_hills(S->ctx))
    return sfail(ABP_E_INVAL, "reserved history slots are pending; commit them before start");
  if (hipSetDevice(S->cv.device) != hipSuccess) return sfail(ABP_E_DEVICE, "cannot select device");
  if (!S->registered) {
    const size_t nl = S->lidx.size();
    if (hipMalloc(&S->d_lidx, sizeof(int32_t) * (nl + 1)) != hipSuccess ||
        hipMalloc(&S->d_rx, sizeof(float) * (nl + 1)) != hipSuccess ||
        hipMalloc(&S->d_ry, sizeof(float) * (nl + 1)) != hipSuccess ||
        hipMalloc(&S->d_rz, sizeof(float) * (nl + 1)) != hipSuccess)
      return sfail(ABP_E_NOMEM, "cannot allocate the CV lists");
    if (nl) {
      SRV_TRY(hipMemcpy(S->d_lidx, S->lidx.data(), sizeof(int32_t) * nl, hipMemcpyHostToDevice));
      SRV_TRY(hipMemcpy(S->d_rx, S->lrx.data(), sizeof(float) * nl, hipMemcpyHostToDevice));
      SRV_TRY(hipMemcpy(S->d_ry, S->lry.data(), sizeof(float) * nl, hipMemcpyHostToDevice));
      SRV_TRY(hipMemcpy(S->d_rz, S->lrz.data(), sizeof(float) * nl, hipMemcpyHostToDevice));
    }
    S->registered = true;
  }
  for (auto& sl : S->slots) {
    SRV_TRY(hipStreamSynchronize(sl.stream));
    sl.busy = false;
  }
  SRV_TRY(hipStreamSynchronize(S->commit_stream));
  if (S->grid_mode) {        // both copies start from the context's grid
    SRV_TRY(hipMemcpy(S->own_grid, S->cv.grid, sizeof(double) * S->cv.grid_doubles, hipMemcpyDeviceToDevice));
    const int64_t v = abp_num_hills(S->ctx);
    S->gcopy[0] = {S->cv.grid, S->cv.grid32, v, 0};
    S->gcopy[1] = {S->own_grid, nullptr, v, 0};
    S->gcur = 0;
    S->gupd = -1;
    S->groups.clear();
    S->gbase = 0;
  }
  abp_status st = size_buffers(S);
  if (st != ABP_OK) return st;
  st = warm_up(S);
  if (st != ABP_OK) return st;
  st = abp_sync(S->ctx, nullptr);
  if (st != ABP_OK) return st;
  reset_residency(S);
  S->launch_order.clear();
  S->dep_done.clear();
  {
    std::lock_guard<std::mutex> lk(S->mu_out);
    S->completed.clear();
  }
  {
    std::lock_guard<std::mutex> lk(S->mu_in);
    S->incoming.clear();
    S->next_id = 0;
  }
  S->outstanding = 0;
  {
    std::lock_guard<std::mutex> lk(S->mu_stats);
    const int64_t pool = S->pool_atoms;
    S->stats = abp_server_stats{};
    S->stats.pool_atoms = pool;
    S->trace.clear();
    S->trace_next = 0;
    S->t_start = now_s(S);
    S->t_stop = -1.0;
  }
  S->thread_status = ABP_OK;
  S->thread_error.clear();
  S->stopping = false;
  S->running = true;
  try {
    S->thread = std::thread(scheduler, S);
  } catch (...) {
    S->running = false;
    return sfail(ABP_E_NOMEM, "cannot start the scheduler thread");
  }
  return ABP_OK;
}

abp_status abp_server_submit(abp_server* S, int32_t walker, int64_t step, const float* xyz, float* force_out,
                             int64_t* request_id) {
  if (!S || !xyz) return sfail(ABP_E_INVAL, "NULL argument");
  if (!S->running.load() || S->stopping.load()) return sfail(ABP_E_INVAL, "the server is not running");
  if (walker < 0 || walker >= (int32_t)S->walkers.size()) return sfail(ABP_E_INVAL, "unknown walker id");
  const int32_t n = S->walkers[walker].n_cv;
  for (int64_t i = 0; i < 3 * (int64_t)n; ++i)
    if (!std::isfinite(xyz[i])) return sfail(ABP_E_NONFINITE, "non-finite CV-atom coordinate");
  int32_t r;
  int64_t id;
  {
    std::lock_guard<std::mutex> lk(S->mu_in);
    if (S->free_records.empty()) return sfail(ABP_E_BUSY, "max_pending requests are outstanding; poll first");
    r = S->free_records.back();
    S->free_records.pop_back();
    id = S->next_id++;
  }
  Record& R = S->records[r];
  float* strip = S->arena + R.arena_off;
  const int64_t M = S->block;
  for (int c = 0; c < 3; ++c) {
    std::memcpy(strip + c * M, xyz + (int64_t)c * n, sizeof(float) * (size_t)n);
    std::memset(strip + (3 + c) * M, 0, sizeof(float) * (size_t)n);     // forces accumulate from zero
  }
  R.id = id;
  R.walker = walker;
  R.n_cv = n;
  R.step = step;
  R.force_out = force_out;
  R.t_submit = now_s(S);
  R.dep_slot = -1;
  S->outstanding.fetch_add(1);
  {
    std::lock_guard<std::mutex> lk(S->mu_in);
    S->incoming.push_back(r);
  }
  S->cv_in.notify_one();
  {
    std::lock_guard<std::mutex> lk(S->mu_stats);
    S->stats.submitted++;
  }
  if (request_id) *request_id = id;
  return ABP_OK;
}

abp_status abp_server_poll(abp_server* S, abp_server_result* out, int64_t max, int64_t* n, int64_t wait_us) {
  if (!S || !n || (max > 0 && !out) || max < 0) return sfail(ABP_E_INVAL, "bad arguments");
  *n = 0;
  std::vector<int32_t> take;
  {
    std::unique_lock<std::mutex> lk(S->mu_out);
    if (S->completed.empty() && wait_us > 0)
      S->cv_out.wait_for(lk, std::chrono::microseconds(wait_us),
                         [S] { return !S->completed.empty() || !S->running.load(); });
    while (!S->completed.empty() && (int64_t)take.size() < max) {
      take.push_back(S->completed.front());
      S->completed.pop_front();
    }
  }
  for (size_t k = 0; k < take.size(); ++k) {
    const Record& R = S->records[take[k]];
    abp_server_result& o = out[k];
    o.request = R.id;
    o.step = R.step;
    o.version = R.version;
    o.deposit_slot = R.dep_slot;
    o.walker = R.walker;
    o.n_cv_atoms = R.n_cv;
    o.t_submit = R.t_submit;
    o.t_done = R.t_done;
    for (int a = 0; a < 3; ++a) {
      o.s[a] = a < S->ncv ? R.s[a] : 0.0;
      o.dVds[a] = a < S->ncv ? R.dV[a] : 0.0;
    }
    o.V = R.V;
    if (R.force_out)
      for (int c = 0; c < 3; ++c)
        std::memcpy(R.force_out + (int64_t)c * R.n_cv, S->arena + R.arena_off + (3 + c) * S->block,
                    sizeof(float) * (size_t)R.n_cv);
  }
  if (!take.empty()) {
    std::lock_guard<std::mutex> lk(S->mu_in);
    for (const int32_t r : take) S->free_records.push_back(r);
  }
  *n = (int64_t)take.size();
  return ABP_OK;
}

abp_status abp_server_get_stats(abp_server* S, abp_server_stats* out) {
  if (!S || !out) return sfail(ABP_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu_stats);
  *out = S->stats;
  out->wall_seconds = (S->t_stop >= 0.0 ? S->t_stop : now_s(S)) - S->t_start;
  return ABP_OK;
}

abp_status abp_server_trace(abp_server* S, abp_server_batch* out, int64_t max, int64_t* n) {
  if (!S || !n || max < 0 || (max > 0 && !out)) return sfail(ABP_E_INVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->mu_stats);
  const size_t have = S->trace.size();
  const size_t take = std::min(have, (size_t)max);
  // oldest first among the last `take` records
  const size_t first = S->trace_next - take;
  for (size_t k = 0; k < take; ++k) {
    const size_t i = first + k;
    out[k] = have < kTraceMax ? S->trace[i] : S->trace[i % kTraceMax];
  }
  *n = (int64_t)take;
  return ABP_OK;
}

}  // extern "C"

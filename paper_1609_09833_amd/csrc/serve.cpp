// Serving loop of libabp (abp_server_*): continuous batching of bias-force
// requests from many walkers sharing one hill history.
//
// One host thread runs the scheduler. Each turn it
//   1. releases requests whose arrival time has passed into per-walker FIFOs,
//   2. retires finished batches (event polled): records completion times and
//      outputs, frees the walkers for their next request, and commits history
//      slots once every earlier slot is done,
//   3. admits waiting walkers first come first served into the device pools,
//      evicting least recently used idle walkers when the budget is short,
//   4. if a stream is free, forms a batch from the walkers that are resident,
//      idle and have a request, and enqueues: descriptor upload (with the
//      base positions and masses of the CV atoms of walkers admitted since
//      their last batch, gathered here), the engine step (those stored into
//      the pool, CV-atom positions for this step, cleared CV-atom forces), the
//      bias-force stages (they write the outputs straight into mapped host
//      memory), an event.
// Requests in one batch see the same history version (hills committed when
// the batch was formed); deposits go to slots reserved in formation order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <functional>
#include <list>
#include <map>
#include <new>
#include <string>
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
constexpr int64_t kBytesPerAtom = ABP_SERVER_BYTES_PER_ATOM;   // ten FP32 pool arrays

struct Walker {
  int32_t n = 0;
  int64_t img_base = 0;      // first entry of the walker's CV image
  int64_t entries = 0;       // CV-list entries, all lists
  int64_t list_base = 0;     // offset in the list pool
  int32_t len[kMaxLists] = {0, 0, 0, 0, 0, 0};
  int64_t atom_base = -1;    // device pool offset when resident
  bool inflight = false;
  bool waiting_admission = false;
  bool in_ready = false;
  bool fresh = false;
  bool in_lru = false;
  std::list<int32_t>::iterator lru_it;
  std::deque<int64_t> queue;  // request indices
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  int64_t nb = 0;
  int64_t version = 0;
  std::vector<int64_t> reqs;
  std::vector<int64_t> dep_slots;   // history slot per request or -1
  char* h_desc = nullptr;            // pinned descriptor, then the staged base positions
  char* d_desc = nullptr;
  size_t desc_cap = 0;               // bytes of h_desc and of d_desc
  double* h_out = nullptr;           // mapped pinned outputs: s[ncv][nb], V[nb], dV[ncv][nb]
  double* m_out = nullptr;           // its device view: the bias-force launches write there directly
  void* d_ws = nullptr;              // bias_force workspace
  size_t ws_bytes = 0;
};

// Byte layout of a batch descriptor with nb requests (arrays packed at stride
// nb). The staging area follows at `total`: (x0, y0, z0, mass) of the CV
// entries of every walker admitted for this batch, in list order.
struct DescLayout {
  size_t atom_base, stage_off, step, dep_slot, dep_height, n_atoms, walker, list_beg, list_len, total;
  static size_t up(size_t x) { return (x + 15) / 16 * 16; }
  DescLayout(int64_t nb, int nlists) {
    size_t o = 0;
    atom_base = o; o = up(o + 8 * nb);
    stage_off = o; o = up(o + 8 * nb);
    step = o; o = up(o + 8 * nb);
    dep_slot = o; o = up(o + 8 * nb);
    dep_height = o; o = up(o + 8 * nb);
    n_atoms = o; o = up(o + 4 * nb);
    walker = o; o = up(o + 4 * nb);
    list_beg = o; o = up(o + 4 * nb * nlists);
    list_len = o; o = up(o + 4 * nb * nlists);
    total = o;
  }
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct abp_server {
  abp_ctx* ctx = nullptr;
  abp::CtxView cv;
  abp_server_desc desc{};
  int ncv = 0;
  int nlists = 0;
  int kind[3] = {0, 0, 0};
  // registered walkers (host copies until the first replay)
  std::vector<Walker> walkers;
  // CV images: (x0, y0, z0, mass) of every walker's CV-list entries, in list
  // order (the only atoms the engine step and the bias path touch)
  std::vector<float4> himg;
  std::vector<int32_t> lidx;
  std::vector<float> lrx, lry, lrz;
  bool dirty = true;
  // device list pool
  int32_t* d_lidx = nullptr;
  float* d_rx = nullptr; float* d_ry = nullptr; float* d_rz = nullptr;
  // device atom pools
  int64_t pool_atoms = 0;
  float* d_pool = nullptr;           // 10 arrays of pool_atoms floats
  abp::RangePool free_atoms;         // free atom ranges of the pools (best fit: admissions are
                                     // frequent and the pools fragment)
  std::list<int32_t> lru;            // idle resident walkers, least recent first
  std::deque<int32_t> admission;     // walkers waiting for memory
  std::deque<int32_t> ready;         // resident, idle, with a request
  std::vector<Slot> slots;
  std::deque<int> launch_order;      // busy slots in launch order
  // deposit commit bookkeeping
  std::map<int64_t, bool> dep_done;  // reserved slot -> done
  int64_t resident = 0;
  abp_server_stats stats{};
};

namespace {

float* pool_array(abp_server* S, int which) { return S->d_pool + (int64_t)which * S->pool_atoms; }

bool pool_alloc(abp_server* S, int64_t n, int64_t* off) { return S->free_atoms.alloc(n, off); }

void pool_free(abp_server* S, int64_t off, int64_t n) { S->free_atoms.free(off, n); }

// Descriptor buffers of every stream, sized once per replay for the largest
// staging a batch can need: the max_batch walkers with the most CV entries,
// all just admitted (never more than all walkers' CV images together). The
// slots must be idle.
abp_status size_descriptors(abp_server* S) {
  std::vector<int64_t> ent;
  ent.reserve(S->walkers.size());
  for (const auto& w : S->walkers) ent.push_back(w.entries);
  const size_t b = std::min(ent.size(), (size_t)S->desc.max_batch);
  std::partial_sort(ent.begin(), ent.begin() + b, ent.end(), std::greater<int64_t>());
  int64_t most = 0;
  for (size_t i = 0; i < b; ++i) most += ent[i];
  const size_t need = DescLayout(S->desc.max_batch, S->nlists).total + (size_t)most * sizeof(float4);
  for (auto& sl : S->slots) {
    if (sl.desc_cap >= need) continue;
    SRV_TRY(hipHostFree(sl.h_desc));
    SRV_TRY(hipFree(sl.d_desc));
    sl.h_desc = nullptr;
    sl.d_desc = nullptr;
    sl.desc_cap = 0;
    SRV_TRY(hipHostMalloc((void**)&sl.h_desc, need, hipHostMallocDefault));
    SRV_TRY(hipMalloc((void**)&sl.d_desc, need));
    sl.desc_cap = need;
  }
  return ABP_OK;
}

abp_status finalize(abp_server* S) {
  if (!S->dirty) return ABP_OK;
  const size_t nl = S->lidx.size();
  if (S->d_lidx) { (void)hipFree(S->d_lidx); S->d_lidx = nullptr; }
  if (S->d_rx) { (void)hipFree(S->d_rx); S->d_rx = nullptr; }
  if (S->d_ry) { (void)hipFree(S->d_ry); S->d_ry = nullptr; }
  if (S->d_rz) { (void)hipFree(S->d_rz); S->d_rz = nullptr; }
  SRV_TRY(hipMalloc(&S->d_lidx, sizeof(int32_t) * (nl + 1)));
  SRV_TRY(hipMalloc(&S->d_rx, sizeof(float) * (nl + 1)));
  SRV_TRY(hipMalloc(&S->d_ry, sizeof(float) * (nl + 1)));
  SRV_TRY(hipMalloc(&S->d_rz, sizeof(float) * (nl + 1)));
  if (nl) {
    SRV_TRY(hipMemcpy(S->d_lidx, S->lidx.data(), sizeof(int32_t) * nl, hipMemcpyHostToDevice));
    SRV_TRY(hipMemcpy(S->d_rx, S->lrx.data(), sizeof(float) * nl, hipMemcpyHostToDevice));
    SRV_TRY(hipMemcpy(S->d_ry, S->lry.data(), sizeof(float) * nl, hipMemcpyHostToDevice));
    SRV_TRY(hipMemcpy(S->d_rz, S->lrz.data(), sizeof(float) * nl, hipMemcpyHostToDevice));
  }
  S->dirty = false;
  return ABP_OK;
}

// Returns every resident walker to the pool and clears all queues.
void reset_residency(abp_server* S) {
  for (auto& w : S->walkers) {
    w.atom_base = -1;
    w.inflight = w.waiting_admission = w.in_ready = w.fresh = w.in_lru = false;
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
  if (w.in_ready || w.inflight || w.atom_base < 0 || w.queue.empty()) return;
  if (w.in_lru) {
    S->lru.erase(w.lru_it);
    w.in_lru = false;
  }
  w.in_ready = true;
  S->ready.push_back(wid);
}

void make_idle(abp_server* S, int32_t wid) {
  Walker& w = S->walkers[wid];
  if (w.in_lru || w.atom_base < 0) return;
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
    bool ok = pool_alloc(S, w.n, &off);
    while (!ok && !S->lru.empty()) {
      const int32_t victim = S->lru.front();
      S->lru.pop_front();
      Walker& v = S->walkers[victim];
      v.in_lru = false;
      pool_free(S, v.atom_base, v.n);
      v.atom_base = -1;
      S->resident--;
      S->stats.evictions++;
      ok = pool_alloc(S, w.n, &off);
    }
    if (!ok) return;                       // wait for a walker to go idle
    S->admission.pop_front();
    w.waiting_admission = false;
    w.atom_base = off;
    w.fresh = true;
    S->resident++;
    S->stats.admissions++;
    if (S->resident > S->stats.peak_resident) S->stats.peak_resident = S->resident;
    make_ready(S, wid);
  }
}

void commit_prefix(abp_server* S, hipStream_t stream) {
  int64_t upto = abp_num_hills(S->ctx);
  auto it = S->dep_done.begin();
  while (it != S->dep_done.end() && it->first == upto && it->second) {
    ++upto;
    it = S->dep_done.erase(it);
  }
  if (upto > abp_num_hills(S->ctx)) {
    const int64_t before = abp_num_hills(S->ctx);
    if (abp_commit(S->ctx, upto, stream) == ABP_OK) S->stats.deposits += upto - before;
  }
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
  if (!std::isfinite(desc->height0) || desc->height0 < 0 || !(desc->height_decay >= 0))
    return sfail(ABP_E_INVAL, "bad deposit height law");
  if (!(desc->amplitude >= 0.0f) || !std::isfinite(desc->amplitude)) return sfail(ABP_E_INVAL, "bad amplitude");
  abp_server* S = new (std::nothrow) abp_server();
  if (!S) return sfail(ABP_E_NOMEM, "host allocation failed");
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
  if (hipSetDevice(S->cv.device) != hipSuccess) {
    delete S;
    return sfail(ABP_E_DEVICE, "cannot select the context's device");
  }
  S->pool_atoms = desc->hbm_budget_bytes / kBytesPerAtom;
  if (hipMalloc(&S->d_pool, sizeof(float) * 10 * S->pool_atoms) != hipSuccess) {
    delete S;
    return sfail(ABP_E_NOMEM, "cannot allocate the walker pool");
  }
  S->stats.pool_atoms = S->pool_atoms;
  reset_residency(S);
  const int64_t B = desc->max_batch;
  DescLayout L(B, S->nlists);
  S->slots.resize(desc->streams);
  for (auto& sl : S->slots) {
    bool good = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
                hipHostMalloc((void**)&sl.h_desc, L.total, hipHostMallocDefault) == hipSuccess &&
                hipMalloc((void**)&sl.d_desc, L.total) == hipSuccess &&
                hipHostMalloc((void**)&sl.h_out, sizeof(double) * B * (2 * S->ncv + 1), hipHostMallocMapped) == hipSuccess &&
                hipHostGetDevicePointer((void**)&sl.m_out, sl.h_out, 0) == hipSuccess;
    if (!good) {
      abp_server_destroy(S);
      return sfail(ABP_E_NOMEM, "cannot allocate per-stream batch buffers");
    }
    sl.desc_cap = L.total;
    sl.reqs.reserve(B);
    sl.dep_slots.reserve(B);
    // Workspace for a full batch at the history's capacity (split shape), so
    // the loop never reallocates; it still grows on demand if this fails.
    const size_t full = abp::force_workspace_bytes(B, abp::force_blocks_per_walker(S->cv.H.capacity, 0, 0), S->ncv);
    if (full <= ((size_t)1 << 30) && hipMalloc(&sl.d_ws, full) == hipSuccess &&
        hipMemset(sl.d_ws, 0, full) == hipSuccess)
      sl.ws_bytes = full;
    else if (sl.d_ws) {
      (void)hipFree(sl.d_ws);
      sl.d_ws = nullptr;
    }
  }
  *out = S;
  return ABP_OK;
}

abp_status abp_server_destroy(abp_server* S) {
  if (!S) return ABP_OK;
  (void)hipSetDevice(S->cv.device);
  for (auto& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_desc) (void)hipHostFree(sl.h_desc);
    if (sl.d_desc) (void)hipFree(sl.d_desc);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.d_ws) (void)hipFree(sl.d_ws);
  }
  if (S->d_lidx) (void)hipFree(S->d_lidx);
  if (S->d_rx) (void)hipFree(S->d_rx);
  if (S->d_ry) (void)hipFree(S->d_ry);
  if (S->d_rz) (void)hipFree(S->d_rz);
  if (S->d_pool) (void)hipFree(S->d_pool);
  delete S;
  return ABP_OK;
}

abp_status abp_server_add_walker(abp_server* S, int32_t n_atoms, const float* x0, const float* y0,
                                 const float* z0, const float* mass, const int32_t* list_len,
                                 const int32_t* list_idx, const float* ref_x, const float* ref_y,
                                 const float* ref_z, int32_t* walker_id) {
  if (!S || !x0 || !y0 || !z0 || !mass || !list_len || !walker_id) return sfail(ABP_E_INVAL, "NULL argument");
  if (n_atoms < 1) return sfail(ABP_E_INVAL, "n_atoms must be >= 1");
  if ((int64_t)n_atoms > S->pool_atoms) return sfail(ABP_E_NOMEM, "walker larger than the whole budget");
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
  Walker w;
  w.n = n_atoms;
  w.img_base = (int64_t)S->himg.size();
  w.entries = total;
  w.list_base = (int64_t)S->lidx.size();
  for (int q = 0; q < S->nlists; ++q) w.len[q] = list_len[q];
  for (int64_t e = 0; e < total; ++e) {
    const int32_t i = list_idx[e];
    S->himg.push_back(make_float4(x0[i], y0[i], z0[i], mass[i]));
    S->lidx.push_back(i);
    S->lrx.push_back(ref_x ? ref_x[e] : 0.0f);
    S->lry.push_back(ref_y ? ref_y[e] : 0.0f);
    S->lrz.push_back(ref_z ? ref_z[e] : 0.0f);
  }
  *walker_id = (int32_t)S->walkers.size();
  S->walkers.push_back(std::move(w));
  S->dirty = true;
  return ABP_OK;
}

abp_status abp_server_replay(abp_server* S, int64_t n, const int32_t* walker, const int64_t* step,
                             const double* t_arrival, double* t_done, int64_t* version, int64_t* deposit_slot,
                             double* s_out, double* V_out, double* dV_out) {
  if (!S || n < 0 || (n > 0 && (!walker || !step || !t_arrival))) return sfail(ABP_E_INVAL, "bad arguments");
  {
    std::vector<int64_t> last(S->walkers.size(), -1);
    for (int64_t i = 0; i < n; ++i) {
      if (walker[i] < 0 || walker[i] >= (int32_t)S->walkers.size()) return sfail(ABP_E_INVAL, "unknown walker id");
      if (!(t_arrival[i] >= 0.0) || (i > 0 && t_arrival[i] < t_arrival[i - 1]))
        return sfail(ABP_E_INVAL, "arrival times must be >= 0 and not decrease");
      if (step[i] <= last[walker[i]]) return sfail(ABP_E_INVAL, "a walker's steps must be >= 0 and increase");
      last[walker[i]] = step[i];
    }
  }
  if (hipSetDevice(S->cv.device) != hipSuccess) return sfail(ABP_E_DEVICE, "cannot select device");
  if (abp::ctx_reserved(S->ctx) != abp_num_hills(S->ctx))
    return sfail(ABP_E_INVAL, "reserved history slots are pending; commit them before a replay");
  abp_status st = finalize(S);
  if (st != ABP_OK) return st;
  for (auto& sl : S->slots) {            // drain whatever an aborted replay left
    SRV_TRY(hipStreamSynchronize(sl.stream));
    sl.busy = false;
  }
  st = size_descriptors(S);
  if (st != ABP_OK) return st;
  S->launch_order.clear();
  reset_residency(S);
  S->dep_done.clear();
  const int64_t pool = S->pool_atoms;
  const abp_server_stats keep{};
  S->stats = keep;
  S->stats.pool_atoms = pool;
  const int ncv = S->ncv;
  const auto t0 = std::chrono::steady_clock::now();
  int64_t next = 0, completed = 0;

  double last_progress = 0.0;
  int64_t progress_mark = -1;
  while (completed < n) {
    const double t = now_s(t0);
    // The loop always progresses (see admit); a stall means a broken invariant.
    const int64_t mark = next + completed + S->stats.batches;
    if (mark != progress_mark) {
      progress_mark = mark;
      last_progress = t;
    } else if (t - last_progress > 60.0 && (next == n || t_arrival[next] < t - 60.0)) {
      for (auto& sl : S->slots) (void)hipStreamSynchronize(sl.stream);
      return sfail(ABP_E_DEVICE, "serving loop made no progress for 60 s");
    }
    // 1. arrivals
    while (next < n && t_arrival[next] <= t) {
      const int32_t wid = walker[next];
      Walker& w = S->walkers[wid];
      w.queue.push_back(next);
      if (w.atom_base < 0) {
        if (!w.waiting_admission) {
          w.waiting_admission = true;
          S->admission.push_back(wid);
        }
      } else {
        make_ready(S, wid);
      }
      ++next;
    }
    // 2. retire finished batches, in launch order
    while (!S->launch_order.empty()) {
      Slot& sl = S->slots[S->launch_order.front()];
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return sfail(ABP_E_DEVICE, std::string("batch failed: ") + hipGetErrorString(q));
      const double td = now_s(t0);
      const int64_t nb = sl.nb;
      for (int64_t j = 0; j < nb; ++j) {
        const int64_t r = sl.reqs[j];
        if (t_done) t_done[r] = td;
        if (version) version[r] = sl.version;
        if (deposit_slot) deposit_slot[r] = sl.dep_slots[j];
        for (int a = 0; a < ncv; ++a) {
          if (s_out) s_out[a * n + r] = sl.h_out[a * nb + j];
          if (dV_out) dV_out[a * n + r] = sl.h_out[(ncv + 1 + a) * nb + j];
        }
        if (V_out) V_out[r] = sl.h_out[ncv * nb + j];
        const int32_t wid = walker[r];
        Walker& w = S->walkers[wid];
        w.inflight = false;
        if (w.queue.empty()) make_idle(S, wid);
        else make_ready(S, wid);
        if (sl.dep_slots[j] >= 0) S->dep_done[sl.dep_slots[j]] = true;
      }
      completed += nb;
      S->stats.completed += nb;
      sl.busy = false;
      const int idx = S->launch_order.front();
      S->launch_order.pop_front();
      commit_prefix(S, S->slots[idx].stream);
    }
    // 3. admission
    admit(S);
    // 4. form and launch a batch on a free stream
    if (S->ready.empty()) continue;
    int free_slot = -1;
    for (int k = 0; k < (int)S->slots.size(); ++k)
      if (!S->slots[k].busy) { free_slot = k; break; }
    if (free_slot < 0) continue;
    Slot& sl = S->slots[free_slot];
    const int64_t nb = std::min<int64_t>((int64_t)S->ready.size(), S->desc.max_batch);
    DescLayout L(nb, S->nlists);
    // Staging for the walkers admitted since their last batch (the buffers
    // were sized for the worst case when the replay began).
    {
      int64_t n_stage = 0;
      for (int64_t j = 0; j < nb; ++j) {
        const Walker& w = S->walkers[S->ready[j]];
        if (w.fresh) n_stage += w.entries;
      }
      if (L.total + (size_t)n_stage * sizeof(float4) > sl.desc_cap)
        return sfail(ABP_E_DEVICE, "batch descriptor larger than sized (internal error)");
    }
    int64_t* d_atom_base = reinterpret_cast<int64_t*>(sl.h_desc + L.atom_base);
    int64_t* d_stage_off = reinterpret_cast<int64_t*>(sl.h_desc + L.stage_off);
    float4* h_stage = reinterpret_cast<float4*>(sl.h_desc + L.total);
    int64_t spos = 0;
    int64_t* d_step = reinterpret_cast<int64_t*>(sl.h_desc + L.step);
    int64_t* d_dep = reinterpret_cast<int64_t*>(sl.h_desc + L.dep_slot);
    double* d_hgt = reinterpret_cast<double*>(sl.h_desc + L.dep_height);
    int32_t* d_n = reinterpret_cast<int32_t*>(sl.h_desc + L.n_atoms);
    int32_t* d_wid = reinterpret_cast<int32_t*>(sl.h_desc + L.walker);
    int32_t* d_lbeg = reinterpret_cast<int32_t*>(sl.h_desc + L.list_beg);
    int32_t* d_llen = reinterpret_cast<int32_t*>(sl.h_desc + L.list_len);
    sl.reqs.clear();
    sl.dep_slots.clear();
    sl.version = abp_num_hills(S->ctx);
    bool any_deposit = false;
    for (int64_t j = 0; j < nb; ++j) {
      const int32_t wid = S->ready.front();
      S->ready.pop_front();
      Walker& w = S->walkers[wid];
      w.in_ready = false;
      w.inflight = true;
      const int64_t r = w.queue.front();
      w.queue.pop_front();
      sl.reqs.push_back(r);
      d_atom_base[j] = w.atom_base;
      d_stage_off[j] = -1;
      if (w.fresh) {          // this walker's CV entries, in list order
        d_stage_off[j] = spos;
        std::memcpy(h_stage + spos, S->himg.data() + w.img_base, sizeof(float4) * (size_t)w.entries);
        spos += w.entries;
        w.fresh = false;
      }
      d_step[j] = step[r];
      d_n[j] = w.n;
      d_wid[j] = wid;
      int64_t lpos = w.list_base;
      for (int q = 0; q < S->nlists; ++q) {
        d_lbeg[q * nb + j] = (int32_t)lpos;
        d_llen[q * nb + j] = w.len[q];
        lpos += w.len[q];
      }
      int64_t slot = -1;
      if (S->desc.deposit_every > 0 && step[r] > 0 && step[r] % S->desc.deposit_every == 0) {
        if (abp_reserve(S->ctx, 1, &slot) != ABP_OK) slot = -1;     // history full: no deposit
        if (slot >= 0) {
          S->dep_done[slot] = false;
          any_deposit = true;
        }
      }
      d_dep[j] = slot;
      d_hgt[j] = S->desc.height_decay > 0 ? S->desc.height0 * std::exp(-(double)std::max<int64_t>(slot, 0) /
                                                                        S->desc.height_decay)
                                          : S->desc.height0;
      sl.dep_slots.push_back(slot);
    }
    sl.nb = nb;
    // Workspace for this batch's partial sums (split or chained shape); grows with the history
    // (the slot is idle here, so freeing its old buffer is safe).
    const size_t need = abp::force_uses_workspace(nb, sl.version, 0, 0)
                            ? abp::force_workspace_bytes(nb, abp::force_blocks_per_walker(sl.version, 0, 0), ncv)
                            : 0;
    if (need > sl.ws_bytes) {
      if (sl.d_ws) SRV_TRY(hipFree(sl.d_ws));
      sl.d_ws = nullptr;
      sl.ws_bytes = 0;
      const size_t want = std::max(need, abp::force_workspace_bytes(
          S->desc.max_batch, abp::force_blocks_per_walker(2 * sl.version + 4096, 0, 0), ncv));
      if (hipMalloc(&sl.d_ws, want) != hipSuccess) return sfail(ABP_E_NOMEM, "cannot grow the batch workspace");
      SRV_TRY(hipMemset(sl.d_ws, 0, want));
      sl.ws_bytes = want;
    }
    SRV_TRY(hipMemcpyAsync(sl.d_desc, sl.h_desc, L.total + (size_t)spos * sizeof(float4), hipMemcpyHostToDevice,
                           sl.stream));
    abp::EngineArgs E;
    E.nb = nb;
    E.atom_base = reinterpret_cast<const int64_t*>(sl.d_desc + L.atom_base);
    E.n_atoms = reinterpret_cast<const int32_t*>(sl.d_desc + L.n_atoms);
    E.stage_off = reinterpret_cast<const int64_t*>(sl.d_desc + L.stage_off);
    E.stage = reinterpret_cast<const float4*>(sl.d_desc + L.total);
    E.walker = reinterpret_cast<const int32_t*>(sl.d_desc + L.walker);
    E.step = reinterpret_cast<const int64_t*>(sl.d_desc + L.step);
    E.nlists = S->nlists;
    E.list_beg = reinterpret_cast<const int32_t*>(sl.d_desc + L.list_beg);
    E.list_len = reinterpret_cast<const int32_t*>(sl.d_desc + L.list_len);
    E.list_idx = S->d_lidx;
    E.amplitude = S->desc.amplitude;
    E.x = pool_array(S, 0);
    E.y = pool_array(S, 1);
    E.z = pool_array(S, 2);
    E.mass = pool_array(S, 3);
    E.fx = pool_array(S, 4);
    E.fy = pool_array(S, 5);
    E.fz = pool_array(S, 6);
    E.x0 = pool_array(S, 7);
    E.y0 = pool_array(S, 8);
    E.z0 = pool_array(S, 9);
    SRV_TRY(abp::launch_engine_step(E, sl.stream));
    abp::ForceArgs A;
    std::memset(&A, 0, sizeof(A));
    A.ncv = ncv;
    for (int a = 0; a < 3; ++a) A.kind[a] = S->kind[a];
    A.list_beg = E.list_beg;
    A.list_len = E.list_len;
    A.list_idx = S->d_lidx;
    A.ref_x = S->d_rx;
    A.ref_y = S->d_ry;
    A.ref_z = S->d_rz;
    A.nw = nb;
    A.atom_base = E.atom_base;
    A.n_atoms = E.n_atoms;
    A.x = E.x;
    A.y = E.y;
    A.z = E.z;
    A.mass = E.mass;
    A.fx = E.fx;
    A.fy = E.fy;
    A.fz = E.fz;
    A.n_visible = nullptr;
    A.n_visible_default = sl.version;
    A.deposit_slot = any_deposit ? reinterpret_cast<const int64_t*>(sl.d_desc + L.dep_slot) : nullptr;
    A.deposit_height = reinterpret_cast<const double*>(sl.d_desc + L.dep_height);
    A.s = sl.m_out;
    A.V = sl.m_out + ncv * nb;
    A.dVds = sl.m_out + (ncv + 1) * nb;
    A.prec = S->desc.prec;
    A.err = S->cv.err;
    SRV_TRY(abp::launch_bias_force(S->cv.K, S->cv.H, A, sl.d_ws, sl.stream));
    SRV_TRY(hipEventRecord(sl.done, sl.stream));
    sl.busy = true;
    S->launch_order.push_back(free_slot);
    S->stats.batches++;
    if (nb > S->stats.max_batch_seen) S->stats.max_batch_seen = nb;
  }
  for (auto& sl : S->slots) SRV_TRY(hipStreamSynchronize(sl.stream));
  S->stats.wall_seconds = now_s(t0);
  // Device-side flags (invalid walker, non-finite input) surface here.
  return abp_sync(S->ctx, nullptr);
}

abp_status abp_server_get_stats(abp_server* S, abp_server_stats* out) {
  if (!S || !out) return sfail(ABP_E_INVAL, "NULL argument");
  *out = S->stats;
  return ABP_OK;
}

}  // extern "C"

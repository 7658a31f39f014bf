// abp_serve_driver.cpp - an open-loop load generator for the serving loop of
// libabp.so, written against the public C-ABI only (include/abp.h): what an
// MD engine, or many of them, would do with abp_server_submit and
// abp_server_poll. The benchmark and the serving tests drive the server
// through it; it is not part of the library.
//
// Engine model (synthetic): the CV atoms of walker w at MD step t sit at
//   x = x0 + amplitude * u(w, t, atom, coordinate),  u in [-1, 1),
// with u from an integer hash (the "lowbias32" mixer, C. Wellons, 2018) and
// float arithmetic whose result does not depend on contraction (amplitude is
// a power of two and u a multiple of 2^-15, so the product is exact), so a
// host reproduces the positions bit for bit.
//
// Build: g++ -O2 -std=c++17 -shared -fPIC -pthread -I<repo>/include abp_serve_driver.cpp
//        -L<dir of libabp.so> -labp -Wl,-rpath,<dir of libabp.so> -o libabp_serve_driver.so
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "abp.h"

namespace {

inline uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  h *= 0x846ca68bu;
  h ^= h >> 16;
  return h;
}

inline float unit_hash(uint32_t w, uint32_t step, uint32_t atom, uint32_t coord) {
  const uint32_t h = mix32(w * 0x9e3779b1u ^ mix32(step * 0x85ebca77u ^ mix32(atom * 0xc2b2ae3du + coord)));
  return (float)(int32_t)((h >> 16) & 0xffffu) * (1.0f / 32768.0f) - 1.0f;
}

void fail_msg(char* err, int errlen, const char* what, abp_status st) {
  if (err && errlen > 0) std::snprintf(err, (size_t)errlen, "%s: %s (%s)", what, abp_status_str(st), abp_last_error());
}

}  // namespace

extern "C" {

// Positions of request i (walker[i] at step[i]) into pos + pos_off[i],
// [3][n] for the walker's n CV atoms (x block, y block, z block), from the
// walker's CV-atom base positions base + base_off[w] (same layout) and its CV
// atom indices atoms + base_off[w] / 3 (n of them). `threads` host threads.
void abp_drv_positions(int64_t n_req, const int32_t* walker, const int64_t* step, const float* base,
                       const int64_t* base_off, const int32_t* n_cv, const int32_t* atoms, float amplitude,
                       float* pos, const int64_t* pos_off, int threads) {
  threads = std::max(1, threads);
  auto work = [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t w = walker[i];
      const int32_t n = n_cv[w];
      const float* b = base + base_off[w];
      const int32_t* at = atoms + base_off[w] / 3;
      float* p = pos + pos_off[i];
      for (int c = 0; c < 3; ++c)
        for (int32_t a = 0; a < n; ++a)
          p[c * n + a] = b[c * n + a] + amplitude * unit_hash((uint32_t)w, (uint32_t)step[i], (uint32_t)at[a], (uint32_t)c);
    }
  };
  std::vector<std::thread> pool;
  const int64_t per = (n_req + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    const int64_t lo = t * per, hi = std::min(n_req, lo + per);
    if (lo < hi) pool.emplace_back(work, lo, hi);
  }
  for (auto& th : pool) th.join();
}

// Replays an open-loop schedule against a started server: request i (walker
// walker[i], MD step step[i], positions pos + pos_off[i] as [3][n_cv]) is
// submitted t_arrival[i] seconds after the call starts (non-decreasing
// times), and results are polled as they come. Outputs per request, each may
// be NULL: t_submit and t_done in seconds since the call started (t_done is
// the scheduler's completion time, moved to this clock), version,
// deposit_slot, s[ncv][n], V[n], dVds[ncv][n], and the bias forces at
// forces + pos_off[i] ([3][n_cv]). Returns 0, or -1 with a message in err.
int abp_drv_replay(abp_server* srv, int32_t ncv, int64_t n, const int32_t* walker, const int64_t* step,
                   const double* t_arrival, const float* pos, const int64_t* pos_off, double* t_submit,
                   double* t_done, int64_t* version, int64_t* deposit_slot, double* s, double* V, double* dVds,
                   float* forces, char* err, int errlen) {
  using clk = std::chrono::steady_clock;
  const auto T0 = clk::now();
  auto now = [&] { return std::chrono::duration<double>(clk::now() - T0).count(); };
  std::vector<int64_t> index;                 // request id -> i
  std::vector<double> offset(n, 0.0);         // this clock minus the server's, per request
  std::vector<abp_server_result> res(4096);
  int64_t next = 0, done = 0, first_id = -1;
  while (done < n) {
    const double t = now();
    while (next < n && t_arrival[next] <= t) {
      int64_t id = -1;
      const double ts = now();
      const abp_status st = abp_server_submit(srv, walker[next], step[next], pos + pos_off[next],
                                              forces ? forces + pos_off[next] : nullptr, &id);
      if (st == ABP_E_BUSY) break;            // poll first
      if (st != ABP_OK) {
        fail_msg(err, errlen, "abp_server_submit", st);
        return -1;
      }
      if (first_id < 0) first_id = id;
      if ((int64_t)index.size() <= id - first_id) index.resize((size_t)(id - first_id) + 1, -1);
      index[(size_t)(id - first_id)] = next;
      if (t_submit) t_submit[next] = ts;
      offset[next] = ts;                      // completed below with the server's submit time
      ++next;
    }
    int64_t got = 0;
    const abp_status st = abp_server_poll(srv, res.data(), (int64_t)res.size(), &got, 0);
    if (st != ABP_OK) {
      fail_msg(err, errlen, "abp_server_poll", st);
      return -1;
    }
    for (int64_t k = 0; k < got; ++k) {
      const abp_server_result& r = res[(size_t)k];
      const int64_t rel = r.request - first_id;
      if (rel < 0 || rel >= (int64_t)index.size() || index[(size_t)rel] < 0) {
        if (err && errlen > 0) std::snprintf(err, (size_t)errlen, "result for an unknown request %lld", (long long)r.request);
        return -1;
      }
      const int64_t i = index[(size_t)rel];
      const double off = offset[i] - r.t_submit;
      if (t_done) t_done[i] = r.t_done + off;
      if (version) version[i] = r.version;
      if (deposit_slot) deposit_slot[i] = r.deposit_slot;
      for (int a = 0; a < ncv; ++a) {
        if (s) s[a * n + i] = r.s[a];
        if (dVds) dVds[a * n + i] = r.dVds[a];
      }
      if (V) V[i] = r.V;
    }
    done += got;
    if (got == 0) {
      // nothing came back: spin (no lock) until the next arrival, at most 5 us
      const double until = std::min(next < n ? t_arrival[next] : 1e300, now() + 5e-6);
      while (now() < until) {
      }
    }
  }
  return 0;
}

}  // extern "C"

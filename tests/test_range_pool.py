"""The serving loop's walker-pool bookkeeping (csrc/range_pool.h, host code)
against a brute-force model: random allocations and frees on a small pool.
After every operation the pool's free ranges must be exactly the maximal free
runs of the model (so freed ranges merged with their neighbours), every
allocation must lie in free slots, be the shortest free run that fits
(lowest offset among equals), and fail only when no free run is long
enough."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_09833_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include "range_pool.h"

static int fail(const char* what, long step) { std::printf("FAIL %s at step %ld\n", what, step); return 1; }

int main() {
  const int64_t size = 1000;
  std::mt19937_64 rng(12345);
  abp::RangePool pool;
  std::vector<char> used(size, 0);
  std::vector<std::pair<int64_t, int64_t>> live;
  for (int round = 0; round < 3; ++round) {
    pool.reset(size);
    std::fill(used.begin(), used.end(), 0);
    live.clear();
    for (long step = 0; step < 20000; ++step) {
      const bool do_alloc = live.empty() || (rng() % 100) < 55;
      if (do_alloc) {
        const int64_t n = 1 + (int64_t)(rng() % 60);
        // model: maximal free runs, the shortest that fits (lowest offset first)
        int64_t best_off = -1, best_len = 0;
        for (int64_t i = 0; i < size;) {
          if (used[i]) { ++i; continue; }
          int64_t j = i;
          while (j < size && !used[j]) ++j;
          const int64_t len = j - i;
          if (len >= n && (best_off < 0 || len < best_len)) { best_off = i; best_len = len; }
          i = j;
        }
        int64_t off = -1;
        const bool ok = pool.alloc(n, &off);
        if (ok != (best_off >= 0)) return fail("alloc success differs from the model", step);
        if (ok) {
          if (off != best_off) return fail("not the best fit", step);
          for (int64_t k = off; k < off + n; ++k) {
            if (k < 0 || k >= size || used[k]) return fail("overlap or out of the pool", step);
            used[k] = 1;
          }
          live.push_back({off, n});
        }
      } else {
        const size_t pick = rng() % live.size();
        const auto r = live[pick];
        live[pick] = live.back();
        live.pop_back();
        pool.free(r.first, r.second);
        for (int64_t k = r.first; k < r.first + r.second; ++k) used[k] = 0;
      }
      // the pool's free ranges are the model's maximal free runs
      std::vector<std::pair<int64_t, int64_t>> runs;
      for (int64_t i = 0; i < size;) {
        if (used[i]) { ++i; continue; }
        int64_t j = i;
        while (j < size && !used[j]) ++j;
        runs.push_back({i, j - i});
        i = j;
      }
      const auto& got = pool.ranges();
      if (got.size() != runs.size()) return fail("free range count", step);
      size_t q = 0;
      for (const auto& kv : got) {
        if (kv.first != runs[q].first || kv.second != runs[q].second) return fail("free ranges differ", step);
        ++q;
      }
    }
  }
  std::printf("ok\n");
  return 0;
}
"""


def test_range_pool_matches_brute_force(tmp_path):
    src = tmp_path / "pool_test.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "pool_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, "-o", str(exe), str(src)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr

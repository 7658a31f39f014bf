/* A plain C client of libabp.so (no Python, no PyTorch): one walker's bias
 * on a 2-D torsion CV space. It creates a context, deposits hills from host
 * data copied to the device with the HIP runtime, evaluates V and dV/ds at a
 * few CV points by the direct sum and the grid, and prints them.
 *
 * Build: gcc -std=c11 -D__HIP_PLATFORM_AMD__ -I<repo>/include -I/opt/rocm/include abp_c_client.c
 *        -L<dir of libabp.so> -labp -Wl,-rpath,<dir of libabp.so> -L/opt/rocm/lib -lamdhip64 -lm
 *        -o abp_c_client
 * Run:   abp_c_client <n_hills> <n_queries> <seed> [hills.bin]
 * Output: one line per query: q0 q1 V_direct dV0 dV1 V_grid (FP64, %.17g);
 * with a fourth argument the hills are also written there as raw FP64
 * (centres [2][n], then heights [n]).
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "abp.h"

static uint64_t lcg(uint64_t* s) {          /* splitmix64 */
  uint64_t z = (*s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static double uniform(uint64_t* s, double lo, double hi) {
  return lo + (hi - lo) * (double)(lcg(s) >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(call)                                                                   \
  do {                                                                                \
    abp_status st_ = (call);                                                          \
    if (st_ != ABP_OK) {                                                              \
      fprintf(stderr, "%s: %s (%s)\n", #call, abp_status_str(st_), abp_last_error()); \
      return 1;                                                                       \
    }                                                                                 \
  } while (0)
#define HCHECK(call)                                      \
  do {                                                    \
    if ((call) != hipSuccess) {                           \
      fprintf(stderr, "%s failed\n", #call);              \
      return 1;                                           \
    }                                                     \
  } while (0)

int main(int argc, char** argv) {
  const int64_t nh = argc > 1 ? atoll(argv[1]) : 1000;
  const int64_t nq = argc > 2 ? atoll(argv[2]) : 8;
  uint64_t seed = argc > 3 ? strtoull(argv[3], NULL, 10) : 1;
  const double pi = 3.14159265358979323846;

  abp_bias_desc d = {0};
  d.ndim = 2;
  d.periodic[0] = d.periodic[1] = 1;
  d.lo[0] = d.lo[1] = -pi;
  d.hi[0] = d.hi[1] = pi;
  d.kernel = ABP_K_GAUSS;
  d.width[0] = d.width[1] = 0.3;
  d.transform = ABP_T_PLAIN;
  d.grid_n[0] = d.grid_n[1] = 128;
  d.capacity = nh;
  abp_ctx* ctx = NULL;
  CHECK(abp_create(&d, 0, &ctx));

  double* hc = malloc(sizeof(double) * 2 * nh);
  double* hw = malloc(sizeof(double) * nh);
  double* hq = malloc(sizeof(double) * 2 * nq);
  for (int64_t k = 0; k < nh; ++k) {
    hc[k] = uniform(&seed, -pi, pi);
    hc[nh + k] = uniform(&seed, -pi, pi);
    hw[k] = uniform(&seed, 0.1, 1.2);
  }
  for (int64_t j = 0; j < nq; ++j) {
    hq[j] = uniform(&seed, -pi, pi);
    hq[nq + j] = uniform(&seed, -pi, pi);
  }
  if (argc > 4) {
    FILE* f = fopen(argv[4], "wb");
    if (!f || fwrite(hc, sizeof(double), 2 * nh, f) != (size_t)(2 * nh) ||
        fwrite(hw, sizeof(double), nh, f) != (size_t)nh) {
      fprintf(stderr, "cannot write %s\n", argv[4]);
      return 1;
    }
    fclose(f);
  }
  double *dc, *dw, *dq, *dV, *ddV, *dVg, *ddVg;
  HCHECK(hipMalloc((void**)&dc, sizeof(double) * 2 * nh));
  HCHECK(hipMalloc((void**)&dw, sizeof(double) * nh));
  HCHECK(hipMalloc((void**)&dq, sizeof(double) * 2 * nq));
  HCHECK(hipMalloc((void**)&dV, sizeof(double) * nq));
  HCHECK(hipMalloc((void**)&ddV, sizeof(double) * 2 * nq));
  HCHECK(hipMalloc((void**)&dVg, sizeof(double) * nq));
  HCHECK(hipMalloc((void**)&ddVg, sizeof(double) * 2 * nq));
  HCHECK(hipMemcpy(dc, hc, sizeof(double) * 2 * nh, hipMemcpyHostToDevice));
  HCHECK(hipMemcpy(dw, hw, sizeof(double) * nh, hipMemcpyHostToDevice));
  HCHECK(hipMemcpy(dq, hq, sizeof(double) * 2 * nq, hipMemcpyHostToDevice));

  CHECK(bias_deposit(ctx, nh, ABP_F64, dc, dw, NULL));
  CHECK(bias_eval(ctx, ABP_EVAL_DIRECT, ABP_PREC_FP32_KAHAN, nq, ABP_F64, dq, -1, dV, ddV, NULL));
  CHECK(bias_eval(ctx, ABP_EVAL_GRID, ABP_PREC_FP64, nq, ABP_F64, dq, -1, dVg, ddVg, NULL));
  CHECK(abp_sync(ctx, NULL));

  double* V = malloc(sizeof(double) * nq);
  double* dV2 = malloc(sizeof(double) * 2 * nq);
  double* Vg = malloc(sizeof(double) * nq);
  HCHECK(hipMemcpy(V, dV, sizeof(double) * nq, hipMemcpyDeviceToHost));
  HCHECK(hipMemcpy(dV2, ddV, sizeof(double) * 2 * nq, hipMemcpyDeviceToHost));
  HCHECK(hipMemcpy(Vg, dVg, sizeof(double) * nq, hipMemcpyDeviceToHost));
  printf("# hills %lld, hills committed %lld\n", (long long)nh, (long long)abp_num_hills(ctx));
  for (int64_t j = 0; j < nq; ++j)
    printf("%.17g %.17g %.17g %.17g %.17g %.17g\n", hq[j], hq[nq + j], V[j], dV2[j], dV2[nq + j], Vg[j]);

  CHECK(abp_destroy(ctx));
  (void)hipFree(dc); (void)hipFree(dw); (void)hipFree(dq); (void)hipFree(dV);
  (void)hipFree(ddV); (void)hipFree(dVg); (void)hipFree(ddVg);
  free(hc); free(hw); free(hq); free(V); free(dV2); free(Vg);
  return 0;
}

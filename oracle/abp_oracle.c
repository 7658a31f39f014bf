/* FP64 CPU oracle for the adaptive-biasing-potential bias-force path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg. The GPU library never links or calls it and
 * shares no code with it.
 *
 * Everything is double precision, written as plain loops in the order of the
 * definitions it follows. Sums over hills run in hill index order with
 * Neumaier's compensated summation (A. Neumaier, ZAMM 54, 1974), which only
 * makes the oracle's own rounding smaller; it does not change what is summed.
 *
 * Paper: Dickson et al., arXiv:1609.09833, Supplemental Material.
 */
#include "abp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Compensated running sum (Neumaier).                                       */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double nsum_get(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Kernels                                                                    */
/* ------------------------------------------------------------------------ */

/* Minimum image: the displacement on a circle of length `period` that is
 * nearest to zero; ties (exactly half a period) round to even multiples. */
double orc_wrap(double delta, double period) {
  return delta - period * nearbyint(delta / period);
}

/* One axis of a hill, evaluated at delta = s - center.
 *
 * Gaussian (eq. ghill): exp(-|xi|^2 / alpha^2) is a product over axes. The
 * width is given as sigma with alpha = sqrt(2) sigma, so each axis factor is
 * exp(-delta^2 / (2 sigma^2)); its derivative with respect to s is
 * -(delta / sigma^2) times the factor.
 *
 * Compact (eq. compacthill): S_a^p(delta) = e^p exp(-p / (1 - (delta/a)^2))
 * for |delta/a| < 1 and 0 otherwise, so that S(0) = 1. Its derivative with
 * respect to s is -2 p delta / (a^2 (1 - (delta/a)^2)^2) times S.
 *
 * The sign convention of the derivative histogram h' is the derivative with
 * respect to the evaluation point, which makes eq. btraj-grad the gradient
 * of eq. apfm. */
void orc_kernel_1d(int32_t kernel, double width, int32_t p, double delta,
                   double* value, double* deriv) {
  if (kernel == ORC_GAUSS) {
    double sigma = width;
    double k = exp(-(delta * delta) / (2.0 * sigma * sigma));
    *value = k;
    *deriv = -(delta / (sigma * sigma)) * k;
  } else {
    double a = width;
    double u = delta / a;
    if (fabs(u) < 1.0) {
      double one_minus = 1.0 - u * u;
      double S = exp((double)p) * exp(-(double)p / one_minus);
      *value = S;
      *deriv = -2.0 * p * delta / (a * a * one_minus * one_minus) * S;
    } else {
      *value = 0.0;
      *deriv = 0.0;
    }
  }
}

static int bias_ok(const orc_bias* B) {
  if (!B || B->ndim < 1 || B->ndim > 3) return 0;
  for (int i = 0; i < B->ndim; ++i) {
    if (!(B->width[i] > 0.0)) return 0;
    if (B->periodic[i] && !(B->hi[i] > B->lo[i])) return 0;
  }
  if (B->kernel != ORC_GAUSS && B->kernel != ORC_COMPACT) return 0;
  if (B->kernel == ORC_COMPACT && B->p < 1) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Quantised mode: the trajectory's CV value is approximated by the nearest  */
/* grid point before the update (text before eq. update). Rounding: floor of  */
/* (x - lo)/dx + 1/2, so a point halfway between nodes goes to the upper one. */
/* ------------------------------------------------------------------------ */
static double node_spacing(const orc_bias* B, int i) {
  const double L = B->hi[i] - B->lo[i];
  return B->periodic[i] ? L / (double)B->grid_n[i] : L / (double)(B->grid_n[i] - 1);
}

int64_t orc_snap_index(const orc_bias* B, int32_t axis, double x) {
  const double n = (double)B->grid_n[axis];
  double t = floor((x - B->lo[axis]) / node_spacing(B, axis) + 0.5);
  if (!isfinite(t)) t = 0.0;
  if (B->periodic[axis]) t -= n * floor(t / n);
  if (t < 0.0) t = 0.0;
  if (t > n - 1.0) t = n - 1.0;
  return (int64_t)t;
}

double orc_snap(const orc_bias* B, int32_t axis, double x) {
  const double j = (double)orc_snap_index(B, axis, x);
  const double p = j * node_spacing(B, axis);
  return B->lo[axis] + p;
}

/* Displacement s - c on axis i, minimum image on periodic axes. */
static double axis_delta(const orc_bias* B, int i, double s, double c) {
  double d = s - c;
  if (B->periodic[i]) d = orc_wrap(d, B->hi[i] - B->lo[i]);
  return d;
}

/* ------------------------------------------------------------------------ */
/* Direct sum: eq. histos with the time integral replaced by the deposited   */
/* hills, h(s) = sum_k w_k K(s - c_k), and its gradient.                      */
/* ------------------------------------------------------------------------ */
static void hill_sum_one(const orc_bias* B, int64_t nh, const double* centers,
                         const double* heights, const double* s,
                         double* h, double* dh, double* A0, double* A) {
  const int d = B->ndim;
  nsum H = {0, 0}, G[3] = {{0, 0}, {0, 0}, {0, 0}}, AH = {0, 0}, AG[3] = {{0, 0}, {0, 0}, {0, 0}};
  double x[3];
  for (int i = 0; i < d; ++i) x[i] = B->quantize ? orc_snap(B, i, s[i]) : s[i];
  for (int64_t k = 0; k < nh; ++k) {
    double val[3], der[3];
    for (int i = 0; i < d; ++i) {
      double ck = centers[(int64_t)i * nh + k];
      if (B->quantize) ck = orc_snap(B, i, ck);
      double delta = axis_delta(B, i, x[i], ck);
      orc_kernel_1d(B->kernel, B->width[i], B->p, delta, &val[i], &der[i]);
    }
    double w = heights[k];
    double K = 1.0;
    for (int i = 0; i < d; ++i) K *= val[i];
    nsum_add(&H, w * K);
    nsum_add(&AH, fabs(w * K));
    for (int i = 0; i < d; ++i) {
      double g = w * der[i];
      for (int j = 0; j < d; ++j)
        if (j != i) g *= val[j];
      nsum_add(&G[i], g);
      nsum_add(&AG[i], fabs(g));
    }
  }
  *h = nsum_get(&H);
  if (A0) *A0 = nsum_get(&AH);
  for (int i = 0; i < d; ++i) {
    dh[i] = nsum_get(&G[i]);
    if (A) A[i] = nsum_get(&AG[i]);
  }
}

int32_t orc_hill_sum(const orc_bias* B, int64_t nh, const double* centers, const double* heights,
                     int64_t nq, const double* q, double* h, double* dh, double* A0, double* A) {
  if (!bias_ok(B) || nh < 0 || nq < 0) return ORC_E_INVAL;
  const int d = B->ndim;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < nq; ++j) {
    double s[3], g[3], a[3], a0;
    for (int i = 0; i < d; ++i) s[i] = q[(int64_t)i * nq + j];
    hill_sum_one(B, nh, centers, heights, s, &h[j], g, &a0, a);
    for (int i = 0; i < d; ++i) {
      dh[(int64_t)i * nq + j] = g[i];
      if (A) A[(int64_t)i * nq + j] = a[i];
    }
    if (A0) A0[j] = a0;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Transform. PLAIN: V = h. MABP (eq. apfm): V = kT b/(1-b) ln(c(1-b)h + 1);  */
/* its gradient (eq. btraj-grad): c b kT h'_i / (1 + c(1-b) h).               */
/* slope = dV/dh, used by tolerance definitions.                              */
/* ------------------------------------------------------------------------ */
static void transform_one(const orc_bias* B, double h, const double* dh, double* V, double* dV,
                          double* slope) {
  const int d = B->ndim;
  if (B->transform == ORC_PLAIN) {
    *V = h;
    for (int i = 0; i < d; ++i) dV[i] = dh[i];
    if (slope) *slope = 1.0;
  } else {
    double kT = B->kT, b = B->b, c = B->c;
    *V = kT * b / (1.0 - b) * log1p(c * (1.0 - b) * h);
    double den = 1.0 + c * (1.0 - b) * h;
    for (int i = 0; i < d; ++i) dV[i] = c * b * kT * dh[i] / den;
    if (slope) *slope = c * b * kT / den;
  }
}

int32_t orc_transform(const orc_bias* B, int64_t nq, const double* h, const double* dh,
                      double* V, double* dV, double* slope) {
  if (!bias_ok(B) || nq < 0) return ORC_E_INVAL;
  if (B->transform == ORC_MABP && !(B->b > 0.0 && B->b < 1.0 && B->c >= 0.0)) return ORC_E_INVAL;
  const int d = B->ndim;
  for (int64_t j = 0; j < nq; ++j) {
    double g[3], o[3];
    for (int i = 0; i < d; ++i) g[i] = dh[(int64_t)i * nq + j];
    transform_one(B, h[j], g, &V[j], o, slope ? &slope[j] : NULL);
    for (int i = 0; i < d; ++i) dV[(int64_t)i * nq + j] = o[i];
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Grid (eq. update / eq. Cupdate accumulated over all hills, at the nodes).  */
/* Periodic axis: nodes lo + j L/n, j = 0..n-1. Non-periodic axis: nodes      */
/* lo + j (hi-lo)/(n-1), j = 0..n-1, both ends included.                      */
/* ------------------------------------------------------------------------ */
double orc_grid_coord(const orc_bias* B, int32_t axis, int64_t j) {
  int64_t n = B->grid_n[axis];
  if (B->periodic[axis]) return B->lo[axis] + (double)j * (B->hi[axis] - B->lo[axis]) / (double)n;
  return B->lo[axis] + (double)j * (B->hi[axis] - B->lo[axis]) / (double)(n - 1);
}

static int grid_ok(const orc_bias* B) {
  if (!bias_ok(B)) return 0;
  for (int i = 0; i < B->ndim; ++i) {
    if (B->periodic[i] && B->grid_n[i] < 2) return 0;
    if (!B->periodic[i] && (B->grid_n[i] < 2 || !(B->hi[i] > B->lo[i]))) return 0;
  }
  return 1;
}

int32_t orc_grid_nodes(const orc_bias* B, int64_t nh, const double* centers, const double* heights,
                       int64_t n_nodes, const int64_t* node_ids, double* out) {
  if (!grid_ok(B) || nh < 0 || n_nodes < 0) return ORC_E_INVAL;
  const int d = B->ndim;
  const int nm = 1 << d;
  int64_t total = 1;
  for (int i = 0; i < d; ++i) total *= B->grid_n[i];
  for (int64_t t = 0; t < n_nodes; ++t)
    if (node_ids[t] < 0 || node_ids[t] >= total) return ORC_E_INDEX;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < n_nodes; ++t) {
    int64_t rem = node_ids[t];
    double x[3];
    for (int i = 0; i < d; ++i) {
      int64_t j = rem % B->grid_n[i];
      rem /= B->grid_n[i];
      x[i] = orc_grid_coord(B, i, j);
    }
    nsum acc[8];
    for (int m = 0; m < nm; ++m) { acc[m].s = 0; acc[m].c = 0; }
    for (int64_t k = 0; k < nh; ++k) {
      double val[3], der[3];
      for (int i = 0; i < d; ++i) {
        double c = centers[(int64_t)i * nh + k];
        if (B->quantize) c = orc_snap(B, i, c);
        double delta = axis_delta(B, i, x[i], c);
        orc_kernel_1d(B->kernel, B->width[i], B->p, delta, &val[i], &der[i]);
      }
      for (int m = 0; m < nm; ++m) {
        double term = heights[k];
        for (int i = 0; i < d; ++i) term *= ((m >> i) & 1) ? der[i] : val[i];
        nsum_add(&acc[m], term);
      }
    }
    for (int m = 0; m < nm; ++m) out[t * nm + m] = nsum_get(&acc[m]);
  }
  return ORC_OK;
}

/* Cubic Hermite basis on t in [0,1]: index [c][m] with c the cell end (0 or 1)
 * and m = 0 for the value, 1 for the derivative datum. */
static void hermite_basis(double t, double phi[2][2], double dphi[2][2]) {
  double t2 = t * t, t3 = t2 * t;
  phi[0][0] = 2 * t3 - 3 * t2 + 1;      /* h00 */
  phi[0][1] = t3 - 2 * t2 + t;          /* h10 */
  phi[1][0] = -2 * t3 + 3 * t2;         /* h01 */
  phi[1][1] = t3 - t2;                  /* h11 */
  dphi[0][0] = 6 * t2 - 6 * t;
  dphi[0][1] = 3 * t2 - 4 * t + 1;
  dphi[1][0] = -6 * t2 + 6 * t;
  dphi[1][1] = 3 * t2 - 2 * t;
}

int32_t orc_grid_eval(const orc_bias* B, const double* H, int64_t nq, const double* q,
                      double* h, double* dh, int64_t* n_clamped) {
  if (!grid_ok(B) || nq < 0) return ORC_E_INVAL;
  const int d = B->ndim;
  const int nm = 1 << d;
  int64_t clamped = 0;
  for (int64_t jq = 0; jq < nq; ++jq) {
    if (B->quantize) {
      /* nearest-node look-up: h and h'_i of eq. btraj-grad at xi* */
      int64_t node = 0, stride = 1;
      int was_out = 0;
      for (int i = 0; i < d; ++i) {
        double s = q[(int64_t)i * nq + jq];
        if (!B->periodic[i] && !(s >= B->lo[i] && s <= B->hi[i])) was_out = 1;
        node += orc_snap_index(B, i, s) * stride;
        stride *= (int64_t)B->grid_n[i];
      }
      clamped += was_out;
      h[jq] = H[node * nm];
      for (int k = 0; k < d; ++k) dh[(int64_t)k * nq + jq] = H[node * nm + (1 << k)];
      continue;
    }
    int64_t j0[3], j1[3];
    double dx[3], phi[3][2][2], dphi[3][2][2];
    int was_clamped = 0;
    for (int i = 0; i < d; ++i) {
      double s = q[(int64_t)i * nq + jq];
      int64_t n = B->grid_n[i];
      double t;
      if (B->periodic[i]) {
        dx[i] = (B->hi[i] - B->lo[i]) / (double)n;
        double u = (s - B->lo[i]) / dx[i];
        double fj = floor(u);
        t = u - fj;
        int64_t j = (int64_t)fj % n;
        if (j < 0) j += n;
        j0[i] = j;
        j1[i] = (j + 1) % n;
      } else {
        dx[i] = (B->hi[i] - B->lo[i]) / (double)(n - 1);
        if (s < B->lo[i]) { s = B->lo[i]; was_clamped = 1; }
        if (s > B->hi[i]) { s = B->hi[i]; was_clamped = 1; }
        double u = (s - B->lo[i]) / dx[i];
        int64_t j = (int64_t)floor(u);
        if (j > n - 2) j = n - 2;
        if (j < 0) j = 0;
        t = u - (double)j;
        j0[i] = j;
        j1[i] = j + 1;
      }
      hermite_basis(t, phi[i], dphi[i]);
    }
    clamped += was_clamped;
    double val = 0.0, grad[3] = {0.0, 0.0, 0.0};
    for (int corner = 0; corner < (1 << d); ++corner) {
      int64_t node = 0, stride = 1;
      for (int i = 0; i < d; ++i) {
        node += (((corner >> i) & 1) ? j1[i] : j0[i]) * stride;
        stride *= B->grid_n[i];
      }
      for (int m = 0; m < nm; ++m) {
        double Hv = H[node * nm + m];
        double w = 1.0;
        for (int i = 0; i < d; ++i) {
          int c = (corner >> i) & 1, mi = (m >> i) & 1;
          w *= phi[i][c][mi] * (mi ? dx[i] : 1.0);
        }
        val += w * Hv;
        for (int k = 0; k < d; ++k) {
          double g = 1.0;
          for (int i = 0; i < d; ++i) {
            int c = (corner >> i) & 1, mi = (m >> i) & 1;
            double scale = mi ? dx[i] : 1.0;
            g *= (i == k) ? dphi[i][c][mi] * scale / dx[i] : phi[i][c][mi] * scale;
          }
          grad[k] += g * Hv;
        }
      }
    }
    h[jq] = val;
    for (int k = 0; k < d; ++k) dh[(int64_t)k * nq + jq] = grad[k];
  }
  if (n_clamped) *n_clamped = clamped;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Collective variables                                                      */
/* ------------------------------------------------------------------------ */

/* Distance between the centres of mass of two groups,
 * R_G = sum_j m_j x_j / sum_j m_j, d = |R_A - R_B|. Gradient:
 * +(m_j/M_A) u for j in A and -(m_j/M_B) u for j in B, u = (R_A - R_B)/d.
 * Below d = 1e-12 nm the gradient is set to zero (the direction is undefined). */
int32_t orc_com_distance(int64_t na, const double* xa, const double* ma,
                         int64_t nb, const double* xb, const double* mb,
                         double* d, double* grad_a, double* grad_b) {
  double RA[3] = {0, 0, 0}, RB[3] = {0, 0, 0}, MA = 0, MB = 0;
  for (int64_t j = 0; j < na; ++j) {
    MA += ma[j];
    for (int c = 0; c < 3; ++c) RA[c] += ma[j] * xa[3 * j + c];
  }
  for (int64_t j = 0; j < nb; ++j) {
    MB += mb[j];
    for (int c = 0; c < 3; ++c) RB[c] += mb[j] * xb[3 * j + c];
  }
  if (!(MA > 0.0) || !(MB > 0.0)) return ORC_E_INVAL;
  double r[3];
  for (int c = 0; c < 3; ++c) r[c] = RA[c] / MA - RB[c] / MB;
  double dist = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  *d = dist;
  double u[3] = {0, 0, 0};
  if (dist >= 1e-12)
    for (int c = 0; c < 3; ++c) u[c] = r[c] / dist;
  for (int64_t j = 0; j < na; ++j)
    for (int c = 0; c < 3; ++c) grad_a[3 * j + c] = ma[j] / MA * u[c];
  for (int64_t j = 0; j < nb; ++j)
    for (int c = 0; c < 3; ++c) grad_b[3 * j + c] = -mb[j] / MB * u[c];
  return ORC_OK;
}

static void cross(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Dihedral angle of atoms 1-2-3-4 (IUPAC sign): with b1 = x2-x1, b2 = x3-x2,
 * b3 = x4-x3, n1 = b1 x b2, n2 = b2 x b3,
 * phi = atan2(|b2| b1.n2, n1.n2) in (-pi, pi].
 * Gradient (Blondel & Karplus, J. Comput. Chem. 17:1132, 1996, rewritten in
 * the b vectors):
 *   dphi/dx1 = -|b2|/|n1|^2 n1,          dphi/dx4 = +|b2|/|n2|^2 n2,
 *   dphi/dx2 = (|b2|/|n1|^2 + (b1.b2)/(|n1|^2 |b2|)) n1 + (b3.b2)/(|n2|^2 |b2|) n2,
 *   dphi/dx3 = -(b1.b2)/(|n1|^2 |b2|) n1 - (|b2|/|n2|^2 + (b3.b2)/(|n2|^2 |b2|)) n2.
 * If |n1|^2 or |n2|^2 falls below 1e-24 (collinear atoms) the gradient is zero. */
int32_t orc_torsion(const double* x4, double* phi, double* grad4) {
  double b1[3], b2[3], b3[3], n1[3], n2[3];
  for (int c = 0; c < 3; ++c) {
    b1[c] = x4[3 + c] - x4[0 + c];
    b2[c] = x4[6 + c] - x4[3 + c];
    b3[c] = x4[9 + c] - x4[6 + c];
  }
  cross(b1, b2, n1);
  cross(b2, b3, n2);
  double lb2 = sqrt(dot(b2, b2));
  *phi = atan2(lb2 * dot(b1, n2), dot(n1, n2));
  double nn1 = dot(n1, n1), nn2 = dot(n2, n2);
  for (int t = 0; t < 12; ++t) grad4[t] = 0.0;
  if (nn1 < 1e-24 || nn2 < 1e-24 || lb2 == 0.0) return ORC_OK;
  double r1 = dot(b1, b2), r3 = dot(b3, b2);
  for (int c = 0; c < 3; ++c) {
    grad4[0 + c] = -lb2 / nn1 * n1[c];
    grad4[9 + c] = lb2 / nn2 * n2[c];
    grad4[3 + c] = (lb2 / nn1 + r1 / (nn1 * lb2)) * n1[c] + r3 / (nn2 * lb2) * n2[c];
    grad4[6 + c] = -r1 / (nn1 * lb2) * n1[c] - (lb2 / nn2 + r3 / (nn2 * lb2)) * n2[c];
  }
  return ORC_OK;
}

/* Offset RMSD ("Definition of the RMSD"): RMSD = ((1/N) sum_i |x_i - x0_i|^2
 * + 0.01)^(1/2), no alignment, lower bound 0.1. Gradient (x_i - x0_i)/(N RMSD). */
int32_t orc_rmsd_off(int64_t n, const double* x, const double* x0, double* r, double* grad) {
  if (n < 1) return ORC_E_INVAL;
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      double dlt = x[3 * i + c] - x0[3 * i + c];
      acc += dlt * dlt;
    }
  double val = sqrt(acc / (double)n + 0.01);
  *r = val;
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) grad[3 * i + c] = (x[3 * i + c] - x0[3 * i + c]) / ((double)n * val);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Bias force for a batch of walkers.                                         */
/*                                                                            */
/* Layout: list_off[(cv*2 + slot)*(nw+1) + w] .. [+1] delimits the local atom */
/* indices of list (cv, slot) of walker w inside list_idx. COM_DIST: slot 0 = */
/* group A, slot 1 = group B. TORSION: slot 0 = the four atoms in order,      */
/* slot 1 empty. RMSD_OFF: slot 0 = the atoms (reference positions ref_* at   */
/* the same list positions), slot 1 empty. Groups must be strictly increasing */
/* (COM_DIST, RMSD_OFF); torsion atoms must be distinct.                      */
/* Forces: F_j += -sum_cv dV/ds_cv * ds_cv/dx_j (the chain rule), applied CV  */
/* by CV and list by list.                                                    */
/* ------------------------------------------------------------------------ */
static int check_lists(int32_t ncv, const int32_t* kind, int64_t nw, int64_t w,
                       const int64_t* list_off, const int32_t* list_idx, int32_t natoms,
                       const double* x, const double* y, const double* z, const double* mass,
                       int64_t base) {
  for (int a = 0; a < ncv; ++a) {
    for (int slot = 0; slot < 2; ++slot) {
      const int64_t* off = list_off + (int64_t)(a * 2 + slot) * (nw + 1);
      int64_t b = off[w], e = off[w + 1];
      if (b < 0 || e < b) return ORC_E_INVAL;
      int64_t len = e - b;
      if (kind[a] == ORC_COM_DIST && len < 1) return ORC_E_INVAL;
      if (kind[a] == ORC_TORSION && len != (slot == 0 ? 4 : 0)) return ORC_E_INVAL;
      if (kind[a] == ORC_RMSD_OFF && (slot == 0 ? len < 1 : len != 0)) return ORC_E_INVAL;
      for (int64_t t = b; t < e; ++t) {
        int32_t i = list_idx[t];
        if (i < 0 || i >= natoms) return ORC_E_INDEX;
        if (kind[a] != ORC_TORSION && t > b && list_idx[t - 1] >= i) return ORC_E_INDEX;
        if (kind[a] == ORC_TORSION)
          for (int64_t u = b; u < t; ++u)
            if (list_idx[u] == i) return ORC_E_INDEX;
        int64_t g = base + i;
        if (!isfinite(x[g]) || !isfinite(y[g]) || !isfinite(z[g]) || !isfinite(mass[g]))
          return ORC_E_NONFINITE;
      }
    }
  }
  return ORC_OK;
}

int32_t orc_bias_force(const orc_bias* B, int64_t nh, const double* centers, const double* heights,
                       int32_t use_grid, const double* H,
                       int32_t ncv, const int32_t* kind, int64_t nw,
                       const int64_t* list_off, const int32_t* list_idx,
                       const double* ref_x, const double* ref_y, const double* ref_z,
                       const int64_t* atom_base, const int32_t* n_atoms,
                       const double* x, const double* y, const double* z, const double* mass,
                       const int64_t* n_visible,
                       double* s, double* V, double* dVds,
                       double* fx, double* fy, double* fz, int32_t* status) {
  if (!bias_ok(B) || ncv != B->ndim || nw < 0) return ORC_E_INVAL;
  for (int a = 0; a < ncv; ++a) {
    if (kind[a] == ORC_TORSION && !B->periodic[a]) return ORC_E_INVAL;
    if (kind[a] != ORC_TORSION && B->periodic[a]) return ORC_E_INVAL;
  }
  if (use_grid && (!grid_ok(B) || !H)) return ORC_E_INVAL;
  for (int64_t w = 0; w < nw; ++w) {
    int64_t base = atom_base[w];
    int st = check_lists(ncv, kind, nw, w, list_off, list_idx, n_atoms[w], x, y, z, mass, base);
    if (st != ORC_OK) { status[w] = st; continue; }
    double sv[3];
    /* per-CV gradient with respect to the atoms of each list: [cv][slot][len*3] */
    double* grad[3][2] = {{NULL, NULL}, {NULL, NULL}, {NULL, NULL}};
    int err = ORC_OK;
    for (int a = 0; a < ncv && err == ORC_OK; ++a) {
      const int64_t* off0 = list_off + (int64_t)(a * 2 + 0) * (nw + 1);
      const int64_t* off1 = list_off + (int64_t)(a * 2 + 1) * (nw + 1);
      int64_t b0 = off0[w], n0 = off0[w + 1] - off0[w];
      int64_t b1 = off1[w], n1 = off1[w + 1] - off1[w];
      double* p0 = (double*)malloc(sizeof(double) * 3 * (n0 + 1));
      double* p1 = (double*)malloc(sizeof(double) * 3 * (n1 + 1));
      double* m0 = (double*)malloc(sizeof(double) * (n0 + 1));
      double* m1 = (double*)malloc(sizeof(double) * (n1 + 1));
      grad[a][0] = (double*)malloc(sizeof(double) * 3 * (n0 + 1));
      grad[a][1] = (double*)malloc(sizeof(double) * 3 * (n1 + 1));
      for (int64_t t = 0; t < n0; ++t) {
        int64_t g = base + list_idx[b0 + t];
        p0[3 * t] = x[g]; p0[3 * t + 1] = y[g]; p0[3 * t + 2] = z[g]; m0[t] = mass[g];
      }
      for (int64_t t = 0; t < n1; ++t) {
        int64_t g = base + list_idx[b1 + t];
        p1[3 * t] = x[g]; p1[3 * t + 1] = y[g]; p1[3 * t + 2] = z[g]; m1[t] = mass[g];
      }
      if (kind[a] == ORC_COM_DIST) {
        err = orc_com_distance(n0, p0, m0, n1, p1, m1, &sv[a], grad[a][0], grad[a][1]);
      } else if (kind[a] == ORC_TORSION) {
        err = orc_torsion(p0, &sv[a], grad[a][0]);
      } else {
        double* r0 = (double*)malloc(sizeof(double) * 3 * (n0 + 1));
        for (int64_t t = 0; t < n0; ++t) {
          r0[3 * t] = ref_x[b0 + t]; r0[3 * t + 1] = ref_y[b0 + t]; r0[3 * t + 2] = ref_z[b0 + t];
        }
        err = orc_rmsd_off(n0, p0, r0, &sv[a], grad[a][0]);
        free(r0);
      }
      free(p0); free(p1); free(m0); free(m1);
    }
    if (err == ORC_OK) {
      double hv, dh[3], Vv, dV[3];
      if (use_grid) {
        double qs[3];
        for (int a = 0; a < ncv; ++a) qs[a] = sv[a];
        orc_grid_eval(B, H, 1, qs, &hv, dh, NULL);
        /* orc_grid_eval with nq = 1 writes dh[k*1 + 0] = dh[k] */
      } else {
        int64_t nvis = n_visible ? n_visible[w] : nh;
        if (nvis < 0 || nvis > nh) nvis = nh;
        /* hills [0, nvis): centers keep their [ndim][nh] stride */
        double* cv = (double*)malloc(sizeof(double) * (size_t)(ncv * (nvis + 1)));
        for (int a = 0; a < ncv; ++a)
          for (int64_t k = 0; k < nvis; ++k) cv[(int64_t)a * nvis + k] = centers[(int64_t)a * nh + k];
        hill_sum_one(B, nvis, cv, heights, sv, &hv, dh, NULL, NULL);
        free(cv);
      }
      transform_one(B, hv, dh, &Vv, dV, NULL);
      for (int a = 0; a < ncv; ++a) {
        s[(int64_t)a * nw + w] = sv[a];
        dVds[(int64_t)a * nw + w] = dV[a];
      }
      V[w] = Vv;
      for (int a = 0; a < ncv; ++a) {
        for (int slot = 0; slot < 2; ++slot) {
          const int64_t* off = list_off + (int64_t)(a * 2 + slot) * (nw + 1);
          for (int64_t t = off[w]; t < off[w + 1]; ++t) {
            int64_t g = base + list_idx[t];
            int64_t r = t - off[w];
            fx[g] += -dV[a] * grad[a][slot][3 * r + 0];
            fy[g] += -dV[a] * grad[a][slot][3 * r + 1];
            fz[g] += -dV[a] * grad[a][slot][3 * r + 2];
          }
        }
      }
    }
    for (int a = 0; a < ncv; ++a) { free(grad[a][0]); free(grad[a][1]); }
    status[w] = err;
  }
  return ORC_OK;
}

/* FP64 CPU oracle for the adaptive-biasing-potential bias-force path.
 *
 * TEST INFRASTRUCTURE ONLY. This library exists so that tests, the smoke
 * check and the benchmark's CPU-baseline leg can check the GPU library
 * against a plain, slow, obviously correct implementation of the paper's
 * definitions. The GPU library never includes, links or calls it; the two
 * share no code.
 *
 * Paper: Dickson, de Waal, Ramjan, Xu, Rothbart, "A fast, open source
 * implementation of adaptive biasing potentials uncovers a ligand design
 * strategy for the chromatin regulator BRD4", arXiv:1609.09833.
 * Equation names refer to its Supplemental Material ("Streamlined bias
 * potential updates", "Convergence with S_a^p", "Definition of the RMSD").
 */
#ifndef ABP_ORACLE_H
#define ABP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GAUSS = 0, ORC_COMPACT = 1 };
enum { ORC_PLAIN = 0, ORC_MABP = 1 };
enum { ORC_COM_DIST = 0, ORC_TORSION = 1, ORC_RMSD_OFF = 2 };
enum { ORC_OK = 0, ORC_E_INVAL = 1, ORC_E_INDEX = 5, ORC_E_NONFINITE = 6 };

typedef struct {
  int32_t ndim;          /* 1..3 */
  int32_t periodic[3];   /* 1: the axis is periodic with period hi-lo */
  double lo[3], hi[3];
  int32_t kernel;        /* ORC_GAUSS or ORC_COMPACT */
  double width[3];       /* Gaussian: sigma_i; compact: a_i */
  int32_t p;             /* compact kernel exponent, >= 1 */
  int32_t transform;     /* ORC_PLAIN or ORC_MABP */
  double kT, b, c;       /* mABP parameters (eq. apfm) */
  int32_t grid_n[3];     /* grid nodes per axis */
  int32_t quantize;      /* 1: hills and evaluation points are moved to their nearest grid
                            node (the nearest-grid-point approximation that precedes
                            eq. update), and the grid is read at that node */
} orc_bias;

/* Minimum-image displacement on a periodic axis. */
double orc_wrap(double delta, double period);

/* One-dimensional kernel value and its derivative with respect to the
 * evaluation point (delta = s - center). */
void orc_kernel_1d(int32_t kernel, double width, int32_t p, double delta,
                   double* value, double* deriv);

/* Direct sum over hills [0, nh): h(s), dh/ds_i, and the condition sums
 * A0 = sum |w K|, A_i = sum |w dK/ds_i|. Arrays are [ndim][n] row-major. */
int32_t orc_hill_sum(const orc_bias* B, int64_t nh, const double* centers, const double* heights,
                     int64_t nq, const double* q, double* h, double* dh, double* A0, double* A);

/* Bias transform (eq. apfm / eq. btraj-grad): V, dV/ds and slope dV/dh. */
int32_t orc_transform(const orc_bias* B, int64_t nq, const double* h, const double* dh,
                      double* V, double* dV, double* slope);

/* Nearest grid node of x on an axis: index floor((x - lo)/dx + 1/2), taken
 * mod n on a periodic axis and clamped to [0, n-1] otherwise (dx the node
 * spacing); orc_snap returns that node's coordinate lo + j dx. */
int64_t orc_snap_index(const orc_bias* B, int32_t axis, double x);
double orc_snap(const orc_bias* B, int32_t axis, double x);

/* Grid node coordinate j on axis i. */
double orc_grid_coord(const orc_bias* B, int32_t axis, int64_t j);

/* Node arrays for the listed nodes: out[n][2^ndim], entry m holds the sum over
 * hills of w * prod_i (bit i of m ? dK_i : K_i) at the node. Node ids are
 * linear, axis 0 fastest. */
int32_t orc_grid_nodes(const orc_bias* B, int64_t nh, const double* centers, const double* heights,
                       int64_t n_nodes, const int64_t* node_ids, double* out);

/* Tensor-product cubic Hermite interpolation of h and its analytic gradient
 * from node arrays H[nodes][2^ndim]. Out-of-range queries on non-periodic axes
 * are clamped to the grid; their number is returned in *n_clamped. In the
 * quantised mode h and dh are the value and first-derivative arrays at the
 * query's nearest node instead. */
int32_t orc_grid_eval(const orc_bias* B, const double* H, int64_t nq, const double* q,
                      double* h, double* dh, int64_t* n_clamped);

/* Collective variables and their gradients. Positions are xyz[3*n] (atom-major). */
int32_t orc_com_distance(int64_t na, const double* xa, const double* ma,
                         int64_t nb, const double* xb, const double* mb,
                         double* d, double* grad_a, double* grad_b);
int32_t orc_torsion(const double* x4, double* phi, double* grad4);
int32_t orc_rmsd_off(int64_t n, const double* x, const double* x0, double* r, double* grad);

/* Bias force for a batch of walkers; see the implementation for the layout.
 * Forces are accumulated (+=) into fx, fy, fz. status[w] receives ORC_OK or
 * an error code; outputs of failed walkers are left untouched. */
int32_t orc_bias_force(const orc_bias* B, int64_t nh, const double* centers, const double* heights,
                       int32_t use_grid, const double* H,
                       int32_t ncv, const int32_t* kind, int64_t nw,
                       const int64_t* list_off, const int32_t* list_idx,
                       const double* ref_x, const double* ref_y, const double* ref_z,
                       const int64_t* atom_base, const int32_t* n_atoms,
                       const double* x, const double* y, const double* z, const double* mass,
                       const int64_t* n_visible,
                       double* s, double* V, double* dVds,
                       double* fx, double* fy, double* fz, int32_t* status);

#ifdef __cplusplus
}
#endif
#endif

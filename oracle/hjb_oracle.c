/*
 * hjb_oracle.c -- plain, slow, CPU FP64 oracle for the patchy semi-Lagrangian
 * scheme for the minimum-time HJB equation (Cacace, Cristiani, Falcone,
 * Picarelli, "A Patchy Dynamic Programming Scheme for a Class of
 * Hamilton-Jacobi-Bellman Equations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * Every floating-point expression below is written as separate IEEE binary64
 * multiplies and adds; with contraction off the compiler must not fuse them.
 *
 * What is computed (paper sections in brackets):
 *   - the SL fixed-point operator F of Section 2.1 (eq. SLscheme) in the
 *     Kruzkov variable v = 1 - exp(-T):
 *         [F(v)]_p = min_k beta * I[v](p + s (c_p a_k + w_p)) + (1 - beta)
 *     on active non-target nodes, 0 on target nodes;
 *   - value iteration v^{n+1} = min(v^n, F(v^n)) from v^0 = 0 on the target,
 *     1 elsewhere (eq. iterativeSLscheme), Jacobi order, until no node changes
 *     (or the sup-norm change is below tol);
 *   - Patchy Algorithm (Section 3): Step 1 coarse solve, Step 2 prolongation
 *     and discrete feedback (eq. feedbackcontrol), Step 3.1 colour transport
 *     with frozen feedback (eq. HJBridotta_discreta) and labels, Step 3.2
 *     independent per-patch iteration, Step 4 merge.
 *
 * Readings where the paper leaves the details open (all documented with the
 * design notes of the repository):
 *   - index-space foot point: displacement d = s * (c a + w) per axis,
 *     cell q = floor(d), local coordinate t = d - q;
 *   - "linear interpolation in R^d" is the tensor product of 1D linear
 *     interpolations in weights form, nested x, then y, then z:
 *         r = (1 - t) * lo + t * hi;
 *   - grid boundary: every box node is an unknown; corners outside the box
 *     take the ghost value (1 for v: state constraint; 0 for the colours);
 *   - patch boundary (state constraint, Section 3 "Details on boundary
 *     conditions"): in patch j, non-target nodes with another label are
 *     ghosts with value 1; all target nodes are 0 in every patch;
 *   - feedback: the first control (ascending k) attaining the minimum of the
 *     scheme's right-hand side beta_k I[U^(0)] + 1 - beta_k; when beta does
 *     not depend on the control this is the minimum of the raw I (compared
 *     before the affine Kruzkov map, which could round distinct I to equal
 *     values); target nodes carry no feedback (255);
 *   - colours: target nodes are fixed (1 on their own part, 0 elsewhere),
 *     non-target nodes start at 0 and rise as phi <- max(phi, Q(beta I[phi]))
 *     until nothing changes.  The factor beta = exp(-h) is the scheme's own
 *     per-step factor in the Kruzkov variable: a colour is the share of
 *     exp(-T) that part j carries along the frozen feedback, and the colour
 *     map is a beta-contraction (without it, near-closed loops of the frozen
 *     feedback -- rotating drifts produce them -- make the iteration
 *     contract arbitrarily slowly).  Q rounds down to a multiple of 2^-24:
 *     the paper allows a very rough stopping rule here since only the
 *     projection of the colours is used, and on this lattice increments
 *     below 2^-24 are not pursued while the map stays monotone (the stop
 *     does not depend on the order of the updates).  The label is the part
 *     with the largest colour, lowest part index on ties; pieces of a patch
 *     that hold no node of its target part (axis neighbours) are uncoloured;
 *     uncoloured nodes then take the smallest label among their nearest
 *     labelled nodes (Remark 3.1: uncovered nodes get the colour of their
 *     neighbours), so -1 remains only where no node is labelled at all;
 *   - merge: target 0, label -1 gives 1, else the value of patch label.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Colours below this floor are set to zero in the unrounded discounted
 * transport (ORC_TRACE_DISCOUNTED). */
#define ORC_COLOUR_FLOOR 1e-9
/* 2^24: the colour lattice of the labels' transport (ORC_TRACE_LATTICE) has
 * spacing 2^-24, the reading of the rough stopping rule of Step 3.1
 * (colours matter only through their final projection). */
#define ORC_COLOUR_LATTICE 16777216.0

/* pi to double precision (C99 has no M_PI) */
#define ORC_PI 3.14159265358979323846

/* target_part value of a node inside an obstacle (Section 4.5): a state
 * constraint inside the box -- never updated, read as the ghost value (1 for
 * v and U^(0), 0 for colours), label -2. */
#define ORC_OBSTACLE (-2)

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOCONV 4
#define ORC_ENOMEM 3

typedef struct {
  int32_t dim;
  int32_t n[3];
  double step[3];
  double beta;
  double omb;
  int32_t n_controls;
  const double *controls;      /* [Nc][dim] */
  const double *speed;         /* [N] */
  const double *drift;         /* [N][dim] or NULL */
  const int16_t *target_part;  /* [N], -1 = not target */
  int32_t n_parts;
  /* Variable step of Section 2.1 (h_i such that the foot point lies one
   * cell away): per-node beta_i = exp(-h_i), 1 - beta_i formed in FP64; or
   * NULL for the scalar beta. */
  const double *beta_node;
  /* Tabulated dynamics (any f, with the step rule of Section 2.1 per node
   * and control), control-major: foot[(k N + q) dim + d] is the foot-point
   * displacement in cells, beta_pk[k N + q] the factor exp(-h_{q,k});
   * either may be NULL (displacement s (c a + w); beta per node or
   * scalar). */
  const double *foot;
  const double *beta_pk;
} orc_problem;

/* Active-set description: patch < 0 means "every box node is active"
 * (global solve); otherwise a node is active iff it is a target node or its
 * label equals patch. */
typedef struct {
  const int16_t *labels;
  int patch;
  /* Control restriction of add-on AO3 (Section "Patchy method's add-ons"):
   * when allow != NULL, node q uses control k only if
   * allow[fb[q] * n_controls + k] is 1 (fb = the Step 2 feedback). */
  const uint8_t *fb;
  const uint8_t *allow;
  /* Dirichlet patch boundary data of eq. dbc (Section 4.4 and the add-ons
   * section): when u0 != NULL, a box node outside the active set reads
   * u0[q] instead of the ghost value 1. */
  const double *u0;
  /* Add-on AO1: the iteration is v <- F(v) from a given start (no min with
   * the old value), for starts that are not above the fixed point. */
  int plain;
} orc_active;

static long long orc_N(const orc_problem *P) {
  return (long long)P->n[0] * P->n[1] * P->n[2];
}

static int orc_check(const orc_problem *P) {
  if (!P || (P->dim != 2 && P->dim != 3)) return ORC_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (P->n[d] < 1) return ORC_EINVAL;
  if (P->n[0] < 2 || P->n[1] < 2 || (P->dim == 3 && P->n[2] < 2)) return ORC_EINVAL;
  if (P->dim == 2 && P->n[2] != 1) return ORC_EINVAL;
  if (P->n_controls < 1 || !P->controls || !P->speed || !P->target_part) return ORC_EINVAL;
  return ORC_OK;
}

/* Value of a corner node: stored value if inside the box and active, else
 * the ghost value (or, inside the box, the Dirichlet data u0 of eq. dbc). */
static double orc_corner(const orc_problem *P, const double *v, const orc_active *A,
                         long long x, long long y, long long z, double ghost) {
  if (x < 0 || y < 0 || z < 0 || x >= P->n[0] || y >= P->n[1] || z >= P->n[2]) return ghost;
  long long q = x + (long long)P->n[0] * (y + (long long)P->n[1] * z);
  if (P->target_part[q] == ORC_OBSTACLE) return ghost;
  if (A) {
    int tp = P->target_part[q];
    if (tp < 0 && A->patch >= 0 && A->labels[q] != A->patch) return A->u0 ? A->u0[q] : ghost;
  }
  return v[q];
}

/* 1D linear interpolation in weights form. */
static double orc_lin(double t, double lo, double hi) {
  double omt = 1.0 - t;
  double a = omt * lo;
  double b = t * hi;
  return a + b;
}

/* Foot-point displacement of node q under control k, in cells, per axis. */
static void orc_displacement(const orc_problem *P, long long q, int k, double disp[3]) {
  double c = P->speed[q];
  for (int d = 0; d < 3; ++d) disp[d] = 0.0;
  if (P->foot) {
    for (int d = 0; d < P->dim; ++d)
      disp[d] = P->foot[((long long)k * orc_N(P) + q) * P->dim + d];
    return;
  }
  for (int d = 0; d < P->dim; ++d) {
    double g = c * P->controls[(long long)k * P->dim + d];
    if (P->drift) g = g + P->drift[q * P->dim + d];
    disp[d] = P->step[d] * g;
  }
}

/* I[v](p + disp): interpolated value at the foot point. */
static double orc_interp(const orc_problem *P, const double *v, const orc_active *A,
                         long long px, long long py, long long pz, const double disp[3],
                         double ghost) {
  double fl[3], t[3];
  long long c0[3];
  for (int d = 0; d < 3; ++d) {
    fl[d] = floor(disp[d]);
    t[d] = disp[d] - fl[d];
    c0[d] = (long long)fl[d];
  }
  long long x0 = px + c0[0], y0 = py + c0[1];
  if (P->dim == 2) {
    double v00 = orc_corner(P, v, A, x0, y0, 0, ghost);
    double v10 = orc_corner(P, v, A, x0 + 1, y0, 0, ghost);
    double v01 = orc_corner(P, v, A, x0, y0 + 1, 0, ghost);
    double v11 = orc_corner(P, v, A, x0 + 1, y0 + 1, 0, ghost);
    double r0 = orc_lin(t[0], v00, v10);
    double r1 = orc_lin(t[0], v01, v11);
    return orc_lin(t[1], r0, r1);
  }
  long long z0 = pz + c0[2];
  double rz[2];
  for (int ez = 0; ez < 2; ++ez) {
    double v00 = orc_corner(P, v, A, x0, y0, z0 + ez, ghost);
    double v10 = orc_corner(P, v, A, x0 + 1, y0, z0 + ez, ghost);
    double v01 = orc_corner(P, v, A, x0, y0 + 1, z0 + ez, ghost);
    double v11 = orc_corner(P, v, A, x0 + 1, y0 + 1, z0 + ez, ghost);
    double r0 = orc_lin(t[0], v00, v10);
    double r1 = orc_lin(t[0], v01, v11);
    rz[ez] = orc_lin(t[1], r0, r1);
  }
  return orc_lin(t[2], rz[0], rz[1]);
}

/* [F(v)]_q for a non-target active node q (Section 2.1, eq. SLscheme in the
 * Kruzkov variable): min over the discrete controls of beta*I + (1-beta). */
static double orc_F_node(const orc_problem *P, const double *v, const orc_active *A, long long q,
                         long long px, long long py, long long pz) {
  double best = INFINITY;
  const uint8_t *row = (A && A->allow) ? A->allow + (long long)A->fb[q] * P->n_controls : NULL;
  for (int k = 0; k < P->n_controls; ++k) {
    if (row && !row[k]) continue;
    double disp[3];
    orc_displacement(P, q, k, disp);
    double I = orc_interp(P, v, A, px, py, pz, disp, 1.0);
    double b = P->beta_pk     ? P->beta_pk[(long long)k * orc_N(P) + q]
               : P->beta_node ? P->beta_node[q]
                              : P->beta;
    double omb = (P->beta_pk || P->beta_node) ? 1.0 - b : P->omb;
    double bI = b * I;
    double cand = bI + omb;
    if (cand < best) best = cand;
  }
  return best;
}

static int orc_is_updated(const orc_problem *P, const orc_active *A, long long q) {
  if (P->target_part[q] >= 0 || P->target_part[q] == ORC_OBSTACLE) return 0;
  if (A && A->patch >= 0 && A->labels[q] != A->patch) return 0;
  return 1;
}

/* Public: apply F once (no min with the old value) to every node, for tests
 * of the operator's invariants.  Inactive non-target nodes copy v_in. */
int orc_apply_F(const orc_problem *P, const int16_t *labels, int patch, const double *v_in,
                double *v_out) {
  if (orc_check(P)) return ORC_EINVAL;
  orc_active A = {labels, patch};
  const orc_active *Ap = (patch >= 0) ? &A : NULL;
  long long nx = P->n[0], ny = P->n[1], nz = P->n[2];
  for (long long z = 0; z < nz; ++z)
    for (long long y = 0; y < ny; ++y)
      for (long long x = 0; x < nx; ++x) {
        long long q = x + nx * (y + ny * z);
        if (P->target_part[q] >= 0) v_out[q] = 0.0;
        else if (!orc_is_updated(P, Ap, q)) v_out[q] = v_in[q];
        else v_out[q] = orc_F_node(P, v_in, Ap, q, x, y, z);
      }
  return ORC_OK;
}

/* Public: F at a list of nodes (raw operator, no min with the old value),
 * so that a large result can be checked node by node. */
int orc_F_at(const orc_problem *P, const int16_t *labels, int patch, const double *v,
             const long long *idx, long long count, double *out) {
  if (orc_check(P)) return ORC_EINVAL;
  orc_active A = {labels, patch};
  const orc_active *Ap = (patch >= 0) ? &A : NULL;
  long long nx = P->n[0], ny = P->n[1];
  for (long long i = 0; i < count; ++i) {
    long long q = idx[i];
    long long x = q % nx, y = (q / nx) % ny, z = q / (nx * ny);
    if (P->target_part[q] >= 0) out[i] = 0.0;
    else if (P->target_part[q] == ORC_OBSTACLE) out[i] = 1.0;
    else out[i] = orc_F_node(P, v, Ap, q, x, y, z);
  }
  return ORC_OK;
}

/* Jacobi value iteration over the node list `nodes` (all updated nodes of
 * the active set), in place on v which must hold the initial values.
 * Stops when the sup-norm change of a sweep is <= tol (tol == 0: exact fixed
 * point, no node changes). */
static int orc_jacobi(const orc_problem *P, const orc_active *A, const long long *nodes,
                      long long count, double tol, int max_sweeps, double *v, int *sweeps_out,
                      double *res_out) {
  long long N = orc_N(P);
  double *vn = (double *)malloc(sizeof(double) * (size_t)N);
  if (!vn) return ORC_ENOMEM;
  memcpy(vn, v, sizeof(double) * (size_t)N);
  long long nx = P->n[0], ny = P->n[1];
  int sweeps = 0;
  double res = 0.0;
  int rc = ORC_ENOCONV;
  while (sweeps < max_sweeps) {
    res = 0.0;
#pragma omp parallel for schedule(static) reduction(max : res)
    for (long long i = 0; i < count; ++i) {
      long long q = nodes[i];
      long long x = q % nx, y = (q / nx) % ny, z = q / (nx * ny);
      double f = orc_F_node(P, v, A, q, x, y, z);
      double nv = (A && A->plain) ? f : (f < v[q] ? f : v[q]);
      double dlt = fabs(v[q] - nv);
      if (dlt > res) res = dlt;
      vn[q] = nv;
    }
    for (long long i = 0; i < count; ++i) v[nodes[i]] = vn[nodes[i]];
    ++sweeps;
    if (res <= tol) { rc = ORC_OK; break; }
  }
  free(vn);
  if (sweeps_out) *sweeps_out = sweeps;
  if (res_out) *res_out = res;
  return rc;
}

/* Public: global solve (every box node active), eq. iterativeSLscheme.
 * Outputs v [N]; sweeps, final residual and node-control updates. */
int orc_solve_global(const orc_problem *P, double tol, int max_sweeps, double *v, int *sweeps,
                     double *residual, long long *updates) {
  if (orc_check(P)) return ORC_EINVAL;
  long long N = orc_N(P), cnt = 0;
  long long *nodes = (long long *)malloc(sizeof(long long) * (size_t)(N > 0 ? N : 1));
  if (!nodes) return ORC_ENOMEM;
  for (long long q = 0; q < N; ++q) {
    if (P->target_part[q] >= 0) v[q] = 0.0;
    else if (P->target_part[q] == ORC_OBSTACLE) v[q] = 1.0;
    else { v[q] = 1.0; nodes[cnt++] = q; }
  }
  int sw = 0;
  int rc = orc_jacobi(P, NULL, nodes, cnt, tol, max_sweeps, v, &sw, residual);
  if (sweeps) *sweeps = sw;
  if (updates) *updates = (long long)sw * cnt * P->n_controls;
  free(nodes);
  return rc;
}

/* Public: Step 2, prolongation of the coarse values onto the fine grid.
 * Fine node p_d maps to coarse index coordinate X = p_d (nc_d-1) / (nf_d-1);
 * Q = min(floor X, nc_d - 2), T = X - Q; nested linear interpolation.
 * Obstacle nodes of the fine grid get 1 (T = +inf). */
int orc_prolong(const orc_problem *C, const double *vc, const orc_problem *F, double *u0) {
  if (orc_check(C) || orc_check(F) || C->dim != F->dim) return ORC_EINVAL;
  int dim = F->dim;
  long long nf[3] = {F->n[0], F->n[1], F->n[2]};
  long long ncn[3] = {C->n[0], C->n[1], C->n[2]};
  for (long long z = 0; z < nf[2]; ++z)
    for (long long y = 0; y < nf[1]; ++y)
      for (long long x = 0; x < nf[0]; ++x) {
        long long p[3] = {x, y, z};
        long long Q[3] = {0, 0, 0};
        double T[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < dim; ++d) {
          double X = (double)(p[d] * (ncn[d] - 1)) / (double)(nf[d] - 1);
          double fq = floor(X);
          if (fq > (double)(ncn[d] - 2)) fq = (double)(ncn[d] - 2);
          Q[d] = (long long)fq;
          T[d] = X - fq;
        }
        double val;
#define CV(a, b, c) vc[(Q[0] + (a)) + ncn[0] * ((Q[1] + (b)) + ncn[1] * (Q[2] + (c)))]
        if (dim == 2) {
          double r0 = orc_lin(T[0], CV(0, 0, 0), CV(1, 0, 0));
          double r1 = orc_lin(T[0], CV(0, 1, 0), CV(1, 1, 0));
          val = orc_lin(T[1], r0, r1);
        } else {
          double rz[2];
          for (int ez = 0; ez < 2; ++ez) {
            double r0 = orc_lin(T[0], CV(0, 0, ez), CV(1, 0, ez));
            double r1 = orc_lin(T[0], CV(0, 1, ez), CV(1, 1, ez));
            rz[ez] = orc_lin(T[1], r0, r1);
          }
          val = orc_lin(T[2], rz[0], rz[1]);
        }
#undef CV
        long long qf = x + nf[0] * (y + nf[1] * z);
        u0[qf] = F->target_part[qf] == ORC_OBSTACLE ? 1.0 : val;
      }
  return ORC_OK;
}

/* The quantity the feedback minimises over k at node q, given the
 * interpolated Step 2 value I at the foot point of control k.  Eq.
 * feedbackcontrol minimises I[U^(0)](foot) + h_{i,a} in the time variable,
 * i.e. the scheme's own right-hand side; in the Kruzkov variable that is
 * beta_k I + (1 - beta_k).  When beta does not depend on the control (one
 * beta, or one per node) that map is increasing in I, so I itself is
 * compared (the affine map could round distinct I to equal values); with
 * per-control factors (the step rule on tabulated dynamics) the step must
 * enter, or slow controls win on the value of their foot alone. */
static double orc_feedback_key(const orc_problem *F, long long q, int k, double I) {
  if (!F->beta_pk) return I;
  double b = F->beta_pk[(long long)k * orc_N(F) + q];
  double bI = b * I;
  return bI + (1.0 - b);
}

/* Public: Step 2, discrete feedback (eq. feedbackcontrol): for every
 * non-target fine node the first k minimising the scheme's right-hand side
 * at I[U^(0)](p + s(c a_k + w)) (orc_feedback_key), ghost 1 outside the
 * box, every node active.  Target nodes get 255. */
int orc_feedback(const orc_problem *F, const double *u0, uint8_t *fb) {
  if (orc_check(F) || F->n_controls > 255) return ORC_EINVAL;
  long long nx = F->n[0], ny = F->n[1], nz = F->n[2];
#pragma omp parallel for schedule(static) collapse(2)
  for (long long z = 0; z < nz; ++z)
    for (long long y = 0; y < ny; ++y)
      for (long long x = 0; x < nx; ++x) {
        long long q = x + nx * (y + ny * z);
        if (F->target_part[q] >= 0 || F->target_part[q] == ORC_OBSTACLE) { fb[q] = 255; continue; }
        double best = INFINITY;
        int bk = 0;
        for (int k = 0; k < F->n_controls; ++k) {
          double disp[3];
          orc_displacement(F, q, k, disp);
          double I = orc_feedback_key(F, q, k, orc_interp(F, u0, NULL, x, y, z, disp, 1.0));
          if (I < best) { best = I; bk = k; }
        }
        fb[q] = (uint8_t)bk;
      }
  return ORC_OK;
}

/* Public: the discrete feedback at a list of nodes only (as orc_feedback),
 * so that a large grid can be checked node by node. */
int orc_feedback_at(const orc_problem *F, const double *u0, const long long *idx, long long count,
                    uint8_t *fb) {
  if (orc_check(F) || F->n_controls > 255) return ORC_EINVAL;
  long long nx = F->n[0], ny = F->n[1];
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < count; ++i) {
    long long q = idx[i];
    long long x = q % nx, y = (q / nx) % ny, z = q / (nx * ny);
    if (F->target_part[q] >= 0 || F->target_part[q] == ORC_OBSTACLE) { fb[i] = 255; continue; }
    double best = INFINITY;
    int bk = 0;
    for (int k = 0; k < F->n_controls; ++k) {
      double disp[3];
      orc_displacement(F, q, k, disp);
      double I = orc_feedback_key(F, q, k, orc_interp(F, u0, NULL, x, y, z, disp, 1.0));
      if (I < best) { best = I; bk = k; }
    }
    fb[i] = (uint8_t)bk;
  }
  return ORC_OK;
}

/* Colour transport modes of orc_trace_part_mode:
 *   ORC_TRACE_LATTICE     the reading used for the labels: the foot point
 *                         of the feedback control under the scheme's own
 *                         step h, the factor beta, and every new colour
 *                         rounded down to a multiple of 2^-24 (the "very
 *                         rough" stop of Step 3.1 made exact: increments
 *                         below the lattice spacing are not pursued, and
 *                         the rounded map is still monotone, so every fair
 *                         order of updates stops at the same colours);
 *   ORC_TRACE_DISCOUNTED  the same foot point and factor, colours below the
 *                         floor 1e-9 set to 0, otherwise unrounded;
 *   ORC_TRACE_PLAIN       the same foot point with no factor and no floor;
 *   ORC_TRACE_PAPER       eq. HJBridotta_discreta as printed: no factor, no
 *                         floor, and the step h_i with |h_i f(x_i, a*)| = k,
 *                         i.e. the foot point one cell away along f (grids
 *                         with equal steps on every axis only). */
#define ORC_TRACE_DISCOUNTED 0
#define ORC_TRACE_PLAIN 1
#define ORC_TRACE_PAPER 2
#define ORC_TRACE_LATTICE 3

/* Public: Step 3.1 for one part j -- colour transport with the frozen
 * feedback (eq. HJBridotta_discreta, in the reading `mode`), iterated
 * (Jacobi) from below to the exact fixed point.  phi [N] is output. */
int orc_trace_part_mode(const orc_problem *F, const uint8_t *fb, int part, int mode,
                        int max_sweeps, double *phi, int *sweeps_out) {
  if (orc_check(F) || mode < 0 || mode > 3) return ORC_EINVAL;
  if (mode == ORC_TRACE_PAPER)
    for (int d = 1; d < F->dim; ++d)
      if (F->step[d] != F->step[0]) return ORC_EINVAL;
  long long N = orc_N(F), nx = F->n[0], ny = F->n[1];
  long long cnt = 0;
  long long *nodes = (long long *)malloc(sizeof(long long) * (size_t)N);
  double *pn = (double *)malloc(sizeof(double) * (size_t)N);
  if (!nodes || !pn) { free(nodes); free(pn); return ORC_ENOMEM; }
  for (long long q = 0; q < N; ++q) {
    int tp = F->target_part[q];
    if (tp >= 0) phi[q] = (tp == part) ? 1.0 : 0.0;
    else if (tp == ORC_OBSTACLE) phi[q] = 0.0;
    else { phi[q] = 0.0; nodes[cnt++] = q; }
  }
  memcpy(pn, phi, sizeof(double) * (size_t)N);
  int sweeps = 0, rc = ORC_ENOCONV;
  while (sweeps < max_sweeps) {
    int changed = 0;
#pragma omp parallel for schedule(static) reduction(| : changed)
    for (long long i = 0; i < cnt; ++i) {
      long long q = nodes[i];
      long long x = q % nx, y = (q / nx) % ny, z = q / (nx * ny);
      double disp[3];
      orc_displacement(F, q, fb[q], disp);
      if (mode == ORC_TRACE_PAPER) {
        /* |h_i f| = k: the displacement in cells scaled to length 1; a node
         * where f vanishes does not move */
        double len2 = 0.0;
        for (int d = 0; d < F->dim; ++d) len2 = len2 + disp[d] * disp[d];
        double len = sqrt(len2);
        for (int d = 0; d < F->dim; ++d) disp[d] = len > 0.0 ? disp[d] / len : 0.0;
      }
      double I = orc_interp(F, phi, NULL, x, y, z, disp, 0.0);
      double bI = I;
      if (mode == ORC_TRACE_DISCOUNTED || mode == ORC_TRACE_LATTICE) {
        double b = F->beta_pk     ? F->beta_pk[(long long)fb[q] * N + q]
                   : F->beta_node ? F->beta_node[q]
                                  : F->beta;
        bI = b * I;
        if (mode == ORC_TRACE_LATTICE) {
          /* scaling by a power of two is exact: floor to the lattice */
          bI = floor(bI * ORC_COLOUR_LATTICE) / ORC_COLOUR_LATTICE;
        } else if (bI < ORC_COLOUR_FLOOR) {
          bI = 0.0;
        }
      }
      double nv = bI > phi[q] ? bI : phi[q];
      if (nv != phi[q]) changed = 1;
      pn[q] = nv;
    }
    for (long long i = 0; i < cnt; ++i) phi[nodes[i]] = pn[nodes[i]];
    ++sweeps;
    if (!changed) { rc = ORC_OK; break; }
  }
  if (sweeps_out) *sweeps_out = sweeps;
  free(nodes);
  free(pn);
  return rc;
}

/* Public: Step 3.1 for one part j in the reading used for the labels. */
int orc_trace_part(const orc_problem *F, const uint8_t *fb, int part, int max_sweeps, double *phi,
                   int *sweeps_out) {
  return orc_trace_part_mode(F, fb, part, ORC_TRACE_LATTICE, max_sweeps, phi, sweeps_out);
}

/* Remark 3.1: nodes no colour reached take the colour of their neighbours.
 * Jacobi layers: an unlabelled node with labelled axis neighbours (4 in 2D,
 * 6 in 3D) takes the smallest of their labels; repeat until no node
 * changes.  The result is the lowest label among the nearest labelled nodes
 * (in steps along the axes), and a filled node joins a piece of its patch
 * through a face.
 * *filled (optional) receives the number of nodes that were unlabelled. */
int orc_fill_labels(const orc_problem *F, int16_t *labels, long long *filled) {
  long long N = orc_N(F), nx = F->n[0], ny = F->n[1], nz = F->n[2];
  int16_t *next = (int16_t *)malloc(sizeof(int16_t) * (size_t)N);
  if (!next) return ORC_ENOMEM;
  long long before = 0;
  for (long long q = 0; q < N; ++q) before += labels[q] == -1;
  int dz0 = nz > 1 ? -1 : 0, dz1 = nz > 1 ? 1 : 0;
  for (;;) {
    int changed = 0;
    memcpy(next, labels, sizeof(int16_t) * (size_t)N);
    for (long long q = 0; q < N; ++q) {
      if (labels[q] != -1) continue;  /* labelled, or an obstacle (-2) */
      long long x = q % nx, y = (q / nx) % ny, z = q / (nx * ny);
      int best = -1;
      for (int dz = dz0; dz <= dz1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (abs(dx) + abs(dy) + abs(dz) != 1) continue; /* axis neighbours */
            long long X = x + dx, Y = y + dy, Z = z + dz;
            if (X < 0 || Y < 0 || Z < 0 || X >= nx || Y >= ny || Z >= nz) continue;
            int L = labels[X + nx * (Y + ny * Z)];
            if (L >= 0 && (best < 0 || L < best)) best = L;
          }
      if (best >= 0) {
        next[q] = (int16_t)best;
        changed = 1;
      }
    }
    memcpy(labels, next, sizeof(int16_t) * (size_t)N);
    if (!changed) break;
  }
  free(next);
  if (filled) *filled = before;
  return ORC_OK;
}

/* Public: pieces of a patch cut off from its own target part (Section 3,
 * Remark 3.1 and the discussion of Fig. independence).  The argmax
 * projection can leave a piece of the nodes of label j that holds no target
 * node of part j: no characteristic of patch j runs from it to Omega_0^j, so
 * under the state constraint of Step 3.2 its values stay at or near 1
 * (T = +inf).  Pieces are connected through the axis neighbours (4 in 2D, 6
 * in 3D): nodes that touch only at a corner form a chain too thin for the
 * interpolation stencil of the scheme to carry values along it.  Such a
 * piece is treated like the nodes no colour reached: its labels become -1,
 * and orc_fill_labels gives them the colour of their neighbours.  Target
 * nodes carry their own part as label, so a piece is attached iff it
 * contains a target node.  Obstacle (-2) and unlabelled (-1) nodes separate
 * pieces.  *detached (optional) receives the number of relabelled nodes.
 * Plain breadth-first search over the grid. */
int orc_detach_fragments(const orc_problem *F, int16_t *labels, long long *detached) {
  long long N = orc_N(F), nx = F->n[0], ny = F->n[1], nz = F->n[2];
  long long *queue = (long long *)malloc(sizeof(long long) * (size_t)(N > 0 ? N : 1));
  uint8_t *seen = (uint8_t *)calloc((size_t)(N > 0 ? N : 1), 1);
  if (!queue || !seen) { free(queue); free(seen); return ORC_ENOMEM; }
  int dz0 = nz > 1 ? -1 : 0, dz1 = nz > 1 ? 1 : 0;
  long long cut = 0;
  for (long long s0 = 0; s0 < N; ++s0) {
    if (seen[s0] || labels[s0] < 0) continue;
    int L = labels[s0];
    long long head = 0, tail = 0;
    int attached = 0;
    queue[tail++] = s0;
    seen[s0] = 1;
    while (head < tail) {
      long long q = queue[head++];
      if (F->target_part[q] == L) attached = 1; /* a target node of part L */
      long long x = q % nx, y = (q / nx) % ny, z = q / (nx * ny);
      for (int dz = dz0; dz <= dz1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (abs(dx) + abs(dy) + abs(dz) != 1) continue; /* axis neighbours */
            long long X = x + dx, Y = y + dy, Z = z + dz;
            if (X < 0 || Y < 0 || Z < 0 || X >= nx || Y >= ny || Z >= nz) continue;
            long long r = X + nx * (Y + ny * Z);
            if (seen[r] || labels[r] != L) continue;
            seen[r] = 1;
            queue[tail++] = r;
          }
    }
    if (!attached) {
      /* the queue still lists the whole piece */
      for (long long i = 0; i < tail; ++i) labels[queue[i]] = -1;
      cut += tail;
    }
  }
  free(queue);
  free(seen);
  if (detached) *detached = cut;
  return ORC_OK;
}

/* Public: Step 3.1 for all parts, then the labels (projection/assembly,
 * eq. proiezionecolore with Remark 3.1): label = target part on target
 * nodes; elsewhere the part with the largest colour (lowest index on ties),
 * -1 where every colour is 0; pieces cut off from their own target part
 * become -1 as well (orc_detach_fragments), and every -1 node takes the
 * colour of its neighbours (orc_fill_labels).  phi_sum (optional) receives
 * sum_j phi^j; *unreached the nodes no colour reached, *detached the nodes
 * of cut-off pieces. */
int orc_labels(const orc_problem *F, const uint8_t *fb, int max_sweeps, int16_t *labels,
               double *phi_sum, int *max_trace_sweeps, long long *unreached,
               long long *detached) {
  if (orc_check(F) || F->n_parts < 1) return ORC_EINVAL;
  long long N = orc_N(F);
  double *phi = (double *)malloc(sizeof(double) * (size_t)N);
  double *best = (double *)malloc(sizeof(double) * (size_t)N);
  if (!phi || !best) { free(phi); free(best); return ORC_ENOMEM; }
  for (long long q = 0; q < N; ++q) {
    best[q] = 0.0;
    labels[q] = -1;
    if (phi_sum) phi_sum[q] = 0.0;
  }
  int mx = 0, rc = ORC_OK;
  for (int j = 0; j < F->n_parts; ++j) {
    int sw = 0;
    int r = orc_trace_part(F, fb, j, max_sweeps, phi, &sw);
    if (r != ORC_OK) rc = r;
    if (sw > mx) mx = sw;
    for (long long q = 0; q < N; ++q) {
      if (phi_sum) phi_sum[q] = phi_sum[q] + phi[q];
      if (phi[q] > best[q]) { best[q] = phi[q]; labels[q] = (int16_t)j; }
    }
  }
  for (long long q = 0; q < N; ++q) {
    if (F->target_part[q] >= 0) labels[q] = F->target_part[q];
    if (F->target_part[q] == ORC_OBSTACLE) labels[q] = ORC_OBSTACLE;
  }
  if (max_trace_sweeps) *max_trace_sweeps = mx;
  free(phi);
  free(best);
  if (unreached) {
    long long u = 0;
    for (long long q = 0; q < N; ++q) u += labels[q] == -1;
    *unreached = u;
  }
  if (rc == ORC_OK) rc = orc_detach_fragments(F, labels, detached);
  if (rc == ORC_OK) rc = orc_fill_labels(F, labels, NULL);
  return rc;
}

/* Public: exclusion of unreachable regions (Section 4.6): after Step 1, a
 * fine node off the target whose U^(0) is at least `theta` is excluded
 * from the rest of the computation, i.e. becomes an obstacle node:
 * tp_out = target_part with ORC_OBSTACLE there.  u0 is the raw
 * prolongation.  Returns the number of excluded nodes, or -1. */
long long orc_exclude(const orc_problem *F, const double *u0, double theta, int16_t *tp_out) {
  if (orc_check(F) || !(theta > 0.0)) return -1;
  long long N = orc_N(F), cnt = 0;
  for (long long q = 0; q < N; ++q) {
    int tp = F->target_part[q];
    if (tp == -1 && u0[q] >= theta) { tp_out[q] = ORC_OBSTACLE; ++cnt; }
    else tp_out[q] = (int16_t)tp;
  }
  return cnt;
}

/* Public: the control sets of add-on AO3 (Section "Patchy method's
 * add-ons"): allow[ks * Nc + k] = 1 iff a_k . a_ks >= cos(pi / r), for every
 * feedback control ks.  The dot product is summed over the axes in order,
 * FP64, no fused multiply-add.  The feedback control itself is always kept
 * (the cone is centred on it; this matters only for controls shorter than
 * cos(pi/r)).  r <= 1 keeps every control.  Returns the largest set size. */
int orc_cone_allowed(const orc_problem *P, double r, uint8_t *allow) {
  if (orc_check(P)) return -1;
  int nc = P->n_controls, dim = P->dim, lmax = 0;
  double cr = r > 1.0 ? cos(ORC_PI / r) : -INFINITY;
  for (int ks = 0; ks < nc; ++ks) {
    int cnt = 0;
    for (int k = 0; k < nc; ++k) {
      double dot = 0.0;
      for (int d = 0; d < dim; ++d) {
        double pr = P->controls[(long long)k * dim + d] * P->controls[(long long)ks * dim + d];
        dot = dot + pr;
      }
      int ok = (k == ks) || r <= 1.0 || dot >= cr;
      allow[(long long)ks * nc + k] = (uint8_t)ok;
      cnt += ok;
    }
    if (cnt > lmax) lmax = cnt;
  }
  return lmax;
}

/* Public: F at a list of nodes for the patch solve with the options of the
 * add-ons section (cones of AO3 around fb when cone_r > 1, Dirichlet data
 * u0 when given), so that a large result can be checked node by node. */
int orc_F_at_ex(const orc_problem *P, const int16_t *labels, int patch, const uint8_t *fb,
                double cone_r, const double *u0, const double *v, const long long *idx,
                long long count, double *out) {
  if (orc_check(P) || patch < 0) return ORC_EINVAL;
  uint8_t *allow = NULL;
  if (fb && cone_r > 1.0) {
    allow = (uint8_t *)malloc((size_t)P->n_controls * (size_t)P->n_controls);
    if (!allow) return ORC_ENOMEM;
    orc_cone_allowed(P, cone_r, allow);
  }
  orc_active A = {labels, patch, fb, allow, u0, 0};
  long long nx = P->n[0], ny = P->n[1];
  for (long long i = 0; i < count; ++i) {
    long long q = idx[i];
    long long x = q % nx, y = (q / nx) % ny, z = q / (nx * ny);
    if (P->target_part[q] >= 0) out[i] = 0.0;
    else out[i] = orc_F_node(P, v, &A, q, x, y, z);
  }
  free(allow);
  return ORC_OK;
}

/* Public: Step 3.2 + Step 4 -- independent value iteration in every patch,
 * then merge.  `only_patch` >= 0 solves that single patch (other nodes of v
 * are left at 1 / 0).  Patch boundary: state constraint (other patches'
 * nodes are ghosts of value 1) or, with u0 != NULL, the Dirichlet data of
 * eq. dbc (they hold u0).  With fb != NULL and cone_r > 1, each node keeps
 * only the controls of add-on AO3 around its feedback control fb[q]
 * (orc_cone_allowed); `updates` then counts the controls evaluated.  With
 * init != NULL (add-on AO1) the patch nodes start at init and iterate
 * v <- F(v) until no node moves by more than tol (> 0) in a sweep. */
int orc_solve_patches_ex(const orc_problem *F, const int16_t *labels, const uint8_t *fb,
                         double cone_r, const double *u0, const double *init, double tol,
                         int max_sweeps, int only_patch, double *v, int *sweeps_per_patch,
                         long long *updates) {
  if (orc_check(F) || F->n_parts < 1) return ORC_EINVAL;
  if (init && !(tol > 0.0)) return ORC_EINVAL;
  uint8_t *allow = NULL;
  long long *row_cnt = NULL;
  if (fb && cone_r > 1.0) {
    long long nc = F->n_controls;
    allow = (uint8_t *)malloc((size_t)(nc * nc));
    row_cnt = (long long *)calloc((size_t)nc, sizeof(long long));
    if (!allow || !row_cnt) { free(allow); free(row_cnt); return ORC_ENOMEM; }
    orc_cone_allowed(F, cone_r, allow);
    for (long long ks = 0; ks < nc; ++ks)
      for (long long k = 0; k < nc; ++k) row_cnt[ks] += allow[ks * nc + k];
    long long Nf = orc_N(F);
    for (long long q = 0; q < Nf; ++q)
      if (F->target_part[q] == -1 && labels[q] >= 0 && fb[q] >= nc) {
        free(allow); free(row_cnt); return ORC_EINVAL;
      }
  }
  long long N = orc_N(F);
  long long *cnt = (long long *)calloc((size_t)F->n_parts, sizeof(long long));
  long long *start = (long long *)calloc((size_t)F->n_parts + 1, sizeof(long long));
  long long *nodes = (long long *)malloc(sizeof(long long) * (size_t)(N > 0 ? N : 1));
  double *work = (double *)malloc(sizeof(double) * (size_t)N);
  if (!cnt || !start || !nodes || !work) {
    free(cnt); free(start); free(nodes); free(work); free(allow); free(row_cnt);
    return ORC_ENOMEM;
  }
  for (long long q = 0; q < N; ++q) {
    if (F->target_part[q] >= 0) { v[q] = 0.0; continue; }
    v[q] = 1.0;
    int L = labels[q];
    if (L >= F->n_parts) {
      free(cnt); free(start); free(nodes); free(work); free(allow); free(row_cnt);
      return ORC_EINVAL;
    }
    if (L >= 0) cnt[L]++;
  }
  for (int j = 0; j < F->n_parts; ++j) start[j + 1] = start[j] + cnt[j];
  for (int j = 0; j < F->n_parts; ++j) cnt[j] = 0;
  for (long long q = 0; q < N; ++q) {
    int L = labels[q];
    if (F->target_part[q] < 0 && L >= 0) nodes[start[L] + cnt[L]++] = q;
  }
  int rc = ORC_OK;
  long long upd = 0;
  for (int j = 0; j < F->n_parts; ++j) {
    if (sweeps_per_patch) sweeps_per_patch[j] = 0;
    if (only_patch >= 0 && j != only_patch) continue;
    /* Patch-local iterate: target 0, patch nodes 1; other nodes are ghosts
     * (never read as values, see orc_corner). */
    for (long long q = 0; q < N; ++q) work[q] = (F->target_part[q] >= 0) ? 0.0 : 1.0;
    if (init)
      for (long long i = start[j]; i < start[j] + cnt[j]; ++i) work[nodes[i]] = init[nodes[i]];
    orc_active A = {labels, j, fb, allow, u0, init != NULL};
    int sw = 0;
    int r = orc_jacobi(F, &A, nodes + start[j], cnt[j], tol, max_sweeps, work, &sw, NULL);
    if (r != ORC_OK) rc = r;
    if (sweeps_per_patch) sweeps_per_patch[j] = sw;
    long long per_sweep = cnt[j] * F->n_controls;
    if (allow) {
      per_sweep = 0;
      for (long long i = start[j]; i < start[j] + cnt[j]; ++i) per_sweep += row_cnt[fb[nodes[i]]];
    }
    upd += (long long)sw * per_sweep;
    for (long long i = start[j]; i < start[j] + cnt[j]; ++i) v[nodes[i]] = work[nodes[i]];
  }
  if (updates) *updates = upd;
  free(cnt); free(start); free(nodes); free(work); free(allow); free(row_cnt);
  return rc;
}

/* Public: Steps 3.2 + 4 of the basic algorithm (every control). */
int orc_solve_patches(const orc_problem *F, const int16_t *labels, double tol, int max_sweeps,
                      int only_patch, double *v, int *sweeps_per_patch, long long *updates) {
  return orc_solve_patches_ex(F, labels, NULL, 0.0, NULL, NULL, tol, max_sweeps, only_patch, v,
                              sweeps_per_patch, updates);
}

/* Public: number of threads the parallel loops use. */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

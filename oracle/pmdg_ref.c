/*
 * pmdg_ref.c -- plain FP64 CPU oracle for the coupled PMUT / DG-SEM acoustic
 * time step (arXiv 2603.06267).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant with the
 * HIP library: every number below is recomputed here from its definition.
 *
 * What it computes (paper sections cited per function):
 *   - GLL / Gauss-Legendre rules and the Lagrange derivative matrix (Sec. 3,
 *     Lagrangian basis, "reduced integration" of the mass form).
 *   - Two axis-aligned hexahedral bricks, each carrying a continuous Q_N
 *     space (Sec. 3, definition of V_a^{r_a}); the bricks meet on one
 *     non-conforming, mixed-order interface Gamma_I treated by symmetric
 *     interior penalty (Sec. 3, bilinear form a, eq. Wf_2, penalty gamma_F).
 *   - Interface integrals evaluated on quadrature points of the finer face,
 *     mapped back into the coarse element (Sec. 5).
 *   - PMUT coupling integrals f_i and g_m (Sec. 3.1, eqs. f_i and g_m) and the
 *     reduced modal ODE (Sec. 2, eq. pmut_problem).
 *   - Newmark beta=0, gamma=1/2 time stepping (Sec. 3.1, Algorithm 1), in the
 *     synchronised ordering (the ODE samples the predicted pressure at the new
 *     time level); the printed ordering is kept behind a switch for tests.
 *   - Trilinear hexahedra (Sec. 3: every element the image of the reference
 *     cube under a trilinear map X_K with positive Jacobian): node
 *     coordinates, lumped mass, element stiffness with the metric terms,
 *     PMUT face weights with the surface Jacobian, receivers located by a
 *     Newton inverse map; and the face matching of Sec. 5, Algorithm 3.
 *   - The smooth drive window g(t) (Sec. 6.1, eq. voltage).
 *   - First-order absorbing faces and the perfectly matched layer (Sec. 2,
 *     eq. full_problem: the damping alpha p_t + beta p, the auxiliary fields
 *     Phi and psi, the profile zeta_i and its constant).
 *
 * Written for clarity, not speed: element loops, explicit Lagrange products,
 * no blocking.  OpenMP is used only over element colours so that no two
 * threads ever add into the same node.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define RMAXN 9 /* orders 1..8 */
#define RMAXQ 10

/* ------------------------------------------------------------------ */
/* Quadrature and Lagrange basis                                       */
/* ------------------------------------------------------------------ */

/* Legendre P_n(x) and P_n'(x) by the three-term recurrence. */
static void legendre(int n, double x, double *P, double *dP) {
  double p0 = 1.0, p1 = x, dp0 = 0.0, dp1 = 1.0;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double dp2 = dp0 + (2.0 * k + 1.0) * p1; /* P'_{k+1} = P'_{k-1} + (2k+1) P_k */
    p0 = p1; p1 = p2; dp0 = dp1; dp1 = dp2;
  }
  *P = p1; *dP = dp1;
}

/* Gauss-Lobatto-Legendre nodes and weights on [-1,1], N+1 points:
 * x = +-1 and the roots of P_N'; w_i = 2 / (N (N+1) P_N(x_i)^2). */
int pmdg_ref_gll(int N, double *x, double *w) {
  if (N < 1 || N >= RMAXN) return -1;
  x[0] = -1.0; x[N] = 1.0;
  for (int j = 1; j < N; ++j) {
    double t = -cos(M_PI * j / N);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(N, t, &P, &dP);
      /* (1-t^2) P'' = 2 t P' - N(N+1) P */
      double d2P = (2.0 * t * dP - N * (N + 1.0) * P) / (1.0 - t * t);
      double dt = dP / d2P;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    x[j] = t;
  }
  for (int j = 0; j <= N; ++j) {
    double P, dP;
    legendre(N, x[j], &P, &dP);
    w[j] = 2.0 / (N * (N + 1.0) * P * P);
  }
  return 0;
}

/* Gauss-Legendre nodes and weights, n points: roots of P_n,
 * w = 2 / ((1 - x^2) P_n'(x)^2). */
int pmdg_ref_gl(int n, double *x, double *w) {
  if (n < 1 || n > RMAXQ) return -1;
  for (int j = 0; j < n; ++j) {
    double t = -cos(M_PI * (j + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, t, &P, &dP);
      double dt = P / dP;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    double P, dP;
    legendre(n, t, &P, &dP);
    x[j] = t;
    w[j] = 2.0 / ((1.0 - t * t) * dP * dP);
  }
  return 0;
}

/* Values and first derivatives of the n+1 Lagrange polynomials through
 * nodes[0..n], at the point t, by the plain product formula. */
void pmdg_ref_lagrange(int n, const double *nodes, double t, double *val, double *der) {
  for (int j = 0; j <= n; ++j) {
    double v = 1.0;
    for (int m = 0; m <= n; ++m)
      if (m != j) v *= (t - nodes[m]) / (nodes[j] - nodes[m]);
    val[j] = v;
    double d = 0.0;
    for (int k = 0; k <= n; ++k) {
      if (k == j) continue;
      double prod = 1.0 / (nodes[j] - nodes[k]);
      for (int m = 0; m <= n; ++m)
        if (m != j && m != k) prod *= (t - nodes[m]) / (nodes[j] - nodes[m]);
      d += prod;
    }
    der[j] = d;
  }
}

/* D[i][j] = l_j'(x_i), row-major (N+1)x(N+1), at the GLL nodes of order N. */
int pmdg_ref_dmat(int N, double *D) {
  double x[RMAXN], w[RMAXN], v[RMAXN];
  if (pmdg_ref_gll(N, x, w)) return -1;
  for (int i = 0; i <= N; ++i) pmdg_ref_lagrange(N, x, x[i], v, D + i * (N + 1));
  return 0;
}

/* ------------------------------------------------------------------ */
/* Mesh: one or two bricks                                             */
/* ------------------------------------------------------------------ */

typedef struct {
  double x0[3], h[3];
  int ne[3], N;
  double c, rho;
  int nn[3];
  long nnodes, off;
  double xg[RMAXN], wg[RMAXN];
  double D[RMAXN][RMAXN];
  /* trilinear hexahedra (Sec. 3, maps X_K): vertex coordinates
   * [(ne0+1)(ne1+1)(ne2+1)][3], x fastest; NULL for an axis-aligned brick */
  double *V;
} rdom;

typedef struct {
  int dom, e[3];
  double l[3][RMAXN];
} rrecv;

typedef struct {
  int ndom;
  rdom d[2];
  long ntot;
  double dt, alpha, gammaF;
  int literal;
  int abs_literal;    /* absorbing damping on the predicted velocity alone, as printed (test switch) */
  double sample_gain; /* 1 normally; 0 removes the sampling term (test hook) */
  double *mass;
  double *cabs;      /* absorbing-boundary matrix C (diagonal), or NULL */
  double *p, *pd, *pdd;
  /* perfectly matched layer, per domain (Sec. 2, eq. full_problem) */
  int pml_on[2];
  double *pzeta[2][3];  /* zeta_i of the layer at the node coordinates of axis i, [nn[i]] */
  long *eslot[2];       /* element -> slot of its Phi values, or -1 */
  long nel[2];          /* elements with zeta > 0 at one of their nodes */
  double *Phi[2];       /* [nel][3][(N+1)^3], element-wise at the GLL nodes */
  double *psi;          /* [ntot], psi_t = p */
  /* interface quadrature-point list (fine-face points mapped to coarse side) */
  int nq;
  double gq[RMAXQ], gw[RMAXQ];
  long nfine;
  int *q_ce;         /* [nfine*nq*nq*2] coarse element (ex,ey) */
  double *q_xi;      /* [nfine*nq*nq*2] coarse reference coordinates */
  /* PMUTs */
  int Np, Nm;
  double *ctr, *rad, *omega, *zeta, *eta;
  double kappa;
  int *fn_cnt;
  long **fn_node;
  double **fn_wf, **fn_shape;
  double *q, *qd, *qdd;
  double *amp, *phase, freq, ncyc;
  int envelope;
  double t_switch, cap;
  /* receivers */
  int R;
  rrecv *rcv;
  long nstep;
} rsolver;

static long nidx(const rdom *d, int i, int j, int k) {
  return d->off + i + (long)d->nn[0] * (j + (long)d->nn[1] * k);
}

static double node_coord(const rdom *d, int axis, int i) {
  int e = i / d->N, a = i % d->N;
  if (e == d->ne[axis]) { e -= 1; a = d->N; }
  return d->x0[axis] + d->h[axis] * (e + 0.5 * (d->xg[a] + 1.0));
}

/* ------------------------------------------------------------------ */
/* Trilinear hexahedra (Sec. 3, maps X_K)                              */
/* ------------------------------------------------------------------ */

/* Corner c = cx + 2 cy + 4 cz of the reference cube sits at
 * ((-1)^(cx+1), (-1)^(cy+1), (-1)^(cz+1)).  X(xi) = sum_c N_c(xi) V_c with
 * N_c = prod_a (1 + s_a xi_a) / 2; J[i][j] = d x_i / d xi_j. */
static void tri_map(const double V8[8][3], const double xi[3], double x[3], double J[3][3]) {
  for (int i = 0; i < 3; ++i) {
    x[i] = 0;
    for (int j = 0; j < 3; ++j) J[i][j] = 0;
  }
  for (int c = 0; c < 8; ++c) {
    double sg[3], f[3];
    for (int a = 0; a < 3; ++a) {
      sg[a] = ((c >> a) & 1) ? 1.0 : -1.0;
      f[a] = 0.5 * (1.0 + sg[a] * xi[a]);
    }
    double Nc = f[0] * f[1] * f[2];
    double dN[3] = {0.5 * sg[0] * f[1] * f[2], 0.5 * sg[1] * f[0] * f[2], 0.5 * sg[2] * f[0] * f[1]};
    for (int i = 0; i < 3; ++i) {
      x[i] += Nc * V8[c][i];
      for (int j = 0; j < 3; ++j) J[i][j] += dN[j] * V8[c][i];
    }
  }
}

static double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* Inverse of a 3x3 matrix by its adjugate; returns the determinant. */
static double inv3(const double J[3][3], double Ji[3][3]) {
  double dt = det3(J);
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / dt;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / dt;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / dt;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / dt;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / dt;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / dt;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / dt;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / dt;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / dt;
  return dt;
}

static long vidx(const rdom *d, int i, int j, int k) {
  return i + (long)(d->ne[0] + 1) * (j + (long)(d->ne[1] + 1) * k);
}

/* The eight vertices of element (ex, ey, ez) in corner order. */
static void elem_vertices(const rdom *d, int ex, int ey, int ez, double V8[8][3]) {
  for (int c = 0; c < 8; ++c) {
    long v = vidx(d, ex + (c & 1), ey + ((c >> 1) & 1), ez + ((c >> 2) & 1));
    for (int a = 0; a < 3; ++a) V8[c][a] = d->V[3 * v + a];
  }
}

/* Element and local index along one axis of global node index i: the lower
 * element owns a shared node, except at the last node of the line. */
static void node_elem(const rdom *d, int axis, int i, int *e, int *a) {
  *e = i / d->N;
  *a = i % d->N;
  if (*e == d->ne[axis]) { *e -= 1; *a = d->N; }
}

/* Coordinates of node (i, j, k): on a brick the tensor grid, on trilinear
 * hexahedra the map of the lowest element containing it at its GLL point. */
static void node_xyz(const rdom *d, int i, int j, int k, double x[3]) {
  if (!d->V) {
    x[0] = node_coord(d, 0, i); x[1] = node_coord(d, 1, j); x[2] = node_coord(d, 2, k);
    return;
  }
  int e[3], a[3], g[3] = {i, j, k};
  for (int t = 0; t < 3; ++t) node_elem(d, t, g[t], &e[t], &a[t]);
  double V8[8][3], J[3][3], xi[3] = {d->xg[a[0]], d->xg[a[1]], d->xg[a[2]]};
  elem_vertices(d, e[0], e[1], e[2], V8);
  tri_map(V8, xi, x, J);
}

/* Element residual r = K_e u of the volume term of a on a trilinear
 * hexahedron with vertices V24 (corner order): the integral of
 * c^2 grad u . grad v over K = X_K(K^), by GLL collocation on the
 * reference cube.  At each node grad_x u = J^{-T} grad_xi u, so the
 * reference flux is w |J| c^2 J^{-1} J^{-T} grad_xi u, tested with
 * grad_xi l_m (Sec. 3, eq. Wf_2, first sum, with the change of variables
 * x = X_K(xi)).  u, r are [(N+1)^3] with a fastest. */
void pmdg_ref_hex_apply(int N, const double *V24, double c, const double *u, double *r) {
  double xg[RMAXN], w[RMAXN], D[RMAXN * RMAXN], V8[8][3];
  pmdg_ref_gll(N, xg, w);
  pmdg_ref_dmat(N, D);
  for (int q = 0; q < 8; ++q)
    for (int a = 0; a < 3; ++a) V8[q][a] = V24[3 * q + a];
  int n1 = N + 1;
#define U(a, b, cc) u[(a) + n1 * ((b) + n1 * (cc))]
  for (int i = 0; i < n1 * n1 * n1; ++i) r[i] = 0.0;
  for (int cc = 0; cc <= N; ++cc)
    for (int b = 0; b <= N; ++b)
      for (int a = 0; a <= N; ++a) {
        double gr[3] = {0, 0, 0};
        for (int m = 0; m <= N; ++m) {
          gr[0] += D[a * n1 + m] * U(m, b, cc);
          gr[1] += D[b * n1 + m] * U(a, m, cc);
          gr[2] += D[cc * n1 + m] * U(a, b, m);
        }
        double xi[3] = {xg[a], xg[b], xg[cc]}, x[3], J[3][3], Ji[3][3];
        tri_map(V8, xi, x, J);
        double dJ = inv3(J, Ji);
        /* physical gradient, then the reference flux J^{-1} (grad_x u) */
        double gx[3], F[3];
        for (int i = 0; i < 3; ++i) gx[i] = Ji[0][i] * gr[0] + Ji[1][i] * gr[1] + Ji[2][i] * gr[2];
        double wq = w[a] * w[b] * w[cc] * dJ * c * c;
        for (int i = 0; i < 3; ++i) F[i] = wq * (Ji[i][0] * gx[0] + Ji[i][1] * gx[1] + Ji[i][2] * gx[2]);
        for (int m = 0; m <= N; ++m) {
          r[m + n1 * (b + n1 * cc)] += D[a * n1 + m] * F[0];
          r[a + n1 * (m + n1 * cc)] += D[b * n1 + m] * F[1];
          r[a + n1 * (b + n1 * m)] += D[cc * n1 + m] * F[2];
        }
      }
#undef U
}

/* Newton's method for the reference point xi of x in the element with
 * vertices V8g, from xi = 0; returns 0 when it converged (|dxi| < 1e-14),
 * -1 otherwise.  Coordinates are taken relative to the first vertex, so the
 * residual's rounding is that of the element's size. */
static int tri_inverse(const double V8g[8][3], const double xg[3], double xi[3]) {
  double V8[8][3], x[3];
  for (int c = 0; c < 8; ++c)
    for (int a = 0; a < 3; ++a) V8[c][a] = V8g[c][a] - V8g[0][a];
  for (int a = 0; a < 3; ++a) x[a] = xg[a] - V8g[0][a];
  xi[0] = xi[1] = xi[2] = 0.0;
  for (int it = 0; it < 60; ++it) {
    double y[3], J[3][3], Ji[3][3], dx[3], st = 0;
    tri_map(V8, xi, y, J);
    if (!(fabs(det3(J)) > 0)) return -1;
    inv3(J, Ji);
    for (int i = 0; i < 3; ++i) dx[i] = x[i] - y[i];
    for (int i = 0; i < 3; ++i) {
      double d = Ji[i][0] * dx[0] + Ji[i][1] * dx[1] + Ji[i][2] * dx[2];
      xi[i] += d;
      st += fabs(d);
    }
    if (!(fabs(xi[0]) < 10 && fabs(xi[1]) < 10 && fabs(xi[2]) < 10)) return -1;
    if (st < 1e-14) return 0;
  }
  return -1;
}

static int setup_dom(rdom *d, const double *prm) {
  /* prm: x0[3], h[3], ne[3], N, c, rho */
  for (int a = 0; a < 3; ++a) { d->x0[a] = prm[a]; d->h[a] = prm[3 + a]; d->ne[a] = (int)prm[6 + a]; }
  d->N = (int)prm[9]; d->c = prm[10]; d->rho = prm[11];
  if (d->N < 1 || d->N >= RMAXN) return -1;
  for (int a = 0; a < 3; ++a) {
    if (d->ne[a] < 1 || !(d->h[a] > 0)) return -1;
    d->nn[a] = d->N * d->ne[a] + 1;
  }
  d->nnodes = (long)d->nn[0] * d->nn[1] * d->nn[2];
  pmdg_ref_gll(d->N, d->xg, d->wg);
  double Dm[RMAXN * RMAXN];
  pmdg_ref_dmat(d->N, Dm);
  for (int i = 0; i <= d->N; ++i)
    for (int j = 0; j <= d->N; ++j) d->D[i][j] = Dm[i * (d->N + 1) + j];
  return 0;
}

/* Lumped mass: the mass form with GLL ("reduced") integration is diagonal,
 * M_ii = sum over elements containing i of w_a w_b w_c |J| (Sec. 3.1). */
static void build_mass(rsolver *s) {
  memset(s->mass, 0, sizeof(double) * s->ntot);
  for (int dd = 0; dd < s->ndom; ++dd) {
    rdom *d = &s->d[dd];
    int N = d->N;
    double J = d->h[0] * d->h[1] * d->h[2] / 8.0;
    for (int ez = 0; ez < d->ne[2]; ++ez)
      for (int ey = 0; ey < d->ne[1]; ++ey)
        for (int ex = 0; ex < d->ne[0]; ++ex) {
          double V8[8][3];
          if (d->V) elem_vertices(d, ex, ey, ez, V8);
          for (int c = 0; c <= N; ++c)
            for (int b = 0; b <= N; ++b)
              for (int a = 0; a <= N; ++a) {
                double Jq = J;
                if (d->V) {
                  double xi[3] = {d->xg[a], d->xg[b], d->xg[c]}, x[3], Jm[3][3];
                  tri_map(V8, xi, x, Jm);
                  Jq = det3(Jm);
                }
                s->mass[nidx(d, N * ex + a, N * ey + b, N * ez + c)] += d->wg[a] * d->wg[b] * d->wg[c] * Jq;
              }
        }
  }
}

/* First-order absorbing boundary (Sec. 2 and 3.1: the term int c pdot v ds
 * on absorbing faces, the damping matrix C of the acoustic solve): C_ii = sum over the
 * element faces on an absorbing face of domain dd that contain i of
 * c w_a w_b |J_f|, GLL collocation on the face, |J_f| the face's area / 4.
 * faces: bit 2a + 0 for the face at the low end of axis a, 2a + 1 for the
 * high end.  Calls accumulate (one per domain). */
void pmdg_ref_set_absorbing(void *h, int dd, int faces) {
  rsolver *s = (rsolver *)h;
  if (s->d[dd].V) return; /* absorbing faces on trilinear hexahedra are not built */
  if (!s->cabs) s->cabs = (double *)calloc(s->ntot, sizeof(double));
  rdom *d = &s->d[dd];
  int N = d->N;
  for (int ax = 0; ax < 3; ++ax)
    for (int side = 0; side < 2; ++side) {
      if (!(faces & (1 << (2 * ax + side)))) continue;
      int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
      double Jf = d->h[t1] * d->h[t2] / 4.0;
      int fixed = side ? d->nn[ax] - 1 : 0;
      for (int e2 = 0; e2 < d->ne[t2]; ++e2)
        for (int e1 = 0; e1 < d->ne[t1]; ++e1)
          for (int b = 0; b <= N; ++b)
            for (int a = 0; a <= N; ++a) {
              int g[3];
              g[ax] = fixed;
              g[t1] = N * e1 + a;
              g[t2] = N * e2 + b;
              s->cabs[nidx(d, g[0], g[1], g[2])] += d->c * d->wg[a] * d->wg[b] * Jf;
            }
    }
}

/* Trilinear hexahedra for the domain of a single-domain solver: V holds
 * the (ne0+1)(ne1+1)(ne2+1) vertices [.. x 3], x fastest (Sec. 3: element
 * (ex, ey, ez) is the trilinear image of the reference cube on its eight
 * vertices).  Returns 0; -1 for a two-domain solver or one with absorbing
 * faces or a layer; -2 when the Jacobian determinant is not positive at a
 * GLL node of some element.  Rebuilds the lumped mass; PMUTs and receivers
 * are set afterwards. */
int pmdg_ref_set_vertices(void *h, int dd, const double *V) {
  rsolver *s = (rsolver *)h;
  if (s->ndom != 1 || dd != 0 || s->cabs || s->pml_on[0]) return -1;
  rdom *d = &s->d[dd];
  long nv = (long)(d->ne[0] + 1) * (d->ne[1] + 1) * (d->ne[2] + 1);
  double *Vc = (double *)malloc(sizeof(double) * 3 * nv);
  memcpy(Vc, V, sizeof(double) * 3 * nv);
  double *old = d->V;
  d->V = Vc;
  int N = d->N;
  for (int ez = 0; ez < d->ne[2]; ++ez)
    for (int ey = 0; ey < d->ne[1]; ++ey)
      for (int ex = 0; ex < d->ne[0]; ++ex) {
        double V8[8][3];
        elem_vertices(d, ex, ey, ez, V8);
        for (int c = 0; c <= N; ++c)
          for (int b = 0; b <= N; ++b)
            for (int a = 0; a <= N; ++a) {
              double xi[3] = {d->xg[a], d->xg[b], d->xg[c]}, x[3], J[3][3];
              tri_map(V8, xi, x, J);
              if (!(det3(J) > 0)) {
                d->V = old;
                free(Vc);
                return -2;
              }
            }
      }
  free(old);
  build_mass(s);
  return 0;
}

/* Outward unit normal at the centre of face f = 2 axis + side of the
 * element with vertices V8, the face's first corner and its diameter (the
 * largest distance between two of its corners, which bounds the distance
 * from a corner to any point of the face). */
static void face_geometry(const double V8[8][3], int f, double n[3], double v0[3], double *diam) {
  int ax = f / 2, side = f % 2, t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
  double xi[3] = {0, 0, 0}, x[3], J[3][3];
  xi[ax] = side ? 1.0 : -1.0;
  tri_map(V8, xi, x, J);
  double a[3] = {J[0][t1], J[1][t1], J[2][t1]}, b[3] = {J[0][t2], J[1][t2], J[2][t2]};
  double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  double l = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]), sg = side ? 1.0 : -1.0;
  for (int i = 0; i < 3; ++i) n[i] = sg * c[i] / l;
  /* corners of the face: bit ax fixed to side; k00, k10, k01, k11 in (t1, t2) */
  int k[4];
  for (int q = 0; q < 4; ++q) k[q] = (side << ax) | ((q & 1) << t1) | (((q >> 1) & 1) << t2);
  for (int i = 0; i < 3; ++i) v0[i] = V8[k[0]][i];
  double dmax = 0;
  for (int p = 0; p < 4; ++p)
    for (int q = p + 1; q < 4; ++q) {
      double d = 0;
      for (int i = 0; i < 3; ++i) d += (V8[k[q]][i] - V8[k[p]][i]) * (V8[k[q]][i] - V8[k[p]][i]);
      if (d > dmax) dmax = d;
    }
  *diam = sqrt(dmax);
}

/* Face matching on Gamma_I (Sec. 5, Algorithm 3).  Fine side: nf
 * hexahedra fine_hex [nf][8][3] (corner order) and the local face of each
 * on Gamma_I, fine_face[nf] = 2 axis + side (side 0: xi_axis = -1, side 1:
 * +1); coarse side likewise (nc, coarse_hex, coarse_face).  For every
 * Gauss-Legendre point (nq per direction) of every fine face, x_q =
 * X_{K+}(xi), the coarse faces are taken in index order; one is a candidate
 * when its outward normal at its centre is opposite to the fine face's,
 * |n+ + n-| < tol, and its first corner lies within
 * r = max(diam F-, diam F+) + eps of x_q (diam: the largest distance
 * between two corners of the face); the first candidate whose
 * element's inverse map (Newton) puts x_q in [-1, 1]^3, up to 1e-10, is the
 * match.  Points are ordered (fine face, j, i) with i along the face's
 * first tangential axis (axis + 1) mod 3.  Writes elem[nf nq^2] (coarse
 * index, or -1) and xi[nf nq^2][3]; returns the number of unmatched points,
 * or -1 for bad arguments. */
int pmdg_ref_match_faces(int nq, int nf, const double *fine_hex, const int *fine_face, int nc,
                         const double *coarse_hex, const int *coarse_face, double tol, double eps,
                         int *elem, double *xi) {
  if (nq < 1 || nq > RMAXQ || nf < 0 || nc < 0) return -1;
  double gq[RMAXQ], gw[RMAXQ];
  pmdg_ref_gl(nq, gq, gw);
  double *cn = (double *)malloc(sizeof(double) * 3 * (nc ? nc : 1));
  double *cv = (double *)malloc(sizeof(double) * 3 * (nc ? nc : 1));
  double *cd = (double *)malloc(sizeof(double) * (nc ? nc : 1));
  for (int c = 0; c < nc; ++c) {
    double V8[8][3];
    memcpy(V8, coarse_hex + 24L * c, sizeof(V8));
    if (coarse_face[c] < 0 || coarse_face[c] > 5) { free(cn); free(cv); free(cd); return -1; }
    face_geometry(V8, coarse_face[c], cn + 3 * c, cv + 3 * c, cd + c);
  }
  int unmatched = 0;
  for (int f = 0; f < nf; ++f) {
    double V8[8][3], nf3[3], vf[3], df;
    memcpy(V8, fine_hex + 24L * f, sizeof(V8));
    if (fine_face[f] < 0 || fine_face[f] > 5) { unmatched = -1; break; }
    face_geometry(V8, fine_face[f], nf3, vf, &df);
    int ax = fine_face[f] / 2, t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
    for (int j = 0; j < nq; ++j)
      for (int i = 0; i < nq; ++i) {
        long q = ((long)f * nq + j) * nq + i;
        double r[3], x[3], J[3][3];
        r[ax] = (fine_face[f] % 2) ? 1.0 : -1.0;
        r[t1] = gq[i];
        r[t2] = gq[j];
        tri_map(V8, r, x, J);
        elem[q] = -1;
        xi[3 * q] = xi[3 * q + 1] = xi[3 * q + 2] = 0.0;
        for (int c = 0; c < nc; ++c) {
          double sn = 0, dv = 0;
          for (int k = 0; k < 3; ++k) {
            sn += (nf3[k] + cn[3 * c + k]) * (nf3[k] + cn[3 * c + k]);
            dv += (cv[3 * c + k] - x[k]) * (cv[3 * c + k] - x[k]);
          }
          double rad = (cd[c] > df ? cd[c] : df) + eps;
          /* |n+ + n-| < tol and |V - x_q| < r, compared as squares */
          if (!(sn < tol * tol && dv < rad * rad)) continue;
          double W8[8][3], t[3];
          memcpy(W8, coarse_hex + 24L * c, sizeof(W8));
          if (tri_inverse(W8, x, t)) continue;
          if (fabs(t[0]) <= 1 + 1e-10 && fabs(t[1]) <= 1 + 1e-10 && fabs(t[2]) <= 1 + 1e-10) {
            elem[q] = c;
            for (int k = 0; k < 3; ++k) xi[3 * q + k] = t[k];
            break;
          }
        }
        if (elem[q] < 0) ++unmatched;
      }
  }
  free(cn); free(cv); free(cd);
  return unmatched;
}

/* Copies C (zeros without absorbing faces) into out [ntot]. */
void pmdg_ref_absorbing(void *h, double *out) {
  rsolver *s = (rsolver *)h;
  for (long i = 0; i < s->ntot; ++i) out[i] = s->cabs ? s->cabs[i] : 0.0;
}

/* ------------------------------------------------------------------ */
/* Stiffness: volume part                                              */
/* ------------------------------------------------------------------ */

/* Element residual r = K_e u for the volume term of a: integral over K of
 * c^2 grad u . grad v, with GLL collocation in all three directions
 * (Sec. 3, eq. Wf_2, first sum).  u, r are [(N+1)^3] with a fastest.
 * Gradient in reference coordinates via D, metric 2/h per axis. */
void pmdg_ref_element_apply(int N, const double *h, double c, const double *u, double *r) {
  double x[RMAXN], w[RMAXN], D[RMAXN * RMAXN];
  pmdg_ref_gll(N, x, w);
  pmdg_ref_dmat(N, D);
  int n1 = N + 1;
  double J = h[0] * h[1] * h[2] / 8.0;
  double g[3] = {4.0 / (h[0] * h[0]), 4.0 / (h[1] * h[1]), 4.0 / (h[2] * h[2])};
#define U(a, b, cc) u[(a) + n1 * ((b) + n1 * (cc))]
  for (int i = 0; i < n1 * n1 * n1; ++i) r[i] = 0.0;
  for (int cc = 0; cc <= N; ++cc)
    for (int b = 0; b <= N; ++b)
      for (int a = 0; a <= N; ++a) {
        /* gradient at quadrature node (a,b,cc) */
        double ux = 0, uy = 0, uz = 0;
        for (int m = 0; m <= N; ++m) {
          ux += D[a * n1 + m] * U(m, b, cc);
          uy += D[b * n1 + m] * U(a, m, cc);
          uz += D[cc * n1 + m] * U(a, b, m);
        }
        double wq = w[a] * w[b] * w[cc] * J * c * c;
        /* test function gradients: d/dxi of l_m at node a is D[a][m] */
        for (int m = 0; m <= N; ++m) {
          r[m + n1 * (b + n1 * cc)] += wq * g[0] * D[a * n1 + m] * ux;
          r[a + n1 * (m + n1 * cc)] += wq * g[1] * D[b * n1 + m] * uy;
          r[a + n1 * (b + n1 * m)] += wq * g[2] * D[cc * n1 + m] * uz;
        }
      }
#undef U
}

static void volume_apply(const rsolver *s, const double *p, double *Kp) {
  for (int dd = 0; dd < s->ndom; ++dd) {
    const rdom *d = &s->d[dd];
    int N = d->N, n1 = N + 1;
    for (int colour = 0; colour < 8; ++colour) {
      int cx = colour & 1, cy = (colour >> 1) & 1, cz = (colour >> 2) & 1;
      int nx = (d->ne[0] - cx + 1) / 2, ny = (d->ne[1] - cy + 1) / 2, nz = (d->ne[2] - cz + 1) / 2;
      long tot = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
      for (long t = 0; t < tot; ++t) {
        int ex = cx + 2 * (int)(t % nx), ey = cy + 2 * (int)((t / nx) % ny), ez = cz + 2 * (int)(t / ((long)nx * ny));
        double u[RMAXN * RMAXN * RMAXN], r[RMAXN * RMAXN * RMAXN];
        for (int c = 0; c <= N; ++c)
          for (int b = 0; b <= N; ++b)
            for (int a = 0; a <= N; ++a)
              u[a + n1 * (b + n1 * c)] = p[nidx(d, N * ex + a, N * ey + b, N * ez + c)];
        if (d->V) {
          double V8[8][3];
          elem_vertices(d, ex, ey, ez, V8);
          pmdg_ref_hex_apply(N, &V8[0][0], d->c, u, r);
        } else {
          pmdg_ref_element_apply(N, d->h, d->c, u, r);
        }
        for (int c = 0; c <= N; ++c)
          for (int b = 0; b <= N; ++b)
            for (int a = 0; a <= N; ++a)
              Kp[nidx(d, N * ex + a, N * ey + b, N * ez + c)] += r[a + n1 * (b + n1 * c)];
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* Stiffness: interface part (SIPG on Gamma_I)                         */
/* ------------------------------------------------------------------ */

/* Interface quadrature-point list (Sec. 5): every Gauss-Legendre point of
 * every fine face is pushed forward with the fine map, then pulled back into
 * the coarse element containing it.  On bricks both maps are affine, so the
 * pull-back is closed-form; the containing coarse element is found by a plain
 * scan that keeps the lowest index whose reference coordinate lies in
 * [-1,1] up to a tolerance. */
static int build_interface(rsolver *s) {
  rdom *f = &s->d[0], *cr = &s->d[1];
  /* geometry must match: fine top face == coarse bottom face */
  double ztop = f->x0[2] + f->ne[2] * f->h[2];
  double tol = 1e-9 * (f->h[2] < cr->h[2] ? f->h[2] : cr->h[2]);
  if (fabs(ztop - cr->x0[2]) > tol) return -1;
  for (int a = 0; a < 2; ++a) {
    double l0 = f->ne[a] * f->h[a], l1 = cr->ne[a] * cr->h[a];
    if (fabs(f->x0[a] - cr->x0[a]) > 1e-9 * l0 || fabs(l0 - l1) > 1e-9 * l0) return -1;
  }
  int nmax = f->N > cr->N ? f->N : cr->N;
  s->nq = nmax + 1;
  pmdg_ref_gl(s->nq, s->gq, s->gw);
  double cbar = 2.0 * f->c * cr->c / (f->c + cr->c);
  double hmin = f->h[2] < cr->h[2] ? f->h[2] : cr->h[2];
  s->gammaF = s->alpha * cbar * cbar * (double)(nmax * nmax) / hmin;
  s->nfine = (long)f->ne[0] * f->ne[1];
  long npts = s->nfine * s->nq * s->nq;
  s->q_ce = (int *)malloc(sizeof(int) * 2 * npts);
  s->q_xi = (double *)malloc(sizeof(double) * 2 * npts);
  for (long fe = 0; fe < s->nfine; ++fe) {
    int ex = (int)(fe % f->ne[0]), ey = (int)(fe / f->ne[0]);
    for (int qb = 0; qb < s->nq; ++qb)
      for (int qa = 0; qa < s->nq; ++qa) {
        long qi = (fe * s->nq + qb) * s->nq + qa;
        double xq[2];
        xq[0] = f->x0[0] + f->h[0] * (ex + 0.5 * (s->gq[qa] + 1.0));
        xq[1] = f->x0[1] + f->h[1] * (ey + 0.5 * (s->gq[qb] + 1.0));
        for (int a = 0; a < 2; ++a) {
          int found = -1;
          double xi = 0;
          for (int e = 0; e < cr->ne[a]; ++e) {
            double r = 2.0 * (xq[a] - (cr->x0[a] + e * cr->h[a])) / cr->h[a] - 1.0;
            if (r >= -1.0 - 1e-12 && r <= 1.0 + 1e-12) { found = e; xi = r; break; }
          }
          if (found < 0) return -1;
          s->q_ce[2 * qi + a] = found;
          s->q_xi[2 * qi + a] = xi;
        }
      }
  }
  return 0;
}

/* The interface quadrature-point list: coarse element (ex, ey) and
 * reference coordinates (xi, eta) of every Gauss-Legendre point of every
 * fine face, [npts][2] each, points ordered (fine face, eta, xi) with the
 * fine face ex + ne0 ey.  Returns npts (0 without an interface). */
long pmdg_ref_interface_points(void *h, int *ce, double *xi) {
  rsolver *s = (rsolver *)h;
  if (s->ndom < 2) return 0;
  long npts = s->nfine * s->nq * s->nq;
  if (ce) memcpy(ce, s->q_ce, sizeof(int) * 2 * npts);
  if (xi) memcpy(xi, s->q_xi, sizeof(double) * 2 * npts);
  return npts;
}

/* Adds the three interface sums of a (Sec. 3, eq. Wf_2) for all test
 * functions: with n = n+ (outward from the fine side), [u] = (u+ - u-) n and
 * {c^2 grad u}.[v] = 1/2 (c+^2 d_n u+ + c-^2 d_n u-) (v+ - v-). */
static void interface_apply(const rsolver *s, const double *p, double *Kp) {
  if (s->ndom < 2) return;
  const rdom *f = &s->d[0], *cr = &s->d[1];
  int Nf = f->N, Nc = cr->N, n1f = Nf + 1, n1c = Nc + 1;
  double Jf = 0.25 * f->h[0] * f->h[1];
  double cf2 = f->c * f->c, cc2 = cr->c * cr->c;
  int ezf = f->ne[2] - 1;
  double lzf[RMAXN], dzf[RMAXN], lzc[RMAXN], dzc[RMAXN];
  pmdg_ref_lagrange(Nf, f->xg, 1.0, lzf, dzf);
  pmdg_ref_lagrange(Nc, cr->xg, -1.0, lzc, dzc);
  for (long fe = 0; fe < s->nfine; ++fe) {
    int ex = (int)(fe % f->ne[0]), ey = (int)(fe / f->ne[0]);
    for (int qb = 0; qb < s->nq; ++qb)
      for (int qa = 0; qa < s->nq; ++qa) {
        long qi = (fe * s->nq + qb) * s->nq + qa;
        double w = s->gw[qa] * s->gw[qb] * Jf;
        double la[RMAXN], da[RMAXN], lb[RMAXN], db[RMAXN];
        pmdg_ref_lagrange(Nf, f->xg, s->gq[qa], la, da);
        pmdg_ref_lagrange(Nf, f->xg, s->gq[qb], lb, db);
        int cx = s->q_ce[2 * qi], cy = s->q_ce[2 * qi + 1];
        double ma[RMAXN], mda[RMAXN], mb[RMAXN], mdb[RMAXN];
        pmdg_ref_lagrange(Nc, cr->xg, s->q_xi[2 * qi], ma, mda);
        pmdg_ref_lagrange(Nc, cr->xg, s->q_xi[2 * qi + 1], mb, mdb);
        double pp = 0, dpp = 0, pm = 0, dpm = 0;
        for (int c = 0; c <= Nf; ++c)
          for (int b = 0; b <= Nf; ++b)
            for (int a = 0; a <= Nf; ++a) {
              double u = p[nidx(f, Nf * ex + a, Nf * ey + b, Nf * ezf + c)];
              pp += u * la[a] * lb[b] * lzf[c];
              dpp += u * la[a] * lb[b] * dzf[c] * (2.0 / f->h[2]);
            }
        for (int c = 0; c <= Nc; ++c)
          for (int b = 0; b <= Nc; ++b)
            for (int a = 0; a <= Nc; ++a) {
              double u = p[nidx(cr, Nc * cx + a, Nc * cy + b, c)];
              pm += u * ma[a] * mb[b] * lzc[c];
              dpm += u * ma[a] * mb[b] * dzc[c] * (2.0 / cr->h[2]);
            }
        double jump = pp - pm;
        double avg = 0.5 * (cf2 * dpp + cc2 * dpm);
        double A = s->gammaF * jump - avg;
        for (int c = 0; c <= Nf; ++c)
          for (int b = 0; b <= Nf; ++b)
            for (int a = 0; a <= Nf; ++a) {
              double phi = la[a] * lb[b] * lzf[c];
              double dphi = la[a] * lb[b] * dzf[c] * (2.0 / f->h[2]);
              Kp[nidx(f, Nf * ex + a, Nf * ey + b, Nf * ezf + c)] += w * (A * phi - 0.5 * jump * cf2 * dphi);
            }
        for (int c = 0; c <= Nc; ++c)
          for (int b = 0; b <= Nc; ++b)
            for (int a = 0; a <= Nc; ++a) {
              double phi = ma[a] * mb[b] * lzc[c];
              double dphi = ma[a] * mb[b] * dzc[c] * (2.0 / cr->h[2]);
              Kp[nidx(cr, Nc * cx + a, Nc * cy + b, c)] += w * (-A * phi - 0.5 * jump * cc2 * dphi);
            }
      }
  }
  (void)n1f; (void)n1c;
}

/* ------------------------------------------------------------------ */
/* Public construction                                                 */
/* ------------------------------------------------------------------ */

/* dom_prm: ndom x 12 doubles {x0[3], h[3], ne[3], N, c, rho}; dom 0 is the
 * primary (fine) brick whose bottom face z = x0[2] carries the PMUTs; dom 1,
 * if present, sits on top of it and meets it on Gamma_I. */
void *pmdg_ref_create(int ndom, const double *dom_prm, double dt, double alpha) {
  if (ndom < 1 || ndom > 2) return NULL;
  rsolver *s = (rsolver *)calloc(1, sizeof(rsolver));
  s->ndom = ndom; s->dt = dt; s->alpha = alpha; s->sample_gain = 1.0;
  s->t_switch = INFINITY; s->cap = 1.0;
  long off = 0;
  for (int d = 0; d < ndom; ++d) {
    if (setup_dom(&s->d[d], dom_prm + 12 * d)) { free(s); return NULL; }
    s->d[d].off = off;
    off += s->d[d].nnodes;
  }
  s->ntot = off;
  if (ndom == 2 && build_interface(s)) { free(s); return NULL; }
  s->mass = (double *)malloc(sizeof(double) * s->ntot);
  s->p = (double *)calloc(s->ntot, sizeof(double));
  s->pd = (double *)calloc(s->ntot, sizeof(double));
  s->pdd = (double *)calloc(s->ntot, sizeof(double));
  build_mass(s);
  s->kappa = s->d[0].rho * s->d[0].c * s->d[0].c;
  return s;
}

static void free_pmuts(rsolver *s) {
  for (int k = 0; k < s->Np; ++k) {
    free(s->fn_node[k]); free(s->fn_wf[k]); free(s->fn_shape[k]);
  }
  free(s->fn_node); free(s->fn_wf); free(s->fn_shape); free(s->fn_cnt);
  free(s->ctr); free(s->rad); free(s->omega); free(s->zeta); free(s->eta);
  free(s->q); free(s->qd); free(s->qdd); free(s->amp); free(s->phase);
  s->Np = 0;
}

void pmdg_ref_destroy(void *h) {
  rsolver *s = (rsolver *)h;
  if (!s) return;
  free_pmuts(s);
  free(s->mass); free(s->cabs); free(s->p); free(s->pd); free(s->pdd);
  free(s->q_ce); free(s->q_xi); free(s->rcv);
  for (int d = 0; d < 2; ++d) {
    free(s->d[d].V);
    for (int a = 0; a < 3; ++a) free(s->pzeta[d][a]);
    free(s->eslot[d]); free(s->Phi[d]);
  }
  free(s->psi);
  free(s);
}

long pmdg_ref_num_nodes(void *h) { return ((rsolver *)h)->ntot; }
long pmdg_ref_dom_nodes(void *h, int d) { return ((rsolver *)h)->d[d].nnodes; }
double pmdg_ref_gamma(void *h) { return ((rsolver *)h)->gammaF; }
void pmdg_ref_set_literal(void *h, int lit) { ((rsolver *)h)->literal = lit; }
/* Test switch: the acoustic solve takes the absorbing term as printed in
 * Algorithm 1, M pdd = f - K p - C pdot* with the predicted velocity alone. */
void pmdg_ref_set_absorbing_literal(void *h, int on) { ((rsolver *)h)->abs_literal = on; }
void pmdg_ref_set_sample_gain(void *h, double g) { ((rsolver *)h)->sample_gain = g; }
void pmdg_ref_set_dt(void *h, double dt) { ((rsolver *)h)->dt = dt; }

/* Node coordinates, concatenated over domains, [ntot x 3]. */
void pmdg_ref_coords(void *h, double *xyz) {
  rsolver *s = (rsolver *)h;
  for (int dd = 0; dd < s->ndom; ++dd) {
    rdom *d = &s->d[dd];
    for (int k = 0; k < d->nn[2]; ++k)
      for (int j = 0; j < d->nn[1]; ++j)
        for (int i = 0; i < d->nn[0]; ++i) {
          node_xyz(d, i, j, k, xyz + 3 * nidx(d, i, j, k));
        }
  }
}

void pmdg_ref_mass(void *h, double *out) {
  rsolver *s = (rsolver *)h;
  memcpy(out, s->mass, sizeof(double) * s->ntot);
}

/* K p = volume part + interface part.  which: 1 volume, 2 interface, 3 both. */
void pmdg_ref_apply_K(void *h, const double *p, double *Kp, int which) {
  rsolver *s = (rsolver *)h;
  memset(Kp, 0, sizeof(double) * s->ntot);
  if (which & 1) volume_apply(s, p, Kp);
  if (which & 2) interface_apply(s, p, Kp);
}

/* Largest eigenvalue of M^{-1} K by power iteration (stability check of the
 * explicit scheme: stable iff dt^2 lambda_max < 4). */
double pmdg_ref_lambda_max(void *h, int iters, unsigned seed) {
  rsolver *s = (rsolver *)h;
  long n = s->ntot;
  double *v = (double *)malloc(sizeof(double) * n), *w = (double *)malloc(sizeof(double) * n);
  unsigned long long st = seed * 2654435761ULL + 12345ULL;
  for (long i = 0; i < n; ++i) {
    st = st * 6364136223846793005ULL + 1442695040888963407ULL;
    v[i] = (double)(st >> 11) / 9007199254740992.0 - 0.5;
  }
  double lam = 0;
  for (int it = 0; it < iters; ++it) {
    pmdg_ref_apply_K(h, v, w, 3);
    double num = 0, den = 0;
    for (long i = 0; i < n; ++i) { w[i] /= s->mass[i]; }
    /* Rayleigh quotient in the M inner product */
    for (long i = 0; i < n; ++i) { num += v[i] * s->mass[i] * w[i]; den += v[i] * s->mass[i] * v[i]; }
    lam = num / den;
    double nrm = 0;
    for (long i = 0; i < n; ++i) nrm += w[i] * w[i] * s->mass[i];
    nrm = sqrt(nrm);
    for (long i = 0; i < n; ++i) v[i] = w[i] / nrm;
  }
  free(v); free(w);
  return lam;
}

/* ------------------------------------------------------------------ */
/* PMUTs, drive, receivers                                             */
/* ------------------------------------------------------------------ */

/* PMUT k covers the primary bottom-face nodes whose in-plane distance to its
 * centre is at most its radius.  Face weight of node i: sum over the bottom
 * faces containing i of w_a w_b |J_face| (GLL collocation on the face).  The
 * coupling matrix is B_{i,(k,m)} = wf_i U_{k,m}.n(x_i), so that
 * f_i = -kappa sum_m qdd_{k,m} B_{i,(k,m)} (eq. f_i) and
 * g_{k,m} = sum_i B_{i,(k,m)} p_i (eq. g_m). */
int pmdg_ref_set_pmuts(void *h, int Np, const double *ctr, const double *rad, int Nm,
                       const double *omega, const double *zeta, const double *eta) {
  rsolver *s = (rsolver *)h;
  free_pmuts(s);
  rdom *d = &s->d[0];
  int N = d->N;
  s->Np = Np; s->Nm = Nm;
  s->ctr = (double *)malloc(sizeof(double) * 2 * Np); memcpy(s->ctr, ctr, sizeof(double) * 2 * Np);
  s->rad = (double *)malloc(sizeof(double) * Np); memcpy(s->rad, rad, sizeof(double) * Np);
  long nm = (long)Np * Nm;
  s->omega = (double *)malloc(sizeof(double) * nm); memcpy(s->omega, omega, sizeof(double) * nm);
  s->zeta = (double *)malloc(sizeof(double) * nm); memcpy(s->zeta, zeta, sizeof(double) * nm);
  s->eta = (double *)malloc(sizeof(double) * nm); memcpy(s->eta, eta, sizeof(double) * nm);
  s->q = (double *)calloc(nm, sizeof(double));
  s->qd = (double *)calloc(nm, sizeof(double));
  s->qdd = (double *)calloc(nm, sizeof(double));
  s->amp = (double *)calloc(Np, sizeof(double));
  s->phase = (double *)calloc(Np, sizeof(double));
  s->fn_cnt = (int *)calloc(Np, sizeof(int));
  s->fn_node = (long **)calloc(Np, sizeof(long *));
  s->fn_wf = (double **)calloc(Np, sizeof(double *));
  s->fn_shape = (double **)calloc(Np, sizeof(double *));
  /* face weights over the whole bottom face */
  int nx = d->nn[0], ny = d->nn[1];
  double *wf = (double *)calloc((size_t)nx * ny, sizeof(double));
  double Jf = 0.25 * d->h[0] * d->h[1];
  for (int ey = 0; ey < d->ne[1]; ++ey)
    for (int ex = 0; ex < d->ne[0]; ++ex) {
      double V8[8][3];
      if (d->V) elem_vertices(d, ex, ey, 0, V8);
      for (int b = 0; b <= N; ++b)
        for (int a = 0; a <= N; ++a) {
          double Jq = Jf;
          if (d->V) {
            /* surface Jacobian |dX/dxi x dX/deta| on the face zeta = -1 */
            double xi[3] = {d->xg[a], d->xg[b], -1.0}, x[3], J[3][3];
            tri_map(V8, xi, x, J);
            double cx = J[1][0] * J[2][1] - J[2][0] * J[1][1];
            double cy = J[2][0] * J[0][1] - J[0][0] * J[2][1];
            double cz = J[0][0] * J[1][1] - J[1][0] * J[0][1];
            Jq = sqrt(cx * cx + cy * cy + cz * cz);
          }
          wf[(N * ex + a) + (long)nx * (N * ey + b)] += d->wg[a] * d->wg[b] * Jq;
        }
    }
  for (int k = 0; k < Np; ++k) {
    int cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
      cnt = 0;
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double xn[3];
          node_xyz(d, i, j, 0, xn);
          double dx = xn[0] - ctr[2 * k], dy = xn[1] - ctr[2 * k + 1];
          if (sqrt(dx * dx + dy * dy) <= rad[k]) {
            if (pass == 1) {
              s->fn_node[k][cnt] = nidx(d, i, j, 0);
              s->fn_wf[k][cnt] = wf[i + (long)nx * j];
            }
            ++cnt;
          }
        }
      if (pass == 0) {
        s->fn_node[k] = (long *)malloc(sizeof(long) * (cnt ? cnt : 1));
        s->fn_wf[k] = (double *)malloc(sizeof(double) * (cnt ? cnt : 1));
        s->fn_shape[k] = (double *)calloc((size_t)(cnt ? cnt : 1) * Nm, sizeof(double));
      }
    }
    s->fn_cnt[k] = cnt;
  }
  free(wf);
  return 0;
}

int pmdg_ref_pmut_nodes(void *h, int k, double *xyz) {
  rsolver *s = (rsolver *)h;
  if (k < 0 || k >= s->Np) return -1;
  if (xyz) {
    double *all = NULL;
    (void)all;
    const rdom *d = &s->d[0];
    for (int n = 0; n < s->fn_cnt[k]; ++n) {
      long g = s->fn_node[k][n] - d->off;
      int i = (int)(g % d->nn[0]), j = (int)((g / d->nn[0]) % d->nn[1]);
      node_xyz(d, i, j, 0, xyz + 3 * n);
    }
  }
  return s->fn_cnt[k];
}

/* shape: [Nm x cnt] samples of U_{k,m}.n at PMUT k's face nodes. */
int pmdg_ref_set_shape(void *h, int k, const double *shape) {
  rsolver *s = (rsolver *)h;
  if (k < 0 || k >= s->Np) return -1;
  memcpy(s->fn_shape[k], shape, sizeof(double) * s->Nm * s->fn_cnt[k]);
  return 0;
}

/* Coupling column B_{.,(k,m)} as (node, value) pairs. */
int pmdg_ref_coupling(void *h, int k, int m, long *node, double *val) {
  rsolver *s = (rsolver *)h;
  for (int n = 0; n < s->fn_cnt[k]; ++n) {
    node[n] = s->fn_node[k][n];
    val[n] = s->fn_wf[k][n] * s->fn_shape[k][(long)m * s->fn_cnt[k] + n];
  }
  return s->fn_cnt[k];
}

void pmdg_ref_set_drive(void *h, const double *amp, const double *phase, double freq, double ncyc, int envelope) {
  rsolver *s = (rsolver *)h;
  memcpy(s->amp, amp, sizeof(double) * s->Np);
  memcpy(s->phase, phase, sizeof(double) * s->Np);
  s->freq = freq; s->ncyc = ncyc; s->envelope = envelope;
}

void pmdg_ref_set_rx(void *h, double t_switch, double cap) {
  rsolver *s = (rsolver *)h;
  s->t_switch = t_switch; s->cap = cap;
}

/* Smooth window (Sec. 6.1, eq. voltage), n = 10:
 * g(t) = exp(1 - alpha(T_d - t)) on [0, T_d/2), exp(1 - alpha(t)) on
 * [T_d/2, T_d], alpha(tau) = (1 - 2 beta^{2n+1} / (1 + beta^{2n}))^{-2},
 * beta(tau) = 2 tau / T_d - 1.  Zero outside [0, T_d]. */
double pmdg_ref_window(double t, double Td) {
  if (t < 0.0 || t > Td) return 0.0;
  double tau = (t < 0.5 * Td) ? (Td - t) : t;
  double beta = 2.0 * tau / Td - 1.0;
  double b20 = pow(beta, 20.0), b21 = pow(beta, 21.0);
  double base = 1.0 - 2.0 * b21 / (1.0 + b20);
  if (base <= 0.0) return 0.0;
  double alpha = 1.0 / (base * base);
  return exp(1.0 - alpha);
}

/* Applied voltage phi_{k,0}(t) = A_k sin(2 pi f t - theta_k) g(t), with
 * T_d = ncyc / f.  envelope 0: window g; 1: rectangular on [0, T_d];
 * 2: rectangular and never switched off. */
double pmdg_ref_drive(double A, double theta, double f, double ncyc, int envelope, double t) {
  double Td = ncyc / f;
  double env;
  if (envelope == 0) env = pmdg_ref_window(t, Td);
  else if (envelope == 1) env = (t >= 0.0 && t <= Td) ? 1.0 : 0.0;
  else env = (t >= 0.0) ? 1.0 : 0.0;
  return A * sin(2.0 * M_PI * f * t - theta) * env;
}

/* Receivers: the lowest-index element (primary first) whose closure holds the
 * point; the trace is the tensor Lagrange interpolant of the element values. */
int pmdg_ref_set_receivers(void *h, int R, const double *xyz) {
  rsolver *s = (rsolver *)h;
  free(s->rcv);
  s->R = R;
  s->rcv = (rrecv *)calloc(R > 0 ? R : 1, sizeof(rrecv));
  for (int r = 0; r < R; ++r) {
    int ok = 0;
    for (int dd = 0; dd < s->ndom && !ok; ++dd) {
      rdom *d = &s->d[dd];
      int e[3];
      double xi[3];
      int inside = 1;
      if (d->V) {
        /* lowest element whose inverse map puts the point in [-1, 1]^3 */
        inside = 0;
        for (int ez = 0; ez < d->ne[2] && !inside; ++ez)
          for (int ey = 0; ey < d->ne[1] && !inside; ++ey)
            for (int ex = 0; ex < d->ne[0] && !inside; ++ex) {
              double V8[8][3], t[3];
              elem_vertices(d, ex, ey, ez, V8);
              if (tri_inverse(V8, xyz + 3 * r, t)) continue;
              if (fabs(t[0]) <= 1 + 1e-10 && fabs(t[1]) <= 1 + 1e-10 && fabs(t[2]) <= 1 + 1e-10) {
                inside = 1;
                e[0] = ex; e[1] = ey; e[2] = ez;
                xi[0] = t[0]; xi[1] = t[1]; xi[2] = t[2];
              }
            }
      }
      for (int a = 0; a < 3 && inside && !d->V; ++a) {
        int found = -1;
        for (int k = 0; k < d->ne[a]; ++k) {
          double t = 2.0 * (xyz[3 * r + a] - (d->x0[a] + k * d->h[a])) / d->h[a] - 1.0;
          if (t >= -1.0 - 1e-12 && t <= 1.0 + 1e-12) { found = k; xi[a] = t; break; }
        }
        if (found < 0) inside = 0; else e[a] = found;
      }
      if (inside) {
        ok = 1;
        s->rcv[r].dom = dd;
        double dummy[RMAXN];
        for (int a = 0; a < 3; ++a) {
          s->rcv[r].e[a] = e[a];
          pmdg_ref_lagrange(d->N, d->xg, xi[a], s->rcv[r].l[a], dummy);
        }
      }
    }
    if (!ok) return -1;
  }
  return 0;
}

static double receiver_value(const rsolver *s, int r, const double *p) {
  const rrecv *rc = &s->rcv[r];
  const rdom *d = &s->d[rc->dom];
  int N = d->N;
  double v = 0;
  for (int c = 0; c <= N; ++c)
    for (int b = 0; b <= N; ++b)
      for (int a = 0; a <= N; ++a)
        v += rc->l[0][a] * rc->l[1][b] * rc->l[2][c] *
             p[nidx(d, N * rc->e[0] + a, N * rc->e[1] + b, N * rc->e[2] + c)];
  return v;
}

/* ------------------------------------------------------------------ */
/* Perfectly matched layer (Sec. 2, eq. full_problem)                  */
/* ------------------------------------------------------------------ */

/* The damping profile of Sec. 2 at distance d into a layer of thickness ell:
 * zeta = zt (d / ell - sin(2 pi d / ell) / (2 pi)) on [0, ell], zero outside,
 * with zt = (c / ell) log(1 / R). */
static double pml_profile(double d, double ell, double c, double R) {
  if (!(ell > 0) || d <= 0) return 0.0;
  if (d > ell) d = ell;
  double zt = c / ell * log(1.0 / R);
  return zt * (d / ell - sin(2.0 * M_PI * d / ell) / (2.0 * M_PI));
}

/* Layers of thickness ell[2a] (low end of axis a) and ell[2a + 1] (high end)
 * inside domain dd, with reflection coefficient R: zeta_a at every node
 * coordinate of axis a is the profile of the layer the node lies in (the
 * distance counted from the layer's inner face), 0 elsewhere.  The interface
 * faces of two coupled domains (primary top, secondary bottom) carry no
 * layer.  Elements with zeta > 0 at one of their nodes hold the auxiliary
 * field Phi; psi is kept at every node.  Returns 0, or -1 on bad input. */
int pmdg_ref_set_pml(void *h, int dd, const double *ell, double R) {
  rsolver *s = (rsolver *)h;
  if (dd < 0 || dd >= s->ndom || !(R > 0 && R < 1)) return -1;
  if (s->d[dd].V) return -1; /* layers on trilinear hexahedra are not built */
  rdom *d = &s->d[dd];
  for (int a = 0; a < 3; ++a) {
    double L = d->h[a] * d->ne[a];
    if (ell[2 * a] < 0 || ell[2 * a + 1] < 0 || ell[2 * a] + ell[2 * a + 1] > L) return -1;
  }
  if (s->ndom == 2 && ((dd == 0 && ell[5] > 0) || (dd == 1 && ell[4] > 0))) return -1;
  for (int a = 0; a < 3; ++a) {
    free(s->pzeta[dd][a]);
    s->pzeta[dd][a] = (double *)calloc(d->nn[a], sizeof(double));
    double lo = d->x0[a] + ell[2 * a], hi = d->x0[a] + d->h[a] * d->ne[a] - ell[2 * a + 1];
    for (int i = 0; i < d->nn[a]; ++i) {
      double x = node_coord(d, a, i);
      double z = 0.0;
      if (ell[2 * a] > 0 && x < lo) z = pml_profile(lo - x, ell[2 * a], d->c, R);
      if (ell[2 * a + 1] > 0 && x > hi) z = pml_profile(x - hi, ell[2 * a + 1], d->c, R);
      s->pzeta[dd][a][i] = z;
    }
  }
  int N = d->N, n3 = (N + 1) * (N + 1) * (N + 1);
  long ne = (long)d->ne[0] * d->ne[1] * d->ne[2];
  free(s->eslot[dd]);
  s->eslot[dd] = (long *)malloc(sizeof(long) * ne);
  long nel = 0;
  for (int ez = 0; ez < d->ne[2]; ++ez)
    for (int ey = 0; ey < d->ne[1]; ++ey)
      for (int ex = 0; ex < d->ne[0]; ++ex) {
        int any = 0;
        for (int m = 0; m <= N; ++m)
          any |= s->pzeta[dd][0][N * ex + m] > 0 || s->pzeta[dd][1][N * ey + m] > 0 || s->pzeta[dd][2][N * ez + m] > 0;
        s->eslot[dd][ex + (long)d->ne[0] * (ey + (long)d->ne[1] * ez)] = any ? nel++ : -1;
      }
  s->nel[dd] = nel;
  free(s->Phi[dd]);
  s->Phi[dd] = (double *)calloc((size_t)(nel > 0 ? nel : 1) * 3 * n3, sizeof(double));
  if (!s->psi) s->psi = (double *)calloc(s->ntot, sizeof(double));
  s->pml_on[dd] = nel > 0;
  return 0;
}

/* zeta of axis a of domain dd at that axis's node coordinates (zeros without
 * a layer), out[nn[a]]. */
void pmdg_ref_pml_profile(void *h, int dd, int a, double *out) {
  rsolver *s = (rsolver *)h;
  for (int i = 0; i < s->d[dd].nn[a]; ++i) out[i] = s->pzeta[dd][a] ? s->pzeta[dd][a][i] : 0.0;
}

/* Element-local gradient (d/dx, d/dy, d/dz) of the nodal field u at the GLL
 * node (a, b, c) of element (ex, ey, ez): the derivative of the element's
 * polynomial, D by the metric 2 / h per axis. */
static void elem_grad(const rdom *d, const double *u, int ex, int ey, int ez, int a, int b, int c, double g[3]) {
  int N = d->N;
  g[0] = g[1] = g[2] = 0.0;
  for (int m = 0; m <= N; ++m) {
    g[0] += d->D[a][m] * u[nidx(d, N * ex + m, N * ey + b, N * ez + c)];
    g[1] += d->D[b][m] * u[nidx(d, N * ex + a, N * ey + m, N * ez + c)];
    g[2] += d->D[c][m] * u[nidx(d, N * ex + a, N * ey + b, N * ez + m)];
  }
  for (int k = 0; k < 3; ++k) g[k] *= 2.0 / d->h[k];
}

/* Phi_t = Z1 Phi + c^2 Z2 grad p + c^2 Z3 grad psi at every GLL node of every
 * layer element, Z1 = diag(-zeta_i), Z2 = diag(alpha - 2 zeta_i), Z3 =
 * diag(zeta_j zeta_k), by the trapezoidal rule over one step: p and psi
 * enter as the averages of their old and new values, so that
 * (1 + dt/2 zeta_i) Phi_i^{n+1} = (1 - dt/2 zeta_i) Phi_i^n
 *   + dt c^2 ((alpha - 2 zeta_i) d_i pbar + zeta_j zeta_k d_i psibar). */
static void pml_update_phi(rsolver *s, const double *pold, const double *pnew, const double *psiold,
                           const double *psinew) {
  double dt = s->dt;
  for (int dd = 0; dd < s->ndom; ++dd) {
    if (!s->pml_on[dd]) continue;
    rdom *d = &s->d[dd];
    int N = d->N, n1 = N + 1, n3 = n1 * n1 * n1;
    double c2 = d->c * d->c;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < (long)d->ne[0] * d->ne[1] * d->ne[2]; ++e) {
      long slot = s->eslot[dd][e];
      if (slot < 0) continue;
      int ex = (int)(e % d->ne[0]), ey = (int)((e / d->ne[0]) % d->ne[1]), ez = (int)(e / ((long)d->ne[0] * d->ne[1]));
      double *Ph = s->Phi[dd] + (size_t)slot * 3 * n3;
      for (int c = 0; c <= N; ++c)
        for (int b = 0; b <= N; ++b)
          for (int a = 0; a <= N; ++a) {
            double z[3] = {s->pzeta[dd][0][N * ex + a], s->pzeta[dd][1][N * ey + b], s->pzeta[dd][2][N * ez + c]};
            double al = z[0] + z[1] + z[2];
            double g0[3], g1[3], s0[3], s1[3];
            elem_grad(d, pold, ex, ey, ez, a, b, c, g0);
            elem_grad(d, pnew, ex, ey, ez, a, b, c, g1);
            elem_grad(d, psiold, ex, ey, ez, a, b, c, s0);
            elem_grad(d, psinew, ex, ey, ez, a, b, c, s1);
            int q = a + n1 * (b + n1 * c);
            for (int i = 0; i < 3; ++i) {
              double zjk = z[(i + 1) % 3] * z[(i + 2) % 3];
              double rhs = c2 * ((al - 2.0 * z[i]) * 0.5 * (g0[i] + g1[i]) + zjk * 0.5 * (s0[i] + s1[i]));
              double *ph = &Ph[i * n3 + q];
              *ph = ((1.0 - 0.5 * dt * z[i]) * *ph + dt * rhs) / (1.0 + 0.5 * dt * z[i]);
            }
          }
    }
  }
}

/* r += (Phi, grad v_i) over the layer elements (the weak form of
 * -div Phi with Phi.n = 0 on the outer boundary), GLL quadrature at the
 * element's nodes, where Phi is stored. */
static void pml_weak_div(const rsolver *s, double *r) {
  for (int dd = 0; dd < s->ndom; ++dd) {
    if (!s->pml_on[dd]) continue;
    const rdom *d = &s->d[dd];
    int N = d->N, n1 = N + 1, n3 = n1 * n1 * n1;
    double J = d->h[0] * d->h[1] * d->h[2] / 8.0;
    for (int colour = 0; colour < 8; ++colour) {
      int cx = colour & 1, cy = (colour >> 1) & 1, cz = (colour >> 2) & 1;
      int nx = (d->ne[0] - cx + 1) / 2, ny = (d->ne[1] - cy + 1) / 2, nz = (d->ne[2] - cz + 1) / 2;
      long tot = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
      for (long t = 0; t < tot; ++t) {
        int ex = cx + 2 * (int)(t % nx), ey = cy + 2 * (int)((t / nx) % ny), ez = cz + 2 * (int)(t / ((long)nx * ny));
        long slot = s->eslot[dd][ex + (long)d->ne[0] * (ey + (long)d->ne[1] * ez)];
        if (slot < 0) continue;
        const double *Ph = s->Phi[dd] + (size_t)slot * 3 * n3;
        for (int c = 0; c <= N; ++c)
          for (int b = 0; b <= N; ++b)
            for (int a = 0; a <= N; ++a) {
              int q = a + n1 * (b + n1 * c);
              double wq = d->wg[a] * d->wg[b] * d->wg[c] * J;
              for (int m = 0; m <= N; ++m) {
                r[nidx(d, N * ex + m, N * ey + b, N * ez + c)] += wq * (2.0 / d->h[0]) * d->D[a][m] * Ph[q];
                r[nidx(d, N * ex + a, N * ey + m, N * ez + c)] += wq * (2.0 / d->h[1]) * d->D[b][m] * Ph[n3 + q];
                r[nidx(d, N * ex + a, N * ey + b, N * ez + m)] += wq * (2.0 / d->h[2]) * d->D[c][m] * Ph[2 * n3 + q];
              }
            }
      }
    }
  }
}

/* alpha, beta, gamma of Sec. 2 at node (i, j, k) of domain dd. */
static void pml_coeffs(const rsolver *s, int dd, int i, int j, int k, double *al, double *be, double *ga) {
  double z0 = s->pzeta[dd][0][i], z1 = s->pzeta[dd][1][j], z2 = s->pzeta[dd][2][k];
  *al = z0 + z1 + z2;
  *be = z0 * z1 + z1 * z2 + z2 * z0;
  *ga = z0 * z1 * z2;
}

/* ------------------------------------------------------------------ */
/* State and time stepping (Sec. 3.1, Algorithm 1)                     */
/* ------------------------------------------------------------------ */

void pmdg_ref_set_state(void *h, const double *p, const double *pd, const double *pdd,
                        const double *q, const double *qd, const double *qdd, long nstep) {
  rsolver *s = (rsolver *)h;
  if (p) memcpy(s->p, p, sizeof(double) * s->ntot);
  if (pd) memcpy(s->pd, pd, sizeof(double) * s->ntot);
  if (pdd) memcpy(s->pdd, pdd, sizeof(double) * s->ntot);
  long nm = (long)s->Np * s->Nm;
  if (q && nm) memcpy(s->q, q, sizeof(double) * nm);
  if (qd && nm) memcpy(s->qd, qd, sizeof(double) * nm);
  if (qdd && nm) memcpy(s->qdd, qdd, sizeof(double) * nm);
  s->nstep = nstep;
}

void pmdg_ref_get_state(void *h, double *p, double *pd, double *pdd, double *q, double *qd, double *qdd, long *nstep) {
  rsolver *s = (rsolver *)h;
  if (p) memcpy(p, s->p, sizeof(double) * s->ntot);
  if (pd) memcpy(pd, s->pd, sizeof(double) * s->ntot);
  if (pdd) memcpy(pdd, s->pdd, sizeof(double) * s->ntot);
  long nm = (long)s->Np * s->Nm;
  if (q && nm) memcpy(q, s->q, sizeof(double) * nm);
  if (qd && nm) memcpy(qd, s->qd, sizeof(double) * nm);
  if (qdd && nm) memcpy(qdd, s->qdd, sizeof(double) * nm);
  if (nstep) *nstep = s->nstep;
}

static double voltage(const rsolver *s, int k, double t) {
  if (t > s->t_switch) {
    double v = 0;
    for (int m = 0; m < s->Nm; ++m) v += s->eta[(long)k * s->Nm + m] * s->q[(long)k * s->Nm + m];
    return v / s->cap;
  }
  return pmdg_ref_drive(s->amp[k], s->phase[k], s->freq, s->ncyc, s->envelope, t);
}

/* PMUT predictor, solve and corrector for all (k,m), sampling pressure p and
 * the voltage at time t (Algorithm 1, PMUT block; damping -2 zeta omega qdot
 * uses the predicted velocity). */
static void pmut_block(rsolver *s, const double *p, double t) {
  double dt = s->dt;
  long nm = (long)s->Np * s->Nm;
  for (long i = 0; i < nm; ++i) {
    s->q[i] += dt * s->qd[i] + 0.5 * dt * dt * s->qdd[i];
    s->qd[i] += 0.5 * dt * s->qdd[i];
  }
  for (int k = 0; k < s->Np; ++k) {
    double phi = voltage(s, k, t);
    for (int m = 0; m < s->Nm; ++m) {
      long i = (long)k * s->Nm + m;
      double g = 0;
      for (int n = 0; n < s->fn_cnt[k]; ++n)
        g += s->fn_wf[k][n] * s->fn_shape[k][(long)m * s->fn_cnt[k] + n] * p[s->fn_node[k][n]];
      double w = s->omega[i];
      s->qdd[i] = -w * w * s->q[i] - 2.0 * s->zeta[i] * w * s->qd[i] + s->sample_gain * g + s->eta[i] * phi;
    }
  }
  for (long i = 0; i < nm; ++i) s->qd[i] += 0.5 * dt * s->qdd[i];
}

/* Runs nsteps of Algorithm 1.  traces: [R x nsteps], column n holds the
 * receiver pressures at time (nstep0 + n + 1) dt.  Synchronised ordering by
 * default (PMUT block after the acoustic predictor, sampling p^{n+1} and
 * phi(t^{n+1})); the printed ordering (PMUT block first, sampling p^n and
 * phi(t^n)) when the literal switch is set. */
void pmdg_ref_step(void *h, int nsteps, double *traces) {
  rsolver *s = (rsolver *)h;
  long n = s->ntot;
  double dt = s->dt;
  int pml = s->psi && (s->pml_on[0] || s->pml_on[1]);
  double *f = (double *)malloc(sizeof(double) * n);
  double *Kp = (double *)malloc(sizeof(double) * n);
  double *pold = pml ? (double *)malloc(sizeof(double) * n) : NULL;
  double *psinew = pml ? (double *)malloc(sizeof(double) * n) : NULL;
  for (int it = 0; it < nsteps; ++it) {
    double tn = s->nstep * dt, tn1 = (s->nstep + 1) * dt;
    if (s->literal) pmut_block(s, s->p, tn);
    if (pml) memcpy(pold, s->p, sizeof(double) * n);
    /* acoustic predictor */
    for (long i = 0; i < n; ++i) {
      s->p[i] += dt * s->pd[i] + 0.5 * dt * dt * s->pdd[i];
      s->pd[i] += 0.5 * dt * s->pdd[i];
    }
    if (!s->literal) pmut_block(s, s->p, tn1);
    /* layer fields: psi_t = p by the trapezoidal rule, then Phi from the
     * averaged gradients of p and psi (Sec. 2, eq. full_problem, rows 2-3) */
    if (pml) {
      for (long i = 0; i < n; ++i) psinew[i] = s->psi[i] + 0.5 * dt * (pold[i] + s->p[i]);
      pml_update_phi(s, pold, s->p, s->psi, psinew);
      memcpy(s->psi, psinew, sizeof(double) * n);
    }
    /* acoustic solve: M pdd + C (pdot* + dt/2 pdd) = f(qdd) - K p, i.e. the
     * damping acts on the corrected velocity of the gamma = 1/2 Newmark
     * scheme: pdd = (f - K p - C pdot*) / (M + dt/2 C), with pdot* the
     * predicted velocity (C = 0 without absorbing faces).  The printed
     * solve takes C pdot* alone, which is stable only while
     * dt (M^{-1} C)_ii <= 2; GLL end weights exceed that at edges and
     * corners of absorbing faces at the configurations' CFL number.  In a
     * layer, the first row of eq. full_problem adds alpha M to C and
     * (Phi, grad v) + M (beta p + gamma psi) to K p. */
    memset(f, 0, sizeof(double) * n);
    for (int k = 0; k < s->Np; ++k)
      for (int m = 0; m < s->Nm; ++m) {
        double qdd = s->qdd[(long)k * s->Nm + m];
        for (int nn = 0; nn < s->fn_cnt[k]; ++nn)
          f[s->fn_node[k][nn]] += -s->kappa * qdd * s->fn_wf[k][nn] * s->fn_shape[k][(long)m * s->fn_cnt[k] + nn];
      }
    pmdg_ref_apply_K(h, s->p, Kp, 3);
    if (pml) pml_weak_div(s, Kp);
    for (int dd = 0; dd < s->ndom; ++dd) {
      const rdom *d = &s->d[dd];
      int lay = pml && s->pml_on[dd];
      for (int k = 0; k < d->nn[2]; ++k)
        for (int j = 0; j < d->nn[1]; ++j)
          for (int i0 = 0; i0 < d->nn[0]; ++i0) {
            long i = nidx(d, i0, j, k);
            double ci = s->cabs ? s->cabs[i] : 0.0, kp = Kp[i];
            if (lay) {
              double al, be, ga;
              pml_coeffs(s, dd, i0, j, k, &al, &be, &ga);
              ci += s->mass[i] * al;
              kp += s->mass[i] * (be * s->p[i] + ga * s->psi[i]);
            }
            double mi = s->abs_literal ? s->mass[i] : s->mass[i] + 0.5 * dt * ci;
            s->pdd[i] = (f[i] - kp - ci * s->pd[i]) / mi;
            s->pd[i] += 0.5 * dt * s->pdd[i];
          }
    }
    s->nstep += 1;
    if (traces)
      for (int r = 0; r < s->R; ++r) traces[(long)r * nsteps + it] = receiver_value(s, r, s->p);
  }
  free(f); free(Kp); free(pold); free(psinew);
}

/* Interpolated pressure at the receivers for an arbitrary field p. */
void pmdg_ref_sample_receivers(void *h, const double *p, double *out) {
  rsolver *s = (rsolver *)h;
  for (int r = 0; r < s->R; ++r) out[r] = receiver_value(s, r, p);
}


/* Time step from the CFL number (the paper only states dt <~ h_min, Sec.
 * 3.1): dt = cfl * min over domains of (smallest GLL node gap in physical
 * units) / c, with the gap h * min_i (x_{i+1} - x_i) / 2 over the shortest
 * element edge h of the domain. */
double pmdg_ref_cfl_dt(void *h, double cfl) {
  rsolver *s = (rsolver *)h;
  double best = INFINITY;
  for (int dd = 0; dd < s->ndom; ++dd) {
    const rdom *d = &s->d[dd];
    double gap = INFINITY, hm = INFINITY;
    for (int i = 0; i < d->N; ++i) if (d->xg[i + 1] - d->xg[i] < gap) gap = d->xg[i + 1] - d->xg[i];
    if (!d->V) {
      for (int a = 0; a < 3; ++a) if (d->h[a] < hm) hm = d->h[a];
    } else {
      /* shortest edge of any element */
      for (int ez = 0; ez < d->ne[2]; ++ez)
        for (int ey = 0; ey < d->ne[1]; ++ey)
          for (int ex = 0; ex < d->ne[0]; ++ex) {
            double V8[8][3];
            elem_vertices(d, ex, ey, ez, V8);
            for (int c = 0; c < 8; ++c)
              for (int a = 0; a < 3; ++a) {
                if ((c >> a) & 1) continue;
                int c2 = c | (1 << a);
                double l = sqrt((V8[c2][0] - V8[c][0]) * (V8[c2][0] - V8[c][0]) +
                                (V8[c2][1] - V8[c][1]) * (V8[c2][1] - V8[c][1]) +
                                (V8[c2][2] - V8[c][2]) * (V8[c2][2] - V8[c][2]));
                if (l < hm) hm = l;
              }
          }
    }
    double v = cfl * hm * gap * 0.5 / d->c;
    if (v < best) best = v;
  }
  return best;
}

/* Thread count of the oracle's OpenMP loops from here on (n >= 1). */
void pmdg_ref_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int pmdg_ref_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

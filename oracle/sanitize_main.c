/*
 * sanitize_main.c -- a driver that runs every entry of the FP64 CPU oracle
 * (oracle/pmdg_ref.c) once on small inputs, for a build with the host
 * address and undefined-behaviour sanitizers (tests/test_oracle_sanitizers.py).
 *
 * TEST INFRASTRUCTURE ONLY, like the oracle itself.  It covers: two bricks
 * with a non-nested interface, PMUTs, drive, receive mode, receivers,
 * stepping, the stability estimate, state get/set; one brick with absorbing
 * faces and a matched layer; one brick of trilinear hexahedra; and the face
 * matching of Algorithm 3.  Exit status 0 when every call returned what it
 * should; the sanitizers abort on their own findings.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void *pmdg_ref_create(int ndom, const double *dom_prm, double dt, double alpha);
void pmdg_ref_destroy(void *h);
long pmdg_ref_num_nodes(void *h);
double pmdg_ref_cfl_dt(void *h, double cfl);
void pmdg_ref_set_dt(void *h, double dt);
void pmdg_ref_coords(void *h, double *xyz);
void pmdg_ref_apply_K(void *h, const double *p, double *Kp, int which);
double pmdg_ref_lambda_max(void *h, int iters, unsigned seed);
int pmdg_ref_set_pmuts(void *h, int Np, const double *ctr, const double *rad, int Nm, const double *omega,
                       const double *zeta, const double *eta);
int pmdg_ref_pmut_nodes(void *h, int k, double *xyz);
int pmdg_ref_set_shape(void *h, int k, const double *shape);
void pmdg_ref_set_drive(void *h, const double *amp, const double *phase, double freq, double ncyc, int envelope);
void pmdg_ref_set_rx(void *h, double t_switch, double cap);
int pmdg_ref_set_receivers(void *h, int R, const double *xyz);
void pmdg_ref_step(void *h, int nsteps, double *traces);
void pmdg_ref_set_state(void *h, const double *p, const double *pd, const double *pdd, const double *q,
                        const double *qd, const double *qdd, long nstep);
void pmdg_ref_get_state(void *h, double *p, double *pd, double *pdd, double *q, double *qd, double *qdd,
                        long *nstep);
void pmdg_ref_set_absorbing(void *h, int dd, int faces);
int pmdg_ref_set_pml(void *h, int dd, const double *ell, double R);
int pmdg_ref_set_vertices(void *h, int dd, const double *V);
int pmdg_ref_match_faces(int nq, int nf, const double *fine_hex, const int *fine_face, int nc,
                         const double *coarse_hex, const int *coarse_face, double tol, double eps, int *elem,
                         double *xi);

static int fails = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                \
    }                                                         \
  } while (0)

static void brick(double *prm, double x0, double y0, double z0, double lx, double ly, double lz, int nx, int ny,
                  int nz, int N) {
  double v[12] = {x0, y0, z0, lx / nx, ly / ny, lz / nz, nx, ny, nz, N, 1.5, 1.0};
  memcpy(prm, v, sizeof(v));
}

static void pmuts_and_receivers(void *h, int R, const double *rxyz) {
  const double ctr[4] = {0.5, 0.5, 1.5, 1.0}, rad[2] = {0.4, 0.3};
  const double om[4] = {6.0, 13.0, 7.0, 15.0}, ze[4] = {0.01, 0.01, 0.02, 0.02}, et[4] = {1, 1, 1, 1};
  CHECK(pmdg_ref_set_pmuts(h, 2, ctr, rad, 2, om, ze, et) == 0);
  for (int k = 0; k < 2; ++k) {
    int n = pmdg_ref_pmut_nodes(h, k, NULL);
    CHECK(n > 0);
    double *xyz = malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    double *shape = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    pmdg_ref_pmut_nodes(h, k, xyz);
    for (int i = 0; i < n; ++i) {
      double r = hypot(xyz[3 * i] - ctr[2 * k], xyz[3 * i + 1] - ctr[2 * k + 1]);
      shape[i] = 1.0 - r / rad[k];
      shape[n + i] = cos(3.0 * r / rad[k]);
    }
    CHECK(pmdg_ref_set_shape(h, k, shape) == 0);
    free(xyz);
    free(shape);
  }
  const double amp[2] = {1.0, 0.5}, ph[2] = {0.0, 1.0};
  pmdg_ref_set_drive(h, amp, ph, 2.0, 3.0, 0);
  CHECK(pmdg_ref_set_receivers(h, R, rxyz) == 0);
}

int main(void) {
  /* two bricks, 4:3 interface */
  {
    double prm[24];
    brick(prm, 0, 0, 0, 2.0, 1.5, 0.5, 8, 6, 2, 3);
    brick(prm + 12, 0, 0, 0.5, 2.0, 1.5, 1.0, 6, 4, 3, 2);
    void *h = pmdg_ref_create(2, prm, 1.0, 2.0);
    CHECK(h != NULL);
    double dt = pmdg_ref_cfl_dt(h, 0.3);
    pmdg_ref_set_dt(h, dt);
    const double rx[9] = {0.3, 0.4, 0.2, 1.0, 0.75, 0.5, 1.7, 1.2, 1.3};
    pmuts_and_receivers(h, 3, rx);
    pmdg_ref_set_rx(h, 20 * dt, 0.2);
    long n = pmdg_ref_num_nodes(h);
    double *xyz = malloc(sizeof(double) * 3 * n), *p = malloc(sizeof(double) * n), *Kp = malloc(sizeof(double) * n);
    pmdg_ref_coords(h, xyz);
    for (long i = 0; i < n; ++i) p[i] = sin(xyz[3 * i]) * cos(2 * xyz[3 * i + 2]);
    pmdg_ref_apply_K(h, p, Kp, 3);
    CHECK(isfinite(Kp[n / 2]));
    double lam = pmdg_ref_lambda_max(h, 30, 1);
    CHECK(lam > 0 && dt * dt * lam < 4.0);
    double tr[3 * 40];
    pmdg_ref_step(h, 40, tr);
    for (int i = 0; i < 120; ++i) CHECK(isfinite(tr[i]));
    double *pd = malloc(sizeof(double) * n), *pdd = malloc(sizeof(double) * n);
    double q[4], qd[4], qdd[4];
    long ns;
    pmdg_ref_get_state(h, p, pd, pdd, q, qd, qdd, &ns);
    CHECK(ns == 40);
    pmdg_ref_set_state(h, p, pd, pdd, q, qd, qdd, ns);
    pmdg_ref_step(h, 5, tr);
    free(xyz); free(p); free(Kp); free(pd); free(pdd);
    pmdg_ref_destroy(h);
  }
  /* one brick: absorbing faces and a matched layer */
  {
    double prm[12];
    brick(prm, 0, 0, 0, 2.0, 2.0, 2.0, 6, 6, 6, 3);
    void *h = pmdg_ref_create(1, prm, 1.0, 2.0);
    pmdg_ref_set_dt(h, pmdg_ref_cfl_dt(h, 0.3));
    pmdg_ref_set_absorbing(h, 0, 0x3e);
    const double ell[6] = {0.5, 0.5, 0.5, 0.5, 0.0, 0.5};
    CHECK(pmdg_ref_set_pml(h, 0, ell, 1e-4) == 0);
    const double bad[6] = {1.5, 1.5, 0, 0, 0, 0};
    CHECK(pmdg_ref_set_pml(h, 0, bad, 1e-4) != 0);
    const double rx[3] = {1.0, 1.0, 1.0};
    pmuts_and_receivers(h, 1, rx);
    double tr[30];
    pmdg_ref_step(h, 30, tr);
    for (int i = 0; i < 30; ++i) CHECK(isfinite(tr[i]));
    pmdg_ref_destroy(h);
  }
  /* one brick of trilinear hexahedra */
  {
    double prm[12];
    const int ne[3] = {4, 3, 2};
    brick(prm, 0, 0, 0, 2.0, 1.5, 1.0, ne[0], ne[1], ne[2], 4);
    void *h = pmdg_ref_create(1, prm, 1.0, 2.0);
    const int nv = (ne[0] + 1) * (ne[1] + 1) * (ne[2] + 1);
    double *V = malloc(sizeof(double) * 3 * nv);
    int v = 0;
    for (int k = 0; k <= ne[2]; ++k)
      for (int j = 0; j <= ne[1]; ++j)
        for (int i = 0; i <= ne[0]; ++i, ++v) {
          double x = 0.5 * i, y = 0.5 * j, z = 0.5 * k;
          int inner = i > 0 && i < ne[0] && j > 0 && j < ne[1] && k > 0 && k < ne[2];
          V[3 * v] = x + (inner ? 0.07 * sin(3.0 * v) : 0.0);
          V[3 * v + 1] = y + (inner ? 0.07 * cos(5.0 * v) : 0.0);
          V[3 * v + 2] = z + (inner ? 0.05 * sin(7.0 * v) : 0.0);
        }
    CHECK(pmdg_ref_set_vertices(h, 0, V) == 0);
    pmdg_ref_set_dt(h, pmdg_ref_cfl_dt(h, 0.3));
    const double rx[6] = {0.7, 0.6, 0.4, 1.3, 1.1, 0.8};
    pmuts_and_receivers(h, 2, rx);
    double tr[2 * 25];
    pmdg_ref_step(h, 25, tr);
    for (int i = 0; i < 50; ++i) CHECK(isfinite(tr[i]));
    /* a folded element is refused */
    double *W = malloc(sizeof(double) * 3 * nv);
    memcpy(W, V, sizeof(double) * 3 * nv);
    W[3 * 1 + 2] = 2.0;
    CHECK(pmdg_ref_set_vertices(h, 0, W) == -2);
    free(V); free(W);
    pmdg_ref_destroy(h);
  }
  /* Algorithm 3: a 3 x 3 fine layer against a 2 x 2 coarse layer */
  {
    double fine[9 * 24], coarse[4 * 24];
    int ff[9], cf[4];
    for (int e = 0; e < 9; ++e) {
      int ex = e % 3, ey = e / 3;
      for (int c = 0; c < 8; ++c) {
        fine[e * 24 + 3 * c] = (ex + (c & 1)) / 3.0;
        fine[e * 24 + 3 * c + 1] = (ey + ((c >> 1) & 1)) / 3.0;
        fine[e * 24 + 3 * c + 2] = ((c >> 2) & 1) - 1.0;
      }
      ff[e] = 5;
    }
    for (int e = 0; e < 4; ++e) {
      int ex = e % 2, ey = e / 2;
      for (int c = 0; c < 8; ++c) {
        coarse[e * 24 + 3 * c] = (ex + (c & 1)) / 2.0;
        coarse[e * 24 + 3 * c + 1] = (ey + ((c >> 1) & 1)) / 2.0;
        coarse[e * 24 + 3 * c + 2] = 0.5 * ((c >> 2) & 1);
      }
      cf[e] = 4;
    }
    int elem[9 * 16];
    double xi[9 * 16 * 3];
    CHECK(pmdg_ref_match_faces(4, 9, fine, ff, 4, coarse, cf, 1e-6, 1e-9, elem, xi) == 0);
    for (int q = 0; q < 9 * 16; ++q) CHECK(elem[q] >= 0 && elem[q] < 4);
    CHECK(pmdg_ref_match_faces(0, 9, fine, ff, 4, coarse, cf, 1e-6, 1e-9, elem, xi) == -1);
  }
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("oracle sanitizer driver: all entries ran\n");
  return 0;
}

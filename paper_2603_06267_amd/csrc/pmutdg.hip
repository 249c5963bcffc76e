// libpmutdg: host side of the C ABI (include/pmutdg.h).
//
// Builds the operator tables of the explicit step on the host once (long
// double), uploads them into a caller-owned device workspace and enqueues
// the per-step kernels of pmutdg_kernels.hip, optionally as hipGraphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <queue>
#include <string>
#include <thread>
#include <vector>

#include "pmutdg_internal.h"
#include "pmutdg.h"

using namespace pmdg;
typedef long double ld;

static thread_local std::string g_err;

static pmdg_status fail(pmdg_status s, const std::string& m) {
  g_err = m;
  return s;
}

namespace pmdg {
void set_last_error(const std::string& m) { g_err = m; }
}  // namespace pmdg

#define HIPCHK(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(PMDG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------------
// 1D spectral-element rules (Sec. 3: Lagrange basis on GLL nodes, reduced
// integration of the mass form; Sec. 5: Gauss-Legendre points on the finer
// interface face).
// ------------------------------------------------------------------------
static void leg(int n, ld t, ld& P, ld& Pm1, ld& dP) {
  // P_n, P_{n-1} and P_n' by the Bonnet recurrence
  ld a = 1, b = t;
  if (n == 0) { P = 1; Pm1 = 0; dP = 0; return; }
  for (int k = 2; k <= n; ++k) {
    ld c = ((2 * k - 1) * t * b - (k - 1) * a) / k;
    a = b;
    b = c;
  }
  P = b;
  Pm1 = a;
  dP = (std::fabs(t) < 1) ? n * (a - t * b) / (1 - t * t) : (t > 0 ? 1 : (n % 2 ? 1 : -1)) * 0.5L * n * (n + 1);
}

struct Rule1D {
  int N = 0;
  std::vector<ld> x, w, lam;  // nodes, weights, barycentric weights
  std::vector<ld> D;          // D[i*(N+1)+j] = l_j'(x_i)
};

// GLL: interior nodes are the zeros of P_{N-1}(t) - t P_N(t), which is
// proportional to (1 - t^2) P_N'(t).
static Rule1D gll_rule(int N) {
  Rule1D r;
  r.N = N;
  r.x.assign(N + 1, 0);
  r.w.assign(N + 1, 0);
  r.x[0] = -1;
  r.x[N] = 1;
  for (int j = 1; j < N; ++j) {
    ld t = -std::cos(M_PI * (ld)j / N);
    for (int it = 0; it < 200; ++it) {
      ld P, Pm1, dP, Q, Qm1, dQ;
      leg(N, t, P, Pm1, dP);
      leg(N - 1, t, Q, Qm1, dQ);
      const ld f = Q - t * P, df = dQ - P - t * dP;
      const ld step = f / df;
      t -= step;
      if (std::fabs(step) < 1e-19L) break;
    }
    r.x[j] = t;
  }
  std::sort(r.x.begin(), r.x.end());
  std::vector<ld> PN(N + 1);
  for (int j = 0; j <= N; ++j) {
    ld P, Pm1, dP;
    leg(N, r.x[j], P, Pm1, dP);
    PN[j] = P;
    r.w[j] = 2.0L / (N * (N + 1.0L) * P * P);
  }
  r.lam.assign(N + 1, 1);
  for (int j = 0; j <= N; ++j)
    for (int m = 0; m <= N; ++m)
      if (m != j) r.lam[j] /= (r.x[j] - r.x[m]);
  r.D.assign((N + 1) * (N + 1), 0);
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N; ++j)
      if (i != j) r.D[i * (N + 1) + j] = PN[i] / (PN[j] * (r.x[i] - r.x[j]));
  r.D[0] = -0.25L * N * (N + 1);
  r.D[N * (N + 1) + N] = 0.25L * N * (N + 1);
  return r;
}

static void gl_rule(int n, std::vector<ld>& x, std::vector<ld>& w) {
  x.assign(n, 0);
  w.assign(n, 0);
  for (int j = 0; j < n; ++j) {
    ld t = -std::cos(M_PI * (4.0L * j + 3.0L) / (4.0L * n + 2.0L));
    ld P, Pm1, dP;
    for (int it = 0; it < 200; ++it) {
      leg(n, t, P, Pm1, dP);
      const ld step = P / dP;
      t -= step;
      if (std::fabs(step) < 1e-19L) break;
    }
    leg(n, t, P, Pm1, dP);
    x[j] = t;
    w[j] = 2.0L / ((1 - t * t) * dP * dP);
  }
}

// Lagrange basis values at t by the barycentric formula.
static void bary_eval(const Rule1D& r, ld t, ld* v) {
  const int n = r.N + 1;
  for (int j = 0; j < n; ++j)
    if (std::fabs(t - r.x[j]) < 1e-16L) {
      for (int k = 0; k < n; ++k) v[k] = (k == j);
      return;
    }
  ld den = 0;
  for (int j = 0; j < n; ++j) den += r.lam[j] / (t - r.x[j]);
  for (int j = 0; j < n; ++j) v[j] = r.lam[j] / (t - r.x[j]) / den;
}

// ------------------------------------------------------------------------
// Solver object
// ------------------------------------------------------------------------
struct Brick {
  double x0[3], h[3];
  int ne[3], N, nn[3];
  long plane, nnodes;   // compact (host / ABI) layout
  int px;               // device row pitch: nn[0] rounded up to a multiple of 64 nodes
  long pplane, pnodes;  // device plane stride and nodes per scenario
  double c, rho;
  Rule1D rule;
  std::vector<double> tap[3];   // [nn][2N]
  std::vector<double> minv[3];  // [nn]
  std::vector<double> mass1[3]; // [nn] assembled 1D lumped mass
  double lam1[3];               // largest eigenvalue of M_d^{-1} K_d
  std::vector<double> ctap[3];  // [N+2][2N] rows by node class (see StiffArgs)
  std::vector<double> cmin[3];  // [N+2]
  int absorbing = 0;            // outer faces with the first-order absorbing condition (bit 2a / 2a+1: low / high end of axis a)
  // perfectly matched layer: zeta per axis at the node coordinates, the
  // layer's elements (slot per element, -1 outside) and their nodes
  bool pml = false;
  std::vector<double> pzeta[3];
  std::vector<int> eslot, pel, pnode;
  // trilinear hexahedra: element vertices [(ne0+1)(ne1+1)(ne2+1)][3] (empty
  // for an axis-aligned brick), the inverse assembled lumped mass in the
  // padded device layout, and each element's corner offsets from corner 0
  std::vector<double> V, hminv, hvert;
  bool mapped() const { return !V.empty(); }
  double coord(int axis, int i) const {
    const int e = i / N, a = i % N;
    return x0[axis] + h[axis] * (e + 0.5 * ((double)rule.x[a] + 1.0));
  }
};

struct Seg {
  size_t off = 0, bytes = 0;
};

struct pmdg_solver {
  pmdg_problem pr;
  int ndom = 1, S = 1, prec = 32;
  long cap = 1;
  double dt = 0;
  double lam_max = 0;  // largest eigenvalue of M^{-1} K (coupled operator for two bricks)
  Brick b[2];
  // interface
  int Nq = 0;
  int xl_max = 0;  // most fine Gauss points inside one coarse element along x
  std::vector<double> Lq, wJ, xw, yw;
  std::vector<int> xcx, ycx, xl_off, xl, yl_off, yl;
  double gamma = 0, dz0[kMaxOrder + 1] = {0}, dz1[kMaxOrder + 1] = {0};
  // PMUTs
  int Np = 0, Nm = 0;
  std::vector<double> ctr, rad, omega, zeta, eta;
  std::vector<int> pm_off, pm_node;
  std::vector<double> pm_wf, pm_B;
  std::vector<char> shape_set;
  // drive
  std::vector<double> amp, phase, freq;
  double ncyc = 3, t_switch = INFINITY, rx_cap = 1;
  int envelope = 0;
  // drive tables as last uploaded (valid once bound: restart uploads them
  // again without recomputing them)
  std::vector<double> dA_h, car_h;
  bool drive_cached = false;
  // receivers
  int R = 0;
  std::vector<int> r_dom;
  std::vector<long> r_base;
  std::vector<double> r_w;
  // device
  bool bound = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_need = 0;  // bytes the layout uses (zeroed by bind and restart)
  std::map<std::string, Seg> seg;
  long steps_done = 0;
  // options
  int use_graph = 1, rows = 0, zchunk = -1, graph_chunk = 64, timing = 0;  // rows 0, zchunk -1: automatic
  int rows1 = 0, zchunk1 = -1;  // secondary brick's tile (0 / -1: as the primary's)
  int waves = 4;                // waves per stiffness workgroup
  int depth = 2;                // stiffness prefetch distance in planes
  int tblock = 1;               // steps per stiffness pass of the primary (1, or 2 for FP32)
  int tblock1 = 0;              // same for the secondary (0: as the primary)
  int overlap = 0;              // PMUT face work alongside the secondary's stiffness
  int resident = 1;             // small single-brick FP32 solvers: whole steps with p in LDS (0: never)
  int batches = 0;              // batches holding this solver (their tile layout is fixed)
  int static_dev = -1;          // device whose library-held workspace this solver is bound to, or -1
  std::map<int, hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;
  // side stream and events for running the PMUT part of the face kernel
  // alongside the secondary brick's stiffness launch
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double ktimes[3] = {0, 0, 0};
};

static int nfine(const pmdg_solver* s) { return s->b[0].ne[0] * s->b[0].ne[1]; }
static int ncoarse(const pmdg_solver* s) { return s->ndom > 1 ? s->b[1].ne[0] * s->b[1].ne[1] : 0; }
static long face0(const pmdg_solver* s) { return (long)s->b[0].nn[0] * s->b[0].nn[1]; }
static long face1(const pmdg_solver* s) { return s->ndom > 1 ? (long)s->b[1].nn[0] * s->b[1].nn[1] : 0; }

static int setup_brick(Brick& B, const pmdg_brick& d, std::string& err) {
  B.N = d.order;
  if (B.N < 1 || B.N > kMaxOrder) { err = "order must be in 1..8"; return -1; }
  if (!(d.c > 0) || !(d.rho > 0)) { err = "c and rho must be positive"; return -1; }
  B.c = d.c;
  B.rho = d.rho;
  for (int a = 0; a < 3; ++a) {
    if (d.ne[a] < 1 || !(d.x1[a] > d.x0[a])) { err = "bad brick extent or element count"; return -1; }
    B.x0[a] = d.x0[a];
    B.ne[a] = d.ne[a];
    B.h[a] = (d.x1[a] - d.x0[a]) / d.ne[a];
    B.nn[a] = B.N * B.ne[a] + 1;
  }
  B.plane = (long)B.nn[0] * B.nn[1];
  B.nnodes = B.plane * B.nn[2];
  B.px = (B.nn[0] + 63) / 64 * 64;
  B.pplane = (long)B.px * B.nn[1];
  B.pnodes = B.pplane * B.nn[2];
  if (B.pnodes > (1L << 31) - 1024) { err = "brick too large"; return -1; }
  // the stiffness kernel stores relative to one plane with 32-bit byte offsets
  if (B.pplane * (long)sizeof(double) >= (1L << 31)) { err = "brick plane too large"; return -1; }
  B.rule = gll_rule(B.N);
  const int N = B.N, n1 = N + 1, NT = 2 * N;
  for (int a = 0; a < 3; ++a) {
    const int n = B.nn[a];
    const ld h = B.h[a];
    // local 1D stiffness (2/h) D^T W D and assembled operator M^{-1} K
    std::vector<ld> kl(n1 * n1, 0);
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n1; ++j) {
        ld sacc = 0;
        for (int q = 0; q < n1; ++q) sacc += B.rule.w[q] * B.rule.D[q * n1 + i] * B.rule.D[q * n1 + j];
        kl[i * n1 + j] = 2.0L / h * sacc;
      }
    std::vector<ld> M(n, 0);
    std::vector<ld> K((size_t)n * (NT + 1), 0);  // band storage K[i][t + N]
    for (int e = 0; e < B.ne[a]; ++e)
      for (int i = 0; i < n1; ++i) {
        M[N * e + i] += 0.5L * h * B.rule.w[i];
        for (int j = 0; j < n1; ++j) K[(size_t)(N * e + i) * (NT + 1) + (j - i + N)] += kl[i * n1 + j];
      }
    B.tap[a].assign((size_t)n * NT, 0);
    B.minv[a].assign(n, 0);
    B.mass1[a].assign(n, 0);
    for (int i = 0; i < n; ++i) {
      B.minv[a][i] = (double)(1.0L / M[i]);
      B.mass1[a][i] = (double)M[i];
      for (int t = -N; t <= N; ++t) {
        if (t == 0) continue;
        const int slot = t < 0 ? (t + N) : (N + t - 1);
        const bool ok = i + t >= 0 && i + t < n;
        B.tap[a][(size_t)i * NT + slot] = ok ? (double)(K[(size_t)i * (NT + 1) + (t + N)] / M[i]) : 0.0;
      }
    }
    // largest eigenvalue of M^{-1} K (similar to M^{-1/2} K M^{-1/2}) by power iteration
    std::vector<ld> v(n), wv(n);
    for (int i = 0; i < n; ++i) v[i] = 1.0L + 0.37L * std::sin(1.3L * i) * ((i % 2) ? 1 : -1);
    ld lam = 0;
    for (int it = 0; it < 4000; ++it) {
      ld nrm = 0;
      for (int i = 0; i < n; ++i) {
        ld acc = 0;
        for (int t = -N; t <= N; ++t)
          if (i + t >= 0 && i + t < n) acc += K[(size_t)i * (NT + 1) + (t + N)] / std::sqrt(M[i] * M[i + t]) * v[i + t];
        wv[i] = acc;
        nrm += acc * acc;
      }
      nrm = std::sqrt(nrm);
      ld vv = 0, vw = 0;
      for (int i = 0; i < n; ++i) { vv += v[i] * v[i]; vw += v[i] * wv[i]; }
      lam = vw / vv;
      for (int i = 0; i < n; ++i) v[i] = wv[i] / nrm;
    }
    B.lam1[a] = (double)lam;
    // rows by node class: interior i mod N, first node, last node
    B.ctap[a].assign((size_t)(N + 2) * NT, 0.0);
    B.cmin[a].assign(N + 2, 0.0);
    auto rep = [&](int cls) -> int {
      if (cls == N) return 0;
      if (cls == N + 1) return n - 1;
      if (cls == 0) return n > N + 1 ? N : -1;
      return cls;
    };
    for (int cls = 0; cls < N + 2; ++cls) {
      const int i = rep(cls);
      if (i < 0) continue;
      for (int t = 0; t < NT; ++t) B.ctap[a][(size_t)cls * NT + t] = B.tap[a][(size_t)i * NT + t];
      B.cmin[a][cls] = B.minv[a][i];
    }
    for (int i = 0; i < n; ++i) {
      const int cls = i == 0 ? N : (i == n - 1 ? N + 1 : i % N);
      for (int t = 0; t < NT; ++t)
        if (std::fabs(B.ctap[a][(size_t)cls * NT + t] - B.tap[a][(size_t)i * NT + t]) >
            1e-12 * std::fabs(B.tap[a][(size_t)i * NT + t]) + 1e-300) {
          err = "internal: 1D operator rows are not periodic by node class";
          return -1;
        }
    }
  }
  return 0;
}

// Interface quadrature-point list (Sec. 5): Gauss-Legendre points of every
// fine face (the primary's top element faces) pushed forward with the fine
// map and pulled back into the lowest-index coarse element containing them.
// On bricks both maps are affine and separable, so the list factors into an
// x table and a y table.
static int setup_interface(pmdg_solver* s, std::string& err) {
  Brick &F = s->b[0], &C = s->b[1];
  const double ztop = F.x0[2] + F.ne[2] * F.h[2];
  const double tolz = 1e-9 * std::min(F.h[2], C.h[2]);
  if (std::fabs(ztop - C.x0[2]) > tolz) { err = "secondary bottom face must be the primary top face"; return -1; }
  for (int a = 0; a < 2; ++a) {
    const double l0 = F.ne[a] * F.h[a], l1 = C.ne[a] * C.h[a];
    if (std::fabs(F.x0[a] - C.x0[a]) > 1e-9 * l0 || std::fabs(l0 - l1) > 1e-9 * l0) {
      err = "primary and secondary must share the same lateral extent";
      return -1;
    }
  }
  const int N0 = F.N, N1 = C.N, n0 = N0 + 1, n1 = N1 + 1;
  if (std::max(N0, N1) > kMaxOrder - 1) { err = "orders of two coupled bricks must be <= 7"; return -1; }
  for (int a = 0; a < 2; ++a)
    if (F.h[a] > C.h[a] * (1 + 1e-12)) { err = "the primary (fine) brick's faces must not be larger than the secondary's"; return -1; }
  s->Nq = std::max(N0, N1) + 1;
  const int Nq = s->Nq;
  std::vector<ld> gx, gw;
  gl_rule(Nq, gx, gw);
  s->Lq.assign(Nq * n0, 0);
  for (int q = 0; q < Nq; ++q) {
    ld v[kMaxOrder + 1];
    bary_eval(F.rule, gx[q], v);
    for (int a = 0; a < n0; ++a) s->Lq[q * n0 + a] = (double)v[a];
  }
  s->wJ.assign(Nq * Nq, 0);
  for (int qb = 0; qb < Nq; ++qb)
    for (int qa = 0; qa < Nq; ++qa) s->wJ[qb * Nq + qa] = (double)(gw[qa] * gw[qb]) * 0.25 * F.h[0] * F.h[1];
  for (int axis = 0; axis < 2; ++axis) {
    std::vector<int>& cx = axis == 0 ? s->xcx : s->ycx;
    std::vector<double>& cw = axis == 0 ? s->xw : s->yw;
    std::vector<int>& off = axis == 0 ? s->xl_off : s->yl_off;
    std::vector<int>& lst = axis == 0 ? s->xl : s->yl;
    const int nef = F.ne[axis], nec = C.ne[axis];
    cx.assign(nef * Nq, 0);
    cw.assign((size_t)nef * Nq * n1, 0);
    std::vector<std::vector<int>> buckets(nec);
    for (int e = 0; e < nef; ++e)
      for (int q = 0; q < Nq; ++q) {
        const ld xq = F.x0[axis] + F.h[axis] * (e + 0.5L * (gx[q] + 1));
        int found = -1;
        ld xi = 0;
        for (int k = 0; k < nec; ++k) {
          const ld r = 2 * (xq - (C.x0[axis] + k * (ld)C.h[axis])) / C.h[axis] - 1;
          if (r >= -1 - 1e-12L && r <= 1 + 1e-12L) { found = k; xi = r; break; }
        }
        if (found < 0) { err = "interface point outside the coarse face"; return -1; }
        cx[e * Nq + q] = found;
        ld v[kMaxOrder + 1];
        bary_eval(C.rule, xi, v);
        for (int a = 0; a < n1; ++a) cw[(size_t)(e * Nq + q) * n1 + a] = (double)v[a];
        buckets[found].push_back(e * Nq + q);
      }
    off.assign(nec + 1, 0);
    lst.clear();
    for (int k = 0; k < nec; ++k) {
      off[k] = (int)lst.size();
      lst.insert(lst.end(), buckets[k].begin(), buckets[k].end());
    }
    off[nec] = (int)lst.size();
    for (int k = 0; k < nec; ++k) {
      if (off[k + 1] - off[k] > 64) { err = "more than 64 fine Gauss points per coarse element along an axis"; return -1; }
      if (axis == 0) s->xl_max = std::max(s->xl_max, off[k + 1] - off[k]);
    }
  }
  const double cbar = 2.0 * F.c * C.c / (F.c + C.c);
  const int nmax = std::max(N0, N1);
  s->gamma = s->pr.penalty_alpha * cbar * cbar * nmax * nmax / std::min(F.h[2], C.h[2]);
  for (int c = 0; c < n0; ++c) s->dz0[c] = (double)(2.0L / F.h[2] * F.rule.D[N0 * n0 + c]);
  for (int c = 0; c < n1; ++c) s->dz1[c] = (double)(2.0L / C.h[2] * C.rule.D[0 * n1 + c]);
  return 0;
}

// ------------------------------------------------------------------------
// Explicit stability of the coupled operator (Sec. 3.1: the leapfrog needs
// dt^2 lambda_max(M^{-1} K) < 4).  The SIPG penalty gamma_F of Sec. 3 lifts
// the largest eigenvalue well above that of either brick's volume operator
// (a factor of about 1.7 at alpha = 2 and 7 at alpha = 10 for the orders
// used here).  Those modes live at the element scale next to Gamma_I, so the
// eigenvalue is computed on a patch of the two bricks with the same element
// sizes, orders, materials and penalty: laterally the shortest run of coarse
// elements that ends on a fine element edge, repeated to at least three
// coarse elements where the brick has them, and up to three element layers
// on each side of Gamma_I (rigid patch walls).  Lanczos iteration in the
// M-inner product on the patch operator (volume stiffness by the assembled
// 1D rows, interface terms of eq. Wf_2 at the fine-face Gauss points).
// ------------------------------------------------------------------------
static long bnode(const Brick& B, int i, int j, int k) { return ((long)k * B.nn[1] + j) * B.nn[0] + i; }

// y = M^{-1} K v on the two bricks of s (host tables of setup_brick and
// setup_interface); v and y hold the primary's nodes, then the secondary's.
static void coupled_apply(const pmdg_solver* s, const std::vector<double>& v, std::vector<double>& y) {
  const long off1 = s->b[0].nnodes;
  std::fill(y.begin(), y.end(), 0.0);
  std::vector<double> r(y.size(), 0.0);
  for (int d = 0; d < s->ndom; ++d) {
    const Brick& B = s->b[d];
    const int N = B.N, NT = 2 * N;
    const double c2 = B.c * B.c;
    const long o = d ? off1 : 0;
    for (int k = 0; k < B.nn[2]; ++k)
      for (int j = 0; j < B.nn[1]; ++j)
        for (int i = 0; i < B.nn[0]; ++i) {
          const int ix[3] = {i, j, k};
          const long me = o + bnode(B, i, j, k);
          double acc = 0;
          for (int a = 0; a < 3; ++a)
            for (int t = -N; t <= N; ++t) {
              if (t == 0 || ix[a] + t < 0 || ix[a] + t >= B.nn[a]) continue;
              int jx[3] = {i, j, k};
              jx[a] += t;
              const int slot = t < 0 ? (t + N) : (N + t - 1);
              acc += B.tap[a][(size_t)ix[a] * NT + slot] * (v[o + bnode(B, jx[0], jx[1], jx[2])] - v[me]);
            }
          y[me] = c2 * acc;
        }
  }
  if (s->ndom < 2) return;
  const Brick &F = s->b[0], &C = s->b[1];
  const int N0 = F.N, N1 = C.N, n0 = N0 + 1, n1 = N1 + 1, Nq = s->Nq;
  const double c0 = F.c * F.c, c1 = C.c * C.c, g = s->gamma;
  const int kt0 = F.nn[2] - 1;
  for (int ey = 0; ey < F.ne[1]; ++ey)
    for (int ex = 0; ex < F.ne[0]; ++ex)
      for (int qb = 0; qb < Nq; ++qb)
        for (int qa = 0; qa < Nq; ++qa) {
          const int px = ex * Nq + qa, py = ey * Nq + qb;
          const int kx = s->xcx[px], ky = s->ycx[py];
          const double* wx = &s->xw[(size_t)px * n1];
          const double* wy = &s->yw[(size_t)py * n1];
          const double* lx = &s->Lq[qa * n0];
          const double* ly = &s->Lq[qb * n0];
          double pp = 0, dp = 0, pm = 0, dm = 0;
          for (int b = 0; b < n0; ++b)
            for (int a = 0; a < n0; ++a) {
              const double w = lx[a] * ly[b];
              const int i = N0 * ex + a, j = N0 * ey + b;
              pp += w * v[bnode(F, i, j, kt0)];
              for (int c = 0; c < n0; ++c) dp += w * s->dz0[c] * v[bnode(F, i, j, kt0 - N0 + c)];
            }
          for (int b = 0; b < n1; ++b)
            for (int a = 0; a < n1; ++a) {
              const double w = wx[a] * wy[b];
              const int i = N1 * kx + a, j = N1 * ky + b;
              pm += w * v[off1 + bnode(C, i, j, 0)];
              for (int c = 0; c < n1; ++c) dm += w * s->dz1[c] * v[off1 + bnode(C, i, j, c)];
            }
          const double W = s->wJ[qb * Nq + qa];
          const double jump = pp - pm, avg = 0.5 * (c0 * dp + c1 * dm);
          for (int b = 0; b < n0; ++b)
            for (int a = 0; a < n0; ++a) {
              const double w = W * lx[a] * ly[b];
              const int i = N0 * ex + a, j = N0 * ey + b;
              r[bnode(F, i, j, kt0)] += w * (g * jump - avg);
              for (int c = 0; c < n0; ++c) r[bnode(F, i, j, kt0 - N0 + c)] -= w * 0.5 * c0 * jump * s->dz0[c];
            }
          for (int b = 0; b < n1; ++b)
            for (int a = 0; a < n1; ++a) {
              const double w = W * wx[a] * wy[b];
              const int i = N1 * kx + a, j = N1 * ky + b;
              r[off1 + bnode(C, i, j, 0)] += w * (avg - g * jump);
              for (int c = 0; c < n1; ++c) r[off1 + bnode(C, i, j, c)] -= w * 0.5 * c1 * jump * s->dz1[c];
            }
        }
  for (int d = 0; d < 2; ++d) {
    const Brick& B = s->b[d];
    const long o = d ? off1 : 0;
    for (int k = 0; k < B.nn[2]; ++k)
      for (int j = 0; j < B.nn[1]; ++j)
        for (int i = 0; i < B.nn[0]; ++i) {
          const long me = o + bnode(B, i, j, k);
          y[me] += r[me] / (B.mass1[0][i] * B.mass1[1][j] * B.mass1[2][k]);
        }
  }
}

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal al and
// off-diagonal be, by Sturm-sequence bisection.
static double tridiag_max_eig(const std::vector<double>& al, const std::vector<double>& be) {
  const int m = (int)al.size();
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(be[i - 1]) : 0) + (i + 1 < m ? std::fabs(be[i]) : 0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  auto count_above = [&](double x) {  // eigenvalues > x
    int n = 0;
    double q = 1;
    for (int i = 0; i < m; ++i) {
      q = al[i] - x - (i > 0 ? be[i - 1] * be[i - 1] / q : 0.0);
      if (q == 0) q = -1e-300;
      if (q > 0) ++n;
    }
    return n;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::fabs(hi); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_above(mid) > 0) lo = mid; else hi = mid;
  }
  return hi;
}

static double patch_lambda_max(const pmdg_solver* s, std::string& err) {
  const Brick &F = s->b[0], &C = s->b[1];
  pmdg_solver P;
  P.pr = s->pr;
  P.ndom = 2;
  pmdg_brick pf = s->pr.dom[0], pc = s->pr.dom[1];
  for (int a = 0; a < 2; ++a) {
    const int nec = C.ne[a];
    int kc = nec;
    for (int k = 1; k <= nec; ++k) {
      const double r = k * C.h[a] / F.h[a];
      if (std::fabs(r - std::round(r)) <= 1e-9 * r) { kc = k; break; }
    }
    const int rep = std::max(1, std::min((3 + kc - 1) / kc, nec / kc));
    kc *= rep;
    const int kf = kc == nec ? F.ne[a] : (int)std::lround(kc * C.h[a] / F.h[a]);
    pf.ne[a] = kf;
    pf.x1[a] = F.x0[a] + kf * F.h[a];
    pc.ne[a] = kc;
    pc.x1[a] = C.x0[a] + kc * C.h[a];
  }
  const double ztop = F.x0[2] + F.ne[2] * F.h[2];
  pf.ne[2] = std::min(F.ne[2], 3);
  pf.x0[2] = ztop - pf.ne[2] * F.h[2];
  pf.x1[2] = ztop;
  pc.ne[2] = std::min(C.ne[2], 3);
  pc.x0[2] = ztop;
  pc.x1[2] = ztop + pc.ne[2] * C.h[2];
  if (setup_brick(P.b[0], pf, err) || setup_brick(P.b[1], pc, err) || setup_interface(&P, err)) return -1;
  const long n = P.b[0].nnodes + P.b[1].nnodes;
  std::vector<double> mass(n);
  for (int d = 0; d < 2; ++d) {
    const Brick& B = P.b[d];
    const long o = d ? P.b[0].nnodes : 0;
    for (int k = 0; k < B.nn[2]; ++k)
      for (int j = 0; j < B.nn[1]; ++j)
        for (int i = 0; i < B.nn[0]; ++i) mass[o + bnode(B, i, j, k)] = B.mass1[0][i] * B.mass1[1][j] * B.mass1[2][k];
  }
  auto dotm = [&](const std::vector<double>& a, const std::vector<double>& b) {
    double acc = 0;
    for (long i = 0; i < n; ++i) acc += mass[i] * a[i] * b[i];
    return acc;
  };
  const int m = (int)std::min<long>(60, n);
  std::vector<std::vector<double>> Q;
  std::vector<double> al, be, w(n), q(n);
  uint64_t st = 0x9E3779B97F4A7C15ull;
  for (long i = 0; i < n; ++i) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    q[i] = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
  double nq = std::sqrt(dotm(q, q));
  for (long i = 0; i < n; ++i) q[i] /= nq;
  Q.push_back(q);
  for (int j = 0; j < m; ++j) {
    coupled_apply(&P, Q[j], w);
    al.push_back(dotm(w, Q[j]));
    for (int pass = 0; pass < 2; ++pass)  // full reorthogonalisation, twice
      for (const auto& qi : Q) {
        const double h = dotm(w, qi);
        for (long i = 0; i < n; ++i) w[i] -= h * qi[i];
      }
    const double b = std::sqrt(dotm(w, w));
    if (j + 1 == m || !(b > 1e-12 * std::fabs(al.back()))) break;
    be.push_back(b);
    for (long i = 0; i < n; ++i) w[i] /= b;
    Q.push_back(w);
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  return tridiag_max_eig(al, be);
}

// ------------------------------------------------------------------------
// Drive tables (Sec. 6.1, eq. voltage): the applied voltage of PMUT k is
// A_k g(t) sin(2 pi f t - theta_k) = (A_k cos theta_k) C_s(t) - (A_k sin theta_k) C_c(t)
// with C_s = g(t) sin(2 pi f t), C_c = g(t) cos(2 pi f t) sampled at t_n = n dt.
// ------------------------------------------------------------------------
static double drive_window(double t, double Td, int envelope) {
  if (envelope == 2) return t >= 0 ? 1.0 : 0.0;
  if (t < 0 || t > Td) return 0.0;
  if (envelope == 1) return 1.0;
  // smooth window with n = 10 in the symmetric variable b = |2t/T_d - 1|
  const double b = std::fabs(2.0 * t / Td - 1.0);
  const double b20 = std::pow(b, 20.0);
  const double base = 1.0 - 2.0 * b20 * b / (1.0 + b20);
  if (base <= 0.0) return 0.0;
  return std::exp(1.0 - 1.0 / (base * base));
}

static void drive_tables(const pmdg_solver* s, std::vector<double>& dA, std::vector<double>& car) {
  dA.assign((size_t)s->S * s->Np * 2, 0.0);
  car.assign((size_t)s->S * (s->cap + 1) * 2, 0.0);
  // scenarios [sc0, sc1): disjoint entries, so several host threads can
  // share the work (the FP64 window and carrier values of a few thousand
  // scenarios take milliseconds on one thread)
  auto fill = [s, &dA, &car](int sc0, int sc1) {
    for (int sc = sc0; sc < sc1; ++sc) {
      for (int k = 0; k < s->Np; ++k) {
        const size_t i = (size_t)sc * s->Np + k;
        dA[2 * i] = s->amp[i] * std::cos(s->phase[i]);
        dA[2 * i + 1] = s->amp[i] * std::sin(s->phase[i]);
      }
      const double f = s->freq[sc], Td = s->ncyc / f;
      for (long n = 0; n <= s->cap; ++n) {
        const double t = n * s->dt;
        const double g = drive_window(t, Td, s->envelope);
        if (g == 0.0) continue;  // outside the burst the carrier entries stay zero
        car[((size_t)sc * (s->cap + 1) + n) * 2] = g * std::sin(2.0 * M_PI * f * t);
        car[((size_t)sc * (s->cap + 1) + n) * 2 + 1] = g * std::cos(2.0 * M_PI * f * t);
      }
    }
  };
  const long work = (long)s->S * (s->cap + 1);
  const int nt = (int)std::min<long>(std::min<long>(std::max(1u, std::thread::hardware_concurrency()), 16L), s->S);
  if (nt <= 1 || work < (1L << 16)) {
    fill(0, s->S);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) pool.emplace_back(fill, (int)((long)s->S * t / nt), (int)((long)s->S * (t + 1) / nt));
  for (std::thread& th : pool) th.join();
}

// ------------------------------------------------------------------------
// Workspace layout
// ------------------------------------------------------------------------
static size_t rbytes(const pmdg_solver* s) { return s->prec == 64 ? 8 : 4; }

static size_t layout(pmdg_solver* s) {
  s->seg.clear();
  size_t off = 0;
  auto add = [&](const std::string& name, size_t bytes) {
    Seg g;
    g.off = off;
    g.bytes = bytes;
    s->seg[name] = g;
    off += (bytes + 255) / 256 * 256;
  };
  const size_t rb = rbytes(s);
  const long S = s->S;
  add("ctl", 256);
  for (int d = 0; d < s->ndom; ++d) {
    const Brick& B = s->b[d];
    const std::string p = "d" + std::to_string(d) + ".";
    add(p + "P0", rb * S * B.pnodes);
    add(p + "P1", rb * S * B.pnodes);
    if (s->prec == 32) {
      add(p + "P2", rb * S * B.pnodes);
      add(p + "X", rb * 2 * S * B.pnodes);
    }
    if (B.mapped()) {
      const size_t nel = (size_t)B.ne[0] * B.ne[1] * B.ne[2], n3 = (size_t)(B.N + 1) * (B.N + 1) * (B.N + 1);
      add(p + "hminv", rb * B.pnodes);
      add(p + "hvert", rb * nel * 24);
      add(p + "hy", rb * S * nel * n3);
    }
    add(p + "taps", rb * 3 * (B.N + 3) * 2 * B.N);
    add(p + "mins", rb * 3 * (B.N + 3));
    add(p + "absg", rb * 3 * (B.N + 3));
    if (B.pml) {
      const size_t n3 = (size_t)(B.N + 1) * (B.N + 1) * (B.N + 1), nel = B.pel.size() / 3;
      for (int a = 0; a < 3; ++a) {
        add(p + "pz" + std::to_string(a), rb * B.nn[a]);
        add(p + "pmi" + std::to_string(a), rb * B.nn[a]);
      }
      add(p + "eslot", sizeof(int) * B.eslot.size());
      add(p + "pel", sizeof(int) * B.pel.size());
      add(p + "pnode", sizeof(int) * B.pnode.size());
      add(p + "phi", rb * S * nel * 3 * n3);
      add(p + "prel", rb * S * nel * n3);
      add(p + "psi", rb * S * B.pnodes);
      add(p + "pacc", rb * S * B.pnodes);
    }
  }
  if (s->Np > 0) {
    add("force", rb * S * s->b[0].pplane);
    add("pm_off", sizeof(int) * (s->Np + 1));
    add("pm_node", sizeof(int) * std::max<size_t>(1, s->pm_node.size()));
    add("pm_B", sizeof(double) * std::max<size_t>(1, s->pm_B.size()));
    add("omega", sizeof(double) * s->Np * s->Nm);
    add("zeta", sizeof(double) * s->Np * s->Nm);
    add("eta", sizeof(double) * s->Np * s->Nm);
    add("dA", sizeof(double) * S * s->Np * 2);
    add("car", sizeof(double) * S * (s->cap + 1) * 2);
    add("q", sizeof(double) * S * s->Np * s->Nm);
    add("qd", sizeof(double) * S * s->Np * s->Nm);
    add("qdd", sizeof(double) * S * s->Np * s->Nm);
  }
  if (s->ndom > 1) {
    const int n0 = s->b[0].N + 1, n1 = s->b[1].N + 1;
    add("tr0", rb * S * face0(s) * 2);
    add("tr1", rb * S * face1(s) * 2);
    add("R0", rb * S * nfine(s) * n0 * n0 * 2);
    add("R1", rb * S * ncoarse(s) * n1 * n1 * 2);
    add("Aq", rb * S * nfine(s) * s->Nq * s->Nq * 2);
    add("Lq", rb * s->Lq.size());
    add("wJ", rb * s->wJ.size());
    add("xw", rb * s->xw.size());
    add("yw", rb * s->yw.size());
    add("xcx", sizeof(int) * s->xcx.size());
    add("ycx", sizeof(int) * s->ycx.size());
    add("xl_off", sizeof(int) * s->xl_off.size());
    add("xl", sizeof(int) * s->xl.size());
    add("yl_off", sizeof(int) * s->yl_off.size());
    add("yl", sizeof(int) * s->yl.size());
  }
  if (s->R > 0) {
    add("r_dom", sizeof(int) * s->R);
    add("r_base", sizeof(long) * s->R);
    add("r_w", sizeof(double) * s->r_w.size());
    add("traces", sizeof(double) * S * s->R * s->cap);
  }
  return off;
}

template <typename T>
static T* dptr(pmdg_solver* s, const std::string& name) {
  auto it = s->seg.find(name);
  if (it == s->seg.end() || !s->ws) return nullptr;
  return (T*)(s->ws + it->second.off);
}

template <typename Real>
static std::vector<Real> conv(const std::vector<double>& v) {
  return std::vector<Real>(v.begin(), v.end());
}

static pmdg_status upload_bytes(pmdg_solver* s, const std::string& name, const void* src, size_t bytes,
                                hipStream_t st) {
  auto it = s->seg.find(name);
  if (it == s->seg.end()) return fail(PMDG_EINVAL, "internal: unknown segment " + name);
  if (bytes > it->second.bytes) return fail(PMDG_EINVAL, "internal: segment overflow " + name);
  if (bytes == 0) return PMDG_OK;
  HIPCHK(hipMemcpyAsync(s->ws + it->second.off, src, bytes, hipMemcpyHostToDevice, st));
  return PMDG_OK;
}

template <typename Real>
static pmdg_status upload_real(pmdg_solver* s, const std::string& name, const std::vector<double>& v,
                               hipStream_t st) {
  std::vector<Real> t = conv<Real>(v);
  pmdg_status r = upload_bytes(s, name, t.data(), t.size() * sizeof(Real), st);
  if (r) return r;
  HIPCHK(hipStreamSynchronize(st));
  return PMDG_OK;
}

template <typename T>
static pmdg_status upload_vec(pmdg_solver* s, const std::string& name, const std::vector<T>& v, hipStream_t st) {
  pmdg_status r = upload_bytes(s, name, v.data(), v.size() * sizeof(T), st);
  if (r) return r;
  HIPCHK(hipStreamSynchronize(st));
  return PMDG_OK;
}

// ------------------------------------------------------------------------
// Kernel argument assembly
// ------------------------------------------------------------------------
template <typename Real>
static DomView<Real> view(pmdg_solver* s, int d) {
  DomView<Real> v;
  const Brick& B = s->b[d];
  for (int a = 0; a < 3; ++a) v.nn[a] = B.nn[a];
  v.N = B.N;
  v.px = B.px;
  v.plane = B.pplane;
  v.nnodes = B.pnodes;
  const std::string p = "d" + std::to_string(d) + ".";
  v.P[0] = dptr<Real>(s, p + "P0");
  v.P[1] = dptr<Real>(s, p + "P1");
  v.P[2] = s->prec == 32 ? dptr<Real>(s, p + "P2") : nullptr;
  v.nbuf = s->prec == 32 ? 3 : 2;
  v.X = s->prec == 32 ? dptr<Real>(s, p + "X") : nullptr;
  v.xstride = (long)s->S * B.pnodes;
  v.xsel = (const int*)(dptr<char>(s, "ctl") + 8 + 4 * d);
  return v;
}

// Planes per stiffness workgroup along z for brick d, whose plane layer
// has layer_tiles workgroup tiles (all scenarios): an explicit chunk, the
// whole brick (0), or automatically (-1) 73 planes unless that leaves fewer
// than 512 workgroups (two per CU), then fewer planes, at least 4.  Each
// workgroup's plane loop is a chain of dependent memory round trips, so a
// small brick needs short chunks to finish quickly.
static int brick_zchunk(const pmdg_solver* s, int d, long layer_tiles) {
  const int zc = (d == 1 && s->zchunk1 >= 0) ? s->zchunk1 : s->zchunk;
  const int nz = s->b[d].nn[2];
  if (zc > 0) return std::min(zc, nz);
  if (zc == 0) return nz;
  const long fit = (long)nz * layer_tiles / 512;
  return (int)std::min<long>(nz, std::max(4L, std::min(73L, fit)));
}

// Rows per wave of brick d's stiffness tile: an explicit choice, or
// automatically (0) 1 for a brick whose whole z extent is one chunk at 2
// rows, else 2.  Such a brick cannot gain workgroups along z without
// reloading 2N halo planes per extra chunk; halving the rows doubles its
// workgroups at the cost of y-halo rows, which mostly hit in L2.
static int brick_rows(const pmdg_solver* s, int d) {
  const int r = (d == 1 && s->rows1 > 0) ? s->rows1 : s->rows;
  if (r > 0) return r;
  const Brick& B = s->b[d];
  const long ty = 2L * s->waves;
  const long layer = (long)(B.px / 64) * ((B.nn[1] + ty - 1) / ty) * s->S;
  return brick_zchunk(s, d, layer) >= B.nn[2] ? 1 : 2;
}

// Planes per workgroup of brick d's single-step stiffness launch.
static int launch_zchunk(const pmdg_solver* s, int d) {
  const Brick& B = s->b[d];
  const int ty = s->waves * brick_rows(s, d);
  return brick_zchunk(s, d, (long)(B.px / 64) * ((B.nn[1] + ty - 1) / ty) * s->S);
}

static bool two_step(const pmdg_solver* s, int d);

// Brick d's stiffness launch writes its own value / normal-derivative
// traces on Gamma_I, so the face kernel skips its trace blocks: two bricks,
// brick d on the single-step pass, and the interface element layer inside
// one z chunk of that launch.
static bool fused_traces(const pmdg_solver* s, int d) {
  if (s->ndom < 2 || two_step(s, d)) return false;
  const int nz = s->b[d].nn[2], N = s->b[d].N, zc = launch_zchunk(s, d);
  const int l0 = d == 0 ? nz - 1 - N : 0, l1 = d == 0 ? nz - 1 : N;
  return l0 / zc == l1 / zc;
}

template <typename Real>
static StiffArgs<Real> stiff_args(pmdg_solver* s, int d) {
  StiffArgs<Real> a;
  memset(&a, 0, sizeof(a));
  a.d = view<Real>(s, d);
  a.S = s->S;
  a.dt2 = (Real)(s->dt * s->dt);
  a.counter = dptr<long>(s, "ctl");
  a.force = (d == 0 && s->Np > 0) ? dptr<Real>(s, "force") : nullptr;
  if (s->ndom > 1) {
    const Brick& B = s->b[d];
    a.iface = dptr<Real>(s, d == 0 ? "R0" : "R1");
    a.iface_side = d == 0 ? 1 : -1;
    a.iface_nex = B.ne[0];
    a.iface_ney = B.ne[1];
    const double c2 = B.c * B.c;
    for (int c = 0; c <= B.N; ++c) a.iface_d[c] = (Real)(c2 * (d == 0 ? s->dz0[c] : s->dz1[c]));
  }
  {
    const std::string p = "d" + std::to_string(d) + ".";
    a.taps = dptr<Real>(s, p + "taps");
    a.mins = dptr<Real>(s, p + "mins");
    a.absg = dptr<Real>(s, p + "absg");
    a.absorb = s->b[d].absorbing != 0;
  }
  const Brick& B = s->b[d];
  a.rows = brick_rows(s, d);
  a.waves = s->waves;
  a.depth = deep_prefetch_built(B.N, a.rows, a.waves) ? s->depth : 2;
  if (B.pml) {
    // the layer's build: 4-wave tiles of 1 or 2 rows, 2-plane prefetch
    const std::string p = "d" + std::to_string(d) + ".";
    a.rows = std::min(a.rows, 2);
    a.waves = 4;
    a.depth = 2;
    a.pml_acc = dptr<Real>(s, p + "pacc");
    a.pml_zx = dptr<Real>(s, p + "pz0");
    a.pml_zy = dptr<Real>(s, p + "pz1");
    a.pml_zz = dptr<Real>(s, p + "pz2");
    a.dt = (Real)s->dt;
  }
  a.nbx = B.px / 64;
  const int TY = a.waves * a.rows;
  a.nby = (B.nn[1] + TY - 1) / TY;
  a.zlo = 0;
  a.zhi = B.nn[2] - 1;
  a.zchunk = brick_zchunk(s, d, (long)a.nbx * a.nby * s->S);
  a.nbz = (B.nn[2] + a.zchunk - 1) / a.zchunk;
  a.nblocks = a.nbx * a.nby * a.nbz * s->S;
  if (fused_traces(s, d)) {
    a.trace = dptr<Real>(s, d == 0 ? "tr0" : "tr1");
    for (int c = 0; c <= B.N; ++c) a.trd[c] = (Real)(d == 0 ? s->dz0[c] : s->dz1[c]);
  }
  return a;
}

template <typename Real>
static FaceArgs<Real> face_args(pmdg_solver* s, int prime) {
  FaceArgs<Real> a;
  memset(&a, 0, sizeof(a));
  a.counter = dptr<long>(s, "ctl");
  a.nonfinite = (int*)(dptr<char>(s, "ctl") + 16);
  a.prime = prime;
  a.S = s->S;
  a.dt = s->dt;
  a.ndom = s->ndom;
  a.d0 = view<Real>(s, 0);
  if (s->ndom > 1) a.d1 = view<Real>(s, 1);
  if (s->ndom > 1) {
    a.tr0 = dptr<Real>(s, "tr0");
    a.tr1 = dptr<Real>(s, "tr1");
    for (int c = 0; c <= s->b[0].N; ++c) a.dz0[c] = (Real)s->dz0[c];
    for (int c = 0; c <= s->b[1].N; ++c) a.dz1[c] = (Real)s->dz1[c];
    a.nb_tr0 = prime || !fused_traces(s, 0) ? (int)((s->S * face0(s) + 255) / 256) : 0;
    a.nb_tr1 = prime || !fused_traces(s, 1) ? (int)((s->S * face1(s) + 255) / 256) : 0;
  }
  if (s->Np > 0) {
    a.Np = s->Np;
    a.Nm = s->Nm;
    a.pm_off = dptr<int>(s, "pm_off");
    a.pm_node = dptr<int>(s, "pm_node");
    a.pm_B = dptr<double>(s, "pm_B");
    a.omega = dptr<double>(s, "omega");
    a.zeta = dptr<double>(s, "zeta");
    a.eta = dptr<double>(s, "eta");
    a.kappa = s->b[0].rho * s->b[0].c * s->b[0].c;
    a.dA = dptr<double>(s, "dA");
    a.car = dptr<double>(s, "car");
    a.ncar = s->cap + 1;
    a.t_switch = s->t_switch;
    a.cap = s->rx_cap;
    a.q = dptr<double>(s, "q");
    a.qd = dptr<double>(s, "qd");
    a.qdd = dptr<double>(s, "qdd");
    a.force = dptr<Real>(s, "force");
    a.nb_pm = s->S * s->Np;
  }
  if (s->R > 0 && !prime) {
    a.R = s->R;
    a.r_dom = dptr<int>(s, "r_dom");
    a.r_base = dptr<long>(s, "r_base");
    a.r_w = dptr<double>(s, "r_w");
    a.traces = dptr<double>(s, "traces");
    a.tcap = s->cap;
    a.nb_rc = (s->S * s->R + kWaves - 1) / kWaves;
  }
  a.nblocks = a.nb_tr0 + a.nb_tr1 + a.nb_pm + a.nb_rc;
  if (a.nblocks == 0) a.nblocks = 1;
  return a;
}

template <typename Real>
static FluxArgs<Real> flux_args(pmdg_solver* s, int tick) {
  FluxArgs<Real> a;
  memset(&a, 0, sizeof(a));
  if (s->ndom < 2) return a;
  a.S = s->S;
  a.N0 = s->b[0].N;
  a.N1 = s->b[1].N;
  a.Nq = s->Nq;
  a.nn0x = s->b[0].nn[0];
  a.nn1x = s->b[1].nn[0];
  a.nex0 = s->b[0].ne[0];
  a.ney0 = s->b[0].ne[1];
  a.nex1 = s->b[1].ne[0];
  a.ney1 = s->b[1].ne[1];
  a.tr0 = dptr<Real>(s, "tr0");
  a.tr1 = dptr<Real>(s, "tr1");
  a.Lq = dptr<Real>(s, "Lq");
  a.wJ = dptr<Real>(s, "wJ");
  a.xcx = dptr<int>(s, "xcx");
  a.ycx = dptr<int>(s, "ycx");
  a.xw = dptr<Real>(s, "xw");
  a.yw = dptr<Real>(s, "yw");
  a.xl_off = dptr<int>(s, "xl_off");
  a.xl = dptr<int>(s, "xl");
  a.yl_off = dptr<int>(s, "yl_off");
  a.yl = dptr<int>(s, "yl");
  a.gamma = (Real)s->gamma;
  a.cf2 = (Real)(s->b[0].c * s->b[0].c);
  a.cc2 = (Real)(s->b[1].c * s->b[1].c);
  a.R0 = dptr<Real>(s, "R0");
  a.R1 = dptr<Real>(s, "R1");
  a.Aq = dptr<Real>(s, "Aq");
  a.counter = dptr<long>(s, "ctl");
  a.tick = tick;
  a.xsel = (int*)(dptr<char>(s, "ctl") + 8);
  a.toggle = 0;  // bit d: swap brick d's live increment copy
  a.nb_fine = (s->S * nfine(s) + 2 * kWaves - 1) / (2 * kWaves);
  a.nb_coarse = (s->S * ncoarse(s) + 2 * kWaves - 1) / (2 * kWaves);
  a.tcap = s->xl_max * (a.N1 + 1);
  return a;
}

// Per-kernel-class HIP events (0 stiffness, 1 face, 2 interface + tick).
struct Timer {
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  hipError_t begin(int cls, hipStream_t st) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    ev.push_back({cls, {a, b}});
    return hipEventRecord(a, st);
  }
  hipError_t end(hipStream_t st) { return hipEventRecord(ev.back().second.second, st); }
  void release() {
    for (auto& e : ev) {
      (void)hipEventDestroy(e.second.first);
      (void)hipEventDestroy(e.second.second);
    }
    ev.clear();
  }
};

#define TBEGIN(cls) \
  if (tm) HIPCHK(tm->begin(cls, st))
#define TEND() \
  if (tm) HIPCHK(tm->end(st))

template <typename Real>
static pmdg_status enqueue_coupling(pmdg_solver* s, hipStream_t st, Timer* tm, int toggle) {
  {
    FaceArgs<Real> a = face_args<Real>(s, 0);
    TBEGIN(1);
    HIPCHK(launch_face<Real>(a, st));
    TEND();
  }
  TBEGIN(2);
  if (s->ndom > 1) {
    FluxArgs<Real> a = flux_args<Real>(s, 1);
    a.toggle = toggle;
    HIPCHK(launch_flux<Real>(a, st));
  } else {
    HIPCHK(launch_tick(dptr<long>(s, "ctl"), (int*)(dptr<char>(s, "ctl") + 8), toggle, st));
  }
  TEND();
  return PMDG_OK;
}

// Two bricks, untimed: after the primary's stiffness launch, the face work
// that needs only the primary (PMUT sampling, modal ODE and force, the
// primary's interface traces) runs on a side stream while the secondary's
// stiffness launch runs; the secondary's interface traces, the receivers and
// the interface kernels follow the join.  Mode 2 also moves the primary's
// stiffness launch to the side stream, so that both bricks' stiffness
// updates (independent of each other within a step) run together.
template <typename Real>
static pmdg_status enqueue_step_split(pmdg_solver* s, hipStream_t st, int toggle) {
  if (!s->side) {
    HIPCHK(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
  }
  const bool incr = s->prec == 32;
  if (s->overlap == 2) {
    HIPCHK(hipEventRecord(s->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(s->side, s->ev_fork, 0));
    HIPCHK(launch_stiff<Real>(stiff_args<Real>(s, 0), incr, s->side));
  } else {
    HIPCHK(launch_stiff<Real>(stiff_args<Real>(s, 0), incr, st));
    HIPCHK(hipEventRecord(s->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(s->side, s->ev_fork, 0));
  }
  FaceArgs<Real> f = face_args<Real>(s, 0);
  FaceArgs<Real> f1 = f, f2 = f;
  f1.nb_tr1 = 0;
  f1.nb_rc = 0;
  f1.R = 0;
  f1.nblocks = std::max(1, f1.nb_tr0 + f1.nb_pm);
  f2.nb_tr0 = 0;
  f2.nb_pm = 0;
  f2.nblocks = std::max(1, f2.nb_tr1 + f2.nb_rc);
  HIPCHK(launch_face<Real>(f1, s->side));
  HIPCHK(hipEventRecord(s->ev_join, s->side));
  HIPCHK(launch_stiff<Real>(stiff_args<Real>(s, 1), incr, st));
  HIPCHK(hipStreamWaitEvent(st, s->ev_join, 0));
  HIPCHK(launch_face<Real>(f2, st));
  FluxArgs<Real> a = flux_args<Real>(s, 1);
  a.toggle = toggle;
  HIPCHK(launch_flux<Real>(a, st));
  return PMDG_OK;
}

static bool any_pml(const pmdg_solver* s) { return s->b[0].pml || (s->ndom > 1 && s->b[1].pml); }

// Two bricks, untimed, overlap mode 3: both stiffness launches in sequence
// (and any interface traces they do not write themselves), then the PMUT
// and receiver blocks of the face kernel on a side stream alongside the two
// interface kernels, both short and bound by latency rather than bandwidth.  The last interface kernel advances the
// step counter, so the face kernel reads a copy of it that the primary's
// stiffness launch writes.
template <typename Real>
static pmdg_status enqueue_step_faceflux(pmdg_solver* s, hipStream_t st, int toggle) {
  if (!s->side) {
    HIPCHK(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
  }
  const bool incr = s->prec == 32;
  long* snap = (long*)(dptr<char>(s, "ctl") + 32);
  StiffArgs<Real> a0 = stiff_args<Real>(s, 0);
  a0.cnt_snap = snap;
  HIPCHK(launch_stiff<Real>(a0, incr, st));
  HIPCHK(launch_stiff<Real>(stiff_args<Real>(s, 1), incr, st));
  FaceArgs<Real> f = face_args<Real>(s, 0);
  f.counter = snap;
  // interface traces the stiffness launches did not write go first: the
  // interface kernels read them
  if (f.nb_tr0 + f.nb_tr1 > 0) {
    FaceArgs<Real> ft = f;
    ft.nb_pm = 0;
    ft.nb_rc = 0;
    ft.R = 0;
    ft.nblocks = f.nb_tr0 + f.nb_tr1;
    HIPCHK(launch_face<Real>(ft, st));
  }
  HIPCHK(hipEventRecord(s->ev_fork, st));
  HIPCHK(hipStreamWaitEvent(s->side, s->ev_fork, 0));
  FaceArgs<Real> fp = f;
  fp.nb_tr0 = 0;
  fp.nb_tr1 = 0;
  fp.nblocks = std::max(1, f.nb_pm + f.nb_rc);
  HIPCHK(launch_face<Real>(fp, s->side));
  HIPCHK(hipEventRecord(s->ev_join, s->side));
  FluxArgs<Real> a = flux_args<Real>(s, 1);
  a.toggle = toggle;
  HIPCHK(launch_flux<Real>(a, st));
  HIPCHK(hipStreamWaitEvent(st, s->ev_join, 0));
  return PMDG_OK;
}

// Arguments of the layer kernels of brick d (prime: the acceleration of the
// current level only).
template <typename Real>
static PmlArgs<Real> pml_args(pmdg_solver* s, int d, int prime) {
  PmlArgs<Real> a;
  memset(&a, 0, sizeof(a));
  const Brick& B = s->b[d];
  const std::string p = "d" + std::to_string(d) + ".";
  a.d = view<Real>(s, d);
  a.S = s->S;
  a.counter = dptr<long>(s, "ctl");
  a.prime = prime;
  a.dt = (Real)s->dt;
  a.c2 = (Real)(B.c * B.c);
  for (int k = 0; k < 3; ++k) {
    a.gh[k] = (Real)(2.0 / B.h[k]);
    a.ne[k] = B.ne[k];
  }
  a.J = (Real)(B.h[0] * B.h[1] * B.h[2] / 8.0);
  a.zx = dptr<Real>(s, p + "pz0");
  a.zy = dptr<Real>(s, p + "pz1");
  a.zz = dptr<Real>(s, p + "pz2");
  a.mix = dptr<Real>(s, p + "pmi0");
  a.miy = dptr<Real>(s, p + "pmi1");
  a.miz = dptr<Real>(s, p + "pmi2");
  a.eslot = dptr<int>(s, p + "eslot");
  a.pel = dptr<int>(s, p + "pel");
  a.nel = (int)(B.pel.size() / 3);
  a.pnode = dptr<int>(s, p + "pnode");
  a.npn = (int)(B.pnode.size() / 3);
  a.phi = dptr<Real>(s, p + "phi");
  a.rel = dptr<Real>(s, p + "prel");
  a.psi = dptr<Real>(s, p + "psi");
  a.acc = dptr<Real>(s, p + "pacc");
  const int n1 = B.N + 1;
  for (int q = 0; q < n1; ++q) {
    a.w[q] = (Real)B.rule.w[q];
    for (int m = 0; m < n1; ++m) a.D[q * n1 + m] = (Real)B.rule.D[q * n1 + m];
  }
  return a;
}

// Kernel arguments of a brick given as trilinear hexahedra.
template <typename Real>
static HexArgs<Real> hex_args(pmdg_solver* s, int d) {
  HexArgs<Real> a;
  memset(&a, 0, sizeof(a));
  const Brick& B = s->b[d];
  const std::string p = "d" + std::to_string(d) + ".";
  a.d = view<Real>(s, d);
  a.S = s->S;
  for (int k = 0; k < 3; ++k) a.ne[k] = B.ne[k];
  a.nel = B.ne[0] * B.ne[1] * B.ne[2];
  // one workgroup per strip of sx elements along x, per element row and scenario
  const int sx = hex_elems_per_block<Real>(B.N);
  a.eblocks = (int)((long)(B.ne[0] + sx - 1) / sx * B.ne[1] * B.ne[2] * s->S);
  a.dt2 = (Real)(s->dt * s->dt);
  a.c2 = (Real)(B.c * B.c);
  a.counter = dptr<long>(s, "ctl");
  a.force = (d == 0 && s->Np > 0) ? dptr<Real>(s, "force") : nullptr;
  a.minv = dptr<Real>(s, p + "hminv");
  a.vert = dptr<Real>(s, p + "hvert");
  a.y = dptr<Real>(s, p + "hy");
  const int n1 = B.N + 1;
  for (int i = 0; i < n1; ++i) {
    a.w[i] = (Real)B.rule.w[i];
    a.xg[i] = (Real)B.rule.x[i];
    for (int j = 0; j < n1; ++j) a.D[i * n1 + j] = (Real)B.rule.D[i * n1 + j];
  }
  return a;
}

template <typename Real>
static pmdg_status enqueue_step(pmdg_solver* s, hipStream_t st, Timer* tm) {
  if (!tm && s->ndom == 2 && s->overlap == 3 && !any_pml(s) && !s->b[0].mapped())
    return enqueue_step_faceflux<Real>(s, st, 0);
  if (!tm && s->ndom == 2 && s->overlap && !any_pml(s)) return enqueue_step_split<Real>(s, st, 0);
  const bool incr = s->prec == 32;
  for (int d = 0; d < s->ndom; ++d) {
    if (s->b[d].mapped()) {
      TBEGIN(0);
      HIPCHK(launch_hex<Real>(hex_args<Real>(s, d), incr, st));
      TEND();
      continue;
    }
    StiffArgs<Real> a = stiff_args<Real>(s, d);
    TBEGIN(0);
    HIPCHK(launch_stiff<Real>(a, incr, st));
    if (s->b[d].pml) HIPCHK(launch_pml<Real>(pml_args<Real>(s, d, 0), st));
    TEND();
  }
  return enqueue_coupling<Real>(s, st, tm, 0);
}

// Planes of brick d whose second step of a two-step pass needs the coupling
// terms of the first: the primary's PMUT plane and interface layers, the
// secondary's interface layers.
static void completion_ranges(const pmdg_solver* s, int d, int r[4]) {
  const Brick& B = s->b[d];
  r[0] = r[2] = 1;
  r[1] = r[3] = 0;
  if (d == 0) {
    if (s->Np > 0) r[0] = r[1] = 0;
    if (s->ndom > 1) { r[2] = B.nn[2] - 1 - B.N; r[3] = B.nn[2] - 1; }
  } else {
    r[0] = 0;
    r[1] = B.N;
  }
}

// brick d advances two steps per stiffness pass
static bool two_step(const pmdg_solver* s, int d) {
  if (s->prec != 32 || s->b[d].absorbing || s->b[0].pml || (s->ndom > 1 && s->b[1].pml) || s->b[d].mapped())
    return false;
  const int tb = (d == 1 && s->tblock1 > 0) ? s->tblock1 : s->tblock;
  return tb == 2 && stiff2_tile_rows(s->b[d].N) > 0;
}

static bool two_step_any(const pmdg_solver* s) {
  for (int d = 0; d < s->ndom; ++d)
    if (two_step(s, d)) return true;
  return false;
}

static StiffArgs<float> stiff2_args(pmdg_solver* s, int d) {
  StiffArgs<float> a = stiff_args<float>(s, d);
  const Brick& B = s->b[d];
  const int TYO = stiff2_tile_rows(B.N), TXO = 64 - 2 * B.N;
  a.nbx = (B.nn[0] + TXO - 1) / TXO;
  a.nby = (B.nn[1] + TYO - 1) / TYO;
  a.zlo = 0;
  a.zhi = B.nn[2] - 1;
  a.zchunk = brick_zchunk(s, d, (long)a.nbx * a.nby * s->S);
  a.nbz = (B.nn[2] + a.zchunk - 1) / a.zchunk;
  a.nblocks = a.nbx * a.nby * a.nbz * s->S;
  int r[4];
  completion_ranges(s, d, r);
  a.cb0 = r[0]; a.ce0 = r[1]; a.cb1 = r[2]; a.ce1 = r[3];
  return a;
}

// Steps n+1 and n+2.  Bricks with two-step passes: the fused pass, then,
// after the coupling of step n+1 (whose tick swaps their live increment
// copies), a single-step completion of their coupled planes.  Other bricks:
// a single step before and a single step after that coupling.
static pmdg_status enqueue_pair(pmdg_solver* s, hipStream_t st, Timer* tm) {
  int mask = 0;
  for (int d = 0; d < s->ndom; ++d) {
    TBEGIN(0);
    if (two_step(s, d)) {
      HIPCHK(launch_stiff2(stiff2_args(s, d), st));
      mask |= 1 << d;
    } else {
      HIPCHK(launch_stiff<float>(stiff_args<float>(s, d), true, st));
    }
    TEND();
  }
  pmdg_status r = enqueue_coupling<float>(s, st, tm, mask);
  if (r) return r;
  for (int d = 0; d < s->ndom; ++d) {
    if (!two_step(s, d)) {
      TBEGIN(0);
      HIPCHK(launch_stiff<float>(stiff_args<float>(s, d), true, st));
      TEND();
      continue;
    }
    int cr[4];
    completion_ranges(s, d, cr);
    for (int j = 0; j < 2; ++j) {
      if (cr[2 * j] > cr[2 * j + 1]) continue;
      StiffArgs<float> a = stiff_args<float>(s, d);
      a.zlo = cr[2 * j];
      a.zhi = cr[2 * j + 1];
      a.zchunk = a.zhi - a.zlo + 1;
      a.nbz = 1;
      a.nblocks = a.nbx * a.nby * s->S;
      TBEGIN(0);
      HIPCHK(launch_stiff<float>(a, true, st));
      TEND();
    }
  }
  return enqueue_coupling<float>(s, st, tm, 0);
}

#undef TBEGIN
#undef TEND

template <typename Real>
static pmdg_status prime(pmdg_solver* s, hipStream_t st) {
  FaceArgs<Real> a = face_args<Real>(s, 1);
  HIPCHK(launch_face<Real>(a, st));
  for (int d = 0; d < s->ndom; ++d)
    if (s->b[d].pml) HIPCHK(launch_pml<Real>(pml_args<Real>(s, d, 1), st));
  if (s->ndom > 1) {
    FluxArgs<Real> f = flux_args<Real>(s, 0);
    HIPCHK(launch_flux<Real>(f, st));
  }
  return PMDG_OK;
}

// n steps: pairs of two-step passes where enabled, single steps otherwise
// The LDS-resident path (one workgroup per scenario, whole steps per
// launch): single-brick FP32 solvers without absorbing faces, layers or
// trilinear vertices, with the default tile options, whose pressure, increment,
// face force and PMUT tables fit one workgroup's LDS.
static bool resident_args(pmdg_solver* s, ResidentArgs* out) {
  if (!s->resident || s->ndom != 1 || s->prec != 32) return false;
  const Brick& B = s->b[0];
  if (B.absorbing || B.pml || B.mapped()) return false;
  if (s->rows != 0 || s->zchunk != -1 || s->waves != 4 || s->depth != 2 || s->tblock != 1 || s->overlap != 0)
    return false;
  if (s->Nm > kMaxModes || B.nnodes > resident_max_nodes() || B.pnodes > (1L << 30)) return false;
  // every table the kernel reads must exist: PMUT tables when there are
  // PMUTs, receiver tables when there are receivers
  if ((s->Np > 0 && !(dptr<int>(s, "pm_off") && dptr<double>(s, "pm_B") && dptr<double>(s, "car"))) ||
      (s->R > 0 && !(dptr<long>(s, "r_base") && dptr<double>(s, "r_w") && dptr<double>(s, "traces"))))
    return false;
  ResidentArgs a;
  memset(&a, 0, sizeof(a));
  const int NT = 2 * B.N, NC = B.N + 3;
  const long nc = B.nnodes, nface = (long)s->pm_node.size();
  auto al = [](long v) { return (v + 15) / 16 * 16; };
  // p with N planes of zero padding on each side, then the increment
  long off = al(4 * (nc + 2L * resident_pad(B.N, B.nn[0], B.nn[1])) + 4 * nc);
  a.off_force = (int)off;
  off = al(off + 4L * B.nn[0] * B.nn[1]);
  a.off_taps = (int)off;
  off = al(off + 4L * 3 * NC * NT);
  a.off_mins = (int)off;
  off = al(off + 4L * 3 * NC);
  a.off_B = (int)off;
  off = al(off + 8L * nface * s->Nm);
  a.off_fn = (int)off;
  off = al(off + 4L * nface);
  a.off_q = (int)off;
  off = al(off + 8L * 3 * s->Np * s->Nm);
  a.off_coef = (int)off;
  off = al(off + 8L * 3 * s->Np * s->Nm);
  a.off_da = (int)off;
  off = al(off + 8L * 2 * s->Np);
  a.off_rw = (int)off;
  off = al(off + 8L * 3 * (B.N + 1) * s->R);
  a.off_poff = (int)off;
  off = al(off + 4L * (s->Np + 1));
  a.off_rb = (int)off;
  off += 4L * s->R;
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  if (off > lim) return false;
  a.lds_bytes = (int)off;
  a.d = view<float>(s, 0);
  a.S = s->S;
  a.nc = (int)nc;
  a.inv_nn0 = 1.0f / B.nn[0];
  a.inv_nn1 = 1.0f / B.nn[1];
  a.counter = dptr<long>(s, "ctl");
  a.dt2 = (float)(s->dt * s->dt);
  a.taps = dptr<float>(s, "d0.taps");
  a.mins = dptr<float>(s, "d0.mins");
  a.nonfinite = (int*)(dptr<char>(s, "ctl") + 16);
  FaceArgs<float> f = face_args<float>(s, 0);
  a.force = s->Np > 0 ? dptr<float>(s, "force") : nullptr;
  a.Np = s->Np;
  a.Nm = s->Nm;
  a.nface = (int)nface;
  for (int k = 0; k < s->Np; ++k)
    if (s->pm_off[k + 1] - s->pm_off[k] > 48) a.pm_wide = 1;
  a.pm_off = f.pm_off;
  a.pm_node = f.pm_node;
  a.pm_B = f.pm_B;
  a.omega = f.omega;
  a.zeta = f.zeta;
  a.eta = f.eta;
  a.kappa = f.kappa;
  a.dt = f.dt;
  a.dA = f.dA;
  a.car = f.car;
  a.ncar = f.ncar;
  a.t_switch = f.t_switch;
  a.cap = f.cap;
  a.q = f.q;
  a.qd = f.qd;
  a.qdd = f.qdd;
  a.R = s->R;
  a.r_base = f.r_base;
  a.r_w = f.r_w;
  a.traces = f.traces;
  a.tcap = f.tcap;
  *out = a;
  return true;
}

static pmdg_status enqueue_resident(pmdg_solver* s, const ResidentArgs& base, hipStream_t st, int n, Timer* tm) {
  for (int i = 0; i < n;) {
    ResidentArgs a = base;
    a.nsteps = std::min(n - i, 2048);
    if (tm) HIPCHK(tm->begin(0, st));
    HIPCHK(launch_resident(a, st));
    HIPCHK(launch_tick_n(const_cast<long*>(a.counter), a.nsteps, st));
    if (tm) HIPCHK(tm->end(st));
    i += a.nsteps;
  }
  return PMDG_OK;
}

static pmdg_status enqueue(pmdg_solver* s, hipStream_t st, int n, Timer* tm) {
  pmdg_status r = PMDG_OK;
  {
    ResidentArgs ra;
    if (resident_args(s, &ra)) return enqueue_resident(s, ra, st, n, tm);
  }
  int i = 0;
  if (two_step_any(s))
    for (; i + 1 < n && !r; i += 2) r = enqueue_pair(s, st, tm);
  for (; i < n && !r; ++i) r = s->prec == 64 ? enqueue_step<double>(s, st, tm) : enqueue_step<float>(s, st, tm);
  return r;
}

static void drop_graphs(pmdg_solver* s) {
  for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
}

template <typename Real>
static pmdg_status bind_tables(pmdg_solver* s, hipStream_t st) {
  pmdg_status r;
  for (int d = 0; d < s->ndom; ++d) {
    const std::string p = "d" + std::to_string(d) + ".";
    const Brick& B = s->b[d];
    const int NT = 2 * B.N, NC = B.N + 3;
    std::vector<double> taps((size_t)3 * NC * NT, 0.0), mins((size_t)3 * NC, 0.0), absg((size_t)3 * NC, 0.0);
    const double sc = -s->dt * s->dt * B.c * B.c;
    for (int ax = 0; ax < 3; ++ax)
      for (int cls = 0; cls < B.N + 2; ++cls) {
        for (int t = 0; t < NT; ++t) taps[((size_t)ax * NC + cls) * NT + t] = sc * B.ctap[ax][(size_t)cls * NT + t];
        mins[(size_t)ax * NC + cls] = B.cmin[ax][cls];
      }
    // first-order absorbing faces: the lumped boundary matrix of a face node
    // is c times the node's face weight, i.e. the 3D lumped mass divided by
    // the 1D mass m_d of the end node along the face normal, so dt M^{-1} C
    // contributes dt c / m_d per absorbing face through the node
    for (int ax = 0; ax < 3; ++ax) {
      if (B.absorbing & (1 << (2 * ax))) absg[(size_t)ax * NC + B.N] = s->dt * B.c * B.cmin[ax][B.N];
      if (B.absorbing & (1 << (2 * ax + 1))) absg[(size_t)ax * NC + B.N + 1] = s->dt * B.c * B.cmin[ax][B.N + 1];
    }
    if (B.mapped()) {
      if ((r = upload_real<Real>(s, p + "hminv", B.hminv, st))) return r;
      if ((r = upload_real<Real>(s, p + "hvert", B.hvert, st))) return r;
    }
    if ((r = upload_real<Real>(s, p + "taps", taps, st))) return r;
    if ((r = upload_real<Real>(s, p + "mins", mins, st))) return r;
    if ((r = upload_real<Real>(s, p + "absg", absg, st))) return r;
    if (B.pml) {
      for (int a = 0; a < 3; ++a) {
        if ((r = upload_real<Real>(s, p + "pz" + std::to_string(a), B.pzeta[a], st))) return r;
        if ((r = upload_real<Real>(s, p + "pmi" + std::to_string(a), B.minv[a], st))) return r;
      }
      if ((r = upload_vec(s, p + "eslot", B.eslot, st))) return r;
      if ((r = upload_vec(s, p + "pel", B.pel, st))) return r;
      if ((r = upload_vec(s, p + "pnode", B.pnode, st))) return r;
    }
  }
  if (s->ndom > 1) {
    if ((r = upload_real<Real>(s, "Lq", s->Lq, st))) return r;
    if ((r = upload_real<Real>(s, "wJ", s->wJ, st))) return r;
    if ((r = upload_real<Real>(s, "xw", s->xw, st))) return r;
    if ((r = upload_real<Real>(s, "yw", s->yw, st))) return r;
    if ((r = upload_vec(s, "xcx", s->xcx, st))) return r;
    if ((r = upload_vec(s, "ycx", s->ycx, st))) return r;
    if ((r = upload_vec(s, "xl_off", s->xl_off, st))) return r;
    if ((r = upload_vec(s, "xl", s->xl, st))) return r;
    if ((r = upload_vec(s, "yl_off", s->yl_off, st))) return r;
    if ((r = upload_vec(s, "yl", s->yl, st))) return r;
  }
  return PMDG_OK;
}

// compact (i + nn0 (j + nn1 k)) <-> device (i + px (j + nn1 k)) node index
static inline long dev_index(const Brick& B, long i) {
  const long row = i / B.nn[0];
  return row * B.px + (i - row * B.nn[0]);
}

template <typename Real>
static pmdg_status get_state_t(pmdg_solver* s, int sc, double* p, double* pp, hipStream_t st) {
  HIPCHK(hipStreamSynchronize(st));
  long cnt = 0;
  HIPCHK(hipMemcpy(&cnt, dptr<long>(s, "ctl"), sizeof(long), hipMemcpyDeviceToHost));
  int xsels[2] = {0, 0};
  HIPCHK(hipMemcpy(xsels, dptr<char>(s, "ctl") + 8, sizeof(xsels), hipMemcpyDeviceToHost));
  const int nbuf = s->prec == 32 ? 3 : 2;
  const int cur = (int)(cnt % nbuf);
  long o = 0;
  for (int d = 0; d < s->ndom; ++d) {
    const Brick& B = s->b[d];
    const std::string pf = "d" + std::to_string(d) + ".";
    std::vector<Real> a(B.pnodes), b(B.pnodes);
    HIPCHK(hipMemcpy(a.data(), dptr<Real>(s, pf + "P" + std::to_string(cur)) + (size_t)sc * B.pnodes,
                     B.pnodes * sizeof(Real), hipMemcpyDeviceToHost));
    if (s->prec == 32)
      HIPCHK(hipMemcpy(b.data(), dptr<Real>(s, pf + "X") + ((size_t)xsels[d] * s->S + sc) * B.pnodes,
                       B.pnodes * sizeof(Real), hipMemcpyDeviceToHost));
    else
      HIPCHK(hipMemcpy(b.data(), dptr<Real>(s, pf + (cur ? "P0" : "P1")) + (size_t)sc * B.pnodes,
                       B.pnodes * sizeof(Real), hipMemcpyDeviceToHost));
    for (long i = 0; i < B.nnodes; ++i) {
      const long di = dev_index(B, i);
      if (p) p[o + i] = (double)a[di];
      if (pp) pp[o + i] = s->prec == 32 ? (double)a[di] - (double)b[di] : (double)b[di];
    }
    o += B.nnodes;
  }
  return PMDG_OK;
}

template <typename Real>
static pmdg_status set_state_t(pmdg_solver* s, int sc, const double* p, const double* pp, const double* q,
                               const double* qd, const double* qdd, long nstep, hipStream_t st) {
  HIPCHK(hipStreamSynchronize(st));
  int xsels[2] = {0, 0};
  HIPCHK(hipMemcpy(xsels, dptr<char>(s, "ctl") + 8, sizeof(xsels), hipMemcpyDeviceToHost));
  const int nbuf = s->prec == 32 ? 3 : 2;
  const int cur = (int)(nstep % nbuf);
  long o = 0;
  for (int d = 0; d < s->ndom; ++d) {
    const Brick& B = s->b[d];
    const std::string pf = "d" + std::to_string(d) + ".";
    std::vector<Real> a(B.pnodes, Real(0)), b(B.pnodes, Real(0));
    for (long i = 0; i < B.nnodes; ++i) {
      const double pv = p ? p[o + i] : 0.0, pq = pp ? pp[o + i] : 0.0;
      const long di = dev_index(B, i);
      a[di] = (Real)pv;
      b[di] = s->prec == 32 ? (Real)(pv - pq) : (Real)pq;
    }
    HIPCHK(hipMemcpy(dptr<Real>(s, pf + "P" + std::to_string(cur)) + (size_t)sc * B.pnodes, a.data(),
                     B.pnodes * sizeof(Real), hipMemcpyHostToDevice));
    if (s->prec == 32)
      HIPCHK(hipMemcpy(dptr<Real>(s, pf + "X") + ((size_t)xsels[d] * s->S + sc) * B.pnodes, b.data(),
                       B.pnodes * sizeof(Real), hipMemcpyHostToDevice));
    else
      HIPCHK(hipMemcpy(dptr<Real>(s, pf + (cur ? "P0" : "P1")) + (size_t)sc * B.pnodes, b.data(),
                       B.pnodes * sizeof(Real), hipMemcpyHostToDevice));
    o += B.nnodes;
  }
  if (s->Np > 0) {
    const size_t nm = (size_t)s->Np * s->Nm, off = nm * sc;
    std::vector<double> z(nm, 0.0);
    HIPCHK(hipMemcpy(dptr<double>(s, "q") + off, q ? q : z.data(), nm * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dptr<double>(s, "qd") + off, qd ? qd : z.data(), nm * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dptr<double>(s, "qdd") + off, qdd ? qdd : z.data(), nm * 8, hipMemcpyHostToDevice));
  }
  // layer fields start at rest (psi = 0, Phi = 0); the layer's acceleration
  // of the set level is formed by prime
  for (int d = 0; d < s->ndom; ++d) {
    const Brick& B = s->b[d];
    if (!B.pml) continue;
    const std::string pf = "d" + std::to_string(d) + ".";
    const long n3 = (long)(B.N + 1) * (B.N + 1) * (B.N + 1), nel = (long)(B.pel.size() / 3);
    HIPCHK(launch_fill<Real>(dptr<Real>(s, pf + "psi") + (size_t)sc * B.pnodes, B.pnodes, Real(0), st));
    HIPCHK(launch_fill<Real>(dptr<Real>(s, pf + "phi") + (size_t)sc * nel * 3 * n3, nel * 3 * n3, Real(0), st));
    HIPCHK(launch_fill<Real>(dptr<Real>(s, pf + "prel") + (size_t)sc * nel * n3, nel * n3, Real(0), st));
  }
  HIPCHK(hipMemcpy(dptr<long>(s, "ctl"), &nstep, sizeof(long), hipMemcpyHostToDevice));
  pmdg_status r = prime<Real>(s, st);
  if (r) return r;
  HIPCHK(hipStreamSynchronize(st));
  s->steps_done = nstep;
  return PMDG_OK;
}

// ------------------------------------------------------------------------
// ABI
// ------------------------------------------------------------------------
// ------------------------------------------------------------------------
// ------------------------------------------------------------------------
// Trilinear hexahedra (host setup)
// ------------------------------------------------------------------------
// Corner c = cx + 2 cy + 4 cz of the reference cube [-1, 1]^3; the map is
// x(xi) = sum_c prod_a (1 + s_a xi_a) / 2 V_c with s_a = +-1 by the bits of c.
static void hex_corners(const Brick& B, int ex, int ey, int ez, double V8[8][3]) {
  const long nx = B.ne[0] + 1, ny = B.ne[1] + 1;
  for (int c = 0; c < 8; ++c) {
    const long v = (ex + (c & 1)) + nx * ((ey + ((c >> 1) & 1)) + ny * (long)(ez + ((c >> 2) & 1)));
    for (int a = 0; a < 3; ++a) V8[c][a] = B.V[3 * v + a];
  }
}

static void hex_map(const double V8[8][3], const double xi[3], double x[3], double J[3][3]) {
  for (int r = 0; r < 3; ++r) {
    x[r] = 0;
    J[r][0] = J[r][1] = J[r][2] = 0;
  }
  for (int c = 0; c < 8; ++c) {
    double f[3], sg[3];
    for (int a = 0; a < 3; ++a) {
      sg[a] = ((c >> a) & 1) ? 1.0 : -1.0;
      f[a] = 0.5 * (1 + sg[a] * xi[a]);
    }
    const double d[3] = {0.5 * sg[0] * f[1] * f[2], 0.5 * sg[1] * f[0] * f[2], 0.5 * sg[2] * f[0] * f[1]};
    for (int r = 0; r < 3; ++r) {
      x[r] += f[0] * f[1] * f[2] * V8[c][r];
      for (int k = 0; k < 3; ++k) J[r][k] += d[k] * V8[c][r];
    }
  }
}

// adj(J) (= det J times J^{-1}); returns det J
static double hex_adj(const double J[3][3], double A[3][3]) {
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  return J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
}

// Coordinates of node (i, j, k): the lowest element holding it, at its GLL point.
static void hex_node_xyz(const Brick& B, int i, int j, int k, double x[3]) {
  const int g[3] = {i, j, k};
  int e[3];
  double xi[3], J[3][3], V8[8][3];
  for (int a = 0; a < 3; ++a) {
    e[a] = std::min(g[a] / B.N, B.ne[a] - 1);
    xi[a] = (double)B.rule.x[g[a] - B.N * e[a]];
  }
  hex_corners(B, e[0], e[1], e[2], V8);
  hex_map(V8, xi, x, J);
}

// Newton's method for the reference point of x in the element with corners
// V8, from the centre; false if it does not converge.  It works in
// coordinates relative to corner 0, so its residual carries rounding of
// the element's size, not of the distance from the origin.
static bool hex_inverse(const double V8g[8][3], const double xg[3], double xi[3]) {
  double V8[8][3], x[3];
  for (int c = 0; c < 8; ++c)
    for (int a = 0; a < 3; ++a) V8[c][a] = V8g[c][a] - V8g[0][a];
  for (int a = 0; a < 3; ++a) x[a] = xg[a] - V8g[0][a];
  xi[0] = xi[1] = xi[2] = 0;
  for (int it = 0; it < 60; ++it) {
    double y[3], J[3][3], A[3][3];
    hex_map(V8, xi, y, J);
    const double det = hex_adj(J, A);
    if (!(std::fabs(det) > 0)) return false;
    const double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double step = 0;
    for (int a = 0; a < 3; ++a) {
      const double dxi = (A[a][0] * r[0] + A[a][1] * r[1] + A[a][2] * r[2]) / det;
      xi[a] += dxi;
      step += std::fabs(dxi);
    }
    if (!(std::fabs(xi[0]) < 10 && std::fabs(xi[1]) < 10 && std::fabs(xi[2]) < 10)) return false;
    if (step < 1e-14) return true;
  }
  return false;
}

// K_e u on one element with corners V8 (without c^2): GLL collocation of
// grad u . grad v |J| on the reference cube, by sum factorisation.
static void hex_apply_host(const Rule1D& R, const double V8[8][3], const double* u, double* r) {
  const int N = R.N, n1 = N + 1, n3 = n1 * n1 * n1;
  std::vector<double> F(3 * (size_t)n3);
  for (int i = 0; i < n3; ++i) {
    const int a = i % n1, b = (i / n1) % n1, c = i / (n1 * n1);
    double g[3] = {0, 0, 0};
    for (int m = 0; m < n1; ++m) {
      g[0] += (double)R.D[a * n1 + m] * u[m + n1 * (b + n1 * c)];
      g[1] += (double)R.D[b * n1 + m] * u[a + n1 * (m + n1 * c)];
      g[2] += (double)R.D[c * n1 + m] * u[a + n1 * (b + n1 * m)];
    }
    const double xi[3] = {(double)R.x[a], (double)R.x[b], (double)R.x[c]};
    double x[3], J[3][3], A[3][3];
    hex_map(V8, xi, x, J);
    const double det = hex_adj(J, A);
    double h[3];
    for (int k = 0; k < 3; ++k) h[k] = A[0][k] * g[0] + A[1][k] * g[1] + A[2][k] * g[2];
    const double sc = (double)(R.w[a] * R.w[b] * R.w[c]) / det;
    for (int k = 0; k < 3; ++k) F[k * (size_t)n3 + i] = sc * (A[k][0] * h[0] + A[k][1] * h[1] + A[k][2] * h[2]);
  }
  for (int i = 0; i < n3; ++i) {
    const int a = i % n1, b = (i / n1) % n1, c = i / (n1 * n1);
    double v = 0;
    for (int m = 0; m < n1; ++m) {
      v += (double)R.D[m * n1 + a] * F[m + n1 * (b + n1 * c)];
      v += (double)R.D[m * n1 + b] * F[n3 + a + n1 * (m + n1 * c)];
      v += (double)R.D[m * n1 + c] * F[2 * (size_t)n3 + a + n1 * (b + n1 * m)];
    }
    r[i] = v;
  }
}

// Largest eigenvalue of Mt^{-1} K_e for one element, Mt the diagonal of
// element-node masses mt: Lanczos with full reorthogonalisation on the
// symmetric form Mt^{-1/2} K_e Mt^{-1/2}.
static double hex_elem_lambda(const Rule1D& R, const double V8[8][3], const double* mt) {
  const int N = R.N, n1 = N + 1, n3 = n1 * n1 * n1;
  std::vector<double> ms(n3);
  for (int i = 0; i < n3; ++i) ms[i] = 1.0 / std::sqrt(mt[i]);
  const int m = std::min(n3, 40);
  std::vector<std::vector<double>> Q;
  std::vector<double> al, be, q(n3), w(n3), t(n3), y(n3);
  unsigned long long st = 0x9e3779b97f4a7c15ULL;
  double nr = 0;
  for (int i = 0; i < n3; ++i) {
    st = st * 6364136223846793005ULL + 1442695040888963407ULL;
    q[i] = (double)(st >> 11) / 9007199254740992.0 - 0.5;
    nr += q[i] * q[i];
  }
  for (int i = 0; i < n3; ++i) q[i] /= std::sqrt(nr);
  for (int k = 0; k < m; ++k) {
    Q.push_back(q);
    for (int i = 0; i < n3; ++i) t[i] = ms[i] * q[i];
    hex_apply_host(R, V8, t.data(), y.data());
    for (int i = 0; i < n3; ++i) w[i] = ms[i] * y[i];
    double a = 0;
    for (int i = 0; i < n3; ++i) a += w[i] * q[i];
    al.push_back(a);
    for (const auto& v : Q) {
      double d = 0;
      for (int i = 0; i < n3; ++i) d += w[i] * v[i];
      for (int i = 0; i < n3; ++i) w[i] -= d * v[i];
    }
    double b = 0;
    for (int i = 0; i < n3; ++i) b += w[i] * w[i];
    b = std::sqrt(b);
    if (k + 1 == m || b < 1e-12 * std::fabs(a)) break;
    be.push_back(b);
    for (int i = 0; i < n3; ++i) q[i] = w[i] / b;
  }
  return tridiag_max_eig(al, be);
}

// Largest eigenvalue of M^{-1} K on a whole trilinear brick (mass: the
// assembled lumped mass, compact layout): Lanczos in the M inner product
// with full reorthogonalisation, as for the coupled operator.
static double hex_mesh_lambda(const Brick& B, const std::vector<double>& mass) {
  const int N = B.N, n1 = N + 1, n3 = n1 * n1 * n1;
  const long n = B.nnodes;
  auto idx = [&](int ex, int ey, int ez, int i) {
    return (N * ex + i % n1) + (long)B.nn[0] * ((N * ey + (i / n1) % n1) + (long)B.nn[1] * (N * ez + i / (n1 * n1)));
  };
  auto apply = [&](const std::vector<double>& u, std::vector<double>& w) {
    std::fill(w.begin(), w.end(), 0.0);
    std::vector<double> ue(n3), re(n3);
    for (int ez = 0; ez < B.ne[2]; ++ez)
      for (int ey = 0; ey < B.ne[1]; ++ey)
        for (int ex = 0; ex < B.ne[0]; ++ex) {
          double V8[8][3];
          hex_corners(B, ex, ey, ez, V8);
          for (int i = 0; i < n3; ++i) ue[i] = u[idx(ex, ey, ez, i)];
          hex_apply_host(B.rule, V8, ue.data(), re.data());
          for (int i = 0; i < n3; ++i) w[idx(ex, ey, ez, i)] += re[i];
        }
    for (long i = 0; i < n; ++i) w[i] *= B.c * B.c / mass[i];
  };
  auto dotm = [&](const std::vector<double>& a, const std::vector<double>& b) {
    double acc = 0;
    for (long i = 0; i < n; ++i) acc += mass[i] * a[i] * b[i];
    return acc;
  };
  const int m = (int)std::min<long>(60, n);
  std::vector<std::vector<double>> Q;
  std::vector<double> al, be, w(n), q(n);
  uint64_t st = 0x9E3779B97F4A7C15ull;
  for (long i = 0; i < n; ++i) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    q[i] = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
  const double nq = std::sqrt(dotm(q, q));
  for (long i = 0; i < n; ++i) q[i] /= nq;
  Q.push_back(q);
  for (int j = 0; j < m; ++j) {
    apply(Q[j], w);
    al.push_back(dotm(w, Q[j]));
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& qi : Q) {
        const double h = dotm(w, qi);
        for (long i = 0; i < n; ++i) w[i] -= h * qi[i];
      }
    const double b = std::sqrt(dotm(w, w));
    if (j + 1 == m || !(b > 1e-12 * std::fabs(al.back()))) break;
    be.push_back(b);
    for (long i = 0; i < n; ++i) w[i] /= b;
    Q.push_back(w);
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  return tridiag_max_eig(al, be);
}

// Library-held workspace (pmdg_bind_static): one static device array per
// GPU, for callers that cannot allocate device memory.  Host code never
// passes the array's name to a kernel or a copy: the device address is
// looked up once per device with hipGetSymbolAddress and kept here.  The
// solver last bound to a device's array owns it; the others are refused.
// ------------------------------------------------------------------------
constexpr size_t kScratchBytes = 32ull << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kScratchDevices];
static const pmdg_solver* g_scratch_owner[kScratchDevices];

// The solver is bound to a library-held workspace that a later
// pmdg_bind_static on the same device has taken over.
static bool ws_lost(const pmdg_solver* s) {
  if (s->static_dev < 0) return false;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_owner[s->static_dev] != s;
}
static const char* kLostMsg = "the library-held workspace of this device was bound to another solver";

extern "C" {

const char* pmdg_last_error(void) { return g_err.c_str(); }

pmdg_status pmdg_create(const pmdg_problem* pr, pmdg_solver** out) {
  if (!out) return fail(PMDG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pr) return fail(PMDG_EINVAL, "problem is NULL");
  if (pr->ndom < 1 || pr->ndom > 2) return fail(PMDG_EINVAL, "ndom must be 1 or 2");
  if (pr->precision != 32 && pr->precision != 64) return fail(PMDG_EINVAL, "precision must be 32 or 64");
  if (pr->n_scenarios < 1) return fail(PMDG_EINVAL, "n_scenarios must be >= 1");
  if (pr->trace_capacity < 1) return fail(PMDG_EINVAL, "trace_capacity must be >= 1");
  if (pr->ndom == 2 && !(pr->penalty_alpha > 0)) return fail(PMDG_EINVAL, "penalty_alpha must be > 0");
  pmdg_solver* s = new (std::nothrow) pmdg_solver();
  if (!s) return fail(PMDG_ENOMEM, "out of host memory");
  s->pr = *pr;
  s->ndom = pr->ndom;
  s->S = pr->n_scenarios;
  s->prec = pr->precision;
  s->cap = pr->trace_capacity;
  std::string err;
  for (int d = 0; d < s->ndom; ++d)
    if (setup_brick(s->b[d], pr->dom[d], err)) {
      delete s;
      return fail(PMDG_EINVAL, "brick " + std::to_string(d) + ": " + err);
    }
  if (s->ndom == 2 && setup_interface(s, err)) {
    delete s;
    return fail(PMDG_EINVAL, err);
  }
  // time step: dt = cfl * h_min * (min GLL gap) / 2 / c over both bricks
  if (pr->dt > 0) {
    s->dt = pr->dt;
  } else {
    if (!(pr->cfl > 0)) { delete s; return fail(PMDG_EINVAL, "cfl must be > 0 when dt <= 0"); }
    double best = INFINITY;
    for (int d = 0; d < s->ndom; ++d) {
      const Brick& B = s->b[d];
      double gap = INFINITY, hm = INFINITY;
      for (int i = 0; i < B.N; ++i) gap = std::min(gap, (double)(B.rule.x[i + 1] - B.rule.x[i]));
      for (int a = 0; a < 3; ++a) hm = std::min(hm, B.h[a]);
      best = std::min(best, pr->cfl * hm * gap * 0.5 / B.c);
    }
    s->dt = best;
  }
  // explicit stability, dt^2 lambda_max < 4: the volume operator of each
  // brick (exact: the Kronecker sum of the 1D operators), then the coupled
  // operator with the interface penalty (patch estimate, with a 2% margin for
  // the difference between the patch and the whole bricks)
  for (int d = 0; d < s->ndom; ++d) {
    const Brick& B = s->b[d];
    const double lam = B.c * B.c * (B.lam1[0] + B.lam1[1] + B.lam1[2]);
    s->lam_max = std::max(s->lam_max, lam);
    if (s->dt * s->dt * lam >= 4.0) {
      delete s;
      return fail(PMDG_EUNSTABLE, "dt exceeds the explicit stability bound of brick " + std::to_string(d));
    }
  }
  if (s->ndom == 2) {
    const double lam = patch_lambda_max(s, err);
    if (!(lam > 0)) {
      delete s;
      return fail(PMDG_EINVAL, "coupled stability estimate failed: " + err);
    }
    s->lam_max = std::max(s->lam_max, lam);
    if (s->dt * s->dt * lam * 1.02 >= 4.0) {
      const double r = s->dt * s->dt * lam;
      delete s;
      return fail(PMDG_EUNSTABLE, "dt^2 lambda_max of the coupled operator is " + std::to_string(r) +
                                      " (>= 4 / 1.02): reduce cfl or penalty_alpha");
    }
  }
  s->amp.assign(s->S, 0.0);
  s->phase.assign(s->S, 0.0);
  s->freq.assign(s->S, 1.0);
  *out = s;
  return PMDG_OK;
}

pmdg_status pmdg_set_pmuts(pmdg_solver* s, int Np, const double* ctr, const double* radius, int Nm,
                           const double* omega, const double* zeta, const double* eta) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (s->bound) return fail(PMDG_ESTATE, "set_pmuts must precede bind");
  if (Np < 0 || Nm < 1 || Nm > kMaxModes || (Np > 0 && (!ctr || !radius || !omega || !zeta || !eta)))
    return fail(PMDG_EINVAL, "bad PMUT arguments (1 <= Nm <= 16)");
  s->Np = Np;
  s->Nm = Nm;
  s->ctr.assign(ctr, ctr + 2 * Np);
  s->rad.assign(radius, radius + Np);
  s->omega.assign(omega, omega + (size_t)Np * Nm);
  s->zeta.assign(zeta, zeta + (size_t)Np * Nm);
  s->eta.assign(eta, eta + (size_t)Np * Nm);
  const Brick& B = s->b[0];
  std::vector<int> owner(face0(s), -1);
  s->pm_off.assign(Np + 1, 0);
  s->pm_node.clear();
  s->pm_wf.clear();
  // trilinear hexahedra: bottom-face node coordinates and the assembled face
  // weights w_a w_b |dX/dxi x dX/deta| of the face zeta = -1
  std::vector<double> hx, hy, hw;
  if (B.mapped()) {
    const long nf = face0(s);
    hx.assign(nf, 0.0);
    hy.assign(nf, 0.0);
    hw.assign(nf, 0.0);
    for (int j = 0; j < B.nn[1]; ++j)
      for (int i = 0; i < B.nn[0]; ++i) {
        double x[3];
        hex_node_xyz(B, i, j, 0, x);
        hx[i + (long)B.nn[0] * j] = x[0];
        hy[i + (long)B.nn[0] * j] = x[1];
      }
    for (int ey = 0; ey < B.ne[1]; ++ey)
      for (int ex = 0; ex < B.ne[0]; ++ex) {
        double V8[8][3];
        hex_corners(B, ex, ey, 0, V8);
        for (int b = 0; b <= B.N; ++b)
          for (int a = 0; a <= B.N; ++a) {
            const double xi[3] = {(double)B.rule.x[a], (double)B.rule.x[b], -1.0};
            double x[3], J[3][3];
            hex_map(V8, xi, x, J);
            const double n0 = J[1][0] * J[2][1] - J[2][0] * J[1][1], n1 = J[2][0] * J[0][1] - J[0][0] * J[2][1],
                         n2 = J[0][0] * J[1][1] - J[1][0] * J[0][1];
            hw[(B.N * ex + a) + (long)B.nn[0] * (B.N * ey + b)] +=
                (double)(B.rule.w[a] * B.rule.w[b]) * std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
          }
      }
  }
  for (int k = 0; k < Np; ++k) {
    s->pm_off[k] = (int)s->pm_node.size();
    for (int j = 0; j < B.nn[1]; ++j)
      for (int i = 0; i < B.nn[0]; ++i) {
        const long f = i + (long)B.nn[0] * j;
        const double xn = B.mapped() ? hx[f] : B.coord(0, i), yn = B.mapped() ? hy[f] : B.coord(1, j);
        const double dx = xn - ctr[2 * k], dy = yn - ctr[2 * k + 1];
        if (std::sqrt(dx * dx + dy * dy) <= radius[k]) {
          if (owner[f] >= 0) return fail(PMDG_EINVAL, "PMUT discs overlap");
          owner[f] = k;
          s->pm_node.push_back(i + B.px * j);  // device (padded) face index
          // face quadrature weight: on bricks the product of the assembled
          // 1D lumped masses
          s->pm_wf.push_back(B.mapped() ? hw[f] : B.mass1[0][i] * B.mass1[1][j]);
        }
      }
  }
  s->pm_off[Np] = (int)s->pm_node.size();
  s->pm_B.assign(s->pm_node.size() * Nm, 0.0);
  s->shape_set.assign(Np, 0);
  s->amp.assign((size_t)s->S * Np, 0.0);
  s->phase.assign((size_t)s->S * Np, 0.0);
  return PMDG_OK;
}

pmdg_status pmdg_pmut_face_nodes(pmdg_solver* s, int k, int* n, double* xyz) {
  if (!s || !n) return fail(PMDG_EINVAL, "NULL argument");
  if (k < 0 || k >= s->Np) return fail(PMDG_EINVAL, "PMUT index out of range");
  const int o = s->pm_off[k], cnt = s->pm_off[k + 1] - o;
  *n = cnt;
  if (xyz) {
    const Brick& B = s->b[0];
    for (int m = 0; m < cnt; ++m) {
      const int f = s->pm_node[o + m];
      if (B.mapped()) {
        hex_node_xyz(B, f % B.px, f / B.px, 0, xyz + 3 * m);
        continue;
      }
      xyz[3 * m] = B.coord(0, f % B.px);
      xyz[3 * m + 1] = B.coord(1, f / B.px);
      xyz[3 * m + 2] = B.x0[2];
    }
  }
  return PMDG_OK;
}

pmdg_status pmdg_set_pmut_shape(pmdg_solver* s, int k, const double* shape) {
  if (!s || !shape) return fail(PMDG_EINVAL, "NULL argument");
  if (s->bound) return fail(PMDG_ESTATE, "set_pmut_shape must precede bind");
  if (k < 0 || k >= s->Np) return fail(PMDG_EINVAL, "PMUT index out of range");
  const int o = s->pm_off[k], cnt = s->pm_off[k + 1] - o, Nm = s->Nm;
  const Brick& B = s->b[0];
  const double kappa = B.rho * B.c * B.c;
  for (int m = 0; m < Nm; ++m) {
    double X = 0;
    for (int n = 0; n < cnt; ++n) {
      const double bv = s->pm_wf[o + n] * shape[(size_t)m * cnt + n];
      s->pm_B[(size_t)(o + n) * Nm + m] = bv;
      const int f = s->pm_node[o + n];
      const double M = B.mass1[0][f % B.px] * B.mass1[1][f / B.px] * B.mass1[2][0];
      X += bv * bv / M;
    }
    X *= kappa * s->dt * s->dt;
    if (X > 2.0)
      return fail(PMDG_EUNSTABLE, "PMUT coupling strength kappa dt^2 b^T M^-1 b = " + std::to_string(X) +
                                      " exceeds 2 (synchronised explicit coupling unstable)");
  }
  s->shape_set[k] = 1;
  return PMDG_OK;
}

pmdg_status pmdg_set_drive(pmdg_solver* s, const double* amp, const double* phase, const double* freq, double ncyc,
                           int envelope) {
  if (!s || (s->Np > 0 && (!amp || !phase)) || !freq) return fail(PMDG_EINVAL, "NULL argument");
  if (envelope < 0 || envelope > 2 || !(ncyc > 0)) return fail(PMDG_EINVAL, "bad envelope or ncyc");
  if (s->bound && ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  for (int i = 0; i < s->S; ++i)
    if (!(freq[i] > 0)) return fail(PMDG_EINVAL, "freq must be > 0");
  const size_t n = (size_t)s->S * s->Np;
  s->amp.assign(amp, amp + n);
  s->phase.assign(phase, phase + n);
  s->freq.assign(freq, freq + s->S);
  s->ncyc = ncyc;
  s->envelope = envelope;
  s->drive_cached = false;
  drop_graphs(s);
  if (s->bound && s->Np > 0) {
    hipStream_t st = nullptr;
    pmdg_status r;
    drive_tables(s, s->dA_h, s->car_h);
    s->drive_cached = true;
    if ((r = upload_vec(s, "dA", s->dA_h, st))) return r;
    if ((r = upload_vec(s, "car", s->car_h, st))) return r;
  }
  return PMDG_OK;
}

pmdg_status pmdg_set_rx(pmdg_solver* s, double t_switch, double cap) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (!(cap != 0)) return fail(PMDG_EINVAL, "capacitance must be non-zero");
  s->t_switch = t_switch;
  s->rx_cap = cap;
  drop_graphs(s);
  return PMDG_OK;
}

pmdg_status pmdg_set_absorbing(pmdg_solver* s, int dom, int faces) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (s->bound) return fail(PMDG_ESTATE, "set_absorbing must precede bind");
  if (dom < 0 || dom >= s->ndom) return fail(PMDG_EINVAL, "no such domain");
  if (faces < 0 || faces > 63) return fail(PMDG_EINVAL, "faces is a mask of 6 bits");
  if (faces && s->b[dom].mapped()) return fail(PMDG_EINVAL, "absorbing faces are not built on trilinear hexahedra");
  if (s->ndom > 1 && (faces & (dom == 0 ? 32 : 16)))
    return fail(PMDG_EINVAL, "the interface face of a coupled brick cannot be absorbing");
  s->b[dom].absorbing = faces;
  return PMDG_OK;
}

pmdg_status pmdg_set_pml(pmdg_solver* s, int dom, const double* ell, double R) {
  if (!s || !ell) return fail(PMDG_EINVAL, "NULL argument");
  if (s->bound) return fail(PMDG_ESTATE, "set_pml must precede bind");
  if (dom < 0 || dom >= s->ndom) return fail(PMDG_EINVAL, "domain out of range");
  if (!(R > 0 && R < 1)) return fail(PMDG_EINVAL, "the reflection coefficient R must be in (0, 1)");
  Brick& B = s->b[dom];
  if (B.mapped()) return fail(PMDG_EINVAL, "layers are not built on trilinear hexahedra");
  for (int a = 0; a < 3; ++a) {
    const double L = B.h[a] * B.ne[a];
    if (!(ell[2 * a] >= 0) || !(ell[2 * a + 1] >= 0) || ell[2 * a] + ell[2 * a + 1] > L * (1 + 1e-12))
      return fail(PMDG_EINVAL, "layer thicknesses must be >= 0 and fit in the brick");
  }
  if (s->ndom == 2 && ((dom == 0 && ell[5] > 0) || (dom == 1 && ell[4] > 0)))
    return fail(PMDG_EINVAL, "the interface faces of two coupled bricks carry no layer");
  if (B.N > kPmlMaxOrder) return fail(PMDG_EINVAL, "layers are built for orders up to 6");
  // the profile of Sec. 2 at distance d into a layer of thickness l
  auto prof = [&](double d, double l) {
    if (!(l > 0) || d <= 0) return 0.0;
    d = std::min(d, l);
    return B.c / l * std::log(1.0 / R) * (d / l - std::sin(2.0 * M_PI * d / l) / (2.0 * M_PI));
  };
  for (int a = 0; a < 3; ++a) {
    B.pzeta[a].assign(B.nn[a], 0.0);
    const double lo = B.x0[a] + ell[2 * a], hi = B.x0[a] + B.h[a] * B.ne[a] - ell[2 * a + 1];
    for (int i = 0; i < B.nn[a]; ++i) {
      const double x = B.coord(a, i);
      double z = 0.0;
      if (ell[2 * a] > 0 && x < lo) z = prof(lo - x, ell[2 * a]);
      if (ell[2 * a + 1] > 0 && x > hi) z = prof(x - hi, ell[2 * a + 1]);
      B.pzeta[a][i] = z;
    }
  }
  const int N = B.N;
  B.eslot.assign((size_t)B.ne[0] * B.ne[1] * B.ne[2], -1);
  B.pel.clear();
  std::vector<char> mark(B.nnodes, 0);
  for (int ez = 0; ez < B.ne[2]; ++ez)
    for (int ey = 0; ey < B.ne[1]; ++ey)
      for (int ex = 0; ex < B.ne[0]; ++ex) {
        bool any = false;
        for (int m = 0; m <= N; ++m)
          any = any || B.pzeta[0][N * ex + m] > 0 || B.pzeta[1][N * ey + m] > 0 || B.pzeta[2][N * ez + m] > 0;
        if (!any) continue;
        B.eslot[ex + (size_t)B.ne[0] * (ey + (size_t)B.ne[1] * ez)] = (int)(B.pel.size() / 3);
        B.pel.insert(B.pel.end(), {ex, ey, ez});
        for (int c = 0; c <= N; ++c)
          for (int b = 0; b <= N; ++b)
            for (int aa = 0; aa <= N; ++aa)
              mark[(N * ex + aa) + (long)B.nn[0] * ((N * ey + b) + (long)B.nn[1] * (N * ez + c))] = 1;
      }
  B.pnode.clear();
  for (int k = 0; k < B.nn[2]; ++k)
    for (int j = 0; j < B.nn[1]; ++j)
      for (int i = 0; i < B.nn[0]; ++i)
        if (mark[i + (long)B.nn[0] * (j + (long)B.nn[1] * k)]) B.pnode.insert(B.pnode.end(), {i, j, k});
  B.pml = !B.pel.empty();
  return PMDG_OK;
}

pmdg_status pmdg_match_faces(int nq, int nf, const double* fine_hex, const int* fine_face, int nc,
                             const double* coarse_hex, const int* coarse_face, double tol, double eps, int* elem,
                             double* xi, int* unmatched, void* stream) {
  if (nq < 1 || nq > kMaxNq) return fail(PMDG_EINVAL, "nq must be in 1..9");
  if (nf < 0 || nc < 0) return fail(PMDG_EINVAL, "face counts must be >= 0");
  if (!(tol > 0) || !(eps >= 0)) return fail(PMDG_EINVAL, "tol must be > 0 and eps >= 0");
  if (!unmatched || (nf > 0 && (!fine_hex || !fine_face || !elem || !xi)) || (nc > 0 && (!coarse_hex || !coarse_face)))
    return fail(PMDG_EINVAL, "NULL array");
  if ((long)nf * nq * nq > (1L << 31) - 1) return fail(PMDG_EINVAL, "too many points");
  MatchArgs a;
  memset(&a, 0, sizeof(a));
  a.nq = nq;
  a.nf = nf;
  a.nc = nc;
  a.fine_hex = fine_hex;
  a.fine_face = fine_face;
  a.coarse_hex = coarse_hex;
  a.coarse_face = coarse_face;
  a.tol = tol;
  a.eps = eps;
  a.elem = elem;
  a.xi = xi;
  a.unmatched = unmatched;
  std::vector<ld> gx, gw;
  gl_rule(nq, gx, gw);
  for (int i = 0; i < nq; ++i) a.gq[i] = (double)gx[i];
  HIPCHK(launch_match(a, (hipStream_t)stream));
  return PMDG_OK;
}

pmdg_status pmdg_set_vertices(pmdg_solver* s, int dom, const double* V) {
  if (!s || !V) return fail(PMDG_EINVAL, "NULL argument");
  if (s->bound) return fail(PMDG_ESTATE, "set_vertices must precede bind");
  if (s->ndom != 1 || dom != 0) return fail(PMDG_EINVAL, "trilinear hexahedra are built for single-brick solvers");
  Brick& B = s->b[0];
  if (B.absorbing || B.pml)
    return fail(PMDG_EINVAL, "absorbing faces and layers are not built on trilinear hexahedra");
  if (s->Np > 0 || s->R > 0) return fail(PMDG_ESTATE, "set_vertices must precede set_pmuts and set_receivers");
  const long nv = (long)(B.ne[0] + 1) * (B.ne[1] + 1) * (B.ne[2] + 1);
  for (long i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(V[i])) return fail(PMDG_EINVAL, "vertex coordinates must be finite");
  std::vector<double> old;
  old.swap(B.V);
  B.V.assign(V, V + 3 * nv);
  const int N = B.N, n1 = N + 1;
  const long nel = (long)B.ne[0] * B.ne[1] * B.ne[2];
  std::vector<double> mass(B.nnodes, 0.0), hvert((size_t)nel * 24, 0.0);
  double hm = INFINITY, lam = 0;
  for (int ez = 0; ez < B.ne[2]; ++ez)
    for (int ey = 0; ey < B.ne[1]; ++ey)
      for (int ex = 0; ex < B.ne[0]; ++ex) {
        const long e = ex + (long)B.ne[0] * (ey + (long)B.ne[1] * ez);
        double V8[8][3];
        hex_corners(B, ex, ey, ez, V8);
        for (int c = 0; c < 8; ++c)
          for (int a = 0; a < 3; ++a) hvert[e * 24 + 3 * c + a] = V8[c][a] - V8[0][a];
        for (int c = 0; c < 8; ++c)
          for (int a = 0; a < 3; ++a) {
            if ((c >> a) & 1) continue;
            const int c2 = c | (1 << a);
            const double d0 = V8[c2][0] - V8[c][0], d1 = V8[c2][1] - V8[c][1], d2 = V8[c2][2] - V8[c][2];
            hm = std::min(hm, std::sqrt(d0 * d0 + d1 * d1 + d2 * d2));
          }
        for (int c = 0; c <= N; ++c)
          for (int b = 0; b <= N; ++b)
            for (int a = 0; a <= N; ++a) {
              const double xi[3] = {(double)B.rule.x[a], (double)B.rule.x[b], (double)B.rule.x[c]};
              double x[3], J[3][3], A[3][3];
              hex_map(V8, xi, x, J);
              const double det = hex_adj(J, A);
              if (!(det > 0)) {
                B.V.swap(old);
                return fail(PMDG_EINVAL, "the Jacobian of element " + std::to_string(e) + " is not positive");
              }
              mass[(N * ex + a) + (long)B.nn[0] * ((N * ey + b) + (long)B.nn[1] * (N * ez + c))] +=
                  (double)(B.rule.w[a] * B.rule.w[b] * B.rule.w[c]) * det;
            }
      }
  // Stability.  Meshes of up to kHexLanczosNodes nodes: Lanczos on the
  // whole operator, with a 2% margin for its estimate from below.  Larger
  // ones: with Mt_e the assembled lumped mass of each node divided by the
  // number of elements holding it, p.M p = sum_e p_e.Mt_e p_e and
  // p.K p = sum_e p_e.K_e p_e, so lambda_max(M^{-1} K) <= max_e
  // lambda_max(Mt_e^{-1} K_e), an upper bound needing no margin.  The
  // element value depends on the element's shape and Mt_e up to translation
  // and scale (lambda ~ 1 / L^2): it is cached by the normalised corner
  // offsets and masses.
  constexpr long kHexLanczosNodes = 150000;
  double margin = 1.0;
  if (B.nnodes <= kHexLanczosNodes) {
    lam = hex_mesh_lambda(B, mass);
    margin = 1.02;
  } else {
    const int n3 = n1 * n1 * n1;
    std::map<std::vector<long long>, double> cache;
    std::vector<double> mt(n3);
    std::vector<long long> key(21 + n3);
    for (int ez = 0; ez < B.ne[2]; ++ez)
      for (int ey = 0; ey < B.ne[1]; ++ey)
        for (int ex = 0; ex < B.ne[0]; ++ex) {
          double V8[8][3], W8[8][3], L = 0;
          hex_corners(B, ex, ey, ez, V8);
          for (int c = 1; c < 8; ++c)
            for (int a = 0; a < 3; ++a) L = std::max(L, std::fabs(V8[c][a] - V8[0][a]));
          for (int c = 0; c < 8; ++c)
            for (int a = 0; a < 3; ++a) {
              W8[c][a] = (V8[c][a] - V8[0][a]) / L;
              if (c > 0) key[3 * (c - 1) + a] = std::llround(W8[c][a] * 1e9);
            }
          const int g0[3] = {N * ex, N * ey, N * ez};
          for (int i = 0; i < n3; ++i) {
            const int l[3] = {i % n1, (i / n1) % n1, i / (n1 * n1)};
            int mult = 1;
            for (int a = 0; a < 3; ++a) {
              const int gi = g0[a] + l[a];
              if (gi % N == 0 && gi > 0 && gi < N * B.ne[a]) mult *= 2;
            }
            mt[i] = mass[(g0[0] + l[0]) + (long)B.nn[0] * ((g0[1] + l[1]) + (long)B.nn[1] * (g0[2] + l[2]))] /
                    mult / (L * L * L);
            key[21 + i] = std::llround(mt[i] * 1e9);
          }
          auto it = cache.find(key);
          double ln;
          if (it != cache.end()) {
            ln = it->second;
          } else {
            ln = hex_elem_lambda(B.rule, W8, mt.data());
            cache.emplace(key, ln);
          }
          lam = std::max(lam, B.c * B.c * ln / (L * L));
        }
  }
  double dt = s->dt;
  if (!(s->pr.dt > 0)) {
    double gap = INFINITY;
    for (int i = 0; i < N; ++i) gap = std::min(gap, (double)(B.rule.x[i + 1] - B.rule.x[i]));
    dt = s->pr.cfl * hm * gap * 0.5 / B.c;
  }
  if (dt * dt * lam * margin >= 4.0) {
    B.V.swap(old);
    return fail(PMDG_EUNSTABLE, "dt^2 lambda_max of the trilinear mesh is " + std::to_string(dt * dt * lam) +
                                    " (>= 4): reduce cfl");
  }
  B.hminv.assign((size_t)B.pnodes, 0.0);
  for (int k = 0; k < B.nn[2]; ++k)
    for (int j = 0; j < B.nn[1]; ++j)
      for (int i = 0; i < B.nn[0]; ++i)
        B.hminv[i + (size_t)B.px * (j + (size_t)B.nn[1] * k)] =
            1.0 / mass[i + (size_t)B.nn[0] * (j + (size_t)B.nn[1] * k)];
  B.hvert.swap(hvert);
  s->dt = dt;
  s->lam_max = lam;
  return PMDG_OK;
}

pmdg_status pmdg_set_receivers(pmdg_solver* s, int R, const double* xyz) {
  if (!s || R < 0 || (R > 0 && !xyz)) return fail(PMDG_EINVAL, "bad receiver arguments");
  if (s->bound) return fail(PMDG_ESTATE, "set_receivers must precede bind");
  s->R = R;
  s->r_dom.assign(R, 0);
  s->r_base.assign(R, 0);
  s->r_w.assign((size_t)R * 3 * (kMaxOrder + 1), 0.0);
  for (int r = 0; r < R; ++r) {
    bool ok = false;
    for (int d = 0; d < s->ndom && !ok; ++d) {
      const Brick& B = s->b[d];
      int e[3];
      ld xi[3];
      bool in = true;
      if (B.mapped()) {
        // lowest element (x fastest) whose inverse map puts the point in
        // [-1, 1]^3 up to 1e-10
        in = false;
        for (int ez = 0; ez < B.ne[2] && !in; ++ez)
          for (int ey = 0; ey < B.ne[1] && !in; ++ey)
            for (int ex = 0; ex < B.ne[0] && !in; ++ex) {
              double V8[8][3], t[3];
              hex_corners(B, ex, ey, ez, V8);
              if (!hex_inverse(V8, xyz + 3 * r, t)) continue;
              if (std::fabs(t[0]) <= 1 + 1e-10 && std::fabs(t[1]) <= 1 + 1e-10 && std::fabs(t[2]) <= 1 + 1e-10) {
                in = true;
                e[0] = ex; e[1] = ey; e[2] = ez;
                for (int a = 0; a < 3; ++a) xi[a] = t[a];
              }
            }
      }
      for (int a = 0; a < 3 && in && !B.mapped(); ++a) {
        int found = -1;
        for (int k = 0; k < B.ne[a]; ++k) {
          const ld t = 2 * (xyz[3 * r + a] - (B.x0[a] + k * (ld)B.h[a])) / B.h[a] - 1;
          if (t >= -1 - 1e-12L && t <= 1 + 1e-12L) { found = k; xi[a] = t; break; }
        }
        if (found < 0) in = false;
        else e[a] = found;
      }
      if (!in) continue;
      ok = true;
      s->r_dom[r] = d;
      s->r_base[r] = (long)B.N * e[0] + (long)B.px * B.N * e[1] + B.pplane * B.N * e[2];
      for (int a = 0; a < 3; ++a) {
        ld v[kMaxOrder + 1];
        bary_eval(B.rule, xi[a], v);
        for (int i = 0; i <= B.N; ++i) s->r_w[((size_t)r * 3 + a) * (kMaxOrder + 1) + i] = (double)v[i];
      }
    }
    if (!ok) return fail(PMDG_EINVAL, "receiver " + std::to_string(r) + " lies outside the mesh");
  }
  return PMDG_OK;
}

pmdg_status pmdg_workspace_size(pmdg_solver* s, size_t* bytes) {
  if (!s || !bytes) return fail(PMDG_EINVAL, "NULL argument");
  *bytes = layout(s);
  return PMDG_OK;
}

}  // extern "C"

// Zeroes the solver's workspace and uploads every table: the state of
// step 0, everything at rest (pmdg_bind and pmdg_restart).
static pmdg_status fill_workspace(pmdg_solver* s, hipStream_t st) {
  // fill kernel: safe under capture on any stream
  HIPCHK(launch_fill_bytes(s->ws, s->ws_need / 4 * 4, st));
  pmdg_status r = s->prec == 64 ? bind_tables<double>(s, st) : bind_tables<float>(s, st);
  if (r) return r;
  if (s->Np > 0) {
    if ((r = upload_vec(s, "pm_off", s->pm_off, st))) return r;
    if ((r = upload_vec(s, "pm_node", s->pm_node, st))) return r;
    if ((r = upload_vec(s, "pm_B", s->pm_B, st))) return r;
    if ((r = upload_vec(s, "omega", s->omega, st))) return r;
    if ((r = upload_vec(s, "zeta", s->zeta, st))) return r;
    if ((r = upload_vec(s, "eta", s->eta, st))) return r;
    if (!s->drive_cached) {
      drive_tables(s, s->dA_h, s->car_h);
      s->drive_cached = true;
    }
    if ((r = upload_vec(s, "dA", s->dA_h, st))) return r;
    if ((r = upload_vec(s, "car", s->car_h, st))) return r;
  }
  if (s->R > 0) {
    if ((r = upload_vec(s, "r_dom", s->r_dom, st))) return r;
    if ((r = upload_vec(s, "r_base", s->r_base, st))) return r;
    if ((r = upload_vec(s, "r_w", s->r_w, st))) return r;
  }
  HIPCHK(hipStreamSynchronize(st));
  s->steps_done = 0;
  return PMDG_OK;
}

extern "C" {

pmdg_status pmdg_bind(pmdg_solver* s, void* dev_ptr, size_t bytes, void* stream) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (s->bound) return fail(PMDG_ESTATE, "already bound");
  if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return fail(PMDG_EINVAL, "workspace must be 256-byte aligned");
  for (int k = 0; k < s->Np; ++k)
    if (!s->shape_set[k]) return fail(PMDG_ESTATE, "mode shape of PMUT " + std::to_string(k) + " not set");
  const size_t need = layout(s);
  if (bytes < need) return fail(PMDG_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  s->ws = (char*)dev_ptr;
  s->ws_bytes = bytes;
  s->ws_need = need;
  const pmdg_status r = fill_workspace(s, (hipStream_t)stream);
  if (r) {
    s->ws = nullptr;
    return r;
  }
  s->bound = true;
  return PMDG_OK;
}

pmdg_status pmdg_restart(pmdg_solver* s, void* stream) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (!s->bound) return fail(PMDG_ESTATE, "not bound");
  if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  drop_graphs(s);
  return fill_workspace(s, (hipStream_t)stream);
}

pmdg_status pmdg_bind_static(pmdg_solver* s, void* stream) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (s->bound) return fail(PMDG_ESTATE, "already bound");
  for (int k = 0; k < s->Np; ++k)
    if (!s->shape_set[k]) return fail(PMDG_ESTATE, "mode shape of PMUT " + std::to_string(k) + " not set");
  const size_t need = layout(s);
  if (need > kScratchBytes)
    return fail(PMDG_ENOMEM, "the solver needs " + std::to_string(need) + " bytes; the library-held workspace holds " +
                                 std::to_string(kScratchBytes) + ": bind caller memory with pmdg_bind");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(PMDG_EINVAL, "device index beyond the library-held workspaces");
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      if (!p || ((uintptr_t)p & 255)) return fail(PMDG_EHIP, "library-held workspace has no aligned device address");
      g_scratch_ptr[dev] = (char*)p;
    }
    base = g_scratch_ptr[dev];
    g_scratch_owner[dev] = s;
  }
  s->static_dev = dev;
  const pmdg_status r = pmdg_bind(s, base, kScratchBytes, stream);
  if (r) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_owner[dev] == s) g_scratch_owner[dev] = nullptr;
    s->static_dev = -1;
  }
  return r;
}

pmdg_status pmdg_get_dt(pmdg_solver* s, double* dt) {
  if (!s || !dt) return fail(PMDG_EINVAL, "NULL argument");
  *dt = s->dt;
  return PMDG_OK;
}

pmdg_status pmdg_lambda_max(pmdg_solver* s, double* lam) {
  if (!s || !lam) return fail(PMDG_EINVAL, "NULL argument");
  *lam = s->lam_max;
  return PMDG_OK;
}

pmdg_status pmdg_num_nodes(pmdg_solver* s, long* n) {
  if (!s || !n) return fail(PMDG_EINVAL, "NULL argument");
  *n = s->b[0].nnodes + (s->ndom > 1 ? s->b[1].nnodes : 0);
  return PMDG_OK;
}

pmdg_status pmdg_node_coords(pmdg_solver* s, double* xyz) {
  if (!s || !xyz) return fail(PMDG_EINVAL, "NULL argument");
  long o = 0;
  for (int d = 0; d < s->ndom; ++d) {
    const Brick& B = s->b[d];
    for (int k = 0; k < B.nn[2]; ++k)
      for (int j = 0; j < B.nn[1]; ++j)
        for (int i = 0; i < B.nn[0]; ++i, ++o) {
          if (B.mapped()) {
            hex_node_xyz(B, i, j, k, xyz + 3 * o);
            continue;
          }
          xyz[3 * o] = B.coord(0, i);
          xyz[3 * o + 1] = B.coord(1, j);
          xyz[3 * o + 2] = B.coord(2, k);
        }
  }
  return PMDG_OK;
}

pmdg_status pmdg_set_option(pmdg_solver* s, int option, long value) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (s->batches > 0 && option != PMDG_OPT_GRAPH && option != PMDG_OPT_GRAPH_CHUNK && option != PMDG_OPT_TIMING)
    return fail(PMDG_ESTATE, "the solver is held by a batch, whose tile layout was fixed at pmdg_batch_create");
  switch (option) {
    case PMDG_OPT_GRAPH: s->use_graph = value ? 1 : 0; break;
    case PMDG_OPT_TILE_ROWS:
      if (!(value == 0 || value == 1 || value == 2 || value == 4))
        return fail(PMDG_EINVAL, "tile rows per wave must be 0 (automatic), 1, 2 or 4");
      s->rows = (int)value;
      break;
    case PMDG_OPT_TILE_ZCHUNK:
      if (value < -1) return fail(PMDG_EINVAL, "zchunk must be >= -1");
      s->zchunk = (int)value;
      break;
    case PMDG_OPT_OVERLAP:
      if (!(value >= 0 && value <= 3)) return fail(PMDG_EINVAL, "overlap mode must be 0, 1, 2 or 3");
      s->overlap = (int)value;
      break;
    case PMDG_OPT_TIME_BLOCK:
      if (!(value == 1 || value == 2)) return fail(PMDG_EINVAL, "steps per stiffness pass must be 1 or 2");
      s->tblock = (int)value;
      break;
    case PMDG_OPT_TIME_BLOCK_SECONDARY:
      if (!(value == 0 || value == 1 || value == 2))
        return fail(PMDG_EINVAL, "steps per stiffness pass must be 0 (as the primary), 1 or 2");
      s->tblock1 = (int)value;
      break;
    case PMDG_OPT_PREFETCH:
      if (!(value >= 2 && value <= 4)) return fail(PMDG_EINVAL, "prefetch distance must be 2, 3 or 4 planes");
      s->depth = (int)value;
      break;
    case PMDG_OPT_TILE_WAVES:
      if (!(value == 4 || value == 8)) return fail(PMDG_EINVAL, "waves per stiffness workgroup must be 4 or 8");
      s->waves = (int)value;
      break;
    case PMDG_OPT_TILE_ROWS_SECONDARY:
      if (!(value == 0 || value == 1 || value == 2 || value == 4))
        return fail(PMDG_EINVAL, "tile rows per wave must be 0 (as the primary), 1, 2 or 4");
      s->rows1 = (int)value;
      break;
    case PMDG_OPT_TILE_ZCHUNK_SECONDARY:
      if (value < -1) return fail(PMDG_EINVAL, "zchunk must be >= -1");
      s->zchunk1 = (int)value;
      break;
    case PMDG_OPT_GRAPH_CHUNK:
      if (value < 1) return fail(PMDG_EINVAL, "graph chunk must be >= 1");
      s->graph_chunk = (int)value;
      break;
    case PMDG_OPT_TIMING: s->timing = value ? 1 : 0; break;
    case PMDG_OPT_RESIDENT:
      if (!(value == 0 || value == 1)) return fail(PMDG_EINVAL, "resident mode must be 0 (never) or 1 (automatic)");
      s->resident = (int)value;
      break;
    default: return fail(PMDG_EINVAL, "unknown option");
  }
  drop_graphs(s);
  return PMDG_OK;
}

pmdg_status pmdg_step(pmdg_solver* s, int n, void* stream) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (!s->bound) return fail(PMDG_ESTATE, "bind before stepping");
  if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  if (n < 0) return fail(PMDG_EINVAL, "n must be >= 0");
  if (s->steps_done + n > s->cap) return fail(PMDG_ESTATE, "trace capacity (maximum step count) exceeded");
  if (n == 0) return PMDG_OK;
  hipStream_t st = (hipStream_t)stream;
  if (s->timing) {
    Timer tm;
    pmdg_status r = enqueue(s, st, n, &tm);
    if (r) {
      tm.release();
      return r;
    }
    HIPCHK(hipStreamSynchronize(st));
    double tot[3] = {0, 0, 0};
    for (auto& e : tm.ev) {
      float ms;
      HIPCHK(hipEventElapsedTime(&ms, e.second.first, e.second.second));
      tot[e.first] += ms;
    }
    tm.release();
    for (int c = 0; c < 3; ++c) s->ktimes[c] = tot[c] / n;
    s->steps_done += n;
    return PMDG_OK;
  }
  ResidentArgs ra;
  if (!s->use_graph || resident_args(s, &ra)) {
    // (the LDS-resident path runs many steps per launch: no graphs needed)
    pmdg_status r = enqueue(s, st, n, nullptr);
    if (r) return r;
    s->steps_done += n;
    return PMDG_OK;
  }
  // graph replay in chunks; capture happens on a private stream so that the
  // caller's stream may be the legacy default stream
  if (!s->cap_stream) HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  int left = n;
  while (left > 0) {
    const int len = std::min(left, s->graph_chunk);
    auto it = s->graphs.find(len);
    if (it == s->graphs.end()) {
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
      pmdg_status r = PMDG_OK;
      r = enqueue(s, s->cap_stream, len, nullptr);
      hipError_t ec = hipStreamEndCapture(s->cap_stream, &g);
      if (r) return r;
      if (ec != hipSuccess) return fail(PMDG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
      hipGraphExec_t ex;
      ec = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (ec != hipSuccess) return fail(PMDG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ec));
      it = s->graphs.emplace(len, ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, st));
    left -= len;
  }
  s->steps_done += n;
  return PMDG_OK;
}

pmdg_status pmdg_resident(pmdg_solver* s, int* on) {
  if (!s || !on) return fail(PMDG_EINVAL, "NULL argument");
  if (!s->bound) return fail(PMDG_ESTATE, "not bound");
  ResidentArgs ra;
  *on = resident_args(s, &ra) ? 1 : 0;
  return PMDG_OK;
}

pmdg_status pmdg_steps_done(pmdg_solver* s, long* n) {
  if (!s || !n) return fail(PMDG_EINVAL, "NULL argument");
  *n = s->steps_done;
  return PMDG_OK;
}

pmdg_status pmdg_kernel_times(pmdg_solver* s, double* ms3) {
  if (!s || !ms3) return fail(PMDG_EINVAL, "NULL argument");
  for (int c = 0; c < 3; ++c) ms3[c] = s->ktimes[c];
  return PMDG_OK;
}

pmdg_status pmdg_read_traces(pmdg_solver* s, double* out, void* stream) {
  if (!s || !out) return fail(PMDG_EINVAL, "NULL argument");
  if (!s->bound) return fail(PMDG_ESTATE, "not bound");
  if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  if (s->R == 0) return PMDG_OK;
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  std::vector<double> all((size_t)s->S * s->R * s->cap);
  HIPCHK(hipMemcpy(all.data(), dptr<double>(s, "traces"), all.size() * sizeof(double), hipMemcpyDeviceToHost));
  const long n = std::min(s->steps_done, s->cap);
  for (long sr = 0; sr < (long)s->S * s->R; ++sr)
    memcpy(out + sr * n, all.data() + sr * s->cap, n * sizeof(double));
  return PMDG_OK;
}

pmdg_status pmdg_read_traces_device(pmdg_solver* s, void* out, int bits, void* stream) {
  if (!s || !out) return fail(PMDG_EINVAL, "NULL argument");
  if (bits != 32 && bits != 64) return fail(PMDG_EINVAL, "bits must be 32 or 64");
  if (!s->bound) return fail(PMDG_ESTATE, "not bound");
  if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  if (s->R == 0) return PMDG_OK;
  const long n = std::min(s->steps_done, s->cap);
  HIPCHK(launch_pack_traces(dptr<double>(s, "traces"), out, bits, s->cap, n, (long)s->S * s->R,
                            (hipStream_t)stream));
  return PMDG_OK;
}

pmdg_status pmdg_read_modal(pmdg_solver* s, int sc, double* q, double* qd, double* qdd, void* stream) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (!s->bound) return fail(PMDG_ESTATE, "not bound");
  if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  if (sc < 0 || sc >= s->S) return fail(PMDG_EINVAL, "scenario out of range");
  if (s->Np == 0) return PMDG_OK;
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  const size_t nm = (size_t)s->Np * s->Nm, off = nm * sc;
  if (q) HIPCHK(hipMemcpy(q, dptr<double>(s, "q") + off, nm * 8, hipMemcpyDeviceToHost));
  if (qd) HIPCHK(hipMemcpy(qd, dptr<double>(s, "qd") + off, nm * 8, hipMemcpyDeviceToHost));
  if (qdd) HIPCHK(hipMemcpy(qdd, dptr<double>(s, "qdd") + off, nm * 8, hipMemcpyDeviceToHost));
  return PMDG_OK;
}

pmdg_status pmdg_get_state(pmdg_solver* s, int sc, double* p, double* p_prev, void* stream) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (!s->bound) return fail(PMDG_ESTATE, "not bound");
  if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  if (sc < 0 || sc >= s->S) return fail(PMDG_EINVAL, "scenario out of range");
  return s->prec == 64 ? get_state_t<double>(s, sc, p, p_prev, (hipStream_t)stream)
                       : get_state_t<float>(s, sc, p, p_prev, (hipStream_t)stream);
}

pmdg_status pmdg_set_state(pmdg_solver* s, int sc, const double* p, const double* p_prev, const double* q,
                           const double* qd, const double* qdd, long nstep, void* stream) {
  if (!s) return fail(PMDG_EINVAL, "NULL solver");
  if (!s->bound) return fail(PMDG_ESTATE, "not bound");
  if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  if (sc < 0 || sc >= s->S) return fail(PMDG_EINVAL, "scenario out of range");
  if (nstep < 0 || (s->R > 0 && nstep > s->cap)) return fail(PMDG_EINVAL, "nstep out of range");
  // the S scenarios share one step counter, which also selects their state
  // buffers: with several scenarios only the current step can be set
  if (s->S > 1 && nstep != s->steps_done)
    return fail(PMDG_ESTATE, "with several scenarios nstep must equal the steps done (" +
                                 std::to_string(s->steps_done) + ")");
  return s->prec == 64 ? set_state_t<double>(s, sc, p, p_prev, q, qd, qdd, nstep, (hipStream_t)stream)
                       : set_state_t<float>(s, sc, p, p_prev, q, qd, qdd, nstep, (hipStream_t)stream);
}

pmdg_status pmdg_status_flags(pmdg_solver* s, int* nonfinite, void* stream) {
  if (!s || !nonfinite) return fail(PMDG_EINVAL, "NULL argument");
  if (!s->bound) return fail(PMDG_ESTATE, "not bound");
  if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  HIPCHK(hipMemcpy(nonfinite, dptr<char>(s, "ctl") + 16, sizeof(int), hipMemcpyDeviceToHost));
  return PMDG_OK;
}

void pmdg_destroy(pmdg_solver* s) {
  if (!s) return;
  if (s->static_dev >= 0) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_owner[s->static_dev] == s) g_scratch_owner[s->static_dev] = nullptr;
  }
  drop_graphs(s);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->side) (void)hipStreamDestroy(s->side);
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  delete s;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Batched form: several bound single-brick solvers stepped together by
// persistent launches over device work lists.
// ------------------------------------------------------------------------
struct pmdg_batch {
  std::vector<pmdg_solver*> sv;
  int nmax = 1;
  int nm_max = 1;               // most modes per PMUT over the problems
  size_t lds = 0;
  int n_stiff = 0, n_face = 0, grid_stiff = 1, grid_face = 1;
  char* ws = nullptr;
  size_t off_sargs = 0, off_fargs = 0, off_sitems = 0, off_fitems = 0, off_ctr = 0, off_woff = 0, bytes = 0;
  bool bound = false;
  int use_graph = 1, graph_chunk = 64;
  std::map<int, hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;
  // kernel arguments of every solver, fixed at create together with the
  // layout, item counts and LDS size they imply
  std::vector<StiffArgs<float>> sa;
  std::vector<FaceArgs<float>> fa;
};

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

static void batch_layout(pmdg_batch* b) {
  const size_t n = b->sv.size();
  size_t o = 0;
  b->off_sargs = o; o = al256(o + n * sizeof(StiffArgs<float>));
  b->off_fargs = o; o = al256(o + n * sizeof(FaceArgs<float>));
  b->off_sitems = o; o = al256(o + (size_t)b->n_stiff * sizeof(int2));
  b->off_fitems = o; o = al256(o + (size_t)b->n_face * sizeof(int2));
  b->off_ctr = o; o = al256(o + n * sizeof(long*));
  // per-workgroup item ranges: at most one workgroup per item
  b->off_woff = o; o = al256(o + ((size_t)b->n_stiff + 1) * sizeof(int));
  b->bytes = o;
}

// Splits the stiffness items of a batch into `grid` per-workgroup lists of
// about equal cost: an item's cost is the plane iterations of its z-march
// (the planes of its chunk plus the 2N that fill the register queue) plus
// two for its set-up.  Longest items first, each to the least loaded list
// (ties to the lower index), so the launch ends with the longest list
// rather than with whichever workgroup a round robin gave the most long
// items.  Every item is computed the same way whichever workgroup takes it.
static void balance_items(const std::vector<StiffArgs<float>>& sa, int grid, std::vector<int2>& items,
                          std::vector<int>& woff) {
  const int n = (int)items.size();
  std::vector<int> cost(n), order(n);
  for (int i = 0; i < n; ++i) {
    const StiffArgs<float>& a = sa[items[i].x];
    const int bz = (items[i].y / (a.nbx * a.nby)) % a.nbz;
    const int k0 = a.zlo + bz * a.zchunk, k1 = std::min(a.zhi + 1, k0 + a.zchunk);
    cost[i] = (k1 - k0) + 2 * a.d.N + 2;
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  typedef std::pair<long, int> Load;  // (cost so far, list)
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int g = 0; g < grid; ++g) heap.push(Load(0, g));
  std::vector<std::vector<int>> lists(grid);
  for (int i : order) {
    Load l = heap.top();
    heap.pop();
    lists[l.second].push_back(i);
    heap.push(Load(l.first + cost[i], l.second));
  }
  std::vector<int2> out;
  out.reserve(n);
  woff.assign(grid + 1, 0);
  for (int g = 0; g < grid; ++g) {
    for (int i : lists[g]) out.push_back(items[i]);
    woff[g + 1] = (int)out.size();
  }
  items.swap(out);
}

static pmdg_status batch_enqueue(pmdg_batch* b, hipStream_t st) {
  HIPCHK(launch_stiff_batch((const StiffArgs<float>*)(b->ws + b->off_sargs), (const int2*)(b->ws + b->off_sitems),
                            b->n_stiff, (const int*)(b->ws + b->off_woff), b->nmax, b->grid_stiff, b->lds, st));
  HIPCHK(launch_face_batch((const FaceArgs<float>*)(b->ws + b->off_fargs), (const int2*)(b->ws + b->off_fitems),
                           b->n_face, b->grid_face, b->nm_max, st));
  HIPCHK(launch_tick_batch((long* const*)(b->ws + b->off_ctr), (int)b->sv.size(), st));
  return PMDG_OK;
}

extern "C" {

pmdg_status pmdg_batch_create(int n, pmdg_solver* const* solvers, pmdg_batch** out) {
  if (!out) return fail(PMDG_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || !solvers) return fail(PMDG_EINVAL, "need at least one solver");
  pmdg_batch* b = new (std::nothrow) pmdg_batch();
  if (!b) return fail(PMDG_ENOMEM, "out of host memory");
  for (int i = 0; i < n; ++i) {
    pmdg_solver* s = solvers[i];
    if (!s || !s->bound) { delete b; return fail(PMDG_ESTATE, "every solver must be bound"); }
    if (ws_lost(s)) { delete b; return fail(PMDG_ESTATE, kLostMsg); }
    if (s->ndom != 1 || s->prec != 32) { delete b; return fail(PMDG_EINVAL, "batches take single-brick FP32 solvers"); }
    if (s->b[0].pml) { delete b; return fail(PMDG_EINVAL, "batches take solvers without a matched layer"); }
    if (s->b[0].mapped()) { delete b; return fail(PMDG_EINVAL, "batches take axis-aligned bricks"); }
    const int rows = brick_rows(s, 0);
    if (rows != 1 && rows != 2) { delete b; return fail(PMDG_EINVAL, "batched tiles use 1 or 2 rows per wave"); }
    if (s->waves != kWaves) { delete b; return fail(PMDG_EINVAL, "batched tiles use 4 waves per workgroup"); }
    b->sv.push_back(s);
    b->nmax = std::max(b->nmax, s->b[0].N);
    b->nm_max = std::max(b->nm_max, s->Nm);
    b->lds = std::max(b->lds, batch_lds_bytes(s->b[0].N, rows));
    b->sa.push_back(stiff_args<float>(s, 0));
    b->fa.push_back(face_args<float>(s, 0));
    b->n_stiff += b->sa.back().nblocks;
    b->n_face += b->fa.back().nblocks;
  }
  batch_layout(b);
  for (pmdg_solver* s : b->sv) ++s->batches;
  *out = b;
  return PMDG_OK;
}

pmdg_status pmdg_batch_workspace_size(pmdg_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(PMDG_EINVAL, "NULL argument");
  *bytes = b->bytes;
  return PMDG_OK;
}

pmdg_status pmdg_batch_bind(pmdg_batch* b, void* dev_ptr, size_t bytes, void* stream) {
  if (!b) return fail(PMDG_EINVAL, "NULL batch");
  if (b->bound) return fail(PMDG_ESTATE, "already bound");
  if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return fail(PMDG_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < b->bytes) return fail(PMDG_ENOMEM, "batch workspace too small: need " + std::to_string(b->bytes));
  hipStream_t st = (hipStream_t)stream;
  b->ws = (char*)dev_ptr;
  const std::vector<StiffArgs<float>>& sa = b->sa;
  const std::vector<FaceArgs<float>>& fa = b->fa;
  std::vector<int2> si, fi;
  std::vector<long*> ctr;
  for (size_t p = 0; p < b->sv.size(); ++p) {
    pmdg_solver* s = b->sv[p];
    for (int t = 0; t < sa[p].nblocks; ++t) si.push_back(make_int2((int)p, t));
    for (int t = 0; t < fa[p].nblocks; ++t) fi.push_back(make_int2((int)p, t));
    ctr.push_back(dptr<long>(s, "ctl"));
  }
  if ((int)si.size() != b->n_stiff || (int)fi.size() != b->n_face)
    return fail(PMDG_EINVAL, "internal: batch item counts differ from the layout");
  int dev = 0, cus = 256, occ = 1;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(batch_occupancy(b->nmax, b->lds, &occ));
  b->grid_stiff = std::max(1, std::min(b->n_stiff, cus * std::max(occ, 1)));
  b->grid_face = std::max(1, std::min(b->n_face, cus * 4));
  std::vector<int> woff;
  balance_items(sa, b->grid_stiff, si, woff);
  HIPCHK(hipMemcpyAsync(b->ws + b->off_sargs, sa.data(), sa.size() * sizeof(sa[0]), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->ws + b->off_fargs, fa.data(), fa.size() * sizeof(fa[0]), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->ws + b->off_sitems, si.data(), si.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->ws + b->off_woff, woff.data(), woff.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->ws + b->off_fitems, fi.data(), fi.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->ws + b->off_ctr, ctr.data(), ctr.size() * sizeof(long*), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  b->bound = true;
  return PMDG_OK;
}

pmdg_status pmdg_batch_set_option(pmdg_batch* b, int option, long value) {
  if (!b) return fail(PMDG_EINVAL, "NULL batch");
  if (option == PMDG_OPT_GRAPH) b->use_graph = value ? 1 : 0;
  else if (option == PMDG_OPT_GRAPH_CHUNK && value >= 1) b->graph_chunk = (int)value;
  else return fail(PMDG_EINVAL, "unsupported batch option");
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
  return PMDG_OK;
}

pmdg_status pmdg_batch_step(pmdg_batch* b, int n, void* stream) {
  if (!b) return fail(PMDG_EINVAL, "NULL batch");
  if (!b->bound) return fail(PMDG_ESTATE, "bind the batch before stepping");
  if (n < 0) return fail(PMDG_EINVAL, "n must be >= 0");
  for (auto* s : b->sv) {
    if (s->steps_done + n > s->cap) return fail(PMDG_ESTATE, "a solver's trace capacity would be exceeded");
    if (ws_lost(s)) return fail(PMDG_ESTATE, kLostMsg);
  }
  if (n == 0) return PMDG_OK;
  hipStream_t st = (hipStream_t)stream;
  if (!b->use_graph) {
    for (int i = 0; i < n; ++i) {
      pmdg_status r = batch_enqueue(b, st);
      if (r) return r;
    }
  } else {
    if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    int left = n;
    while (left > 0) {
      const int len = std::min(left, b->graph_chunk);
      auto it = b->graphs.find(len);
      if (it == b->graphs.end()) {
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        pmdg_status r = PMDG_OK;
        for (int i = 0; i < len && !r; ++i) r = batch_enqueue(b, b->cap_stream);
        hipError_t ec = hipStreamEndCapture(b->cap_stream, &g);
        if (r) return r;
        if (ec != hipSuccess) return fail(PMDG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        hipGraphExec_t ex;
        ec = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ec != hipSuccess) return fail(PMDG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ec));
        it = b->graphs.emplace(len, ex).first;
      }
      HIPCHK(hipGraphLaunch(it->second, st));
      left -= len;
    }
  }
  for (auto* s : b->sv) s->steps_done += n;
  return PMDG_OK;
}

void pmdg_batch_destroy(pmdg_batch* b) {
  if (!b) return;
  for (pmdg_solver* s : b->sv) --s->batches;
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"

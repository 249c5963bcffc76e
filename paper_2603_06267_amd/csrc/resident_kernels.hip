// Steps of a small single-brick FP32 solver with the pressure held in LDS.
//
// One workgroup (1024 threads) per scenario keeps p on every node in LDS
// together with the increment X = p^n - p^{n-1}, and runs whole steps
// (Sec. 3.1, Algorithm 1 in its synchronised reading) back to back inside
// one launch:
//   1. stiffness and update at every node: the difference-form Kronecker
//      stencil of the tiled kernel, in the same operation order, and the
//      PMUT face force on the bottom plane; X += a is formed from p^n for
//      every node first, then p += X in place after a barrier;
//   2. PMUT sampling of p^{n+1} (FP64), the modal Newmark update with its
//      drive (or the receive-mode feedback), and the new face force, 16
//      lanes per PMUT (Sec. 2, eq. pmut_problem; Sec. 3.1, eqs. f_i, g_m);
//   3. receiver traces of p^{n+1} (FP64), 16 lanes per receiver.
// HBM is touched only to read the state at the start, to write the traces
// of each step and to write the state back at the end.  A one-thread launch
// then advances the device step counter by the number of steps.
#include "pmutdg_internal.h"

namespace pmdg {

// Zero padding before and after p in LDS: N planes for the z neighbours, and
// room for the last x window of the last row.
__host__ __device__ int resident_pad(int N, int nx, int ny) { return N * nx * ny + 8 + N; }

namespace {

constexpr int kResThreads = 1024;
constexpr int kResRun = 8;  // nodes per x run of the stiffness phase (room for it in resident_pad)
constexpr int kResMaxPer = 32;  // nodes per thread (the LDS bound comes first)

template <int N>
__device__ __forceinline__ int res_class(int i, int n) {
  return i == 0 ? N : (i == n - 1 ? N + 1 : i % N);
}

// floor(n / d) for 0 <= n < 2^20 from a float reciprocal, corrected by one
__device__ __forceinline__ int res_div(int n, int d, float inv) {
  int q = (int)((float)n * inv);
  const int r = n - q * d;
  if (r < 0) --q;
  else if (r >= d) ++q;
  return q;
}

// sum over the G lanes of a lane group
template <int G>
__device__ __forceinline__ double res_group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

template <int N, int MM, int G>
__global__ void __launch_bounds__(kResThreads) k_resident(const ResidentArgs a) {
  constexpr int NT = 2 * N, NC = N + 3, n1 = N + 1;
  extern __shared__ __align__(16) unsigned char lds[];
  // p with N planes of zeros before and after: every neighbour of the
  // stencil is a valid address, and those outside the brick carry zero taps
  const int pad = resident_pad(N, a.d.nn[0], a.d.nn[1]);
  float* P = reinterpret_cast<float*>(lds) + pad;
  float* XS = P + a.nc + pad;
  float* FZ = reinterpret_cast<float*>(lds + a.off_force);
  float* TP = reinterpret_cast<float*>(lds + a.off_taps);
  float* MI = reinterpret_cast<float*>(lds + a.off_mins);
  double* BB = reinterpret_cast<double*>(lds + a.off_B);
  int* FN = reinterpret_cast<int*>(lds + a.off_fn);
  double* QS = reinterpret_cast<double*>(lds + a.off_q);  // q, qd, qdd: [3][Np Nm]
  double* CF = reinterpret_cast<double*>(lds + a.off_coef);  // omega, zeta, eta: [3][Np Nm]
  double* DA = reinterpret_cast<double*>(lds + a.off_da);    // [Np][2]: A cos theta, A sin theta
  double* RW = reinterpret_cast<double*>(lds + a.off_rw);    // [R][3][N+1]
  int* PO = reinterpret_cast<int*>(lds + a.off_poff);        // [Np+1]
  int* RB = reinterpret_cast<int*>(lds + a.off_rb);          // [R] compact first node
  const int tid = threadIdx.x;
  const int s = blockIdx.x;
  const int nx = a.d.nn[0], ny = a.d.nn[1], nz = a.d.nn[2], nc = a.nc, px = a.d.px;
  const long cnt0 = *a.counter;
  const float* Pg = a.d.P[(int)(cnt0 % 3)] + (long)s * a.d.nnodes;
  float* Xg = a.d.X + (long)(*a.d.xsel) * a.d.xstride + (long)s * a.d.nnodes;
  const int nfz = nx * ny, Nm = a.Nm, npm = a.Np * Nm;

  for (int n = tid; n < nc; n += kResThreads) {
    const int jk = res_div(n, nx, a.inv_nn0), i = n - jk * nx;
    const int k = res_div(jk, ny, a.inv_nn1), j = jk - k * ny;
    const long g = i + (long)px * (j + (long)ny * k);
    P[n] = Pg[g];
    XS[n] = Xg[g];
  }
  for (int t = tid; t < pad; t += kResThreads) {
    P[-pad + t] = 0.f;
    P[nc + t] = 0.f;
  }
  for (int f = tid; f < nfz; f += kResThreads) {
    const int j = res_div(f, nx, a.inv_nn0), i = f - j * nx;
    FZ[f] = a.force ? a.force[(long)s * a.d.plane + i + (long)px * j] : 0.f;
  }
  for (int t = tid; t < 3 * NC * NT; t += kResThreads) TP[t] = a.taps[t];
  for (int t = tid; t < 3 * NC; t += kResThreads) MI[t] = a.mins[t];
  for (int t = tid; t < a.nface * Nm; t += kResThreads) BB[t] = a.pm_B[t];
  for (int t = tid; t < a.nface; t += kResThreads) {
    const int f = a.pm_node[t];
    FN[t] = f % px + nx * (f / px);
  }
  for (int t = tid; t < npm; t += kResThreads) {
    const long o = (long)s * npm + t;
    QS[t] = a.q[o];
    QS[npm + t] = a.qd[o];
    QS[2 * npm + t] = a.qdd[o];
    CF[t] = a.omega[t];
    CF[npm + t] = a.zeta[t];
    CF[2 * npm + t] = a.eta[t];
  }
  for (int t = tid; t < 2 * a.Np; t += kResThreads) DA[t] = a.dA[(long)s * a.Np * 2 + t];
  // (a solver without PMUTs has no PMUT tables at all)
  if (a.Np > 0)
    for (int t = tid; t <= a.Np; t += kResThreads) PO[t] = a.pm_off[t];
  for (int t = tid; t < a.R * 3 * n1; t += kResThreads) {
    const int r = t / (3 * n1), q = t - r * 3 * n1, ax = q / n1, i = q - ax * n1;
    RW[t] = a.r_w[(long)r * 3 * (kMaxOrder + 1) + ax * (kMaxOrder + 1) + i];
  }
  for (int r = tid; r < a.R; r += kResThreads) {
    // padded node index of the element's first node (small brick: 32-bit)
    const int b = (int)a.r_base[r];
    const int i0 = b % px, jk = b / px;
    RB[r] = i0 + nx * jk;
  }
  __syncthreads();

  const double dt = a.dt;
  // runs along x: each row split into nseg runs of at most kResRun nodes
  const int nseg = (nx + kResRun - 1) / kResRun, seglen = (nx + nseg - 1) / nseg;
  const int nseg_all = nseg * ny * nz;
  for (int st = 0; st < a.nsteps; ++st) {
    const long cnt = cnt0 + st;
    // this step's drive carrier, loaded ahead of the stiffness phase
    const long lev = cnt + 1;
    const double* c2 = a.car + ((long)s * a.ncar + min(lev, a.ncar - 1)) * 2;
    const double car0 = a.Np > 0 ? c2[0] : 0.0, car1 = a.Np > 0 ? c2[1] : 0.0;
    // (1) stiffness and update: X += a from p^n at every node, then p += X.
    // A thread takes a run of up to kResRun nodes along x: the x line comes
    // from one window of registers, the y and z rows of the operator once
    // per run.
    for (int sgi = tid; sgi < nseg_all; sgi += kResThreads) {
      const int row = sgi / nseg, sg = sgi - row * nseg;
      const int k = res_div(row, ny, a.inv_nn1), j = row - k * ny;
      const int i0 = sg * seglen, len = min(seglen, nx - i0);
      const int base = row * nx + i0;
      const int cy = res_class<N>(j, ny), cz = res_class<N>(k, nz);
      float ty[NT], tz[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        ty[t] = TP[(NC + cy) * NT + t];
        tz[t] = TP[(2 * NC + cz) * NT + t];
      }
      const float myz = MI[NC + cy], mz = MI[2 * NC + cz];
      // the x window: nodes i0 - N .. i0 + kResRun + N - 1 of this row (the
      // padding keeps every address valid)
      float w[kResRun + 2 * N];
#pragma unroll
      for (int q = 0; q < kResRun + 2 * N; ++q) w[q] = P[base - N + q];
      const int sy = nx, sz = nx * ny;
#pragma unroll
      for (int u = 0; u < kResRun; ++u) {
        if (u < len) {
          const int n = base + u, i = i0 + u;
          const int cx = res_class<N>(i, nx);
          const float* tx = TP + cx * NT;
          const float p0 = w[u + N];
          float ac = 0.f;
#pragma unroll
          for (int t = 0; t < N; ++t) {
            // a neighbour outside the brick has a zero tap; its address (the
            // zero padding, or a node of the next or previous row or plane)
            // holds a finite value
            const float ya = P[n + (t - N) * sy];
            const float yb = P[n + (1 + t) * sy];
            const float za = P[n + (t - N) * sz];
            const float zb = P[n + (1 + t) * sz];
            ac += tx[t] * (w[u + t] - p0);
            ac += tx[N + t] * (w[u + N + 1 + t] - p0);
            ac += ty[t] * (ya - p0);
            ac += ty[N + t] * (yb - p0);
            ac += tz[t] * (za - p0);
            ac += tz[N + t] * (zb - p0);
          }
          const float minv = MI[cx] * myz * mz;
          if (k == 0) ac += a.dt2 * minv * FZ[i + nx * j];
          XS[n] = XS[n] + ac;
        }
      }
    }
    __syncthreads();
    for (int n = tid; n < nc; n += kResThreads) P[n] = P[n] + XS[n];
    __syncthreads();
    // (2) PMUTs: sample p^{n+1}, modal update, face force; G lanes per PMUT
    // (16, or 64 for PMUTs of more than 48 face nodes; lane m of the group
    // also carries mode m)
    const bool driven = !(lev * dt > a.t_switch);
    {
      const int grp = tid / G, l16 = tid % G;
      for (int k0 = 0; k0 < a.Np; k0 += kResThreads / G) {
        const int k = k0 + grp;
        if (k >= a.Np) continue;
        const int f0 = PO[k], f1 = PO[k + 1], po = k * Nm;
        double g[MM];
#pragma unroll
        for (int m = 0; m < MM; ++m) g[m] = 0.0;
        bool bad = false;
        for (int f = f0 + l16; f < f1; f += G) {
          const double p = (double)P[FN[f]];
          bad |= !__builtin_isfinite(p);
#pragma unroll
          for (int m = 0; m < MM; ++m)
            if (m < Nm) g[m] += BB[f * Nm + m] * p;
        }
        if (bad) atomicOr(a.nonfinite, 1);
#pragma unroll
        for (int m = 0; m < MM; ++m)
          if (m < Nm) g[m] = res_group_sum<G>(g[m]);
        double qp = 0.0, qds = 0.0;
        if (l16 < Nm) {
          const double q = QS[po + l16], qd = QS[npm + po + l16], qdd = QS[2 * npm + po + l16];
          qp = q + dt * qd + 0.5 * dt * dt * qdd;
          qds = qd + 0.5 * dt * qdd;
        }
        double phi;
        if (driven) {
          phi = DA[2 * k] * car0 - DA[2 * k + 1] * car1;
        } else {
          phi = res_group_sum<G>(l16 < Nm ? CF[2 * npm + po + l16] * qp : 0.0) / a.cap;
        }
        double qa = 0.0;
        if (l16 < Nm) {
          double gm = 0.0;
#pragma unroll
          for (int m = 0; m < MM; ++m)
            if (m == l16) gm = g[m];
          const double w = CF[po + l16], ze = CF[npm + po + l16], et = CF[2 * npm + po + l16];
          qa = -w * w * qp - 2.0 * ze * w * qds + gm + et * phi;
          QS[po + l16] = qp;
          QS[npm + po + l16] = qds + 0.5 * dt * qa;
          QS[2 * npm + po + l16] = qa;
        }
        double qm[MM];
#pragma unroll
        for (int m = 0; m < MM; ++m) qm[m] = __shfl(qa, m, G);
        for (int f = f0 + l16; f < f1; f += G) {
          double fv = 0.0;
#pragma unroll
          for (int m = 0; m < MM; ++m)
            if (m < Nm) fv += qm[m] * BB[f * Nm + m];
          FZ[FN[f]] = (float)(-a.kappa * fv);
        }
      }
    }
    // (3) receivers: 16 lanes per receiver, all 64 groups of the workgroup
    // at once
    {
      const int grp = tid >> 4, l16 = tid & 15;
      for (int r0 = 0; r0 < a.R; r0 += kResThreads / 16) {
        const int r = r0 + grp;
        double v = 0.0;
        if (r < a.R) {
          const int cb = RB[r];
          const double* w = RW + r * 3 * n1;
          for (int idx = l16; idx < n1 * n1 * n1; idx += 16) {
            const int i = idx % n1, j = (idx / n1) % n1, c = idx / (n1 * n1);
            v += w[i] * w[n1 + j] * w[2 * n1 + c] * (double)P[cb + i + nx * (j + ny * c)];
          }
        }
        v = res_group_sum<16>(v);
        if (r < a.R && l16 == 0) {
          if (cnt < a.tcap) a.traces[((long)s * a.R + r) * a.tcap + cnt] = v;
          if (!__builtin_isfinite(v)) atomicOr(a.nonfinite, 1);
        }
      }
    }
    __syncthreads();
  }

  // state out: the level cnt0 + nsteps, its increment, the face force and
  // the modal state
  float* PgE = a.d.P[(int)((cnt0 + a.nsteps) % 3)] + (long)s * a.d.nnodes;
  for (int n = tid; n < nc; n += kResThreads) {
    const int jk = res_div(n, nx, a.inv_nn0), i = n - jk * nx;
    const int k = res_div(jk, ny, a.inv_nn1), j = jk - k * ny;
    const long g = i + (long)px * (j + (long)ny * k);
    PgE[g] = P[n];
    Xg[g] = XS[n];
  }
  if (a.force)
    for (int f = tid; f < nfz; f += kResThreads) {
      const int j = res_div(f, nx, a.inv_nn0), i = f - j * nx;
      a.force[(long)s * a.d.plane + i + (long)px * j] = FZ[f];
    }
  for (int t = tid; t < npm; t += kResThreads) {
    const long o = (long)s * npm + t;
    a.q[o] = QS[t];
    a.qd[o] = QS[npm + t];
    a.qdd[o] = QS[2 * npm + t];
  }
}

__global__ void k_tick_n(long* counter, long n) {
  if (threadIdx.x == 0) *counter += n;
}

template <int N, int MM, int G>
hipError_t res_launch_nmg(const ResidentArgs& a, hipStream_t st) {
  if (a.lds_bytes > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_resident<N, MM, G>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_resident<N, MM, G>), dim3(a.S), dim3(kResThreads), a.lds_bytes, st, a);
  return hipGetLastError();
}

template <int N, int MM>
hipError_t res_launch_nm(const ResidentArgs& a, hipStream_t st) {
  return a.pm_wide ? res_launch_nmg<N, MM, 64>(a, st) : res_launch_nmg<N, MM, 16>(a, st);
}

template <int N>
hipError_t res_launch_n(const ResidentArgs& a, hipStream_t st) {
  return a.Nm <= 4 ? res_launch_nm<N, 4>(a, st) : res_launch_nm<N, kMaxModes>(a, st);
}

}  // namespace

int resident_max_nodes() { return kResMaxPer * kResThreads; }

hipError_t launch_resident(const ResidentArgs& a, hipStream_t st) {
  if (a.nc > resident_max_nodes() || a.Nm > kMaxModes || a.nsteps < 1) return hipErrorInvalidValue;
  switch (a.d.N) {
    case 1: return res_launch_n<1>(a, st);
    case 2: return res_launch_n<2>(a, st);
    case 3: return res_launch_n<3>(a, st);
    case 4: return res_launch_n<4>(a, st);
    case 5: return res_launch_n<5>(a, st);
    case 6: return res_launch_n<6>(a, st);
    case 7: return res_launch_n<7>(a, st);
    case 8: return res_launch_n<8>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tick_n(long* counter, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_tick_n, dim3(1), dim3(64), 0, st, counter, n);
  return hipGetLastError();
}

}  // namespace pmdg

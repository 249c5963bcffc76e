// HIP kernels of libpmutdg for CDNA4 (gfx950): one explicit time step of the
// coupled PMUT / DG spectral-element acoustic model (arXiv 2603.06267).
//
// Per step, in stream order:
//   k_stiff (one launch per brick)  p^{n+1} from p^n with the volume
//       stiffness, the interface residual of p^n and the PMUT face force of
//       qddot^n (Sec. 3.1, Algorithm 1 acoustic block, explicit form);
//   k_face   PMUT sampling of p^{n+1}, modal ODE to level n+1 and the new
//       face force (Algorithm 1 PMUT block, synchronised with p^{n+1};
//       eqs. g_m, f_i); receiver traces of p^{n+1}; value / normal-derivative
//       traces of p^{n+1} on Gamma_I; advances the device step counter;
//   k_flux   SIPG terms (eq. Wf_2, interface sums) at the Gauss points of the
//       fine faces (Sec. 5), reduced onto the faces of both sides for the
//       next k_stiff.
//
// The volume operator of a uniform brick with GLL collocation is the
// Kronecker sum c^2 (A_x (x) I (x) I + I (x) A_y (x) I + I (x) I (x) A_z),
// A_d = M_d^{-1} K_d the assembled 1D operator (an exact identity of the
// tensor-product spectral element, equivalent to element-wise sum
// factorisation followed by assembly).  Each node therefore needs the 2N
// off-centre taps of its three grid lines; the kernel applies them in
// difference form sum_t a_t (p_{i+t} - p_i), which keeps the zero row sum of
// A_d exact in finite precision.
#include <utility>

#include "pmutdg_internal.h"
#include "stiff_kernel.h"

namespace pmdg {


// ------------------------------------------------------------------------
// Face kernel.
// ------------------------------------------------------------------------
__device__ __forceinline__ double window_g(double t, double Td) {
  // smooth window of Sec. 6.1 (eq. voltage), exponent n = 10, written in the
  // symmetric variable b = |2t/T_d - 1|
  if (t < 0.0 || t > Td) return 0.0;
  const double b = fabs(2.0 * t / Td - 1.0);
  const double b2 = b * b, b4 = b2 * b2, b5 = b4 * b, b10 = b5 * b5, b20 = b10 * b10;
  const double base = 1.0 - 2.0 * b20 * b / (1.0 + b20);
  if (base <= 0.0) return 0.0;
  return exp(1.0 - 1.0 / (base * base));
}

__device__ __forceinline__ double drive_phi(double A, double th, double f, double ncyc, int env, double t) {
  const double Td = ncyc / f;
  double e;
  if (env == 0) e = window_g(t, Td);
  else if (env == 1) e = (t >= 0.0 && t <= Td) ? 1.0 : 0.0;
  else e = (t >= 0.0) ? 1.0 : 0.0;
  return A * sin(2.0 * M_PI * f * t - th) * e;
}

template <typename Real>
__device__ void face_traces(const FaceArgs<Real>& a, int side, int item, int buf) {
  const DomView<Real>& D = side == 0 ? a.d0 : a.d1;
  const long nf = D.plane;
  if (item >= (long)a.S * nf) return;
  const int s = item / nf;
  const long f = item - (long)s * nf;
  const Real* P = D.P[buf] + (long)s * D.nnodes;
  const int N = D.N;
  Real val, der = 0;
  if (side == 0) {
    const int top = D.nn[2] - 1;
    val = P[f + D.plane * top];
    for (int c = 0; c <= N; ++c) der += a.dz0[c] * P[f + D.plane * (top - N + c)];
    a.tr0[((long)s * nf + f) * 2] = val;
    a.tr0[((long)s * nf + f) * 2 + 1] = der;
  } else {
    val = P[f];
    for (int c = 0; c <= N; ++c) der += a.dz1[c] * P[f + D.plane * c];
    a.tr1[((long)s * nf + f) * 2] = val;
    a.tr1[((long)s * nf + f) * 2 + 1] = der;
  }
}

template <typename Real>
__global__ void __launch_bounds__(256) k_face(const FaceArgs<Real> a) {
  __shared__ double red[kWaves][kMaxModes];
  __shared__ double qp_s[kMaxModes], qds_s[kMaxModes], qdd_s[kMaxModes];
  __shared__ double phi_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long cnt = *a.counter;
  const long lev = a.prime ? cnt : cnt + 1;  // time level of the pressure to sample
  const int buf = (int)(lev & 1);
  int b = blockIdx.x;

  if (b < a.nb_tr0) {
    face_traces(a, 0, b * 256 + tid, buf);
  } else if ((b -= a.nb_tr0) < a.nb_tr1) {
    face_traces(a, 1, b * 256 + tid, buf);
  } else if ((b -= a.nb_tr1) < a.nb_pm) {
    const int s = b / a.Np, k = b - s * a.Np;
    const int Nm = a.Nm;
    const long qo = ((long)s * a.Np + k) * Nm;
    const int n0 = a.pm_off[k], n1 = a.pm_off[k + 1];
    const double dt = a.dt;
    if (!a.prime) {
      if (tid < Nm) {
        const double q = a.q[qo + tid], qd = a.qd[qo + tid], qdd = a.qdd[qo + tid];
        qp_s[tid] = q + dt * qd + 0.5 * dt * dt * qdd;
        qds_s[tid] = qd + 0.5 * dt * qdd;
      }
      double acc[kMaxModes];
#pragma unroll
      for (int m = 0; m < kMaxModes; ++m) acc[m] = 0.0;
      const Real* P0 = a.d0.P[buf] + (long)s * a.d0.nnodes;
      bool bad = false;
      for (int n = n0 + tid; n < n1; n += 256) {
        const double p = (double)P0[a.pm_node[n]];
        bad |= !__builtin_isfinite(p);
        const double* B = a.pm_B + (long)n * Nm;
#pragma unroll
        for (int m = 0; m < kMaxModes; ++m)
          if (m < Nm) acc[m] += B[m] * p;
      }
      if (bad) atomicOr(a.nonfinite, 1);
#pragma unroll
      for (int m = 0; m < kMaxModes; ++m) {
        if (m < Nm) {
          const double v = wave_sum(acc[m]);
          if (lane == 0) red[wave][m] = v;
        }
      }
      __syncthreads();
      if (tid == 0) {
        const double t = lev * dt;
        double phi;
        if (t > a.t_switch) {
          phi = 0.0;
          for (int m = 0; m < Nm; ++m) phi += a.eta[(long)k * Nm + m] * qp_s[m];
          phi /= a.cap;
        } else {
          phi = drive_phi(a.amp[(long)s * a.Np + k], a.phase[(long)s * a.Np + k], a.freq[s], a.ncyc,
                          a.envelope, t);
        }
        phi_s = phi;
      }
      __syncthreads();
      if (tid < Nm) {
        const double g = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
        const long pi = (long)k * Nm + tid;
        const double w = a.omega[pi];
        const double qdd = -w * w * qp_s[tid] - 2.0 * a.zeta[pi] * w * qds_s[tid] + g + a.eta[pi] * phi_s;
        a.q[qo + tid] = qp_s[tid];
        a.qd[qo + tid] = qds_s[tid] + 0.5 * dt * qdd;
        a.qdd[qo + tid] = qdd;
        qdd_s[tid] = qdd;
      }
    } else {
      if (tid < Nm) qdd_s[tid] = a.qdd[qo + tid];
    }
    __syncthreads();
    Real* F = a.force + (long)s * a.d0.plane;
    for (int n = n0 + tid; n < n1; n += 256) {
      const double* B = a.pm_B + (long)n * Nm;
      double f = 0.0;
      for (int m = 0; m < Nm; ++m) f += qdd_s[m] * B[m];
      F[a.pm_node[n]] = (Real)(-a.kappa * f);
    }
  } else if (!a.prime) {
    b -= a.nb_pm;
    const int item = b * kWaves + wave;
    if (item < a.S * a.R) {
      const int s = item / a.R, r = item - s * a.R;
      const DomView<Real>& D = a.r_dom[r] == 0 ? a.d0 : a.d1;
      const int n1 = D.N + 1;
      const double* w = a.r_w + (long)r * 3 * (kMaxOrder + 1);
      const Real* Pd = D.P[buf] + (long)s * D.nnodes;
      const long base = a.r_base[r];
      double acc = 0.0;
      for (int idx = lane; idx < n1 * n1 * n1; idx += 64) {
        const int i = idx % n1, j = (idx / n1) % n1, c = idx / (n1 * n1);
        acc += w[i] * w[kMaxOrder + 1 + j] * w[2 * (kMaxOrder + 1) + c] *
               (double)Pd[base + i + (long)D.nn[0] * j + D.plane * c];
      }
      acc = wave_sum(acc);
      if (lane == 0 && cnt < a.tcap) a.traces[((long)s * a.R + r) * a.tcap + cnt] = acc;
      if (lane == 0 && !__builtin_isfinite(acc)) atomicOr(a.nonfinite, 1);
    }
  }

  if (!a.prime) {
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      const unsigned prev = atomicAdd(a.done, 1u);
      if (prev == (unsigned)a.nblocks - 1u) {
        // every block has read the counter: advance the step
        atomicExch(a.done, 0u);
        atomicAdd((unsigned long long*)a.counter, 1ull);
        __threadfence();
      }
    }
  }
}

// ------------------------------------------------------------------------
// Interface flux.
// ------------------------------------------------------------------------
template <typename Real>
__device__ __forceinline__ void flux_point(const FluxArgs<Real>& a, int s, int ex, int ey, int qa, int qb,
                                           Real& A, Real& B) {
  const int N0 = a.N0, N1 = a.N1, n0 = N0 + 1, n1 = N1 + 1, Nq = a.Nq;
  const long nf0 = (long)a.nn0x * (a.ney0 * N0 + 1), nf1 = (long)a.nn1x * (a.ney1 * N1 + 1);
  const Real* T0 = a.tr0 + (long)s * nf0 * 2;
  const Real* T1 = a.tr1 + (long)s * nf1 * 2;
  Real pP = 0, dP = 0, pM = 0, dM = 0;
  for (int bb = 0; bb < n0; ++bb) {
    const Real lb = a.Lq[qb * n0 + bb];
    const long row = (long)a.nn0x * (N0 * ey + bb) + N0 * ex;
    for (int aa = 0; aa < n0; ++aa) {
      const Real w = a.Lq[qa * n0 + aa] * lb;
      pP += w * T0[(row + aa) * 2];
      dP += w * T0[(row + aa) * 2 + 1];
    }
  }
  const int cx = a.xcx[ex * Nq + qa], cy = a.ycx[ey * Nq + qb];
  const Real* wx = a.xw + (long)(ex * Nq + qa) * n1;
  const Real* wy = a.yw + (long)(ey * Nq + qb) * n1;
  for (int bb = 0; bb < n1; ++bb) {
    const long row = (long)a.nn1x * (N1 * cy + bb) + N1 * cx;
    for (int aa = 0; aa < n1; ++aa) {
      const Real w = wx[aa] * wy[bb];
      pM += w * T1[(row + aa) * 2];
      dM += w * T1[(row + aa) * 2 + 1];
    }
  }
  const Real jump = pP - pM;
  const Real avg = Real(0.5) * (a.cf2 * dP + a.cc2 * dM);
  const Real wj = a.wJ[qb * Nq + qa];
  A = wj * (a.gamma * jump - avg);
  B = Real(-0.5) * wj * jump;
}

template <typename Real>
__global__ void __launch_bounds__(256) k_flux(const FluxArgs<Real> a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int Nq = a.Nq;
  int b = blockIdx.x;
  if (b < a.nb_fine) {
    const int nfine = a.nex0 * a.ney0;
    const int item = b * kWaves + wave;
    if (item >= a.S * nfine) return;
    const int s = item / nfine, f = item - s * nfine;
    const int ex = f % a.nex0, ey = f / a.nex0;
    Real A = 0, B = 0;
    if (lane < Nq * Nq) flux_point(a, s, ex, ey, lane % Nq, lane / Nq, A, B);
    const int n0 = a.N0 + 1;
    Real RA = 0, RB = 0;
    const int aa = lane % n0, bb = lane / n0;
    for (int qq = 0; qq < Nq * Nq; ++qq) {
      const Real Aq = __shfl(A, qq, 64), Bq = __shfl(B, qq, 64);
      if (lane < n0 * n0) {
        const Real w = a.Lq[(qq % Nq) * n0 + aa] * a.Lq[(qq / Nq) * n0 + bb];
        RA += w * Aq;
        RB += w * Bq;
      }
    }
    if (lane < n0 * n0) {
      Real* R = a.R0 + (((long)s * nfine + f) * n0 * n0 + lane) * 2;
      R[0] = RA;
      R[1] = RB;
    }
  } else {
    b -= a.nb_fine;
    const int ncoarse = a.nex1 * a.ney1;
    const int item = b * kWaves + wave;
    if (item >= a.S * ncoarse) return;
    const int s = item / ncoarse, f = item - s * ncoarse;
    const int cx = f % a.nex1, cy = f / a.nex1;
    const int xo0 = a.xl_off[cx], nxl = a.xl_off[cx + 1] - xo0;
    const int yo0 = a.yl_off[cy], nyl = a.yl_off[cy + 1] - yo0;
    const int nqc = nxl * nyl;
    const int n1 = a.N1 + 1;
    const int aa = lane % n1, bb = lane / n1;
    Real RA = 0, RB = 0;
    for (int base = 0; base < nqc; base += 64) {
      Real A = 0, B = 0;
      int px = 0, py = 0;
      const int qi = base + lane;
      if (qi < nqc) {
        px = a.xl[xo0 + qi % nxl];
        py = a.yl[yo0 + qi / nxl];
        flux_point(a, s, px / Nq, py / Nq, px % Nq, py % Nq, A, B);
      }
      const int cntq = min(64, nqc - base);
      for (int qq = 0; qq < cntq; ++qq) {
        const Real Aq = __shfl(A, qq, 64), Bq = __shfl(B, qq, 64);
        const int pxq = __shfl(px, qq, 64), pyq = __shfl(py, qq, 64);
        if (lane < n1 * n1) {
          const Real w = a.xw[(long)pxq * n1 + aa] * a.yw[(long)pyq * n1 + bb];
          RA += w * Aq;
          RB += w * Bq;
        }
      }
    }
    if (lane < n1 * n1) {
      Real* R = a.R1 + (((long)s * ncoarse + f) * n1 * n1 + lane) * 2;
      R[0] = RA;  // the stiffness kernel applies the coarse side's minus sign
      R[1] = RB;
    }
  }
}

template <typename Real>
__global__ void k_fill(Real* p, long n, Real v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------
template <>
hipError_t launch_stiff<float>(const StiffArgs<float>& a, int ry, int wv, bool incr, hipStream_t st) {
  if (!incr) return hipErrorInvalidValue;  // FP32 state always uses the increment form
  return a.d.N <= 4 ? launch_stiff_f32_lo(a, ry, wv, st) : launch_stiff_f32_hi(a, ry, wv, st);
}

template <>
hipError_t launch_stiff<double>(const StiffArgs<double>& a, int ry, int wv, bool incr, hipStream_t st) {
  if (incr) return hipErrorInvalidValue;  // FP64 state uses the two-level form
  return a.d.N <= 4 ? launch_stiff_f64_lo(a, ry, wv, st) : launch_stiff_f64_hi(a, ry, wv, st);
}

template <typename Real>
hipError_t launch_face(const FaceArgs<Real>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_face<Real>, dim3(a.nblocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_flux(const FluxArgs<Real>& a, hipStream_t st) {
  const int nb = a.nb_fine + a.nb_coarse;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flux<Real>, dim3(nb), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_fill(Real* p, long n, Real v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill<Real>, dim3((unsigned)nb), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_bytes(void* p, size_t n, hipStream_t st) {
  // n is a multiple of 4 (workspace sub-allocations are 256-byte aligned)
  return launch_fill<unsigned>((unsigned*)p, (long)(n / 4), 0u, st);
}

template hipError_t launch_face<float>(const FaceArgs<float>&, hipStream_t);
template hipError_t launch_face<double>(const FaceArgs<double>&, hipStream_t);
template hipError_t launch_flux<float>(const FluxArgs<float>&, hipStream_t);
template hipError_t launch_flux<double>(const FluxArgs<double>&, hipStream_t);
template hipError_t launch_fill<float>(float*, long, float, hipStream_t);
template hipError_t launch_fill<double>(double*, long, double, hipStream_t);
template hipError_t launch_fill<unsigned>(unsigned*, long, unsigned, hipStream_t);

}  // namespace pmdg

// HIP kernels of libpmutdg for CDNA4 (gfx950): one explicit time step of the
// coupled PMUT / DG spectral-element acoustic model (arXiv 2603.06267).
//
// Per step, in stream order:
//   k_stiff (one launch per brick)  p^{n+1} from p^n with the volume
//       stiffness, the interface residual of p^n and the PMUT face force of
//       qddot^n (Sec. 3.1, Algorithm 1 acoustic block, explicit form); where
//       a brick's interface element layer lies in one z chunk, also the
//       value / normal-derivative traces of p^{n+1} on Gamma_I;
//   k_face   PMUT sampling of p^{n+1}, modal ODE to level n+1 and the new
//       face force (Algorithm 1 PMUT block, synchronised with p^{n+1};
//       eqs. g_m, f_i); receiver traces of p^{n+1}; the Gamma_I traces the
//       stiffness launches do not write;
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
template <typename Real>
__device__ void face_traces(const FaceArgs<Real>& a, int side, int item, int buf) {
  // item runs over the compact face grid nn[0] x nn[1] of every scenario
  const DomView<Real>& D = side == 0 ? a.d0 : a.d1;
  const long nf = (long)D.nn[0] * D.nn[1];
  if (item >= (long)a.S * nf) return;
  const int s = item / nf;
  const long f = item - (long)s * nf;
  const long j = f / D.nn[0], i = f - j * D.nn[0];
  const long g = i + (long)D.px * j;  // device index within a plane
  const Real* P = D.P[buf] + (long)s * D.nnodes;
  const int N = D.N;
  Real val, der = 0;
  if (side == 0) {
    const int top = D.nn[2] - 1;
    val = P[g + D.plane * top];
    for (int c = 0; c <= N; ++c) der += a.dz0[c] * P[g + D.plane * (top - N + c)];
    a.tr0[((long)s * nf + f) * 2] = val;
    a.tr0[((long)s * nf + f) * 2 + 1] = der;
  } else {
    val = P[g];
    for (int c = 0; c <= N; ++c) der += a.dz1[c] * P[g + D.plane * c];
    a.tr1[((long)s * nf + f) * 2] = val;
    a.tr1[((long)s * nf + f) * 2 + 1] = der;
  }
}

// Sums v[0..MM) over the 64 lanes of a wave by recursive halving.  At the
// step with lane offset o, a lane whose o bit is clear keeps the lower half
// of its values and one whose bit is set the upper half, and each adds its
// partner's copy of the half it keeps; after log2(MM) such steps every lane
// holds one value and plain butterfly steps over the remaining lane bits
// finish the sums.  Returns the sum held by this lane; *m is its index, and
// the lanes whose low 6 - log2(MM) bits are zero hold the MM sums once each.
// 6 dependent exchange rounds for all MM values, instead of 6 per value.
template <int MM>
__device__ __forceinline__ double wave_sum_many(double (&v)[MM], int lane, int* m) {
  static_assert(MM == 4 || MM == 8 || MM == 16, "MM must be 4, 8 or 16");
  constexpr int LG = MM == 4 ? 2 : (MM == 8 ? 3 : 4);
  int idx = 0;
  static_for<LG>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int o = 32 >> i, h = MM >> (i + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int j = 0; j < h; ++j) {
      const double send = up ? v[j] : v[j + h];
      const double keep = up ? v[j + h] : v[j];
      v[j] = keep + __shfl_xor(send, o, 64);
    }
    if (up) idx += h;
  });
  double r = v[0];
#pragma unroll
  for (int o = 32 >> LG; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
  *m = idx;
  return r;
}

// One workgroup-sized unit b of the face work of one problem.
// MM bounds the mode loops (a multiple of 4, >= the problem's Nm).  KEEP
// holds each PMUT node's projection row in LDS between the sampling and the
// force scatter (the batch kernel, whose persistent loop needs more
// registers, reloads it instead).
template <typename Real, int MM, bool KEEP>
__device__ void face_block(const FaceArgs<Real>& a, int b) {
  __shared__ double red[kWaves][kMaxModes];
  __shared__ double qp_s[kMaxModes], qds_s[kMaxModes], qdd_s[kMaxModes];
  __shared__ double phi_s;
  __shared__ double sB[KEEP ? MM : 1][256];  // PMUT blocks: each thread's projection row
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long cnt = *a.counter;
  const long lev = a.prime ? cnt : cnt + 1;  // time level of the pressure to sample
  const int buf = (int)(lev % a.d0.nbuf);

  // PMUT blocks come first: they carry the longest chains of dependent
  // loads, so they should all be resident from the start of the launch
  if (b < a.nb_pm) {
    // One PMUT.  Every load the update needs is issued up front (state,
    // ODE coefficients and drive value by the first threads, the sampled
    // pressures by all), so the block waits for memory once for the gather
    // of the samples and once for the force scatter's operands.
    const int s = b / a.Np, k = b - s * a.Np;
    const int Nm = a.Nm;
    const long qo = ((long)s * a.Np + k) * Nm;
    const int n0 = a.pm_off[k], n1 = a.pm_off[k + 1];
    const double dt = a.dt;
    // The block's first 256 face nodes (every node of a disc of up to 256):
    // the node index stays in a register and the projection row in the
    // thread's own LDS column from the sampling to the force scatter, which
    // then loads nothing from memory but the new accelerations.
    const int nf = n0 + tid;
    const bool mine = KEEP && nf < n1;
    const int nrest = KEEP ? nf + 256 : nf;  // nodes past the first 256
    const int node0 = mine ? a.pm_node[nf] : 0;
    if (!a.prime) {
      double q = 0, qd = 0, qdd = 0, w = 0, ze = 0, et = 0;
      const long pi = (long)k * Nm + tid;
      if (tid < Nm) {
        q = a.q[qo + tid];
        qd = a.qd[qo + tid];
        qdd = a.qdd[qo + tid];
        w = a.omega[pi];
        ze = a.zeta[pi];
        et = a.eta[pi];
      }
      const double t = lev * dt;
      const bool driven = !(t > a.t_switch);
      double c2x = 0, c2y = 0, d2x = 0, d2y = 0;
      if (tid == 0 && driven) {
        // A g(t) sin(2 pi f t - theta) = (A cos theta) g sin(2 pi f t) - (A sin theta) g cos(2 pi f t)
        const double* c2 = a.car + ((long)s * a.ncar + min(lev, a.ncar - 1)) * 2;
        const double* d2 = a.dA + ((long)s * a.Np + k) * 2;
        c2x = c2[0];
        c2y = c2[1];
        d2x = d2[0];
        d2y = d2[1];
      }
      double acc[MM];
#pragma unroll
      for (int m = 0; m < MM; ++m) acc[m] = 0.0;
      const Real* P0 = a.d0.P[buf] + (long)s * a.d0.nnodes;
      bool bad = false;
      if (mine) {
        const double p = (double)P0[node0];
        bad |= !__builtin_isfinite(p);
        const double* B = a.pm_B + (long)nf * Nm;
        double bm[MM];
#pragma unroll
        for (int m = 0; m < MM; ++m) bm[m] = B[min(m, Nm - 1)];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
          if (KEEP) sB[m][tid] = bm[m];
          if (m < Nm) acc[m] += bm[m] * p;
        }
      }
      // mode loops run over MM with clamped, unconditional loads: a
      // load under a per-mode condition would be waited for one mode at a time
      for (int n = nrest; n < n1; n += 256) {
        const double p = (double)P0[a.pm_node[n]];
        bad |= !__builtin_isfinite(p);
        const double* B = a.pm_B + (long)n * Nm;
        double bm[MM];
#pragma unroll
        for (int m = 0; m < MM; ++m) bm[m] = B[min(m, Nm - 1)];
#pragma unroll
        for (int m = 0; m < MM; ++m)
          if (m < Nm) acc[m] += bm[m] * p;
      }
      if (bad) atomicOr(a.nonfinite, 1);
      if (tid < Nm) {
        qp_s[tid] = q + dt * qd + 0.5 * dt * dt * qdd;
        qds_s[tid] = qd + 0.5 * dt * qdd;
      }
      {
        int m;
        const double v = wave_sum_many<MM>(acc, lane, &m);
        if ((lane & ((64 / MM) - 1)) == 0 && m < Nm) red[wave][m] = v;
      }
      __syncthreads();
      if (tid == 0) {
        double phi;
        if (!driven) {
          double em[MM];
#pragma unroll
          for (int m = 0; m < MM; ++m) em[m] = a.eta[(long)k * Nm + min(m, Nm - 1)];
          phi = 0.0;
#pragma unroll
          for (int m = 0; m < MM; ++m)
            if (m < Nm) phi += em[m] * qp_s[m];
          phi /= a.cap;
        } else {
          phi = d2x * c2x - d2y * c2y;
        }
        phi_s = phi;
      }
      __syncthreads();
      if (tid < Nm) {
        const double g = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
        const double qa = -w * w * qp_s[tid] - 2.0 * ze * w * qds_s[tid] + g + et * phi_s;
        a.q[qo + tid] = qp_s[tid];
        a.qd[qo + tid] = qds_s[tid] + 0.5 * dt * qa;
        a.qdd[qo + tid] = qa;
        qdd_s[tid] = qa;
      }
    } else {
      if (tid < Nm) qdd_s[tid] = a.qdd[qo + tid];
      if (mine) {
        const double* B = a.pm_B + (long)nf * Nm;
#pragma unroll
        for (int m = 0; m < MM; ++m)
          if (KEEP) sB[m][tid] = B[min(m, Nm - 1)];
      }
    }
    __syncthreads();
    Real* F = a.force + (long)s * a.d0.plane;  // padded bottom plane
    if (mine) {
      double f = 0.0;
#pragma unroll
      for (int m = 0; m < MM; ++m)
        if (m < Nm && KEEP) f += qdd_s[m] * sB[m][tid];
      F[node0] = (Real)(-a.kappa * f);
    }
    for (int n = nrest; n < n1; n += 256) {
      const double* B = a.pm_B + (long)n * Nm;
      double bm[MM];
#pragma unroll
      for (int m = 0; m < MM; ++m) bm[m] = B[min(m, Nm - 1)];
      double f = 0.0;
#pragma unroll
      for (int m = 0; m < MM; ++m)
        if (m < Nm) f += qdd_s[m] * bm[m];
      F[a.pm_node[n]] = (Real)(-a.kappa * f);
    }
  } else if ((b -= a.nb_pm) < a.nb_tr0) {
    face_traces(a, 0, b * 256 + tid, buf);
  } else if ((b -= a.nb_tr0) < a.nb_tr1) {
    face_traces(a, 1, b * 256 + tid, buf);
  } else if (!a.prime) {
    b -= a.nb_tr1;
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
               (double)Pd[base + i + (long)D.px * j + D.plane * c];
      }
      acc = wave_sum(acc);
      if (lane == 0 && cnt < a.tcap) a.traces[((long)s * a.R + r) * a.tcap + cnt] = acc;
      if (lane == 0 && !__builtin_isfinite(acc)) atomicOr(a.nonfinite, 1);
    }
  }


}

template <typename Real, int MM>
__global__ void __launch_bounds__(256) k_face(const FaceArgs<Real> a) {
  face_block<Real, MM, true>(a, blockIdx.x);
}

// Persistent face kernel over the (problem, unit) work list of a batch.
template <typename Real, int MM>
__global__ void __launch_bounds__(256) k_face_batch(const FaceArgs<Real>* __restrict__ probs,
                                                    const int2* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    __syncthreads();
    face_block<Real, MM, false>(probs[w.x], w.y);
  }
}

// Advances the step counters of all problems of a batch.
__global__ void k_tick_batch(long* const* __restrict__ counters, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd((unsigned long long*)counters[i], 1ull);
}

// ------------------------------------------------------------------------
// Interface flux, in two passes over Gamma_I.
//   k_flux_fine: one half-wave per fine face.  The face's value / normal-derivative
//     traces are staged in LDS and interpolated to its Nq x Nq Gauss points by
//     two 1D contractions; the coarse traces are interpolated the same way
//     (x first, over the at most 2 N1 + 1 coarse node rows the face touches,
//     then y).  At each point the SIPG integrand gives
//       A_q = w J (gamma [p] - {c^2 d_n p}),  B_q = -w J [p] / 2,
//     stored for the coarse pass and reduced onto the fine face's nodes.
//   k_flux_coarse: one half-wave per coarse face: reduces the A_q, B_q of the
//     points mapped into it onto its nodes (two 1D contractions), and, in the
//     last launch of a step, advances the step counter.
// ------------------------------------------------------------------------
// LDS of a fine-pass workgroup, in Real entries: the two tables, then per
// face slot the fine traces, the x-contracted rows, the x-contracted coarse
// rows (a fine face meets at most two coarse element rows: 2 N1 + 1 node
// rows), the SIPG terms and the coarse y basis; the slots' coarse element
// rows (ints) follow.
__host__ __device__ inline int flux_fine_slot(int Nq, int N0, int N1) {
  const int n0 = N0 + 1, n1 = N1 + 1;
  return 2 * n0 * n0 + 2 * Nq * n0 + 2 * Nq * (2 * N1 + 1) + 2 * Nq * Nq + Nq * n1;
}

template <typename Real>
__device__ __forceinline__ void flux_fine_block(const FluxArgs<Real>& a, int blk, unsigned char* raw) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // two fine faces per wave, one per half-wave, so that a launch over the
  // interface fits the machine's wave slots in one round
  const int hl = lane & 31, slot = 2 * w + (lane >> 5);
  const int Nq = a.Nq, N0 = a.N0, N1 = a.N1, n0 = N0 + 1, n1 = N1 + 1;
  const int crow = 2 * N1 + 1, fs = flux_fine_slot(Nq, N0, N1);
  Real* sL = reinterpret_cast<Real*>(raw);
  Real* sW = sL + Nq * n0;
  Real* base = sW + Nq * Nq + slot * fs;
  Real* T0v = base;                  // fine traces: value, normal derivative
  Real* T0d = T0v + n0 * n0;
  Real* Rv = T0d + n0 * n0;          // x-contracted rows
  Real* Rd = Rv + Nq * n0;
  Real* Cv = Rd + Nq * n0;           // x-contracted coarse rows
  Real* Cd = Cv + Nq * crow;
  Real* Av = Cd + Nq * crow;         // SIPG terms at the Gauss points
  Real* Ad = Av + Nq * Nq;
  Real* Yw = Ad + Nq * Nq;           // coarse y basis of each Gauss row
  int* CY = reinterpret_cast<int*>(sW + Nq * Nq + 2 * kWaves * fs) + slot * Nq;
  const int nfine = a.nex0 * a.ney0;
  for (int i = threadIdx.x; i < Nq * n0; i += 64 * kWaves) sL[i] = a.Lq[i];
  for (int i = threadIdx.x; i < Nq * Nq; i += 64 * kWaves) sW[i] = a.wJ[i];
  const int item = blk * (2 * kWaves) + slot;
  const bool valid = item < a.S * nfine;
  const int s = valid ? item / nfine : 0, f = valid ? item - s * nfine : 0;
  const int ex = f % a.nex0, ey = f / a.nex0;
  const long nf0 = (long)a.nn0x * (a.ney0 * N0 + 1), nf1 = (long)a.nn1x * (a.ney1 * N1 + 1);
  const Real* T0 = a.tr0 + (long)s * nf0 * 2;
  const Real* T1 = a.tr1 + (long)s * nf1 * 2;
  // coarse node rows touched by this face (one lane per Gauss row, reduced
  // across the half-wave)
  int cy_lo = 1 << 30, cy_hi = -1;
  if (hl < Nq) {
    const int c = a.ycx[ey * Nq + hl];
    CY[hl] = c;
    cy_lo = cy_hi = c;
  }
  for (int l = hl; l < Nq * n1; l += 32) Yw[l] = a.yw[(long)(ey * Nq) * n1 + l];
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) {
    cy_lo = min(cy_lo, __shfl_xor(cy_lo, o, 64));
    cy_hi = max(cy_hi, __shfl_xor(cy_hi, o, 64));
  }
  const int ry0 = N1 * cy_lo, nrow = N1 * (cy_hi - cy_lo) + n1;
  // (1) fine traces into LDS; coarse traces contracted along x
  if (valid)
    for (int l = hl; l < n0 * n0; l += 32) {
      const long node = (long)(N0 * ex + l % n0) + (long)a.nn0x * (N0 * ey + l / n0);
      T0v[l] = T0[node * 2];
      T0d[l] = T0[node * 2 + 1];
    }
  // two items per lane and trip (a face meeting two coarse element rows has
  // up to Nq (2 N1 + 1) of them, more than 32 at N1 = 3), gathered in one
  // loop so that both items' loads are in flight together
  const int ncl = Nq * nrow;
  for (int l = hl; l < ncl; l += 64) {
    const int m = min(l + 32, ncl - 1);  // second item, or the first again
    const int qa = l % Nq, row = ry0 + l / Nq, qm = m % Nq, rowm = ry0 + m / Nq;
    const int cx = a.xcx[ex * Nq + qa], cxm = a.xcx[ex * Nq + qm];
    const Real* wx = a.xw + (long)(ex * Nq + qa) * n1;
    const Real* wm = a.xw + (long)(ex * Nq + qm) * n1;
    Real cv = 0, cd = 0, cvm = 0, cdm = 0;
    if (valid)
      for (int aa = 0; aa < n1; ++aa) {
        const long node = (long)(N1 * cx + aa) + (long)a.nn1x * row;
        const long nodm = (long)(N1 * cxm + aa) + (long)a.nn1x * rowm;
        cv += wx[aa] * T1[node * 2];
        cd += wx[aa] * T1[node * 2 + 1];
        cvm += wm[aa] * T1[nodm * 2];
        cdm += wm[aa] * T1[nodm * 2 + 1];
      }
    Cv[l] = cv;
    Cd[l] = cd;
    if (l + 32 < ncl) {
      Cv[m] = cvm;
      Cd[m] = cdm;
    }
  }
  __syncthreads();
  // (2) fine traces contracted along x: R[qa + Nq b]
  for (int l = hl; l < Nq * n0; l += 32) {
    const int qa = l % Nq, b = l / Nq;
    Real rv = 0, rd = 0;
    for (int aa = 0; aa < n0; ++aa) {
      const Real lq = sL[qa * n0 + aa];
      rv += lq * T0v[aa + n0 * b];
      rd += lq * T0d[aa + n0 * b];
    }
    Rv[l] = rv;
    Rd[l] = rd;
  }
  __syncthreads();
  // (3) SIPG integrand at the Gauss points
  for (int l = hl; l < Nq * Nq; l += 32) {
    const int qa = l % Nq, qb = l / Nq;
    Real pP = 0, dP = 0, pM = 0, dM = 0;
    for (int b = 0; b < n0; ++b) {
      const Real lq = sL[qb * n0 + b];
      pP += lq * Rv[qa + Nq * b];
      dP += lq * Rd[qa + Nq * b];
    }
    const int cy = CY[qb];
    const Real* wy = &Yw[qb * n1];
    for (int b = 0; b < n1; ++b) {
      const int li = qa + Nq * (N1 * cy + b - ry0);
      pM += wy[b] * Cv[li];
      dM += wy[b] * Cd[li];
    }
    const Real jump = pP - pM;
    const Real avg = Real(0.5) * (a.cf2 * dP + a.cc2 * dM);
    const Real wj = sW[qb * Nq + qa];
    const Real A = wj * (a.gamma * jump - avg), B = Real(-0.5) * wj * jump;
    Av[l] = A;
    Ad[l] = B;
    if (valid) {
      Real* o = a.Aq + (((long)s * nfine + f) * Nq * Nq + l) * 2;
      o[0] = A;
      o[1] = B;
    }
  }
  __syncthreads();
  // (4) reduce onto the fine nodes: contract along qb, then along qa
  for (int l = hl; l < Nq * n0; l += 32) {
    const int qa = l % Nq, b = l / Nq;
    Real ta = 0, tb = 0;
    for (int qb = 0; qb < Nq; ++qb) {
      const Real lq = sL[qb * n0 + b];
      ta += lq * Av[qa + Nq * qb];
      tb += lq * Ad[qa + Nq * qb];
    }
    Rv[l] = ta;
    Rd[l] = tb;
  }
  __syncthreads();
  if (valid)
    for (int l = hl; l < n0 * n0; l += 32) {
      const int aa = l % n0, b = l / n0;
      Real RA = 0, RB = 0;
      for (int qa = 0; qa < Nq; ++qa) {
        const Real lq = sL[qa * n0 + aa];
        RA += lq * Rv[qa + Nq * b];
        RB += lq * Rd[qa + Nq * b];
      }
      Real* R = a.R0 + (((long)s * nfine + f) * n0 * n0 + l) * 2;
      R[0] = RA;
      R[1] = RB;
    }
}

template <typename Real>
__global__ void __launch_bounds__(256) k_flux_fine(const FluxArgs<Real> a) {
  extern __shared__ __align__(16) unsigned char flux_lds[];
  flux_fine_block(a, blockIdx.x, flux_lds);
}

template <typename Real>
__global__ void __launch_bounds__(256) k_flux_coarse(const FluxArgs<Real> a) {
  // Two coarse faces per wave, one per half-wave, so that a launch over the
  // interface fits the machine's wave slots in one round.  Each face keeps
  // its y-contracted sums (tcap entries per component) in dynamic LDS.
  extern __shared__ __align__(16) unsigned char flux_lds[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int hl = lane & 31, slot = 2 * w + (lane >> 5);
  const int Nq = a.Nq, N1 = a.N1, n1 = N1 + 1, tc = a.tcap;
  const int nfine = a.nex0 * a.ney0, ncoarse = a.nex1 * a.ney1;
  const int item = blockIdx.x * (2 * kWaves) + slot;
  const bool valid = item < a.S * ncoarse;
  const int s = valid ? item / ncoarse : 0, f = valid ? item - s * ncoarse : 0;
  const int cx = f % a.nex1, cy = f / a.nex1;
  const int xo0 = a.xl_off[cx], nxl = a.xl_off[cx + 1] - xo0;
  const int yo0 = a.yl_off[cy], nyl = a.yl_off[cy + 1] - yo0;
  Real* TA = reinterpret_cast<Real*>(flux_lds) + 2 * slot * tc;
  Real* TB = TA + tc;
  // (1) contract along y: T[ix + nxl b] = sum_iy wy(iy)[b] A(ix, iy)
  for (int l = hl; l < nxl * n1; l += 32) {
    const int ix = l % nxl, b = l / nxl;
    const int ex_qa = a.xl[xo0 + ix];
    const int ex = ex_qa / Nq, qa = ex_qa % Nq;
    Real ta = 0, tb = 0;
    // unrolled so that the point-list loads of several rows are in flight
    // together ahead of the loads they address
    if (valid)
#pragma unroll 4
      for (int iy = 0; iy < nyl; ++iy) {
        const int ey_qb = a.yl[yo0 + iy];
        const int ey = ey_qb / Nq, qb = ey_qb % Nq;
        const Real wy = a.yw[(long)ey_qb * n1 + b];
        const Real* A = a.Aq + (((long)s * nfine + ex + (long)a.nex0 * ey) * Nq * Nq + qa + Nq * qb) * 2;
        ta += wy * A[0];
        tb += wy * A[1];
      }
    TA[l] = ta;
    TB[l] = tb;
  }
  __syncthreads();
  // (2) contract along x onto the coarse face's nodes
  if (valid)
    for (int l = hl; l < n1 * n1; l += 32) {
      const int aa = l % n1, b = l / n1;
      Real RA = 0, RB = 0;
      for (int ix = 0; ix < nxl; ++ix) {
        const Real wx = a.xw[(long)a.xl[xo0 + ix] * n1 + aa];
        RA += wx * TA[ix + nxl * b];
        RB += wx * TB[ix + nxl * b];
      }
      Real* R = a.R1 + (((long)s * ncoarse + f) * n1 * n1 + l) * 2;
      R[0] = RA;  // the stiffness kernel applies the coarse side's minus sign
      R[1] = RB;
    }
  if (a.tick && blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd((unsigned long long*)a.counter, 1ull);
    for (int d = 0; d < 2; ++d)
      if (a.toggle & (1 << d)) atomicXor(a.xsel + d, 1);
  }
}

// Advances the step counter when no interface pass ends the step.
__global__ void k_tick(long* counter, int* xsel, int toggle) {
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)counter, 1ull);
    for (int d = 0; d < 2; ++d)
      if (toggle & (1 << d)) atomicXor(xsel + d, 1);
  }
}

template <typename Real>
__global__ void k_fill(Real* p, long n, Real v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

// Packs rows of the trace buffer (leading dimension cap) into a dense
// [rows][n] array of type Out.
template <typename Out>
__global__ void k_pack_traces(const double* __restrict__ src, Out* __restrict__ dst, long cap, long n, long rows) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= rows * n) return;
  const long r = i / n, j = i - r * n;
  dst[i] = (Out)src[r * cap + j];
}

// ------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------
hipError_t launch_pack_traces(const double* src, void* dst, int bits, long cap, long n, long rows, hipStream_t st) {
  const long total = rows * n;
  if (total <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((total + 255) / 256);
  if (bits == 32)
    hipLaunchKernelGGL(k_pack_traces<float>, dim3(grid), dim3(256), 0, st, src, (float*)dst, cap, n, rows);
  else
    hipLaunchKernelGGL(k_pack_traces<double>, dim3(grid), dim3(256), 0, st, src, (double*)dst, cap, n, rows);
  return hipGetLastError();
}

template <>
hipError_t launch_stiff<float>(const StiffArgs<float>& a, bool incr, hipStream_t st) {
  if (!incr) return hipErrorInvalidValue;  // FP32 state always uses the increment form
  if (a.pml_acc) return launch_stiff_pml<float>(a, incr, st);
  return a.d.N <= 4 ? launch_stiff_f32_lo(a, st) : launch_stiff_f32_hi(a, st);
}

template <>
hipError_t launch_stiff<double>(const StiffArgs<double>& a, bool incr, hipStream_t st) {
  if (incr) return hipErrorInvalidValue;  // FP64 state uses the two-level form
  if (a.pml_acc) return launch_stiff_pml<double>(a, incr, st);
  return a.d.N <= 4 ? launch_stiff_f64_lo(a, st) : launch_stiff_f64_hi(a, st);
}

hipError_t launch_stiff2(const StiffArgs<float>& a, hipStream_t st) {
  if (stiff2_tile_rows(a.d.N) <= 0) return hipErrorInvalidValue;
  return launch_stiff2_lo(a, st);
}

// owned rows of the two-step tile: 16 extended rows less an N-row halo on
// each side (orders above 4 are not supported)
int stiff2_tile_rows(int N) { return (N >= 1 && N <= 4) ? 16 - 2 * N : 0; }

template <typename Real>
hipError_t launch_face(const FaceArgs<Real>& a, hipStream_t st) {
  if (a.Nm <= 4)
    hipLaunchKernelGGL((k_face<Real, 4>), dim3(a.nblocks), dim3(256), 0, st, a);
  else if (a.Nm <= 8)
    hipLaunchKernelGGL((k_face<Real, 8>), dim3(a.nblocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_face<Real, kMaxModes>), dim3(a.nblocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_flux(const FluxArgs<Real>& a, hipStream_t st) {
  if (a.nb_fine == 0) return hipSuccess;
  const size_t fine_lds = sizeof(Real) * ((size_t)a.Nq * (a.N0 + 1) + (size_t)a.Nq * a.Nq +
                                          2 * kWaves * (size_t)flux_fine_slot(a.Nq, a.N0, a.N1)) +
                          sizeof(int) * 2 * kWaves * (size_t)a.Nq;
  hipLaunchKernelGGL(k_flux_fine<Real>, dim3(a.nb_fine), dim3(256), fine_lds, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(Real) * 2 * (2 * kWaves) * (size_t)a.tcap;
  hipLaunchKernelGGL(k_flux_coarse<Real>, dim3(a.nb_coarse), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_face_batch(const FaceArgs<float>* probs, const int2* items, int nitems, int grid, int nm_max,
                             hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  if (nm_max <= 4)
    hipLaunchKernelGGL((k_face_batch<float, 4>), dim3(grid), dim3(256), 0, st, probs, items, nitems);
  else if (nm_max <= 8)
    hipLaunchKernelGGL((k_face_batch<float, 8>), dim3(grid), dim3(256), 0, st, probs, items, nitems);
  else
    hipLaunchKernelGGL((k_face_batch<float, kMaxModes>), dim3(grid), dim3(256), 0, st, probs, items, nitems);
  return hipGetLastError();
}

hipError_t launch_tick_batch(long* const* counters, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_tick_batch, dim3((n + 63) / 64), dim3(64), 0, st, counters, n);
  return hipGetLastError();
}

hipError_t launch_tick(long* counter, int* xsel, int toggle, hipStream_t st) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, counter, xsel, toggle);
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

// Perfectly matched layer of libpmutdg (Sec. 2, eq. full_problem):
//   p_tt + alpha p_t + beta p = div(c^2 grad p) + div Phi - gamma psi,
//   Phi_t = Z1 Phi + c^2 Z2 grad p + c^2 Z3 grad psi,   psi_t = p,
// Z1 = diag(-zeta_i), Z2 = diag(alpha - 2 zeta_i), Z3 = diag(zeta_j zeta_k),
// alpha, beta, gamma the sum, pair sum and product of the zeta_i.
//
// A brick with a layer runs its stiffness update with the layer's terms
// (k_stiff_pml: the damping alpha joins the absorbing term on the corrected
// velocity, and the layer's acceleration -(M^{-1} (Phi, grad v) + beta p +
// gamma psi) of the current level is added), then two kernels advance the
// auxiliary fields to the new level and form the next acceleration:
//   k_pml_phi   per layer element: Phi at its GLL nodes by the trapezoidal
//               rule, from the element-local gradients of the averaged p and
//               psi of the two levels (Phi is discontinuous across elements),
//               then the element's share of the weak divergence (Phi, grad v)
//               at each of its nodes;
//   k_pml_node  per node of the layer's elements: psi by the trapezoidal
//               rule, the shares of the (up to eight) layer elements sharing
//               the node, and the new acceleration.  No atomics: every node
//               sums its own terms in a fixed order.
#include "stiff_kernel.h"

namespace pmdg {

template <typename Real, int N, bool INCR, int RY>
__global__ void __launch_bounds__(256) k_stiff_pml(const StiffArgs<Real> a) {
  __shared__ Real lds[stiff_lds_elems<N, RY, 4>()];
  stiff_tile<Real, N, INCR, RY, 4, 2, true, true, true>(a, xcd_remap(blockIdx.x, a.nblocks), lds);
}

template <typename Real, int N, bool INCR>
static hipError_t stiff_pml_rows(const StiffArgs<Real>& a, hipStream_t st) {
  if (a.waves != 4 || a.depth != 2) return hipErrorInvalidValue;
  if (a.rows == 1) hipLaunchKernelGGL((k_stiff_pml<Real, N, INCR, 1>), dim3(a.nblocks), dim3(256), 0, st, a);
  else if (a.rows == 2) hipLaunchKernelGGL((k_stiff_pml<Real, N, INCR, 2>), dim3(a.nblocks), dim3(256), 0, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_stiff_pml(const StiffArgs<Real>& a, bool incr, hipStream_t st) {
  constexpr bool I = sizeof(Real) == 4;  // FP32: increment form; FP64: two-level form
  if (incr != I) return hipErrorInvalidValue;
  switch (a.d.N) {
    case 1: return stiff_pml_rows<Real, 1, I>(a, st);
    case 2: return stiff_pml_rows<Real, 2, I>(a, st);
    case 3: return stiff_pml_rows<Real, 3, I>(a, st);
    case 4: return stiff_pml_rows<Real, 4, I>(a, st);
    case 5: return stiff_pml_rows<Real, 5, I>(a, st);
    case 6: return stiff_pml_rows<Real, 6, I>(a, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_stiff_pml<float>(const StiffArgs<float>&, bool, hipStream_t);
template hipError_t launch_stiff_pml<double>(const StiffArgs<double>&, bool, hipStream_t);

// device index of node (i, j, k) of a brick
template <typename Real>
__device__ __forceinline__ long pml_dev(const DomView<Real>& d, int i, int j, int k) {
  return (long)i + (long)d.px * j + d.plane * k;
}

// Layer elements in groups of EPB per workgroup (one thread per GLL node).
// Levels: p^n = P[cnt % nbuf], p^{n+1} = P[(cnt + 1) % nbuf] (the step
// counter advances at the end of the step); psi still holds psi^n, so the
// average of psi over the step is psi^n + dt/4 (p^n + p^{n+1}).  After Phi,
// the element's share of the weak divergence at each of its nodes,
// r_E(i) = sum_q w_q J Phi(q) . grad v_i(q), which depends on this
// element's Phi only, is written per element node for k_pml_node to gather.
template <int N>
constexpr int pml_epb() {
  return (N + 1) * (N + 1) * (N + 1) <= 256 ? 256 / ((N + 1) * (N + 1) * (N + 1)) : 1;
}

template <typename Real, int N>
__global__ void __launch_bounds__(256) k_pml_phi(const PmlArgs<Real> a) {
  constexpr int n1 = N + 1, n3 = n1 * n1 * n1, EPB = pml_epb<N>();
  __shared__ Real pb[EPB * n3], sb[EPB * n3], pf[EPB * 3 * n3];
  const int s = blockIdx.y;
  const long cnt = *a.counter;
  const Real* P0 = a.d.P[cnt % a.d.nbuf] + (long)s * a.d.nnodes;
  const Real* P1 = a.d.P[(cnt + 1) % a.d.nbuf] + (long)s * a.d.nnodes;
  const Real* PS = a.psi + (long)s * a.d.nnodes;
  for (int t = threadIdx.x; t < EPB * n3; t += blockDim.x) {
    const int el = t / n3, q = t % n3, e = blockIdx.x * EPB + el;
    if (e >= a.nel) continue;
    const int ia = q % n1, ib = (q / n1) % n1, ic = q / (n1 * n1);
    const long g = pml_dev(a.d, N * a.pel[3 * e] + ia, N * a.pel[3 * e + 1] + ib, N * a.pel[3 * e + 2] + ic);
    const Real p0 = P0[g], p1 = P1[g];
    pb[t] = Real(0.5) * (p0 + p1);
    sb[t] = PS[g] + Real(0.25) * a.dt * (p0 + p1);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < EPB * n3; t += blockDim.x) {
    const int el = t / n3, q = t % n3, e = blockIdx.x * EPB + el;
    if (e >= a.nel) continue;
    const int ia = q % n1, ib = (q / n1) % n1, ic = q / (n1 * n1);
    const Real* PB = pb + el * n3;
    const Real* SB = sb + el * n3;
    Real gp[3] = {0, 0, 0}, gs[3] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < n1; ++m) {
      const Real dx = a.D[ia * n1 + m], dy = a.D[ib * n1 + m], dz = a.D[ic * n1 + m];
      gp[0] += dx * PB[m + n1 * (ib + n1 * ic)];
      gp[1] += dy * PB[ia + n1 * (m + n1 * ic)];
      gp[2] += dz * PB[ia + n1 * (ib + n1 * m)];
      gs[0] += dx * SB[m + n1 * (ib + n1 * ic)];
      gs[1] += dy * SB[ia + n1 * (m + n1 * ic)];
      gs[2] += dz * SB[ia + n1 * (ib + n1 * m)];
    }
    const int ex = a.pel[3 * e], ey = a.pel[3 * e + 1], ez = a.pel[3 * e + 2];
    const Real z[3] = {a.zx[N * ex + ia], a.zy[N * ey + ib], a.zz[N * ez + ic]};
    const Real al = z[0] + z[1] + z[2];
    Real* ph = a.phi + ((long)s * a.nel + e) * 3 * n3 + q;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const Real zjk = z[(i + 1) % 3] * z[(i + 2) % 3];
      const Real rhs = a.c2 * a.gh[i] * ((al - Real(2) * z[i]) * gp[i] + zjk * gs[i]);
      const Real hz = Real(0.5) * a.dt * z[i];
      const Real v = ((Real(1) - hz) * ph[i * n3] + a.dt * rhs) / (Real(1) + hz);
      ph[i * n3] = v;
      pf[(el * 3 + i) * n3 + q] = v;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < EPB * n3; t += blockDim.x) {
    const int el = t / n3, q = t % n3, e = blockIdx.x * EPB + el;
    if (e >= a.nel) continue;
    const int la = q % n1, lb = (q / n1) % n1, lc = q / (n1 * n1);
    const Real* F = pf + el * 3 * n3;
    Real gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int m = 0; m < n1; ++m) {
      gx += a.w[m] * a.D[m * n1 + la] * F[m + n1 * (lb + n1 * lc)];
      gy += a.w[m] * a.D[m * n1 + lb] * F[n3 + la + n1 * (m + n1 * lc)];
      gz += a.w[m] * a.D[m * n1 + lc] * F[2 * n3 + la + n1 * (lb + n1 * m)];
    }
    a.rel[((long)s * a.nel + e) * n3 + q] =
        a.J * (a.gh[0] * a.w[lb] * a.w[lc] * gx + a.gh[1] * a.w[la] * a.w[lc] * gy + a.gh[2] * a.w[la] * a.w[lb] * gz);
  }
}

// One thread per (node of the layer's elements, scenario).
template <typename Real, int N>
__global__ void __launch_bounds__(256) k_pml_node(const PmlArgs<Real> a) {
  constexpr int n1 = N + 1, n3 = n1 * n1 * n1;
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (tid >= (long)a.npn * a.S) return;
  const int s = (int)(tid / a.npn), v = (int)(tid % a.npn);
  const int I = a.pnode[3 * v], J = a.pnode[3 * v + 1], K = a.pnode[3 * v + 2];
  const long g = pml_dev(a.d, I, J, K);
  const long cnt = *a.counter;
  const long so = (long)s * a.d.nnodes;
  const Real pc = a.d.P[cnt % a.d.nbuf][so + g];
  Real pn = pc, ps = a.psi[so + g];
  if (!a.prime) {
    pn = a.d.P[(cnt + 1) % a.d.nbuf][so + g];
    ps += Real(0.5) * a.dt * (pc + pn);
    a.psi[so + g] = ps;
  }
  // (Phi, grad v) at this node: the shares of the layer elements containing it
  Real G = 0;
  const int exs[2] = {I / N - ((I % N == 0 && I > 0) ? 1 : 0), I / N};
  const int eys[2] = {J / N - ((J % N == 0 && J > 0) ? 1 : 0), J / N};
  const int ezs[2] = {K / N - ((K % N == 0 && K > 0) ? 1 : 0), K / N};
  for (int jz = 0; jz < 2; ++jz) {
    const int ez = ezs[jz];
    if ((jz && ez == ezs[0]) || ez < 0 || ez >= a.ne[2]) continue;
    for (int jy = 0; jy < 2; ++jy) {
      const int ey = eys[jy];
      if ((jy && ey == eys[0]) || ey < 0 || ey >= a.ne[1]) continue;
      for (int jx = 0; jx < 2; ++jx) {
        const int ex = exs[jx];
        if ((jx && ex == exs[0]) || ex < 0 || ex >= a.ne[0]) continue;
        const int slot = a.eslot[ex + a.ne[0] * (ey + a.ne[1] * ez)];
        if (slot < 0) continue;
        const int la = I - N * ex, lb = J - N * ey, lc = K - N * ez;
        G += a.rel[((long)s * a.nel + slot) * n3 + la + n1 * (lb + n1 * lc)];
      }
    }
  }
  const Real z0 = a.zx[I], z1 = a.zy[J], z2 = a.zz[K];
  const Real be = z0 * z1 + z1 * z2 + z2 * z0, ga = z0 * z1 * z2;
  const Real minv = a.mix[I] * a.miy[J] * a.miz[K];
  a.acc[so + g] = -(minv * G + be * pn + ga * ps);
}

template <typename Real, int N>
static hipError_t pml_order(const PmlArgs<Real>& a, hipStream_t st) {
  if (!a.prime && a.nel > 0)
    hipLaunchKernelGGL((k_pml_phi<Real, N>), dim3((a.nel + pml_epb<N>() - 1) / pml_epb<N>(), a.S), dim3(256), 0, st,
                       a);
  const long nt = (long)a.npn * a.S;
  if (nt > 0) hipLaunchKernelGGL((k_pml_node<Real, N>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_pml(const PmlArgs<Real>& a, hipStream_t st) {
  switch (a.d.N) {
    case 1: return pml_order<Real, 1>(a, st);
    case 2: return pml_order<Real, 2>(a, st);
    case 3: return pml_order<Real, 3>(a, st);
    case 4: return pml_order<Real, 4>(a, st);
    case 5: return pml_order<Real, 5>(a, st);
    case 6: return pml_order<Real, 6>(a, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_pml<float>(const PmlArgs<float>&, hipStream_t);
template hipError_t launch_pml<double>(const PmlArgs<double>&, hipStream_t);

}  // namespace pmdg

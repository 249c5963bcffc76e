// Stiffness update on trilinear hexahedra (Sec. 3: every element is the
// image of the reference cube under a trilinear map X_K; the volume term of
// the bilinear form a, eq. Wf_2, becomes, after the change of variables
// x = X_K(xi), the integral over the reference cube of
// c^2 (J^{-T} grad_xi p) . (J^{-T} grad_xi v) |J|, taken by GLL collocation).
//
// Two launches per step:
//   k_hex_elem: per element, the reference gradient of p by the 1D
//     derivative matrix along each axis (sum factorisation), the metric
//     G = w |J| c^2 J^{-1} J^{-T} from the trilinear map at each node
//     (computed from the element's eight corners, nothing stored per node),
//     and the transposed contraction; each element writes its residual at
//     its own (N+1)^3 nodes, so no two workgroups add into one address.
//   k_hex_node: per node, the sum of the residuals of the (up to eight)
//     elements holding it, the PMUT face force, the inverse lumped mass and
//     the explicit Newmark update (increment form in FP32, two-level form in
//     FP64), the same update as on bricks.
#include "pmutdg_internal.h"

namespace pmdg {

template <int N>
__host__ __device__ constexpr int hex_epb() {
  return (N + 1) * (N + 1) * (N + 1) <= 256 ? 256 / ((N + 1) * (N + 1) * (N + 1)) : 1;
}

template <typename Real, int N>
__global__ void __launch_bounds__(256) k_hex_elem(const HexArgs<Real> a) {
  constexpr int n1 = N + 1, n3 = n1 * n1 * n1, EPB = hex_epb<N>();
  __shared__ Real u[EPB][n3];
  __shared__ Real F[EPB][3][n3];
  __shared__ Real V[EPB][24];
  __shared__ Real Dm[n1 * n1];
  const int tid = threadIdx.x;
  const long total = (long)a.S * a.nel;
  const long g0 = (long)blockIdx.x * EPB;
  const long cnt = *a.counter;
  const Real* __restrict__ P = a.d.P[(int)(cnt % a.d.nbuf)];
  if (tid < n1 * n1) Dm[tid] = a.D[tid];
  for (int t = tid; t < EPB * 24; t += 256) {
    const int es = t / 24, j = t - es * 24;
    const long ge = g0 + es;
    V[es][j] = ge < total ? a.vert[(ge % a.nel) * 24 + j] : Real(0);
  }
  for (int t = tid; t < EPB * n3; t += 256) {
    const int es = t / n3, i = t - es * n3;
    const long ge = g0 + es;
    Real v = Real(0);
    if (ge < total) {
      const int s = (int)(ge / a.nel), e = (int)(ge % a.nel);
      const int ex = e % a.ne[0], ey = (e / a.ne[0]) % a.ne[1], ez = e / (a.ne[0] * a.ne[1]);
      const int ia = i % n1, ib = (i / n1) % n1, ic = i / (n1 * n1);
      const long node = (long)(N * ex + ia) + (long)a.d.px * (N * ey + ib) + a.d.plane * (N * ez + ic);
      v = P[(long)s * a.d.nnodes + node];
    }
    u[es][i] = v;
  }
  __syncthreads();
  // reference flux G grad_xi (p - p_0) at every node (p_0: the element's
  // first nodal value; grad_xi of a constant is zero, so subtracting it only
  // removes rounding from the sums)
  for (int t = tid; t < EPB * n3; t += 256) {
    const int es = t / n3, i = t - es * n3;
    const int ia = i % n1, ib = (i / n1) % n1, ic = i / (n1 * n1);
    const Real u0 = u[es][0];
    Real g0r = 0, g1r = 0, g2r = 0;
#pragma unroll
    for (int m = 0; m < n1; ++m) {
      g0r += Dm[ia * n1 + m] * (u[es][m + n1 * (ib + n1 * ic)] - u0);
      g1r += Dm[ib * n1 + m] * (u[es][ia + n1 * (m + n1 * ic)] - u0);
      g2r += Dm[ic * n1 + m] * (u[es][ia + n1 * (ib + n1 * m)] - u0);
    }
    // J[r][c] = d x_r / d xi_c of the trilinear map at this node
    const Real xi[3] = {a.xg[ia], a.xg[ib], a.xg[ic]};
    Real J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int c = 1; c < 8; ++c) {
      const Real s0 = (c & 1) ? Real(1) : Real(-1), s1 = (c & 2) ? Real(1) : Real(-1), s2 = (c & 4) ? Real(1) : Real(-1);
      const Real f0 = Real(0.5) * (Real(1) + s0 * xi[0]), f1 = Real(0.5) * (Real(1) + s1 * xi[1]),
                 f2 = Real(0.5) * (Real(1) + s2 * xi[2]);
      const Real d0 = Real(0.5) * s0 * f1 * f2, d1 = Real(0.5) * s1 * f0 * f2, d2 = Real(0.5) * s2 * f0 * f1;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const Real vc = V[es][3 * c + r];
        J[r][0] += d0 * vc;
        J[r][1] += d1 * vc;
        J[r][2] += d2 * vc;
      }
    }
    // cofactors: adj(J) = det(J) J^{-1}
    const Real A00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], A01 = J[0][2] * J[2][1] - J[0][1] * J[2][2],
               A02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    const Real A10 = J[1][2] * J[2][0] - J[1][0] * J[2][2], A11 = J[0][0] * J[2][2] - J[0][2] * J[2][0],
               A12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    const Real A20 = J[1][0] * J[2][1] - J[1][1] * J[2][0], A21 = J[0][1] * J[2][0] - J[0][0] * J[2][1],
               A22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const Real det = J[0][0] * A00 + J[0][1] * A10 + J[0][2] * A20;
    // grad_x p = J^{-T} grad_xi p = adj^T g / det; flux = w |J| c^2 J^{-1} grad_x p
    //          = w c^2 adj (adj^T g) / det
    const Real hx = A00 * g0r + A10 * g1r + A20 * g2r;
    const Real hy = A01 * g0r + A11 * g1r + A21 * g2r;
    const Real hz = A02 * g0r + A12 * g1r + A22 * g2r;
    const Real sc = a.w[ia] * a.w[ib] * a.w[ic] * a.c2 / det;
    F[es][0][i] = sc * (A00 * hx + A01 * hy + A02 * hz);
    F[es][1][i] = sc * (A10 * hx + A11 * hy + A12 * hz);
    F[es][2][i] = sc * (A20 * hx + A21 * hy + A22 * hz);
  }
  __syncthreads();
  for (int t = tid; t < EPB * n3; t += 256) {
    const int es = t / n3, i = t - es * n3;
    const long ge = g0 + es;
    if (ge >= total) continue;
    const int ia = i % n1, ib = (i / n1) % n1, ic = i / (n1 * n1);
    Real r = 0;
#pragma unroll
    for (int m = 0; m < n1; ++m) {
      r += Dm[m * n1 + ia] * F[es][0][m + n1 * (ib + n1 * ic)];
      r += Dm[m * n1 + ib] * F[es][1][ia + n1 * (m + n1 * ic)];
      r += Dm[m * n1 + ic] * F[es][2][ia + n1 * (ib + n1 * m)];
    }
    a.y[ge * n3 + i] = r;
  }
}

// Elements along one axis holding node index i (at most two) and the
// node's local index in each.
template <int N>
__device__ __forceinline__ int hex_owners(int i, int ne, int e[2], int l[2]) {
  int n = 0;
  const int q = i / N, r = i - q * N;
  if (q < ne) { e[n] = q; l[n] = r; ++n; }
  if (r == 0 && q > 0) { e[n] = q - 1; l[n] = N; ++n; }
  return n;
}

template <typename Real, int N, bool INCR>
__global__ void __launch_bounds__(256) k_hex_node(const HexArgs<Real> a) {
  constexpr int n1 = N + 1, n3 = n1 * n1 * n1;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = a.d.nnodes;
  if (id >= (long)a.S * per) return;
  const int s = (int)(id / per);
  const long node = id - (long)s * per;
  const int i = (int)(node % a.d.px);
  const long jk = node / a.d.px;
  const int j = (int)(jk % a.d.nn[1]), k = (int)(jk / a.d.nn[1]);
  if (i >= a.d.nn[0]) return;  // row padding
  int ex[2], lx[2], ey[2], ly[2], ez[2], lz[2];
  const int cx = hex_owners<N>(i, a.ne[0], ex, lx);
  const int cy = hex_owners<N>(j, a.ne[1], ey, ly);
  const int cz = hex_owners<N>(k, a.ne[2], ez, lz);
  const Real* __restrict__ Y = a.y + (long)s * a.nel * n3;
  Real kp = 0;
  for (int z = 0; z < cz; ++z)
    for (int yy = 0; yy < cy; ++yy)
      for (int x = 0; x < cx; ++x) {
        const long e = ex[x] + (long)a.ne[0] * (ey[yy] + (long)a.ne[1] * ez[z]);
        kp += Y[e * n3 + lx[x] + n1 * (ly[yy] + n1 * lz[z])];
      }
  const long cnt = *a.counter;
  const int cur = (int)(cnt % a.d.nbuf), nxt = (int)((cnt + 1) % a.d.nbuf);
  const long o = (long)s * per + node;
  const Real p0 = a.d.P[cur][o];
  const Real mi = a.minv[node];
  Real f = -kp;
  if (a.force && k == 0) f += a.force[(long)s * a.d.plane + node];
  const Real acc = a.dt2 * mi * f;
  if (INCR) {
    Real* X = a.d.X + (long)(*a.d.xsel) * a.d.xstride;
    const Real xv = X[o] + acc;
    X[o] = xv;
    a.d.P[nxt][o] = p0 + xv;
  } else {
    const Real pm = a.d.P[nxt][o];
    a.d.P[nxt][o] = p0 + (p0 - pm) + acc;
  }
}

template <typename Real, int N>
static hipError_t hex_launch_n(const HexArgs<Real>& a, bool incr, hipStream_t st) {
  hipLaunchKernelGGL((k_hex_elem<Real, N>), dim3(a.eblocks), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long nodes = (long)a.S * a.d.nnodes;
  const dim3 g((unsigned)((nodes + 255) / 256));
  if (incr)
    hipLaunchKernelGGL((k_hex_node<Real, N, true>), g, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_hex_node<Real, N, false>), g, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename Real>
int hex_elems_per_block(int N) {
  switch (N) {
    case 1: return hex_epb<1>();
    case 2: return hex_epb<2>();
    case 3: return hex_epb<3>();
    case 4: return hex_epb<4>();
    case 5: return hex_epb<5>();
    case 6: return hex_epb<6>();
    case 7: return hex_epb<7>();
    case 8: return hex_epb<8>();
  }
  return 0;
}

template <typename Real>
hipError_t launch_hex(const HexArgs<Real>& a, bool incr, hipStream_t st) {
  if (incr != std::is_same<Real, float>::value) return hipErrorInvalidValue;
  switch (a.d.N) {
    case 1: return hex_launch_n<Real, 1>(a, incr, st);
    case 2: return hex_launch_n<Real, 2>(a, incr, st);
    case 3: return hex_launch_n<Real, 3>(a, incr, st);
    case 4: return hex_launch_n<Real, 4>(a, incr, st);
    case 5: return hex_launch_n<Real, 5>(a, incr, st);
    case 6: return hex_launch_n<Real, 6>(a, incr, st);
    case 7: return hex_launch_n<Real, 7>(a, incr, st);
    case 8: return hex_launch_n<Real, 8>(a, incr, st);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_hex<float>(const HexArgs<float>&, bool, hipStream_t);
template hipError_t launch_hex<double>(const HexArgs<double>&, bool, hipStream_t);
template int hex_elems_per_block<float>(int);
template int hex_elems_per_block<double>(int);

}  // namespace pmdg

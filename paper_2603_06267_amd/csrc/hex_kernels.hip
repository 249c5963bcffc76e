// Stiffness update on trilinear hexahedra (Sec. 3: every element is the
// image of the reference cube under a trilinear map X_K; the volume term of
// the bilinear form a, eq. Wf_2, becomes, after the change of variables
// x = X_K(xi), the integral over the reference cube of
// c^2 (J^{-T} grad_xi p) . (J^{-T} grad_xi v) |J|, taken by GLL collocation).
//
// Two launches per step:
//   k_hex_elem: per strip of elements along x (p staged in LDS row by row,
//     shared nodes loaded once), one thread per (element, a, b) column of
//     nodes marching along c: the reference gradient of p by the 1D
//     derivative matrix along each axis (sum factorisation), the metric
//     G = w |J| c^2 J^{-1} J^{-T} at each node (the Jacobian's column d is
//     the bilinear interpolation of the element's four half edges along d;
//     nothing is stored per node), and the transposed contraction, whose
//     component along c stays in the thread's registers; each element
//     writes its residual at its own (N+1)^3 nodes, so no two workgroups add
//     into one address.
//   k_hex_node: per node, the sum of the residuals of the (up to eight)
//     elements holding it, the PMUT face force, the inverse lumped mass and
//     the explicit Newmark update (increment form in FP32, two-level form in
//     FP64), the same update as on bricks.
#include <algorithm>

#include "pmutdg_internal.h"

namespace pmdg {

// Elements per workgroup: a strip of SX consecutive elements along x, one
// thread per (element, a, b) column of nodes.
template <int N>
__host__ __device__ constexpr int hex_sx() {
  return 256 / ((N + 1) * (N + 1));
}

// Residual layout (x-contiguous): for element row (ey, ez) and local row
// (b, c), the entries of all elements of the row follow each other along x,
// element ex at ex (N+1) + a; so a wave writing one strip and a wave
// gathering one node row both touch consecutive addresses.
template <int N, typename Real>
__device__ __forceinline__ long hex_yidx(const HexArgs<Real>& a, int ex, int ey, int ez, int la, int lb, int lc) {
  constexpr int n1 = N + 1;
  return (((long)(ez * a.ne[1] + ey) * n1 + lc) * n1 + lb) * ((long)a.ne[0] * n1) + (long)ex * n1 + la;
}

// 1 / x: the hardware reciprocal in FP32 (1 ulp, for the metric's 1 / |J|
// with |J| > 0), IEEE division in FP64
template <typename Real>
__device__ __forceinline__ Real hex_rcp(Real x) {
  return Real(1) / x;
}
template <>
__device__ __forceinline__ float hex_rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// One element strip of a workgroup: position in the mesh and scenario.
struct HexStrip {
  int ex0, ey, ez, s, nsx;  // first element along x, row, layer, scenario, elements in the strip
};

template <int SX>
__device__ __forceinline__ HexStrip hex_strip(const int ne[3], int t) {
  const int nsx = (ne[0] + SX - 1) / SX;
  HexStrip q;
  const int sx = t % nsx;
  t /= nsx;
  q.ey = t % ne[1];
  t /= ne[1];
  q.ez = t % ne[2];
  q.s = t / ne[2];
  q.ex0 = sx * SX;
  q.nsx = min(SX, ne[0] - q.ex0);
  return q;
}

// Persistent: workgroup b takes strips b, b + gridDim.x, ...  The next
// strip's p and corner offsets are loaded into registers before the current
// strip's arithmetic and written to LDS after it, so their memory latency
// overlaps the arithmetic; two barriers per strip, as without the overlap.
template <typename Real, int N>
__global__ void __launch_bounds__(256) k_hex_elem(const HexArgs<Real> a) {
  constexpr int n1 = N + 1, n2 = n1 * n1, n3 = n2 * n1, SX = hex_sx<N>(), UX = SX * N + 1;
  constexpr int NW = (n2 * UX + 255) / 256, NE = (SX * 36 + 255) / 256;  // staged values per thread
  __shared__ Real u[n2 * UX];      // p on the strip's nodes, [c][b][x]
  __shared__ Real F0[SX * n3];     // reference flux components 0 and 1,
  __shared__ Real F1[SX * n3];     //   [element][c][b][a]
  __shared__ Real E[SX][12][3];    // half edge vectors: 4 along each axis
  __shared__ Real Dm[n2], Wq[n1], Xq[n1];
  const int tid = threadIdx.x;
  const int nstrips = a.eblocks;
  const long cnt = *a.counter;
  const Real* __restrict__ Pl = a.d.P[(int)(cnt % a.d.nbuf)];
  if (tid < n2) Dm[tid] = a.D[tid];
  if (tid < n1) {
    Wq[tid] = a.w[tid];
    Xq[tid] = a.xg[tid];
  }
  Real pu[NW], pe[NE];
  // p on the strip: rows of nsx N + 1 consecutive nodes (indices split by
  // the compile-time row width UX; entries past the strip are zero and never
  // read); half edge vectors: edges along axis d join corners c and
  // c | (1 << d) for the four c with bit d clear, in increasing order of c
  auto fetch = [&](const HexStrip& q) {
    const Real* __restrict__ P0 =
        Pl + (long)q.s * a.d.nnodes + (long)q.ex0 * N + (long)a.d.px * (q.ey * N) + a.d.plane * (q.ez * N);
    const int ux = q.nsx * N + 1;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int w = tid + 256 * i, row = w / UX, xl = w - row * UX, lb = row % n1, lc = row / n1;
      pu[i] = (w < n2 * UX && xl < ux) ? P0[xl + (long)a.d.px * lb + a.d.plane * lc] : Real(0);
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int w = tid + 256 * i, el = w / 36, r = w - el * 36, q3 = r / 3, k = r - 3 * q3, d = q3 / 4, m = q3 % 4;
      Real v = 0;
      if (w < SX * 36 && el < q.nsx) {
        const int lo = m & ((1 << d) - 1), c0 = lo | ((m >> d) << (d + 1));
        const long e = (long)(q.ex0 + el) + (long)a.ne[0] * (q.ey + (long)a.ne[1] * q.ez);
        const Real* V = a.vert + e * 24;
        v = Real(0.5) * (V[3 * (c0 | (1 << d)) + k] - V[3 * c0 + k]);
      }
      pe[i] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int w = tid + 256 * i;
      if (w < n2 * UX) u[w] = pu[i];
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int w = tid + 256 * i;
      if (w < SX * 36) (&E[0][0][0])[w] = pe[i];
    }
  };
  int t = (int)blockIdx.x;
  HexStrip cur = hex_strip<SX>(a.ne, t < nstrips ? t : 0);
  if (t < nstrips) {
    fetch(cur);
    stash();
  }
  __syncthreads();
  // thread -> (a fastest, element, b): consecutive threads write consecutive
  // residual addresses
  const int ia = tid % n1, el = (tid / n1) % SX, ib = tid / (n1 * SX);
  for (; t < nstrips; t += gridDim.x) {
    const int tn = t + (int)gridDim.x;
    HexStrip nxt = cur;
    if (tn < nstrips) {
      nxt = hex_strip<SX>(a.ne, tn);
      fetch(nxt);
    }
    const int ex0 = cur.ex0, ey = cur.ey, ez = cur.ez, s = cur.s;
    const bool active = tid < SX * n2 && el < cur.nsx;
    Real f2[n1];
    if (active) {
      // Jacobian column d at a node is the bilinear interpolation of the four
      // half edges along d in the other two reference coordinates: column 2
      // depends on (a, b) only; columns 0 and 1 are blended along c below
      const Real xa = Xq[ia], xb = Xq[ib];
      // columns 0 and 1 are linear in the third coordinate zc: M + zc D
      Real c2[3], MA[3], DA[3], MB[3], DB[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // axis 2 edges: bits (0, 1) = (a, b)
        const Real lo = Real(0.5) * ((1 - xa) * E[el][8][k] + (1 + xa) * E[el][9][k]);
        const Real hi = Real(0.5) * ((1 - xa) * E[el][10][k] + (1 + xa) * E[el][11][k]);
        c2[k] = Real(0.5) * ((1 - xb) * lo + (1 + xb) * hi);
        // axis 0 edges: bits (1, 2) = (b, c); blend along b now, along c later
        const Real A0 = Real(0.5) * ((1 - xb) * E[el][0][k] + (1 + xb) * E[el][1][k]);
        const Real A1 = Real(0.5) * ((1 - xb) * E[el][2][k] + (1 + xb) * E[el][3][k]);
        // axis 1 edges: bits (0, 2) = (a, c)
        const Real B0 = Real(0.5) * ((1 - xa) * E[el][4][k] + (1 + xa) * E[el][5][k]);
        const Real B1 = Real(0.5) * ((1 - xa) * E[el][6][k] + (1 + xa) * E[el][7][k]);
        MA[k] = Real(0.5) * (A0 + A1);
        DA[k] = Real(0.5) * (A1 - A0);
        MB[k] = Real(0.5) * (B0 + B1);
        DB[k] = Real(0.5) * (B1 - B0);
      }
      const Real* ue = u + el * N;
      Real da[n1], db[n1], ucol[n1];
#pragma unroll
      for (int m = 0; m < n1; ++m) {
        da[m] = Dm[ia * n1 + m];
        db[m] = Dm[ib * n1 + m];
        ucol[m] = ue[(m * n1 + ib) * UX + ia];
      }
      const Real wab = Wq[ia] * Wq[ib] * a.c2;
#pragma unroll
      for (int ic = 0; ic < n1; ++ic) {
        Real g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
        for (int m = 0; m < n1; ++m) {
          g0 += da[m] * ue[(ic * n1 + ib) * UX + m];
          g1 += db[m] * ue[(ic * n1 + m) * UX + ia];
          g2 += Dm[ic * n1 + m] * ucol[m];
        }
        const Real zc = Xq[ic];
        const Real J00 = MA[0] + zc * DA[0], J10 = MA[1] + zc * DA[1], J20 = MA[2] + zc * DA[2];
        const Real J01 = MB[0] + zc * DB[0], J11 = MB[1] + zc * DB[1], J21 = MB[2] + zc * DB[2];
        const Real J02 = c2[0], J12 = c2[1], J22 = c2[2];
        const Real A00 = J11 * J22 - J12 * J21, A01 = J02 * J21 - J01 * J22, A02 = J01 * J12 - J02 * J11;
        const Real A10 = J12 * J20 - J10 * J22, A11 = J00 * J22 - J02 * J20, A12 = J02 * J10 - J00 * J12;
        const Real A20 = J10 * J21 - J11 * J20, A21 = J01 * J20 - J00 * J21, A22 = J00 * J11 - J01 * J10;
        const Real det = J00 * A00 + J01 * A10 + J02 * A20;
        // flux = w |J| c^2 J^{-1} J^{-T} grad_xi p = w c^2 adj (adj^T g) / det
        const Real hx = A00 * g0 + A10 * g1 + A20 * g2;
        const Real hy = A01 * g0 + A11 * g1 + A21 * g2;
        const Real hz = A02 * g0 + A12 * g1 + A22 * g2;
        const Real sc = wab * Wq[ic] * hex_rcp(det);
        const int o = el * n3 + (ic * n1 + ib) * n1 + ia;
        F0[o] = sc * (A00 * hx + A01 * hy + A02 * hz);
        F1[o] = sc * (A10 * hx + A11 * hy + A12 * hz);
        f2[ic] = sc * (A20 * hx + A21 * hy + A22 * hz);
      }
    }
    __syncthreads();
    if (active) {
      // transposed contraction: the test function's reference gradient at each
      // node; component 2 runs along this thread's own column
      // this thread's column of residual entries: consecutive c are one
      // (N+1) x (row length) block apart
      Real* __restrict__ Yc = a.y + (long)s * a.nel * n3 + hex_yidx<N>(a, ex0 + el, ey, ez, ia, ib, 0);
      const long ystride = (long)n1 * n1 * a.ne[0];
      const Real* f0 = F0 + el * n3;
      const Real* f1 = F1 + el * n3;
      Real dta[n1], dtb[n1];
#pragma unroll
      for (int m = 0; m < n1; ++m) {
        dta[m] = Dm[m * n1 + ia];
        dtb[m] = Dm[m * n1 + ib];
      }
#pragma unroll
      for (int ic = 0; ic < n1; ++ic) {
        Real v = 0;
#pragma unroll
        for (int m = 0; m < n1; ++m) {
          v += dta[m] * f0[(ic * n1 + ib) * n1 + m];
          v += dtb[m] * f1[(ic * n1 + m) * n1 + ia];
          v += Dm[m * n1 + ic] * f2[m];
        }
        Yc[ic * ystride] = v;
      }
    }
    // every thread is past its last read of u and E for this strip
    if (tn < nstrips) stash();
    __syncthreads();
    cur = nxt;
  }
}

// Elements along one axis holding node index i: element q = i / N at local
// index r = i - q N when q < ne, and element q - 1 at local index N when
// r = 0 and q > 0.
struct HexOwners {
  int q, r;
  bool lo, hi;  // element q holds the node; element q - 1 holds it
};

template <int N>
__device__ __forceinline__ HexOwners hex_owners(int i, int ne) {
  HexOwners o;
  o.q = i / N;
  o.r = i - o.q * N;
  o.lo = o.q < ne;
  o.hi = o.r == 0 && o.q > 0;
  return o;
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
  const HexOwners ox = hex_owners<N>(i, a.ne[0]), oy = hex_owners<N>(j, a.ne[1]), oz = hex_owners<N>(k, a.ne[2]);
  const Real* __restrict__ Y = a.y + (long)s * a.nel * n3;
  // the residual of (ex, ey, ez) at local (la, lb, lc) sits at
  // ((ez ne1 + ey) n1 + lc) n1 + lb) rows of ne0 n1 entries, then ex n1 + la
  const long rowlen = (long)a.ne[0] * n1;
  Real kp = 0;
#pragma unroll
  for (int z = 0; z < 2; ++z) {
    if (!(z ? oz.hi : oz.lo)) continue;
    const int ez = oz.q - z, lc = z ? N : oz.r;
#pragma unroll
    for (int yy = 0; yy < 2; ++yy) {
      if (!(yy ? oy.hi : oy.lo)) continue;
      const int ey = oy.q - yy, lb = yy ? N : oy.r;
      const Real* row = Y + ((((long)ez * a.ne[1] + ey) * n1 + lc) * n1 + lb) * rowlen;
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        if (!(x ? ox.hi : ox.lo)) continue;
        kp += row[(long)(ox.q - x) * n1 + (x ? N : ox.r)];
      }
    }
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
  const long strips = (long)(a.ne[0] + hex_sx<N>() - 1) / hex_sx<N>() * a.ne[1] * a.ne[2] * a.S;
  if (strips != a.eblocks) return hipErrorInvalidValue;
  // persistent: as many workgroups as fit the chip at once, at most one per
  // strip (the count is queried once per device and kept)
  constexpr int kDevices = 64;
  static int slots[kDevices] = {0};
  int dev = 0;
  hipError_t e0 = hipGetDevice(&dev);
  if (e0 != hipSuccess) return e0;
  int fit = (dev >= 0 && dev < kDevices) ? slots[dev] : 0;
  if (fit <= 0) {
    int cus = 0, per_cu = 0;
    e0 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e0 == hipSuccess) e0 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_hex_elem<Real, N>, 256, 0);
    if (e0 != hipSuccess) return e0;
    fit = std::max(1, cus * std::max(per_cu, 1));
    if (dev >= 0 && dev < kDevices) slots[dev] = fit;
  }
  const long grid = std::max(1L, std::min(strips, (long)fit));
  hipLaunchKernelGGL((k_hex_elem<Real, N>), dim3((unsigned)grid), dim3(256), 0, st, a);
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
    case 1: return hex_sx<1>();
    case 2: return hex_sx<2>();
    case 3: return hex_sx<3>();
    case 4: return hex_sx<4>();
    case 5: return hex_sx<5>();
    case 6: return hex_sx<6>();
    case 7: return hex_sx<7>();
    case 8: return hex_sx<8>();
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

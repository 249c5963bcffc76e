// Stiffness + update kernel of libpmutdg (CDNA4 / gfx950), included by the
// per-precision compilation units stiff_f32_*.hip and stiff_f64_*.hip.
//
// The volume operator of a uniform brick with GLL collocation is the
// Kronecker sum c^2 (A_x (x) I (x) I + I (x) A_y (x) I + I (x) I (x) A_z),
// A_d = M_d^{-1} K_d the assembled 1D operator (an exact identity of the
// tensor-product spectral element, equivalent to element-wise sum
// factorisation followed by assembly).  Each node therefore needs the 2N
// off-centre taps of its three grid lines; the kernel applies them in
// difference form sum_t a_t (p_{i+t} - p_i), which keeps the zero row sum of
// A_d exact in finite precision.
#pragma once

#include <utility>

#include "pmutdg_internal.h"

namespace pmdg {

// Compile-time loop: f(std::integral_constant<int, 0>{}) ... f(<N-1>).
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD works on a contiguous range of tiles (neighbouring tiles share halo
// planes through that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int xcd = b & 7, slot = b >> 3;
  return xcd * q + min(xcd, r) + slot;
}

// Masked store without a branch: a raw buffer store relative to one plane,
// where lanes outside the brick pass an offset beyond the plane's extent and
// the hardware drops them.  (A global store under a divergent branch makes the
// compiler's wait counting merge the taken and skipped paths conservatively:
// a later wait for an earlier prefetch then also waits for loads issued after
// the store.)  The plane must span fewer than 2^31 bytes.  NT selects
// non-temporal stores, for bricks far larger than L2: nothing reads the new
// level before the step's face kernel, and keeping it out of the way in L2
// leaves room for the halo rows of p that neighbouring tiles re-read.  (The
// batched form, whose meshes are small, keeps plain stores.)
constexpr unsigned kDropOffset = 0x80000000u;
template <bool NT, typename Real>
__device__ __forceinline__ void plane_store(Real* base, unsigned plane_bytes, unsigned off_bytes, Real v) {
  constexpr int cpol = NT ? 2 : 0;  // cache-policy operand: 2 = non-temporal
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)plane_bytes, 0x00020000);
  if constexpr (sizeof(Real) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, off_bytes, 0, cpol);
  } else {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, off_bytes, 0, cpol);
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------------
// Stiffness + update: 2.5D tiles (64 x TY nodes in x-y) marching along z.
// Rows are padded to a multiple of 64 nodes, so each wave's row segment is a
// cache-line aligned 64-lane access.  The z line lives in a register queue
// of 2N+1 planes per owned node (its rotation is unrolled so that no register
// moves are needed); the x and y lines are read from a double-buffered LDS
// copy of the current plane with an N-node halo.  Everything a plane needs
// (lead plane, halos, the increment or previous level) is fetched D planes
// ahead (two by default) so that memory latency overlaps the arithmetic of
// the planes in between, with one barrier per plane.  Operator rows come by
// node class (x per lane, y per wave row, z per plane, all uniform where the
// class is), as do the absorbing-face coefficients.
// Increment form (FP32): X holds p^n - p^{n-1}, X += a, p^{n+1} = p^n + X.
// Two-level form (FP64): p^{n+1} = p^n + (p^n - p^{n-1}) + a over p^{n-1}.
// ------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ int node_class(int i, int n) {
  return i == 0 ? N : (i == n - 1 ? N + 1 : i % N);
}

// LDS (in Real elements) of one stiffness workgroup: two plane buffers and
// the z rows by node class (2N taps, inverse mass, absorbing coefficient)
__host__ __device__ constexpr int stiff_lds_elems_rt(int N, int RY, int WV) {
  return 2 * (64 + 2 * N) * (WV * RY + 2 * N) + (N + 2) * (2 * N + 2);
}
template <int N, int RY, int WV>
__host__ __device__ constexpr int stiff_lds_elems() {
  return stiff_lds_elems_rt(N, RY, WV);
}

constexpr int ct_gcd(int a, int b) { return b == 0 ? a : ct_gcd(b, a % b); }

// One tile of the stiffness update (tile = linear tile index of the brick
// and scenario); lds holds stiff_lds_elems<N, RY, WV>() elements.  D is the
// prefetch distance in planes (the loads for plane k + D are issued while
// plane k is updated); NTS selects non-temporal stores; IFT builds in the
// interface traces (off for the batch kernel, whose problems have none).
template <typename Real, int N, bool INCR, int RY, int WV, int D = 2, bool NTS = true, bool IFT = true,
          bool PML = false>
__device__ __forceinline__ void stiff_tile(const StiffArgs<Real>& a, int tile_id, Real* __restrict__ lds) {
  constexpr int TX = 64, TY = WV * RY, W = TX + 2 * N, H = TY + 2 * N, NT = 2 * N, NQ = NT + 1;
  static_assert(D >= 2, "prefetch distance of at least two planes");
  // unrolled planes per loop trip: queue position (mod NQ) and prefetch slot
  // (mod D) are compile-time constants
  constexpr int U = NQ / ct_gcd(NQ, D) * D;
  constexpr int HYR = (NT + WV - 1) / WV;              // y-halo rows per wave
  constexpr int NXH = (TY * NT + 64 * WV - 1) / (64 * WV);  // x-halo loads per thread
  Real (*tile)[H * W] = reinterpret_cast<Real (*)[H * W]>(lds);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int t = tile_id;
  const int bx = t % a.nbx; t /= a.nbx;
  const int by = t % a.nby; t /= a.nby;
  const int bz = t % a.nbz; t /= a.nbz;
  const int s = t;

  const int nx = a.d.nn[0], ny = a.d.nn[1], nz = a.d.nn[2];
  const unsigned plane = (unsigned)a.d.plane;
  const unsigned plane_bytes = plane * (unsigned)sizeof(Real);
  const long cnt = *a.counter;
  if (a.cnt_snap && tile_id == 0 && tid == 0) *a.cnt_snap = cnt;
  const int cur = (int)(cnt % a.d.nbuf), nxt = (int)((cnt + 1) % a.d.nbuf);
  const Real* __restrict__ P = a.d.P[cur] + (long)s * a.d.nnodes;
  Real* __restrict__ Pn = a.d.P[nxt] + (long)s * a.d.nnodes;
  // increment (live copy), or p^{n-1}
  Real* __restrict__ X = INCR ? a.d.X + (long)(*a.d.xsel) * a.d.xstride + (long)s * a.d.nnodes : Pn;

  // Every load below is unconditional on a clamped address and masked
  // afterwards, so no load needs its own branch.
  constexpr int NC = N + 3;
  const Real* __restrict__ TP = a.taps;
  const Real* __restrict__ MI = a.mins;
  const unsigned px = (unsigned)a.d.px;
  // rows are padded to a multiple of 64 nodes: every lane's x is inside the
  // row.  Lanes past the last node load from the last node's address, so a
  // tile that holds the row's tail touches no cache line of padding alone.
  const int x = bx * TX + lane;
  const bool xin = x < nx;
  const unsigned xl = (unsigned)min(x, nx - 1);
  const int ybase = by * TY + wave * RY;

  Real tx[NT];
  const int cxl = xin ? node_class<N>(x, nx) : N + 2;  // class N+2: all-zero row
#pragma unroll
  for (int i = 0; i < NT; ++i) tx[i] = TP[cxl * NT + i];
  const Real mx = MI[cxl];
  // absorbing faces: g = dt (M^{-1} C)_ii = gx + gy + gz, dt c / m_d of the
  // end node of each absorbing face through the node (zero elsewhere).  The
  // solve (M + dt/2 C) pdd = f - K p - C pdot* with pdot* = (p^n - p^{n-1})
  // / dt turns the update into (acc - g (p^n - p^{n-1})) / (1 + g/2), which
  // is acc itself wherever g = 0; bricks without absorbing faces skip it.
  const bool absorb = a.absorb;
  const Real* __restrict__ AG = a.absg;
  const Real gx = AG[cxl];
  // layer damping per axis (PML build): dt zeta at the lane's x, row's y
  Real pzx = Real(0), pzy[RY];
  const Real* __restrict__ PA = PML ? a.pml_acc + (long)s * a.d.nnodes : nullptr;
  if constexpr (PML) pzx = a.dt * a.pml_zx[xl];
  int cyr[RY];
  bool in[RY];
  unsigned roff[RY];
  Real ty[RY][NT], my[RY], gxy[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = ybase + r;
    cyr[r] = y < ny ? node_class<N>(y, ny) : N + 2;
    in[r] = xin && y < ny;
    roff[r] = xl + px * (unsigned)min(y, ny - 1);
#pragma unroll
    for (int i = 0; i < NT; ++i) ty[r][i] = TP[(NC + cyr[r]) * NT + i];
    my[r] = MI[NC + cyr[r]];
    gxy[r] = gx + AG[NC + cyr[r]];
    pzy[r] = PML ? a.dt * a.pml_zy[min(y, ny - 1)] : Real(0);
  }
  // z operator rows by class, staged in LDS (read with uniform addresses)
  Real* ztab = lds + 2 * H * W;
  for (int i = tid; i < (N + 2) * (NT + 2); i += 64 * WV) {
    const int cls = i / (NT + 2), j = i % (NT + 2);
    ztab[i] = j < NT ? TP[(2 * NC + cls) * NT + j] : (j == NT ? MI[2 * NC + cls] : AG[2 * NC + cls]);
  }
  // x-halo slots of this thread: (row, column) pairs of the 2N x TY halo
  unsigned xh_off[NXH];
  int xh_dst[NXH];
  bool xh_ok[NXH];
#pragma unroll
  for (int j = 0; j < NXH; ++j) {
    const int e = tid + j * 64 * WV;
    const int hrow = e / NT, hc = e % NT;
    const int hx = hc < N ? (bx * TX - N + hc) : (bx * TX + TX + hc - N);
    const int y = by * TY + hrow;
    xh_ok[j] = e < TY * NT && hx >= 0 && hx < nx && y < ny;
    // a slot that loads nothing useful reads the lane's own row segment, so
    // that the wave's unused lanes share cache lines the wave loads anyway
    // instead of touching a line each
    xh_off[j] = xh_ok[j] ? (unsigned)hx + px * (unsigned)y : roff[0];
    xh_dst[j] = e < TY * NT ? ((N + hrow) * W + (hc < N ? hc : TX + hc)) : -1;
  }
  // y-halo rows of this wave
  unsigned yh_off[HYR];
  int yh_dst[HYR];
  bool yh_ok[HYR];
#pragma unroll
  for (int j = 0; j < HYR; ++j) {
    const int hr = wave + j * WV;
    const int trow = hr < N ? hr : (TY + hr);
    const int y = by * TY - N + trow;
    yh_ok[j] = hr < NT && xin && y >= 0 && y < ny;
    yh_off[j] = yh_ok[j] ? xl + px * (unsigned)y : roff[0];
    yh_dst[j] = hr < NT ? trow * W + N + lane : -1;
  }

  const int k0 = a.zlo + bz * a.zchunk;
  const int k1 = min(a.zhi + 1, k0 + a.zchunk);

  Real q[RY][NQ];
  Real xc[RY], ac[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int kk = k0 - N + i;
      const Real v = P[roff[r] + (unsigned)min(max(kk, 0), nz - 1) * plane];
      q[r][i] = (in[r] && kk >= 0 && kk < nz) ? v : Real(0);
    }
    const Real v = X[roff[r] + (unsigned)k0 * plane];
    xc[r] = in[r] ? v : Real(0);
    ac[r] = Real(0);
    if constexpr (PML) {
      const Real va = PA[roff[r] + (unsigned)k0 * plane];
      ac[r] = in[r] ? va : Real(0);
    }
  }
  {
    Real* T = tile[0];
#pragma unroll
    for (int r = 0; r < RY; ++r) T[(N + wave * RY + r) * W + N + lane] = q[r][N];
#pragma unroll
    for (int j = 0; j < NXH; ++j) {
      const Real v = P[xh_off[j] + (unsigned)k0 * plane];
      if (xh_dst[j] >= 0) T[xh_dst[j]] = xh_ok[j] ? v : Real(0);
    }
#pragma unroll
    for (int j = 0; j < HYR; ++j) {
      const Real v = P[yh_off[j] + (unsigned)k0 * plane];
      if (yh_dst[j] >= 0) T[yh_dst[j]] = yh_ok[j] ? v : Real(0);
    }
  }

  int lay0 = 1 << 30, lay1 = -1;
  if (a.iface) {
    if (a.iface_side > 0) { lay0 = nz - 1 - N; lay1 = nz - 1; }
    else { lay0 = 0; lay1 = N; }
  }
  constexpr int n1 = N + 1;
  // The PMUT force (plane 0) and the interface residual of a node's column
  // do not change along z: gather them once per tile, so that the plane loop
  // issues no loads but the streaming ones.
  Real fr[RY], RA[RY], RB[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) fr[r] = RA[r] = RB[r] = Real(0);
  if (a.force && k0 == 0) {
#pragma unroll
    for (int r = 0; r < RY; ++r)
      if (in[r]) fr[r] = a.force[(long)s * plane + roff[r]];
  }
  if (a.iface && k1 > lay0 && k0 <= lay1) {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (!in[r]) continue;
      // residual of the (up to 4) interface faces sharing (x, y)
      const int y = ybase + r;
      const int ex1 = min(x / N, a.iface_nex - 1), ey1 = min(y / N, a.iface_ney - 1);
      const int ax1 = x - N * ex1, by1 = y - N * ey1;
      const long fbase = (long)s * a.iface_nex * a.iface_ney;
#pragma unroll
      for (int jy = 0; jy < 2; ++jy) {
        const int ey = ey1 - jy, bb = jy ? N : by1;
        if (jy && !(by1 == 0 && ey1 > 0)) continue;
#pragma unroll
        for (int jx = 0; jx < 2; ++jx) {
          const int ex = ex1 - jx, aa = jx ? N : ax1;
          if (jx && !(ax1 == 0 && ex1 > 0)) continue;
          const Real* R = a.iface + ((fbase + ex + (long)a.iface_nex * ey) * (n1 * n1) + aa + n1 * bb) * 2;
          RA[r] += R[0];
          RB[r] += R[1];
        }
      }
    }
  }

  // Prefetch D planes ahead: iteration k consumes the loads for plane k+1
  // (issued at iteration k+1-D) and issues those for plane k+D, so each load
  // has D-1 plane updates of work to hide behind.  Slot (j - k0) mod D holds
  // the data for plane j: the queue's lead plane j+N, the increment (or
  // p^{n-1}) of plane j and the x/y halos of plane j.
  Real fq[D][RY], fx[D][RY], fa[D][RY], fhx[D][NXH], fhy[D][HYR];
  auto fetch = [&](int slot, int j) {
    const unsigned kl_off = (unsigned)min(j + N, nz - 1) * plane;
    const unsigned kn_off = (unsigned)min(j, nz - 1) * plane;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      fq[slot][r] = P[roff[r] + kl_off];
      fx[slot][r] = X[roff[r] + kn_off];
      if constexpr (PML) fa[slot][r] = PA[roff[r] + kn_off];
    }
    // unused halo slots read the lead-plane line of the lane's first row,
    // which the fetch has just requested: no further L2 request
#pragma unroll
    for (int jj = 0; jj < NXH; ++jj) fhx[slot][jj] = P[xh_off[jj] + (xh_ok[jj] ? kn_off : kl_off)];
#pragma unroll
    for (int jj = 0; jj < HYR; ++jj) fhy[slot][jj] = P[yh_off[jj] + (yh_ok[jj] ? kn_off : kl_off)];
  };
  static_for<D - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value + 1;
    fetch(i, k0 + i);
  });
  // value and normal derivative of p^{n+1} on Gamma_I, accumulated over the
  // interface element layer as its planes are updated (when the launch
  // writes the traces itself; the layer then lies inside one z chunk)
  Real tv[RY], td[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) tv[r] = td[r] = Real(0);
  const bool traces = IFT && a.trace != nullptr;
  const int tval = a.iface_side > 0 ? N : 0;  // layer index of the interface plane

  for (int kb = k0; kb < k1; kb += U) {
    static_for<U>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      constexpr int uq = u % NQ;
      constexpr int cs = (u + 1) % D;  // slot of plane k+1 (k - k0 = kb - k0 + u, U a multiple of D)
      constexpr int ns = u % D;        // slot of plane k+D
      const int k = kb + u;
      if (k >= k1) return;
      const int b = (k - k0) & 1;
      const int kn = k + 1;
      const bool more = kn < k1;
      // (1) fetch for plane k+D (unconditional on clamped addresses: a
      // conditional load would make its registers a join that the compiler
      // settles with copies, i.e. an early wait for the load)
      fetch(ns, k + D);
      // (2) plane k is complete in buffer b
      __syncthreads();
      // every LDS operand of the plane is read up front, so that the reads
      // overlap one another rather than each being waited for at its use
      const Real* T = tile[b];
      Real col[RY + NT], xl[RY][NT], tz[NT + 2];
#pragma unroll
      for (int j = 0; j < RY + NT; ++j) col[j] = T[(wave * RY + j) * W + N + lane];
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const int row = N + wave * RY + r;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          xl[r][i] = T[row * W + lane + i];
          xl[r][N + i] = T[row * W + N + lane + 1 + i];
        }
      }
      const int cz = node_class<N>(k, nz);
#pragma unroll
      for (int i = 0; i < NT + 2; ++i) tz[i] = ztab[cz * (NT + 2) + i];
      __builtin_amdgcn_sched_barrier(0);
      const Real mz = tz[NT];
      const Real pzz = PML ? a.dt * a.pml_zz[k] : Real(0);
      const bool in_layer = (k >= lay0 && k <= lay1);
      const int cl = k - lay0;
      // (3) update the nodes of plane k
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const Real p0 = q[r][(uq + N) % NQ];

        Real acc = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          acc += tx[i] * (xl[r][i] - p0);
          acc += tx[N + i] * (xl[r][N + i] - p0);
          acc += ty[r][i] * (col[r + i] - p0);
          acc += ty[r][N + i] * (col[r + N + 1 + i] - p0);
          acc += tz[i] * (q[r][(uq + i) % NQ] - p0);
          acc += tz[N + i] * (q[r][(uq + N + 1 + i) % NQ] - p0);
        }
        // lanes outside the brick compute on zeros and their stores are dropped
        const Real minv = mx * my[r] * mz;
        if (k == 0) acc += a.dt2 * minv * fr[r];
        if (in_layer) {
          Real rif = RB[r] * a.iface_d[cl];
          if (a.iface_side > 0) { if (cl == N) rif += RA[r]; }
          else { if (cl == 0) rif -= RA[r]; }
          acc -= a.dt2 * minv * rif;
        }
        if constexpr (PML) {
          // layer terms of the first row of eq. full_problem: the layer's
          // acceleration, and the damping alpha on the corrected velocity
          acc += a.dt2 * ac[r];
          const Real g = (absorb ? gxy[r] + tz[NT + 1] : Real(0)) + pzx + pzy[r] + pzz;
          acc = (acc - g * (INCR ? xc[r] : p0 - xc[r])) / (Real(1) + Real(0.5) * g);
        } else if (absorb) {
          const Real g = gxy[r] + tz[NT + 1];
          acc = (acc - g * (INCR ? xc[r] : p0 - xc[r])) / (Real(1) + Real(0.5) * g);
        }
        const unsigned soff = in[r] ? roff[r] * (unsigned)sizeof(Real) : kDropOffset;
        const long kp = (long)k * plane;
        Real pn;
        if (INCR) {
          const Real xv = xc[r] + acc;
          pn = p0 + xv;
          plane_store<NTS>(X + kp, plane_bytes, soff, xv);
        } else {
          pn = p0 + (p0 - xc[r]) + acc;
        }
        plane_store<NTS>(Pn + kp, plane_bytes, soff, pn);
        if (traces && in_layer) {
          td[r] += a.trd[cl] * pn;
          if (cl == tval) tv[r] = pn;
        }
      }
      // (4) plane k+1 into the other buffer
      if (more) {
        Real* Tn = tile[b ^ 1];
#pragma unroll
        for (int r = 0; r < RY; ++r) Tn[(N + wave * RY + r) * W + N + lane] = q[r][(uq + N + 1) % NQ];
#pragma unroll
        for (int j = 0; j < NXH; ++j)
          if (xh_dst[j] >= 0) Tn[xh_dst[j]] = xh_ok[j] ? fhx[cs][j] : Real(0);
#pragma unroll
        for (int j = 0; j < HYR; ++j)
          if (yh_dst[j] >= 0) Tn[yh_dst[j]] = yh_ok[j] ? fhy[cs][j] : Real(0);
      }
      // (5) rotate the queue: plane k+N+1 replaces plane k-N
      const int kl = k + N + 1;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        q[r][uq] = (in[r] && kl < nz) ? fq[cs][r] : Real(0);
        xc[r] = (in[r] && more) ? fx[cs][r] : Real(0);
        if constexpr (PML) ac[r] = (in[r] && more) ? fa[cs][r] : Real(0);
      }
    });
  }
  if (traces && k0 <= lay0 && lay1 < k1) {
    Real* TR = a.trace + (long)s * nx * ny * 2;
#pragma unroll
    for (int r = 0; r < RY; ++r)
      if (in[r]) {
        const long f = x + (long)nx * (ybase + r);
        TR[f * 2] = tv[r];
        TR[f * 2 + 1] = td[r];
      }
  }
}


template <typename Real, int N, bool INCR, int RY, int WV, int D = 2>
__global__ void __launch_bounds__(64 * WV) k_stiff(const StiffArgs<Real> a) {
  __shared__ Real lds[stiff_lds_elems<N, RY, WV>()];
  stiff_tile<Real, N, INCR, RY, WV, D>(a, xcd_remap(blockIdx.x, a.nblocks), lds);
}

template <typename Real, int N, bool INCR>
static hipError_t stiff_rows(const StiffArgs<Real>& a, hipStream_t st) {
  dim3 g(a.nblocks);
  if constexpr (deep_prefetch_built(N, 1, 4)) {
    if (a.depth > 2) {
      switch (a.rows + 8 * a.depth) {
        case 1 + 24: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 1, 4, 3>), g, dim3(256), 0, st, a); break;
        case 2 + 24: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 2, 4, 3>), g, dim3(256), 0, st, a); break;
        case 1 + 32: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 1, 4, 4>), g, dim3(256), 0, st, a); break;
        case 2 + 32: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 2, 4, 4>), g, dim3(256), 0, st, a); break;
        default: return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
  }
  switch (a.rows + 8 * a.waves) {
    case 1 + 32: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 1, 4>), g, dim3(256), 0, st, a); break;
    case 2 + 32: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 2, 4>), g, dim3(256), 0, st, a); break;
    case 4 + 32: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 4, 4>), g, dim3(256), 0, st, a); break;
    case 1 + 64: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 1, 8>), g, dim3(512), 0, st, a); break;
    case 2 + 64: hipLaunchKernelGGL((k_stiff<Real, N, INCR, 2, 8>), g, dim3(512), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Launchers for one precision and a range of orders (one per unit).
hipError_t launch_stiff_f32_lo(const StiffArgs<float>& a, hipStream_t st);
hipError_t launch_stiff_f32_hi(const StiffArgs<float>& a, hipStream_t st);
hipError_t launch_stiff_f64_lo(const StiffArgs<double>& a, hipStream_t st);
hipError_t launch_stiff_f64_hi(const StiffArgs<double>& a, hipStream_t st);

}  // namespace pmdg

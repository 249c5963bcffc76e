// Two steps of the FP32 increment-form stiffness update in one pass over
// memory (temporal blocking of the explicit Newmark scheme), included by
// stiff2_lo.hip.
//
// A workgroup owns a (64 - 2N) x TY node tile of every plane of a z range and
// computes, for the tile extended by N nodes on each side (64 lanes x
// TY + 2N rows),
//   stage 1   p^{n+1} = p^n + X^{n+1},  X^{n+1} = X^n + a(p^n)        (as the
//             single-step kernel: register queue along z, LDS plane of p^n),
//             kept in an LDS ring of the last 2N+2 planes,
//   stage 2   p^{n+2} = p^{n+1} + X^{n+2},  X^{n+2} = X^{n+1} + a(p^{n+1})
//             on the owned nodes, N+1 planes behind stage 1, from the ring.
// With stage 2 one plane further behind than its stencil needs, it reads
// only ring planes completed before the iteration's barrier and never the
// slot stage 1 is writing, so one barrier per plane suffices and the two
// stages of different waves overlap.
// So p^n and X^n are read once and p^{n+1}, p^{n+2}, X^{n+2} written once
// for two steps.  Stage 1 runs N planes beyond both ends of the z range so
// that stage 2 has its z neighbours.  Planes whose second step needs the
// coupling terms of step n+1 (PMUT force on the primary's bottom plane,
// interface residual on the interface layers) are left at p^{n+1} with
// X^{n+1} for a single-step completion pass after the face and interface
// kernels of step n+1.  The increment is read from one copy and written to
// the other, since stage 1 reads X^n on halo nodes that other workgroups
// update.
#pragma once

#include "stiff_kernel.h"

namespace pmdg {

// LDS (floats): two p^n plane buffers, the p^{n+1} ring, the z rows
template <int N, int RY, int WV>
__host__ __device__ constexpr int stiff2_lds_elems() {
  return 2 * (64 + 2 * N) * (WV * RY + 2 * N) + (2 * N + 2) * (WV * RY) * 64 + (N + 2) * (2 * N + 1);
}

template <int N, int RY, int WV>
__device__ __forceinline__ void stiff2_tile(const StiffArgs<float>& a, int tile_id, float* __restrict__ lds) {
  constexpr int TYE = WV * RY, TXO = 64 - 2 * N, TYO = TYE - 2 * N;
  constexpr int W = 64 + 2 * N, H = TYE + 2 * N, NT = 2 * N, NQ = NT + 1, NR = NT + 2;
  constexpr int HYR = (NT + WV - 1) / WV;                     // y-halo rows per wave
  constexpr int NXH = (TYE * NT + 64 * WV - 1) / (64 * WV);  // x-halo loads per thread
  static_assert(TYO >= 1, "tile too small for this order");
  float (*tile)[H * W] = reinterpret_cast<float (*)[H * W]>(lds);
  float (*ring)[TYE * 64] = reinterpret_cast<float (*)[TYE * 64]>(lds + 2 * H * W);
  float* ztab = lds + 2 * H * W + NR * TYE * 64;

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
  const long cnt = *a.counter;
  const int xs = *a.d.xsel;
  const float* __restrict__ P = a.d.P[cnt % 3] + (long)s * a.d.nnodes;
  float* __restrict__ P1 = a.d.P[(cnt + 1) % 3] + (long)s * a.d.nnodes;
  float* __restrict__ P2 = a.d.P[(cnt + 2) % 3] + (long)s * a.d.nnodes;
  const float* __restrict__ X0 = a.d.X + (long)xs * a.d.xstride + (long)s * a.d.nnodes;
  float* __restrict__ X1 = a.d.X + (long)(xs ^ 1) * a.d.xstride + (long)s * a.d.nnodes;

  constexpr int NC = N + 3;
  const float* __restrict__ TP = a.taps;
  const float* __restrict__ MI = a.mins;
  const unsigned px = (unsigned)a.d.px;
  // extended tile: lane <-> x = bx TXO - N + lane, row e <-> y = by TYO - N + e
  const int x = bx * TXO - N + lane;
  const bool xin = x >= 0 && x < nx;
  const unsigned xc_ = (unsigned)min(max(x, 0), nx - 1);
  const bool xown = lane >= N && lane < 64 - N && xin;
  const int ybase = by * TYO - N + wave * RY;

  float tx[NT];
  const int cxl = xin ? node_class<N>(x, nx) : N + 2;
#pragma unroll
  for (int i = 0; i < NT; ++i) tx[i] = TP[cxl * NT + i];
  const float mx = MI[cxl];
  bool in[RY], own[RY];
  unsigned roff[RY];
  float ty[RY][NT], my[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = ybase + r;
    const int e = wave * RY + r;
    const bool yin = y >= 0 && y < ny;
    const int cy = yin ? node_class<N>(y, ny) : N + 2;
    in[r] = xin && yin;
    own[r] = xown && yin && e >= N && e < TYE - N;
    roff[r] = xc_ + px * (unsigned)min(max(y, 0), ny - 1);
#pragma unroll
    for (int i = 0; i < NT; ++i) ty[r][i] = TP[(NC + cy) * NT + i];
    my[r] = MI[NC + cy];
  }
  for (int i = tid; i < (N + 2) * (NT + 1); i += 64 * WV) {
    const int cls = i / (NT + 1), j = i % (NT + 1);
    ztab[i] = j < NT ? TP[(2 * NC + cls) * NT + j] : MI[2 * NC + cls];
  }
  // x halo of the p^n plane: the N columns left and right of the extended
  // tile, for its TYE rows
  unsigned xh_off[NXH];
  int xh_dst[NXH];
  bool xh_ok[NXH];
#pragma unroll
  for (int j = 0; j < NXH; ++j) {
    const int e = tid + j * 64 * WV;
    const int hrow = e / NT, hc = e % NT;
    const int hx = hc < N ? (bx * TXO - 2 * N + hc) : (bx * TXO - N + 64 + hc - N);
    const int y = by * TYO - N + hrow;
    xh_ok[j] = e < TYE * NT && hx >= 0 && hx < nx && y >= 0 && y < ny;
    // unused slots read the lane's own row segment (no extra cache lines)
    xh_off[j] = xh_ok[j] ? (unsigned)hx + px * (unsigned)y : roff[0];
    xh_dst[j] = e < TYE * NT ? ((N + hrow) * W + (hc < N ? hc : 64 + hc)) : -1;
  }
  // y halo: N rows above and below the extended tile, 64 lanes each
  unsigned yh_off[HYR];
  int yh_dst[HYR];
  bool yh_ok[HYR];
#pragma unroll
  for (int j = 0; j < HYR; ++j) {
    const int hr = wave + j * WV;
    const int trow = hr < N ? hr : (TYE + hr);
    const int y = by * TYO - 2 * N + trow;
    yh_ok[j] = hr < NT && xin && y >= 0 && y < ny;
    yh_off[j] = yh_ok[j] ? xc_ + px * (unsigned)y : roff[0];
    yh_dst[j] = hr < NT ? trow * W + N + lane : -1;
  }

  // output planes [k0, k1); stage 1 runs over [k0 - N, k1 + N], stage 2
  // N+1 planes behind it
  const int k0 = a.zlo + bz * a.zchunk;
  const int k1 = min(a.zhi + 1, k0 + a.zchunk);
  const int ks = k0 - N, ke = k1 + N + 1;
  auto valid_plane = [&](int k) { return k >= 0 && k < nz; };
  auto completion = [&](int k) { return (k >= a.cb0 && k <= a.ce0) || (k >= a.cb1 && k <= a.ce1); };

  int lay0 = 1 << 30, lay1 = -1;
  if (a.iface) {
    if (a.iface_side > 0) { lay0 = nz - 1 - N; lay1 = nz - 1; }
    else { lay0 = 0; lay1 = N; }
  }
  constexpr int n1 = N + 1;
  // coupling terms of step n+1 (force f^n on plane 0, interface residual
  // R^n on the layers) for the extended nodes: stage 1 needs them
  float fr[RY], RA[RY], RB[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) fr[r] = RA[r] = RB[r] = 0.f;
  if (a.force && ks <= 0) {
#pragma unroll
    for (int r = 0; r < RY; ++r)
      if (in[r]) fr[r] = a.force[(long)s * plane + roff[r]];
  }
  if (a.iface && ke > lay0 && ks <= lay1) {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (!in[r]) continue;
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
          const float* R = a.iface + ((fbase + ex + (long)a.iface_nex * ey) * (n1 * n1) + aa + n1 * bb) * 2;
          RA[r] += R[0];
          RB[r] += R[1];
        }
      }
    }
  }

  // register queue of p^n along z for the extended nodes: planes k-N..k+N
  float q[RY][NQ];
  float xc[RY];
  auto zoff = [&](int k) { return (unsigned)min(max(k, 0), nz - 1) * plane; };
#pragma unroll
  for (int r = 0; r < RY; ++r) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int kk = ks - N + i;
      const float v = P[roff[r] + zoff(kk)];
      q[r][i] = (in[r] && valid_plane(kk)) ? v : 0.f;
    }
    const float v = X0[roff[r] + zoff(ks)];
    xc[r] = (in[r] && valid_plane(ks)) ? v : 0.f;
  }
  {
    float* T = tile[0];
    const bool vk = valid_plane(ks);
#pragma unroll
    for (int r = 0; r < RY; ++r) T[(N + wave * RY + r) * W + N + lane] = q[r][N];
#pragma unroll
    for (int j = 0; j < NXH; ++j) {
      const float v = P[xh_off[j] + zoff(ks)];
      if (xh_dst[j] >= 0) T[xh_dst[j]] = (xh_ok[j] && vk) ? v : 0.f;
    }
#pragma unroll
    for (int j = 0; j < HYR; ++j) {
      const float v = P[yh_off[j] + zoff(ks)];
      if (yh_dst[j] >= 0) T[yh_dst[j]] = (yh_ok[j] && vk) ? v : 0.f;
    }
  }

  // prefetch slots (two planes ahead, as the single-step kernel)
  float fq[2][RY], fx[2][RY], fhx[2][NXH], fhy[2][HYR];
  auto fetch = [&](int slot, int j) {
    const unsigned kl_off = zoff(j + N), kn_off = zoff(j);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      fq[slot][r] = P[roff[r] + kl_off];
      fx[slot][r] = X0[roff[r] + kn_off];
    }
#pragma unroll
    for (int jj = 0; jj < NXH; ++jj) fhx[slot][jj] = P[xh_off[jj] + kn_off];
#pragma unroll
    for (int jj = 0; jj < HYR; ++jj) fhy[slot][jj] = P[yh_off[jj] + kn_off];
  };
  fetch(1, ks + 1);

  // X^{n+1} of the owned nodes of the last NQ planes (stage 2 uses plane k-N-1)
  float xq[RY][NQ];
#pragma unroll
  for (int r = 0; r < RY; ++r)
#pragma unroll
    for (int i = 0; i < NQ; ++i) xq[r][i] = 0.f;

  int rslot = 0;  // ring slot of plane k: (k - ks) mod NR
  for (int kb = ks; kb < ke; kb += 2 * NQ) {
    static_for<2 * NQ>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      constexpr int uq = u % NQ;           // (k - ks) mod NQ
      constexpr int cs = (u + 1) & 1, ns = u & 1;
      const int k = kb + u;
      if (k >= ke) return;
      const int b = (k - ks) & 1;
      const bool more = k + 1 < ke;
      const bool vk = valid_plane(k);
      // (1) fetch for plane k+2
      fetch(ns, k + 2);
      // (2) plane k of p^n complete in buffer b, ring plane k-1 complete,
      // and stage 2 of the previous iteration done with the slot stage 1
      // overwrites now
      __syncthreads();
      const float* T = tile[b];
      float col[RY + NT];
#pragma unroll
      for (int j = 0; j < RY + NT; ++j) col[j] = T[(wave * RY + j) * W + N + lane];
      const int cz = vk ? node_class<N>(k, nz) : N + 2;
      const float* tz = ztab + min(cz, N + 1) * (NT + 1);
      const float mz = tz[NT];
      const bool in_layer = (k >= lay0 && k <= lay1);
      const int cl = k - lay0;
      const bool emit = k >= k0 && k < k1;
      // (3) stage 1: p^{n+1} of the extended nodes of plane k
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const int row = N + wave * RY + r;
        const float p0 = q[r][(uq + N) % NQ];
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          acc += tx[i] * (T[row * W + lane + i] - p0);
          acc += tx[N + i] * (T[row * W + N + lane + 1 + i] - p0);
          acc += ty[r][i] * (col[r + i] - p0);
          acc += ty[r][N + i] * (col[r + N + 1 + i] - p0);
          acc += tz[i] * (q[r][(uq + i) % NQ] - p0);
          acc += tz[N + i] * (q[r][(uq + N + 1 + i) % NQ] - p0);
        }
        float p1 = 0.f, x1 = 0.f;
        if (in[r] && vk) {
          const float minv = mx * my[r] * mz;
          if (k == 0) acc += a.dt2 * minv * fr[r];
          if (in_layer) {
            float rif = RB[r] * a.iface_d[cl];
            if (a.iface_side > 0) { if (cl == N) rif += RA[r]; }
            else { if (cl == 0) rif -= RA[r]; }
            acc -= a.dt2 * minv * rif;
          }
          x1 = xc[r] + acc;
          p1 = p0 + x1;
        }
        ring[rslot][(wave * RY + r) * 64 + lane] = p1;
        xq[r][uq] = x1;
        if (own[r] && emit) {
          const unsigned idx = roff[r] + (unsigned)k * plane;
          __builtin_nontemporal_store(p1, &P1[idx]);
          if (completion(k)) __builtin_nontemporal_store(x1, &X1[idx]);
        }
      }
      // (4) plane k+1 of p^n into the other buffer
      if (more) {
        float* Tn = tile[b ^ 1];
        const bool vn = valid_plane(k + 1);
#pragma unroll
        for (int r = 0; r < RY; ++r) Tn[(N + wave * RY + r) * W + N + lane] = q[r][(uq + N + 1) % NQ];
#pragma unroll
        for (int j = 0; j < NXH; ++j)
          if (xh_dst[j] >= 0) Tn[xh_dst[j]] = (xh_ok[j] && vn) ? fhx[cs][j] : 0.f;
#pragma unroll
        for (int j = 0; j < HYR; ++j)
          if (yh_dst[j] >= 0) Tn[yh_dst[j]] = (yh_ok[j] && vn) ? fhy[cs][j] : 0.f;
      }
      // (5) rotate the p^n queue: plane k+N+1 replaces plane k-N
      const int kl = k + N + 1;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        q[r][uq] = (in[r] && valid_plane(kl)) ? fq[cs][r] : 0.f;
        xc[r] = (in[r] && valid_plane(k + 1)) ? fx[cs][r] : 0.f;
      }
      // (6) stage 2: p^{n+2} of the owned nodes of plane m = k - N - 1 from
      // ring planes m-N .. m+N = k-2N-1 .. k-1
      const int m = k - N - 1;
      if (m >= k0 && m < k1 && !completion(m)) {
        constexpr int um = (u + 2 * NQ - N - 1) % NQ;  // xq slot of plane m
        const int rm = (rslot + NR - N - 1) % NR;       // ring slot of plane m
        int rz[NT];                                     // ring slots of m-N..m-1, m+1..m+N
#pragma unroll
        for (int i = 0; i < N; ++i) {
          rz[i] = (rm + NR - N + i) % NR;
          rz[N + i] = (rm + 1 + i) % NR;
        }
        const int czm = node_class<N>(m, nz);
        const float* tzm = ztab + czm * (NT + 1);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          if (!own[r]) continue;
          const int e = wave * RY + r;
          const float* Rm = ring[rm] + e * 64 + lane;
          const float c0 = Rm[0];
          float acc = 0.f;
#pragma unroll
          for (int i = 0; i < N; ++i) {
            acc += tx[i] * (Rm[i - N] - c0);
            acc += tx[N + i] * (Rm[1 + i] - c0);
            acc += ty[r][i] * (Rm[(i - N) * 64] - c0);
            acc += ty[r][N + i] * (Rm[(1 + i) * 64] - c0);
            acc += tzm[i] * (ring[rz[i]][e * 64 + lane] - c0);
            acc += tzm[N + i] * (ring[rz[N + i]][e * 64 + lane] - c0);
          }
          const float x2 = xq[r][um] + acc;
          const unsigned idx = roff[r] + (unsigned)m * plane;
          __builtin_nontemporal_store(c0 + x2, &P2[idx]);
          __builtin_nontemporal_store(x2, &X1[idx]);
        }
      }
      rslot = rslot + 1 == NR ? 0 : rslot + 1;
    });
  }
}

template <int N, int RY, int WV>
__global__ void __launch_bounds__(64 * WV) k_stiff2(const StiffArgs<float> a) {
  __shared__ float lds[stiff2_lds_elems<N, RY, WV>()];
  stiff2_tile<N, RY, WV>(a, xcd_remap(blockIdx.x, a.nblocks), lds);
}

// one tile shape per order: 8 waves x 2 rows (16 extended rows); orders up
// to 4 (the LDS of order 5 would exceed 64 KB)
template <int N>
static hipError_t stiff2_launch(const StiffArgs<float>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_stiff2<N, 2, 8>), dim3(a.nblocks), dim3(512), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_stiff2_lo(const StiffArgs<float>& a, hipStream_t st);

}  // namespace pmdg

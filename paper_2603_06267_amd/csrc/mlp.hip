// libpmutdg, surrogate form: a fully connected network that maps the drive
// parameters of a PMUT array (per-PMUT phase, frequency, amplitude) to
// receiver traces, trained and evaluated by hand-written BF16 MFMA kernels
// (CDNA4 v_mfma_f32_32x32x16_bf16) that accumulate in FP32, on FP32 master
// weights updated by Adam.
//
//   input     x_0 = bf16(embed(u)), rows optionally gathered: each network
//             input column takes one raw feature u_c, either affinely,
//             (u_c - shift) * scale, or through cos / sin (scale u_c + shift)
//             (angles, and Fourier features of a scalar)
//   forward   z_l = x_l W_l^T + b_l, x_{l+1} = bf16(gelu(z_l)) (hidden layers),
//             y = z_{L-1}; inference returns out_scale * a * y, where a is one
//             raw feature the output is proportional to (or 1)
//   loss      mean squared error against t / (out_scale a),
//             dz_{L-1} = 2 (y - t / (out_scale a)) / (B n_out)
//   backward  dW_l = dz_l^T x_l, db_l = sum over rows of dz_l,
//             dz_{l-1} = (dz_l W_l) * gelu'(z_{l-1})
//   update    Adam with bias correction on the FP32 masters; the BF16 copies
//             used by the GEMMs are refreshed in the same pass
//
// Layouts (row-major): activations [batch][width], the input width padded
// with zeros to a multiple of 32; W_l [n_out][n_in padded].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "pmutdg.h"
#include "pmutdg_internal.h"

namespace {

typedef unsigned short bf16_t;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

__device__ __forceinline__ bf16_t f2bf(float f) {
  // round to nearest, ties to even (operands are finite)
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// EPI_FWD_LIN_STAGED: EPI_FWD_LIN for outputs with 16-byte aligned rows and
// no split-K, stored through LDS as 16-byte row segments
enum { EPI_FWD_GELU = 0, EPI_FWD_LIN = 1, EPI_DX_GELU = 2, EPI_DW = 3, EPI_FWD_LIN_STAGED = 4 };

struct GemmArgs {
  int M, N, K;           // C[M][N] = sum_r A(i, r) B(r, j)
  const bf16_t* A;       // A(i, r) = A[i*lda + r] (ACON) or A[r*lda + i]
  const bf16_t* B;       // B(r, j) = B[j*ldb + r] (BCON) or B[r*ldb + j]
  int lda, ldb;
  const float* bias;     // [N] (forward epilogues)
  float* Cf;             // FP32 result (z, dz or dW), ld = ldc
  bf16_t* Cb;            // BF16 copy (activation or dz), ld = ldc
  int ldc;
  const float* Zprev;    // pre-activation for gelu' (EPI_DX_GELU), ld = ldc
  float* Y;              // EPI_FWD_LIN: if set, out_scale * rowscale[row] * z goes here instead of Cf
  float out_scale;
  const float* rowscale; // [M] per-row output factor
  float* part;           // split-K partial sums [ks][M][N]
  int mt, nt, ks, kchunk;
};

template <int EPI>
__device__ __forceinline__ void epilogue(const GemmArgs& g, int row, int col, float v) {
  const long o = (long)row * g.ldc + col;
  if (EPI == EPI_FWD_GELU) {
    const float z = v + g.bias[col];
    g.Cf[o] = z;
    g.Cb[o] = f2bf(gelu(z));
  } else if (EPI == EPI_FWD_LIN) {
    const float z = v + g.bias[col];
    if (g.Y) g.Y[o] = g.out_scale * g.rowscale[row] * z;
    else g.Cf[o] = z;
  } else if (EPI == EPI_DX_GELU) {
    const float d = v * gelu_d(g.Zprev[o]);
    g.Cf[o] = d;
    g.Cb[o] = f2bf(d);
  } else {
    g.Cf[o] = v;
  }
}

// Tile shape: 4 waves in 2 x 2, each wave TM x TN MFMA 32x32 blocks, so a
// workgroup computes (64 TM) x (64 TN) outputs over BK-deep slices.
template <int TM, int TN, int BK>
struct Tile {
  static constexpr int BM = 64 * TM, BN = 64 * TN, LDK = BK + 8;
};

// One output tile per workgroup of 4 waves.  MFMA 32x32x16 operand layout:
// lane l supplies row (A) or column (B) l % 32 and eight reduction indices
// chosen by l / 32 (the same for A and B, so the exact order within the 16
// does not matter); accumulator element r of lane l is row 8 (r / 4) +
// 4 (l / 32) + r % 4, column l % 32.  The linear grid is remapped so that the
// workgroups one XCD receives (dispatch is round-robin over the 8 XCDs) are
// consecutive tiles that share the same B (weight) tile, which then stays in
// that XCD's L2.  Operand rows are staged in LDS padded by 8 elements, so
// the 16-byte fragment reads of 32 consecutive rows hit distinct banks.
// The next slice is fetched into registers before the MFMAs of the current
// one and written to the other LDS buffer after them, so its memory latency
// overlaps the arithmetic; one barrier per slice.  LDS is dynamic:
// 2 (BM + BN) LDK elements.
template <bool ACON, bool BCON, int EPI, int TM, int TN, int BK>
__global__ void __launch_bounds__(256) k_gemm(const GemmArgs g) {
  using TL = Tile<TM, TN, BK>;
  constexpr int BM = TL::BM, BN = TL::BN, LDK = TL::LDK;
  constexpr int CA = BM * BK / 8 / 256, CB = BN * BK / 8 / 256;  // 8-element chunks per thread
  static_assert(CA * 256 * 8 == BM * BK && CB * 256 * 8 == BN * BK, "tile must split into chunks");
  extern __shared__ __attribute__((aligned(16))) bf16_t gemm_lds[];
  bf16_t* const As0 = gemm_lds;
  bf16_t* const Bs0 = gemm_lds + 2 * BM * LDK;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;

  const int nb = g.mt * g.nt * g.ks;
  int t = blockIdx.x;
  if ((nb & 7) == 0) t = (t & 7) * (nb >> 3) + (t >> 3);
  const int z = t / (g.mt * g.nt);
  const int rem = t - z * g.mt * g.nt;
  const int m0 = (rem % g.mt) * BM, n0 = (rem / g.mt) * BN;
  const int kbeg = z * g.kchunk, kend = min(g.K, kbeg + g.kchunk);

  // contiguous operand: chunk c covers row c / (BK/8), reduction 8 (c % (BK/8));
  // strided operand: chunk c covers reduction c / (B?/8), rows 8 (c % (B?/8))
  uint4 ra[CA], rb[CB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int c2 = 0; c2 < CA; ++c2) {
      const int c = tid + 256 * c2;
      ra[c2] = make_uint4(0, 0, 0, 0);
      if (ACON) {
        const int row = c / (BK / 8), kc = (c % (BK / 8)) * 8;
        if (m0 + row < g.M && k0 + kc < kend) ra[c2] = *(const uint4*)(g.A + (long)(m0 + row) * g.lda + k0 + kc);
      } else {
        const int r = c / (BM / 8), ic = (c % (BM / 8)) * 8;
        if (k0 + r < kend && m0 + ic < g.M) ra[c2] = *(const uint4*)(g.A + (long)(k0 + r) * g.lda + m0 + ic);
      }
    }
#pragma unroll
    for (int c2 = 0; c2 < CB; ++c2) {
      const int c = tid + 256 * c2;
      rb[c2] = make_uint4(0, 0, 0, 0);
      if (BCON) {
        const int col = c / (BK / 8), kc = (c % (BK / 8)) * 8;
        if (n0 + col < g.N && k0 + kc < kend) rb[c2] = *(const uint4*)(g.B + (long)(n0 + col) * g.ldb + k0 + kc);
      } else {
        const int r = c / (BN / 8), jc = (c % (BN / 8)) * 8;
        if (k0 + r < kend && n0 + jc < g.N) rb[c2] = *(const uint4*)(g.B + (long)(k0 + r) * g.ldb + n0 + jc);
      }
    }
  };
  auto stash = [&](int buf) {
    bf16_t* As = As0 + buf * BM * LDK;
    bf16_t* Bs = Bs0 + buf * BN * LDK;
#pragma unroll
    for (int c2 = 0; c2 < CA; ++c2) {
      const int c = tid + 256 * c2;
      if (ACON) {
        const int row = c / (BK / 8), kc = (c % (BK / 8)) * 8;
        *(uint4*)&As[row * LDK + kc] = ra[c2];
      } else {
        const int r = c / (BM / 8), ic = (c % (BM / 8)) * 8;
        const bf16_t* e = (const bf16_t*)&ra[c2];
#pragma unroll
        for (int q = 0; q < 8; ++q) As[(ic + q) * LDK + r] = e[q];
      }
    }
#pragma unroll
    for (int c2 = 0; c2 < CB; ++c2) {
      const int c = tid + 256 * c2;
      if (BCON) {
        const int col = c / (BK / 8), kc = (c % (BK / 8)) * 8;
        *(uint4*)&Bs[col * LDK + kc] = rb[c2];
      } else {
        const int r = c / (BN / 8), jc = (c % (BN / 8)) * 8;
        const bf16_t* e = (const bf16_t*)&rb[c2];
#pragma unroll
        for (int q = 0; q < 8; ++q) Bs[(jc + q) * LDK + r] = e[q];
      }
    }
  };

  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  const int nk = (kend - kbeg + BK - 1) / BK;
  if (nk > 0) {
    fetch(kbeg);
    stash(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) fetch(kbeg + (kt + 1) * BK);
    const bf16_t* As = As0 + buf * BM * LDK;
    const bf16_t* Bs = Bs0 + buf * BN * LDK;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8 af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int row = wm * 32 * TM + i * 32 + (lane & 31);
        af[i] = *(const bf16x8*)&As[row * LDK + kk + (lane >> 5) * 8];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = wn * 32 * TN + j * 32 + (lane & 31);
        bfr[j] = *(const bf16x8*)&Bs[col * LDK + kk + (lane >> 5) * 8];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    // buffer buf ^ 1 was last read in the previous slice, before its barrier
    if (more) stash(buf ^ 1);
    __syncthreads();
  }

  auto row_of = [&](int i, int r) { return m0 + wm * 32 * TM + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3); };
  // Linear outputs with 16-byte aligned rows: the tile goes through LDS (the
  // operand buffers are free: the loop ended with a barrier), so that every
  // thread then stores whole 16-byte row segments: a quarter of the store
  // instructions, and no accumulator copies held for the epilogue.  Same
  // arithmetic as the per-element epilogue below.
  if constexpr (EPI == EPI_FWD_LIN_STAGED) {
    // in one pass, or in two halves of rows (one per row of waves) when the
    // whole tile does not fit the operand buffers
    float* out = g.Y ? g.Y : g.Cf;
    constexpr int LDC = BN + 8, F4 = BN / 4, RPP = 256 / F4;
    constexpr size_t kLds = 2 * (BM + BN) * LDK * sizeof(bf16_t);
    constexpr int HALVES = BM * LDC * sizeof(float) <= kLds ? 1 : 2, HR = BM / HALVES, PASSES = HR / RPP;
    static_assert(HR * LDC * sizeof(float) <= kLds, "a half tile fits the LDS");
    static_assert(256 % F4 == 0 && HR % RPP == 0 && (HALVES == 1 || HR == 32 * TM), "tile splits into passes");
    float* T = reinterpret_cast<float*>(gemm_lds);
    const int cl = (tid % F4) * 4, rl0 = tid / F4, col = n0 + cl;
    const bool scaled = g.Y != nullptr;
    float b4[4], rsp[HALVES][PASSES];
#pragma unroll
    for (int c = 0; c < 4; ++c) b4[c] = g.bias[min(col + c, g.N - 1)];
#pragma unroll
    for (int h = 0; h < HALVES; ++h)
#pragma unroll
      for (int k = 0; k < PASSES; ++k)
        rsp[h][k] = scaled ? g.out_scale * g.rowscale[min(m0 + h * HR + rl0 + k * RPP, g.M - 1)] : 0.0f;
#pragma unroll
    for (int h = 0; h < HALVES; ++h) {
      if (HALVES == 1 || wm == h) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
              T[(wm * 32 * TM - h * HR + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3)) * LDC + wn * 32 * TN +
                j * 32 + (lane & 31)] = acc[i][j][r];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PASSES; ++k) {
        const int rl = rl0 + k * RPP, row = m0 + h * HR + rl;
        if (row >= g.M || col >= g.N) continue;
        const float4 v = *reinterpret_cast<const float4*>(&T[rl * LDC + cl]);
        const float vv[4] = {v.x, v.y, v.z, v.w};
        float o[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float zz = vv[c] + b4[c];
          o[c] = scaled ? rsp[h][k] * zz : zz;
        }
        float* dst = out + (long)row * g.ldc + col;
        if (col + 3 < g.N) {
          // non-temporal: nothing in this launch reads the output back
          typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4v;
          f4v ov = {o[0], o[1], o[2], o[3]};
          __builtin_nontemporal_store(ov, reinterpret_cast<f4v*>(dst));
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (col + c < g.N) dst[c] = o[c];
        }
      }
      if (HALVES > 1) __syncthreads();  // the next half reuses T
    }
  } else {
  auto col_of = [&](int j) { return n0 + wn * 32 * TN + j * 32 + (lane & 31); };
  if (g.ks > 1) {
    float* part = g.part + (long)z * g.M * g.N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row_of(i, r), col = col_of(j);
          if (row < g.M && col < g.N) part[(long)row * g.N + col] = acc[i][j][r];
        }
    return;
  }
  // The epilogue's operands (bias, row factors, pre-activations) are all
  // loaded before the first store, unconditionally from clamped indices:
  // the stores may alias them as far as the compiler knows, and a load
  // under a branch, or after a store, waits for its own result there, once
  // per element.
  float bj[TN], rs[TM][16];
  const bool scaled = EPI == EPI_FWD_LIN && g.Y != nullptr;
  if (EPI == EPI_FWD_GELU || EPI == EPI_FWD_LIN) {
#pragma unroll
    for (int j = 0; j < TN; ++j) bj[j] = g.bias[min(col_of(j), g.N - 1)];
  }
  if (scaled) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) rs[i][r] = g.out_scale * g.rowscale[min(row_of(i, r), g.M - 1)];
  }
  if (EPI == EPI_DX_GELU) {
    float zp[TM][TN][16];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          zp[i][j][r] = g.Zprev[(long)min(row_of(i, r), g.M - 1) * g.ldc + min(col_of(j), g.N - 1)];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] *= gelu_d(zp[i][j][r]);
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = row_of(i, r), col = col_of(j);
        if (row >= g.M || col >= g.N) continue;
        const long o = (long)row * g.ldc + col;
        const float v = acc[i][j][r];
        if (EPI == EPI_FWD_GELU) {
          const float zz = v + bj[j];
          g.Cf[o] = zz;
          g.Cb[o] = f2bf(gelu(zz));
        } else if (EPI == EPI_FWD_LIN) {
          const float zz = v + bj[j];
          if (scaled) g.Y[o] = rs[i][r] * zz;
          else g.Cf[o] = zz;
        } else if (EPI == EPI_DX_GELU) {
          g.Cf[o] = v;
          g.Cb[o] = f2bf(v);
        } else {
          g.Cf[o] = v;
        }
      }
  }
}

// split-K: sum the ks partial tiles in a fixed order, then the epilogue
template <int EPI>
__global__ void k_splitk_reduce(const GemmArgs g) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long MN = (long)g.M * g.N;
  if (i >= MN) return;
  float s = 0.f;
  for (int z = 0; z < g.ks; ++z) s += g.part[z * MN + i];
  epilogue<EPI>(g, (int)(i / g.N), (int)(i % g.N), s);
}

// One network input column: raw feature src (-1: zero padding) and how it
// enters (0: (u - shift) * scale, 1: cos(scale u + shift), 2: sin(scale u + shift)).
// Input column: g(u[src]; op, shift, scale), times a second such factor of
// u[src2] when src2 >= 0 (op 0: (x - shift) scale, 1: cos(scale x + shift),
// 2: sin(scale x + shift)).
struct EmbCol {
  int src, op;
  float shift, scale;
  int src2, op2;
  float shift2, scale2;
};

__device__ __forceinline__ float emb_factor(float x, int op, float shift, float scale) {
  return op == 0 ? (x - shift) * scale : (op == 1 ? cosf(scale * x + shift) : sinf(scale * x + shift));
}

// x_0[r][c] = bf16(embed column c of u[row r]), rowscale[r] = u[row r][amp]
__global__ void k_pack_input(const float* __restrict__ u, const int* __restrict__ idx, int nrows, int B, int nu, int ld,
                             const EmbCol* __restrict__ emb, int amp, bf16_t* __restrict__ X,
                             float* __restrict__ rowscale) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * ld) return;
  const int r = (int)(i / ld), c = (int)(i % ld);
  const long src = idx ? min(max(idx[r], 0), nrows - 1) : r;
  const EmbCol e = emb[c];
  float v = 0.f;
  if (e.src >= 0) {
    v = emb_factor(u[src * nu + e.src], e.op, e.shift, e.scale);
    if (e.src2 >= 0) v *= emb_factor(u[src * nu + e.src2], e.op2, e.shift2, e.scale2);
  }
  X[i] = f2bf(v);
  if (c == 0) rowscale[r] = amp >= 0 ? u[src * nu + amp] : 1.0f;
}

// per-row squared error and squared target norm (normalised units), and
// dz = 2 (y - t / (out_scale a)) / (B n); n a multiple of 4
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ Y, const float* __restrict__ T,
                                              const int* __restrict__ idx, int nrows, int B, int n, float inv_scale,
                                              const float* __restrict__ rowscale, float* __restrict__ dZ,
                                              bf16_t* __restrict__ dZb, float* __restrict__ rowerr,
                                              float* __restrict__ rownorm) {
  const int r = blockIdx.x;
  const long src = idx ? min(max(idx[r], 0), nrows - 1) : r;
  float se = 0.f, sn = 0.f;
  const float sc = 2.0f / ((float)B * (float)n);
  const float rs = rowscale[r];
  const float inv = rs != 0.f ? inv_scale / rs : 0.f;
  const float4* __restrict__ Y4 = (const float4*)(Y + (long)r * n);
  const float4* __restrict__ T4 = (const float4*)(T + src * n);
  float4* __restrict__ D4 = (float4*)(dZ + (long)r * n);
  uint2* __restrict__ Db = (uint2*)(dZb + (long)r * n);
  for (int c = threadIdx.x; c < n / 4; c += blockDim.x) {
    const float4 yv = Y4[c], tv4 = T4[c];
    const float t0 = tv4.x * inv, t1 = tv4.y * inv, t2 = tv4.z * inv, t3 = tv4.w * inv;
    const float d0 = yv.x - t0, d1 = yv.y - t1, d2 = yv.z - t2, d3 = yv.w - t3;
    se += (d0 * d0 + d1 * d1) + (d2 * d2 + d3 * d3);
    sn += (t0 * t0 + t1 * t1) + (t2 * t2 + t3 * t3);
    const float4 g = make_float4(sc * d0, sc * d1, sc * d2, sc * d3);
    D4[c] = g;
    Db[c] = make_uint2((unsigned)f2bf(g.x) | ((unsigned)f2bf(g.y) << 16), (unsigned)f2bf(g.z) | ((unsigned)f2bf(g.w) << 16));
  }
  __shared__ float s1[256], s2[256];
  s1[threadIdx.x] = se;
  s2[threadIdx.x] = sn;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s1[threadIdx.x] += s1[threadIdx.x + s];
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rowerr[r] = s1[0];
    rownorm[r] = s2[0];
  }
}

// db[c] = sum_r dz[r][c] in two passes: partial sums over chunks of 64
// rows (64 columns x 4 row groups per workgroup), then over the chunks
constexpr int kColChunk = 64;
__global__ void __launch_bounds__(256) k_colsum_part(const float* __restrict__ dZ, int B, int n,
                                                     float* __restrict__ part) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), rg = threadIdx.x >> 6;
  const int r0 = blockIdx.y * kColChunk, r1 = min(B, r0 + kColChunk);
  float s = 0.f;
  if (c < n)
    for (int r = r0 + rg; r < r1; r += 4) s += dZ[(long)r * n + c];
  __shared__ float sh[4][64];
  sh[rg][threadIdx.x & 63] = s;
  __syncthreads();
  if (rg == 0 && c < n)
    part[(long)blockIdx.y * n + c] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

__global__ void k_colsum_fin(const float* __restrict__ part, int nchunk, int n, float* __restrict__ db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float s = 0.f;
  for (int j = 0; j < nchunk; ++j) s += part[(long)j * n + c];
  db[c] = s;
}

// Adam on 4 consecutive values per thread (n a multiple of 4)
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, bf16_t* __restrict__ wb, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n / 4) return;
  const float4 g = ((const float4*)gr)[i];
  float4 mi = ((float4*)m)[i], vi = ((float4*)v)[i], wi = ((float4*)w)[i];
  const float ga[4] = {g.x, g.y, g.z, g.w};
  float ma[4] = {mi.x, mi.y, mi.z, mi.w}, va[4] = {vi.x, vi.y, vi.z, vi.w}, wa[4] = {wi.x, wi.y, wi.z, wi.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ma[j] = b1 * ma[j] + (1.f - b1) * ga[j];
    va[j] = b2 * va[j] + (1.f - b2) * ga[j] * ga[j];
    wa[j] = wa[j] - lr * (ma[j] / c1) / (sqrtf(va[j] / c2) + eps);
  }
  ((float4*)m)[i] = make_float4(ma[0], ma[1], ma[2], ma[3]);
  ((float4*)v)[i] = make_float4(va[0], va[1], va[2], va[3]);
  ((float4*)w)[i] = make_float4(wa[0], wa[1], wa[2], wa[3]);
  if (wb)
    ((uint2*)wb)[i] = make_uint2((unsigned)f2bf(wa[0]) | ((unsigned)f2bf(wa[1]) << 16),
                                 (unsigned)f2bf(wa[2]) | ((unsigned)f2bf(wa[3]) << 16));
}

__global__ void k_to_bf16(const float* __restrict__ w, bf16_t* __restrict__ wb, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) wb[i] = f2bf(w[i]);
}

// ensemble of two: mean into out and the per-row relative spread
// |a - b| / |(a + b) / 2| (0 where the mean vanishes)
// (out may alias a or b: each element is read before it is written, by the
// same thread)
__global__ void __launch_bounds__(256) k_pair_combine(const float* a, const float* b, int n, float* out,
                                                      float* __restrict__ spread) {
  const long base = (long)blockIdx.x * n;
  float s1 = 0.f, s2 = 0.f;
  for (int c = threadIdx.x * 4; c < n; c += 1024) {
    const float4 x = *(const float4*)(a + base + c), y = *(const float4*)(b + base + c);
    const float4 m = make_float4(0.5f * (x.x + y.x), 0.5f * (x.y + y.y), 0.5f * (x.z + y.z), 0.5f * (x.w + y.w));
    const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z, dw = x.w - y.w;
    s1 += dx * dx + dy * dy + dz * dz + dw * dw;
    s2 += m.x * m.x + m.y * m.y + m.z * m.z + m.w * m.w;
    *(float4*)(out + base + c) = m;
  }
  __shared__ float t1[256], t2[256];
  t1[threadIdx.x] = s1;
  t2[threadIdx.x] = s2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      t1[threadIdx.x] += t1[threadIdx.x + s];
      t2[threadIdx.x] += t2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) spread[blockIdx.x] = t2[0] > 0.f ? sqrtf(t1[0] / t2[0]) : 0.f;
}

inline long nblk(long n, int b) { return (n + b - 1) / b; }

pmdg_status mfail(pmdg_status s, const std::string& m) {
  pmdg::set_last_error(m);
  return s;
}

constexpr int kTargetBlocks = 256;  // one workgroup per CU
constexpr size_t kPartFloats = (size_t)384 * 128 * 128;

// split-K factor: ks * tiles <= kTargetBlocks + tiles, chunks of >= 64
void plan_split(GemmArgs& g, int BM, int BN) {
  g.mt = (g.M + BM - 1) / BM;
  g.nt = (g.N + BN - 1) / BN;
  const int tiles = g.mt * g.nt;
  int ks = 1;
  if (tiles < kTargetBlocks / 2) {
    ks = (kTargetBlocks + tiles - 1) / tiles;
    ks = std::min(ks, std::max(1, g.K / 64));
  }
  g.kchunk = (int)((g.K + ks - 1) / ks + 31) / 32 * 32;
  g.ks = (g.K + g.kchunk - 1) / g.kchunk;
}

template <bool ACON, bool BCON, int EPI, int TM, int TN, int BK>
hipError_t gemm_t_launch(const GemmArgs& g, hipStream_t st) {
  using TL = Tile<TM, TN, BK>;
  const size_t lds = sizeof(bf16_t) * 2 * (TL::BM + TL::BN) * TL::LDK;
  if (lds > 65536) {
    const hipError_t attr = hipFuncSetAttribute((const void*)k_gemm<ACON, BCON, EPI, TM, TN, BK>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
  }
  hipLaunchKernelGGL((k_gemm<ACON, BCON, EPI, TM, TN, BK>), dim3(g.mt * g.nt * g.ks), dim3(256), lds, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.ks == 1) return e;
  hipLaunchKernelGGL((k_splitk_reduce<EPI>), dim3((unsigned)nblk((long)g.M * g.N, 256)), dim3(256), 0, st, g);
  return hipGetLastError();
}

template <bool ACON, bool BCON, int EPI, int TM, int TN, int BK>
hipError_t gemm_t(GemmArgs g, float* part, hipStream_t st) {
  using TL = Tile<TM, TN, BK>;
  plan_split(g, TL::BM, TL::BN);
  g.part = part;
  if (g.ks > 1 && (size_t)g.ks * g.M * g.N > kPartFloats) {
    g.kchunk = ((g.K + 31) / 32) * 32;
    g.ks = 1;
  }
  if constexpr (EPI == EPI_FWD_LIN) {
    // linear outputs staged through LDS where half the tile fits the operand
    // buffers and the rows are 16-byte aligned
    constexpr bool fits =
        TL::BM / 2 * (TL::BN + 8) * sizeof(float) <= 2 * (TL::BM + TL::BN) * TL::LDK * sizeof(bf16_t);
    const float* out = g.Y ? g.Y : g.Cf;
    if constexpr (fits) {
      if (g.ks == 1 && (g.ldc & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0)
        return gemm_t_launch<ACON, BCON, EPI_FWD_LIN_STAGED, TM, TN, BK>(g, st);
    }
  }
  return gemm_t_launch<ACON, BCON, EPI, TM, TN, BK>(g, st);
}

// Tile choice: 64 x 64 tiles where 128 x 128 tiles would leave most CUs
// idle and the reduction is short (the hidden and first layers), else
// 128 x 128 with split-K, over 64-deep slices (32-deep when both operands
// are strided: their LDS scatter then measured faster).  (Wider 2 x 4 blocks
// per wave measured slower: at 268 registers one wave per SIMD cannot hide
// the LDS and memory latency.)
template <bool ACON, bool BCON, int EPI>
hipError_t gemm(GemmArgs g, float* part, hipStream_t st) {
  const long mid = (long)((g.M + 127) / 128) * ((g.N + 127) / 128);
  if (mid < kTargetBlocks / 4 && g.K <= 2048) return gemm_t<ACON, BCON, EPI, 1, 1, 32>(g, part, st);
  if (!ACON && !BCON) return gemm_t<ACON, BCON, EPI, 2, 2, 32>(g, part, st);
  // Linear outputs over many tiles: 32-deep slices, whose 40 KB of LDS and
  // (staged epilogue) 64 VGPRs let four workgroups share a CU; with fewer
  // tiles the deeper slices measured faster.
  if (EPI == EPI_FWD_LIN && ACON && BCON && mid >= 1024) return gemm_t<ACON, BCON, EPI, 2, 2, 32>(g, part, st);
  return gemm_t<ACON, BCON, EPI, 2, 2, 64>(g, part, st);
}


// ------------------------------------------------------------------------
// Least-squares fit of the network (pmdg_mlp_fit_linear).  The surrogate's
// target is linear in the embedded input columns when those are products of
// each PMUT's drive (cos / sin of its phase) with a basis in frequency, so a
// linear map of rank r fitted by least squares is a network whose hidden
// layers pass r signals through: the leading ones as pairs (gelu(z) -
// gelu(-z) = z exactly), the rest shifted by beta so that gelu(z + beta) is
// z + beta to within the BF16 rounding.  The large products run here on the
// GPU in FP32; the factorisations of the n_0 x n_0 matrices run on the host
// in FP64.
// ------------------------------------------------------------------------

// C[i][j] = alpha sum_k A(i, k) B(k, j) over FP32 operands with arbitrary
// strides: A(i, k) = A[i sai + k sak], B(k, j) = B[g(k) sbk + j sbj], g(k) =
// gidx[k] (row gather) or k.  64 x 64 tiles, 16-deep slices staged in LDS;
// each slice is loaded along whichever index has unit stride.
__global__ void __launch_bounds__(256) k_sgemm(int M, int N, int K, const float* __restrict__ A, long sai, long sak,
                                              const float* __restrict__ B, long sbk, long sbj,
                                              const int* __restrict__ gidx, float alpha, float* __restrict__ C,
                                              long ldc) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int t = threadIdx.x, tx = t % 16, ty = t / 16;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const bool a_k_fast = sak == 1 && sai != 1, b_k_fast = sbk == 1 && sbj != 1;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      const int ii = a_k_fast ? e / 16 : e % 64, kk = a_k_fast ? e % 16 : e / 64;
      const int i = i0 + ii, k = k0 + kk;
      As[kk][ii] = (i < M && k < K) ? A[(long)i * sai + (long)k * sak] : 0.f;
      const int jj = b_k_fast ? e / 16 : e % 64, kb = b_k_fast ? e % 16 : e / 64;
      const int j = j0 + jj, k2 = k0 + kb;
      float bv = 0.f;
      if (j < N && k2 < K) bv = B[(long)(gidx ? gidx[k2] : k2) * sbk + (long)j * sbj];
      Bs[kb][jj] = bv;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
    }
    __syncthreads();
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + ty * 4 + r, j = j0 + tx * 4 + c;
      if (i < M && j < N) C[(long)i * ldc + j] = alpha * acc[r][c];
    }
}

// X[r][c] = embed column c of u[idx[r]] (FP32, n_0 columns), Xs = X / (s a_r)
// with a_r the amplitude feature (or 1), s the output scale.
__global__ void k_embed_f32(const float* __restrict__ u, const int* __restrict__ idx, int nrows, int n, int nu, int n0,
                            const EmbCol* __restrict__ emb, int amp, float inv_scale, float* __restrict__ X,
                            float* __restrict__ Xs) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)n * n0) return;
  const int r = (int)(i / n0), c = (int)(i % n0);
  const long src = idx ? min(max(idx[r], 0), nrows - 1) : r;
  const EmbCol e = emb[c];
  float v = 0.f;
  if (e.src >= 0) {
    v = emb_factor(u[src * nu + e.src], e.op, e.shift, e.scale);
    if (e.src2 >= 0) v *= emb_factor(u[src * nu + e.src2], e.op2, e.shift2, e.scale2);
  }
  const float a = amp >= 0 ? u[src * nu + amp] : 1.0f;
  X[i] = v;
  Xs[i] = a != 0.f ? v * inv_scale / a : 0.f;
}

// sum over the fit rows of (t[idx[r]] / a_r)^2: one partial per workgroup
// (row r = blockIdx.x), summed on the host in a fixed order.
__global__ void __launch_bounds__(256) k_row_sq(const float* __restrict__ t, const float* __restrict__ u,
                                               const int* __restrict__ idx, int nrows, int nu, int amp, int nL,
                                               double* __restrict__ part) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  const long src = idx ? min(max(idx[r], 0), nrows - 1) : r;
  const float a = amp >= 0 ? u[src * nu + amp] : 1.0f;
  const float inv = a != 0.f ? 1.0f / a : 0.f;
  double s = 0;
  for (int j = threadIdx.x; j < nL; j += 256) {
    const double v = (double)(t[src * (long)nL + j] * inv);
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[r] = red[0];
}

// Output layer of the fitted network from the rank-r coefficients C [r][nL]:
// W[j][c] = +C[c][j] (c < P), -C[c - P][j] (P <= c < 2P), C[c - P][j]
// (2P <= c < P + r), 0 beyond; b[j] = -beta sum_{i >= P} C[i][j] (removes the
// shift of the singly passed signals).  W is [nL][ld] FP32 with its BF16 copy.
__global__ void k_fit_out_layer(const float* __restrict__ C, int r, int P, int nL, int width, int ld, float beta,
                                float* __restrict__ W, bf16_t* __restrict__ Wb, float* __restrict__ b) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)nL * ld) return;
  const int j = (int)(i / ld), c = (int)(i % ld);
  float v = 0.f;
  if (c < P) v = C[(long)c * nL + j];
  else if (c < 2 * P) v = -C[(long)(c - P) * nL + j];
  else if (c < P + r && c < width) v = C[(long)(c - P) * nL + j];
  W[i] = v;
  Wb[i] = f2bf(v);
  if (c == 0) {
    float acc = 0.f;
    for (int k = P; k < r; ++k) acc += C[(long)k * nL + j];
    b[j] = -beta * acc;
  }
}

// max |Z| over a block of columns [c0, c1) of Z [n][ld] (non-negative floats
// compare as their bit patterns)
__global__ void k_absmax_cols(const float* __restrict__ Z, long n, int ld, int c0, int c1, unsigned* __restrict__ out) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n * ld) return;
  const int c = (int)(i % ld);
  if (c < c0 || c >= c1) return;
  atomicMax(out, __float_as_uint(fabsf(Z[i])));
}

// per-row relative L2 error ||y_r - t[idx[r]]|| / ||t[idx[r]]||
__global__ void __launch_bounds__(256) k_row_relerr(const float* __restrict__ y, const float* __restrict__ t,
                                                   const int* __restrict__ idx, int nrows, int n,
                                                   float* __restrict__ err) {
  __shared__ double red[2][256];
  const int r = blockIdx.x;
  const long src = idx ? min(max(idx[r], 0), nrows - 1) : r;
  double se = 0, sn = 0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double tv = t[src * (long)n + j], d = (double)y[(long)r * n + j] - tv;
    se += d * d;
    sn += tv * tv;
  }
  red[0][threadIdx.x] = se;
  red[1][threadIdx.x] = sn;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) err[r] = red[1][0] > 0 ? (float)sqrt(red[0][0] / red[1][0]) : 0.f;
}

// dst[rows[i]] = src[i] for i < nr, rows of n floats
__global__ void k_scatter_rows(const float* __restrict__ src, const int* __restrict__ rows, int nr, int n,
                               float* __restrict__ dst) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)nr * n) return;
  const int r = (int)(i / n), c = (int)(i % n);
  dst[(long)rows[r] * n + c] = src[i];
}
}  // namespace

#define MCHK(call)                                                                                  \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return mfail(PMDG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct pmdg_mlp {
  int L = 0;                       // weight matrices
  std::vector<int> width;          // L + 1 widths
  std::vector<int> kin;            // padded input width of layer l
  int max_batch = 0;
  char* ws = nullptr;
  bool bound = false;
  bool have_z = false;             // last forward kept the normalised output
  int last_batch = 0;
  const int* last_idx = nullptr;
  int last_nrows = 0;
  int n_u = 0;                     // raw features per input row
  int amp_col = -1;                // raw feature the output is proportional to
  std::vector<EmbCol> emb;         // input map per network input column (kin[0])
  float out_scale = 1.f;
  // byte offsets into the workspace
  std::vector<size_t> oW, ob, oWb, omW, ovW, omb, ovb, odW, odb, oZ, oXb, odZ, odZb;
  size_t oRowErr = 0, oRowNorm = 0, oEmb = 0, oRowScale = 0, oPart = 0, bytes = 0;
  long nparams = 0;
  int adam_t = 0;
};

static size_t a256(size_t x) { return (x + 255) / 256 * 256; }

static void mlp_layout(pmdg_mlp* m) {
  const int L = m->L;
  const size_t B = m->max_batch;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = a256(o + bytes); return r; };
  for (auto* v : {&m->oW, &m->ob, &m->oWb, &m->omW, &m->ovW, &m->omb, &m->ovb, &m->odW, &m->odb, &m->oZ, &m->odZ,
                  &m->odZb})
    v->assign(L, 0);
  m->oXb.assign(L, 0);
  for (int l = 0; l < L; ++l) {
    const size_t nw = (size_t)m->width[l + 1] * m->kin[l], nb = m->width[l + 1];
    m->oW[l] = take(4 * nw); m->ob[l] = take(4 * nb); m->oWb[l] = take(2 * nw);
    m->omW[l] = take(4 * nw); m->ovW[l] = take(4 * nw); m->omb[l] = take(4 * nb); m->ovb[l] = take(4 * nb);
    m->odW[l] = take(4 * nw); m->odb[l] = take(4 * nb);
    m->oZ[l] = take(4 * B * m->width[l + 1]);
    m->odZ[l] = take(4 * B * m->width[l + 1]);
    m->odZb[l] = take(2 * B * m->width[l + 1]);
    m->oXb[l] = take(2 * B * m->kin[l]);
  }
  m->oRowErr = take(4 * B);
  m->oRowNorm = take(4 * B);
  m->oEmb = take(sizeof(EmbCol) * (size_t)m->kin[0]);
  m->oRowScale = take(4 * B);
  // split-K partial tiles, and the column-sum partials of the bias gradients
  int wmax = 0;
  for (int l = 1; l <= L; ++l) wmax = std::max(wmax, m->width[l]);
  const size_t colpart = (size_t)((B + kColChunk - 1) / kColChunk) * wmax;
  m->oPart = take(4 * std::max(kPartFloats, colpart));
  m->bytes = o;
}

template <typename T>
static T* at(pmdg_mlp* m, size_t off) { return (T*)(m->ws + off); }

// ---- host FP64 linear algebra for the least-squares fit (n of a few hundred)

// Cholesky factor L (lower, row-major) of the SPD matrix A [n][n]; false if
// a pivot is not positive.
static bool chol_lower(int n, const std::vector<double>& A, std::vector<double>& L) {
  L.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0)) return false;
    const double ljj = std::sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / ljj;
    }
  }
  return true;
}

// B <- L^{-1} B for B [n][m] (forward substitution, column by column of B)
static void solve_lower(int n, int m, const std::vector<double>& L, std::vector<double>& B) {
  for (int i = 0; i < n; ++i) {
    double* bi = &B[(size_t)i * m];
    for (int k = 0; k < i; ++k) {
      const double l = L[(size_t)i * n + k];
      if (l == 0) continue;
      const double* bk = &B[(size_t)k * m];
      for (int j = 0; j < m; ++j) bi[j] -= l * bk[j];
    }
    const double inv = 1.0 / L[(size_t)i * n + i];
    for (int j = 0; j < m; ++j) bi[j] *= inv;
  }
}

// B <- L^{-T} B for B [n][m] (back substitution with the transpose)
static void solve_lower_t(int n, int m, const std::vector<double>& L, std::vector<double>& B) {
  for (int i = n - 1; i >= 0; --i) {
    double* bi = &B[(size_t)i * m];
    for (int k = i + 1; k < n; ++k) {
      const double l = L[(size_t)k * n + i];
      if (l == 0) continue;
      const double* bk = &B[(size_t)k * m];
      for (int j = 0; j < m; ++j) bi[j] -= l * bk[j];
    }
    const double inv = 1.0 / L[(size_t)i * n + i];
    for (int j = 0; j < m; ++j) bi[j] *= inv;
  }
}

// Eigen-decomposition of the symmetric A [n][n] (destroyed): eigenvalues w in
// descending order, eigenvectors as the columns of V [n][n].  Householder
// reduction to tridiagonal form with the reflections accumulated, then the
// implicit QL iteration with Wilkinson-type shifts (Golub and Van Loan,
// Matrix Computations, Sec. 8.3).  false if an eigenvalue does not converge.
static bool sym_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& V) {
  std::vector<double> d(n), e(n, 0.0);
  // Vt holds the accumulated transformation by rows (row i = column i of
  // the eigenvector matrix), so every update runs along contiguous rows
  std::vector<double> Vt((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Vt[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), sv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    double xn = 0;
    for (int i = 0; i < m; ++i) xn += A[(size_t)(k + 1 + i) * n + k] * A[(size_t)(k + 1 + i) * n + k];
    xn = std::sqrt(xn);
    if (xn == 0) { e[k] = 0; continue; }
    const double x0 = A[(size_t)(k + 1) * n + k];
    const double alpha = x0 >= 0 ? -xn : xn;
    double vn2 = 0;
    for (int i = 0; i < m; ++i) {
      v[i] = A[(size_t)(k + 1 + i) * n + k] - (i == 0 ? alpha : 0.0);
      vn2 += v[i] * v[i];
    }
    if (vn2 == 0) { e[k] = x0; continue; }
    const double beta = 2.0 / vn2;
    // p = beta A22 v, K = beta/2 v.p, w = p - K v; A22 -= v w^T + w v^T
    double vp = 0;
    for (int i = 0; i < m; ++i) {
      const double* ai = &A[(size_t)(k + 1 + i) * n + k + 1];
      double s = 0;
      for (int j = 0; j < m; ++j) s += ai[j] * v[j];
      p[i] = beta * s;
      vp += v[i] * p[i];
    }
    const double K = 0.5 * beta * vp;
    for (int i = 0; i < m; ++i) p[i] -= K * v[i];
    for (int i = 0; i < m; ++i) {
      double* ai = &A[(size_t)(k + 1 + i) * n + k + 1];
      for (int j = 0; j < m; ++j) ai[j] -= v[i] * p[j] + p[i] * v[j];
    }
    for (int i = 0; i < m; ++i) {
      A[(size_t)(k + 1 + i) * n + k] = i == 0 ? alpha : 0.0;
      A[(size_t)k * n + k + 1 + i] = i == 0 ? alpha : 0.0;
    }
    e[k] = alpha;
    // rows k+1.. of Vt: Vt_j -= beta v_j sum_i v_i Vt_i
    std::fill(sv.begin(), sv.end(), 0.0);
    for (int j = 0; j < m; ++j) {
      const double* vj = &Vt[(size_t)(k + 1 + j) * n];
      for (int r = 0; r < n; ++r) sv[r] += v[j] * vj[r];
    }
    for (int j = 0; j < m; ++j) {
      double* vj = &Vt[(size_t)(k + 1 + j) * n];
      const double f = beta * v[j];
      for (int r = 0; r < n; ++r) vj[r] -= f * sv[r];
    }
  }
  if (n >= 2) e[n - 2] = A[(size_t)(n - 1) * n + n - 2];
  e[n - 1] = 0;
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  // implicit QL on (d, e): e[i] couples i and i + 1
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < n - 1; ++m)
        if (std::fabs(e[m]) <= eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
      if (m == l) break;
      if (iter == 100) return false;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1, c = 1, pp = 0;
      int i = m - 1;
      bool early = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0) {  // split: d[i+1] converged early
          d[i + 1] -= pp;
          e[m] = 0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        double* va = &Vt[(size_t)i * n];
        double* vb = &Vt[(size_t)(i + 1) * n];
        for (int k = 0; k < n; ++k) {
          const double fv = vb[k];
          vb[k] = s * va[k] + c * fv;
          va[k] = c * va[k] - s * fv;
        }
      }
      if (early) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0;
    }
  }
  // descending order
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
  w.resize(n);
  V.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    w[c] = d[ord[c]];
    const double* src = &Vt[(size_t)ord[c] * n];
    for (int r = 0; r < n; ++r) V[(size_t)r * n + c] = src[r];
  }
  return true;
}

// Device buffers of the least-squares fit (byte offsets into the caller's
// fit workspace).
struct FitLayout {
  size_t X, Xs, G, Bt, S, M, C, Z, part, zmax, bytes;
};

static FitLayout fit_layout(const pmdg_mlp* m, int n, int rank) {
  const size_t n0 = m->width[0], nL = m->width[m->L];
  FitLayout f;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = a256(o + bytes); return r; };
  f.X = take(4 * (size_t)n * n0);
  f.Xs = take(4 * (size_t)n * n0);
  f.G = take(4 * n0 * n0);
  f.Bt = take(4 * n0 * nL);
  f.S = take(4 * n0 * n0);
  f.M = take(4 * n0 * (size_t)rank);
  f.C = take(4 * (size_t)rank * nL);
  f.Z = take(4 * (size_t)n * rank);
  f.part = take(8 * (size_t)n);
  f.zmax = take(4);
  f.bytes = o;
  return f;
}

// out_scale = RMS over rows idx of t / a (a the amplitude feature or 1);
// part: n doubles of device scratch
static pmdg_status target_scale(pmdg_mlp* m, const float* u, const float* t, const int* idx, int nrows, int n,
                                double* part, hipStream_t st) {
  const int nL = m->width[m->L];
  hipLaunchKernelGGL(k_row_sq, dim3(n), dim3(256), 0, st, t, u, idx, nrows, m->n_u, m->amp_col, nL, part);
  MCHK(hipGetLastError());
  std::vector<double> hp(n);
  MCHK(hipMemcpyAsync(hp.data(), part, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
  MCHK(hipStreamSynchronize(st));
  double ss = 0;
  for (int r = 0; r < n; ++r) ss += hp[r];
  const double oscale = std::sqrt(ss / ((double)n * nL));
  if (!(oscale > 0) || !std::isfinite(oscale)) return mfail(PMDG_EINVAL, "targets are zero or not finite");
  m->out_scale = (float)oscale;
  return PMDG_OK;
}

static hipError_t sgemm(int M, int N, int K, const float* A, long sai, long sak, const float* B, long sbk, long sbj,
                        const int* gidx, float alpha, float* C, long ldc, hipStream_t st) {
  hipLaunchKernelGGL(k_sgemm, dim3((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64)), dim3(256), 0, st, M, N, K,
                     A, sai, sak, B, sbk, sbj, gidx, alpha, C, ldc);
  return hipGetLastError();
}

static pmdg_status check_batch(pmdg_mlp* m, const int* idx, int nrows, int B) {
  if (!m->bound) return mfail(PMDG_ESTATE, "model not bound");
  if (B < 8 || B > m->max_batch || B % 8) return mfail(PMDG_EINVAL, "batch must be a multiple of 8 in [8, max_batch]");
  if (nrows < 1 || (!idx && nrows < B)) return mfail(PMDG_EINVAL, "nrows must be >= 1, and >= B without idx");
  return PMDG_OK;
}

static pmdg_status mlp_forward_dev(pmdg_mlp* m, const float* u, const int* idx, int nrows, int B, float* y,
                                   hipStream_t st) {
  const int L = m->L;
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)nblk((long)B * m->kin[0], 256)), dim3(256), 0, st, u, idx, nrows, B,
                     m->n_u, m->kin[0], at<EmbCol>(m, m->oEmb), m->amp_col, at<bf16_t>(m, m->oXb[0]),
                     at<float>(m, m->oRowScale));
  MCHK(hipGetLastError());
  for (int l = 0; l < L; ++l) {
    GemmArgs g;
    memset(&g, 0, sizeof(g));
    g.M = B; g.N = m->width[l + 1]; g.K = m->kin[l];
    g.A = at<bf16_t>(m, m->oXb[l]); g.lda = m->kin[l];
    g.B = at<bf16_t>(m, m->oWb[l]); g.ldb = m->kin[l];
    g.bias = at<float>(m, m->ob[l]);
    g.Cf = at<float>(m, m->oZ[l]); g.ldc = m->width[l + 1];
    if (l < L - 1) {
      g.Cb = at<bf16_t>(m, m->oXb[l + 1]);
      MCHK((gemm<true, true, EPI_FWD_GELU>(g, at<float>(m, m->oPart), st)));
    } else {
      g.Y = y;
      g.out_scale = m->out_scale;
      g.rowscale = at<float>(m, m->oRowScale);
      MCHK((gemm<true, true, EPI_FWD_LIN>(g, at<float>(m, m->oPart), st)));
    }
  }
  m->have_z = (y == nullptr);
  m->last_batch = B;
  m->last_idx = idx;
  m->last_nrows = nrows;
  return PMDG_OK;
}

static pmdg_status mlp_backward_dev(pmdg_mlp* m, const float* t, const int* idx, int nrows, int B, hipStream_t st) {
  const int L = m->L, nout = m->width[L];
  hipLaunchKernelGGL(k_loss, dim3(B), dim3(256), 0, st, at<float>(m, m->oZ[L - 1]), t, idx, nrows, B, nout,
                     1.0f / m->out_scale, at<float>(m, m->oRowScale), at<float>(m, m->odZ[L - 1]),
                     at<bf16_t>(m, m->odZb[L - 1]),
                     at<float>(m, m->oRowErr), at<float>(m, m->oRowNorm));
  MCHK(hipGetLastError());
  for (int l = L - 1; l >= 0; --l) {
    const int n = m->width[l + 1], k = m->kin[l];
    {  // dW_l [n][k] = dz_l^T x_l
      GemmArgs g;
      memset(&g, 0, sizeof(g));
      g.M = n; g.N = k; g.K = B;
      g.A = at<bf16_t>(m, m->odZb[l]); g.lda = n;
      g.B = at<bf16_t>(m, m->oXb[l]); g.ldb = k;
      g.Cf = at<float>(m, m->odW[l]); g.ldc = k;
      MCHK((gemm<false, false, EPI_DW>(g, at<float>(m, m->oPart), st)));
    }
    {
      const int nchunk = (B + kColChunk - 1) / kColChunk;
      hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)nblk(n, 64), nchunk), dim3(256), 0, st,
                         at<float>(m, m->odZ[l]), B, n, at<float>(m, m->oPart));
      MCHK(hipGetLastError());
      hipLaunchKernelGGL(k_colsum_fin, dim3((unsigned)nblk(n, 256)), dim3(256), 0, st, at<float>(m, m->oPart), nchunk,
                         n, at<float>(m, m->odb[l]));
      MCHK(hipGetLastError());
    }
    if (l > 0) {  // dz_{l-1} [B][width_l] = (dz_l W_l) * gelu'(z_{l-1})
      GemmArgs g;
      memset(&g, 0, sizeof(g));
      g.M = B; g.N = m->width[l]; g.K = n;
      g.A = at<bf16_t>(m, m->odZb[l]); g.lda = n;
      g.B = at<bf16_t>(m, m->oWb[l]); g.ldb = k;
      g.Cf = at<float>(m, m->odZ[l - 1]); g.Cb = at<bf16_t>(m, m->odZb[l - 1]); g.ldc = m->width[l];
      g.Zprev = at<float>(m, m->oZ[l - 1]);
      MCHK((gemm<true, false, EPI_DX_GELU>(g, at<float>(m, m->oPart), st)));
    }
  }
  return PMDG_OK;
}

static pmdg_status copy_out(pmdg_mlp* m, const std::vector<size_t>& oW, const std::vector<size_t>& ob, float* host) {
  float* p = host;
  for (int l = 0; l < m->L; ++l) {
    const int no = m->width[l + 1], ni = m->width[l], kp = m->kin[l];
    std::vector<float> w((size_t)no * kp);
    MCHK(hipMemcpy(w.data(), at<float>(m, oW[l]), w.size() * 4, hipMemcpyDeviceToHost));
    for (int r = 0; r < no; ++r)
      for (int c = 0; c < ni; ++c) p[(size_t)r * ni + c] = w[(size_t)r * kp + c];
    p += (size_t)no * ni;
    MCHK(hipMemcpy(p, at<float>(m, ob[l]), (size_t)no * 4, hipMemcpyDeviceToHost));
    p += no;
  }
  return PMDG_OK;
}

extern "C" {

pmdg_status pmdg_mlp_create(int nlayers, const int* widths, pmdg_mlp** out) {
  if (!out) return mfail(PMDG_EINVAL, "out is NULL");
  *out = nullptr;
  if (nlayers < 1 || nlayers > 16 || !widths) return mfail(PMDG_EINVAL, "nlayers must be in [1, 16]");
  for (int l = 0; l <= nlayers; ++l)
    if (widths[l] < 1 || widths[l] > (1 << 20)) return mfail(PMDG_EINVAL, "widths must be in [1, 2^20]");
  for (int l = 1; l <= nlayers; ++l)
    if (widths[l] % 8) return mfail(PMDG_EINVAL, "hidden and output widths must be multiples of 8");
  // a hidden layer's activations are the next layer's input rows, whose
  // leading dimension is the input width rounded up to 32
  for (int l = 1; l < nlayers; ++l)
    if (widths[l] % 32) return mfail(PMDG_EINVAL, "hidden widths must be multiples of 32");
  pmdg_mlp* m = new (std::nothrow) pmdg_mlp();
  if (!m) return mfail(PMDG_ENOMEM, "out of host memory");
  m->L = nlayers;
  m->width.assign(widths, widths + nlayers + 1);
  m->kin.resize(nlayers);
  for (int l = 0; l < nlayers; ++l) m->kin[l] = (m->width[l] + 31) / 32 * 32;
  for (int l = 0; l < nlayers; ++l) m->nparams += (long)m->width[l + 1] * (m->width[l] + 1);
  m->n_u = m->width[0];
  m->emb.assign(m->kin[0], EmbCol{-1, 0, 0.f, 1.f, -1, 0, 0.f, 1.f});
  for (int c = 0; c < m->width[0]; ++c) m->emb[c].src = c;
  *out = m;
  return PMDG_OK;
}

pmdg_status pmdg_mlp_num_params(pmdg_mlp* m, long* n) {
  if (!m || !n) return mfail(PMDG_EINVAL, "NULL argument");
  *n = m->nparams;
  return PMDG_OK;
}

pmdg_status pmdg_mlp_workspace_size(pmdg_mlp* m, int max_batch, size_t* bytes) {
  if (!m || !bytes) return mfail(PMDG_EINVAL, "NULL argument");
  if (m->bound) return mfail(PMDG_ESTATE, "already bound");
  if (max_batch < 8 || max_batch % 8 || max_batch > (1 << 16))
    return mfail(PMDG_EINVAL, "max_batch must be a multiple of 8 in [8, 65536]");
  m->max_batch = max_batch;
  mlp_layout(m);
  *bytes = m->bytes;
  return PMDG_OK;
}

pmdg_status pmdg_mlp_bind(pmdg_mlp* m, void* dev, size_t bytes, void* stream) {
  if (!m) return mfail(PMDG_EINVAL, "NULL model");
  if (m->bound) return mfail(PMDG_ESTATE, "already bound");
  if (m->max_batch == 0) return mfail(PMDG_ESTATE, "call pmdg_mlp_workspace_size first");
  if (!dev || ((uintptr_t)dev & 255)) return mfail(PMDG_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < m->bytes) return mfail(PMDG_ENOMEM, "workspace too small: need " + std::to_string(m->bytes));
  hipStream_t st = (hipStream_t)stream;
  m->ws = (char*)dev;
  MCHK(hipMemsetAsync(m->ws, 0, m->bytes, st));
  MCHK(hipMemcpyAsync(at<EmbCol>(m, m->oEmb), m->emb.data(), sizeof(EmbCol) * m->emb.size(), hipMemcpyHostToDevice,
                      st));
  MCHK(hipStreamSynchronize(st));
  m->bound = true;
  m->adam_t = 0;
  return PMDG_OK;
}

pmdg_status pmdg_mlp_set_io_map(pmdg_mlp* m, int n_u, int ncols, const int* src, const int* op, const float* shift,
                                const float* scale, int amp_col, float out_scale, void* stream) {
  if (!m || !src || !op || !shift || !scale) return mfail(PMDG_EINVAL, "NULL argument");
  if (n_u < 1 || n_u > (1 << 20)) return mfail(PMDG_EINVAL, "n_u out of range");
  if (ncols != m->width[0]) return mfail(PMDG_EINVAL, "ncols must equal widths[0] = " + std::to_string(m->width[0]));
  if (!(out_scale > 0.f) || !std::isfinite(out_scale)) return mfail(PMDG_EINVAL, "out_scale must be finite and > 0");
  if (amp_col < -1 || amp_col >= n_u) return mfail(PMDG_EINVAL, "amp_col must be -1 or a feature index");
  std::vector<EmbCol> emb(m->kin[0], EmbCol{-1, 0, 0.f, 1.f, -1, 0, 0.f, 1.f});
  for (int c = 0; c < ncols; ++c) {
    if (src[c] < 0 || src[c] >= n_u) return mfail(PMDG_EINVAL, "src must index a raw feature");
    if (op[c] < 0 || op[c] > 2) return mfail(PMDG_EINVAL, "op must be 0 (affine), 1 (cos) or 2 (sin)");
    if (!std::isfinite(shift[c]) || !std::isfinite(scale[c])) return mfail(PMDG_EINVAL, "non-finite input map");
    emb[c] = EmbCol{src[c], op[c], shift[c], scale[c], -1, 0, 0.f, 1.f};
  }
  m->emb = emb;
  m->n_u = n_u;
  m->amp_col = amp_col;
  m->out_scale = out_scale;
  if (m->bound) {
    hipStream_t st = (hipStream_t)stream;
    MCHK(hipMemcpyAsync(at<EmbCol>(m, m->oEmb), m->emb.data(), sizeof(EmbCol) * m->emb.size(),
                        hipMemcpyHostToDevice, st));
    MCHK(hipStreamSynchronize(st));
  }
  return PMDG_OK;
}

pmdg_status pmdg_mlp_set_io_factors(pmdg_mlp* m, int ncols, const int* src2, const int* op2, const float* shift2,
                                    const float* scale2, void* stream) {
  if (!m || !src2 || !op2 || !shift2 || !scale2) return mfail(PMDG_EINVAL, "NULL argument");
  if (ncols != m->width[0]) return mfail(PMDG_EINVAL, "ncols must equal widths[0] = " + std::to_string(m->width[0]));
  if ((int)m->emb.size() != m->kin[0]) return mfail(PMDG_ESTATE, "set the input map first");
  std::vector<EmbCol> emb = m->emb;
  for (int c = 0; c < ncols; ++c) {
    if (src2[c] < -1 || src2[c] >= m->n_u) return mfail(PMDG_EINVAL, "src2 must be -1 or index a raw feature");
    if (op2[c] < 0 || op2[c] > 2) return mfail(PMDG_EINVAL, "op2 must be 0 (affine), 1 (cos) or 2 (sin)");
    if (!std::isfinite(shift2[c]) || !std::isfinite(scale2[c])) return mfail(PMDG_EINVAL, "non-finite input map");
    emb[c].src2 = src2[c];
    emb[c].op2 = op2[c];
    emb[c].shift2 = shift2[c];
    emb[c].scale2 = scale2[c];
  }
  m->emb = emb;
  if (m->bound) {
    hipStream_t st = (hipStream_t)stream;
    MCHK(hipMemcpyAsync(at<EmbCol>(m, m->oEmb), m->emb.data(), sizeof(EmbCol) * m->emb.size(),
                        hipMemcpyHostToDevice, st));
    MCHK(hipStreamSynchronize(st));
  }
  return PMDG_OK;
}

pmdg_status pmdg_mlp_set_params(pmdg_mlp* m, const float* host, void* stream) {
  if (!m || !host) return mfail(PMDG_EINVAL, "NULL argument");
  if (!m->bound) return mfail(PMDG_ESTATE, "model not bound");
  hipStream_t st = (hipStream_t)stream;
  MCHK(hipStreamSynchronize(st));
  const float* p = host;
  for (int l = 0; l < m->L; ++l) {
    const int no = m->width[l + 1], ni = m->width[l], kp = m->kin[l];
    std::vector<float> w((size_t)no * kp, 0.f);
    for (int r = 0; r < no; ++r)
      for (int c = 0; c < ni; ++c) w[(size_t)r * kp + c] = p[(size_t)r * ni + c];
    p += (size_t)no * ni;
    MCHK(hipMemcpy(at<float>(m, m->oW[l]), w.data(), w.size() * 4, hipMemcpyHostToDevice));
    MCHK(hipMemcpy(at<float>(m, m->ob[l]), p, (size_t)no * 4, hipMemcpyHostToDevice));
    p += no;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)nblk((long)w.size(), 256)), dim3(256), 0, st,
                       at<float>(m, m->oW[l]), at<bf16_t>(m, m->oWb[l]), (long)w.size());
    MCHK(hipGetLastError());
  }
  // fresh optimiser state
  for (int l = 0; l < m->L; ++l) {
    const size_t nw = (size_t)m->width[l + 1] * m->kin[l], nb = m->width[l + 1];
    MCHK(hipMemsetAsync(at<float>(m, m->omW[l]), 0, 4 * nw, st));
    MCHK(hipMemsetAsync(at<float>(m, m->ovW[l]), 0, 4 * nw, st));
    MCHK(hipMemsetAsync(at<float>(m, m->omb[l]), 0, 4 * nb, st));
    MCHK(hipMemsetAsync(at<float>(m, m->ovb[l]), 0, 4 * nb, st));
  }
  m->adam_t = 0;
  MCHK(hipStreamSynchronize(st));
  return PMDG_OK;
}

pmdg_status pmdg_mlp_get_params(pmdg_mlp* m, float* host, void* stream) {
  if (!m || !host) return mfail(PMDG_EINVAL, "NULL argument");
  if (!m->bound) return mfail(PMDG_ESTATE, "model not bound");
  MCHK(hipStreamSynchronize((hipStream_t)stream));
  return copy_out(m, m->oW, m->ob, host);
}

pmdg_status pmdg_mlp_get_grads(pmdg_mlp* m, float* host, void* stream) {
  if (!m || !host) return mfail(PMDG_EINVAL, "NULL argument");
  if (!m->bound) return mfail(PMDG_ESTATE, "model not bound");
  MCHK(hipStreamSynchronize((hipStream_t)stream));
  return copy_out(m, m->odW, m->odb, host);
}

pmdg_status pmdg_mlp_forward(pmdg_mlp* m, const float* u, const int* idx, int nrows, int B, float* y, void* stream) {
  if (!m || !u) return mfail(PMDG_EINVAL, "NULL argument");
  pmdg_status r = check_batch(m, idx, nrows, B);
  if (r) return r;
  return mlp_forward_dev(m, u, idx, nrows, B, y, (hipStream_t)stream);
}

pmdg_status pmdg_mlp_backward(pmdg_mlp* m, const float* t, int B, float* rowerr, float* rownorm, void* stream) {
  if (!m || !t) return mfail(PMDG_EINVAL, "NULL argument");
  pmdg_status r = check_batch(m, m->last_idx, m->last_nrows, B);
  if (r) return r;
  if ((uintptr_t)t & 15) return mfail(PMDG_EINVAL, "targets must be 16-byte aligned");
  if (!m->have_z || m->last_batch != B)
    return mfail(PMDG_ESTATE, "backward needs a preceding training forward (y == NULL) of the same batch");
  hipStream_t st = (hipStream_t)stream;
  if ((r = mlp_backward_dev(m, t, m->last_idx, m->last_nrows, B, st))) return r;
  if (rowerr) MCHK(hipMemcpyAsync(rowerr, at<float>(m, m->oRowErr), (size_t)B * 4, hipMemcpyDeviceToDevice, st));
  if (rownorm) MCHK(hipMemcpyAsync(rownorm, at<float>(m, m->oRowNorm), (size_t)B * 4, hipMemcpyDeviceToDevice, st));
  return PMDG_OK;
}

pmdg_status pmdg_mlp_adam(pmdg_mlp* m, float lr, float b1, float b2, float eps, void* stream) {
  if (!m) return mfail(PMDG_EINVAL, "NULL model");
  if (!m->bound) return mfail(PMDG_ESTATE, "model not bound");
  if (!(lr >= 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return mfail(PMDG_EINVAL, "need lr >= 0, 0 <= b1, b2 < 1, eps > 0");
  hipStream_t st = (hipStream_t)stream;
  m->adam_t += 1;
  const float c1 = (float)(1.0 - std::pow((double)b1, m->adam_t));
  const float c2 = (float)(1.0 - std::pow((double)b2, m->adam_t));
  for (int l = 0; l < m->L; ++l) {
    const long nw = (long)m->width[l + 1] * m->kin[l], nb = m->width[l + 1];
    hipLaunchKernelGGL(k_adam, dim3((unsigned)nblk(nw / 4, 256)), dim3(256), 0, st, at<float>(m, m->oW[l]),
                       at<float>(m, m->odW[l]), at<float>(m, m->omW[l]), at<float>(m, m->ovW[l]),
                       at<bf16_t>(m, m->oWb[l]), nw, lr, b1, b2, eps, c1, c2);
    MCHK(hipGetLastError());
    hipLaunchKernelGGL(k_adam, dim3((unsigned)nblk(nb / 4, 256)), dim3(256), 0, st, at<float>(m, m->ob[l]),
                       at<float>(m, m->odb[l]), at<float>(m, m->omb[l]), at<float>(m, m->ovb[l]), (bf16_t*)nullptr,
                       nb, lr, b1, b2, eps, c1, c2);
    MCHK(hipGetLastError());
  }
  return PMDG_OK;
}

pmdg_status pmdg_mlp_train_step(pmdg_mlp* m, const float* u, const float* t, const int* idx, int nrows, int B,
                                float lr, float b1, float b2, float eps, float* rowerr, float* rownorm, void* stream) {
  if (!m || !u || !t) return mfail(PMDG_EINVAL, "NULL argument");
  pmdg_status r = check_batch(m, idx, nrows, B);
  if (r) return r;
  hipStream_t st = (hipStream_t)stream;
  if ((r = mlp_forward_dev(m, u, idx, nrows, B, nullptr, st))) return r;
  if ((r = pmdg_mlp_backward(m, t, B, rowerr, rownorm, stream))) return r;
  return pmdg_mlp_adam(m, lr, b1, b2, eps, stream);
}

pmdg_status pmdg_mlp_pair_combine(const float* a, const float* b, int B, int n, float* mean, float* spread,
                                  void* stream) {
  if (!a || !b || !mean || !spread) return mfail(PMDG_EINVAL, "NULL argument");
  if (B < 1 || n < 4 || n % 4) return mfail(PMDG_EINVAL, "need B >= 1 and n a positive multiple of 4");
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)mean) & 15) return mfail(PMDG_EINVAL, "arrays must be 16-byte aligned");
  hipLaunchKernelGGL(k_pair_combine, dim3(B), dim3(256), 0, (hipStream_t)stream, a, b, n, mean, spread);
  MCHK(hipGetLastError());
  return PMDG_OK;
}

pmdg_status pmdg_mlp_fit_linear_workspace(pmdg_mlp* m, int n, int rank, size_t* bytes) {
  if (!m || !bytes) return mfail(PMDG_EINVAL, "NULL argument");
  if (n < 1 || rank < 1) return mfail(PMDG_EINVAL, "n and rank must be >= 1");
  *bytes = fit_layout(m, n, rank).bytes;
  return PMDG_OK;
}

pmdg_status pmdg_mlp_fit_linear(pmdg_mlp* m, const float* u, const float* t, const int* idx, int nrows, int n,
                                int npairs, int rank, float ridge, void* work, size_t work_bytes, void* stream) {
  if (!m || !u || !t || !work) return mfail(PMDG_EINVAL, "NULL argument");
  if (!m->bound) return mfail(PMDG_ESTATE, "model not bound");
  if ((int)m->emb.size() != m->kin[0]) return mfail(PMDG_ESTATE, "set the input map first");
  const int L = m->L, n0 = m->width[0], nL = m->width[L];
  if (L < 2) return mfail(PMDG_EINVAL, "the fit needs at least one hidden layer");
  const int Wd = m->width[1];
  for (int l = 1; l < L; ++l)
    if (m->width[l] != Wd) return mfail(PMDG_EINVAL, "the fit needs hidden layers of one width");
  if (n < 1 || nrows < 1 || (!idx && nrows < n)) return mfail(PMDG_EINVAL, "bad row counts");
  if (npairs < 0 || rank < 1 || npairs > rank || npairs + rank > Wd || rank > n0 || rank > n)
    return mfail(PMDG_EINVAL, "need 0 <= npairs <= rank, npairs + rank <= hidden width, rank <= n_0 and rank <= n");
  if (!(ridge >= 0.f) || !std::isfinite(ridge)) return mfail(PMDG_EINVAL, "ridge must be finite and >= 0");
  const FitLayout f = fit_layout(m, n, rank);
  if (((uintptr_t)work & 255) || work_bytes < f.bytes)
    return mfail(PMDG_ENOMEM, "fit workspace must be 256-byte aligned and hold " + std::to_string(f.bytes) + " bytes");
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)work;
  float *X = (float*)(w + f.X), *Xs = (float*)(w + f.Xs), *G = (float*)(w + f.G), *Bt = (float*)(w + f.Bt);
  float *S = (float*)(w + f.S), *Md = (float*)(w + f.M), *C = (float*)(w + f.C), *Z = (float*)(w + f.Z);
  double* part = (double*)(w + f.part);
  unsigned* zmax = (unsigned*)(w + f.zmax);
  // output scale: RMS of the amplitude-normalised targets over the fit rows
  pmdg_status rs = target_scale(m, u, t, idx, nrows, n, part, st);
  if (rs) return rs;
  const double oscale = m->out_scale;
  // X, Xs = X / (out_scale a); G = X^T X; Bt = Xs^T t; S = Bt Bt^T
  hipLaunchKernelGGL(k_embed_f32, dim3((unsigned)nblk((long)n * n0, 256)), dim3(256), 0, st, u, idx, nrows, n,
                     m->n_u, n0, at<EmbCol>(m, m->oEmb), m->amp_col, (float)(1.0 / oscale), X, Xs);
  MCHK(hipGetLastError());
  MCHK(sgemm(n0, n0, n, X, 1, n0, X, n0, 1, nullptr, 1.f, G, n0, st));
  MCHK(sgemm(n0, nL, n, Xs, 1, n0, t, nL, 1, idx, 1.f, Bt, nL, st));
  MCHK(sgemm(n0, n0, nL, Bt, nL, 1, Bt, 1, nL, nullptr, 1.f, S, n0, st));
  std::vector<float> hG((size_t)n0 * n0), hS((size_t)n0 * n0);
  MCHK(hipMemcpyAsync(hG.data(), G, 4 * hG.size(), hipMemcpyDeviceToHost, st));
  MCHK(hipMemcpyAsync(hS.data(), S, 4 * hS.size(), hipMemcpyDeviceToHost, st));
  MCHK(hipStreamSynchronize(st));
  // host, FP64: G + ridge = L L^T; H = L^{-1} S L^{-T} = V diag(w) V^T;
  // M0 = L^{-T} V_r gives x M0 orthonormal over the fit rows and
  // x M0 M0^T Bt the rank-r least-squares predictor
  std::vector<double> Gd(hG.begin(), hG.end()), H(hS.begin(), hS.end()), Lc;
  double tr = 0;
  for (int i = 0; i < n0; ++i) tr += Gd[(size_t)i * n0 + i];
  const double lam = std::max((double)ridge * tr / n0, 1e-12 * tr / n0);
  for (int i = 0; i < n0; ++i) Gd[(size_t)i * n0 + i] += lam;
  if (!chol_lower(n0, Gd, Lc)) return mfail(PMDG_EINVAL, "the embedded columns are linearly dependent on the fit rows");
  solve_lower(n0, n0, Lc, H);  // L^{-1} S
  for (int i = 0; i < n0; ++i)  // transpose in place: (L^{-1} S)^T = S L^{-T}
    for (int j = i + 1; j < n0; ++j) std::swap(H[(size_t)i * n0 + j], H[(size_t)j * n0 + i]);
  solve_lower(n0, n0, Lc, H);  // L^{-1} S L^{-T}
  for (int i = 0; i < n0; ++i)
    for (int j = i + 1; j < n0; ++j) {
      const double a = 0.5 * (H[(size_t)i * n0 + j] + H[(size_t)j * n0 + i]);
      H[(size_t)i * n0 + j] = H[(size_t)j * n0 + i] = a;
    }
  std::vector<double> ev, V;
  if (!sym_eig(n0, H, ev, V)) return mfail(PMDG_EINVAL, "eigenvalue iteration did not converge");
  std::vector<double> M0((size_t)n0 * rank);
  for (int i = 0; i < n0; ++i)
    for (int c = 0; c < rank; ++c) M0[(size_t)i * rank + c] = V[(size_t)i * n0 + c];
  solve_lower_t(n0, rank, Lc, M0);
  // z = x M with M = alpha M0 has unit RMS per column over the fit rows
  const double alpha = std::sqrt((double)n);
  std::vector<float> hM((size_t)n0 * rank);
  for (size_t i = 0; i < hM.size(); ++i) hM[i] = (float)(alpha * M0[i]);
  MCHK(hipMemcpyAsync(Md, hM.data(), 4 * hM.size(), hipMemcpyHostToDevice, st));
  // C = M^T Bt / alpha^2 (so that z C = x M0 M0^T Bt); Z = X M
  MCHK(sgemm(rank, nL, n0, Md, 1, rank, Bt, nL, 1, nullptr, (float)(1.0 / (alpha * alpha)), C, nL, st));
  MCHK(sgemm(n, rank, n0, X, n0, 1, Md, rank, 1, nullptr, 1.f, Z, rank, st));
  MCHK(hipMemsetAsync(zmax, 0, 4, st));
  hipLaunchKernelGGL(k_absmax_cols, dim3((unsigned)nblk((long)n * rank, 256)), dim3(256), 0, st, Z, (long)n, rank,
                     npairs, rank, zmax);
  MCHK(hipGetLastError());
  unsigned zbits = 0;
  MCHK(hipMemcpyAsync(&zbits, zmax, 4, hipMemcpyDeviceToHost, st));
  MCHK(hipStreamSynchronize(st));
  float zm;
  memcpy(&zm, &zbits, 4);
  // shift of the singly passed signals: gelu(u) = u Phi(u) is u to within
  // 1.4e-3 u for u >= 3, with a 25% margin on the largest |z| of the fit rows
  const float beta = npairs < rank ? 1.25f * zm + 3.0f : 0.f;
  const int P = npairs, ns = rank - npairs;
  // first layer: rows [M_c; -M_c] for the pairs, M_c + beta for the singles
  {
    const int kp = m->kin[0];
    std::vector<float> W((size_t)Wd * kp, 0.f), b(Wd, 0.f);
    for (int c = 0; c < P; ++c)
      for (int i = 0; i < n0; ++i) {
        W[(size_t)c * kp + i] = hM[(size_t)i * rank + c];
        W[(size_t)(P + c) * kp + i] = -hM[(size_t)i * rank + c];
      }
    for (int c = 0; c < ns; ++c) {
      for (int i = 0; i < n0; ++i) W[(size_t)(2 * P + c) * kp + i] = hM[(size_t)i * rank + P + c];
      b[2 * P + c] = beta;
    }
    MCHK(hipMemcpy(at<float>(m, m->oW[0]), W.data(), 4 * W.size(), hipMemcpyHostToDevice));
    MCHK(hipMemcpy(at<float>(m, m->ob[0]), b.data(), 4 * b.size(), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)nblk((long)W.size(), 256)), dim3(256), 0, st,
                       at<float>(m, m->oW[0]), at<bf16_t>(m, m->oWb[0]), (long)W.size());
    MCHK(hipGetLastError());
  }
  // hidden layers: z_pair -> [z; -z] from (gelu(z), gelu(-z)); singles pass
  for (int l = 1; l + 1 < L; ++l) {
    const int kp = m->kin[l];
    std::vector<float> W((size_t)Wd * kp, 0.f), b(Wd, 0.f);
    for (int c = 0; c < P; ++c) {
      W[(size_t)c * kp + c] = 1.f;
      W[(size_t)c * kp + P + c] = -1.f;
      W[(size_t)(P + c) * kp + c] = -1.f;
      W[(size_t)(P + c) * kp + P + c] = 1.f;
    }
    for (int c = 2 * P; c < 2 * P + ns; ++c) W[(size_t)c * kp + c] = 1.f;
    MCHK(hipMemcpy(at<float>(m, m->oW[l]), W.data(), 4 * W.size(), hipMemcpyHostToDevice));
    MCHK(hipMemcpy(at<float>(m, m->ob[l]), b.data(), 4 * b.size(), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)nblk((long)W.size(), 256)), dim3(256), 0, st,
                       at<float>(m, m->oW[l]), at<bf16_t>(m, m->oWb[l]), (long)W.size());
    MCHK(hipGetLastError());
  }
  // output layer from C
  hipLaunchKernelGGL(k_fit_out_layer, dim3((unsigned)nblk((long)nL * m->kin[L - 1], 256)), dim3(256), 0, st, C, rank,
                     P, nL, Wd, m->kin[L - 1], beta, at<float>(m, m->oW[L - 1]), at<bf16_t>(m, m->oWb[L - 1]),
                     at<float>(m, m->ob[L - 1]));
  MCHK(hipGetLastError());
  for (int l = 0; l < L; ++l) {
    const size_t nw = (size_t)m->width[l + 1] * m->kin[l], nb = m->width[l + 1];
    MCHK(hipMemsetAsync(at<float>(m, m->omW[l]), 0, 4 * nw, st));
    MCHK(hipMemsetAsync(at<float>(m, m->ovW[l]), 0, 4 * nw, st));
    MCHK(hipMemsetAsync(at<float>(m, m->omb[l]), 0, 4 * nb, st));
    MCHK(hipMemsetAsync(at<float>(m, m->ovb[l]), 0, 4 * nb, st));
  }
  m->adam_t = 0;
  m->have_z = false;
  MCHK(hipStreamSynchronize(st));
  return PMDG_OK;
}

pmdg_status pmdg_mlp_set_target_scale(pmdg_mlp* m, const float* u, const float* t, const int* idx, int nrows, int n,
                                      void* work, size_t work_bytes, void* stream) {
  if (!m || !u || !t || !work) return mfail(PMDG_EINVAL, "NULL argument");
  if (!m->bound) return mfail(PMDG_ESTATE, "model not bound");
  if (n < 1 || nrows < 1 || (!idx && nrows < n)) return mfail(PMDG_EINVAL, "bad row counts");
  if (((uintptr_t)work & 7) || work_bytes < 8 * (size_t)n) return mfail(PMDG_ENOMEM, "work must hold n doubles");
  return target_scale(m, u, t, idx, nrows, n, (double*)work, (hipStream_t)stream);
}

pmdg_status pmdg_mlp_out_scale(pmdg_mlp* m, float* out_scale) {
  if (!m || !out_scale) return mfail(PMDG_EINVAL, "NULL argument");
  *out_scale = m->out_scale;
  return PMDG_OK;
}

pmdg_status pmdg_mlp_row_errors(const float* y, const float* t, const int* idx, int nrows, int B, int n, float* err,
                                void* stream) {
  if (!y || !t || !err) return mfail(PMDG_EINVAL, "NULL argument");
  if (B < 1 || n < 1 || nrows < 1 || (!idx && nrows < B)) return mfail(PMDG_EINVAL, "bad sizes");
  hipLaunchKernelGGL(k_row_relerr, dim3(B), dim3(256), 0, (hipStream_t)stream, y, t, idx, nrows, n, err);
  MCHK(hipGetLastError());
  return PMDG_OK;
}

pmdg_status pmdg_mlp_scatter_rows(const float* src, const int* rows, int nr, int n, float* dst, void* stream) {
  if (!src || !rows || !dst) return mfail(PMDG_EINVAL, "NULL argument");
  if (nr < 0 || n < 1) return mfail(PMDG_EINVAL, "bad sizes");
  if (nr == 0) return PMDG_OK;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)nblk((long)nr * n, 256)), dim3(256), 0, (hipStream_t)stream, src,
                     rows, nr, n, dst);
  MCHK(hipGetLastError());
  return PMDG_OK;
}

void pmdg_mlp_destroy(pmdg_mlp* m) { delete m; }

}  // extern "C"

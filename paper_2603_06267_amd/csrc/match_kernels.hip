// Face matching on the non-conforming interface (Sec. 5, Algorithm 3), in
// parallel over the Gauss-Legendre points of the finer faces.
//
// One thread per fine-face point x_q = X_{K+}(xi).  The coarse faces are
// scanned in index order in chunks staged through LDS: each chunk's outward
// unit normal at the face centre, first corner and diameter (the largest
// distance between two of its corners) are computed once per workgroup from
// the coarse element's corners.  A coarse face is a candidate when |n+ + n-| < tol and its first
// corner lies within r = max(diam F-, diam F+) + eps of x_q; the first
// candidate whose element's inverse map (Newton, in coordinates relative to
// its first corner) puts x_q inside [-1, 1]^3 up to 1e-10 is the match.
// The unmatched points are counted by one atomic per wave into a counter
// that a one-thread launch clears first.  FP64 throughout; nothing is
// allocated.
#include "pmutdg_internal.h"

namespace pmdg {

namespace {

constexpr int kMatchThreads = 256;
constexpr int kMatchChunk = 256;

__device__ void tri_map_d(const double V[8][3], const double xi[3], double x[3], double J[3][3]) {
  for (int r = 0; r < 3; ++r) {
    x[r] = 0;
    J[r][0] = J[r][1] = J[r][2] = 0;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const double s0 = (c & 1) ? 1.0 : -1.0, s1 = (c & 2) ? 1.0 : -1.0, s2 = (c & 4) ? 1.0 : -1.0;
    const double f0 = 0.5 * (1 + s0 * xi[0]), f1 = 0.5 * (1 + s1 * xi[1]), f2 = 0.5 * (1 + s2 * xi[2]);
    const double d0 = 0.5 * s0 * f1 * f2, d1 = 0.5 * s1 * f0 * f2, d2 = 0.5 * s2 * f0 * f1, n = f0 * f1 * f2;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      x[r] += n * V[c][r];
      J[r][0] += d0 * V[c][r];
      J[r][1] += d1 * V[c][r];
      J[r][2] += d2 * V[c][r];
    }
  }
}

// Outward unit normal at the centre of face f of the element with corners
// V, its first corner (the lowest-index corner on the face) and diameter
// (the largest distance between two of its corners: a bound on the distance
// from a corner to any point of the face).
__device__ void face_geom_d(const double V[8][3], int f, double n[3], double v0[3], double* diam) {
  const int ax = f >> 1, side = f & 1, t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
  double xi[3] = {0, 0, 0}, x[3], J[3][3];
  xi[ax] = side ? 1.0 : -1.0;
  tri_map_d(V, xi, x, J);
  const double a0 = J[0][t1], a1 = J[1][t1], a2 = J[2][t1], b0 = J[0][t2], b1 = J[1][t2], b2 = J[2][t2];
  const double c0 = a1 * b2 - a2 * b1, c1 = a2 * b0 - a0 * b2, c2 = a0 * b1 - a1 * b0;
  const double sg = (side ? 1.0 : -1.0) / sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  n[0] = sg * c0;
  n[1] = sg * c1;
  n[2] = sg * c2;
  const int k0 = side << ax, k1 = k0 | (1 << t1), k2 = k0 | (1 << t2), k3 = k1 | (1 << t2);
  const int k[4] = {k0, k1, k2, k3};
  for (int r = 0; r < 3; ++r) v0[r] = V[k0][r];
  double dmax = 0;
  for (int p = 0; p < 4; ++p)
    for (int q = p + 1; q < 4; ++q) {
      const double e0 = V[k[q]][0] - V[k[p]][0], e1 = V[k[q]][1] - V[k[p]][1], e2 = V[k[q]][2] - V[k[p]][2];
      dmax = fmax(dmax, e0 * e0 + e1 * e1 + e2 * e2);
    }
  *diam = sqrt(dmax);
}

__device__ bool tri_inverse_d(const double* __restrict__ hex, const double xg[3], double xi[3]) {
  double V[8][3], x[3];
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int r = 0; r < 3; ++r) V[c][r] = hex[3 * c + r] - hex[r];
  for (int r = 0; r < 3; ++r) x[r] = xg[r] - hex[r];
  xi[0] = xi[1] = xi[2] = 0;
  for (int it = 0; it < 60; ++it) {
    double y[3], J[3][3];
    tri_map_d(V, xi, y, J);
    const double A00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], A01 = J[0][2] * J[2][1] - J[0][1] * J[2][2],
                 A02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    const double A10 = J[1][2] * J[2][0] - J[1][0] * J[2][2], A11 = J[0][0] * J[2][2] - J[0][2] * J[2][0],
                 A12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    const double A20 = J[1][0] * J[2][1] - J[1][1] * J[2][0], A21 = J[0][1] * J[2][0] - J[0][0] * J[2][1],
                 A22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * A00 + J[0][1] * A10 + J[0][2] * A20;
    if (!(fabs(det) > 0)) return false;
    const double r0 = x[0] - y[0], r1 = x[1] - y[1], r2 = x[2] - y[2];
    const double e0 = (A00 * r0 + A01 * r1 + A02 * r2) / det, e1 = (A10 * r0 + A11 * r1 + A12 * r2) / det,
                 e2 = (A20 * r0 + A21 * r1 + A22 * r2) / det;
    xi[0] += e0;
    xi[1] += e1;
    xi[2] += e2;
    if (!(fabs(xi[0]) < 10 && fabs(xi[1]) < 10 && fabs(xi[2]) < 10)) return false;
    if (fabs(e0) + fabs(e1) + fabs(e2) < 1e-14) return true;
  }
  return false;
}

__global__ void __launch_bounds__(kMatchThreads) k_match(const MatchArgs a) {
  __shared__ double cn[kMatchChunk][3], cv[kMatchChunk][3], cd[kMatchChunk];
  __shared__ int ok[kMatchChunk];
  const int tid = threadIdx.x;
  const long npts = (long)a.nf * a.nq * a.nq;
  const long q = (long)blockIdx.x * kMatchThreads + tid;
  const bool live = q < npts;
  double x[3] = {0, 0, 0}, nf[3] = {0, 0, 0}, df = 0;
  int found = -1;
  double fxi[3] = {0, 0, 0};
  bool searching = false;
  if (live) {
    const long f = q / (a.nq * a.nq);
    const int rem = (int)(q - f * a.nq * a.nq), j = rem / a.nq, i = rem - j * a.nq;
    const int face = a.fine_face[f];
    if (face >= 0 && face < 6) {
      double V[8][3];
      for (int c = 0; c < 8; ++c)
        for (int r = 0; r < 3; ++r) V[c][r] = a.fine_hex[f * 24 + 3 * c + r];
      const int ax = face >> 1, t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
      double r3[3], J[3][3], v0[3];
      r3[ax] = (face & 1) ? 1.0 : -1.0;
      r3[t1] = a.gq[i];
      r3[t2] = a.gq[j];
      tri_map_d(V, r3, x, J);
      face_geom_d(V, face, nf, v0, &df);
      searching = true;
    }
  }
  for (int c0 = 0; c0 < a.nc; c0 += kMatchChunk) {
    __syncthreads();
    for (int t = tid; t < kMatchChunk; t += kMatchThreads) {
      const int c = c0 + t;
      int good = 0;
      if (c < a.nc) {
        const int face = a.coarse_face[c];
        if (face >= 0 && face < 6) {
          double V[8][3];
          for (int k = 0; k < 8; ++k)
            for (int r = 0; r < 3; ++r) V[k][r] = a.coarse_hex[(long)c * 24 + 3 * k + r];
          double n[3], v0[3], d;
          face_geom_d(V, face, n, v0, &d);
          for (int r = 0; r < 3; ++r) {
            cn[t][r] = n[r];
            cv[t][r] = v0[r];
          }
          cd[t] = d;
          good = 1;
        }
      }
      ok[t] = good;
    }
    __syncthreads();
    if (!searching) continue;
    const int m = min(kMatchChunk, a.nc - c0);
    for (int t = 0; t < m; ++t) {
      if (!ok[t]) continue;
      const double s0 = nf[0] + cn[t][0], s1 = nf[1] + cn[t][1], s2 = nf[2] + cn[t][2];
      const double e0 = cv[t][0] - x[0], e1 = cv[t][1] - x[1], e2 = cv[t][2] - x[2];
      const double rad = (cd[t] > df ? cd[t] : df) + a.eps;
      // |n+ + n-| < tol and |V - x_q| < r, compared as squares
      if (!(s0 * s0 + s1 * s1 + s2 * s2 < a.tol * a.tol && e0 * e0 + e1 * e1 + e2 * e2 < rad * rad)) continue;
      double t3[3];
      if (!tri_inverse_d(a.coarse_hex + (long)(c0 + t) * 24, x, t3)) continue;
      if (fabs(t3[0]) <= 1 + 1e-10 && fabs(t3[1]) <= 1 + 1e-10 && fabs(t3[2]) <= 1 + 1e-10) {
        found = c0 + t;
        fxi[0] = t3[0];
        fxi[1] = t3[1];
        fxi[2] = t3[2];
        searching = false;
        break;
      }
    }
  }
  if (live) {
    a.elem[q] = found;
    a.xi[3 * q] = fxi[0];
    a.xi[3 * q + 1] = fxi[1];
    a.xi[3 * q + 2] = fxi[2];
  }
  // unmatched points: one integer atomic per wave (an exact sum in any order)
  const unsigned long long miss = __ballot(live && found < 0);
  if ((tid & 63) == 0 && miss) atomicAdd(a.unmatched, (int)__popcll(miss));
}

__global__ void k_match_zero(int* out) {
  if (threadIdx.x == 0) *out = 0;
}

}  // namespace

hipError_t launch_match(const MatchArgs& a, hipStream_t st) {
  const long npts = (long)a.nf * a.nq * a.nq;
  hipLaunchKernelGGL(k_match_zero, dim3(1), dim3(64), 0, st, a.unmatched);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || npts == 0) return e;
  hipLaunchKernelGGL(k_match, dim3((unsigned)((npts + kMatchThreads - 1) / kMatchThreads)), dim3(kMatchThreads), 0, st,
                     a);
  return hipGetLastError();
}

}  // namespace pmdg

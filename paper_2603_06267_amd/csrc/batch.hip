// Persistent stiffness kernel of the batched form: one launch updates the
// tiles of every problem of a batch (uneven single-brick meshes of different
// orders, each with its own drive scenarios), looping over a device work list
// of (problem, tile) items.  The order and tile rows of each item select the
// device tile function; all items share one dynamic LDS allocation sized for
// the largest of them.
#include "stiff_kernel.h"

namespace pmdg {

template <int N, int RY>
__device__ __forceinline__ bool run_tile(const StiffArgs<float>& a, int key, int tile, float* lds) {
  if (key != N * 4 + RY) return false;
  // single-brick problems: no interface traces, and none of their registers
  stiff_tile<float, N, true, RY, kWaves, 2, false, false>(a, tile, lds);
  return true;
}

// Workgroup b takes the items woff[b] .. woff[b+1]-1 of the work list (the
// host balances the lists by each item's plane count), or, without woff,
// every gridDim.x-th item from b.
template <int NMAX>
__global__ void __launch_bounds__(256) k_stiff_batch(const StiffArgs<float>* __restrict__ probs,
                                                     const int2* __restrict__ items, int nitems,
                                                     const int* __restrict__ woff) {
  extern __shared__ float lds[];
  const int beg = woff ? woff[blockIdx.x] : (int)blockIdx.x;
  const int end = woff ? woff[blockIdx.x + 1] : nitems;
  const int inc = woff ? 1 : (int)gridDim.x;
  for (int it = beg; it < end; it += inc) {
    const int2 w = items[it];
    const StiffArgs<float>& a = probs[w.x];
    const int key = a.d.N * 4 + a.rows;
    __syncthreads();  // the previous item's LDS readers are done
    static_for<NMAX>([&](auto nc) {
      constexpr int N = decltype(nc)::value + 1;
      run_tile<N, 1>(a, key, w.y, lds);
      run_tile<N, 2>(a, key, w.y, lds);
    });
  }
}

size_t batch_lds_bytes(int N, int rows) {
  switch (rows) {
    case 1: return sizeof(float) * stiff_lds_elems_rt(N, 1, kWaves);
    case 2: return sizeof(float) * stiff_lds_elems_rt(N, 2, kWaves);
    default: return 0;
  }
}

static int nmax_of(int nmax) { return nmax <= 4 ? 4 : (nmax <= 6 ? 6 : 8); }

hipError_t batch_occupancy(int nmax, size_t lds, int* blocks_per_cu) {
  switch (nmax_of(nmax)) {
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_stiff_batch<4>, 256, lds);
    case 6: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_stiff_batch<6>, 256, lds);
    default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_stiff_batch<8>, 256, lds);
  }
}

hipError_t launch_stiff_batch(const StiffArgs<float>* probs, const int2* items, int nitems, const int* woff,
                              int nmax, int grid, size_t lds, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  switch (nmax_of(nmax)) {
    case 4: hipLaunchKernelGGL(k_stiff_batch<4>, dim3(grid), dim3(256), lds, st, probs, items, nitems, woff); break;
    case 6: hipLaunchKernelGGL(k_stiff_batch<6>, dim3(grid), dim3(256), lds, st, probs, items, nitems, woff); break;
    default: hipLaunchKernelGGL(k_stiff_batch<8>, dim3(grid), dim3(256), lds, st, probs, items, nitems, woff); break;
  }
  return hipGetLastError();
}

}  // namespace pmdg

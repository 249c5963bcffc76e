// Stiffness kernel instantiations: float, orders 1..4.
#include "stiff_kernel.h"

namespace pmdg {

hipError_t launch_stiff_f32_lo(const StiffArgs<float>& a, int ry, int wv, hipStream_t st) {
  switch (a.d.N) {
    case 1: return stiff_waves<float, 1, true>(a, ry, wv, st);
    case 2: return stiff_waves<float, 2, true>(a, ry, wv, st);
    case 3: return stiff_waves<float, 3, true>(a, ry, wv, st);
    case 4: return stiff_waves<float, 4, true>(a, ry, wv, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmdg

// Stiffness kernel instantiations: float, orders 1..4.
#include "stiff_kernel.h"

namespace pmdg {

hipError_t launch_stiff_f32_lo(const StiffArgs<float>& a, hipStream_t st) {
  switch (a.d.N) {
    case 1: return stiff_rows<float, 1, true>(a, st);
    case 2: return stiff_rows<float, 2, true>(a, st);
    case 3: return stiff_rows<float, 3, true>(a, st);
    case 4: return stiff_rows<float, 4, true>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmdg

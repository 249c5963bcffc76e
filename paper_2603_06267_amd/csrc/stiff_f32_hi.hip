// Stiffness kernel instantiations: float, orders 5..8.
#include "stiff_kernel.h"

namespace pmdg {

hipError_t launch_stiff_f32_hi(const StiffArgs<float>& a, hipStream_t st) {
  switch (a.d.N) {
    case 5: return stiff_rows<float, 5, true>(a, st);
    case 6: return stiff_rows<float, 6, true>(a, st);
    case 7: return stiff_rows<float, 7, true>(a, st);
    case 8: return stiff_rows<float, 8, true>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmdg

// Stiffness kernel instantiations: double, orders 5..8.
#include "stiff_kernel.h"

namespace pmdg {

hipError_t launch_stiff_f64_hi(const StiffArgs<double>& a, hipStream_t st) {
  switch (a.d.N) {
    case 5: return stiff_rows<double, 5, false>(a, st);
    case 6: return stiff_rows<double, 6, false>(a, st);
    case 7: return stiff_rows<double, 7, false>(a, st);
    case 8: return stiff_rows<double, 8, false>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmdg

// Stiffness kernel instantiations: double, orders 1..4.
#include "stiff_kernel.h"

namespace pmdg {

hipError_t launch_stiff_f64_lo(const StiffArgs<double>& a, hipStream_t st) {
  switch (a.d.N) {
    case 1: return stiff_rows<double, 1, false>(a, st);
    case 2: return stiff_rows<double, 2, false>(a, st);
    case 3: return stiff_rows<double, 3, false>(a, st);
    case 4: return stiff_rows<double, 4, false>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmdg

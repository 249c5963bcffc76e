// Stiffness kernel instantiations: double, orders 1..4.
#include "stiff_kernel.h"

namespace pmdg {

hipError_t launch_stiff_f64_lo(const StiffArgs<double>& a, int ry, int wv, hipStream_t st) {
  switch (a.d.N) {
    case 1: return stiff_waves<double, 1, false>(a, ry, wv, st);
    case 2: return stiff_waves<double, 2, false>(a, ry, wv, st);
    case 3: return stiff_waves<double, 3, false>(a, ry, wv, st);
    case 4: return stiff_waves<double, 4, false>(a, ry, wv, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmdg

// Two-step stiffness kernel instantiations: orders 1..4.
#include "stiff2_kernel.h"

namespace pmdg {

hipError_t launch_stiff2_lo(const StiffArgs<float>& a, hipStream_t st) {
  switch (a.d.N) {
    case 1: return stiff2_launch<1>(a, st);
    case 2: return stiff2_launch<2>(a, st);
    case 3: return stiff2_launch<3>(a, st);
    case 4: return stiff2_launch<4>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmdg

// Two-step stiffness kernel instantiations: order 5 (higher orders leave too
// few owned rows in a 16-row extended tile and use the single-step kernel).
#include "stiff2_kernel.h"

namespace pmdg {

hipError_t launch_stiff2_hi(const StiffArgs<float>& a, hipStream_t st) {
  switch (a.d.N) {
    case 5: return stiff2_launch<5>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmdg

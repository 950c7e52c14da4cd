// Solve-kernel instantiations with 16 lane(s) per column (nqp_kernel.h).
// Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_nqp_l16(int E, const NqpParams &p, hipStream_t s) {
    switch (E) {
    case 1: return launch_nqp_t<1, 16>(p, s);
    case 2: return launch_nqp_t<2, 16>(p, s);
    case 3: return launch_nqp_t<3, 16>(p, s);
    case 4: return launch_nqp_t<4, 16>(p, s);
    case 5: return launch_nqp_t<5, 16>(p, s);
    case 6: return launch_nqp_t<6, 16>(p, s);
    case 7: return launch_nqp_t<7, 16>(p, s);
    case 8: return launch_nqp_t<8, 16>(p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

// Solve-kernel instantiations with 8 lane(s) per column (nqp_kernel.h).
// Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_nqp_l8(int E, const NqpParams &p, hipStream_t s) {
    switch (E) {
    case 1: return launch_nqp_t<1, 8>(p, s);
    case 2: return launch_nqp_t<2, 8>(p, s);
    case 3: return launch_nqp_t<3, 8>(p, s);
    case 4: return launch_nqp_t<4, 8>(p, s);
    case 6: return launch_nqp_t<6, 8>(p, s);
    case 8: return launch_nqp_t<8, 8>(p, s);
    case 10: return launch_nqp_t<10, 8>(p, s);
    case 12: return launch_nqp_t<12, 8>(p, s);
    case 13: return launch_nqp_t<13, 8>(p, s);
    case 16: return launch_nqp_t<16, 8>(p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

// Solve-kernel instantiations with 2 lane(s) per column (nqp_kernel.h).
// Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_nqp_l2(int E, const NqpParams &p, hipStream_t s) {
    switch (E) {
    case 2: return launch_nqp_t<2, 2>(p, s);
    case 4: return launch_nqp_t<4, 2>(p, s);
    case 6: return launch_nqp_t<6, 2>(p, s);
    case 8: return launch_nqp_t<8, 2>(p, s);
    case 12: return launch_nqp_t<12, 2>(p, s);
    case 16: return launch_nqp_t<16, 2>(p, s);
    case 20: return launch_nqp_t<20, 2>(p, s);
    case 24: return launch_nqp_t<24, 2>(p, s);
    case 28: return launch_nqp_t<28, 2>(p, s);
    case 32: return launch_nqp_t<32, 2>(p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

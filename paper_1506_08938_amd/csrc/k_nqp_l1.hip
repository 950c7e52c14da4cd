// Solve-kernel instantiations with 1 lane(s) per column (nqp_kernel.h).
// Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_nqp_l1(int E, const NqpParams &p, hipStream_t s) {
    switch (E) {
    case 1: return launch_nqp_t<1, 1>(p, s);
    case 2: return launch_nqp_t<2, 1>(p, s);
    case 4: return launch_nqp_t<4, 1>(p, s);
    case 6: return launch_nqp_t<6, 1>(p, s);
    case 8: return launch_nqp_t<8, 1>(p, s);
    case 12: return launch_nqp_t<12, 1>(p, s);
    case 16: return launch_nqp_t<16, 1>(p, s);
    case 20: return launch_nqp_t<20, 1>(p, s);
    case 24: return launch_nqp_t<24, 1>(p, s);
    case 28: return launch_nqp_t<28, 1>(p, s);
    case 32: return launch_nqp_t<32, 1>(p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

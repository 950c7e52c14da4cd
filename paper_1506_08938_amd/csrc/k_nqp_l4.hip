// Solve-kernel instantiations with 4 lane(s) per column (nqp_kernel.h).
// Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_nqp_l4(int E, const NqpParams &p, hipStream_t s) {
    switch (E) {
    case 1: return launch_nqp_t<1, 4>(p, s);
    case 2: return launch_nqp_t<2, 4>(p, s);
    case 4: return launch_nqp_t<4, 4>(p, s);
    case 6: return launch_nqp_t<6, 4>(p, s);
    case 8: return launch_nqp_t<8, 4>(p, s);
    case 12: return launch_nqp_t<12, 4>(p, s);
    case 16: return launch_nqp_t<16, 4>(p, s);
    case 18: return launch_nqp_t<18, 4>(p, s);
    case 20: return launch_nqp_t<20, 4>(p, s);
    case 22: return launch_nqp_t<22, 4>(p, s);
    case 24: return launch_nqp_t<24, 4>(p, s);
    case 25: return launch_nqp_t<25, 4>(p, s);
    case 26: return launch_nqp_t<26, 4>(p, s);
    case 28: return launch_nqp_t<28, 4>(p, s);
    case 30: return launch_nqp_t<30, 4>(p, s);
    case 32: return launch_nqp_t<32, 4>(p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

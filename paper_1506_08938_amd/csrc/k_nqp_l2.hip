// Solve-kernel instantiations with 2 lane(s) per column (see nqp_kernel.h).
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_nqp_l2(int E, const NqpParams &p, hipStream_t s) {
    switch (E) {
    case 20: return launch_nqp_t<20, 2>(p, s);
    case 24: return launch_nqp_t<24, 2>(p, s);
    case 28: return launch_nqp_t<28, 2>(p, s);
    case 32: return launch_nqp_t<32, 2>(p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

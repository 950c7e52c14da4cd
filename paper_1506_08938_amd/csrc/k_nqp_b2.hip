// Batched solve-kernel instantiations with 2 lane(s) per column
// (nqp_kernel.h).  Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_bnqp_l2(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s) {
    switch (E) {
    case 2: return launch_bnqp_t<2, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 4: return launch_bnqp_t<4, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 6: return launch_bnqp_t<6, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 8: return launch_bnqp_t<8, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 12: return launch_bnqp_t<12, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 16: return launch_bnqp_t<16, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 20: return launch_bnqp_t<20, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 24: return launch_bnqp_t<24, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 28: return launch_bnqp_t<28, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 32: return launch_bnqp_t<32, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

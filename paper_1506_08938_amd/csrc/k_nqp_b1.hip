// Batched solve-kernel instantiations with 1 lane(s) per column
// (nqp_kernel.h).  Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_bnqp_l1(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s) {
    switch (E) {
    case 1: return launch_bnqp_t<1, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 2: return launch_bnqp_t<2, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 4: return launch_bnqp_t<4, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 6: return launch_bnqp_t<6, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 8: return launch_bnqp_t<8, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 12: return launch_bnqp_t<12, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 16: return launch_bnqp_t<16, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 20: return launch_bnqp_t<20, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 24: return launch_bnqp_t<24, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 28: return launch_bnqp_t<28, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 32: return launch_bnqp_t<32, 1>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

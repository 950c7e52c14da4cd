// Batched solve-kernel instantiations with 8 lane(s) per column
// (nqp_kernel.h).  Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_bnqp_l8(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s) {
    switch (E) {
    case 1: return launch_bnqp_t<1, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 2: return launch_bnqp_t<2, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 3: return launch_bnqp_t<3, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 4: return launch_bnqp_t<4, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 6: return launch_bnqp_t<6, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 8: return launch_bnqp_t<8, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 10: return launch_bnqp_t<10, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 12: return launch_bnqp_t<12, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 13: return launch_bnqp_t<13, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 16: return launch_bnqp_t<16, 8>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

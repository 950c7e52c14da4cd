// Batched solve-kernel instantiations with 16 lane(s) per column
// (nqp_kernel.h).  Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_bnqp_l16(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s) {
    switch (E) {
    case 1: return launch_bnqp_t<1, 16>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 2: return launch_bnqp_t<2, 16>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 3: return launch_bnqp_t<3, 16>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 4: return launch_bnqp_t<4, 16>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 5: return launch_bnqp_t<5, 16>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 6: return launch_bnqp_t<6, 16>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 7: return launch_bnqp_t<7, 16>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 8: return launch_bnqp_t<8, 16>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

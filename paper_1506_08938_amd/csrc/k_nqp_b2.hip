// Batched solve-kernel instantiations with 2 lane(s) per column (see nqp_kernel.h).
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_bnqp_l2(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          hipStream_t s) {
    switch (E) {
    case 20: return launch_bnqp_t<20, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, s);
    case 24: return launch_bnqp_t<24, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, s);
    case 28: return launch_bnqp_t<28, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, s);
    case 32: return launch_bnqp_t<32, 2>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

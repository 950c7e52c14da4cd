// Batched solve-kernel instantiations with 4 lane(s) per column
// (nqp_kernel.h).  Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {

hipError_t launch_bnqp_l4(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s) {
    switch (E) {
    case 1: return launch_bnqp_t<1, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 2: return launch_bnqp_t<2, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 4: return launch_bnqp_t<4, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 6: return launch_bnqp_t<6, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 8: return launch_bnqp_t<8, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 12: return launch_bnqp_t<12, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 16: return launch_bnqp_t<16, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 18: return launch_bnqp_t<18, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 20: return launch_bnqp_t<20, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 22: return launch_bnqp_t<22, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 24: return launch_bnqp_t<24, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 25: return launch_bnqp_t<25, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 26: return launch_bnqp_t<26, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 28: return launch_bnqp_t<28, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 30: return launch_bnqp_t<30, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 32: return launch_bnqp_t<32, 4>(chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nmfi

// Compiled solve-kernel variants (entries per lane E for each lanes-per-
// column L).  Written by variants.py.
#pragma once

#include <hip/hip_runtime.h>

namespace nmfi {

struct NqpParams;
struct BSolveChunk;
struct BSolveProb;

constexpr int kNqpE1[] = {1, 2, 4, 6, 8, 12, 16, 20, 24, 28, 32};
constexpr int kNqpE2[] = {2, 4, 6, 8, 12, 16, 20, 24, 28, 32};
constexpr int kNqpE4[] = {1, 2, 4, 6, 8, 12, 16, 18, 20, 22, 24, 25, 26, 28, 30, 32};
constexpr int kNqpE8[] = {1, 2, 3, 4, 6, 8, 10, 12, 13, 16};
constexpr int kNqpE16[] = {1, 2, 3, 4, 5, 6, 7, 8};

// E values compiled for L lanes per column (nullptr if none); *n = count.
inline const int *nqp_e_table(int L, int *n) {
    switch (L) {
    case 1: *n = (int)(sizeof kNqpE1 / sizeof(int)); return kNqpE1;
    case 2: *n = (int)(sizeof kNqpE2 / sizeof(int)); return kNqpE2;
    case 4: *n = (int)(sizeof kNqpE4 / sizeof(int)); return kNqpE4;
    case 8: *n = (int)(sizeof kNqpE8 / sizeof(int)); return kNqpE8;
    case 16: *n = (int)(sizeof kNqpE16 / sizeof(int)); return kNqpE16;
    default: *n = 0; return nullptr;
    }
}

hipError_t launch_nqp_l1(int E, const NqpParams &p, hipStream_t s);
hipError_t launch_bnqp_l1(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s);
hipError_t launch_nqp_l2(int E, const NqpParams &p, hipStream_t s);
hipError_t launch_bnqp_l2(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s);
hipError_t launch_nqp_l4(int E, const NqpParams &p, hipStream_t s);
hipError_t launch_bnqp_l4(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s);
hipError_t launch_nqp_l8(int E, const NqpParams &p, hipStream_t s);
hipError_t launch_bnqp_l8(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s);
hipError_t launch_nqp_l16(int E, const NqpParams &p, hipStream_t s);
hipError_t launch_bnqp_l16(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s);

}  // namespace nmfi

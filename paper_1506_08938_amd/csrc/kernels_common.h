// Vector types and small helpers shared by the product kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace nmfi {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// float -> bfloat16 with round-to-nearest-even, eight at a time
__device__ __forceinline__ bf16x8 pack_bf16x8(const float (&f)[8]) {
    bf16x8 v;
#pragma unroll
    for (int q = 0; q < 8; q++) v[q] = (__bf16)f[q];
    return v;
}

}  // namespace nmfi

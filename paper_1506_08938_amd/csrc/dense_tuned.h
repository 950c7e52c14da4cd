// Split-K slices of the dense product, measured by autotune.py --dense on an
// MI355X at each grid point: 0 keeps the rule in k_dense.hip (not measured, or
// no count beat it by more than 10%); k_dense.hip reads an entry as the block
// count it gave at its grid point.
// Command: python -m paper_1506_08938_amd.autotune --dense OUT_DIR (sweep on the GPU), then --dense-from-json dense_tuned.json
#pragma once

namespace nmfi {

constexpr long long kDenseTunedC[] = {128, 512, 2048, 8192, 32768};
constexpr long long kDenseTunedK[] = {256, 1024, 4096, 16384, 65536};
// [kernel: 0 FP32 V, 1 FP32 V' (k-major), 2 BF16][column tiles - 1][C index][K index]
constexpr int kDenseTunedSplit[3][4][5][5] = {
    {
        {{4, 16, 64, 128, 0}, {4, 8, 64, 0, 0}, {4, 12, 0, 0, 48}, {4, 0, 0, 12, 16}, {0, 0, 3, 4, 0}},
        {{4, 16, 64, 128, 0}, {4, 16, 64, 0, 0}, {4, 8, 0, 0, 0}, {2, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
        {{4, 16, 64, 128, 0}, {4, 16, 64, 0, 128}, {4, 8, 0, 32, 32}, {4, 0, 8, 8, 8}, {0, 2, 2, 2, 0}},
        {{4, 16, 64, 256, 0}, {4, 16, 64, 0, 128}, {4, 16, 0, 32, 0}, {4, 0, 8, 0, 0}, {0, 2, 0, 0, 0}},
    },
    {
        {{4, 12, 64, 128, 0}, {4, 12, 64, 0, 0}, {4, 8, 0, 0, 0}, {4, 0, 0, 0, 16}, {0, 0, 0, 4, 0}},
        {{4, 16, 64, 128, 0}, {4, 16, 64, 0, 0}, {4, 8, 0, 0, 0}, {4, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
        {{4, 16, 64, 128, 0}, {4, 16, 64, 0, 128}, {4, 8, 0, 32, 32}, {4, 0, 8, 8, 24}, {0, 2, 2, 6, 0}},
        {{4, 16, 64, 128, 0}, {4, 16, 64, 0, 128}, {4, 16, 0, 32, 0}, {4, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
    },
    {
        {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 96}, {0, 4, 0, 0, 0}, {0, 0, 8, 0, 0}, {0, 1, 0, 0, 0}},
        {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 64}, {0, 0, 0, 16, 0}, {0, 0, 0, 0, 0}, {0, 1, 0, 0, 0}},
        {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 64}, {0, 0, 0, 16, 24}, {0, 1, 6, 8, 8}, {0, 1, 3, 2, 0}},
        {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 64}, {0, 0, 0, 16, 24}, {0, 1, 6, 6, 8}, {0, 1, 3, 2, 0}},
    },
};

}  // namespace nmfi

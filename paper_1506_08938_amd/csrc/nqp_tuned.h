// Lanes per column of the solve kernel, measured by autotune.py on an
// MI355X: the fastest value for each (rank, launch size) grid point.
// Command: python -m paper_1506_08938_amd.autotune (sweep on the GPU), then --from-json nqp_tuned.json
#pragma once

namespace nmfi {

constexpr int kTunedRanks[] = {4, 8, 12, 16, 20, 24, 32, 40, 48, 56, 64, 72, 80, 90, 100, 112, 128};
constexpr long long kTunedCols[] = {256, 1024, 4096, 16384, 32768, 65536, 131072, 262144};
// [rank index][column index]
constexpr int kTunedLanes[17][8] = {
    {16, 4, 4, 1, 1, 1, 1, 1},
    {4, 4, 4, 2, 2, 1, 1, 1},
    {16, 16, 4, 2, 2, 1, 1, 1},
    {16, 16, 8, 4, 2, 2, 1, 1},
    {16, 16, 16, 4, 4, 2, 1, 1},
    {16, 16, 8, 4, 4, 2, 2, 1},
    {16, 16, 16, 8, 4, 2, 2, 2},
    {16, 16, 16, 8, 4, 2, 4, 2},
    {16, 16, 16, 8, 4, 4, 4, 4},
    {16, 16, 16, 8, 8, 4, 4, 4},
    {16, 16, 16, 8, 8, 4, 4, 4},
    {16, 16, 16, 8, 8, 8, 4, 4},
    {16, 16, 16, 8, 8, 8, 8, 4},
    {16, 16, 16, 16, 8, 8, 8, 8},
    {16, 16, 16, 16, 8, 8, 8, 8},
    {16, 16, 16, 16, 16, 16, 8, 8},
    {16, 16, 16, 16, 16, 16, 8, 8},
};

}  // namespace nmfi

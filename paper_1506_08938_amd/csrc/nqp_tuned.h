// Lanes per column of the solve kernel, measured by autotune.py on an
// MI355X: the fastest value for each (rank, launch size) grid point.
// Command: python -m paper_1506_08938_amd.autotune (sweep on the GPU), then --from-json nqp_tuned.json
#pragma once

namespace nmfi {

constexpr int kTunedRanks[] = {4, 8, 16, 24, 32, 48, 64, 80, 100, 128};
constexpr long long kTunedCols[] = {256, 1024, 4096, 16384, 65536, 262144};
// [rank index][column index]
constexpr int kTunedLanes[10][6] = {
    {16, 8, 2, 1, 1, 1},
    {8, 8, 4, 2, 1, 1},
    {16, 16, 8, 4, 2, 1},
    {8, 16, 8, 4, 2, 2},
    {16, 16, 16, 8, 4, 2},
    {16, 16, 16, 8, 4, 4},
    {16, 16, 16, 8, 8, 4},
    {16, 16, 16, 16, 8, 8},
    {16, 16, 16, 16, 8, 4},
    {16, 16, 16, 16, 16, 8},
};

}  // namespace nmfi

// Tile variant of the batched FP64 MFMA products per degree p (row) and call
// site (column: trailing update, Schur product), indices into the variant
// list of k_condense.hpp, and outer blocks per group of delayed trailing
// updates of the LU of S per degree.  Written by `python -m
// paper_2507_22195_amd.autotune --render`; edit by rerunning the sweep, not
// by hand.
//
// sweep on AMD Radeon Graphics: milliseconds per condensation spent at the site,
// best of the repetitions, viscous Taylor-Green batch of each degree; then,
// with the fastest variants, milliseconds per condensation (all its kernels)
// at each depth
//   p = 1, 4096 macro-elements (16x16x16):
//     update 0:128x64/16 1.05, 1:128x128/16 1.36, 2:128x128/16 1.41, 3:128x64/32 1.25, 4:64x64/16 0.69, 5:128x128/16 1.31, 6:64x128/16 0.85
//     schur  0:128x64/16 3.25, 1:128x128/16 4.08, 2:128x128/16 4.13, 3:128x64/32 4.22, 4:64x64/16 3.05, 5:128x128/16 3.98, 6:64x128/16 3.55
//     depth  (2 blocks) 1:13.5, 2:14.0
//   p = 2, 4096 macro-elements (16x16x16):
//     update 0:128x64/16 22.26, 1:128x128/16 24.44, 2:128x128/16 24.13, 3:128x64/32 25.65, 4:64x64/16 22.27, 5:128x128/16 23.34, 6:64x128/16 22.86
//     schur  0:128x64/16 50.29, 1:128x128/16 55.40, 2:128x128/16 54.63, 3:128x64/32 59.18, 4:64x64/16 51.02, 5:128x128/16 52.16, 6:64x128/16 52.74
//     depth  (5 blocks) 1:177.7, 2:174.0, 3:173.8, 4:174.4, 5:174.9
//   p = 3, 2048 macro-elements (16x16x8):
//     update 0:128x64/16 170.06, 1:128x128/16 185.09, 2:128x128/16 182.90, 3:128x64/32 195.96, 4:64x64/16 166.80, 5:128x128/16 176.15, 6:64x128/16 170.98
//     schur  0:128x64/16 249.87, 1:128x128/16 281.30, 2:128x128/16 276.99, 3:128x64/32 289.92, 4:64x64/16 259.34, 5:128x128/16 263.89, 6:64x128/16 269.32
//     depth  (14 blocks) 1:1036.2, 2:976.8, 3:965.4, 4:958.4, 7:957.7, 14:964.1
//   p = 4, 64 macro-elements (4x4x4):
//     update 0:128x64/16 64.06, 1:128x128/16 67.77, 2:128x128/16 68.73, 3:128x64/32 71.47, 4:64x64/16 68.11, 5:128x128/16 66.39, 6:64x128/16 67.78
//     schur  0:128x64/16 46.67, 1:128x128/16 48.30, 2:128x128/16 49.03, 3:128x64/32 52.29, 4:64x64/16 52.99, 5:128x128/16 46.33, 6:64x128/16 49.20
//     depth  (29 blocks) 1:249.2, 2:236.7, 3:232.2, 4:229.7, 7:226.9, 29:230.5
#pragma once

namespace mehdg {
constexpr int kTileTable[5][2] = {
    {0, 0},   // (unused)
    {4, 4},   // p = 1
    {0, 0},   // p = 2
    {4, 0},   // p = 3
    {0, 5},   // p = 4
};
constexpr int kLuDepth[5] = {1, 1, 3, 7, 7};   // (unused), p = 1, 2, 3, 4
}  // namespace mehdg

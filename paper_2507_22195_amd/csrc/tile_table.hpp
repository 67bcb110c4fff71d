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
//     update 0:128x64/16 28.70, 1:128x128/16 31.40, 2:128x128/16 31.55, 3:128x64/32 33.03, 4:64x64/16 30.10, 5:128x128/16 30.66, 6:64x128/16 30.55
//     schur  0:128x64/16 53.31, 1:128x128/16 57.38, 2:128x128/16 58.47, 3:128x64/32 62.52, 4:64x64/16 55.63, 5:128x128/16 55.39, 6:64x128/16 57.32
//     depth  (5 blocks) 1:179.9, 2:177.3, 3:177.1, 4:177.9, 5:179.1
//   p = 3, 2048 macro-elements (16x16x8):
//     update 0:128x64/16 178.17, 1:128x128/16 191.02, 2:128x128/16 194.44, 3:128x64/32 204.86, 4:64x64/16 176.58, 5:128x128/16 185.17, 6:64x128/16 181.38
//     schur  0:128x64/16 264.37, 1:128x128/16 292.13, 2:128x128/16 298.28, 3:128x64/32 305.43, 4:64x64/16 272.05, 5:128x128/16 282.00, 6:64x128/16 285.58
//     depth  (14 blocks) 1:1059.3, 2:1007.2, 3:991.3, 4:983.9, 7:981.9, 14:987.1
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

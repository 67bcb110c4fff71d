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
//     update 0:128x64/16 1.02, 1:128x128/16 1.33, 2:128x128/16 1.32, 3:128x64/32 1.25, 4:64x64/16 0.67, 5:128x128/16 1.28, 6:64x128/16 0.83
//     schur  0:128x64/16 3.35, 1:128x128/16 4.17, 2:128x128/16 4.18, 3:128x64/32 4.41, 4:64x64/16 3.13, 5:128x128/16 4.01, 6:64x128/16 3.52
//     depth  (2 blocks) 1:13.7, 2:14.1
//   p = 2, 4096 macro-elements (16x16x16):
//     update 0:128x64/16 30.62, 1:128x128/16 32.96, 2:128x128/16 32.89, 3:128x64/32 36.22, 4:64x64/16 32.06, 5:128x128/16 31.64, 6:64x128/16 32.22
//     schur  0:128x64/16 57.09, 1:128x128/16 60.80, 2:128x128/16 61.53, 3:128x64/32 70.71, 4:64x64/16 62.00, 5:128x128/16 58.28, 6:64x128/16 62.12
//     depth  (5 blocks) 1:188.0, 2:184.9, 3:185.1, 4:185.1, 5:186.4
//   p = 3, 2048 macro-elements (16x16x8):
//     update 0:128x64/16 190.33, 1:128x128/16 203.98, 2:128x128/16 206.82, 3:128x64/32 232.05, 4:64x64/16 195.18, 5:128x128/16 193.88, 6:64x128/16 196.98
//     schur  0:128x64/16 285.29, 1:128x128/16 313.65, 2:128x128/16 318.63, 3:128x64/32 349.35, 4:64x64/16 301.08, 5:128x128/16 295.30, 6:64x128/16 310.91
//     depth  (14 blocks) 1:1111.5, 2:1057.5, 3:1042.3, 4:1040.2, 7:1038.2, 14:1044.6
//   p = 4, 64 macro-elements (4x4x4):
//     update 0:128x64/16 108.39, 1:128x128/16 115.14, 2:128x128/16 115.82, 3:128x64/32 125.64, 4:64x64/16 113.17, 5:128x128/16 114.02, 6:64x128/16 114.28
//     schur  0:128x64/16 49.96, 1:128x128/16 51.38, 2:128x128/16 52.57, 3:128x64/32 61.13, 4:64x64/16 58.90, 5:128x128/16 49.11, 6:64x128/16 53.69
//     depth  (29 blocks) 1:262.7, 2:248.3, 3:243.7, 4:239.9, 7:236.5, 29:242.6
#pragma once

namespace mehdg {
constexpr int kTileTable[5][2] = {
    {0, 0},   // (unused)
    {4, 4},   // p = 1
    {0, 0},   // p = 2
    {0, 0},   // p = 3
    {0, 5},   // p = 4
};
constexpr int kLuDepth[5] = {1, 1, 2, 7, 7};   // (unused), p = 1, 2, 3, 4
}  // namespace mehdg

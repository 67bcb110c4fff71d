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
//     update 0:128x64/16 21.82, 1:128x128/16 24.16, 2:128x128/16 24.27, 3:128x64/32 25.79, 4:64x64/16 22.02, 5:128x128/16 23.48, 6:64x128/16 23.35, 7:128x64/16 21.40
//     schur  0:128x64/16 49.10, 1:128x128/16 54.80, 2:128x128/16 55.20, 3:128x64/32 60.08, 4:64x64/16 50.02, 5:128x128/16 52.17, 6:64x128/16 52.27, 7:128x64/16 48.02
//     depth  (5 blocks) 1:172.9, 2:169.6, 3:169.8, 4:170.4, 5:171.2
//   p = 3, 2048 macro-elements (16x16x8):
//     update 0:128x64/16 165.61, 1:128x128/16 183.15, 2:128x128/16 184.06, 3:128x64/32 196.65, 4:64x64/16 161.44, 5:128x128/16 174.64, 6:64x128/16 167.12, 7:128x64/16 162.76
//     schur  0:128x64/16 240.13, 1:128x128/16 278.40, 2:128x128/16 279.73, 3:128x64/32 291.58, 4:64x64/16 243.07, 5:128x128/16 261.48, 6:64x128/16 254.19, 7:128x64/16 237.12
//     depth  (14 blocks) 1:1016.4, 2:954.8, 3:936.9, 4:930.2, 7:926.5, 14:933.2
//   p = 4, 64 macro-elements (4x4x4):
//     update 0:128x64/16 64.06, 1:128x128/16 67.77, 2:128x128/16 68.73, 3:128x64/32 71.47, 4:64x64/16 68.11, 5:128x128/16 66.39, 6:64x128/16 67.78
//     schur  0:128x64/16 46.67, 1:128x128/16 48.30, 2:128x128/16 49.03, 3:128x64/32 52.29, 4:64x64/16 52.99, 5:128x128/16 46.33, 6:64x128/16 49.20
//     depth  (29 blocks) 1:249.2, 2:236.7, 3:232.2, 4:229.7, 7:226.9, 29:230.5
#pragma once

namespace mehdg {
constexpr int kTileTable[5][2] = {
    {0, 0},   // (unused)
    {4, 4},   // p = 1
    {7, 7},   // p = 2
    {4, 7},   // p = 3
    {0, 5},   // p = 4
};
constexpr int kLuDepth[5] = {1, 1, 2, 7, 7};   // (unused), p = 1, 2, 3, 4
}  // namespace mehdg

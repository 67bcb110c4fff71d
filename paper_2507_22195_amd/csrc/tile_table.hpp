// Tile variant of the batched FP64 MFMA products per degree p (row) and call
// site (column: trailing update, Schur product), indices into the variant
// list of k_condense.hpp.  Written by `python -m paper_2507_22195_amd.autotune
// --render`; edit by rerunning the sweep, not by hand.
//
// sweep on AMD Radeon Graphics: milliseconds per condensation spent at the site,
// best of the repetitions, viscous Taylor-Green batch of each degree
//   p = 1, 4096 macro-elements (16x16x16):
//     update 0:128x64/16 1.01, 1:128x128/16 1.32, 2:128x128/16 1.31, 3:128x64/32 1.19, 4:64x64/16 0.66, 5:128x128/16 1.25, 6:64x128/16 0.82
//     schur  0:128x64/16 3.36, 1:128x128/16 4.12, 2:128x128/16 4.18, 3:128x64/32 4.36, 4:64x64/16 3.11, 5:128x128/16 4.03, 6:64x128/16 3.59
//   p = 2, 4096 macro-elements (16x16x16):
//     update 0:128x64/16 42.39, 1:128x128/16 44.70, 2:128x128/16 44.98, 3:128x64/32 49.07, 4:64x64/16 43.69, 5:128x128/16 43.78, 6:64x128/16 43.68
//     schur  0:128x64/16 57.25, 1:128x128/16 61.09, 2:128x128/16 61.80, 3:128x64/32 71.00, 4:64x64/16 62.26, 5:128x128/16 58.36, 6:64x128/16 62.37
//   p = 3, 2048 macro-elements (16x16x8):
//     update 0:128x64/16 396.66, 1:128x128/16 416.39, 2:128x128/16 415.90, 3:128x64/32 467.80, 4:64x64/16 402.07, 5:128x128/16 405.94, 6:64x128/16 403.01
//     schur  0:128x64/16 284.89, 1:128x128/16 314.13, 2:128x128/16 319.02, 3:128x64/32 349.84, 4:64x64/16 301.76, 5:128x128/16 295.46, 6:64x128/16 311.30
#pragma once

namespace mehdg {
constexpr int kTileTable[5][2] = {
    {0, 0},   // (unused)
    {4, 4},   // p = 1
    {0, 0},   // p = 2
    {0, 0},   // p = 3
    {0, 0},   // p = 4 (not swept yet)
};
}  // namespace mehdg

// Tile shapes of the grouped products of the batched form, written by
// paper_1310_7202_amd/tune.py from timings on MI355X (see the record below).
// kGroupedTile[product][storage]: product 0 sketch, 1 Gram, 2 projection,
// 3 S^{-1} C, 4 L = Lv L_b; storage 0 FP64, 1 FP32.  -1 keeps the built-in
// rule (a tile at least as wide as l for the sketch, 64 x 64 otherwise).
//
// Record: phase time (ms, best of 3) of a batch of 256 problems (m, n ~
// U[256, 4096], r ~ U[8, 64], k = r, l = r + 8) per tile shape:
//   sketch_gemm   FP64: 64x64x16 5.297, 64x112x16 7.201, 112x64x16 5.104, 64x112x32 8.668, 112x64x32 5.638, 64x64x32 5.618, 128x64x16 4.782, 64x128x16 7.696  -> 128x64x16
//   sketch_gemm   FP32: 64x64x16 3.015, 64x112x16 3.749, 112x64x16 2.771, 64x112x32 4.035, 112x64x32 2.977, 64x64x32 2.992, 128x64x16 2.552, 64x128x16 3.964  -> 128x64x16
//   gram_gemm     FP64: 64x64x16 0.226, 64x112x16 0.356, 112x64x16 0.374, 64x112x32 0.426, 112x64x32 0.436, 64x64x32 0.275, 128x64x16 0.368, 64x128x16 0.373  -> 64x64x16
//   gram_gemm     FP32: 64x64x16 0.225, 64x112x16 0.365, 112x64x16 0.359, 64x112x32 0.430, 112x64x32 0.438, 64x64x32 0.275, 128x64x16 0.379, 64x128x16 0.381  -> 64x64x16
//   project_gemm  FP64: 64x64x16 4.749, 64x112x16 4.504, 112x64x16 6.926, 64x112x32 7.443, 112x64x32 12.490, 64x64x32 5.794, 128x64x16 8.441, 64x128x16 4.735  -> 64x112x16
//   project_gemm  FP32: 64x64x16 3.061, 64x112x16 2.947, 112x64x16 4.569, 64x112x32 3.072, 112x64x32 4.804, 64x64x32 3.192, 128x64x16 4.720, 64x128x16 2.609  -> 64x128x16
//   solve_gemm    FP64: 64x64x16 0.121, 64x112x16 0.138, 112x64x16 0.195, 64x112x32 0.209, 112x64x32 0.312, 64x64x32 0.166, 128x64x16 0.206, 64x128x16 0.136  -> 64x64x16
//   solve_gemm    FP32: 64x64x16 0.121, 64x112x16 0.140, 112x64x16 0.195, 64x112x32 0.209, 112x64x32 0.308, 64x64x32 0.165, 128x64x16 0.205, 64x128x16 0.135  -> 64x64x16
//   form_l_gemm   FP64: 64x64x16 0.200, 64x112x16 0.314, 112x64x16 0.293, 64x112x32 0.504, 112x64x32 0.458, 64x64x32 0.290, 128x64x16 0.283, 64x128x16 0.353  -> 64x64x16
//   form_l_gemm   FP32: 64x64x16 0.212, 64x112x16 0.310, 112x64x16 0.284, 64x112x32 0.496, 112x64x32 0.450, 64x64x32 0.279, 128x64x16 0.268, 64x128x16 0.350  -> 64x64x16
#pragma once

namespace rlu {
namespace tuned {

constexpr int kGroupedTile[5][2] = {{7, 7}, {0, 0}, {1, 8}, {0, 0}, {0, 0}};

}  // namespace tuned
}  // namespace rlu

// Tile shapes of the grouped products of the batched form, written by
// paper_1310_7202_amd/tune.py from timings on MI355X (see the record below).
// kGroupedTile[product][storage]: product 0 sketch, 1 Gram, 2 projection,
// 3 S^{-1} C, 4 L = Lv L_b; storage 0 FP64, 1 FP32.  -1 keeps the built-in
// rule (a tile at least as wide as l for the sketch, 64 x 64 otherwise).
//
// Record: phase time (ms, best of 3) of a batch of 256 problems (m, n ~
// U[256, 4096], r ~ U[8, 64], k = r, l = r + 8) per tile shape:
//   sketch_gemm   FP64: 64x64x16 5.112, 64x112x16 7.118, 112x64x16 5.118, 64x112x32 8.590, 112x64x32 5.667, 64x64x32 5.472, 128x64x16 4.664, 64x128x16 7.528  -> 128x64x16
//   sketch_gemm   FP32: 64x64x16 2.889, 64x112x16 3.706, 112x64x16 2.753, 64x112x32 3.907, 112x64x32 2.984, 64x64x32 2.869, 128x64x16 2.549, 64x128x16 3.948  -> 128x64x16
//   gram_gemm     FP64: 64x64x16 0.155, 64x112x16 0.304, 112x64x16 0.299, 64x112x32 0.320, 112x64x32 0.326, 64x64x32 0.189, 128x64x16 0.318, 64x128x16 0.318  -> 64x64x16
//   gram_gemm     FP32: 64x64x16 0.156, 64x112x16 0.296, 112x64x16 0.295, 64x112x32 0.318, 112x64x32 0.320, 64x64x32 0.184, 128x64x16 0.312, 64x128x16 0.314  -> 64x64x16
//   project_gemm  FP64: 64x64x16 4.082, 64x112x16 4.139, 112x64x16 7.003, 64x112x32 5.326, 112x64x32 8.826, 64x64x32 4.337, 128x64x16 7.543, 64x128x16 4.235  -> 64x64x16
//   project_gemm  FP32: 64x64x16 2.564, 64x112x16 2.436, 112x64x16 3.851, 64x112x32 2.409, 112x64x32 4.202, 64x64x32 2.543, 128x64x16 4.025, 64x128x16 2.366  -> 64x128x16
//   solve_gemm    FP64: 64x64x16 0.123, 64x112x16 0.144, 112x64x16 0.198, 64x112x32 0.210, 112x64x32 0.314, 64x64x32 0.167, 128x64x16 0.207, 64x128x16 0.137  -> 64x64x16
//   solve_gemm    FP32: 64x64x16 0.124, 64x112x16 0.147, 112x64x16 0.203, 64x112x32 0.218, 112x64x32 0.329, 64x64x32 0.174, 128x64x16 0.216, 64x128x16 0.143  -> 64x64x16
//   form_l_gemm   FP64: 64x64x16 0.198, 64x112x16 0.313, 112x64x16 0.291, 64x112x32 0.501, 112x64x32 0.458, 64x64x32 0.287, 128x64x16 0.285, 64x128x16 0.353  -> 64x64x16
//   form_l_gemm   FP32: 64x64x16 0.211, 64x112x16 0.308, 112x64x16 0.279, 64x112x32 0.496, 112x64x32 0.450, 64x64x32 0.279, 128x64x16 0.276, 64x128x16 0.351  -> 64x64x16
#pragma once

namespace rlu {
namespace tuned {

constexpr int kGroupedTile[5][2] = {{7, 7}, {0, 0}, {0, 8}, {0, 0}, {0, 0}};

}  // namespace tuned
}  // namespace rlu

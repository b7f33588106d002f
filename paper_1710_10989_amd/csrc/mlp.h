// Small MLP of the learned (m, s) selector: 8 features -> 64 (ReLU) -> 64 (ReLU) -> 16 classes.
#pragma once

namespace expm {

constexpr int kMlpIn = 8, kMlpH = 64, kMlpOut = 16;
// Packed FP32 parameters: W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [16][64], b3 [16].
constexpr int kMlpW1 = 0, kMlpB1 = kMlpW1 + kMlpH * kMlpIn, kMlpW2 = kMlpB1 + kMlpH,
              kMlpB2 = kMlpW2 + kMlpH * kMlpH, kMlpW3 = kMlpB2 + kMlpH, kMlpB3 = kMlpW3 + kMlpOut * kMlpH,
              kMlpParams = kMlpB3 + kMlpOut;

// Class c <-> (m, s): c = 0..4 -> (1, 0), (2, 0), (4, 0), (8, 0), (12, 0); c = 5..15 -> (18, c - 5).
__host__ __device__ inline void mlp_class_ms(int c, int *m, int *s) {
  const int ms[5] = {1, 2, 4, 8, 12};
  if (c < 5) { *m = ms[c]; *s = 0; } else { *m = 18; *s = c - 5; }
}
__host__ __device__ inline int mlp_ms_class(int m, int s) {
  if (m == 18) return s <= 10 ? 5 + s : -1;
  if (s != 0) return -1;
  switch (m) { case 1: return 0; case 2: return 1; case 4: return 2; case 8: return 3; case 12: return 4; }
  return -1;
}

}  // namespace expm

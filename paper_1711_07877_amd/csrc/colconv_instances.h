// Compiled instances of the whole-column convolution: X(L, R0, R1, R2, R3, tag).
// Lengths form a ladder (about 1.2x apart) with four-stage radix sequences (R0 even);
// 8640 = 12 12 12 5 is the length of the 1e7-point grids.  The plan takes the
// smallest instance at or above the length it needs when it is within 15% of the
// generic transform's size, else the generic column passes.
#pragma once

#define SBD_CC_F32R_A(X)                                                                   \
  X(216, 4, 3, 9, 2, f32r) X(256, 4, 4, 8, 2, f32r) X(324, 4, 3, 3, 9, f32r) X(384, 8, 3, 8, 2, f32r) \
  X(432, 4, 4, 3, 9, f32r) X(480, 4, 3, 5, 8, f32r) X(576, 4, 8, 9, 2, f32r) X(720, 8, 5, 9, 2, f32r) X(864, 4, 3, 8, 9, f32r) \
  X(1024, 8, 8, 8, 2, f32r) X(1296, 8, 9, 9, 2, f32r) X(1536, 8, 3, 8, 8, f32r) X(1728, 8, 3, 8, 9, f32r) \
  X(2048, 4, 8, 8, 8, f32r) X(2592, 4, 8, 9, 9, f32r)
#define SBD_CC_F32R_B(X)                                                                   \
  X(3072, 8, 3, 8, 16, f32r) X(3456, 8, 3, 9, 16, f32r) X(4096, 8, 8, 8, 8, f32r) X(4608, 8, 8, 8, 9, f32r) \
  X(5184, 8, 8, 9, 9, f32r) X(5832, 8, 9, 9, 9, f32r) X(6912, 8, 8, 9, 12, f32r) X(7776, 8, 9, 9, 12, f32r) \
  X(8640, 12, 12, 12, 5, f32r) X(9216, 8, 8, 9, 16, f32r) X(10368, 8, 9, 9, 16, f32r) X(11664, 16, 9, 9, 9, f32r) \
  X(13824, 8, 9, 12, 16, f32r) X(15552, 12, 9, 9, 16, f32r)
#define SBD_CC_F32C(X)                                                                     \
  X(432, 4, 4, 3, 9, f32c) X(480, 4, 3, 5, 8, f32c) X(576, 4, 8, 9, 2, f32c) X(1296, 8, 9, 9, 2, f32c) X(2592, 4, 8, 9, 9, f32c) X(5184, 8, 8, 9, 9, f32c)
#define SBD_CC_F64R(X)                                                                     \
  X(432, 4, 4, 3, 9, f64r) X(1296, 8, 9, 9, 2, f64r) X(2592, 4, 8, 9, 9, f64r) X(5184, 8, 8, 9, 9, f64r) \
  X(8640, 12, 12, 12, 5, f64r)
#define SBD_CC_F64C(X) X(576, 4, 8, 9, 2, f64c) X(5184, 8, 8, 9, 9, f64c)

// Compiled instances of the real-row transforms: X(N, R0, R1, R2, R3, tag), N the complex
// length (real row length 2 N).  The forward transform runs the radices in this order
// (R0 even: its first stage drops the zero upper half), the inverse in reverse order (its
// last stage, radix R0, keeps the lower half).  The plan takes the smallest N >= nx when
// it is within 15% of the generic transform's size.
#pragma once

#define SBD_RR_F32(X)                                                                                       \
  X(120, 4, 3, 5, 2, rf32) X(144, 4, 4, 3, 3, rf32) X(192, 4, 4, 4, 3, rf32) X(216, 4, 3, 9, 2, rf32)        \
  X(256, 4, 4, 8, 2, rf32) X(324, 4, 3, 3, 9, rf32) X(384, 8, 3, 8, 2, rf32) X(432, 4, 4, 3, 9, rf32)        \
  X(480, 4, 3, 5, 8, rf32) X(576, 4, 8, 9, 2, rf32) X(720, 8, 5, 9, 2, rf32) X(864, 4, 3, 8, 9, rf32)        \
  X(1024, 8, 8, 8, 2, rf32) X(1296, 8, 9, 9, 2, rf32) X(1536, 8, 3, 8, 8, rf32) X(1728, 8, 3, 8, 9, rf32)    \
  X(2048, 4, 8, 8, 8, rf32) X(2592, 4, 8, 9, 9, rf32) X(3072, 8, 3, 8, 16, rf32) X(3456, 8, 3, 9, 16, rf32)  \
  X(4096, 8, 8, 8, 8, rf32) X(4320, 8, 5, 9, 12, rf32) X(4608, 8, 8, 8, 9, rf32) X(5184, 8, 8, 9, 9, rf32)   \
  X(5832, 8, 9, 9, 9, rf32) X(6912, 8, 8, 9, 12, rf32) X(7776, 8, 9, 9, 12, rf32)
#define SBD_RR_F64(X)                                                                                       \
  X(216, 4, 3, 9, 2, rf64) X(432, 4, 4, 3, 9, rf64) X(1296, 8, 9, 9, 2, rf64) X(2592, 4, 8, 9, 9, rf64)      \
  X(4320, 8, 5, 9, 12, rf64)

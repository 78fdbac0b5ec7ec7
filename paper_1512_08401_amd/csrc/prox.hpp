// Coordinate step of the proximal update (Alg. 1 steps 3-4; Alg. 2 with a
// diagonal P), shared by the float32 proximal kernels.
//
// The iterate may be held as a float64 anchor a plus a float32 displacement
// (x = a + d): the float32 vectors of the iteration then carry differences
// from a, whose size shrinks as the solve converges, instead of the
// coefficients themselves (the approximation coefficients reach 2^J times
// the image mean, and their float32 rounding alone moves the gradient by
// far more than the optimality conditions of the l1 problem can absorb).
// The threshold decision is taken on the whole coefficient in float64.
#pragma once

#include <hip/hip_runtime.h>

namespace wdb {

// x = S_t(z), z = y - sg (float32 iterate).
__device__ __forceinline__ float prox_plain(float y, float sg, float t) {
  const float z = y - sg;
  return copysignf(fmaxf(fabsf(z) - t, 0.0f), z);
}

// Anchored iterate: z = a + y - sg in float64, x = S_t(z); returns the
// displacement x - a rounded to float32 (-a when the coefficient is zeroed).
__device__ __forceinline__ float prox_anchored(double a, float y, float sg, float t) {
  const double z = (a + static_cast<double>(y)) - static_cast<double>(sg);
  const double xa = copysign(fmax(fabs(z) - static_cast<double>(t), 0.0), z);
  return static_cast<float>(xa - a);
}

}  // namespace wdb

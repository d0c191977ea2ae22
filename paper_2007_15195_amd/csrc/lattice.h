// Randomized Richtmyer lattice points (device side).
//
// Generator z_j = frac(sqrt(p_j)), p_j the j-th prime, held as the 64-bit
// fixed-point integer Z_j (computed on the host by an exact integer square
// root and passed to the kernels). Shift S = SplitMix64 output number
// n = (term << 21) | (shift << 5) | dim (dim < 32) of the stream seeded with
// the call's seed (Steele, Lea & Flood 2014). Point p: U = p Z_j + S mod 2^64; baker
// transform W = |2U - 2^64| (2^64 saturates); the coordinate is the midpoint
// of W's cell on the 2^-52 grid (FP64) or, from U's upper half, on the 2^-23
// grid (FP32).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vecchia {

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Dimensions 32..62 (terms of more than 32 variables) take the key
// 2^62 + (term << 22) + (shift << 6) + dim, a range the first form never reaches.
// A term's second lattice (the denominators of the independent-points
// estimator) adds 2^61 to the key: no first-lattice key has that bit set.
__device__ __forceinline__ uint64_t lattice_shift(uint64_t seed, int64_t term, int r, int dim, bool second) {
  const uint64_t salt = second ? (1ULL << 61) : 0ULL;
  if (dim < 32) return splitmix64(seed, salt | ((uint64_t)term << 21) | ((uint64_t)r << 5) | (uint64_t)dim);
  return splitmix64(seed, salt | (1ULL << 62) | ((uint64_t)term << 22) | ((uint64_t)r << 6) | (uint64_t)dim);
}

// FP64 coordinate (2 floor(W / 2^12) + 1) 2^-53.
__device__ __forceinline__ double lattice_coord_f64(uint64_t U) {
  const uint64_t twice = U << 1;
  uint64_t W = (U >> 63) ? twice : (0 - twice);
  W = U ? W : ~0ULL;
  const uint64_t odd = (W >> 11) | 1ULL;   // 2 floor(W/2^12) + 1 < 2^53
  return (double)odd * 0x1p-53;
}

// FP32 coordinate of U, from its upper 32 bits only: with s = U_hi - 2^31 as a
// signed 32-bit integer, the cell is c = |s| >> 8 for s >= 0 and
// (|s| - 1) >> 8 for s < 0, and w = (c + 1/2) 2^-23, the midpoint of the 2^-23
// cell of the baker-transformed point (within 2^-24 of the FP64 coordinate;
// exactly its cell unless U's low 40 bits are all zero). With
// g = (signed U_hi) >> 8 this is w = 1 - |g + 1/2| 2^-23, so 1 - w = |g + 1/2| 2^-23;
// both are exact in FP32.
struct CoordF32 {
  float w, wc;   // w and 1 - w
};
__device__ __forceinline__ CoordF32 lattice_coord_f32(uint32_t hi) {
  const float g = (float)((int32_t)hi >> 8);
  CoordF32 c;
  c.wc = fabsf(fmaf(g, 0x1p-23f, 0x1p-24f));
  c.w = 1.0f - c.wc;
  return c;
}

}  // namespace vecchia

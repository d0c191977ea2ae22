// Randomized Richtmyer lattice points (device side).
//
// Generator z_j = frac(sqrt(p_j)), p_j the j-th prime, held as the 64-bit
// fixed-point integer Z_j (computed on the host by an exact integer square
// root and passed to the kernels). Shift S = SplitMix64 output number
// n = (term << 21) | (shift << 5) | dim of the stream seeded with the call's
// seed (Steele, Lea & Flood 2014). Point p: U = p Z_j + S mod 2^64; baker
// transform W = |2U - 2^64| (2^64 saturates); the coordinate is the midpoint
// of W's cell on the 2^-52 (FP64) or 2^-23 (FP32) grid.
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

__device__ __forceinline__ uint64_t lattice_shift(uint64_t seed, int64_t term, int r, int dim) {
  return splitmix64(seed, ((uint64_t)term << 21) | ((uint64_t)r << 5) | (uint64_t)dim);
}

// FP64 coordinate (2 floor(W / 2^12) + 1) 2^-53.
__device__ __forceinline__ double lattice_coord_f64(uint64_t U) {
  const uint64_t twice = U << 1;
  uint64_t W = (U >> 63) ? twice : (0 - twice);
  W = U ? W : ~0ULL;
  const uint64_t odd = (W >> 11) | 1ULL;   // 2 floor(W/2^12) + 1 < 2^53
  return (double)odd * 0x1p-53;
}

// FP32 coordinate (2 floor(W / 2^41) + 1) 2^-24, from the two 32-bit halves of U.
// U >= 2^63: floor(W/2^41) = bits 62..40 of U.
// U <  2^63: W = 2X with X = 2^63 - U in (0, 2^63], floor(W/2^41) = min(X >> 40, 2^23 - 1).
__device__ __forceinline__ uint32_t lattice_cell_f32(uint32_t hi, uint32_t lo) {
  const uint32_t up = (hi >> 8) & 0x7fffffu;
  const uint32_t borrow = lo != 0u;
  const uint32_t xhi = 0x80000000u - hi - borrow;
  uint32_t dn = xhi >> 8;
  dn = dn < 0x7fffffu ? dn : 0x7fffffu;
  return (hi & 0x80000000u) ? up : dn;
}

}  // namespace vecchia

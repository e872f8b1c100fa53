// Shared pieces of the fused column-projection kernels (FP64 in proj.hip,
// FP32 and split-BF16 in proj_lp.hip).  Internal to the library.
#pragma once

#include "kernels.h"

namespace ttice {
namespace proj {

template <typename T, int VEC>
struct Vec;
template <typename T>
struct Vec<T, 1> {
  T v[1];
  __device__ static Vec load(const T* p) { return Vec{{p[0]}}; }
};
template <typename T>
struct Vec<T, 2> {
  T v[2];
  __device__ static Vec load(const T* p) {
    Vec r;
    __builtin_memcpy(&r.v[0], __builtin_assume_aligned(p, 2 * sizeof(T)), 2 * sizeof(T));
    return r;
  }
};
template <typename T>
struct Vec<T, 4> {
  T v[4];
  __device__ static Vec load(const T* p) {
    Vec r;
    __builtin_memcpy(&r.v[0], __builtin_assume_aligned(p, 4 * sizeof(T)), 4 * sizeof(T));
    return r;
  }
};

template <int VEC>
__device__ __forceinline__ void store_vec(double* p, const double* v) {
  if constexpr (VEC == 1) {
    p[0] = v[0];
  } else {
    __builtin_memcpy(__builtin_assume_aligned(p, VEC * sizeof(double)), v, VEC * sizeof(double));
  }
}

// True when every lane's VEC columns of view v (elements of esize bytes at
// base) are consecutive in memory and VEC-aligned.
inline bool aligned_cols(const View& v, const void* base, size_t esize, int vec) {
  if (v.cs != 1 || (v.rs % vec) != 0) return false;
  if (v.cpf != kUnframed && ((v.cpf % vec) != 0 || (v.cfs % vec) != 0)) return false;
  return ((uintptr_t)base % (vec * esize)) == 0;
}

constexpr int kChunkQuads = 8;  // row quads whose loads are issued together

// LDS bytes of the fixed-order tree over W waves with NV doubles per lane
constexpr size_t red_bytes(int W, int NV) { return (size_t)(W / 2) * NV * 64 * sizeof(double); }

}  // namespace proj
}  // namespace ttice

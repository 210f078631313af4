// Bucket gather of one staged chunk, shared by the stored-A and the matrix-free
// SJLT kernels.  For each of the wave's NJ output columns, every entry of the
// column's bucket for this chunk names a staged source (entry >> 1) and a sign
// (entry & 1); the source's RPL values of this lane are read from LDS through
// LD(entry) and added with that sign.  Entries are wave-uniform (scalar loads).
#pragma once
#include "internal.hpp"

namespace sk {

// +-1 from an entry's sign bit, built with integer operations on the uniform
// entry so that it stays a scalar operand of the FMA
template <typename T>
__device__ __forceinline__ T entry_sign(int v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(float, ((uint32_t)v << 31) | 0x3f800000u);
  } else {
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)v << 63) | 0x3ff0000000000000ull);
  }
}

// P: the wave's bucket bounds for this chunk (NJ + 1 values), ent: entries
template <typename T, int NJ, int RPL, typename VT, typename LoadFn>
__device__ __forceinline__ void gather_chunk(const int32_t* __restrict__ P, const int32_t* __restrict__ ent,
                                             LoadFn LD, T (&acc)[NJ][RPL]) {
  int pv[NJ + 1];  // loaded once per chunk
#pragma unroll
  for (int jj = 0; jj <= NJ; ++jj) pv[jj] = P[jj];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    // accumulate straight into acc: separate partial sums per column get sunk
    // to the end of the chunk by the compiler and inflate VGPR use
    const int p1 = pv[jj + 1];
    int e = pv[jj];
    for (; e + 4 <= p1; e += 4) {
      const int v0 = ent[e], v1 = ent[e + 1], v2 = ent[e + 2], v3 = ent[e + 3];
      const VT x0 = LD(v0), x1 = LD(v1), x2 = LD(v2), x3 = LD(v3);
      const T s0 = entry_sign<T>(v0), s1 = entry_sign<T>(v1), s2 = entry_sign<T>(v2), s3 = entry_sign<T>(v3);
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        T a = fma(((const T*)&x0)[r], s0, acc[jj][r]);
        a = fma(((const T*)&x1)[r], s1, a);
        a = fma(((const T*)&x2)[r], s2, a);
        acc[jj][r] = fma(((const T*)&x3)[r], s3, a);
      }
    }
    for (; e < p1; ++e) {
      const int v0 = ent[e];
      const VT x0 = LD(v0);
      const T s0 = entry_sign<T>(v0);
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[jj][r] = fma(((const T*)&x0)[r], s0, acc[jj][r]);
    }
  }
}

}  // namespace sk

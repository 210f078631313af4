// Bucket gather of one staged chunk, shared by the stored-A and the matrix-free
// SJLT kernels.  For each of the wave's NJ output columns, every entry of the
// column's bucket for this chunk names a staged source (entry >> 1) and a sign
// (entry & 1); the source's RPL values of this lane are read from LDS through
// LD(entry) and added with that sign.  Entries are wave-uniform (scalar loads).
#pragma once
#include <type_traits>
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

namespace sk {

// Bucket gather with the chunk's entries staged in LDS.  E holds EW words per
// entry: word 0 is the LDS address of the entry's source row in the staged tile
// (XOR the lane's part gives the lane's address) and the last one (FP32) or
// two (FP64) words the sign as a +-1.0 of type T.  The wave's bucket bounds
// arrive in a VGPR (lane jj holds the start of column jj, bndN the end of the
// last column).
//
// Bucket lengths vary (about KC * alpha / w entries per column and chunk), and
// a data-dependent loop per column leaves one dependent chain of LDS reads in
// flight.  So the first ms (4 or 8) slots of every bucket are gathered by
// straight-line code (slots past the bucket's end read the zero row at zaddr),
// four independent reads at a time; the rest of a longer bucket follows in
// pairs (and a last single entry).
// With PACK, E holds one word per entry instead: the address with the sign in
// bit 31.  With NEG the tile holds a negated copy of every staged source and
// an entry is one word, the address of the source row or of its negated copy:
// the gather adds without a sign.
template <typename T, int NJ, int RPL, typename VT, bool PACK = false, bool NEG = false>
__device__ __forceinline__ void gather_chunk_lds(const uint32_t* E, int ebase, uint32_t bnd, uint32_t bndN,
                                                 uint32_t lane_part, uint32_t zaddr, int ms,
                                                 T (&acc)[NJ][RPL]) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(3))) const VT* lds_vt;
  constexpr int EW = sizeof(T) == 8 ? 4 : 2;
  // a + s x: an add when the sign is in the staged value
  auto madd = [](T x, T s, T a) -> T {
    if constexpr (NEG) {
      (void)s;
      return a + x;
    } else {
      return fma(x, s, a);
    }
  };
  auto entry = [&](int e, uint32_t& addr, T& sgn) {
    if constexpr (NEG) {
      addr = E[e] ^ lane_part;
      sgn = T(1);
    } else if constexpr (PACK) {
      const uint32_t w = E[e];
      addr = (w & 0x7fffffffu) ^ lane_part;
      if constexpr (sizeof(T) == 8)
        sgn = __builtin_bit_cast(T, (uint64_t)((w & 0x80000000u) | 0x3ff00000u) << 32);
      else
        sgn = __builtin_bit_cast(T, (w & 0x80000000u) | 0x3f800000u);
    } else if constexpr (EW == 4) {
      const u4 a = *(const u4*)&E[e * 4];
      addr = a[0] ^ lane_part;
      sgn = __builtin_bit_cast(T, ((uint64_t)a[3] << 32) | a[2]);
    } else {
      const uint32_t* p = &E[e * 2];
      addr = p[0] ^ lane_part;
      sgn = __builtin_bit_cast(T, p[1]);
    }
  };
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int e0 = (int)__builtin_amdgcn_readlane(bnd, jj) - ebase;
    const int e1 = (jj + 1 < NJ ? (int)__builtin_amdgcn_readlane(bnd, jj + 1)
                                : (int)__builtin_amdgcn_readfirstlane(bndN)) - ebase;
    // slots [e0 + m0, e0 + m0 + 4), masked past the bucket's end
    auto four = [&](int m0) {
      uint32_t ad[4];
      T sg[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        entry(e0 + m0 + q, ad[q], sg[q]);
        ad[q] = e0 + m0 + q < e1 ? ad[q] : zaddr;
      }
      VT x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = *(lds_vt)(uintptr_t)ad[q];
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        T a = acc[jj][r];
#pragma unroll
        for (int q = 0; q < 4; ++q) a = madd(((const T*)&x[q])[r], sg[q], a);
        acc[jj][r] = a;
      }
    };
    four(0);
    if (ms > 4) four(4);  // buckets of about eight entries: eight straight-line slots
    int e = e0 + ms;
    for (; e + 1 < e1; e += 2) {
      uint32_t a0, a1;
      T s0, s1;
      entry(e, a0, s0);
      entry(e + 1, a1, s1);
      const VT x0 = *(lds_vt)(uintptr_t)a0, x1 = *(lds_vt)(uintptr_t)a1;
#pragma unroll
      for (int r = 0; r < RPL; ++r)
        acc[jj][r] = madd(((const T*)&x1)[r], s1, madd(((const T*)&x0)[r], s0, acc[jj][r]));
    }
    if (e < e1) {  // odd bucket length
      uint32_t a0;
      T s0;
      entry(e, a0, s0);
      const VT x0 = *(lds_vt)(uintptr_t)a0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[jj][r] = madd(((const T*)&x0)[r], s0, acc[jj][r]);
    }
  }
}

// The same gather with the straight-line slot count MS (2, 4 or 8) fixed at
// compile time, for kernels instantiated per bucket-length class.
template <typename T, int NJ, int RPL, typename VT, int MS>
__device__ __forceinline__ void gather_chunk_lds_ms(const uint32_t* E, int ebase, uint32_t bnd, uint32_t bndN,
                                                    uint32_t lane_part, uint32_t zaddr, T (&acc)[NJ][RPL]) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(3))) const VT* lds_vt;
  constexpr int EW = sizeof(T) == 8 ? 4 : 2;
  constexpr int NQ = MS < 4 ? MS : 4;
  auto entry = [&](int e, uint32_t& addr, T& sgn) {
    if constexpr (EW == 4) {
      const u4 a = *(const u4*)&E[e * 4];
      addr = a[0] ^ lane_part;
      sgn = __builtin_bit_cast(T, ((uint64_t)a[3] << 32) | a[2]);
    } else {
      const uint32_t* p = &E[e * 2];
      addr = p[0] ^ lane_part;
      sgn = __builtin_bit_cast(T, p[1]);
    }
  };
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int e0 = (int)__builtin_amdgcn_readlane(bnd, jj) - ebase;
    const int e1 = (jj + 1 < NJ ? (int)__builtin_amdgcn_readlane(bnd, jj + 1)
                                : (int)__builtin_amdgcn_readfirstlane(bndN)) - ebase;
#pragma unroll
    for (int m0 = 0; m0 < MS; m0 += NQ) {
      uint32_t ad[NQ];
      T sg[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        entry(e0 + m0 + q, ad[q], sg[q]);
        ad[q] = e0 + m0 + q < e1 ? ad[q] : zaddr;
      }
      VT x[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) x[q] = *(lds_vt)(uintptr_t)ad[q];
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        T a = acc[jj][r];
#pragma unroll
        for (int q = 0; q < NQ; ++q) a = fma(((const T*)&x[q])[r], sg[q], a);
        acc[jj][r] = a;
      }
    }
    int e = e0 + MS;
    for (; e + 1 < e1; e += 2) {
      uint32_t a0, a1;
      T s0, s1;
      entry(e, a0, s0);
      entry(e + 1, a1, s1);
      const VT x0 = *(lds_vt)(uintptr_t)a0, x1 = *(lds_vt)(uintptr_t)a1;
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[jj][r] = fma(((const T*)&x1)[r], s1, fma(((const T*)&x0)[r], s0, acc[jj][r]));
    }
    if (e < e1) {  // odd bucket length
      uint32_t a0;
      T s0;
      entry(e, a0, s0);
      const VT x0 = *(lds_vt)(uintptr_t)a0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[jj][r] = fma(((const T*)&x0)[r], s0, acc[jj][r]);
    }
  }
}


// Gather with one 32-bit word per staged entry: the LDS address of the source
// row with the sign in bit 31 (RPL = 1).  Two adjacent entries come in one
// ds_read2_b32; the sign is applied by flipping the sign bit of the value.
template <typename T>
__device__ __forceinline__ T flip_sign(T v, uint32_t w) {
  if constexpr (sizeof(T) == 8) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    u ^= (uint64_t)(w & 0x80000000u) << 32;
    return __builtin_bit_cast(T, u);
  } else {
    return __builtin_bit_cast(T, __builtin_bit_cast(uint32_t, v) ^ (w & 0x80000000u));
  }
}

template <typename T, int NJ, int MS>
__device__ __forceinline__ void gather_chunk_e32(const uint32_t* E, int ebase, uint32_t bnd, uint32_t bndN,
                                                 uint32_t lane_part, uint32_t zaddr, T (&acc)[NJ][1]) {
  typedef __attribute__((address_space(3))) const T* lds_t;
  static_assert(MS % 2 == 0, "slots come in pairs");
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int e0 = (int)__builtin_amdgcn_readlane(bnd, jj) - ebase;
    const int e1 = (jj + 1 < NJ ? (int)__builtin_amdgcn_readlane(bnd, jj + 1)
                                : (int)__builtin_amdgcn_readfirstlane(bndN)) - ebase;
    uint32_t w[MS];
#pragma unroll
    for (int q = 0; q < MS; ++q) w[q] = E[e0 + q];
    T x[MS];
#pragma unroll
    for (int q = 0; q < MS; ++q) {
      const uint32_t ad = e0 + q < e1 ? ((w[q] & 0x7fffffffu) ^ lane_part) : zaddr;
      x[q] = *(lds_t)(uintptr_t)ad;
    }
    T a = acc[jj][0];
#pragma unroll
    for (int q = 0; q < MS; ++q) a += flip_sign(x[q], w[q]);
    int e = e0 + MS;
    for (; e + 1 < e1; e += 2) {
      const uint32_t w0 = E[e], w1 = E[e + 1];
      const T x0 = *(lds_t)(uintptr_t)((w0 & 0x7fffffffu) ^ lane_part);
      const T x1 = *(lds_t)(uintptr_t)((w1 & 0x7fffffffu) ^ lane_part);
      a += flip_sign(x0, w0);  // one add at a time: the order of the FMA gathers
      a += flip_sign(x1, w1);
    }
    if (e < e1) {  // odd overflow
      const uint32_t w0 = E[e];
      a += flip_sign(*(lds_t)(uintptr_t)((w0 & 0x7fffffffu) ^ lane_part), w0);
    }
    acc[jj][0] = a;
  }
}


// The same with RPL rows per lane (VT holds RPL consecutive elements).
template <typename T, int NJ, int RPL, typename VT, int MS>
__device__ __forceinline__ void gather_chunk_e32_rpl(const uint32_t* E, int ebase, uint32_t bnd, uint32_t bndN,
                                                     uint32_t lane_part, uint32_t zaddr, T (&acc)[NJ][RPL]) {
  typedef __attribute__((address_space(3))) const VT* lds_vt;
  auto add = [&](T(&a)[RPL], const VT& x, uint32_t w) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) a[r] += flip_sign(((const T*)&x)[r], w);
  };
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int e0 = (int)__builtin_amdgcn_readlane(bnd, jj) - ebase;
    const int e1 = (jj + 1 < NJ ? (int)__builtin_amdgcn_readlane(bnd, jj + 1)
                                : (int)__builtin_amdgcn_readfirstlane(bndN)) - ebase;
    uint32_t w[MS];
#pragma unroll
    for (int q = 0; q < MS; ++q) w[q] = E[e0 + q];
    VT x[MS];
#pragma unroll
    for (int q = 0; q < MS; ++q) {
      const uint32_t ad = e0 + q < e1 ? ((w[q] & 0x7fffffffu) ^ lane_part) : zaddr;
      x[q] = *(lds_vt)(uintptr_t)ad;
    }
#pragma unroll
    for (int q = 0; q < MS; ++q) add(acc[jj], x[q], w[q]);
    int e = e0 + MS;
    for (; e + 1 < e1; e += 2) {
      const uint32_t w0 = E[e], w1 = E[e + 1];
      const VT x0 = *(lds_vt)(uintptr_t)((w0 & 0x7fffffffu) ^ lane_part);
      const VT x1 = *(lds_vt)(uintptr_t)((w1 & 0x7fffffffu) ^ lane_part);
      add(acc[jj], x0, w0);
      add(acc[jj], x1, w1);
    }
    if (e < e1) {
      const uint32_t w0 = E[e];
      const VT x0 = *(lds_vt)(uintptr_t)((w0 & 0x7fffffffu) ^ lane_part);
      add(acc[jj], x0, w0);
    }
  }
}

// Bucket gather for one-word entries: the LDS address of the source row with
// the sign in bit 31 (SGN; FP64 one row per lane, FP32 RPL rows), or, for FP32
// with negated tile rows (!SGN), the address of the source row or of its
// negated copy.  The wave first reads the bucket of each of a group of PG
// columns into a VGPR window (lane k holds the bucket's entry k, lanes past the
// end the null entry, i.e. the zero row), all windows of the group before any
// value: a slot is then a v_readlane of a uniform word (its sign built by
// scalar operations), and the value reads of all columns of the group depend
// on no further LDS read, so they overlap across columns (gather_chunk_lds
// reads the entries of a column right before its values, one dependent pair of
// LDS round trips per column).  An entry costs one LDS value read; a window
// costs one 4-byte read per column instead of a broadcast read per entry.
// NS straight-line slots per bucket (4, or about the mean bucket length), then
// the rest in pairs (the lane past an odd end holds the null entry); with TWO
// the straight-line slots of every column of the group come first, so that the
// value reads of the group are in flight together (this costs NS PG RPL VGPRs).  Buckets of more than 64 entries (a
// chunk of more than 64 sources) take more windows.  The additions are those of gather_chunk_lds in the same order
// (a + (+-1) x is exact in the product, so fma and add agree).
template <typename T, int NJ, int RPL, typename VT, int PG, bool SGN, bool TWO, int NS = 4>
__device__ __forceinline__ void gather_chunk_lds_win(const uint32_t* E, int ebase, uint32_t bnd, uint32_t bndN,
                                                     uint32_t lane_part, uint32_t zaddr, T (&acc)[NJ][RPL]) {
  typedef __attribute__((address_space(3))) const VT* lds_vt;
  static_assert(NJ % PG == 0, "whole column groups");
  const uint32_t zword = __builtin_amdgcn_readfirstlane(zaddr ^ lane_part);  // the zero row, sign +
  const int lane = (int)__lane_id();
  // slot of the uniform entry word w: this lane's staged values, signed
  auto slot = [&](T(&a)[RPL], uint32_t w) {
    if constexpr (SGN) {
      const uint32_t ad = __builtin_amdgcn_bitop3_b32(w, lane_part, 0x7fffffffu, 0x6c);  // (w & 0x7fffffff) ^ lane_part
      const VT x = *(lds_vt)(uintptr_t)ad;
      T sg;  // +-1 from bit 31 of w
      if constexpr (sizeof(T) == 8)
        sg = __builtin_bit_cast(T, (uint64_t)((w & 0x80000000u) | 0x3ff00000u) << 32);
      else
        sg = __builtin_bit_cast(T, (w & 0x80000000u) | 0x3f800000u);
#pragma unroll
      for (int r = 0; r < RPL; ++r) a[r] = fma(((const T*)&x)[r], sg, a[r]);
    } else {
      const VT x = *(lds_vt)(uintptr_t)(w ^ lane_part);
#pragma unroll
      for (int r = 0; r < RPL; ++r) a[r] += ((const T*)&x)[r];
    }
  };
#pragma unroll
  for (int g0 = 0; g0 < NJ; g0 += PG) {
    uint32_t win[PG];
    int e0s[PG], cnts[PG];
#pragma unroll
    for (int j = 0; j < PG; ++j) {
      const int jj = g0 + j;
      e0s[j] = (int)__builtin_amdgcn_readlane(bnd, jj) - ebase;
      const int e1 = (jj + 1 < NJ ? (int)__builtin_amdgcn_readlane(bnd, jj + 1)
                                  : (int)__builtin_amdgcn_readfirstlane(bndN)) - ebase;
      cnts[j] = e1 - e0s[j];
      win[j] = lane < cnts[j] ? E[e0s[j] + lane] : zword;
    }
    // TWO: the four straight-line slots of every column of the group, then the
    // rest of the longer buckets (per column the same order of additions)
    if constexpr (TWO) {
#pragma unroll
      for (int j = 0; j < PG; ++j) {
#pragma unroll
        for (int q = 0; q < NS; ++q) slot(acc[g0 + j], __builtin_amdgcn_readlane(win[j], q));
      }
    }
#pragma unroll
    for (int j = 0; j < PG; ++j) {
      const int cnt = cnts[j];
      T(&a)[RPL] = acc[g0 + j];
      if constexpr (!TWO) {
#pragma unroll
        for (int q = 0; q < NS; ++q) slot(a, __builtin_amdgcn_readlane(win[j], q));
      }
      if (cnt > NS) {
        const int lim = cnt < 64 ? cnt : 64;
        for (int q = NS; q < lim; q += 2) {
          slot(a, __builtin_amdgcn_readlane(win[j], q));
          slot(a, __builtin_amdgcn_readlane(win[j], q + 1));
        }
        for (int base = 64; base < cnt; base += 64) {  // buckets of more than 64 entries
          const int c2 = cnt - base;
          const uint32_t w2 = lane < c2 ? E[e0s[j] + base + lane] : zword;
          const int l2 = c2 < 64 ? c2 : 64;
          for (int q = 0; q < l2; q += 2) {
            slot(a, __builtin_amdgcn_readlane(w2, q));
            slot(a, __builtin_amdgcn_readlane(w2, q + 1));
          }
        }
      }
    }
  }
}

}  // namespace sk

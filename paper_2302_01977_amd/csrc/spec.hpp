// Operator specification: every entry of R is a pure function of (seed, counter).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the 64-bit seed
// (low word first).  Counters, all indices 0-based:
//   SJLT offset, row k, chunk c, block b : (1, b, k, c >> 2), word c & 3,
//                                          offset = mulhi32(word, w_b / alpha)
//   SJLT sign,   row k, chunk c, block b : (2, b, k, 0), word 0, bit c (1 = negative)
//   SRHT diagonal D_k                    : (3, 0, k, 0), word 0, bit 0 (1 = -1)
//   SRHT sample mu_j, global column j    : (4, 0, j >> 2, 0), word j & 3,
//                                          mu = mulhi32(word, nu), nu = 2^ceil(log2 n)
//   Gaussian g_{k,j}, global column j    : (5, j, k, 0), words 0 and 1, Box-Muller
//                                          in FP64, rounded to bfloat16 (RNE).
//   SJLT graph draw, row k, step c, blk b: (6, b, k, c >> 2), word c & 3,
//                                          t_c = mulhi32(word, w_b - alpha + c + 1)
// Compiled for host and device so that the library's host queries
// (sketch_get_rows) and its kernels evaluate the same definition.
#pragma once
#include <stdint.h>
#include <math.h>
#include <string.h>

#ifdef __HIPCC__
#define SK_HD __host__ __device__ __forceinline__
#else
#define SK_HD inline
#endif

namespace sk {

struct U4 {
  uint32_t v[4];
};

SK_HD U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  U4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

SK_HD uint32_t mulhi(uint32_t u, uint32_t r) { return (uint32_t)(((uint64_t)u * r) >> 32); }

struct Key {
  uint32_t k0, k1;
};
SK_HD Key key_of(uint64_t seed) {
  Key k;
  k.k0 = (uint32_t)seed;
  k.k1 = (uint32_t)(seed >> 32);
  return k;
}

// SJLT (block construction): column inside the block and sign of the nonzero of
// row k in chunk c.  Returns (col << 1) | negative.
SK_HD uint32_t sjlt_code(Key key, uint32_t block, uint32_t k, uint32_t c, uint32_t wc) {
  const U4 o = philox(1u, block, k, c >> 2, key.k0, key.k1);
  const uint32_t off = mulhi(o.v[c & 3], wc);
  const U4 s = philox(2u, block, k, 0u, key.k0, key.k1);
  return ((c * wc + off) << 1) | ((s.v[0] >> c) & 1u);
}

// SJLT (graph construction, section 2.4.3): the alpha distinct columns of row
// k of a block of width w, as codes (col << 1) | negative in code[0..alpha).
// A uniformly random alpha-subset by Floyd's sampling: step c draws t uniform
// in [0, j], j = w - alpha + c, and takes t unless an earlier step took it,
// else j.  The signs use the block construction's counter (2, b, k, 0), bit c.
SK_HD void sjlt_graph_codes(Key key, uint32_t block, uint32_t k, int alpha, uint32_t w, uint32_t* code) {
  const uint32_t sbits = philox(2u, block, k, 0u, key.k0, key.k1).v[0];
  U4 o = philox(6u, block, k, 0u, key.k0, key.k1);
  for (int c = 0; c < alpha; ++c) {
    if (c > 0 && (c & 3) == 0) o = philox(6u, block, k, (uint32_t)(c >> 2), key.k0, key.k1);
    const uint32_t j = w - (uint32_t)alpha + (uint32_t)c;
    uint32_t t = mulhi(o.v[c & 3], j + 1u);
    for (int q = 0; q < c; ++q)
      if ((code[q] >> 1) == t) t = j;  // j itself is never taken before step c
    code[c] = (t << 1) | ((sbits >> c) & 1u);
  }
}

SK_HD int srht_neg(Key key, uint32_t k) {
  return (int)(philox(3u, 0u, k, 0u, key.k0, key.k1).v[0] & 1u);
}

// Hadamard dimension of an SRHT on n rows: nu = 2^ceil(log2 n) (section 7.2:
// for n not a power of two only the first n rows of H_nu are used, D padded
// with zeros).
SK_HD uint32_t srht_nu(int64_t n) {
  uint32_t nu = 1;
  while ((int64_t)nu < n) nu <<= 1;
  return nu;
}

SK_HD uint32_t srht_mu(Key key, uint32_t j, uint32_t nu) {
  const U4 o = philox(4u, 0u, j >> 2, 0u, key.k0, key.k1);
  return mulhi(o.v[j & 3], nu);
}

// Round a finite FP64 value to the nearest bfloat16 value (ties to even); the
// result is returned as FP64 and is exact in bf16, fp32 and fp64.
SK_HD double bf16_rne(double z) {
  uint64_t b;
  memcpy(&b, &z, 8);
  const uint64_t lsb = (b >> 45) & 1u;
  b += 0x00000FFFFFFFFFFFull + lsb;
  b &= ~((1ull << 45) - 1ull);
  memcpy(&z, &b, 8);
  return z;
}

SK_HD double gauss_raw(Key key, uint32_t k, uint32_t j) {
  const U4 o = philox(5u, j, k, 0u, key.k0, key.k1);
  const double u1 = ((double)o.v[0] + 0.5) * 0x1p-32;
  const double u2 = ((double)o.v[1] + 0.5) * 0x1p-32;
  const double z = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2);
  return bf16_rne(z);
}

SK_HD uint16_t bf16_bits_of_grid_value(double g) {
  const float f = (float)g;  // exact: g is on the bf16 grid
  uint32_t u;
  memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}

SK_HD int popc32(uint32_t x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __popc(x);
#else
  return __builtin_popcount(x);
#endif
}

}  // namespace sk

// SJLT sketch of a stored, column-major A: the per-workgroup tile routine shared
// by the per-pass and the batched kernels.
//
// SJLT sketch of a stored, column-major A (section 6.3 computes A R by an outer
// product over the rows of R and A^* R by inner products with the columns of R).
//
// GPU formulation: a hashed gather.  A workgroup owns TL = 64 * RPL "lanes"
// (rows of A for S = A R, columns of A for S' = A^T R; RPL consecutive lanes per
// thread) and walks the sources (columns of A for S, rows for S') in chunks of
// KC.  Each chunk is staged once in LDS; it is loaded with coalesced 16-byte
// accesses into registers one chunk ahead, so HBM traffic overlaps the gather.
// Every wave owns NJ output columns; for each of them it adds or subtracts the
// staged sources listed in that column's bucket for the chunk.  Bucket entries
// are wave-uniform, so each LDS read is a contiguous access of RPL elements per
// lane and the sign is folded into an FMA with a uniform +-1.  Accumulators stay
// in VGPRs; the 1/sqrt(alpha) scale is applied once at the end, as in the paper.
// KC is chosen per operator so that a bucket holds about four entries per chunk.
// When the lane tiles cannot fill the chip the source range is split and the
// partial sums are reduced in a fixed order (deterministic, no atomics).
//
// S' stages a transposed tile: each thread loads VECN x VECN blocks (VECN
// sources of VECN columns, one 16-byte load per column), transposes them in
// registers and writes 16-byte chunks whose position within the tile row is
// XOR-swizzled by the source index; both the writes and the per-lane reads are
// then free of bank conflicts.
#pragma once
#include <algorithm>
#include <type_traits>

#include "gather.hpp"
#include "internal.hpp"

namespace sk {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// 16-byte global load at a 4-byte aligned address (lda may be odd)
__device__ __forceinline__ u32x4 ld16(const void* p) {
  u32x4 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}

template <typename T, int N>
struct VecT;
template <>
struct VecT<float, 1> {
  typedef float type;
};
template <>
struct VecT<float, 2> {
  typedef f32x2 type;
};
template <>
struct VecT<float, 4> {
  typedef f32x4 type;
};
template <>
struct VecT<double, 1> {
  typedef double type;
};
template <>
struct VecT<double, 2> {
  typedef f64x2 type;
};

// One workgroup's tile: lanes [l0, l0 + TL) against the sources of chunks
// [t0, t1), for the NJ columns of this wave's group.  The caller resolves the
// wave's group: `active`, its bucket table row pointer `ptr` (column jb of the
// block, rows of length prow), the block's entries `ent`, the block's position
// `blk` among the staged entry regions and this thread's staging pointers
// eptr[2] (null when the thread stages nothing); dst points at the group's
// first output column (leading dimension ldd), scaled by sc.
// NEG (FP32 with staged entries): the tile also holds the negated sources in
// rows KCK + 1 .. 2 KCK, and an entry is the address of the source row or of
// its negated copy, so the gather adds without a sign (the wide passes are
// bound by LDS bytes).
template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK, bool LDSE, bool NEG = false>
__device__ __forceinline__ void sjlt_tile(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, int64_t l0,
                                          int t0, int t1, bool active, const int32_t* __restrict__ ptr,
                                          int64_t prow, const int32_t* __restrict__ ent, int blk,
                                          const uint32_t* eptr0, const uint32_t* eptr1, int kcap, int epad,
                                          int ms, T* __restrict__ dst, int64_t ldd, T sc) {
  constexpr int SZ = sizeof(T);
  constexpr int VECN = 16 / SZ;  // elements per 16-byte vector
  constexpr int TL = 64 * RPL;   // lanes (rows of A, or columns of A for S') per workgroup
  constexpr int NTHR = NW * 64;
  constexpr int NV = KCK * TL / (NTHR * VECN);  // 16-byte vectors per thread per chunk
  constexpr int NRB = KCK / VECN;               // S': row blocks per chunk
  static_assert((KCK * TL) % (NTHR * VECN) == 0, "tile must split evenly");
  static_assert(!TRANS || NV % VECN == 0, "S' staging moves whole VECN x VECN blocks");
  static_assert(RPL <= VECN, "a lane reads at most one 16-byte chunk");
  typedef typename VecT<T, RPL>::type VT;

  // Dynamic LDS: the staged tile, whose extra source slot KCK holds zeros (the
  // source of null entries), then (LDSE) the chunk's bucket entries, one word
  // each: the entry's LDS address in the tile with its sign in bit 31 (PACK),
  // or with NEG the address of the source row or of its negated copy.
  constexpr int NSLOT = NEG ? 2 * KCK + 1 : KCK + 1;
  constexpr bool PACK = !NEG;
  static_assert(!NEG || (LDSE && SZ == 4), "negated rows: FP32 with staged entries");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* tile = (T*)smem;
  uint32_t* ents = (uint32_t*)(smem + NSLOT * TL * SZ);
  // LDS address of the tile.  The kernels have no static LDS, so the dynamic
  // block starts at 0 and the tile base is a multiple of the row stride TL * SZ:
  // base + row offset + swizzle key combine with the lane part by XOR.
  const uint32_t tile_lds = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char*)smem;
  const int tid = threadIdx.x;
  const int lane = tid & 63;

  // LDSE staging of entries: thread tid moves entries [4 tid, 4 tid + 4) and
  // [4 (tid + NTHR), ...) of the concatenated chunk regions of the blocks
  const int q0[2] = {tid * 4, (tid + NTHR) * 4};
  const uint32_t* __restrict__ eptr[2] = {eptr0, eptr1};
  u32x4 ebuf[2] = {u32x4{0u, 0u, 0u, 0u}, u32x4{0u, 0u, 0u, 0u}};
  uint32_t bnd = 0, bndN = 0, bnd_nx = 0, bndN_nx = 0;
  for (int e = tid; e < TL; e += NTHR) tile[KCK * TL + e] = T(0);
  // The straight-line slots of the last bucket may read up to 7 entries past
  // the staged regions (entries epad..epad+7); they hold the null entry (zero
  // row, +) instead of whatever the LDS held before.
  if constexpr (LDSE) {
    if (tid < 8) ents[epad + tid] = tile_lds + (uint32_t)(KCK * TL * SZ);
  }
  // ---------------------------------------------------------------- staging
  u32x4 buf[NV];
  // Per-thread geometry of the staged tile.  NTHR * VECN is a multiple of TL
  // (S) and NTHR a multiple of NRB (S'), so each thread keeps the same row (S)
  // or row block (S') in every vector and only a uniform column step changes.
  constexpr int CSTEP = NTHR * VECN / TL;   // S: columns advanced per vector
  constexpr int CBSTEP = NTHR / NRB;        // S': column blocks advanced per block
  static_assert((NTHR * VECN) % TL == 0 && NTHR % NRB == 0, "staging geometry");
  const int my_row = (tid * VECN) % TL;           // S: row inside the tile
  const int my_col = (tid * VECN) / TL;           // S: first column
  const int my_rb = tid % NRB;                    // S': row block
  const int my_cb = tid / NRB;                    // S': first column block
  auto vec_rc = [&](int it, int64_t& gr, int64_t& gc, int64_t k0) {
    if (!TRANS) {
      gr = l0 + my_row;
      gc = k0 + my_col + (int64_t)it * CSTEP;
    } else {
      gr = k0 + (int64_t)my_rb * VECN;
      gc = l0 + ((int64_t)my_cb + (int64_t)(it / VECN) * CBSTEP) * VECN + (it % VECN);
    }
  };
  auto load_meta = [&](int t) {
    if constexpr (LDSE) {
#pragma unroll
      for (int h = 0; h < 2; ++h)  // whole regions: null entries past the end
        if (eptr[h]) ebuf[h] = *(const u32x4*)(eptr[h] + (int64_t)t * kcap);
      if (active) {
        const int32_t* pb = ptr + (int64_t)t * prow;
        bnd_nx = lane < NJ ? (uint32_t)pb[lane] : 0u;
        bndN_nx = (uint32_t)pb[NJ];
      }
    }
  };
  // FULL: every chunk of the tile is known to lie inside A
  auto load_chunk = [&](int t, auto fullc) __attribute__((always_inline)) {
    load_meta(t);
    const int64_t k0 = (int64_t)t * KCK;
    const bool full = decltype(fullc)::value || (l0 + TL <= L && k0 + KCK <= K);  // uniform
    if (full) {
      int64_t gr, gc;
      vec_rc(0, gr, gc, k0);
      const T* base = A + gr + gc * lda;
#pragma unroll
      for (int it = 0; it < NV; ++it) {
        const int64_t off = TRANS ? ((int64_t)(it / VECN) * CBSTEP * VECN + (it % VECN)) * lda
                                  : (int64_t)it * CSTEP * lda;
        buf[it] = ld16(base + off);
      }
    } else {
#pragma unroll
      for (int it = 0; it < NV; ++it) {
        int64_t gr, gc;
        vec_rc(it, gr, gc, k0);
        const int64_t rlim = TRANS ? K : L;
        const bool cok = TRANS ? gc < L : gc < K;
        const T* p = A + gr + gc * lda;
        T v[VECN];
#pragma unroll
        for (int q = 0; q < VECN; ++q) v[q] = (cok && gr + q < rlim) ? p[q] : T(0);
        __builtin_memcpy(&buf[it], v, 16);
      }
    }
  };
  auto store_chunk = [&]() {
    if constexpr (LDSE) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (!eptr[h]) continue;
        uint32_t ad[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t src = ebuf[h][q] >> 1;
          // NEG: negative entries address the negated copy (null entries, source
          // KCK, always the zero row)
          const uint32_t row = NEG && (ebuf[h][q] & 1u) && src < (uint32_t)KCK ? src + KCK + 1 : src;
          ad[q] = (tile_lds + row * (uint32_t)(TL * SZ)) | (TRANS ? ((src / VECN) & 15u) * 16u : 0u);
          if constexpr (PACK) ad[q] |= ebuf[h][q] << 31;
        }
        *(u32x4*)&ents[q0[h]] = u32x4{ad[0], ad[1], ad[2], ad[3]};
      }
      bnd = bnd_nx;
      bndN = bndN_nx;
    }
    if (!TRANS) {
#pragma unroll
      for (int it = 0; it < NV; ++it) {
        *(u32x4*)(&tile[(my_col + it * CSTEP) * TL + my_row]) = buf[it];
        if constexpr (NEG)
          *(u32x4*)(&tile[(KCK + 1 + my_col + it * CSTEP) * TL + my_row]) =
              buf[it] ^ u32x4{0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u};
      }
    } else {
#pragma unroll
      for (int ib = 0; ib < NV / VECN; ++ib) {
        const int cb = my_cb + ib * CBSTEP;
        const int pos = (cb ^ (my_rb & 15)) * VECN;
        T blkv[VECN][VECN];  // [column][source]
#pragma unroll
        for (int j = 0; j < VECN; ++j) __builtin_memcpy(blkv[j], &buf[ib * VECN + j], 16);
#pragma unroll
        for (int i = 0; i < VECN; ++i) {
          T rowv[VECN];
#pragma unroll
          for (int j = 0; j < VECN; ++j) rowv[j] = blkv[j][i];
          __builtin_memcpy(&tile[(my_rb * VECN + i) * TL + pos], rowv, 16);
          if constexpr (NEG) {
#pragma unroll
            for (int j = 0; j < VECN; ++j) rowv[j] = -rowv[j];
            __builtin_memcpy(&tile[(KCK + 1 + my_rb * VECN + i) * TL + pos], rowv, 16);
          }
        }
      }
    }
  };

  T acc[NJ][RPL];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
    for (int r = 0; r < RPL; ++r) acc[jj][r] = T(0);

  // per-lane part of the LDS read address (bytes)
  const int lane_elem = lane * RPL;
  const uint32_t lane_q16 = (uint32_t)(lane_elem / VECN) * 16u;  // S': 16-byte chunk before the swizzle
  const uint32_t lane_in = (uint32_t)(lane_elem % VECN) * SZ;     // S': offset inside the chunk
  const uint32_t lane_off = (uint32_t)lane_elem * SZ;             // S
  // LDSE: an entry's address is its staged word XOR this lane's part (the
  // source's row offset and the S' swizzle key occupy disjoint bits)
  const uint32_t lane_part = TRANS ? (lane_q16 | lane_in) : lane_off;
  const uint32_t zaddr = (tile_lds + (uint32_t)(KCK * TL * SZ)) ^ lane_part;  // this lane's zero of slot KCK
  const char* tbase = (const char*)tile;

  auto LD = [&](int v) -> VT {
    const uint32_t src = (uint32_t)v >> 1;
    uint32_t a;
    if (!TRANS) {
      a = src * (uint32_t)(TL * SZ) + lane_off;
    } else {
      const uint32_t key16 = ((src / VECN) & 15u) * 16u;
      a = src * (uint32_t)(TL * SZ) + ((lane_q16 ^ key16) + lane_in);
    }
    return *(const VT*)(tbase + a);
  };

  // the entry-window gather, windows of 4 columns at a time; FP64 with one row
  // per lane takes the straight-line slots of the 4 columns first (n = 16384
  // step: S 0.473 -> 0.461 ms against 16-column windows; in FP32 the value
  // registers of the group would push the kernels past their VGPR budget)
  constexpr bool WIN = NJ <= 16;
  constexpr int WPG = NJ < 4 ? NJ : 4;
  constexpr bool WTWO = SZ == 8 && RPL == 1;
  auto run = [&](auto fullc) __attribute__((always_inline)) {
    if (t0 < t1) load_chunk(t0, fullc);
    for (int t = t0; t < t1; ++t) {
      __syncthreads();  // the previous chunk is fully consumed
      store_chunk();
      __syncthreads();
      if (t + 1 < t1) load_chunk(t + 1, fullc);  // in flight during the gather below
      if (active) {
        if constexpr (LDSE && WIN)
          gather_chunk_lds_win<T, NJ, RPL, VT, WPG, PACK, WTWO>(ents, (t - blk) * kcap, bnd, bndN, lane_part, zaddr, acc);
        else if constexpr (LDSE)
          gather_chunk_lds<T, NJ, RPL, VT, PACK, NEG>(ents, (t - blk) * kcap, bnd, bndN, lane_part, zaddr, ms, acc);
        else
          gather_chunk<T, NJ, RPL, VT>(ptr + (int64_t)t * prow, ent, LD, acc);
      }
    }
  };
  // S': when no chunk of the tile reaches past A, a loop without the
  // bounds-checked staging.  With both staging forms in one loop the compiler
  // merges their registers after the load and waits there for the loads of
  // the next chunk, so they would not overlap the gather.
  if (TRANS && l0 + TL <= L && (int64_t)t1 * KCK <= K)
    run(std::true_type{});
  else
    run(std::false_type{});

  if (!active) return;
  const int64_t row0 = l0 + lane_elem;
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
#pragma unroll
    for (int r = 0; r < RPL; ++r)
      if (row0 + r < L) dst[row0 + r + (int64_t)jj * ldd] = acc[jj][r] * sc;
  }
}

// dynamic LDS of one workgroup: the tile with its zero slot (and with neg the
// negated rows), then the entries
inline size_t gather_lds_bytes(int esz, int kc, int tl, bool ldse, int nblk, int kcap, bool neg = false) {
  const size_t ew = 4;  // one word per entry
  const size_t rows = neg ? 2 * (size_t)kc + 1 : (size_t)kc + 1;
  // (+8 entries: the straight-line slots of the last bucket may read up to 7 past it)
  return rows * tl * esz + (ldse ? ((size_t)nblk * kcap + 8) * ew : 0);
}

struct GatherCfg {
  int nw, nj, rpl, kc;
  bool ldse;  // bucket entries staged in LDS (else read through the scalar cache)
  bool neg;   // FP32 staged entries of one word with negated tile rows
};

template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK>
struct GatherValid {
  static constexpr int VECN = 16 / (int)sizeof(T);
  static constexpr int NV = KCK * 64 * RPL / (NW * 64 * VECN);
  static constexpr bool value = (KCK * 64 * RPL) % (NW * 64 * VECN) == 0 && NV >= 1 && (!TRANS || NV % VECN == 0) &&
                                RPL <= VECN;
};

// the launch table skips 8-wave variants whose tile does not split evenly
template <typename T, bool TRANS>
inline bool cfg_valid(int nw, int rpl, int kc) {
  const int vecn = 16 / (int)sizeof(T);
  const long tile = (long)kc * 64 * rpl;
  const long per = (long)nw * 64 * vecn;
  if (tile % per) return false;
  const long nv = tile / per;
  return nv >= 1 && (!TRANS || nv % vecn == 0) && rpl <= vecn;
}

}  // namespace sk

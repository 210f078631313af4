// SJLT sketch S = A R of a stored, column-major A with the chunks of A moved
// into LDS by direct-to-LDS loads (global_load_lds_dwordx4): no registers hold
// the next chunk, so more waves fit on a CU and the loads of chunk t + 1 stay in
// flight during the whole gather of chunk t.  The tile and the bucket entries
// are double-buffered in LDS (one barrier per chunk).  The tile layout is the
// column-major one of the register-staged kernel: a source occupies TL
// consecutive elements, so each wave instruction fills one contiguous KB.
// Chunks that reach past the edge of A (last row tile or last source chunk) are
// staged element by element with bounds checks instead.
#include "sjlt_tile.hpp"

namespace sk {

template <typename T, int NW, int NJ, int RPL, int KCK, int MS>
__global__ void __launch_bounds__(NW * 64)
    sjlt_dma_kernel(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, SjltPass pass,
                    T* __restrict__ out, int64_t ldo, T scale, int split, T* __restrict__ part) {
  constexpr int SZ = sizeof(T);
  constexpr int VECN = 16 / SZ;
  constexpr int TL = 64 * RPL;
  constexpr int NTHR = NW * 64;
  constexpr int NSLOT = KCK + 1;
  constexpr int TBYTES = NSLOT * TL * SZ;        // one tile buffer, zero slot included
  constexpr int UNITS = KCK * TL * SZ / 1024;    // 1 KB wave loads per chunk
  static_assert((KCK * TL * SZ) % 1024 == 0, "a chunk is a whole number of KB");
  typedef typename VecT<T, RPL>::type VT;

  extern __shared__ __attribute__((aligned(16))) char smem[];
  // the same block as an LDS-address-space pointer (direct-to-LDS destinations)
  __attribute__((address_space(3))) char* const smem3 = (__attribute__((address_space(3))) char*)smem;
  const uint32_t lds0 = (uint32_t)(uintptr_t)smem3;
  // entries in LDS: one word (address, sign in bit 31), read through entry
  // windows (gather.hpp)
  const int ebytes = (pass.nblk * pass.kcap + 8) * 4;  // one entry buffer (+8 spare)
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * TL;
  const int s = blockIdx.y;
  const int nT = pass.nT;
  const int t0 = (int)(((int64_t)nT * s) / split);
  const int t1 = (int)(((int64_t)nT * (s + 1)) / split);
  const int g = blockIdx.z * NW + wave;
  const bool active = g < pass.ngroups;
  const int blk = active ? pass.grp_blk[g] : 0;
  const int jb = active ? pass.grp_col[g] : 0;
  const int32_t* __restrict__ ptr = pass.ptr[blk] + jb;
  const int64_t prow = pass.wtot[blk] + 1;

  // entry staging (as in the register-staged kernel): thread tid moves entries
  // [4 tid, 4 tid + 4) and [4 (tid + NTHR), ...) of the pass's chunk regions
  const uint32_t* eptr[2] = {nullptr, nullptr};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q0 = (tid + h * NTHR) * 4;
    const int eb = __builtin_amdgcn_readfirstlane(q0 / pass.kcap);
    if (eb < pass.nblk) eptr[h] = (const uint32_t*)pass.ent[eb] + (q0 - eb * pass.kcap);
  }
  u32x4 ebuf[2] = {u32x4{0u, 0u, 0u, 0u}, u32x4{0u, 0u, 0u, 0u}};
  uint32_t bnd = 0, bndN = 0, bnd_nx = 0, bndN_nx = 0;

  auto tile_base = [&](int b) -> uint32_t { return lds0 + (uint32_t)(b * TBYTES); };
  auto ents_of = [&](int b) -> uint32_t* { return (uint32_t*)(smem + 2 * TBYTES + b * ebytes); };
  // zero slot of both buffers
  for (int e = tid; e < TL; e += NTHR) {
    ((T*)smem)[KCK * TL + e] = T(0);
    ((T*)(smem + TBYTES))[KCK * TL + e] = T(0);
  }

  auto load_meta = [&](int t) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (eptr[h]) ebuf[h] = *(const u32x4*)(eptr[h] + (int64_t)t * pass.kcap);
    if (active) {
      const int32_t* pb = ptr + (int64_t)t * prow;
      bnd_nx = lane < NJ ? (uint32_t)pb[lane] : 0u;
      bndN_nx = (uint32_t)pb[NJ];
    }
  };
  // chunk t of A into tile buffer b: 1 KB unit u covers tile bytes [1024 u, 1024 (u + 1))
  auto load_tile = [&](int t, int b) {
    const int64_t k0 = (int64_t)t * KCK;
    const bool full = l0 + TL <= L && k0 + KCK <= K;  // uniform
    char* tb = smem + b * TBYTES;
    for (int u = wave; u < UNITS; u += NW) {
      const int byte = u * 1024 + lane * 16;
      const int src = byte / (TL * SZ);
      const int row = (byte % (TL * SZ)) / SZ;
      const T* gp = A + (l0 + row) + (k0 + src) * lda;
      if (full) {
        // (the builtin takes a non-const pointer; without the cast the host pass
        // silently drops the kernel's launch stub)
        __builtin_amdgcn_global_load_lds((void*)gp, (__attribute__((address_space(3))) void*)(smem3 + b * TBYTES + u * 1024),
                                         16, 0, 0);
      } else {
        T v[VECN];
#pragma unroll
        for (int q = 0; q < VECN; ++q) v[q] = (k0 + src < K && l0 + row + q < L) ? gp[q] : T(0);
        __builtin_memcpy(tb + byte, v, 16);
      }
    }
  };
  auto store_meta = [&](int t, int b) {
    uint32_t* ents = ents_of(b);
    const uint32_t base = tile_base(b);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!eptr[h]) continue;
      const int qb = (tid + h * NTHR) * 4;
      u32x4 wd;
#pragma unroll
      for (int q = 0; q < 4; ++q) wd[q] = (base + (ebuf[h][q] >> 1) * (uint32_t)(TL * SZ)) | (ebuf[h][q] << 31);
      *(u32x4*)&ents[qb] = wd;
    }
    bnd = bnd_nx;
    bndN = bndN_nx;
  };

  T acc[NJ][RPL];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
    for (int r = 0; r < RPL; ++r) acc[jj][r] = T(0);
  const int lane_elem = lane * RPL;
  const uint32_t lane_part = (uint32_t)lane_elem * SZ;
  // this lane's zero of slot KCK in either buffer (buffer bases are multiples of
  // the row stride, so base + row offset and the lane part combine by XOR)
  const uint32_t zaddr0 = (tile_base(0) + (uint32_t)(KCK * TL * SZ)) ^ lane_part;
  const uint32_t zaddr1 = (tile_base(1) + (uint32_t)(KCK * TL * SZ)) ^ lane_part;

  if (t0 < t1) {
    load_meta(t0);
    load_tile(t0, 0);
  }
  for (int t = t0; t < t1; ++t) {
    const int b = (t - t0) & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's tile and meta loads for chunk t
    store_meta(t, b);
    __syncthreads();  // chunk t complete in LDS; every wave is past the gather of t - 1
    if (t + 1 < t1) {
      load_meta(t + 1);
      load_tile(t + 1, b ^ 1);
    }
    if (active)
      gather_chunk_lds_win<T, NJ, RPL, VT, (NJ < 4 ? NJ : 4), true, false, MS>(
          ents_of(b), (t - blk) * pass.kcap, bnd, bndN, lane_part, b ? zaddr1 : zaddr0, acc);
  }

  if (!active) return;
  const int64_t row0 = l0 + lane_elem;
  const int64_t jc = (int64_t)g * NJ;
  T* dst = split > 1 ? part + (int64_t)s * L * ((int64_t)pass.ngroups * NJ) + jc * L : out + jc * ldo;
  const int64_t ldd = split > 1 ? L : ldo;
  const T sc = split > 1 ? T(1) : scale;
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
#pragma unroll
    for (int r = 0; r < RPL; ++r)
      if (row0 + r < L) dst[row0 + r + (int64_t)jj * ldd] = acc[jj][r] * sc;
  }
}

// S' = A^T R with direct-to-LDS loads.  A workgroup owns 64 columns of A (the
// rows of S'); chunk t of column p is KC contiguous elements (KC SZ = 1 KB, one
// wave load), placed at p (KC + 8) elements so that the reads below are free of
// bank conflicts.  Per chunk, waves 0..7 move the tile into rows of sources with
// the 64 columns contiguous, column p at slot p XOR 8 (c mod 8) of row c
// (conflict-free writes), and zero row KC; the bucket entries carry that
// row address, so the gather is the one of the S kernel.
template <typename T, int NW, int NJ, int KCK, int MS>
__global__ void __launch_bounds__(NW * 64)
    sjlt_dma_t_kernel(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, SjltPass pass,
                      T* __restrict__ out, int64_t ldo, T scale, int split, T* __restrict__ part) {
  constexpr int SZ = sizeof(T);
  constexpr int VECN = 16 / SZ;
  constexpr int TL = 64;
  constexpr int NTHR = NW * 64;
  constexpr int CSTR = (KCK + 8) * SZ;   // bytes between the staged columns
  constexpr int TBYTES = TL * CSTR;      // one tile buffer (also holds rows 0..KC of the moved tile)
  constexpr int RB = TL * SZ;            // bytes of one moved row
  constexpr int NH = KCK / 8;
  static_assert(KCK * SZ == 1024, "one column chunk is one 1 KB wave load");
  static_assert((KCK + 1) * RB <= TBYTES, "the moved tile and its zero row fit the buffer");
  static_assert(NW >= 8, "the move uses 8 waves");
  typedef T VT;

  extern __shared__ __attribute__((aligned(16))) char smem[];
  __attribute__((address_space(3))) char* const smem3 = (__attribute__((address_space(3))) char*)smem;
  const uint32_t lds0 = (uint32_t)(uintptr_t)smem3;
  const int ebytes = (pass.nblk * pass.kcap + 8) * 4;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * TL;
  const int s = blockIdx.y;
  const int nT = pass.nT;
  const int t0 = (int)(((int64_t)nT * s) / split);
  const int t1 = (int)(((int64_t)nT * (s + 1)) / split);
  const int g = blockIdx.z * NW + wave;
  const bool active = g < pass.ngroups;
  const int blk = active ? pass.grp_blk[g] : 0;
  const int jb = active ? pass.grp_col[g] : 0;
  const int32_t* __restrict__ ptr = pass.ptr[blk] + jb;
  const int64_t prow = pass.wtot[blk] + 1;

  const uint32_t* eptr[2] = {nullptr, nullptr};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q0 = (tid + h * NTHR) * 4;
    const int eb = __builtin_amdgcn_readfirstlane(q0 / pass.kcap);
    if (eb < pass.nblk) eptr[h] = (const uint32_t*)pass.ent[eb] + (q0 - eb * pass.kcap);
  }
  u32x4 ebuf[2] = {u32x4{0u, 0u, 0u, 0u}, u32x4{0u, 0u, 0u, 0u}};
  uint32_t bnd = 0, bndN = 0, bnd_nx = 0, bndN_nx = 0;

  auto tile_base = [&](int b) -> uint32_t { return lds0 + (uint32_t)(b * TBYTES); };
  auto ents_of = [&](int b) -> uint32_t* { return (uint32_t*)(smem + 2 * TBYTES + b * ebytes); };

  auto load_meta = [&](int t) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (eptr[h]) ebuf[h] = *(const u32x4*)(eptr[h] + (int64_t)t * pass.kcap);
    if (active) {
      const int32_t* pb = ptr + (int64_t)t * prow;
      bnd_nx = lane < NJ ? (uint32_t)pb[lane] : 0u;
      bndN_nx = (uint32_t)pb[NJ];
    }
  };
  auto load_tile = [&](int t, int b) {
    const int64_t k0 = (int64_t)t * KCK;
    const bool full = l0 + TL <= L && k0 + KCK <= K;  // uniform
    for (int p = wave; p < TL; p += NW) {
      const T* gp = A + (k0 + lane * VECN) + (l0 + p) * lda;
      if (full) {
        // (the builtin takes a non-const pointer; without the cast the host pass
        // silently drops the kernel's launch stub)
        __builtin_amdgcn_global_load_lds((void*)gp,
                                         (__attribute__((address_space(3))) void*)(smem3 + b * TBYTES + p * CSTR),
                                         16, 0, 0);
      } else {
        T v[VECN];
#pragma unroll
        for (int q = 0; q < VECN; ++q) v[q] = (k0 + lane * VECN + q < K && l0 + p < L) ? gp[q] : T(0);
        __builtin_memcpy(smem + b * TBYTES + p * CSTR + lane * 16, v, 16);
      }
    }
  };
  // entries as one word: address of the source's moved row, sign in bit 31
  auto store_meta = [&](int b) {
    uint32_t* ents = ents_of(b);
    const uint32_t base = tile_base(b);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!eptr[h]) continue;
      u32x4 wd;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t src = ebuf[h][q] >> 1;
        wd[q] = (base + src * (uint32_t)RB + ((src & 7u) * 8u) * (uint32_t)SZ) | (ebuf[h][q] << 31);
      }
      *(u32x4*)&ents[(tid + h * NTHR) * 4] = wd;
    }
    bnd = bnd_nx;
    bndN = bndN_nx;
  };

  T acc[NJ][1];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) acc[jj][0] = T(0);
  const uint32_t lane_part = (uint32_t)lane * SZ;
  // move role: column tp = 8 wave + lane / 8, sources e + 8 m
  const int tp = 8 * wave + (lane >> 3);
  const int e = lane & 7;

  if (t0 < t1) {
    load_meta(t0);
    load_tile(t0, 0);
  }
  for (int t = t0; t < t1; ++t) {
    const int b = (t - t0) & 1;
    char* const tb = smem + b * TBYTES;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's tile and meta loads for chunk t
    store_meta(b);
    __syncthreads();  // chunk t complete in LDS; every wave is past the gather of t - 1
    if (t + 1 < t1) {
      load_meta(t + 1);
      load_tile(t + 1, b ^ 1);
    }
    T x[NH];
    if (wave < 8) {
#pragma unroll
      for (int m = 0; m < NH; ++m) x[m] = *(const T*)(tb + tp * CSTR + (e + 8 * m) * SZ);
    }
    __syncthreads();  // the staged columns are read
    if (wave < 8) {
#pragma unroll
      for (int m = 0; m < NH; ++m) *(T*)(tb + (e + 8 * m) * RB + ((tp ^ (8 * e)) * SZ)) = x[m];
    }
    if (wave == NW - 1) *(T*)(tb + KCK * RB + lane * SZ) = T(0);  // row KC: masked slots and null entries
    __syncthreads();
    if (active)
      gather_chunk_e32<T, NJ, MS>(ents_of(b), (t - blk) * pass.kcap, bnd, bndN, lane_part,
                                  (tile_base(b) + (uint32_t)(KCK * RB)) ^ lane_part, acc);
  }

  if (!active) return;
  const int64_t row0 = l0 + lane;
  const int64_t jc = (int64_t)g * NJ;
  T* dst = split > 1 ? part + (int64_t)s * L * ((int64_t)pass.ngroups * NJ) + jc * L : out + jc * ldo;
  const int64_t ldd = split > 1 ? L : ldo;
  const T sc = split > 1 ? T(1) : scale;
  if (row0 >= L) return;
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) dst[row0 + (int64_t)jj * ldd] = acc[jj][0] * sc;
}

size_t dma_t_lds_bytes(int esz, int kc, int nblk, int kcap) {
  return 2 * (size_t)64 * (kc + 8) * esz + 2 * ((size_t)nblk * kcap + 8) * 4;
}

template <typename T, int NW, int NJ, int KCK>
static int run_dma_t(Ctx* c, const T* A, int64_t lda, int64_t L, int64_t K, const SjltPass& pass, T* out,
                     int64_t ldo, T scale, int split, T* part, hipStream_t st) {
  dim3 grid((unsigned)((L + 63) / 64), (unsigned)split, (unsigned)((pass.ngroups + NW - 1) / NW));
  const size_t shmem = dma_t_lds_bytes((int)sizeof(T), KCK, pass.nblk, pass.kcap);
  auto kern = pass.ms == 2 ? sjlt_dma_t_kernel<T, NW, NJ, KCK, 2>
                            : pass.ms == 4 ? sjlt_dma_t_kernel<T, NW, NJ, KCK, 4> : sjlt_dma_t_kernel<T, NW, NJ, KCK, 8>;
  static bool attr_set[3] = {false, false, false};
  const int ai = pass.ms == 2 ? 0 : pass.ms == 4 ? 1 : 2;
  if (!attr_set[ai]) {
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_set[ai] = true;
  }
  ProfScope ps(c, "sjlt_gather_t", st);
  kern<<<grid, NW * 64, shmem, st>>>(A, lda, L, K, pass, out, ldo, scale, split, part);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// shapes of the direct-to-LDS S' kernel: returns 1 when (nw, nj, kc) has none
int launch_sjlt_dma_t(Ctx* c, int dtype, int nw, int nj, int kc, const void* A, int64_t lda, int64_t L, int64_t K,
                      const SjltPass& pass, void* out, int64_t ldo, double scale, int split, void* part,
                      hipStream_t st) {
#define SK_DMAT(T_, NW_, NJ_, KC_)                                                                          \
  if (nw == NW_ && nj == NJ_ && kc == KC_)                                                                  \
    return run_dma_t<T_, NW_, NJ_, KC_>(c, (const T_*)A, lda, L, K, pass, (T_*)out, ldo, (T_)scale, split, \
                                        (T_*)part, st);
  if (dtype == SK_F32) {
    SK_DMAT(float, 16, 8, 256) SK_DMAT(float, 16, 4, 256)
  }
#undef SK_DMAT
  return 1;
}

size_t dma_lds_bytes(int esz, int kc, int tl, int nblk, int kcap) {
  return 2 * (size_t)(kc + 1) * tl * esz + 2 * ((size_t)nblk * kcap + 8) * 4;
}

template <typename T, int NW, int NJ, int RPL, int KCK>
static int run_dma(Ctx* c, const T* A, int64_t lda, int64_t L, int64_t K, const SjltPass& pass, T* out,
                   int64_t ldo, T scale, int split, T* part, int gz, hipStream_t st) {
  dim3 grid((unsigned)((L + 64 * RPL - 1) / (64 * RPL)), (unsigned)split, (unsigned)gz);
  const size_t shmem = dma_lds_bytes((int)sizeof(T), KCK, 64 * RPL, pass.nblk, pass.kcap);
  auto kern = pass.ms == 2 ? sjlt_dma_kernel<T, NW, NJ, RPL, KCK, 2>
                            : pass.ms == 4 ? sjlt_dma_kernel<T, NW, NJ, RPL, KCK, 4> : sjlt_dma_kernel<T, NW, NJ, RPL, KCK, 8>;
  static bool attr_set[3] = {false, false, false};
  const int ai = pass.ms == 2 ? 0 : pass.ms == 4 ? 1 : 2;
  if (!attr_set[ai]) {
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_set[ai] = true;
  }
  ProfScope ps(c, "sjlt_gather", st);
  kern<<<grid, NW * 64, shmem, st>>>(A, lda, L, K, pass, out, ldo, scale, split, part);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// shapes with a direct-to-LDS kernel: returns 1 when (nw, nj, rpl, kc) has none
int launch_sjlt_dma(Ctx* c, int dtype, int nw, int nj, int rpl, int kc, const void* A, int64_t lda, int64_t L,
                    int64_t K, const SjltPass& pass, void* out, int64_t ldo, double scale, int split, void* part,
                    int gz, hipStream_t st) {
#define SK_DMA(T_, NW_, NJ_, RPL_, KC_)                                                                       \
  if (nw == NW_ && nj == NJ_ && rpl == RPL_ && kc == KC_)                                                     \
    return run_dma<T_, NW_, NJ_, RPL_, KC_>(c, (const T_*)A, lda, L, K, pass, (T_*)out, ldo, (T_)scale, split, \
                                            (T_*)part, gz, st);
  if (dtype == SK_F64) {
    SK_DMA(double, 16, 16, 1, 128) SK_DMA(double, 8, 32, 1, 128) SK_DMA(double, 8, 16, 1, 128)
    SK_DMA(double, 4, 16, 1, 128) SK_DMA(double, 16, 16, 1, 64) SK_DMA(double, 8, 16, 2, 64)
  } else {
    SK_DMA(float, 16, 16, 1, 256) SK_DMA(float, 8, 32, 1, 256) SK_DMA(float, 16, 16, 2, 128)
    SK_DMA(float, 8, 16, 2, 128) SK_DMA(float, 16, 16, 1, 128)
  }
#undef SK_DMA
  return 1;
}

}  // namespace sk

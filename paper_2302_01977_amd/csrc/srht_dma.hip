// SRHT sketch S = (1/sqrt(w)) A D H P of a stored, column-major A (section 7.1),
// with the chunks of A moved into LDS by direct-to-LDS loads
// (global_load_lds_dwordx4).
//
// Sampled column j picks Hadamard column mu_j (section 7.2, entry
// (-1)^{popcount(k & mu)} with 0-based indices).  Split the source index as
// k = t KC + c and mu_j = hi_j KC + lo_j; the sign factors into
// (-1)^{popcount(t & hi_j)} (-1)^{popcount(c & lo_j)}, so
//     S(i, j) = (1/sqrt(w)) sum_t (-1)^{popcount(t & hi_j)} Y_t(i, lo_j),
//     Y_t(i, .) = KC-point Walsh-Hadamard transform of A(i, t KC + c) D_{t KC + c}.
// A workgroup owns 64 rows of A (one per lane) and walks the chunks t:
//   * chunk t + 1 is in flight to the second LDS buffer (no registers hold it)
//     while chunk t is transformed and gathered;
//   * the transform of chunk t runs in place in LDS in two passes, each a set of
//     butterflies in registers: first over the high log2(KC) - 3 bits of c
//     (applying D, kept as sign bits, on the way), then over the low three bits;
//   * every wave owns NJ sampled columns and adds one LDS value per column and
//     chunk with the sign (-1)^{popcount(t & hi_j)} (wave-uniform).
// Only the w sampled outputs of the last factor are formed, so a chunk costs
// log2(KC) butterflies per element plus w / KC gathered reads.  LDS accesses are
// whole 64-lane rows of one source column: contiguous, free of bank conflicts.
// Sources past n read as zero, which leaves Y at the sampled indices unchanged.
// When the row tiles cannot fill the chip, the chunk range is split across
// workgroups and the partial sums are reduced in a fixed order.
#include "sjlt_tile.hpp"

namespace sk {

template <typename T, int N>
__device__ __forceinline__ void fwht_regs(T* x) {
#pragma unroll
  for (int h = 1; h < N; h <<= 1) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      if (c & h) continue;
      const T a = x[c], b = x[c + h];
      x[c] = a + b;
      x[c + h] = a - b;
    }
  }
}

template <typename T, int NW, int NJ, int KCK>
__global__ void __launch_bounds__(NW * 64)
    srht_dma_kernel(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, const uint32_t* __restrict__ Db,
                    const uint32_t* __restrict__ mu, int64_t col0, int W, T* __restrict__ out, int64_t ldo, T scale,
                    int split, T* __restrict__ part) {
  constexpr int SZ = sizeof(T);
  constexpr int VECN = 16 / SZ;
  constexpr int TL = 64;         // rows of A per workgroup, one per lane
  constexpr int CB = TL * SZ;    // bytes of one source column of the tile
  constexpr int TBYTES = KCK * CB;
  constexpr int UNITS = TBYTES / 1024;  // 1 KB wave loads per chunk
  constexpr int LOGKC = __builtin_ctz(KCK);
  constexpr int NH = KCK / 8;    // elements of the first pass (high bits of c)
  static_assert(KCK >= 16 && (KCK & (KCK - 1)) == 0, "KC is a power of two");
  static_assert(TBYTES % 1024 == 0, "a chunk is a whole number of KB");

  extern __shared__ __attribute__((aligned(16))) char smem[];
  __attribute__((address_space(3))) char* const smem3 = (__attribute__((address_space(3))) char*)smem;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * TL;
  const int s = blockIdx.y;
  const int nT = (int)((K + KCK - 1) / KCK);
  const int t0 = (int)(((int64_t)nT * s) / split);
  const int t1 = (int)(((int64_t)nT * (s + 1)) / split);
  const int jw = (blockIdx.z * NW + wave) * NJ;  // first sampled column of this wave
  const bool active = jw < W;

  // this wave's sampled columns: tile byte offset of lo_j, and hi_j
  uint32_t moff[NJ], mhi[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int j = jw + jj;
    const uint32_t m = (active && j < W) ? mu[col0 + j] : 0u;
    moff[jj] = (m & (KCK - 1)) * CB + lane * SZ;
    mhi[jj] = m >> LOGKC;
  }

  // chunk t of A into tile buffer b: 1 KB unit u covers tile bytes [1024 u, 1024 (u + 1))
  auto load_tile = [&](int t, int b) {
    const int64_t k0 = (int64_t)t * KCK;
    const bool full = l0 + TL <= L && k0 + KCK <= K;  // uniform
    for (int u = wave; u < UNITS; u += NW) {
      const int byte = u * 1024 + lane * 16;
      const int src = byte / CB;
      const int row = (byte % CB) / SZ;
      const T* gp = A + (l0 + row) + (k0 + src) * lda;
      if (full) {
        // (the builtin takes a non-const pointer; without the cast the host pass
        // silently drops the kernel's launch stub)
        __builtin_amdgcn_global_load_lds((void*)gp,
                                         (__attribute__((address_space(3))) void*)(smem3 + b * TBYTES + u * 1024),
                                         16, 0, 0);
      } else {
        T v[VECN];
#pragma unroll
        for (int q = 0; q < VECN; ++q) v[q] = (k0 + src < K && l0 + row + q < L) ? gp[q] : T(0);
        __builtin_memcpy(smem + b * TBYTES + byte, v, 16);
      }
    }
  };

  T acc[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) acc[jj] = T(0);

  if (t0 < t1) load_tile(t0, 0);
  for (int t = t0; t < t1; ++t) {
    const int b = (t - t0) & 1;
    char* const tb = smem + b * TBYTES;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of chunk t
    __syncthreads();                // chunk t complete in LDS; every wave is past the gather of t - 1
    if (t + 1 < t1) load_tile(t + 1, b ^ 1);
    // pass 1: D, then butterflies over the high bits of c (c = u + 8 m); the
    // signs of the chunk are KC / 32 words (sources past n hold zeros in the tile)
    const uint32_t* __restrict__ db = Db + (int64_t)t * (KCK / 32);
    for (int u = wave; u < 8; u += NW) {
      T x[NH];
#pragma unroll
      for (int m = 0; m < NH; ++m) {
        const int c = u + 8 * m;
        const T v = *(const T*)(tb + c * CB + lane * SZ);
        x[m] = (db[c >> 5] >> (c & 31)) & 1u ? -v : v;
      }
      fwht_regs<T, NH>(x);
#pragma unroll
      for (int m = 0; m < NH; ++m) *(T*)(tb + (u + 8 * m) * CB + lane * SZ) = x[m];
    }
    __syncthreads();
    // pass 2: butterflies over the low three bits of c (c = 8 q + e)
    for (int q = wave; q < KCK / 8; q += NW) {
      T y[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) y[e] = *(const T*)(tb + (8 * q + e) * CB + lane * SZ);
      fwht_regs<T, 8>(y);
#pragma unroll
      for (int e = 0; e < 8; ++e) *(T*)(tb + (8 * q + e) * CB + lane * SZ) = y[e];
    }
    __syncthreads();
    // gather the sampled columns of Y_t
    if (active) {
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) {
        const T v = *(const T*)(tb + moff[jj]);
        acc[jj] += (__builtin_popcount((uint32_t)t & mhi[jj]) & 1) ? -v : v;
      }
    }
  }

  const int64_t row = l0 + lane;
  if (!active || row >= L) return;
  T* dst = split > 1 ? part + (int64_t)s * L * W : out;
  const int64_t ldd = split > 1 ? L : ldo;
  const T sc = split > 1 ? T(1) : scale;
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int j = jw + jj;
    if (j < W) dst[row + (int64_t)j * ldd] = acc[jj] * sc;
  }
}

// S' = (1/sqrt(w)) A^T D H P: a workgroup owns 64 columns of A (the rows of S')
// and walks the rows of A in chunks of KC; chunk t of column p is KC contiguous
// elements, one 1 KB direct-to-LDS wave load, placed at p (KC + 8) elements
// (the pad keeps the transform's reads free of bank conflicts).  Per chunk:
//   * thread (p, e) with e = lane mod 8 holds the KC / 8 elements
//     c = e + 8 m of column p: D, butterflies over m in registers, then the
//     three low bits of c across the 8 lanes of e (DPP lane exchanges);
//   * the transformed chunk is written back over the tile as rows of c with
//     the 64 columns contiguous (slot p XOR 8 (c mod 8): conflict-free writes);
//   * every lane (column p) gathers its sampled values from those rows.
template <typename T, int CTRL>
__device__ __forceinline__ T dpp_move(T v) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
  }
}

// DPP controls: quad_perm [1,0,3,2] (lane ^ 1), quad_perm [2,3,0,1] (lane ^ 2),
// row_half_mirror (lane ^ 7 within 8 lanes) then quad_perm [3,2,1,0] (lane ^ 3): lane ^ 4
constexpr int DPP_XOR1 = 0xB1;
constexpr int DPP_XOR2 = 0x4E;
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_XOR3 = 0x1B;

template <typename T, int NW, int NJ, int KCK>
__global__ void __launch_bounds__(NW * 64)
    srht_dma_t_kernel(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, const uint32_t* __restrict__ Db,
                      const uint32_t* __restrict__ mu, int64_t col0, int W, T* __restrict__ out, int64_t ldo,
                      T scale, int split, T* __restrict__ part) {
  constexpr int SZ = sizeof(T);
  constexpr int VECN = 16 / SZ;
  constexpr int TL = 64;                  // columns of A per workgroup, one per lane
  constexpr int CSTR = (KCK + 8) * SZ;    // bytes between the tile's columns
  constexpr int TBYTES = TL * CSTR;
  constexpr int LOGKC = __builtin_ctz(KCK);
  constexpr int NH = KCK / 8;
  static_assert(KCK * SZ == 1024, "one column chunk is one 1 KB wave load");
  static_assert(NW >= 8, "the transform uses 8 waves");

  extern __shared__ __attribute__((aligned(16))) char smem[];
  __attribute__((address_space(3))) char* const smem3 = (__attribute__((address_space(3))) char*)smem;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * TL;
  const int s = blockIdx.y;
  const int nT = (int)((K + KCK - 1) / KCK);
  const int t0 = (int)(((int64_t)nT * s) / split);
  const int t1 = (int)(((int64_t)nT * (s + 1)) / split);
  const int jw = (blockIdx.z * NW + wave) * NJ;
  const bool active = jw < W;

  // gathered value of sampled column j for this lane: row lo_j of the
  // transformed chunk, slot lane ^ 8 (lo_j mod 8)
  uint32_t moff[NJ], mhi[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int j = jw + jj;
    const uint32_t m = (active && j < W) ? mu[col0 + j] : 0u;
    const uint32_t lo = m & (KCK - 1);
    moff[jj] = lo * (TL * SZ) + (uint32_t)((lane ^ (8 * (lo & 7))) * SZ);
    mhi[jj] = m >> LOGKC;
  }
  // transform role: column tp = 8 wave + lane / 8, low bits e = lane mod 8
  const int tp = 8 * wave + (lane >> 3);
  const int e = lane & 7;
  const T sg1 = (e & 1) ? T(-1) : T(1), sg2 = (e & 2) ? T(-1) : T(1), sg4 = (e & 4) ? T(-1) : T(1);

  auto load_tile = [&](int t, int b) {
    const int64_t k0 = (int64_t)t * KCK;
    const bool full = l0 + TL <= L && k0 + KCK <= K;  // uniform
    for (int p = wave; p < TL; p += NW) {
      const T* gp = A + (k0 + lane * VECN) + (l0 + p) * lda;
      if (full) {
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

  T acc[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) acc[jj] = T(0);

  if (t0 < t1) load_tile(t0, 0);
  for (int t = t0; t < t1; ++t) {
    const int b = (t - t0) & 1;
    char* const tb = smem + b * TBYTES;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // chunk t complete in LDS; every wave is past the gather of t - 1
    if (t + 1 < t1) load_tile(t + 1, b ^ 1);
    const uint32_t* __restrict__ db = Db + (int64_t)t * (KCK / 32);
    T x[NH];
    if (wave < 8) {
#pragma unroll
      for (int m = 0; m < NH; ++m) {
        const int c = e + 8 * m;  // word m / 4, bit e + 8 (m mod 4)
        const T v = *(const T*)(tb + tp * CSTR + c * SZ);
        x[m] = (db[m >> 2] >> (e + 8 * (m & 3))) & 1u ? -v : v;
      }
      fwht_regs<T, NH>(x);
#pragma unroll
      for (int m = 0; m < NH; ++m) {
        T v = x[m];
        v = sg1 * v + dpp_move<T, DPP_XOR1>(v);
        v = sg2 * v + dpp_move<T, DPP_XOR2>(v);
        v = sg4 * v + dpp_move<T, DPP_XOR3>(dpp_move<T, DPP_HALF_MIRROR>(v));
        x[m] = v;
      }
    }
    __syncthreads();  // the tile is read
    if (wave < 8) {
#pragma unroll
      for (int m = 0; m < NH; ++m) *(T*)(tb + (e + 8 * m) * (TL * SZ) + ((tp ^ (8 * e)) * SZ)) = x[m];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) {
        const T v = *(const T*)(tb + moff[jj]);
        acc[jj] += (__builtin_popcount((uint32_t)t & mhi[jj]) & 1) ? -v : v;
      }
    }
  }

  const int64_t row = l0 + lane;
  if (!active || row >= L) return;
  T* dst = split > 1 ? part + (int64_t)s * L * W : out;
  const int64_t ldd = split > 1 ? L : ldo;
  const T sc = split > 1 ? T(1) : scale;
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int j = jw + jj;
    if (j < W) dst[row + (int64_t)j * ldd] = acc[jj] * sc;
  }
}

template <typename T, bool TRANS, int NJ, int KCK>
static int run_srht_dma(Ctx* c, const T* A, int64_t lda, int64_t L, int64_t K, const uint32_t* Db, const uint32_t* mu,
                        int64_t col0, int W, T* out, int64_t ldo, T scale, hipStream_t st) {
  constexpr int NW = 16;
  const int gz = (W + NW * NJ - 1) / (NW * NJ);
  const int64_t tiles = ((L + 63) / 64) * gz;
  const int nT = (int)((K + KCK - 1) / KCK);
  int split = 1;
  if (tiles < c->num_cu)
    split = (int)std::min<int64_t>((c->num_cu + tiles - 1) / tiles, std::max(1, nT / 4));
  T* part = nullptr;
  if (split > 1) {
    const int rc = ensure_work(c, (size_t)split * (size_t)L * (size_t)W * sizeof(T));
    if (rc) return rc;
    part = (T*)work_ptr(c);
  }
  const size_t shmem = TRANS ? 2 * (size_t)64 * (KCK + 8) * sizeof(T) : 2 * (size_t)KCK * 64 * sizeof(T);
  auto kern = TRANS ? srht_dma_t_kernel<T, NW, NJ, KCK> : srht_dma_kernel<T, NW, NJ, KCK>;
  static bool attr_set = false;  // once per instantiation (the limit is the same on every device)
  if (!attr_set) {
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_set = true;
  }
  dim3 grid((unsigned)((L + 63) / 64), (unsigned)split, (unsigned)gz);
  {
    ProfScope ps(c, TRANS ? "srht_t" : "srht", st);
    kern<<<grid, NW * 64, shmem, st>>>(A, lda, L, K, Db, mu, col0, W, out, ldo, scale, split, part);
    SK_HIP(hipGetLastError());
  }
  if (split > 1) {
    ProfScope ps(c, TRANS ? "srht_reduce_t" : "srht_reduce", st);
    split_reduce_any(sizeof(T) == 8 ? SK_F64 : SK_F32, part, split, L, W, out, ldo, (double)scale, st);
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

int launch_srht_dma(Ctx* c, int dtype, bool trans, const void* A, int64_t lda, int64_t L, int64_t K,
                    const uint32_t* Db, const uint32_t* mu, int64_t col0, int W, void* out, int64_t ldo, double scale,
                    hipStream_t st) {
  // direct-to-LDS 16-byte loads: A and its columns 16-byte aligned
  const size_t esz = dtype == SK_F64 ? 8 : 4;
  if ((uintptr_t)A % 16 != 0 || (lda * (int64_t)esz) % 16 != 0) return 1;
#define SK_SRHT_DMA(T_, KC_)                                                                                   \
  {                                                                                                            \
    const T_* a = (const T_*)A;                                                                                \
    T_* o = (T_*)out;                                                                                          \
    const T_ sc = (T_)scale;                                                                                   \
    if (W <= 64)                                                                                               \
      return trans ? run_srht_dma<T_, true, 4, KC_>(c, a, lda, L, K, Db, mu, col0, W, o, ldo, sc, st)          \
                   : run_srht_dma<T_, false, 4, KC_>(c, a, lda, L, K, Db, mu, col0, W, o, ldo, sc, st);        \
    if (W <= 128)                                                                                              \
      return trans ? run_srht_dma<T_, true, 8, KC_>(c, a, lda, L, K, Db, mu, col0, W, o, ldo, sc, st)          \
                   : run_srht_dma<T_, false, 8, KC_>(c, a, lda, L, K, Db, mu, col0, W, o, ldo, sc, st);        \
    return trans ? run_srht_dma<T_, true, 16, KC_>(c, a, lda, L, K, Db, mu, col0, W, o, ldo, sc, st)           \
                 : run_srht_dma<T_, false, 16, KC_>(c, a, lda, L, K, Db, mu, col0, W, o, ldo, sc, st);         \
  }
  if (dtype == SK_F64) SK_SRHT_DMA(double, 128)
  SK_SRHT_DMA(float, 256)
#undef SK_SRHT_DMA
}

}  // namespace sk

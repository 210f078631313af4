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
#include <algorithm>

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

template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK, bool LDSE>
__global__ void __launch_bounds__(NW * 64)
    sjlt_gather_kernel(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, SjltPass pass,
                       T* __restrict__ out, int64_t ldo, T scale, int split, T* __restrict__ part) {
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
  // source of null entries), then (LDSE) the chunk's bucket entries, EW words
  // each: the entry's LDS address in the tile and its sign as +-1.0.
  constexpr int NSLOT = KCK + 1;
  constexpr int EW = SZ == 8 ? 4 : 2;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* tile = (T*)smem;
  uint32_t* ents = (uint32_t*)(smem + NSLOT * TL * SZ);
  // LDS address of the tile.  The kernel has no static LDS, so the dynamic
  // block starts at 0 and the tile base is a multiple of the row stride TL * SZ:
  // base + row offset + swizzle key combine with the lane part by XOR.
  const uint32_t tile_lds = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char*)smem;
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
  const int64_t prow = pass.wtot[blk] + 1;
  const int32_t* __restrict__ ptr = pass.ptr[blk] + jb;
  const int32_t* __restrict__ ent = pass.ent[blk];

  // LDSE staging of entries: thread tid moves entries [4 tid, 4 tid + 4) and
  // [4 (tid + NTHR), ...) of the concatenated chunk regions of the pass's blocks
  // (kcap is a multiple of 256, so a wave's entries lie in one block)
  int q0[2], eloc[2];
  bool e_on[2];
  const uint32_t* __restrict__ eptr[2];
  u32x4 ebuf[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    q0[h] = (tid + h * NTHR) * 4;
    const int eb = LDSE ? __builtin_amdgcn_readfirstlane(q0[h] / pass.kcap) : 0;
    eloc[h] = q0[h] - eb * (LDSE ? pass.kcap : 0);
    e_on[h] = LDSE && eb < pass.nblk;
    eptr[h] = e_on[h] ? (const uint32_t*)pass.ent[eb] + eloc[h] : nullptr;
    ebuf[h] = u32x4{0u, 0u, 0u, 0u};
  }
  uint32_t bnd = 0, bndN = 0, bnd_nx = 0, bndN_nx = 0;
  for (int e = tid; e < TL; e += NTHR) tile[KCK * TL + e] = T(0);

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
        if (e_on[h]) ebuf[h] = *(const u32x4*)(eptr[h] + (int64_t)t * pass.kcap);
      if (active) {
        const int32_t* pb = ptr + (int64_t)t * prow;
        bnd_nx = lane < NJ ? (uint32_t)pb[lane] : 0u;
        bndN_nx = (uint32_t)pb[NJ];
      }
    }
  };
  auto load_chunk = [&](int t) {
    load_meta(t);
    const int64_t k0 = (int64_t)t * KCK;
    const bool full = l0 + TL <= L && k0 + KCK <= K;  // uniform
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
        if (!e_on[h]) continue;
        uint32_t ad[4], sg[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t src = ebuf[h][q] >> 1;
          ad[q] = (tile_lds + src * (uint32_t)(TL * SZ)) | (TRANS ? ((src / VECN) & 15u) * 16u : 0u);
          // the sign as +-1.0 (high word of the double for FP64)
          sg[q] = ((ebuf[h][q] & 1u) << 31) | (SZ == 8 ? 0x3ff00000u : 0x3f800000u);
        }
        const int qb = q0[h];
        if constexpr (EW == 4) {
#pragma unroll
          for (int q = 0; q < 4; ++q) *(u32x4*)&ents[(qb + q) * 4] = u32x4{ad[q], 0u, 0u, sg[q]};
        } else {
          *(u32x4*)&ents[qb * 2] = u32x4{ad[0], sg[0], ad[1], sg[1]};
          *(u32x4*)&ents[qb * 2 + 4] = u32x4{ad[2], sg[2], ad[3], sg[3]};
        }
      }
      bnd = bnd_nx;
      bndN = bndN_nx;
    }
    if (!TRANS) {
#pragma unroll
      for (int it = 0; it < NV; ++it) *(u32x4*)(&tile[(my_col + it * CSTEP) * TL + my_row]) = buf[it];
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

  if (t0 < t1) load_chunk(t0);
  for (int t = t0; t < t1; ++t) {
    __syncthreads();  // the previous chunk is fully consumed
    store_chunk();
    __syncthreads();
    if (t + 1 < t1) load_chunk(t + 1);  // in flight during the gather below
    if (active) {
      if constexpr (LDSE)
        gather_chunk_lds<T, NJ, RPL, VT>(ents, (t - blk) * pass.kcap, bnd, bndN, lane_part, zaddr, pass.ms, acc);
      else
        gather_chunk<T, NJ, RPL, VT>(ptr + (int64_t)t * prow, ent, LD, acc);
    }
  }

  if (!active) return;
  const int64_t row0 = l0 + lane_elem;
  const int64_t jc = (int64_t)g * NJ;
  T* dst = out;
  int64_t ldd = ldo;
  T sc = scale;
  if (split > 1) {
    dst = part + (int64_t)s * L * ((int64_t)pass.ngroups * NJ);
    ldd = L;
    sc = T(1);
  }
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
#pragma unroll
    for (int r = 0; r < RPL; ++r)
      if (row0 + r < L) dst[row0 + r + (jc + jj) * ldd] = acc[jj][r] * sc;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) split_reduce_kernel(const T* __restrict__ part, int split, int64_t L,
                                                          int64_t W, T* __restrict__ out, int64_t ldo, T scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= L * W) return;
  const int64_t row = idx % L, j = idx / L;
  T a = T(0);
  for (int s = 0; s < split; ++s) a += part[(int64_t)s * L * W + idx];
  out[row + j * ldo] = a * scale;
}

void split_reduce_f32(const float* part, int split, int64_t L, int64_t W, float* out, int64_t ldo, float scale,
                      hipStream_t st) {
  const int64_t tot = L * W;
  split_reduce_kernel<float><<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(part, split, L, W, out, ldo, scale);
}

// ------------------------------------------------------------------ dispatch
// dynamic LDS of one workgroup: the tile with its zero slot, then the entries
static size_t gather_lds_bytes(int esz, int kc, int tl, bool ldse, int nblk, int kcap) {
  const size_t ew = esz == 8 ? 16 : 8;
  return (size_t)(kc + 1) * tl * esz + (ldse ? ((size_t)nblk * kcap + 4) * ew : 0);
}

struct GatherCfg {
  int nw, nj, rpl, kc;
  bool ldse;  // bucket entries staged in LDS (else read through the scalar cache)
};

template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK, bool LDSE>
static int run_gather(Ctx* c, const T* A, int64_t lda, int64_t L, int64_t K, const SjltPass& pass, T* out,
                      int64_t ldo, T scale, int split, T* part, int gz, hipStream_t st) {
  dim3 grid((unsigned)((L + 64 * RPL - 1) / (64 * RPL)), (unsigned)split, (unsigned)gz);
  const size_t shmem = gather_lds_bytes((int)sizeof(T), KCK, 64 * RPL, LDSE, pass.nblk, pass.kcap);
  auto kern = sjlt_gather_kernel<T, TRANS, NW, NJ, RPL, KCK, LDSE>;
  static bool attr_set = false;  // once per instantiation (the limit is the same on every device)
  if (!attr_set) {
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_set = true;
  }
  ProfScope ps(c, TRANS ? "sjlt_gather_t" : "sjlt_gather", st);
  kern<<<grid, NW * 64, shmem, st>>>(A, lda, L, K, pass, out, ldo, scale, split, part);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK>
struct GatherValid {
  static constexpr int VECN = 16 / (int)sizeof(T);
  static constexpr int NV = KCK * 64 * RPL / (NW * 64 * VECN);
  static constexpr bool value = (KCK * 64 * RPL) % (NW * 64 * VECN) == 0 && NV >= 1 && (!TRANS || NV % VECN == 0) &&
                                RPL <= VECN;
};

// returns 1 when the configuration does not match (caller tries the next one)
template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK>
static int try_cfg(const GatherCfg& cfg, Ctx* c, const T* A, int64_t lda, int64_t L, int64_t K, const SjltPass& pass,
                   T* out, int64_t ldo, T scale, int split, T* part, int gz, hipStream_t st) {
  if (cfg.nw != NW || cfg.nj != NJ || cfg.rpl != RPL || cfg.kc != KCK) return 1;
  if constexpr (GatherValid<T, TRANS, NW, NJ, RPL, KCK>::value) {
    if (cfg.ldse)
      return run_gather<T, TRANS, NW, NJ, RPL, KCK, true>(c, A, lda, L, K, pass, out, ldo, scale, split, part, gz, st);
    return run_gather<T, TRANS, NW, NJ, RPL, KCK, false>(c, A, lda, L, K, pass, out, ldo, scale, split, part, gz, st);
  } else {
    return 1;
  }
}

#define SK_TRY(NW_, NJ_, RPL_, KC_)                                                                              \
  if ((rc = try_cfg<T, TRANS, NW_, NJ_, RPL_, KC_>(cfg, c, A, lda, L, K, pass, out, ldo, scale, split, part, gz, \
                                                   st)) != 1)                                                   \
    return rc;
#define SK_TRY_NW(NJ_, RPL_, KC_) SK_TRY(4, NJ_, RPL_, KC_) SK_TRY(8, NJ_, RPL_, KC_)

template <typename T, bool TRANS>
static int dispatch(Ctx* c, const GatherCfg& cfg, const T* A, int64_t lda, int64_t L, int64_t K,
                    const SjltPass& pass, T* out, int64_t ldo, T scale, int split, T* part, int gz,
                    hipStream_t st) {
  int rc;
  if constexpr (sizeof(T) == 4) {
    SK_TRY_NW(16, 4, 64)
    SK_TRY_NW(16, 2, 128)
    SK_TRY_NW(32, 2, 128)
    SK_TRY_NW(16, 1, 64)
    SK_TRY_NW(32, 1, 64)
    SK_TRY_NW(64, 1, 64)
    SK_TRY_NW(16, 1, 128)
    SK_TRY_NW(32, 1, 128)
    SK_TRY_NW(64, 1, 128)
    SK_TRY_NW(16, 1, 256)
    SK_TRY_NW(32, 1, 256)
    SK_TRY_NW(64, 1, 256)
  } else {
    SK_TRY_NW(16, 2, 64)
    SK_TRY_NW(16, 1, 64)
    SK_TRY_NW(32, 1, 64)
    SK_TRY_NW(16, 1, 128)
    SK_TRY_NW(32, 1, 128)
    SK_TRY_NW(16, 1, 256)
    SK_TRY_NW(32, 1, 256)
  }
  set_error("internal: no SJLT kernel for NW=%d NJ=%d RPL=%d KC=%d", cfg.nw, cfg.nj, cfg.rpl, cfg.kc);
  return SK_EINVAL;
}

// the launch table skips 8-wave variants whose tile does not split evenly
template <typename T, bool TRANS>
static bool cfg_valid(int nw, int rpl, int kc) {
  const int vecn = 16 / (int)sizeof(T);
  const long tile = (long)kc * 64 * rpl;
  const long per = (long)nw * 64 * vecn;
  if (tile % per) return false;
  const long nv = tile / per;
  return nv >= 1 && (!TRANS || nv % vecn == 0) && rpl <= vecn;
}

static int gcd_int(int a, int b) {
  while (b) {
    const int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

int sjlt_chunk_for(int w, int alpha) {
  // about four entries per bucket and chunk: KC * alpha / w >= 4
  int kc = 64;
  while (kc < 256 && kc * alpha < 4 * w) kc *= 2;
  return kc;
}

// rows per lane, columns per wave and waves per workgroup for a pass of width W
// whose block widths share the divisor g
static GatherCfg choose_cfg(int dtype, int kc, int W, int g) {
  GatherCfg c;
  c.kc = kc;
  if (dtype == SK_F32) c.rpl = kc == 64 ? 4 : kc == 128 ? 2 : 1;
  else c.rpl = kc == 64 ? 2 : 1;
  // accumulators per lane stay at or below 64 VGPRs
  int njmax = (dtype == SK_F32 ? 64 : 32) / c.rpl;
  // a pass wider than 8 waves x njmax columns would re-read A: fewer rows per lane
  if (W > 8 * njmax && c.rpl > 1) {
    c.rpl = 1;
    njmax = dtype == SK_F32 ? 64 : 32;
  }
  int nj = 16;
  for (int cand = njmax; cand >= 16; cand /= 2)
    if (g % cand == 0 && (cand * 4 <= W || cand == 16)) {
      nj = cand;
      break;
    }
  c.nj = nj;
  c.nw = W / nj <= 4 ? 4 : 8;
  return c;
}

int launch_sjlt_pass(Handle* h, const sk_input* in, int b0, int b1, bool trans, void* out, int64_t ldo,
                     hipStream_t st) {
  const int nblk = b1 - b0;
  SK_REQUIRE(nblk >= 1 && nblk <= MAX_PASS_BLOCKS, SK_EINVAL, "a pass covers 1..%d blocks", MAX_PASS_BLOCKS);
  int W = 0, g = 0;
  for (int b = b0; b < b1; ++b) {
    W += h->blocks[b].w;
    g = gcd_int(g, h->blocks[b].w);
  }
  SK_REQUIRE(g % 16 == 0, SK_EINVAL, "SJLT block widths must be multiples of 16");
  GatherCfg cfg = choose_cfg(h->dtype, h->kc, W, g);
  if (cfg.nw == 8) {
    const bool ok = h->dtype == SK_F64 ? (trans ? cfg_valid<double, true>(8, cfg.rpl, cfg.kc)
                                               : cfg_valid<double, false>(8, cfg.rpl, cfg.kc))
                                       : (trans ? cfg_valid<float, true>(8, cfg.rpl, cfg.kc)
                                                : cfg_valid<float, false>(8, cfg.rpl, cfg.kc));
    if (!ok) cfg.nw = 4;
  }
  const int ngroups = W / cfg.nj;
  SK_REQUIRE(ngroups <= MAX_PASS_GROUPS, SK_EINVAL, "pass too wide (%d columns)", W);
  const int gz = (ngroups + cfg.nw - 1) / cfg.nw;

  SjltPass pass;
  memset(&pass, 0, sizeof(pass));
  pass.nT = (int)((h->n + h->kc - 1) / h->kc);
  pass.ngroups = ngroups;
  int gi = 0;
  for (int b = b0; b < b1; ++b) {
    const Block& B = h->blocks[b];
    pass.ptr[b - b0] = B.ptr;
    pass.ent[b - b0] = B.ent;
    pass.wtot[b - b0] = B.w;
    for (int c = 0; c < B.w; c += cfg.nj) {
      pass.grp_blk[gi] = b - b0;
      pass.grp_col[gi] = c;
      ++gi;
    }
  }

  pass.nblk = nblk;
  pass.kcap = 0;
  // straight-line slots per bucket: about the mean bucket length KC * alpha / w
  pass.ms = (int64_t)h->kc * h->alpha >= 7LL * W / nblk ? 8 : 4;
  for (int b = b0; b < b1; ++b) pass.kcap = std::max(pass.kcap, sjlt_kcap(h->kc, h->alpha, h->blocks[b].w));
  // entries staged in LDS when every block of the pass has the same chunk region
  // size, the regions fit four entries per thread and the LDS holds them
  bool same = true;
  for (int b = b0; b < b1; ++b) same = same && sjlt_kcap(h->kc, h->alpha, h->blocks[b].w) == pass.kcap;
  const size_t esz = h->dtype == SK_F64 ? 8 : 4;
  const int TL = 64 * cfg.rpl;
  cfg.ldse = same && (int64_t)nblk * pass.kcap <= (int64_t)cfg.nw * 64 * 8 &&
             gather_lds_bytes((int)esz, cfg.kc, TL, true, nblk, pass.kcap) <= 160 * 1024;

  const int64_t L = trans ? in->n : in->m;  // lanes
  const int64_t K = trans ? in->m : in->n;  // sources (= rows of R)
  const int64_t tiles = ((L + TL - 1) / TL) * gz;
  const size_t tile_bytes = gather_lds_bytes((int)esz, cfg.kc, TL, cfg.ldse, nblk, pass.kcap);
  const int64_t per_cu = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)tile_bytes);
  const int64_t target = per_cu * (int64_t)h->ctx->num_cu;
  int split = 1;
  if (tiles < target) split = (int)std::min<int64_t>((target + tiles - 1) / tiles, std::max(1, pass.nT / 4));
  void* part = nullptr;
  if (split > 1) {
    const int rc = ensure_work(h->ctx, (size_t)split * (size_t)L * (size_t)W * esz);
    if (rc) return rc;
    part = h->ctx->work;
  }
  const double scale = 1.0 / sqrt((double)h->alpha);
  Ctx* c = h->ctx;
  int rc;
  if (h->dtype == SK_F64) {
    const double* A = (const double*)in->A;
    rc = trans ? dispatch<double, true>(c, cfg, A, in->lda, L, K, pass, (double*)out, ldo, scale, split,
                                        (double*)part, gz, st)
               : dispatch<double, false>(c, cfg, A, in->lda, L, K, pass, (double*)out, ldo, scale, split,
                                         (double*)part, gz, st);
  } else {
    const float* A = (const float*)in->A;
    rc = trans ? dispatch<float, true>(c, cfg, A, in->lda, L, K, pass, (float*)out, ldo, (float)scale, split,
                                       (float*)part, gz, st)
               : dispatch<float, false>(c, cfg, A, in->lda, L, K, pass, (float*)out, ldo, (float)scale, split,
                                        (float*)part, gz, st);
  }
  if (rc) return rc;
  if (split > 1) {
    const int64_t tot = L * (int64_t)W;
    const unsigned nb = (unsigned)((tot + 255) / 256);
    ProfScope ps(h->ctx, "sjlt_reduce", st);
    if (h->dtype == SK_F64)
      split_reduce_kernel<double><<<nb, 256, 0, st>>>((const double*)part, split, L, W, (double*)out, ldo, scale);
    else
      split_reduce_kernel<float><<<nb, 256, 0, st>>>((const float*)part, split, L, W, (float*)out, ldo,
                                                     (float)scale);
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

}  // namespace sk

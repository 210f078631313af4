// SJLT sketch of a stored, column-major A: kernels over one pass of operator
// blocks (S = A R_b... and S' = A^T R_b...), with the source range split across
// workgroups when the lane tiles cannot fill the chip.
#include "sjlt_tile.hpp"

namespace sk {

template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK, bool LDSE, bool NEG>
__global__ void __launch_bounds__(NW * 64)
    sjlt_gather_kernel(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, SjltPass pass,
                       T* __restrict__ out, int64_t ldo, T scale, int split, T* __restrict__ part) {
  constexpr int TL = 64 * RPL;
  constexpr int NTHR = NW * 64;
  const int tid = threadIdx.x;
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
  const uint32_t* eptr[2] = {nullptr, nullptr};
  if constexpr (LDSE) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q0 = (tid + h * NTHR) * 4;
      const int eb = __builtin_amdgcn_readfirstlane(q0 / pass.kcap);  // a wave's entries lie in one block
      if (eb < pass.nblk) eptr[h] = (const uint32_t*)pass.ent[eb] + (q0 - eb * pass.kcap);
    }
  }
  const int64_t jc = (int64_t)g * NJ;
  T* dst = split > 1 ? part + (int64_t)s * L * ((int64_t)pass.ngroups * NJ) + jc * L : out + jc * ldo;
  sjlt_tile<T, TRANS, NW, NJ, RPL, KCK, LDSE, NEG>(A, lda, L, K, l0, t0, t1, active, pass.ptr[blk] + jb,
                                              (int64_t)pass.wtot[blk] + 1, pass.ent[blk], blk, eptr[0], eptr[1],
                                              pass.kcap, pass.nblk * pass.kcap, pass.ms, dst, split > 1 ? L : ldo,
                                              split > 1 ? T(1) : scale);
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

void split_reduce_any(int dtype, const void* part, int split, int64_t L, int64_t W, void* out, int64_t ldo,
                      double scale, hipStream_t st) {
  const unsigned nb = (unsigned)((L * W + 255) / 256);
  if (dtype == SK_F64)
    split_reduce_kernel<double><<<nb, 256, 0, st>>>((const double*)part, split, L, W, (double*)out, ldo, scale);
  else
    split_reduce_kernel<float><<<nb, 256, 0, st>>>((const float*)part, split, L, W, (float*)out, ldo, (float)scale);
}

// ------------------------------------------------------------------ dispatch
template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK, bool LDSE, bool NEG = false>
static int run_gather(Ctx* c, const T* A, int64_t lda, int64_t L, int64_t K, const SjltPass& pass, T* out,
                      int64_t ldo, T scale, int split, T* part, int gz, hipStream_t st) {
  dim3 grid((unsigned)((L + 64 * RPL - 1) / (64 * RPL)), (unsigned)split, (unsigned)gz);
  const size_t shmem = gather_lds_bytes((int)sizeof(T), KCK, 64 * RPL, LDSE, pass.nblk, pass.kcap, NEG);
  auto kern = sjlt_gather_kernel<T, TRANS, NW, NJ, RPL, KCK, LDSE, NEG>;
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

// returns 1 when the configuration does not match (caller tries the next one)
template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK>
static int try_cfg(const GatherCfg& cfg, Ctx* c, const T* A, int64_t lda, int64_t L, int64_t K, const SjltPass& pass,
                   T* out, int64_t ldo, T scale, int split, T* part, int gz, hipStream_t st) {
  if (cfg.nw != NW || cfg.nj != NJ || cfg.rpl != RPL || cfg.kc != KCK) return 1;
  if constexpr (GatherValid<T, TRANS, NW, NJ, RPL, KCK>::value) {
    if constexpr (sizeof(T) == 4 && NW == 16 && RPL > 1) {  // the wide FP32 passes
      if (cfg.ldse && cfg.neg)
        return run_gather<T, TRANS, NW, NJ, RPL, KCK, true, true>(c, A, lda, L, K, pass, out, ldo, scale, split,
                                                                  part, gz, st);
    }
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
    SK_TRY(16, 16, 1, 64) SK_TRY(16, 16, 1, 128) SK_TRY(16, 16, 1, 256)
    SK_TRY(16, 16, 4, 64) SK_TRY(16, 16, 2, 128) SK_TRY(8, 8, 4, 64)
  } else {
    SK_TRY_NW(16, 2, 64)
    SK_TRY_NW(16, 1, 64)
    SK_TRY_NW(32, 1, 64)
    SK_TRY_NW(16, 1, 128)
    SK_TRY_NW(32, 1, 128)
    SK_TRY_NW(16, 1, 256)
    SK_TRY_NW(32, 1, 256)
    SK_TRY(16, 16, 1, 64) SK_TRY(16, 16, 1, 128) SK_TRY(16, 16, 1, 256)
    SK_TRY(16, 16, 2, 64)
  }
  set_error("internal: no SJLT kernel for NW=%d NJ=%d RPL=%d KC=%d", cfg.nw, cfg.nj, cfg.rpl, cfg.kc);
  return SK_EINVAL;
}

static int gcd_int(int a, int b) {
  while (b) {
    const int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Shape of the direct-to-LDS S kernel for a pass: every column group in one
// workgroup (nw * nj == W), the double-buffered tile and entries in LDS, the
// entries within the staging capacity; nw = 0 when none fits.
struct DmaShape {
  int nw, nj, rpl;
};
static DmaShape choose_dma(int dtype, int kc, int W, int g, int nblk, int kcap) {
  static const int f64[][4] = {{128, 16, 16, 1}, {128, 8, 32, 1}, {128, 8, 16, 1}, {128, 4, 16, 1},
                               {64, 16, 16, 1},  {64, 8, 16, 2}};
  static const int f32[][4] = {{256, 16, 16, 1}, {256, 8, 32, 1}, {128, 16, 16, 2},
                               {128, 8, 16, 2},  {128, 16, 16, 1}};
  const int esz = dtype == SK_F64 ? 8 : 4;
  const int(*tab)[4] = dtype == SK_F64 ? f64 : f32;
  const int ntab = dtype == SK_F64 ? (int)(sizeof(f64) / sizeof(f64[0])) : (int)(sizeof(f32) / sizeof(f32[0]));
  for (int i = 0; i < ntab; ++i) {
    const int* r = tab[i];
    if (r[0] != kc || r[1] * r[2] != W || g % r[2] != 0) continue;
    if ((int64_t)nblk * kcap > (int64_t)r[1] * 64 * 8) continue;
    if (dma_lds_bytes(esz, kc, 64 * r[3], nblk, kcap) > 160 * 1024) continue;
    return DmaShape{r[1], r[2], r[3]};
  }
  return DmaShape{0, 0, 0};
}

// Chunk sizes of a dense operator of width d.  S: about two entries per bucket
// when the direct-to-LDS kernel has a shape for it (it double-buffers the tile,
// so shorter chunks keep it in LDS), else about four (and four for FP64 from
// 256 columns on).  S': the 1 KB column
// chunks of the direct-to-LDS S' kernel when it applies (and in FP32 from 256
// columns on, for the register-staged kernel), else (register-staged kernel)
// about four entries per bucket in FP64, two in FP32.  kct = 0 when S' shares
// the S tables.
// Shape of the direct-to-LDS S' kernel: one 1 KB chunk per column (KC = 256
// sources in FP32), NJ columns per wave; nw = 0 when it does not apply.  The
// FP64 instances (KC = 128) were measured no faster than the register-staged
// kernel on MI355X (w = 256) or slower (w = 64, 0.70 against 0.52 ms at
// n = 16384), so FP64 keeps the register-staged S'.  From 256 columns on, the
// register-staged kernel with the same 1 KB pieces is faster in FP32 too
// (n = 16384, w = 256: 0.369 against 0.433 ms; w = 128: 0.43 against 0.39 ms).
static DmaShape choose_dma_t(int dtype, int kc, int W, int g, int nblk, int kcap) {
  const int esz = dtype == SK_F64 ? 8 : 4;
  if (dtype == SK_F64 || kc * esz != 1024 || W >= 256) return DmaShape{0, 0, 0};
  const int nj = W >= 128 ? 8 : 4;
  if (g % nj != 0 || W / nj > MAX_PASS_GROUPS) return DmaShape{0, 0, 0};
  // long buckets (more than about eight entries per chunk) gather faster in the
  // register-staged kernel (measured: w = 64, alpha = 8)
  if ((int64_t)nblk * kcap > 8 * (int64_t)W) return DmaShape{0, 0, 0};
  if ((int64_t)nblk * kcap > 16 * 64 * 8) return DmaShape{0, 0, 0};
  if (dma_t_lds_bytes(esz, kc, nblk, kcap) > 160 * 1024) return DmaShape{0, 0, 0};
  return DmaShape{16, nj, 1};
}

void sjlt_pick_chunks(int dtype, int d, int alpha, bool want_t, int* kc, int* kct) {
  const int k2 = sjlt_chunk_for(d, alpha, 2);
  *kc = choose_dma(dtype, k2, d, d, 1, sjlt_kcap(k2, alpha, d)).nw ? k2 : sjlt_chunk_for(d, alpha, 4);
  // FP64 from 256 columns on: the register-staged kernel with 16 waves and
  // about four entries per bucket beats the direct-to-LDS one (n = 16384,
  // w = 256: 0.517 against 0.569 ms), and S' shares its tables
  if (dtype == SK_F64 && d >= 256) *kc = sjlt_chunk_for(d, alpha, 4);
  const int kd = dtype == SK_F64 ? 128 : 256;
  const int kt = (dtype == SK_F32 && d >= 256) || choose_dma_t(dtype, kd, d, d, 1, sjlt_kcap(kd, alpha, d)).nw
                     ? kd
                     : sjlt_chunk_for(d, alpha, dtype == SK_F64 ? 4 : 2);
  *kct = want_t && kt != *kc ? kt : 0;
}

int sjlt_chunk_for(int w, int alpha, int lam) {
  // smallest chunk with about lam entries per bucket (KC * alpha / w >= lam)
  int kc = 64;
  while (kc < 256 && kc * alpha < lam * w) kc *= 2;
  return kc;
}

// rows per lane, columns per wave and waves per workgroup for a pass of width W
// whose block widths share the divisor g
static GatherCfg choose_cfg(int dtype, int kc, int W, int g) {
  GatherCfg c = {};
  c.kc = kc;
  if (dtype == SK_F32) c.rpl = kc == 64 ? 4 : kc == 128 ? 2 : 1;
  else c.rpl = kc == 64 ? 2 : 1;
  // accumulators per lane stay at or below 64 VGPRs
  int njmax = (dtype == SK_F32 ? 64 : 32) / c.rpl;
  // A pass wider than 8 waves x njmax columns: 16 waves of 16 columns keep the
  // RPL rows per lane, one workgroup per 256 columns (A is staged once per 256
  // columns).  One row per lane instead would double the LDS bytes per add
  // (each bucket entry read then serves one element per lane, not RPL):
  // measured on FP32, alpha = 8, w = 64, n = 65536, four blocks in one pass:
  // 30.2 ms with one row per lane, 11.2 ms with four.
  if (W > 8 * njmax && c.rpl > 1) {
    if (g % 16 == 0) {
      c.nj = 16;
      c.nw = 16;
      return c;
    }
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
  // a 64-column FP32 pass with four rows per lane: 8 waves of 8 columns rather
  // than 4 of 16 (twice the waves per CU to cover the loads; measured on FP32,
  // alpha = 8, n = 65536: 4.82 -> 3.92 ms)
  if (dtype == SK_F32 && c.rpl == 4 && W == 64 && g % 8 == 0) {
    c.nj = 8;
    c.nw = 8;
  }
  // passes of 256 columns or more: 16 waves of 16 columns (fewer VGPRs per
  // wave, twice the waves per CU; measured for FP64 S' at n = 16384, w = 256:
  // 0.74 -> 0.57 ms; slower at w = 128)
  if (c.rpl == 1 && W >= 256 && g % 16 == 0) {
    c.nj = 16;
    c.nw = 16;
  }
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
  // S' may use bucket tables of its own chunk size
  const bool own_t = trans && h->kct && h->blocks[b0].ptr_t;
  const int kc = own_t ? h->kct : h->kc;
  GatherCfg cfg = choose_cfg(h->dtype, kc, W, g);
  if (cfg.nw == 16) {
    const bool ok = h->dtype == SK_F64 ? (trans ? cfg_valid<double, true>(16, cfg.rpl, cfg.kc)
                                               : cfg_valid<double, false>(16, cfg.rpl, cfg.kc))
                                       : (trans ? cfg_valid<float, true>(16, cfg.rpl, cfg.kc)
                                                : cfg_valid<float, false>(16, cfg.rpl, cfg.kc));
    if (!ok) cfg.nw = 8;
  }
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
  pass.nT = (int)((h->n + kc - 1) / kc);
  pass.ngroups = ngroups;
  int gi = 0;
  for (int b = b0; b < b1; ++b) {
    const Block& B = h->blocks[b];
    pass.ptr[b - b0] = own_t ? B.ptr_t : B.ptr;
    pass.ent[b - b0] = own_t ? B.ent_t : B.ent;
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
  {
    const int64_t lam2 = 2LL * kc * h->alpha * nblk / W;  // twice the mean bucket length per chunk
    pass.ms = lam2 >= 14 ? 8 : lam2 >= 6 ? 4 : 2;
  }
  for (int b = b0; b < b1; ++b) pass.kcap = std::max(pass.kcap, sjlt_kcap(kc, h->alpha, h->blocks[b].w));
  // entries staged in LDS when every block of the pass has the same chunk region
  // size, the regions fit four entries per thread and the LDS holds them
  bool same = true;
  for (int b = b0; b < b1; ++b) same = same && sjlt_kcap(kc, h->alpha, h->blocks[b].w) == pass.kcap;
  const size_t esz = h->dtype == SK_F64 ? 8 : 4;
  const int TL = 64 * cfg.rpl;
  cfg.ldse = same && (int64_t)nblk * pass.kcap <= (int64_t)cfg.nw * 64 * 8 &&
             gather_lds_bytes((int)esz, cfg.kc, TL, true, nblk, pass.kcap) <= 160 * 1024;
  // wide FP32 passes (16 waves, several rows per lane): with negated tile
  // rows an entry is a bare address and the gather adds without a sign
  // (measured at alpha = 8, n = 65536, 3 passes: 21.5 against 23.9 ms)
  cfg.neg = cfg.ldse && h->dtype == SK_F32 && cfg.nw == 16 && cfg.rpl > 1 &&
            gather_lds_bytes((int)esz, cfg.kc, TL, true, nblk, pass.kcap, true) <= 160 * 1024;

  const int64_t L = trans ? in->n : in->m;  // lanes
  const int64_t K = trans ? in->m : in->n;  // sources (= rows of R)
  const int64_t tiles = ((L + TL - 1) / TL) * gz;
  const size_t tile_bytes = gather_lds_bytes((int)esz, cfg.kc, TL, cfg.ldse, nblk, pass.kcap, cfg.neg);
  const int64_t per_cu = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)tile_bytes);
  const int64_t target = per_cu * (int64_t)h->ctx->num_cu;
  const int ms_raw = pass.ms;
  pass.ms = std::max(pass.ms, 4);  // the register-staged gather takes 4 or 8 straight-line slots
  int split = 1;
  // slices of at least 4 chunks; at least 2 when the tiles fill under a quarter
  // of the chip (small matrices are latency-bound)
  const int min_chunks = tiles * 4 < target ? 2 : 4;
  if (tiles < target)
    split = (int)std::min<int64_t>((target + tiles - 1) / tiles, std::max(1, pass.nT / min_chunks));
  void* part = nullptr;
  if (split > 1) {
    const int rc = ensure_work(h->ctx, (size_t)split * (size_t)L * (size_t)W * esz);
    if (rc) return rc;
    part = work_ptr(h->ctx);
  }
  const double scale = 1.0 / sqrt((double)h->alpha);
  Ctx* c = h->ctx;
  int rc;
  // S with whole-workgroup column coverage: the direct-to-LDS kernel when a
  // shape fits (it splits the source range by the same rule)
  {
    // (direct-to-LDS 16-byte loads: A and its columns 16-byte aligned)
    const bool al16 = (uintptr_t)in->A % 16 == 0 && (in->lda * (int64_t)esz) % 16 == 0;
    DmaShape ds = !al16 ? DmaShape{0, 0, 0}
                  : trans ? choose_dma_t(h->dtype, kc, W, g, nblk, pass.kcap)
                          : choose_dma(h->dtype, kc, W, g, nblk, pass.kcap);
    if (ds.nw) {
      const size_t dbytes = trans ? dma_t_lds_bytes((int)esz, kc, nblk, pass.kcap)
                                  : dma_lds_bytes((int)esz, kc, 64 * ds.rpl, nblk, pass.kcap);
      const int64_t dtiles = (L + 64 * ds.rpl - 1) / (64 * ds.rpl);
      const int64_t dtarget = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)dbytes) * c->num_cu;
      int dsplit = 1;
      if (dtiles < dtarget)
        dsplit = (int)std::min<int64_t>((dtarget + dtiles - 1) / dtiles,
                                        std::max(1, pass.nT / (dtiles * 4 < dtarget ? 2 : 4)));
      SjltPass dp = pass;  // the register-staged pass below keeps its own column groups
      dp.ms = ms_raw;
      dp.ngroups = W / ds.nj;
      int di = 0;
      for (int b = b0; b < b1; ++b)
        for (int cc = 0; cc < h->blocks[b].w; cc += ds.nj) {
          dp.grp_blk[di] = b - b0;
          dp.grp_col[di] = cc;
          ++di;
        }
      void* dpart = nullptr;
      if (dsplit > 1) {
        if ((rc = ensure_work(c, (size_t)dsplit * (size_t)L * (size_t)W * esz))) return rc;
        dpart = work_ptr(c);
      }
      rc = trans ? launch_sjlt_dma_t(c, h->dtype, ds.nw, ds.nj, kc, in->A, in->lda, L, K, dp, out, ldo, scale,
                                     dsplit, dpart, st)
                 : launch_sjlt_dma(c, h->dtype, ds.nw, ds.nj, ds.rpl, kc, in->A, in->lda, L, K, dp, out, ldo, scale,
                                   dsplit, dpart, 1, st);
      if (rc != 1) {
        if (rc) return rc;
        if (dsplit > 1) {
          const int64_t tot = L * (int64_t)W;
          const unsigned nb = (unsigned)((tot + 255) / 256);
          ProfScope ps(h->ctx, "sjlt_reduce", st);
          if (h->dtype == SK_F64)
            split_reduce_kernel<double><<<nb, 256, 0, st>>>((const double*)dpart, dsplit, L, W, (double*)out, ldo,
                                                            scale);
          else
            split_reduce_kernel<float><<<nb, 256, 0, st>>>((const float*)dpart, dsplit, L, W, (float*)out, ldo,
                                                           (float)scale);
          SK_HIP(hipGetLastError());
        }
        return SK_OK;
      }
      if (split > 1) part = work_ptr(c);  // the workspace may have grown above
    }
  }
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


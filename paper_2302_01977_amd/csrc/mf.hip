// Matrix-free Gaussian-kernel sketch S = K(X, h) R with an SJLT R, and its
// hand-written backward.  K_ij = exp(-|x_i - x_j|^2 / (2 h^2)) (+ shift on the
// diagonal) is never stored: every kernel recomputes the tiles it needs.
// (The paper's construction is only partially matrix-free, section 2.3; here the
// sketch itself is.)
//
// Forward: the stored-A SJLT gather with the LDS tile produced in registers:
// a workgroup owns 64 points i (lanes) and, per chunk of KC source points k,
// each wave evaluates K_ik for a slice of the chunk; the bucket gather then adds
// the signed entries exactly as for a stored matrix.
//
// Backward for L = sum(W o S) (W = dL/dS): with G = W R^T,
//   dL/dx_i = -(1/h^2) sum_j (G_ij + G_ji) K_ij (x_i - x_j),
//   dL/dh   =  sum_ij G_ij K_ij |x_i - x_j|^2 / h^3.
// G_ij = sum_c sign(j,c) W(i, col(j,c)) / sqrt(alpha) reads the columns named by
// the (uniform) hash of j from an LDS copy of W's rows i; G_ji reads row j of W
// at the columns named by the hash of lane i, from an LDS slot of the wave into
// which row j of a row-major copy of W (1 KB) is staged.  dL/dx terms are summed in FP32 over a
// chunk of sources and in FP64 across chunks; dL/dh, a sum with heavy
// cancellation, is accumulated in FP64 term by term.  Waves and workgroups are
// combined in a fixed order, so the result is deterministic.
#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

#include "gather.hpp"
#include "internal.hpp"

namespace sk {

// RPL consecutive points i per lane (TL = 64 RPL per workgroup): the gather's
// per-entry work (address, mask, bounds) is shared by RPL additions.
// cs = sqrt(log2(e) / (2 h^2)): coordinates are scaled by cs as they are
// loaded, so that K = exp2(-|cs x_i - cs x_k|^2) needs no multiply per pair.
template <int NW, int NJ, int KCK, int DIM, bool LDSE, int RPL>
__global__ void __launch_bounds__(NW * 64)
    mf_sjlt_kernel(const float* __restrict__ X, int64_t N, float cs, float shift, SjltPass pass,
                   float* __restrict__ out, int64_t ldo, float scale, int split, float* __restrict__ part) {
  constexpr int TL = 64 * RPL;
  constexpr uint32_t ROWB = TL * 4;  // bytes of one staged source row
  static_assert(KCK % TL == 0, "a tile's own points lie in one chunk");
  typedef typename std::conditional<RPL == 1, float, float __attribute__((ext_vector_type(2)))>::type VT;
  static_assert(RPL == 1 || RPL == 2, "one or two points per lane");
  // dynamic LDS: the tile (slot KCK: zeros for null entries), then (LDSE) the
  // chunk's bucket entries, one word each (LDS address of the source row, the
  // sign in bit 31; the region keeps room for two words per entry)
  extern __shared__ __attribute__((aligned(16))) char smem[];
  float* const tile = (float*)smem;
  uint32_t* const ents = (uint32_t*)(smem + (KCK + 1) * ROWB);
  constexpr int NTHR = NW * 64;
  const uint32_t tile_lds = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char*)smem;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * TL;
  const int64_t i0 = l0 + (int64_t)lane * RPL;  // this lane's first point
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

  float xi[RPL][DIM];
#pragma unroll
  for (int r = 0; r < RPL; ++r)
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[r][d] = i0 + r < N ? X[(i0 + r) * DIM + d] * cs : 0.f;
  for (int e = tid; e < TL; e += NTHR) tile[KCK * TL + e] = 0.f;

  // LDSE staging (as in the stored-A kernels): thread tid moves entries
  // [4 tid, 4 tid + 4) and [4 (tid + NTHR), ...) of the pass's chunk regions,
  // one chunk ahead; lane jj of bnd holds the start of the wave's column jj
  const uint32_t* eptr[2] = {nullptr, nullptr};
  if constexpr (LDSE) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q0 = (tid + h * NTHR) * 4;
      const int eb = __builtin_amdgcn_readfirstlane(q0 / pass.kcap);
      if (eb < pass.nblk) eptr[h] = (const uint32_t*)pass.ent[eb] + (q0 - eb * pass.kcap);
    }
  }
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  u4 ebuf[2] = {u4{0u, 0u, 0u, 0u}, u4{0u, 0u, 0u, 0u}};
  uint32_t bnd = 0, bndN = 0, bnd_nx = 0, bndN_nx = 0;
  auto load_meta = [&](int t) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (eptr[h]) ebuf[h] = *(const u4*)(eptr[h] + (int64_t)t * pass.kcap);
    if (active) {
      const int32_t* pb = ptr + (int64_t)t * prow;
      bnd_nx = lane < NJ ? (uint32_t)pb[lane] : 0u;
      bndN_nx = (uint32_t)pb[NJ];
    }
  };
  auto store_meta = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!eptr[h]) continue;
      uint32_t ad[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) ad[q] = (tile_lds + (ebuf[h][q] >> 1) * ROWB) | (ebuf[h][q] << 31);
      const int qb = (tid + h * NTHR) * 4;
      *(u4*)&ents[qb] = u4{ad[0], ad[1], ad[2], ad[3]};
    }
    bnd = bnd_nx;
    bndN = bndN_nx;
  };

  float acc[NJ][RPL];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
    for (int r = 0; r < RPL; ++r) acc[jj][r] = 0.f;
  const uint32_t lane_off = (uint32_t)lane * RPL * 4u;
  const uint32_t zaddr = (tile_lds + (uint32_t)KCK * ROWB) ^ lane_off;
  const char* tbase = (const char*)tile;
  auto LD = [&](int v) -> VT { return *(const VT*)(tbase + ((uint32_t)v >> 1) * ROWB + lane_off); };

  // the wave's sources of a chunk are src = wave + NW r (r < SPW); lane r
  // loads the coordinates of source r one chunk ahead and parks them in the
  // wave's own LDS slots (after the entries), whence the evaluation reads them
  // as one broadcast per source: no VALU slots, and no barrier beyond the
  // chunk's, since no other wave touches the slots
  constexpr int SPW = KCK / NW;
  static_assert(SPW <= 64 && KCK % NW == 0 && DIM <= 4, "one source per lane");
  typedef float f4 __attribute__((ext_vector_type(4)));
  f4* const xsl = (f4*)(smem + (size_t)(KCK + 1) * ROWB + (LDSE ? ((size_t)pass.nblk * pass.kcap + 8) * 8 : 0)) +
                  wave * SPW;
  float xs[DIM];
  auto load_xs = [&](int t) {
    const int64_t k = (int64_t)t * KCK + wave + NW * lane;
#pragma unroll
    for (int d = 0; d < DIM; ++d) xs[d] = (lane < SPW && k < N) ? X[k * DIM + d] * cs : 0.f;
  };
  auto store_xs = [&]() {
    f4 q = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < DIM; ++d) q[d] = xs[d];
    if (lane < SPW) xsl[lane] = q;
  };
  // kernel entries of the chunk into the tile; only the chunk that holds the
  // rows' own indices adds the diagonal shift
  auto eval = [&](int64_t k0, auto diag) {
    // sources of this chunk that exist (a uniform 32-bit bound: scalar compares)
    const int kn = (int)std::min<int64_t>(N - k0, (int64_t)KCK);
    // (unrolled by 4 only: a full unroll takes the kernel past 64 VGPRs, which
    // halves the workgroups per CU)
#pragma unroll 4
    for (int r = 0; r < SPW; ++r) {
      const int src = wave + NW * r;
      const int64_t k = k0 + src;
      float v[RPL];
#pragma unroll
      for (int p = 0; p < RPL; ++p) v[p] = 0.f;
      if (src < kn) {
        const f4 q = xsl[r];
#pragma unroll
        for (int p = 0; p < RPL; ++p) {
          float d2 = 0.f;
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            const float df = xi[p][d] - q[d];
            d2 = fmaf(df, df, d2);
          }
          v[p] = __builtin_amdgcn_exp2f(-d2);
          if constexpr (decltype(diag)::value)
            if (k == i0 + p) v[p] += shift;
        }
      }
      VT vv;
      __builtin_memcpy(&vv, v, sizeof(VT));
      *(VT*)(tile + src * TL + lane * RPL) = vv;
    }
  };
  const int tdiag = (int)(l0 / KCK);  // KCK is a multiple of TL: the tile's rows lie in one chunk

  if (t0 < t1) {
    if (LDSE) load_meta(t0);
    load_xs(t0);
    store_xs();
  }
  for (int t = t0; t < t1; ++t) {
    const int64_t k0 = (int64_t)t * KCK;
    __syncthreads();  // previous chunk consumed
    if constexpr (LDSE) store_meta();
    if (t + 1 < t1) load_xs(t + 1);
    if (t == tdiag) eval(k0, std::true_type{});
    else eval(k0, std::false_type{});
    if (LDSE && t + 1 < t1) load_meta(t + 1);  // in flight during the gather
    __syncthreads();
    if (active) {
      if constexpr (LDSE)
        gather_chunk_lds_win<float, NJ, RPL, VT, 4, true, RPL == 2>(ents, (t - blk) * pass.kcap, bnd, bndN,
                                                                           lane_off, zaddr, acc);
      else
        gather_chunk<float, NJ, RPL, VT>(ptr + (int64_t)t * prow, ent, LD, acc);
    }
    if (t + 1 < t1) store_xs();  // this wave's evaluation of chunk t is done
  }
  if (!active) return;
  const int64_t jc = (int64_t)g * NJ;
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int64_t i = i0 + p;
    if (i >= N) continue;
    if (split == 1) {
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) out[i + (jc + jj) * ldo] = acc[jj][p] * scale;
    } else {
      float* q = part + (int64_t)s * N * ((int64_t)pass.ngroups * NJ);
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) q[i + (jc + jj) * N] = acc[jj][p];
    }
  }
}

// ----------------------------------------------------------------- backward
struct MfBlocks {
  const uint32_t* codes[MAX_PASS_BLOCKS];  // per block: n * alpha hash codes
  int32_t coloff[MAX_PASS_BLOCKS];         // first column of the block inside W
  int32_t nb;
};

// row-major copy of the column-major N x w matrix W (tiled transpose)
__global__ void __launch_bounds__(256) transpose_kernel(const float* __restrict__ W, int64_t ldw, int64_t N, int w,
                                                        float* __restrict__ Wrm) {
  __shared__ float t[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + tx;
    const int c = c0 + y;
    t[y][tx] = (r < N && c < w) ? W[r + (int64_t)c * ldw] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + y;
    const int c = c0 + tx;
    if (r < N && c < w) Wrm[r * w + c] = t[tx][y];
  }
}

// One workgroup owns 64 points i (lanes); its NWB waves split the sources j
// into contiguous ranges.  G_ij reads the LDS copy of W's rows i (column named
// by the uniform hash of j: conflict-free); G_ji reads row j of W, which each
// wave stages in its own LDS slot (two rows at a time, the next two already in
// flight in registers), at the columns named by the hash of lane i.
//
// NA is the number of hash codes per source (blocks x alpha) rounded up to a
// multiple of 4; the codes past the true count na carry weight 0 (scalar
// selects, no branches), so the loop over codes is straight-line code with
// every per-code constant hoisted: per code and pair one readlane of the
// source's code, one address add, two FMAs.  Calls with more codes or columns
// run in groups of blocks; `mode` tells a group whether it writes dX (0: the
// only group), starts (1), adds to (2) or finishes (3) the FP64 sum in dXacc.
template <int DIM, int NWB, int NA>
__global__ void __launch_bounds__(NWB * 64)
    mf_bwd_kernel(const float* __restrict__ X, int64_t N, float c2, const float* __restrict__ W, int64_t ldw,
                  const float* __restrict__ Wrm, int Wt, MfBlocks mb, int alpha, float* __restrict__ dX,
                  float xscale, double* __restrict__ dh_part, double* __restrict__ dXacc, int mode) {
  constexpr int SRC = 2;    // sources staged per step and wave
  constexpr int GRP = 32;   // sources summed in FP32 before the FP64 accumulators
  extern __shared__ __attribute__((aligned(16))) float smem_f[];
  float* const Wr = smem_f;                   // Wr[col * 64 + lane] = W(l0 + lane, col), col < Wt
  float* const Wj = smem_f + (size_t)Wt * 64;  // per wave: SRC staged rows of Wt floats
  typedef __attribute__((address_space(3))) const float* lds_f;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * 64;
  const int64_t i = l0 + lane;
  const bool lane_ok = i < N;
  float* const myrows = Wj + (size_t)wave * SRC * Wt;

  for (int e = tid; e < Wt * 64; e += NWB * 64) {
    const int col = e >> 6, r = e & 63;
    Wr[e] = (l0 + r < N) ? W[(l0 + r) + (int64_t)col * ldw] : 0.f;
  }
  float xi[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xi[d] = lane_ok ? X[i * DIM + d] : 0.f;
  const int na = mb.nb * alpha;
  // per code q: the block's first column (uniform), this lane's own hash
  // column and sign (G_ji) and the LDS addresses of that column in the wave's
  // staged rows
  int cof[NA];
  float sgL[NA];
  uint32_t gja[SRC][NA];
  const uint32_t rows_lds = (uint32_t)(uintptr_t)(lds_f)myrows;
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    const int b = q < na ? q / alpha : 0, c = q % alpha;
    cof[q] = q < na ? mb.coloff[b] : 0;
    int colL = 0;
    sgL[q] = 0.f;
    if (q < na && lane_ok) {
      const uint32_t code = mb.codes[b][i * alpha + c];
      colL = (int)(code >> 1) + mb.coloff[b];
      sgL[q] = (code & 1u) ? -1.f : 1.f;
    }
#pragma unroll
    for (int u = 0; u < SRC; ++u) gja[u][q] = rows_lds + (uint32_t)(u * Wt + colL) * 4u;
  }
  const uint32_t wr_lane = (uint32_t)(uintptr_t)(lds_f)Wr + (uint32_t)lane * 4u;
  __syncthreads();

  // this wave's sources [js, js + len); rows are Wt / 4 pieces of 16 bytes
  const int64_t js = N * wave / NWB;
  const int len = (int)(N * (wave + 1) / NWB - js);
  const int npc = Wt / 4;
  typedef float f4v __attribute__((ext_vector_type(4)));
  f4v pf[SRC];
  auto fetch = [&](int r0) {
#pragma unroll
    for (int u = 0; u < SRC; ++u) {
      const int r = r0 + u;
      pf[u] = (lane < npc && r < len) ? *(const f4v*)(Wrm + (js + r) * Wt + 4 * lane) : f4v{0.f, 0.f, 0.f, 0.f};
    }
  };

  double ax[DIM], ah = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) ax[d] = 0.0;
  float px[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) px[d] = 0.f;
  int ng = 0;
  // coordinates and hash codes of the sources, 64 at a time: lane r holds those
  // of source jg + r, broadcast with readlane (no scalar-memory round trip per source)
  float xg[DIM];
  uint32_t cg[NA];
  auto load_group = [&](int r0) {
    const int r = r0 + lane;
    const bool ok = r < len;
    const int64_t j = js + r;
#pragma unroll
    for (int d = 0; d < DIM; ++d) xg[d] = ok ? X[j * DIM + d] : 0.f;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      cg[q] = 0u;
      if (q < na && ok) cg[q] = mb.codes[q / alpha][j * alpha + q % alpha];
    }
  };
  if (len > 0) fetch(0);
  for (int r0 = 0; r0 < len; r0 += SRC) {
    const int rl = r0 & 63;  // lane of source r0 in the group registers
    if (rl == 0) load_group(r0);
    // stage this step's rows (the wave's earlier reads of its slot are done:
    // LDS operations of one wave complete in order), then fetch the next step
#pragma unroll
    for (int u = 0; u < SRC; ++u)
      if (lane < npc) *(f4v*)(myrows + u * Wt + 4 * lane) = pf[u];
    if (r0 + SRC < len) fetch(r0 + SRC);
#pragma unroll
    for (int u = 0; u < SRC; ++u) {
      if (r0 + u >= len) break;
      float df[DIM], r2 = 0.f;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        df[d] = xi[d] - __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, xg[d]), rl + u));
        r2 = fmaf(df[d], df[d], r2);
      }
      const float K = __builtin_amdgcn_exp2f(-r2 * c2);
      float gij = 0.f, gji = 0.f;
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const uint32_t code = (uint32_t)__builtin_amdgcn_readlane((int)cg[q], rl + u);
        // +-1.0f, or +0.0f past the true code count (integer select: stays scalar)
        const uint32_t keep = q < na ? 0xffffffffu : 0u;
        const float sg = __builtin_bit_cast(float, ((code << 31) | 0x3f800000u) & keep);
        const uint32_t wa = (((code >> 1) + (uint32_t)cof[q]) << 8) + wr_lane;
        gij = fmaf(*(lds_f)(uintptr_t)wa, sg, gij);
        gji = fmaf(*(lds_f)(uintptr_t)gja[u][q], sgL[q], gji);
      }
      const float M = (gij + gji) * K;
#pragma unroll
      for (int d = 0; d < DIM; ++d) px[d] = fmaf(M, df[d], px[d]);
      ah += (double)(gij * K * r2);  // dL/dh cancels heavily: accumulate its terms in FP64
    }
    ng += SRC;
    if (ng >= GRP) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        ax[d] += (double)px[d];
        px[d] = 0.f;
      }
      ng = 0;
    }
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d) ax[d] += (double)px[d];
  // combine the waves in a fixed order (the LDS rows of W are no longer read)
  __syncthreads();
  double* const red = (double*)smem_f;  // [NWB][DIM + 1][64]
#pragma unroll
  for (int d = 0; d < DIM; ++d) red[(wave * (DIM + 1) + d) * 64 + lane] = ax[d];
  red[(wave * (DIM + 1) + DIM) * 64 + lane] = lane_ok ? ah : 0.0;
  __syncthreads();
  if (wave == 0) {
    double sx[DIM], sh = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) sx[d] = 0.0;
    for (int q = 0; q < NWB; ++q) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) sx[d] += red[(q * (DIM + 1) + d) * 64 + lane];
      sh += red[(q * (DIM + 1) + DIM) * 64 + lane];
    }
    if (lane_ok) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double v = sx[d] * (double)xscale;
        if (mode == 0) dX[i * DIM + d] = (float)v;
        else if (mode == 1) dXacc[i * DIM + d] = v;
        else if (mode == 2) dXacc[i * DIM + d] += v;
        else dX[i * DIM + d] = (float)(dXacc[i * DIM + d] + v);
      }
    }
    red[DIM * 64 + lane] = sh;  // slot of wave 0, item DIM: read back below by thread 0 only
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int l = 0; l < 64; ++l) t += red[DIM * 64 + l];
    dh_part[blockIdx.x] = t;
  }
}

__global__ void dh_reduce_kernel(const double* __restrict__ part, int64_t np, double scale, double* __restrict__ dh) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int64_t q = 0; q < np; ++q) t += part[q];
  *dh = t * scale;
}

// ------------------------------------------------------------------ launch
// dynamic LDS of the forward: tile with its zero slot, (ldse) the entries, the
// per-wave source coordinates
static size_t mf_lds_bytes(int kc, int rpl, bool ldse, int nblk, int kcap) {
  return (size_t)(kc + 1) * 64 * rpl * 4 + (ldse ? ((size_t)nblk * kcap + 8) * 8 : 0) + (size_t)kc * 16;
}

template <int NW, int NJ, int KCK, bool LDSE, int RPL = 1>
static int run_mf(Ctx* c, int dim, const float* X, int64_t N, float cs, float shift, const SjltPass& pass,
                  float* out, int64_t ldo, float scale, int split, float* part, int gz, hipStream_t st) {
  constexpr int TL = 64 * RPL;
  dim3 grid((unsigned)((N + TL - 1) / TL), (unsigned)split, (unsigned)gz);
  // tile with its zero slot, (LDSE) the entries, the per-wave source coordinates
  const size_t shmem = mf_lds_bytes(KCK, RPL, LDSE, pass.nblk, pass.kcap);
  auto kern = dim == 1 ? mf_sjlt_kernel<NW, NJ, KCK, 1, LDSE, RPL>
              : dim == 2 ? mf_sjlt_kernel<NW, NJ, KCK, 2, LDSE, RPL>
              : dim == 3 ? mf_sjlt_kernel<NW, NJ, KCK, 3, LDSE, RPL> : mf_sjlt_kernel<NW, NJ, KCK, 4, LDSE, RPL>;
  static bool attr_set[4] = {false, false, false, false};
  if (!attr_set[dim - 1]) {
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_set[dim - 1] = true;
  }
  ProfScope ps(c, "mf_fwd", st);
  kern<<<grid, NW * 64, shmem, st>>>(X, N, cs, shift, pass, out, ldo, scale, split, part);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

static constexpr double LOG2E = 1.4426950408889634;

int launch_mf_pass(Handle* h, const sk_input* in, int b0, int b1, void* out, int64_t ldo, hipStream_t st) {
  SK_REQUIRE(h->kind == SK_SJLT, SK_EUNSUPPORTED, "the matrix-free kernel sketch uses the SJLT operator");
  const int nblk = b1 - b0;
  SK_REQUIRE(nblk >= 1 && nblk <= MAX_PASS_BLOCKS, SK_EINVAL, "a pass covers 1..%d blocks", MAX_PASS_BLOCKS);
  int W = 0, g = 0;
  for (int b = b0; b < b1; ++b) {
    W += h->blocks[b].w;
    int a = g, bb = h->blocks[b].w;
    while (bb) {
      const int t = a % bb;
      a = bb;
      bb = t;
    }
    g = a;
  }
  // 16 columns per wave and 16 waves from 256 columns on (more waves per CU to
  // overlap the kernel evaluation with the gather: N = 32768, d = 256 forward
  // 1.71 -> 1.52 ms), else 32 columns
  const bool wide = W >= 256;
  const int nj = wide ? 16 : (g % 32 == 0 && W >= 128) ? 32 : 16;
  const int ngroups = W / nj;
  SK_REQUIRE(ngroups <= MAX_PASS_GROUPS, SK_EINVAL, "pass too wide (%d columns)", W);
  const int nw = wide ? 16 : ngroups <= 4 ? 4 : 8;
  const int gz = (ngroups + nw - 1) / nw;
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
    for (int c = 0; c < B.w; c += nj) {
      pass.grp_blk[gi] = b - b0;
      pass.grp_col[gi] = c;
      ++gi;
    }
  }
  const int64_t N = in->N;
  const int kc = h->kc;
  // bucket entries staged in LDS (four per thread and staging round, one chunk
  // ahead) when every block of the pass has the same chunk region size
  pass.nblk = nblk;
  pass.kcap = 0;
  bool same = true;
  for (int b = b0; b < b1; ++b) pass.kcap = std::max(pass.kcap, sjlt_kcap(kc, h->alpha, h->blocks[b].w));
  for (int b = b0; b < b1; ++b) same = same && sjlt_kcap(kc, h->alpha, h->blocks[b].w) == pass.kcap;
  {
    const int64_t lam2 = 2LL * kc * h->alpha * nblk / W;
    pass.ms = lam2 >= 14 ? 8 : 4;
  }
  const bool ldse = same && (int64_t)nblk * pass.kcap <= (int64_t)nw * 64 * 8 &&
                    mf_lds_bytes(kc, 1, true, nblk, pass.kcap) <= 160 * 1024;
  // wide passes: two points per lane when the 128-point tile fits beside the
  // entries (one workgroup of 16 waves per CU): every staged entry then serves
  // two additions, which halves the gather's address, mask and bound work
  const int rpl = ldse && wide && kc >= 128 && mf_lds_bytes(kc, 2, true, nblk, pass.kcap) <= 160 * 1024 ? 2 : 1;
  const int64_t tiles = ((N + 64 * rpl - 1) / (64 * rpl)) * gz;
  const size_t tile_bytes = mf_lds_bytes(kc, rpl, ldse, nblk, pass.kcap);
  const int64_t per_cu = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)tile_bytes);
  const int64_t target = per_cu * (int64_t)h->ctx->num_cu;
  int split = 1;
  if (tiles < target) split = (int)std::min<int64_t>((target + tiles - 1) / tiles, std::max(1, pass.nT / 4));
  float* part = nullptr;
  if (split > 1) {
    if (int rc = ensure_work(h->ctx, (size_t)split * (size_t)N * (size_t)W * 4)) return rc;
    part = (float*)work_ptr(h->ctx);
  }
  const float cs = (float)sqrt(LOG2E / (2.0 * (double)in->h * (double)in->h));
  const float scale = (float)(1.0 / sqrt((double)h->alpha));
  int rc = SK_EINVAL;
#define SK_MF(NW_, NJ_, KC_)                                                                                          \
  if (nw == NW_ && nj == NJ_ && kc == KC_ && rpl == 1)                                                                \
    rc = ldse ? run_mf<NW_, NJ_, KC_, true>(h->ctx, in->dim, in->X, N, cs, in->shift, pass, (float*)out, ldo, scale, \
                                            split, part, gz, st)                                                     \
              : run_mf<NW_, NJ_, KC_, false>(h->ctx, in->dim, in->X, N, cs, in->shift, pass, (float*)out, ldo, scale, \
                                             split, part, gz, st);                                                   \
  else
#define SK_MF2(NW_, NJ_, KC_)                                                                                        \
  if (nw == NW_ && nj == NJ_ && kc == KC_ && rpl == 2)                                                               \
    rc = run_mf<NW_, NJ_, KC_, true, 2>(h->ctx, in->dim, in->X, N, cs, in->shift, pass, (float*)out, ldo, scale,    \
                                        split, part, gz, st);                                                       \
  else
  SK_MF(4, 16, 64) SK_MF(8, 16, 64) SK_MF(4, 32, 64) SK_MF(8, 32, 64)
  SK_MF(4, 16, 128) SK_MF(8, 16, 128) SK_MF(4, 32, 128) SK_MF(8, 32, 128)
  SK_MF(4, 16, 256) SK_MF(8, 16, 256) SK_MF(4, 32, 256) SK_MF(8, 32, 256)
  SK_MF(16, 16, 64) SK_MF(16, 16, 128) SK_MF(16, 16, 256)
  SK_MF2(16, 16, 128) SK_MF2(16, 16, 256) {
    set_error("internal: no matrix-free kernel for NW=%d NJ=%d KC=%d RPL=%d", nw, nj, kc, rpl);
  }
#undef SK_MF2
#undef SK_MF
  if (rc) return rc;
  if (split > 1) {
    ProfScope ps(h->ctx, "sjlt_reduce", st);
    split_reduce_f32(part, split, N, W, (float*)out, ldo, scale, st);
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

int launch_mf_backward(Handle* h, const sk_input* in, int b0, int b1, const float* Wd, int64_t ldw, float* dX,
                       double* dh, hipStream_t st) {
  SK_REQUIRE(h->kind == SK_SJLT, SK_EUNSUPPORTED, "the matrix-free backward uses the SJLT operator");
  const int nblk = b1 - b0;
  SK_REQUIRE(nblk >= 1, SK_EINVAL, "the backward covers at least one block");
  SK_REQUIRE(h->alpha <= 16, SK_EUNSUPPORTED, "the matrix-free backward supports alpha <= 16");
  for (int b = b0; b < b1; ++b)
    SK_REQUIRE(h->blocks[b].w <= 256, SK_EUNSUPPORTED, "the matrix-free backward supports blocks of <= 256 columns");
  // groups of consecutive blocks with at most 16 hash codes per source and 256
  // columns each; every group recomputes the kernel entries and adds its part
  // of dL/dX (FP64 across groups) and its dL/dh partials
  std::vector<std::pair<int, int>> groups;
  for (int p0 = b0; p0 < b1;) {
    int p1 = p0, codes = 0, cols = 0;
    while (p1 < b1 && p1 - p0 < MAX_PASS_BLOCKS && codes + h->alpha <= 16 && cols + h->blocks[p1].w <= 256) {
      codes += h->alpha;
      cols += h->blocks[p1++].w;
    }
    groups.emplace_back(p0, p1);
    p0 = p1;
  }
  const int ng = (int)groups.size();
  const int64_t N = in->N;
  const int64_t nwg = (N + 63) / 64;
  int Wmax = 0;
  for (auto& gp : groups) {
    int w = 0;
    for (int b = gp.first; b < gp.second; ++b) w += h->blocks[b].w;
    Wmax = std::max(Wmax, w);
  }
  // workspace: row-major copy of the group's columns of W, the dh partials of
  // every group, and (several groups) the FP64 sum of dL/dX
  const size_t wrm_bytes = ((size_t)N * Wmax * 4 + 255) & ~(size_t)255;
  const size_t dhp_bytes = ((size_t)ng * nwg * 8 + 255) & ~(size_t)255;
  const size_t acc_bytes = ng > 1 ? (size_t)N * in->dim * 8 : 0;
  if (int rc = ensure_work(h->ctx, wrm_bytes + dhp_bytes + acc_bytes)) return rc;
  float* Wrm = (float*)work_ptr(h->ctx);
  double* dh_part = (double*)((char*)work_ptr(h->ctx) + wrm_bytes);
  double* dXacc = ng > 1 ? (double*)((char*)work_ptr(h->ctx) + wrm_bytes + dhp_bytes) : nullptr;
  const double hh = (double)in->h;
  const float c2 = (float)(LOG2E / (2.0 * hh * hh));
  const double ga = 1.0 / sqrt((double)h->alpha);
  const float xscale = (float)(-ga / (hh * hh));
  constexpr int NWB = 8;
  int col0 = 0;
  for (int gi = 0; gi < ng; ++gi) {
    const int p0 = groups[gi].first, p1 = groups[gi].second;
    MfBlocks mb;
    memset(&mb, 0, sizeof(mb));
    int Wt = 0;
    for (int b = p0; b < p1; ++b) {
      mb.codes[b - p0] = h->blocks[b].codes;
      mb.coloff[b - p0] = Wt;
      Wt += h->blocks[b].w;
    }
    mb.nb = p1 - p0;
    const float* Wg = Wd + (int64_t)col0 * ldw;
    {
      dim3 grid((unsigned)((N + 31) / 32), (unsigned)((Wt + 31) / 32));
      transpose_kernel<<<grid, 256, 0, st>>>(Wg, ldw, N, Wt, Wrm);
      SK_HIP(hipGetLastError());
    }
    // W rows i + two staged rows j per wave; the end-of-kernel reduction reuses it
    const size_t shmem = std::max((size_t)Wt * 64 * 4 + (size_t)NWB * 2 * Wt * 4, (size_t)NWB * 5 * 64 * 8);
    const int na = mb.nb * h->alpha;
    const int NAr = (na + 3) / 4 * 4;
    const int mode = ng == 1 ? 0 : gi == 0 ? 1 : gi + 1 < ng ? 2 : 3;
    ProfScope ps(h->ctx, "mf_bwd", st);
    const dim3 grid((unsigned)nwg);
    typedef void (*KernT)(const float*, int64_t, float, const float*, int64_t, const float*, int, MfBlocks, int,
                          float*, float, double*, double*, int);
    KernT kern = nullptr;
#define SK_MFB(D_)                                                                                               \
  if (in->dim == D_)                                                                                             \
    kern = NAr == 4 ? mf_bwd_kernel<D_, NWB, 4> : NAr == 8 ? mf_bwd_kernel<D_, NWB, 8>                          \
         : NAr == 12 ? mf_bwd_kernel<D_, NWB, 12> : mf_bwd_kernel<D_, NWB, 16>;
    SK_MFB(1) SK_MFB(2) SK_MFB(3) SK_MFB(4)
#undef SK_MFB
    SK_REQUIRE(kern, SK_EINVAL, "internal: no matrix-free backward for dim %d", in->dim);
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    kern<<<grid, NWB * 64, shmem, st>>>(in->X, N, c2, Wg, ldw, Wrm, Wt, mb, h->alpha, dX, xscale,
                                        dh_part + (size_t)gi * nwg, dXacc, mode);
    SK_HIP(hipGetLastError());
    col0 += Wt;
  }
  dh_reduce_kernel<<<1, 64, 0, st>>>(dh_part, (int64_t)ng * nwg, ga / (hh * hh * hh), dh);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk

// Gaussian sketch S = A R_b on the matrix cores (section 2.4.1: R_b has i.i.d.
// N(0, 1/w_b) entries; the product is a dense contraction, O(m n w) flops).
// The draws g are stored on the bfloat16 grid, column-major; the 1/sqrt(w_b)
// scale is applied to the result.
//
// gauss_f64_kernel: v_mfma_f64_16x16x4_f64.  A workgroup of 4 waves owns 64 rows;
//   wave q computes rows 16q..16q+15 against up to 256 columns.  A fragments are
//   read straight from global memory (16 consecutive rows per column, coalesced);
//   the R chunk (16 k x W, exact in FP64) is staged once per workgroup in LDS.
//   FP32 inputs are promoted on load, so this is also the FP64 reference for FP32 A.
// gauss_bf16_kernel: v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  The 16x32
//   A fragment needs 8 consecutive k per row while A is column-major, so each
//   64 x 64 chunk of A is loaded in 4x4 blocks, rounded to bf16 (and, for
//   bf16x3, split exactly a = a1 + a2 + a3 into three bf16 parts), transposed in
//   registers and written to LDS rows of k (padded rows: conflict-free reads).
#include <algorithm>

#include "internal.hpp"

namespace sk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4g __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double bf16_bits_to_double(uint16_t b) {
  return (double)__builtin_bit_cast(float, (uint32_t)b << 16);
}

// ------------------------------------------------------------------- FP64
// Element (i, k) of the contracted matrix: A(i, k) for S, A(k, i) for S' = A^T R.
template <bool TRANS, typename TA>
__device__ __forceinline__ TA aelem(const TA* __restrict__ A, int64_t lda, int64_t i, int64_t k) {
  return TRANS ? A[k + i * lda] : A[i + k * lda];
}

template <typename TA, typename TS, bool TRANS, int NB>
__global__ void __launch_bounds__(256)
    gauss_f64_kernel(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n, const uint16_t* __restrict__ g,
                     int64_t ldg, int W, TS* __restrict__ S, int64_t ldS, double scale) {
  constexpr int KT = 16;
  constexpr int WP = NB * 16;
  __shared__ double Rl[KT * WP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int q = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + 16 * q;
  const int jbase = blockIdx.z * WP;  // first column of this workgroup inside the block
  const int wloc = std::min(WP, W - jbase);
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t arow = row0 + lr;

  d4 acc[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) acc[cb] = d4{0, 0, 0, 0};

  // R staging: thread -> column j = tid % WP and a run of KS consecutive k
  constexpr int KS = KT * WP / 256;
  const int sj = tid % WP, sk0 = (tid / WP) * KS;

  for (int64_t k0 = 0; k0 < n; k0 += KT) {
    double rv[KS];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int64_t k = k0 + sk0 + u;
      rv[u] = (sj < wloc && k < n) ? bf16_bits_to_double(g[k + (int64_t)(jbase + sj) * ldg]) : 0.0;
    }
    double af[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * s + lk;
      af[s] = (arow < m && k < n) ? (double)aelem<TRANS>(A, lda, arow, k) : 0.0;
    }
    __syncthreads();  // previous chunk consumed
#pragma unroll
    for (int u = 0; u < KS; ++u) Rl[(sk0 + u) * WP + sj] = rv[u];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const double b = Rl[(4 * s + lk) * WP + cb * 16 + lr];
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s], b, acc[cb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int j = jbase + cb * 16 + lr;
    if (j >= W) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // v_mfma_f64_16x16x4f64 returns D[4 v + lane / 16][lane % 16] in item v
      const int64_t r = row0 + 4 * v + lk;
      if (r < m) S[r + (int64_t)j * ldS] = (TS)(acc[cb][v] * scale);
    }
  }
}

// ------------------------------------------------------------------- BF16
template <int NB, bool X3, bool TRANS>
__global__ void __launch_bounds__(256)
    gauss_bf16_kernel(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                      const uint16_t* __restrict__ g, int64_t ldg, int W, float* __restrict__ S, int64_t ldS,
                      float scale) {
  constexpr int KT = 64;
  constexpr int NP = X3 ? 3 : 1;
  constexpr int RS = KT + 8;  // padded row length (bf16 elements): 144 bytes
  constexpr int WP = NB * 16;
  __shared__ __attribute__((aligned(16))) __bf16 At[NP][64 * RS];
  __shared__ __attribute__((aligned(16))) __bf16 Rt[WP * RS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int q = tid >> 6;
  const int64_t rowblk = (int64_t)blockIdx.x * 64;
  const int jbase = blockIdx.z * WP;
  const int wloc = std::min(WP, W - jbase);
  const int lr = lane & 15, lk = lane >> 4;

  // A staging: thread -> 4x4 block (rows 4*rb.., columns 4*cb..)
  const int rb = tid >> 4, cbk = tid & 15;  // 16 row blocks x 16 column blocks
  const int64_t ar0 = rowblk + 4 * rb;
  f4 acc[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) acc[cb] = f4{0.f, 0.f, 0.f, 0.f};

  for (int64_t k0 = 0; k0 < n; k0 += KT) {
    float a[4][4];  // [column][row]
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t k = k0 + 4 * cbk + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = ar0 + r;
        a[c][r] = (row < m && k < n) ? aelem<TRANS>(A, lda, row, k) : 0.f;
      }
    }
    // R chunk: WP columns x KT k, thread -> (column, 8 consecutive k)
    constexpr int RV = WP * KT / 8 / 256;  // 16-byte pieces per thread (>= 1 for WP >= 32)
    uint32_t rpiece[RV > 0 ? RV : 1][4];
#pragma unroll
    for (int u = 0; u < (RV > 0 ? RV : 1); ++u) {
      const int pid = u * 256 + tid;
      const int j = pid / (KT / 8), kk = (pid % (KT / 8)) * 8;
      uint16_t hv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + kk + e;
        hv[e] = (pid < WP * KT / 8 && j < wloc && k < n) ? g[k + (int64_t)(jbase + j) * ldg] : (uint16_t)0;
      }
      __builtin_memcpy(rpiece[u], hv, 16);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      __bf16 p1[4], p2[4], p3[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float x = a[c][r];
        const __bf16 h1 = (__bf16)x;
        p1[c] = h1;
        if (X3) {
          const float r1 = x - (float)h1;
          const __bf16 h2 = (__bf16)r1;
          p2[c] = h2;
          p3[c] = (__bf16)(r1 - (float)h2);
        }
      }
      const int off = (4 * rb + r) * RS + 4 * cbk;
      __builtin_memcpy(&At[0][off], p1, 8);
      if (X3) {
        __builtin_memcpy(&At[1 % NP][off], p2, 8);
        __builtin_memcpy(&At[2 % NP][off], p3, 8);
      }
    }
#pragma unroll
    for (int u = 0; u < (RV > 0 ? RV : 1); ++u) {
      const int pid = u * 256 + tid;
      if (pid < WP * KT / 8) {
        const int j = pid / (KT / 8), kk = (pid % (KT / 8)) * 8;
        __builtin_memcpy(&Rt[j * RS + kk], rpiece[u], 16);
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KT / 32; ++ks) {
      bf8 af[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) __builtin_memcpy(&af[p], &At[p][(16 * q + lr) * RS + 32 * ks + 8 * lk], 16);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        bf8 bfr;
        __builtin_memcpy(&bfr, &Rt[(cb * 16 + lr) * RS + 32 * ks + 8 * lk], 16);
#pragma unroll
        for (int p = NP - 1; p >= 0; --p)  // small parts first
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[p], bfr, acc[cb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int j = jbase + cb * 16 + lr;
    if (j >= W) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // v_mfma_f32_16x16x32_bf16 returns D[4 (lane / 16) + v][lane % 16] in item v
      const int64_t r = rowblk + 16 * q + 4 * lk + v;
      if (r < m) S[r + (int64_t)j * ldS] = acc[cb][v] * scale;
    }
  }
}

// ------------------------------------------------------------------ launch
template <typename TA, typename TS, bool TRANS>
static int run_f64(Ctx* c, const TA* A, int64_t lda, int64_t m, int64_t n, const uint16_t* g, int W, TS* S,
                   int64_t ldS, double scale, hipStream_t st) {
  // columns per workgroup: W rounded up to 16, at most 256
  const int nb = std::min(16, (W + 15) / 16);
  const int nbk = nb <= 2 ? 2 : nb <= 4 ? 4 : nb <= 8 ? 8 : 16;
  const int gz = (W + nbk * 16 - 1) / (nbk * 16);
  dim3 grid((unsigned)((m + 63) / 64), 1, (unsigned)gz);
  ProfScope ps(c, TRANS ? "gauss_f64_t" : "gauss_f64", st);
  if (nbk == 2) gauss_f64_kernel<TA, TS, TRANS, 2><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale);
  else if (nbk == 4) gauss_f64_kernel<TA, TS, TRANS, 4><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale);
  else if (nbk == 8) gauss_f64_kernel<TA, TS, TRANS, 8><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale);
  else gauss_f64_kernel<TA, TS, TRANS, 16><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <bool TRANS>
static int run_bf16(Ctx* c, bool x3, const float* A, int64_t lda, int64_t m, int64_t n, const uint16_t* g, int W,
                    float* S, int64_t ldS, float scale, hipStream_t st) {
  const int nb = std::min(16, (W + 15) / 16);
  const int nbk = nb <= 2 ? 2 : nb <= 4 ? 4 : nb <= 8 ? 8 : 16;
  const int gz = (W + nbk * 16 - 1) / (nbk * 16);
  dim3 grid((unsigned)((m + 63) / 64), 1, (unsigned)gz);
  ProfScope ps(c, x3 ? (TRANS ? "gauss_bf16x3_t" : "gauss_bf16x3") : (TRANS ? "gauss_bf16_t" : "gauss_bf16"), st);
#define SK_BF_CASE(NB_)                                                                                      \
  if (nbk == NB_) {                                                                                          \
    if (x3) gauss_bf16_kernel<NB_, true, TRANS><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale); \
    else gauss_bf16_kernel<NB_, false, TRANS><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale);  \
  }
  SK_BF_CASE(2) SK_BF_CASE(4) SK_BF_CASE(8) SK_BF_CASE(16)
#undef SK_BF_CASE
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_gauss_pass(Handle* h, const sk_input* in, int b0, int b1, bool trans, void* out, int64_t ldo,
                      hipStream_t st) {
  // one launch per block: each block has its own draws and its own 1/sqrt(w_b)
  int64_t col = 0;
  const size_t esz = h->dtype == SK_F64 ? 8 : 4;
  const int64_t M = trans ? in->n : in->m;  // rows of the result
  const int64_t K = trans ? in->m : in->n;  // contraction length = rows of R
  for (int b = b0; b < b1; ++b) {
    const Block& B = h->blocks[b];
    const double scale = 1.0 / sqrt((double)B.w);
    char* o = (char*)out + (size_t)col * ldo * esz;
    int rc;
    if (h->prec == SK_PREC_NATIVE) {
      if (h->dtype == SK_F64)
        rc = trans ? run_f64<double, double, true>(h->ctx, (const double*)in->A, in->lda, M, K, B.gbf, B.w,
                                                   (double*)o, ldo, scale, st)
                   : run_f64<double, double, false>(h->ctx, (const double*)in->A, in->lda, M, K, B.gbf, B.w,
                                                    (double*)o, ldo, scale, st);
      else
        rc = trans ? run_f64<float, float, true>(h->ctx, (const float*)in->A, in->lda, M, K, B.gbf, B.w, (float*)o,
                                                 ldo, scale, st)
                   : run_f64<float, float, false>(h->ctx, (const float*)in->A, in->lda, M, K, B.gbf, B.w,
                                                  (float*)o, ldo, scale, st);
    } else {
      const bool x3 = h->prec == SK_PREC_BF16X3;
      rc = trans ? run_bf16<true>(h->ctx, x3, (const float*)in->A, in->lda, M, K, B.gbf, B.w, (float*)o, ldo,
                                  (float)scale, st)
                 : run_bf16<false>(h->ctx, x3, (const float*)in->A, in->lda, M, K, B.gbf, B.w, (float*)o, ldo,
                                   (float)scale, st);
    }
    if (rc) return rc;
    col += B.w;
  }
  return SK_OK;
}

}  // namespace sk

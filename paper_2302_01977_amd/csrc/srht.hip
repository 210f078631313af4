// SRHT sketch of a stored, column-major A (section 7.1: S = A D H P, the cost
// dominated by the Hadamard transform), any n: H = H_nu with nu = 2^ceil(log2 n)
// and A, D padded with zeros past n (section 7.2).
//
// Sampled output column j picks Hadamard column mu_j (section 7.2, element
// formula (H)_{k,mu} = (-1)^{popcount(k & mu)}), so
//     S(i, j) = (1/sqrt(w)) sum_k A(i,k) D_k (-1)^{popcount(k & mu_j)}.
// With k = i2 * G + i1 and mu = j2 * G + j1 the sign factors as
// (-1)^{popcount(i1 & j1)} (-1)^{popcount(i2 & j2)}, i.e. H_nu = H_{nu/G} (x) H_G.
//
// A workgroup owns 64 lanes (rows of A for S, columns of A for S') and walks the
// source index k in batches of NW groups of G consecutive sources:
//   1. each wave loads one group for its 64 lanes, applies D and a G-point fast
//      Walsh-Hadamard transform in registers (natural order, unnormalised) and
//      writes the result Z_{i2}[i1] to LDS;
//   2. a NW-point transform across the batch's groups is done in LDS, giving
//      Y_p[j1] = sum_q (-1)^{popcount(q & p)} Z_{g0+q}[j1];
//   3. every wave gathers its sampled columns:
//         acc_j += (-1)^{popcount(g0 & j2)} Y_{j2 mod NW}[j1],
//      one LDS read per sampled column and batch (g0 is a multiple of NW).
// Only the sampled outputs of the last factor are formed.  Sources past n are
// zero, which leaves the transform at indices < n unchanged, so any n works.
#include <algorithm>

#include "internal.hpp"

namespace sk {

template <typename T, bool TRANS, int G, int NW, int NJ>
__global__ void __launch_bounds__(NW * 64)
    srht_kernel(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, const T* __restrict__ Dv,
                const uint32_t* __restrict__ mu, int64_t col0, int W, T* __restrict__ out, int64_t ldo, T scale) {
  static_assert((G & (G - 1)) == 0 && (NW & (NW - 1)) == 0, "powers of two");
  constexpr int LG = __builtin_ctz(G);
  __shared__ T Z[NW * G * 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * 64;
  const int64_t lrow = l0 + lane;  // this lane's row of S (row of A, or column of A for S')
  const int jw = (blockIdx.z * NW + wave) * NJ;  // first sampled column of this wave
  const bool lane_ok = lrow < L;

  T acc[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) acc[jj] = T(0);

  const int64_t ngroups = (K + G - 1) / G;
  for (int64_t g0 = 0; g0 < ngroups; g0 += NW) {
    // ---- 1. group transform in registers
    const int64_t g = g0 + wave;
    T x[G];
    if (g < ngroups) {
      const int64_t k0 = g * G;
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const int64_t k = k0 + c;
        T v = T(0);
        if (lane_ok && k < K) v = TRANS ? A[k + lrow * lda] : A[lrow + k * lda];
        x[c] = k < K ? v * Dv[k] : T(0);
      }
    } else {
#pragma unroll
      for (int c = 0; c < G; ++c) x[c] = T(0);
    }
#pragma unroll
    for (int h = 1; h < G; h <<= 1) {
#pragma unroll
      for (int c = 0; c < G; ++c) {
        if (c & h) continue;
        const T a = x[c], b = x[c + h];
        x[c] = a + b;
        x[c + h] = a - b;
      }
    }
    __syncthreads();  // the previous batch's gather is done with Z
#pragma unroll
    for (int c = 0; c < G; ++c) Z[(wave * G + c) * 64 + lane] = x[c];
    __syncthreads();
    // ---- 2. NW-point transform across the groups of the batch
    if (NW > 1) {
      for (int pos = tid; pos < G * 64; pos += NW * 64) {
        T y[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) y[q] = Z[q * G * 64 + pos];
#pragma unroll
        for (int h = 1; h < NW; h <<= 1) {
#pragma unroll
          for (int q = 0; q < NW; ++q) {
            if (q & h) continue;
            const T a = y[q], b = y[q + h];
            y[q] = a + b;
            y[q + h] = a - b;
          }
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) Z[q * G * 64 + pos] = y[q];
      }
      __syncthreads();
    }
    // ---- 3. gather the sampled columns
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const int j = jw + jj;
      if (j < W) {
        const uint32_t m = mu[col0 + j];
        const uint32_t j1 = m & (G - 1), j2 = m >> LG;
        const uint32_t p = j2 & (NW - 1);
        const T sg = (__popcll((uint64_t)g0 & (uint64_t)j2) & 1) ? T(-1) : T(1);
        acc[jj] = fma(Z[(p * G + j1) * 64 + lane], sg, acc[jj]);
      }
    }
  }
  if (!lane_ok) return;
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int j = jw + jj;
    if (j < W) out[lrow + (int64_t)j * ldo] = acc[jj] * scale;
  }
}

template <typename T, bool TRANS, int G, int NJ>
static int run_srht(Ctx* c, const T* A, int64_t lda, int64_t L, int64_t K, const T* Dv, const uint32_t* mu,
                    int64_t col0, int W, T* out, int64_t ldo, T scale, hipStream_t st) {
  constexpr int NW = 4;
  const int gz = (W + NW * NJ - 1) / (NW * NJ);
  dim3 grid((unsigned)((L + 63) / 64), 1, (unsigned)gz);
  ProfScope ps(c, TRANS ? "srht_t" : "srht", st);
  srht_kernel<T, TRANS, G, NW, NJ><<<grid, NW * 64, 0, st>>>(A, lda, L, K, Dv, mu, col0, W, out, ldo, scale);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename T, bool TRANS>
static int srht_dispatch(Ctx* c, int W, const T* A, int64_t lda, int64_t L, int64_t K, const T* Dv,
                         const uint32_t* mu, int64_t col0, T* out, int64_t ldo, T scale, hipStream_t st) {
  constexpr int G = sizeof(T) == 8 ? 32 : 64;
  if (W <= 64) return run_srht<T, TRANS, G, 16>(c, A, lda, L, K, Dv, mu, col0, W, out, ldo, scale, st);
  if (W <= 128) return run_srht<T, TRANS, G, 32>(c, A, lda, L, K, Dv, mu, col0, W, out, ldo, scale, st);
  return run_srht<T, TRANS, G, 64>(c, A, lda, L, K, Dv, mu, col0, W, out, ldo, scale, st);
}

int launch_srht_pass(Handle* h, const sk_input* in, int b0, int b1, bool trans, void* out, int64_t ldo,
                     hipStream_t st) {
  // every block of the pass is normalised by its own width: run block by block
  // when the widths differ, otherwise in one launch
  const int64_t L = trans ? in->n : in->m;
  const int64_t K = trans ? in->m : in->n;
  int64_t col = 0;
  const size_t esz = h->dtype == SK_F64 ? 8 : 4;
  int b = b0;
  while (b < b1) {
    int e = b + 1;
    while (e < b1 && h->blocks[e].w == h->blocks[b].w) ++e;
    int W = 0;
    for (int q = b; q < e; ++q) W += h->blocks[q].w;
    const double scale = 1.0 / sqrt((double)h->blocks[b].w);
    char* o = (char*)out + (size_t)col * ldo * esz;
    int rc = launch_srht_dma(h->ctx, h->dtype, trans, in->A, in->lda, L, K, h->srht_Db, h->srht_mu,
                             h->blocks[b].col0, W, o, ldo, scale, st);
    if (rc != 1) {
      if (rc) return rc;
    } else if (h->dtype == SK_F64) {
      rc = trans ? srht_dispatch<double, true>(h->ctx, W, (const double*)in->A, in->lda, L, K,
                                               (const double*)h->srht_Dv, h->srht_mu, h->blocks[b].col0,
                                               (double*)o, ldo, scale, st)
                 : srht_dispatch<double, false>(h->ctx, W, (const double*)in->A, in->lda, L, K,
                                                (const double*)h->srht_Dv, h->srht_mu, h->blocks[b].col0,
                                                (double*)o, ldo, scale, st);
    } else {
      rc = trans ? srht_dispatch<float, true>(h->ctx, W, (const float*)in->A, in->lda, L, K,
                                              (const float*)h->srht_Dv, h->srht_mu, h->blocks[b].col0,
                                              (float*)o, ldo, (float)scale, st)
                 : srht_dispatch<float, false>(h->ctx, W, (const float*)in->A, in->lda, L, K,
                                               (const float*)h->srht_Dv, h->srht_mu, h->blocks[b].col0,
                                               (float*)o, ldo, (float)scale, st);
    }
    if (rc) return rc;
    col += W;
    b = e;
  }
  return SK_OK;
}

}  // namespace sk

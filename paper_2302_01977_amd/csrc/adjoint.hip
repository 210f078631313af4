// Adjoint of the stored-A SJLT sketch: dA = dS R^T, the transpose of A -> A R.
// Column k of dA gathers the alpha columns of dS named by row k of R:
//     dA(:, k) = (1/sqrt(alpha)) sum_c sign(k, c) dS(:, col(k, c)).
// A workgroup owns 64 rows; their slab of dS (64 rows x the blocks' columns) is
// staged in LDS once, then each wave writes whole columns of dA (coalesced,
// write-bound), reading the hash of row k of R as uniform scalars.  Blocks wider
// than the LDS slab are handled in several passes that accumulate into dA.
#include <algorithm>

#include "internal.hpp"

namespace sk {

struct AdjBlocks {
  const uint32_t* codes[MAX_PASS_BLOCKS];
  int32_t coloff[MAX_PASS_BLOCKS];  // first column of the block inside dS
  int32_t nb;
};

template <typename T, int MAXW>
__global__ void __launch_bounds__(256)
    sjlt_adjoint_kernel(const T* __restrict__ dS, int64_t lddS, int64_t m, int64_t n, AdjBlocks ab, int alpha,
                        int c0, int wcnt, T* __restrict__ dA, int64_t lddA, T scale, int kper, int accumulate) {
  __shared__ __attribute__((aligned(16))) T St[MAXW * 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * 64;
  const int64_t row = l0 + lane;
  for (int e = tid; e < wcnt * 64; e += 256) {
    const int col = e >> 6, r = e & 63;
    St[e] = (l0 + r < m) ? dS[(l0 + r) + (int64_t)(c0 + col) * lddS] : T(0);
  }
  __syncthreads();
  const int64_t k0 = (int64_t)blockIdx.y * kper;
  const int64_t k1 = std::min<int64_t>(n, k0 + kper);
  for (int64_t k = k0 + wave; k < k1; k += 4) {
    T a = T(0);
    for (int b = 0; b < ab.nb; ++b) {
      for (int c = 0; c < alpha; ++c) {
        const uint32_t code = ab.codes[b][k * alpha + c];
        const int col = (int)(code >> 1) + ab.coloff[b] - c0;  // column inside the staged slab
        if (col >= 0 && col < wcnt) a += (code & 1u) ? -St[col * 64 + lane] : St[col * 64 + lane];
      }
    }
    if (row < m) {
      T* p = dA + row + k * lddA;
      *p = accumulate ? *p + a * scale : a * scale;
    }
  }
}

int launch_sjlt_adjoint(Handle* h, const sk_input* in, int b0, int b1, const void* dS, int64_t lddS, void* dA,
                        int64_t lddA, hipStream_t st) {
  SK_REQUIRE(h->kind == SK_SJLT, SK_EUNSUPPORTED, "the stored-A adjoint is implemented for the SJLT operator");
  const int nblk = b1 - b0;
  SK_REQUIRE(nblk >= 1 && nblk <= MAX_PASS_BLOCKS, SK_EINVAL, "the adjoint covers 1..%d blocks", MAX_PASS_BLOCKS);
  AdjBlocks ab;
  memset(&ab, 0, sizeof(ab));
  int Wt = 0;
  for (int b = b0; b < b1; ++b) {
    ab.codes[b - b0] = h->blocks[b].codes;
    ab.coloff[b - b0] = Wt;
    Wt += h->blocks[b].w;
  }
  ab.nb = nblk;
  const int64_t m = in->m, n = in->n;
  const int64_t rt = (m + 63) / 64;
  // spread the columns of dA so that the grid holds ~4 workgroups per CU
  const int64_t want = 4 * (int64_t)h->ctx->num_cu;
  const int64_t ksplit = std::max<int64_t>(1, std::min<int64_t>(n, (want + rt - 1) / rt));
  const int kper = (int)((n + ksplit - 1) / ksplit);
  const dim3 grid((unsigned)rt, (unsigned)((n + kper - 1) / kper));
  const double scale = 1.0 / sqrt((double)h->alpha);
  ProfScope ps(h->ctx, "sjlt_adjoint", st);
  constexpr int MAXW = 128;  // LDS slab: 64 rows x 128 columns (64 KB in FP64)
  for (int c0 = 0; c0 < Wt; c0 += MAXW) {
    const int wcnt = std::min(MAXW, Wt - c0);
    if (h->dtype == SK_F64)
      sjlt_adjoint_kernel<double, MAXW><<<grid, 256, 0, st>>>((const double*)dS, lddS, m, n, ab, h->alpha, c0, wcnt,
                                                              (double*)dA, lddA, scale, kper, c0 > 0);
    else
      sjlt_adjoint_kernel<float, MAXW><<<grid, 256, 0, st>>>((const float*)dS, lddS, m, n, ab, h->alpha, c0, wcnt,
                                                             (float*)dA, lddA, (float)scale, kper, c0 > 0);
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

}  // namespace sk

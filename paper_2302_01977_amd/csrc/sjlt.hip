// SJLT sketch of a stored, column-major A (section 6.3 computes A R by an outer
// product over the rows of R and A^* R by inner products with the columns of R).
//
// GPU formulation: a hashed gather.  A workgroup owns 64 "lanes" (rows of A for
// S = A R, columns of A for S' = A^T R) and walks the sources (columns of A for
// S, rows for S') in chunks of KC = 64.  Each chunk is staged once, coalesced,
// in LDS; every wave then owns NJ output columns and, for each of them, adds or
// subtracts the staged sources listed in that column's bucket for the chunk
// (wave-uniform indices, so every LDS read is a contiguous 64-lane access).
// Accumulators stay in VGPRs; no multiplies, the 1/sqrt(alpha) scale is applied
// once at the end, as in the paper.  When the lane tiles alone cannot fill the
// chip the source range is split and the partial sums are reduced in a fixed
// order (deterministic, no atomics).
#include "internal.hpp"

namespace sk {

template <typename T, bool TRANS, int NW, int NJ>
__global__ void __launch_bounds__(NW * 64)
    sjlt_gather_kernel(const T* __restrict__ A, int64_t lda, int64_t L, int64_t K, SjltPass pass,
                       T* __restrict__ out, int64_t ldo, T scale, int split, T* __restrict__ part) {
  constexpr int STRIDE = TRANS ? 65 : 64;
  constexpr int DUMMY = KC << 1;  // entry that reads the all-zero tile row KC
  __shared__ T tile[(KC + 1) * STRIDE];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t l0 = (int64_t)blockIdx.x * 64;
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
  if (threadIdx.x < STRIDE) tile[KC * STRIDE + threadIdx.x] = T(0);

  T acc[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) acc[jj] = T(0);

  for (int t = t0; t < t1; ++t) {
    const int64_t k0 = (int64_t)t * KC;
    if (!TRANS) {
      const int64_t row = l0 + lane;
      for (int kk = threadIdx.x >> 6; kk < KC; kk += NW) {
        const int64_t col = k0 + kk;
        tile[kk * STRIDE + lane] = (row < L && col < K) ? A[row + col * lda] : T(0);
      }
    } else {
      const int64_t row = k0 + lane;
      for (int l = threadIdx.x >> 6; l < 64; l += NW) {
        const int64_t col = l0 + l;
        tile[lane * STRIDE + l] = (row < K && col < L) ? A[row + col * lda] : T(0);
      }
    }
    __syncthreads();
    if (active) {
      const int32_t* __restrict__ P = ptr + (int64_t)t * prow;
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) {
        const int p1 = P[jj + 1];
        T a0 = T(0), a1 = T(0);
        for (int e = P[jj]; e < p1; e += 4) {
          // four entries per step, reads in flight together; past the end of
          // the bucket the dummy entry adds the zero row
          int v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = (e + u < p1) ? ent[e + u] : DUMMY;
          T x[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) x[u] = tile[(v[u] >> 1) * STRIDE + lane];
#pragma unroll
          for (int u = 0; u < 4; u += 2) {
            a0 = fma(x[u], (v[u] & 1) ? T(-1) : T(1), a0);
            a1 = fma(x[u + 1], (v[u + 1] & 1) ? T(-1) : T(1), a1);
          }
        }
        acc[jj] += a0 + a1;
      }
    }
    __syncthreads();
  }

  if (!active) return;
  const int64_t row = l0 + lane;
  if (row >= L) return;
  const int64_t jc = (int64_t)g * NJ;
  if (split == 1) {
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) out[row + (jc + jj) * ldo] = acc[jj] * scale;
  } else {
    T* p = part + (int64_t)s * L * ((int64_t)pass.ngroups * NJ);
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) p[row + (jc + jj) * L] = acc[jj];
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

static thread_local Ctx* prof_ctx = nullptr;

template <typename T, bool TRANS, int NW, int NJ>
static int run_gather(const T* A, int64_t lda, int64_t L, int64_t K, const SjltPass& pass, T* out, int64_t ldo,
                      T scale, int split, T* part, int gz, hipStream_t st) {
  dim3 grid((unsigned)((L + 63) / 64), (unsigned)split, (unsigned)gz);
  ProfScope ps(prof_ctx, TRANS ? "sjlt_gather_t" : "sjlt_gather", st);
  sjlt_gather_kernel<T, TRANS, NW, NJ><<<grid, NW * 64, 0, st>>>(A, lda, L, K, pass, out, ldo, scale, split, part);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename T, bool TRANS>
static int dispatch(int nw, int nj, const T* A, int64_t lda, int64_t L, int64_t K, const SjltPass& pass, T* out,
                    int64_t ldo, T scale, int split, T* part, int gz, hipStream_t st) {
  if (nw == 4 && nj == 16) return run_gather<T, TRANS, 4, 16>(A, lda, L, K, pass, out, ldo, scale, split, part, gz, st);
  if (nw == 4 && nj == 32) return run_gather<T, TRANS, 4, 32>(A, lda, L, K, pass, out, ldo, scale, split, part, gz, st);
  if (nw == 4 && nj == 64) return run_gather<T, TRANS, 4, 64>(A, lda, L, K, pass, out, ldo, scale, split, part, gz, st);
  if (nw == 8 && nj == 16) return run_gather<T, TRANS, 8, 16>(A, lda, L, K, pass, out, ldo, scale, split, part, gz, st);
  if (nw == 8 && nj == 32) return run_gather<T, TRANS, 8, 32>(A, lda, L, K, pass, out, ldo, scale, split, part, gz, st);
  if (nw == 8 && nj == 64) return run_gather<T, TRANS, 8, 64>(A, lda, L, K, pass, out, ldo, scale, split, part, gz, st);
  set_error("internal: no SJLT kernel for NW=%d NJ=%d", nw, nj);
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

int launch_sjlt_pass(Handle* h, const sk_input* in, int b0, int b1, bool trans, void* out, int64_t ldo,
                     hipStream_t st) {
  const int nblk = b1 - b0;
  SK_REQUIRE(nblk >= 1 && nblk <= MAX_PASS_BLOCKS, SK_EINVAL, "a pass covers 1..%d blocks", MAX_PASS_BLOCKS);
  int W = 0, g = 0;
  for (int b = b0; b < b1; ++b) {
    W += h->blocks[b].w;
    g = gcd_int(g, h->blocks[b].w);
  }
  // columns per wave: the largest of 64/32/16 dividing every width, at most W/4
  int nj = 16;
  const int nj_max = h->dtype == SK_F64 ? 32 : 64;  // FP64 x 64 columns spills
  for (int c : {64, 32}) {
    if (c > nj_max) continue;
    if (g % c == 0 && c <= (W >= 64 ? W / 4 : 16)) {
      nj = c;
      break;
    }
  }
  SK_REQUIRE(g % nj == 0, SK_EINVAL, "SJLT block widths must be multiples of 16");
  const int ngroups = W / nj;
  SK_REQUIRE(ngroups <= MAX_PASS_GROUPS, SK_EINVAL, "pass too wide (%d columns)", W);
  const int nw = ngroups <= 4 ? 4 : 8;
  const int gz = (ngroups + nw - 1) / nw;

  SjltPass pass;
  memset(&pass, 0, sizeof(pass));
  pass.nT = (int)((h->n + KC - 1) / KC);
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

  const int64_t L = trans ? in->n : in->m;  // lanes
  const int64_t K = trans ? in->m : in->n;  // sources (= rows of R)
  const int64_t tiles = ((L + 63) / 64) * gz;
  int split = 1;
  const int64_t target = 2 * (int64_t)h->ctx->num_cu;
  if (tiles < target) split = (int)std::min<int64_t>((target + tiles - 1) / tiles, std::max(1, pass.nT / 4));
  const size_t esz = h->dtype == SK_F64 ? 8 : 4;
  void* part = nullptr;
  if (split > 1) {
    const int rc = ensure_work(h->ctx, (size_t)split * (size_t)L * (size_t)W * esz);
    if (rc) return rc;
    part = h->ctx->work;
  }
  const double scale = 1.0 / sqrt((double)h->alpha);
  prof_ctx = h->ctx;
  int rc;
  if (h->dtype == SK_F64) {
    const double* A = (const double*)in->A;
    rc = trans ? dispatch<double, true>(nw, nj, A, in->lda, L, K, pass, (double*)out, ldo, scale, split, (double*)part, gz, st)
               : dispatch<double, false>(nw, nj, A, in->lda, L, K, pass, (double*)out, ldo, scale, split, (double*)part, gz, st);
  } else {
    const float* A = (const float*)in->A;
    rc = trans ? dispatch<float, true>(nw, nj, A, in->lda, L, K, pass, (float*)out, ldo, (float)scale, split, (float*)part, gz, st)
               : dispatch<float, false>(nw, nj, A, in->lda, L, K, pass, (float*)out, ldo, (float)scale, split, (float*)part, gz, st);
  }
  if (rc) return rc;
  if (split > 1) {
    const int64_t tot = L * (int64_t)W;
    const unsigned nb = (unsigned)((tot + 255) / 256);
    ProfScope ps(h->ctx, "sjlt_reduce", st);
    if (h->dtype == SK_F64)
      split_reduce_kernel<double><<<nb, 256, 0, st>>>((const double*)part, split, L, W, (double*)out, ldo, scale);
    else
      split_reduce_kernel<float><<<nb, 256, 0, st>>>((const float*)part, split, L, W, (float*)out, ldo, (float)scale);
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

}  // namespace sk

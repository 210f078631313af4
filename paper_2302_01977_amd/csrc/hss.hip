// Batched FP64 kernels for the per-node work of adaptive HSS compression
// (Algorithm 1 and the appendix "HSS Algorithm Detailed Description"): the
// small dense products of the local sketches and local operators, the
// Householder QR of the stopping test (section 3, eq. "stopping_criteria-1"),
// the column-pivoted QR of the interpolative decomposition, Frobenius norms,
// row / column selections, and the rows of R on the device.
//
// Every kernel takes its descriptors by value in the kernel arguments (one per
// node of a tree level; a call with more runs several launches), so a batched
// call copies nothing and never waits for the device; it runs one workgroup
// (or a grid of tiles) per descriptor, and sizes are per descriptor, so the
// nodes of a level need not match.
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace sk {

// descriptors of one launch, passed by value (kernel arguments stay under 4 KB)
template <typename D, int CAP>
struct DescPack {
  D d[CAP];
};
constexpr int CAP_GEMM = 40, CAP_QR = 64, CAP_ID = 48, CAP_NORM = 96, CAP_GATHER = 40;
static_assert(sizeof(DescPack<sk_gemm_desc, CAP_GEMM>) <= 3584 && sizeof(DescPack<sk_qr_desc, CAP_QR>) <= 3584 &&
                  sizeof(DescPack<sk_id_desc, CAP_ID>) <= 3584 && sizeof(DescPack<sk_norm_desc, CAP_NORM>) <= 3584 &&
                  sizeof(DescPack<sk_gather_desc, CAP_GATHER>) <= 3584,
              "descriptor packs fit the kernel arguments");

// QR, ID and norms: one workgroup of NT threads (NWV waves) per node
constexpr int NT = 1024, NWV = NT / 64;

// ------------------------------------------------------------------ products
// C = beta C + alpha op(A) op(B): 64 x 64 output tiles, 256 threads, each
// thread 4 x 4 outputs; k in steps of 16 staged in LDS.
constexpr int GT = 64, GK = 16;

__global__ void __launch_bounds__(256) bgemm_kernel(const DescPack<sk_gemm_desc, CAP_GEMM> pk) {
  const sk_gemm_desc g = pk.d[blockIdx.z];
  const int tm = (g.m + GT - 1) / GT, tn = (g.n + GT - 1) / GT;
  if ((int)blockIdx.x >= tm * tn) return;
  const int i0 = ((int)blockIdx.x % tm) * GT, j0 = ((int)blockIdx.x / tm) * GT;
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x;
  const int ti = (tid % 16) * 4, tj = (tid / 16) * 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k0 = 0; k0 < g.k; k0 += GK) {
    // stage A(i0 : i0 + 64, k0 : k0 + 16) and B(k0 : k0 + 16, j0 : j0 + 64)
    for (int e = tid; e < GK * GT; e += 256) {
      const int kk = e / GT, ii = e % GT;
      const int i = i0 + ii, k = k0 + kk;
      double v = 0.0;
      if (i < g.m && k < g.k) v = g.transA ? g.A[k + (int64_t)i * g.lda] : g.A[i + (int64_t)k * g.lda];
      As[kk][ii] = v;
      const int j = j0 + ii;
      double w = 0.0;
      if (j < g.n && k < g.k) w = g.transB ? g.B[j + (int64_t)k * g.ldb] : g.B[k + (int64_t)j * g.ldb];
      Bs[kk][ii] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ti + q];
        b[q] = Bs[kk][tj + q];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = i0 + ti + x, j = j0 + tj + y;
      if (i < g.m && j < g.n) {
        double* c = g.C + i + (int64_t)j * g.ldc;
        *c = (g.beta == 0.0 ? 0.0 : g.beta * *c) + g.alpha * acc[x][y];
      }
    }
}

// ------------------------------------------------------------------ helpers
// sum over the workgroup (NT threads) in a fixed order; every thread gets it
__device__ __forceinline__ double wg_sum(double v, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();  // red is free
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < NWV; ++u) t += red[u];
  return t;
}

// Householder reflector of x = M(k:m, col): on exit M(k, col) holds beta
// (= -sign(x0) ||x||), M(k+1:m, col) the vector v scaled so that v0 = 1
// (implicit), and tau = (beta - x0) / beta; tau = 0 when x is zero below k
// (no reflection).  Returns tau.
__device__ double house(double* __restrict__ M, int64_t ld, int m, int k, int col, double* red) {
  const int tid = threadIdx.x;
  double* x = M + (int64_t)col * ld;
  double s = 0.0;
  for (int i = k + 1 + tid; i < m; i += NT) s = fma(x[i], x[i], s);
  const double sigma = wg_sum(s, red);
  const double x0 = x[k];
  double tau = 0.0, beta = x0, scale = 0.0;
  if (sigma > 0.0) {
    const double nrm = sqrt(x0 * x0 + sigma);
    beta = x0 > 0.0 ? -nrm : nrm;
    tau = (beta - x0) / beta;
    scale = 1.0 / (x0 - beta);
  }
  __syncthreads();  // every thread has read x0
  if (sigma > 0.0)
    for (int i = k + 1 + tid; i < m; i += NT) x[i] *= scale;
  if (tid == 0) x[k] = beta;
  __syncthreads();
  return tau;
}

// apply H = I - tau v v^T (v from column vc, v0 = 1) to columns [c0, c1) of M
__device__ void apply_house(double* __restrict__ M, int64_t ld, int m, int k, int vc, double tau, int c0, int c1,
                            double* red) {
  if (tau == 0.0) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double* v = M + (int64_t)vc * ld;
  // one wave per column: dot, then update
  for (int j = c0 + w; j < c1; j += NWV) {
    double* y = M + (int64_t)j * ld;
    double s = 0.0;
    for (int i = k + lane; i < m; i += 64) s = fma(i == k ? 1.0 : v[i], y[i], s);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    const double f = tau * s;
    for (int i = k + lane; i < m; i += 64) y[i] -= f * (i == k ? 1.0 : v[i]);
  }
  __syncthreads();
  (void)red;
}

// ---------------------------------------------------------------------- QR
// In place: A (m x n) -> R in the upper triangle, reflectors below.  Writes
// the explicit Q (m x r, r = min(m, n)) and |R_jj| (r values).
__global__ void __launch_bounds__(NT) bqr_kernel(const DescPack<sk_qr_desc, CAP_QR> pk) {
  const sk_qr_desc g = pk.d[blockIdx.x];
  __shared__ double red[NWV];
  __shared__ double taus[1024];
  const int m = g.m, n = g.n, r = min(m, n);
  const int tid = threadIdx.x;
  for (int k = 0; k < r; ++k) {
    const double tau = house(g.A, g.lda, m, k, k, red);
    if (tid == 0) taus[k] = tau;
    apply_house(g.A, g.lda, m, k, k, tau, k + 1, n, red);
  }
  __syncthreads();
  for (int k = tid; k < r; k += NT) g.rdiag[k] = fabs(g.A[k + (int64_t)k * g.lda]);
  if (!g.Q) return;
  // Q = H_0 ... H_{r-1} [I; 0], accumulated backwards
  for (int e = tid; e < m * r; e += NT) {
    const int i = e % m, j = e / m;
    g.Q[i + (int64_t)j * g.ldq] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = r - 1; k >= 0; --k) {
    const double tau = taus[k];
    if (tau == 0.0) continue;
    const double* v = g.A + (int64_t)k * g.lda;
    const int lane = tid & 63, w = tid >> 6;
    for (int j = k + w; j < r; j += NWV) {
      double* y = g.Q + (int64_t)j * g.ldq;
      double s = 0.0;
      for (int i = k + lane; i < m; i += 64) s = fma(i == k ? 1.0 : v[i], y[i], s);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
      const double f = tau * s;
      for (int i = k + lane; i < m; i += 64) y[i] -= f * (i == k ? 1.0 : v[i]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------- ID
// Column-pivoted Householder QR of M (p x q, in place) with the column norms
// recomputed exactly at every step; the pivot is the first column of maximal
// norm; stop at the first k with norm < max(eps_a, eps_r * |R_00|).  Writes the
// rank k, the permutation (perm[0:k] the selected columns) and
// Y = [I, R11^{-1} R12] P^T (k x q, column j of Y for column j of M).
__global__ void __launch_bounds__(NT) bid_kernel(const DescPack<sk_id_desc, CAP_ID> pk) {
  const sk_id_desc g = pk.d[blockIdx.x];
  __shared__ double red[NWV];
  __shared__ double bestv[NWV];
  __shared__ int besti[NWV];
  __shared__ int s_piv;
  __shared__ double s_nk;
  const int p = g.p, q = g.q, r = min(p, q);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* M = g.M;
  for (int j = tid; j < q; j += NT) g.perm[j] = j;
  __syncthreads();
  int rank = 0;
  double r00 = -1.0;
  for (int k = 0; k < r; ++k) {
    // exact norms of the trailing columns, one wave per column; best = first max
    double bv = -1.0;
    int bi = q;
    for (int j = k + w; j < q; j += NWV) {
      const double* y = M + (int64_t)j * g.ldm;
      double s = 0.0;
      for (int i = k + lane; i < p; i += 64) s = fma(y[i], y[i], s);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
      const double nr = sqrt(s);
      if (nr > bv) {  // j increases: keeps the first maximum of this wave
        bv = nr;
        bi = j;
      }
    }
    if (lane == 0) {
      bestv[w] = bv;
      besti[w] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = -1.0;
      int bj = q;
      for (int u = 0; u < NWV; ++u)
        if (bestv[u] > b || (bestv[u] == b && besti[u] < bj)) {
          b = bestv[u];
          bj = besti[u];
        }
      s_piv = bj;
      s_nk = b;
    }
    __syncthreads();
    const double nk = s_nk;
    const int piv = s_piv;
    if (r00 < 0.0) r00 = nk;
    if (nk == 0.0 || nk < fmax(g.eps_a, g.eps_r * r00)) break;
    if (piv != k) {  // swap columns k and piv
      double* a = M + (int64_t)k * g.ldm;
      double* b = M + (int64_t)piv * g.ldm;
      for (int i = tid; i < p; i += NT) {
        const double t = a[i];
        a[i] = b[i];
        b[i] = t;
      }
      if (tid == 0) {
        const int t = g.perm[k];
        g.perm[k] = g.perm[piv];
        g.perm[piv] = t;
      }
      __syncthreads();
    }
    const double tau = house(M, g.ldm, p, k, k, red);
    apply_house(M, g.ldm, p, k, k, tau, k + 1, q, red);
    rank = k + 1;
  }
  if (tid == 0) *g.rank = rank;
  // Y (k x q): identity on the selected columns, X = R11^{-1} R12 on the rest,
  // by back substitution, one thread per column of R12
  for (int e = tid; e < rank * q; e += NT) g.Y[(e % rank) + (int64_t)(e / rank) * g.ldy] = 0.0;
  __syncthreads();
  for (int j = tid; j < rank; j += NT) g.Y[j + (int64_t)g.perm[j] * g.ldy] = 1.0;
  for (int c = rank + tid; c < q; c += NT) {
    double* y = g.Y + (int64_t)g.perm[c] * g.ldy;
    const double* rc = M + (int64_t)c * g.ldm;
    for (int i = rank - 1; i >= 0; --i) {
      double s = rc[i];
      for (int l = i + 1; l < rank; ++l) s -= M[i + (int64_t)l * g.ldm] * y[l];
      y[i] = s / M[i + (int64_t)i * g.ldm];
    }
  }
}

// ----------------------------------------------------------- norms, gathers
__global__ void __launch_bounds__(NT) bnorm_kernel(const DescPack<sk_norm_desc, CAP_NORM> pk) {
  const sk_norm_desc g = pk.d[blockIdx.x];
  __shared__ double red[NWV];
  double s = 0.0;
  const int64_t tot = (int64_t)g.m * g.n;
  for (int64_t e = threadIdx.x; e < tot; e += NT) {
    const double v = g.A[(e % g.m) + (e / g.m) * g.lda];
    s = fma(v, v, s);
  }
  s = wg_sum(s, red);
  if (threadIdx.x == 0) *g.out = sqrt(s);
}

// dst(i, j) = src(rows[i], cols[j]) (rows / cols NULL: row0 + i / col0 + j)
__global__ void __launch_bounds__(256) bgather_kernel(const DescPack<sk_gather_desc, CAP_GATHER> pk) {
  const sk_gather_desc g = pk.d[blockIdx.y];
  const int64_t tot = (int64_t)g.m * g.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % g.m), j = (int)(e / g.m);
    const int64_t si = g.rows ? g.rows[i] : g.row0 + i;
    const int64_t sj = g.cols ? g.cols[j] : g.col0 + j;
    g.dst[i + (int64_t)j * g.ldd] = g.trans ? g.src[sj + si * g.lds] : g.src[si + sj * g.lds];
  }
}

// R(i0:i1, j0:j1) from the handle's device metadata (FP64, column-major)
struct RRowsArgs {
  int kind, alpha, construction;
  int64_t n, i0, i1, j0, j1;
  int nb;
  int32_t w[64];
  int64_t col0[64];
  const uint32_t* codes[64];
  const uint16_t* gbf[64];
  const int8_t* D;
  const uint32_t* mu;
  double* out;
  int64_t ldo;
};

__global__ void __launch_bounds__(256) rrows_kernel(RRowsArgs a, int bsel) {
  const int64_t rows = a.i1 - a.i0;
  const int b = bsel;
  const int64_t c0 = a.col0[b], w = a.w[b];
  const int64_t jlo = std::max<int64_t>(a.j0, c0), jhi = std::min<int64_t>(a.j1, c0 + w);
  const int64_t tot = rows * (jhi > jlo ? jhi - jlo : 0);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t ii = e % rows, j = jlo + e / rows;
    const int64_t i = a.i0 + ii;
    const int jj = (int)(j - c0);
    double v = 0.0;
    if (a.kind == SK_SJLT) {
      const double s = 1.0 / sqrt((double)a.alpha);
      const uint32_t* cd = a.codes[b] + i * a.alpha;
      if (a.construction == SK_SJLT_GRAPH) {
        for (int c = 0; c < a.alpha; ++c)
          if ((int)(cd[c] >> 1) == jj) v = (cd[c] & 1u) ? -s : s;
      } else {
        const int c = jj / (int)(w / a.alpha);
        if ((int)(cd[c] >> 1) == jj) v = (cd[c] & 1u) ? -s : s;
      }
    } else if (a.kind == SK_GAUSSIAN) {
      const uint32_t bits = (uint32_t)a.gbf[b][i + (int64_t)jj * a.n] << 16;
      v = (double)__builtin_bit_cast(float, bits) / sqrt((double)w);
    } else {
      const int neg = (a.D[i] < 0) ^ (__popc((uint32_t)i & a.mu[j]) & 1);
      v = (neg ? -1.0 : 1.0) / sqrt((double)w);
    }
    a.out[ii + (j - a.j0) * a.ldo] = v;
  }
}

// copy descriptors [b0, b0 + n) of a call into a launch's pack
template <typename D, int CAP>
static DescPack<D, CAP> pack(const D* descs, int b0, int n) {
  DescPack<D, CAP> pk;
  memset(&pk, 0, sizeof(pk));
  memcpy(pk.d, descs + b0, sizeof(D) * (size_t)n);
  return pk;
}

}  // namespace sk

using namespace sk;

static int check_live(const sk_ctx* c) {
  SK_REQUIRE(c && c->c.magic == CTX_MAGIC, SK_ESTATE, "not a live sketch context");
  return SK_OK;
}

extern "C" {

int sketch_batched_gemm(sk_ctx* ctx, const sk_gemm_desc* descs, int32_t count, void* stream) {
  if (int rc = check_live(ctx)) return rc;
  SK_REQUIRE(count >= 0 && (count == 0 || descs), SK_EINVAL, "bad descriptor array");
  if (count == 0) return SK_OK;
  for (int b = 0; b < count; ++b) {
    const sk_gemm_desc& g = descs[b];
    SK_REQUIRE(g.m >= 0 && g.n >= 0 && g.k >= 0, SK_EINVAL, "gemm %d: negative size", b);
    SK_REQUIRE(g.m == 0 || g.n == 0 || g.C, SK_EINVAL, "gemm %d: C is NULL", b);
    SK_REQUIRE(g.k == 0 || g.m == 0 || g.n == 0 || (g.A && g.B), SK_EINVAL, "gemm %d: A or B is NULL", b);
    SK_REQUIRE(g.ldc >= std::max(1, g.m), SK_EINVAL, "gemm %d: ldc < m", b);
    SK_REQUIRE(g.lda >= std::max(1, g.transA ? g.k : g.m), SK_EINVAL, "gemm %d: lda too small", b);
    SK_REQUIRE(g.ldb >= std::max(1, g.transB ? g.n : g.k), SK_EINVAL, "gemm %d: ldb too small", b);
  }
  SK_HIP(hipSetDevice(ctx->c.device));
  hipStream_t st = (hipStream_t)stream;
  ProfScope ps(&ctx->c, "hss_gemm", st);
  for (int b0 = 0; b0 < count; b0 += CAP_GEMM) {
    const int n = std::min(CAP_GEMM, count - b0);
    int tl = 1;
    for (int b = b0; b < b0 + n; ++b)
      tl = std::max(tl, ((descs[b].m + GT - 1) / GT) * ((descs[b].n + GT - 1) / GT));
    bgemm_kernel<<<dim3((unsigned)tl, 1, (unsigned)n), 256, 0, st>>>(pack<sk_gemm_desc, CAP_GEMM>(descs, b0, n));
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

int sketch_batched_qr(sk_ctx* ctx, const sk_qr_desc* descs, int32_t count, void* stream) {
  if (int rc = check_live(ctx)) return rc;
  SK_REQUIRE(count >= 0 && (count == 0 || descs), SK_EINVAL, "bad descriptor array");
  if (count == 0) return SK_OK;
  for (int b = 0; b < count; ++b) {
    const sk_qr_desc& g = descs[b];
    SK_REQUIRE(g.m >= 1 && g.n >= 1 && g.A && g.rdiag, SK_EINVAL, "qr %d: empty matrix or NULL pointer", b);
    SK_REQUIRE(std::min(g.m, g.n) <= 1024, SK_EINVAL, "qr %d: min(m, n) above 1024", b);
    SK_REQUIRE(g.lda >= g.m && (!g.Q || g.ldq >= g.m), SK_EINVAL, "qr %d: leading dimension too small", b);
  }
  SK_HIP(hipSetDevice(ctx->c.device));
  hipStream_t st = (hipStream_t)stream;
  ProfScope ps(&ctx->c, "hss_qr", st);
  for (int b0 = 0; b0 < count; b0 += CAP_QR) {
    const int n = std::min(CAP_QR, count - b0);
    bqr_kernel<<<(unsigned)n, NT, 0, st>>>(pack<sk_qr_desc, CAP_QR>(descs, b0, n));
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

int sketch_batched_id(sk_ctx* ctx, const sk_id_desc* descs, int32_t count, void* stream) {
  if (int rc = check_live(ctx)) return rc;
  SK_REQUIRE(count >= 0 && (count == 0 || descs), SK_EINVAL, "bad descriptor array");
  if (count == 0) return SK_OK;
  for (int b = 0; b < count; ++b) {
    const sk_id_desc& g = descs[b];
    SK_REQUIRE(g.p >= 1 && g.q >= 1 && g.M && g.perm && g.rank && g.Y, SK_EINVAL,
               "id %d: empty matrix or NULL pointer", b);
    SK_REQUIRE(g.ldm >= g.p && g.ldy >= std::min(g.p, g.q), SK_EINVAL, "id %d: leading dimension too small", b);
  }
  SK_HIP(hipSetDevice(ctx->c.device));
  hipStream_t st = (hipStream_t)stream;
  ProfScope ps(&ctx->c, "hss_id", st);
  for (int b0 = 0; b0 < count; b0 += CAP_ID) {
    const int n = std::min(CAP_ID, count - b0);
    bid_kernel<<<(unsigned)n, NT, 0, st>>>(pack<sk_id_desc, CAP_ID>(descs, b0, n));
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

int sketch_batched_norm(sk_ctx* ctx, const sk_norm_desc* descs, int32_t count, void* stream) {
  if (int rc = check_live(ctx)) return rc;
  SK_REQUIRE(count >= 0 && (count == 0 || descs), SK_EINVAL, "bad descriptor array");
  if (count == 0) return SK_OK;
  for (int b = 0; b < count; ++b) {
    const sk_norm_desc& g = descs[b];
    SK_REQUIRE(g.m >= 0 && g.n >= 0 && g.out && (g.m * (int64_t)g.n == 0 || g.A), SK_EINVAL, "norm %d: bad", b);
    SK_REQUIRE(g.lda >= std::max(1, g.m), SK_EINVAL, "norm %d: lda < m", b);
  }
  SK_HIP(hipSetDevice(ctx->c.device));
  hipStream_t st = (hipStream_t)stream;
  ProfScope ps(&ctx->c, "hss_norm", st);
  for (int b0 = 0; b0 < count; b0 += CAP_NORM) {
    const int n = std::min(CAP_NORM, count - b0);
    bnorm_kernel<<<(unsigned)n, NT, 0, st>>>(pack<sk_norm_desc, CAP_NORM>(descs, b0, n));
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

int sketch_batched_gather(sk_ctx* ctx, const sk_gather_desc* descs, int32_t count, void* stream) {
  if (int rc = check_live(ctx)) return rc;
  SK_REQUIRE(count >= 0 && (count == 0 || descs), SK_EINVAL, "bad descriptor array");
  if (count == 0) return SK_OK;
  for (int b = 0; b < count; ++b) {
    const sk_gather_desc& g = descs[b];
    SK_REQUIRE(g.m >= 0 && g.n >= 0, SK_EINVAL, "gather %d: negative size", b);
    SK_REQUIRE((int64_t)g.m * g.n == 0 || (g.src && g.dst), SK_EINVAL, "gather %d: NULL pointer", b);
    SK_REQUIRE(g.ldd >= std::max(1, g.m), SK_EINVAL, "gather %d: ldd < m", b);
  }
  SK_HIP(hipSetDevice(ctx->c.device));
  hipStream_t st = (hipStream_t)stream;
  ProfScope ps(&ctx->c, "hss_gather", st);
  for (int b0 = 0; b0 < count; b0 += CAP_GATHER) {
    const int n = std::min(CAP_GATHER, count - b0);
    int64_t mx = 1;
    for (int b = b0; b < b0 + n; ++b) mx = std::max<int64_t>(mx, (int64_t)descs[b].m * descs[b].n);
    const unsigned gx = (unsigned)std::min<int64_t>((mx + 255) / 256, 1024);
    bgather_kernel<<<dim3(gx, (unsigned)n), 256, 0, st>>>(pack<sk_gather_desc, CAP_GATHER>(descs, b0, n));
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

int sketch_get_rows_device(const sk_handle* H, int64_t i0, int64_t i1, int64_t j0, int64_t j1, double* out,
                           int64_t ldo, void* stream) {
  SK_REQUIRE(H && H->h.magic == HND_MAGIC, SK_ESTATE, "not a live sketch handle");
  const Handle* h = &H->h;
  SK_REQUIRE(0 <= i0 && i0 <= i1 && i1 <= h->n, SK_EINVAL, "row range out of bounds");
  SK_REQUIRE(0 <= j0 && j0 <= j1 && j1 <= h->d, SK_EINVAL, "column range out of bounds");
  SK_REQUIRE(out || i1 == i0 || j1 == j0, SK_EINVAL, "out is NULL");
  SK_REQUIRE(ldo >= std::max<int64_t>(1, i1 - i0), SK_EINVAL, "ldo too small");
  if (i1 == i0 || j1 == j0) return SK_OK;
  SK_HIP(hipSetDevice(h->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  RRowsArgs a;
  memset(&a, 0, sizeof(a));
  a.kind = h->kind;
  a.alpha = h->alpha;
  a.construction = h->construction;
  a.n = h->n;
  a.i0 = i0;
  a.i1 = i1;
  a.j0 = j0;
  a.j1 = j1;
  a.D = h->srht_D;
  a.mu = h->srht_mu;
  a.out = out;
  a.ldo = ldo;
  ProfScope ps(h->ctx, "hss_rrows", st);
  for (size_t b0 = 0; b0 < h->blocks.size(); b0 += 64) {
    a.nb = (int)std::min<size_t>(64, h->blocks.size() - b0);
    for (int q = 0; q < a.nb; ++q) {
      const Block& B = h->blocks[b0 + q];
      a.w[q] = B.w;
      a.col0[q] = B.col0;
      a.codes[q] = B.codes;
      a.gbf[q] = B.gbf;
    }
    for (int q = 0; q < a.nb; ++q) {
      if (a.col0[q] >= j1 || a.col0[q] + a.w[q] <= j0) continue;
      const int64_t cols = std::min<int64_t>(j1, a.col0[q] + a.w[q]) - std::max<int64_t>(j0, a.col0[q]);
      const unsigned gx = (unsigned)std::min<int64_t>(((i1 - i0) * cols + 255) / 256, 4096);
      rrows_kernel<<<gx, 256, 0, st>>>(a, q);
      SK_HIP(hipGetLastError());
    }
  }
  return SK_OK;
}

}  // extern "C"

// Operator block generation on the device (random matrix construction; the paper
// notes its cost is negligible next to the sketch, section 8 serial results).
//
// SJLT: the hash of every (row, chunk) and, per block, bucket tables that list
// for each output column and each chunk of KC consecutive sources the sources
// that feed it, in ascending order (a counting sort, deterministic).
// SRHT: the Rademacher diagonal D and the sampled Hadamard columns mu.
// Gaussian: the bf16-grid draws of the block, column-major.
#include "internal.hpp"

namespace sk {

__device__ __forceinline__ void hash_row(uint32_t* __restrict__ codes, int64_t k, int alpha, uint32_t wc,
                                         uint32_t block, Key key) {
  const uint32_t sbits = philox(2u, block, (uint32_t)k, 0u, key.k0, key.k1).v[0];
  for (int c4 = 0; c4 < alpha; c4 += 4) {
    const U4 o = philox(1u, block, (uint32_t)k, (uint32_t)(c4 >> 2), key.k0, key.k1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = c4 + q;
      if (c < alpha) {
        const uint32_t off = mulhi(o.v[q], wc);
        codes[k * alpha + c] = (((uint32_t)c * wc + off) << 1) | ((sbits >> c) & 1u);
      }
    }
  }
}

__global__ void __launch_bounds__(256) sjlt_hash_kernel(uint32_t* __restrict__ codes, int64_t n, int alpha,
                                                        uint32_t wc, uint32_t block, Key key) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) hash_row(codes, k, alpha, wc, block, key);
}

// Bucket table, chunk-major: ptr[t * (w + 1) + j] = first entry of column j in
// chunk t; slot w holds the end of the chunk's entries.  Chunk t owns the entry
// slots [t * kcap, (t + 1) * kcap); its unused slots hold null entries (source
// KC, sign +, a staged slot of zeros).  count_chunk stores the counts,
// scan_chunk turns them into starts.
__device__ __forceinline__ void count_chunk(const uint32_t* __restrict__ codes, int32_t* __restrict__ ptr,
                                            int64_t n, int alpha, int w, int kc, int t, int* cnt) {
  for (int j = threadIdx.x; j < w; j += blockDim.x) cnt[j] = 0;
  __syncthreads();
  const int64_t k0 = (int64_t)t * kc;
  const int nk = (int)min((int64_t)kc, n - k0);
  for (int e = threadIdx.x; e < nk * alpha; e += blockDim.x) atomicAdd(&cnt[codes[k0 * alpha + e] >> 1], 1);
  __syncthreads();
  for (int j = threadIdx.x; j <= w; j += blockDim.x)
    ptr[(int64_t)t * (w + 1) + j] = j < w ? cnt[j] : 0;
}

__global__ void __launch_bounds__(256) sjlt_count_kernel(const uint32_t* __restrict__ codes,
                                                         int32_t* __restrict__ ptr, int64_t n, int alpha,
                                                         int w, int kc) {
  __shared__ int cnt[1024];
  count_chunk(codes, ptr, n, alpha, w, kc, blockIdx.x, cnt);
}

// Exclusive scan of chunk t's w + 1 counts, offset by the chunk's region
// start (thread 0 walks the row in order).
__device__ __forceinline__ void scan_chunk(int32_t* __restrict__ ptr, int w, int kcap, int t) {
  if (threadIdx.x != 0) return;
  int32_t* row = ptr + (int64_t)t * (w + 1);
  int32_t run = (int32_t)t * kcap;
  for (int j = 0; j <= w; ++j) {
    const int32_t c = row[j];
    row[j] = run;
    run += c;
  }
}

__global__ void __launch_bounds__(64) chunk_scan_kernel(int32_t* __restrict__ ptr, int w, int kcap) {
  scan_chunk(ptr, w, kcap, blockIdx.x);
}

// One thread per source of chunk t; a source's rank inside its bucket counts the
// earlier sources of the chunk in the same bucket, so every bucket lists its
// sources in ascending order.
__device__ __forceinline__ void scatter_chunk(const uint32_t* __restrict__ codes, const int32_t* __restrict__ ptr,
                                              int32_t* __restrict__ ent, int64_t n, int alpha, int w, int kc,
                                              int kcap, int t, uint32_t* sc) {
  const int kk = threadIdx.x;
  const int64_t k0 = (int64_t)t * kc;
  const int nk = (int)min((int64_t)kc, n - k0);
  for (int e = threadIdx.x; e < nk * alpha; e += blockDim.x) sc[e] = codes[k0 * alpha + e];
  for (int e = threadIdx.x; e < kcap; e += blockDim.x) ent[(int64_t)t * kcap + e] = kc << 1;  // null entries
  __syncthreads();
  if (kk >= nk) return;
  for (int c = 0; c < alpha; ++c) {
    const uint32_t code = sc[kk * alpha + c];
    const uint32_t col = code >> 1;
    int rank = 0;
    for (int q = 0; q < kk; ++q) rank += (sc[q * alpha + c] >> 1) == col;
    ent[ptr[(int64_t)t * (w + 1) + col] + rank] = (kk << 1) | (int)(code & 1u);
  }
}

__global__ void __launch_bounds__(KC_MAX) sjlt_scatter_kernel(const uint32_t* __restrict__ codes,
                                                              const int32_t* __restrict__ ptr,
                                                              int32_t* __restrict__ ent, int64_t n, int alpha,
                                                              int w, int kc, int kcap) {
  __shared__ uint32_t sc[KC_MAX * 32];
  scatter_chunk(codes, ptr, ent, n, alpha, w, kc, kcap, blockIdx.x, sc);
}

// ---- batched: one launch per step over the blocks of many operators; list[i]
// = (item, row block of 256 sources) for hashing, (item, chunk) otherwise
__global__ void __launch_bounds__(256) sjlt_hash_batch(const MetaItem* __restrict__ items,
                                                       const int2* __restrict__ list) {
  const int2 l = list[blockIdx.x];
  const MetaItem& m = items[l.x];
  const int64_t k = (int64_t)l.y + threadIdx.x;
  if (k < m.n) hash_row(m.codes, k, m.alpha, (uint32_t)(m.w / m.alpha), (uint32_t)m.block, Key{m.k0, m.k1});
}

__global__ void __launch_bounds__(256) sjlt_count_batch(const MetaItem* __restrict__ items,
                                                        const int2* __restrict__ list) {
  __shared__ int cnt[1024];
  const int2 l = list[blockIdx.x];
  const MetaItem& m = items[l.x];
  count_chunk(m.codes, m.ptr, m.n, m.alpha, m.w, m.kc, l.y, cnt);
}

__global__ void __launch_bounds__(64) chunk_scan_batch(const MetaItem* __restrict__ items,
                                                       const int2* __restrict__ list) {
  const int2 l = list[blockIdx.x];
  const MetaItem& m = items[l.x];
  scan_chunk(m.ptr, m.w, m.kcap, l.y);
}

__global__ void __launch_bounds__(KC_MAX) sjlt_scatter_batch(const MetaItem* __restrict__ items,
                                                             const int2* __restrict__ list) {
  __shared__ uint32_t sc[KC_MAX * 32];
  const int2 l = list[blockIdx.x];
  const MetaItem& m = items[l.x];
  scatter_chunk(m.codes, m.ptr, m.ent, m.n, m.alpha, m.w, m.kc, m.kcap, l.y, sc);
}

int launch_sjlt_meta_batch(const MetaItem* items, const int2* rows, int nrows, const int2* chunks, int nchunks,
                           int kc, hipStream_t st) {
  if (nrows == 0 || nchunks == 0) return SK_OK;
  sjlt_hash_batch<<<nrows, 256, 0, st>>>(items, rows);
  SK_HIP(hipGetLastError());
  sjlt_count_batch<<<nchunks, 256, 0, st>>>(items, chunks);
  SK_HIP(hipGetLastError());
  chunk_scan_batch<<<nchunks, 64, 0, st>>>(items, chunks);
  SK_HIP(hipGetLastError());
  sjlt_scatter_batch<<<nchunks, kc, 0, st>>>(items, chunks);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// Fused generation of one block's tables: one workgroup per chunk of one table
// set (S tables with chunk kc; optionally S' tables with chunk kct).  The
// workgroup hashes its chunk's sources (the S set also writes the codes), then
// counts, scans and scatters in LDS.  One launch replaces hash + count + scan +
// scatter per set, which were dominated by launch gaps.
struct MetaSet {
  int32_t* ptr;
  int32_t* ent;
  int32_t kc, kcap, nT;
};

__global__ void __launch_bounds__(KC_MAX) sjlt_meta_fused(uint32_t* __restrict__ codes, int64_t n, int alpha,
                                                          int w, uint32_t block, Key key, MetaSet s0, MetaSet s1) {
  __shared__ uint32_t sc[KC_MAX * 32];
  __shared__ int cnt[1025];
  const bool first = (int)blockIdx.x < s0.nT;
  const MetaSet& m = first ? s0 : s1;
  const int t = first ? blockIdx.x : blockIdx.x - s0.nT;
  const int kc = m.kc;
  const int64_t k0 = (int64_t)t * kc;
  const int nk = (int)min((int64_t)kc, n - k0);
  const uint32_t wc = (uint32_t)(w / alpha);
  // hash of the chunk's sources (same draws as hash_row)
  for (int kk = threadIdx.x; kk < nk; kk += blockDim.x) {
    const int64_t k = k0 + kk;
    const uint32_t sbits = philox(2u, block, (uint32_t)k, 0u, key.k0, key.k1).v[0];
    for (int c4 = 0; c4 < alpha; c4 += 4) {
      const U4 o = philox(1u, block, (uint32_t)k, (uint32_t)(c4 >> 2), key.k0, key.k1);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = c4 + q;
        if (c < alpha) {
          const uint32_t code = (((uint32_t)c * wc + mulhi(o.v[q], wc)) << 1) | ((sbits >> c) & 1u);
          sc[kk * alpha + c] = code;
          if (first) codes[k * alpha + c] = code;
        }
      }
    }
  }
  for (int j = threadIdx.x; j <= w; j += blockDim.x) cnt[j] = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < nk * alpha; e += blockDim.x) atomicAdd(&cnt[sc[e] >> 1], 1);
  __syncthreads();
  // exclusive scan of the counts (thread 0, in order), offset by the region start
  if (threadIdx.x == 0) {
    int32_t run = (int32_t)t * m.kcap;
    for (int j = 0; j < w; ++j) {
      const int32_t c = cnt[j];
      cnt[j] = run;
      run += c;
    }
    cnt[w] = run;
  }
  for (int e = threadIdx.x; e < m.kcap; e += blockDim.x) m.ent[(int64_t)t * m.kcap + e] = kc << 1;  // nulls
  __syncthreads();
  for (int j = threadIdx.x; j <= w; j += blockDim.x) m.ptr[(int64_t)t * (w + 1) + j] = cnt[j];
  const int kk = threadIdx.x;
  if (kk < nk) {
    for (int c = 0; c < alpha; ++c) {
      const uint32_t code = sc[kk * alpha + c];
      const uint32_t col = code >> 1;
      int rank = 0;
      for (int q = 0; q < kk; ++q) rank += (sc[q * alpha + c] >> 1) == col;
      m.ent[cnt[col] + rank] = (kk << 1) | (int)(code & 1u);
    }
  }
}

int launch_sjlt_meta(Handle* h, Block& b, hipStream_t st) {
  const int64_t n = h->n;
  SK_REQUIRE(b.w <= 1024 && (int64_t)h->alpha * KC_MAX <= KC_MAX * 32, SK_EINVAL, "block too wide for the tables");
  MetaSet s0{b.ptr, b.ent, h->kc, sjlt_kcap(h->kc, h->alpha, b.w), (int)((n + h->kc - 1) / h->kc)};
  MetaSet s1{nullptr, nullptr, 64, 0, 0};
  if (b.ptr_t) s1 = MetaSet{b.ptr_t, b.ent_t, h->kct, sjlt_kcap(h->kct, h->alpha, b.w), (int)((n + h->kct - 1) / h->kct)};
  ProfScope ps(h->ctx, "sjlt_meta", st);
  sjlt_meta_fused<<<s0.nT + s1.nT, KC_MAX, 0, st>>>(b.codes, n, h->alpha, b.w, (uint32_t)b.index, key_of(h->seed),
                                                     s0, s1);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename T>
__global__ void __launch_bounds__(256) srht_D_kernel(int8_t* __restrict__ D, T* __restrict__ Dv, int64_t n, Key key) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int neg = srht_neg(key, (uint32_t)k);
  D[k] = neg ? (int8_t)-1 : (int8_t)1;
  Dv[k] = neg ? T(-1) : T(1);
}

// word q of the sign bits: bit b set when D_{32 q + b} = -1 (zero past n)
__global__ void __launch_bounds__(256) srht_Db_kernel(uint32_t* __restrict__ Db, int64_t nwords, int64_t n, Key key) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nwords) return;
  uint32_t w = 0;
  for (int b = 0; b < 32; ++b) {
    const int64_t k = 32 * q + b;
    if (k < n && srht_neg(key, (uint32_t)k)) w |= 1u << b;
  }
  Db[q] = w;
}

__global__ void __launch_bounds__(256) srht_mu_kernel(uint32_t* __restrict__ mu, int64_t j0, int64_t j1,
                                                      uint32_t nu, Key key) {
  const int64_t j = j0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < j1) mu[j] = srht_mu(key, (uint32_t)j, nu);
}

int launch_srht_meta(Handle* h, int64_t j0, int64_t j1, bool draw_D, hipStream_t st) {
  const Key key = key_of(h->seed);
  if (draw_D) {
    const unsigned nb = (unsigned)((h->n + 255) / 256);
    if (h->dtype == SK_F64) srht_D_kernel<double><<<nb, 256, 0, st>>>(h->srht_D, (double*)h->srht_Dv, h->n, key);
    else srht_D_kernel<float><<<nb, 256, 0, st>>>(h->srht_D, (float*)h->srht_Dv, h->n, key);
    SK_HIP(hipGetLastError());
    const int64_t nwords = (h->n + 255) / 256 * 8;
    srht_Db_kernel<<<(unsigned)((nwords + 255) / 256), 256, 0, st>>>(h->srht_Db, nwords, h->n, key);
    SK_HIP(hipGetLastError());
  }
  if (j1 > j0) {
    srht_mu_kernel<<<(unsigned)((j1 - j0 + 255) / 256), 256, 0, st>>>(h->srht_mu, j0, j1, (uint32_t)h->n, key);
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

__global__ void __launch_bounds__(256) gauss_kernel(uint16_t* __restrict__ g, int64_t n, int w, int64_t col0,
                                                    Key key) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int jj = blockIdx.y;
  if (k < n) g[k + (int64_t)jj * n] = bf16_bits_of_grid_value(gauss_raw(key, (uint32_t)k, (uint32_t)(col0 + jj)));
}

int launch_gauss_meta(Handle* h, Block& b, hipStream_t st) {
  dim3 grid((unsigned)((h->n + 255) / 256), (unsigned)b.w);
  gauss_kernel<<<grid, 256, 0, st>>>(b.gbf, h->n, b.w, b.col0, key_of(h->seed));
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk

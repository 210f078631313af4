// Operator block generation on the device (random matrix construction; the paper
// notes its cost is negligible next to the sketch, section 8 serial results).
//
// SJLT: the hash of every (row, chunk) and, per block, bucket tables that list
// for each output column and each chunk of KC consecutive sources the sources
// that feed it, in ascending order (a counting sort, deterministic).
// SRHT: the Rademacher diagonal D and the sampled Hadamard columns mu.
// Gaussian: the bf16-grid draws of the block, column-major.
#include <algorithm>

#include "internal.hpp"

namespace sk {

// ---------------------------------------------------------------- SJLT tables
// Bucket table, chunk-major: ptr[t * (w + 1) + j] = first entry of column j in
// chunk t; slot w holds the end of the chunk's entries.  Chunk t owns the entry
// slots [t * kcap, (t + 1) * kcap); its unused slots hold null entries (source
// KC, sign +, a staged slot of zeros).  One workgroup of KC_MAX threads (four
// waves) builds one chunk: it hashes the chunk's sources into LDS, then counts,
// scans and scatters there.
constexpr int META_WAVES = KC_MAX / 64;

struct MetaLds {
  uint32_t sc[KC_MAX * 32];       // codes of the chunk; bits 16.. later hold the rank within the wave
  int cnt[1025];                  // per column: count, then first entry
  int wh[META_WAVES * 1024];      // per wave and column: count, then the count of the earlier waves
  int wsum[META_WAVES];
};

// Hash of source k0 + kk (one thread per source): for every chunk c of the
// block an offset in [0, w/alpha) and a sign, as code = (column << 1) | negative.
// With GRAPH the alpha columns of a source are the graph construction's
// distinct draws over the whole block (width w = wc * alpha is not required:
// wc carries w itself).
template <bool GRAPH>
__device__ __forceinline__ void hash_chunk(MetaLds& L, uint32_t* __restrict__ codes, bool write_codes, int64_t k0,
                                           int nk, int alpha, uint32_t wc, uint32_t block, Key key) {
  const int kk = threadIdx.x;
  if (kk >= nk) return;
  const int64_t k = k0 + kk;
  if constexpr (GRAPH) {
    uint32_t* sc = &L.sc[kk * alpha];
    sjlt_graph_codes(key, block, (uint32_t)k, alpha, wc, sc);
    if (write_codes)
      for (int c = 0; c < alpha; ++c) codes[k * alpha + c] = sc[c];
    return;
  }
  const uint32_t sbits = philox(2u, block, (uint32_t)k, 0u, key.k0, key.k1).v[0];
  for (int c4 = 0; c4 < alpha; c4 += 4) {
    const U4 o = philox(1u, block, (uint32_t)k, (uint32_t)(c4 >> 2), key.k0, key.k1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = c4 + q;
      if (c < alpha) {
        const uint32_t code = (((uint32_t)c * wc + mulhi(o.v[q], wc)) << 1) | ((sbits >> c) & 1u);
        L.sc[kk * alpha + c] = code;
        if (write_codes) codes[k * alpha + c] = code;
      }
    }
  }
}

// Tables of chunk t from the codes in L.sc.  A source's rank inside its bucket
// counts the earlier sources of the chunk in the same bucket, so every bucket
// lists its sources in ascending order.  Within a wave the rank comes from
// matching lanes by ballot (one round per distinct column among the wave's
// lanes); the earlier waves contribute their per-column counts.  Column starts
// come from a workgroup-wide exclusive scan.  Requires blockDim.x == KC_MAX and
// w <= 1024; the caller's writes of L.sc are ordered by the first barrier.
//
// GRAPH: a column may come from any c (the columns of one source are distinct,
// so a lane holds a column at most once).  One round per distinct column among
// the wave's entries matches it against all alpha codes of every lane: the
// lanes holding it form one mask M, and a lane's rank is the number of lanes
// of M below it.
template <bool GRAPH>
__device__ __forceinline__ void bucket_chunk(MetaLds& L, int nk, int alpha, int w, int kc, int kcap, int t,
                                             int32_t* __restrict__ ptr, int32_t* __restrict__ ent) {
  const int kk = threadIdx.x, lane = kk & 63, wv = kk >> 6;
  for (int j = kk; j < META_WAVES * w; j += KC_MAX) L.wh[j] = 0;
  for (int e = kk; e < kcap; e += KC_MAX) ent[(int64_t)t * kcap + e] = kc << 1;  // null entries
  __syncthreads();
  const bool act = kk < nk;
  const uint64_t below = (1ull << lane) - 1ull;
  if constexpr (GRAPH) {
    // bits of this lane's codes not yet ranked (codes hold (col << 1) | neg in
    // their low 16 bits; ranks go to bits 16.. as they are found)
    uint32_t pend = act ? (alpha >= 32 ? 0xFFFFFFFFu : (1u << alpha) - 1u) : 0u;
    for (;;) {
      const uint64_t any = __ballot(pend != 0u);
      if (!any) break;
      const int lead = __builtin_ctzll(any);
      const int c0 = pend ? __builtin_ctz(pend) : 0;
      const uint32_t mine = act ? (L.sc[kk * alpha + c0] & 0xFFFFu) >> 1 : 0u;
      const uint32_t lc = __builtin_amdgcn_readlane(mine, lead);  // this round's column
      int hit = -1;
      if (act)
        for (int c = 0; c < alpha; ++c)
          if (((L.sc[kk * alpha + c] & 0xFFFFu) >> 1) == lc) hit = c;
      const uint64_t M = __ballot(hit >= 0);
      if (hit >= 0) {
        L.sc[kk * alpha + hit] |= (uint32_t)__popcll(M & below) << 16;
        pend &= ~(1u << hit);
      }
      if (lane == lead) L.wh[wv * w + lc] = __popcll(M);
    }
  } else {
  for (int c = 0; c < alpha; ++c) {
    const uint32_t col = act ? (L.sc[kk * alpha + c] >> 1) : 0xFFFFFFFFu;
    uint64_t todo = __ballot(act);
    uint32_t r = 0;
    while (todo) {
      const int lead = __builtin_ctzll(todo);
      const uint32_t lc = __builtin_amdgcn_readlane(col, lead);
      const uint64_t same = __ballot(col == lc);
      if (col == lc) r = (uint32_t)__popcll(same & below);
      if (lane == lead) L.wh[wv * w + lc] = __popcll(same);  // chunks c own disjoint columns
      todo &= ~same;
    }
    if (act) L.sc[kk * alpha + c] |= r << 16;
  }
  }
  __syncthreads();
  // per column: the counts of the earlier waves (in place) and the chunk's count
  for (int j = kk; j < w; j += KC_MAX) {
    int run = 0;
    for (int v = 0; v < META_WAVES; ++v) {
      const int x = L.wh[v * w + j];
      L.wh[v * w + j] = run;
      run += x;
    }
    L.cnt[j] = run;
  }
  __syncthreads();
  // exclusive scan of the w counts from the region start, four columns per thread
  int loc[4], own = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 4 * kk + q;
    loc[q] = j < w ? L.cnt[j] : 0;
    own += loc[q];
  }
  int inc = own;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) L.wsum[wv] = inc;
  __syncthreads();
  int run = t * kcap + inc - own;
  for (int v = 0; v < wv; ++v) run += L.wsum[v];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 4 * kk + q;
    if (j < w) L.cnt[j] = run;
    run += loc[q];
  }
  if (kk == KC_MAX - 1) L.cnt[w] = run;  // the end of the chunk's entries
  __syncthreads();
  for (int j = kk; j <= w; j += KC_MAX) ptr[(int64_t)t * (w + 1) + j] = L.cnt[j];
  if (!act) return;
  for (int c = 0; c < alpha; ++c) {
    const uint32_t v = L.sc[kk * alpha + c];
    const uint32_t col = (v & 0xFFFFu) >> 1;
    ent[L.cnt[col] + L.wh[wv * w + col] + (int)(v >> 16)] = (kk << 1) | (int)(v & 1u);
  }
}

// Batched: one workgroup per (item, chunk) of every operator block of a round.
__global__ void __launch_bounds__(KC_MAX) sjlt_meta_batch(const MetaItem* __restrict__ items,
                                                          const int2* __restrict__ list) {
  __shared__ MetaLds L;
  const int2 l = list[blockIdx.x];
  const MetaItem& m = items[l.x];
  const int64_t k0 = (int64_t)l.y * m.kc;
  const int nk = (int)min((int64_t)m.kc, m.n - k0);
  hash_chunk<false>(L, m.codes, true, k0, nk, m.alpha, (uint32_t)(m.w / m.alpha), (uint32_t)m.block,
                    Key{m.k0, m.k1});
  bucket_chunk<false>(L, nk, m.alpha, m.w, m.kc, m.kcap, l.y, m.ptr, m.ent);
}

int launch_sjlt_meta_batch(const MetaItem* items, const int2* chunks, int nchunks, hipStream_t st) {
  if (nchunks == 0) return SK_OK;
  sjlt_meta_batch<<<nchunks, KC_MAX, 0, st>>>(items, chunks);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// The tables of up to META_MAX_BLOCKS blocks in one launch: one workgroup per
// chunk of each table set of each block (S tables with chunk kc; optionally S'
// tables with chunk kct).  The S set also writes the block's codes.
struct MetaSet {
  int32_t* ptr;
  int32_t* ent;
  int32_t kc, kcap, nT;
};
constexpr int META_MAX_BLOCKS = 8;
struct MetaBlocks {
  uint32_t* codes[META_MAX_BLOCKS];
  MetaSet set[META_MAX_BLOCKS][2];
  int32_t w[META_MAX_BLOCKS];
  uint32_t index[META_MAX_BLOCKS];
  int32_t first[META_MAX_BLOCKS + 1];  // first workgroup of each block
  int32_t nb;
};

template <bool GRAPH>
__global__ void __launch_bounds__(KC_MAX) sjlt_meta_fused(MetaBlocks mb, int64_t n, int alpha, Key key) {
  __shared__ MetaLds L;
  int b = 0;
  while (b + 1 < mb.nb && (int)blockIdx.x >= mb.first[b + 1]) ++b;
  int t = (int)blockIdx.x - mb.first[b];
  const bool s0 = t < mb.set[b][0].nT;
  if (!s0) t -= mb.set[b][0].nT;
  const MetaSet& m = mb.set[b][s0 ? 0 : 1];
  const int w = mb.w[b];
  const int64_t k0 = (int64_t)t * m.kc;
  const int nk = (int)min((int64_t)m.kc, n - k0);
  hash_chunk<GRAPH>(L, mb.codes[b], s0, k0, nk, alpha, GRAPH ? (uint32_t)w : (uint32_t)(w / alpha), mb.index[b],
                    key);
  bucket_chunk<GRAPH>(L, nk, alpha, w, m.kc, m.kcap, t, m.ptr, m.ent);
}

int launch_sjlt_meta(Handle* h, int b0, int b1, hipStream_t st) {
  const int64_t n = h->n;
  SK_REQUIRE(h->alpha <= 32, SK_EINVAL, "alpha too large for the tables");
  for (int c0 = b0; c0 < b1; c0 += META_MAX_BLOCKS) {
    MetaBlocks mb{};
    mb.nb = std::min(META_MAX_BLOCKS, b1 - c0);
    int grid = 0;
    for (int i = 0; i < mb.nb; ++i) {
      const Block& b = h->blocks[c0 + i];
      SK_REQUIRE(b.w <= 1024, SK_EINVAL, "block too wide for the tables");
      mb.codes[i] = b.codes;
      mb.set[i][0] = MetaSet{b.ptr, b.ent, h->kc, sjlt_kcap(h->kc, h->alpha, b.w), (int)((n + h->kc - 1) / h->kc)};
      mb.set[i][1] = b.ptr_t ? MetaSet{b.ptr_t, b.ent_t, h->kct, sjlt_kcap(h->kct, h->alpha, b.w),
                                       (int)((n + h->kct - 1) / h->kct)}
                             : MetaSet{nullptr, nullptr, 64, 0, 0};
      mb.w[i] = b.w;
      mb.index[i] = (uint32_t)b.index;
      mb.first[i] = grid;
      grid += mb.set[i][0].nT + mb.set[i][1].nT;
    }
    mb.first[mb.nb] = grid;
    ProfScope ps(h->ctx, "sjlt_meta", st);
    if (h->construction == SK_SJLT_GRAPH)
      sjlt_meta_fused<true><<<grid, KC_MAX, 0, st>>>(mb, n, h->alpha, key_of(h->seed));
    else
      sjlt_meta_fused<false><<<grid, KC_MAX, 0, st>>>(mb, n, h->alpha, key_of(h->seed));
    SK_HIP(hipGetLastError());
  }
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
    srht_mu_kernel<<<(unsigned)((j1 - j0 + 255) / 256), 256, 0, st>>>(h->srht_mu, j0, j1, srht_nu(h->n), key);
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

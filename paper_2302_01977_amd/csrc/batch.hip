// Batched persistent SJLT sketch: many stored, column-major matrices of uneven
// size, each with its own operator grown in blocks of dd columns (the adaptive
// extension of Algorithm 1, run for a whole batch of independent compressions).
// Round r draws block r of every operator whose target width exceeds r * dd and
// computes S_i(:, r dd : (r+1) dd) = A_i R_i,r (and S'_i = A_i^T R_i,r), with
// one launch per step: four batched operator-generation kernels and one
// persistent sketch kernel walking an (item, row tile) work list, optionally
// captured once per round in a HIP graph and replayed.  The tile shape comes
// from a built-in heuristic or from an autotuner that times the candidate shapes
// on the batch itself and caches the winner in the context.
#include <algorithm>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "sjlt_tile.hpp"

namespace sk {

// One matrix of a batch: a single operator block applied as S = A R_b (or
// S' = A^T R_b), written to out (the block's first column, leading dimension
// ldo).
struct BatchItem {
  const void* A;
  int64_t lda, L, K;
  void* out;
  int64_t ldo;
  const int32_t* ptr;  // bucket table of the block
  const int32_t* ent;  // entries of the block
  int32_t nT, w, kcap, ms;
  double scale;
};

// Persistent batched sketch: a grid sized to the resident capacity walks the
// work list (item, row tile) with a static stride; the list is sorted by
// decreasing work, so the largest tiles start first.  Every item's columns fit
// one workgroup (NW * NJ >= w).
template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK, bool LDSE>
__global__ void __launch_bounds__(NW * 64)
    sjlt_batch_kernel(const BatchItem* __restrict__ items, const int2* __restrict__ work, int nwork) {
  constexpr int TL = 64 * RPL;
  constexpr int NTHR = NW * 64;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const int2 wk = work[wi];
    const BatchItem& it = items[wk.x];
    const int64_t l0 = (int64_t)wk.y * TL;
    const int jb = wave * NJ;
    const bool active = jb < it.w;
    const uint32_t* eptr[2] = {nullptr, nullptr};
    if constexpr (LDSE) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q0 = (tid + h * NTHR) * 4;
        if (q0 < it.kcap) eptr[h] = (const uint32_t*)it.ent + q0;
      }
    }
    sjlt_tile<T, TRANS, NW, NJ, RPL, KCK, LDSE>((const T*)it.A, it.lda, it.L, it.K, l0, 0, it.nT, active,
                                                it.ptr + jb, (int64_t)it.w + 1, it.ent, 0, eptr[0], eptr[1],
                                                it.kcap, it.kcap, it.ms, (T*)it.out + (int64_t)jb * it.ldo, it.ldo,
                                                (T)it.scale);
    __syncthreads();  // the next item reuses the LDS
  }
}

// ------------------------------------------------------------ shape table
struct BatchCfg {
  int kc, nw, nj, rpl;
};

template <typename T, bool TRANS, int NW, int NJ, int RPL, int KCK>
static int run_batch(const BatchItem* items, const int2* work, int nwork, int kcap, int num_cu, bool launch,
                     hipStream_t st) {
  if constexpr (!GatherValid<T, TRANS, NW, NJ, RPL, KCK>::value) {
    return 1;
  } else {
    const size_t shmem = gather_lds_bytes((int)sizeof(T), KCK, 64 * RPL, true, 1, kcap);
    if (shmem > 160 * 1024) return 1;
    auto kern = sjlt_batch_kernel<T, TRANS, NW, NJ, RPL, KCK, true>;
    static bool attr_set = false;
    if (!attr_set) {
      SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
      attr_set = true;
    }
    if (!launch || nwork == 0) return SK_OK;
    // resident capacity: LDS per workgroup, and at most 32 waves per CU
    const int per_cu = std::max(1, std::min((int)((160 * 1024) / shmem), 32 / NW));
    const int grid = std::min(nwork, per_cu * num_cu);
    kern<<<grid, NW * 64, shmem, st>>>(items, work, nwork);
    SK_HIP(hipGetLastError());
    return SK_OK;
  }
}

#define SK_BT(NW_, NJ_, RPL_, KC_)                                                                         \
  if (c.nw == NW_ && c.nj == NJ_ && c.rpl == RPL_ && c.kc == KC_) {                                       \
    rc = trans ? run_batch<T, true, NW_, NJ_, RPL_, KC_>(items, work, nwork, kcap, num_cu, launch, st)   \
               : run_batch<T, false, NW_, NJ_, RPL_, KC_>(items, work, nwork, kcap, num_cu, launch, st); \
    return rc;                                                                                             \
  }
#define SK_BT_NW(RPL_, KC_)                                                                    \
  SK_BT(4, 16, RPL_, KC_) SK_BT(8, 16, RPL_, KC_) SK_BT(8, 32, RPL_, KC_) SK_BT(8, 8, RPL_, KC_) \
  SK_BT(16, 4, RPL_, KC_) SK_BT(16, 8, RPL_, KC_) SK_BT(16, 16, RPL_, KC_)

// 0 = launched (or prepared), 1 = shape not available, < 0 = error
template <typename T>
static int batch_dispatch(const BatchCfg& c, bool trans, const BatchItem* items, const int2* work, int nwork,
                          int kcap, int num_cu, bool launch, hipStream_t st) {
  int rc = 1;
  if constexpr (sizeof(T) == 4) {
    SK_BT_NW(4, 64) SK_BT_NW(2, 64) SK_BT_NW(1, 64) SK_BT_NW(2, 128) SK_BT_NW(1, 128) SK_BT_NW(1, 256)
  } else {
    SK_BT_NW(2, 64) SK_BT_NW(1, 64) SK_BT_NW(1, 128) SK_BT_NW(1, 256)
  }
  return rc;
}
#undef SK_BT_NW
#undef SK_BT

static int batch_launch(int dtype, const BatchCfg& c, bool trans, const BatchItem* items, const int2* work,
                        int nwork, int kcap, int num_cu, bool launch, hipStream_t st) {
  return dtype == SK_F64 ? batch_dispatch<double>(c, trans, items, work, nwork, kcap, num_cu, launch, st)
                         : batch_dispatch<float>(c, trans, items, work, nwork, kcap, num_cu, launch, st);
}

// candidate shapes for a block width: every wave owns NJ of the dd columns
// (fewer columns per wave = more waves per workgroup)
static std::vector<BatchCfg> batch_candidates(int dtype, int dd, int alpha, bool need_t = true) {
  std::vector<BatchCfg> out;
  std::vector<std::pair<int, int>> wj;  // (waves, columns per wave)
  if (dd == 64) wj = {{4, 16}, {8, 8}, {16, 4}};
  else if (dd == 128) wj = {{8, 16}, {16, 8}};
  else if (dd == 256) wj = {{8, 32}, {16, 16}};
  else return out;
  const int kr32[][2] = {{64, 4}, {64, 2}, {64, 1}, {128, 2}, {128, 1}, {256, 1}};
  const int kr64[][2] = {{64, 2}, {64, 1}, {128, 1}, {256, 1}};
  const int nkr = dtype == SK_F64 ? 4 : 6;
  for (const auto& p : wj) {
    const int nw = p.first, nj = p.second;
    for (int i = 0; i < nkr; ++i) {
      const int kc = dtype == SK_F64 ? kr64[i][0] : kr32[i][0];
      const int rpl = dtype == SK_F64 ? kr64[i][1] : kr32[i][1];
      if ((int64_t)kc * alpha > 32 * (int64_t)KC_MAX) continue;       // scatter staging capacity
      if (nj * rpl * (dtype == SK_F64 ? 2 : 1) > 64) continue;       // accumulators per lane
      if (sjlt_kcap(kc, alpha, dd) > nw * 64 * 8) continue;          // entry staging capacity
      // the tile must split evenly over the workgroup (S' moves whole blocks)
      const bool ok = dtype == SK_F64 ? cfg_valid<double, false>(nw, rpl, kc) &&
                                            (!need_t || cfg_valid<double, true>(nw, rpl, kc))
                                      : cfg_valid<float, false>(nw, rpl, kc) &&
                                            (!need_t || cfg_valid<float, true>(nw, rpl, kc));
      if (!ok) continue;
      if (gather_lds_bytes(dtype == SK_F64 ? 8 : 4, kc, 64 * rpl, true, 1, sjlt_kcap(kc, alpha, dd)) > 160 * 1024)
        continue;
      out.push_back(BatchCfg{kc, nw, nj, rpl});
    }
  }
  return out;
}

static BatchCfg batch_default(int dtype, int dd, int alpha) {
  std::vector<BatchCfg> c = batch_candidates(dtype, dd, alpha);
  const int kc = sjlt_chunk_for(dd, alpha, 4);
  const int rpl = dtype == SK_F32 ? (kc == 64 ? 4 : kc == 128 ? 2 : 1) : (kc == 64 ? 2 : 1);
  for (const BatchCfg& b : c)
    if (b.kc == kc && b.rpl == rpl) return b;
  return c.empty() ? BatchCfg{0, 0, 0, 0} : c.front();
}

// ------------------------------------------------------------ batch object
struct BatchRound {
  MetaItem* d_meta = nullptr;
  int2* d_chunks = nullptr;
  BatchItem* d_items = nullptr;
  int2* d_work[2] = {nullptr, nullptr};  // S, S'
  int nmeta = 0, nchunks = 0, nwork[2] = {0, 0};
  std::vector<MetaItem> h_meta;
  std::vector<int> meta_matrix;  // matrix of each meta item
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool eager = false;  // graph capture failed: the round runs launch by launch
};

struct Batch {
  uint32_t magic = 0x534b4254u;  // "SKBT"
  Ctx* ctx = nullptr;
  int dtype = 0, alpha = 4, dd = 64, count = 0, flags = 0, kcap = 0;
  BatchCfg cfg{};
  std::vector<sk_input> ins;
  std::vector<sk_output> outs;
  std::vector<int32_t> d;
  std::vector<uint64_t> seeds;
  char* meta_buf = nullptr;  // operator metadata of every (matrix, block)
  std::vector<BatchRound> rounds;
  hipStream_t cap = nullptr;  // private stream for graph capture
};

static void free_round(BatchRound& r) {
  if (r.gexec) (void)hipGraphExecDestroy(r.gexec);
  if (r.graph) (void)hipGraphDestroy(r.graph);
  void* ps[] = {r.d_meta, r.d_chunks, r.d_items, r.d_work[0], r.d_work[1]};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  r = BatchRound();
}

static void free_batch_buffers(Batch* b) {
  for (auto& r : b->rounds) free_round(r);
  b->rounds.clear();
  if (b->meta_buf) (void)hipFree(b->meta_buf);
  b->meta_buf = nullptr;
}

template <typename P>
static int upload(Ctx* c, P** dst, const std::vector<P>& v, hipStream_t st) {
  if (v.empty()) return SK_OK;
  if (int rc = ctx_malloc(c, (void**)dst, sizeof(P) * v.size())) return rc;
  SK_HIP(hipMemcpyAsync(*dst, v.data(), sizeof(P) * v.size(), hipMemcpyHostToDevice, st));
  return SK_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Lay out the metadata of every (matrix, block) for shape c and build the
// per-round launch lists.  Host arrays are uploaded on st (the call returns
// after st has finished them, so they can be freed).
static int build_rounds(Batch* b, const BatchCfg& c, int max_rounds, hipStream_t st) {
  free_batch_buffers(b);
  b->cfg = c;
  b->kcap = sjlt_kcap(c.kc, b->alpha, b->dd);
  const int nr = std::min(max_rounds, *std::max_element(b->d.begin(), b->d.end()) / b->dd);
  // metadata sizes
  std::vector<size_t> off_codes, off_ptr, off_ent;
  size_t total = 0;
  for (int r = 0; r < nr; ++r)
    for (int i = 0; i < b->count; ++i) {
      if (b->d[i] <= r * b->dd) continue;
      const int64_t n = b->ins[i].n;
      const int64_t nT = (n + c.kc - 1) / c.kc;
      off_codes.push_back(total);
      total += align256(sizeof(uint32_t) * n * b->alpha);
      off_ptr.push_back(total);
      total += align256(sizeof(int32_t) * nT * (b->dd + 1));
      off_ent.push_back(total);
      total += align256(sizeof(int32_t) * nT * b->kcap);
    }
  if (int rc = ctx_malloc(b->ctx, (void**)&b->meta_buf, std::max<size_t>(total, 256))) return rc;
  const Key dummy{0, 0};
  (void)dummy;
  const int TL = 64 * c.rpl;
  b->rounds.resize(nr);
  size_t q = 0;
  for (int r = 0; r < nr; ++r) {
    BatchRound& R = b->rounds[r];
    std::vector<int2> chunks;
    std::vector<BatchItem> items;
    std::vector<std::pair<int64_t, int2>> work[2];
    for (int i = 0; i < b->count; ++i) {
      if (b->d[i] <= r * b->dd) continue;
      const sk_input& in = b->ins[i];
      const int64_t n = in.n;
      const int nT = (int)((n + c.kc - 1) / c.kc);
      MetaItem m;
      m.codes = (uint32_t*)(b->meta_buf + off_codes[q]);
      m.ptr = (int32_t*)(b->meta_buf + off_ptr[q]);
      m.ent = (int32_t*)(b->meta_buf + off_ent[q]);
      ++q;
      m.n = n;
      m.w = b->dd;
      m.alpha = b->alpha;
      m.kc = c.kc;
      m.kcap = b->kcap;
      m.block = r;
      const Key k = key_of(b->seeds[i]);
      m.k0 = k.k0;
      m.k1 = k.k1;
      const int mi = (int)R.h_meta.size();
      R.h_meta.push_back(m);
      R.meta_matrix.push_back(i);
      for (int t = 0; t < nT; ++t) chunks.push_back(make_int2(mi, t));
      const int ms = (int64_t)c.kc * b->alpha >= 7LL * b->dd ? 8 : 4;  // straight-line slots (4 or 8)
      const sk_output& o = b->outs[i];
      const size_t esz = b->dtype == SK_F64 ? 8 : 4;
      for (int tr = 0; tr < 2; ++tr) {
        void* base = tr ? o.St : o.S;
        if (!base) continue;
        const int64_t ld = tr ? o.ldSt : o.ldS;
        BatchItem it;
        it.A = in.A;
        it.lda = in.lda;
        it.L = tr ? in.n : in.m;
        it.K = tr ? in.m : in.n;
        it.out = (char*)base + (size_t)r * b->dd * ld * esz;
        it.ldo = ld;
        it.ptr = m.ptr;
        it.ent = m.ent;
        it.nT = nT;
        it.w = b->dd;
        it.kcap = b->kcap;
        it.ms = ms;
        it.scale = 1.0 / sqrt((double)b->alpha);
        const int ii = (int)items.size();
        items.push_back(it);
        for (int64_t p = 0; p * TL < it.L; ++p) work[tr].push_back({it.K, make_int2(ii, (int)p)});
      }
    }
    R.nmeta = (int)R.h_meta.size();
    R.nchunks = (int)chunks.size();
    if (int rc = upload(b->ctx, &R.d_meta, R.h_meta, st)) return rc;
    if (int rc = upload(b->ctx, &R.d_chunks, chunks, st)) return rc;
    if (int rc = upload(b->ctx, &R.d_items, items, st)) return rc;
    for (int tr = 0; tr < 2; ++tr) {
      // largest tiles (most sources) first; ties in item order
      std::stable_sort(work[tr].begin(), work[tr].end(),
                       [](const std::pair<int64_t, int2>& a, const std::pair<int64_t, int2>& c2) {
                         return a.first > c2.first;
                       });
      std::vector<int2> wl;
      for (auto& w : work[tr]) wl.push_back(w.second);
      R.nwork[tr] = (int)wl.size();
      if (int rc = upload(b->ctx, &R.d_work[tr], wl, st)) return rc;
    }
    SK_HIP(hipStreamSynchronize(st));  // the host vectors above go out of scope
  }
  return SK_OK;
}

// the kernels of one round, in stream order
static int round_kernels(Batch* b, BatchRound& R, hipStream_t st) {
  if (int rc = launch_sjlt_meta_batch(R.d_meta, R.d_chunks, R.nchunks, st)) return rc;
  for (int tr = 0; tr < 2; ++tr) {
    if (!R.nwork[tr]) continue;
    const int rc = batch_launch(b->dtype, b->cfg, tr == 1, R.d_items, R.d_work[tr], R.nwork[tr], b->kcap,
                                b->ctx->num_cu, true, st);
    if (rc == 1) {
      set_error("internal: no batched SJLT kernel for KC=%d NW=%d NJ=%d RPL=%d", b->cfg.kc, b->cfg.nw, b->cfg.nj,
                b->cfg.rpl);
      return SK_EINVAL;
    }
    if (rc) return rc;
  }
  return SK_OK;
}

// Capture round R into a graph on the private stream.  Returns SK_OK with
// R.gexec set, or an error code; on error nothing of the capture is left.
static int capture_round(Batch* b, BatchRound& R) {
  if (!b->cap) SK_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  SK_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
  const int rc = round_kernels(b, R, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (rc || e != hipSuccess || b->ctx->fail_graph) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    set_error("graph capture failed (injected by the graph-failure test hook)");
    return SK_EHIP;
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return hip_fail(ei, "hipGraphInstantiate");
  }
  R.graph = g;
  R.gexec = x;
  return SK_OK;
}

static int run_round(Batch* b, int r, hipStream_t st) {
  BatchRound& R = b->rounds[r];
  ProfScope ps(b->ctx, "sjlt_batch", st);
  if (!(b->flags & SK_BATCH_GRAPH) || R.eager) return round_kernels(b, R, st);
  if (!R.gexec && capture_round(b, R) != SK_OK) {
    // a round that cannot be captured (the runtime refuses the capture or the
    // instantiation) runs launch by launch from now on: same kernels, same
    // arguments, so the results do not change
    R.eager = true;
    return round_kernels(b, R, st);
  }
  SK_HIP(hipGraphLaunch(R.gexec, st));
  return SK_OK;
}

// time round 0 for every candidate shape and keep the fastest
static int autotune(Batch* b, hipStream_t st, BatchCfg* best) {
  char key[160];
  int64_t nsum = 0, nmax = 0;
  bool any_t = false;
  for (int i = 0; i < b->count; ++i) {
    nsum += b->ins[i].n;
    nmax = std::max<int64_t>(nmax, b->ins[i].n);
    any_t = any_t || b->outs[i].St;
  }
  snprintf(key, sizeof(key), "batch:%d:%d:%d:%d:%d:%lld:%lld", b->dtype, b->dd, b->alpha, (int)any_t, b->count,
           (long long)nsum, (long long)nmax);
  auto hit = b->ctx->tune.find(key);
  if (hit != b->ctx->tune.end()) {
    *best = BatchCfg{hit->second[0], hit->second[1], hit->second[2], hit->second[3]};
    return SK_OK;
  }
  std::vector<BatchCfg> cand = batch_candidates(b->dtype, b->dd, b->alpha, any_t);
  SK_REQUIRE(!cand.empty(), SK_EUNSUPPORTED, "batched sketch supports block widths 64, 128 and 256");
  hipEvent_t e0, e1;
  SK_HIP(hipEventCreate(&e0));
  SK_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  int rc = SK_OK;
  const int saved_flags = b->flags;
  b->flags &= ~SK_BATCH_GRAPH;
  for (const BatchCfg& c : cand) {
    if ((rc = build_rounds(b, c, 1, st))) break;
    if ((rc = round_kernels(b, b->rounds[0], st))) break;  // warm-up
    float tot = 0.f;
    for (int rep = 0; rep < 3 && !rc; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) rc = SK_EHIP;
      if (!rc) rc = round_kernels(b, b->rounds[0], st);
      if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = SK_EHIP;
      if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = SK_EHIP;
      float ms = 0.f;
      if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = SK_EHIP;
      tot += ms;
    }
    if (rc) break;
    if (tot < best_ms) {
      best_ms = tot;
      *best = c;
    }
  }
  b->flags = saved_flags;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    if (rc == SK_EHIP) set_error("autotune: event timing failed");
    return rc;
  }
  b->ctx->tune[key] = {best->kc, best->nw, best->nj, best->rpl};
  return SK_OK;
}

}  // namespace sk

using namespace sk;

struct sk_batch {
  Batch b;
};

extern "C" {

int sketch_batch_create(sk_ctx* ctx, const sk_input* ins, int32_t count, const int32_t* d, int32_t dd,
                        int32_t alpha, const uint64_t* seeds, const sk_output* outs, int32_t flags, sk_batch** out,
                        void* stream) {
  SK_REQUIRE(ctx && ctx->c.magic == CTX_MAGIC, SK_ESTATE, "invalid or released context");
  SK_REQUIRE(ins && d && seeds && outs && out, SK_EINVAL, "NULL argument");
  SK_REQUIRE(count >= 1, SK_EINVAL, "count must be >= 1");
  SK_REQUIRE(alpha >= 1 && alpha <= 32, SK_EINVAL, "alpha must be in [1, 32]");
  SK_REQUIRE(dd == 64 || dd == 128 || dd == 256, SK_EUNSUPPORTED, "batched block width must be 64, 128 or 256");
  SK_REQUIRE(dd % alpha == 0, SK_EINVAL, "alpha must divide the block width");
  const int dtype = ins[0].dtype;
  SK_REQUIRE(dtype == SK_F64 || dtype == SK_F32, SK_EINVAL, "dtype must be SK_F64 or SK_F32");
  for (int i = 0; i < count; ++i) {
    const sk_input& in = ins[i];
    SK_REQUIRE(in.input == SK_DENSE && in.A, SK_EINVAL, "matrix %d: dense input with non-NULL A required", i);
    SK_REQUIRE(in.dtype == dtype, SK_EINVAL, "matrix %d: all matrices must share one dtype", i);
    SK_REQUIRE(in.m >= 1 && in.n >= 1 && in.n <= 0x7fffffffLL && in.m <= 0x7fffffffLL, SK_EINVAL,
               "matrix %d: sizes out of range", i);
    SK_REQUIRE(in.lda >= in.m, SK_EINVAL, "matrix %d: lda < m", i);
    SK_REQUIRE(d[i] >= dd && d[i] % dd == 0, SK_EINVAL, "matrix %d: d must be a positive multiple of dd", i);
    SK_REQUIRE(outs[i].S && outs[i].ldS >= in.m, SK_EINVAL, "matrix %d: S is NULL or ldS < m", i);
    SK_REQUIRE(!outs[i].St || (in.m == in.n && outs[i].ldSt >= in.n), SK_EINVAL,
               "matrix %d: S' needs a square matrix and ldSt >= n", i);
  }
  Ctx* c = &ctx->c;
  SK_HIP(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  sk_batch* B = new sk_batch();
  Batch* b = &B->b;
  b->ctx = c;
  b->dtype = dtype;
  b->alpha = alpha;
  b->dd = dd;
  b->count = count;
  b->flags = flags;
  b->ins.assign(ins, ins + count);
  b->outs.assign(outs, outs + count);
  b->d.assign(d, d + count);
  b->seeds.assign(seeds, seeds + count);
  BatchCfg cfg = batch_default(dtype, dd, alpha);
  int rc = cfg.kc ? SK_OK : SK_EUNSUPPORTED;
  if (rc) set_error("no batched shape for dd=%d alpha=%d", dd, alpha);
  if (!rc && (flags & SK_BATCH_AUTOTUNE)) rc = autotune(b, st, &cfg);
  if (!rc) rc = build_rounds(b, cfg, 1 << 30, st);
  if (!rc) {  // kernel attributes are set outside any capture
    bool any_t = false;
    for (int i = 0; i < count; ++i) any_t = any_t || outs[i].St;
    rc = batch_launch(dtype, cfg, false, nullptr, nullptr, 0, b->kcap, c->num_cu, false, st);
    if (!rc && any_t) rc = batch_launch(dtype, cfg, true, nullptr, nullptr, 0, b->kcap, c->num_cu, false, st);
    if (rc == 1) {
      set_error("internal: batched shape unavailable");
      rc = SK_EINVAL;
    }
  }
  if (rc) {
    const std::string msg = sketch_last_error();
    (void)hipStreamSynchronize(st);
    free_batch_buffers(b);
    delete B;
    set_error("%s", msg.c_str());
    return rc;
  }
  c->live_handles++;
  *out = B;
  return SK_OK;
}

int sketch_batch_run(sk_batch* B, int32_t r0, int32_t r1, void* stream) {
  SK_REQUIRE(B && B->b.magic == 0x534b4254u, SK_ESTATE, "invalid or destroyed batch");
  Batch* b = &B->b;
  SK_REQUIRE(0 <= r0 && r0 <= r1 && r1 <= (int)b->rounds.size(), SK_EINVAL, "rounds [%d, %d) outside [0, %d)", r0,
             r1, (int)b->rounds.size());
  SK_HIP(hipSetDevice(b->ctx->device));
  for (int r = r0; r < r1; ++r)
    if (int rc = run_round(b, r, (hipStream_t)stream)) return rc;
  return SK_OK;
}

int sketch_batch_reseed(sk_batch* B, const uint64_t* seeds, void* stream) {
  SK_REQUIRE(B && B->b.magic == 0x534b4254u, SK_ESTATE, "invalid or destroyed batch");
  SK_REQUIRE(seeds, SK_EINVAL, "seeds is NULL");
  Batch* b = &B->b;
  SK_HIP(hipSetDevice(b->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  b->seeds.assign(seeds, seeds + b->count);
  for (BatchRound& R : b->rounds) {
    for (int q = 0; q < R.nmeta; ++q) {
      const Key k = key_of(b->seeds[R.meta_matrix[q]]);
      R.h_meta[q].k0 = k.k0;
      R.h_meta[q].k1 = k.k1;
    }
    if (R.nmeta)
      SK_HIP(hipMemcpyAsync(R.d_meta, R.h_meta.data(), sizeof(MetaItem) * R.nmeta, hipMemcpyHostToDevice, st));
  }
  SK_HIP(hipStreamSynchronize(st));  // the host copies stay valid, but keep the call's effect complete
  return SK_OK;
}

int sketch_batch_info(const sk_batch* B, int32_t* nrounds, int32_t* shape) {
  SK_REQUIRE(B && B->b.magic == 0x534b4254u, SK_ESTATE, "invalid or destroyed batch");
  if (nrounds) *nrounds = (int32_t)B->b.rounds.size();
  if (shape) {
    shape[0] = B->b.cfg.kc;
    shape[1] = B->b.cfg.nw;
    shape[2] = B->b.cfg.nj;
    shape[3] = B->b.cfg.rpl;
  }
  return SK_OK;
}

int sketch_batch_mode(const sk_batch* B, int32_t round, int32_t* mode) {
  SK_REQUIRE(B && B->b.magic == 0x534b4254u, SK_ESTATE, "invalid or destroyed batch");
  const Batch* b = &B->b;
  SK_REQUIRE(round >= 0 && round < (int)b->rounds.size() && mode, SK_EINVAL, "round out of range or mode NULL");
  const BatchRound& R = b->rounds[round];
  *mode = !(b->flags & SK_BATCH_GRAPH) ? SK_ROUND_EAGER
          : R.eager                    ? SK_ROUND_CAPTURE_FAILED
          : R.gexec                    ? SK_ROUND_GRAPH
                                       : SK_ROUND_NOT_CAPTURED;
  return SK_OK;
}

int sketch_batch_destroy(sk_batch* B) {
  SK_REQUIRE(B && B->b.magic == 0x534b4254u, SK_ESTATE, "invalid or destroyed batch");
  Batch* b = &B->b;
  SK_HIP(hipSetDevice(b->ctx->device));
  SK_HIP(hipDeviceSynchronize());
  free_batch_buffers(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  b->ctx->live_handles--;
  b->magic = 0;
  delete B;
  return SK_OK;
}

int sketch_apply_batched(sk_ctx* ctx, const sk_input* ins, const sk_op_desc* op, const int32_t* d, int32_t dd,
                         const uint64_t* seeds, const sk_output* outs, int32_t count, int32_t flags, sk_handle** hs,
                         void* stream) {
  SK_REQUIRE(ctx && ctx->c.magic == CTX_MAGIC, SK_ESTATE, "invalid or released context");
  SK_REQUIRE(op, SK_EINVAL, "operator description is NULL");
  SK_REQUIRE(op->kind == SK_SJLT && op->construction == SK_SJLT_BLOCK, SK_EUNSUPPORTED,
             "the batched sketch uses the SJLT operator with the block construction");
  SK_REQUIRE(op->flags == 0, SK_EINVAL, "flags of the operator description must be 0");
  SK_REQUIRE((flags & ~(SK_BATCH_GRAPH | SK_BATCH_AUTOTUNE)) == 0, SK_EINVAL, "unknown batch flags 0x%x", flags);
  if (hs)
    for (int i = 0; i < count; ++i) hs[i] = nullptr;
  sk_batch* B = nullptr;
  if (int rc = sketch_batch_create(ctx, ins, count, d, dd, op->alpha, seeds, outs, flags, &B, stream)) return rc;
  hipStream_t st = (hipStream_t)stream;
  int rc = sketch_batch_run(B, 0, (int)B->b.rounds.size(), stream);
  // per-matrix handles hold the same operators (blocks of width dd drawn from
  // seeds[i]) with their own bucket tables, as apply(dd) + extend(dd) would
  for (int i = 0; hs && !rc && i < count; ++i) {
    const int nb = d[i] / dd;
    std::vector<int32_t> widths((size_t)nb, dd);
    int kc = 64, kct = 0;
    sjlt_pick_chunks(ins[i].dtype, dd, op->alpha, outs[i].St != nullptr, &kc, &kct);
    rc = make_operator_handle(&ctx->c, SK_SJLT, op->alpha, SK_SJLT_BLOCK, SK_PREC_NATIVE, ins[i].dtype, SK_DENSE,
                              ins[i].n, seeds[i], kc, kct, widths.data(), nb, &hs[i], st);
  }
  const std::string msg = rc ? std::string(sketch_last_error()) : std::string();
  const int rc2 = sketch_batch_destroy(B);  // synchronises the device
  if (rc && hs) {
    for (int i = 0; i < count; ++i)
      if (hs[i]) {
        (void)sketch_release(hs[i]);
        hs[i] = nullptr;
      }
  }
  if (rc) {
    set_error("%s", msg.c_str());
    return rc;
  }
  return rc2;
}

}  // extern "C"

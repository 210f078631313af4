// Library-internal types shared by the ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/sketch.h"
#include "spec.hpp"

namespace sk {

constexpr uint32_t CTX_MAGIC = 0x534b4358u;  // "SKCX"
constexpr uint32_t HND_MAGIC = 0x534b4844u;  // "SKHD"
constexpr int KC_MAX = 256;   // largest chunk of sources of the SJLT bucket tables
constexpr int MAX_PASS_BLOCKS = 16;
constexpr int MAX_PASS_GROUPS = 64;
constexpr int MAX_PASS_COLS = 1024;  // columns of one pass (MAX_PASS_GROUPS groups of 16)

void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

#define SK_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return ::sk::hip_fail(e_, #call); \
  } while (0)

#define SK_REQUIRE(cond, code, ...)  \
  do {                               \
    if (!(cond)) {                   \
      ::sk::set_error(__VA_ARGS__);  \
      return (code);                 \
    }                                \
  } while (0)

struct Block {
  int32_t w = 0;       // width w_b
  int32_t index = 0;   // block number b (counter word of the SJLT hash)
  int64_t col0 = 0;    // first global column c_b
  // SJLT metadata
  uint32_t* codes = nullptr;  // n * alpha: (col << 1) | neg
  int32_t* ptr = nullptr;     // nT * (w + 1): bucket starts, chunk-major (ptr[t * (w + 1) + j])
  int32_t* ent = nullptr;     // nT * kcap: (local source << 1) | neg, sorted by (chunk, col, source)
  int32_t* ptr_t = nullptr;   // the same tables for S' when it uses another chunk size (Handle::kct)
  int32_t* ent_t = nullptr;
  // Gaussian draws of the block: bf16 bits, n x w column-major (k contiguous)
  uint16_t* gbf = nullptr;
  // Gaussian draws as FP64, w x n (row j of R^T contiguous over k) for the FP64 kernel
  double* gf64 = nullptr;
};

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};

struct Ctx {
  uint32_t magic = CTX_MAGIC;
  int device = 0;
  int num_cu = 256;
  int live_handles = 0;
  void* work = nullptr;  // split-K partial sums, grow-only
  size_t work_bytes = 0;
  // launch timing (sketch_profile_*): events recorded around each kernel
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  // autotuner results: shape key -> tuned parameters
  std::map<std::string, std::vector<int>> tune;
  // test hooks (sketch_test_hook): the fail_alloc-th device allocation from
  // now on fails (0: off); graph capture reports failure
  int64_t fail_alloc = 0;
  bool fail_graph = false;
  // allocation-free calls: while use_fixed is set, kernels take their scratch
  // from the library's fixed per-device array (fixed_work, fixed_bytes) and
  // ensure_work never allocates
  void* fixed_work = nullptr;
  size_t fixed_bytes = 0;
  bool use_fixed = false;
};

// the workspace the kernels write (valid after a successful ensure_work)
inline void* work_ptr(const Ctx* c) { return c->use_fixed ? c->fixed_work : c->work; }

// Every device allocation made for a context goes through here (the allocation
// failure hook counts them).  SK_ENOMEM with a message on failure.
int ctx_malloc(Ctx* c, void** p, size_t bytes);

// Brackets one kernel launch with HIP events on its stream when profiling is on.
struct ProfScope {
  Ctx* c;
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(Ctx* c_, const char* n_, hipStream_t s_);
  ~ProfScope();
};

struct Handle {
  uint32_t magic = HND_MAGIC;
  Ctx* ctx = nullptr;
  int32_t kind = 0, alpha = 1, prec = 0, dtype = 0, input = 0;
  int32_t construction = 0;  // SJLT: SK_SJLT_BLOCK or SK_SJLT_GRAPH
  int64_t n = 0;  // rows of R
  int32_t kc = 64;  // SJLT: sources per chunk of the bucket tables
  int32_t kct = 0;  // SJLT: chunk of the S' tables when it differs from kc (0: S' uses the S tables)
  uint64_t seed = 0;
  int32_t d = 0;
  std::vector<Block> blocks;
  // SRHT
  int8_t* srht_D = nullptr;     // n signs (+1 / -1)
  void* srht_Dv = nullptr;      // the same signs as +-1.0 in the element type
  uint32_t* srht_Db = nullptr;  // the same signs as bits (bit k % 32 of word k / 32 set when D_k = -1),
                                // words for roundup(n, 256) sources (zero past n)
  uint32_t* srht_mu = nullptr;  // capacity mu_cap
  int32_t mu_cap = 0;
};

// Pass over a set of consecutive blocks: output column group g (of NJ columns)
// reads block slot grp_blk[g] starting at column grp_col[g] of that block.
struct SjltPass {
  int32_t nT;       // number of source chunks of KC
  int32_t wtot[MAX_PASS_BLOCKS];  // block widths (row length of ptr is w + 1)
  int32_t ngroups;  // W / NJ
  int32_t grp_blk[MAX_PASS_GROUPS];
  int32_t grp_col[MAX_PASS_GROUPS];
  const int32_t* ptr[MAX_PASS_BLOCKS];
  const int32_t* ent[MAX_PASS_BLOCKS];
  int32_t nblk;     // blocks in the pass
  int32_t kcap;     // entry slots of one block per chunk (sjlt_kcap)
  int32_t ms;       // straight-line bucket slots in the LDS-staged gather (4 or 8)
};

// Entry slots reserved per chunk of one block: the chunk's KC * alpha entries,
// rounded up to 256 so that chunk regions start on 1 KB boundaries.
inline int sjlt_kcap(int kc, int alpha, int w) {
  (void)w;
  return (kc * alpha + 255) / 256 * 256;
}

// One SJLT operator block to generate in a batched launch.
struct MetaItem {
  uint32_t* codes;  // n * alpha
  int32_t* ptr;     // nT * (w + 1)
  int32_t* ent;     // nT * kcap
  int64_t n;
  int32_t w, alpha, kc, kcap, block;
  uint32_t k0, k1;  // Philox key of the operator's seed
};

// ---- launchers (each returns SK_OK or an error code after checking the launch)
int launch_sjlt_meta_batch(const MetaItem* items, const int2* chunks, int nchunks, hipStream_t st);
// bucket tables of blocks [b0, b1), as few launches as possible
int launch_sjlt_meta(Handle* h, int b0, int b1, hipStream_t st);
int launch_srht_meta(Handle* h, int64_t j0, int64_t j1, bool draw_D, hipStream_t st);
int launch_gauss_meta(Handle* h, Block& b, hipStream_t st);

// dense SJLT pass over blocks [b0, b1): S (trans = false) or S' (trans = true)
int launch_sjlt_pass(Handle* h, const sk_input* in, int b0, int b1, bool trans, void* out, int64_t ldo,
                     hipStream_t st);
int launch_srht_pass(Handle* h, const sk_input* in, int b0, int b1, bool trans, void* out, int64_t ldo,
                     hipStream_t st);
int launch_gauss_pass(Handle* h, const sk_input* in, int b0, int b1, bool trans, void* out, int64_t ldo,
                      hipStream_t st);
int launch_mf_pass(Handle* h, const sk_input* in, int b0, int b1, void* out, int64_t ldo, hipStream_t st);
int launch_mf_backward(Handle* h, const sk_input* in, int b0, int b1, const float* W, int64_t ldw, float* dX,
                       double* dh, hipStream_t st);
int launch_sjlt_adjoint(Handle* h, const sk_input* in, int b0, int b1, const void* dS, int64_t lddS, void* dA,
                        int64_t lddA, hipStream_t st);
void split_reduce_f32(const float* part, int split, int64_t L, int64_t W, float* out, int64_t ldo, float scale,
                      hipStream_t st);
// out(:, j) = scale * sum_s part[s](:, j) for the split-source partials (L x W each, packed)
void split_reduce_any(int dtype, const void* part, int split, int64_t L, int64_t W, void* out, int64_t ldo,
                      double scale, hipStream_t st);
// SRHT S = A D H P (trans: S' = A^T D H P) with direct-to-LDS loads; returns 1
// when A's alignment rules them out
int launch_srht_dma(Ctx* c, int dtype, bool trans, const void* A, int64_t lda, int64_t L, int64_t K,
                    const uint32_t* Db, const uint32_t* mu, int64_t col0, int W, void* out, int64_t ldo, double scale,
                    hipStream_t st);

int launch_sjlt_dma(Ctx* c, int dtype, int nw, int nj, int rpl, int kc, const void* A, int64_t lda, int64_t L,
                    int64_t K, const SjltPass& pass, void* out, int64_t ldo, double scale, int split, void* part,
                    int gz, hipStream_t st);
size_t dma_lds_bytes(int esz, int kc, int tl, int nblk, int kcap);
int launch_sjlt_dma_t(Ctx* c, int dtype, int nw, int nj, int kc, const void* A, int64_t lda, int64_t L, int64_t K,
                      const SjltPass& pass, void* out, int64_t ldo, double scale, int split, void* part,
                      hipStream_t st);
size_t dma_t_lds_bytes(int esz, int kc, int nblk, int kcap);

int ensure_work(Ctx* c, size_t bytes);
int make_operator_handle(Ctx* c, int kind, int alpha, int construction, int prec, int dtype, int input, int64_t n,
                         uint64_t seed, int kc, int kct, const int32_t* widths, int nb, sk_handle** out,
                         hipStream_t st);
int sjlt_chunk_for(int w, int alpha, int lam);
// chunk sizes of a new dense SJLT operator of width d: for S, and for S'
void sjlt_pick_chunks(int dtype, int d, int alpha, bool want_t, int* kc, int* kct);

}  // namespace sk

struct sk_ctx {
  sk::Ctx c;
};
struct sk_handle {
  sk::Handle h;
};

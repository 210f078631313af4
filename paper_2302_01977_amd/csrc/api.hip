// C ABI: argument checking, handle bookkeeping, device metadata ownership and
// dispatch to the kernel launchers.  Nothing here computes sketch values.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "internal.hpp"

namespace sk {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

int hip_fail(hipError_t e, const char* what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  return SK_EHIP;
}

static hipEvent_t pool_event(Ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(Ctx* c_, const char* n_, hipStream_t s_) : c(c_), name(n_), st(s_) {
  if (!c->prof || c->use_fixed) return;  // (event creation may allocate)
  a = pool_event(c);
  if (a) (void)hipEventRecord(a, st);
}

ProfScope::~ProfScope() {
  if (!a) return;
  hipEvent_t b = pool_event(c);
  if (!b) {
    c->pool.push_back(a);
    return;
  }
  (void)hipEventRecord(b, st);
  c->recs.push_back(ProfRec{name, a, b});
}

int ctx_malloc(Ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (c->fail_alloc > 0 && --c->fail_alloc == 0) {
    set_error("device allocation of %zu bytes failed (injected by the allocation-failure test hook)", bytes);
    return SK_ENOMEM;
  }
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error("device allocation of %zu bytes failed", bytes);
    return SK_ENOMEM;
  }
  return SK_OK;
}

int ensure_work(Ctx* c, size_t bytes) {
  if (c->use_fixed) {
    SK_REQUIRE(bytes <= c->fixed_bytes, SK_EINVAL,
               "this call needs %zu bytes of scratch; the allocation-free entry point has %zu (use sketch_rerun)",
               bytes, c->fixed_bytes);
    return SK_OK;
  }
  if (bytes <= c->work_bytes) return SK_OK;
  if (c->work) {
    SK_HIP(hipFree(c->work));  // implicit device synchronisation: no kernel still reads it
    c->work = nullptr;
    c->work_bytes = 0;
  }
  if (int rc = ctx_malloc(c, &c->work, bytes)) return rc;
  c->work_bytes = bytes;
  return SK_OK;
}

template <typename P>
static int dev_alloc(Ctx* c, P** p, size_t count) {
  *p = nullptr;
  if (count == 0) return SK_OK;
  return ctx_malloc(c, (void**)p, count * sizeof(P));
}

static void free_block(Block& b) {
  if (b.codes) (void)hipFree(b.codes);
  if (b.ptr) (void)hipFree(b.ptr);
  if (b.ent) (void)hipFree(b.ent);
  if (b.ptr_t) (void)hipFree(b.ptr_t);
  if (b.ent_t) (void)hipFree(b.ent_t);
  if (b.gbf) (void)hipFree(b.gbf);
  if (b.gf64) (void)hipFree(b.gf64);
  b = Block();
}

static int check_ctx(const sk_ctx* c) {
  SK_REQUIRE(c && c->c.magic == CTX_MAGIC, SK_ESTATE, "not a live sketch context");
  return SK_OK;
}

static int check_handle(const sk_handle* h) {
  SK_REQUIRE(h && h->h.magic == HND_MAGIC, SK_ESTATE, "not a live sketch handle");
  return SK_OK;
}

// rows of R implied by the input
static int64_t op_rows(const sk_input* in) { return in->input == SK_POINTS ? in->N : in->n; }

static int validate_input(const sk_input* in) {
  SK_REQUIRE(in, SK_EINVAL, "input is NULL");
  if (in->input == SK_DENSE) {
    SK_REQUIRE(in->dtype == SK_F64 || in->dtype == SK_F32, SK_EINVAL, "dtype must be SK_F64 or SK_F32");
    SK_REQUIRE(in->m >= 1 && in->n >= 1, SK_EINVAL, "A must have m >= 1 and n >= 1 (got %lld x %lld)",
               (long long)in->m, (long long)in->n);
    SK_REQUIRE(in->lda >= in->m, SK_EINVAL, "lda (%lld) < m (%lld)", (long long)in->lda, (long long)in->m);
    SK_REQUIRE(in->A, SK_EINVAL, "A is NULL");
    SK_REQUIRE(in->n <= 0x7fffffffLL && in->m <= 0x7fffffffLL, SK_EUNSUPPORTED, "dimensions above 2^31-1");
  } else if (in->input == SK_POINTS) {
    SK_REQUIRE(in->dtype == SK_F32, SK_EINVAL, "point input is FP32");
    SK_REQUIRE(in->N >= 1 && in->N <= 0x7fffffffLL, SK_EINVAL, "N out of range");
    SK_REQUIRE(in->dim >= 1 && in->dim <= 4, SK_EINVAL, "dim must be 1..4");
    SK_REQUIRE(in->X, SK_EINVAL, "X is NULL");
    SK_REQUIRE(in->h > 0.f, SK_EINVAL, "bandwidth h must be > 0");
  } else {
    SK_REQUIRE(false, SK_EINVAL, "unknown input kind %d", in->input);
  }
  return SK_OK;
}

static int validate_out(const sk_input* in, const sk_output* out, bool want_t) {
  SK_REQUIRE(out && out->S, SK_EINVAL, "output S is NULL");
  const int64_t rows = in->input == SK_POINTS ? in->N : in->m;
  SK_REQUIRE(out->ldS >= rows, SK_EINVAL, "ldS (%lld) < rows (%lld)", (long long)out->ldS, (long long)rows);
  if (want_t) {
    SK_REQUIRE(in->input == SK_DENSE, SK_EINVAL, "S' is only defined for stored A");
    SK_REQUIRE(in->m == in->n, SK_EINVAL, "S' = A^T R needs a square A (m == n)");
    SK_REQUIRE(!in->symmetric, SK_EINVAL, "symmetric input: S' equals S, pass St = NULL");
    SK_REQUIRE(out->ldSt >= in->n, SK_EINVAL, "ldSt < n");
  }
  return SK_OK;
}

static int validate_width(const Handle* h, int32_t w) {
  SK_REQUIRE(w >= 1 && w <= 1024, SK_EINVAL, "block width must be in 1..1024 (got %d)", w);
  if (h->kind == SK_SJLT && h->construction == SK_SJLT_GRAPH) {
    SK_REQUIRE(h->alpha <= w, SK_EINVAL, "graph construction: alpha (%d) exceeds the block width (%d)", h->alpha, w);
  } else if (h->kind == SK_SJLT) {
    SK_REQUIRE(w % h->alpha == 0, SK_EINVAL, "alpha (%d) must divide the block width (%d)", h->alpha, w);
  }
  if (h->kind == SK_SJLT || h->kind == SK_SRHT) {
    SK_REQUIRE(w % 16 == 0, SK_EINVAL, "SJLT/SRHT block widths must be multiples of 16 (got %d)", w);
  }
  return SK_OK;
}

static int add_block(Handle* h, int32_t w) {
  Block b;
  b.w = w;
  b.index = (int32_t)h->blocks.size();
  b.col0 = h->d;
  int rc = SK_OK;
  if (h->kind == SK_SJLT) {
    const int64_t nT = (h->n + h->kc - 1) / h->kc;
    if (!rc) rc = dev_alloc(h->ctx, &b.codes, (size_t)h->n * h->alpha);
    if (!rc) rc = dev_alloc(h->ctx, &b.ptr, (size_t)nT * (w + 1));
    if (!rc) rc = dev_alloc(h->ctx, &b.ent, (size_t)nT * sjlt_kcap(h->kc, h->alpha, w));
    if (h->kct) {
      const int64_t nTt = (h->n + h->kct - 1) / h->kct;
      if (!rc) rc = dev_alloc(h->ctx, &b.ptr_t, (size_t)nTt * (w + 1));
      if (!rc) rc = dev_alloc(h->ctx, &b.ent_t, (size_t)nTt * sjlt_kcap(h->kct, h->alpha, w));
    }
  } else if (h->kind == SK_GAUSSIAN) {
    if (!rc) rc = dev_alloc(h->ctx, &b.gbf, (size_t)h->n * w);
  } else if (h->kind == SK_SRHT) {
    if (h->d + w > h->mu_cap) {
      const int cap = std::max<int>(h->d + w, 2 * h->mu_cap);
      uint32_t* nmu = nullptr;
      rc = dev_alloc(h->ctx, &nmu, (size_t)cap);
      if (!rc && h->srht_mu) {
        SK_HIP(hipMemcpy(nmu, h->srht_mu, sizeof(uint32_t) * h->d, hipMemcpyDeviceToDevice));
        (void)hipFree(h->srht_mu);
      }
      if (!rc) {
        h->srht_mu = nmu;
        h->mu_cap = cap;
      }
    }
  }
  if (rc) {
    free_block(b);
    return rc;
  }
  h->blocks.push_back(b);
  h->d += w;
  return SK_OK;
}

// operator metadata of blocks [b0, b1)
static int gen_blocks(Handle* h, int b0, int b1, hipStream_t st) {
  if (h->kind == SK_SJLT) return launch_sjlt_meta(h, b0, b1, st);
  for (int bi = b0; bi < b1; ++bi) {
    Block& b = h->blocks[bi];
    const int rc = h->kind == SK_GAUSSIAN ? launch_gauss_meta(h, b, st)
                                          : launch_srht_meta(h, b.col0, b.col0 + b.w, bi == 0, st);
    if (rc) return rc;
  }
  return SK_OK;
}

static int compute_pass(Handle* h, const sk_input* in, int b0, int b1, const sk_output* out, hipStream_t st) {
  if (in->input == SK_DENSE) {
    auto pass = h->kind == SK_SJLT ? launch_sjlt_pass : h->kind == SK_SRHT ? launch_srht_pass : launch_gauss_pass;
    int rc = pass(h, in, b0, b1, false, out->S, out->ldS, st);
    if (!rc && out->St) rc = pass(h, in, b0, b1, true, out->St, out->ldSt, st);
    return rc;
  }
  return launch_mf_pass(h, in, b0, b1, out->S, out->ldS, st);
}

// split a run of blocks into passes of at most MAX_PASS_BLOCKS blocks and
// MAX_PASS_COLS columns (a single block is at most MAX_PASS_COLS wide)
static int compute_blocks(Handle* h, const sk_input* in, int b0, int b1, const sk_output* out, hipStream_t st) {
  int64_t col = 0;
  const size_t esz = h->dtype == SK_F64 ? 8 : 4;
  int p0 = b0;
  while (p0 < b1) {
    int p1 = p0;
    int64_t w = 0;
    while (p1 < b1 && p1 - p0 < MAX_PASS_BLOCKS && w + h->blocks[p1].w <= MAX_PASS_COLS) w += h->blocks[p1++].w;
    SK_REQUIRE(p1 > p0, SK_EINVAL, "internal: block %d wider than a pass", p0);
    sk_output o = *out;
    o.S = (char*)out->S + (size_t)col * out->ldS * esz;
    if (out->St) o.St = (char*)out->St + (size_t)col * out->ldSt * esz;
    const int rc = compute_pass(h, in, p0, p1, &o, st);
    if (rc) return rc;
    col += w;
    p0 = p1;
  }
  return SK_OK;
}

// undo add_block for blocks [b0, end) after a failed extension: the handle's
// width and block list return to what they were before the call
static void drop_blocks(Handle* h, int b0, int32_t d0, hipStream_t st) {
  (void)hipStreamSynchronize(st);  // launches already queued may read the metadata
  for (int b = (int)h->blocks.size() - 1; b >= b0; --b) free_block(h->blocks[b]);
  h->blocks.resize(b0);
  h->d = d0;
}

// A new handle for an operator with no blocks yet (SRHT sign arrays allocated).
static int new_handle(Ctx* c, int kind, int alpha, int construction, int prec, int dtype, int input, int64_t n,
                      uint64_t seed, int kc, int kct, sk_handle** out) {
  *out = nullptr;
  sk_handle* H = new (std::nothrow) sk_handle;
  SK_REQUIRE(H, SK_ENOMEM, "host allocation failed");
  Handle* h = &H->h;
  h->ctx = c;
  h->kind = kind;
  h->alpha = kind == SK_SJLT ? alpha : 1;
  h->construction = kind == SK_SJLT ? construction : 0;
  h->prec = prec;
  h->dtype = dtype;
  h->input = input;
  h->n = n;
  h->seed = seed;
  h->kc = kc;
  h->kct = kct;
  int rc = SK_OK;
  if (kind == SK_SRHT) {
    rc = dev_alloc(c, &h->srht_D, (size_t)n);
    if (!rc) rc = dev_alloc(c, &h->srht_Db, (size_t)((n + 255) / 256 * 8));
    if (!rc) {
      if (dtype == SK_F64) rc = dev_alloc(c, (double**)&h->srht_Dv, (size_t)n);
      else rc = dev_alloc(c, (float**)&h->srht_Dv, (size_t)n);
    }
  }
  if (rc) {
    if (h->srht_D) (void)hipFree(h->srht_D);
    if (h->srht_Db) (void)hipFree(h->srht_Db);
    h->magic = 0;
    delete H;
    return rc;
  }
  *out = H;
  return SK_OK;
}

// Frees a handle that failed before it was handed out (st: the stream its
// launches went to); keeps the error message of the failure.
static void discard_handle(sk_handle* H, hipStream_t st) {
  const std::string msg = g_err;
  Handle* h = &H->h;
  (void)hipStreamSynchronize(st);
  for (auto& b : h->blocks) free_block(b);
  if (h->srht_D) (void)hipFree(h->srht_D);
  if (h->srht_Dv) (void)hipFree(h->srht_Dv);
  if (h->srht_Db) (void)hipFree(h->srht_Db);
  if (h->srht_mu) (void)hipFree(h->srht_mu);
  h->magic = 0;
  delete H;
  g_err = msg;
}

// A handle holding the operator of blocks of the given widths drawn from
// `seed`, metadata generated on st (nothing computed).  Used by state import
// and by the batched call's per-matrix handles.
int make_operator_handle(Ctx* c, int kind, int alpha, int construction, int prec, int dtype, int input, int64_t n,
                         uint64_t seed, int kc, int kct, const int32_t* widths, int nb, sk_handle** out,
                         hipStream_t st) {
  sk_handle* H = nullptr;
  if (int rc = new_handle(c, kind, alpha, construction, prec, dtype, input, n, seed, kc, kct, &H)) return rc;
  Handle* h = &H->h;
  int rc = SK_OK;
  for (int b = 0; b < nb && !rc; ++b) {
    rc = validate_width(h, widths[b]);
    if (!rc) rc = add_block(h, widths[b]);
  }
  if (!rc) rc = gen_blocks(h, 0, nb, st);
  if (rc) {
    discard_handle(H, st);
    return rc;
  }
  c->live_handles++;
  *out = H;
  return SK_OK;
}

static int check_same_input(const Handle* h, const sk_input* in) {
  SK_REQUIRE(in->input == h->input, SK_EINVAL, "input kind differs from the one the handle was applied to");
  SK_REQUIRE(op_rows(in) == h->n, SK_EINVAL, "input size differs from the handle's operator (n = %lld)",
             (long long)h->n);
  SK_REQUIRE(in->input == SK_POINTS || in->dtype == h->dtype, SK_EINVAL, "dtype differs from the handle's");
  return SK_OK;
}

// Scratch of the allocation-free entry point: a fixed array in device memory,
// one copy per GPU the library runs on, held until the process ends.  Host code
// never uses its name as an address: sketch_init looks up each device's copy
// with hipGetSymbolAddress and the kernels receive that pointer.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[256];  // per device: address of its copy of `scratch`

// Address of this device's copy of the scratch array (the device is current).
static int static_scratch(int device, void** out) {
  SK_REQUIRE(device >= 0 && device < 256, SK_EINVAL, "device index %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return SK_OK;
}

// Fills the whole 160 KB LDS allocation of each workgroup with `pattern`
// (test hook: later kernels on the same CUs start with those bits in LDS).
__global__ void __launch_bounds__(1024) poison_lds_kernel(uint32_t pattern) {
  extern __shared__ uint32_t lds_words[];
  for (int i = threadIdx.x; i < 160 * 1024 / 4; i += blockDim.x) lds_words[i] = pattern;
  __syncthreads();
  asm volatile("" ::: "memory");  // the stores are the point: keep them
}

}  // namespace sk

using namespace sk;

extern "C" {

int sketch_init(sk_ctx** ctx, int32_t device, uint32_t flags) {
  SK_REQUIRE(ctx, SK_EINVAL, "ctx is NULL");
  *ctx = nullptr;
  SK_REQUIRE((flags & ~SK_INIT_PROFILE) == 0, SK_EINVAL, "unknown sketch_init flags 0x%x", flags);
  int count = 0;
  SK_HIP(hipGetDeviceCount(&count));
  SK_REQUIRE(device >= 0 && device < count, SK_EINVAL, "device %d out of range (%d devices)", device, count);
  SK_HIP(hipSetDevice(device));
  hipDeviceProp_t p;
  SK_HIP(hipGetDeviceProperties(&p, device));
  sk_ctx* c = new (std::nothrow) sk_ctx;
  SK_REQUIRE(c, SK_ENOMEM, "host allocation failed");
  c->c.device = device;
  c->c.num_cu = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
  c->c.prof = (flags & SK_INIT_PROFILE) != 0;
  if (int rc = static_scratch(device, &c->c.fixed_work)) {
    c->c.magic = 0;
    delete c;
    return rc;
  }
  c->c.fixed_bytes = STATIC_SCRATCH_BYTES;
  *ctx = c;
  return SK_OK;
}

int sketch_finalize(sk_ctx* ctx) {
  if (int rc = check_ctx(ctx)) return rc;
  SK_REQUIRE(ctx->c.live_handles == 0, SK_ESTATE, "%d handles still live", ctx->c.live_handles);
  SK_HIP(hipDeviceSynchronize());
  if (ctx->c.work) (void)hipFree(ctx->c.work);
  for (auto& r : ctx->c.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->c.pool) (void)hipEventDestroy(e);
  ctx->c.magic = 0;
  delete ctx;
  return SK_OK;
}

const char* sketch_last_error(void) { return g_err.c_str(); }

int sketch_profile_enable(sk_ctx* ctx, int32_t on) {
  if (int rc = check_ctx(ctx)) return rc;
  ctx->c.prof = on != 0;
  return SK_OK;
}

int sketch_profile_read(sk_ctx* ctx, const char* name, double* ms, int64_t* count, int32_t reset) {
  if (int rc = check_ctx(ctx)) return rc;
  SK_REQUIRE(name && ms && count, SK_EINVAL, "NULL argument");
  Ctx* c = &ctx->c;
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : c->recs) {
    if (strcmp(r.name, name) != 0) continue;
    SK_HIP(hipEventSynchronize(r.b));
    float e = 0.f;
    SK_HIP(hipEventElapsedTime(&e, r.a, r.b));
    tot += e;
    ++cnt;
  }
  *ms = tot;
  *count = cnt;
  if (reset) {
    for (auto& r : c->recs) {
      (void)hipEventSynchronize(r.b);
      c->pool.push_back(r.a);
      c->pool.push_back(r.b);
    }
    c->recs.clear();
  }
  return SK_OK;
}

int sketch_apply(sk_ctx* ctx, const sk_input* in, const sk_op_desc* op, int32_t d, uint64_t seed,
                 const sk_output* out, sk_handle** hout, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  SK_REQUIRE(hout, SK_EINVAL, "handle output pointer is NULL");
  *hout = nullptr;
  if (int rc = validate_input(in)) return rc;
  SK_REQUIRE(op, SK_EINVAL, "operator description is NULL");
  SK_REQUIRE(op->kind >= SK_GAUSSIAN && op->kind <= SK_SRHT, SK_EINVAL, "unknown operator kind %d", op->kind);
  SK_REQUIRE(op->flags == 0, SK_EINVAL, "flags must be 0");
  if (op->kind == SK_SJLT) {
    SK_REQUIRE(op->alpha >= 1 && op->alpha <= 32, SK_EINVAL, "alpha must be in 1..32 (got %d)", op->alpha);
    SK_REQUIRE(op->construction == SK_SJLT_BLOCK || op->construction == SK_SJLT_GRAPH, SK_EINVAL,
               "unknown SJLT construction %d", op->construction);
  } else {
    SK_REQUIRE(op->construction == 0, SK_EINVAL, "construction applies to the SJLT operator only");
  }
  if (in->input == SK_POINTS)
    SK_REQUIRE(op->kind == SK_SJLT, SK_EUNSUPPORTED, "the matrix-free kernel sketch uses the SJLT operator");
  SK_REQUIRE(op->prec >= SK_PREC_NATIVE && op->prec <= SK_PREC_BF16X3, SK_EINVAL, "unknown precision %d", op->prec);
  if (op->kind == SK_GAUSSIAN && op->prec != SK_PREC_NATIVE)
    SK_REQUIRE(in->dtype == SK_F32, SK_EINVAL, "bf16 Gaussian arithmetic needs FP32 A");
  if (int rc = validate_out(in, out, out && out->St)) return rc;
  SK_HIP(hipSetDevice(ctx->c.device));

  hipStream_t st = (hipStream_t)stream;
  int kc = 64, kct = 0;
  if (op->kind == SK_SJLT) {
    if (in->input == SK_DENSE) sjlt_pick_chunks(in->dtype, d, op->alpha, out && out->St, &kc, &kct);
    else kc = sjlt_chunk_for(d, op->alpha, 4);
  }
  sk_handle* H = nullptr;
  if (int rc = new_handle(&ctx->c, op->kind, op->alpha, op->construction, op->prec, in->dtype, in->input,
                          op_rows(in), seed, kc, kct, &H))
    return rc;
  Handle* h = &H->h;
  int rc = validate_width(h, d);
  if (!rc) rc = add_block(h, d);
  if (!rc) rc = gen_blocks(h, 0, 1, st);
  if (!rc) rc = compute_blocks(h, in, 0, 1, out, st);
  if (rc) {
    discard_handle(H, st);
    return rc;
  }
  ctx->c.live_handles++;
  *hout = H;
  return SK_OK;
}

int sketch_extend(sk_handle* H, const sk_input* in, int32_t dd, int32_t nblocks, const sk_output* out_new,
                  void* stream) {
  if (int rc = check_handle(H)) return rc;
  Handle* h = &H->h;
  if (int rc = validate_input(in)) return rc;
  if (int rc = check_same_input(h, in)) return rc;
  SK_REQUIRE(nblocks >= 1 && nblocks <= 64, SK_EINVAL, "nblocks must be in 1..64");
  if (int rc = validate_width(h, dd)) return rc;
  if (int rc = validate_out(in, out_new, out_new && out_new->St)) return rc;
  SK_REQUIRE((int64_t)h->d + (int64_t)dd * nblocks <= 0x7fffffffLL, SK_EINVAL, "total width above 2^31-1");
  SK_HIP(hipSetDevice(h->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int b0 = (int)h->blocks.size();
  const int32_t d0 = h->d;
  int rc = SK_OK;
  for (int i = 0; i < nblocks && !rc; ++i) rc = add_block(h, dd);
  if (!rc) rc = gen_blocks(h, b0, b0 + nblocks, st);
  if (!rc) rc = compute_blocks(h, in, b0, b0 + nblocks, out_new, st);
  if (rc) {
    const std::string msg = g_err;
    drop_blocks(h, b0, d0, st);
    g_err = msg;
  }
  return rc;
}

int sketch_rerun(sk_handle* H, const sk_input* in, uint64_t seed, const sk_output* out, void* stream) {
  if (int rc = check_handle(H)) return rc;
  Handle* h = &H->h;
  if (int rc = validate_input(in)) return rc;
  if (int rc = check_same_input(h, in)) return rc;
  if (int rc = validate_out(in, out, out && out->St)) return rc;
  SK_HIP(hipSetDevice(h->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  h->seed = seed;
  if (int rc = gen_blocks(h, 0, (int)h->blocks.size(), st)) return rc;
  return compute_blocks(h, in, 0, (int)h->blocks.size(), out, st);
}

int sketch_rerun_static(sk_handle* H, const sk_input* in, uint64_t seed, const sk_output* out, void* stream) {
  if (int rc = check_handle(H)) return rc;
  Handle* h = &H->h;
  if (int rc = validate_input(in)) return rc;
  if (int rc = check_same_input(h, in)) return rc;
  if (int rc = validate_out(in, out, out && out->St)) return rc;
  Ctx* c = h->ctx;
  SK_REQUIRE(c->fixed_work, SK_ESTATE, "the context has no scratch array");
  SK_HIP(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const uint64_t seed0 = h->seed;
  const int nb = (int)h->blocks.size();
  c->use_fixed = true;
  h->seed = seed;
  int rc = gen_blocks(h, 0, nb, st);
  if (!rc) rc = compute_blocks(h, in, 0, nb, out, st);
  if (rc) {  // the handle keeps its previous operator
    const std::string msg = g_err;
    h->seed = seed0;
    (void)gen_blocks(h, 0, nb, st);
    g_err = msg;
  }
  c->use_fixed = false;
  return rc;
}

int sketch_adjoint(sk_handle* H, const sk_input* in, int32_t block0, int32_t nblocks, const void* dS, int64_t lddS,
                   void* dA, int64_t lddA, float* dX, double* dh, void* stream) {
  if (int rc = check_handle(H)) return rc;
  Handle* h = &H->h;
  if (int rc = validate_input(in)) return rc;
  if (int rc = check_same_input(h, in)) return rc;
  SK_REQUIRE(nblocks >= 1 && block0 >= 0 && block0 + nblocks <= (int)h->blocks.size(), SK_EINVAL,
             "block range [%d, %d) outside the operator's %d blocks", block0, block0 + nblocks,
             (int)h->blocks.size());
  SK_REQUIRE(dS, SK_EINVAL, "dS is NULL");
  const int64_t rows = in->input == SK_POINTS ? in->N : in->m;
  SK_REQUIRE(lddS >= rows, SK_EINVAL, "lddS < rows");
  SK_HIP(hipSetDevice(h->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (in->input == SK_DENSE) {
    SK_REQUIRE(dA && lddA >= in->m, SK_EINVAL, "dA is NULL or lddA < m");
    return launch_sjlt_adjoint(h, in, block0, block0 + nblocks, dS, lddS, dA, lddA, st);
  }
  SK_REQUIRE(dX && dh, SK_EINVAL, "dX and dh are required for point input");
  return launch_mf_backward(h, in, block0, block0 + nblocks, (const float*)dS, lddS, dX, dh, st);
}

int sketch_width(const sk_handle* H, int32_t* d, int32_t* nblocks) {
  if (int rc = check_handle(H)) return rc;
  if (d) *d = H->h.d;
  if (nblocks) *nblocks = (int32_t)H->h.blocks.size();
  return SK_OK;
}

int sketch_release(sk_handle* H) {
  if (int rc = check_handle(H)) return rc;
  Handle* h = &H->h;
  SK_HIP(hipSetDevice(h->ctx->device));
  SK_HIP(hipDeviceSynchronize());
  for (auto& b : h->blocks) free_block(b);
  if (h->srht_D) (void)hipFree(h->srht_D);
  if (h->srht_Dv) (void)hipFree(h->srht_Dv);
  if (h->srht_Db) (void)hipFree(h->srht_Db);
  if (h->srht_mu) (void)hipFree(h->srht_mu);
  h->ctx->live_handles--;
  h->magic = 0;
  delete H;
  return SK_OK;
}

int sketch_get_rows(const sk_handle* H, int64_t i0, int64_t i1, int64_t j0, int64_t j1, double* out, int64_t ldo) {
  if (int rc = check_handle(H)) return rc;
  const Handle* h = &H->h;
  SK_REQUIRE(0 <= i0 && i0 <= i1 && i1 <= h->n, SK_EINVAL, "row range out of bounds");
  SK_REQUIRE(0 <= j0 && j0 <= j1 && j1 <= h->d, SK_EINVAL, "column range out of bounds");
  SK_REQUIRE(out || i1 == i0 || j1 == j0, SK_EINVAL, "out is NULL");
  SK_REQUIRE(ldo >= i1 - i0, SK_EINVAL, "ldo too small");
  const Key key = key_of(h->seed);
  for (int64_t j = j0; j < j1; ++j) {
    int b = 0;
    while (b + 1 < (int)h->blocks.size() && h->blocks[b + 1].col0 <= j) ++b;
    const Block& B = h->blocks[b];
    const int jj = (int)(j - B.col0);
    double* o = out + (j - j0) * ldo;
    if (h->kind == SK_SJLT && h->construction == SK_SJLT_GRAPH) {
      const double s = 1.0 / sqrt((double)h->alpha);
      uint32_t codes[32];
      for (int64_t i = i0; i < i1; ++i) {
        sjlt_graph_codes(key, (uint32_t)B.index, (uint32_t)i, h->alpha, (uint32_t)B.w, codes);
        double v = 0.0;
        for (int c = 0; c < h->alpha; ++c)
          if ((int)(codes[c] >> 1) == jj) v = (codes[c] & 1u) ? -s : s;
        o[i - i0] = v;
      }
    } else if (h->kind == SK_SJLT) {
      const uint32_t wc = (uint32_t)(B.w / h->alpha);
      const uint32_t c = (uint32_t)jj / wc;
      const double s = 1.0 / sqrt((double)h->alpha);
      for (int64_t i = i0; i < i1; ++i) {
        const uint32_t code = sjlt_code(key, (uint32_t)B.index, (uint32_t)i, c, wc);
        o[i - i0] = ((int)(code >> 1) == jj) ? ((code & 1u) ? -s : s) : 0.0;
      }
    } else if (h->kind == SK_GAUSSIAN) {
      const double sw = sqrt((double)B.w);
      for (int64_t i = i0; i < i1; ++i) o[i - i0] = gauss_raw(key, (uint32_t)i, (uint32_t)j) / sw;
    } else {
      const uint32_t mu = srht_mu(key, (uint32_t)j, srht_nu(h->n));
      const double s = 1.0 / sqrt((double)B.w);
      for (int64_t i = i0; i < i1; ++i) {
        const int neg = srht_neg(key, (uint32_t)i) ^ (popc32((uint32_t)i & mu) & 1);
        o[i - i0] = neg ? -s : s;
      }
    }
  }
  return SK_OK;
}

int sketch_get_sjlt(const sk_handle* H, int32_t block, uint32_t* codes) {
  if (int rc = check_handle(H)) return rc;
  const Handle* h = &H->h;
  SK_REQUIRE(h->kind == SK_SJLT, SK_EINVAL, "handle is not an SJLT operator");
  SK_REQUIRE(block >= 0 && block < (int)h->blocks.size(), SK_EINVAL, "block out of range");
  SK_REQUIRE(codes, SK_EINVAL, "codes is NULL");
  SK_HIP(hipSetDevice(h->ctx->device));
  SK_HIP(hipDeviceSynchronize());
  SK_HIP(hipMemcpy(codes, h->blocks[block].codes, sizeof(uint32_t) * h->n * h->alpha, hipMemcpyDeviceToHost));
  return SK_OK;
}

int sketch_get_srht(const sk_handle* H, int8_t* D, uint32_t* mu, int32_t j0, int32_t j1) {
  if (int rc = check_handle(H)) return rc;
  const Handle* h = &H->h;
  SK_REQUIRE(h->kind == SK_SRHT, SK_EINVAL, "handle is not an SRHT operator");
  SK_REQUIRE(0 <= j0 && j0 <= j1 && j1 <= h->d, SK_EINVAL, "column range out of bounds");
  SK_HIP(hipSetDevice(h->ctx->device));
  SK_HIP(hipDeviceSynchronize());
  if (D) SK_HIP(hipMemcpy(D, h->srht_D, (size_t)h->n, hipMemcpyDeviceToHost));
  if (mu && j1 > j0) SK_HIP(hipMemcpy(mu, h->srht_mu + j0, sizeof(uint32_t) * (j1 - j0), hipMemcpyDeviceToHost));
  return SK_OK;
}

int sketch_get_gaussian(const sk_handle* H, int32_t block, uint16_t* bits) {
  if (int rc = check_handle(H)) return rc;
  const Handle* h = &H->h;
  SK_REQUIRE(h->kind == SK_GAUSSIAN, SK_EINVAL, "handle is not a Gaussian operator");
  SK_REQUIRE(block >= 0 && block < (int)h->blocks.size(), SK_EINVAL, "block out of range");
  SK_REQUIRE(bits, SK_EINVAL, "bits is NULL");
  SK_HIP(hipSetDevice(h->ctx->device));
  SK_HIP(hipDeviceSynchronize());
  SK_HIP(hipMemcpy(bits, h->blocks[block].gbf, sizeof(uint16_t) * h->n * h->blocks[block].w,
                   hipMemcpyDeviceToHost));
  return SK_OK;
}

int sketch_test_hook(sk_ctx* ctx, int32_t hook, int64_t arg) {
  if (int rc = check_ctx(ctx)) return rc;
  if (hook == SK_HOOK_FAIL_ALLOC) {
    SK_REQUIRE(arg >= 0, SK_EINVAL, "allocation countdown must be >= 0");
    ctx->c.fail_alloc = arg;
  } else if (hook == SK_HOOK_FAIL_GRAPH) {
    ctx->c.fail_graph = arg != 0;
  } else {
    SK_REQUIRE(false, SK_EINVAL, "unknown test hook %d", hook);
  }
  return SK_OK;
}

int sketch_test_poison_lds(sk_ctx* ctx, uint32_t pattern, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  SK_HIP(hipSetDevice(ctx->c.device));
  static bool attr_set = false;
  if (!attr_set) {
    SK_HIP(hipFuncSetAttribute((const void*)poison_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024));
    attr_set = true;
  }
  poison_lds_kernel<<<4 * ctx->c.num_cu, 1024, 160 * 1024, (hipStream_t)stream>>>(pattern);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// ---- operator state: the handle's operator is a pure function of these fields
// (Algorithm 1's JL-Operator(d, n) per block, drawn from the seed), so the
// state is a few hundred bytes and import regenerates every block's metadata.
namespace {
constexpr uint32_t STATE_MAGIC = 0x54534b53u;  // "SKST"
constexpr uint32_t STATE_VERSION = 1;
struct StateHead {
  uint32_t magic, version;
  int32_t kind, alpha, construction, prec, dtype, input;
  int64_t n;
  uint64_t seed;
  int32_t kc, kct, nblocks, d;
};
static_assert(sizeof(StateHead) == 64, "state header layout: the block widths follow at byte 64");
uint64_t fnv1a(const unsigned char* p, size_t len) {
  uint64_t x = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < len; ++i) x = (x ^ p[i]) * 0x100000001b3ull;
  return x;
}
}  // namespace

int sketch_state_export(const sk_handle* H, void* buf, size_t* len) {
  if (int rc = check_handle(H)) return rc;
  SK_REQUIRE(len, SK_EINVAL, "len is NULL");
  const Handle* h = &H->h;
  const size_t need = sizeof(StateHead) + sizeof(int32_t) * h->blocks.size() + sizeof(uint64_t);
  if (!buf) {
    *len = need;
    return SK_OK;
  }
  SK_REQUIRE(*len >= need, SK_EINVAL, "buffer of %zu bytes, %zu needed", *len, need);
  StateHead hd;
  memset(&hd, 0, sizeof(hd));
  hd.magic = STATE_MAGIC;
  hd.version = STATE_VERSION;
  hd.kind = h->kind;
  hd.alpha = h->alpha;
  hd.construction = h->construction;
  hd.prec = h->prec;
  hd.dtype = h->dtype;
  hd.input = h->input;
  hd.n = h->n;
  hd.seed = h->seed;
  hd.kc = h->kc;
  hd.kct = h->kct;
  hd.nblocks = (int32_t)h->blocks.size();
  hd.d = h->d;
  unsigned char* p = (unsigned char*)buf;
  memcpy(p, &hd, sizeof(hd));
  for (size_t b = 0; b < h->blocks.size(); ++b)
    memcpy(p + sizeof(hd) + sizeof(int32_t) * b, &h->blocks[b].w, sizeof(int32_t));
  const uint64_t sum = fnv1a(p, need - sizeof(uint64_t));
  memcpy(p + need - sizeof(uint64_t), &sum, sizeof(sum));
  *len = need;
  return SK_OK;
}

int sketch_state_import(sk_ctx* ctx, const void* buf, size_t len, sk_handle** out) {
  if (int rc = check_ctx(ctx)) return rc;
  SK_REQUIRE(buf && out, SK_EINVAL, "NULL argument");
  *out = nullptr;
  SK_REQUIRE(len >= sizeof(StateHead) + sizeof(uint64_t), SK_EINVAL, "state too short (%zu bytes)", len);
  StateHead hd;
  memcpy(&hd, buf, sizeof(hd));
  SK_REQUIRE(hd.magic == STATE_MAGIC, SK_EINVAL, "not a sketch operator state");
  SK_REQUIRE(hd.version == STATE_VERSION, SK_EINVAL, "state version %u, expected %u", hd.version, STATE_VERSION);
  SK_REQUIRE(hd.nblocks >= 1 && hd.nblocks <= (1 << 20), SK_EINVAL, "state holds %d blocks", hd.nblocks);
  const size_t need = sizeof(StateHead) + sizeof(int32_t) * (size_t)hd.nblocks + sizeof(uint64_t);
  SK_REQUIRE(len == need, SK_EINVAL, "state of %zu bytes, %zu expected for %d blocks", len, need, hd.nblocks);
  const unsigned char* p = (const unsigned char*)buf;
  uint64_t sum;
  memcpy(&sum, p + need - sizeof(uint64_t), sizeof(sum));
  SK_REQUIRE(sum == fnv1a(p, need - sizeof(uint64_t)), SK_EINVAL, "state checksum mismatch (corrupted)");
  SK_REQUIRE(hd.kind >= SK_GAUSSIAN && hd.kind <= SK_SRHT, SK_EINVAL, "state: unknown kind %d", hd.kind);
  SK_REQUIRE(hd.input == SK_DENSE || hd.input == SK_POINTS, SK_EINVAL, "state: unknown input kind");
  SK_REQUIRE(hd.dtype == SK_F64 || hd.dtype == SK_F32, SK_EINVAL, "state: unknown dtype");
  SK_REQUIRE(hd.prec >= SK_PREC_NATIVE && hd.prec <= SK_PREC_BF16X3, SK_EINVAL, "state: unknown precision");
  SK_REQUIRE(hd.n >= 1 && hd.n <= 0x7fffffffLL, SK_EINVAL, "state: n out of range");
  if (hd.kind == SK_SJLT) {
    SK_REQUIRE(hd.alpha >= 1 && hd.alpha <= 32, SK_EINVAL, "state: alpha out of range");
    SK_REQUIRE(hd.construction == SK_SJLT_BLOCK || hd.construction == SK_SJLT_GRAPH, SK_EINVAL,
               "state: unknown construction");
    SK_REQUIRE(hd.kc == 64 || hd.kc == 128 || hd.kc == 256, SK_EINVAL, "state: chunk %d", hd.kc);
    SK_REQUIRE(hd.kct == 0 || hd.kct == 64 || hd.kct == 128 || hd.kct == 256, SK_EINVAL, "state: chunk %d", hd.kct);
  }
  std::vector<int32_t> widths((size_t)hd.nblocks);
  memcpy(widths.data(), p + sizeof(hd), sizeof(int32_t) * widths.size());
  int64_t d = 0;
  for (int32_t w : widths) d += w;
  SK_REQUIRE(d == hd.d, SK_EINVAL, "state: block widths sum to %lld, not %d", (long long)d, hd.d);
  SK_HIP(hipSetDevice(ctx->c.device));
  // metadata generated on the null stream, then waited for: the call returns a
  // handle whose device data is complete
  if (int rc = make_operator_handle(&ctx->c, hd.kind, hd.alpha, hd.construction, hd.prec, hd.dtype, hd.input, hd.n,
                                    hd.seed, hd.kc, hd.kct, widths.data(), hd.nblocks, out, nullptr))
    return rc;
  SK_HIP(hipStreamSynchronize(nullptr));
  return SK_OK;
}

}  // extern "C"

// Gaussian sketch S = A R_b on the matrix cores (section 2.4.1: R_b has i.i.d.
// N(0, 1/w_b) entries; the product is a dense contraction, O(m n w) flops).
// The draws g are stored on the bfloat16 grid, column-major; the 1/sqrt(w_b)
// scale is applied to the result.
//
// gauss_f64_kernel: v_mfma_f64_16x16x4_f64.  A workgroup of 4 waves owns 64 rows
//   and a slice of the source range (split so that two workgroups fit per CU);
//   wave q computes rows 16q..16q+15 against up to 256 columns.  A fragments are
//   read straight from global memory (16 consecutive rows per column, coalesced);
//   the R chunk (16 k x W, exact in FP64) is staged once per workgroup in LDS.
//   FP32 inputs are promoted on load, so this is also the FP64 reference for FP32 A.
// gauss_bf16_kernel: v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  The 16x32
//   A fragment needs 8 consecutive k per row while A is column-major, so each
//   128 x 32 step of A is loaded in 4x4 blocks, rounded to bf16 (and, for
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
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    gauss_f64_kernel(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n, const uint16_t* __restrict__ g,
                     int64_t ldg, int W, TS* __restrict__ S, int64_t ldS, double scale, int split,
                     TS* __restrict__ part) {
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

  // the draws (bf16 bits) and the A fragments of chunk k0 + KT are loaded while
  // chunk k0 is multiplied
  uint16_t rb[KS];
  TA ar[4];
  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int64_t k = k0 + sk0 + u;
      rb[u] = (sj < wloc && k < n) ? g[k + (int64_t)(jbase + sj) * ldg] : (uint16_t)0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * s + lk;
      ar[s] = (arow < m && k < n) ? aelem<TRANS>(A, lda, arow, k) : TA(0);
    }
  };
  // this workgroup's slice of the source range, in whole chunks
  const int64_t nK = (n + KT - 1) / KT;
  const int64_t kb = nK * blockIdx.y / split * KT, ke = std::min<int64_t>(n, nK * (blockIdx.y + 1) / split * KT);
  if (kb < ke) load_chunk(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += KT) {
    double af[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) af[s] = (double)ar[s];
    __syncthreads();  // previous chunk consumed
#pragma unroll
    for (int u = 0; u < KS; ++u) Rl[(sk0 + u) * WP + sj] = bf16_bits_to_double(rb[u]);
    __syncthreads();
    if (k0 + KT < ke) load_chunk(k0 + KT);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const double b = Rl[(4 * s + lk) * WP + cb * 16 + lr];
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s], b, acc[cb], 0, 0, 0);
      }
      // one k-step of R fragments in flight at a time (keeps two waves per SIMD)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  TS* dst = split > 1 ? part + (int64_t)blockIdx.y * m * W : S;
  const int64_t ldd = split > 1 ? m : ldS;
  const double sc = split > 1 ? 1.0 : scale;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int j = jbase + cb * 16 + lr;
    if (j >= W) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // v_mfma_f64_16x16x4f64 returns D[4 v + lane / 16][lane % 16] in item v
      const int64_t r = row0 + 4 * v + lk;
      if (r < m) dst[r + (int64_t)j * ldd] = (TS)(acc[cb][v] * sc);
    }
  }
}

// ------------------------------------------------------------------- BF16
// A workgroup of 4 waves owns 128 rows of the result and up to 256 of its
// columns; wave q computes rows 32 q .. 32 q + 31 (two 16-row blocks, so every R
// fragment read from LDS feeds two MFMAs per part).  The source range is walked
// in steps of 32 (one MFMA depth) and split across workgroups (partial sums
// reduced in a fixed order) so that the row tiles fill the chip and the slice of
// R that one workgroup reads fits an XCD's L2: workgroups are dealt to the 8 XCDs
// in turn, so the launch gives every source slice its own XCDs and R is read
// from HBM about once per XCD.  Step kt + 1 of A and R is loaded into registers
// while step kt is multiplied.
struct Bf16Grid {
  int64_t tiles;  // row tiles x column slices
  int gz;         // column slices
  int split;      // source slices
  int xcd;        // 1: source slice s runs on XCDs [s 8 / split, (s + 1) 8 / split)
};

template <int NB, bool X3, bool TRANS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    gauss_bf16_kernel(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                      const uint16_t* __restrict__ g, int64_t ldg, int W, float* __restrict__ S, int64_t ldS,
                      float scale, Bf16Grid gr, float* __restrict__ part) {
  constexpr int KT = 32;
  constexpr int RS = KT + 8;  // padded LDS row (bf16 elements): 80 bytes, conflict-free 16-byte reads
  constexpr int MR = 128;
  constexpr int NP = X3 ? 3 : 1;
  constexpr int WP = NB * 16;
  constexpr int NPIECE = WP * KT / 8;  // 16-byte pieces of the R step
  constexpr int RV = (NPIECE + 255) / 256;
  __shared__ __attribute__((aligned(16))) __bf16 At[NP][MR * RS];
  __shared__ __attribute__((aligned(16))) __bf16 Rt[WP * RS];
  // work item of this workgroup
  const int64_t lin = blockIdx.x;
  int64_t tile;
  int s;
  if (gr.xcd) {
    const int per = 8 / gr.split;  // XCDs per source slice
    const int x = (int)(lin & 7);
    s = x / per;
    tile = (x % per) + per * (lin >> 3);
  } else {
    s = (int)(lin / gr.tiles);
    tile = lin % gr.tiles;
  }
  if (tile >= gr.tiles) return;  // whole workgroup: no barrier is reached
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int q = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t row0 = (tile / gr.gz) * MR;
  const int jbase = (int)(tile % gr.gz) * WP;
  const int wloc = std::min(WP, W - jbase);
  const int64_t nK = (n + KT - 1) / KT;
  const int64_t kt0 = nK * s / gr.split, kt1 = nK * (s + 1) / gr.split;
  const bool g16 = (ldg & 7) == 0 && ((uintptr_t)g & 15) == 0;  // R pieces are 16-byte aligned

  // staging roles.  S: a 4 x 4 block (rows 4 rg.., sources 4 kg..) transposed in
  // registers.  S' (A^T): piece p = 256 u + tid is row p / 8 (a column of A),
  // sources 4 (p mod 8) .. + 3: eight lanes read one column's 128 contiguous
  // bytes, so a wave instruction covers 8 whole 128-byte segments.
  // S places the 16-byte source units of an LDS row XOR-swizzled by row / 16
  // (measured, paired: n = 32768, w = 64: 1.42 -> 1.22 ms; at w = 256 the
  // plain layout is faster, 0.62 against 0.65 ms, and is kept there).
  auto swz = [](int row) -> int { return (TRANS || NB > 8) ? 0 : (row >> 4) & 3; };
  const int rg = tid & 31, kg = tid >> 5;

  float areg[4][4];
  uint32_t rreg[RV][4];

  auto load_step = [&](int64_t kt) {
    const int64_t k0 = kt * KT;
    if (!TRANS) {
      const int64_t r = row0 + 4 * rg;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t k = k0 + 4 * kg + c;
        const float* p = A + r + k * lda;
        if (k < n && r + 4 <= m) {
          __builtin_memcpy(areg[c], p, 16);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) areg[c][e] = (k < n && r + e < m) ? p[e] : 0.f;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int pc = u * 256 + tid;
        const int64_t r = row0 + (pc >> 3);
        const int64_t k = k0 + 4 * (pc & 7);
        const float* p = A + k + r * lda;
        if (r < m && k + 4 <= n) {
          __builtin_memcpy(areg[u], p, 16);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) areg[u][e] = (r < m && k + e < n) ? p[e] : 0.f;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < RV; ++u) {
      const int pid = u * 256 + tid;
      const int j = pid >> 2, kk = (pid & 3) * 8;
      const int64_t k = k0 + kk;
      const uint16_t* p = g + k + (int64_t)(jbase + j) * ldg;
      if (pid < NPIECE && j < wloc && g16 && k + 8 <= n) {
        __builtin_memcpy(rreg[u], p, 16);
      } else {
        uint16_t hv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[e] = (pid < NPIECE && j < wloc && k + e < n) ? p[e] : (uint16_t)0;
        __builtin_memcpy(rreg[u], hv, 16);
      }
    }
  };

  auto split_store = [&](const float (&x)[4], int off) {
    __bf16 p1[4], p2[4], p3[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const __bf16 h1 = (__bf16)x[e];
      p1[e] = h1;
      if (X3) {
        const float r1 = x[e] - (float)h1;
        const __bf16 h2 = (__bf16)r1;
        p2[e] = h2;
        p3[e] = (__bf16)(r1 - (float)h2);
      }
    }
    __builtin_memcpy(&At[0][off], p1, 8);
    if (X3) {
      __builtin_memcpy(&At[1 % NP][off], p2, 8);
      __builtin_memcpy(&At[2 % NP][off], p3, 8);
    }
  };

  f4 acc[2][NB];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};

  if (kt0 < kt1) load_step(kt0);
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    __syncthreads();  // the previous step's fragments are read
    if (!TRANS) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float x[4] = {areg[0][r], areg[1][r], areg[2][r], areg[3][r]};
        // 16-byte unit kg / 2 of row 4 rg + r at unit (kg / 2) ^ swz(row): the
        // rows of one store are 4 apart, and without the swizzle 8 lanes would
        // share each bank
        const int row = 4 * rg + r;
        split_store(x, row * RS + 8 * ((kg >> 1) ^ swz(row)) + 4 * (kg & 1));
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int pc = u * 256 + tid;
        split_store(areg[u], (pc >> 3) * RS + 4 * (pc & 7));
      }
    }
#pragma unroll
    for (int u = 0; u < RV; ++u) {
      const int pid = u * 256 + tid;
      if (pid < NPIECE) __builtin_memcpy(&Rt[(pid >> 2) * RS + (pid & 3) * 8], rreg[u], 16);
    }
    if (kt + 1 < kt1) load_step(kt + 1);
    __syncthreads();
    bf8 af[2][NP];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int row = 32 * q + 16 * rb + lr;
        __builtin_memcpy(&af[rb][p], &At[p][row * RS + 8 * (lk ^ swz(row))], 16);
      }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      bf8 bfr;
      __builtin_memcpy(&bfr, &Rt[(cb * 16 + lr) * RS + 8 * lk], 16);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int p = NP - 1; p >= 0; --p)  // small parts first
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[rb][p], bfr, acc[rb][cb], 0, 0, 0);
    }
  }
  float* dst = gr.split > 1 ? part + (int64_t)s * m * W : S;
  const int64_t ldd = gr.split > 1 ? m : ldS;
  const float sc = gr.split > 1 ? 1.f : scale;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int j = jbase + cb * 16 + lr;
    if (j >= W) continue;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // v_mfma_f32_16x16x32_bf16 returns D[4 (lane / 16) + v][lane % 16] in item v
        const int64_t r = row0 + 32 * q + 16 * rb + 4 * lk + v;
        if (r < m) dst[r + (int64_t)j * ldd] = acc[rb][cb][v] * sc;
      }
  }
}

// S = A R in BF16 / bf16x3 with A and R moved by direct-to-LDS loads into rings
// of stages (A: three 32-deep steps, R: two), so that two steps of A are in
// flight while one is multiplied, with no prefetch registers and one barrier
// per step.  Full tiles only (rows, sources and columns multiples of the tile;
// A, its columns and the draws 16-byte aligned); other shapes take the
// register-staged kernel above.  The A fragments are built in registers from
// the raw FP32 stage (rounded / split there), so no converted copy is stored.
// Raw A stage: 32 source columns of 512 bytes (128 rows); the 16-byte unit of
// rows 4u..4u+3 of source k sits at unit u ^ 4 ((k / 8) mod 4), which makes the
// fragment reads (16 rows x 4 source groups per wave instruction) conflict-free.
// R stage: column j's 64 bytes with unit q at q ^ ((j / 4) mod 4).
// S' (A^T) stage: 128 columns of A, 128 bytes (32 sources) each, the 16-byte
// piece p of column c at slot p ^ ((c / 2) mod 8).
template <int NB, bool X3, bool TRANS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    gauss_bf16_dma_kernel(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                          const uint16_t* __restrict__ g, int64_t ldg, int W, float* __restrict__ S, int64_t ldS,
                          float scale, Bf16Grid gr, float* __restrict__ part) {
  constexpr int KT = 32;
  constexpr int MR = 128;
  constexpr int NP = X3 ? 3 : 1;
  constexpr int WP = NB * 16;
  constexpr int ABYTES = MR * KT * 4;   // raw A stage
  constexpr int RBYTES = WP * KT * 2;   // R stage
  constexpr int NA = 3, NR = 2;         // ring depths
  constexpr int AUNITS = ABYTES / 1024;
  constexpr int RUNITS = RBYTES / 1024;
  static_assert(AUNITS % 4 == 0 && RBYTES % 1024 == 0, "whole KB per stage");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __attribute__((address_space(3))) char* const smem3 = (__attribute__((address_space(3))) char*)smem;

  const int64_t lin = blockIdx.x;
  int64_t tile;
  int s;
  {
    const int per = 8 / gr.split;
    const int x = (int)(lin & 7);
    s = x / per;
    tile = (x % per) + per * (lin >> 3);
  }
  if (tile >= gr.tiles) return;  // whole workgroup: no barrier is reached
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t row0 = (tile / gr.gz) * MR;
  const int jbase = (int)(tile % gr.gz) * WP;
  const int64_t nK = n / KT;
  const int64_t kt0 = nK * s / gr.split, kt1 = nK * (s + 1) / gr.split;

  // step kt of A into ring slot kt % NA.  S: unit u holds source columns 2u and
  // 2u + 1; S': unit u holds columns 8u .. 8u + 7 of A
  auto issue_a = [&](int64_t kt) {
    char* const dst = (char*)smem3 + (int)(kt % NA) * ABYTES;
#pragma unroll
    for (int i = 0; i < AUNITS / 4; ++i) {
      const int u = wave + 4 * i;
      const float* gp;
      if constexpr (!TRANS) {
        const int k = 2 * u + (lane >> 5);                  // source column within the step
        const int ur = (lane & 31) ^ (4 * ((k >> 3) & 3));  // unit of rows held by this lane's slot
        gp = A + (row0 + 4 * ur) + (kt * KT + k) * lda;
      } else {
        const int c = 8 * u + (lane >> 3);                  // column of A (row of S')
        const int pc = (lane & 7) ^ ((c >> 1) & 7);         // 16-byte piece held by this lane's slot
        gp = A + (kt * KT + 4 * pc) + (row0 + c) * lda;
      }
      __builtin_amdgcn_global_load_lds((void*)gp, (__attribute__((address_space(3))) void*)(dst + u * 1024), 16, 0,
                                       0);
    }
  };
  // step kt of R into ring slot kt % NR: unit u holds columns 16u .. 16u + 15
  auto issue_r = [&](int64_t kt) {
    char* const dst = (char*)smem3 + NA * ABYTES + (int)(kt % NR) * RBYTES;
    for (int u = wave; u < RUNITS; u += 4) {
      const int j = 16 * u + (lane >> 2);
      const int kq = (lane & 3) ^ ((j >> 2) & 3);
      const uint16_t* gp = g + (kt * KT + 8 * kq) + (int64_t)(jbase + j) * ldg;
      __builtin_amdgcn_global_load_lds((void*)gp, (__attribute__((address_space(3))) void*)(dst + u * 1024), 16, 0,
                                       0);
    }
  };

  f4 acc[2][NB];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};

  // issue order keeps "everything but the last 4 instructions of this wave"
  // equal to "steps up to t complete" at the top of step t: A(t+1) is always the
  // last thing issued before step t begins, and it is 4 instructions per wave
  if (kt0 < kt1) {
    issue_a(kt0);
    issue_r(kt0);
    if (kt0 + 1 < kt1) issue_a(kt0 + 1);
  }
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    if (kt + 1 < kt1) __builtin_amdgcn_s_waitcnt(0xF74);  // vmcnt(4): A(kt + 1) may stay in flight
    else __builtin_amdgcn_s_waitcnt(0xF70);               // vmcnt(0)
    __builtin_amdgcn_s_barrier();  // every wave's loads of step kt landed; step kt - 1 is consumed
    if (kt + 1 < kt1) issue_r(kt + 1);
    if (kt + 2 < kt1) issue_a(kt + 2);
    const char* const as = smem + (int)(kt % NA) * ABYTES;
    const char* const rs = smem + NA * ABYTES + (int)(kt % NR) * RBYTES;
    bf8 af[2][NP];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int r = 32 * wave + 16 * rb + lr;
      float x[8];
      if constexpr (!TRANS) {
        const int pos = ((((r >> 2) ^ (4 * lk)) << 2) | (r & 3)) * 4;  // byte position in a source column
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = *(const float*)(as + (8 * lk + e) * 512 + pos);
      } else {
        const int f = (r >> 1) & 7;
        __builtin_memcpy(&x[0], as + r * 128 + 16 * ((2 * lk) ^ f), 16);
        __builtin_memcpy(&x[4], as + r * 128 + 16 * ((2 * lk + 1) ^ f), 16);
      }
      __bf16 p1[8], p2[8], p3[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const __bf16 h1 = (__bf16)x[e];
        p1[e] = h1;
        if (X3) {
          const float r1 = x[e] - (float)h1;
          const __bf16 h2 = (__bf16)r1;
          p2[e] = h2;
          p3[e] = (__bf16)(r1 - (float)h2);
        }
      }
      __builtin_memcpy(&af[rb][0], p1, 16);
      if (X3) {
        __builtin_memcpy(&af[rb][1 % NP], p2, 16);
        __builtin_memcpy(&af[rb][2 % NP], p3, 16);
      }
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      bf8 bfr;
      __builtin_memcpy(&bfr, rs + (cb * 16 + lr) * 64 + 16 * (lk ^ ((lr >> 2) & 3)), 16);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int p = NP - 1; p >= 0; --p)  // small parts first
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[rb][p], bfr, acc[rb][cb], 0, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's reads of the stages are done
  }
  float* dst = gr.split > 1 ? part + (int64_t)s * m * W : S;
  const int64_t ldd = gr.split > 1 ? m : ldS;
  const float sc = gr.split > 1 ? 1.f : scale;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int j = jbase + cb * 16 + lr;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // v_mfma_f32_16x16x32_bf16 returns D[4 (lane / 16) + v][lane % 16] in item v
        const int64_t r = row0 + 32 * wave + 16 * rb + 4 * lk + v;
        dst[r + (int64_t)j * ldd] = acc[rb][cb][v] * sc;
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
  // about two workgroups per CU (two waves per SIMD): split the source range
  // when the row tiles are fewer, at least 8 chunks per slice
  const int64_t tiles = ((m + 63) / 64) * gz;
  const int64_t nK = (n + 15) / 16;
  int split = 1;
  if (tiles < 2 * (int64_t)c->num_cu)
    split = (int)std::max<int64_t>(1, std::min<int64_t>((2 * c->num_cu + tiles - 1) / tiles, nK / 8));
  TS* part = nullptr;
  if (split > 1) {
    const int rc = ensure_work(c, (size_t)split * (size_t)m * (size_t)W * sizeof(TS));
    if (rc) return rc;
    part = (TS*)work_ptr(c);
  }
  dim3 grid((unsigned)((m + 63) / 64), (unsigned)split, (unsigned)gz);
  {
    ProfScope ps(c, TRANS ? "gauss_f64_t" : "gauss_f64", st);
#define SK_F64_CASE(NB_)                                                                                       \
  if (nbk == NB_)                                                                                              \
    gauss_f64_kernel<TA, TS, TRANS, NB_><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale, split, part);
    SK_F64_CASE(2) SK_F64_CASE(4) SK_F64_CASE(8) SK_F64_CASE(16)
#undef SK_F64_CASE
    SK_HIP(hipGetLastError());
  }
  if (split > 1) {
    ProfScope ps(c, "gauss_reduce", st);
    split_reduce_any(sizeof(TS) == 8 ? SK_F64 : SK_F32, part, split, m, W, S, ldS, scale, st);
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

template <bool TRANS>
static int run_bf16(Ctx* c, bool x3, const float* A, int64_t lda, int64_t m, int64_t n, const uint16_t* g, int W,
                    float* S, int64_t ldS, float scale, hipStream_t st) {
  const int nb = std::min(16, (W + 15) / 16);
  const int nbk = nb <= 2 ? 2 : nb <= 4 ? 4 : nb <= 8 ? 8 : 16;
  Bf16Grid gr;
  gr.gz = (W + nbk * 16 - 1) / (nbk * 16);
  gr.tiles = ((m + 127) / 128) * gr.gz;
  // source slices: enough for about two workgroups per CU, and for the slice of
  // R (n x W bf16) read on one XCD to take at most half of its 4 MB L2; a power
  // of two up to 8 (then each slice owns whole XCDs), at least 8 steps each
  const int64_t nK = (n + 31) / 32;
  const double rbytes = 2.0 * (double)n * (double)std::min(W, nbk * 16);
  int split = 1;
  while (split < 8 && (gr.tiles * split < 2 * (int64_t)c->num_cu || rbytes / split > 2.0 * 1024 * 1024) &&
         nK / (2 * split) >= 8)
    split *= 2;
  gr.split = split;
  gr.xcd = 1;
  float* part = nullptr;
  if (split > 1) {
    const int rc = ensure_work(c, (size_t)split * (size_t)m * (size_t)W * sizeof(float));
    if (rc) return rc;
    part = (float*)work_ptr(c);
  }
  // XCD-major order: 8 / split XCDs per source slice, row tiles dealt over them
  const int per = 8 / split;
  const int64_t nblk = 8 * ((gr.tiles + per - 1) / per);
  dim3 grid((unsigned)nblk);
  // full tiles with 16-byte aligned A columns and draws: the direct-to-LDS kernel
  const int WPk = nbk * 16;
  const bool dma = m % 128 == 0 && n % 32 == 0 && W % WPk == 0 && (lda * 4) % 16 == 0 &&
                   (uintptr_t)A % 16 == 0 && (uintptr_t)g % 16 == 0;
  if (dma) {
    const size_t shmem = 3 * (size_t)128 * 32 * 4 + 2 * (size_t)WPk * 32 * 2;
    ProfScope ps(c, x3 ? (TRANS ? "gauss_bf16x3_t" : "gauss_bf16x3") : (TRANS ? "gauss_bf16_t" : "gauss_bf16"), st);
#define SK_BFD_CASE(NB_)                                                                                      \
  if (nbk == NB_) {                                                                                           \
    auto kern = x3 ? gauss_bf16_dma_kernel<NB_, true, TRANS> : gauss_bf16_dma_kernel<NB_, false, TRANS>;     \
    static bool attr_set[2] = {false, false};                                                                 \
    if (!attr_set[x3]) {                                                                                      \
      SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024)); \
      attr_set[x3] = true;                                                                                    \
    }                                                                                                         \
    kern<<<grid, 256, shmem, st>>>(A, lda, m, n, g, n, W, S, ldS, scale, gr, part);                           \
  }
    SK_BFD_CASE(2) SK_BFD_CASE(4) SK_BFD_CASE(8) SK_BFD_CASE(16)
#undef SK_BFD_CASE
    SK_HIP(hipGetLastError());
  } else {
    ProfScope ps(c, x3 ? (TRANS ? "gauss_bf16x3_t" : "gauss_bf16x3") : (TRANS ? "gauss_bf16_t" : "gauss_bf16"), st);
#define SK_BF_CASE(NB_)                                                                                       \
  if (nbk == NB_) {                                                                                           \
    if (x3)                                                                                                   \
      gauss_bf16_kernel<NB_, true, TRANS><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale, gr, part); \
    else                                                                                                      \
      gauss_bf16_kernel<NB_, false, TRANS><<<grid, 256, 0, st>>>(A, lda, m, n, g, n, W, S, ldS, scale, gr, part); \
  }
    SK_BF_CASE(2) SK_BF_CASE(4) SK_BF_CASE(8) SK_BF_CASE(16)
#undef SK_BF_CASE
    SK_HIP(hipGetLastError());
  }

  if (split > 1) {
    ProfScope ps(c, "gauss_reduce", st);
    split_reduce_any(SK_F32, part, split, m, W, S, ldS, (double)scale, st);
    SK_HIP(hipGetLastError());
  }
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

// Grid-sized complex FP64 GEMMs on the matrix cores (v_mfma_f64_16x16x4_f64),
// complex products by three real MFMAs (Gauss's 3M form).
//
//  * zgemm_nn: C[b] = A[b] * op(B[b]) with A (M x K, c128, small, L2-resident)
//    and B (K x N) / C (M x N) long row-major panels over the grid (N = N_g).
//    Used for Gamma^n = Psi^n conj(psi^n) and for the fit solve xi = S^+ Z.
//    Operand fragments are read straight from global memory (no LDS): a lane
//    loads one complex of a 16-column B strip, so each 16-lane group reads a
//    contiguous 256-byte segment.
//  * The workgroup order is XCD-aware: hardware deals workgroups round robin
//    over the 8 XCDs; remapping gives every XCD a contiguous range of tiles,
//    so the row tiles that share one B column strip run on the same XCD and
//    reuse it from that XCD's L2.
#include "common.h"

namespace exx {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NXCD = 8;

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// logical tile index from the hardware workgroup id (XCD-contiguous ranges)
__device__ __forceinline__ long xcd_remap(long bid, long total_padded) {
  const long per = total_padded / NXCD;
  return (bid % NXCD) * per + bid / NXCD;
}

// Wave tile: WM x WN blocks of 16x16; workgroup = 2 x 2 waves.
// ACC = 0: C = A op(B); ACC = +1 / -1: C = C +/- A op(B) (arithmetic in FP64).
template <typename TB, typename TC, int WM, int WN, int CONJB, int ACC, int LOWER>
__global__ __launch_bounds__(256) void zgemm_nn_mfma(int M, int N, int K, int nrt, long ntiles,
                                                     long ntiles_pad, const double2* __restrict__ A,
                                                     long lda, long sA,
                                                     const cplx<TB>* __restrict__ B, long ldb,
                                                     long sB, cplx<TC>* __restrict__ C, long ldc,
                                                     long sC) {
  const long t = xcd_remap(blockIdx.x, ntiles_pad);
  if (t >= ntiles) return;
  const int rt = (int)(t % nrt);
  const long ct = t / nrt;
  const long b = blockIdx.y;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = rt * (2 * WM * 16) + (wave & 1) * (WM * 16);
  const long col0 = ct * (2 * WN * 16) + (wave >> 1) * (WN * 16);
  // LOWER: A is lower triangular, so this wave's rows need k < row0 + WM * 16
  // (skipping the blocks above the diagonal within that range was measured
  // slower here: the branches cost more than the three-product MFMAs they save)
  const int Kb = LOWER ? min(K, row0 + WM * 16) : K;

  // Gauss's three-product form of the complex product: T1 = Re A Re B,
  // T2 = Im A Im B, T3 = (Re A + Im A)(Re B + Im B); then Re C = T1 - T2 and
  // Im C = T3 - T1 - T2. Three real MFMAs per complex k-step instead of four.
  d4 t1[WM][WN], t2[WM][WN], t3[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      t1[i][j] = d4{0, 0, 0, 0};
      t2[i][j] = d4{0, 0, 0, 0};
      t3[i][j] = d4{0, 0, 0, 0};
    }

  // NPF-deep register pipeline: slot s holds the fragments of k-step s (mod NPF).
  // Loads are unconditional with indices clamped into the operands: rows past M
  // and columns past N only feed outputs that are never stored, and k past K is
  // zeroed on the A side when the slot is consumed. With no branch or select
  // between a load and its use, the wait before each k-step covers only that
  // slot's loads. B fragments stay in their storage type until consumed.
  constexpr int NPF = 3;
  double2 fa[NPF][WM];
  cplx<TB> fb[NPF][WN];
  // 32-bit element offsets from the uniform operand bases (the launcher checks
  // that they fit), so the loads use a scalar base plus a vector offset
  unsigned aoff[WM], boff[WN];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    const int r = row0 + i * 16 + li;
    aoff[i] = (unsigned)((r < M ? r : M - 1) * lda);
  }
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long c = col0 + j * 16 + li;
    boff[j] = (unsigned)(c < N ? c : N - 1);
  }
  const unsigned ldb32 = (unsigned)ldb;
  auto load = [&](int k0, double2* xa, cplx<TB>* xb) {
    const int k = k0 + lk;
    const unsigned kc = (unsigned)(k < K ? k : K - 1);
#pragma unroll
    for (int i = 0; i < WM; ++i) xa[i] = A[aoff[i] + kc];
#pragma unroll
    for (int j = 0; j < WN; ++j) xb[j] = B[kc * ldb32 + boff[j]];
  };
#pragma unroll
  for (int s = 0; s < NPF; ++s) load(4 * s, fa[s], fb[s]);
  // let the first loads land before the loop, so that the wait counts at the
  // loop head see only the loop's own refills (the differently ordered prologue
  // otherwise forces a full wait there on every iteration)
  __builtin_amdgcn_s_waitcnt(0);
  const int niter = (Kb + 4 * NPF - 1) / (4 * NPF);
  for (int it = 0; it < niter; ++it) {
#pragma unroll
    for (int s = 0; s < NPF; ++s) {
      const bool kin = 4 * (it * NPF + s) + lk < Kb;
      double br[WN], bi[WN], bs[WN];
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        br[j] = (double)fb[s][j].x;
        bi[j] = CONJB ? -(double)fb[s][j].y : (double)fb[s][j].y;
        bs[j] = br[j] + bi[j];
      }
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const double ar = kin ? fa[s][i].x : 0.0, ai = kin ? fa[s][i].y : 0.0;
        const double as = ar + ai;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          t1[i][j] = mfma64(ar, br[j], t1[i][j]);
          t2[i][j] = mfma64(ai, bi[j], t2[i][j]);
          t3[i][j] = mfma64(as, bs[j], t3[i][j]);
        }
      }
      // refill the slot with k-step (it + 1) * NPF + s (masked at use past K). The
      // scheduling barriers keep the refill after this slot's MFMAs, so it lands
      // in the same registers and the loop carries no copies.
      __builtin_amdgcn_sched_barrier(0);
      load(4 * ((it + 1) * NPF + s), fa[s], fb[s]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // D layout of v_mfma_f64_16x16x4_f64: register v of a lane holds row
  // 4*v + lane/16, column lane%16 of the 16x16 block.
  // Combining T1..T3 needs the accumulators in VALU registers. Each lane
  // round-trips its own values through this wave's LDS slice (the LDS write
  // takes matrix registers directly, and LDS accesses of one wave complete in
  // order); arithmetic on the accumulators themselves makes the compiler carry
  // them in VALU registers and copy them in and out of the matrix registers on
  // every iteration.
  __shared__ double stage[4][3][64 * 4];
  typedef __attribute__((address_space(3))) volatile double lds_f64;
  lds_f64* s1 = (lds_f64*)stage[wave][0];
  lds_f64* s2 = (lds_f64*)stage[wave][1];
  lds_f64* s3 = (lds_f64*)stage[wave][2];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        s1[v * 64 + lane] = t1[i][j][v];
        s2[v * 64 + lane] = t2[i][j][v];
        s3[v * 64 + lane] = t3[i][j][v];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double x1 = s1[v * 64 + lane], x2 = s2[v * 64 + lane], x3 = s3[v * 64 + lane];
        double xr = x1 - x2, xi = x3 - x1 - x2;
        const int r = row0 + i * 16 + 4 * v + lk;
        const long c = col0 + j * 16 + li;
        if (r < M && c < N) {
          if constexpr (ACC != 0) {
            const cplx<TC> o = C[(long)r * ldc + c];
            xr = (double)o.x + ACC * xr;
            xi = (double)o.y + ACC * xi;
          }
          C[(long)r * ldc + c] = mk<TC>((TC)xr, (TC)xi);
        }
      }
    }
}

// FP32 matrix-core form for FP32 storage: C = A op(B) with A (c128) rounded to
// FP32 at load, v_mfma_f32_16x16x4_f32, FP32 accumulation (the products of
// the FP32 build path; K is short there). Same tiling, pipeline and workgroup
// order as zgemm_nn_mfma. D layout: register v of a lane holds row
// 4*(lane/16) + v, column lane%16 of the 16x16 block.
typedef float f4 __attribute__((ext_vector_type(4)));

template <int WM, int WN, int CONJB>
__global__ __launch_bounds__(256) void cgemm_nn_mfma32(int M, int N, int K, int nrt, long ntiles,
                                                       long ntiles_pad,
                                                       const double2* __restrict__ A, long lda,
                                                       long sA, const float2* __restrict__ B,
                                                       long ldb, long sB, float2* __restrict__ C,
                                                       long ldc, long sC) {
  const long t = xcd_remap(blockIdx.x, ntiles_pad);
  if (t >= ntiles) return;
  const int rt = (int)(t % nrt);
  const long ct = t / nrt;
  const long b = blockIdx.y;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = rt * (2 * WM * 16) + (wave & 1) * (WM * 16);
  const long col0 = ct * (2 * WN * 16) + (wave >> 1) * (WN * 16);
  f4 are[WM][WN], aim[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      are[i][j] = f4{0, 0, 0, 0};
      aim[i][j] = f4{0, 0, 0, 0};
    }
  constexpr int NPF = 3;
  double2 fa[NPF][WM];
  float2 fb[NPF][WN];
  // 32-bit element offsets from the uniform operand bases (the launcher checks
  // that they fit), so the loads use a scalar base plus a vector offset
  unsigned aoff[WM], boff[WN];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    const int r = row0 + i * 16 + li;
    aoff[i] = (unsigned)((r < M ? r : M - 1) * lda);
  }
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long c = col0 + j * 16 + li;
    boff[j] = (unsigned)(c < N ? c : N - 1);
  }
  const unsigned ldb32 = (unsigned)ldb;
  auto load = [&](int k0, double2* xa, float2* xb) {
    const int k = k0 + lk;
    const unsigned kc = (unsigned)(k < K ? k : K - 1);
#pragma unroll
    for (int i = 0; i < WM; ++i) xa[i] = A[aoff[i] + kc];
#pragma unroll
    for (int j = 0; j < WN; ++j) xb[j] = B[kc * ldb32 + boff[j]];
  };
#pragma unroll
  for (int s = 0; s < NPF; ++s) load(4 * s, fa[s], fb[s]);
  __builtin_amdgcn_s_waitcnt(0);  // as in zgemm_nn_mfma
  const int niter = (K + 4 * NPF - 1) / (4 * NPF);
  for (int it = 0; it < niter; ++it) {
#pragma unroll
    for (int s = 0; s < NPF; ++s) {
      const bool kin = 4 * (it * NPF + s) + lk < K;
      float br[WN], bi[WN];
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        br[j] = fb[s][j].x;
        bi[j] = CONJB ? -fb[s][j].y : fb[s][j].y;
      }
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const float ar = kin ? (float)fa[s][i].x : 0.f, ai = kin ? (float)fa[s][i].y : 0.f;
        const float nai = -ai;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          are[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br[j], are[i][j], 0, 0, 0);
          are[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai, bi[j], are[i][j], 0, 0, 0);
          aim[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi[j], aim[i][j], 0, 0, 0);
          aim[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br[j], aim[i][j], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      load(4 * ((it + 1) * NPF + s), fa[s], fb[s]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + i * 16 + 4 * lk + v;
      if (r >= M) continue;
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const long c = col0 + j * 16 + li;
        if (c < N) C[(long)r * ldc + c] = make_float2(are[i][j][v], aim[i][j][v]);
      }
    }
}

// Real form for the fit solve of meshes whose transfers are all self-conjugate:
// C[b] = Re(A[b]) B[b] with A (M x K) stored complex (its imaginary part is
// zero there) and real B (K x N, storage TB) and C (M x N, storage TC). One
// FP64 MFMA per block and k-step. Wave tile 4 x 4 blocks (64 x 64); the four
// waves of a workgroup take consecutive column strips of one 64-row band, so
// they share the A rows through L1. Same register pipeline as zgemm_nn_mfma.
// LOWER: A is lower triangular (zero above its diagonal), so the band of rows
// [r0, r0 + 64) stops its k loop at r0 + 64 and skips the 16-row blocks that a
// k-step cannot reach (above the diagonal, or past M).
// ACC = 0: C = A B; ACC = +1 / -1: C = C +/- A B (sum formed in FP64).
template <typename TB, typename TC, int LOWER, int ACC = 0>
__global__ __launch_bounds__(256) void dgemm_nn_mfma(int M, int N, int K, int nrt, long ntiles,
                                                     long ntiles_pad, const double2* __restrict__ A,
                                                     long lda, long sA, const TB* __restrict__ B,
                                                     long ldb, long sB, TC* __restrict__ C,
                                                     long ldc, long sC) {
  constexpr int WM = 4, WN = 4;
  const long t = xcd_remap(blockIdx.x, ntiles_pad);
  if (t >= ntiles) return;
  const int rt = (int)(t % nrt);
  const long ct = t / nrt;
  const long b = blockIdx.y;
  const double* Ar = (const double*)(A + b * sA);  // real parts at even offsets
  B += b * sB;
  C += b * sC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = rt * (WM * 16);
  const long col0 = ct * (4 * WN * 16) + wave * (WN * 16);
  const int Kb = LOWER ? min(K, row0 + WM * 16) : K;
  d4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = d4{0, 0, 0, 0};
  constexpr int NPF = 3;
  double fa[NPF][WM];
  TB fb[NPF][WN];
  unsigned aoff[WM], boff[WN];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    const int r = row0 + i * 16 + li;
    aoff[i] = (unsigned)(2 * (r < M ? r : M - 1) * lda);
  }
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long c = col0 + j * 16 + li;
    boff[j] = (unsigned)(c < N ? c : N - 1);
  }
  const unsigned ldb32 = (unsigned)ldb;
  // 32-bit byte offsets from the uniform bases (the launcher checks that the
  // bytes of one batch item's operands fit), so the loads take a scalar base
  // plus a vector offset
  const char* Ab = (const char*)Ar;
  const char* Bb = (const char*)B;
  auto load = [&](int k0, double* xa, TB* xb) {
    const int k = k0 + lk;
    const unsigned kc = (unsigned)(k < K ? k : K - 1);
#pragma unroll
    for (int i = 0; i < WM; ++i) xa[i] = *(const double*)(Ab + (aoff[i] + 2 * kc) * 8u);
#pragma unroll
    for (int j = 0; j < WN; ++j)
      xb[j] = *(const TB*)(Bb + (kc * ldb32 + boff[j]) * (unsigned)sizeof(TB));
  };
#pragma unroll
  for (int s = 0; s < NPF; ++s) load(4 * s, fa[s], fb[s]);
  __builtin_amdgcn_s_waitcnt(0);  // as in zgemm_nn_mfma
  const int niter = (Kb + 4 * NPF - 1) / (4 * NPF);
  for (int it = 0; it < niter; ++it) {
#pragma unroll
    for (int s = 0; s < NPF; ++s) {
      const bool kin = 4 * (it * NPF + s) + lk < Kb;
      double bv[WN];
#pragma unroll
      for (int j = 0; j < WN; ++j) bv[j] = (double)fb[s][j];
      const int kb = 4 * (it * NPF + s);  // this k-step's first column (wave-uniform)
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        // LOWER: a row block past M, or one whose rows all lie above this
        // k-step's columns, contributes nothing; its MFMAs are skipped by a
        // wave-uniform branch (the full product keeps its branch-free loop)
        const int rb = row0 + i * 16;
        if (LOWER && (rb >= M || kb > rb + 15)) continue;
        const double av = kin ? fa[s][i] : 0.0;
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = mfma64(av, bv[j], acc[i][j]);
      }
      __builtin_amdgcn_sched_barrier(0);
      load(4 * ((it + 1) * NPF + s), fa[s], fb[s]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // register v of a lane holds row 4 v + lane/16, column lane%16 of a block;
  // stored through this wave's LDS slice (see zgemm_nn_mfma)
  __shared__ double stage[4][64 * 4];
  typedef __attribute__((address_space(3))) volatile double lds_f64;
  lds_f64* sv = (lds_f64*)stage[wave];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) sv[v * 64 + lane] = acc[i][j][v];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double x = sv[v * 64 + lane];
        const int r = row0 + i * 16 + 4 * v + lk;
        const long c = col0 + j * 16 + li;
        if (r < M && c < N) {
          TC* dst = C + (long)r * ldc + c;
          *dst = ACC ? (TC)((double)*dst + (double)ACC * x) : (TC)x;
        }
      }
    }
}

template <typename TB, typename TC, int WM, int WN, int CONJB, int ACC = 0, int LOWER = 0>
hipError_t run_nn(int M, int N, int K, int batch, const void* A, long lda, long sA, const void* B,
                  long ldb, long sB, void* C, long ldc, long sC, hipStream_t st) {
  const int nrt = (M + 2 * WM * 16 - 1) / (2 * WM * 16);
  const long nct = ((long)N + 2 * WN * 16 - 1) / (2 * WN * 16);
  const long ntiles = nrt * nct;
  const long pad = (ntiles + NXCD - 1) / NXCD * NXCD;
  hipLaunchKernelGGL((zgemm_nn_mfma<TB, TC, WM, WN, CONJB, ACC, LOWER>), dim3((unsigned)pad, batch),
                     dim3(256),
                     0, st, M, N, K, nrt, ntiles, pad, (const double2*)A, lda, sA,
                     (const cplx<TB>*)B, ldb, sB, (cplx<TC>*)C, ldc, sC);
  return hipGetLastError();
}

template <typename TB, typename TC, int CONJB, int LOWER>
hipError_t run_nn_tile(int tile, int M, int N, int K, int batch, const void* A, long lda, long sA,
                       const void* B, long ldb, long sB, void* C, long ldc, long sC,
                       hipStream_t st) {
  switch (tile) {
    case 22:
      return run_nn<TB, TC, 2, 2, CONJB, 0, LOWER>(M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc,
                                                   sC, st);
    case 42:
      return run_nn<TB, TC, 4, 2, CONJB, 0, LOWER>(M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc,
                                                   sC, st);
    default:
      return run_nn<TB, TC, 2, 4, CONJB, 0, LOWER>(M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc,
                                                   sC, st);
  }
}

// operand offsets of one batch item must fit the kernels' 32-bit arithmetic
bool offsets_fit(int M, int N, int K, long lda, long ldb) {
  if (K <= 0) return false;
  const long lim = 0x7fffffffL;
  return (long)M * lda < lim && (long)K * ldb < lim && (long)N <= ldb;
}

}  // namespace

template <typename TB, typename TC>
hipError_t zgemm_nn_grid(int M, int N, int K, int batch, const void* A, long lda, long sA,
                         bool conjB, const void* B, long ldb, long sB, void* C, long ldc, long sC,
                         hipStream_t st, int tile, bool lower) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (!offsets_fit(M, N, K, lda, ldb)) return hipErrorInvalidValue;
  if (conjB && lower) return hipErrorInvalidValue;  // not instantiated
  if (conjB)
    return run_nn_tile<TB, TC, 1, 0>(tile, M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc, sC, st);
  if (lower)
    return run_nn_tile<TB, TC, 0, 1>(tile, M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc, sC, st);
  return run_nn_tile<TB, TC, 0, 0>(tile, M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc, sC, st);
}

namespace {
typedef __bf16 gb_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short gb_u16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ gb_bf16x8 gb_as_bf16(gb_u16x8 v) {
  gb_bf16x8 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

// BF16 matrix-core form of cgemm_nn_mfma32 with conj(B): v_mfma_f32_16x16x32_bf16,
// a k-step of 32 with lane group lk = lane/16 holding k = 8 lk .. 8 lk + 7 of its
// row of A and column of B (the same pairing on both operands), operands
// rounded to bfloat16 at load, FP32 accumulation. Wave tile WM x WN blocks,
// workgroup 2 x 2 waves, XCD-contiguous tile order as zgemm_nn_mfma.
template <int WM, int WN>
__global__ __launch_bounds__(256) void cgemm_nn_bf16(int M, int N, int K, int nrt, long ntiles,
                                                     long ntiles_pad,
                                                     const double2* __restrict__ A, long lda,
                                                     long sA, const float2* __restrict__ B,
                                                     long ldb, long sB, float2* __restrict__ C,
                                                     long ldc, long sC) {
  const long t = xcd_remap(blockIdx.x, ntiles_pad);
  if (t >= ntiles) return;
  const int rt = (int)(t % nrt);
  const long ct = t / nrt;
  const long b = blockIdx.y;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = rt * (2 * WM * 16) + (wave & 1) * (WM * 16);
  const long col0 = ct * (2 * WN * 16) + (wave >> 1) * (WN * 16);
  f4 are[WM][WN], aim[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) are[i][j] = aim[i][j] = f4{0, 0, 0, 0};
  long arow[WM], bcol[WN];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    const int r = row0 + i * 16 + li;
    arow[i] = (long)(r < M ? r : M - 1) * lda;
  }
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long c = col0 + j * 16 + li;
    bcol[j] = c < N ? c : N - 1;
  }
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int kb = k0 + 8 * lk;
    gb_u16x8 br[WN], bi[WN];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = min(kb + e, K - 1);  // the A side is zero past K
        const float2 v = B[(long)k * ldb + bcol[j]];
        br[j][e] = bf16_rne(v.x);
        bi[j][e] = bf16_rne(v.y);
      }
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      gb_u16x8 ar, ai, nar;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = kb + e;
        const double2 v = k < K ? A[arow[i] + k] : make_double2(0.0, 0.0);
        ar[e] = bf16_rne((float)v.x);
        ai[e] = bf16_rne((float)v.y);
        nar[e] = ar[e] ^ 0x8000u;
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        // C = A conj(B): Re += ar br + ai bi, Im += ai br - ar bi
        are[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gb_as_bf16(ar), gb_as_bf16(br[j]),
                                                            are[i][j], 0, 0, 0);
        are[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gb_as_bf16(ai), gb_as_bf16(bi[j]),
                                                            are[i][j], 0, 0, 0);
        aim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gb_as_bf16(ai), gb_as_bf16(br[j]),
                                                            aim[i][j], 0, 0, 0);
        aim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gb_as_bf16(nar), gb_as_bf16(bi[j]),
                                                            aim[i][j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + i * 16 + 4 * lk + v;
      if (r >= M) continue;
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const long c = col0 + j * 16 + li;
        if (c < N) C[(long)r * ldc + c] = make_float2(are[i][j][v], aim[i][j][v]);
      }
    }
}
}  // namespace

hipError_t cgemm_nn_grid_bf16(int M, int N, int K, int batch, const void* A, long lda, long sA,
                              const void* B, long ldb, long sB, void* C, long ldc, long sC,
                              hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (!offsets_fit(M, N, K, lda, ldb)) return hipErrorInvalidValue;
  constexpr int WM = 2, WN = 2;
  const int nrt = (M + 2 * WM * 16 - 1) / (2 * WM * 16);
  const long nct = ((long)N + 2 * WN * 16 - 1) / (2 * WN * 16);
  const long ntiles = nrt * nct;
  const long pad = (ntiles + NXCD - 1) / NXCD * NXCD;
  hipLaunchKernelGGL((cgemm_nn_bf16<WM, WN>), dim3((unsigned)pad, batch), dim3(256), 0, st, M, N,
                     K, nrt, ntiles, pad, (const double2*)A, lda, sA, (const float2*)B, ldb, sB,
                     (float2*)C, ldc, sC);
  return hipGetLastError();
}

hipError_t cgemm_nn_grid32(int M, int N, int K, int batch, const void* A, long lda, long sA,
                          bool conjB, const void* B, long ldb, long sB, void* C, long ldc, long sC,
                          hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (!offsets_fit(M, N, K, lda, ldb)) return hipErrorInvalidValue;
  constexpr int WM = 2, WN = 2;
  const int nrt = (M + 2 * WM * 16 - 1) / (2 * WM * 16);
  const long nct = ((long)N + 2 * WN * 16 - 1) / (2 * WN * 16);
  const long ntiles = nrt * nct;
  const long pad = (ntiles + NXCD - 1) / NXCD * NXCD;
  if (conjB)
    hipLaunchKernelGGL((cgemm_nn_mfma32<WM, WN, 1>), dim3((unsigned)pad, batch), dim3(256), 0, st, M,
                       N, K, nrt, ntiles, pad, (const double2*)A, lda, sA, (const float2*)B, ldb,
                       sB, (float2*)C, ldc, sC);
  else
    hipLaunchKernelGGL((cgemm_nn_mfma32<WM, WN, 0>), dim3((unsigned)pad, batch), dim3(256), 0, st, M,
                       N, K, nrt, ntiles, pad, (const double2*)A, lda, sA, (const float2*)B, ldb,
                       sB, (float2*)C, ldc, sC);
  return hipGetLastError();
}

template <typename TB, typename TC>
hipError_t dgemm_nn_grid(int M, int N, int K, int batch, const void* A, long lda, long sA,
                         const void* B, long ldb, long sB, void* C, long ldc, long sC,
                         hipStream_t st, bool lower) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (!offsets_fit(M, N, K, 2 * lda, ldb)) return hipErrorInvalidValue;
  if ((long)M * 2 * lda * 8 >= 0xffffffffL || (long)K * ldb * (long)sizeof(TB) >= 0xffffffffL)
    return hipErrorInvalidValue;
  const int nrt = (M + 63) / 64;
  const long nct = ((long)N + 255) / 256;
  const long ntiles = nrt * nct;
  const long pad = (ntiles + NXCD - 1) / NXCD * NXCD;
  if (lower)
    hipLaunchKernelGGL((dgemm_nn_mfma<TB, TC, 1>), dim3((unsigned)pad, batch), dim3(256), 0, st, M,
                       N, K, nrt, ntiles, pad, (const double2*)A, lda, sA, (const TB*)B, ldb, sB,
                       (TC*)C, ldc, sC);
  else
    hipLaunchKernelGGL((dgemm_nn_mfma<TB, TC, 0>), dim3((unsigned)pad, batch), dim3(256), 0, st, M,
                       N, K, nrt, ntiles, pad, (const double2*)A, lda, sA, (const TB*)B, ldb, sB,
                       (TC*)C, ldc, sC);
  return hipGetLastError();
}
template hipError_t dgemm_nn_grid<double, double>(int, int, int, int, const void*, long, long,
                                                  const void*, long, long, void*, long, long,
                                                  hipStream_t, bool);
template hipError_t dgemm_nn_grid<double, float>(int, int, int, int, const void*, long, long,
                                                 const void*, long, long, void*, long, long,
                                                 hipStream_t, bool);
template hipError_t dgemm_nn_grid<float, float>(int, int, int, int, const void*, long, long,
                                                const void*, long, long, void*, long, long,
                                                hipStream_t, bool);

template <typename TB, typename TC>
hipError_t dgemm_nn_grid_acc(int M, int N, int K, int batch, const void* A, long lda, long sA,
                             const void* B, long ldb, long sB, void* C, long ldc, long sC,
                             int sign, hipStream_t st, bool lower) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (!offsets_fit(M, N, K, 2 * lda, ldb)) return hipErrorInvalidValue;
  if ((long)M * 2 * lda * 8 >= 0xffffffffL || (long)K * ldb * (long)sizeof(TB) >= 0xffffffffL)
    return hipErrorInvalidValue;
  if (sign != 1 && sign != -1) return hipErrorInvalidValue;
  const int nrt = (M + 63) / 64;
  const long nct = ((long)N + 255) / 256;
  const long ntiles = nrt * nct;
  const long pad = (ntiles + NXCD - 1) / NXCD * NXCD;
#define EXX_DACC(LW, SG)                                                                      \
  hipLaunchKernelGGL((dgemm_nn_mfma<TB, TC, LW, SG>), dim3((unsigned)pad, batch), dim3(256), 0, \
                     st, M, N, K, nrt, ntiles, pad, (const double2*)A, lda, sA, (const TB*)B,  \
                     ldb, sB, (TC*)C, ldc, sC)
  if (lower && sign > 0)
    EXX_DACC(1, 1);
  else if (lower)
    EXX_DACC(1, -1);
  else if (sign > 0)
    EXX_DACC(0, 1);
  else
    EXX_DACC(0, -1);
#undef EXX_DACC
  return hipGetLastError();
}
#define EXX_DACC_INST(TB, TC)                                                                 \
  template hipError_t dgemm_nn_grid_acc<TB, TC>(int, int, int, int, const void*, long, long, \
                                                const void*, long, long, void*, long, long,  \
                                                int, hipStream_t, bool);
EXX_DACC_INST(double, double)
EXX_DACC_INST(float, double)
EXX_DACC_INST(double, float)
EXX_DACC_INST(float, float)
#undef EXX_DACC_INST

namespace {

// Small real FP64 products C[b] = alpha A[b] B[b] (+ C[b] with ACC) with every
// operand addressed by element strides (a view may be the real parts of complex
// storage or a transpose). Workgroup tile 64 x 64 of four 32 x 32 wave tiles;
// operands are read from global memory (they are small and stay in L2), four
// k-steps in flight per wave. CPLX: C is complex storage and gets (x, 0).
template <int CPLX, int ACC>
__global__ __launch_bounds__(256) void dgemm_strided_kernel(const double* __restrict__ A,
                                                            const double* __restrict__ B,
                                                            double* __restrict__ C,
                                                            StridedGemm s, double alpha) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int col0 = blockIdx.x * 64 + (wave & 1) * 32;
  const long b = blockIdx.z;
  A += b * s.sA;
  B += b * s.sB;
  C += b * s.sC;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
  for (int k0 = 0; k0 < s.K; k0 += 16) {
    double a[4][2], bv[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + lk;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = row0 + i * 16 + li;
        a[u][i] = (r < s.M && k < s.K) ? A[r * s.ar + k * s.ak] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = col0 + j * 16 + li;
        bv[u][j] = (c < s.N && k < s.K) ? B[k * s.bk + c * s.bc] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma64(a[u][i], bv[u][j], acc[i][j]);
  }
  // register v of a lane holds row 4 v + lane/16, column lane%16 of a block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + i * 16 + 4 * v + lk;
        const int c = col0 + j * 16 + li;
        if (r >= s.M || c >= s.N) continue;
        const long o = r * s.cr + c * s.cc;
        const double x = alpha * acc[i][j][v] + (ACC ? C[o] : 0.0);
        if (CPLX)
          *(double2*)(C + o) = make_double2(x, 0.0);
        else
          C[o] = x;
      }
}

}  // namespace

hipError_t dgemm_strided(const StridedGemm& s, int batch, const double* A, const double* B,
                         double* C, bool cplx_out, hipStream_t st, double alpha, bool acc) {
  if (s.M <= 0 || s.N <= 0 || batch <= 0) return hipSuccess;
  if (s.K <= 0 || (cplx_out && ((s.cr | s.cc | s.sC) & 1))) return hipErrorInvalidValue;
  if (s.ar < 0 || s.ak < 0 || s.bk < 0 || s.bc < 0 || s.cr < 0 || s.cc < 0)
    return hipErrorInvalidValue;
  const long lim = 0x7fffffffL;
  if ((long)(s.M - 1) * s.ar + (long)(s.K - 1) * s.ak >= lim ||
      (long)(s.K - 1) * s.bk + (long)(s.N - 1) * s.bc >= lim ||
      (long)(s.M - 1) * s.cr + (long)(s.N - 1) * s.cc + 1 >= lim)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((s.N + 63) / 64), (unsigned)((s.M + 63) / 64), (unsigned)batch);
#define EXX_STRIDED(CX, AC)                                                                  \
  hipLaunchKernelGGL((dgemm_strided_kernel<CX, AC>), grid, dim3(256), 0, st, A, B, C, s, alpha)
  if (cplx_out) {
    if (acc)
      EXX_STRIDED(1, 1);
    else
      EXX_STRIDED(1, 0);
  } else {
    if (acc)
      EXX_STRIDED(0, 1);
    else
      EXX_STRIDED(0, 0);
  }
#undef EXX_STRIDED
  return hipGetLastError();
}

template <typename TB, typename TC>
hipError_t zgemm_nn_grid_acc(int M, int N, int K, int batch, const void* A, long lda, long sA,
                             const void* B, long ldb, long sB, void* C, long ldc, long sC,
                             int sign, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (!offsets_fit(M, N, K, lda, ldb)) return hipErrorInvalidValue;
  if (sign > 0)
    return run_nn<TB, TC, 2, 2, 0, 1>(M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc, sC, st);
  return run_nn<TB, TC, 2, 2, 0, -1>(M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc, sC, st);
}

#define EXX_ACC_INST(TB, TC)                                                                  \
  template hipError_t zgemm_nn_grid_acc<TB, TC>(int, int, int, int, const void*, long, long, \
                                                const void*, long, long, void*, long, long,  \
                                                int, hipStream_t);
EXX_ACC_INST(double, double)
EXX_ACC_INST(float, double)
EXX_ACC_INST(double, float)
EXX_ACC_INST(float, float)
#undef EXX_ACC_INST

template hipError_t zgemm_nn_grid<double, double>(int, int, int, int, const void*, long, long,
                                                  bool, const void*, long, long, void*, long, long,
                                                  hipStream_t, int, bool);
template hipError_t zgemm_nn_grid<float, float>(int, int, int, int, const void*, long, long, bool,
                                                const void*, long, long, void*, long, long,
                                                hipStream_t, int, bool);
template hipError_t zgemm_nn_grid<double, float>(int, int, int, int, const void*, long, long, bool,
                                                 const void*, long, long, void*, long, long,
                                                 hipStream_t, int, bool);
template hipError_t zgemm_nn_grid<float, double>(int, int, int, int, const void*, long, long, bool,
                                                 const void*, long, long, void*, long, long,
                                                 hipStream_t, int, bool);

}  // namespace exx

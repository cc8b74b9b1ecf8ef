// Batched complex GEMM, LDS-tiled, vector FMA. Serves the small and medium
// contractions of the build (G^n, S^+, K^n) and is the portable baseline for
// the grid-sized ones.
#include <algorithm>

#include "common.h"

namespace exx {

namespace {

constexpr int BM = 64, BN = 64, BK = 8, NT = 256;

template <typename T, typename TA, typename TB, typename TC, int OA, int OB>
__global__ __launch_bounds__(NT) void gemm_tiled(int M, int N, int K, const cplx<TA>* __restrict__ A,
                                                 long lda, long sA, const cplx<TB>* __restrict__ B,
                                                 long ldb, long sB, cplx<TC>* __restrict__ C,
                                                 long ldc, long sC, T alpha, int accumulate,
                                                 int nsplit, int kc, long sCs) {
  __shared__ cplx<T> As[BK][BM];
  __shared__ cplx<T> Bs[BK][BN];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  // split-K: slice s of the K range [s kc, min(K, (s + 1) kc)) into C + s sCs
  const long b = blockIdx.z / nsplit;
  const int sk = blockIdx.z % nsplit;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
  const int kb = sk * kc, ke = min(K, kb + kc);
  A += b * sA;
  B += b * sB;
  C += b * sC + sk * sCs;

  cplx<T> acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = mk<T>(0, 0);

  for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
    for (int s = 0; s < (BM * BK) / NT; ++s) {
      int e = tid + NT * s;
      int i, k;
      if (OA == A_N) {
        i = e / BK;
        k = e % BK;
      } else {
        k = e / BM;
        i = e % BM;
      }
      int gi = i0 + i, gk = k0 + k;
      cplx<T> val = mk<T>(0, 0);
      if (gi < M && gk < ke) {
        if (OA == A_N)
          val = cload<T, TA>(A + (long)gi * lda + gk);
        else
          val = cconj<T>(cload<T, TA>(A + (long)gk * lda + gi));
      }
      As[k][i] = val;
    }
#pragma unroll
    for (int s = 0; s < (BN * BK) / NT; ++s) {
      int e = tid + NT * s;
      int j, k;
      if (OB == B_C) {
        j = e / BK;
        k = e % BK;
      } else {
        k = e / BN;
        j = e % BN;
      }
      int gj = j0 + j, gk = k0 + k;
      cplx<T> val = mk<T>(0, 0);
      if (gj < N && gk < ke) {
        if (OB == B_N)
          val = cload<T, TB>(B + (long)gk * ldb + gj);
        else if (OB == B_R)
          val = cconj<T>(cload<T, TB>(B + (long)gk * ldb + gj));
        else
          val = cconj<T>(cload<T, TB>(B + (long)gj * ldb + gk));
      }
      Bs[k][j] = val;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      cplx<T> a[4], bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[kk][ty + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) bb[v] = Bs[kk][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc[u][v].x += a[u].x * bb[v].x - a[u].y * bb[v].y;
          acc[u][v].y += a[u].x * bb[v].y + a[u].y * bb[v].x;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int gi = i0 + ty + 16 * u;
    if (gi >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int gj = j0 + tx + 16 * v;
      if (gj >= N) continue;
      cplx<T> val = cscale<T>(acc[u][v], alpha);
      cplx<TC>* p = C + (long)gi * ldc + gj;
      if (accumulate) val = cadd<T>(val, cload<T, TC>(p));
      cstore<TC, T>(p, val);
    }
  }
}

template <typename T, typename TA, typename TB, typename TC, int OA, int OB>
hipError_t run(int M, int N, int K, int batch, const void* A, long lda, long sA, const void* B,
               long ldb, long sB, void* C, long ldc, long sC, T alpha, bool accumulate,
               hipStream_t st, int nsplit = 1, int kc = 0, long sCs = 0) {
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch * nsplit);
  hipLaunchKernelGGL((gemm_tiled<T, TA, TB, TC, OA, OB>), grid, dim3(NT), 0, st, M, N, K,
                     (const cplx<TA>*)A, lda, sA, (const cplx<TB>*)B, ldb, sB, (cplx<TC>*)C, ldc,
                     sC, alpha, accumulate ? 1 : 0, nsplit, nsplit > 1 ? kc : K, sCs);
  return hipGetLastError();
}

// C[b][i][j] = alpha sum_s part[s][b][i][j] (+ C[b][i][j]), the slices added in order
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const double2* __restrict__ part,
                                                            double2* __restrict__ C, int M, int N,
                                                            long ldc, long sC, int nsplit,
                                                            long per, double alpha,
                                                            int accumulate) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= per) return;
  const long mn = (long)M * N;
  const long b = e / mn;
  const int i = (int)((e % mn) / N), j = (int)(e % N);
  double sx = 0.0, sy = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    const double2 v = part[(long)s * per + e];
    sx += v.x;
    sy += v.y;
  }
  double2* p = C + b * sC + (long)i * ldc + j;
  double2 r = make_double2(alpha * sx, alpha * sy);
  if (accumulate) {
    const double2 c = *p;
    r.x += c.x;
    r.y += c.y;
  }
  *p = r;
}

// the K range of one slice: a multiple of BK
int splitk_chunk(int K, int nsplit) { return ((K + nsplit - 1) / nsplit + BK - 1) / BK * BK; }

}  // namespace

template <typename T, typename TA, typename TB, typename TC>
hipError_t gemm(int M, int N, int K, int batch, OpA oa, const void* A, long lda, long sA, OpB ob,
                const void* B, long ldb, long sB, void* C, long ldc, long sC, T alpha,
                bool accumulate, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
#define EXX_GEMM_CASE(oa_, ob_)                                                                 \
  if (oa == oa_ && ob == ob_)                                                                   \
    return run<T, TA, TB, TC, oa_, ob_>(M, N, K, batch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, \
                                        accumulate, st);
  EXX_GEMM_CASE(A_N, B_N)
  EXX_GEMM_CASE(A_N, B_R)
  EXX_GEMM_CASE(A_N, B_C)
  EXX_GEMM_CASE(A_C, B_N)
  EXX_GEMM_CASE(A_C, B_R)
#undef EXX_GEMM_CASE
  return hipErrorInvalidValue;
}

int gemm_splitk_parts(int M, int N, int K, int batch) {
  const long blocks = (long)((N + BN - 1) / BN) * ((M + BM - 1) / BM) * batch;
  long ns = (2048 + blocks - 1) / blocks;  // about 2048 workgroups
  ns = std::min(ns, (long)std::max(1, K / 512));
  ns = std::min(ns, 64L);
  return (int)std::max(1L, ns);
}

hipError_t zgemm_splitk(int M, int N, int K, int batch, OpA oa, const void* A, long lda, long sA,
                        OpB ob, const void* B, long ldb, long sB, void* C, long ldc, long sC,
                        double alpha, bool accumulate, void* part, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  const int ns = gemm_splitk_parts(M, N, K, batch);
  const int kc = splitk_chunk(K, ns);
  const long per = (long)batch * M * N;
  hipError_t e = hipErrorInvalidValue;
  if (oa == A_N && ob == B_C)  // C = A B^H: the slices on the FP64 matrix cores
    e = zgemm_abh_parts(M, N, K, batch, A, lda, sA, B, ldb, sB, part, ns, kc, st);
  else if (oa == A_N && ob == B_R)
    e = run<double, double, double, double, A_N, B_R>(M, N, K, batch, A, lda, sA, B, ldb, sB, part,
                                                      N, (long)M * N, 1.0, false, st, ns, kc, per);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, st,
                     (const double2*)part, (double2*)C, M, N, ldc, sC, ns, per, alpha,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

template hipError_t gemm<double, double, double, double>(int, int, int, int, OpA, const void*,
                                                         long, long, OpB, const void*, long, long,
                                                         void*, long, long, double, bool,
                                                         hipStream_t);
template hipError_t gemm<float, double, float, float>(int, int, int, int, OpA, const void*, long,
                                                      long, OpB, const void*, long, long, void*,
                                                      long, long, float, bool, hipStream_t);
template hipError_t gemm<double, double, float, float>(int, int, int, int, OpA, const void*, long,
                                                       long, OpB, const void*, long, long, void*,
                                                       long, long, double, bool, hipStream_t);

template <typename T>
hipError_t launch_gamma(const Geom& g, const void* occ_pts, const void* psi, void* gam,
                        hipStream_t st) {
  return gemm<T, double, T, T>(g.ni, g.ng, g.no, g.nk, A_N, occ_pts, g.no, (long)g.ni * g.no, B_R,
                               psi, g.ng, (long)g.no * g.ng, gam, g.ng, (long)g.ni * g.ng, (T)1,
                               false, st);
}
template hipError_t launch_gamma<double>(const Geom&, const void*, const void*, void*, hipStream_t);
template hipError_t launch_gamma<float>(const Geom&, const void*, const void*, void*, hipStream_t);

}  // namespace exx

// Exchange contraction helpers: the k-mesh convolution of the Bloch-gauge
// Coulomb matrices with the occupied point Gram matrices, and the FP64
// exchange-energy reduction.
#include "common.h"

namespace exx {

namespace {

struct KconvArgs {
  int N[3];
  int nk;
  long nn;
};

// The k-mesh convolution Y^n = sum_m Vb^m o G^{n+m}, elementwise over the
// N_I x N_I matrices, by DFTs over the mesh: with F[x](k) = sum_n x^n e^{-2 pi i
// k.n / N}, F[Y](k) = F[Vb](-k) F[G](k), so Y = F^{-1}[F[Vb](-k) F[G](k)]. Each
// mesh DFT runs axis by axis as direct DFTs of the axis length (at most 8):
// N_k (N_1 + N_2 + N_3) complex products per element and transform, against N_k^2
// for the direct sum, and every operand value is read from memory once. A
// workgroup stages KC_E consecutive elements of every transfer of both operands
// in LDS; a thread transforms whole lines of one element.
constexpr int KC_E = 16;
constexpr int KC_NT = 256;

// one axis of the mesh DFT on buf[k][j] (k the flat mesh index, j < KC_E)
__device__ __forceinline__ void kconv_axis(double2* buf, const KconvArgs& a, int ax,
                                           const double2* tw, bool inverse) {
  const int na = a.N[ax];
  if (na == 1) return;
  const int st = ax == 0 ? a.N[1] * a.N[2] : (ax == 1 ? a.N[2] : 1);
  const int nlines = a.nk / na;
  for (int it = threadIdx.x; it < nlines * KC_E; it += KC_NT) {
    const int j = it % KC_E, l = it / KC_E;
    const int base = (l / st) * (na * st) + l % st;
    double2 x[8];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (t < na) x[t] = buf[(base + t * st) * KC_E + j];
    for (int s = 0; s < na; ++s) {
      double yr = x[0].x, yi = x[0].y;
#pragma unroll
      for (int t = 1; t < 8; ++t) {
        if (t >= na) break;
        const double2 w = tw[(s * t) % na];
        const double wi = inverse ? -w.y : w.y;
        yr += x[t].x * w.x - x[t].y * wi;
        yi += x[t].x * wi + x[t].y * w.x;
      }
      buf[(base + s * st) * KC_E + j] = make_double2(yr, yi);
    }
  }
}

__global__ __launch_bounds__(KC_NT) void kconv_dft_kernel(const double2* __restrict__ Vb,
                                                          const double2* __restrict__ G,
                                                          double2* __restrict__ Y, KconvArgs a) {
  __shared__ double2 sv[64 * KC_E];
  __shared__ double2 sg[64 * KC_E];
  __shared__ double2 tw[3][8];
  const long e0 = (long)blockIdx.x * KC_E;
  const int ne = (int)min((long)KC_E, a.nn - e0);
  const int tot = a.nk * KC_E;
  for (int it = threadIdx.x; it < tot; it += KC_NT) {
    const int k = it / KC_E, j = it % KC_E;
    const long src = (long)k * a.nn + e0 + j;
    sv[it] = j < ne ? Vb[src] : make_double2(0.0, 0.0);
    sg[it] = j < ne ? G[src] : make_double2(0.0, 0.0);
  }
  if (threadIdx.x < 24) {  // e^{-2 pi i u / N_a}
    const int ax = threadIdx.x / 8, u = threadIdx.x % 8;
    double sn = 0.0, cs = 1.0;
    if (u < a.N[ax]) sincospi(-2.0 * u / a.N[ax], &sn, &cs);
    tw[ax][u] = make_double2(cs, sn);
  }
  __syncthreads();
  for (int ax = 2; ax >= 0; --ax) {
    if (a.N[ax] == 1) continue;
    kconv_axis(sv, a, ax, tw[ax], false);
    kconv_axis(sg, a, ax, tw[ax], false);
    __syncthreads();
  }
  // F[Y](k) = F[Vb](-k) F[G](k)
  for (int it = threadIdx.x; it < tot; it += KC_NT) {
    const int k = it / KC_E, j = it % KC_E;
    const int k1 = k / (a.N[1] * a.N[2]), k2 = (k / a.N[2]) % a.N[1], k3 = k % a.N[2];
    const int kr = (((a.N[0] - k1) % a.N[0]) * a.N[1] + (a.N[1] - k2) % a.N[1]) * a.N[2] +
                   (a.N[2] - k3) % a.N[2];
    const double2 v = sv[kr * KC_E + j], g = sg[it];
    sg[it] = make_double2(v.x * g.x - v.y * g.y, v.x * g.y + v.y * g.x);
  }
  __syncthreads();
  for (int ax = 2; ax >= 0; --ax) {
    if (a.N[ax] == 1) continue;
    kconv_axis(sg, a, ax, tw[ax], true);
    __syncthreads();
  }
  const double inv = 1.0 / a.nk;
  for (int it = threadIdx.x; it < tot; it += KC_NT) {
    const int k = it / KC_E, j = it % KC_E;
    if (j < ne) {
      const double2 y = sg[it];
      Y[(long)k * a.nn + e0 + j] = make_double2(y.x * inv, y.y * inv);
    }
  }
}

// AH[b][c][r] = s * conj(A[b][r][c]) for an (rows x cols) matrix per batch item
__global__ __launch_bounds__(256) void conj_transpose_kernel(const double2* __restrict__ A,
                                                             double2* __restrict__ AH, int rows,
                                                             int cols, double s) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)rows * cols;
  if (e >= n) return;
  const long b = blockIdx.y;
  const int c = (int)(e / rows), r = (int)(e % rows);  // output order: consecutive r
  const double2 v = A[b * n + (long)r * cols + c];
  AH[b * n + e] = make_double2(s * v.x, -s * v.y);
}

constexpr int EN_NT = 256;

// partial[b] = sum over block b of Re(Y conj G)
__global__ __launch_bounds__(EN_NT) void energy_partial_kernel(const double2* __restrict__ Y,
                                                               const double2* __restrict__ G,
                                                               long total,
                                                               double* __restrict__ partial) {
  __shared__ double red[EN_NT];
  double s = 0.0;
  for (long e = (long)blockIdx.x * EN_NT + threadIdx.x; e < total; e += (long)gridDim.x * EN_NT) {
    const double2 y = Y[e], g = G[e];
    s += y.x * g.x + y.y * g.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = EN_NT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(EN_NT) void energy_final_kernel(const double* __restrict__ partial,
                                                             int nb, double scale,
                                                             double* __restrict__ Ex) {
  __shared__ double red[EN_NT];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += EN_NT) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = EN_NT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *Ex = scale * red[0];
}

}  // namespace

hipError_t launch_kconv(const Geom& g, const double2* Vb, const double2* G, double2* Y,
                        hipStream_t st) {
  KconvArgs a;
  for (int i = 0; i < 3; ++i) a.N[i] = g.N[i];
  a.nk = g.nk;
  a.nn = (long)g.ni * g.ni;
  if (g.nk > 64 || g.N[0] > 8 || g.N[1] > 8 || g.N[2] > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kconv_dft_kernel, dim3((unsigned)((a.nn + KC_E - 1) / KC_E)), dim3(KC_NT), 0,
                     st, Vb, G, Y, a);
  return hipGetLastError();
}

hipError_t launch_energy(const Geom& g, const double2* Y, const double2* G, double* partial,
                         double* Ex, hipStream_t st) {
  const long total = (long)g.nk * g.ni * g.ni;
  const int nb = 512;
  hipLaunchKernelGGL(energy_partial_kernel, dim3(nb), dim3(EN_NT), 0, st, Y, G, total, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double scale = -1.0 / ((double)g.nk * (double)g.nk);
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(EN_NT), 0, st, partial, nb, scale, Ex);
  return hipGetLastError();
}

hipError_t launch_conj_transpose(const double2* A, double2* AH, int rows, int cols, int batch,
                                 double s, hipStream_t st) {
  const long n = (long)rows * cols;
  if (n <= 0 || batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(conj_transpose_kernel, dim3((unsigned)((n + 255) / 256), batch), dim3(256), 0,
                     st, A, AH, rows, cols, s);
  return hipGetLastError();
}

}  // namespace exx

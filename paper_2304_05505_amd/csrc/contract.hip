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

// Y[n][e] = sum_{n'} Vb[m(n, n')][e] * G[n'][e], m = (n' - n) mod N per axis
__global__ __launch_bounds__(256) void kconv_kernel(const double2* __restrict__ Vb,
                                                    const double2* __restrict__ G,
                                                    double2* __restrict__ Y, KconvArgs a) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (e >= a.nn) return;
  const int n1 = n / (a.N[1] * a.N[2]), n2 = (n / a.N[2]) % a.N[1], n3 = n % a.N[2];
  double sx = 0.0, sy = 0.0;
  for (int q = 0; q < a.nk; ++q) {
    const int q1 = q / (a.N[1] * a.N[2]), q2 = (q / a.N[2]) % a.N[1], q3 = q % a.N[2];
    const int m1 = (q1 - n1 + a.N[0]) % a.N[0];
    const int m2 = (q2 - n2 + a.N[1]) % a.N[1];
    const int m3 = (q3 - n3 + a.N[2]) % a.N[2];
    const int m = (m1 * a.N[1] + m2) * a.N[2] + m3;
    const double2 v = Vb[(long)m * a.nn + e];
    const double2 gq = G[(long)q * a.nn + e];
    sx += v.x * gq.x - v.y * gq.y;
    sy += v.x * gq.y + v.y * gq.x;
  }
  Y[(long)n * a.nn + e] = make_double2(sx, sy);
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
  hipLaunchKernelGGL(kconv_kernel, dim3((unsigned)((a.nn + 255) / 256), g.nk), dim3(256), 0, st, Vb,
                     G, Y, a);
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

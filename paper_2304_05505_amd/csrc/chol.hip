// Blocked FP64 Cholesky factorisation of the fit metrics S^m in point order
// with pivot drop, and the blocked inverse of the factor, batched over the
// transfers m. Panels of NB columns are factorised by one workgroup per m in
// LDS; the trailing updates and the off-diagonal blocks of the inverse are
// batched complex GEMMs over all m.
//
// Drop rule: a point whose Schur-complement pivot falls below
// rel_tol * max_P S^m_PP is dropped: its column of L is zero, it does not
// update later columns, and its row and column of L^{-1} are zero. The
// retained block then satisfies S_RR = L_RR L_RR^H.
#include <algorithm>
#include <climits>

#include "common.h"

namespace exx {

namespace {

constexpr int NB = 32;
constexpr int PNT = 256;

// tol[m] = rel_tol * max_P Re S^m_PP; rank[m] = 0
__global__ __launch_bounds__(PNT) void chol_init_kernel(const double2* __restrict__ A, int n,
                                                        double rel_tol, double* __restrict__ tol,
                                                        int32_t* __restrict__ rank) {
  const int m = blockIdx.x;
  const double2* Am = A + (long)m * n * n;
  __shared__ double red[PNT];
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += PNT) mx = fmax(mx, Am[(long)i * n + i].x);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = PNT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tol[m] = rel_tol * red[0];
    rank[m] = 0;
  }
}

// Factorise the diagonal block at c0 (width w) and solve the rows below it.
// status (may be null): a non-finite pivot sets ST_NONFINITE with site
// SITE_METRIC; with strict, a pivot dropped by the rule sets ST_NOT_PD and
// lowers status[1] to the transfer label of this metric.
__global__ __launch_bounds__(PNT) void chol_panel_kernel(double2* __restrict__ A, int n, int c0,
                                                         const double* __restrict__ tol,
                                                         int32_t* __restrict__ keep,
                                                         int32_t* __restrict__ rank,
                                                         int32_t* __restrict__ status, int strict,
                                                         QLabel lab) {
  const int m = blockIdx.x;
  double2* Am = A + (long)m * n * n;
  int32_t* km = keep + (long)m * n;
  const int w = min(NB, n - c0);
  __shared__ double2 D[NB][NB + 1];
  __shared__ int kp[NB];
  __shared__ int s_kept;
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += PNT) {
    const int i = e / w, j = e % w;
    D[i][j] = (j <= i) ? Am[(long)(c0 + i) * n + c0 + j] : make_double2(0.0, 0.0);
  }
  if (tid == 0) s_kept = 0;
  __syncthreads();
  const double tl = tol[m];
  for (int p = 0; p < w; ++p) {
    const double d = D[p][p].x;
    const bool ok = (d >= tl) && (d > 0.0) && isfinite(d);
    __syncthreads();
    if (ok) {
      const double s = sqrt(d), inv = 1.0 / s;
      for (int i = p + tid; i < w; i += PNT)
        D[i][p] = (i == p) ? make_double2(s, 0.0) : make_double2(D[i][p].x * inv, D[i][p].y * inv);
    } else {
      for (int i = p + tid; i < w; i += PNT) D[i][p] = make_double2(0.0, 0.0);
    }
    if (tid == 0) {
      kp[p] = ok ? 1 : 0;
      s_kept += ok ? 1 : 0;
      if (!ok && status) {
        if (!isfinite(d)) {
          atomicOr(status, (int)ST_NONFINITE);
          atomicMin(status + 2, (int)SITE_METRIC);
        } else if (strict) {
          atomicOr(status, (int)ST_NOT_PD);
          atomicMin(status + 1, lab.q[m]);
        }
      }
    }
    __syncthreads();
    if (ok) {
      const int r = w - p - 1;
      for (int e = tid; e < r * r; e += PNT) {
        const int i = p + 1 + e / r, j = p + 1 + e % r;
        if (j > i) continue;
        const double2 li = D[i][p], lj = D[j][p];
        D[i][j].x -= li.x * lj.x + li.y * lj.y;
        D[i][j].y -= li.y * lj.x - li.x * lj.y;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < w * w; e += PNT) {
    const int i = e / w, j = e % w;
    if (j <= i) Am[(long)(c0 + i) * n + c0 + j] = D[i][j];
  }
  for (int p = tid; p < w; p += PNT) km[c0 + p] = kp[p];
  if (tid == 0) rank[m] += s_kept;
  // rows below: x L_D^H = a  ->  x_p = (a_p - sum_{c<p} x_c conj L_D[p][c]) / L_D[p][p]
  for (int i = c0 + w + tid; i < n; i += PNT) {
    double2* row = Am + (long)i * n + c0;
    double2 x[NB];
#pragma unroll
    for (int p = 0; p < NB; ++p) x[p] = (p < w) ? row[p] : make_double2(0.0, 0.0);
#pragma unroll
    for (int p = 0; p < NB; ++p) {
      if (p >= w) break;
      if (!kp[p]) {
        x[p] = make_double2(0.0, 0.0);
        continue;
      }
      double sx = x[p].x, sy = x[p].y;
#pragma unroll
      for (int c = 0; c < p; ++c) {
        const double2 l = D[p][c];  // x_c * conj(l)
        sx -= x[c].x * l.x + x[c].y * l.y;
        sy -= x[c].y * l.x - x[c].x * l.y;
      }
      const double inv = 1.0 / D[p][p].x;
      x[p] = make_double2(sx * inv, sy * inv);
    }
#pragma unroll
    for (int p = 0; p < NB; ++p)
      if (p < w) row[p] = x[p];
  }
}

// status[0] |= ST_NONFINITE, status[2] = min(status[2], site) if any value is not finite
__global__ __launch_bounds__(256) void check_finite_kernel(const double* __restrict__ p, long n,
                                                           int32_t* __restrict__ status, int site) {
  bool bad = false;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256)
    bad |= !isfinite(p[e]);
  if (__any(bad) && (threadIdx.x & 63) == 0) {
    atomicOr(status, (int)ST_NONFINITE);
    atomicMin(status + 2, site);
  }
}

__global__ void copy_kernel(double2* __restrict__ dst, const double2* __restrict__ src, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

// W := 0 (whole n x n of every m)
__global__ void zero_kernel(double2* __restrict__ W, long total) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) W[e] = make_double2(0.0, 0.0);
}

// Diagonal blocks of the inverse: W_bb = L_bb^{-1} on the retained points.
__global__ __launch_bounds__(PNT) void diag_inv_kernel(const double2* __restrict__ Lf, int n,
                                                       const int32_t* __restrict__ keep,
                                                       double2* __restrict__ W) {
  const int m = blockIdx.y;
  const int c0 = blockIdx.x * NB;
  const int w = min(NB, n - c0);
  const double2* Lm = Lf + (long)m * n * n;
  const int32_t* km = keep + (long)m * n;
  double2* Wm = W + (long)m * n * n;
  __shared__ double2 D[NB][NB + 1];
  for (int e = threadIdx.x; e < w * w; e += PNT) {
    const int i = e / w, j = e % w;
    D[i][j] = (j <= i) ? Lm[(long)(c0 + i) * n + c0 + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int j = threadIdx.x;  // one column of the block per thread
  if (j >= w) return;
  double2 x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = make_double2(0.0, 0.0);
  if (km[c0 + j]) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (i >= w) break;
      if (i < j || !km[c0 + i]) continue;
      double sx = (i == j) ? 1.0 : 0.0, sy = 0.0;
#pragma unroll
      for (int c = 0; c < i; ++c) {
        if (c < j) continue;
        const double2 l = D[i][c];
        sx -= l.x * x[c].x - l.y * x[c].y;
        sy -= l.x * x[c].y + l.y * x[c].x;
      }
      const double inv = 1.0 / D[i][i].x;
      x[i] = make_double2(sx * inv, sy * inv);
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < w) Wm[(long)(c0 + i) * n + c0 + j] = x[i];
}

}  // namespace

struct RankMap {
  int rep[64], bar[64];
  int n;
};

// rank[rep[s]] = rc[s] and, for a conjugate partner, rank[bar[s]] = rc[s]
__global__ void rank_scatter_kernel(const int32_t* __restrict__ rc, int32_t* __restrict__ rank,
                                    RankMap mp) {
  const int s = threadIdx.x;
  if (s >= mp.n) return;
  rank[mp.rep[s]] = rc[s];
  if (mp.bar[s] >= 0) rank[mp.bar[s]] = rc[s];
}

hipError_t launch_rank_scatter(const int32_t* rc, int32_t* rank, const int* rep, const int* bar,
                               int n, hipStream_t st) {
  RankMap mp;
  for (int s = 0; s < 64; ++s) {
    mp.rep[s] = s < n ? rep[s] : 0;
    mp.bar[s] = s < n ? bar[s] : -1;
  }
  mp.n = n;
  hipLaunchKernelGGL(rank_scatter_kernel, dim3(1), dim3(64), 0, st, rc, rank, mp);
  return hipGetLastError();
}

// rank[m] = rc[0] for every transfer (one fit shared by all transfers)
__global__ void rank_broadcast_kernel(const int32_t* __restrict__ rc, int32_t* __restrict__ rank,
                                      int nk) {
  const int m = threadIdx.x;
  if (m < nk) rank[m] = rc[0];
}

hipError_t launch_rank_broadcast(const int32_t* rc, int32_t* rank, int nk, hipStream_t st) {
  if (nk <= 0 || nk > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rank_broadcast_kernel, dim3(1), dim3(64), 0, st, rc, rank, nk);
  return hipGetLastError();
}

__global__ void status_reset_kernel(int32_t* __restrict__ status) {
  if (threadIdx.x == 0) {
    status[0] = 0;
    status[1] = INT_MAX;
    status[2] = INT_MAX;
    status[3] = 0;
  }
}

__global__ void zero_upper_kernel(double2* __restrict__ A, int n, long total) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long w = e % ((long)n * n);
  if (w % n > w / n) A[e] = make_double2(0.0, 0.0);
}

hipError_t launch_zero_upper(double2* A, int n, int batch, hipStream_t st) {
  const long total = (long)batch * n * n;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A,
                     n, total);
  return hipGetLastError();
}

hipError_t launch_status_reset(int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(status_reset_kernel, dim3(1), dim3(64), 0, st, status);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* p, long n, int32_t* status, int site,
                               hipStream_t st) {
  if (n <= 0 || !status) return hipSuccess;
  const long blocks = std::min<long>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, status,
                     site);
  return hipGetLastError();
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void convert_kernel(const cplx<TS>* __restrict__ src,
                                                      cplx<TD>* __restrict__ dst, long n) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < n) dst[e] = mk<TD>((TD)src[e].x, (TD)src[e].y);
}

template <typename TS, typename TD>
hipError_t launch_convert(const void* src, void* dst, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<TS, TD>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const cplx<TS>*)src, (cplx<TD>*)dst, n);
  return hipGetLastError();
}
template hipError_t launch_convert<double, double>(const void*, void*, long, hipStream_t);
template hipError_t launch_convert<double, float>(const void*, void*, long, hipStream_t);
template hipError_t launch_convert<float, float>(const void*, void*, long, hipStream_t);

hipError_t launch_copy(double2* dst, const double2* src, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

static QLabel labels(const QLabel* lab) {
  QLabel l;
  for (int s = 0; s < 64; ++s) l.q[s] = lab ? lab->q[s] : s;
  return l;
}

hipError_t launch_chol_blocked(const Geom& g, double2* A, int32_t* keep, int32_t* rank,
                               double* tol, double rel_tol, hipStream_t st, int32_t* status,
                               bool strict, const QLabel* lab) {
  const int n = g.ni;
  const long nn = (long)n * n;
  const QLabel ql = labels(lab);
  hipLaunchKernelGGL(chol_init_kernel, dim3(g.nk), dim3(PNT), 0, st, A, n, rel_tol, tol, rank);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int c0 = 0; c0 < n; c0 += NB) {
    const int w = n - c0 < NB ? n - c0 : NB;
    hipLaunchKernelGGL(chol_panel_kernel, dim3(g.nk), dim3(PNT), 0, st, A, n, c0, tol, keep, rank,
                       status, strict ? 1 : 0, ql);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int r = n - c0 - w;
    if (r <= 0) break;
    double2* Lp = A + (long)(c0 + w) * n + c0;
    double2* Ct = A + (long)(c0 + w) * n + c0 + w;
    // trailing update A22 -= L21 L21^H
    e = gemm<double, double, double, double>(r, r, w, g.nk, A_N, Lp, n, nn, B_C, Lp, n, nn, Ct, n,
                                             nn, -1.0, true, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_tri_inv_blocked(const Geom& g, const double2* Lf, const int32_t* keep,
                                  double2* W, double2* T, hipStream_t st) {
  const int n = g.ni;
  const long nn = (long)n * n;
  const long total = (long)g.nk * nn;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, W, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = (n + NB - 1) / NB;
  hipLaunchKernelGGL(diag_inv_kernel, dim3(nb, g.nk), dim3(PNT), 0, st, Lf, n, keep, W);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // block row i: W[i, 0:ci] = -W_ii (L[i, 0:ci] W[0:ci, 0:ci])
  for (int b = 1; b < nb; ++b) {
    const int ci = b * NB;
    const int w = n - ci < NB ? n - ci : NB;
    e = gemm<double, double, double, double>(w, ci, ci, g.nk, A_N, Lf + (long)ci * n, n, nn, B_N, W,
                                             n, nn, T, ci, (long)NB * n, 1.0, false, st);
    if (e != hipSuccess) return e;
    e = gemm<double, double, double, double>(w, ci, w, g.nk, A_N, W + (long)ci * n + ci, n, nn, B_N,
                                             T, ci, (long)NB * n, W + (long)ci * n, n, nn, -1.0,
                                             false, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Real-path forms (the metric S~ is real, stored complex with a zero imaginary
// part): the trailing updates and the off-diagonal blocks of the inverse run on
// the real parts through the strided FP64 matrix-core product; the panel and
// diagonal-block kernels are the complex ones, exact on real data.
hipError_t launch_chol_blocked_real(const Geom& g, double2* A, int32_t* keep, int32_t* rank,
                                   double* tol, double rel_tol, hipStream_t st, int32_t* status,
                                   bool strict) {
  const int n = g.ni;
  const long nn = (long)n * n;
  const QLabel ql = labels(nullptr);
  hipLaunchKernelGGL(chol_init_kernel, dim3(g.nk), dim3(PNT), 0, st, A, n, rel_tol, tol, rank);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double* Ad = (double*)A;
  for (int c0 = 0; c0 < n; c0 += NB) {
    const int w = n - c0 < NB ? n - c0 : NB;
    hipLaunchKernelGGL(chol_panel_kernel, dim3(g.nk), dim3(PNT), 0, st, A, n, c0, tol, keep, rank,
                       status, strict ? 1 : 0, ql);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int r = n - c0 - w;
    if (r <= 0) break;
    // A22 -= L21 L21^T: L21(i, k) at row c0 + w + i, column c0 + k
    const double* L21 = Ad + 2 * ((long)(c0 + w) * n + c0);
    StridedGemm p{2 * nn, 2 * nn, 2 * nn, 2 * n, 2, 2, 2 * n, 2 * n, 2, r, r, w};
    e = dgemm_strided(p, g.nk, L21, L21, Ad + 2 * ((long)(c0 + w) * n + c0 + w), true, st, -1.0,
                      true);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_tri_inv_real(const Geom& g, const double2* Lf, const int32_t* keep, double2* W,
                               double2* T, hipStream_t st) {
  const int n = g.ni;
  const long nn = (long)n * n;
  const long total = (long)g.nk * nn;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, W, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = (n + NB - 1) / NB;
  hipLaunchKernelGGL(diag_inv_kernel, dim3(nb, g.nk), dim3(PNT), 0, st, Lf, n, keep, W);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double* Ld = (const double*)Lf;
  double* Wd = (double*)W;
  double* Td = (double*)T;  // w x ci real per transfer, NB n doubles apart
  for (int b = 1; b < nb; ++b) {
    const int ci = b * NB;
    const int w = n - ci < NB ? n - ci : NB;
    // T = L[ci:ci+w, 0:ci] W[0:ci, 0:ci]
    StridedGemm p1{2 * nn, 2 * nn, (long)NB * n, 2 * n, 2, 2 * n, 2, ci, 1, w, ci, ci};
    e = dgemm_strided(p1, g.nk, Ld + 2 * (long)ci * n, Wd, Td, false, st);
    if (e != hipSuccess) return e;
    // W[ci:ci+w, 0:ci] = -W[ci:ci+w, ci:ci+w] T
    StridedGemm p2{2 * nn, (long)NB * n, 2 * nn, 2 * n, 2, ci, 1, 2 * n, 2, w, ci, w};
    e = dgemm_strided(p2, g.nk, Wd + 2 * ((long)ci * n + ci), Td, Wd + 2 * (long)ci * n, true, st,
                      -1.0, false);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace exx

// ISDF fit kernels: Bloch-phase tables, the k-mesh autocorrelation that forms
// the fit metric S^m and the right-hand side Z^m, the FP64 Cholesky with pivot
// drop and the triangular inverse used for the least-squares solve.
#include <cmath>

#include "common.h"

namespace exx {

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------
exx_status get_tables(exx_context* h, const Geom& g, Tables* t, hipStream_t st) {
  int key[6] = {g.n[0], g.n[1], g.n[2], g.N[0], g.N[1], g.N[2]};
  size_t nroot = 0, ntw = 0;
  for (int a = 0; a < 3; ++a) {
    nroot += (size_t)g.n[a] * g.N[a];
    ntw += (size_t)g.n[a];
  }
  size_t bytes = nroot * sizeof(double2) + ntw * (sizeof(double2) + sizeof(float2)) + 256;
  bool same = h->tables != nullptr;
  for (int a = 0; a < 6; ++a) same = same && key[a] == h->tab_key[a];
  if (!same) {
    if (h->tables_cap < bytes) {
      if (h->tables) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_check(h, e, "hipStreamSynchronize");
        (void)hipFree(h->tables);
        h->tables = nullptr;
        h->tables_cap = 0;
      }
      hipError_t e = hipMalloc(&h->tables, bytes);
      if (e != hipSuccess) return fail(h, EXX_ERR_NOMEM, "table allocation failed");
      h->tables_cap = bytes;
    }
    std::vector<double2> r64;
    std::vector<double2> w64;
    std::vector<float2> w32;
    for (int a = 0; a < 3; ++a) {
      int Lr = g.n[a] * g.N[a];
      for (int s = 0; s < Lr; ++s) {
        double ang = -2.0 * M_PI * (double)s / (double)Lr;
        r64.push_back(make_double2(std::cos(ang), std::sin(ang)));
      }
    }
    for (int a = 0; a < 3; ++a) {
      for (int s = 0; s < g.n[a]; ++s) {
        double ang = -2.0 * M_PI * (double)s / (double)g.n[a];
        w64.push_back(make_double2(std::cos(ang), std::sin(ang)));
        w32.push_back(make_float2((float)std::cos(ang), (float)std::sin(ang)));
      }
    }
    char* base = (char*)h->tables;
    // synchronous upload: tables change only with the geometry
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(base, r64.data(), r64.size() * sizeof(double2), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(base + nroot * sizeof(double2), w64.data(), w64.size() * sizeof(double2),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(base + (nroot + ntw) * sizeof(double2), w32.data(), w32.size() * sizeof(float2),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_check(h, e, "table upload");
    for (int a = 0; a < 6; ++a) h->tab_key[a] = key[a];
  }
  const double2* r = (const double2*)h->tables;
  const double2* w = r + nroot;
  const float2* w2 = (const float2*)(w + ntw);
  size_t o1 = 0, o2 = 0;
  for (int a = 0; a < 3; ++a) {
    t->root[a] = r + o1;
    t->tw64[a] = w + o2;
    t->tw32[a] = w2 + o2;
    o1 += (size_t)g.n[a] * g.N[a];
    o2 += g.n[a];
  }
  return EXX_OK;
}

// ---------------------------------------------------------------------------
// k-mesh DFT helpers (register arrays, compile-time mesh)
// ---------------------------------------------------------------------------
template <typename T, int N>
__device__ __forceinline__ cplx<T> kroot(int t) {
  // e^{-2 pi i t / N}, 0 <= t < N
  if (N == 1) return mk<T>(1, 0);
  if (N == 2) return t ? mk<T>(-1, 0) : mk<T>(1, 0);
  if (N == 4) {
    switch (t & 3) {
      case 0: return mk<T>(1, 0);
      case 1: return mk<T>(0, -1);
      case 2: return mk<T>(-1, 0);
      default: return mk<T>(0, 1);
    }
  }
  if (N == 3) {
    const T s = (T)0.86602540378443864676372317075294;
    switch (t) {
      case 0: return mk<T>(1, 0);
      case 1: return mk<T>(-0.5, -s);
      default: return mk<T>(-0.5, s);
    }
  }
  double sn, cs;
  sincospi(-2.0 * (double)t / (double)N, &sn, &cs);
  return mk<T>((T)cs, (T)sn);
}

// forward DFT along one axis of an N1 x N2 x N3 register array
template <typename T, int N1, int N2, int N3, int AX>
__device__ __forceinline__ void kdft_axis(cplx<T>* a) {
  constexpr int NA = AX == 0 ? N1 : (AX == 1 ? N2 : N3);
  if (NA == 1) return;
  constexpr int ST = AX == 0 ? N2 * N3 : (AX == 1 ? N3 : 1);
  constexpr int NK = N1 * N2 * N3;
#pragma unroll
  for (int base = 0; base < NK; ++base) {
    // process each line once, from its first element
    const int pos = (base / ST) % NA;
    if (pos != 0) continue;
    cplx<T> tmp[NA];
#pragma unroll
    for (int t = 0; t < NA; ++t) tmp[t] = a[base + t * ST];
#pragma unroll
    for (int s = 0; s < NA; ++s) {
      cplx<T> acc = tmp[0];
#pragma unroll
      for (int t = 1; t < NA; ++t) acc = cadd<T>(acc, cmul<T>(tmp[t], kroot<T, NA>((s * t) % NA)));
      a[base + s * ST] = acc;
    }
  }
}

template <typename T, int N1, int N2, int N3>
__device__ __forceinline__ void kdft3(cplx<T>* a) {
  kdft_axis<T, N1, N2, N3, 2>(a);
  kdft_axis<T, N1, N2, N3, 1>(a);
  kdft_axis<T, N1, N2, N3, 0>(a);
}

// e^{-i q_m . r} for grid coordinates (g1, g2, g3), transfer (m1, m2, m3)
__device__ __forceinline__ double2 bloch(const double2* const* root, const int* nn, const int* NN,
                                         int m1, int m2, int m3, int g1, int g2, int g3) {
  double2 p = root[0][(m1 * g1) % (NN[0] * nn[0])];
  double2 b = root[1][(m2 * g2) % (NN[1] * nn[1])];
  double2 c = root[2][(m3 * g3) % (NN[2] * nn[2])];
  double2 pb = make_double2(p.x * b.x - p.y * b.y, p.x * b.y + p.y * b.x);
  return make_double2(pb.x * c.x - pb.y * c.y, pb.x * c.y + pb.y * c.x);
}

struct KcorrArgs {
  const double2* root[3];
  int n[3];
  int N[3];
};

// out[m][P][c] = e^{i q_m.(r_P - r_c)} (1/N_k) DFT_k(|DFT_k in|^2)[m]
//             = e^{i q_m.(r_P - r_c)} sum_n in[n][P][c] conj in[n+m][P][c]
template <typename T, int N1, int N2, int N3>
// `in` and `out` may alias (in place): each thread reads all of its inputs
// before it writes.
__global__ __launch_bounds__(256) void kcorr_kernel(const cplx<T>* in, cplx<T>* out, int ni, int ncol,
                                                    const int32_t* __restrict__ pts,
                                                    int cols_are_points, KcorrArgs ka) {
  constexpr int NK = N1 * N2 * N3;
  const long total = (long)ni * ncol;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int P = (int)(idx / ncol);
  const int c = (int)(idx % ncol);
  cplx<T> a[NK];
#pragma unroll
  for (int n = 0; n < NK; ++n) a[n] = in[(long)n * total + idx];
  if (NK > 1) {
    kdft3<T, N1, N2, N3>(a);
#pragma unroll
    for (int n = 0; n < NK; ++n) a[n] = mk<T>(a[n].x * a[n].x + a[n].y * a[n].y, 0);
    kdft3<T, N1, N2, N3>(a);
  } else {
    a[0] = mk<T>(a[0].x * a[0].x + a[0].y * a[0].y, 0);
  }
  const T inv = (T)1 / (T)NK;
  // grid coordinates of the point P and the column
  const int n23 = ka.n[1] * ka.n[2];
  int gp = pts[P];
  int p1 = gp / n23, p2 = (gp / ka.n[2]) % ka.n[1], p3 = gp % ka.n[2];
  int gc = cols_are_points ? pts[c] : c;
  int c1 = gc / n23, c2 = (gc / ka.n[2]) % ka.n[1], c3 = gc % ka.n[2];
#pragma unroll
  for (int m = 0; m < NK; ++m) {
    const int m1 = m / (N2 * N3), m2 = (m / N3) % N2, m3 = m % N3;
    cplx<T> v = cscale<T>(a[m], inv);
    if (m) {
      double2 fp = bloch(ka.root, ka.n, ka.N, m1, m2, m3, p1, p2, p3);  // e^{-iq.r_P}
      double2 fc = bloch(ka.root, ka.n, ka.N, m1, m2, m3, c1, c2, c3);  // e^{-iq.r_c}
      // e^{iq.(r_P - r_c)} = conj(fp) * fc
      double2 ph = make_double2(fp.x * fc.x + fp.y * fc.y, fp.x * fc.y - fp.y * fc.x);
      v = cmul<T>(v, mk<T>((T)ph.x, (T)ph.y));
    }
    out[(long)m * total + idx] = v;
  }
}

#define EXX_KMESH_LIST(X) \
  X(1, 1, 1)              \
  X(2, 2, 2)              \
  X(3, 3, 3)              \
  X(4, 4, 4)              \
  X(2, 1, 1)              \
  X(1, 2, 1)              \
  X(1, 1, 2)              \
  X(2, 2, 1)              \
  X(3, 2, 1)              \
  X(1, 2, 3)

bool kcorr_supported(const Geom& g) {
#define EXX_KSUP(a, b, c) \
  if (g.N[0] == a && g.N[1] == b && g.N[2] == c) return true;
  EXX_KMESH_LIST(EXX_KSUP)
#undef EXX_KSUP
  return false;
}

template <typename T>
hipError_t launch_kcorr(const Geom& g, const Tables& tb, const void* in, void* out, int ncol,
                        const int32_t* pts, bool cols_are_points, hipStream_t st) {
  KcorrArgs ka;
  for (int a = 0; a < 3; ++a) {
    ka.root[a] = tb.root[a];
    ka.n[a] = g.n[a];
    ka.N[a] = g.N[a];
  }
  long total = (long)g.ni * ncol;
  dim3 grid((unsigned)((total + 255) / 256));
#define EXX_KLAUNCH(a, b, c)                                                                    \
  if (g.N[0] == a && g.N[1] == b && g.N[2] == c) {                                              \
    hipLaunchKernelGGL((kcorr_kernel<T, a, b, c>), grid, dim3(256), 0, st, (const cplx<T>*)in,  \
                       (cplx<T>*)out, g.ni, ncol, pts, cols_are_points ? 1 : 0, ka);                             \
    return hipGetLastError();                                                                   \
  }
  EXX_KMESH_LIST(EXX_KLAUNCH)
#undef EXX_KLAUNCH
  return hipErrorInvalidValue;
}
template hipError_t launch_kcorr<double>(const Geom&, const Tables&, const void*, void*, int,
                                         const int32_t*, bool, hipStream_t);
template hipError_t launch_kcorr<float>(const Geom&, const Tables&, const void*, void*, int,
                                        const int32_t*, bool, hipStream_t);

// ---------------------------------------------------------------------------
// Cholesky in point order with pivot drop: one workgroup per transfer m.
// A (n x n, row-major) holds S^m on entry and L in its lower triangle on exit
// (dropped columns zero, strict upper triangle undefined).
// ---------------------------------------------------------------------------
constexpr int CH_NT = 1024;

__global__ __launch_bounds__(CH_NT) void chol_drop_kernel(double2* Aall, int n, int32_t* keepall,
                                                          int32_t* rank, double rel_tol) {
  const int m = blockIdx.x;
  double2* A = Aall + (long)m * n * n;
  int32_t* keep = keepall + (long)m * n;
  __shared__ double red[CH_NT];
  __shared__ int s_kept;
  const int tid = threadIdx.x;
  double mx = 0.0;
  for (int i = tid; i < n; i += CH_NT) mx = fmax(mx, A[(long)i * n + i].x);
  red[tid] = mx;
  __syncthreads();
  for (int s = CH_NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double tol = rel_tol * red[0];
  if (tid == 0) s_kept = 0;
  __syncthreads();
  for (int p = 0; p < n; ++p) {
    const double d = A[(long)p * n + p].x;
    const bool kp = (d >= tol) && isfinite(d) && d > 0.0;
    __syncthreads();  // every thread has read the pivot before it is overwritten
    if (!kp) {
      for (int i = p + tid; i < n; i += CH_NT) A[(long)i * n + p] = make_double2(0.0, 0.0);
      if (tid == 0) keep[p] = 0;
      __syncthreads();
      continue;
    }
    const double sd = sqrt(d), inv = 1.0 / sd;
    for (int i = p + tid; i < n; i += CH_NT) {
      double2 v = A[(long)i * n + p];
      A[(long)i * n + p] = (i == p) ? make_double2(sd, 0.0) : make_double2(v.x * inv, v.y * inv);
    }
    if (tid == 0) {
      keep[p] = 1;
      s_kept += 1;
    }
    __syncthreads();
    // trailing update of the lower triangle: A[i][j] -= L[i][p] conj(L[j][p]), p < j <= i
    const int w = n - p - 1;
    const long tot = (long)w * w;
    for (long e = tid; e < tot; e += CH_NT) {
      const int i = p + 1 + (int)(e / w);
      const int j = p + 1 + (int)(e % w);
      if (j > i) continue;
      double2 li = A[(long)i * n + p];
      double2 lj = A[(long)j * n + p];
      double2 a = A[(long)i * n + j];
      a.x -= li.x * lj.x + li.y * lj.y;
      a.y -= li.y * lj.x - li.x * lj.y;
      A[(long)i * n + j] = a;
    }
    __syncthreads();
  }
  if (tid == 0) rank[m] = s_kept;
}

hipError_t launch_chol_drop(const Geom& g, double2* A, int32_t* keep, int32_t* rank,
                            double rel_tol, hipStream_t st) {
  hipLaunchKernelGGL(chol_drop_kernel, dim3(g.nk), dim3(CH_NT), 0, st, A, g.ni, keep, rank,
                     rel_tol);
  return hipGetLastError();
}

// W = L_RR^{-1} scattered back to n x n (zero rows/cols for dropped points).
// One thread per column j, forward substitution down the column.
__global__ __launch_bounds__(256) void tri_inv_kernel(const double2* __restrict__ Lall,
                                                      const int32_t* __restrict__ keepall,
                                                      double2* __restrict__ Wall, int n) {
  const int m = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double2* L = Lall + (long)m * n * n;
  const int32_t* keep = keepall + (long)m * n;
  double2* W = Wall + (long)m * n * n;
  for (int i = 0; i < j; ++i) W[(long)i * n + j] = make_double2(0.0, 0.0);
  if (!keep[j]) {
    for (int i = j; i < n; ++i) W[(long)i * n + j] = make_double2(0.0, 0.0);
    return;
  }
  W[(long)j * n + j] = make_double2(1.0 / L[(long)j * n + j].x, 0.0);
  for (int i = j + 1; i < n; ++i) {
    if (!keep[i]) {
      W[(long)i * n + j] = make_double2(0.0, 0.0);
      continue;
    }
    double sx = 0.0, sy = 0.0;
    for (int k = j; k < i; ++k) {
      double2 l = L[(long)i * n + k];
      double2 w = W[(long)k * n + j];
      sx += l.x * w.x - l.y * w.y;
      sy += l.x * w.y + l.y * w.x;
    }
    const double inv = 1.0 / L[(long)i * n + i].x;
    W[(long)i * n + j] = make_double2(-sx * inv, -sy * inv);
  }
}

hipError_t launch_tri_inv(const Geom& g, const double2* Lf, const int32_t* keep, double2* W,
                          hipStream_t st) {
  dim3 grid((g.ni + 255) / 256, g.nk);
  hipLaunchKernelGGL(tri_inv_kernel, grid, dim3(256), 0, st, Lf, keep, W, g.ni);
  return hipGetLastError();
}

}  // namespace exx

// Kernels of the density derivative of the fitted exchange energy (the
// occupied-virtual block of Sec. 2.3, Eq. 19) and of the robust-fit exchange
// matrix (one fitted and one exact pair density per integral, the one-sided fit
// discussed in Sec. 5): the potentials of the fitted functions on the grid,
// their k-mesh cross-correlations with Gamma^n and G^n, the grid-length AO-basis
// contraction C = A B^H on the FP64 matrix cores (split over the grid, the slices
// added in order by the split-K reduction of gemm.hip), and the Hermitian
// assemblies. The transforms and the Gamma^n reuse the build's FFT and GEMM
// kernels.
#include "common.h"

namespace exx {

namespace {

struct GradMesh {
  int N[3];
  int nk;
  int src[64];  // P^m is slice src[m] of P ...
  int cj[64];   // ... conjugated where cj[m]
};

__device__ __forceinline__ int mesh_add(const GradMesh& a, int n, int m, int sign) {
  const int n1 = n / (a.N[1] * a.N[2]), n2 = (n / a.N[2]) % a.N[1], n3 = n % a.N[2];
  const int m1 = m / (a.N[1] * a.N[2]), m2 = (m / a.N[2]) % a.N[1], m3 = m % a.N[2];
  const int r1 = (n1 + sign * m1 + a.N[0]) % a.N[0];
  const int r2 = (n2 + sign * m2 + a.N[1]) % a.N[1];
  const int r3 = (n3 + sign * m3 + a.N[2]) % a.N[2];
  return (r1 * a.N[1] + r2) * a.N[2] + r3;
}

// a complex value of storage T as FP64
template <typename T>
__device__ __forceinline__ double2 ld2(const cplx<T>* __restrict__ p, long i) {
  const cplx<T> v = p[i];
  return make_double2((double)v.x, (double)v.y);
}

// F[m][P][g] <- conj(v^m(g) F[m][P][g]), F of storage T (FP64 arithmetic)
template <typename T>
__global__ __launch_bounds__(256) void kernel_scale_conj_kernel(cplx<T>* __restrict__ F,
                                                                const double* __restrict__ vt,
                                                                long per_m, long ng, long total) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const long m = e / per_m;
  const long g = e % ng;
  const double v = vt[m * ng + g];
  const double2 f = ld2<T>(F, e);
  F[e] = mk<T>((T)(v * f.x), (T)(-v * f.y));
}

struct PhaseArgs {
  const double2* root[3];  // e^{-2 pi i t / (N_a n_a)}
  int n[3], N[3];
  int ni;
  long ng;
  double scale;
  int nrb;      // workgroups per row (1024 grid points each)
  int rep[64];  // slice s holds transfer rep[s]
};

// X[m][P][r] <- scale e^{i q_m.(r_P - r)} X[m][P][r]: workgroup (row, rb) with
// row = (m, P), whose factor scale e^{i q.r_P} is uniform; a thread takes four grid
// points r (stride 256), each with e^{-i q.r} from the three axis tables
// (root_a[m_a c_a mod N_a n_a] = e^{-2 pi i m_a c_a / (N_a n_a)}).
template <typename T>
__global__ __launch_bounds__(256) void potential_phase_kernel(cplx<T>* __restrict__ X,
                                                              const int32_t* __restrict__ pts,
                                                              PhaseArgs a) {
  const int row = blockIdx.x / a.nrb, rb = blockIdx.x % a.nrb;
  const int P = row % a.ni, m = a.rep[row / a.ni];
  const int n2 = a.n[1], n3 = a.n[2], n23 = n2 * n3;
  const int gp = pts[P];
  const int mm[3] = {m / (a.N[1] * a.N[2]), (m / a.N[2]) % a.N[1], m % a.N[2]};
  const int pc[3] = {gp / n23, (gp / n3) % n2, gp % n3};
  // scale e^{i q.r_P} = scale prod_a conj(root_a[m_a p_a])
  double px = a.scale, py = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    const double2 f = a.root[ax][(mm[ax] * pc[ax]) % (a.N[ax] * a.n[ax])];
    const double tx = px * f.x + py * f.y;
    py = py * f.x - px * f.y;
    px = tx;
  }
  cplx<T>* Xr = X + (long)row * a.ng;
  const int ng = (int)a.ng;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = (rb * 4 + u) * 256 + threadIdx.x;
    if (r >= ng) break;
    const int c0 = r / n23, c1 = (r / n3) % n2, c2 = r % n3;
    const double2 f0 = a.root[0][(mm[0] * c0) % (a.N[0] * a.n[0])];
    const double2 f1 = a.root[1][(mm[1] * c1) % (a.N[1] * a.n[1])];
    const double2 f2 = a.root[2][(mm[2] * c2) % (a.N[2] * a.n[2])];
    double wx = f0.x * f1.x - f0.y * f1.y, wy = f0.x * f1.y + f0.y * f1.x;
    const double tx = wx * f2.x - wy * f2.y;
    wy = wx * f2.y + wy * f2.x;
    wx = tx;
    const double qx = px * wx - py * wy, qy = px * wy + py * wx;
    const double2 x = ld2<T>(Xr, r);
    Xr[r] = mk<T>((T)(qx * x.x - qy * x.y), (T)(qx * x.y + qy * x.x));
  }
}

// out[n][e] = sum_m [p^m(e) conj Q^{n+m}(e) + conj(p^m(e)) conj Q^{n-m}(e)],
// p^m = P^m, or conj(P^m) with CONJ_P; UP_ONLY keeps the first term
template <typename TP, bool CONJ_P, bool UP_ONLY>
__global__ __launch_bounds__(256) void grad_xcorr_kernel(const cplx<TP>* __restrict__ P,
                                                         const double2* __restrict__ Q,
                                                         double2* __restrict__ out, long elems,
                                                         GradMesh a) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= elems) return;
  for (int n = 0; n < a.nk; ++n) {
    double sx = 0.0, sy = 0.0;
    for (int m = 0; m < a.nk; ++m) {
      double2 p = ld2<TP>(P, (long)a.src[m] * elems + e);
      if (CONJ_P != (a.cj[m] != 0)) p.y = -p.y;
      const double2 qu = Q[(long)mesh_add(a, n, m, 1) * elems + e];
      // p conj(qu) (+ conj(p) conj(qd))
      sx += p.x * qu.x + p.y * qu.y;
      sy += p.y * qu.x - p.x * qu.y;
      if (!UP_ONLY) {
        const double2 qd = Q[(long)mesh_add(a, n, m, -1) * elems + e];
        sx += p.x * qd.x - p.y * qd.y;
        sy += -p.x * qd.y - p.y * qd.x;
      }
    }
    out[(long)n * elems + e] = make_double2(sx, sy);
  }
}

// The same sums with each element's N_k values of P and Q staged once in LDS
// (each lane reads back only its own column, so no barrier is needed): 2 N_k
// loads per element instead of up to 3 N_k^2. One wave per workgroup, 64
// elements; LDS 2 N_k x 64 x 16 bytes.
template <typename TP, bool CONJ_P, bool UP_ONLY>
__global__ __launch_bounds__(64) void grad_xcorr_lds_kernel(const cplx<TP>* __restrict__ P,
                                                            const double2* __restrict__ Q,
                                                            double2* __restrict__ out, long elems,
                                                            GradMesh a) {
  extern __shared__ double2 stage[];
  double2* Ps = stage;
  double2* Qs = stage + a.nk * 64;
  const int t = threadIdx.x;
  const long e = (long)blockIdx.x * 64 + t;
  const bool in = e < elems;
  for (int m = 0; m < a.nk; ++m) {
    double2 p = in ? ld2<TP>(P, (long)a.src[m] * elems + e) : make_double2(0.0, 0.0);
    if (CONJ_P != (a.cj[m] != 0)) p.y = -p.y;
    Ps[m * 64 + t] = p;
    Qs[m * 64 + t] = in ? Q[(long)m * elems + e] : make_double2(0.0, 0.0);
  }
  for (int n = 0; n < a.nk; ++n) {
    double sx = 0.0, sy = 0.0;
    for (int m = 0; m < a.nk; ++m) {
      const double2 p = Ps[m * 64 + t];
      const double2 qu = Qs[mesh_add(a, n, m, 1) * 64 + t];
      sx += p.x * qu.x + p.y * qu.y;
      sy += p.y * qu.x - p.x * qu.y;
      if (!UP_ONLY) {
        const double2 qd = Qs[mesh_add(a, n, m, -1) * 64 + t];
        sx += p.x * qd.x - p.y * qd.y;
        sy += -p.x * qd.y - p.y * qd.x;
      }
    }
    if (in) out[(long)n * elems + e] = make_double2(sx, sy);
  }
}

// index of k_n + sign * q_m on an N1 x N2 x N3 mesh (constant once unrolled)
template <int N1, int N2, int N3>
__device__ constexpr int mesh_add_c(int n, int m, int sign) {
  return ((n / (N2 * N3) + sign * (m / (N2 * N3)) + N1) % N1 * N2 +
          ((n / N3) % N2 + sign * ((m / N3) % N2) + N2) % N2) * N3 +
         (n % N3 + sign * (m % N3) + N3) % N3;
}

// The same sums (p^m = P^m) on a mesh known at compile time: each element's N_k
// values of P (storage TP, read as FP64) and Q are held in registers, every
// transfer index is a constant.
// MODE: XR_BOTH writes both terms, XR_UP the first term alone, XR_DOWN adds the
// second term to out (a larger mesh runs XR_UP then XR_DOWN, so that one pass
// holds no more than 2 N_k complex values in registers).
enum { XR_BOTH = 0, XR_UP = 1, XR_DOWN = 2 };
template <typename TP, int MODE, int N1, int N2, int N3>
__global__ __launch_bounds__(256) void grad_xcorr_reg_kernel(const cplx<TP>* __restrict__ P,
                                                            const double2* __restrict__ Q,
                                                            double2* __restrict__ out, long elems,
                                                            GradMesh a) {
  constexpr int NK = N1 * N2 * N3;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= elems) return;
  double2 p[NK], q[NK];
#pragma unroll
  for (int m = 0; m < NK; ++m) {
    p[m] = ld2<TP>(P, (long)a.src[m] * elems + e);
    if (a.cj[m]) p[m].y = -p[m].y;
    q[m] = Q[(long)m * elems + e];
  }
#pragma unroll
  for (int n = 0; n < NK; ++n) {
    double sx = 0.0, sy = 0.0;
    if (MODE == XR_DOWN) {
      const double2 o = out[(long)n * elems + e];
      sx = o.x;
      sy = o.y;
    }
#pragma unroll
    for (int m = 0; m < NK; ++m) {
      if (MODE != XR_DOWN) {
        const double2 qu = q[mesh_add_c<N1, N2, N3>(n, m, 1)];
        sx += p[m].x * qu.x + p[m].y * qu.y;
        sy += p[m].y * qu.x - p[m].x * qu.y;
      }
      if (MODE != XR_UP) {
        const double2 qd = q[mesh_add_c<N1, N2, N3>(n, m, -1)];
        sx += p[m].x * qd.x - p[m].y * qd.y;
        sy += -p[m].x * qd.y - p[m].y * qd.x;
      }
    }
    out[(long)n * elems + e] = make_double2(sx, sy);
  }
}

// Kg[n][mu][nu] = -(N_k/4) (Ac[n][mu][nu] + conj(Ac[n][nu][mu]))
__global__ __launch_bounds__(256) void grad_assemble_kernel(const double2* __restrict__ Ac,
                                                            double2* __restrict__ Kg, int nao,
                                                            long total, double f) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const long nn = (long)nao * nao;
  const long n = e / nn;
  const int mu = (int)((e % nn) / nao), nu = (int)(e % nao);
  const double2 a = Ac[e], b = Ac[n * nn + (long)nu * nao + mu];
  Kg[e] = make_double2(f * (a.x + b.x), f * (a.y - b.y));
}

// robust K: Kr[n][mu][nu] = conj(Ac[n][mu][nu]) + Ac[n][nu][mu] - Kr[n][mu][nu],
// Ac = conj of the one-sided term, Kr holding the fitted K on entry
__global__ __launch_bounds__(256) void robust_assemble_kernel(const double2* __restrict__ Ac,
                                                              double2* __restrict__ Kr, int nao,
                                                              long total) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const long nn = (long)nao * nao;
  const long n = e / nn;
  const int mu = (int)((e % nn) / nao), nu = (int)(e % nao);
  const double2 a = Ac[e], b = Ac[n * nn + (long)nu * nao + mu], k = Kr[e];
  Kr[e] = make_double2(a.x + b.x - k.x, -a.y + b.y - k.y);
}

}  // namespace

hipError_t launch_kernel_scale_conj(const Geom& g, void* F, const double* vt, hipStream_t st,
                                    bool f32) {
  const long per_m = (long)g.ni * g.ng, total = per_m * g.nk;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (f32)
    hipLaunchKernelGGL(kernel_scale_conj_kernel<float>, grid, dim3(256), 0, st, (float2*)F, vt,
                       per_m, (long)g.ng, total);
  else
    hipLaunchKernelGGL(kernel_scale_conj_kernel<double>, grid, dim3(256), 0, st, (double2*)F, vt,
                       per_m, (long)g.ng, total);
  return hipGetLastError();
}

hipError_t launch_potential_phase(const Geom& g, const Tables& tb, void* X, const int32_t* pts,
                                  double scale, hipStream_t st, bool f32, const int* rep, int ns) {
  if (!rep) ns = g.nk;
  PhaseArgs a;
  for (int ax = 0; ax < 3; ++ax) {
    a.root[ax] = tb.root[ax];
    a.n[ax] = g.n[ax];
    a.N[ax] = g.N[ax];
  }
  a.ni = g.ni;
  a.ng = g.ng;
  a.scale = scale;
  a.nrb = (int)((g.ng + 1023) / 1024);
  for (int m = 0; m < 64; ++m) a.rep[m] = m < ns ? (rep ? rep[m] : m) : 0;
  const long nblk = (long)ns * g.ni * a.nrb;
  if (f32)
    hipLaunchKernelGGL(potential_phase_kernel<float>, dim3((unsigned)nblk), dim3(256), 0, st,
                       (float2*)X, pts, a);
  else
    hipLaunchKernelGGL(potential_phase_kernel<double>, dim3((unsigned)nblk), dim3(256), 0, st,
                       (double2*)X, pts, a);
  return hipGetLastError();
}

namespace {

template <typename TP>
hipError_t grad_xcorr_run(const Geom& g, const void* P, bool conj_p, const void* Q, void* out,
                          long elems, hipStream_t st, bool up_only, const int* src,
                          const int* cj) {
  GradMesh gm;
  for (int ax = 0; ax < 3; ++ax) gm.N[ax] = g.N[ax];
  gm.nk = g.nk;
  for (int m = 0; m < 64; ++m) {
    gm.src[m] = src && m < g.nk ? src[m] : m;
    gm.cj[m] = cj && m < g.nk ? cj[m] : 0;
  }
  const dim3 grid((unsigned)((elems + 255) / 256));
  const cplx<TP>* p = (const cplx<TP>*)P;
  const double2* q = (const double2*)Q;
  double2* o = (double2*)out;
  if (!conj_p) {  // register-resident forms for the common small meshes
#define EXX_XREG(a, b, c)                                                                      \
  if (g.N[0] == a && g.N[1] == b && g.N[2] == c) {                                             \
    if (up_only)                                                                               \
      hipLaunchKernelGGL((grad_xcorr_reg_kernel<TP, XR_UP, a, b, c>), grid, dim3(256), 0, st, p,   \
                         q, o, elems, gm);                                                     \
    else                                                                                       \
      hipLaunchKernelGGL((grad_xcorr_reg_kernel<TP, XR_BOTH, a, b, c>), grid, dim3(256), 0, st, p, \
                         q, o, elems, gm);                                                     \
    return hipGetLastError();                                                                  \
  }
    EXX_XREG(1, 1, 1)
    EXX_XREG(2, 1, 1)
    EXX_XREG(1, 2, 1)
    EXX_XREG(1, 1, 2)
    EXX_XREG(2, 2, 1)
    EXX_XREG(2, 1, 2)
    EXX_XREG(1, 2, 2)
    EXX_XREG(2, 2, 2)
    EXX_XREG(3, 1, 1)
    EXX_XREG(1, 3, 1)
    EXX_XREG(1, 1, 3)
    EXX_XREG(3, 2, 1)
    EXX_XREG(1, 2, 3)
    EXX_XREG(2, 3, 1)
#undef EXX_XREG
    if (g.N[0] == 3 && g.N[1] == 3 && g.N[2] == 3) {  // two passes: 2 x 27 values each
      hipLaunchKernelGGL((grad_xcorr_reg_kernel<TP, XR_UP, 3, 3, 3>), grid, dim3(256), 0, st, p, q,
                         o, elems, gm);
      if (!up_only)
        hipLaunchKernelGGL((grad_xcorr_reg_kernel<TP, XR_DOWN, 3, 3, 3>), grid, dim3(256), 0, st, p,
                           q, o, elems, gm);
      return hipGetLastError();
    }
  }
  if (g.nk <= 32) {  // LDS staging, at most 64 KiB per workgroup
    const dim3 gl((unsigned)((elems + 63) / 64));
    const size_t lds = sizeof(double2) * 2 * 64 * (size_t)g.nk;
    if (up_only) {
      if (conj_p)
        hipLaunchKernelGGL((grad_xcorr_lds_kernel<TP, true, true>), gl, dim3(64), lds, st, p, q, o,
                           elems, gm);
      else
        hipLaunchKernelGGL((grad_xcorr_lds_kernel<TP, false, true>), gl, dim3(64), lds, st, p, q, o,
                           elems, gm);
    } else {
      if (conj_p)
        hipLaunchKernelGGL((grad_xcorr_lds_kernel<TP, true, false>), gl, dim3(64), lds, st, p, q,
                           o, elems, gm);
      else
        hipLaunchKernelGGL((grad_xcorr_lds_kernel<TP, false, false>), gl, dim3(64), lds, st, p, q,
                           o, elems, gm);
    }
    return hipGetLastError();
  }
  if (up_only) {
    if (conj_p)
      hipLaunchKernelGGL((grad_xcorr_kernel<TP, true, true>), grid, dim3(256), 0, st, p, q, o,
                         elems, gm);
    else
      hipLaunchKernelGGL((grad_xcorr_kernel<TP, false, true>), grid, dim3(256), 0, st, p, q, o,
                         elems, gm);
  } else {
    if (conj_p)
      hipLaunchKernelGGL((grad_xcorr_kernel<TP, true, false>), grid, dim3(256), 0, st, p, q, o,
                         elems, gm);
    else
      hipLaunchKernelGGL((grad_xcorr_kernel<TP, false, false>), grid, dim3(256), 0, st, p, q, o,
                         elems, gm);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grad_xcorr(const Geom& g, const void* P, bool conj_p, const void* Q, void* out,
                             long elems, hipStream_t st, bool up_only, bool p_f32, const int* src,
                             const int* cj) {
  if (p_f32) return grad_xcorr_run<float>(g, P, conj_p, Q, out, elems, st, up_only, src, cj);
  return grad_xcorr_run<double>(g, P, conj_p, Q, out, elems, st, up_only, src, cj);
}

hipError_t launch_robust_assemble(const Geom& g, const void* Ac, void* K, hipStream_t st) {
  const long total = (long)g.nk * g.nao * g.nao;
  hipLaunchKernelGGL(robust_assemble_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     st, (const double2*)Ac, (double2*)K, g.nao, total);
  return hipGetLastError();
}

hipError_t launch_grad_assemble(const Geom& g, const void* Ac, void* Kg, hipStream_t st) {
  const long total = (long)g.nk * g.nao * g.nao;
  hipLaunchKernelGGL(grad_assemble_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     (const double2*)Ac, (double2*)Kg, g.nao, total, -0.25 * g.nk);
  return hipGetLastError();
}

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// One slice [k0, k1) of C = A B^H (A [M][K], B [N][K], FP64 complex, K the long
// axis): a workgroup of 2 x 2 waves computes a 64 x 64 tile, each wave a 32 x 32
// tile of 2 x 2 blocks of 16 x 16 on the FP64 matrix cores with three real
// products per complex one (Re x conj y = T1 + T2, Im = T3 - T1 + T2 from
// T1 = sum xr yr, T2 = sum xi yi, T3 = sum (xr + xi)(yr - yi)). A lane feeds two
// consecutive k of its row per step (eight k per step); loads are clamped into
// the arrays and masked to zero past the slice, and three steps' operands are
// in flight while a step's products issue. Work item w = ((b ns + s) tm + ti)
// tn + tj, laid out XCD-contiguously so that the tiles of one slice share an L2.
__global__ __launch_bounds__(256, 2) void zgemm_abh_kernel(
    const double2* __restrict__ A, long lda, long sA, const double2* __restrict__ B, long ldb,
    long sB, double2* __restrict__ part, int M, int N, int K, int kc, int tm, int tn, int batch,
    int ns, long nwork, long nwork_pad) {
  const long w = (blockIdx.x % 8) * (nwork_pad / 8) + blockIdx.x / 8;
  if (w >= nwork) return;
  const int tj = (int)(w % tn);
  long r = w / tn;
  const int ti = (int)(r % tm);
  r /= tm;
  const int sk = (int)(r % ns);
  const long b = r / ns;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, gq = lane >> 4;
  const int P0 = ti * 64 + (wave & 1) * 32, Q0 = tj * 64 + (wave >> 1) * 32;
  const long k0 = (long)sk * kc, k1 = min((long)K, k0 + kc);
  const double2* Ab = A + b * sA;
  const double2* Bb = B + b * sB;
  long xrow[2], yrow[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    xrow[i] = (long)min(P0 + 16 * i + li, M - 1) * lda;
    yrow[i] = (long)min(Q0 + 16 * i + li, N - 1) * ldb;
  }
  d4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) t1[i][j] = t2[i][j] = t3[i][j] = d4{0, 0, 0, 0};
  // operands of the step at kb; NPF steps are in flight in registers (a slot is
  // refilled with the step NPF ahead as soon as its products are issued)
  constexpr int NPF = 3;
  auto load = [&](long kb, double2 (*x)[2], double2 (*y)[2]) {
    const long g = kb + 2 * gq;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const long gi = min(g + t, (long)K - 1);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        x[i][t] = Ab[xrow[i] + gi];
        y[i][t] = Bb[yrow[i] + gi];
      }
    }
  };
  double2 xb[NPF][2][2], yb[NPF][2][2];
#pragma unroll
  for (int sl = 0; sl < NPF; ++sl) load(k0 + 8 * sl, xb[sl], yb[sl]);
  for (long kc0 = k0; kc0 < k1; kc0 += 8 * NPF) {
#pragma unroll
    for (int sl = 0; sl < NPF; ++sl) {
      const long kb = kc0 + 8 * sl;
      const long g = kb + 2 * gq;
      double2 x[2][2], y[2][2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const bool ok = g + t < k1;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          x[i][t] = ok ? xb[sl][i][t] : make_double2(0.0, 0.0);
          y[i][t] = ok ? yb[sl][i][t] : make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        double ys[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) ys[j] = y[j][t].x - y[j][t].y;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const double xs = x[i][t].x + x[i][t].y;
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            t1[i][j] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(x[i][t].x, y[j][t].x, t1[i][j], 0, 0, 0);
            t2[i][j] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(x[i][t].y, y[j][t].y, t2[i][j], 0, 0, 0);
            t3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs, ys[j], t3[i][j], 0, 0, 0);
          }
        }
      }
      // refill the slot (clamped into the arrays past the end; masked at use)
      __builtin_amdgcn_sched_barrier(0);
      load(kb + 8 * NPF, xb[sl], yb[sl]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // register v of a lane holds row 4 v + lane/16, column lane%16 of a block
  double2* out = part + ((long)sk * batch + b) * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int P = P0 + 16 * i + 4 * v + gq, Q = Q0 + 16 * j + li;
        if (P < M && Q < N)
          out[(long)P * N + Q] = make_double2(t1[i][j][v] + t2[i][j][v],
                                              t3[i][j][v] - t1[i][j][v] + t2[i][j][v]);
      }
}

}  // namespace

hipError_t zgemm_abh_parts(int M, int N, int K, int batch, const void* A, long lda, long sA,
                           const void* B, long ldb, long sB, void* part, int ns, int kc,
                           hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0 || batch <= 0 || ns <= 0 || kc <= 0 || kc % 8)
    return hipErrorInvalidValue;
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  const long nwork = (long)batch * ns * tm * tn;
  const long pad = (nwork + 7) / 8 * 8;
  hipLaunchKernelGGL(zgemm_abh_kernel, dim3((unsigned)pad), dim3(256), 0, st, (const double2*)A,
                     lda, sA, (const double2*)B, ldb, sB, (double2*)part, M, N, K, kc, tm, tn,
                     batch, ns, nwork, pad);
  return hipGetLastError();
}

}  // namespace exx

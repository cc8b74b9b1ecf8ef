// Coulomb matrices of the interpolating vectors in reciprocal space:
//   V^m_PQ = (Omega/N_g^2) sum_g v^m(g) F_P(g) conj F_Q(g),  v^m = 4 pi/|K|^2,
// as a Hermitian rank-N_g update split over grid chunks. sqrt(v^m(g)) scales
// both operands while they are staged in LDS; the kernel value is generated
// on the fly from the K-box rule. A reduction kernel sums the chunks, mirrors
// the upper triangle and applies the Bloch-gauge phase.
#include <cmath>

#include "common.h"

namespace exx {

namespace {

constexpr int TM = 64, TK = 16, NT = 256;

struct CoulArgs {
  double L[3];
  int n[3];
  int N[3];
  int ng, ni, nk, nsplit, chunk, ntile;
};

__device__ __forceinline__ double sqrt_kernel(const CoulArgs& a, int m, long g) {
  const int n23 = a.n[1] * a.n[2];
  const int g1 = (int)(g / n23), g2 = (int)((g / a.n[2]) % a.n[1]), g3 = (int)(g % a.n[2]);
  const int m1 = m / (a.N[1] * a.N[2]), m2 = (m / a.N[2]) % a.N[1], m3 = m % a.N[2];
  const int k1 = wrap_sym(a.N[0] * g1 + m1, a.N[0] * a.n[0]);
  const int k2 = wrap_sym(a.N[1] * g2 + m2, a.N[1] * a.n[1]);
  const int k3 = wrap_sym(a.N[2] * g3 + m3, a.N[2] * a.n[2]);
  const double K1 = k1 * (2.0 * M_PI / (a.N[0] * a.L[0]));
  const double K2 = k2 * (2.0 * M_PI / (a.N[1] * a.L[1]));
  const double K3 = k3 * (2.0 * M_PI / (a.N[2] * a.L[2]));
  const double kk = K1 * K1 + K2 * K2 + K3 * K3;
  // sqrt(4 pi / |K|^2)
  return kk > 0.0 ? 3.5449077018110320546 / sqrt(kk) : 0.0;
}

// partial[m][s][P][Q] = sum_{g in chunk s} w(g) F[m][P][g] conj F[m][Q][g] for lower tiles
template <typename T>
__global__ __launch_bounds__(NT) void coulomb_partial_kernel(const cplx<T>* __restrict__ F,
                                                             cplx<T>* __restrict__ part,
                                                             CoulArgs a) {
  __shared__ cplx<T> As[TK][TM];
  __shared__ cplx<T> Bs[TK][TM];
  __shared__ T sw[TK];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  // triangular tile index -> (ti, tj), ti >= tj
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tj = t;
  const int m = blockIdx.y / a.nsplit, s = blockIdx.y % a.nsplit;
  const long g0 = (long)s * a.chunk;
  const long g1 = min((long)a.ng, g0 + a.chunk);
  const cplx<T>* Fm = F + (long)m * a.ni * a.ng;
  const int i0 = ti * TM, j0 = tj * TM;
  cplx<T> acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = mk<T>(0, 0);
  for (long k0 = g0; k0 < g1; k0 += TK) {
    if (tid < TK) {
      long g = k0 + tid;
      sw[tid] = (g < g1) ? (T)sqrt_kernel(a, m, g) : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (TM * TK) / NT; ++r) {
      const int e = tid + NT * r;
      const int i = e / TK, k = e % TK;
      const long g = k0 + k;
      cplx<T> va = mk<T>(0, 0), vb = mk<T>(0, 0);
      if (g < g1) {
        if (i0 + i < a.ni) va = cscale<T>(Fm[(long)(i0 + i) * a.ng + g], sw[k]);
        if (j0 + i < a.ni) vb = cscale<T>(Fm[(long)(j0 + i) * a.ng + g], sw[k]);
      }
      As[k][i] = va;
      Bs[k][i] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      cplx<T> x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = As[kk][ty + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] = Bs[kk][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // x * conj(y)
          acc[u][v].x += x[u].x * y[v].x + x[u].y * y[v].y;
          acc[u][v].y += x[u].y * y[v].x - x[u].x * y[v].y;
        }
    }
    __syncthreads();
  }
  cplx<T>* out = part + ((long)m * a.nsplit + s) * a.ni * a.ni;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int P = i0 + ty + 16 * u;
    if (P >= a.ni) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int Q = j0 + tx + 16 * v;
      if (Q < a.ni) out[(long)P * a.ni + Q] = acc[u][v];
    }
  }
}

// ---------------------------------------------------------------------------
// Matrix-core version of the partial contraction. A lane (row li = lane % 16,
// group gq = lane / 16) loads 4 consecutive grid values of its row, so the k
// index of MFMA step t is g0 + 4 gq + t for both operands (the k order of a
// sum is free). X = v(g) F_P (rows P), Y = conj F_Q (rows Q):
//   Re += Re X Re F_Q + Im X Im F_Q,  Im += Im X Re F_Q - Re X Im F_Q.
// FP64 storage: v_mfma_f64_16x16x4_f64. FP32 storage: v_mfma_f32_16x16x4_f32
// whose FP32 accumulators are flushed into FP64 every FLUSH grid points.
// ---------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int MW = 2;       // 16-blocks per wave in each direction (wave tile 32 x 32)
constexpr int MTILE = 64;   // workgroup tile (2 x 2 waves)
constexpr int FLUSH = 64;   // FP32 accumulation length before the FP64 flush

__device__ __forceinline__ double kernel_v(const CoulArgs& a, int m1, int m2, int m3, long g) {
  const int n23 = a.n[1] * a.n[2];
  const int g1 = (int)(g / n23), g2 = (int)((g / a.n[2]) % a.n[1]), g3 = (int)(g % a.n[2]);
  const int k1 = wrap_sym(a.N[0] * g1 + m1, a.N[0] * a.n[0]);
  const int k2 = wrap_sym(a.N[1] * g2 + m2, a.N[1] * a.n[1]);
  const int k3 = wrap_sym(a.N[2] * g3 + m3, a.N[2] * a.n[2]);
  const double K1 = k1 * (2.0 * M_PI / (a.N[0] * a.L[0]));
  const double K2 = k2 * (2.0 * M_PI / (a.N[1] * a.L[1]));
  const double K3 = k3 * (2.0 * M_PI / (a.N[2] * a.L[2]));
  const double kk = K1 * K1 + K2 * K2 + K3 * K3;
  return kk > 0.0 ? 4.0 * M_PI / kk : 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void coulomb_mfma_kernel(const cplx<T>* __restrict__ F,
                                                           double2* __restrict__ part, CoulArgs a,
                                                           long nwork, long nwork_pad) {
  const long per = nwork_pad / 8;
  const long w = (blockIdx.x % 8) * per + blockIdx.x / 8;  // XCD-contiguous ranges
  if (w >= nwork) return;
  int tile = (int)(w % a.ntile);
  const long ms = w / a.ntile;
  const int m = (int)(ms / a.nsplit), s = (int)(ms % a.nsplit);
  int ti = 0;
  while (tile > ti) {
    tile -= ti + 1;
    ++ti;
  }
  const int tj = tile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, gq = lane >> 4;
  const int P0 = ti * MTILE + (wave & 1) * (MW * 16);
  const int Q0 = tj * MTILE + (wave >> 1) * (MW * 16);
  const long g0 = (long)s * a.chunk;
  const long g1 = min((long)a.ng, g0 + a.chunk);
  const cplx<T>* Fm = F + (long)m * a.ni * a.ng;
  const int m1 = m / (a.N[1] * a.N[2]), m2 = (m / a.N[2]) % a.N[1], m3 = m % a.N[2];

  constexpr bool F64 = sizeof(T) == 8;
  double accr[MW][MW][4], acci[MW][MW][4];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) accr[i][j][v] = acci[i][j][v] = 0.0;
  d4v dr[MW][MW], di[MW][MW];
  f4v fr[MW][MW], fi[MW][MW];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      dr[i][j] = d4v{0, 0, 0, 0};
      di[i][j] = d4v{0, 0, 0, 0};
      fr[i][j] = f4v{0, 0, 0, 0};
      fi[i][j] = f4v{0, 0, 0, 0};
    }

  int since = 0;
  for (long k0 = g0; k0 < g1; k0 += 16) {
    const long gb = k0 + 4 * gq;
    T vv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) vv[t] = (gb + t < g1) ? (T)kernel_v(a, m1, m2, m3, gb + t) : (T)0;
    cplx<T> x[MW][4], y[MW][4];
#pragma unroll
    for (int i = 0; i < MW; ++i) {
      const int P = P0 + 16 * i + li;
      const int Q = Q0 + 16 * i + li;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool ok = gb + t < g1;
        cplx<T> xv = (ok && P < a.ni) ? Fm[(long)P * a.ng + gb + t] : mk<T>(0, 0);
        x[i][t] = mk<T>(xv.x * vv[t], xv.y * vv[t]);
        y[i][t] = (ok && Q < a.ni) ? Fm[(long)Q * a.ng + gb + t] : mk<T>(0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < MW; ++i)
#pragma unroll
        for (int j = 0; j < MW; ++j) {
          if constexpr (F64) {
            dr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i][t].x, y[j][t].x, dr[i][j], 0, 0, 0);
            dr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i][t].y, y[j][t].y, dr[i][j], 0, 0, 0);
            di[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i][t].y, y[j][t].x, di[i][j], 0, 0, 0);
            di[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x[i][t].x, y[j][t].y, di[i][j], 0, 0, 0);
          } else {
            fr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)x[i][t].x, (float)y[j][t].x, fr[i][j], 0, 0, 0);
            fr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)x[i][t].y, (float)y[j][t].y, fr[i][j], 0, 0, 0);
            fi[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)x[i][t].y, (float)y[j][t].x, fi[i][j], 0, 0, 0);
            fi[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-(float)x[i][t].x, (float)y[j][t].y, fi[i][j], 0, 0, 0);
          }
        }
    if constexpr (!F64) {
      since += 16;
      if (since >= FLUSH) {
        since = 0;
#pragma unroll
        for (int i = 0; i < MW; ++i)
#pragma unroll
          for (int j = 0; j < MW; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              accr[i][j][v] += (double)fr[i][j][v];
              acci[i][j][v] += (double)fi[i][j][v];
            }
            fr[i][j] = f4v{0, 0, 0, 0};
            fi[i][j] = f4v{0, 0, 0, 0};
          }
      }
    }
  }
  double2* out = part + ((long)m * a.nsplit + s) * a.ni * a.ni;
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // output rows: f64 MFMA register v holds row 4 v + lane/16, f32 holds 4 (lane/16) + v
      const int P = P0 + 16 * i + (F64 ? 4 * v + gq : 4 * gq + v);
      if (P >= a.ni) continue;
#pragma unroll
      for (int j = 0; j < MW; ++j) {
        const int Q = Q0 + 16 * j + li;
        if (Q >= a.ni) continue;
        double re, im;
        if constexpr (F64) {
          re = dr[i][j][v];
          im = di[i][j][v];
        } else {
          re = accr[i][j][v] + (double)fr[i][j][v];
          im = acci[i][j][v] + (double)fi[i][j][v];
        }
        out[(long)P * a.ni + Q] = make_double2(re, im);
      }
    }
}

struct ReduceArgs {
  const double2* root[3];
  int n[3];
  int N[3];
  int ni, nsplit;
  double scale;
};

// V[m][P][Q] = scale * e^{-i q_m.(r_P - r_Q)} sum_s part (mirrored for upper tiles)
__global__ __launch_bounds__(256) void coulomb_reduce_kernel(const double2* __restrict__ part,
                                                             const int32_t* __restrict__ pts,
                                                             double2* __restrict__ V,
                                                             ReduceArgs a) {
  const long nn = (long)a.ni * a.ni;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (idx >= nn) return;
  const int P = (int)(idx / a.ni), Q = (int)(idx % a.ni);
  const bool lower = (P / MTILE) >= (Q / MTILE);
  const long src = lower ? ((long)P * a.ni + Q) : ((long)Q * a.ni + P);
  double sx = 0.0, sy = 0.0;
  for (int s = 0; s < a.nsplit; ++s) {
    const double2 v = part[((long)m * a.nsplit + s) * nn + src];
    sx += v.x;
    sy += v.y;
  }
  if (!lower) sy = -sy;
  sx *= a.scale;
  sy *= a.scale;
  if (m) {
    const int m1 = m / (a.N[1] * a.N[2]), m2 = (m / a.N[2]) % a.N[1], m3 = m % a.N[2];
    const int n23 = a.n[1] * a.n[2];
    const int gp = pts[P], gq = pts[Q];
    int pc[3] = {gp / n23, (gp / a.n[2]) % a.n[1], gp % a.n[2]};
    int qc[3] = {gq / n23, (gq / a.n[2]) % a.n[1], gq % a.n[2]};
    int mm[3] = {m1, m2, m3};
    // e^{-i q.r_P} * conj(e^{-i q.r_Q})
    double px = 1.0, py = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
      const int Lr = a.N[ax] * a.n[ax];
      double2 fp = a.root[ax][(mm[ax] * pc[ax]) % Lr];
      double2 fq = a.root[ax][(mm[ax] * qc[ax]) % Lr];
      double2 r = make_double2(fp.x * fq.x + fp.y * fq.y, fp.y * fq.x - fp.x * fq.y);
      double tx = px * r.x - py * r.y;
      py = px * r.y + py * r.x;
      px = tx;
    }
    double vx = sx * px - sy * py;
    sy = sx * py + sy * px;
    sx = vx;
  }
  V[(long)m * nn + idx] = make_double2(sx, sy);
}

}  // namespace

int coulomb_nsplit(const Geom& g) {
  const int nt = (g.ni + MTILE - 1) / MTILE;
  const long tiles = (long)nt * (nt + 1) / 2 * g.nk;
  long ns = (4096 + tiles - 1) / tiles;
  const long maxs = (g.ng + 1023) / 1024;  // keep chunks >= ~1k points
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  return (int)ns;
}

size_t coulomb_partial_bytes(const Geom& g, int nsplit) {
  return (size_t)g.nk * nsplit * g.ni * g.ni * sizeof(double2);
}

template <typename T>
hipError_t launch_coulomb(const Geom& g, const Tables& tb, const void* F, const int32_t* pts,
                          void* partial, int nsplit, double2* V, hipStream_t st) {
  CoulArgs a;
  for (int i = 0; i < 3; ++i) {
    a.L[i] = g.L[i];
    a.n[i] = g.n[i];
    a.N[i] = g.N[i];
  }
  a.ng = g.ng;
  a.ni = g.ni;
  a.nk = g.nk;
  a.nsplit = nsplit;
  a.chunk = (int)((((long)g.ng + nsplit - 1) / nsplit + FLUSH - 1) / FLUSH * FLUSH);
  const int nt = (g.ni + MTILE - 1) / MTILE;
  a.ntile = nt * (nt + 1) / 2;
  const long nwork = (long)a.ntile * g.nk * nsplit;
  const long pad = (nwork + 7) / 8 * 8;
  hipLaunchKernelGGL(coulomb_mfma_kernel<T>, dim3((unsigned)pad), dim3(256), 0, st,
                     (const cplx<T>*)F, (double2*)partial, a, nwork, pad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ReduceArgs r;
  for (int i = 0; i < 3; ++i) {
    r.root[i] = tb.root[i];
    r.n[i] = g.n[i];
    r.N[i] = g.N[i];
  }
  r.ni = g.ni;
  r.nsplit = nsplit;
  r.scale = g.omega / ((double)g.ng * (double)g.ng);
  const long nn = (long)g.ni * g.ni;
  hipLaunchKernelGGL(coulomb_reduce_kernel, dim3((unsigned)((nn + 255) / 256), g.nk), dim3(256), 0,
                     st, (const double2*)partial, pts, V, r);
  return hipGetLastError();
}

template hipError_t launch_coulomb<double>(const Geom&, const Tables&, const void*, const int32_t*,
                                           void*, int, double2*, hipStream_t);
template hipError_t launch_coulomb<float>(const Geom&, const Tables&, const void*, const int32_t*,
                                          void*, int, double2*, hipStream_t);

}  // namespace exx

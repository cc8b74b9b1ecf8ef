// Coulomb matrices of the interpolating vectors in reciprocal space:
//   V^m_PQ = (Omega/N_g^2) sum_g v^m(g) F_P(g) conj F_Q(g),  v^m = 4 pi/|K|^2,
// as a Hermitian rank-N_g update split over grid chunks. sqrt(v^m(g)) scales
// both operands while they are staged in LDS; the kernel value is generated
// on the fly from the K-box rule. A reduction kernel sums the chunks, mirrors
// the upper triangle and applies the Bloch-gauge phase.
#include <cmath>
#include <type_traits>

#include "common.h"

namespace exx {

namespace {

struct CoulArgs {
  double L[3];
  int n[3];
  int N[3];
  int ng, ni, nk, nsplit, chunk, ntile;
};

// ---------------------------------------------------------------------------
// Matrix-core version of the partial contraction. A lane (row li = lane % 16,
// group gq = lane / 16) loads TPL consecutive grid values of its row, so the k
// index of MFMA step t is g0 + TPL gq + t for both operands (the k order of a
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
constexpr int TPL = 2;      // consecutive grid values per lane and chunk
constexpr int CK = 4 * TPL; // grid points per chunk

// Accumulators of one wave tile (MW x MW blocks of 16x16, real and imaginary).
template <bool F64MMA>
struct CAcc;

template <>
struct CAcc<true> {  // FP64 matrix cores, FP64 accumulation
  d4v r[MW][MW], i[MW][MW];
  __device__ void init() {
#pragma unroll
    for (int a = 0; a < MW; ++a)
#pragma unroll
      for (int b = 0; b < MW; ++b) r[a][b] = i[a][b] = d4v{0, 0, 0, 0};
  }
  // (xr + i xi) * conj(yr + i yi) for block (a, b)
  __device__ void mac(int a, int b, double xr, double xi, double yr, double yi) {
    r[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, yr, r[a][b], 0, 0, 0);
    r[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, yi, r[a][b], 0, 0, 0);
    i[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, yr, i[a][b], 0, 0, 0);
    i[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xr, yi, i[a][b], 0, 0, 0);
  }
  __device__ void chunk_done(int) {}
  __device__ double re(int a, int b, int v) const { return r[a][b][v]; }
  __device__ double im(int a, int b, int v) const { return i[a][b][v]; }
  // register v of a lane holds row 4 v + lane/16 of the block
  static __device__ int row(int gq, int v) { return 4 * v + gq; }
};

template <>
struct CAcc<false> {  // FP32 matrix cores, FP32 accumulation flushed into FP64
  f4v r[MW][MW], i[MW][MW];
  double sr[MW][MW][4], si[MW][MW][4];
  int since;
  __device__ void init() {
    since = 0;
#pragma unroll
    for (int a = 0; a < MW; ++a)
#pragma unroll
      for (int b = 0; b < MW; ++b) {
        r[a][b] = i[a][b] = f4v{0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < 4; ++v) sr[a][b][v] = si[a][b][v] = 0.0;
      }
  }
  __device__ void mac(int a, int b, float xr, float xi, float yr, float yi) {
    r[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, yr, r[a][b], 0, 0, 0);
    r[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi, yi, r[a][b], 0, 0, 0);
    i[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi, yr, i[a][b], 0, 0, 0);
    i[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-xr, yi, i[a][b], 0, 0, 0);
  }
  __device__ void flush() {
#pragma unroll
    for (int a = 0; a < MW; ++a)
#pragma unroll
      for (int b = 0; b < MW; ++b) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          sr[a][b][v] += (double)r[a][b][v];
          si[a][b][v] += (double)i[a][b][v];
        }
        r[a][b] = i[a][b] = f4v{0, 0, 0, 0};
      }
  }
  __device__ void chunk_done(int npts) {
    since += npts;
    if (since >= FLUSH) {
      since = 0;
      flush();
    }
  }
  __device__ double re(int a, int b, int v) const { return sr[a][b][v] + (double)r[a][b][v]; }
  __device__ double im(int a, int b, int v) const { return si[a][b][v] + (double)i[a][b][v]; }
  // register v of a lane holds row 4 (lane/16) + v of the block
  static __device__ int row(int gq, int v) { return 4 * gq + v; }
};

// T: storage of F. F64MMA: FP64 matrix cores (exact products of FP32 inputs, FP64
// accumulation) even for FP32 storage; otherwise FP32 matrix cores with flushes.
template <typename T, bool F64MMA>
__global__ __launch_bounds__(256, 2) void coulomb_mfma_kernel(const cplx<T>* __restrict__ F,
                                                           double2* __restrict__ part, CoulArgs a,
                                                           long nwork, long nwork_pad) {
  using TO = typename std::conditional<F64MMA, double, float>::type;
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

  // per-axis squared components of K for this transfer: |K|^2 = T0[g1] + T1[g2] + T2[g3]
  __shared__ double sK2[3][128];
  for (int e = threadIdx.x; e < a.n[0] + a.n[1] + a.n[2]; e += 256) {
    const int ax = e < a.n[0] ? 0 : (e < a.n[0] + a.n[1] ? 1 : 2);
    const int gi = e - (ax == 0 ? 0 : (ax == 1 ? a.n[0] : a.n[0] + a.n[1]));
    const int mi = ax == 0 ? m1 : (ax == 1 ? m2 : m3);
    const int kap = wrap_sym(a.N[ax] * gi + mi, a.N[ax] * a.n[ax]);
    const double K = kap * (2.0 * M_PI / (a.N[ax] * a.L[ax]));
    sK2[ax][gi] = K * K;
  }
  __syncthreads();
  const int n2 = a.n[1], n3 = a.n[2];
  // v^m at TPL consecutive grid points starting at gb (int32 index arithmetic)
  auto vchunk = [&](long gb, double* vv) {
    int g = (int)gb;
    int q = g / n3;
    int c3 = g - q * n3;
    int c1 = q / n2;
    int c2 = q - c1 * n2;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
      const double kk = sK2[0][c1] + sK2[1][c2] + sK2[2][c3];
      vv[t] = (gb + t < g1 && kk > 0.0) ? 4.0 * M_PI / kk : 0.0;
      if (++c3 == n3) {
        c3 = 0;
        if (++c2 == n2) {
          c2 = 0;
          if (++c1 == a.n[0]) c1 = 0;
        }
      }
    }
  };

  CAcc<F64MMA> acc;
  acc.init();
  // double-buffered register pipeline over CK-point grid chunks
  cplx<T> rx[2][MW][TPL], ry[2][MW][TPL];
  auto load = [&](long k0, cplx<T> (*xx)[TPL], cplx<T> (*yy)[TPL]) {
    const long gb = k0 + TPL * gq;
#pragma unroll
    for (int i = 0; i < MW; ++i) {
      const int P = P0 + 16 * i + li;
      const int Q = Q0 + 16 * i + li;
#pragma unroll
      for (int t = 0; t < TPL; ++t) {
        const bool ok = gb + t < g1;
        xx[i][t] = (ok && P < a.ni) ? Fm[(long)P * a.ng + gb + t] : mk<T>(0, 0);
        yy[i][t] = (ok && Q < a.ni) ? Fm[(long)Q * a.ng + gb + t] : mk<T>(0, 0);
      }
    }
  };
  auto compute = [&](long k0, cplx<T> (*xx)[TPL], cplx<T> (*yy)[TPL]) {
    const long gb = k0 + TPL * gq;
    double vd[TPL];
    vchunk(gb, vd);
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
      const TO vv = (TO)vd[t];
#pragma unroll
      for (int i = 0; i < MW; ++i) {
        const TO xr = (TO)xx[i][t].x * vv, xi = (TO)xx[i][t].y * vv;
#pragma unroll
        for (int j = 0; j < MW; ++j) acc.mac(i, j, xr, xi, (TO)yy[j][t].x, (TO)yy[j][t].y);
      }
    }
    acc.chunk_done(CK);
  };
  // ping-pong between two statically indexed register buffers
  if (g0 < g1) load(g0, rx[0], ry[0]);
  for (long k0 = g0; k0 < g1; k0 += 2 * CK) {
    if (k0 + CK < g1) load(k0 + CK, rx[1], ry[1]);
    compute(k0, rx[0], ry[0]);
    if (k0 + CK >= g1) break;
    if (k0 + 2 * CK < g1) load(k0 + 2 * CK, rx[0], ry[0]);
    compute(k0 + CK, rx[1], ry[1]);
  }
  double2* out = part + ((long)m * a.nsplit + s) * a.ni * a.ni;
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int P = P0 + 16 * i + CAcc<F64MMA>::row(gq, v);
      if (P >= a.ni) continue;
#pragma unroll
      for (int j = 0; j < MW; ++j) {
        const int Q = Q0 + 16 * j + li;
        if (Q < a.ni) out[(long)P * a.ni + Q] = make_double2(acc.re(i, j, v), acc.im(i, j, v));
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
                          void* partial, int nsplit, double2* V, bool f64mma, hipStream_t st) {
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
  if (f64mma || sizeof(T) == 8)
    hipLaunchKernelGGL((coulomb_mfma_kernel<T, true>), dim3((unsigned)pad), dim3(256), 0, st,
                       (const cplx<T>*)F, (double2*)partial, a, nwork, pad);
  else
    hipLaunchKernelGGL((coulomb_mfma_kernel<T, false>), dim3((unsigned)pad), dim3(256), 0, st,
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
                                           void*, int, double2*, bool, hipStream_t);
template hipError_t launch_coulomb<float>(const Geom&, const Tables&, const void*, const int32_t*,
                                          void*, int, double2*, bool, hipStream_t);

}  // namespace exx

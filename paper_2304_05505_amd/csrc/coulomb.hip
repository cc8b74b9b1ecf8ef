// Coulomb matrices of the interpolating vectors in reciprocal space:
//   V^m_PQ = (Omega/N_g^2) sum_g v^m(g) F_P(g) conj F_Q(g),  v^m = 4 pi/|K|^2,
// as a Hermitian rank-N_g update split over grid chunks on the matrix cores.
// The kernel values v^m(g) (K-box rule, K = 0 dropped) are tabulated once per
// call; a reduction kernel sums the chunks, mirrors the upper triangle and
// applies the Bloch-gauge phase.
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
  long fstride;  // elements of F per slice (0: every slice reads the same F)
  int rep[64];   // transfer of each slice (slices may hold a subset of the transfers)
};

// ---------------------------------------------------------------------------
// Matrix-core partial contraction. A lane (row li = lane % 16, group
// gq = lane / 16) loads TPL consecutive grid values of its row, so the k index
// of MFMA step t is g0 + TPL gq + t for both operands (the k order of a sum is
// free). X = v(g) F_P (rows P), Y = conj F_Q (rows Q):
//   Re = sum Re X Re F_Q + Im X Im F_Q,  Im = sum Im X Re F_Q - Re X Im F_Q,
// on the FP64 matrix cores (v_mfma_f64_16x16x4_f64) in Gauss's three-product
// form: T1 = sum Re X Re F_Q, T2 = sum Im X Im F_Q, T3 = sum (Re X + Im X)
// (Re F_Q - Im F_Q), then Re = T1 + T2 and Im = T3 - T1 + T2. FP32-stored F is
// widened at use, so its products are exact and the accumulation is FP64.
// ---------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int MW = 2;      // 16-blocks per wave in each direction (wave tile 32 x 32)
constexpr int WTILE = MW * 16;  // wave tile
constexpr int CALIGN = 64; // grid chunks of the split start at multiples of this

// v^m(g) for every transfer m and grid point g: 4 pi/|K|^2 with the K-box
// representative of each axis, 0 for K = 0
__global__ __launch_bounds__(256) void coulomb_vtab_kernel(double* __restrict__ vt, CoulArgs a) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  const int sl = blockIdx.y, m = a.rep[sl];
  if (g >= a.ng) return;
  const int n23 = a.n[1] * a.n[2];
  const int gc[3] = {(int)(g / n23), (int)((g / a.n[2]) % a.n[1]), (int)(g % a.n[2])};
  const int mm[3] = {m / (a.N[1] * a.N[2]), (m / a.N[2]) % a.N[1], m % a.N[2]};
  double kk = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    const int kap = wrap_sym(a.N[ax] * gc[ax] + mm[ax], a.N[ax] * a.n[ax]);
    const double K = kap * (2.0 * M_PI / (a.N[ax] * a.L[ax]));
    kk += K * K;
  }
  vt[(long)sl * a.ng + g] = kk > 0.0 ? 4.0 * M_PI / kk : 0.0;
}

// Real path: the kernel table over the kept half grid (z index g3 < hz of the
// [x][y][hz] layout) with the pairing weights of G <-> G' = -G - 2 q_m: 2 where
// the partner lies outside the kept set or after G, 1 where G' = G, 0 for
// partners already counted and for z columns past the transfer's half range.
__global__ __launch_bounds__(256) void coulomb_vtab_half_kernel(double* __restrict__ vt,
                                                                CoulArgs a, int hz) {
  const long gh = (long)blockIdx.x * 256 + threadIdx.x;
  const int sl = blockIdx.y, m = a.rep[sl];
  const long ngh = (long)a.n[0] * a.n[1] * hz;
  if (gh >= ngh) return;
  const int g1 = (int)(gh / ((long)a.n[1] * hz)), g2 = (int)((gh / hz) % a.n[1]),
            g3 = (int)(gh % hz);
  const int mm[3] = {m / (a.N[1] * a.N[2]), (m / a.N[2]) % a.N[1], m % a.N[2]};
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  const int h3 = mm[2] == 0 ? n3 / 2 + 1 : (n3 + 1) / 2;
  int w = 0;
  if (g3 < h3) {
    const int p3 = ((-g3 - mm[2]) % n3 + n3) % n3;
    if (p3 != g3) {
      w = 2;
    } else {
      const int p1 = ((-g1 - mm[0]) % n1 + n1) % n1, p2 = ((-g2 - mm[1]) % n2 + n2) % n2;
      const long lin = (long)g1 * n2 + g2, plin = (long)p1 * n2 + p2;
      w = lin < plin ? 2 : (lin == plin ? 1 : 0);
    }
  }
  double v = 0.0;
  if (w) {
    const int gc[3] = {g1, g2, g3};
    double kk = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
      const int kap = wrap_sym(a.N[ax] * gc[ax] + mm[ax], a.N[ax] * a.n[ax]);
      const double K = kap * (2.0 * M_PI / (a.N[ax] * a.L[ax]));
      kk += K * K;
    }
    v = kk > 0.0 ? w * 4.0 * M_PI / kk : 0.0;
  }
  vt[(long)sl * ngh + gh] = v;
}

// One wave computes one 32 x 32 wave tile (2 x 2 blocks of 16 x 16) of the
// lower triangle for one transfer m and one grid chunk [g0, g1). MASK selects
// the blocks that are computed and stored (bit 2 i + j for block row i, column
// j). On diagonal tiles without block (0, 1) the row and column operands are
// the same rows of F and are loaded once. Loads are unconditional with clamped
// indices (clamped rows only feed outputs that are never stored; grid points
// past the chunk get v = 0 at use), and NPF chunks are in flight in registers.
// VEC (FP32 storage, even N_g): a lane's two grid values of a row are one
// aligned 16-byte load, so a load instruction touches each row's cache line
// once. stage: this wave's 3 x 256 doubles of LDS (epilogue staging).
// RE: accumulate only Re(X conj Y) = Re X Re Y + Im X Im Y (two MFMAs into one
// accumulator; the real path, whose Coulomb matrices are real).
template <typename T, int MASK, bool VEC, int NPF, bool RE = false>
__device__ __forceinline__ void coulomb_wave_tile(const cplx<T>* __restrict__ Fm,
                                                  const double* __restrict__ vm,
                                                  double2* __restrict__ out, const CoulArgs& a,
                                                  int P0, int Q0, long g0, long g1,
                                                  double* stage) {
  constexpr int TPL = 2;  // grid values per lane and MFMA step group
  constexpr int CK = 4 * TPL;
  constexpr bool DIAG = (MASK & 2) == 0;
  constexpr bool XU[MW] = {(MASK & 3) != 0, (MASK & 12) != 0};
  constexpr bool YU[MW] = {(MASK & 5) != 0, (MASK & 10) != 0};
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, gq = lane >> 4;
  // 32-bit row offsets from the uniform base Fm (N_ISDF N_g < 2^31 is checked by
  // the launcher)
  unsigned xrow[MW], yrow[MW];
#pragma unroll
  for (int i = 0; i < MW; ++i) {
    const int P = min(P0 + 16 * i + li, a.ni - 1), Q = min(Q0 + 16 * i + li, a.ni - 1);
    xrow[i] = (unsigned)P * (unsigned)a.ng;
    yrow[i] = (unsigned)Q * (unsigned)a.ng;
  }
  d4v t1[MW][MW], t2[MW][MW], t3[MW][MW];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < MW; ++j) t1[i][j] = t2[i][j] = t3[i][j] = d4v{0, 0, 0, 0};
  cplx<T> fx[NPF][MW][TPL], fy[NPF][MW][TPL];
  double fv[NPF][TPL];
  auto load = [&](long k0, cplx<T> (*xx)[TPL], cplx<T> (*yy)[TPL], double* vv) {
    const long gb = k0 + TPL * gq;
    if constexpr (VEC) {
      // gb is even; past the end the base is clamped to N_g - 2 (v = 0 at use)
      const unsigned g = (unsigned)min(gb, (long)a.ng - 2);
      const double2 v2 = *(const double2*)(vm + g);
      vv[0] = v2.x;
      vv[1] = v2.y;
#pragma unroll
      for (int i = 0; i < MW; ++i) {
        if (DIAG ? (XU[i] || YU[i]) : XU[i]) {
          const float4 q = *(const float4*)(Fm + xrow[i] + g);
          xx[i][0] = mk<T>(q.x, q.y);
          xx[i][1] = mk<T>(q.z, q.w);
        }
        if (!DIAG && YU[i]) {
          const float4 q = *(const float4*)(Fm + yrow[i] + g);
          yy[i][0] = mk<T>(q.x, q.y);
          yy[i][1] = mk<T>(q.z, q.w);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < TPL; ++t) {
        const unsigned g = (unsigned)min(gb + t, (long)a.ng - 1);
        vv[t] = vm[g];
#pragma unroll
        for (int i = 0; i < MW; ++i) {
          if (DIAG ? (XU[i] || YU[i]) : XU[i]) xx[i][t] = Fm[xrow[i] + g];
          if (!DIAG && YU[i]) yy[i][t] = Fm[yrow[i] + g];
        }
      }
    }
  };
  const long nchunk = (g1 - g0 + CK - 1) / CK;
#pragma unroll
  for (int sl = 0; sl < NPF; ++sl) load(g0 + (long)sl * CK, fx[sl], fy[sl], fv[sl]);
  // FP32 storage: let the first loads land before the loop, so that the wait
  // counts at the loop head see only the loop's own refills (otherwise the
  // differently ordered prologue forces a full wait there on every iteration)
  if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_waitcnt(0);
  for (long c = 0; c < nchunk; c += NPF) {
#pragma unroll
    for (int sl = 0; sl < NPF; ++sl) {
      const long k0 = g0 + (c + sl) * CK;
      const long gb = k0 + TPL * gq;
#pragma unroll
      for (int t = 0; t < TPL; ++t) {
        const double vv = (gb + t < g1) ? fv[sl][t] : 0.0;
        double yr[MW], yi[MW], ys[MW];
#pragma unroll
        for (int j = 0; j < MW; ++j) {
          if (!YU[j]) continue;
          const cplx<T> y = DIAG ? fx[sl][j][t] : fy[sl][j][t];
          yr[j] = (double)y.x;
          yi[j] = (double)y.y;
          if (!RE) ys[j] = yr[j] - yi[j];
        }
#pragma unroll
        for (int i = 0; i < MW; ++i) {
          if (!XU[i]) continue;
          const double xr = (double)fx[sl][i][t].x * vv, xi = (double)fx[sl][i][t].y * vv;
          const double xs = RE ? 0.0 : xr + xi;
#pragma unroll
          for (int j = 0; j < MW; ++j) {
            if (!(MASK & (1 << (2 * i + j)))) continue;
            t1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, yr[j], t1[i][j], 0, 0, 0);
            if (RE) {
              t1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, yi[j], t1[i][j], 0, 0, 0);
            } else {
              t2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, yi[j], t2[i][j], 0, 0, 0);
              t3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs, ys[j], t3[i][j], 0, 0, 0);
            }
          }
        }
      }
      // refill the slot (clamped loads past the end are discarded by v = 0)
      __builtin_amdgcn_sched_barrier(0);
      load(k0 + NPF * CK, fx[sl], fy[sl], fv[sl]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // D layout: register v of a lane holds row 4 v + lane/16 of the block.
  // Combining T1..T3 needs the accumulators in VALU registers: each lane
  // round-trips its own values through its wave's LDS slice (LDS accesses of
  // one wave complete in order), which keeps the accumulators in the matrix
  // registers during the loop.
  typedef __attribute__((address_space(3))) volatile double lds_f64;
  lds_f64* s1 = (lds_f64*)stage;
  lds_f64* s2 = s1 + 64 * 4;
  lds_f64* s3 = s2 + 64 * 4;
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      if (!(MASK & (1 << (2 * i + j)))) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        s1[v * 64 + lane] = t1[i][j][v];
        if (!RE) {
          s2[v * 64 + lane] = t2[i][j][v];
          s3[v * 64 + lane] = t3[i][j][v];
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int P = P0 + 16 * i + 4 * v + gq;
        const int Q = Q0 + 16 * j + li;
        const double x1 = s1[v * 64 + lane];
        if (RE) {
          if (P < a.ni && Q < a.ni) out[(long)P * a.ni + Q] = make_double2(x1, 0.0);
        } else {
          const double x2 = s2[v * 64 + lane], x3 = s3[v * 64 + lane];
          if (P < a.ni && Q < a.ni) out[(long)P * a.ni + Q] = make_double2(x1 + x2, x3 - x1 + x2);
        }
      }
    }
}

// (transfer m, grid split s, lower-triangle tile t) of work item w; the order of
// w is XCD-contiguous so that the tiles of one (m, s) share an L2
__device__ __forceinline__ void coulomb_work(long w, const CoulArgs& a, int& m, int& s, int& ti,
                                             int& tj) {
  int tile = (int)(w % a.ntile);
  const long ms = w / a.ntile;
  m = (int)(ms / a.nsplit);
  s = (int)(ms % a.nsplit);
  ti = 0;
  while (tile > ti) {
    tile -= ti + 1;
    ++ti;
  }
  tj = tile;
}

// FP64 storage: 64 x 64 tiles of 2 x 2 waves, whose waves share the rows of F
// through L1 (the redundant upper-triangle blocks of diagonal tiles are
// computed; the reduction reads only P >= Q).
template <bool RE>
__global__ __launch_bounds__(256, 2) void coulomb_kernel_f64(const double2* __restrict__ F,
                                                          const double* __restrict__ vt,
                                                          double2* __restrict__ part, CoulArgs a,
                                                          long nwork, long nwork_pad) {
  const long w = (blockIdx.x % 8) * (nwork_pad / 8) + blockIdx.x / 8;
  if (w >= nwork) return;
  int m, s, ti, tj;
  coulomb_work(w, a, m, s, ti, tj);
  const int wave = threadIdx.x >> 6;
  const int P0 = ti * 2 * WTILE + (wave & 1) * WTILE;
  const int Q0 = tj * 2 * WTILE + (wave >> 1) * WTILE;
  const long g0 = (long)s * a.chunk;
  const long g1 = min((long)a.ng, g0 + a.chunk);
  __shared__ double stage[4 * 3 * 64 * 4];
  coulomb_wave_tile<double, 0xF, false, 2, RE>(
      F + (long)m * a.fstride, vt + (long)m * a.ng,
      part + ((long)m * a.nsplit + s) * a.ni * a.ni, a, P0, Q0, g0, g1,
      stage + wave * 3 * 64 * 4);
}

// FP32 storage: one wave per workgroup and 32 x 32 tiles, so that only the
// blocks that hold needed entries are computed (the all-upper block of a
// diagonal tile and block rows past N_ISDF are skipped) without leaving a SIMD
// of a multi-wave workgroup short of waves.
template <bool VEC, bool RE>
__global__ __launch_bounds__(64) void coulomb_kernel_f32(const float2* __restrict__ F,
                                                      const double* __restrict__ vt,
                                                      double2* __restrict__ part, CoulArgs a,
                                                      long nwork, long nwork_pad) {
  const long w = (blockIdx.x % 8) * (nwork_pad / 8) + blockIdx.x / 8;
  if (w >= nwork) return;
  int m, s, ti, tj;
  coulomb_work(w, a, m, s, ti, tj);
  const int P0 = ti * WTILE, Q0 = tj * WTILE;
  const long g0 = (long)s * a.chunk;
  const long g1 = min((long)a.ng, g0 + a.chunk);
  const float2* Fm = F + (long)m * a.fstride;
  const double* vm = vt + (long)m * a.ng;
  double2* out = part + ((long)m * a.nsplit + s) * a.ni * a.ni;
  constexpr int NPF = 4;
  __shared__ double stage[3 * 64 * 4];
  const bool row1 = P0 + 16 < a.ni;  // block row 1 holds rows below N_ISDF
  if (ti != tj) {
    if (row1)
      coulomb_wave_tile<float, 0xF, VEC, NPF, RE>(Fm, vm, out, a, P0, Q0, g0, g1, stage);
    else
      coulomb_wave_tile<float, 0x3, VEC, NPF, RE>(Fm, vm, out, a, P0, Q0, g0, g1, stage);
  } else {
    if (row1)
      coulomb_wave_tile<float, 0xD, VEC, NPF, RE>(Fm, vm, out, a, P0, Q0, g0, g1, stage);
    else
      coulomb_wave_tile<float, 0x1, VEC, NPF, RE>(Fm, vm, out, a, P0, Q0, g0, g1, stage);
  }
}

// Real path: one wave per 64 x 64 tile (4 x 4 blocks of 16 x 16) of the lower
// triangle, which halves the operand loads per MFMA and the re-reads of F
// against 32 x 32 tiles. T: storage of the half-grid transform; a lane loads 16
// bytes of a row per k-step (two consecutive FP32 values, which needs an even
// number of points, or one FP64 value). NR: block rows that hold rows below
// N_ISDF (1..4); DIAG: a diagonal tile, whose column operand rows are its row
// operand rows and whose blocks above the diagonal are skipped. Accumulates
// Re(X conj Y) = Re X Re Y + Im X Im Y in FP64 (two MFMAs per block and value).
template <typename T, int NR, bool DIAG>
__device__ __forceinline__ void coulomb_tile64_re(const cplx<T>* __restrict__ Fm,
                                                  const double* __restrict__ vm,
                                                  double2* __restrict__ out, const CoulArgs& a,
                                                  int P0, int Q0, long g0, long g1,
                                                  double* stage) {
  constexpr int TPL = 16 / sizeof(cplx<T>);  // grid values per lane and k-step
  constexpr int NPF = 2, CK = 4 * TPL;
  constexpr int NC = DIAG ? NR : 4;  // column blocks read
  using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, gq = lane >> 4;
  unsigned xrow[NR], yrow[NC];
#pragma unroll
  for (int i = 0; i < NR; ++i)
    xrow[i] = (unsigned)min(P0 + 16 * i + li, a.ni - 1) * (unsigned)a.ng;
#pragma unroll
  for (int j = 0; j < NC; ++j)
    yrow[j] = (unsigned)min(Q0 + 16 * j + li, a.ni - 1) * (unsigned)a.ng;
  d4v acc[NR][NC];
#pragma unroll
  for (int i = 0; i < NR; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[i][j] = d4v{0, 0, 0, 0};
  V fx[NPF][NR], fy[NPF][DIAG ? 1 : NC];
  double fv[NPF][TPL];
  // the lane's first grid index; past the end the base is clamped to N_g - TPL
  // and the values are discarded (v = 0 at use)
  auto load = [&](long k0, V* xx, V* yy, double* vv) {
    const unsigned g = (unsigned)min(k0 + TPL * gq, (long)a.ng - TPL);
    if constexpr (TPL == 2) {
      const double2 v2 = *(const double2*)(vm + g);
      vv[0] = v2.x;
      vv[1] = v2.y;
    } else {
      vv[0] = vm[g];
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) xx[i] = *(const V*)(Fm + xrow[i] + g);
    if constexpr (!DIAG) {
#pragma unroll
      for (int j = 0; j < NC; ++j) yy[j] = *(const V*)(Fm + yrow[j] + g);
    }
  };
  // value t of a lane's 16 bytes as (re, im) in FP64
  auto re = [](const V& q, int t) -> double {
    if constexpr (sizeof(T) == 4) return (double)(t ? q.z : q.x);
    else return q.x;
  };
  auto im = [](const V& q, int t) -> double {
    if constexpr (sizeof(T) == 4) return (double)(t ? q.w : q.y);
    else return q.y;
  };
  const long nchunk = (g1 - g0 + CK - 1) / CK;
#pragma unroll
  for (int sl = 0; sl < NPF; ++sl) load(g0 + (long)sl * CK, fx[sl], fy[sl], fv[sl]);
  __builtin_amdgcn_s_waitcnt(0);  // as in coulomb_wave_tile
  for (long c = 0; c < nchunk; c += NPF) {
#pragma unroll
    for (int sl = 0; sl < NPF; ++sl) {
      const long k0 = g0 + (c + sl) * CK;
      const long gb = k0 + TPL * gq;
#pragma unroll
      for (int t = 0; t < TPL; ++t) {
        const double vv = (gb + t < g1) ? fv[sl][t] : 0.0;
        double yr[NC], yi[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const V& q = DIAG ? fx[sl][j] : fy[sl][DIAG ? 0 : j];
          yr[j] = re(q, t);
          yi[j] = im(q, t);
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          const double xr = re(fx[sl][i], t) * vv, xi = im(fx[sl][i], t) * vv;
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            if (DIAG && j > i) continue;
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, yr[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, yi[j], acc[i][j], 0, 0, 0);
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      load(k0 + NPF * CK, fx[sl], fy[sl], fv[sl]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // register v of a lane holds row 4 v + lane/16 of a block; each lane
  // round-trips its own values through the wave's LDS slice (keeps the
  // accumulators in matrix registers during the loop)
  typedef __attribute__((address_space(3))) volatile double lds_f64;
  lds_f64* s1 = (lds_f64*)stage;
#pragma unroll
  for (int i = 0; i < NR; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (DIAG && j > i) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) s1[v * 64 + lane] = acc[i][j][v];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int P = P0 + 16 * i + 4 * v + gq;
        const int Q = Q0 + 16 * j + li;
        const double x = s1[v * 64 + lane];
        if (P < a.ni && Q < a.ni) out[(long)P * a.ni + Q] = make_double2(x, 0.0);
      }
    }
}

// one wave per (transfer, grid split, 64 x 64 lower-triangle tile)
template <typename T>
__global__ __launch_bounds__(64) void coulomb_kernel_t64(const cplx<T>* __restrict__ F,
                                                         const double* __restrict__ vt,
                                                         double2* __restrict__ part, CoulArgs a,
                                                         long nwork, long nwork_pad) {
  const long w = (blockIdx.x % 8) * (nwork_pad / 8) + blockIdx.x / 8;
  if (w >= nwork) return;
  int m, s, ti, tj;
  coulomb_work(w, a, m, s, ti, tj);
  const int P0 = ti * 64, Q0 = tj * 64;
  const long g0 = (long)s * a.chunk;
  const long g1 = min((long)a.ng, g0 + a.chunk);
  const cplx<T>* Fm = F + (long)m * a.fstride;
  const double* vm = vt + (long)m * a.ng;
  double2* out = part + ((long)m * a.nsplit + s) * a.ni * a.ni;
  __shared__ double stage[64 * 4];
  const int nr = min(4, (a.ni - P0 + 15) / 16);
#define EXX_T64(R)                                                                 \
  case R:                                                                          \
    if (ti == tj)                                                                  \
      coulomb_tile64_re<T, R, true>(Fm, vm, out, a, P0, Q0, g0, g1, stage);        \
    else                                                                           \
      coulomb_tile64_re<T, R, false>(Fm, vm, out, a, P0, Q0, g0, g1, stage);       \
    break;
  switch (nr) {
    EXX_T64(1)
    EXX_T64(2)
    EXX_T64(3)
    default:
      if (ti == tj)
        coulomb_tile64_re<T, 4, true>(Fm, vm, out, a, P0, Q0, g0, g1, stage);
      else
        coulomb_tile64_re<T, 4, false>(Fm, vm, out, a, P0, Q0, g0, g1, stage);
  }
#undef EXX_T64
}

// ---------------------------------------------------------------------------
// BF16 matrix-core forms (FP32-stored transforms). v_mfma_f32_16x16x32_bf16: a
// k-step covers 16 complex grid points; lane group lk = lane / 16 holds points
// g0 + 4 lk .. g0 + 4 lk + 3 of its row as k values (Re, Im, Re, Im, ...), the
// same pairing on both operands, so that with X = v(g) F_P and Y = F_Q
//   sum_k X_k Y_k   = sum_g Re X Re Y + Im X Im Y = Re(X conj Y),
// and with the column operand rearranged per point to (-Im Y, Re Y)
//   sum_k X_k Y'_k  = sum_g Im X Re Y - Re X Im Y = Im(X conj Y).
// X is formed in FP32 and rounded to bfloat16 (ties to even). SPLIT: every
// operand is carried as hi + lo with hi = bf16(x), lo = bf16(x - hi) (16
// significant bits), and a product is hi hi + hi lo + lo hi (the dropped lo lo
// term is ~2^-16 relative). The FP32 matrix accumulators are added into FP64
// registers every BF_FLUSH k-steps (256 points) and zeroed, so no FP32 sum runs
// over more than 256 points; the partial sums leave the kernel in FP64.
// ---------------------------------------------------------------------------
typedef __bf16 cb_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short cb_u16x8 __attribute__((ext_vector_type(8)));
typedef float cb_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ cb_bf16x8 cb_as_bf16(cb_u16x8 v) {
  cb_bf16x8 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

// x = hi + lo to 16 significant bits
__device__ __forceinline__ void cb_split(float x, unsigned short& hi, unsigned short& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - __uint_as_float((unsigned)hi << 16));
}

constexpr int BF_FLUSH = 16;  // k-steps (of 16 points) per FP32 accumulation
constexpr int BF_NPF = 2;     // k-steps of operands in flight in registers

// lower-triangle 32 x 32 wave tile (MASK as coulomb_wave_tile) of transfer m and
// grid chunk [g0, g1). VEC: N_g % 4 == 0, so a lane's four points of a row are
// two aligned 16-byte loads, and a lane group's points are all inside or all
// outside a chunk (chunks start at multiples of 64). Loads past the end of the
// grid are clamped and their points get v = 0. RE: Re(X conj Y) only.
template <int MASK, bool VEC, bool SPLIT, bool RE>
__device__ __forceinline__ void coulomb_tile_bf16(const float2* __restrict__ Fm,
                                                  const double* __restrict__ vm,
                                                  double2* __restrict__ out, const CoulArgs& a,
                                                  int P0, int Q0, long g0, long g1) {
  constexpr bool DIAG = (MASK & 2) == 0;
  constexpr bool XU[MW] = {(MASK & 3) != 0, (MASK & 12) != 0};
  constexpr bool YU[MW] = {(MASK & 5) != 0, (MASK & 10) != 0};
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  unsigned xrow[MW], yrow[MW];
#pragma unroll
  for (int i = 0; i < MW; ++i) {
    const int P = min(P0 + 16 * i + li, a.ni - 1), Q = min(Q0 + 16 * i + li, a.ni - 1);
    xrow[i] = (unsigned)P * (unsigned)a.ng;
    yrow[i] = (unsigned)Q * (unsigned)a.ng;
  }
  cb_f4 cre[MW][MW], cim[MW][MW];
  double dre[MW][MW][4], dim[MW][MW][4];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      cre[i][j] = cim[i][j] = cb_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) dre[i][j][v] = dim[i][j][v] = 0.0;
    }
  float2 fx[BF_NPF][MW][4], fy[BF_NPF][MW][4];
  double fv[BF_NPF][4];
  auto load = [&](long k0, float2 (*xx)[4], float2 (*yy)[4], double* vv) {
    const long gb = k0 + 4 * lk;
    if constexpr (VEC) {
      const unsigned g = (unsigned)min(gb, (long)a.ng - 4);
      const double2 va = *(const double2*)(vm + g), vb = *(const double2*)(vm + g + 2);
      vv[0] = va.x;
      vv[1] = va.y;
      vv[2] = vb.x;
      vv[3] = vb.y;
#pragma unroll
      for (int i = 0; i < MW; ++i) {
        if (DIAG ? (XU[i] || YU[i]) : XU[i]) {
          const float4 q0 = *(const float4*)(Fm + xrow[i] + g);
          const float4 q1 = *(const float4*)(Fm + xrow[i] + g + 2);
          xx[i][0] = make_float2(q0.x, q0.y);
          xx[i][1] = make_float2(q0.z, q0.w);
          xx[i][2] = make_float2(q1.x, q1.y);
          xx[i][3] = make_float2(q1.z, q1.w);
        }
        if (!DIAG && YU[i]) {
          const float4 q0 = *(const float4*)(Fm + yrow[i] + g);
          const float4 q1 = *(const float4*)(Fm + yrow[i] + g + 2);
          yy[i][0] = make_float2(q0.x, q0.y);
          yy[i][1] = make_float2(q0.z, q0.w);
          yy[i][2] = make_float2(q1.x, q1.y);
          yy[i][3] = make_float2(q1.z, q1.w);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const unsigned g = (unsigned)min(gb + t, (long)a.ng - 1);
        vv[t] = vm[g];
#pragma unroll
        for (int i = 0; i < MW; ++i) {
          if (DIAG ? (XU[i] || YU[i]) : XU[i]) xx[i][t] = Fm[xrow[i] + g];
          if (!DIAG && YU[i]) yy[i][t] = Fm[yrow[i] + g];
        }
      }
    }
  };
  auto step = [&](float2 (*xx)[4], float2 (*yy)[4], const double* vv, long gb) {
    float w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) w[t] = (gb + t < g1) ? (float)vv[t] : 0.f;
    cb_u16x8 yh[MW], yl[MW], yhi[MW], yli[MW];
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      if (!YU[j]) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float2 y = DIAG ? xx[j][t] : yy[j][t];
        unsigned short rh, rl = 0, ih, il = 0;
        if (SPLIT) {
          cb_split(y.x, rh, rl);
          cb_split(y.y, ih, il);
        } else {
          rh = bf16_rne(y.x);
          ih = bf16_rne(y.y);
        }
        yh[j][2 * t] = rh;
        yh[j][2 * t + 1] = ih;
        yhi[j][2 * t] = ih ^ 0x8000u;
        yhi[j][2 * t + 1] = rh;
        if (SPLIT) {
          yl[j][2 * t] = rl;
          yl[j][2 * t + 1] = il;
          yli[j][2 * t] = il ^ 0x8000u;
          yli[j][2 * t + 1] = rl;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < MW; ++i) {
      if (!XU[i]) continue;
      cb_u16x8 xh, xl;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float xr = xx[i][t].x * w[t], xi = xx[i][t].y * w[t];
        if (SPLIT) {
          unsigned short h0, l0, h1, l1;
          cb_split(xr, h0, l0);
          cb_split(xi, h1, l1);
          xh[2 * t] = h0;
          xh[2 * t + 1] = h1;
          xl[2 * t] = l0;
          xl[2 * t + 1] = l1;
        } else {
          xh[2 * t] = bf16_rne(xr);
          xh[2 * t + 1] = bf16_rne(xi);
        }
      }
#pragma unroll
      for (int j = 0; j < MW; ++j) {
        if (!(MASK & (1 << (2 * i + j)))) continue;
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cb_as_bf16(xh), cb_as_bf16(yh[j]),
                                                            cre[i][j], 0, 0, 0);
        if (SPLIT) {
          cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cb_as_bf16(xh), cb_as_bf16(yl[j]),
                                                              cre[i][j], 0, 0, 0);
          cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cb_as_bf16(xl), cb_as_bf16(yh[j]),
                                                              cre[i][j], 0, 0, 0);
        }
        if (!RE) {
          cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cb_as_bf16(xh), cb_as_bf16(yhi[j]),
                                                              cim[i][j], 0, 0, 0);
          if (SPLIT) {
            cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                cb_as_bf16(xh), cb_as_bf16(yli[j]), cim[i][j], 0, 0, 0);
            cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                cb_as_bf16(xl), cb_as_bf16(yhi[j]), cim[i][j], 0, 0, 0);
          }
        }
      }
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < MW; ++i)
#pragma unroll
      for (int j = 0; j < MW; ++j) {
        if (!(MASK & (1 << (2 * i + j)))) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          dre[i][j][v] += (double)cre[i][j][v];
          if (!RE) dim[i][j][v] += (double)cim[i][j][v];
        }
        cre[i][j] = cim[i][j] = cb_f4{0.f, 0.f, 0.f, 0.f};
      }
  };
  const long nstep = (g1 - g0 + 15) / 16;
#pragma unroll
  for (int sl = 0; sl < BF_NPF; ++sl) load(g0 + (long)sl * 16, fx[sl], fy[sl], fv[sl]);
  for (long c = 0; c < nstep; c += BF_NPF) {
#pragma unroll
    for (int sl = 0; sl < BF_NPF; ++sl) {
      const long k0 = g0 + (c + sl) * 16;
      step(fx[sl], fy[sl], fv[sl], k0 + 4 * lk);
      // refill the slot (clamped loads past the end are discarded by v = 0)
      __builtin_amdgcn_sched_barrier(0);
      load(k0 + BF_NPF * 16, fx[sl], fy[sl], fv[sl]);
      __builtin_amdgcn_sched_barrier(0);
    }
    if ((c + BF_NPF) % BF_FLUSH == 0) flush();
  }
  flush();
  // D layout: register v of a lane holds row 4 lk + v, column li of the block
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      if (!(MASK & (1 << (2 * i + j)))) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int P = P0 + 16 * i + 4 * lk + v;
        const int Q = Q0 + 16 * j + li;
        if (P < a.ni && Q < a.ni)
          out[(long)P * a.ni + Q] = make_double2(dre[i][j][v], RE ? 0.0 : dim[i][j][v]);
      }
    }
}

// one wave per 32 x 32 lower-triangle tile, as coulomb_kernel_f32
template <bool VEC, bool SPLIT, bool RE>
__global__ __launch_bounds__(64) void coulomb_kernel_bf16(const float2* __restrict__ F,
                                                       const double* __restrict__ vt,
                                                       double2* __restrict__ part, CoulArgs a,
                                                       long nwork, long nwork_pad) {
  const long w = (blockIdx.x % 8) * (nwork_pad / 8) + blockIdx.x / 8;
  if (w >= nwork) return;
  int m, s, ti, tj;
  coulomb_work(w, a, m, s, ti, tj);
  const int P0 = ti * WTILE, Q0 = tj * WTILE;
  const long g0 = (long)s * a.chunk;
  const long g1 = min((long)a.ng, g0 + a.chunk);
  const float2* Fm = F + (long)m * a.fstride;
  const double* vm = vt + (long)m * a.ng;
  double2* out = part + ((long)m * a.nsplit + s) * a.ni * a.ni;
  const bool row1 = P0 + 16 < a.ni;
  if (ti != tj) {
    if (row1)
      coulomb_tile_bf16<0xF, VEC, SPLIT, RE>(Fm, vm, out, a, P0, Q0, g0, g1);
    else
      coulomb_tile_bf16<0x3, VEC, SPLIT, RE>(Fm, vm, out, a, P0, Q0, g0, g1);
  } else {
    if (row1)
      coulomb_tile_bf16<0xD, VEC, SPLIT, RE>(Fm, vm, out, a, P0, Q0, g0, g1);
    else
      coulomb_tile_bf16<0x1, VEC, SPLIT, RE>(Fm, vm, out, a, P0, Q0, g0, g1);
  }
}

struct ReduceArgs {
  const double2* root[3];
  int n[3];
  int N[3];
  int ni, nsplit;
  int real;
  int raw;  // write the slice's scaled sum, unphased, to V[slice] and nothing else
  double scale;
  int rep[64];  // transfer of each slice
  int bar[64];  // its conjugate partner -m, written as conj(Vb^m); -1: none
};

// V[m][P][Q] = scale * e^{-i q_m.(r_P - r_Q)} sum_s part (P < Q mirrored from Q > P),
// m = rep[slice]; also V[-m] = conj V[m] where bar[slice] names -m
__global__ __launch_bounds__(256) void coulomb_reduce_kernel(const double2* __restrict__ part,
                                                             const int32_t* __restrict__ pts,
                                                             double2* __restrict__ V,
                                                             ReduceArgs a) {
  // one thread per lower-triangle entry (P >= Q; the others exit), so that the
  // partial sums are read once and along rows; (Q, P) is written as the
  // conjugate (V^m is Hermitian)
  const long nn = (long)a.ni * a.ni;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = blockIdx.y, m = a.rep[sl];
  if (idx >= nn) return;
  const int P = (int)(idx / a.ni), Q = (int)(idx % a.ni);
  if (P < Q) return;
  const long up = (long)Q * a.ni + P;
  double sx = 0.0, sy = 0.0;
  for (int s = 0; s < a.nsplit; ++s) {
    const double2 v = part[((long)sl * a.nsplit + s) * nn + idx];
    sx += v.x;
    sy += v.y;
  }
  sx *= a.scale;
  sy *= a.scale;
  if (a.raw) {
    V[(long)sl * nn + idx] = make_double2(sx, sy);
    if (P != Q) V[(long)sl * nn + up] = make_double2(sx, -sy);
    return;
  }
  if (a.real) {
    sy = 0.0;  // the real path's partials are already the Bloch-gauge matrix
  } else if (m) {
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
  double2* Vm = V + (long)m * nn;
  Vm[idx] = make_double2(sx, sy);
  if (P != Q) Vm[up] = make_double2(sx, -sy);
  // Vb^{-m} = conj Vb^m
  if (a.bar[sl] >= 0) {
    double2* Vb = V + (long)a.bar[sl] * nn;
    Vb[idx] = make_double2(sx, -sy);
    if (P != Q) Vb[up] = make_double2(sx, sy);
  }
}

}  // namespace

int coulomb_nsplit(const Geom& g) {
  const int nt = (g.ni + 2 * WTILE - 1) / (2 * WTILE);  // 64-row blocks
  const long tiles = (long)nt * (nt + 1) / 2 * g.nk;
  long ns = (4096 + tiles - 1) / tiles;
  const long maxs = (g.ng + 1023) / 1024;  // keep chunks >= ~1k points
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  return (int)ns;
}

// partial sums [slices][nsplit][N_I][N_I] c128, then the kernel table [slices][N_g] double
static size_t partial_only(const Geom& g, int nslice, int nsplit) {
  return ((size_t)nslice * nsplit * g.ni * g.ni * sizeof(double2) + 255) / 256 * 256;
}

// scratch of a launch over all N_k transfers with nsplit splits; a launch over
// fewer slices may use proportionally more splits in the same bytes
size_t coulomb_partial_bytes(const Geom& g, int nsplit) {
  return partial_only(g, g.nk, nsplit) + (size_t)g.nk * g.ng * sizeof(double);
}

// half = false: F is [N_k][N_ISDF][N_g] (complex path). half = true (real
// path): F is [N_k][N_ISDF][n1 n2 hz] with hz = n3/2 + 1, the contraction takes
// the real part with the pairing weights, and the reduction applies no phase.
// form (FP32 storage only): COUL_F64 on the FP64 matrix cores, COUL_BF16 or
// COUL_BF16X3 on the BF16 matrix cores (coulomb_tile_bf16).
template <typename T>
hipError_t launch_coulomb(const Geom& g, const Tables& tb, const void* F, const int32_t* pts,
                          void* partial, int nsplit, double2* V, bool half, hipStream_t st,
                          const int* rep, const int* bar, int nslice, bool raw, int form,
                          bool shared_f) {
  CoulArgs a;
  const int ns = rep ? nslice : g.nk;
  for (int m = 0; m < 64; ++m) a.rep[m] = rep && m < ns ? rep[m] : m;
  for (int i = 0; i < 3; ++i) {
    a.L[i] = g.L[i];
    a.n[i] = g.n[i];
    a.N[i] = g.N[i];
  }
  const int hz = g.n[2] / 2 + 1;
  a.ng = half ? g.n[0] * g.n[1] * hz : g.ng;
  a.ni = g.ni;
  a.nk = ns;
  a.fstride = shared_f ? 0 : (long)a.ni * a.ng;
  const bool vec = a.ng % 2 == 0;
  const bool bf = sizeof(T) == 4 && form != COUL_F64;
  const bool split = form == COUL_BF16X3;
  const bool vec4 = a.ng % 4 == 0;
  // complex path: FP64 storage on 64 x 64 workgroup tiles, FP32 storage on
  // 32 x 32 wave tiles; real path: 64 x 64 wave tiles (FP32 storage needs an even
  // half grid for its 16-byte loads, else 32 x 32 wave tiles); BF16 forms: 32 x 32
  // wave tiles
  const bool t64 = !bf && half && (sizeof(T) == 8 || vec);
  const int tw = (sizeof(T) == 8 || t64) ? 2 * WTILE : WTILE;
  const int nt = (g.ni + tw - 1) / tw;
  a.ntile = nt * (nt + 1) / 2;
  // Grid splits: whole rounds of the kernel's resident workgroups (a work item
  // runs for its whole chunk, so a last round that is mostly empty costs as
  // much as a full one), within the scratch capacity (nsplit splits over N_k
  // slices) and with chunks of at least ~1k points.
  {
    const void* kfn;
    int threads = 64;
    if (bf) {
#define EXX_BFK(V, S, R) (const void*)coulomb_kernel_bf16<V, S, R>
      kfn = vec4 ? (split ? (half ? EXX_BFK(true, true, true) : EXX_BFK(true, true, false))
                          : (half ? EXX_BFK(true, false, true) : EXX_BFK(true, false, false)))
                 : (split ? (half ? EXX_BFK(false, true, true) : EXX_BFK(false, true, false))
                          : (half ? EXX_BFK(false, false, true) : EXX_BFK(false, false, false)));
#undef EXX_BFK
    } else if (t64) {
      kfn = (const void*)coulomb_kernel_t64<T>;
    } else if (sizeof(T) == 8) {
      kfn = half ? (const void*)coulomb_kernel_f64<true> : (const void*)coulomb_kernel_f64<false>;
      threads = 256;
    } else if (half) {
      kfn = vec ? (const void*)coulomb_kernel_f32<true, true>
                : (const void*)coulomb_kernel_f32<false, true>;
    } else {
      kfn = vec ? (const void*)coulomb_kernel_f32<true, false>
                : (const void*)coulomb_kernel_f32<false, false>;
    }
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, threads, 0) == hipSuccess &&
        ncu > 0 && per_cu > 0) {
      const long slots = (long)ncu * per_cu;
      const long per_split = (long)a.ntile * ns;
      long cap = (long)nsplit * g.nk / ns;
      const long maxs = ((long)a.ng + 1023) / 1024;
      if (cap > maxs) cap = maxs;
      const long rounds = cap * per_split / slots;
      if (rounds >= 1) {
        const long want = rounds * slots / per_split;
        nsplit = (int)(want < 1 ? 1 : want);
      }
    }
  }
  a.nsplit = nsplit;
  a.chunk = (int)((((long)a.ng + nsplit - 1) / nsplit + CALIGN - 1) / CALIGN * CALIGN);
  if ((long)g.ni * a.ng >= 0x7fffffffL) return hipErrorInvalidValue;
  const long nwork = (long)a.ntile * ns * nsplit;
  const long pad = (nwork + 7) / 8 * 8;
  double* vt = (double*)((char*)partial + partial_only(g, ns, nsplit));
  if (half)
    hipLaunchKernelGGL(coulomb_vtab_half_kernel, dim3((unsigned)((a.ng + 255) / 256), ns),
                       dim3(256), 0, st, vt, a, hz);
  else
    hipLaunchKernelGGL(coulomb_vtab_kernel, dim3((unsigned)((g.ng + 255) / 256), ns), dim3(256),
                       0, st, vt, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define EXX_COUL(RE)                                                                            \
  if constexpr (sizeof(T) == 8) {                                                               \
    hipLaunchKernelGGL(coulomb_kernel_f64<RE>, dim3((unsigned)pad), dim3(256), 0, st,            \
                       (const double2*)F, (const double*)vt, (double2*)partial, a, nwork, pad);  \
  } else if (vec) {                                                                             \
    hipLaunchKernelGGL((coulomb_kernel_f32<true, RE>), dim3((unsigned)pad), dim3(64), 0, st,     \
                       (const float2*)F, (const double*)vt, (double2*)partial, a, nwork, pad);   \
  } else {                                                                                      \
    hipLaunchKernelGGL((coulomb_kernel_f32<false, RE>), dim3((unsigned)pad), dim3(64), 0, st,    \
                       (const float2*)F, (const double*)vt, (double2*)partial, a, nwork, pad);   \
  }
#define EXX_BFL(V, S, R)                                                                   \
  hipLaunchKernelGGL((coulomb_kernel_bf16<V, S, R>), dim3((unsigned)pad), dim3(64), 0, st,  \
                     (const float2*)F, (const double*)vt, (double2*)partial, a, nwork, pad)
#define EXX_BFL2(V, S) \
  if (half)            \
    EXX_BFL(V, S, true); \
  else                 \
    EXX_BFL(V, S, false);
  if (bf) {
    if (vec4) {
      if (split) {
        EXX_BFL2(true, true)
      } else {
        EXX_BFL2(true, false)
      }
    } else {
      if (split) {
        EXX_BFL2(false, true)
      } else {
        EXX_BFL2(false, false)
      }
    }
  } else if (t64) {
    hipLaunchKernelGGL(coulomb_kernel_t64<T>, dim3((unsigned)pad), dim3(64), 0, st,
                       (const cplx<T>*)F, (const double*)vt, (double2*)partial, a, nwork, pad);
  } else if (half) {
    EXX_COUL(true)
  } else {
    EXX_COUL(false)
  }
#undef EXX_COUL
#undef EXX_BFL2
#undef EXX_BFL
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  ReduceArgs r;
  for (int i = 0; i < 3; ++i) {
    r.root[i] = tb.root[i];
    r.n[i] = g.n[i];
    r.N[i] = g.N[i];
  }
  r.ni = g.ni;
  r.nsplit = nsplit;
  r.real = half ? 1 : 0;
  r.raw = raw ? 1 : 0;
  r.scale = g.omega / ((double)g.ng * (double)g.ng);
  for (int m = 0; m < 64; ++m) {
    r.rep[m] = a.rep[m];
    r.bar[m] = bar && m < ns ? bar[m] : -1;
  }
  const long nn = (long)g.ni * g.ni;
  hipLaunchKernelGGL(coulomb_reduce_kernel, dim3((unsigned)((nn + 255) / 256), ns), dim3(256), 0,
                     st, (const double2*)partial, pts, V, r);
  return hipGetLastError();
}

template hipError_t launch_coulomb<double>(const Geom&, const Tables&, const void*, const int32_t*,
                                           void*, int, double2*, bool, hipStream_t, const int*,
                                           const int*, int, bool, int, bool);
template hipError_t launch_coulomb<float>(const Geom&, const Tables&, const void*, const int32_t*,
                                          void*, int, double2*, bool, hipStream_t, const int*,
                                          const int*, int, bool, int, bool);

// v^m(g) of every transfer (or of the transfers rep[s], s < ns): vt [slice][N_g]
hipError_t launch_kernel_table(const Geom& g, double* vt, hipStream_t st, const int* rep,
                               int ns) {
  if (!rep) ns = g.nk;
  CoulArgs a;
  for (int m = 0; m < 64; ++m) a.rep[m] = m < ns ? (rep ? rep[m] : m) : 0;
  for (int i = 0; i < 3; ++i) {
    a.L[i] = g.L[i];
    a.n[i] = g.n[i];
    a.N[i] = g.N[i];
  }
  a.ng = g.ng;
  a.ni = g.ni;
  a.nk = g.nk;
  hipLaunchKernelGGL(coulomb_vtab_kernel, dim3((unsigned)((g.ng + 255) / 256), ns), dim3(256),
                     0, st, vt, a);
  return hipGetLastError();
}

// V[rep[s]] = e^{-i q.(r_P - r_Q)} U[s] (lower triangle of U mirrored) and
// V[bar[s]] = conj of that, for the nslice unphased matrices U
hipError_t launch_coulomb_phase(const Geom& g, const Tables& tb, const int32_t* pts,
                                const double2* U, double2* V, const int* rep, const int* bar,
                                int nslice, hipStream_t st) {
  if (nslice <= 0 || nslice > 64) return hipErrorInvalidValue;
  ReduceArgs r;
  for (int i = 0; i < 3; ++i) {
    r.root[i] = tb.root[i];
    r.n[i] = g.n[i];
    r.N[i] = g.N[i];
  }
  r.ni = g.ni;
  r.nsplit = 1;
  r.real = 0;
  r.raw = 0;
  r.scale = 1.0;
  for (int m = 0; m < 64; ++m) {
    r.rep[m] = m < nslice ? rep[m] : 0;
    r.bar[m] = m < nslice ? bar[m] : -1;
  }
  const long nn = (long)g.ni * g.ni;
  hipLaunchKernelGGL(coulomb_reduce_kernel, dim3((unsigned)((nn + 255) / 256), nslice), dim3(256),
                     0, st, U, pts, V, r);
  return hipGetLastError();
}

}  // namespace exx

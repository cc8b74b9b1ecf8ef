// 3-D forward FFT of many functions on the cell grid, mixed radix 2/3/4/5,
// Stockham autosort in LDS. Pass 1 transforms whole (y, z) planes held in LDS
// (one HBM read and one write per plane); pass 2 transforms x lines for a block
// of contiguous (y, z) columns. Twiddle tables are staged in LDS; butterflies
// are dealt to threads so that neighbouring lanes touch neighbouring LDS
// addresses (unit-stride direction fastest).
#include <algorithm>

#include "common.h"

namespace exx {

namespace {

constexpr int NT1 = 512;          // threads of the plane pass
constexpr int NT2 = 256;          // threads of the x pass
constexpr int FFT_MAXPTS = 6144;  // largest (y, z) plane held in LDS by one workgroup
constexpr int FFT_CB = 32;        // largest (y, z) column block per workgroup in pass 2
// (y, z) columns per workgroup in pass 2: 32 in FP32; 16 in FP64, where the
// smaller block halves the stage registers (measured faster)
template <typename T>
constexpr int fft_cb = sizeof(T) == 8 ? 16 : 32;
constexpr int FFT_MAXX = 128;     // longest x line

struct Plan1 {
  int n;
  int ns;
  int r[10];
};

// Radices of a line of length n (a 2*3*5-smooth n), largest first from the
// list below so that a line takes as few LDS stages as possible; composite
// radices run their own small Cooley-Tukey in registers. maxr caps the radix
// (16 in every kernel).
Plan1 plan_for(int n, int maxr = 16) {
  Plan1 p{};
  p.n = n;
  int m = n;
  const int pr[13] = {16, 25, 12, 15, 20, 9, 10, 8, 6, 5, 4, 3, 2};
  while (m > 1 && p.ns < 10) {
    int k = 0;
    while (k < 13 && (pr[k] > maxr || m % pr[k] != 0)) ++k;
    if (k == 13) break;
    p.r[p.ns++] = pr[k];
    m /= pr[k];
  }
  if (m != 1) p.ns = -1;
  return p;
}

// cos and sin of 2 pi m / R, evaluated by the compiler: octant reduction and
// Taylor series on [0, pi/4]
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr void taylor_cs(double x, double& c, double& s) {
  double t = 1.0, cs = 1.0;
  double u = x, ss = x;
  for (int k = 1; k < 14; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    cs += t;
    u *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    ss += u;
  }
  c = cs;
  s = ss;
}

constexpr void cs_2pi_frac(int m, int R, double& c, double& s) {
  const int q = (4 * m) / R, r4 = 4 * m - q * R;  // 2 pi m/R = q pi/2 + (pi/2) r4/R
  double cc = 0.0, sc = 0.0;
  if (2 * r4 <= R) {
    taylor_cs(0.5 * kPi * r4 / R, cc, sc);
  } else {
    double c2 = 0.0, s2 = 0.0;
    taylor_cs(0.5 * kPi * (R - r4) / R, c2, s2);
    cc = s2;
    sc = c2;
  }
  switch (q & 3) {
    case 0: c = cc; s = sc; break;
    case 1: c = -sc; s = cc; break;
    case 2: c = -cc; s = -sc; break;
    default: c = sc; s = -cc; break;
  }
}

template <int R>
struct RootsR {
  double c[R], s[R];
  constexpr RootsR() : c(), s() {
    for (int m = 0; m < R; ++m) cs_2pi_frac(m, R, c[m], s[m]);
  }
};

template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T>* v) {
  if (R == 2) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
  } else if (R == 4) {
    cplx<T> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    cplx<T> s02 = cadd<T>(a0, a2), d02 = csub<T>(a0, a2);
    cplx<T> s13 = cadd<T>(a1, a3), d13 = csub<T>(a1, a3);
    v[0] = cadd<T>(s02, s13);
    v[2] = csub<T>(s02, s13);
    // -i * d13 = (d13.y, -d13.x)
    v[1] = mk<T>(d02.x + d13.y, d02.y - d13.x);
    v[3] = mk<T>(d02.x - d13.y, d02.y + d13.x);
  } else if (R == 3) {
    const T s = (T)0.86602540378443864676372317075294;
    cplx<T> a0 = v[0], a1 = v[1], a2 = v[2];
    cplx<T> t = cadd<T>(a1, a2), d = csub<T>(a1, a2);
    v[0] = cadd<T>(a0, t);
    cplx<T> m = mk<T>(a0.x - (T)0.5 * t.x, a0.y - (T)0.5 * t.y);
    // -i s d = (s d.y, -s d.x)
    v[1] = mk<T>(m.x + s * d.y, m.y - s * d.x);
    v[2] = mk<T>(m.x - s * d.y, m.y + s * d.x);
  } else if (R == 5) {
    const T c1 = (T)0.30901699437494742410229341718282;   // cos(2 pi/5)
    const T c2 = (T)-0.80901699437494742410229341718282;  // cos(4 pi/5)
    const T s1 = (T)0.95105651629515357211643933337938;   // sin(2 pi/5)
    const T s2 = (T)0.58778525229247312916870595463907;   // sin(4 pi/5)
    cplx<T> a0 = v[0];
    cplx<T> t1 = cadd<T>(v[1], v[4]), d1 = csub<T>(v[1], v[4]);
    cplx<T> t2 = cadd<T>(v[2], v[3]), d2 = csub<T>(v[2], v[3]);
    v[0] = cadd<T>(a0, cadd<T>(t1, t2));
    cplx<T> m1 = mk<T>(a0.x + c1 * t1.x + c2 * t2.x, a0.y + c1 * t1.y + c2 * t2.y);
    cplx<T> m2 = mk<T>(a0.x + c2 * t1.x + c1 * t2.x, a0.y + c2 * t1.y + c1 * t2.y);
    // X1 = m1 - i (s1 d1 + s2 d2); X4 = m1 + i (...)
    cplx<T> e1 = mk<T>(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    // X2 = m2 - i (s2 d1 - s1 d2); X3 = m2 + i (...)
    cplx<T> e2 = mk<T>(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    v[1] = mk<T>(m1.x + e1.y, m1.y - e1.x);
    v[4] = mk<T>(m1.x - e1.y, m1.y + e1.x);
    v[2] = mk<T>(m2.x + e2.y, m2.y - e2.x);
    v[3] = mk<T>(m2.x - e2.y, m2.y + e2.x);
  }
}

template <typename T, int R>
__device__ __forceinline__ void dft_any(cplx<T>* v);

// DFT of length R = R1 R2 in registers (forward, natural order in and out):
// X[k1 + R1 k2] = sum_j2 W_R2^{j2 k2} W_R^{j2 k1} sum_j1 W_R1^{j1 k1} x[R2 j1 + j2]
template <typename T, int R1, int R2>
__device__ __forceinline__ void dft_comp(cplx<T>* v) {
  constexpr int R = R1 * R2;
  constexpr RootsR<R> w{};
  cplx<T> y[R];
#pragma unroll
  for (int j2 = 0; j2 < R2; ++j2) {
    cplx<T> t[R1];
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) t[j1] = v[R2 * j1 + j2];
    dft_any<T, R1>(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      const int m = (j2 * k1) % R;
      y[j2 * R1 + k1] = m == 0 ? t[k1] : cmul<T>(t[k1], mk<T>((T)w.c[m], (T)-w.s[m]));
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cplx<T> u[R2];
#pragma unroll
    for (int j2 = 0; j2 < R2; ++j2) u[j2] = y[j2 * R1 + k1];
    dft_any<T, R2>(u);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = u[k2];
  }
}

template <typename T, int R>
__device__ __forceinline__ void dft_any(cplx<T>* v) {
  if constexpr (R == 2 || R == 3 || R == 4 || R == 5) dft_small<T, R>(v);
  else if constexpr (R == 6) dft_comp<T, 2, 3>(v);
  else if constexpr (R == 8) dft_comp<T, 2, 4>(v);
  else if constexpr (R == 9) dft_comp<T, 3, 3>(v);
  else if constexpr (R == 10) dft_comp<T, 2, 5>(v);
  else if constexpr (R == 12) dft_comp<T, 3, 4>(v);
  else if constexpr (R == 15) dft_comp<T, 3, 5>(v);
  else if constexpr (R == 16) dft_comp<T, 4, 4>(v);
}

// x / d for 0 <= x < 2^22 and d >= 1 from a float reciprocal: the float
// quotient is off by at most one, which the remainder test corrects
__device__ __forceinline__ int small_div(int x, int d, float inv) {
  int q = (int)((float)x * inv);
  const int r = x - q * d;
  q += (r >= d) - (r < 0);
  return q;
}

// One Stockham stage of radix R on `nlines` lines of length n stored in LDS
// (element stride es, line stride ls); Ns = product of the radices done so far.
// With LINE_FAST the butterfly index runs over lines first (use when ls == 1).
// The index decomposition is done once per butterfly, without integer division.
template <typename T, int R, int NT, int MAXPTS, bool LINE_FAST>
__device__ __forceinline__ void stage(cplx<T>* buf, int n, int Ns, int nlines, int es, int ls,
                                      const cplx<T>* tw) {
  constexpr int MAXB = (MAXPTS / R + NT - 1) / NT;
  const int nb = n / R;
  const int total = nlines * nb;
  // an opaque copy of the thread index per stage: without it the compiler
  // hoists the index arithmetic of every radix out of the stage loop and keeps
  // it live across all stages (twice the registers, half the occupancy)
  int tid = threadIdx.x;
  __asm__ volatile("" : "+v"(tid));
  const int dmaj = LINE_FAST ? nlines : nb;  // divisor splitting b into (line, j)
  const float imaj = 1.0f / (float)dmaj, ins = 1.0f / (float)Ns;
  cplx<T> v[MAXB][R];
  int src[MAXB], dst[MAXB], stp[MAXB];
#pragma unroll
  for (int s = 0; s < MAXB; ++s) {
    const int b = tid + s * NT;
    if (b < total) {
      const int q = small_div(b, dmaj, imaj);
      const int rem = b - q * dmaj;
      const int line = LINE_FAST ? rem : q;
      const int j = LINE_FAST ? q : rem;
      const int jq = small_div(j, Ns, ins);
      const int jm = j - jq * Ns;
      src[s] = line * ls + j * es;
      dst[s] = line * ls + (jq * Ns * R + jm) * es;
      stp[s] = jm * (nb / Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) v[s][r] = buf[src[s] + r * nb * es];
    }
  }
  __syncthreads();
  const bool first = Ns == 1;  // the first stage's twiddles are all 1 (uniform branch)
#pragma unroll
  for (int s = 0; s < MAXB; ++s) {
    const int b = tid + s * NT;
    if (b < total) {
      if (!first) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[s][r] = cmul<T>(v[s][r], tw[stp[s] * r]);
      }
      dft_any<T, R>(v[s]);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[s] + r * Ns * es] = v[s][r];
    }
  }
  __syncthreads();
}

template <typename T, int NT, int MAXPTS, bool LINE_FAST>
__device__ void fft_lines(cplx<T>* buf, const Plan1& p, int nlines, int es, int ls,
                          const cplx<T>* tw) {
  int Ns = 1;
  for (int s = 0; s < p.ns; ++s) {
    const int R = p.r[s];
#define EXX_STAGE(RR) \
  if (R == RR) stage<T, RR, NT, MAXPTS, LINE_FAST>(buf, p.n, Ns, nlines, es, ls, tw);
    EXX_STAGE(2)
    EXX_STAGE(3)
    EXX_STAGE(4)
    EXX_STAGE(5)
    // composite radices in both precisions: the FP64 plane kernels are held to
    // two workgroups per CU by LDS, so their extra registers cost no occupancy
    {
      EXX_STAGE(6)
      EXX_STAGE(8)
      EXX_STAGE(9)
      EXX_STAGE(10)
      EXX_STAGE(12)
      EXX_STAGE(15)
      EXX_STAGE(16)
    }
#undef EXX_STAGE
    Ns *= R;
  }
}

// pass 1: one (function, x) plane per workgroup; z lines then y lines
template <typename T>
__global__ __launch_bounds__(NT1) void fft_yz1_kernel(const cplx<T>* __restrict__ in,
                                                     cplx<T>* __restrict__ out, Plan1 py, Plan1 pz,
                                                     const cplx<T>* __restrict__ twy,
                                                     const cplx<T>* __restrict__ twz) {
  extern __shared__ char smem_raw[];
  const int n2 = py.n, n3 = pz.n, np = n2 * n3;
  cplx<T>* buf = (cplx<T>*)smem_raw;
  cplx<T>* ty = buf + np;
  cplx<T>* tz = ty + n2;
  const long off = (long)blockIdx.x * np;
  for (int e = threadIdx.x; e < np; e += NT1) buf[e] = in[off + e];
  for (int e = threadIdx.x; e < n2; e += NT1) ty[e] = twy[e];
  for (int e = threadIdx.x; e < n3; e += NT1) tz[e] = twz[e];
  __syncthreads();
  fft_lines<T, NT1, FFT_MAXPTS, false>(buf, pz, n2, 1, n3, tz);
  fft_lines<T, NT1, FFT_MAXPTS, true>(buf, py, n3, n3, 1, ty);
  for (int e = threadIdx.x; e < np; e += NT1) out[off + e] = buf[e];
}

// pass 2: x lines of fft_cb<T> contiguous (y, z) columns of one function
template <typename T>
__global__ __launch_bounds__(NT2) void fft_x1_kernel(cplx<T>* __restrict__ data, Plan1 px, int np,
                                                    int nblk, const cplx<T>* __restrict__ twx) {
  extern __shared__ char smem_raw[];
  const int n1 = px.n;
  cplx<T>* buf = (cplx<T>*)smem_raw;
  cplx<T>* tx = buf + n1 * fft_cb<T>;
  const long f = blockIdx.x / nblk;
  const int c0 = (blockIdx.x % nblk) * fft_cb<T>;
  const int cw = min(fft_cb<T>, np - c0);
  cplx<T>* base = data + f * (long)n1 * np + c0;
  for (int e = threadIdx.x; e < n1 * fft_cb<T>; e += NT2) {
    const int x = e / fft_cb<T>, c = e % fft_cb<T>;
    buf[e] = (c < cw) ? base[(long)x * np + c] : mk<T>(0, 0);
  }
  for (int e = threadIdx.x; e < n1; e += NT2) tx[e] = twx[e];
  __syncthreads();
  fft_lines<T, NT2, fft_cb<T> * FFT_MAXX, true>(buf, px, fft_cb<T>, fft_cb<T>, 1, tx);
  for (int e = threadIdx.x; e < n1 * fft_cb<T>; e += NT2) {
    const int x = e / fft_cb<T>, c = e % fft_cb<T>;
    if (c < cw) base[(long)x * np + c] = buf[e];
  }
}

// pass 1: (function, x) planes, z lines then y lines. Workgroups loop over
// planes; the next plane is loaded into registers while the current one is
// transformed in LDS.
constexpr int PRE1 = (FFT_MAXPTS + NT1 - 1) / NT1;
template <typename T>
__global__ __launch_bounds__(NT1) void fft_yz_kernel(const cplx<T>* __restrict__ in,
                                                     cplx<T>* __restrict__ out, long nplanes,
                                                     Plan1 py, Plan1 pz,
                                                     const cplx<T>* __restrict__ twy,
                                                     const cplx<T>* __restrict__ twz) {
  extern __shared__ char smem_raw[];
  const int n2 = py.n, n3 = pz.n, np = n2 * n3;
  cplx<T>* buf = (cplx<T>*)smem_raw;
  cplx<T>* ty = buf + np;
  cplx<T>* tz = ty + n2;
  for (int e = threadIdx.x; e < n2; e += NT1) ty[e] = twy[e];
  for (int e = threadIdx.x; e < n3; e += NT1) tz[e] = twz[e];
  cplx<T> pre[PRE1];
  long p = blockIdx.x;
  if (p < nplanes) {
#pragma unroll
    for (int k = 0; k < PRE1; ++k) {
      const int e = threadIdx.x + k * NT1;
      if (e < np) pre[k] = in[p * np + e];
    }
  }
  for (; p < nplanes; p += gridDim.x) {
#pragma unroll
    for (int k = 0; k < PRE1; ++k) {
      const int e = threadIdx.x + k * NT1;
      if (e < np) buf[e] = pre[k];
    }
    __syncthreads();
    const long pn = p + gridDim.x;
    if (pn < nplanes) {
#pragma unroll
      for (int k = 0; k < PRE1; ++k) {
        const int e = threadIdx.x + k * NT1;
        if (e < np) pre[k] = in[pn * np + e];
      }
    }
    fft_lines<T, NT1, FFT_MAXPTS, false>(buf, pz, n2, 1, n3, tz);
    fft_lines<T, NT1, FFT_MAXPTS, true>(buf, py, n3, n3, 1, ty);
    for (int e = threadIdx.x; e < np; e += NT1) out[p * np + e] = buf[e];
    __syncthreads();
  }
}

// pass 2: x lines of fft_cb<T> contiguous (y, z) columns; workgroups loop over
// column blocks with a register prefetch of the next block.
constexpr int PRE2 = (FFT_CB * FFT_MAXX + NT2 - 1) / NT2;
template <typename T>
__global__ __launch_bounds__(NT2) void fft_x_kernel(cplx<T>* __restrict__ data, long nwork,
                                                    Plan1 px, int np, int nblk,
                                                    const cplx<T>* __restrict__ twx) {
  extern __shared__ char smem_raw[];
  const int n1 = px.n;
  cplx<T>* buf = (cplx<T>*)smem_raw;
  cplx<T>* tx = buf + n1 * fft_cb<T>;
  for (int e = threadIdx.x; e < n1; e += NT2) tx[e] = twx[e];
  const int npts = n1 * fft_cb<T>;
  cplx<T> pre[PRE2];
  auto fetch = [&](long w) {
    const long f = w / nblk;
    const int c0 = (int)(w % nblk) * fft_cb<T>;
    const int cw = min(fft_cb<T>, np - c0);
    const cplx<T>* base = data + f * (long)n1 * np + c0;
#pragma unroll
    for (int k = 0; k < PRE2; ++k) {
      const int e = threadIdx.x + k * NT2;
      if (e < npts) {
        const int x = e / fft_cb<T>, c = e % fft_cb<T>;
        pre[k] = (c < cw) ? base[(long)x * np + c] : mk<T>(0, 0);
      }
    }
  };
  long w = blockIdx.x;
  if (w < nwork) fetch(w);
  for (; w < nwork; w += gridDim.x) {
#pragma unroll
    for (int k = 0; k < PRE2; ++k) {
      const int e = threadIdx.x + k * NT2;
      if (e < npts) buf[e] = pre[k];
    }
    __syncthreads();
    if (w + gridDim.x < nwork) fetch(w + gridDim.x);
    fft_lines<T, NT2, fft_cb<T> * FFT_MAXX, true>(buf, px, fft_cb<T>, fft_cb<T>, 1, tx);
    const long f = w / nblk;
    const int c0 = (int)(w % nblk) * fft_cb<T>;
    const int cw = min(fft_cb<T>, np - c0);
    cplx<T>* base = data + f * (long)n1 * np + c0;
    for (int e = threadIdx.x; e < npts; e += NT2) {
      const int x = e / fft_cb<T>, c = e % fft_cb<T>;
      if (c < cw) base[(long)x * np + c] = buf[e];
    }
    __syncthreads();
  }
}

// Real path (meshes whose transfers are all self-conjugate): the input is the
// real fit eta_P(r) of transfer m, the transform wanted is
// H_P(G) = sum_r eta_P(r) e^{-i (G + q_m).r}, and only the z frequencies
// g3 < hz = n3/2 + 1 are kept (the others follow from the pairing
// H(G) = conj H(-G - 2 q_m)). Pass 1 loads a (function, x) plane times the
// twist e^{-i q_m.r}, transforms all z lines, then the y lines of the first hz
// z columns only, and writes [function][x][y][hz].
struct TwistArgs {
  const double2* root[3];  // e^{-2 pi i t / (N_a n_a)}
  int n[3], N[3];
  int ni;
  int m0;  // transfer of the first function (functions are N_ISDF per transfer)
};

// Real path, two real lines per complex transform: the twisted input of a
// plane is v(y, z) ry[y] rz[z] with real v, and the y (and x) phase ry[y] is
// constant along z, so it is applied after the z transform. Lines a = 2q and
// b = 2q + 1 are packed as c(z) = (v_a(z) + i v_b(z)) rz[z]; with the z twist
// rz[z] = e^{-i pi d z / n3} (d = 2 m3 / N3, 0 or 1 on the real path), the
// transform X of a real line obeys conj X(g) = X((-g - d) mod n3), so
//   X_a(g) = (C(g) + conj C(g')) / 2,  X_b(g) = (C(g) - conj C(g')) / (2i),
// g' = (-g - d) mod n3, for the kept g < hz. Half the z work and half the LDS
// of fft_yz_half_kernel, so twice the planes per CU with 256-thread workgroups.
constexpr int NTH = 256;            // threads of the paired plane pass
constexpr int FFT_MAXPTS_H = 3200;  // points of the paired z lines or of the kept half plane
constexpr int SEP_MAX = 8;          // separated (pair, g) entries per thread

template <typename TI, typename T>
__global__ __launch_bounds__(NTH) void fft_yz_half2_kernel(const TI* __restrict__ in,
                                                           cplx<T>* __restrict__ out, Plan1 py,
                                                           Plan1 pz, int hz, TwistArgs ta,
                                                           const cplx<T>* __restrict__ twy,
                                                           const cplx<T>* __restrict__ twz) {
  extern __shared__ char smem_raw[];
  const int n2 = py.n, n3 = pz.n, n2p = (n2 + 1) / 2;
  const int nbuf = max(n2p * n3, n2 * hz);
  cplx<T>* buf = (cplx<T>*)smem_raw;
  cplx<T>* ty = buf + nbuf;
  cplx<T>* tz = ty + n2;
  cplx<T>* ry = tz + n3;
  cplx<T>* rz = ry + n2;
  const long p = blockIdx.x;  // plane = function * n1 + x
  const int n1 = ta.n[0];
  const long f = p / n1;
  const int g1 = (int)(p % n1);
  const int m = ta.m0 + (int)(f / ta.ni);
  const int m1 = m / (ta.N[1] * ta.N[2]), m2 = (m / ta.N[2]) % ta.N[1], m3 = m % ta.N[2];
  const int d = (2 * m3) / ta.N[2];
  const double2 c0 = ta.root[0][(m1 * g1) % (ta.N[0] * n1)];
  for (int e = threadIdx.x; e < n2; e += NTH) {
    ty[e] = twy[e];
    const double2 r = ta.root[1][(m2 * e) % (ta.N[1] * n2)];
    ry[e] = mk<T>((T)(c0.x * r.x - c0.y * r.y), (T)(c0.x * r.y + c0.y * r.x));
  }
  for (int e = threadIdx.x; e < n3; e += NTH) {
    tz[e] = twz[e];
    const double2 r = ta.root[2][(m3 * e) % (ta.N[2] * n3)];
    rz[e] = mk<T>((T)r.x, (T)r.y);
  }
  __syncthreads();
  const TI* src = in + p * (long)(n2 * n3);
  const float in3 = 1.0f / (float)n3, ihz = 1.0f / (float)hz;
  for (int e = threadIdx.x; e < n2p * n3; e += NTH) {
    const int q = small_div(e, n3, in3), z = e - q * n3;
    const T va = (T)src[(2 * q) * n3 + z];
    const T vb = 2 * q + 1 < n2 ? (T)src[(2 * q + 1) * n3 + z] : (T)0;
    const cplx<T> w = rz[z];
    buf[e] = mk<T>(va * w.x - vb * w.y, va * w.y + vb * w.x);
  }
  __syncthreads();
  fft_lines<T, NTH, FFT_MAXPTS_H, false>(buf, pz, n2p, 1, n3, tz);
  // separate the pairs (all reads into registers, then the [y][hz] layout is
  // written over the same LDS)
  cplx<T> za[SEP_MAX], zb[SEP_MAX];
  const T half = (T)0.5;
#pragma unroll
  for (int s = 0; s < SEP_MAX; ++s) {
    const int e = threadIdx.x + s * NTH;
    if (e < n2p * hz) {
      const int q = small_div(e, hz, ihz), g = e - q * hz;
      const int gp = (2 * n3 - g - d) % n3;
      const cplx<T> c = buf[q * n3 + g], cp = buf[q * n3 + gp];
      const cplx<T> xa = mk<T>(half * (c.x + cp.x), half * (c.y - cp.y));
      const cplx<T> xb = mk<T>(half * (c.y + cp.y), half * (cp.x - c.x));
      za[s] = cmul<T>(ry[2 * q], xa);
      zb[s] = 2 * q + 1 < n2 ? cmul<T>(ry[2 * q + 1], xb) : mk<T>((T)0, (T)0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SEP_MAX; ++s) {
    const int e = threadIdx.x + s * NTH;
    if (e < n2p * hz) {
      const int q = small_div(e, hz, ihz), g = e - q * hz;
      buf[(2 * q) * hz + g] = za[s];
      if (2 * q + 1 < n2) buf[(2 * q + 1) * hz + g] = zb[s];
    }
  }
  __syncthreads();
  fft_lines<T, NTH, FFT_MAXPTS_H, true>(buf, py, hz, hz, 1, ty);
  cplx<T>* dst = out + p * ((long)n2 * hz);
  for (int e = threadIdx.x; e < n2 * hz; e += NTH) dst[e] = buf[e];
}

template <typename TI, typename T>
__global__ __launch_bounds__(NT1) void fft_yz_half_kernel(const TI* __restrict__ in,
                                                          cplx<T>* __restrict__ out, Plan1 py,
                                                          Plan1 pz, int hz, TwistArgs ta,
                                                          const cplx<T>* __restrict__ twy,
                                                          const cplx<T>* __restrict__ twz) {
  extern __shared__ char smem_raw[];
  const int n2 = py.n, n3 = pz.n, np = n2 * n3;
  cplx<T>* buf = (cplx<T>*)smem_raw;
  cplx<T>* ty = buf + np;
  cplx<T>* tz = ty + n2;
  cplx<T>* ry = tz + n3;
  cplx<T>* rz = ry + n2;
  const long p = blockIdx.x;  // plane = function * n1 + x
  const int n1 = ta.n[0];
  const long f = p / n1;
  const int g1 = (int)(p % n1);
  const int m = ta.m0 + (int)(f / ta.ni);
  const int m1 = m / (ta.N[1] * ta.N[2]), m2 = (m / ta.N[2]) % ta.N[1], m3 = m % ta.N[2];
  const double2 c0 = ta.root[0][(m1 * g1) % (ta.N[0] * n1)];
  for (int e = threadIdx.x; e < n2; e += NT1) {
    ty[e] = twy[e];
    const double2 r = ta.root[1][(m2 * e) % (ta.N[1] * n2)];
    ry[e] = mk<T>((T)(c0.x * r.x - c0.y * r.y), (T)(c0.x * r.y + c0.y * r.x));
  }
  for (int e = threadIdx.x; e < n3; e += NT1) {
    tz[e] = twz[e];
    const double2 r = ta.root[2][(m3 * e) % (ta.N[2] * n3)];
    rz[e] = mk<T>((T)r.x, (T)r.y);
  }
  __syncthreads();
  const TI* src = in + p * np;
  const float in3 = 1.0f / (float)n3, ihz = 1.0f / (float)hz;
  for (int e = threadIdx.x; e < np; e += NT1) {
    const int y = small_div(e, n3, in3), z = e - y * n3;
    const cplx<T> w = cmul<T>(ry[y], rz[z]);
    const T v = (T)src[e];
    buf[e] = mk<T>(v * w.x, v * w.y);
  }
  __syncthreads();
  fft_lines<T, NT1, FFT_MAXPTS, false>(buf, pz, n2, 1, n3, tz);
  fft_lines<T, NT1, FFT_MAXPTS, true>(buf, py, hz, n3, 1, ty);
  cplx<T>* dst = out + p * ((long)n2 * hz);
  for (int e = threadIdx.x; e < n2 * hz; e += NT1) {
    const int y = small_div(e, hz, ihz), z = e - y * hz;
    dst[e] = buf[y * n3 + z];
  }
}

template <typename T>
const cplx<T>* twp(const Tables& tb, int a);
template <>
const double2* twp<double>(const Tables& tb, int a) {
  return tb.tw64[a];
}
template <>
const float2* twp<float>(const Tables& tb, int a) {
  return tb.tw32[a];
}

}  // namespace

bool fft_supported(const Geom& g, bool fp64) {
  (void)fp64;
  for (int a = 0; a < 3; ++a) {
    if (g.n[a] < 1 || g.n[a] > 128) return false;
    if (plan_for(g.n[a]).ns < 0) return false;
  }
  if (g.n[1] * g.n[2] > FFT_MAXPTS) return false;
  if (g.n[0] > FFT_MAXX) return false;
  return true;
}

// Raise the dynamic-LDS limit of the FFT plane and line kernels to what grids up to the
// supported maximum need. Called once per process before any launch (and
// therefore never inside a captured launch sequence).
static hipError_t fft_attributes() {
  static hipError_t done = hipErrorNotReady;
  if (done != hipErrorNotReady) return done;
  const int l1d = (FFT_MAXPTS + 2 * 128) * (int)sizeof(double2);
  const int l2d = (FFT_MAXX * FFT_CB + FFT_MAXX) * (int)sizeof(double2);
  const int l1f = (FFT_MAXPTS + 2 * 128) * (int)sizeof(float2);
  const int l2f = (FFT_MAXX * FFT_CB + FFT_MAXX) * (int)sizeof(float2);
  hipError_t e = hipFuncSetAttribute((const void*)fft_yz1_kernel<double>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, l1d);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)fft_x1_kernel<double>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l2d);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)fft_yz_kernel<float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l1f);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)fft_x_kernel<float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l2f);
  const int lhd = (FFT_MAXPTS + 4 * 128) * (int)sizeof(double2);
  const int lhf = (FFT_MAXPTS + 4 * 128) * (int)sizeof(float2);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)fft_yz_half_kernel<double, double>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lhd);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)fft_yz_half_kernel<float, float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lhf);
  done = e;
  return e;
}

hipError_t fft_prepare(int* ncu) {
  hipError_t e = fft_attributes();
  if (e != hipSuccess) return e;
  int dev = 0, v = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess && v > 0) *ncu = v;
  return e;
}

template <typename T>
hipError_t launch_fft3d(const Geom& g, const Tables& tb, const void* in, void* out, long nfun,
                        int ncu, hipStream_t st) {
  const int maxr = 16;
  Plan1 px = plan_for(g.n[0], maxr), py = plan_for(g.n[1], maxr), pz = plan_for(g.n[2], maxr);
  const int np = g.n[1] * g.n[2];
  size_t lds1 = (size_t)(np + g.n[1] + g.n[2]) * sizeof(cplx<T>);
  size_t lds2 = (size_t)(g.n[0] * fft_cb<T> + g.n[0]) * sizeof(cplx<T>);
  const long nplanes = nfun * g.n[0];
  const int nblk = (np + fft_cb<T> - 1) / fft_cb<T>;
  hipError_t e;
  if constexpr (sizeof(T) == 8) {
    // FP64 planes: a register copy of the next plane would spill, so one plane
    // per workgroup (two workgroups per CU by LDS)
    hipLaunchKernelGGL(fft_yz1_kernel<T>, dim3((unsigned)nplanes), dim3(NT1), lds1, st,
                       (const cplx<T>*)in, (cplx<T>*)out, py, pz, twp<T>(tb, 1), twp<T>(tb, 2));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fft_x1_kernel<T>, dim3((unsigned)(nfun * nblk)), dim3(NT2), lds2, st,
                       (cplx<T>*)out, px, np, nblk, twp<T>(tb, 0));
    return hipGetLastError();
  } else {
    // FP32 planes: persistent workgroups that prefetch the next plane
    const long wpc1 = std::max<long>(1, (160L * 1024) / (long)lds1);
    const long grid1 = std::min<long>(nplanes, (long)ncu * std::min<long>(wpc1, 4) * 2);
    hipLaunchKernelGGL(fft_yz_kernel<T>, dim3((unsigned)grid1), dim3(NT1), lds1, st,
                       (const cplx<T>*)in, (cplx<T>*)out, nplanes, py, pz, twp<T>(tb, 1),
                       twp<T>(tb, 2));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long nwork = nfun * nblk;
    const long wpc2 = std::max<long>(1, (160L * 1024) / (long)lds2);
    const long grid2 = std::min<long>(nwork, (long)ncu * std::min<long>(wpc2, 8) * 2);
    hipLaunchKernelGGL(fft_x_kernel<T>, dim3((unsigned)grid2), dim3(NT2), lds2, st,
                       (cplx<T>*)out, nwork, px, np, nblk, twp<T>(tb, 0));
    return hipGetLastError();
  }
}

int fft_half_z(const Geom& g) { return g.n[2] / 2 + 1; }

template <typename TI, typename T>
hipError_t launch_fft3d_half(const Geom& g, const Tables& tb, const void* in, void* out, long nfun,
                             int m0, int ncu, hipStream_t st) {
  const int maxr = 16;
  Plan1 px = plan_for(g.n[0], maxr), py = plan_for(g.n[1], maxr), pz = plan_for(g.n[2], maxr);
  const int hz = fft_half_z(g);
  const int np = g.n[1] * g.n[2], nph = g.n[1] * hz;
  const size_t lds1 = (size_t)(np + 2 * g.n[1] + 2 * g.n[2]) * sizeof(cplx<T>);
  const size_t lds2 = (size_t)(g.n[0] * fft_cb<T> + g.n[0]) * sizeof(cplx<T>);
  const long nplanes = nfun * g.n[0];
  const int nblk = (nph + fft_cb<T> - 1) / fft_cb<T>;
  TwistArgs ta;
  for (int a = 0; a < 3; ++a) {
    ta.root[a] = tb.root[a];
    ta.n[a] = g.n[a];
    ta.N[a] = g.N[a];
  }
  ta.ni = g.ni;
  ta.m0 = m0;
  const int n2p = (g.n[1] + 1) / 2;
  const bool paired = n2p * g.n[2] <= FFT_MAXPTS_H && nph <= FFT_MAXPTS_H &&
                      n2p * hz <= SEP_MAX * NTH;
  if (paired) {
    const size_t ldsp =
        (size_t)(std::max(n2p * g.n[2], nph) + 2 * g.n[1] + 2 * g.n[2]) * sizeof(cplx<T>);
    hipLaunchKernelGGL((fft_yz_half2_kernel<TI, T>), dim3((unsigned)nplanes), dim3(NTH), ldsp, st,
                       (const TI*)in, (cplx<T>*)out, py, pz, hz, ta, twp<T>(tb, 1),
                       twp<T>(tb, 2));
  } else {
    hipLaunchKernelGGL((fft_yz_half_kernel<TI, T>), dim3((unsigned)nplanes), dim3(NT1), lds1, st,
                       (const TI*)in, (cplx<T>*)out, py, pz, hz, ta, twp<T>(tb, 1),
                       twp<T>(tb, 2));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (sizeof(T) == 8) {
    hipLaunchKernelGGL(fft_x1_kernel<T>, dim3((unsigned)(nfun * nblk)), dim3(NT2), lds2, st,
                       (cplx<T>*)out, px, nph, nblk, twp<T>(tb, 0));
    return hipGetLastError();
  }
  const long nwork = nfun * nblk;
  const long wpc2 = std::max<long>(1, (160L * 1024) / (long)lds2);
  const long grid2 = std::min<long>(nwork, (long)ncu * std::min<long>(wpc2, 8) * 2);
  hipLaunchKernelGGL(fft_x_kernel<T>, dim3((unsigned)grid2), dim3(NT2), lds2, st, (cplx<T>*)out,
                     nwork, px, nph, nblk, twp<T>(tb, 0));
  return hipGetLastError();
}
template hipError_t launch_fft3d_half<double, double>(const Geom&, const Tables&, const void*,
                                                      void*, long, int, int, hipStream_t);
template hipError_t launch_fft3d_half<float, float>(const Geom&, const Tables&, const void*, void*,
                                                    long, int, int, hipStream_t);

template hipError_t launch_fft3d<double>(const Geom&, const Tables&, const void*, void*, long,
                                         int, hipStream_t);
template hipError_t launch_fft3d<float>(const Geom&, const Tables&, const void*, void*, long, int,
                                        hipStream_t);

}  // namespace exx

// ISDF fit kernels: Bloch-phase tables and the k-mesh autocorrelation that
// forms the fit metric S^m and the right-hand side Z^m.
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
  const exx_context::TabEntry* hit = nullptr;
  for (const auto& te : h->tabs) {
    bool same = true;
    for (int a = 0; a < 6; ++a) same = same && te.key[a] == key[a];
    if (same) {
      hit = &te;
      break;
    }
  }
  if (!hit) {
    size_t bytes = nroot * sizeof(double2) + ntw * (sizeof(double2) + sizeof(float2)) + 256;
    void* buf = nullptr;
    hipError_t e = hipMalloc(&buf, bytes);
    if (e != hipSuccess) return fail(h, EXX_ERR_NOMEM, "table allocation failed");
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
    char* base = (char*)buf;
    // synchronous upload, once per shape (never inside a captured sequence)
    e = hipStreamSynchronize(st);
    if (e == hipSuccess)
      e = hipMemcpy(base, r64.data(), r64.size() * sizeof(double2), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(base + nroot * sizeof(double2), w64.data(), w64.size() * sizeof(double2),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(base + (nroot + ntw) * sizeof(double2), w32.data(), w32.size() * sizeof(float2),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(buf);
      return hip_check(h, e, "table upload");
    }
    exx_context::TabEntry te;
    for (int a = 0; a < 6; ++a) te.key[a] = key[a];
    te.buf = buf;
    te.bytes = bytes;
    h->tabs.push_back(te);
    hit = &h->tabs.back();
  }
  const double2* r = (const double2*)hit->buf;
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

// v e^{-2 pi i t / N} for a compile-time root: the roots 1, -1 and -+i are
// applied as exact swaps and sign changes (a multiply by 0 or 1 is not folded
// away in IEEE arithmetic, and would cost instructions and registers)
template <typename T, int N>
__device__ __forceinline__ cplx<T> cmul_kroot(cplx<T> v, int t) {
  if (t == 0) return v;
  if (N == 2) return mk<T>(-v.x, -v.y);
  if (N == 4) {
    if (t == 1) return mk<T>(v.y, -v.x);   // * (-i)
    if (t == 2) return mk<T>(-v.x, -v.y);  // * (-1)
    return mk<T>(-v.y, v.x);               // * (+i)
  }
  return cmul<T>(v, kroot<T, N>(t));
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
      for (int t = 1; t < NA; ++t) acc = cadd<T>(acc, cmul_kroot<T, NA>(tmp[t], (s * t) % NA));
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

// the Bloch phases of a (point, column) element for every transfer of an
// N1 x N2 x N3 mesh: e^{i q_m.(r_P - r_c)} = prod_a w_a^{m_a} with
// w_a = conj(root_a[p_a]) root_a[c_a] (root_a[t] = e^{-2 pi i t/(N_a n_a)}, so
// root_a[m_a t mod N_a n_a] = root_a[t]^{m_a}); pw[a][j] = w_a^j, j < N_a.
// Three table reads per position instead of three per transfer.
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int NMAX>
__device__ __forceinline__ void axis_powers(const double2* root, int pa, int ca, int Na, double2* pw) {
  const double2 rp = root[pa], rc = root[ca];
  const double2 w = make_double2(rp.x * rc.x + rp.y * rc.y, rp.x * rc.y - rp.y * rc.x);
  pw[0] = make_double2(1.0, 0.0);
#pragma unroll
  for (int j = 1; j < NMAX; ++j)
    if (j < Na) pw[j] = zmul(pw[j - 1], w);
}

struct KcorrArgs {
  const double2* root[3];
  int n[3];
  int N[3];
  // output slice of transfer m, or -1 to skip it (compacted output); slot[m] <= m
  int slot[64];
  int col0;  // grid index of column 0 (grid columns)
};

// out[m][P][c] = e^{i q_m.(r_P - r_c)} (1/N_k) DFT_k(|DFT_k in|^2)[m]
//             = e^{i q_m.(r_P - r_c)} sum_n in[n][P][c] conj in[n+m][P][c]
template <typename T, int N1, int N2, int N3>
// `in` and `out` may alias (in place): each thread reads all of its inputs
// before it writes, and writes only its own element of each slice (slices may
// be compacted: transfer m goes to slice slot[m] <= m, or nowhere).
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
  int gc = cols_are_points ? pts[c] : ka.col0 + c;
  int c1 = gc / n23, c2 = (gc / ka.n[2]) % ka.n[1], c3 = gc % ka.n[2];
  double2 w1[N1], w2[N2], w3[N3];
  axis_powers<N1>(ka.root[0], p1, c1, N1, w1);
  axis_powers<N2>(ka.root[1], p2, c2, N2, w2);
  axis_powers<N3>(ka.root[2], p3, c3, N3, w3);
#pragma unroll
  for (int m = 0; m < NK; ++m) {
    const int m1 = m / (N2 * N3), m2 = (m / N3) % N2, m3 = m % N3;
    const int sm = ka.slot[m];
    if (sm < 0) continue;
    cplx<T> v = cscale<T>(a[m], inv);
    if (m) {
      const double2 ph = zmul(zmul(w1[m1], w2[m2]), w3[m3]);  // e^{iq.(r_P - r_c)}
      v = cmul<T>(v, mk<T>((T)ph.x, (T)ph.y));
    }
    out[(long)sm * total + idx] = v;
  }
}

// Meshes whose every axis has N_i <= 2: every transfer m satisfies 2m = 0 on
// the mesh, so the unphased sums sum_n in[n] o conj in[n+m] are real (the
// conjugate sum is the same sum with n relabelled n + m). This kernel writes
// that real value: to a real array (grid columns) or as a complex number with
// zero imaginary part (point columns, for the metric).
template <typename T, typename TO, int N1, int N2, int N3>
__global__ __launch_bounds__(256) void kcorr_real_kernel(const cplx<T>* __restrict__ in,
                                                         TO* __restrict__ out, int ni, int ncol) {
  constexpr int NK = N1 * N2 * N3;
  const long total = (long)ni * ncol;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
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
#pragma unroll
  for (int m = 0; m < NK; ++m) {
    if constexpr (sizeof(TO) == 2 * sizeof(T))
      out[(long)m * total + idx] = mk<T>(a[m].x * inv, 0);
    else
      out[(long)m * total + idx] = (TO)(a[m].x * inv);
  }
}

// ---------------------------------------------------------------------------
// Real path, Gamma and the k-correlation fused: a workgroup (4 waves stacked
// along P) owns a 64 x (16 WN) tile of (P, r). For every k-point n the product
// Gamma^n = occ^n conj(psi^n) of that tile accumulates in matrix registers
// (occ in the storage type T)
// (four real MFMAs per complex step, FP32 or FP64 matrix cores by T); then each
// lane forms Z~[m] = (1/N_k) DFT_k(|DFT_k Gamma|^2)[m] for its elements, which is
// real on these meshes, and only Z~ is written. Gamma never reaches memory.
// ---------------------------------------------------------------------------
typedef float gk_f4 __attribute__((ext_vector_type(4)));
typedef double gk_d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct GkMma;
template <>
struct GkMma<float> {
  using acc = gk_f4;
  static __device__ acc zero() { return acc{0, 0, 0, 0}; }
  static __device__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // register v of a lane holds row 4 (lane/16) + v, column lane % 16
  static __device__ int row(int lk, int v) { return 4 * lk + v; }
};
template <>
struct GkMma<double> {
  using acc = gk_d4;
  static __device__ acc zero() { return acc{0, 0, 0, 0}; }
  static __device__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // register v of a lane holds row 4 v + lane/16, column lane % 16
  static __device__ int row(int lk, int v) { return 4 * v + lk; }
};

template <typename T, typename TZ, int N1, int N2, int N3, int WN>
__global__ __launch_bounds__(256) void gamma_kcorr_kernel(int ni, int ng, int no, int nrt,
                                                          long ntiles, long ntiles_pad,
                                                          const cplx<T>* __restrict__ occ,
                                                          const cplx<T>* __restrict__ psi,
                                                          TZ* __restrict__ Z) {
  using M = GkMma<T>;
  using acc_t = typename M::acc;
  constexpr int NK = N1 * N2 * N3;
  constexpr int NPF = 3;
  const long per = ntiles_pad / 8;
  const long t = (blockIdx.x % 8) * per + blockIdx.x / 8;  // XCD-contiguous tile ranges
  if (t >= ntiles) return;
  const int rt = (int)(t % nrt);
  const long ct = t / nrt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = rt * 64 + wave * 16;
  const long col0 = ct * (16 * WN);
  const int ra = min(row0 + li, ni - 1);
  unsigned boff[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long c = col0 + 16 * j + li;
    boff[j] = (unsigned)(c < ng ? c : ng - 1);
  }
  acc_t are[NK][WN], aim[NK][WN];
#pragma unroll
  for (int n = 0; n < NK; ++n)
#pragma unroll
    for (int j = 0; j < WN; ++j) are[n][j] = aim[n][j] = M::zero();
  // k-steps of 4 per k-point, padded to a multiple of the slot count so that
  // every k-point starts at slot 0; the refills run across k-points (the last
  // slots of k-point n fetch the first steps of n + 1), so the pipeline fills
  // once per tile
  const int nks = ((no + 3) / 4 + NPF - 1) / NPF * NPF;
  cplx<T> fa[NPF];
  cplx<T> fb[NPF][WN];
  // k-point bases are wave-uniform (scalar registers); lane offsets are 32-bit
  // byte offsets (the launcher checks the bytes of one k-point's occ and psi
  // against 2^32), so the loads take a scalar base plus a vector offset
  const unsigned aoff = (unsigned)ra * (unsigned)no, ng32 = (unsigned)ng;
  auto load = [&](int n, int ks, cplx<T>& xa, cplx<T>* xb) {
    if (ks >= nks) {  // first steps of the next k-point (clamped past the last)
      ks -= nks;
      n = n + 1 < NK ? n + 1 : NK - 1;
    }
    const char* An = (const char*)(occ + (long)n * ni * no);
    const char* Bn = (const char*)(psi + (long)n * no * ng);
    const int k = 4 * ks + lk;
    const unsigned kc = (unsigned)(k < no ? k : no - 1);
    constexpr unsigned es = sizeof(cplx<T>);
    xa = *(const cplx<T>*)(An + (aoff + kc) * es);
#pragma unroll
    for (int j = 0; j < WN; ++j) xb[j] = *(const cplx<T>*)(Bn + (kc * ng32 + boff[j]) * es);
  };
#pragma unroll
  for (int s = 0; s < NPF; ++s) load(0, s, fa[s], fb[s]);
  // the first loads land before the loops, so that the wait counts at the loop
  // heads see only the loops' own refills
  __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
  for (int n = 0; n < NK; ++n) {
    for (int it = 0; it < nks; it += NPF) {
#pragma unroll
      for (int s = 0; s < NPF; ++s) {
        const int ks = it + s;
        const bool kin = 4 * ks + lk < no;
        // Gamma = A conj(B): Re += ar br + ai bi, Im += ai br - ar bi
        const T ar = kin ? fa[s].x : (T)0, ai = kin ? fa[s].y : (T)0;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const T br = (T)fb[s][j].x, bi = (T)fb[s][j].y;
          are[n][j] = M::mma(ar, br, are[n][j]);
          are[n][j] = M::mma(ai, bi, are[n][j]);
          aim[n][j] = M::mma(ai, br, aim[n][j]);
          aim[n][j] = M::mma(-ar, bi, aim[n][j]);
        }
        __builtin_amdgcn_sched_barrier(0);
        load(n, ks + NPF, fa[s], fb[s]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // each lane round-trips its accumulators through its wave's LDS slice (keeps
  // them in matrix registers during the loops), then correlates over the mesh
  __shared__ T stage[4][2 * NK][64];
  typedef __attribute__((address_space(3))) volatile T lds_t;
  lds_t* sw = (lds_t*)&stage[wave][0][0];
  const T inv = (T)1 / (T)NK;
  const long nz = (long)ni * ng;
#pragma unroll
  for (int j = 0; j < WN; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int n = 0; n < NK; ++n) {
        sw[(2 * n) * 64 + lane] = are[n][j][v];
        sw[(2 * n + 1) * 64 + lane] = aim[n][j][v];
      }
      cplx<T> a[NK];
#pragma unroll
      for (int n = 0; n < NK; ++n) a[n] = mk<T>(sw[(2 * n) * 64 + lane], sw[(2 * n + 1) * 64 + lane]);
      if (NK > 1) {
        kdft3<T, N1, N2, N3>(a);
#pragma unroll
        for (int n = 0; n < NK; ++n) a[n] = mk<T>(a[n].x * a[n].x + a[n].y * a[n].y, 0);
        kdft3<T, N1, N2, N3>(a);
      } else {
        a[0] = mk<T>(a[0].x * a[0].x + a[0].y * a[0].y, 0);
      }
      const int r = row0 + M::row(lk, v);
      const long c = col0 + 16 * j + li;
      if (r < ni && c < ng) {
        TZ* dst = Z + (long)r * ng + c;
#pragma unroll
        for (int m = 0; m < NK; ++m) dst[(long)m * nz] = (TZ)(a[m].x * inv);
      }
    }
}

// ---------------------------------------------------------------------------
// BF16 form of the fused Gamma + real k-correlation. Same tile and lane roles as
// gamma_kcorr_kernel, with v_mfma_f32_16x16x32_bf16: a k-step covers 32 occupied
// orbitals, lane group lk = lane/16 holds orbitals 8 lk .. 8 lk + 7 of its row
// (occ) or column (psi), rounded to bfloat16; the same (lk, item) pairing on both
// operands makes the instruction sum over all 32. FP32 accumulation.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 as_bf16x8(u16x8 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

template <typename TZ, int N1, int N2, int N3, int WN>
__global__ __launch_bounds__(256) void gamma_kcorr_bf16_kernel(int ni, int ng, int no, int nrt,
                                                               long ntiles, long ntiles_pad,
                                                               const float2* __restrict__ occ,
                                                               const float2* __restrict__ psi,
                                                               TZ* __restrict__ Z) {
  constexpr int NK = N1 * N2 * N3;
  const long per = ntiles_pad / 8;
  const long t = (blockIdx.x % 8) * per + blockIdx.x / 8;  // XCD-contiguous tile ranges
  if (t >= ntiles) return;
  const int rt = (int)(t % nrt);
  const long ct = t / nrt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = rt * 64 + wave * 16;
  const long col0 = ct * (16 * WN);
  const int ra = min(row0 + li, ni - 1);
  long bcol[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long c = col0 + 16 * j + li;
    bcol[j] = c < ng ? c : ng - 1;
  }
  gk_f4 are[NK][WN], aim[NK][WN];
#pragma unroll
  for (int n = 0; n < NK; ++n)
#pragma unroll
    for (int j = 0; j < WN; ++j) are[n][j] = aim[n][j] = gk_f4{0, 0, 0, 0};
  const int nks = (no + 31) / 32;
#pragma unroll
  for (int n = 0; n < NK; ++n) {
    const float2* An = occ + ((long)n * ni + ra) * no;
    const float2* Bn = psi + (long)n * no * ng;
    for (int ks = 0; ks < nks; ++ks) {
      const int k0 = 32 * ks + 8 * lk;
      u16x8 ar, ai, nar;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        const float2 a = k < no ? An[k] : make_float2(0.f, 0.f);
        ar[e] = bf16_rne(a.x);
        ai[e] = bf16_rne(a.y);
        nar[e] = ar[e] ^ 0x8000u;
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        u16x8 br, bi;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = min(k0 + e, no - 1);  // the A side is zero past no
          const float2 b = Bn[(long)k * ng + bcol[j]];
          br[e] = bf16_rne(b.x);
          bi[e] = bf16_rne(b.y);
        }
        // Gamma = A conj(B): Re += ar br + ai bi, Im += ai br - ar bi
        are[n][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ar), as_bf16x8(br),
                                                            are[n][j], 0, 0, 0);
        are[n][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ai), as_bf16x8(bi),
                                                            are[n][j], 0, 0, 0);
        aim[n][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ai), as_bf16x8(br),
                                                            aim[n][j], 0, 0, 0);
        aim[n][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(nar), as_bf16x8(bi),
                                                            aim[n][j], 0, 0, 0);
      }
    }
  }
  // the k-mesh correlation of each element, as in gamma_kcorr_kernel
  __shared__ float stage[4][2 * NK][64];
  typedef __attribute__((address_space(3))) volatile float lds_t;
  lds_t* sw = (lds_t*)&stage[wave][0][0];
  const float inv = 1.0f / (float)NK;
  const long nz = (long)ni * ng;
#pragma unroll
  for (int j = 0; j < WN; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int n = 0; n < NK; ++n) {
        sw[(2 * n) * 64 + lane] = are[n][j][v];
        sw[(2 * n + 1) * 64 + lane] = aim[n][j][v];
      }
      cplx<float> a[NK];
#pragma unroll
      for (int n = 0; n < NK; ++n)
        a[n] = mk<float>(sw[(2 * n) * 64 + lane], sw[(2 * n + 1) * 64 + lane]);
      if (NK > 1) {
        kdft3<float, N1, N2, N3>(a);
#pragma unroll
        for (int n = 0; n < NK; ++n) a[n] = mk<float>(a[n].x * a[n].x + a[n].y * a[n].y, 0);
        kdft3<float, N1, N2, N3>(a);
      } else {
        a[0] = mk<float>(a[0].x * a[0].x + a[0].y * a[0].y, 0);
      }
      const int r = row0 + 4 * lk + v;
      const long c = col0 + 16 * j + li;
      if (r < ni && c < ng) {
        TZ* dst = Z + (long)r * ng + c;
#pragma unroll
        for (int m = 0; m < NK; ++m) dst[(long)m * nz] = (TZ)(a[m].x * inv);
      }
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
  X(3, 1, 1)              \
  X(3, 2, 1)              \
  X(1, 2, 3)

// meshes with a compile-time kernel (register-resident k-mesh DFTs); any other
// mesh of at most 64 points takes kcorr_direct_kernel
static bool kcorr_compiled(const Geom& g) {
#define EXX_KSUP(a, b, c) \
  if (g.N[0] == a && g.N[1] == b && g.N[2] == c) return true;
  EXX_KMESH_LIST(EXX_KSUP)
#undef EXX_KSUP
  return false;
}

bool kcorr_supported(const Geom& g) { return g.nk >= 1 && g.nk <= 64; }

// Any mesh of at most 64 points: the k-correlation by its direct sum,
// out[slot[m]][P][c] = e^{i q_m.(r_P - r_c)} sum_n in[n][P][c] conj in[n+m][P][c]
// (n + m per axis mod N). Each thread first copies its element of every slice
// (in and out may alias, as in kcorr_kernel), then forms the N_k sums.
template <typename T>
__global__ __launch_bounds__(256) void kcorr_direct_kernel(const cplx<T>* in, cplx<T>* out, int ni,
                                                           int ncol, const int32_t* __restrict__ pts,
                                                           int cols_are_points, KcorrArgs ka) {
  const int N1 = ka.N[0], N2 = ka.N[1], N3 = ka.N[2];
  const int nk = N1 * N2 * N3;
  const long total = (long)ni * ncol;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int P = (int)(idx / ncol);
  const int c = (int)(idx % ncol);
  cplx<T> a[64];
  for (int n = 0; n < nk; ++n) a[n] = in[(long)n * total + idx];
  const int n23 = ka.n[1] * ka.n[2];
  const int gp = pts[P];
  const int p1 = gp / n23, p2 = (gp / ka.n[2]) % ka.n[1], p3 = gp % ka.n[2];
  const int gc = cols_are_points ? pts[c] : ka.col0 + c;
  const int c1 = gc / n23, c2 = (gc / ka.n[2]) % ka.n[1], c3 = gc % ka.n[2];
  double2 w1[8], w2[8], w3[8];  // mesh axes are at most 8 points long
  axis_powers<8>(ka.root[0], p1, c1, N1, w1);
  axis_powers<8>(ka.root[1], p2, c2, N2, w2);
  axis_powers<8>(ka.root[2], p3, c3, N3, w3);
  for (int m = 0; m < nk; ++m) {
    const int sm = ka.slot[m];
    if (sm < 0) continue;
    const int m1 = m / (N2 * N3), m2 = (m / N3) % N2, m3 = m % N3;
    cplx<T> v = mk<T>(0, 0);
    for (int n = 0; n < nk; ++n) {
      const int n1 = n / (N2 * N3), n2 = (n / N3) % N2, n3 = n % N3;
      const int q = (((n1 + m1) % N1) * N2 + (n2 + m2) % N2) * N3 + (n3 + m3) % N3;
      v = cadd<T>(v, cmulc<T>(a[n], a[q]));
    }
    if (m) {
      const double2 ph = zmul(zmul(w1[m1], w2[m2]), w3[m3]);  // e^{iq.(r_P - r_c)}
      v = cmul<T>(v, mk<T>((T)ph.x, (T)ph.y));
    }
    out[(long)sm * total + idx] = v;
  }
}

// ---------------------------------------------------------------------------
// 4 x 4 x 4 meshes: one element's 64 values span a lane quad. Lane q of the
// quad holds the 16 values of first-axis index q; the DFTs along the other two
// axes run in the lane, the one along the first axis across the quad with DPP
// broadcasts (quad_perm [j, j, j, j] reads lane j of each quad). A thread then
// holds 16 values instead of 64, so the FP64 form stays within the register
// file (the one-thread form spills there). Same results as kcorr_kernel; in and
// out may alias: a quad's lanes are in one wavefront, and every store depends
// on values exchanged after all four lanes' loads.
// ---------------------------------------------------------------------------
template <int J>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), J * 0x55, 0xF, 0xF,
                                                    false));
}
template <int J>
__device__ __forceinline__ double quad_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), J * 0x55, 0xF, 0xF,
                                             false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), J * 0x55, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// v (-i)^r for a run-time r in 0..3, without branches: odd r swaps the parts,
// and the real (imaginary) part changes sign for r = 2, 3 (r = 1, 2)
template <typename T>
__device__ __forceinline__ cplx<T> mul_mi_pow(cplx<T> v, int r) {
  const bool odd = (r & 1) != 0;
  const T re = odd ? v.y : v.x, im = odd ? v.x : v.y;
  return mk<T>(r >= 2 ? -re : re, (r == 1 || r == 2) ? -im : im);
}

// X_q = sum_j x_j e^{-2 pi i j q / 4} across the quad, for lane q
template <typename T>
__device__ __forceinline__ cplx<T> quad_dft(cplx<T> x, int q) {
  const cplx<T> x0 = mk<T>(quad_bcast<0>(x.x), quad_bcast<0>(x.y));
  const cplx<T> x1 = mk<T>(quad_bcast<1>(x.x), quad_bcast<1>(x.y));
  const cplx<T> x2 = mk<T>(quad_bcast<2>(x.x), quad_bcast<2>(x.y));
  const cplx<T> x3 = mk<T>(quad_bcast<3>(x.x), quad_bcast<3>(x.y));
  cplx<T> acc = cadd<T>(x0, mul_mi_pow<T>(x1, q & 3));
  acc = cadd<T>(acc, mul_mi_pow<T>(x2, (2 * q) & 3));
  return cadd<T>(acc, mul_mi_pow<T>(x3, (3 * q) & 3));
}

template <typename T>
__global__ __launch_bounds__(256) void kcorr_quad_kernel(const cplx<T>* in, cplx<T>* out, int ni,
                                                         int ncol, const int32_t* __restrict__ pts,
                                                         int cols_are_points, KcorrArgs ka) {
  constexpr int NL = 16;  // values per lane (second and third axes)
  const long total = (long)ni * ncol;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long idx = tid >> 2;  // element (all four lanes of a quad share it)
  const int q = (int)(tid & 3);
  if (idx >= total) return;
  const int P = (int)(idx / ncol);
  const int c = (int)(idx % ncol);
  cplx<T> a[NL];
#pragma unroll
  for (int p = 0; p < NL; ++p) a[p] = in[(long)(q * NL + p) * total + idx];
  kdft_axis<T, 1, 4, 4, 2>(a);
  kdft_axis<T, 1, 4, 4, 1>(a);
  // one position at a time across the quad (the barriers keep the scheduler
  // from hoisting all 64 broadcasts, whose temporaries would fill the registers)
#pragma unroll
  for (int p = 0; p < NL; ++p) {
    a[p] = quad_dft<T>(a[p], q);
    a[p] = mk<T>(a[p].x * a[p].x + a[p].y * a[p].y, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int p = 0; p < NL; ++p) {
    a[p] = quad_dft<T>(a[p], q);
    __builtin_amdgcn_sched_barrier(0);
  }
  kdft_axis<T, 1, 4, 4, 2>(a);
  kdft_axis<T, 1, 4, 4, 1>(a);
  const T inv = (T)1 / (T)64;
  const int n23 = ka.n[1] * ka.n[2];
  const int gp = pts[P];
  const int p1 = gp / n23, p2 = (gp / ka.n[2]) % ka.n[1], p3 = gp % ka.n[2];
  const int gc = cols_are_points ? pts[c] : ka.col0 + c;
  const int c1 = gc / n23, c2 = (gc / ka.n[2]) % ka.n[1], c3 = gc % ka.n[2];
  double2 w1[4], w2[4], w3[4];
  axis_powers<4>(ka.root[0], p1, c1, 4, w1);
  axis_powers<4>(ka.root[1], p2, c2, 4, w2);
  axis_powers<4>(ka.root[2], p3, c3, 4, w3);
  // this lane's first-axis factor w1^q without indexing the array by q
  double2 f1 = w1[0];
#pragma unroll
  for (int j = 1; j < 4; ++j)
    if (j == q) f1 = w1[j];
#pragma unroll
  for (int p = 0; p < NL; ++p) {
    const int m = q * NL + p;
    const int sm = ka.slot[m];
    if (sm < 0) continue;
    cplx<T> v = cscale<T>(a[p], inv);
    const double2 ph = zmul(zmul(f1, w2[p / 4]), w3[p % 4]);  // e^{iq.(r_P - r_c)}
    v = cmul<T>(v, mk<T>((T)ph.x, (T)ph.y));
    out[(long)sm * total + idx] = v;
  }
}

template <typename T>
hipError_t launch_kcorr(const Geom& g, const Tables& tb, const void* in, void* out, int ncol,
                        const int32_t* pts, bool cols_are_points, hipStream_t st,
                        const int* slot, int col0) {
  KcorrArgs ka;
  ka.col0 = col0;
  for (int a = 0; a < 3; ++a) {
    ka.root[a] = tb.root[a];
    ka.n[a] = g.n[a];
    ka.N[a] = g.N[a];
  }
  for (int m = 0; m < 64; ++m) ka.slot[m] = slot ? slot[m] : m;
  long total = (long)g.ni * ncol;
  dim3 grid((unsigned)((total + 255) / 256));
  if (g.N[0] == 4 && g.N[1] == 4 && g.N[2] == 4) {
    hipLaunchKernelGGL(kcorr_quad_kernel<T>, dim3((unsigned)((4 * total + 255) / 256)), dim3(256),
                       0, st, (const cplx<T>*)in, (cplx<T>*)out, g.ni, ncol, pts,
                       cols_are_points ? 1 : 0, ka);
    return hipGetLastError();
  }
#define EXX_KLAUNCH(a, b, c)                                                                    \
  if (g.N[0] == a && g.N[1] == b && g.N[2] == c) {                                              \
    hipLaunchKernelGGL((kcorr_kernel<T, a, b, c>), grid, dim3(256), 0, st, (const cplx<T>*)in,  \
                       (cplx<T>*)out, g.ni, ncol, pts, cols_are_points ? 1 : 0, ka);                             \
    return hipGetLastError();                                                                   \
  }
  EXX_KMESH_LIST(EXX_KLAUNCH)
#undef EXX_KLAUNCH
  if (!kcorr_compiled(g) && kcorr_supported(g)) {
    hipLaunchKernelGGL((kcorr_direct_kernel<T>), grid, dim3(256), 0, st, (const cplx<T>*)in,
                       (cplx<T>*)out, g.ni, ncol, pts, cols_are_points ? 1 : 0, ka);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
bool kcorr_real(const Geom& g) { return g.N[0] <= 2 && g.N[1] <= 2 && g.N[2] <= 2; }

// unphased real k-correlation (meshes with every N_i <= 2): grid columns to a
// real array of TO, or point columns (ncol = N_ISDF) to a complex matrix
template <typename T, typename TO>
hipError_t launch_kcorr_real(const Geom& g, const void* in, void* out, int ncol, hipStream_t st) {
  long total = (long)g.ni * ncol;
  dim3 grid((unsigned)((total + 255) / 256));
#define EXX_KRLAUNCH(a, b, c)                                                                    \
  if (g.N[0] == a && g.N[1] == b && g.N[2] == c) {                                               \
    hipLaunchKernelGGL((kcorr_real_kernel<T, TO, a, b, c>), grid, dim3(256), 0, st,              \
                       (const cplx<T>*)in, (TO*)out, g.ni, ncol);                                 \
    return hipGetLastError();                                                                    \
  }
  EXX_KRLAUNCH(1, 1, 1)
  EXX_KRLAUNCH(2, 2, 2)
  EXX_KRLAUNCH(2, 1, 1)
  EXX_KRLAUNCH(1, 2, 1)
  EXX_KRLAUNCH(1, 1, 2)
  EXX_KRLAUNCH(2, 2, 1)
  EXX_KRLAUNCH(2, 1, 2)
  EXX_KRLAUNCH(1, 2, 2)
#undef EXX_KRLAUNCH
  return hipErrorInvalidValue;
}
template hipError_t launch_kcorr_real<double, double>(const Geom&, const void*, void*, int,
                                                      hipStream_t);
template hipError_t launch_kcorr_real<float, float>(const Geom&, const void*, void*, int,
                                                    hipStream_t);
template hipError_t launch_kcorr_real<double, double2>(const Geom&, const void*, void*, int,
                                                       hipStream_t);

__global__ __launch_bounds__(256) void narrow_kernel(const double2* __restrict__ in,
                                                     float2* __restrict__ out, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

hipError_t launch_narrow(const double2* in, float2* out, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out,
                     n);
  return hipGetLastError();
}

// fused Gamma + real k-correlation of the real path: T is the storage of occ
// and psi and the matrix-core precision, TZ that of Z~
template <typename T, typename TZ>
hipError_t launch_gamma_kcorr(const Geom& g, const void* occ, const void* psi, void* Z,
                              hipStream_t st) {
  constexpr int WN = sizeof(T) == 4 ? 2 : 1;
  const int nrt = (g.ni + 63) / 64;
  const long nct = ((long)g.ng + 16 * WN - 1) / (16 * WN);
  const long ntiles = nrt * nct;
  const long pad = (ntiles + 7) / 8 * 8;
  const long es = (long)sizeof(cplx<T>);
  if ((long)g.no * g.ng * es >= 0xffffffffL || (long)g.ni * g.no * es >= 0xffffffffL)
    return hipErrorInvalidValue;
#define EXX_GKLAUNCH(a, b, c)                                                                    \
  if (g.N[0] == a && g.N[1] == b && g.N[2] == c) {                                               \
    hipLaunchKernelGGL((gamma_kcorr_kernel<T, TZ, a, b, c, WN>), dim3((unsigned)pad), dim3(256), \
                       0, st, g.ni, g.ng, g.no, nrt, ntiles, pad, (const cplx<T>*)occ,           \
                       (const cplx<T>*)psi, (TZ*)Z);                                             \
    return hipGetLastError();                                                                    \
  }
  EXX_GKLAUNCH(1, 1, 1)
  EXX_GKLAUNCH(2, 2, 2)
  EXX_GKLAUNCH(2, 1, 1)
  EXX_GKLAUNCH(1, 2, 1)
  EXX_GKLAUNCH(1, 1, 2)
  EXX_GKLAUNCH(2, 2, 1)
  EXX_GKLAUNCH(2, 1, 2)
  EXX_GKLAUNCH(1, 2, 2)
#undef EXX_GKLAUNCH
  return hipErrorInvalidValue;
}
template hipError_t launch_gamma_kcorr<float, float>(const Geom&, const void*, const void*, void*,
                                                     hipStream_t);

hipError_t launch_gamma_kcorr_bf16(const Geom& g, const void* occ, const void* psi, void* Z,
                                   hipStream_t st) {
  constexpr int WN = 2;
  const int nrt = (g.ni + 63) / 64;
  const long nct = ((long)g.ng + 16 * WN - 1) / (16 * WN);
  const long ntiles = nrt * nct;
  const long pad = (ntiles + 7) / 8 * 8;
#define EXX_GKB(a, b, c)                                                                         \
  if (g.N[0] == a && g.N[1] == b && g.N[2] == c) {                                               \
    hipLaunchKernelGGL((gamma_kcorr_bf16_kernel<float, a, b, c, WN>), dim3((unsigned)pad),       \
                       dim3(256), 0, st, g.ni, g.ng, g.no, nrt, ntiles, pad, (const float2*)occ, \
                       (const float2*)psi, (float*)Z);                                           \
    return hipGetLastError();                                                                    \
  }
  EXX_GKB(1, 1, 1)
  EXX_GKB(2, 2, 2)
  EXX_GKB(2, 1, 1)
  EXX_GKB(1, 2, 1)
  EXX_GKB(1, 1, 2)
  EXX_GKB(2, 2, 1)
  EXX_GKB(2, 1, 2)
  EXX_GKB(1, 2, 2)
#undef EXX_GKB
  return hipErrorInvalidValue;
}

template hipError_t launch_kcorr<double>(const Geom&, const Tables&, const void*, void*, int,
                                          const int32_t*, bool, hipStream_t, const int*, int);
template hipError_t launch_kcorr<float>(const Geom&, const Tables&, const void*, void*, int,
                                          const int32_t*, bool, hipStream_t, const int*, int);

// out[e] = sum_s in[s * stride + e], e < n (out may be slice 0 of in: each
// element is read for every slice before it is written)
template <typename T>
__global__ __launch_bounds__(256) void sum_slices_kernel(const cplx<T>* in, cplx<T>* out, long n,
                                                         int nslice, long stride) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  T re = 0, im = 0;
  for (int s = 0; s < nslice; ++s) {
    const cplx<T> v = in[(long)s * stride + e];
    re += v.x;
    im += v.y;
  }
  out[e] = mk<T>(re, im);
}

template <typename T>
hipError_t launch_sum_slices(const void* in, void* out, long n, int nslice, long stride,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_slices_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const cplx<T>*)in, (cplx<T>*)out, n, nslice, stride);
  return hipGetLastError();
}
template hipError_t launch_sum_slices<double>(const void*, void*, long, int, long, hipStream_t);
template hipError_t launch_sum_slices<float>(const void*, void*, long, int, long, hipStream_t);

}  // namespace exx

// Shared device helpers and internal declarations of the exchange library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/exx.h"

namespace exx {

// ---------------------------------------------------------------------------
// complex helpers: float2 / double2 storage, arithmetic in the element type
// ---------------------------------------------------------------------------
template <typename T> struct c2t;
template <> struct c2t<double> { using type = double2; };
template <> struct c2t<float> { using type = float2; };
template <typename T> using cplx = typename c2t<T>::type;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T x, T y) {
  cplx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x - b.x, a.y - b.y);
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) {
  return mk<T>(a.x, -a.y);
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) {
  return mk<T>(a.x * s, a.y * s);
}
// load an element of storage type S and widen/narrow it to compute type T
template <typename T, typename S>
__device__ __forceinline__ cplx<T> cload(const cplx<S>* p) {
  cplx<S> v = *p;
  return mk<T>((T)v.x, (T)v.y);
}
template <typename S, typename T>
__device__ __forceinline__ void cstore(cplx<S>* p, cplx<T> v) {
  *p = mk<S>((S)v.x, (S)v.y);
}

// bfloat16 by round-to-nearest-even of an FP32 value (finite inputs): the top
// 16 bits of x + 0x7fff + (bit 16 of x)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__host__ __device__ __forceinline__ int wrap_sym(int x, int L) {
  // ((x + floor(L/2)) mod L) - floor(L/2), with a non-negative mod
  int h = L / 2;
  int t = (x + h) % L;
  if (t < 0) t += L;
  return t - h;
}

// ---------------------------------------------------------------------------
// geometry passed to kernels by value
// ---------------------------------------------------------------------------
struct Geom {
  double L[3];
  int n[3];    // grid
  int N[3];    // k-mesh
  int nk, ng, no, nao, ni;
  double omega;
};

Geom make_geom(const exx_cell& c);

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
};

}  // namespace exx

struct exx_context {
  int device = 0;
  std::string err;
  exx::Arena ws;            // grid-sized scratch + small matrices
  // caller-owned workspace (exx_set_workspace): when set, every scratch request
  // is served from it and the library allocates no scratch of its own
  char* user_ws = nullptr;
  size_t user_ws_bytes = 0;
  // device status words (exx_get_status): [0] flag bits, [1] first transfer
  // whose metric lost a pivot under EXX_STRICT_PD, [2] first non-finite site
  int32_t* dstat = nullptr;
  int checks = 1;           // EXX_CHECK_* flags
  // per-axis root tables e^{-2 pi i t / (N_i n_i)} for the Bloch phases and
  // twiddle tables for the FFT, one device buffer per (grid, k-mesh) shape
  struct TabEntry {
    int key[6];
    void* buf;
    size_t bytes;
  };
  std::vector<TabEntry> tabs;
  // persistent small buffers for exx_build
  void* small = nullptr;
  size_t small_cap = 0;
  // wave tiles of the grid GEMMs (see zgemm_nn_grid)
  int tile_gamma = 22;
  int tile_solve = 22;
  // steps of iterative refinement after the fit solve (0 or 1)
  int refine = 0;
  int contract = 0;  // EXX_CONTRACT_* of the Coulomb contraction
  int fit_mode = 0;  // EXX_FIT_* of the fused builds
  // second stream (default priority) for the point-metric chain of the fit,
  // which overlaps the grid-sized Gamma and Z; fork/join events
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // paired path: end of the metric chain, and the two transform buffers'
  // release (their contraction has read them)
  hipEvent_t chain_ev = nullptr;
  hipEvent_t fb_ev[2] = {nullptr, nullptr};
  // grid columns per chunk of the paired path's fit: the Gamma/Z buffer holds
  // at most this many bytes (EXX_FIT_CHUNK_MB overrides)
  size_t fit_chunk_bytes = (size_t)8 << 30;
  int ncu = 256;
  // concurrent lanes of a batched build (lane 0 is the handle's own stream set
  // and scratch; lanes 1.. have their own streams, events and scratch)
  struct Lane {
    hipStream_t st = nullptr, aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr, chain_ev = nullptr, done_ev = nullptr;
    hipEvent_t fb_ev[2] = {nullptr, nullptr};
    char* ws = nullptr;
    size_t cap = 0;
  };
  std::vector<Lane> lanes;
  hipEvent_t batch_ev = nullptr;
  // autotuned wave tiles per size class: key (ni, ng, no, nk, prec) -> (gamma, solve)
  struct Tune {
    long key[5];
    int gamma, solve;
  };
  std::vector<Tune> tuned;
  // cached graphs of batched builds, keyed by a signature of the batch
  struct GraphEntry {
    std::vector<long> sig;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  // per-phase timing: recorded (phase, start, stop) events and a free pool
  bool timing = false;
  // with timing: run the phases that normally overlap (factorisation chain and
  // Gamma; transform and contraction chunks) one after another, so that each
  // phase's events bracket its own kernels only
  bool serial = false;
  struct Rec {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
};

namespace exx {

// status helpers
exx_status fail(exx_context* h, exx_status s, const std::string& msg);
// bits of the device status word
enum StatusBits { ST_NONFINITE = 1, ST_NOT_PD = 2 };
// sites of the first non-finite value (status word [2])
enum FiniteSite { SITE_OCC = 1, SITE_AO = 2, SITE_METRIC = 3, SITE_COULOMB = 4, SITE_OUTPUT = 5 };
// transfer label of each factorised metric (slot s of the batch is transfer q[s])
struct QLabel {
  int q[64];
};
// status[0] |= ST_NONFINITE and status[2] = min(status[2], site) if any of the n
// doubles at p is not finite
hipError_t launch_check_finite(const double* p, long n, int32_t* status, int site,
                               hipStream_t st);
// status = {0, INT_MAX, INT_MAX, 0} (a kernel, so that it can be captured)
hipError_t launch_status_reset(int32_t* status, hipStream_t st);
exx_status hip_check(exx_context* h, hipError_t e, const char* what);

// scratch: returns pointer to >= bytes of workspace (grown on demand)
void* ws_get(exx_context* h, size_t bytes, exx_status* st);

enum Phase {
  PH_GRAM = 0,
  PH_METRIC,
  PH_CHOL,
  PH_PINV,
  PH_GAMMA,
  PH_KCORR,
  PH_SOLVE,
  PH_FFT,
  PH_COULOMB,
  PH_KCONV,
  PH_KMAT,
  PH_ENERGY,
  PH_COUNT
};

// records events around a phase when timing is enabled on the handle
class PhaseTimer {
 public:
  PhaseTimer(exx_context* h, int phase, hipStream_t st);
  ~PhaseTimer();

 private:
  exx_context* h_;
  int phase_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr;
};

// ---------------------------------------------------------------------------
// launchers (each returns hipGetLastError() of its launches)
// ---------------------------------------------------------------------------
enum OpA { A_N = 0, A_C = 1 };           // A[i][k]  or conj(A[k][i])
enum OpB { B_N = 0, B_R = 1, B_C = 2 };  // B[k][j], conj(B[k][j]) or conj(B[j][k])

// C[b] = alpha * opA(A[b]) * opB(B[b]) (+ C[b] if accumulate), complex,
// computed in type T, with storage types TA, TB, TC.
template <typename T, typename TA, typename TB, typename TC>
hipError_t gemm(int M, int N, int K, int batch, OpA oa, const void* A, long lda, long sA, OpB ob,
                const void* B, long ldb, long sB, void* C, long ldc, long sC, T alpha_re,
                bool accumulate, hipStream_t st);

// gemm in FP64 (c128 operands) for a long K (a sum over the grid): the K range is
// split into gemm_splitk_parts(M, N, K, batch) slices whose products go to `part`
// (that many x batch x M x N c128) and are then added in slice order
// (deterministic) into C, scaled by alpha; op cases (A_N, B_C) and (A_N, B_R).
int gemm_splitk_parts(int M, int N, int K, int batch);
hipError_t zgemm_splitk(int M, int N, int K, int batch, OpA oa, const void* A, long lda, long sA,
                        OpB ob, const void* B, long ldb, long sB, void* C, long ldc, long sC,
                        double alpha, bool accumulate, void* part, hipStream_t st);

// slices of C = A B^H (A [M][K], B [N][K] c128) on the FP64 matrix cores:
// part[s][b][M][N] = sum over k in [s kc, min(K, (s + 1) kc)) of A[b][i][k] conj B[b][j][k],
// s < ns; kc a multiple of 8
hipError_t zgemm_abh_parts(int M, int N, int K, int batch, const void* A, long lda, long sA,
                           const void* B, long ldb, long sB, void* part, int ns, int kc,
                           hipStream_t st);

// C[b] = A[b] * op(B[b]) on the matrix cores in FP64: A (M x K) c128, B (K x N) and
// C (M x N) row-major with storage types TB, TC; op = conj if conjB. `tile` picks the
// wave tile in 16x16 blocks (22, 24 or 42; any other value means 24; workgroup =
// 2 x 2 waves). lower: A is lower triangular (each wave's rows stop at the
// diagonal); lower with conjB returns hipErrorInvalidValue.
template <typename TB, typename TC>
hipError_t zgemm_nn_grid(int M, int N, int K, int batch, const void* A, long lda, long sA,
                         bool conjB, const void* B, long ldb, long sB, void* C, long ldc, long sC,
                         hipStream_t st, int tile, bool lower = false);

// C[b] = A[b] * op(B[b]) on the FP32 matrix cores: A c128 (rounded to FP32), B and C c64
hipError_t cgemm_nn_grid32(int M, int N, int K, int batch, const void* A, long lda, long sA,
                          bool conjB, const void* B, long ldb, long sB, void* C, long ldc, long sC,
                          hipStream_t st);

// real form: C[b] = Re(A[b]) B[b], A (M x K) c128, B (K x N) real TB, C real TC;
// lower: A is lower triangular (each 64-row band stops at its diagonal and skips
// the 16-row blocks a k-step cannot reach)
template <typename TB, typename TC>
hipError_t dgemm_nn_grid(int M, int N, int K, int batch, const void* A, long lda, long sA,
                         const void* B, long ldb, long sB, void* C, long ldc, long sC,
                         hipStream_t st, bool lower = false);

// AH[b] = s * A[b]^H for (rows x cols) complex matrices, batch items contiguous
hipError_t launch_conj_transpose(const double2* A, double2* AH, int rows, int cols, int batch,
                                 double s, hipStream_t st);

// Small real FP64 product C[b] = alpha A[b] B[b] (+ C[b] if acc), M x K times
// K x N, with operands given by element strides in doubles: A(r, k) =
// A[b sA + r ar + k ak], B(k, c) = B[b sB + k bk + c bc], C(r, c) =
// C[b sC + r cr + c cc]. Strided views cover transposes and the real parts of
// complex storage. cplx_out: C is complex storage (cr, cc, sC even) and gets
// (x, 0). Offsets within one batch item are 32-bit. Invalid strides return
// hipErrorInvalidValue.
struct StridedGemm {
  long sA, sB, sC;
  int ar, ak, bk, bc, cr, cc;
  int M, N, K;
};
hipError_t dgemm_strided(const StridedGemm& s, int batch, const double* A, const double* B,
                         double* C, bool cplx_out, hipStream_t st, double alpha = 1.0,
                         bool acc = false);
// real form of the accumulating product: C[b] = C[b] + sign Re(A[b]) B[b]
// (sign = +1 or -1, sum in FP64), same operands as dgemm_nn_grid
template <typename TB, typename TC>
hipError_t dgemm_nn_grid_acc(int M, int N, int K, int batch, const void* A, long lda, long sA,
                             const void* B, long ldb, long sB, void* C, long ldc, long sC,
                             int sign, hipStream_t st, bool lower = false);
// zero the strict upper triangle of N_k complex n x n matrices
hipError_t launch_zero_upper(double2* A, int n, int batch, hipStream_t st);
// C[b] = C[b] + sign * A[b] * B[b] (sign = +1 or -1), same operands as zgemm_nn_grid
// (tile 22, no conjugation); used by the iterative refinement of the fit
template <typename TB, typename TC>
hipError_t zgemm_nn_grid_acc(int M, int N, int K, int batch, const void* A, long lda, long sA,
                             const void* B, long ldb, long sB, void* C, long ldc, long sC,
                             int sign, hipStream_t st);

// Gamma^n(P, r) = sum_i occ[n][P][i] conj psi[n][i][r]  (fit right-hand side factor)
template <typename T>
hipError_t launch_gamma(const Geom& g, const void* occ_pts, const void* psi, void* gam,
                        hipStream_t st);

// Per-axis phase tables: tab[a][t] = exp(-2 pi i t / (N_a n_a)), t in [0, N_a n_a)
// FFT twiddles: tw[a][t] = exp(-2 pi i t / n_a)
struct Tables {
  const double2* root[3];
  const double2* tw64[3];
  const float2* tw32[3];
};
exx_status get_tables(exx_context* h, const Geom& g, Tables* t, hipStream_t st);

// k-autocorrelation with Bloch phase:
// out[m][P][c] = e^{i q_m.(r_P - r_c)} sum_n in[n][P][c] conj in[n+m][P][c]
// columns c are grid points (cols_are_points false) or the points pts[c].
// slot (64 entries, host): transfer m goes to output slice slot[m] <= m, or is
// skipped for -1; nullptr writes every m to slice m.
// col0: grid index of column 0 (grid columns: column c is grid point col0 + c).
template <typename T>
hipError_t launch_kcorr(const Geom& g, const Tables& tb, const void* in, void* out, int ncol,
                        const int32_t* pts, bool cols_are_points, hipStream_t st,
                        const int* slot = nullptr, int col0 = 0);
bool kcorr_supported(const Geom& g);
// meshes whose every axis has N_i <= 2 (all transfers self-conjugate)
bool kcorr_real(const Geom& g);
// unphased real k-correlation: out[m][P][c] = sum_n in[n][P][c] conj in[n+m][P][c]
// (real there); TO real for grid columns, double2 (imaginary part 0) for points
template <typename T, typename TO>
hipError_t launch_kcorr_real(const Geom& g, const void* in, void* out, int ncol, hipStream_t st);
// c128 -> c64, n elements
hipError_t launch_narrow(const double2* in, float2* out, long n, hipStream_t st);
// real path, Gamma^n = occ^n conj(psi^n) and the real k-correlation fused:
// Z~ [N_k][N_ISDF][N_g] (TZ) from occ [N_k][N_ISDF][n_occ] and psi, both storage T
template <typename T, typename TZ>
hipError_t launch_gamma_kcorr(const Geom& g, const void* occ, const void* psi, void* Z,
                              hipStream_t st);

// BF16 form of launch_gamma_kcorr: occ and psi (c64) rounded to bfloat16 at
// load, products on the BF16 matrix cores with FP32 accumulation, Z~ in FP32
hipError_t launch_gamma_kcorr_bf16(const Geom& g, const void* occ, const void* psi, void* Z,
                                   hipStream_t st);
// BF16 form of cgemm_nn_grid32 with conjB: C = A conj(B), A c128 and B c64 rounded
// to bfloat16 at load, BF16 matrix cores, FP32 accumulation, C c64
hipError_t cgemm_nn_grid_bf16(int M, int N, int K, int batch, const void* A, long lda, long sA,
                              const void* B, long ldb, long sB, void* C, long ldc, long sC,
                              hipStream_t st);

// dst[0:n] = src[0:n] (a kernel, so that captured sequences hold no copy nodes)
hipError_t launch_copy(double2* dst, const double2* src, long n, hipStream_t st);
// dst[0:n] = src[0:n] for complex arrays, converting storage TS to TD
template <typename TS, typename TD>
hipError_t launch_convert(const void* src, void* dst, long n, hipStream_t st);
// rank[rep[s]] = rc[s], and rank[bar[s]] = rc[s] where bar[s] >= 0 (host lists, n <= 64)
hipError_t launch_rank_scatter(const int32_t* rc, int32_t* rank, const int* rep, const int* bar,
                               int n, hipStream_t st);
// rank[m] = rc[0], m < nk (<= 64)
hipError_t launch_rank_broadcast(const int32_t* rc, int32_t* rank, int nk, hipStream_t st);
// out[e] = sum_s in[s * stride + e] over nslice slices, e < n (complex T; out may
// be slice 0 of in)
template <typename T>
hipError_t launch_sum_slices(const void* in, void* out, long n, int nslice, long stride,
                             hipStream_t st);

// Blocked Cholesky with pivot drop (A: S^m in, L in the lower triangle out;
// tol: [N_k] scratch) and blocked inverse W = L^{-1} (T: [N_k][32][N_I] scratch)
// status/strict: a non-finite pivot sets ST_NONFINITE (site SITE_METRIC); with
// strict, a dropped pivot sets ST_NOT_PD and status[1] = min(status[1], lab.q[m])
// (status may be nullptr: no reporting). lab == nullptr labels slot m as m.
hipError_t launch_chol_blocked(const Geom& g, double2* A, int32_t* keep, int32_t* rank,
                               double* tol, double rel_tol, hipStream_t st,
                               int32_t* status = nullptr, bool strict = false,
                               const QLabel* lab = nullptr);
// real-path forms of launch_chol_blocked and launch_tri_inv_blocked (S~ real,
// complex storage): same results, with the GEMMs on the real parts (strided FP64
// matrix-core product)
hipError_t launch_chol_blocked_real(const Geom& g, double2* A, int32_t* keep, int32_t* rank,
                                   double* tol, double rel_tol, hipStream_t st,
                                   int32_t* status = nullptr, bool strict = false);
hipError_t launch_tri_inv_real(const Geom& g, const double2* Lf, const int32_t* keep, double2* W,
                               double2* T, hipStream_t st);
hipError_t launch_tri_inv_blocked(const Geom& g, const double2* Lf, const int32_t* keep,
                                  double2* W, double2* T, hipStream_t st);

// 3-D FFT of nfun functions (forward); pass 1 reads `in`, writes `out`; pass 2 in place.
// fft_prepare sets kernel attributes once and returns the CU count.
hipError_t fft_prepare(int* ncu);
template <typename T>
hipError_t launch_fft3d(const Geom& g, const Tables& tb, const void* in, void* out, long nfun,
                        int ncu, hipStream_t st);
bool fft_supported(const Geom& g, bool fp64);
// real path: twisted FFT of the real fit eta (storage TI), keeping the z
// frequencies below fft_half_z(g) = n3/2 + 1: out [nfun][n1][n2][hz] complex T;
// function f belongs to transfer m0 + f / N_ISDF
template <typename TI, typename T>
hipError_t launch_fft3d_half(const Geom& g, const Tables& tb, const void* in, void* out, long nfun,
                             int m0, int ncu, hipStream_t st);
int fft_half_z(const Geom& g);

// shared_f: every slice contracts the same transforms F (one fit shared by all
// transfers; the transfer enters only through the kernel table v^m).
// Coulomb contraction: V^m (Bloch gauge) from F^m (storage T) on the FP64 matrix cores,
// or with FP32 storage on the BF16 matrix cores (form COUL_BF16: operands rounded to
// bfloat16; COUL_BF16X3: split hi + lo operands, three products), FP32 accumulation
// over at most 256 points added into FP64;
// half: F is the real path's half-grid transform (launch_fft3d_half)
// rep/bar/nslice (host arrays): F holds nslice transfers, slice s being transfer
// rep[s]; V[rep[s]] is written and, where bar[s] >= 0, V[bar[s]] = conj V[rep[s]]
// (bar[s] = -rep[s] on the mesh). rep == nullptr: slice m is transfer m.
// raw: V[s] = the scaled sum of slice s, unphased (lower triangle mirrored), and
// nothing else is written (the factor-split build applies W^H (.) W and then
// launch_coulomb_phase).
template <typename T>
hipError_t launch_coulomb(const Geom& g, const Tables& tb, const void* F, const int32_t* pts,
                          void* partial, int nsplit, double2* V, bool half, hipStream_t st,
                          const int* rep = nullptr, const int* bar = nullptr, int nslice = 0,
                          bool raw = false, int form = 0, bool shared_f = false);
enum { COUL_F64 = 0, COUL_BF16 = 1, COUL_BF16X3 = 2 };
// v^m(g) = 4 pi/|K|^2 (K-box rule, K = 0 dropped) of every transfer: vt [N_k][N_g]
// (rep: the transfers rep[s] of ns slices instead of all)
hipError_t launch_kernel_table(const Geom& g, double* vt, hipStream_t st,
                               const int* rep = nullptr, int ns = 0);

// density derivative of the fitted exchange energy (grad.hip), FP64:
// F <- conj(v^m F) over [N_k][N_ISDF][N_g]; f32: F stored as c64
hipError_t launch_kernel_scale_conj(const Geom& g, void* F, const double* vt, hipStream_t st,
                                    bool f32 = false);
// X[m][P][r] <- scale e^{i q_m.(r_P - r)} X[m][P][r]; f32: X stored as c64; rep: slice s
// holds transfer rep[s] (ns slices) instead of slice m transfer m
hipError_t launch_potential_phase(const Geom& g, const Tables& tb, void* X, const int32_t* pts,
                                  double scale, hipStream_t st, bool f32 = false,
                                  const int* rep = nullptr, int ns = 0);
// out[n] = sum_m [p^m conj Q^{n+m} + conj(p^m) conj Q^{n-m}] over `elems` elements per
// k, p^m = P^m (or conj P^m); up_only: the first term alone; P stored as c64 with p_f32
// (Q and out c128, FP64 arithmetic). src/cj (N_k entries): P^m is slice src[m] of P,
// conjugated where cj[m] (one transfer of each conjugate pair stored); default src[m] = m
hipError_t launch_grad_xcorr(const Geom& g, const void* P, bool conj_p, const void* Q, void* out,
                             long elems, hipStream_t st, bool up_only = false, bool p_f32 = false,
                             const int* src = nullptr, const int* cj = nullptr);
// K[n][mu][nu] <- conj(Ac[n][mu][nu]) + Ac[n][nu][mu] - K[n][mu][nu]
hipError_t launch_robust_assemble(const Geom& g, const void* Ac, void* K, hipStream_t st);
// Kg[n][mu][nu] = -(N_k/4) (Ac[n][mu][nu] + conj Ac[n][nu][mu])
hipError_t launch_grad_assemble(const Geom& g, const void* Ac, void* Kg, hipStream_t st);
// V[rep[s]] = e^{-i q_m.(r_P - r_Q)} U[s] (lower triangle of U mirrored) and, where
// bar[s] >= 0, V[bar[s]] = conj of that; U holds nslice (<= 64) matrices
hipError_t launch_coulomb_phase(const Geom& g, const Tables& tb, const int32_t* pts,
                                const double2* U, double2* V, const int* rep, const int* bar,
                                int nslice, hipStream_t st);
size_t coulomb_partial_bytes(const Geom& g, int nsplit);
int coulomb_nsplit(const Geom& g);

// k-convolution Y^n = sum_m Vb^m o G^{n+m}
hipError_t launch_kconv(const Geom& g, const double2* Vb, const double2* G, double2* Y,
                        hipStream_t st);
// E_x = -(1/N_k^2) sum Re(Y conj G)
hipError_t launch_energy(const Geom& g, const double2* Y, const double2* G, double* partial,
                         double* Ex, hipStream_t st);

// point selection kernels
hipError_t launch_select(const Geom& g, const double2* psi, int32_t* pts, int32_t* n_pivot,
                         void* scratch, hipStream_t st);
size_t select_scratch_bytes(const Geom& g);

// learned selector: descriptors, network, training step, targets, NMS, probe
hipError_t launch_mlp_features(const Geom& g, const double2* psi, const double* norm, float* feat,
                               void* scratch, hipStream_t st);
size_t mlp_feature_scratch_bytes(const Geom& g);
hipError_t launch_mlp_forward(long n, const float* feat, const float* theta, float* score,
                              hipStream_t st);
hipError_t launch_mlp_grad(long n, const int32_t* idx, long rows, const float* feat,
                           const float* tgt, float wpos, const float* theta, float* grad,
                           double* loss, void* scratch, hipStream_t st);
size_t mlp_grad_scratch_bytes(long n);
// sums[0..2] += column sums, sums[3..5] += column sums of squares of feat [n][3]
hipError_t launch_mlp_moments(long n, const float* feat, double* sums, void* scratch,
                              hipStream_t st);
size_t mlp_moments_scratch_bytes(long n);
hipError_t launch_adam(int np, float* theta, const float* g, float* m, float* v, int step, float lr,
                       float b1, float b2, float eps, hipStream_t st);
hipError_t launch_targets(const Geom& g, const int32_t* pts, int npts, double sigma, float* t,
                          hipStream_t st);
hipError_t launch_nms(const Geom& g, const float* score, int k, int32_t* pts, void* scratch,
                      hipStream_t st);
size_t mlp_nms_scratch_bytes(const Geom& g);
hipError_t launch_mlp_probe(const Geom& g, const double2* psi, const int32_t* pts, int nr,
                            unsigned long long seed, double* resid, void* scratch, hipStream_t st);
size_t mlp_probe_scratch_bytes(const Geom& g, int nr);

}  // namespace exx

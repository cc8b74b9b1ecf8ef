/*
 * exx.h -- C ABI of the THC-oo-K k-point exact-exchange build for gfx950.
 *
 * Method: Rettig, Lee, Head-Gordon, "Even Faster Exact Exchange for Solids via
 * Tensor Hypercontraction" (THC-oo-K, Sec. 2.3, Algorithm 2). Given occupied
 * orbitals on the real-space grid of every k-point and a fixed set of N_ISDF
 * interpolation points, one "K-build" returns the exchange matrix K^k for every
 * k and the exchange energy E_x. It runs in three calls:
 *
 *   exx_isdf_fit   occupied-pair ISDF fit, one per momentum transfer q
 *                  (Eqs. 7-8 and 13 restricted to occupied pairs, Eq. 16);
 *   exx_coulomb_V  FFT-Poisson Coulomb matrices of the interpolating vectors
 *                  (Eq. 9 / Eq. 15 by GPW, Algorithm 2 "FFT" and "M^q" lines);
 *   exx_build_K    k-convolution and exchange contraction (Eq. 14, the X^k and
 *                  K_ij lines of Algorithm 2) and E_x (Eq. 18).
 *
 * Conventions
 * -----------
 * Cell: orthorhombic, edges L[3] (bohr). Grid point g = (g1,g2,g3) sits at
 *   r_g = sum_i (g_i/n_i) L_i e_i; flat grid index r = (g1*n2 + g2)*n3 + g3.
 * k-mesh: Gamma-centred, k_n = sum_i (n_i/N_i) b_i, b_i = 2 pi/L_i e_i, flat
 *   index n in C order. Momentum transfer m(n, n') = (n' - n) mod N per axis,
 *   q_m = sum_i (m_i/N_i) b_i.
 * Orbitals: psi_in(r) is the full Bloch orbital (no e^{-ik.r} removed), one
 *   row of N_g values per (n, i).
 * Coulomb kernel for transfer m at FFT index g: v^m(g) = 4 pi/|K|^2 with
 *   K = sum_i kappa_i b_i/N_i, kappa_i = wrap_{N_i n_i}(N_i g_i + m_i),
 *   wrap_L(x) = ((x + floor(L/2)) mod L) - floor(L/2); the K = 0 term is
 *   dropped (no Madelung correction).
 * Forward FFT sign: F(g) = sum_r f(r) exp(-2 pi i g.r/n).
 * Complex numbers are interleaved (re, im) pairs: "c128" = 2 x double,
 *   "c64" = 2 x float. Arrays are C order (last index fastest).
 * Fit gauge: xi^m_P(r) interpolates e^{-i q_m.r} conj psi_in(r) psi_{j,n+m}(r).
 *   Bloch gauge: Vb^m_PQ = e^{-i q_m.(r_P - r_Q)} V^m_PQ, with
 *   V^m_PQ = (Omega/N_g^2) sum_g v^m(g) F_P(g) conj F_Q(g), F_P = FFT(xi^m_P).
 *
 * Ownership and errors
 * --------------------
 * Every array argument is caller-owned DEVICE memory unless marked "host";
 * the library never frees caller memory. Scratch memory belongs to the handle
 * (allocated on first use, grown on demand, released by exx_destroy) unless
 * the caller provides it (exx_set_workspace). Calls
 * are asynchronous on the given stream (0 = default stream) and return a
 * status; no C++ exception crosses the ABI. Shape and argument checks happen
 * before any launch; on error nothing is launched and exx_last_error(h)
 * returns a message. A handle must not be used by two host threads at once.
 * Calls that share a handle must be ordered (same stream or synchronised),
 * because they share the handle's scratch memory.
 */
#ifndef EXX_H
#define EXX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EXX_OK = 0,
  EXX_ERR_ARG = -1,         /* null pointer, bad enum, bad handle */
  EXX_ERR_SHAPE = -2,       /* sizes out of the supported range */
  EXX_ERR_NOMEM = -3,       /* scratch allocation failed */
  EXX_ERR_NOT_PD = -4,      /* a fit metric lost a pivot (EXX_STRICT_PD only) */
  EXX_ERR_NONFINITE = -5,   /* a non-finite value reached a checked array */
  EXX_ERR_DEVICE = -6,      /* a HIP runtime call failed */
  EXX_ERR_UNSUPPORTED = -7  /* precision or size not built in */
} exx_status;

/* Arithmetic precision of the build. G^n, S^m, the Cholesky factorisation,
 * the pseudo-inverse, the k-convolution, K^n and E_x are FP64 in every mode.
 *   EXX_F64    everything FP64; psi_grid and xi are c128.
 *   EXX_MIXED  the whole fit in FP64 (psi_grid c128); xi stored c64; FFT in
 *              FP32; the Coulomb contraction multiplies the FP32-stored
 *              transforms on the FP64 matrix cores (exact products, FP64
 *              accumulation).
 *   EXX_F32    the grid-sized fit GEMM (Gamma^n, FP32 matrix cores) and the
 *              k-correlation Z^m in FP32 (psi_grid and xi c64); the fit solve
 *              applies the FP64 pseudo-inverse in FP64 arithmetic; FFT in
 *              FP32; the Coulomb contraction as in EXX_MIXED (FP64 matrix
 *              cores on the FP32-stored transforms).
 *   EXX_BF16   as EXX_F32, but the grid-sized fit GEMM Gamma^n runs on the
 *              BF16 matrix cores: occ_pts and psi_grid (c64) are rounded to
 *              bfloat16 (nearest even) as they are loaded, FP32 accumulation,
 *              Gamma kept in FP32; and the Coulomb contraction runs on the
 *              BF16 matrix cores (EXX_CONTRACT_BF16, exx_set_contraction).
 *              psi_grid and xi are c64. Its error is that of 8-bit
 *              significands amplified by the metric's conditioning (reported,
 *              not within the 1e-5 / 1e-6 accuracy target). */
/* The precision is a plain 32-bit integer holding one of these constants, so
 * that any value a caller passes can be checked (an enum type would make an
 * out-of-range value undefined in the C++ implementation); anything else is
 * rejected with EXX_ERR_ARG. */
typedef int32_t exx_prec;
enum { EXX_F64 = 0, EXX_F32 = 1, EXX_BF16 = 2, EXX_MIXED = 3 };

typedef struct {
  double L[3];       /* orthorhombic cell edges, bohr */
  int32_t grid[3];   /* n1, n2, n3: each 2..128, 2*3*5-smooth, n2*n3 <= 6144 */
  int32_t kmesh[3];  /* N1, N2, N3: each 1..8, N1 N2 N3 <= 64. The k-correlation
                        of 1x1x1, 2x2x2, 3x3x3, 4x4x4, 2x1x1, 1x2x1, 1x1x2,
                        2x2x1, 2x1x2, 1x2x2, 3x1x1, 3x2x1 and 1x2x3 runs on
                        register-resident k-mesh DFTs; other meshes take a
                        direct-sum kernel (same results, slower) */
  int32_t n_occ;     /* occupied orbitals per k, 1..512 */
  int32_t n_ao;      /* basis functions per k, 1..4096 */
  int32_t n_isdf;    /* interpolation points, 1..2048 */
} exx_cell;
/* Besides the ranges above: n_isdf N_g < 2^28 and n_occ N_g < 2^28 (N_g =
 * n1 n2 n3), because one transfer's grid-sized arrays are addressed with 32-bit
 * byte offsets; larger cells are rejected with EXX_ERR_UNSUPPORTED before any
 * work is queued. */

typedef struct exx_context* exx_handle_t;

/* Create a handle bound to HIP device `device`. */
exx_status exx_create(exx_handle_t* h, int device);
/* Release the handle and its scratch memory (synchronises the device). */
exx_status exx_destroy(exx_handle_t h);
/* Message of the last failing call on this handle ("" if none). Never NULL. */
const char* exx_last_error(exx_handle_t h);
/* Bytes of scratch the handle currently holds. */
exx_status exx_scratch_bytes(exx_handle_t h, size_t* bytes);

/*
 * Caller-owned scratch. exx_workspace_size returns the scratch bytes that one
 * kind of call needs for this cell (and precision, for the K-build calls):
 *   EXX_CALL_BUILD       exx_isdf_fit, exx_coulomb_V, exx_build_K, exx_build and
 *                        an exx_build_batched item (the largest of them)
 *   EXX_CALL_SELECT      exx_select_points
 *   EXX_CALL_SELECT_MLP  exx_select_points_mlp (n_probe up to 8192)
 *   EXX_CALL_GRADIENT    exx_exchange_gradient, exx_build_robust (EXX_F64 or EXX_MIXED)
 * exx_set_workspace hands the handle a device buffer (256-byte aligned, caller
 * owned, e.g. a torch tensor) that every later call uses as its scratch; the
 * library then allocates no scratch of its own and releases what it held. A
 * call needing more than `bytes` fails with EXX_ERR_NOMEM before any launch.
 * dev = NULL returns to library-owned scratch. The call synchronises the device
 * first. The buffer must stay valid until it is replaced or the handle is
 * destroyed, and calls sharing it must be ordered. The handle still keeps a
 * few small tables of its own (FFT twiddles and Bloch phases per grid shape,
 * the status word).
 */
#define EXX_CALL_BUILD 0
#define EXX_CALL_SELECT 1
#define EXX_CALL_SELECT_MLP 2
#define EXX_CALL_GRADIENT 3
exx_status exx_workspace_size(exx_handle_t h, const exx_cell* cell, exx_prec prec, int32_t call,
                              size_t* bytes);
exx_status exx_set_workspace(exx_handle_t h, void* dev, size_t bytes);

/*
 * Run-time checks (failure detection). The K-build calls report into a device
 * status word of the handle; kernels set its bits and the host reads them with
 * exx_get_status, so the checks never stall the stream.
 *   EXX_CHECK_FINITE  (default on) scan the small inputs occ_pts and ao_pts, the
 *                     Coulomb matrices given to or returned by the stage-wise
 *                     calls, and the outputs K and E_x for NaN or Inf; the
 *                     Cholesky factorisation reports a non-finite pivot. A
 *                     non-finite psi_grid reaches V, K and E_x and is reported
 *                     there (exx_isdf_fit alone does not scan xi).
 *   EXX_STRICT_PD     the drop rule (a Schur pivot below 1e-12 max_P S_PP) still
 *                     applies, but a dropped pivot is reported as EXX_ERR_NOT_PD
 *                     with the lowest transfer index m whose metric lost one.
 *   EXX_CHECK_SYNC    every K-build call synchronises its stream at the end and
 *                     returns the status (EXX_ERR_NONFINITE before
 *                     EXX_ERR_NOT_PD) instead of EXX_OK.
 * exx_get_status synchronises `stream`, reads and clears the status word and
 * returns EXX_OK, EXX_ERR_NONFINITE or EXX_ERR_NOT_PD. info (host, may be NULL):
 * info[0] = the first transfer that lost a pivot under EXX_STRICT_PD (-1 if
 * none), info[1] = where the first non-finite value was seen (0 none, 1 occ_pts,
 * 2 ao_pts, 3 fit metric, 4 Coulomb matrices, 5 K or E_x). The status word
 * accumulates over calls until it is read.
 */
#define EXX_CHECK_FINITE 1
#define EXX_STRICT_PD 2
#define EXX_CHECK_SYNC 4
exx_status exx_set_checks(exx_handle_t h, int32_t flags);
exx_status exx_get_status(exx_handle_t h, hipStream_t stream, int32_t* info);

/*
 * exx_isdf_fit -- occupied-pair ISDF fit per transfer q (Sec. 2.2-2.3,
 * Eqs. 7-8 and 13 restricted to occupied pairs as in Eq. 16; Algorithm 2
 * "Compute xi"). For every transfer m it forms the fit metric
 *   S^m_PQ = e^{i q_m.(r_P - r_Q)} sum_n G^n_PQ conj G^{n+m}_PQ,
 *   G^n_PQ = sum_i psi_in(r_P) conj psi_in(r_Q),
 * the right-hand side
 *   Z^m_P(r) = e^{i q_m.(r_P - r)} sum_n Gamma^n(P,r) conj Gamma^{n+m}(P,r),
 *   Gamma^n(P,r) = sum_i psi_in(r_P) conj psi_in(r)
 * (the k-sum evaluated as a circular correlation by DFTs over the k-mesh),
 * factorises S^m by FP64 Cholesky in point order -- a point whose Schur
 * pivot is below 1e-12 * max_P S^m_PP is dropped and gets xi_P = 0 -- and
 * solves S^m xi^m(r) = Z^m(r) on every grid point.
 *
 *   psi_grid [N_k][n_occ][N_g]    c128 (EXX_F64, EXX_MIXED) or c64 (EXX_F32)
 *   occ_pts  [N_k][n_isdf][n_occ] c128: psi_in(r_P), used for G^n and S^m
 *   pts      [n_isdf] int32 flat grid indices of the points, distinct
 *   xi       out [N_k][n_isdf][N_g], c128 (EXX_F64) or c64 (other modes)
 *   S        out [N_k][n_isdf][n_isdf] c128, full Hermitian S^m
 *   rank     out [N_k] int32: retained points per q
 */
exx_status exx_isdf_fit(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                        const void* psi_grid, const void* occ_pts, const int32_t* pts,
                        void* xi, void* S, int32_t* rank, hipStream_t stream);

/*
 * exx_coulomb_V -- Coulomb matrices of the interpolating vectors by
 * FFT-Poisson (Eq. 9 and Eq. 15 evaluated by GPW; Algorithm 2 "FFT" and
 * "M^q" lines): F^m_P = FFT(xi^m_P), V^m = (Omega/N_g^2) F diag(v^m) F^H,
 * returned in the Bloch gauge Vb^m_PQ = e^{-i q_m.(r_P - r_Q)} V^m_PQ.
 *
 *   xi  [N_k][n_isdf][N_g] as written by exx_isdf_fit (not modified)
 *   pts [n_isdf] int32
 *   V   out [N_k][n_isdf][n_isdf] c128, Vb^m (Hermitian)
 */
exx_status exx_coulomb_V(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                         const void* xi, const int32_t* pts, void* V, hipStream_t stream);

/*
 * exx_build_K -- exchange matrices and energy (Eq. 14 with the oo fit,
 * Algorithm 2 X^k and K lines, Eq. 18):
 *   Y^n = sum_m Vb^m o G^{n+m}   (k-convolution, by DFTs over the k-mesh)
 *   K^n = (1/N_k) A^n^H Y^n A^n,  A^n_{P mu} = phi_mu^n(r_P)
 *   E_x = -(1/N_k^2) sum_n sum_PQ Y^n_PQ conj G^n_PQ   (Ha per cell, FP64)
 *
 *   ao_pts  [N_k][n_isdf][n_ao] c128: phi_mu^n(r_P)
 *   occ_pts [N_k][n_isdf][n_occ] c128
 *   V       [N_k][n_isdf][n_isdf] c128 from exx_coulomb_V
 *   K       out [N_k][n_ao][n_ao] c128
 *   Ex      out [1] double (device)
 */
exx_status exx_build_K(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                       const void* ao_pts, const void* occ_pts, const void* V,
                       void* K, double* Ex, hipStream_t stream);

/*
 * exx_build_K_noalloc -- exx_build_K for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, results and checks as exx_build_K; it
 * calls no hipMalloc, hipFree or allocating library routine. Its scratch
 * (G^n, Y^n, the contraction intermediates) lives in a fixed device array of
 * EXX_NOALLOC_MAX_BYTES per GPU, reserved when the library's code is loaded on
 * that GPU and held until the process ends; its address is looked up in
 * exx_create. A cell needing more, 2 N_k N_ISDF^2 + 2 N_k N_ISDF n_ao complex128
 * values plus 8 KiB (the second N_k N_ISDF n_ao term only when n_ao <= N_ISDF),
 * returns EXX_ERR_SHAPE before any launch. Every call on a GPU shares that GPU's
 * array, whatever its handle: calls that overlap in time on one GPU (two
 * streams, two host threads) race and must be ordered by the caller.
 */
#define EXX_NOALLOC_MAX_BYTES (256u << 20)
exx_status exx_build_K_noalloc(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                               const void* ao_pts, const void* occ_pts, const void* V, void* K,
                               double* Ex, hipStream_t stream);

/*
 * exx_build -- one whole K-build (Algorithm 2: fit, Coulomb matrices, K and
 * E_x) with the results of exx_isdf_fit, exx_coulomb_V and exx_build_K called
 * in turn, to rounding; xi, S and V stay in the handle's scratch. It reaches
 * them by identities of the method instead of forming xi: on meshes whose
 * every axis has N_i <= 2 it works in the unphased gauge in real arithmetic,
 * elsewhere it fits and contracts one transfer of each pair (m, -m); both
 * apply the triangular inverse Cholesky factor W (S^+ = W^H W) to the grid
 * and form Vb = W^H Vy W from the contraction of its transform (with
 * refinement on, exx_set_refinement, Y is refined in the factor form:
 * R = Z - L Y, Y += W R). It forks a
 * second stream of the handle (the Gamma fit beside the factorisation; on the
 * paired path, and in EXX_F64 on the real path, also the contraction of each
 * chunk of transfers beside the transform of the next) and joins it back into
 * `stream` before returning, so work
 * ordered on `stream` before and after the call stays ordered. Arguments as
 * above; error behaviour as above.
 */
exx_status exx_build(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                     const void* psi_grid, const void* occ_pts, const void* ao_pts,
                     const int32_t* pts, void* K, double* Ex, int32_t* rank,
                     hipStream_t stream);

/*
 * exx_exchange_gradient -- the derivative of the fitted exchange energy in the
 * AO density matrices (Sec. 2.3, Eq. 19: its occupied-virtual block C_v^H Kgrad
 * C_o is the orbital gradient of the exchange energy), together with the
 * K-build of exx_build. The fit xi^m and the Coulomb matrices depend on the
 * density through G^n and Gamma^n, so the derivative of
 * E_x = -(1/N_k^2) sum_m Tr((S^m)^+ Z^m Vop Z^m^H) has, besides the fixed-fit
 * term that gives K, the terms of dS^m and dZ^m:
 *   dE_x = (1/N_k^2) sum_m [Tr(V^m dS^m) - 2 Re sum_{P,r} dZ^m(P,r) conj Phi^m_P(r)],
 *   Phi^m_P(r) = (Omega/N_g^2) sum_g e^{i g.r} v^m(g) F^m_P(g)
 * (the potential of xi^m_P, F^m_P its transform). With A^n the coefficient of
 * dD^n in dE_x = Re sum_n sum_{mu nu} dD^n_{mu nu} A^n_{mu nu}, the output is
 *   Kgrad^n = -(N_k/4) (A^n + A^n^H)^T,
 * normalised like K (dE_x = -(2/N_k) sum_n Tr(Kgrad^n dD^n) for Hermitian dD^n,
 * E_x = -(1/N_k) sum_n Tr(Kgrad^n D^n)); holding V^m fixed instead gives K.
 * The per-transfer fit is formed for every transfer (its xi^m are needed), the
 * potentials by one more forward transform of conj(v^m F^m), the k-mesh sums
 * in registers and the AO contractions on the FP64 matrix cores.
 *
 *   psi_grid, occ_pts, ao_pts, pts, K, Ex, rank as in exx_build
 *   ao_grid  [N_k][n_ao][N_g] c128: the AO functions phi^n_mu on the grid
 *   Kgrad    out [N_k][n_ao][n_ao] c128, Hermitian
 * prec: EXX_F64, or EXX_MIXED (the fit as in the MIXED builds, xi, the
 * transforms and the potentials stored as c64, everything after them in FP64);
 * anything else returns EXX_ERR_UNSUPPORTED. Scratch: three grid-sized arrays
 * [N_k][N_ISDF][N_g] (c128; in MIXED one of them c64) plus the build's
 * point-sized ones (exx_workspace_size with EXX_CALL_GRADIENT). Ordered on
 * `stream` like exx_build; error behaviour as above.
 */
exx_status exx_exchange_gradient(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                                 const void* psi_grid, const void* occ_pts, const void* ao_pts,
                                 const void* ao_grid, const int32_t* pts, void* K, void* Kgrad,
                                 double* Ex, int32_t* rank, hipStream_t stream);

/*
 * exx_build_robust -- the robust-fit exchange matrix (the one-sided fit that
 * the discussion of Sec. 5 proposes for THC-oo-K): every exchange integral
 * takes one exact and one fitted pair density,
 *   K_rob = K[rho, rho~] + K[rho~, rho] - K[rho~, rho~],
 * with K[a, b]^n_{mu nu} = (1/N_k) sum_{n' j} J^m[a_{mu j}, b_{nu j}] over the
 * pairs rho_{mu j} = e^{-i q.r} conj phi_mu^n psi_jn' of direct exchange and
 * rho~ their interpolation by the per-transfer occupied-pair fit; K[rho~, rho~]
 * is exx_build's K. The error K_direct - K_rob = K[delta, delta] is second order
 * in the fit's residual delta = rho - rho~ (first order for the plain fit), and
 * at full occupied-pair rank the occupied rows C^H K_rob are exact. The
 * one-sided term uses the potentials Phi^m of the fitted functions on the grid
 * (one more transform of every F^m) and Gamma^n:
 *   K[rho, rho~]^n = (1/N_k) conj(phi^n) R^n^T A^n,
 *   R^n(Q, r) = sum_m e^{i q_m.(r_Q - r)} conj Phi^m_Q(r) conj Gamma^{n+m}(Q, r).
 * E_x is the fitted one, which is also the robust energy (the least-squares
 * fit projects the occupied pairs, so the two one-sided terms add up to the
 * fitted energy).
 *
 *   psi_grid, occ_pts, ao_pts, pts, Ex, rank as in exx_build
 *   ao_grid  [N_k][n_ao][N_g] c128: the AO functions phi^n_mu on the grid
 *   K        out [N_k][n_ao][n_ao] c128: K_rob, Hermitian
 * prec: EXX_F64 or EXX_MIXED, as for exx_exchange_gradient (else
 * EXX_ERR_UNSUPPORTED); scratch as for exx_exchange_gradient
 * (EXX_CALL_GRADIENT). Ordered on `stream` like exx_build; error behaviour as
 * above.
 */
exx_status exx_build_robust(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                            const void* psi_grid, const void* occ_pts, const void* ao_pts,
                            const void* ao_grid, const int32_t* pts, void* K, double* Ex,
                            int32_t* rank, hipStream_t stream);

/*
 * exx_select_points -- interpolation points by QR with column pivoting
 * (Sec. 2.1 after Eq. 5), computed as greedy pivoted Cholesky of the pair
 * Gram matrix |Gamma(r, r')|^2, Gamma(r, r') = sum_{n,i} psi_in(r) conj
 * psi_in(r'), in FP64: pivot = argmax of the Schur diagonal (ties to the
 * smallest index); pivoting stops when the pivot drops below 1e-12 times the
 * first one, and the remaining slots take the unselected points of highest
 * density sum_{n,i} |psi_in(r)|^2 (ties to the smallest index).
 *
 *   psi_grid [N_k][n_occ][N_g] c128
 *   pts      out [n_isdf] int32
 *   n_pivot  out [1] int32: number of points chosen by pivoting
 */
exx_status exx_select_points(exx_handle_t h, const exx_cell* cell, const void* psi_grid,
                             int32_t* pts, int32_t* n_pivot, hipStream_t stream);

/*
 * Learned point selection. The paper picks the interpolation points by QRCP
 * or k-means (Sec. 2.1 after Eq. 5); here a small network scores every grid
 * point from three descriptors of the occupied density and a greedy
 * non-maximum suppression turns the scores into N_ISDF points. It is trained
 * to reproduce QRCP selections, and a fit-residual probe sends a cell back to
 * QRCP (exx_select_points) when the proposal is poor.
 *
 * Network: 3 -> 64 -> 64 -> 1, SiLU after both hidden layers, output = logit.
 * Parameters theta: EXX_MLP_NPARAM float32 values, in order W1 (64 x 3, row
 * major), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1). Evaluation rounds
 * the weights W1, W2, w3 to bfloat16 (nearest even) and keeps the biases and
 * all arithmetic in FP32. Features are float32 [N_g][3].
 */
#define EXX_MLP_NPARAM 4481

/*
 * exx_mlp_features -- descriptors of every grid point, from
 *   rho(r) = (1/N_k) sum_{n,i} |psi_in(r)|^2:
 *   f0 = ln(rho / mean_r rho)
 *   f1 = ln|grad rho| - (4/3) ln rho (fourth-order periodic central differences)
 *   f2 = sum |psi_in(r)|^4 / (sum |psi_in(r)|^2)^2 (local orbital weight)
 * each standardised as (f_j - norm[2j]) / norm[2j+1].
 *
 *   psi_grid [N_k][n_occ][N_g] c128
 *   norm     host [6] double: mean and scale of f0, f1, f2 (scales > 0)
 *   feat     out [N_g][3] float32
 */
exx_status exx_mlp_features(exx_handle_t h, const exx_cell* cell, const void* psi_grid,
                            const double* norm, float* feat, hipStream_t stream);

/*
 * exx_mlp_moments -- the standardisation constants' raw moments (the training
 * driver accumulates them over cells before exx_mlp_features is called with
 * the resulting means and scales): sums[j] += sum_i feat[i][j] and
 * sums[3 + j] += sum_i feat[i][j]^2, j < 3, in FP64 with a fixed summation
 * order (deterministic); what sums holds is added to.
 *   feat [n][3] float32 (n >= 0);  sums in/out [6] double (device)
 */
exx_status exx_mlp_moments(exx_handle_t h, int64_t n, const float* feat, double* sums,
                           hipStream_t stream);

/*
 * exx_mlp_forward -- score[i] = network logit of feat[i], i < n (n >= 0).
 *   feat [n][3] float32, theta [EXX_MLP_NPARAM] float32, score out [n] float32
 */
exx_status exx_mlp_forward(exx_handle_t h, int64_t n, const float* feat, const float* theta,
                           float* score, hipStream_t stream);

/*
 * exx_mlp_backward -- gradient of the weighted binary cross-entropy
 *   L = sum_q w_q (softplus(s_q) - t_q s_q) / sum_q w_q,  w_q = 1 + wpos t_q,
 * over the batch q < n of rows idx[q] of feat and target (rows 0..n-1 when
 * idx is NULL), with respect to theta (through the bfloat16-rounded weights:
 * the gradient of the rounded network is returned for the FP32 parameters).
 * Per-block partial sums are reduced in a fixed order, so the result is
 * deterministic. An idx entry outside [0, rows) contributes nothing.
 *
 *   idx    [n] int32 or NULL (then rows == n)
 *   feat   [rows][3], target [rows] float32 (targets in [0, 1]); wpos >= 0
 *   grad   out [EXX_MLP_NPARAM] float32;  loss out [1] double
 */
exx_status exx_mlp_backward(exx_handle_t h, int64_t n, const int32_t* idx, int64_t rows,
                            const float* feat, const float* target, float wpos, const float* theta,
                            float* grad, double* loss, hipStream_t stream);

/*
 * exx_mlp_adam -- one Adam step (Kingma and Ba) in place, all float32 [np]:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   theta -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps);  step >= 1.
 */
exx_status exx_mlp_adam(exx_handle_t h, int32_t np, float* theta, const float* grad, float* m,
                        float* v, int32_t step, float lr, float beta1, float beta2, float eps,
                        hipStream_t stream);

/*
 * exx_mlp_targets -- soft training targets t(r) = exp(-d(r)^2 / (2 sigma^2)), d
 * the periodic minimum-image distance from grid point r to the nearest of the
 * npts points pts (flat grid indices, 1 <= npts <= 2048); sigma > 0 in bohr.
 *   target out [N_g] float32
 */
exx_status exx_mlp_targets(exx_handle_t h, const exx_cell* cell, const int32_t* pts, int32_t npts,
                           double sigma, float* target, hipStream_t stream);

/*
 * exx_mlp_nms -- greedy selection of k points (1 <= k <= N_g): the highest
 * score first (NaN below every number, ties to the smaller index), each pick
 * removing the unpicked points closer than h = (Omega/k)^{1/3}/2 (periodic
 * minimum image); if fewer than k survive, the rest of the slots take the
 * unpicked points in score order.
 *   score [N_g] float32;  pts out [k] int32 in pick order
 */
exx_status exx_mlp_nms(exx_handle_t h, const exx_cell* cell, const float* score, int32_t k,
                       int32_t* pts, hipStream_t stream);

/*
 * exx_mlp_probe -- relative fit residual of the point set pts (n_isdf points)
 * on n_probe grid points r_j drawn by SplitMix64 from seed (j-th draw mod N_g):
 *   resid = sum_j max(C(r_j,r_j) - C(r_j,P) C(P,P)^+ C(P,r_j), 0) / sum_j C(r_j,r_j)
 * with C(r,r') = |Gamma(r,r')|^2, Gamma(r,r') = sum_{n,i} psi_in(r) conj psi_in(r'),
 * the Gram matrix that QRCP pivots on (the Schur complement is the squared
 * distance of the pair row at r_j from the span of the rows at the points);
 * C(P,P)^+ uses the fit's Cholesky with pivot drop. 1 <= n_probe <= 8192,
 * N_k n_occ <= 65536. Point indices outside [0, N_g) are clamped into it.
 *   psi_grid [N_k][n_occ][N_g] c128;  pts [n_isdf] int32;  resid out [1] double
 */
exx_status exx_mlp_probe(exx_handle_t h, const exx_cell* cell, const void* psi_grid,
                         const int32_t* pts, int32_t n_probe, uint64_t seed, double* resid,
                         hipStream_t stream);

/*
 * exx_select_points_mlp -- features, network, NMS for n_isdf points, then the
 * probe (n_probe points, a fixed seed). If the residual exceeds tau (or is not
 * a number) the points are recomputed by exx_select_points and
 * *used_fallback = 1, else 0. Synchronises the stream to read the residual.
 *   psi_grid, norm, theta as above;  pts out [n_isdf] int32
 *   used_fallback  out, host int32;  resid_out  out, host double (may be NULL)
 */
exx_status exx_select_points_mlp(exx_handle_t h, const exx_cell* cell, const void* psi_grid,
                                 const double* norm, const float* theta, double tau,
                                 int32_t n_probe, int32_t* pts, int32_t* used_fallback,
                                 double* resid_out, hipStream_t stream);

/*
 * exx_build_batched -- many independent K-builds (cells of different shapes,
 * k-meshes and sizes) in one call, each exactly as exx_build. All items use
 * the same precision mode. Without EXX_BATCH_CONCURRENT the handle's scratch
 * is sized once for the largest item and the items run one after another on
 * `stream`.
 *
 * flags:
 *   EXX_BATCH_GRAPH  record the whole batch once into a HIP graph (stream
 *                    capture) and launch it as one graph; a later call with
 *                    the same items (same shapes and pointers) and precision
 *                    replays the cached graph. No allocation or host copy
 *                    happens inside the recorded sequence. Needs a
 *                    non-default stream (EXX_ERR_ARG otherwise).
 *   EXX_BATCH_TUNE   before the first launch, time the candidate wave tiles
 *                    of the two grid-sized GEMMs (Gamma^n and the fit solve)
 *                    once per size class (n_isdf, N_g, n_occ, N_k) and keep
 *                    the fastest in the handle; later builds of the same
 *                    class use it.
 *
 *   EXX_BATCH_CONCURRENT  run the items on up to four concurrent lanes: each
 *                    lane has its own streams and scratch (sized for its
 *                    largest item); items go longest first to the least
 *                    loaded lane; the most lanes whose scratch fits in 85% of
 *                    the device memory free at the call are used (one lane,
 *                    the sequential order, when none fits or when the caller's
 *                    workspace is set). Lanes fork from and join back into
 *                    `stream`, so small cells run beside large ones. Results do
 *                    not depend on the lane plan. Not combinable with
 *                    EXX_BATCH_GRAPH (EXX_ERR_UNSUPPORTED).
 *
 *   items  [n] host array; every pointer in it is device memory as in
 *          exx_build (psi_grid, occ_pts, ao_pts, pts in; K, Ex, rank out)
 */
typedef struct {
  exx_cell cell;
  const void* psi_grid;
  const void* occ_pts;
  const void* ao_pts;
  const int32_t* pts;
  void* K;
  double* Ex;
  int32_t* rank;
} exx_batch_item;

#define EXX_BATCH_GRAPH 1
#define EXX_BATCH_TUNE 2
#define EXX_BATCH_CONCURRENT 4
exx_status exx_build_batched(exx_handle_t h, int32_t n, const exx_batch_item* items,
                             exx_prec prec, int32_t flags, hipStream_t stream);

/*
 * exx_save_tuning / exx_load_tuning -- write the handle's autotuned tile table
 * (EXX_BATCH_TUNE results, one line per size class: n_isdf, N_g, n_occ, N_k,
 * precision, Gamma tile, solve tile) to a text file, and read such a file into
 * the handle (entries replace those of the same class), so that later
 * processes skip the timing runs. A malformed file is rejected (EXX_ERR_ARG)
 * without changing the table.
 */
exx_status exx_save_tuning(exx_handle_t h, const char* path);
exx_status exx_load_tuning(exx_handle_t h, const char* path);

/*
 * exx_set_refinement -- steps (0, the default, or 1) of iterative refinement
 * applied by every later fit of this handle. exx_isdf_fit: after
 * xi^m = S^+ Z^m, the residual R^m = Z^m - S^m xi^m and the correction
 * xi^m += S^+ R^m. exx_build and exx_build_batched (which keep Y = W Z, W the
 * inverse Cholesky factor, S = L L^H on the retained points): R = Z - L Y and
 * Y += W R. Either way two more grid-sized GEMMs per fit, formed with FP64
 * sums on the stored operands; with the pivot-drop rule the correction is
 * confined to the retained points like the solve.
 */
exx_status exx_set_refinement(exx_handle_t h, int32_t steps);

/*
 * exx_set_contraction -- arithmetic of the Coulomb contraction
 *   V^m_PQ = (Omega/N_g^2) sum_g v^m(g) F_P(g) conj F_Q(g)
 * (Sec. 2.2, Eq. 15; the step the paper finds rate-limiting) in every later
 * build and exx_coulomb_V call of this handle whose transforms F are stored in
 * FP32 (EXX_MIXED, EXX_F32, EXX_BF16):
 *   EXX_CONTRACT_AUTO    (default) EXX_CONTRACT_BF16 in EXX_BF16, else
 *                        EXX_CONTRACT_F64;
 *   EXX_CONTRACT_F64     FP64 matrix cores, FP32 operands widened exactly,
 *                        FP64 accumulation;
 *   EXX_CONTRACT_BF16    BF16 matrix cores: v F_P formed in FP32, both operands
 *                        rounded to bfloat16 (nearest even), FP32 accumulation
 *                        over at most 256 grid points, added into FP64;
 *   EXX_CONTRACT_BF16X3  BF16 matrix cores on split operands x = hi + lo
 *                        (hi = bf16(x), lo = bf16(x - hi), 16 significant
 *                        bits), three products hi hi + hi lo + lo hi per term,
 *                        accumulation as EXX_CONTRACT_BF16.
 * EXX_F64 builds (FP64-stored transforms) return EXX_ERR_UNSUPPORTED while a
 * BF16 form is set. Returns EXX_ERR_ARG for an unknown form.
 */
/*
 * exx_set_fit -- the ISDF fit of every later exx_build and exx_build_batched
 * call of this handle (exx_isdf_fit always fits per transfer):
 *   EXX_FIT_PER_Q   (default) one fit per transfer q (Sec. 2.3, Eq. 16):
 *                   S^m xi^m = Z^m for every m;
 *   EXX_FIT_SHARED  one fit for all transfers: the k-point fit of Sec. 2.2
 *                   (Eq. 13) restricted to occupied pairs, i.e. the least-
 *                   squares problem over the pairs of every transfer,
 *                   (sum_m S^m) xi = sum_m Z^m in the cell-periodic gauge of the
 *                   per-transfer fit. One factorisation, one grid-sized solve and
 *                   one 3-D FFT per point serve every transfer; the Coulomb
 *                   matrices V^m_PQ = (Omega/N_g^2) sum_g v^m(g) F_P conj F_Q
 *                   differ only in the kernel v^m, then the Bloch phases. Less
 *                   accurate than the per-transfer fit at the same N_ISDF (one
 *                   set of functions spans the pairs of every transfer). rank[m]
 *                   is the shared metric's rank for every m; with
 *                   EXX_STRICT_PD a lost pivot reports transfer 0. Scratch: Gamma
 *                   and Z of one chunk of grid columns, Y = W Z and its
 *                   transform (N_ISDF N_g each) instead of one per transfer.
 * Returns EXX_ERR_ARG for an unknown mode.
 */
#define EXX_FIT_PER_Q 0
#define EXX_FIT_SHARED 1
exx_status exx_set_fit(exx_handle_t h, int32_t mode);

#define EXX_CONTRACT_AUTO 0
#define EXX_CONTRACT_F64 1
#define EXX_CONTRACT_BF16 2
#define EXX_CONTRACT_BF16X3 3
exx_status exx_set_contraction(exx_handle_t h, int32_t form);

/*
 * Per-phase timing (instrumentation, not part of the method). When enabled,
 * the library records a pair of HIP events on the call's stream around each
 * phase of every subsequent call. exx_phase_times synchronises on those
 * events and returns, per phase, the summed elapsed milliseconds and the
 * number of recorded intervals since timing was enabled or last read, then
 * resets the counters.
 *
 * enable = 2 also runs the phases that normally overlap on the build's two
 * streams (the factorisation chain beside Gamma, each chunk's transform beside
 * the previous chunk's contraction) one after another, so that every phase's
 * interval covers its own kernels only (slower builds; for per-kernel rates).
 *
 * Phases: 0 G^n, 1 S^m, 2 Cholesky, 3 S^+ (triangular inverse and W^H W),
 * 4 Gamma^n, 5 Z^m k-correlation, 6 fit solve, 7 grid FFT, 8 Coulomb
 * contraction, 9 k-convolution Y^n, 10 K^n, 11 E_x.
 *
 *   ms    out [n] double (host), calls out [n] int32 (host), n <= EXX_NPHASE
 */
#define EXX_NPHASE 12
exx_status exx_set_timing(exx_handle_t h, int enable);
exx_status exx_phase_times(exx_handle_t h, double* ms, int32_t* calls, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* EXX_H */

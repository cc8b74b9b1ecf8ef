// C ABI entry points: argument checks, scratch layout and the launch sequence
// of one THC-oo-K exchange build.
#include <algorithm>
#include <cerrno>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <optional>
#include <type_traits>

#include "common.h"

// Scratch of the allocation-free exchange contraction (exx_build_K_noalloc):
// one copy per GPU, placed by the loader with the code object and held until
// the process ends. Host code never uses this name as an address; it uses the
// device address from hipGetSymbolAddress, kept per device in noalloc_ptr.
static __device__ __align__(256) char scratch[EXX_NOALLOC_MAX_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex noalloc_mu;
char* noalloc_ptr[MAX_DEVICES] = {};

// With `device` current: the device address of its copy of `scratch`, looked
// up once per device.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (noalloc_ptr[device]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  noalloc_ptr[device] = (char*)p;
  return hipSuccess;
}

char* noalloc_base(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  return noalloc_ptr[device];
}
}  // namespace

namespace exx {

Geom make_geom(const exx_cell& c) {
  Geom g;
  for (int a = 0; a < 3; ++a) {
    g.L[a] = c.L[a];
    g.n[a] = c.grid[a];
    g.N[a] = c.kmesh[a];
  }
  g.nk = c.kmesh[0] * c.kmesh[1] * c.kmesh[2];
  g.ng = c.grid[0] * c.grid[1] * c.grid[2];
  g.no = c.n_occ;
  g.nao = c.n_ao;
  g.ni = c.n_isdf;
  g.omega = c.L[0] * c.L[1] * c.L[2];
  return g;
}

exx_status fail(exx_context* h, exx_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

exx_status hip_check(exx_context* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return EXX_OK;
  return fail(h, EXX_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void* ws_get(exx_context* h, size_t bytes, exx_status* st) {
  *st = EXX_OK;
  if (h->user_ws) {
    if (bytes <= h->user_ws_bytes) return h->user_ws;
    *st = fail(h, EXX_ERR_NOMEM,
               "the workspace set by exx_set_workspace holds " + std::to_string(h->user_ws_bytes) +
                   " bytes; this call needs " + std::to_string(bytes));
    return nullptr;
  }
  if (h->ws.cap >= bytes) return h->ws.base;
  if (h->ws.base) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      *st = hip_check(h, e, "hipDeviceSynchronize");
      return nullptr;
    }
    (void)hipFree(h->ws.base);
    h->ws.base = nullptr;
    h->ws.cap = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *st = fail(h, EXX_ERR_NOMEM, "scratch allocation of " + std::to_string(bytes) + " bytes failed");
    return nullptr;
  }
  h->ws.base = (char*)p;
  h->ws.cap = bytes;
  return p;
}

static hipEvent_t take_event(exx_context* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

PhaseTimer::PhaseTimer(exx_context* h, int phase, hipStream_t st) : h_(h), phase_(phase), st_(st) {
  if (!h_->timing) return;
  a_ = take_event(h_);
  if (a_ && hipEventRecord(a_, st_) != hipSuccess) a_ = nullptr;
}

PhaseTimer::~PhaseTimer() {
  if (!a_) return;
  hipEvent_t b = take_event(h_);
  if (!b) return;
  if (hipEventRecord(b, st_) != hipSuccess) return;
  h_->recs.push_back({phase_, a_, b});
}

namespace {

size_t al(size_t b) { return (b + 255) / 256 * 256; }

bool smooth235(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

// the contraction form of a call in precision prec (COUL_*), or -1 where the
// handle asks for a BF16 form on FP64-stored transforms
int coul_form(const exx_context* h, exx_prec prec) {
  int f = h->contract;
  if (f == EXX_CONTRACT_AUTO) f = prec == EXX_BF16 ? EXX_CONTRACT_BF16 : EXX_CONTRACT_F64;
  if (f == EXX_CONTRACT_F64) return COUL_F64;
  if (prec == EXX_F64) return -1;
  return f == EXX_CONTRACT_BF16 ? COUL_BF16 : COUL_BF16X3;
}

exx_status check_form(exx_context* h, exx_prec prec) {
  if (coul_form(h, prec) < 0)
    return fail(h, EXX_ERR_UNSUPPORTED,
                "a BF16 contraction form needs FP32-stored transforms (not EXX_F64)");
  return EXX_OK;
}

exx_status check_cell(exx_context* h, const exx_cell* c, exx_prec prec) {
  if (!c) return fail(h, EXX_ERR_ARG, "cell is NULL");
  if (prec != EXX_F64 && prec != EXX_F32 && prec != EXX_BF16 && prec != EXX_MIXED)
    return fail(h, EXX_ERR_ARG, "unknown precision");
  for (int a = 0; a < 3; ++a) {
    if (!(c->L[a] > 0.0)) return fail(h, EXX_ERR_SHAPE, "cell edges must be positive");
    if (c->grid[a] < 2 || c->grid[a] > 128 || !smooth235(c->grid[a]))
      return fail(h, EXX_ERR_SHAPE, "grid sizes must be 2..128 and 2*3*5-smooth");
    if (c->kmesh[a] < 1 || c->kmesh[a] > 8) return fail(h, EXX_ERR_SHAPE, "k-mesh sizes must be 1..8");
  }
  if (c->n_occ < 1 || c->n_occ > 512) return fail(h, EXX_ERR_SHAPE, "n_occ must be 1..512");
  if (c->n_ao < 1 || c->n_ao > 4096) return fail(h, EXX_ERR_SHAPE, "n_ao must be 1..4096");
  if (c->n_isdf < 1 || c->n_isdf > 2048) return fail(h, EXX_ERR_SHAPE, "n_isdf must be 1..2048");
  Geom g = make_geom(*c);
  if (g.ni > g.ng) return fail(h, EXX_ERR_SHAPE, "n_isdf exceeds the number of grid points");
  if (!kcorr_supported(g)) return fail(h, EXX_ERR_SHAPE, "the k-mesh may hold at most 64 points");
  if (!fft_supported(g, prec == EXX_F64))
    return fail(h, EXX_ERR_UNSUPPORTED, "grid shape not supported by the FFT (n2*n3 <= 6144)");
  // the grid GEMMs and k-correlations address one transfer's grid-sized arrays
  // (n_isdf or n_occ complex128 functions over the grid) with 32-bit byte offsets
  if ((long)std::max(g.ni, g.no) * g.ng * (long)sizeof(double2) >= 0xffffffffL)
    return fail(h, EXX_ERR_UNSUPPORTED,
                "n_isdf * N_g and n_occ * N_g must be below 2^28 (one transfer's grid arrays "
                "are addressed with 32-bit offsets)");
  return EXX_OK;
}

// Transfers m and -m of the mesh: the fitted pair functions of -m are the
// conjugates of those of m (relabelling n), so Vb^{-m} = conj Vb^m and the
// Cholesky pivots (hence the ranks) agree. The paired path below fits and
// contracts one transfer of each pair (rep, slice order), then writes both.
// It splits the solve at the factor as the real path does:
// Y = W Z on the grid (W lower triangular), the contraction of the transform of
// Y gives Vy, and V^m = W^H Vy W before the Bloch phases are applied.
struct Pairs {
  int n = 0;
  int rep[64], bar[64], slot[64];
};

Pairs make_pairs(const Geom& g) {
  Pairs p;
  for (int m = 0; m < 64; ++m) p.slot[m] = -1;
  for (int m = 0; m < g.nk; ++m) {
    const int m1 = m / (g.N[1] * g.N[2]), m2 = (m / g.N[2]) % g.N[1], m3 = m % g.N[2];
    const int b = (((g.N[0] - m1) % g.N[0]) * g.N[1] + (g.N[1] - m2) % g.N[1]) * g.N[2] +
                  (g.N[2] - m3) % g.N[2];
    if (m <= b) {
      p.slot[m] = p.n;
      p.rep[p.n] = m;
      p.bar[p.n] = b != m ? b : -1;
      ++p.n;
    }
  }
  return p;
}

// which form the fused build takes (fit_coulomb)
enum BuildPath { PATH_STAGES = 0, PATH_REAL = 1, PATH_PAIRED = 2, PATH_SHARED = 3 };

BuildPath build_path(const exx_context* h, const Geom& g) {
  if (h->fit_mode == EXX_FIT_SHARED) return PATH_SHARED;
  if (kcorr_real(g)) return PATH_REAL;
  return make_pairs(g).n < g.nk ? PATH_PAIRED : PATH_STAGES;
}

// the paired path's chunking: fit over `cols` grid columns at a time, the
// transform and contraction over `per` transfers at a time (two buffers)
struct PairedDims {
  int cols, per, nchunk;
};

PairedDims paired_dims(const exx_context* h, const Geom& g, size_t cs) {
  PairedDims d;
  const size_t per_col = cs * (size_t)g.nk * g.ni;
  size_t cols = h->fit_chunk_bytes / per_col;
  cols = cols / 256 * 256;
  if (cols < 256) cols = 256;
  d.cols = (int)std::min<size_t>(cols, (size_t)g.ng);
  const int np = make_pairs(g).n;
  d.nchunk = std::min(4, np);
  d.per = (np + d.nchunk - 1) / d.nchunk;
  return d;
}

// scratch layout shared by the three calls
struct Layout {
  size_t G, Lf, W, Sp, keep, Y, T, epart, cpart, S2, V2, rank2, tol, Tinv, grid, grid2, F, total;
  // the exchange gradient's buffers: a third grid-sized array, the kernel table,
  // the point-sized correlation and the AO-sized products
  size_t g3, gvt, gCS, gT, gA, gP;
  int nsplit;
  PairedDims pd;
};

// what a call needs besides the point-sized matrices
enum Need { NEED_FIT = 1, NEED_COULOMB = 2, NEED_K = 4, NEED_BUILD = 8, NEED_GRAD = 16 };

Layout layout(const exx_context* h, const Geom& g, exx_prec prec, int need) {
  const bool grad = (need & NEED_GRAD) != 0;
  const bool build = (need & NEED_BUILD) != 0 || grad;
  const bool grid = (need & (NEED_FIT | NEED_COULOMB | NEED_BUILD | NEED_GRAD)) != 0;
  const bool paired = !grad && build && build_path(h, g) == PATH_PAIRED;
  const bool shared = !grad && build && build_path(h, g) == PATH_SHARED;
  Layout L;
  const size_t mat = al(sizeof(double2) * (size_t)g.nk * g.ni * g.ni);
  // Gamma/Z (and F) buffer: FP64 unless the fit itself runs in FP32; xi: FP64 only in EXX_F64
  const size_t cs = (prec == EXX_F64 || prec == EXX_MIXED) ? sizeof(double2) : sizeof(float2);
  const size_t cx = prec == EXX_F64 ? sizeof(double2) : sizeof(float2);
  size_t o = 0;
  L.G = o;
  o += mat;
  L.Lf = o;
  o += mat;
  L.W = o;
  o += mat;
  L.Sp = o;
  o += mat;
  L.keep = o;
  o += al(sizeof(int32_t) * (size_t)g.nk * g.ni);
  L.Y = o;
  o += mat;
  L.T = o;
  o += al(sizeof(double2) * (size_t)g.nk * g.ni * g.nao);
  L.epart = o;
  o += al(sizeof(double) * 1024);
  L.nsplit = coulomb_nsplit(g);
  L.cpart = o;
  o += grid ? al(coulomb_partial_bytes(g, L.nsplit)) : 0;
  L.S2 = o;
  o += build ? mat : 0;
  L.V2 = o;
  o += build ? mat : 0;
  L.rank2 = o;
  o += al(sizeof(int32_t) * g.nk);
  L.tol = o;
  o += al(sizeof(double) * g.nk);
  L.Tinv = o;
  o += al(sizeof(double2) * (size_t)g.nk * 32 * g.ni);
  L.pd = paired_dims(h, g, cs);
  L.grid = o;
  if (paired || shared)  // Gamma / Z of one chunk of grid columns
    o += al(cs * (size_t)g.nk * g.ni * L.pd.cols);
  else
    o += grid ? al(cs * (size_t)g.nk * g.ni * g.ng) : 0;
  L.grid2 = o;
  if (paired)  // Y = W Z of the representative transfers
    o += al(cx * (size_t)make_pairs(g).n * g.ni * g.ng);
  else if (shared)  // Y = W Z of the shared fit
    o += al(cx * (size_t)g.ni * g.ng);
  else
    o += build ? al(cx * (size_t)g.nk * g.ni * g.ng) : 0;
  L.F = o;
  if (paired)  // transforms of two chunks of transfers
    o += 2 * al(cx * (size_t)L.pd.per * g.ni * g.ng);
  else if (shared)  // the one transform
    o += al(cx * (size_t)g.ni * g.ng);
  L.g3 = L.gvt = L.gCS = L.gT = L.gA = L.gP = o;
  if (grad) {
    L.g3 = o;
    o += al(sizeof(double2) * (size_t)g.nk * g.ni * g.ng);
    L.gvt = o;
    o += al(sizeof(double) * (size_t)g.nk * g.ng);
    L.gCS = o;
    o += mat;
    L.gT = o;
    o += al(sizeof(double2) * (size_t)g.nk * g.ni * g.nao);
    L.gA = o;
    o += al(sizeof(double2) * (size_t)g.nk * g.nao * g.nao);
    L.gP = o;  // slices of the split sum over the grid
    o += al(sizeof(double2) * (size_t)gemm_splitk_parts(g.ni, g.nao, g.ng, g.nk) * g.nk * g.ni *
            g.nao);
  }
  L.total = o;
  return L;
}

// the second stream of a build and its events (default priority)
hipError_t make_lane_streams(hipStream_t* aux, hipEvent_t* fork, hipEvent_t* join, hipEvent_t* chain,
                             hipEvent_t* fb) {
  hipError_t e = hipStreamCreateWithFlags(aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(chain, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fb[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fb[1], hipEventDisableTiming);
  return e;
}

// serial timing (exx_set_timing(h, 2)): `after` waits for everything queued so
// far on `before`, so that two phases on different streams do not overlap
hipError_t serialize(exx_context* h, hipStream_t before, hipStream_t after) {
  if (!(h->timing && h->serial)) return hipSuccess;
  hipError_t e = hipEventRecord(h->join_ev, before);
  if (e == hipSuccess) e = hipStreamWaitEvent(after, h->join_ev, 0);
  return e;
}

// status word for the kernels' reports (null when no check is enabled)
int32_t* stat_ptr(exx_context* h) {
  return (h->checks & (EXX_CHECK_FINITE | EXX_STRICT_PD)) ? h->dstat : nullptr;
}
bool strict_pd(exx_context* h) { return (h->checks & EXX_STRICT_PD) != 0; }

// non-finite scans of a call's small inputs and outputs (EXX_CHECK_FINITE)
exx_status scan(exx_context* h, const void* p, long n_doubles, int site, hipStream_t st) {
  if (!(h->checks & EXX_CHECK_FINITE) || !p) return EXX_OK;
  return hip_check(h, launch_check_finite((const double*)p, n_doubles, h->dstat, site, st),
                   "finite check");
}

// read and clear the status word after synchronising st
exx_status read_status(exx_context* h, hipStream_t st, int32_t* info) {
  int32_t v[3] = {0, INT_MAX, INT_MAX};
  hipError_t e = hipMemcpyAsync(v, h->dstat, sizeof(v), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = launch_status_reset(h->dstat, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_check(h, e, "status read");
  if (info) {
    info[0] = (v[0] & ST_NOT_PD) ? v[1] : -1;
    info[1] = (v[0] & ST_NONFINITE) ? v[2] : 0;
  }
  if (v[0] & ST_NONFINITE)
    return fail(h, EXX_ERR_NONFINITE, "non-finite value (site " + std::to_string(v[2]) +
                                          ": 1 occ_pts, 2 ao_pts, 3 fit metric, 4 Coulomb "
                                          "matrices, 5 K or E_x)");
  if (v[0] & ST_NOT_PD)
    return fail(h, EXX_ERR_NOT_PD, "fit metric of transfer " + std::to_string(v[1]) +
                                       " lost a pivot to the drop rule (EXX_STRICT_PD)");
  return EXX_OK;
}

// end of a K-build call: with EXX_CHECK_SYNC the call waits for its work and
// returns the status word
exx_status finish(exx_context* h, hipStream_t st) {
  if (!(h->checks & EXX_CHECK_SYNC)) return EXX_OK;
  return read_status(h, st, nullptr);
}

// TF: type of Gamma^n / Z^m (and of psi_grid); TX: storage type of xi
// bf16 (with TF = float): Gamma^n on the BF16 matrix cores
// in_grid (TF == TX): leave xi where Z^m was (the grid buffer, or zbuf) and use
// `xi` only as the solve's scratch (no final copy)
template <typename TF, typename TX>
exx_status fit_impl(exx_context* h, const Geom& g, const Tables& tb, char* ws, const Layout& L,
                    const void* psi, const void* occ, const int32_t* pts, void* xi, void* S,
                    int32_t* rank, hipStream_t st, bool bf16 = false, bool in_grid = false,
                    void* zbuf = nullptr, const Pairs* pr = nullptr) {
  double2* G = (double2*)(ws + L.G);
  double2* Lf = (double2*)(ws + L.Lf);
  double2* W = (double2*)(ws + L.W);
  double2* Sp = (double2*)(ws + L.Sp);
  double2* WH = (double2*)(ws + L.Y);  // W^H (the K-build's Y region is free during a fit)
  int32_t* keep = (int32_t*)(ws + L.keep);
  void* grid = ws + L.grid;
  // Z^m (and then the solve's output) go to zbuf when given, so that Gamma^n
  // stays in grid; otherwise Z^m replaces Gamma^n in place
  void* zg = zbuf ? zbuf : grid;
  // pr: fit one transfer of each conjugate pair (its slices compacted in the
  // order of pr->rep); the ranks are copied to the partners
  Geom gr = g;
  int32_t* rk = rank;
  QLabel lab;
  if (pr) {
    gr.nk = pr->n;
    rk = (int32_t*)(ws + L.rank2);
    for (int k = 0; k < 64; ++k) lab.q[k] = k < pr->n ? pr->rep[k] : 0;
  }
  const int* slot = pr ? pr->slot : nullptr;
  const long nn = (long)g.ni * g.ni;
  hipError_t e;
  // The point-metric chain (a0, a2 at the points, a3) runs on the handle's
  // second stream while the grid-sized Gamma and Z run on st; the solve waits
  // for both. Both streams touch disjoint scratch.
  hipStream_t ax = h->aux;
  e = hipEventRecord(h->fork_ev, st);
  if (e != hipSuccess) return hip_check(h, e, "fork event");
  e = hipStreamWaitEvent(ax, h->fork_ev, 0);
  if (e != hipSuccess) return hip_check(h, e, "fork wait");
  const char* what = nullptr;
  // a0: G^n = Psi^n Psi^n^H (FP64)
  {
    PhaseTimer pt(h, PH_GRAM, ax);
    e = gemm<double, double, double, double>(g.ni, g.ni, g.no, g.nk, A_N, occ, g.no,
                                             (long)g.ni * g.no, B_C, occ, g.no,
                                             (long)g.ni * g.no, G, g.ni, nn, 1.0, false, ax);
  }
  if (e != hipSuccess) what = "G gemm";
  // a2 at the points: S^m = e^{iq(r_P - r_Q)} sum_n G^n o conj G^{n+m}
  if (!what) {
    PhaseTimer pt(h, PH_METRIC, ax);
    e = launch_kcorr<double>(g, tb, G, S, g.ni, pts, true, ax, slot);
    if (e != hipSuccess) what = "S kcorr";
  }
  // a3: Cholesky with drop, inverse factor, S^+ = W^H W
  if (!what) {
    PhaseTimer pt(h, PH_CHOL, ax);
    e = launch_copy(Lf, (const double2*)S, (long)gr.nk * nn, ax);
    if (e != hipSuccess) what = "copy S";
    if (!what) {
      e = launch_chol_blocked(gr, Lf, keep, rk, (double*)(ws + L.tol), 1e-12, ax, stat_ptr(h),
                              strict_pd(h), pr ? &lab : nullptr);
      if (e != hipSuccess) what = "cholesky";
    }
  }
  if (!what) {
    PhaseTimer pt(h, PH_PINV, ax);
    e = launch_tri_inv_blocked(gr, Lf, keep, W, (double2*)(ws + L.Tinv), ax);
    if (e != hipSuccess) what = "triangular inverse";
    if (!what) {
      e = gemm<double, double, double, double>(g.ni, g.ni, g.ni, gr.nk, A_C, W, g.ni, nn, B_N, W,
                                               g.ni, nn, Sp, g.ni, nn, 1.0, false, ax);
      if (e != hipSuccess) what = "S+ gemm";
    }
    if (!what) {
      e = launch_conj_transpose(W, WH, g.ni, g.ni, gr.nk, 1.0, ax);
      if (e != hipSuccess) what = "W^H";
    }
    if (!what && pr) {
      e = launch_rank_scatter(rk, rank, pr->rep, pr->bar, pr->n, ax);
      if (e != hipSuccess) what = "rank scatter";
    }
  }
  // join back into st even after an error, so that st never runs ahead of the
  // chain (and a capture stays joined)
  hipError_t ej = hipEventRecord(h->join_ev, ax);
  if (what) {
    if (ej == hipSuccess) (void)hipStreamWaitEvent(st, h->join_ev, 0);
    return hip_check(h, e, what);
  }
  if (ej != hipSuccess) return hip_check(h, ej, "join event");
  // a1: Gamma^n(P, r)
  {
    PhaseTimer pt(h, PH_GAMMA, st);
    if (std::is_same<TF, double>::value)
      e = zgemm_nn_grid<double, double>(g.ni, g.ng, g.no, g.nk, occ, g.no, (long)g.ni * g.no, true,
                                        psi, g.ng, (long)g.no * g.ng, grid, g.ng,
                                        (long)g.ni * g.ng, st, h->tile_gamma);
    else if (bf16)
      e = cgemm_nn_grid_bf16(g.ni, g.ng, g.no, g.nk, occ, g.no, (long)g.ni * g.no, psi, g.ng,
                             (long)g.no * g.ng, grid, g.ng, (long)g.ni * g.ng, st);
    else
      e = cgemm_nn_grid32(g.ni, g.ng, g.no, g.nk, occ, g.no, (long)g.ni * g.no, true, psi, g.ng,
                          (long)g.no * g.ng, grid, g.ng, (long)g.ni * g.ng, st);
  }
  if (e != hipSuccess) what = "Gamma gemm";
  // a2: Z^m in place
  if (!what) {
    PhaseTimer pt(h, PH_KCORR, st);
    e = launch_kcorr<TF>(g, tb, grid, zg, g.ng, pts, false, st, slot);
    if (e != hipSuccess) what = "Z kcorr";
  }
  hipError_t ew = hipStreamWaitEvent(st, h->join_ev, 0);
  if (what) return hip_check(h, e, what);
  if (ew != hipSuccess) return hip_check(h, ew, "join wait");
  // a4: xi^m = S^+ Z^m in FP64 arithmetic. Without refinement it is applied in
  // the factor form xi = W^H (W Z) (S^+ = W^H W): Y = W Z into xi, then W^H Y
  // into the Z buffer and back into xi. Applying the explicitly formed S^+
  // instead squares the metric's conditioning in the rounding error, which
  // loses every digit where Z lies close to the range of a metric with
  // cond 1e9 (a fit at full pair rank). With refinement the explicit S^+ is
  // applied and then refined below.
  if (h->refine == 0) {
    PhaseTimer pt(h, PH_SOLVE, st);
    e = zgemm_nn_grid<TF, TX>(g.ni, g.ng, g.ni, gr.nk, W, g.ni, nn, false, zg, g.ng,
                              (long)g.ni * g.ng, xi, g.ng, (long)g.ni * g.ng, st, h->tile_solve,
                              true);
    if (e == hipSuccess)
      e = zgemm_nn_grid<TX, TF>(g.ni, g.ng, g.ni, gr.nk, WH, g.ni, nn, false, xi, g.ng,
                                (long)g.ni * g.ng, zg, g.ng, (long)g.ni * g.ng, st,
                                h->tile_solve);
    if (e == hipSuccess && !in_grid)
      e = launch_convert<TF, TX>(zg, xi, (long)gr.nk * g.ni * g.ng, st);
    if (e != hipSuccess) return hip_check(h, e, "solve gemm");
    return EXX_OK;
  }
  {
    PhaseTimer pt(h, PH_SOLVE, st);
    e = zgemm_nn_grid<TF, TX>(g.ni, g.ng, g.ni, gr.nk, Sp, g.ni, nn, false, zg, g.ng,
                            (long)g.ni * g.ng, xi, g.ng, (long)g.ni * g.ng, st, h->tile_solve);
  }
  if (e != hipSuccess) return hip_check(h, e, "solve gemm");
  if (h->refine > 0) {
    // one step of iterative refinement: Z <- Z - S^m xi (the residual, over Z),
    // then xi <- xi + S^+ Z; both products in FP64 arithmetic
    PhaseTimer pt(h, PH_SOLVE, st);
    e = zgemm_nn_grid_acc<TX, TF>(g.ni, g.ng, g.ni, gr.nk, S, g.ni, nn, xi, g.ng,
                                  (long)g.ni * g.ng, zg, g.ng, (long)g.ni * g.ng, -1, st);
    if (e != hipSuccess) return hip_check(h, e, "refinement residual");
    e = zgemm_nn_grid_acc<TF, TX>(g.ni, g.ng, g.ni, gr.nk, Sp, g.ni, nn, zg, g.ng,
                                  (long)g.ni * g.ng, xi, g.ng, (long)g.ni * g.ng, 1, st);
    if (e != hipSuccess) return hip_check(h, e, "refinement update");
  }
  if (in_grid) {
    e = launch_convert<TX, TF>(xi, zg, (long)gr.nk * g.ni * g.ng, st);
    if (e != hipSuccess) return hip_check(h, e, "xi into the grid buffer");
  }
  return EXX_OK;
}

// T: storage of xi and F; cform: the contraction's form (COUL_*; FP32 storage only)
// pr: xi holds one transfer of each conjugate pair (slices in the order of
// pr->rep); V is written for every transfer (Vb^{-m} = conj Vb^m)
template <typename T>
exx_status coulomb_impl(exx_context* h, const Geom& g, const Tables& tb, char* ws, const Layout& L,
                        const void* xi, const int32_t* pts, void* V, hipStream_t st,
                        int cform = COUL_F64, void* Fout = nullptr, const Pairs* pr = nullptr) {
  void* F = Fout ? Fout : ws + L.grid;  // the transforms F^m
  const int ns = pr ? pr->n : g.nk;
  hipError_t e;
  {
    PhaseTimer pt(h, PH_FFT, st);
    e = launch_fft3d<T>(g, tb, xi, F, (long)ns * g.ni, h->ncu, st);
  }
  if (e != hipSuccess) return hip_check(h, e, "fft");
  {
    PhaseTimer pt(h, PH_COULOMB, st);
    e = launch_coulomb<T>(g, tb, F, pts, ws + L.cpart, L.nsplit, (double2*)V, false, st,
                          pr ? pr->rep : nullptr, pr ? pr->bar : nullptr, pr ? pr->n : 0, false,
                          cform);
  }
  if (e != hipSuccess) return hip_check(h, e, "coulomb");
  return EXX_OK;
}

// Fit and Coulomb matrices of the fused build on meshes whose every axis has
// N_i <= 2 (every transfer self-conjugate, refinement off). There the unphased
// metric S~ and right-hand side Z~ are real, S^m = D S~ D^H and
// Z^m = D Z~ e^{-iq.r} with D = diag(e^{iq.r_P}), so xi^m = D eta e^{-iq.r} with
// the real eta = S~^+ Z~; the Bloch-gauge Vb^m is the real
// sum_G v(G) Re(H_P conj H_Q) over the pairs G <-> -G - 2q of the twisted
// transform H = FFT(eta e^{-iq.r}). Same quantities as fit_impl + coulomb_impl,
// in real arithmetic. TF: Gamma storage, TZ: Z~, TX: eta and the transform.
// The factorisation chain of the metric (many short launches) runs on the
// caller's stream and the grid-sized Gamma and Z~ on the handle's second
// stream; the solve waits for both.
//
// The solve is split at the factor: with S~^+ = W^T W (W the inverted Cholesky
// factor, lower triangular in point order) the grid-sized product is Y = W Z~,
// half the multiply-adds of S~^+ Z~; Y is transformed and contracted like eta,
// giving Vy = sum_G v Re(HY_P conj HY_Q), and Vb = W^T Vy W by two small
// products. Rounding of Y, of its transform and of Vy reaches Vb through
// W^T (.) W, amplified by cond(S~) at most, as rounding of Z~ is in the eta
// form. With Z~ in FP64 and Y stored in FP32 (MIXED) the measured errors are
// lower than with eta stored in FP32, not higher.
template <typename TF, typename TZ, typename TX>
exx_status fit_coulomb_real(exx_context* h, const Geom& g, const Tables& tb, char* ws,
                            const Layout& L, const void* psi, const void* occ, const int32_t* pts,
                            void* S, void* V, int32_t* rank, hipStream_t st, bool bf16 = false,
                            int cform = COUL_F64) {
  double2* G = (double2*)(ws + L.G);
  double2* Lf = (double2*)(ws + L.Lf);
  double2* W = (double2*)(ws + L.W);
  double2* Sp = (double2*)(ws + L.Sp);
  int32_t* keep = (int32_t*)(ws + L.keep);
  void* grid = ws + L.grid;    // Gamma (FP64), then eta
  void* grid2 = ws + L.grid2;  // Z~, then the half-grid transform
  const long nn = (long)g.ni * g.ni;
  hipError_t e;
  hipStream_t ax = st;           // the factorisation chain stays on the caller's stream
  hipStream_t gs = h->aux;       // Gamma and Z~ go to the second stream
  e = hipEventRecord(h->fork_ev, st);
  if (e != hipSuccess) return hip_check(h, e, "fork event");
  e = hipStreamWaitEvent(gs, h->fork_ev, 0);
  if (e != hipSuccess) return hip_check(h, e, "fork wait");
  const char* what = nullptr;
  {
    PhaseTimer pt(h, PH_GRAM, ax);
    e = gemm<double, double, double, double>(g.ni, g.ni, g.no, g.nk, A_N, occ, g.no,
                                             (long)g.ni * g.no, B_C, occ, g.no,
                                             (long)g.ni * g.no, G, g.ni, nn, 1.0, false, ax);
  }
  if (e != hipSuccess) what = "G gemm";
  if (!what) {
    PhaseTimer pt(h, PH_METRIC, ax);
    e = launch_kcorr_real<double, double2>(g, G, S, g.ni, ax);
    if (e != hipSuccess) what = "S kcorr";
  }
  if (!what) {
    PhaseTimer pt(h, PH_CHOL, ax);
    e = launch_copy(Lf, (const double2*)S, (long)g.nk * nn, ax);
    if (e != hipSuccess) what = "copy S";
    if (!what) {
      e = launch_chol_blocked_real(g, Lf, keep, rank, (double*)(ws + L.tol), 1e-12, ax,
                                   stat_ptr(h), strict_pd(h));
      if (e != hipSuccess) what = "cholesky";
    }
  }
  if (!what) {
    PhaseTimer pt(h, PH_PINV, ax);
    e = launch_tri_inv_real(g, Lf, keep, W, (double2*)(ws + L.Tinv), ax);
    if (e != hipSuccess) what = "triangular inverse";
    // the refinement multiplies by L itself: clear what the factorisation left
    // above its diagonal
    if (!what && h->refine > 0) {
      e = launch_zero_upper(Lf, g.ni, g.nk, ax);
      if (e != hipSuccess) what = "factor";
    }
  }
  if (what) {
    (void)hipEventRecord(h->join_ev, gs);
    (void)hipStreamWaitEvent(st, h->join_ev, 0);
    return hip_check(h, e, what);
  }
  e = serialize(h, ax, gs);
  if (e != hipSuccess) return hip_check(h, e, "serial timing");
  if constexpr (std::is_same<TF, float>::value) {
    // FP32: Gamma^n and the real k-correlation in one pass; only Z~ is written.
    // occ is narrowed to c64 first, into the K-build's scratch (free until then)
    PhaseTimer pt(h, PH_GAMMA, gs);
    float2* occ32 = (float2*)(ws + L.T);
    e = launch_narrow((const double2*)occ, occ32, (long)g.nk * g.ni * g.no, gs);
    if (e == hipSuccess)
      e = bf16 ? launch_gamma_kcorr_bf16(g, occ32, psi, grid2, gs)
               : launch_gamma_kcorr<float, float>(g, occ32, psi, grid2, gs);
    if (e != hipSuccess) what = "Gamma and Z kcorr";
  } else {
    // FP64: the three-product Gamma GEMM, then the real k-correlation
    {
      PhaseTimer pt(h, PH_GAMMA, gs);
      e = zgemm_nn_grid<double, double>(g.ni, g.ng, g.no, g.nk, occ, g.no, (long)g.ni * g.no, true,
                                        psi, g.ng, (long)g.no * g.ng, grid, g.ng,
                                        (long)g.ni * g.ng, gs, h->tile_gamma);
    }
    if (e != hipSuccess) what = "Gamma gemm";
    if (!what) {
      PhaseTimer pt(h, PH_KCORR, gs);
      e = launch_kcorr_real<TF, TZ>(g, grid, grid2, g.ng, gs);
      if (e != hipSuccess) what = "Z kcorr";
    }
  }
  hipError_t ej = hipEventRecord(h->join_ev, gs);
  hipError_t ew = ej == hipSuccess ? hipStreamWaitEvent(st, h->join_ev, 0) : ej;
  if (what) return hip_check(h, e, what);
  if (ew != hipSuccess) return hip_check(h, ew, "join wait");
  {
    PhaseTimer pt(h, PH_SOLVE, st);
    e = dgemm_nn_grid<TZ, TX>(g.ni, g.ng, g.ni, g.nk, W, g.ni, nn, grid2, g.ng,
                              (long)g.ni * g.ng, grid, g.ng, (long)g.ni * g.ng, st, true);
  }
  if (e != hipSuccess) return hip_check(h, e, "solve gemm");
  if (h->refine > 0) {
    // one step of iterative refinement in the factor form: with S~ = L L^T on the
    // retained points, the residual of eta = W^T Y is L (W Z~ - Y), so
    // R = Z~ - L Y (over Z~) and Y += W R, both sums in FP64
    PhaseTimer pt(h, PH_SOLVE, st);
    e = dgemm_nn_grid_acc<TX, TZ>(g.ni, g.ng, g.ni, g.nk, Lf, g.ni, nn, grid, g.ng,
                                  (long)g.ni * g.ng, grid2, g.ng, (long)g.ni * g.ng, -1, st, true);
    if (e == hipSuccess)
      e = dgemm_nn_grid_acc<TZ, TX>(g.ni, g.ng, g.ni, g.nk, W, g.ni, nn, grid2, g.ng,
                                    (long)g.ni * g.ng, grid, g.ng, (long)g.ni * g.ng, 1, st, true);
    if (e != hipSuccess) return hip_check(h, e, "refinement");
  }
  // FP64 storage: the transfers go in four chunks, the transform of each chunk
  // on the caller's stream and its contraction on the second stream, so that
  // the transform of one chunk runs beside the contraction of the one before
  // (the FP64 transform is latency bound, the contraction matrix-core bound).
  // With FP32 storage the two contend for the CUs and nothing is gained, so
  // that path keeps one transform and one contraction. The timed phases of the
  // chunked form overlap.
  const int nchunk = sizeof(TX) == 8 ? std::min(4, g.nk) : 1;
  if (nchunk == 1) {
    {
      PhaseTimer pt(h, PH_FFT, st);
      e = launch_fft3d_half<TX, TX>(g, tb, grid, grid2, (long)g.nk * g.ni, 0, h->ncu, st);
    }
    if (e != hipSuccess) return hip_check(h, e, "fft");
    PhaseTimer pt(h, PH_COULOMB, st);
    e = launch_coulomb<TX>(g, tb, grid2, pts, ws + L.cpart, L.nsplit, (double2*)V, true, st,
                           nullptr, nullptr, 0, false, cform);
    if (e != hipSuccess) return hip_check(h, e, "coulomb");
  } else {
    const int per = (g.nk + nchunk - 1) / nchunk;
    const size_t fin = (size_t)g.ni * g.ng * sizeof(TX);  // solved functions per transfer
    const size_t fout = (size_t)g.ni * g.n[0] * g.n[1] * (g.n[2] / 2 + 1) * sizeof(cplx<TX>);
    // timed per launch, so that serial timing gives each phase its own kernels
    for (int c0 = 0; c0 < g.nk && !what; c0 += per) {
      const int cn = std::min(per, g.nk - c0);
      {
        PhaseTimer pt(h, PH_FFT, st);
        e = launch_fft3d_half<TX, TX>(g, tb, (const char*)grid + c0 * fin,
                                      (char*)grid2 + c0 * fout, (long)cn * g.ni, c0, h->ncu, st);
      }
      if (e != hipSuccess) what = "fft";
      if (!what) e = hipEventRecord(h->fork_ev, st);
      if (!what && e == hipSuccess) e = hipStreamWaitEvent(gs, h->fork_ev, 0);
      if (!what && e != hipSuccess) what = "chunk fork";
      int rep[64];
      for (int m = 0; m < cn; ++m) rep[m] = c0 + m;
      if (!what) {
        PhaseTimer pt(h, PH_COULOMB, gs);
        e = launch_coulomb<TX>(g, tb, (const char*)grid2 + c0 * fout, pts, ws + L.cpart,
                               L.nsplit, (double2*)V, true, gs, rep, nullptr, cn, false, cform);
      }
      if (!what && e != hipSuccess) what = "coulomb";
      if (!what && serialize(h, gs, st) != hipSuccess) what = "serial timing";
    }
    ej = hipEventRecord(h->join_ev, gs);
    ew = ej == hipSuccess ? hipStreamWaitEvent(st, h->join_ev, 0) : ej;
    if (what) return hip_check(h, e, what);
    if (ew != hipSuccess) return hip_check(h, ew, "join wait");
  }
  {
    PhaseTimer pt(h, PH_COULOMB, st);
    {
      // Vb = W^T Vy W: T = Vy W (real, in the S~^+ scratch), then Vb = W^T T
      const int n = g.ni;
      double* T = (double*)Sp;
      StridedGemm p1{2 * nn, 2 * nn, nn, 2 * n, 2, 2 * n, 2, n, 1, n, n, n};
      e = dgemm_strided(p1, g.nk, (const double*)V, (const double*)W, T, false, st);
      if (e == hipSuccess) {
        StridedGemm p2{2 * nn, nn, 2 * nn, 2, 2 * n, n, 1, 2 * n, 2, n, n, n};
        e = dgemm_strided(p2, g.nk, (const double*)W, T, (double*)V, true, st);
      }
    }
  }
  if (e != hipSuccess) return hip_check(h, e, "coulomb");
  return EXX_OK;
}

// The complex path of the fused build with one transfer per pair (meshes with
// an axis of 3 or more, refinement off): same steps as fit_impl + coulomb_impl
// over the representative transfers, Vb of the partners by conjugation.
//
// Memory is bounded independently of N_k N_ISDF N_g: the fit runs over chunks
// of grid columns (Gamma^n, Z^m and Y = W Z are column-local), writing Y of the
// representative transfers; the transform and the contraction then run over
// chunks of transfers through two transform buffers, the transform of one
// chunk on the caller's stream beside the contraction of the previous one on
// the second stream. Results do not depend on the chunk sizes.
template <typename TF, typename TX>
exx_status fit_coulomb_pairs(exx_context* h, const Geom& g, const Tables& tb, char* ws,
                             const Layout& L, const Pairs& pr, const void* psi, const void* occ,
                             const int32_t* pts, void* V, int32_t* rank, hipStream_t st,
                             bool bf16 = false, int cform = COUL_F64) {
  double2* G = (double2*)(ws + L.G);
  double2* Lf = (double2*)(ws + L.Lf);
  double2* W = (double2*)(ws + L.W);
  double2* Sp = (double2*)(ws + L.Sp);
  int32_t* keep = (int32_t*)(ws + L.keep);
  int32_t* rank_c = (int32_t*)(ws + L.rank2);
  void* gam = ws + L.grid;     // Gamma, then Z (compacted in place), of one column chunk
  char* xi = ws + L.grid2;     // Y = W Z of the representative transfers, full grid
  char* fbuf = ws + L.F;       // transforms of two chunks of transfers
  Geom gr = g;                 // batch over the representative transfers
  gr.nk = pr.n;
  const long nn = (long)g.ni * g.ni;
  const int cc = L.pd.cols;
  hipError_t e;
  hipStream_t ax = st;         // factorisation chain on the caller's stream
  hipStream_t gs = h->aux;     // the fit over column chunks on the second stream
  e = hipEventRecord(h->fork_ev, st);
  if (e != hipSuccess) return hip_check(h, e, "fork event");
  e = hipStreamWaitEvent(gs, h->fork_ev, 0);
  if (e != hipSuccess) return hip_check(h, e, "fork wait");
  const char* what = nullptr;
  {
    PhaseTimer pt(h, PH_GRAM, ax);
    e = gemm<double, double, double, double>(g.ni, g.ni, g.no, g.nk, A_N, occ, g.no,
                                             (long)g.ni * g.no, B_C, occ, g.no,
                                             (long)g.ni * g.no, G, g.ni, nn, 1.0, false, ax);
  }
  if (e != hipSuccess) what = "G gemm";
  if (!what) {
    // S^m of the representative transfers, straight into the factor buffer
    PhaseTimer pt(h, PH_METRIC, ax);
    e = launch_kcorr<double>(g, tb, G, Lf, g.ni, pts, true, ax, pr.slot);
    if (e != hipSuccess) what = "S kcorr";
  }
  if (!what) {
    PhaseTimer pt(h, PH_CHOL, ax);
    QLabel lab;
    for (int k = 0; k < 64; ++k) lab.q[k] = k < pr.n ? pr.rep[k] : 0;
    e = launch_chol_blocked(gr, Lf, keep, rank_c, (double*)(ws + L.tol), 1e-12, ax, stat_ptr(h),
                            strict_pd(h), &lab);
    if (e != hipSuccess) what = "cholesky";
  }
  if (!what) {
    PhaseTimer pt(h, PH_PINV, ax);
    e = launch_tri_inv_blocked(gr, Lf, keep, W, (double2*)(ws + L.Tinv), ax);
    if (e != hipSuccess) what = "triangular inverse";
  }
  if (!what) {
    e = launch_rank_scatter(rank_c, rank, pr.rep, pr.bar, pr.n, ax);
    if (e != hipSuccess) what = "rank scatter";
  }
  if (!what && h->refine > 0) {
    e = launch_zero_upper(Lf, g.ni, gr.nk, ax);
    if (e != hipSuccess) what = "factor";
  }
  if (!what) {
    e = hipEventRecord(h->chain_ev, ax);
    if (e != hipSuccess) what = "chain event";
  }
  if (what) {
    (void)hipEventRecord(h->join_ev, gs);
    (void)hipStreamWaitEvent(st, h->join_ev, 0);
    return hip_check(h, e, what);
  }
  // the fit, one chunk of grid columns at a time; the first chunk's Gamma and Z
  // run beside the factorisation chain, every solve waits for it
  if (h->timing && h->serial) {
    e = hipStreamWaitEvent(gs, h->chain_ev, 0);
    if (e != hipSuccess) what = "serial timing";
  }
  for (int c0 = 0; c0 < g.ng && !what; c0 += cc) {
    const int cn = std::min(cc, g.ng - c0);
    const char* psi_c = (const char*)psi + (size_t)c0 * sizeof(cplx<TF>);
    {
      PhaseTimer pt(h, PH_GAMMA, gs);
      if (std::is_same<TF, double>::value)
        e = zgemm_nn_grid<double, double>(g.ni, cn, g.no, g.nk, occ, g.no, (long)g.ni * g.no, true,
                                          psi_c, g.ng, (long)g.no * g.ng, gam, cn, (long)g.ni * cn,
                                          gs, h->tile_gamma);
      else if (bf16)
        e = cgemm_nn_grid_bf16(g.ni, cn, g.no, g.nk, occ, g.no, (long)g.ni * g.no, psi_c, g.ng,
                               (long)g.no * g.ng, gam, cn, (long)g.ni * cn, gs);
      else
        e = cgemm_nn_grid32(g.ni, cn, g.no, g.nk, occ, g.no, (long)g.ni * g.no, true, psi_c, g.ng,
                            (long)g.no * g.ng, gam, cn, (long)g.ni * cn, gs);
    }
    if (e != hipSuccess) {
      what = "Gamma gemm";
      break;
    }
    {
      // Z^m of the representative transfers, compacted in place
      PhaseTimer pt(h, PH_KCORR, gs);
      e = launch_kcorr<TF>(g, tb, gam, gam, cn, pts, false, gs, pr.slot, c0);
    }
    if (e != hipSuccess) {
      what = "Z kcorr";
      break;
    }
    if (c0 == 0) {
      e = hipStreamWaitEvent(gs, h->chain_ev, 0);
      if (e != hipSuccess) {
        what = "chain wait";
        break;
      }
    }
    PhaseTimer pt(h, PH_SOLVE, gs);
    char* y = xi + (size_t)c0 * sizeof(cplx<TX>);
    e = zgemm_nn_grid<TF, TX>(g.ni, cn, g.ni, gr.nk, W, g.ni, nn, false, gam, cn,
                              (long)g.ni * cn, y, g.ng, (long)g.ni * g.ng, gs, h->tile_solve, true);
    if (e != hipSuccess) what = "solve gemm";
    if (!what && h->refine > 0) {
      // refinement in the factor form: R = Z - L Y (over Z), Y += W R (FP64 sums)
      e = zgemm_nn_grid_acc<TX, TF>(g.ni, cn, g.ni, gr.nk, Lf, g.ni, nn, y, g.ng,
                                    (long)g.ni * g.ng, gam, cn, (long)g.ni * cn, -1, gs);
      if (e == hipSuccess)
        e = zgemm_nn_grid_acc<TF, TX>(g.ni, cn, g.ni, gr.nk, W, g.ni, nn, gam, cn,
                                      (long)g.ni * cn, y, g.ng, (long)g.ni * g.ng, 1, gs);
      if (e != hipSuccess) what = "refinement";
    }
  }
  hipError_t ej = hipEventRecord(h->join_ev, gs);
  hipError_t ew = ej == hipSuccess ? hipStreamWaitEvent(st, h->join_ev, 0) : ej;
  if (what) return hip_check(h, e, what);
  if (ew != hipSuccess) return hip_check(h, ew, "join wait");
  // Vy (unphased, slice order) into V: the transform of each chunk of transfers
  // on the caller's stream into one of two buffers, its contraction on the
  // second stream; a buffer is refilled only after the contraction that read it
  double2* Vy = (double2*)V;
  const int per = L.pd.per;
  const size_t fb = (size_t)g.ni * g.ng * sizeof(cplx<TX>);  // functions of one slice
  {
    // timed per launch, so that serial timing gives each phase its own kernels
    int chunk = 0;
    for (int s0 = 0; s0 < gr.nk && !what; s0 += per, ++chunk) {
      const int cn = std::min(per, gr.nk - s0);
      const int b = chunk & 1;
      char* F = fbuf + (size_t)b * al(per * fb);
      if (chunk >= 2) {
        e = hipStreamWaitEvent(st, h->fb_ev[b], 0);
        if (e != hipSuccess) {
          what = "buffer wait";
          break;
        }
      }
      {
        PhaseTimer pt(h, PH_FFT, st);
        e = launch_fft3d<TX>(g, tb, xi + s0 * fb, F, (long)cn * g.ni, h->ncu, st);
      }
      if (e != hipSuccess) what = "fft";
      if (!what) e = hipEventRecord(h->fork_ev, st);
      if (!what && e == hipSuccess) e = hipStreamWaitEvent(gs, h->fork_ev, 0);
      if (!what && e != hipSuccess) what = "chunk fork";
      if (!what) {
        PhaseTimer pt(h, PH_COULOMB, gs);
        e = launch_coulomb<TX>(g, tb, F, pts, ws + L.cpart, L.nsplit, Vy + (long)s0 * nn, false, gs,
                               pr.rep + s0, pr.bar + s0, cn, true, cform);
      }
      if (!what && e != hipSuccess) what = "coulomb";
      if (!what) {
        e = hipEventRecord(h->fb_ev[b], gs);
        if (e != hipSuccess) what = "buffer event";
      }
      if (!what && h->timing && h->serial) {
        e = hipStreamWaitEvent(st, h->fb_ev[b], 0);
        if (e != hipSuccess) what = "serial timing";
      }
    }
  }
  ej = hipEventRecord(h->join_ev, gs);
  ew = ej == hipSuccess ? hipStreamWaitEvent(st, h->join_ev, 0) : ej;
  if (what) return hip_check(h, e, what);
  if (ew != hipSuccess) return hip_check(h, ew, "join wait");
  {
    PhaseTimer pt(h, PH_COULOMB, st);
    // V^m = W^H Vy W with T = Vy W in the S^+ scratch and the product in the
    // consumed partial sums, then the phases and the conjugate partners
    double2* T = Sp;
    double2* U = (double2*)(ws + L.cpart);
    e = gemm<double, double, double, double>(g.ni, g.ni, g.ni, gr.nk, A_N, Vy, g.ni, nn, B_N, W,
                                             g.ni, nn, T, g.ni, nn, 1.0, false, st);
    if (e == hipSuccess)
      e = gemm<double, double, double, double>(g.ni, g.ni, g.ni, gr.nk, A_C, W, g.ni, nn, B_N,
                                               T, g.ni, nn, U, g.ni, nn, 1.0, false, st);
    if (e == hipSuccess)
      e = launch_coulomb_phase(g, tb, pts, U, (double2*)V, pr.rep, pr.bar, pr.n, st);
  }
  if (e != hipSuccess) return hip_check(h, e, "coulomb");
  return EXX_OK;
}

// One fit shared by all transfers (the k-point fit of Sec. 2.2, Eq. 13, on
// occupied pairs): the least-squares problem over the pairs of every transfer
// has the metric S = sum_m S^m and the right-hand side Z = sum_m Z^m (each in
// the cell-periodic gauge of the per-transfer fit), so one Cholesky factor
// S = L L^H, W = L^{-1} and one grid-sized product Y = W Z serve every
// transfer, and one transform F_Y = FFT(Y). The transfer enters only through
// the kernel: Vy^m = (Omega/N_g^2) sum_g v^m(g) F_Y,P conj F_Y,Q, then
// V^m = W^H Vy^m W and the Bloch phases. The fit runs over chunks of grid
// columns (Gamma^n, Z^m, their sum over m and Y are column-local); the
// factorisation chain runs on the caller's stream beside it.
template <typename TF, typename TX>
exx_status fit_coulomb_shared(exx_context* h, const Geom& g, const Tables& tb, char* ws,
                              const Layout& L, const void* psi, const void* occ,
                              const int32_t* pts, void* V, int32_t* rank, hipStream_t st,
                              bool bf16 = false, int cform = COUL_F64) {
  double2* G = (double2*)(ws + L.G);
  double2* Lf = (double2*)(ws + L.Lf);
  double2* W = (double2*)(ws + L.W);
  double2* Sall = (double2*)(ws + L.S2);
  int32_t* keep = (int32_t*)(ws + L.keep);
  int32_t* rank_c = (int32_t*)(ws + L.rank2);
  void* gam = ws + L.grid;   // Gamma, then Z^m, then sum_m Z^m (slice 0), of one column chunk
  char* y = ws + L.grid2;    // Y = W Z, full grid
  char* F = ws + L.F;        // its transform
  Geom g1 = g;               // the one shared metric
  g1.nk = 1;
  const long nn = (long)g.ni * g.ni;
  const int cc = L.pd.cols;
  hipError_t e;
  hipStream_t ax = st;
  hipStream_t gs = h->aux;
  e = hipEventRecord(h->fork_ev, st);
  if (e != hipSuccess) return hip_check(h, e, "fork event");
  e = hipStreamWaitEvent(gs, h->fork_ev, 0);
  if (e != hipSuccess) return hip_check(h, e, "fork wait");
  const char* what = nullptr;
  {
    PhaseTimer pt(h, PH_GRAM, ax);
    e = gemm<double, double, double, double>(g.ni, g.ni, g.no, g.nk, A_N, occ, g.no,
                                             (long)g.ni * g.no, B_C, occ, g.no,
                                             (long)g.ni * g.no, G, g.ni, nn, 1.0, false, ax);
  }
  if (e != hipSuccess) what = "G gemm";
  if (!what) {
    // S^m of every transfer, then S = sum_m S^m into the factor buffer
    PhaseTimer pt(h, PH_METRIC, ax);
    e = launch_kcorr<double>(g, tb, G, Sall, g.ni, pts, true, ax);
    if (e == hipSuccess) e = launch_sum_slices<double>(Sall, Lf, nn, g.nk, nn, ax);
    if (e != hipSuccess) what = "S kcorr";
  }
  if (!what) {
    PhaseTimer pt(h, PH_CHOL, ax);
    QLabel lab;
    for (int k = 0; k < 64; ++k) lab.q[k] = 0;
    e = launch_chol_blocked(g1, Lf, keep, rank_c, (double*)(ws + L.tol), 1e-12, ax, stat_ptr(h),
                            strict_pd(h), &lab);
    if (e != hipSuccess) what = "cholesky";
  }
  if (!what) {
    PhaseTimer pt(h, PH_PINV, ax);
    e = launch_tri_inv_blocked(g1, Lf, keep, W, (double2*)(ws + L.Tinv), ax);
    if (e != hipSuccess) what = "triangular inverse";
  }
  if (!what) {
    e = launch_rank_broadcast(rank_c, rank, g.nk, ax);
    if (e != hipSuccess) what = "rank broadcast";
  }
  if (!what && h->refine > 0) {
    e = launch_zero_upper(Lf, g.ni, 1, ax);
    if (e != hipSuccess) what = "factor";
  }
  if (!what) {
    e = hipEventRecord(h->chain_ev, ax);
    if (e != hipSuccess) what = "chain event";
  }
  if (what) {
    (void)hipEventRecord(h->join_ev, gs);
    (void)hipStreamWaitEvent(st, h->join_ev, 0);
    return hip_check(h, e, what);
  }
  if (h->timing && h->serial) {
    e = hipStreamWaitEvent(gs, h->chain_ev, 0);
    if (e != hipSuccess) what = "serial timing";
  }
  for (int c0 = 0; c0 < g.ng && !what; c0 += cc) {
    const int cn = std::min(cc, g.ng - c0);
    const char* psi_c = (const char*)psi + (size_t)c0 * sizeof(cplx<TF>);
    {
      PhaseTimer pt(h, PH_GAMMA, gs);
      if (std::is_same<TF, double>::value)
        e = zgemm_nn_grid<double, double>(g.ni, cn, g.no, g.nk, occ, g.no, (long)g.ni * g.no, true,
                                          psi_c, g.ng, (long)g.no * g.ng, gam, cn, (long)g.ni * cn,
                                          gs, h->tile_gamma);
      else if (bf16)
        e = cgemm_nn_grid_bf16(g.ni, cn, g.no, g.nk, occ, g.no, (long)g.ni * g.no, psi_c, g.ng,
                               (long)g.no * g.ng, gam, cn, (long)g.ni * cn, gs);
      else
        e = cgemm_nn_grid32(g.ni, cn, g.no, g.nk, occ, g.no, (long)g.ni * g.no, true, psi_c, g.ng,
                            (long)g.no * g.ng, gam, cn, (long)g.ni * cn, gs);
    }
    if (e != hipSuccess) {
      what = "Gamma gemm";
      break;
    }
    {
      // Z^m of every transfer in place, then their sum into slice 0
      PhaseTimer pt(h, PH_KCORR, gs);
      e = launch_kcorr<TF>(g, tb, gam, gam, cn, pts, false, gs, nullptr, c0);
      if (e == hipSuccess)
        e = launch_sum_slices<TF>(gam, gam, (long)g.ni * cn, g.nk, (long)g.ni * cn, gs);
    }
    if (e != hipSuccess) {
      what = "Z kcorr";
      break;
    }
    if (c0 == 0) {
      e = hipStreamWaitEvent(gs, h->chain_ev, 0);
      if (e != hipSuccess) {
        what = "chain wait";
        break;
      }
    }
    PhaseTimer pt(h, PH_SOLVE, gs);
    char* yc = y + (size_t)c0 * sizeof(cplx<TX>);
    e = zgemm_nn_grid<TF, TX>(g.ni, cn, g.ni, 1, W, g.ni, nn, false, gam, cn, (long)g.ni * cn, yc,
                              g.ng, (long)g.ni * g.ng, gs, h->tile_solve, true);
    if (e != hipSuccess) what = "solve gemm";
    if (!what && h->refine > 0) {
      // refinement in the factor form: R = Z - L Y (over Z), Y += W R (FP64 sums)
      e = zgemm_nn_grid_acc<TX, TF>(g.ni, cn, g.ni, 1, Lf, g.ni, nn, yc, g.ng, (long)g.ni * g.ng,
                                    gam, cn, (long)g.ni * cn, -1, gs);
      if (e == hipSuccess)
        e = zgemm_nn_grid_acc<TF, TX>(g.ni, cn, g.ni, 1, W, g.ni, nn, gam, cn, (long)g.ni * cn, yc,
                                      g.ng, (long)g.ni * g.ng, 1, gs);
      if (e != hipSuccess) what = "refinement";
    }
  }
  hipError_t ej = hipEventRecord(h->join_ev, gs);
  hipError_t ew = ej == hipSuccess ? hipStreamWaitEvent(st, h->join_ev, 0) : ej;
  if (what) return hip_check(h, e, what);
  if (ew != hipSuccess) return hip_check(h, ew, "join wait");
  {
    PhaseTimer pt(h, PH_FFT, st);
    e = launch_fft3d<TX>(g, tb, y, F, g.ni, h->ncu, st);
  }
  if (e != hipSuccess) return hip_check(h, e, "fft");
  int rep[64], bar[64];
  for (int m = 0; m < 64; ++m) {
    rep[m] = m < g.nk ? m : 0;
    bar[m] = -1;
  }
  double2* Vy = (double2*)V;
  {
    PhaseTimer pt(h, PH_COULOMB, st);
    e = launch_coulomb<TX>(g, tb, F, pts, ws + L.cpart, L.nsplit, Vy, false, st, rep, bar, g.nk,
                           true, cform, true);
  }
  if (e != hipSuccess) return hip_check(h, e, "coulomb");
  {
    PhaseTimer pt(h, PH_COULOMB, st);
    // V^m = W^H Vy^m W (W shared: stride 0), then the phases
    double2* T = (double2*)(ws + L.Sp);
    double2* U = (double2*)(ws + L.cpart);
    e = gemm<double, double, double, double>(g.ni, g.ni, g.ni, g.nk, A_N, Vy, g.ni, nn, B_N, W,
                                             g.ni, 0, T, g.ni, nn, 1.0, false, st);
    if (e == hipSuccess)
      e = gemm<double, double, double, double>(g.ni, g.ni, g.ni, g.nk, A_C, W, g.ni, 0, B_N, T,
                                               g.ni, nn, U, g.ni, nn, 1.0, false, st);
    if (e == hipSuccess) e = launch_coulomb_phase(g, tb, pts, U, (double2*)V, rep, bar, g.nk, st);
  }
  if (e != hipSuccess) return hip_check(h, e, "Coulomb products");
  return EXX_OK;
}

// the fused fit + Coulomb of one build in precision prec
exx_status fit_coulomb(exx_context* h, const Geom& g, const Tables& tb, char* ws, const Layout& L,
                       exx_prec prec, const void* psi, const void* occ, const int32_t* pts,
                       int32_t* rank, hipStream_t st) {
  void* xi = ws + L.grid2;
  void* S = ws + L.S2;
  void* V = ws + L.V2;
  exx_status s;
  const Pairs pr = make_pairs(g);
  const int cf = coul_form(h, prec);
  if (cf < 0) return check_form(h, prec);
  const bool bf = prec == EXX_BF16;
  if (build_path(h, g) == PATH_SHARED) {
    if (prec == EXX_F64)
      return fit_coulomb_shared<double, double>(h, g, tb, ws, L, psi, occ, pts, V, rank, st);
    if (prec == EXX_MIXED)
      return fit_coulomb_shared<double, float>(h, g, tb, ws, L, psi, occ, pts, V, rank, st, false,
                                               cf);
    return fit_coulomb_shared<float, float>(h, g, tb, ws, L, psi, occ, pts, V, rank, st, bf, cf);
  }
  if (!kcorr_real(g) && pr.n < g.nk) {
    if (prec == EXX_F64)
      return fit_coulomb_pairs<double, double>(h, g, tb, ws, L, pr, psi, occ, pts, V, rank, st);
    if (prec == EXX_MIXED)
      return fit_coulomb_pairs<double, float>(h, g, tb, ws, L, pr, psi, occ, pts, V, rank, st,
                                              false, cf);
    return fit_coulomb_pairs<float, float>(h, g, tb, ws, L, pr, psi, occ, pts, V, rank, st, bf,
                                           cf);
  }
  if (kcorr_real(g)) {
    if (prec == EXX_F64)
      return fit_coulomb_real<double, double, double>(h, g, tb, ws, L, psi, occ, pts, S, V, rank,
                                                      st);
    if (prec == EXX_MIXED)
      return fit_coulomb_real<double, double, float>(h, g, tb, ws, L, psi, occ, pts, S, V, rank,
                                                     st, false, cf);
    return fit_coulomb_real<float, float, float>(h, g, tb, ws, L, psi, occ, pts, S, V, rank, st,
                                                 bf, cf);
  }
  if (prec == EXX_F64) {
    s = fit_impl<double, double>(h, g, tb, ws, L, psi, occ, pts, xi, S, rank, st);
    if (s == EXX_OK) s = coulomb_impl<double>(h, g, tb, ws, L, xi, pts, V, st);
  } else if (prec == EXX_MIXED) {
    s = fit_impl<double, float>(h, g, tb, ws, L, psi, occ, pts, xi, S, rank, st);
    if (s == EXX_OK) s = coulomb_impl<float>(h, g, tb, ws, L, xi, pts, V, st, cf);
  } else {
    s = fit_impl<float, float>(h, g, tb, ws, L, psi, occ, pts, xi, S, rank, st, bf);
    if (s == EXX_OK) s = coulomb_impl<float>(h, g, tb, ws, L, xi, pts, V, st, cf);
  }
  return s;
}

// scratch of the exchange contraction: G^n and Y^n [N_k][N_ISDF][N_ISDF],
// T [N_k][N_ISDF][n_ao], AH [N_k][n_ao][N_ISDF] (used when n_ao <= N_ISDF),
// epart [1024] doubles
struct KScratch {
  double2 *G, *Y, *T, *AH;
  double* epart;
};

KScratch kscratch(char* ws, const Layout& L) {
  return {(double2*)(ws + L.G), (double2*)(ws + L.Y), (double2*)(ws + L.T), (double2*)(ws + L.Sp),
          (double*)(ws + L.epart)};
}

// have_G: the point Gram G^n is already in ks.G (the fused build's fit formed it
// from the same occ and nothing since has written that region)
exx_status buildK_impl(exx_context* h, const Geom& g, const KScratch& ks, const void* ao,
                       const void* occ, const void* V, void* K, double* Ex, hipStream_t st,
                       bool have_G = false) {
  double2* G = ks.G;
  double2* Y = ks.Y;
  double2* T = ks.T;
  const long nn = (long)g.ni * g.ni;
  hipError_t e = hipSuccess;
  if (!have_G) {
    PhaseTimer pt(h, PH_GRAM, st);
    e = gemm<double, double, double, double>(g.ni, g.ni, g.no, g.nk, A_N, occ, g.no,
                                             (long)g.ni * g.no, B_C, occ, g.no, (long)g.ni * g.no,
                                             G, g.ni, nn, 1.0, false, st);
  }
  if (e != hipSuccess) return hip_check(h, e, "G gemm");
  // c1: Y^n = sum_m Vb^m o G^{n+m}
  {
    PhaseTimer pt(h, PH_KCONV, st);
    e = launch_kconv(g, (const double2*)V, G, Y, st);
  }
  if (e != hipSuccess) return hip_check(h, e, "k-convolution");
  // c2: K^n = (1/N_k) A^H (Y A)
  PhaseTimer ptk(h, PH_KMAT, st);
  const long na_i = (long)g.ni * g.nao;
  if (g.nao <= g.ni) {
    // both products on the FP64 matrix cores: T = Y A, then K = ((1/N_k) A^H) T
    // with A^H written once
    double2* AH = ks.AH;
    e = zgemm_nn_grid<double, double>(g.ni, g.nao, g.ni, g.nk, Y, g.ni, nn, false, ao, g.nao,
                                      na_i, T, g.nao, na_i, st, 22);
    if (e != hipSuccess) return hip_check(h, e, "Y A gemm");
    e = launch_conj_transpose((const double2*)ao, AH, g.ni, g.nao, g.nk, 1.0 / g.nk, st);
    if (e != hipSuccess) return hip_check(h, e, "A^H");
    e = zgemm_nn_grid<double, double>(g.nao, g.nao, g.ni, g.nk, AH, g.ni, na_i, false, T, g.nao,
                                      na_i, K, g.nao, (long)g.nao * g.nao, st, 22);
    if (e != hipSuccess) return hip_check(h, e, "A^H T gemm");
  } else {
    e = gemm<double, double, double, double>(g.ni, g.nao, g.ni, g.nk, A_N, Y, g.ni, nn, B_N, ao,
                                             g.nao, na_i, T, g.nao, na_i, 1.0, false, st);
    if (e != hipSuccess) return hip_check(h, e, "Y A gemm");
    e = gemm<double, double, double, double>(g.nao, g.nao, g.ni, g.nk, A_C, ao, g.nao, na_i, B_N,
                                             T, g.nao, na_i, K, g.nao, (long)g.nao * g.nao,
                                             1.0 / g.nk, false, st);
    if (e != hipSuccess) return hip_check(h, e, "A^H T gemm");
  }
  // c3: E_x
  PhaseTimer pte(h, PH_ENERGY, st);
  e = launch_energy(g, Y, G, ks.epart, Ex, st);
  if (e != hipSuccess) return hip_check(h, e, "energy");
  exx_status s = scan(h, K, 2L * g.nk * g.nao * g.nao, SITE_OUTPUT, st);
  if (s == EXX_OK) s = scan(h, Ex, 1, SITE_OUTPUT, st);
  return s;
}

exx_status setup(exx_context* h, const exx_cell* cell, exx_prec prec, int need, Geom* g,
                 Tables* tb, Layout* L, char** ws, hipStream_t st) {
  exx_status s = check_cell(h, cell, prec);
  if (s != EXX_OK) return s;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  if (!h->aux) {
    e = make_lane_streams(&h->aux, &h->fork_ev, &h->join_ev, &h->chain_ev, h->fb_ev);
    if (e != hipSuccess) return hip_check(h, e, "auxiliary stream");
  }
  e = fft_prepare(&h->ncu);
  if (e != hipSuccess) return hip_check(h, e, "FFT set-up");
  *g = make_geom(*cell);
  *L = layout(h, *g, prec, need);
  *ws = (char*)ws_get(h, L->total, &s);
  if (s != EXX_OK) return s;
  return get_tables(h, *g, tb, st);
}

}  // namespace
}  // namespace exx

using namespace exx;

extern "C" {

exx_status exx_create(exx_handle_t* h, int device) {
  if (!h) return EXX_ERR_ARG;
  *h = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return EXX_ERR_DEVICE;
  exx_context* c = new (std::nothrow) exx_context();
  if (!c) return EXX_ERR_NOMEM;
  c->device = device;
  // the device status word, cleared once here and after every exx_get_status
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = noalloc_setup(device);
  if (e == hipSuccess) e = hipMalloc((void**)&c->dstat, 4 * sizeof(int32_t));
  if (e == hipSuccess) e = launch_status_reset(c->dstat, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    if (c->dstat) (void)hipFree(c->dstat);
    delete c;
    return EXX_ERR_DEVICE;
  }
  // wave tiles of the grid GEMMs (16x16 blocks); EXX_TILE_GAMMA / EXX_TILE_SOLVE override
  if (const char* v = getenv("EXX_TILE_GAMMA")) c->tile_gamma = atoi(v);
  if (const char* v = getenv("EXX_TILE_SOLVE")) c->tile_solve = atoi(v);
  // grid-column chunk of the paired path's fit, in MiB of Gamma (experiments)
  if (const char* v = getenv("EXX_FIT_CHUNK_MB"))
    if (atol(v) > 0) c->fit_chunk_bytes = (size_t)atol(v) << 20;
  *h = c;
  return EXX_OK;
}

exx_status exx_destroy(exx_handle_t h) {
  if (!h) return EXX_ERR_ARG;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  if (h->ws.base) (void)hipFree(h->ws.base);
  for (auto& te : h->tabs) (void)hipFree(te.buf);
  for (auto& ge : h->graphs) (void)hipGraphExecDestroy(ge.exec);
  if (h->small) (void)hipFree(h->small);
  if (h->dstat) (void)hipFree(h->dstat);
  for (auto& r : h->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : h->pool) (void)hipEventDestroy(e);
  if (h->chain_ev) (void)hipEventDestroy(h->chain_ev);
  for (auto ev : h->fb_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  for (size_t l = 1; l < h->lanes.size(); ++l) {
    auto& ln = h->lanes[l];
    if (ln.ws) (void)hipFree(ln.ws);
    for (hipEvent_t ev : {ln.fork_ev, ln.join_ev, ln.chain_ev, ln.done_ev, ln.fb_ev[0], ln.fb_ev[1]})
      if (ev) (void)hipEventDestroy(ev);
    if (ln.aux) (void)hipStreamDestroy(ln.aux);
    if (ln.st) (void)hipStreamDestroy(ln.st);
  }
  if (h->batch_ev) (void)hipEventDestroy(h->batch_ev);
  delete h;
  return EXX_OK;
}

const char* exx_last_error(exx_handle_t h) { return h ? h->err.c_str() : "null handle"; }

exx_status exx_scratch_bytes(exx_handle_t h, size_t* bytes) {
  if (!h || !bytes) return EXX_ERR_ARG;
  size_t tb = 0;
  for (auto& te : h->tabs) tb += te.bytes;
  size_t lb = 0;
  for (size_t l = 1; l < h->lanes.size(); ++l) lb += h->lanes[l].cap;
  *bytes = h->ws.cap + tb + h->small_cap + lb;
  return EXX_OK;
}

exx_status exx_isdf_fit(exx_handle_t h, const exx_cell* cell, exx_prec prec, const void* psi_grid,
                        const void* occ_pts, const int32_t* pts, void* xi, void* S, int32_t* rank,
                        hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!psi_grid || !occ_pts || !pts || !xi || !S || !rank)
    return fail(h, EXX_ERR_ARG, "exx_isdf_fit: null array argument");
  Geom g;
  Tables tb;
  Layout L;
  char* ws;
  exx_status s = setup(h, cell, prec, NEED_FIT, &g, &tb, &L, &ws, stream);
  if (s != EXX_OK) return s;
  s = scan(h, occ_pts, 2L * g.nk * g.ni * g.no, SITE_OCC, stream);
  if (s != EXX_OK) return s;
  if (prec == EXX_F64)
    s = fit_impl<double, double>(h, g, tb, ws, L, psi_grid, occ_pts, pts, xi, S, rank, stream);
  else if (prec == EXX_MIXED)
    s = fit_impl<double, float>(h, g, tb, ws, L, psi_grid, occ_pts, pts, xi, S, rank, stream);
  else
    s = fit_impl<float, float>(h, g, tb, ws, L, psi_grid, occ_pts, pts, xi, S, rank, stream,
                               prec == EXX_BF16);
  return s == EXX_OK ? finish(h, stream) : s;
}

exx_status exx_coulomb_V(exx_handle_t h, const exx_cell* cell, exx_prec prec, const void* xi,
                         const int32_t* pts, void* V, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!xi || !pts || !V) return fail(h, EXX_ERR_ARG, "exx_coulomb_V: null array argument");
  Geom g;
  Tables tb;
  Layout L;
  char* ws;
  if (cell && check_form(h, prec) != EXX_OK) return EXX_ERR_UNSUPPORTED;
  exx_status s = setup(h, cell, prec, NEED_COULOMB, &g, &tb, &L, &ws, stream);
  if (s != EXX_OK) return s;
  if (prec == EXX_F64)
    s = coulomb_impl<double>(h, g, tb, ws, L, xi, pts, V, stream);
  else
    s = coulomb_impl<float>(h, g, tb, ws, L, xi, pts, V, stream, coul_form(h, prec));
  if (s == EXX_OK) s = scan(h, V, 2L * g.nk * g.ni * g.ni, SITE_COULOMB, stream);
  return s == EXX_OK ? finish(h, stream) : s;
}

exx_status exx_build_K(exx_handle_t h, const exx_cell* cell, exx_prec prec, const void* ao_pts,
                       const void* occ_pts, const void* V, void* K, double* Ex,
                       hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!ao_pts || !occ_pts || !V || !K || !Ex)
    return fail(h, EXX_ERR_ARG, "exx_build_K: null array argument");
  Geom g;
  Tables tb;
  Layout L;
  char* ws;
  exx_status s = setup(h, cell, prec, NEED_K, &g, &tb, &L, &ws, stream);
  if (s != EXX_OK) return s;
  s = scan(h, occ_pts, 2L * g.nk * g.ni * g.no, SITE_OCC, stream);
  if (s == EXX_OK) s = scan(h, ao_pts, 2L * g.nk * g.ni * g.nao, SITE_AO, stream);
  if (s == EXX_OK) s = scan(h, V, 2L * g.nk * g.ni * g.ni, SITE_COULOMB, stream);
  if (s == EXX_OK) s = buildK_impl(h, g, kscratch(ws, L), ao_pts, occ_pts, V, K, Ex, stream);
  return s == EXX_OK ? finish(h, stream) : s;
}

exx_status exx_build(exx_handle_t h, const exx_cell* cell, exx_prec prec, const void* psi_grid,
                     const void* occ_pts, const void* ao_pts, const int32_t* pts, void* K,
                     double* Ex, int32_t* rank, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!psi_grid || !occ_pts || !ao_pts || !pts || !K || !Ex || !rank)
    return fail(h, EXX_ERR_ARG, "exx_build: null array argument");
  if (cell && check_form(h, prec) != EXX_OK) return EXX_ERR_UNSUPPORTED;
  Geom g;
  Tables tb;
  Layout L;
  char* ws;
  exx_status s = setup(h, cell, prec, NEED_BUILD, &g, &tb, &L, &ws, stream);
  if (s != EXX_OK) return s;
  s = scan(h, occ_pts, 2L * g.nk * g.ni * g.no, SITE_OCC, stream);
  if (s == EXX_OK) s = scan(h, ao_pts, 2L * g.nk * g.ni * g.nao, SITE_AO, stream);
  if (s == EXX_OK) s = fit_coulomb(h, g, tb, ws, L, prec, psi_grid, occ_pts, pts, rank, stream);
  if (s == EXX_OK)
    s = buildK_impl(h, g, kscratch(ws, L), ao_pts, occ_pts, ws + L.V2, K, Ex, stream, true);
  return s == EXX_OK ? finish(h, stream) : s;
}

}  // extern "C"

namespace exx {
namespace {

// The build followed by the potentials of the fitted functions, shared by the
// gradient and the robust-fit K. The fit writes Z^m to a buffer of its own so
// that Gamma^n survives it; on meshes with conjugate pairs it fits one transfer
// of each pair (the slices of xi, F and Pw then follow pairs order). On return *pw holds
// Pw^m(P, r) = e^{i q_m.(r_P - r)} conj Phi^m_P(r) [N_k][N_ISDF][N_g] (c64 when
// *pw_f32), *gam holds Gamma^n [N_k][N_ISDF][N_g] (c128), *cz is a free
// grid-sized c128 buffer, G = G^n, V2 = Vb^m.
//   EXX_F64: Gamma^n in grid; Z^m and then xi in g3 (grid2 the solve's
//     scratch); the transforms to grid2, the potentials to g3; cz = grid2.
//   EXX_MIXED: as the MIXED builds (Gamma^n, Z^m and the solve in FP64, xi
//     stored as c64): Gamma^n in grid, Z^m in g3, xi (c64) in grid2; the
//     transforms (c64) to g3, the potentials (c64, FP64 arithmetic) to grid2;
//     cz = g3.
exx_status build_with_potentials(exx_context* h, const Geom& g, const Tables& tb, char* ws,
                                 const Layout& L, exx_prec prec, const void* psi_grid,
                                 const void* occ_pts, const void* ao_pts, const int32_t* pts,
                                 void* K, double* Ex, int32_t* rank, hipStream_t stream,
                                 void** pw, void** gam, bool* pw_f32, void** cz, int* src,
                                 int* cj) {
  exx_status s = scan(h, occ_pts, 2L * g.nk * g.ni * g.no, SITE_OCC, stream);
  if (s == EXX_OK) s = scan(h, ao_pts, 2L * g.nk * g.ni * g.nao, SITE_AO, stream);
  if (s != EXX_OK) return s;
  const bool f32 = prec == EXX_MIXED;
  // On meshes with conjugate pairs the fit, the transforms and the potentials
  // cover one transfer of each pair (Pw^{-m} = conj Pw^m): slice s holds
  // transfer prs.rep[s]; src/cj tell the correlation where each transfer is.
  const Pairs prs = make_pairs(g);
  const Pairs* pp = prs.n < g.nk ? &prs : nullptr;
  const int ns = pp ? pp->n : g.nk;
  Geom gs = g;
  gs.nk = ns;
  for (int m = 0; m < 64; ++m) {
    src[m] = m;
    cj[m] = 0;
  }
  if (pp) {
    for (int m = 0; m < g.nk; ++m) {
      if (prs.slot[m] >= 0) {
        src[m] = prs.slot[m];
      } else {
        for (int k = 0; k < prs.n; ++k)
          if (prs.bar[k] == m) src[m] = k;
        cj[m] = 1;
      }
    }
  }
  // the fit (S into S2), V^m (Bloch gauge, into V2), K and E_x with the fit's G^n
  void* gm = ws + L.grid;  // Gamma^n, kept by the fit
  void* xi;                // the fitted functions, then the potentials
  void* F;                 // their transforms, then conj(v F), then free
  if (!f32) {
    xi = ws + L.g3;
    F = ws + L.grid2;
    s = fit_impl<double, double>(h, g, tb, ws, L, psi_grid, occ_pts, pts, ws + L.grid2,
                                 ws + L.S2, rank, stream, false, true, ws + L.g3, pp);
    if (s == EXX_OK)
      s = coulomb_impl<double>(h, g, tb, ws, L, xi, pts, ws + L.V2, stream, COUL_F64, F, pp);
  } else {
    xi = ws + L.grid2;
    F = ws + L.g3;
    s = fit_impl<double, float>(h, g, tb, ws, L, psi_grid, occ_pts, pts, xi, ws + L.S2, rank,
                                stream, false, false, ws + L.g3, pp);
    if (s == EXX_OK)
      s = coulomb_impl<float>(h, g, tb, ws, L, xi, pts, ws + L.V2, stream, coul_form(h, prec), F,
                              pp);
  }
  void* pot = xi;  // xi is no longer needed once the transforms exist
  if (s == EXX_OK)
    s = buildK_impl(h, g, kscratch(ws, L), ao_pts, occ_pts, ws + L.V2, K, Ex, stream, true);
  if (s != EXX_OK) return s;
  double* vt = (double*)(ws + L.gvt);
  hipError_t e = launch_kernel_table(g, vt, stream, pp ? pp->rep : nullptr, ns);
  if (e != hipSuccess) return hip_check(h, e, "kernel table");
  // conj Phi^m scaled by N_g^2 / Omega: the forward transform of conj(v^m F^m)
  e = launch_kernel_scale_conj(gs, F, vt, stream, f32);
  if (e == hipSuccess) {
    if (f32)
      e = launch_fft3d<float>(g, tb, F, pot, (long)ns * g.ni, h->ncu, stream);
    else
      e = launch_fft3d<double>(g, tb, F, pot, (long)ns * g.ni, h->ncu, stream);
  }
  if (e != hipSuccess) return hip_check(h, e, "potentials");
  const double omega = (double)g.L[0] * g.L[1] * g.L[2];
  e = launch_potential_phase(g, tb, pot, pts, omega / ((double)g.ng * g.ng), stream, f32,
                             pp ? pp->rep : nullptr, ns);
  if (e != hipSuccess) return hip_check(h, e, "potential phase");
  *pw = pot;
  *gam = gm;
  *pw_f32 = f32;
  *cz = F;
  return EXX_OK;
}

exx_status potential_args(exx_context* h, const exx_cell* cell, exx_prec prec, const char* name,
                          bool ok) {
  if (!ok) return fail(h, EXX_ERR_ARG, std::string(name) + ": null array argument");
  if (cell && prec != EXX_F64 && prec != EXX_MIXED)
    return fail(h, EXX_ERR_UNSUPPORTED,
                std::string(name) + ": FP64 or MIXED only (EXX_F64, EXX_MIXED)");
  if (cell && prec == EXX_MIXED && check_form(h, prec) != EXX_OK) return EXX_ERR_UNSUPPORTED;
  return EXX_OK;
}

}  // namespace
}  // namespace exx

extern "C" {

exx_status exx_exchange_gradient(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                                 const void* psi_grid, const void* occ_pts, const void* ao_pts,
                                 const void* ao_grid, const int32_t* pts, void* K, void* Kgrad,
                                 double* Ex, int32_t* rank, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  exx_status s = potential_args(h, cell, prec, "exx_exchange_gradient",
                                psi_grid && occ_pts && ao_pts && ao_grid && pts && K && Kgrad &&
                                    Ex && rank);
  if (s != EXX_OK) return s;
  Geom g;
  Tables tb;
  Layout L;
  char* ws;
  s = setup(h, cell, prec, NEED_GRAD, &g, &tb, &L, &ws, stream);
  void *pw = nullptr, *gam = nullptr, *cz = nullptr;
  bool pw_f32 = false;
  int src[64], cj[64];
  if (s == EXX_OK)
    s = build_with_potentials(h, g, tb, ws, L, prec, psi_grid, occ_pts, ao_pts, pts, K, Ex, rank,
                              stream, &pw, &gam, &pw_f32, &cz, src, cj);
  if (s != EXX_OK) return s;
  const long nn = (long)g.ni * g.ni, na_i = (long)g.ni * g.nao, nig = (long)g.ni * g.ng;
  // CZ^n over the grid and CS^n over the points (U^m = conj Vb^m: Vb^m is Hermitian)
  hipError_t e = launch_grad_xcorr(g, pw, false, gam, cz, nig, stream, false, pw_f32, src, cj);
  if (e == hipSuccess)
    e = launch_grad_xcorr(g, ws + L.V2, true, ws + L.G, ws + L.gCS, nn, stream);
  if (e != hipSuccess) return hip_check(h, e, "k-correlation of the derivative");
  // T = CS X^T - 2 CZ phi^H [N_ISDF][n_ao] (X_{mu P} = conj phi_mu(r_P): the conjugated
  // ao_pts, transposed), then conj A = (1/N_k^2) X conj T
  double2* T = (double2*)(ws + L.gT);
  e = zgemm_splitk(g.ni, g.nao, g.ng, g.nk, A_N, cz, g.ng, nig, B_C, ao_grid, g.ng,
                   (long)g.nao * g.ng, T, g.nao, na_i, -2.0, false, ws + L.gP, stream);
  if (e == hipSuccess)
    e = gemm<double, double, double, double>(g.ni, g.nao, g.ni, g.nk, A_N, ws + L.gCS, g.ni, nn,
                                             B_R, ao_pts, g.nao, na_i, T, g.nao, na_i, 1.0, true,
                                             stream);
  if (e == hipSuccess)
    e = gemm<double, double, double, double>(g.nao, g.nao, g.ni, g.nk, A_C, ao_pts, g.nao, na_i,
                                             B_R, T, g.nao, na_i, ws + L.gA, g.nao,
                                             (long)g.nao * g.nao, 1.0 / ((double)g.nk * g.nk),
                                             false, stream);
  if (e != hipSuccess) return hip_check(h, e, "AO contraction of the derivative");
  e = launch_grad_assemble(g, ws + L.gA, Kgrad, stream);
  if (e != hipSuccess) return hip_check(h, e, "gradient assembly");
  s = scan(h, Kgrad, 2L * g.nk * g.nao * g.nao, SITE_OUTPUT, stream);
  return s == EXX_OK ? finish(h, stream) : s;
}

exx_status exx_build_robust(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                            const void* psi_grid, const void* occ_pts, const void* ao_pts,
                            const void* ao_grid, const int32_t* pts, void* K, double* Ex,
                            int32_t* rank, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  exx_status s = potential_args(h, cell, prec, "exx_build_robust",
                                psi_grid && occ_pts && ao_pts && ao_grid && pts && K && Ex && rank);
  if (s != EXX_OK) return s;
  Geom g;
  Tables tb;
  Layout L;
  char* ws;
  s = setup(h, cell, prec, NEED_GRAD, &g, &tb, &L, &ws, stream);
  void *pw = nullptr, *gam = nullptr, *cz = nullptr;
  bool pw_f32 = false;
  int src[64], cj[64];
  if (s == EXX_OK)
    s = build_with_potentials(h, g, tb, ws, L, prec, psi_grid, occ_pts, ao_pts, pts, K, Ex, rank,
                              stream, &pw, &gam, &pw_f32, &cz, src, cj);
  if (s != EXX_OK) return s;
  const long na_i = (long)g.ni * g.nao, nig = (long)g.ni * g.ng;
  // R^n = sum_m Pw^m o conj Gamma^{n+m}
  hipError_t e = launch_grad_xcorr(g, pw, false, gam, cz, nig, stream, true, pw_f32, src, cj);
  if (e != hipSuccess) return hip_check(h, e, "k-correlation of the one-sided term");
  // T = R conj(phi)^T [N_ISDF][n_ao], then conj of the one-sided term
  // (1/N_k) T^T A = conj((1/N_k) T^H conj A)
  double2* T = (double2*)(ws + L.gT);
  e = zgemm_splitk(g.ni, g.nao, g.ng, g.nk, A_N, cz, g.ng, nig, B_C, ao_grid, g.ng,
                   (long)g.nao * g.ng, T, g.nao, na_i, 1.0, false, ws + L.gP, stream);
  if (e == hipSuccess)
    e = gemm<double, double, double, double>(g.nao, g.nao, g.ni, g.nk, A_C, T, g.nao, na_i, B_R,
                                             ao_pts, g.nao, na_i, ws + L.gA, g.nao,
                                             (long)g.nao * g.nao, 1.0 / g.nk, false, stream);
  if (e != hipSuccess) return hip_check(h, e, "AO contraction of the one-sided term");
  // K <- K_cross + K_cross^H - K_fit
  e = launch_robust_assemble(g, ws + L.gA, K, stream);
  if (e != hipSuccess) return hip_check(h, e, "robust assembly");
  s = scan(h, K, 2L * g.nk * g.nao * g.nao, SITE_OUTPUT, stream);
  return s == EXX_OK ? finish(h, stream) : s;
}

exx_status exx_workspace_size(exx_handle_t h, const exx_cell* cell, exx_prec prec, int32_t call,
                              size_t* bytes) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!bytes) return fail(h, EXX_ERR_ARG, "exx_workspace_size: bytes is NULL");
  exx_status s = check_cell(h, cell, call == EXX_CALL_BUILD ? prec : EXX_F64);
  if (s != EXX_OK) return s;
  const Geom g = make_geom(*cell);
  if (call == EXX_CALL_BUILD) {
    size_t b = layout(h, g, prec, NEED_BUILD).total;
    b = std::max(b, layout(h, g, prec, NEED_FIT | NEED_COULOMB | NEED_K).total);
    *bytes = b;
    return EXX_OK;
  }
  if (call == EXX_CALL_GRADIENT) {  // also exx_build_robust
    *bytes = layout(h, g, prec == EXX_MIXED ? EXX_MIXED : EXX_F64, NEED_GRAD).total;
    return EXX_OK;
  }
  if (call == EXX_CALL_SELECT) {
    *bytes = select_scratch_bytes(g);
    return EXX_OK;
  }
  if (call == EXX_CALL_SELECT_MLP) {
    size_t inner = mlp_feature_scratch_bytes(g);
    inner = std::max(inner, mlp_nms_scratch_bytes(g));
    inner = std::max(inner, mlp_probe_scratch_bytes(g, 8192));
    inner = std::max(inner, select_scratch_bytes(g));
    *bytes = al(sizeof(float) * 3 * (size_t)g.ng) + al(sizeof(float) * (size_t)g.ng) +
             al(sizeof(double)) + inner;
    return EXX_OK;
  }
  return fail(h, EXX_ERR_ARG, "exx_workspace_size: unknown call");
}

exx_status exx_set_workspace(exx_handle_t h, void* dev, size_t bytes) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (dev && ((uintptr_t)dev % 256 != 0))
    return fail(h, EXX_ERR_ARG, "exx_set_workspace: the workspace must be 256-byte aligned");
  if (dev && bytes == 0) return fail(h, EXX_ERR_ARG, "exx_set_workspace: zero bytes");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  // work queued on the old scratch must finish before it is released or replaced
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_check(h, e, "hipDeviceSynchronize");
  if (h->ws.base) {
    (void)hipFree(h->ws.base);
    h->ws.base = nullptr;
    h->ws.cap = 0;
  }
  h->user_ws = (char*)dev;
  h->user_ws_bytes = dev ? bytes : 0;
  return EXX_OK;
}

exx_status exx_set_checks(exx_handle_t h, int32_t flags) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (flags & ~(EXX_CHECK_FINITE | EXX_STRICT_PD | EXX_CHECK_SYNC))
    return fail(h, EXX_ERR_ARG, "exx_set_checks: unknown flag");
  h->checks = flags;
  return EXX_OK;
}

exx_status exx_get_status(exx_handle_t h, hipStream_t stream, int32_t* info) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  return read_status(h, stream, info);
}

exx_status exx_build_K_noalloc(exx_handle_t h, const exx_cell* cell, exx_prec prec,
                               const void* ao_pts, const void* occ_pts, const void* V, void* K,
                               double* Ex, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!ao_pts || !occ_pts || !V || !K || !Ex)
    return fail(h, EXX_ERR_ARG, "exx_build_K_noalloc: null array argument");
  exx_status s = check_cell(h, cell, prec);
  if (s != EXX_OK) return s;
  const Geom g = make_geom(*cell);
  // G, Y [N_k][N_ISDF][N_ISDF], T [N_k][N_ISDF][n_ao], A^H (n_ao <= N_ISDF), partial sums
  const size_t mat = al(sizeof(double2) * (size_t)g.nk * g.ni * g.ni);
  const size_t tb = al(sizeof(double2) * (size_t)g.nk * g.ni * g.nao);
  const size_t need = 2 * mat + tb + (g.nao <= g.ni ? tb : 0) + al(sizeof(double) * 1024);
  if (need > (size_t)EXX_NOALLOC_MAX_BYTES)
    return fail(h, EXX_ERR_SHAPE, "exx_build_K_noalloc: this cell needs " + std::to_string(need) +
                                      " bytes of scratch; the allocation-free scratch holds " +
                                      std::to_string((size_t)EXX_NOALLOC_MAX_BYTES));
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  char* base = noalloc_base(h->device);
  if (!base) return fail(h, EXX_ERR_DEVICE, "exx_build_K_noalloc: scratch address not set up");
  KScratch ks;
  ks.G = (double2*)base;
  ks.Y = (double2*)(base + mat);
  ks.T = (double2*)(base + 2 * mat);
  ks.AH = g.nao <= g.ni ? (double2*)(base + 2 * mat + tb) : nullptr;
  ks.epart = (double*)(base + 2 * mat + tb + (g.nao <= g.ni ? tb : 0));
  // no phase events here: taking one may create it
  const bool timing = h->timing;
  h->timing = false;
  s = scan(h, occ_pts, 2L * g.nk * g.ni * g.no, SITE_OCC, stream);
  if (s == EXX_OK) s = scan(h, ao_pts, 2L * g.nk * g.ni * g.nao, SITE_AO, stream);
  if (s == EXX_OK) s = scan(h, V, 2L * g.nk * g.ni * g.ni, SITE_COULOMB, stream);
  if (s == EXX_OK) s = buildK_impl(h, g, ks, ao_pts, occ_pts, V, K, Ex, stream);
  h->timing = timing;
  return s == EXX_OK ? finish(h, stream) : s;
}

exx_status exx_set_refinement(exx_handle_t h, int32_t steps) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (steps < 0 || steps > 1) return fail(h, EXX_ERR_ARG, "exx_set_refinement: steps must be 0 or 1");
  h->refine = steps;
  return EXX_OK;
}

exx_status exx_set_fit(exx_handle_t h, int32_t mode) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (mode != EXX_FIT_PER_Q && mode != EXX_FIT_SHARED)
    return fail(h, EXX_ERR_ARG, "exx_set_fit: unknown mode");
  h->fit_mode = mode;
  return EXX_OK;
}

exx_status exx_set_contraction(exx_handle_t h, int32_t form) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (form < EXX_CONTRACT_AUTO || form > EXX_CONTRACT_BF16X3)
    return fail(h, EXX_ERR_ARG, "exx_set_contraction: unknown form");
  h->contract = form;
  return EXX_OK;
}

exx_status exx_set_timing(exx_handle_t h, int enable) {
  if (!h) return EXX_ERR_ARG;
  (void)hipSetDevice(h->device);
  for (auto& r : h->recs) {
    (void)hipEventSynchronize(r.b);
    h->pool.push_back(r.a);
    h->pool.push_back(r.b);
  }
  h->recs.clear();
  h->timing = enable != 0;
  h->serial = enable == 2;
  return EXX_OK;
}

exx_status exx_phase_times(exx_handle_t h, double* ms, int32_t* calls, int32_t n) {
  if (!h || !ms || !calls || n < 0) return EXX_ERR_ARG;
  (void)hipSetDevice(h->device);
  for (int i = 0; i < n; ++i) {
    ms[i] = 0.0;
    calls[i] = 0;
  }
  exx_status st = EXX_OK;
  for (auto& r : h->recs) {
    hipError_t e = hipEventSynchronize(r.b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) st = hip_check(h, e, "phase timing");
    if (r.phase < n) {
      ms[r.phase] += (double)t;
      calls[r.phase] += 1;
    }
    h->pool.push_back(r.a);
    h->pool.push_back(r.b);
  }
  h->recs.clear();
  return st;
}

}  // extern "C"

namespace {

exx_status build_one(exx_context* h, const Geom& g, const Tables& tb, char* ws, const Layout& L,
                     exx_prec prec, const exx_batch_item& it, hipStream_t st) {
  exx_status s = scan(h, it.occ_pts, 2L * g.nk * g.ni * g.no, SITE_OCC, st);
  if (s == EXX_OK) s = scan(h, it.ao_pts, 2L * g.nk * g.ni * g.nao, SITE_AO, st);
  if (s == EXX_OK)
    s = fit_coulomb(h, g, tb, ws, L, prec, it.psi_grid, it.occ_pts, it.pts, it.rank, st);
  if (s != EXX_OK) return s;
  return buildK_impl(h, g, kscratch(ws, L), it.ao_pts, it.occ_pts, ws + L.V2, it.K, it.Ex, st,
                     true);
}

void tune_key(const Geom& g, exx_prec prec, long* key) {
  key[0] = g.ni;
  key[1] = g.ng;
  key[2] = g.no;
  key[3] = g.nk;
  key[4] = (long)prec;
}

const exx_context::Tune* find_tune(const exx_context* h, const long* key) {
  for (const auto& t : h->tuned) {
    bool same = true;
    for (int i = 0; i < 5; ++i) same = same && t.key[i] == key[i];
    if (same) return &t;
  }
  return nullptr;
}

// time the candidate wave tiles of the Gamma and solve GEMMs on one real build
exx_status autotune(exx_context* h, const Geom& g, const Tables& tb, char* ws, const Layout& L,
                    exx_prec prec, const exx_batch_item& it, hipStream_t st) {
  long key[5];
  tune_key(g, prec, key);
  if (find_tune(h, key)) return EXX_OK;
  const int cand[3] = {22, 24, 42};
  double best_g = 1e300, best_s = 1e300;
  int tg = h->tile_gamma, ts = h->tile_solve;
  const int sg = h->tile_gamma, ss = h->tile_solve;
  const bool timing = h->timing;
  for (int c : cand) {
    h->tile_gamma = h->tile_solve = c;
    exx_status s = exx_set_timing(h, 1);
    if (s != EXX_OK) break;
    s = build_one(h, g, tb, ws, L, prec, it, st);
    double ms[EXX_NPHASE];
    int32_t calls[EXX_NPHASE];
    exx_status s2 = exx_phase_times(h, ms, calls, EXX_NPHASE);
    if (s != EXX_OK || s2 != EXX_OK) {
      h->tile_gamma = sg;
      h->tile_solve = ss;
      exx_set_timing(h, timing ? 1 : 0);
      return s != EXX_OK ? s : s2;
    }
    if (ms[PH_GAMMA] < best_g) {
      best_g = ms[PH_GAMMA];
      tg = c;
    }
    if (ms[PH_SOLVE] < best_s) {
      best_s = ms[PH_SOLVE];
      ts = c;
    }
  }
  exx_set_timing(h, timing ? 1 : 0);
  h->tile_gamma = sg;
  h->tile_solve = ss;
  exx_context::Tune t;
  for (int i = 0; i < 5; ++i) t.key[i] = key[i];
  t.gamma = tg;
  t.solve = ts;
  h->tuned.push_back(t);
  return EXX_OK;
}

}  // namespace

namespace {

// cost of one build in multiply-adds of its grid-sized steps (for lane balance)
double build_cost(const Geom& g) {
  return (double)g.nk * g.ni * (double)g.ng * (g.no + 2.0 * g.ni);
}

// swap the handle's second stream and events with those of a lane (the host
// enqueues the lanes one after another, so the build code sees one set)
void swap_lane(exx_context* h, exx_context::Lane& l) {
  std::swap(h->aux, l.aux);
  std::swap(h->fork_ev, l.fork_ev);
  std::swap(h->join_ev, l.join_ev);
  std::swap(h->chain_ev, l.chain_ev);
  std::swap(h->fb_ev[0], l.fb_ev[0]);
  std::swap(h->fb_ev[1], l.fb_ev[1]);
}

// Split the items over up to 4 lanes, longest first onto the least loaded lane,
// using the most lanes whose scratch (each lane sized for its largest item) fits
// in `budget` bytes. Returns the lane of every item.
std::vector<int> plan_lanes(const std::vector<Geom>& geo, const std::vector<Layout>& lay,
                            size_t budget, int max_lanes, std::vector<size_t>* need) {
  const int n = (int)geo.size();
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return build_cost(geo[a]) > build_cost(geo[b]); });
  for (int L = std::min(max_lanes, n); L >= 1; --L) {
    std::vector<double> load(L, 0.0);
    std::vector<size_t> nd(L, 0);
    std::vector<int> lane(n, 0);
    for (int i : order) {
      int best = 0;
      for (int l = 1; l < L; ++l)
        if (load[l] < load[best]) best = l;
      lane[i] = best;
      load[best] += build_cost(geo[i]);
      nd[best] = std::max(nd[best], lay[i].total);
    }
    size_t tot = 0;
    for (size_t x : nd) tot += x;
    if (L == 1 || tot <= budget) {
      *need = nd;
      return lane;
    }
  }
  return std::vector<int>(n, 0);
}

exx_status ensure_lanes(exx_context* h, int L, const std::vector<size_t>& need) {
  if ((int)h->lanes.size() < L) h->lanes.resize(L);
  for (int l = 1; l < L; ++l) {
    exx_context::Lane& ln = h->lanes[l];
    hipError_t e = hipSuccess;
    if (!ln.st) {
      e = hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking);
      if (e == hipSuccess)
        e = make_lane_streams(&ln.aux, &ln.fork_ev, &ln.join_ev, &ln.chain_ev, ln.fb_ev);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ln.done_ev, hipEventDisableTiming);
      if (e != hipSuccess) return hip_check(h, e, "lane streams");
    }
    if (ln.cap < need[l]) {
      if (ln.ws) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_check(h, e, "hipDeviceSynchronize");
        (void)hipFree(ln.ws);
        ln.ws = nullptr;
        ln.cap = 0;
      }
      void* p = nullptr;
      e = hipMalloc(&p, need[l]);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, EXX_ERR_NOMEM, "lane scratch of " + std::to_string(need[l]) + " bytes");
      }
      ln.ws = (char*)p;
      ln.cap = need[l];
    }
  }
  if (!h->batch_ev) {
    hipError_t e = hipEventCreateWithFlags(&h->batch_ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_check(h, e, "batch event");
  }
  return EXX_OK;
}

}  // namespace

extern "C" exx_status exx_build_batched(exx_handle_t h, int32_t n, const exx_batch_item* items,
                                        exx_prec prec, int32_t flags, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (n < 0 || (n > 0 && !items)) return fail(h, EXX_ERR_ARG, "exx_build_batched: bad item list");
  if (flags & ~(EXX_BATCH_GRAPH | EXX_BATCH_TUNE | EXX_BATCH_CONCURRENT))
    return fail(h, EXX_ERR_ARG, "exx_build_batched: unknown flag");
  if (n == 0) return EXX_OK;
  if (check_form(h, prec) != EXX_OK) return EXX_ERR_UNSUPPORTED;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  if (!h->aux) {
    e = make_lane_streams(&h->aux, &h->fork_ev, &h->join_ev, &h->chain_ev, h->fb_ev);
    if (e != hipSuccess) return hip_check(h, e, "auxiliary stream");
  }
  e = fft_prepare(&h->ncu);
  if (e != hipSuccess) return hip_check(h, e, "FFT set-up");
  // validate everything and size the scratch before anything is launched
  std::vector<Geom> geo(n);
  std::vector<Layout> lay(n);
  std::vector<Tables> tabs(n);
  for (int i = 0; i < n; ++i) {
    const exx_batch_item& it = items[i];
    exx_status s = check_cell(h, &it.cell, prec);
    if (s != EXX_OK) return fail(h, s, "item " + std::to_string(i) + ": " + h->err);
    if (!it.psi_grid || !it.occ_pts || !it.ao_pts || !it.pts || !it.K || !it.Ex || !it.rank)
      return fail(h, EXX_ERR_ARG, "item " + std::to_string(i) + ": null array");
    geo[i] = make_geom(it.cell);
    lay[i] = layout(h, geo[i], prec, NEED_BUILD);
  }
  if ((flags & EXX_BATCH_GRAPH) && stream == nullptr)
    return fail(h, EXX_ERR_ARG, "EXX_BATCH_GRAPH needs a non-default stream (capture)");
  // capturing several lanes into one graph ended in a host-side segmentation
  // fault inside the capture, launch or instantiation, whose cause has not been
  // found; that combination is switched off
  if ((flags & EXX_BATCH_GRAPH) && (flags & EXX_BATCH_CONCURRENT))
    return fail(h, EXX_ERR_UNSUPPORTED,
                "EXX_BATCH_GRAPH with EXX_BATCH_CONCURRENT is not supported");
  // lanes: several only when asked for, with library-owned scratch, within the
  // device memory that is free now (plus what lane 0 already holds)
  int max_lanes = 1;
  size_t budget = 0;
  if ((flags & EXX_BATCH_CONCURRENT) && !h->user_ws && n > 1) {
    size_t fr = 0, tot = 0;
    e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) return hip_check(h, e, "hipMemGetInfo");
    size_t held = h->ws.cap;
    for (size_t l = 1; l < h->lanes.size(); ++l) held += h->lanes[l].cap;
    budget = (size_t)(0.85 * (double)(fr + held));
    max_lanes = 4;
  }
  std::vector<size_t> need;
  const std::vector<int> lane =
      plan_lanes(geo, lay, budget, max_lanes, &need);
  const int L = (int)need.size();
  exx_status s;
  char* ws0 = (char*)ws_get(h, need[0], &s);
  if (s != EXX_OK) return s;
  s = ensure_lanes(h, L, need);
  if (s != EXX_OK) return s;
  auto ws_of = [&](int i) { return lane[i] == 0 ? ws0 : h->lanes[lane[i]].ws; };
  for (int i = 0; i < n; ++i) {
    s = get_tables(h, geo[i], &tabs[i], stream);
    if (s != EXX_OK) return s;
  }
  if (flags & EXX_BATCH_TUNE) {
    for (int i = 0; i < n; ++i) {
      s = autotune(h, geo[i], tabs[i], ws_of(i), lay[i], prec, items[i], stream);
      if (s != EXX_OK) return s;
    }
  }
  // enqueue lane by lane: lane 0 on `stream`, lanes 1.. on their own streams
  // forked from `stream` and joined back into it
  auto run_all = [&]() -> exx_status {
    const int sg = h->tile_gamma, ss = h->tile_solve;
    hipError_t ee = hipSuccess;
    if (L > 1) {
      ee = hipEventRecord(h->batch_ev, stream);
      for (int l = 1; l < L && ee == hipSuccess; ++l)
        ee = hipStreamWaitEvent(h->lanes[l].st, h->batch_ev, 0);
      if (ee != hipSuccess) return hip_check(h, ee, "lane fork");
    }
    exx_status r = EXX_OK;
    for (int l = 0; l < L && r == EXX_OK; ++l) {
      hipStream_t ls = l == 0 ? stream : h->lanes[l].st;
      if (l > 0) swap_lane(h, h->lanes[l]);
      for (int i = 0; i < n && r == EXX_OK; ++i) {
        if (lane[i] != l) continue;
        long key[5];
        tune_key(geo[i], prec, key);
        if (const exx_context::Tune* t = find_tune(h, key)) {
          h->tile_gamma = t->gamma;
          h->tile_solve = t->solve;
        }
        r = build_one(h, geo[i], tabs[i], ws_of(i), lay[i], prec, items[i], ls);
        h->tile_gamma = sg;
        h->tile_solve = ss;
      }
      if (l > 0) {
        swap_lane(h, h->lanes[l]);
        // join the lane back even after an error, so that a capture stays joined
        hipError_t ej = hipEventRecord(h->lanes[l].done_ev, ls);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(stream, h->lanes[l].done_ev, 0);
        if (ej != hipSuccess && r == EXX_OK) r = hip_check(h, ej, "lane join");
      }
    }
    return r;
  };
  if (!(flags & EXX_BATCH_GRAPH)) {
    s = run_all();
    return s == EXX_OK ? finish(h, stream) : s;
  }

  // signature: precision, refinement, contraction form, checks, lane plan and scratch, every item field
  std::vector<long> sig;
  sig.push_back((long)prec);
  sig.push_back((long)h->refine);
  sig.push_back((long)h->contract);
  sig.push_back((long)h->fit_mode);
  sig.push_back((long)h->checks);
  sig.push_back((long)L);
  sig.push_back((long)(size_t)ws0);
  for (int l = 1; l < L; ++l) sig.push_back((long)(size_t)h->lanes[l].ws);
  for (int i = 0; i < n; ++i) {
    const exx_batch_item& it = items[i];
    const int32_t* c = (const int32_t*)&it.cell;
    for (size_t k = 0; k < sizeof(exx_cell) / sizeof(int32_t); ++k) sig.push_back(c[k]);
    for (const void* p : {(const void*)it.psi_grid, it.occ_pts, it.ao_pts, (const void*)it.pts,
                          (const void*)it.K, (const void*)it.Ex, (const void*)it.rank})
      sig.push_back((long)(size_t)p);
    long key[5];
    tune_key(geo[i], prec, key);
    const exx_context::Tune* t = find_tune(h, key);
    sig.push_back(t ? t->gamma * 100 + t->solve : 0);
    sig.push_back(lane[i]);
  }
  for (const auto& ge : h->graphs)
    if (ge.sig == sig) {
      s = hip_check(h, hipGraphLaunch(ge.exec, stream), "hipGraphLaunch");
      return s == EXX_OK ? finish(h, stream) : s;
    }
  const bool timing = h->timing;
  h->timing = false;  // no event records inside the captured sequence
  e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    h->timing = timing;
    return hip_check(h, e, "hipStreamBeginCapture");
  }
  s = run_all();
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(stream, &graph);
  h->timing = timing;
  if (s != EXX_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return hip_check(h, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_check(h, e, "hipGraphInstantiate");
  h->graphs.push_back({sig, exec});
  s = hip_check(h, hipGraphLaunch(exec, stream), "hipGraphLaunch");
  return s == EXX_OK ? finish(h, stream) : s;
}

extern "C" exx_status exx_save_tuning(exx_handle_t h, const char* path) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!path) return fail(h, EXX_ERR_ARG, "exx_save_tuning: path is NULL");
  FILE* f = fopen(path, "w");
  if (!f) return fail(h, EXX_ERR_ARG, std::string("exx_save_tuning: cannot write ") + path);
  fprintf(f, "# exx tile table v1: n_isdf n_grid n_occ n_k prec tile_gamma tile_solve\n");
  for (const auto& t : h->tuned)
    fprintf(f, "%ld %ld %ld %ld %ld %d %d\n", t.key[0], t.key[1], t.key[2], t.key[3], t.key[4],
            t.gamma, t.solve);
  const bool ok = fclose(f) == 0;
  return ok ? EXX_OK : fail(h, EXX_ERR_ARG, std::string("exx_save_tuning: write failed: ") + path);
}

extern "C" exx_status exx_load_tuning(exx_handle_t h, const char* path) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!path) return fail(h, EXX_ERR_ARG, "exx_load_tuning: path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return fail(h, EXX_ERR_ARG, std::string("exx_load_tuning: cannot read ") + path);
  std::vector<exx_context::Tune> got;
  bool bad = false;
  std::string line;
  char buf[256];
  for (;;) {
    // one whole line, however long
    line.clear();
    while (fgets(buf, sizeof buf, f)) {
      line += buf;
      if (!line.empty() && line.back() == '\n') break;
    }
    if (line.empty()) break;  // end of file
    if (line[0] == '#' || line[0] == '\n') continue;
    // seven decimal integers: five key fields, then the two wave tiles
    long v[7];
    const char* p = line.c_str();
    for (int i = 0; i < 7 && !bad; ++i) {
      char* end = nullptr;
      errno = 0;
      v[i] = strtol(p, &end, 10);
      if (end == p || errno == ERANGE) bad = true;
      p = end;
    }
    while (!bad && (*p == ' ' || *p == '\t' || *p == '\r' || *p == '\n')) ++p;
    if (bad || *p != '\0') {
      bad = true;
      break;
    }
    exx_context::Tune t;
    std::copy(v, v + 5, t.key);
    auto tile_ok = [](long x) { return x == 22 || x == 24 || x == 42; };
    if (!tile_ok(v[5]) || !tile_ok(v[6])) {
      bad = true;
      break;
    }
    t.gamma = (int)v[5];
    t.solve = (int)v[6];
    got.push_back(t);
  }
  fclose(f);
  if (bad) return fail(h, EXX_ERR_ARG, std::string("exx_load_tuning: malformed line in ") + path);
  for (const auto& t : got) {
    bool found = false;
    for (auto& u : h->tuned)
      if (std::equal(u.key, u.key + 5, t.key)) {
        u = t;
        found = true;
      }
    if (!found) h->tuned.push_back(t);
  }
  return EXX_OK;
}

namespace {

// limits of the fit-residual probe (scratch grows with N_k n_occ (N_ISDF + n_probe))
exx_status probe_args(exx_context* h, const Geom& g, int32_t n_probe) {
  if (n_probe < 1 || n_probe > 8192)
    return fail(h, EXX_ERR_SHAPE, "probe: n_probe must be 1..8192");
  if ((long)g.nk * g.no > 65536) return fail(h, EXX_ERR_SHAPE, "probe: N_k n_occ above 65536");
  return EXX_OK;
}
}  // namespace

extern "C" {

exx_status exx_select_points(exx_handle_t h, const exx_cell* cell, const void* psi_grid,
                             int32_t* pts, int32_t* n_pivot, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!psi_grid || !pts || !n_pivot)
    return fail(h, EXX_ERR_ARG, "exx_select_points: null array argument");
  exx_status s = check_cell(h, cell, EXX_F64);
  if (s != EXX_OK) return s;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  Geom g = make_geom(*cell);
  void* ws = ws_get(h, select_scratch_bytes(g), &s);
  if (s != EXX_OK) return s;
  e = launch_select(g, (const double2*)psi_grid, pts, n_pivot, ws, stream);
  return hip_check(h, e, "select");
}

// ---------------------------------------------------------------------------
// learned selector
// ---------------------------------------------------------------------------
exx_status exx_mlp_features(exx_handle_t h, const exx_cell* cell, const void* psi_grid,
                            const double* norm, float* feat, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!psi_grid || !norm || !feat) return fail(h, EXX_ERR_ARG, "exx_mlp_features: null argument");
  for (int i = 0; i < 3; ++i)
    if (!(norm[2 * i + 1] > 0.0) || !std::isfinite(norm[2 * i]))
      return fail(h, EXX_ERR_ARG, "exx_mlp_features: scales must be positive, means finite");
  exx_status s = check_cell(h, cell, EXX_F64);
  if (s != EXX_OK) return s;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  Geom g = make_geom(*cell);
  void* ws = ws_get(h, mlp_feature_scratch_bytes(g), &s);
  if (s != EXX_OK) return s;
  return hip_check(h, launch_mlp_features(g, (const double2*)psi_grid, norm, feat, ws, stream),
                   "features");
}

exx_status exx_mlp_forward(exx_handle_t h, int64_t n, const float* feat, const float* theta,
                           float* score, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (n < 0 || n > INT32_MAX) return fail(h, EXX_ERR_SHAPE, "exx_mlp_forward: n out of range");
  if (n == 0) return EXX_OK;
  if (!feat || !theta || !score) return fail(h, EXX_ERR_ARG, "exx_mlp_forward: null argument");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  return hip_check(h, launch_mlp_forward((long)n, feat, theta, score, stream), "forward");
}

exx_status exx_mlp_backward(exx_handle_t h, int64_t n, const int32_t* idx, int64_t rows,
                            const float* feat, const float* target, float wpos, const float* theta,
                            float* grad, double* loss, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (n < 1 || n > INT32_MAX) return fail(h, EXX_ERR_SHAPE, "exx_mlp_backward: n out of range");
  if (rows < 1 || rows > INT32_MAX || (!idx && rows != n))
    return fail(h, EXX_ERR_SHAPE, "exx_mlp_backward: rows out of range (must equal n without idx)");
  if (!feat || !target || !theta || !grad || !loss)
    return fail(h, EXX_ERR_ARG, "exx_mlp_backward: null argument");
  if (!(wpos >= 0.0f) || !std::isfinite(wpos))
    return fail(h, EXX_ERR_ARG, "exx_mlp_backward: wpos must be finite and >= 0");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  exx_status s;
  void* ws = ws_get(h, mlp_grad_scratch_bytes((long)n), &s);
  if (s != EXX_OK) return s;
  return hip_check(h, launch_mlp_grad((long)n, idx, (long)rows, feat, target, wpos, theta, grad,
                                      loss, ws, stream),
                   "backward");
}

exx_status exx_mlp_moments(exx_handle_t h, int64_t n, const float* feat, double* sums,
                           hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (n < 0) return fail(h, EXX_ERR_SHAPE, "exx_mlp_moments: n < 0");
  if ((n > 0 && !feat) || !sums) return fail(h, EXX_ERR_ARG, "exx_mlp_moments: null argument");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  exx_status s;
  void* ws = ws_get(h, mlp_moments_scratch_bytes((long)n), &s);
  if (s != EXX_OK) return s;
  return hip_check(h, launch_mlp_moments((long)n, feat, sums, ws, stream), "moments");
}

exx_status exx_mlp_adam(exx_handle_t h, int32_t np, float* theta, const float* grad, float* m,
                        float* v, int32_t step, float lr, float beta1, float beta2, float eps,
                        hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (np < 1) return fail(h, EXX_ERR_SHAPE, "exx_mlp_adam: np must be >= 1");
  if (!theta || !grad || !m || !v) return fail(h, EXX_ERR_ARG, "exx_mlp_adam: null argument");
  if (step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps >= 0.0f) || !std::isfinite(lr))
    return fail(h, EXX_ERR_ARG, "exx_mlp_adam: step >= 1, 0 <= beta < 1, eps >= 0 required");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  return hip_check(h, launch_adam(np, theta, grad, m, v, step, lr, beta1, beta2, eps, stream),
                   "adam");
}

exx_status exx_mlp_targets(exx_handle_t h, const exx_cell* cell, const int32_t* pts, int32_t npts,
                           double sigma, float* target, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!pts || !target) return fail(h, EXX_ERR_ARG, "exx_mlp_targets: null argument");
  if (!(sigma > 0.0) || !std::isfinite(sigma))
    return fail(h, EXX_ERR_ARG, "exx_mlp_targets: sigma must be positive and finite");
  exx_status s = check_cell(h, cell, EXX_F64);
  if (s != EXX_OK) return s;
  Geom g = make_geom(*cell);
  if (npts < 1 || npts > 2048 || npts > g.ng)
    return fail(h, EXX_ERR_SHAPE, "exx_mlp_targets: npts must be 1..min(2048, N_g)");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  return hip_check(h, launch_targets(g, pts, npts, sigma, target, stream), "targets");
}

exx_status exx_mlp_nms(exx_handle_t h, const exx_cell* cell, const float* score, int32_t k,
                       int32_t* pts, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!score || !pts) return fail(h, EXX_ERR_ARG, "exx_mlp_nms: null argument");
  exx_status s = check_cell(h, cell, EXX_F64);
  if (s != EXX_OK) return s;
  Geom g = make_geom(*cell);
  if (k < 1 || k > g.ng) return fail(h, EXX_ERR_SHAPE, "exx_mlp_nms: k must be 1..N_g");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  void* ws = ws_get(h, mlp_nms_scratch_bytes(g), &s);
  if (s != EXX_OK) return s;
  return hip_check(h, launch_nms(g, score, k, pts, ws, stream), "nms");
}

exx_status exx_mlp_probe(exx_handle_t h, const exx_cell* cell, const void* psi_grid,
                         const int32_t* pts, int32_t n_probe, uint64_t seed, double* resid,
                         hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!psi_grid || !pts || !resid) return fail(h, EXX_ERR_ARG, "exx_mlp_probe: null argument");
  exx_status s = check_cell(h, cell, EXX_F64);
  if (s != EXX_OK) return s;
  Geom g = make_geom(*cell);
  if ((s = probe_args(h, g, n_probe)) != EXX_OK) return s;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  void* ws = ws_get(h, mlp_probe_scratch_bytes(g, n_probe), &s);
  if (s != EXX_OK) return s;
  return hip_check(
      h, launch_mlp_probe(g, (const double2*)psi_grid, pts, n_probe, seed, resid, ws, stream),
      "probe");
}

exx_status exx_select_points_mlp(exx_handle_t h, const exx_cell* cell, const void* psi_grid,
                                 const double* norm, const float* theta, double tau,
                                 int32_t n_probe, int32_t* pts, int32_t* used_fallback,
                                 double* resid_out, hipStream_t stream) {
  if (!h) return EXX_ERR_ARG;
  h->err.clear();
  if (!psi_grid || !norm || !theta || !pts || !used_fallback)
    return fail(h, EXX_ERR_ARG, "exx_select_points_mlp: null argument");
  if (!(tau >= 0.0)) return fail(h, EXX_ERR_ARG, "exx_select_points_mlp: tau must be >= 0");
  for (int i = 0; i < 3; ++i)
    if (!(norm[2 * i + 1] > 0.0) || !std::isfinite(norm[2 * i]))
      return fail(h, EXX_ERR_ARG, "exx_select_points_mlp: scales must be positive, means finite");
  exx_status s = check_cell(h, cell, EXX_F64);
  if (s != EXX_OK) return s;
  Geom g = make_geom(*cell);
  if ((s = probe_args(h, g, n_probe)) != EXX_OK) return s;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_check(h, e, "hipSetDevice");
  // scratch: [feat | score | resid | max(feature, nms, probe, QRCP scratch)]
  const size_t fb = al(sizeof(float) * 3 * (size_t)g.ng), sb = al(sizeof(float) * (size_t)g.ng);
  size_t inner = mlp_feature_scratch_bytes(g);
  inner = std::max(inner, mlp_nms_scratch_bytes(g));
  inner = std::max(inner, mlp_probe_scratch_bytes(g, n_probe));
  inner = std::max(inner, select_scratch_bytes(g));
  char* ws = (char*)ws_get(h, fb + sb + al(sizeof(double)) + inner, &s);
  if (s != EXX_OK) return s;
  float* feat = (float*)ws;
  float* score = (float*)(ws + fb);
  double* dres = (double*)(ws + fb + sb);
  void* rest = ws + fb + sb + al(sizeof(double));
  const double2* psi = (const double2*)psi_grid;
  e = launch_mlp_features(g, psi, norm, feat, rest, stream);
  if (e == hipSuccess) e = launch_mlp_forward((long)g.ng, feat, theta, score, stream);
  if (e == hipSuccess) e = launch_nms(g, score, g.ni, pts, rest, stream);
  if (e == hipSuccess)
    e = launch_mlp_probe(g, psi, pts, n_probe, 0x2304055050ull, dres, rest, stream);
  double resid = 0.0;
  if (e == hipSuccess) e = hipMemcpyAsync(&resid, dres, sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_check(h, e, "learned selection");
  if (resid_out) *resid_out = resid;
  *used_fallback = 0;
  if (!(resid <= tau)) {  // also taken when the residual is not a number
    int32_t* npiv = (int32_t*)(ws + fb);  // the score buffer is free again
    e = launch_select(g, psi, pts, npiv, rest, stream);
    if (e != hipSuccess) return hip_check(h, e, "QRCP fallback");
    *used_fallback = 1;
  }
  return EXX_OK;
}

}  // extern "C"

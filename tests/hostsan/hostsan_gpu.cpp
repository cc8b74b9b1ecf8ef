// The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
// during real GPU builds (the library objects are compiled with the sanitizers
// on their host pass only; the kernels are the usual ones).
//
// Reads the seeded cells that tests/test_gpu_hostsan.py writes (raw arrays
// and cells.txt) and runs, per cell: the fused build in FP64 and MIXED, the
// stage-wise calls, the allocation-free contraction, the exchange gradient,
// the robust fit, a build on a caller-owned workspace and QRCP point
// selection; then the batched call on two copies of every cell (plain, lanes,
// a captured graph twice, tuned, tuned with lanes), the tile table's file
// round trip and a timed MIXED batch. The calls are compared with each other:
// the FP64 routes to the fused build within what the cells' conditioning
// allows (stage-wise, allocation-free and gradient K to 1e-6 / 1e-8 / 1e-8,
// batched to 1e-8, E_x to 1e-9), MIXED to 1e-5, the caller workspace exactly.
// Agreement with the oracle is the parity tests' concern; this driver is about
// the host code. Prints "hostsan-gpu ok" and exits 0 when every check holds.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/exx.h"

typedef std::complex<double> cd;

static int fails = 0;
#define CHECK(c, ...)                                  \
  do {                                                 \
    if (!(c)) {                                        \
      fprintf(stderr, "FAIL %s:%d ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);                    \
      fprintf(stderr, "\n");                           \
      ++fails;                                         \
    }                                                  \
  } while (0)
#define HIPOK(x)                                                   \
  do {                                                             \
    hipError_t e_ = (x);                                           \
    if (e_ != hipSuccess) {                                        \
      fprintf(stderr, "HIP %s at %d\n", hipGetErrorString(e_), __LINE__); \
      exit(3);                                                     \
    }                                                              \
  } while (0)

template <typename T>
std::vector<T> readf(const std::string& p, size_t n) {
  std::vector<T> v(n);
  FILE* f = fopen(p.c_str(), "rb");
  if (!f || fread(v.data(), sizeof(T), n, f) != n) {
    fprintf(stderr, "cannot read %s\n", p.c_str());
    exit(3);
  }
  fclose(f);
  return v;
}

template <typename T>
T* up(const std::vector<T>& v) {
  T* d = nullptr;
  HIPOK(hipMalloc((void**)&d, v.size() * sizeof(T)));
  HIPOK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

template <typename T>
std::vector<T> down(const T* d, size_t n) {
  std::vector<T> v(n);
  HIPOK(hipMemcpy(v.data(), d, n * sizeof(T), hipMemcpyDeviceToHost));
  return v;
}

double reldiff(const std::vector<cd>& a, const std::vector<cd>& b) {
  double m = 0, s = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    m = std::max(m, std::abs(a[i] - b[i]));
    s = std::max(s, std::abs(b[i]));
  }
  return m / std::max(s, 1e-300);
}

struct Case {
  exx_cell c;
  int nk, ng;
  cd *psi, *occ, *ao, *aog;
  int32_t* pts;
  std::vector<cd> K0;
  double E0;
  std::vector<int32_t> r0;
};

int main(int argc, char** argv) {
  if (argc < 3) {
    fprintf(stderr, "usage: %s <input dir> <scratch dir>\n", argv[0]);
    return 2;
  }
  const std::string dir = argv[1];
  const std::string tmp = argv[2];
  exx_handle_t h = nullptr;
  CHECK(exx_create(&h, 0) == EXX_OK, "create");
  std::vector<Case> cs;
  FILE* f = fopen((dir + "/cells.txt").c_str(), "r");
  if (!f) {
    fprintf(stderr, "cannot read %s/cells.txt\n", dir.c_str());
    return 3;
  }
  Case x;
  while (fscanf(f, "%lf %lf %lf %d %d %d %d %d %d %d %d %d", &x.c.L[0], &x.c.L[1], &x.c.L[2],
                &x.c.grid[0], &x.c.grid[1], &x.c.grid[2], &x.c.kmesh[0], &x.c.kmesh[1],
                &x.c.kmesh[2], &x.c.n_occ, &x.c.n_ao, &x.c.n_isdf) == 12)
    cs.push_back(x);
  fclose(f);
  for (size_t i = 0; i < cs.size(); ++i) {
    Case& c = cs[i];
    c.nk = c.c.kmesh[0] * c.c.kmesh[1] * c.c.kmesh[2];
    c.ng = c.c.grid[0] * c.c.grid[1] * c.c.grid[2];
    const int no = c.c.n_occ, na = c.c.n_ao, ni = c.c.n_isdf, nk = c.nk, ng = c.ng;
    const std::string s = std::to_string(i);
    c.psi = up(readf<cd>(dir + "/psi" + s + ".bin", (size_t)nk * no * ng));
    c.occ = up(readf<cd>(dir + "/occ" + s + ".bin", (size_t)nk * ni * no));
    c.ao = up(readf<cd>(dir + "/ao" + s + ".bin", (size_t)nk * ni * na));
    c.aog = up(readf<cd>(dir + "/aog" + s + ".bin", (size_t)nk * na * ng));
    c.pts = up(readf<int32_t>(dir + "/pts" + s + ".bin", ni));
  }
  hipStream_t st;
  HIPOK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  for (size_t i = 0; i < cs.size(); ++i) {
    Case& c = cs[i];
    const int na = c.c.n_ao, ni = c.c.n_isdf, nk = c.nk, ng = c.ng;
    const size_t nK = (size_t)nk * na * na;
    cd *K, *K2, *Kg, *xi, *S, *V;
    double* Ex;
    int32_t* rank;
    HIPOK(hipMalloc((void**)&K, nK * 16));
    HIPOK(hipMalloc((void**)&K2, nK * 16));
    HIPOK(hipMalloc((void**)&Kg, nK * 16));
    HIPOK(hipMalloc((void**)&Ex, 8));
    HIPOK(hipMalloc((void**)&rank, 4 * nk));
    HIPOK(hipMalloc((void**)&xi, (size_t)nk * ni * ng * 16));
    HIPOK(hipMalloc((void**)&S, (size_t)nk * ni * ni * 16));
    HIPOK(hipMalloc((void**)&V, (size_t)nk * ni * ni * 16));
    // fused FP64 and MIXED
    CHECK(exx_build(h, &c.c, EXX_F64, c.psi, c.occ, c.ao, c.pts, K, Ex, rank, st) == EXX_OK,
          "build %zu: %s", i, exx_last_error(h));
    HIPOK(hipStreamSynchronize(st));
    c.K0 = down(K, nK);
    c.E0 = down(Ex, 1)[0];
    c.r0 = down(rank, nk);
    CHECK(exx_build(h, &c.c, EXX_MIXED, c.psi, c.occ, c.ao, c.pts, K2, Ex, rank, st) == EXX_OK,
          "mixed %zu", i);
    HIPOK(hipStreamSynchronize(st));
    const double dm = reldiff(down(K2, nK), c.K0);
    // stage-wise FP64
    CHECK(exx_isdf_fit(h, &c.c, EXX_F64, c.psi, c.occ, c.pts, xi, S, rank, st) == EXX_OK, "fit");
    CHECK(exx_coulomb_V(h, &c.c, EXX_F64, xi, c.pts, V, st) == EXX_OK, "coulomb");
    CHECK(exx_build_K(h, &c.c, EXX_F64, c.ao, c.occ, V, K2, Ex, st) == EXX_OK, "build_K");
    HIPOK(hipStreamSynchronize(st));
    const double ds = reldiff(down(K2, nK), c.K0);
    // allocation-free contraction
    exx_status sn = exx_build_K_noalloc(h, &c.c, EXX_F64, c.ao, c.occ, V, K2, Ex, st);
    HIPOK(hipStreamSynchronize(st));
    double dn = -1;
    if (sn == EXX_OK) dn = reldiff(down(K2, nK), c.K0);
    // gradient and robust
    CHECK(exx_exchange_gradient(h, &c.c, EXX_F64, c.psi, c.occ, c.ao, c.aog, c.pts, K2, Kg, Ex,
                                rank, st) == EXX_OK,
          "gradient %zu: %s", i, exx_last_error(h));
    HIPOK(hipStreamSynchronize(st));
    const double dg = reldiff(down(K2, nK), c.K0);
    CHECK(exx_build_robust(h, &c.c, EXX_MIXED, c.psi, c.occ, c.ao, c.aog, c.pts, K2, Ex, rank,
                           st) == EXX_OK,
          "robust %zu: %s", i, exx_last_error(h));
    HIPOK(hipStreamSynchronize(st));
    // caller workspace
    size_t need = 0;
    CHECK(exx_workspace_size(h, &c.c, EXX_F64, EXX_CALL_BUILD, &need) == EXX_OK, "ws size");
    void* ws = nullptr;
    HIPOK(hipMalloc(&ws, need));
    CHECK(exx_set_workspace(h, ws, need) == EXX_OK, "set ws");
    CHECK(exx_build(h, &c.c, EXX_F64, c.psi, c.occ, c.ao, c.pts, K2, Ex, rank, st) == EXX_OK,
          "ws build");
    HIPOK(hipStreamSynchronize(st));
    const double dw = reldiff(down(K2, nK), c.K0);
    CHECK(exx_set_workspace(h, nullptr, 0) == EXX_OK, "unset ws");
    HIPOK(hipFree(ws));
    // selection
    int32_t *p2, *npiv;
    HIPOK(hipMalloc((void**)&p2, 4 * ni));
    HIPOK(hipMalloc((void**)&npiv, 4));
    CHECK(exx_select_points(h, &c.c, c.psi, p2, npiv, st) == EXX_OK, "select %s",
          exx_last_error(h));
    HIPOK(hipStreamSynchronize(st));
    printf("cell %zu: mixed %.1e stages %.1e noalloc %.1e (status %d) gradient-K %.1e ws %.1e\n",
           i, dm, ds, dn, (int)sn, dg, dw);
    CHECK(dm < 1e-5 && ds < 1e-6 && dg < 1e-8 && dw == 0.0, "cell %zu differences", i);
    CHECK(sn != EXX_OK || dn < 1e-8, "noalloc");
    for (void* p : {(void*)K, (void*)K2, (void*)Kg, (void*)Ex, (void*)rank, (void*)xi, (void*)S,
                    (void*)V, (void*)p2, (void*)npiv})
      HIPOK(hipFree(p));
  }
  // batched: two copies of every cell, plain, lanes, captured graph (replayed), tuned
  const int n = 2 * (int)cs.size();
  std::vector<exx_batch_item> items(n);
  std::vector<cd*> Ks(n);
  std::vector<double*> Es(n);
  std::vector<int32_t*> Rs(n);
  for (int j = 0; j < n; ++j) {
    Case& c = cs[j % cs.size()];
    const size_t nK = (size_t)c.nk * c.c.n_ao * c.c.n_ao;
    HIPOK(hipMalloc((void**)&Ks[j], nK * 16));
    HIPOK(hipMalloc((void**)&Es[j], 8));
    HIPOK(hipMalloc((void**)&Rs[j], 4 * c.nk));
    items[j] = exx_batch_item{c.c, c.psi, c.occ, c.ao, c.pts, Ks[j], Es[j], Rs[j]};
  }
  const int flag_sets[] = {0, EXX_BATCH_CONCURRENT, EXX_BATCH_GRAPH, EXX_BATCH_GRAPH,
                           EXX_BATCH_TUNE, EXX_BATCH_TUNE | EXX_BATCH_CONCURRENT};
  for (int fl : flag_sets) {
    for (int j = 0; j < n; ++j) HIPOK(hipMemsetAsync(Ks[j], 0, 16, st));
    HIPOK(hipStreamSynchronize(st));
    CHECK(exx_build_batched(h, n, items.data(), EXX_F64, fl, st) == EXX_OK, "batched %d: %s", fl,
          exx_last_error(h));
    HIPOK(hipStreamSynchronize(st));
    double worst = 0;
    for (int j = 0; j < n; ++j) {
      Case& c = cs[j % cs.size()];
      const size_t nK = (size_t)c.nk * c.c.n_ao * c.c.n_ao;
      worst = std::max(worst, reldiff(down(Ks[j], nK), c.K0));
      CHECK(std::abs(down(Es[j], 1)[0] - c.E0) <= 1e-9 * std::abs(c.E0), "batched Ex");
      CHECK(down(Rs[j], c.nk) == c.r0, "batched rank");
    }
    printf("batched flags %d: worst rel dK %.1e\n", fl, worst);
    CHECK(worst < 1e-8, "batched flags %d", fl);
  }
  const std::string tf = tmp + "/tiles.txt";
  CHECK(exx_save_tuning(h, tf.c_str()) == EXX_OK, "save");
  CHECK(exx_load_tuning(h, tf.c_str()) == EXX_OK, "load");
  // MIXED batch with timing
  CHECK(exx_set_timing(h, 1) == EXX_OK, "timing");
  CHECK(exx_build_batched(h, n, items.data(), EXX_MIXED, EXX_BATCH_CONCURRENT, st) == EXX_OK,
        "mixed batch");
  HIPOK(hipStreamSynchronize(st));
  double ms[32];
  int32_t calls[32];
  CHECK(exx_phase_times(h, ms, calls, 32) == EXX_OK, "phase times");
  CHECK(exx_set_timing(h, 0) == EXX_OK, "timing off");
  size_t sb = 0;
  CHECK(exx_scratch_bytes(h, &sb) == EXX_OK && sb > 0, "scratch bytes");
  for (int j = 0; j < n; ++j) {
    HIPOK(hipFree(Ks[j]));
    HIPOK(hipFree(Es[j]));
    HIPOK(hipFree(Rs[j]));
  }
  for (Case& c : cs)
    for (void* p : {(void*)c.psi, (void*)c.occ, (void*)c.ao, (void*)c.aog, (void*)c.pts})
      HIPOK(hipFree(p));
  CHECK(exx_destroy(h) == EXX_OK, "destroy");
  HIPOK(hipStreamDestroy(st));
  printf("%s: %d failures, scratch %zu bytes\n", fails ? "FAILED" : "hostsan-gpu ok", fails, sb);
  return fails ? 1 : 0;
}

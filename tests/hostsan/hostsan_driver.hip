// Host-side checks of the exchange library under AddressSanitizer and
// UndefinedBehaviorSanitizer, on a machine without a GPU.
//
// The library's entry-point source is compiled into this file, so that the host
// logic behind the C ABI is reachable without a device: argument and shape
// validation of every entry point, the scratch layouts of every call form, the
// conjugate-pair table of the k-mesh, the lane plan of the batched call and the
// tile-table file format. Every call here returns before its first HIP runtime
// call (or fails that call on a handle whose device does not exist); no kernel
// is launched. Prints "hostsan ok" after the last check, "hostsan skip" when a
// GPU is visible (the checks rely on device calls failing), and exits non-zero
// on the first failed check.
#include "../../paper_2304_05505_amd/csrc/api.hip"

#include <cstdarg>
#include <unistd.h>

namespace {

int n_checks = 0;

void check(bool ok, const char* fmt, ...) {
  ++n_checks;
  if (ok) return;
  va_list ap;
  va_start(ap, fmt);
  fprintf(stderr, "hostsan check failed: ");
  vfprintf(stderr, fmt, ap);
  fprintf(stderr, "\n");
  va_end(ap);
  exit(2);
}

exx_cell make_cell(int n1, int n2, int n3, int N1, int N2, int N3, int no, int nao, int ni) {
  exx_cell c;
  c.L[0] = 5.0;
  c.L[1] = 5.5;
  c.L[2] = 6.0;
  c.grid[0] = n1;
  c.grid[1] = n2;
  c.grid[2] = n3;
  c.kmesh[0] = N1;
  c.kmesh[1] = N2;
  c.kmesh[2] = N3;
  c.n_occ = no;
  c.n_ao = nao;
  c.n_isdf = ni;
  return c;
}

// a device-less handle: every HIP call on it fails, nothing is allocated
exx_context* fake_handle() {
  exx_context* h = new exx_context();
  h->device = -1;
  return h;
}

// every entry point refuses a NULL handle
void null_handle_calls() {
  int dummy = 0;
  void* p = &dummy;
  int32_t* ip = &dummy;
  double d = 0.0;
  size_t sz = 0;
  exx_cell c = make_cell(8, 8, 8, 1, 1, 1, 1, 1, 1);
  check(strcmp(exx_last_error(nullptr), "null handle") == 0, "exx_last_error(NULL)");
  check(exx_create(nullptr, 0) == EXX_ERR_ARG, "exx_create(NULL)");
  check(exx_destroy(nullptr) == EXX_ERR_ARG, "exx_destroy(NULL)");
  check(exx_scratch_bytes(nullptr, &sz) == EXX_ERR_ARG, "scratch_bytes");
  check(exx_workspace_size(nullptr, &c, EXX_F64, EXX_CALL_BUILD, &sz) == EXX_ERR_ARG, "ws size");
  check(exx_set_workspace(nullptr, nullptr, 0) == EXX_ERR_ARG, "set_workspace");
  check(exx_set_checks(nullptr, 0) == EXX_ERR_ARG, "set_checks");
  check(exx_get_status(nullptr, nullptr, ip) == EXX_ERR_ARG, "get_status");
  check(exx_isdf_fit(nullptr, &c, EXX_F64, p, p, ip, p, p, ip, nullptr) == EXX_ERR_ARG, "fit");
  check(exx_coulomb_V(nullptr, &c, EXX_F64, p, ip, p, nullptr) == EXX_ERR_ARG, "coulomb");
  check(exx_build_K(nullptr, &c, EXX_F64, p, p, p, p, &d, nullptr) == EXX_ERR_ARG, "build_K");
  check(exx_build_K_noalloc(nullptr, &c, EXX_F64, p, p, p, p, &d, nullptr) == EXX_ERR_ARG,
        "build_K_noalloc");
  check(exx_build(nullptr, &c, EXX_F64, p, p, p, ip, p, &d, ip, nullptr) == EXX_ERR_ARG, "build");
  check(exx_exchange_gradient(nullptr, &c, EXX_F64, p, p, p, p, ip, p, p, &d, ip, nullptr) ==
            EXX_ERR_ARG,
        "gradient");
  check(exx_build_robust(nullptr, &c, EXX_F64, p, p, p, p, ip, p, &d, ip, nullptr) == EXX_ERR_ARG,
        "robust");
  check(exx_select_points(nullptr, &c, p, ip, ip, nullptr) == EXX_ERR_ARG, "select");
  check(exx_mlp_features(nullptr, &c, p, &d, (float*)p, nullptr) == EXX_ERR_ARG, "features");
  check(exx_mlp_moments(nullptr, 1, (float*)p, &d, nullptr) == EXX_ERR_ARG, "moments");
  check(exx_mlp_forward(nullptr, 1, (float*)p, (float*)p, (float*)p, nullptr) == EXX_ERR_ARG,
        "forward");
  check(exx_mlp_backward(nullptr, 1, ip, 1, (float*)p, (float*)p, 1.f, (float*)p, (float*)p, &d,
                         nullptr) == EXX_ERR_ARG,
        "backward");
  check(exx_mlp_adam(nullptr, 1, (float*)p, (float*)p, (float*)p, (float*)p, 1, 1e-3f, 0.9f,
                     0.999f, 1e-8f, nullptr) == EXX_ERR_ARG,
        "adam");
  check(exx_mlp_targets(nullptr, &c, ip, 1, 1.0, (float*)p, nullptr) == EXX_ERR_ARG, "targets");
  check(exx_mlp_nms(nullptr, &c, (float*)p, 1, ip, nullptr) == EXX_ERR_ARG, "nms");
  check(exx_mlp_probe(nullptr, &c, p, ip, 1, 7, &d, nullptr) == EXX_ERR_ARG, "probe");
  check(exx_select_points_mlp(nullptr, &c, p, &d, (float*)p, 0.1, 1, ip, ip, &d, nullptr) ==
            EXX_ERR_ARG,
        "select_mlp");
  check(exx_build_batched(nullptr, 0, nullptr, EXX_F64, 0, nullptr) == EXX_ERR_ARG, "batched");
  check(exx_save_tuning(nullptr, "x") == EXX_ERR_ARG, "save_tuning");
  check(exx_load_tuning(nullptr, "x") == EXX_ERR_ARG, "load_tuning");
  check(exx_set_refinement(nullptr, 0) == EXX_ERR_ARG, "set_refinement");
  check(exx_set_fit(nullptr, 0) == EXX_ERR_ARG, "set_fit");
  check(exx_set_contraction(nullptr, 0) == EXX_ERR_ARG, "set_contraction");
  check(exx_set_timing(nullptr, 0) == EXX_ERR_ARG, "set_timing");
  check(exx_phase_times(nullptr, &d, ip, 1) == EXX_ERR_ARG, "phase_times");
}

// the shape checks: every out-of-range field gives its status and a message
void shape_errors(exx_context* h) {
  struct Bad {
    exx_cell c;
    exx_prec prec;
    exx_status want;
  };
  std::vector<Bad> bad;
  const exx_cell ok = make_cell(12, 10, 10, 2, 1, 1, 2, 14, 16);
  auto with = [&](auto edit, exx_status want, exx_prec prec = EXX_F64) {
    exx_cell c = ok;
    edit(c);
    bad.push_back({c, prec, want});
  };
  with([](exx_cell& c) { c.L[1] = 0.0; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.L[2] = -1.0; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.L[0] = NAN; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.grid[0] = 1; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.grid[1] = 7; }, EXX_ERR_SHAPE);  // not 2*3*5-smooth
  with([](exx_cell& c) { c.grid[2] = 256; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.grid[2] = INT_MIN; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.kmesh[0] = 0; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.kmesh[2] = 9; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.kmesh[0] = c.kmesh[1] = c.kmesh[2] = 5; }, EXX_ERR_SHAPE);  // 125 > 64
  with([](exx_cell& c) { c.n_occ = 0; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.n_occ = 513; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.n_ao = 4097; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.n_isdf = 0; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.n_isdf = 2049; }, EXX_ERR_SHAPE);
  with([](exx_cell& c) { c.grid[0] = c.grid[1] = c.grid[2] = 2; }, EXX_ERR_SHAPE);  // n_isdf > N_g
  with([](exx_cell& c) { c.grid[1] = c.grid[2] = 120; }, EXX_ERR_UNSUPPORTED);    // n2 n3 > 6144
  // one transfer's grid arrays beyond 32-bit byte offsets: n_isdf N_g or n_occ N_g >= 2^28
  with([](exx_cell& c) {
    c.grid[0] = 128, c.grid[1] = 48, c.grid[2] = 48;
    c.n_isdf = 2048;
  }, EXX_ERR_UNSUPPORTED);
  with([](exx_cell& c) {
    c.grid[0] = 128, c.grid[1] = 48, c.grid[2] = 128;
    c.n_occ = 512;
  }, EXX_ERR_UNSUPPORTED);
  with([](exx_cell&) {}, EXX_ERR_ARG, (exx_prec)7);
  with([](exx_cell&) {}, EXX_ERR_ARG, (exx_prec)-1);
  int dummy = 0;
  void* p = &dummy;
  int32_t* ip = &dummy;
  double d = 0.0;
  size_t sz = 0;
  for (size_t i = 0; i < bad.size(); ++i) {
    const exx_cell* c = &bad[i].c;
    const exx_prec pr = bad[i].prec;
    const exx_status w = bad[i].want;
    exx_status got[] = {
        exx_workspace_size(h, c, pr, EXX_CALL_BUILD, &sz),
        exx_isdf_fit(h, c, pr, p, p, ip, p, p, ip, nullptr),
        exx_coulomb_V(h, c, pr, p, ip, p, nullptr),
        exx_build_K(h, c, pr, p, p, p, p, &d, nullptr),
        exx_build_K_noalloc(h, c, pr, p, p, p, p, &d, nullptr),
        exx_build(h, c, pr, p, p, p, ip, p, &d, ip, nullptr),
    };
    for (size_t j = 0; j < sizeof got / sizeof got[0]; ++j)
      check(got[j] == w && !h->err.empty(), "bad cell %zu call %zu: status %d (want %d), '%s'", i,
            j, (int)got[j], (int)w, h->err.c_str());
    if (pr == EXX_F64 || pr == EXX_MIXED) {
      // the gradient calls check the cell as FP64 (or MIXED) builds
      const exx_status g = exx_exchange_gradient(h, c, pr, p, p, p, p, ip, p, p, &d, ip, nullptr);
      const exx_status r = exx_build_robust(h, c, pr, p, p, p, p, ip, p, &d, ip, nullptr);
      check(g == w && r == w, "bad cell %zu gradient %d robust %d (want %d)", i, (int)g, (int)r,
            (int)w);
    }
  }
  // the largest accepted cell: every size at its maximum, n_isdf N_g just below 2^28
  const exx_cell big = make_cell(128, 32, 30, 1, 1, 1, 512, 4096, 2048);
  for (exx_prec pr : {EXX_F64, EXX_F32, EXX_BF16, EXX_MIXED})
    for (int call = 0; call < 4; ++call)
      check(exx_workspace_size(h, &big, pr, call, &sz) == EXX_OK && sz > 0,
            "largest cell, call %d: %s", call, h->err.c_str());
  // a NULL cell and NULL arrays
  check(exx_workspace_size(h, nullptr, EXX_F64, EXX_CALL_BUILD, &sz) == EXX_ERR_ARG, "NULL cell");
  check(exx_workspace_size(h, &ok, EXX_F64, EXX_CALL_BUILD, nullptr) == EXX_ERR_ARG, "NULL bytes");
  check(exx_workspace_size(h, &ok, EXX_F64, 99, &sz) == EXX_ERR_ARG, "unknown call");
  check(exx_build(h, &ok, EXX_F64, nullptr, p, p, ip, p, &d, ip, nullptr) == EXX_ERR_ARG,
        "build NULL psi");
  check(exx_isdf_fit(h, &ok, EXX_F64, p, p, nullptr, p, p, ip, nullptr) == EXX_ERR_ARG,
        "fit NULL pts");
  check(exx_exchange_gradient(h, &ok, EXX_F64, p, p, p, nullptr, ip, p, p, &d, ip, nullptr) ==
            EXX_ERR_ARG,
        "gradient NULL ao_grid");
  check(exx_exchange_gradient(h, &ok, EXX_F32, p, p, p, p, ip, p, p, &d, ip, nullptr) ==
            EXX_ERR_UNSUPPORTED,
        "gradient in F32");
  // the batched call: bad lists and flags are refused before the device
  check(exx_build_batched(h, -1, nullptr, EXX_F64, 0, nullptr) == EXX_ERR_ARG, "batched n < 0");
  check(exx_build_batched(h, 2, nullptr, EXX_F64, 0, nullptr) == EXX_ERR_ARG, "batched NULL");
  check(exx_build_batched(h, 0, nullptr, EXX_F64, 64, nullptr) == EXX_ERR_ARG, "batched flag");
  check(exx_build_batched(h, 0, nullptr, EXX_F64, 0, nullptr) == EXX_OK, "batched empty");
  // setters
  check(exx_set_refinement(h, 2) == EXX_ERR_ARG && exx_set_refinement(h, 1) == EXX_OK &&
            exx_set_refinement(h, 0) == EXX_OK,
        "set_refinement");
  check(exx_set_fit(h, 5) == EXX_ERR_ARG && exx_set_fit(h, EXX_FIT_PER_Q) == EXX_OK, "set_fit");
  check(exx_set_contraction(h, -1) == EXX_ERR_ARG && exx_set_contraction(h, 4) == EXX_ERR_ARG &&
            exx_set_contraction(h, EXX_CONTRACT_AUTO) == EXX_OK,
        "set_contraction");
  // a BF16 contraction form on FP64 transforms
  check(exx_set_contraction(h, EXX_CONTRACT_BF16) == EXX_OK, "bf16 form");
  check(exx_build(h, &ok, EXX_F64, p, p, p, ip, p, &d, ip, nullptr) == EXX_ERR_UNSUPPORTED,
        "bf16 form with F64");
  check(exx_set_contraction(h, EXX_CONTRACT_AUTO) == EXX_OK, "auto form");
  check(exx_set_workspace(h, (char*)p + 1, 64) == EXX_ERR_ARG, "unaligned workspace");
  double ms[4];
  int32_t calls[4];
  check(exx_phase_times(h, ms, calls, -1) == EXX_ERR_ARG, "phase_times n < 0");
  check(exx_phase_times(h, ms, calls, 4) == EXX_OK && calls[3] == 0 && ms[0] == 0.0,
        "phase_times empty");
  check(exx_scratch_bytes(h, &sz) == EXX_OK && sz == 0, "scratch_bytes %zu", sz);
}

// -m is the partner of m; pairs cover the mesh once
void pair_tables() {
  for (int N1 = 1; N1 <= 8; ++N1)
    for (int N2 = 1; N2 <= 8; ++N2)
      for (int N3 = 1; N3 <= 8; ++N3) {
        if (N1 * N2 * N3 > 64) continue;
        const exx_cell c = make_cell(8, 8, 8, N1, N2, N3, 1, 1, 1);
        const exx::Geom g = exx::make_geom(c);
        const Pairs p = make_pairs(g);
        std::vector<int> seen(g.nk, 0);
        for (int s = 0; s < p.n; ++s) {
          const int m = p.rep[s], b = p.bar[s];
          check(m >= 0 && m < g.nk && p.slot[m] == s, "pairs %dx%dx%d slot", N1, N2, N3);
          ++seen[m];
          if (b >= 0) {
            check(b > m && b < g.nk && p.slot[b] == -1, "pairs %dx%dx%d bar", N1, N2, N3);
            ++seen[b];
            // m + b = 0 on the mesh
            const int m1 = m / (N2 * N3), m2 = (m / N3) % N2, m3 = m % N3;
            const int b1 = b / (N2 * N3), b2 = (b / N3) % N2, b3 = b % N3;
            check((m1 + b1) % N1 == 0 && (m2 + b2) % N2 == 0 && (m3 + b3) % N3 == 0,
                  "pairs %dx%dx%d: %d + %d != 0", N1, N2, N3, m, b);
          }
        }
        for (int m = 0; m < g.nk; ++m) check(seen[m] == 1, "pairs %dx%dx%d cover", N1, N2, N3);
      }
}

// scratch layouts: every offset 256-byte aligned and in order, within the total
void layouts(exx_context* h) {
  const int meshes[][3] = {{1, 1, 1}, {2, 1, 1}, {3, 1, 1}, {2, 2, 2}, {3, 3, 3}, {4, 4, 4},
                           {3, 2, 1}, {1, 2, 3}, {5, 1, 1}, {4, 2, 1}, {8, 8, 1}, {2, 3, 4}};
  const int grids[][3] = {{12, 10, 10}, {36, 36, 36}, {2, 4, 8}, {120, 48, 128}, {30, 45, 64}};
  const int dims[][3] = {{1, 1, 1}, {2, 14, 16}, {8, 32, 176}, {35, 118, 1376}, {512, 4096, 2048}};
  const exx_prec precs[] = {EXX_F64, EXX_F32, EXX_BF16, EXX_MIXED};
  const int needs[] = {NEED_FIT, NEED_COULOMB, NEED_K, NEED_BUILD, NEED_GRAD,
                       NEED_FIT | NEED_COULOMB | NEED_K};
  size_t nlay = 0;
  for (int mode : {EXX_FIT_PER_Q, EXX_FIT_SHARED})
    for (auto& M : meshes)
      for (auto& G : grids)
        for (auto& D : dims)
          for (exx_prec pr : precs) {
            h->fit_mode = mode;
            const exx_cell c = make_cell(G[0], G[1], G[2], M[0], M[1], M[2], D[0], D[1], D[2]);
            if (check_cell(h, &c, pr) != EXX_OK) {
              h->err.clear();
              continue;
            }
            const exx::Geom g = exx::make_geom(c);
            for (int need : needs) {
              const Layout L = layout(h, g, pr, need);
              const size_t off[] = {L.G,     L.Lf,  L.W,    L.Sp,  L.keep, L.Y,     L.T,
                                    L.epart, L.cpart, L.S2, L.V2,  L.rank2, L.tol, L.Tinv,
                                    L.grid,  L.grid2, L.F,  L.g3,  L.gvt,  L.gCS,  L.gT,
                                    L.gA,    L.gP,  L.total};
              for (size_t i = 0; i < sizeof off / sizeof off[0]; ++i) {
                check(off[i] % 256 == 0, "layout offset %zu not aligned", i);
                if (i) check(off[i] >= off[i - 1], "layout offset %zu out of order", i);
              }
              check(L.total >= L.F && L.nsplit >= 1, "layout total");
              if (mode == EXX_FIT_PER_Q && build_path(h, g) == PATH_PAIRED) {
                check(L.pd.cols >= 1 && L.pd.cols <= g.ng && L.pd.per >= 1 && L.pd.nchunk >= 1 &&
                          L.pd.per * L.pd.nchunk >= make_pairs(g).n,
                      "paired chunking");
              }
              ++nlay;
            }
            size_t b[4];
            for (int call = 0; call < 4; ++call)
              check(exx_workspace_size(h, &c, pr, call, &b[call]) == EXX_OK && b[call] > 0,
                    "workspace_size call %d: %s", call, h->err.c_str());
          }
  h->fit_mode = EXX_FIT_PER_Q;
  check(nlay > 1000, "only %zu layouts", nlay);
}

// lanes: each item on one lane, each lane sized for its largest item, one lane
// when nothing fits the budget
void lane_plans(exx_context* h) {
  const int shapes[][9] = {{36, 36, 36, 2, 2, 2, 8, 32, 176},   {12, 10, 10, 2, 1, 1, 2, 14, 16},
                           {48, 48, 48, 1, 1, 1, 16, 64, 320},  {36, 36, 36, 3, 3, 3, 8, 32, 176},
                           {30, 30, 30, 2, 2, 1, 4, 20, 120},   {24, 24, 24, 1, 1, 2, 6, 24, 96}};
  for (int n = 1; n <= 24; ++n) {
    std::vector<exx::Geom> geo;
    std::vector<Layout> lay;
    for (int i = 0; i < n; ++i) {
      const int* s = shapes[(i * 5 + n) % 6];
      const exx_cell c = make_cell(s[0], s[1], s[2], s[3], s[4], s[5], s[6], s[7], s[8]);
      geo.push_back(exx::make_geom(c));
      lay.push_back(layout(h, geo.back(), EXX_MIXED, NEED_BUILD));
    }
    for (size_t budget : {(size_t)0, (size_t)1 << 30, (size_t)64 << 30, (size_t)-1}) {
      for (int max_lanes : {1, 2, 4}) {
        std::vector<size_t> need;
        const std::vector<int> lane = plan_lanes(geo, lay, budget, max_lanes, &need);
        const int L = (int)need.size();
        check(L >= 1 && L <= std::min(max_lanes, n) && (int)lane.size() == n, "lanes n=%d", n);
        size_t tot = 0;
        for (size_t x : need) tot += x;
        check(L == 1 || tot <= budget, "lanes over budget");
        for (int i = 0; i < n; ++i)
          check(lane[i] >= 0 && lane[i] < L && need[lane[i]] >= lay[i].total, "lane of item %d",
                i);
        if (budget == 0) check(L == 1, "zero budget uses one lane");
      }
    }
  }
}

// the tile table file: round trip, malformed lines, long lines, missing files
void tuning_files(exx_context* h, const char* dir) {
  const std::string f1 = std::string(dir) + "/tiles.txt";
  exx_context::Tune t;
  for (int i = 0; i < 5; ++i) {
    for (int k = 0; k < 5; ++k) t.key[k] = 100 * i + k;
    t.gamma = (i % 2) ? 24 : 42;
    t.solve = 22;
    h->tuned.push_back(t);
  }
  check(exx_save_tuning(h, f1.c_str()) == EXX_OK, "save: %s", h->err.c_str());
  exx_context* h2 = fake_handle();
  check(exx_load_tuning(h2, f1.c_str()) == EXX_OK && h2->tuned.size() == 5, "load round trip");
  for (size_t i = 0; i < 5; ++i)
    check(std::equal(h->tuned[i].key, h->tuned[i].key + 5, h2->tuned[i].key) &&
              h->tuned[i].gamma == h2->tuned[i].gamma && h->tuned[i].solve == h2->tuned[i].solve,
          "entry %zu", i);
  // loading again replaces, does not duplicate
  check(exx_load_tuning(h2, f1.c_str()) == EXX_OK && h2->tuned.size() == 5, "reload");
  auto write = [&](const char* name, const std::string& text) {
    const std::string path = std::string(dir) + "/" + name;
    FILE* f = fopen(path.c_str(), "w");
    check(f != nullptr, "cannot write %s", path.c_str());
    fputs(text.c_str(), f);
    fclose(f);
    return path;
  };
  const std::string bad_tile = write("bad_tile.txt", "1 2 3 4 0 33 22\n");
  const std::string short_line = write("short.txt", "# header\n1 2 3\n");
  const std::string words = write("words.txt", "tile gamma solve\n");
  const std::string digits = write("digits.txt", "1 2 3 4 0 22 22\n" + std::string(700, '7') +
                                                    " 1 1 1 0 22 22\n");
  const std::string range = write("range.txt", "99999999999999999999999 1 1 1 0 22 22\n");
  const std::string trail = write("trail.txt", "1 2 3 4 0 22 22 5\n");
  for (const std::string& path : {bad_tile, short_line, words, digits, range, trail}) {
    const size_t before = h2->tuned.size();
    check(exx_load_tuning(h2, path.c_str()) == EXX_ERR_ARG && !h2->err.empty() &&
              h2->tuned.size() == before,
          "malformed %s accepted", path.c_str());
  }
  // a comment longer than the read buffer, a CRLF line and no final newline
  const std::string longc =
      write("long_comment.txt", "# " + std::string(1000, 'x') + "\n7 7 7 7 1 24 42\r\n8 8 8 8 1 42 22");
  check(exx_load_tuning(h2, longc.c_str()) == EXX_OK && h2->tuned.size() == 7 &&
            h2->tuned[5].key[0] == 7 && h2->tuned[5].gamma == 24 && h2->tuned[5].solve == 42 &&
            h2->tuned[6].key[3] == 8 && h2->tuned[6].gamma == 42,
        "long comment: %s", h2->err.c_str());
  const std::string empty = write("empty.txt", "");
  check(exx_load_tuning(h2, empty.c_str()) == EXX_OK && h2->tuned.size() == 7, "empty file");
  check(exx_load_tuning(h2, (std::string(dir) + "/missing.txt").c_str()) == EXX_ERR_ARG,
        "missing file");
  check(exx_load_tuning(h2, nullptr) == EXX_ERR_ARG && exx_save_tuning(h2, nullptr) == EXX_ERR_ARG,
        "NULL path");
  check(exx_save_tuning(h2, (std::string(dir) + "/no/such/dir/t.txt").c_str()) == EXX_ERR_ARG,
        "unwritable path");
  delete h2;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: %s <scratch dir>\n", argv[0]);
    return 2;
  }
  exx_handle_t real = nullptr;
  const exx_status st = exx_create(&real, 0);
  if (st == EXX_OK) {
    exx_destroy(real);
    printf("hostsan skip: a GPU is visible\n");
    return 0;
  }
  check(st == EXX_ERR_DEVICE && real == nullptr, "exx_create without a GPU: %d", (int)st);
  null_handle_calls();
  exx_context* h = fake_handle();
  shape_errors(h);
  pair_tables();
  layouts(h);
  lane_plans(h);
  tuning_files(h, argv[1]);
  check(exx_destroy(h) == EXX_OK, "destroy");
  printf("hostsan ok: %d checks\n", n_checks);
  return 0;
}

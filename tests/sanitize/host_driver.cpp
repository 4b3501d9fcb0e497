// Host-only driver of the library's CPU code (option validation, geometry, Hamiltonian builder, Pauli
// tables, momenta, site fields, the product kernels' tile maps), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Every check prints a line; any failure
// or sanitizer report ends the process with a non-zero status.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "host_model.h"
#include "tile_map.h"

using namespace vemb;

static int failures = 0;
#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);    \
      ++failures;                                                    \
    }                                                                \
  } while (0)

static vemb_lattice ring(int N) { return vemb_lattice{1, {N, 1}, {1, 1}}; }
static vemb_lattice torus(int Nx, int Ny) { return vemb_lattice{2, {Nx, Ny}, {1, 1}}; }

static vemb_term term1(double c, int p) { return vemb_term{c, 1, {p, 0}, {{0, 0}, {0, 0}}}; }
static vemb_term term2(double c, int p, int q, int dx, int dy) { return vemb_term{c, 2, {p, q}, {{0, 0}, {dx, dy}}}; }

static void options() {
  vemb_options o;
  std::string err;
  CHECK(normalize_options(nullptr, o, err) == VEMB_OK && o.mu == 10.0 && o.max_sweeps == 40 && o.warm_refresh == 64);
  vemb_options in;
  vemb_default_options(&in);
  in.mu = -1.0;
  CHECK(normalize_options(&in, o, err) == VEMB_E_INVALID);
  vemb_default_options(&in);
  in.precision = 7;
  CHECK(normalize_options(&in, o, err) == VEMB_E_INVALID);
  vemb_default_options(&in);
  in.lb_every = -3;
  CHECK(normalize_options(&in, o, err) == VEMB_E_INVALID);
  vemb_default_options(&in);
  in.adapt_every = -1;
  CHECK(normalize_options(&in, o, err) == VEMB_E_INVALID);
  vemb_default_options(&in);
  in.fermionic = 1;
  in.opset = VEMB_OPSET_PAULI1;
  CHECK(normalize_options(&in, o, err) == VEMB_E_UNSUPPORTED);
  vemb_default_options(&in);
  in.nu = std::nan("");
  CHECK(normalize_options(&in, o, err) == VEMB_E_INVALID);
  std::printf("options: ok\n");
}

static void geometry() {
  Geometry g;
  std::string err;
  CHECK(parse_geometry(ring(8), vemb_clusters{{2, 1}}, g, err) == VEMB_OK && g.M == 4 && g.L == 2 && g.n == 16);
  CHECK(parse_geometry(torus(16, 16), vemb_clusters{{2, 2}}, g, err) == VEMB_OK && g.M == 64 && g.n == 256);
  CHECK(parse_geometry(ring(9), vemb_clusters{{2, 1}}, g, err) == VEMB_E_INVALID);        // no tiling
  CHECK(parse_geometry(ring(4), vemb_clusters{{4, 1}}, g, err) == VEMB_E_UNSUPPORTED);    // M = 1
  CHECK(parse_geometry(ring(10), vemb_clusters{{5, 1}}, g, err) == VEMB_E_UNSUPPORTED);   // 5-site clusters
  CHECK(parse_geometry(ring(0), vemb_clusters{{1, 1}}, g, err) == VEMB_E_INVALID);
  CHECK(parse_geometry(vemb_lattice{3, {4, 4}, {1, 1}}, vemb_clusters{{1, 1}}, g, err) == VEMB_E_INVALID);
  CHECK(parse_geometry(vemb_lattice{1, {8, 1}, {0, 1}}, vemb_clusters{{1, 1}}, g, err) == VEMB_E_UNSUPPORTED);
  CHECK(parse_geometry(ring(8), vemb_clusters{{1, 2}}, g, err) == VEMB_E_INVALID);        // 2D cluster on a ring
  // cluster counts whose product overflows int are refused, not wrapped
  CHECK(parse_geometry(torus(1 << 30, 1 << 30), vemb_clusters{{1, 1}}, g, err) != VEMB_OK);
  CHECK(parse_geometry(torus(1 << 16, 1 << 16), vemb_clusters{{1, 1}}, g, err) != VEMB_OK);
  std::printf("geometry: ok\n");
}

static double hermitian_defect(const std::vector<double>& A, int n) {
  double d = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) d = std::fmax(d, std::fabs(A[(size_t)i * n + j] - A[(size_t)j * n + i]));
  return d;
}

static void models() {
  std::string err;
  for (int L : {1, 2, 3, 4}) {
    Geometry g;
    CHECK(parse_geometry(ring(4 * L), vemb_clusters{{L, 1}}, g, err) == VEMB_OK);
    std::vector<vemb_term> tfi = {term2(-1.0, VEMB_Z, VEMB_Z, 1, 0), term1(-0.7, VEMB_X)};
    HostModel h;
    CHECK(build_model(vemb_hamiltonian{(int)tfi.size(), tfi.data()}, g, h, err) == VEMB_OK);
    CHECK((int)h.H0.size() == g.m * g.m && (int)h.hd_index.size() == g.M - 1);
    CHECK(hermitian_defect(h.H0, g.m) == 0.0);
    const size_t blocks = h.Hd.size() / ((size_t)g.n * g.n);
    for (size_t b = 0; b < blocks; ++b)
      CHECK(hermitian_defect(std::vector<double>(h.Hd.begin() + b * g.n * g.n, h.Hd.begin() + (b + 1) * g.n * g.n),
                             g.n) == 0.0);
    for (int d : h.hd_index) CHECK(d >= -1 && d < (int)blocks);
    std::vector<vemb_term> xxz = {term2(1.0, VEMB_X, VEMB_X, 1, 0), term2(1.0, VEMB_Y, VEMB_Y, 1, 0),
                                  term2(0.5, VEMB_Z, VEMB_Z, 1, 0)};
    CHECK(build_model(vemb_hamiltonian{(int)xxz.size(), xxz.data()}, g, h, err) == VEMB_OK);
    std::vector<vemb_term> hop = {term2(-1.0, VEMB_FHOP, VEMB_FHOP, 1, 0), term2(0.25, VEMB_Z, VEMB_Z, 1, 0)};
    CHECK(build_model(vemb_hamiltonian{(int)hop.size(), hop.data()}, g, h, err, true) == VEMB_OK);
    CHECK(build_model(vemb_hamiltonian{(int)hop.size(), hop.data()}, g, h, err, false) != VEMB_OK);
    std::vector<vemb_term> bad = {term1(1.0, 9)};
    CHECK(build_model(vemb_hamiltonian{1, bad.data()}, g, h, err) != VEMB_OK);
    std::vector<vemb_term> far = {term2(1.0, VEMB_Z, VEMB_Z, 1 << 20, 0)};  // range wraps on the ring
    build_model(vemb_hamiltonian{1, far.data()}, g, h, err);
    std::vector<vemb_term> neg = {term2(1.0, VEMB_Z, VEMB_Z, -3, 0)};
    build_model(vemb_hamiltonian{1, neg.data()}, g, h, err);
    OpTables T;
    build_pauli1_tables(L, T);
    CHECK(T.n_op == 3 * L);
    for (int a = 0; a < T.n_op; ++a)
      for (int v = 0; v < g.m; ++v) CHECK(T.perm[a][v] >= 0 && T.perm[a][v] < g.m && (T.sign[a][v] == 1 || T.sign[a][v] == -1));
  }
  Geometry g;
  CHECK(parse_geometry(torus(8, 4), vemb_clusters{{2, 2}}, g, err) == VEMB_OK);
  std::vector<vemb_term> t2 = {term2(-1.0, VEMB_Z, VEMB_Z, 1, 0), term2(-1.0, VEMB_Z, VEMB_Z, 0, 1), term1(-3.0, VEMB_X)};
  HostModel h;
  CHECK(build_model(vemb_hamiltonian{(int)t2.size(), t2.data()}, g, h, err) == VEMB_OK);
  std::printf("models: ok\n");
}

static void momenta_and_fields() {
  std::string err;
  for (auto dims : {std::make_pair(8, 1), std::make_pair(9, 1), std::make_pair(4, 4), std::make_pair(6, 3)}) {
    Geometry g;
    vemb_lattice lat = dims.second == 1 ? ring(dims.first) : torus(dims.first, dims.second);
    CHECK(parse_geometry(lat, vemb_clusters{{1, 1}}, g, err) == VEMB_OK);
    std::vector<double> tw, wk;
    int Ku = 0;
    build_momenta(g, tw, wk, Ku);
    double total = 0.0;
    for (double w : wk) total += w;
    CHECK(Ku > 0 && (int)wk.size() == Ku && (int)tw.size() == 2 * Ku * g.M && total == (double)g.M);
    std::vector<double> Hc((size_t)g.M * g.m * g.m, 0.0);
    CHECK(add_site_field(g, 0, 0, VEMB_X, 0.5, Hc, err) == VEMB_OK);
    CHECK(add_site_field(g, g.Nx - 1, g.Ny - 1, VEMB_Z, 0.5, Hc, err) == VEMB_OK);
    CHECK(add_site_field(g, g.Nx, 0, VEMB_Z, 0.5, Hc, err) == VEMB_OK);  // coordinates wrap (periodic)
    CHECK(add_site_field(g, -1, -7, VEMB_Z, 0.5, Hc, err) == VEMB_OK);
    CHECK(add_site_field(g, 0, 0, VEMB_Y, 0.5, Hc, err) != VEMB_OK);
    CHECK(add_site_field(g, 0, 0, VEMB_Z, std::nan(""), Hc, err) != VEMB_OK);
  }
  std::printf("momenta and fields: ok\n");
}

static void tile_maps() {
  for (int tiles = 1; tiles <= 64; ++tiles) {
    const int cnt = upper_tile_count(tiles);
    std::set<std::pair<int, int>> seen;
    for (int idx = 0; idx < cnt; ++idx) {
      int ti = -1, tj = -1;
      CHECK(upper_tile(idx, tiles, &ti, &tj));
      CHECK(0 <= ti && ti <= tj && tj < tiles);
      seen.insert({ti, tj});
    }
    CHECK((int)seen.size() == cnt);
    int ti, tj, blk;
    CHECK(!upper_tile(cnt, tiles, &ti, &tj) && !upper_tile(-1, tiles, &ti, &tj));
    CHECK(!batched_tile_of(0, 3, 3, tiles, &blk, &ti, &tj) && batched_tile_of(cnt - 1, 2, 3, tiles, &blk, &ti, &tj));
  }
  std::printf("tile maps: ok\n");
}

int main() {
  options();
  geometry();
  models();
  momenta_and_fields();
  tile_maps();
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "all passed", failures);
  return failures ? 1 : 0;
}

// Host-side mesh and geometric-map code (csrc/mesh.cpp, csrc/geomap.cpp) exercised over its
// construction paths and its validation cases, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (and libstdc++ bounds assertions).  Any sanitizer report aborts
// the run; a wrong result or a missing error message exits with status 1.  Prints
// "host-mesh-driver ok <checks>" on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <stdexcept>
#include <string>
#include <vector>

#include "geomap.hpp"
#include "mesh.hpp"

using decmg::Mesh;

static int checks = 0;

static void expect(bool ok, const std::string& what) {
  ++checks;
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what.c_str());
    std::exit(1);
  }
}

static void expect_error(const std::string& err, const char* part, const std::string& what) {
  expect(err.find(part) != std::string::npos, what + ": got \"" + err + "\"");
}

// topology, stars and boundary of a mesh that must be valid; Euler characteristic chi
static Mesh finish(Mesh m, int64_t chi, const std::string& what) {
  expect(m.validate_vertices().empty(), what + " vertices");
  expect(m.build_topology().empty(), what + " topology");
  m.build_stars();
  m.build_boundary();
  expect(m.nv - m.ne + m.nt == chi, what + " Euler characteristic");
  expect(int64_t(m.star0.size()) == m.nv && int64_t(m.star1.size()) == m.ne, what + " stars");
  double area = 0.0;
  for (double a : m.star0) area += a;
  expect(std::isfinite(area) && area > 0.0, what + " dual area");
  return m;
}

static Mesh from_arrays(std::vector<double> xyz, std::vector<int32_t> tri) {
  Mesh m;
  m.nv = int64_t(xyz.size() / 3);
  m.nt = int64_t(tri.size() / 3);
  m.xyz = std::move(xyz);
  m.tri = std::move(tri);
  return m;
}

// the first check that fails among validate_vertices and build_topology ("" when none)
static std::string validate(Mesh m) {
  std::string err = m.validate_vertices();
  if (err.empty()) err = m.build_topology();
  return err;
}

static void meshes() {
  for (int n = 1; n <= 5; ++n) {
    Mesh m = finish(decmg::square_grid(n), 1, "square " + std::to_string(n));
    int64_t nb = 0;
    for (uint8_t b : m.bnd) nb += b;
    expect(nb == 4 * n, "square boundary vertices");
    Mesh f = finish(decmg::subdivide(m, false), 1, "binary subdivision");
    expect(f.nv == m.nv + m.ne && f.nt == 4 * m.nt, "binary counts");
    Mesh g = finish(decmg::subdivide(f, false), 1, "second binary subdivision");
    Mesh c = finish(decmg::subdivide_cubic(m, false), 1, "cubic subdivision");
    expect(c.nv == m.nv + 2 * m.ne + m.nt && c.nt == 9 * m.nt, "cubic counts");
    finish(decmg::subdivide_cubic(c, false), 1, "second cubic subdivision");
    finish(decmg::subdivide(c, false), 1, "binary after cubic");
    (void)g;
  }
  Mesh s = finish(decmg::icosahedron(), 2, "icosahedron");
  expect(s.nv == 12 && s.ne == 30 && s.nt == 20, "icosahedron counts");
  for (int i = 0; i < 3; ++i) s = finish(decmg::subdivide(s, true), 2, "sphere subdivision");
  for (int64_t v = 0; v < s.nv; ++v) {
    const double* p = &s.xyz[3 * v];
    expect(std::fabs(std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - 1.0) < 1e-14,
           "projected vertex on the unit sphere");
  }
  finish(decmg::subdivide_cubic(finish(decmg::icosahedron(), 2, "icosahedron"), true), 2,
         "cubic sphere");
  // subdivision needs the coarse topology: refused, not read out of bounds
  bool refused = false;
  try {
    (void)decmg::subdivide(decmg::icosahedron(), true);
  } catch (const std::logic_error&) {
    refused = true;
  }
  expect(refused, "subdivision without topology refused");

  const std::vector<double> sq = {0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0};
  expect(validate(from_arrays(sq, {0, 1, 2, 1, 3, 2})).empty(), "two-triangle square");
  expect_error(validate(from_arrays(sq, {0, 1, 1, 1, 3, 2})), "degenerate", "degenerate");
  expect_error(validate(from_arrays(sq, {0, 1, 2, 1, 3, 2, 2, 1, 0})), "duplicate", "duplicate");
  expect_error(validate(from_arrays(sq, {0, 1, 2})), "in no triangle", "isolated vertex");
  std::vector<double> bad = sq;
  bad[9] = std::numeric_limits<double>::quiet_NaN();
  expect_error(validate(from_arrays(bad, {0, 1, 2, 1, 3, 2})), "non-finite", "NaN coordinate");
  bad[9] = std::numeric_limits<double>::infinity();
  expect_error(validate(from_arrays(bad, {0, 1, 2, 1, 3, 2})), "non-finite", "inf coordinate");
  std::vector<double> five = sq;
  five.insert(five.end(), {0.5, -1, 0});
  expect_error(validate(from_arrays(five, {0, 1, 2, 1, 3, 2, 1, 2, 4})), "more than two",
               "edge of three triangles");
}

// M(f) of a binary subdivision X of Y from X's parent pairs, in CSC form
struct Csc {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> colptr;
  std::vector<int32_t> rowval;
  std::vector<double> nzval;
  mg_geomap view() const {
    return mg_geomap{rows, cols, colptr.data(), rowval.data(), nzval.data()};
  }
};

static Csc binary_map(const Mesh& Y, const Mesh& X) {
  Csc f;
  f.rows = Y.nv;
  f.cols = X.nv;
  f.colptr.push_back(0);
  for (int64_t j = 0; j < X.nv; ++j) {
    const int32_t a = X.parent[2 * j], b = X.parent[2 * j + 1];
    if (a == b) {
      f.rowval.push_back(a);
      f.nzval.push_back(1.0);
    } else {
      f.rowval.insert(f.rowval.end(), {a, b});
      f.nzval.insert(f.nzval.end(), {0.5, 0.5});
    }
    f.colptr.push_back(int64_t(f.rowval.size()));
  }
  return f;
}

static void geomaps() {
  Mesh Z = finish(decmg::square_grid(1), 1, "Z");
  Mesh Y = finish(decmg::subdivide(Z, false), 1, "Y");
  Mesh X = finish(decmg::subdivide(Y, false), 1, "X");
  Csc f = binary_map(Y, X), g = binary_map(Z, Y);
  expect(decmg::check_geomap(Y, X.nv, f.view()).empty(), "binary map accepted");
  expect(decmg::geomap_keeps_ids(f.view()), "binary map keeps ids");
  Mesh Xi = X;
  decmg::set_interp_from_geomap(Xi, f.view());
  for (int64_t j = 0; j < X.nv; ++j)
    for (int q = 0; q < 3; ++q)
      expect(Xi.parent3[3 * j + q] == X.parent3[3 * j + q] &&
                 Xi.pweight[3 * j + q] == X.pweight[3 * j + q],
             "interpolation rows from the map");

  // rejected maps: each mutation of f and the message part it must produce
  auto mutated = [&](const char* part, const std::string& what, auto&& change) {
    Csc h = f;
    int64_t nx = X.nv;
    change(h, nx);
    expect_error(decmg::check_geomap(Y, nx, h.view()), part, what);
  };
  mutated("does not match", "shape", [](Csc&, int64_t& nx) { nx -= 1; });
  mutated("does not match", "negative rows", [](Csc& h, int64_t&) { h.rows = -1; });
  mutated("colptr[0]", "colptr start", [](Csc& h, int64_t&) { h.colptr[0] = 1; });
  mutated("colptr decreases", "colptr order", [](Csc& h, int64_t&) {
    std::swap(h.colptr[3], h.colptr[4]);
  });
  mutated("row out of range", "row range", [](Csc& h, int64_t&) { h.rowval[5] = int32_t(h.rows); });
  mutated("row out of range", "negative row", [](Csc& h, int64_t&) { h.rowval[2] = -3; });
  mutated("1 to 3 entries", "empty column", [](Csc& h, int64_t&) {
    // column 0 (one entry) becomes empty: drop its entry
    h.rowval.erase(h.rowval.begin());
    h.nzval.erase(h.nzval.begin());
    for (size_t j = 1; j < h.colptr.size(); ++j) h.colptr[j] -= 1;
  });
  mutated("finite and >= 0", "negative weight", [](Csc& h, int64_t&) { h.nzval[0] = -1.0; });
  mutated("finite and >= 0", "NaN weight", [](Csc& h, int64_t&) {
    h.nzval[0] = std::numeric_limits<double>::quiet_NaN();
  });
  mutated("sum to 1", "weight sum", [](Csc& h, int64_t&) { h.nzval[0] = 0.75; });
  // a midpoint column (two entries) with its rows made equal
  int64_t two = -1;
  for (int64_t j = 0; j < X.nv && two < 0; ++j)
    if (f.colptr[j + 1] - f.colptr[j] == 2) two = j;
  expect(two >= 0, "a midpoint column exists");
  mutated("repeats a row", "repeated row", [&](Csc& h, int64_t&) {
    h.rowval[h.colptr[two] + 1] = h.rowval[h.colptr[two]];
  });
  // two vertices of Y that share no triangle
  int32_t u = -1, w = -1;
  for (int32_t a = 0; a < Y.nv && u < 0; ++a)
    for (int32_t b = a + 1; b < Y.nv && u < 0; ++b) {
      bool shared = false;
      for (int64_t t = 0; t < Y.nt && !shared; ++t) {
        const int32_t* T = &Y.tri[3 * t];
        shared = (T[0] == a || T[1] == a || T[2] == a) && (T[0] == b || T[1] == b || T[2] == b);
      }
      if (!shared) {
        u = a;
        w = b;
      }
    }
  expect(u >= 0, "a pair of vertices in no common triangle");
  mutated("one simplex", "rows of no simplex", [&](Csc& h, int64_t&) {
    h.rowval[h.colptr[two]] = u;
    h.rowval[h.colptr[two] + 1] = w;
  });
  mutated("1 to 3 entries", "four entries", [&](Csc& h, int64_t&) {
    const int64_t p = h.colptr[two + 1];
    h.rowval.insert(h.rowval.begin() + p, {0, 1});
    h.nzval.insert(h.nzval.begin() + p, {0.0, 0.0});
    for (size_t j = size_t(two) + 1; j < h.colptr.size(); ++j) h.colptr[j] += 2;
  });
  {
    Csc h = f;
    mg_geomap v = h.view();
    v.colptr = nullptr;
    expect_error(decmg::check_geomap(Y, X.nv, v), "null colptr", "null colptr");
  }

  // composition M(g o f) = M(g) M(f): sizes, capacity protocol, columns summing to 1
  int64_t nnz = 0;
  expect(decmg::compose_geomaps(g.view(), f.view(), nullptr, nullptr, nullptr, &nnz).empty(),
         "compose count");
  expect(nnz > 0, "compose entries");
  std::vector<int64_t> cp(size_t(X.nv) + 1);
  std::vector<int32_t> rv(static_cast<size_t>(nnz));
  std::vector<double> nz(static_cast<size_t>(nnz));
  int64_t cap = nnz - 1;
  expect_error(decmg::compose_geomaps(g.view(), f.view(), cp.data(), rv.data(), nz.data(), &cap),
               "too small", "compose capacity");
  cap = nnz;
  expect(decmg::compose_geomaps(g.view(), f.view(), cp.data(), rv.data(), nz.data(), &cap)
             .empty(),
         "compose fill");
  expect(cap == nnz && cp.back() == nnz, "compose fill count");
  for (int64_t j = 0; j < X.nv; ++j) {
    double s = 0.0;
    for (int64_t p = cp[j]; p < cp[j + 1]; ++p) {
      s += nz[p];
      expect(rv[p] >= 0 && rv[p] < Z.nv, "composed row in range");
      if (p > cp[j]) expect(rv[p] > rv[p - 1], "composed rows ascend");
    }
    expect(std::fabs(s - 1.0) < 1e-15, "composed column sums to 1");
  }
  Mesh Zc = Z;
  expect(decmg::check_geomap(Zc, X.nv,
                             mg_geomap{Z.nv, X.nv, cp.data(), rv.data(), nz.data()})
             .empty(),
         "composed map is a geometric map");
  expect_error(decmg::compose_geomaps(f.view(), f.view(), nullptr, nullptr, nullptr, &nnz),
               "not composable", "compose shapes");
  // compose checks index ranges only; a negative dimension or a bad row stops it first
  {
    Csc h = g;
    h.cols = -1;
    mg_geomap fv = f.view();
    fv.n_rows = -1;
    expect_error(decmg::compose_geomaps(h.view(), fv, nullptr, nullptr, nullptr, &nnz),
                 "negative dimension", "compose negative dimension");
    h = g;
    h.rowval[1] = int32_t(Z.nv);
    expect_error(decmg::compose_geomaps(h.view(), f.view(), nullptr, nullptr, nullptr, &nnz),
                 "row out of range", "compose row range");
    expect_error(decmg::compose_geomaps(g.view(), f.view(), cp.data(), nullptr, nz.data(), &cap),
                 "rowval and nzval", "compose null outputs");
  }
}

int main() {
  meshes();
  geomaps();
  std::printf("host-mesh-driver ok %d\n", checks);
  return 0;
}

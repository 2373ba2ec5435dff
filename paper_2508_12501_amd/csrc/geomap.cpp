#include "geomap.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace decmg {

namespace {

std::string col_msg(int64_t j, const char* what) {
  return "map column " + std::to_string(j) + ": " + what;
}

// Index ranges and monotone column pointers.
std::string check_ranges(const mg_geomap& f) {
  if (f.n_rows < 0 || f.n_cols < 0) return "map has a negative dimension";
  if (!f.colptr) return "map has a null colptr";
  if (f.colptr[0] != 0) return "map colptr[0] must be 0";
  if (f.colptr[f.n_cols] > 0 && (!f.rowval || !f.nzval)) return "map has null arrays";
  for (int64_t j = 0; j < f.n_cols; ++j) {
    if (f.colptr[j + 1] < f.colptr[j]) return col_msg(j, "colptr decreases");
    for (int64_t p = f.colptr[j]; p < f.colptr[j + 1]; ++p)
      if (f.rowval[p] < 0 || f.rowval[p] >= f.n_rows) return col_msg(j, "row out of range");
  }
  return "";
}

}  // namespace

std::string check_geomap(const Mesh& Y, int64_t nx, const mg_geomap& f) {
  if (f.n_rows != Y.nv || f.n_cols != nx)
    return "map shape " + std::to_string(f.n_rows) + " x " + std::to_string(f.n_cols) +
           " does not match the meshes (" + std::to_string(Y.nv) + " x " + std::to_string(nx) +
           ")";
  if (std::string err = check_ranges(f); !err.empty()) return err;
  // triangles of Y around each vertex, to decide whether rows span one simplex
  std::vector<int64_t> off(Y.nv + 1, 0);
  for (int64_t i = 0; i < 3 * Y.nt; ++i) ++off[Y.tri[i] + 1];
  for (int64_t v = 0; v < Y.nv; ++v) off[v + 1] += off[v];
  std::vector<int32_t> inc(3 * Y.nt);
  {
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int64_t t = 0; t < Y.nt; ++t)
      for (int q = 0; q < 3; ++q) inc[pos[Y.tri[3 * t + q]]++] = int32_t(t);
  }
  for (int64_t j = 0; j < nx; ++j) {
    const int64_t b = f.colptr[j], k = f.colptr[j + 1] - b;
    if (k < 1 || k > 3) return col_msg(j, "must hold 1 to 3 entries");
    const int32_t* r = f.rowval + b;
    double sum = 0.0;
    for (int64_t q = 0; q < k; ++q) {
      const double w = f.nzval[b + q];
      if (!std::isfinite(w) || w < 0.0) return col_msg(j, "weights must be finite and >= 0");
      sum += w;
      for (int64_t s = 0; s < q; ++s)
        if (r[s] == r[q]) return col_msg(j, "repeats a row");
    }
    if (std::fabs(sum - 1.0) > 1e-12) return col_msg(j, "weights must sum to 1");
    if (k == 1) continue;
    bool found = false;
    for (int64_t p = off[r[0]]; p < off[r[0] + 1] && !found; ++p) {
      const int32_t* T = &Y.tri[3 * size_t(inc[p])];
      bool all = true;
      for (int64_t q = 1; q < k; ++q) all = all && (r[q] == T[0] || r[q] == T[1] || r[q] == T[2]);
      found = all;
    }
    if (!found) return col_msg(j, "rows are not the vertices of one simplex of the coarser mesh");
  }
  return "";
}

void set_interp_from_geomap(Mesh& X, const mg_geomap& f) {
  X.scheme = 3;
  X.parent.clear();
  X.parent3.assign(3 * size_t(X.nv), 0);
  X.pweight.assign(3 * size_t(X.nv), 0.0);
  for (int64_t j = 0; j < X.nv; ++j) {
    const int64_t b = f.colptr[j], k = f.colptr[j + 1] - b;
    for (int q = 0; q < 3; ++q) {
      X.parent3[3 * j + q] = f.rowval[b + (q < k ? q : 0)];
      X.pweight[3 * j + q] = q < k ? f.nzval[b + q] : 0.0;
    }
  }
}

bool geomap_keeps_ids(const mg_geomap& f) {
  if (f.n_cols < f.n_rows) return false;
  for (int64_t j = 0; j < f.n_rows; ++j) {
    const int64_t b = f.colptr[j];
    if (f.colptr[j + 1] - b != 1 || f.rowval[b] != j || f.nzval[b] != 1.0) return false;
  }
  return true;
}

std::string compose_geomaps(const mg_geomap& g, const mg_geomap& f, int64_t* colptr,
                            int32_t* rowval, double* nzval, int64_t* nnz) {
  if (f.n_rows != g.n_cols) return "maps are not composable (f.n_rows != g.n_cols)";
  if (std::string err = check_ranges(f); !err.empty()) return "f: " + err;
  if (std::string err = check_ranges(g); !err.empty()) return "g: " + err;
  const bool fill = colptr != nullptr;
  if (fill && (!rowval || !nzval)) return "rowval and nzval are needed with colptr";
  const int64_t cap = fill ? *nnz : 0;
  std::vector<double> acc(g.n_rows, 0.0);
  std::vector<int64_t> mark(g.n_rows, -1);
  std::vector<int32_t> rows;
  int64_t count = 0;
  if (fill) colptr[0] = 0;
  for (int64_t j = 0; j < f.n_cols; ++j) {
    rows.clear();
    for (int64_t p = f.colptr[j]; p < f.colptr[j + 1]; ++p) {
      const int32_t k = f.rowval[p];
      const double a = f.nzval[p];
      for (int64_t q = g.colptr[k]; q < g.colptr[k + 1]; ++q) {
        const int32_t r = g.rowval[q];
        if (mark[r] != j) {
          mark[r] = j;
          acc[r] = 0.0;
          rows.push_back(r);
        }
        acc[r] += a * g.nzval[q];
      }
    }
    std::sort(rows.begin(), rows.end());
    for (int32_t r : rows) {
      if (acc[r] == 0.0) continue;
      if (fill) {
        if (count >= cap) return "output capacity *nnz is too small";
        rowval[count] = r;
        nzval[count] = acc[r];
      }
      ++count;
    }
    if (fill) colptr[j + 1] = count;
  }
  *nnz = count;
  return "";
}

}  // namespace decmg

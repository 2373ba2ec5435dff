// Hierarchy construction: subdivision levels, locality ordering, SELL-64 operators, transfer
// lists, the coarsest dense inverse and device upload.  Host code, compiled with
// -ffp-contract=off so that host sums match the kernels' plain IEEE order.
#include <algorithm>
#include <map>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <stdexcept>

#include "hier.hpp"
#include "solver.hpp"
#include "util.hpp"

namespace decmg {

namespace {

uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t m = 0;
  for (int b = 0; b < 21; ++b) {
    m |= uint64_t((x >> b) & 1u) << (3 * b);
    m |= uint64_t((y >> b) & 1u) << (3 * b + 1);
    m |= uint64_t((z >> b) & 1u) << (3 * b + 2);
  }
  return m;
}

// Internal order of the unknowns.  MORTON: Z-order of the coordinates quantised on a 2^20
// grid of the level's bounding box.  STRIPES: strips one median edge length wide across the
// axis of largest extent, each sorted along the second axis; on a grid this is row-major
// order, so a wavefront's 64 rows are 64 consecutive vertices of one grid row and the
// neighbours in the adjacent rows are consecutive too.  Both orders nest across levels
// (coordinates are kept by subdivision), and the stripes order keeps neighbour offsets small.
void order_level(Level& L, int bc, int order) {
  const Mesh& m = L.mesh;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < m.nv; ++v)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], m.xyz[3 * v + c]);
      hi[c] = std::max(hi[c], m.xyz[3 * v + c]);
    }
  L.bnd_h.clear();
  std::vector<int32_t> unk;
  unk.reserve(m.nv);
  for (int64_t v = 0; v < m.nv; ++v) {
    if (bc == MG_BC_DIRICHLET0 && m.bnd[v])
      L.bnd_h.push_back(int32_t(v));
    else
      unk.push_back(int32_t(v));
  }
  if (order == MG_ORDER_MORTON) {
    std::vector<std::pair<uint64_t, int32_t>> keys;
    keys.reserve(unk.size());
    for (int32_t v : unk) {
      uint32_t q[3];
      for (int c = 0; c < 3; ++c) {
        const double span = hi[c] - lo[c];
        q[c] = span > 0 ? uint32_t(std::floor((m.xyz[3 * v + c] - lo[c]) / span * 1048576.0)) : 0u;
      }
      keys.emplace_back(morton3(q[0], q[1], q[2]), v);
    }
    std::sort(keys.begin(), keys.end());
    for (size_t k = 0; k < keys.size(); ++k) unk[k] = keys[k].second;
  } else {
    int ax[3] = {0, 1, 2};
    std::stable_sort(ax, ax + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
    std::vector<double> len(m.ne);
    for (int64_t e = 0; e < m.ne; ++e) {
      const double* a = &m.xyz[3 * m.edge[2 * e]];
      const double* b = &m.xyz[3 * m.edge[2 * e + 1]];
      len[e] = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                         (b[2] - a[2]) * (b[2] - a[2]));
    }
    std::nth_element(len.begin(), len.begin() + len.size() / 2, len.end());
    const double h = len.empty() ? 1.0 : len[len.size() / 2];
    struct Key {
      int64_t strip;
      double b, c;
      int32_t v;
    };
    std::vector<Key> keys;
    keys.reserve(unk.size());
    for (int32_t v : unk) {
      const double* p = &m.xyz[3 * v];
      keys.push_back({int64_t(std::floor((p[ax[0]] - lo[ax[0]]) / h + 0.5)), p[ax[1]], p[ax[2]], v});
    }
    std::sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
      if (a.strip != b.strip) return a.strip < b.strip;
      if (a.b != b.b) return a.b < b.b;
      if (a.c != b.c) return a.c < b.c;
      return a.v < b.v;
    });
    for (size_t k = 0; k < keys.size(); ++k) unk[k] = keys[k].v;
  }
  L.n = int32_t(unk.size());
  L.perm_h = unk;
  L.inv_h.assign(m.nv, -1);
  for (int32_t k = 0; k < L.n; ++k) L.inv_h[L.perm_h[k]] = k;
}

// Vertex -> incident edges (all edges, CSR).
void vertex_edges(const Mesh& m, std::vector<int64_t>& off, std::vector<int32_t>& inc) {
  off.assign(m.nv + 1, 0);
  for (int64_t e = 0; e < m.ne; ++e) {
    off[m.edge[2 * e] + 1]++;
    off[m.edge[2 * e + 1] + 1]++;
  }
  for (int64_t v = 0; v < m.nv; ++v) off[v + 1] += off[v];
  inc.resize(off[m.nv]);
  std::vector<int64_t> pos(off.begin(), off.end() - 1);
  for (int64_t e = 0; e < m.ne; ++e) {
    inc[pos[m.edge[2 * e]]++] = int32_t(e);
    inc[pos[m.edge[2 * e + 1]]++] = int32_t(e);
  }
}

template <typename T>
T* upload(const std::vector<T>& h) {
  T* d = nullptr;
  if (h.empty()) return nullptr;
  check_hip(hipMalloc(&d, h.size() * sizeof(T)), "hipMalloc");
  check_hip(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  return d;
}

template <typename T>
T* zeros(int64_t n) {
  T* d = nullptr;
  check_hip(hipMalloc(&d, std::max<int64_t>(n, 1) * sizeof(T)), "hipMalloc");
  check_hip(hipMemset(d, 0, std::max<int64_t>(n, 1) * sizeof(T)), "hipMemset");
  return d;
}

// Pads every slice of a SELL-64 layout (`col` per entry, `aux` per entry when not null, slice
// pointers `sptr` in columns) to the widest slice when that adds at most 1/16 of the entries:
// the kernels then compute slice bounds instead of loading them.  Returns the uniform width, or
// -1 (layout unchanged).  Padding entries are `fill_col` / `fill_aux`.
int32_t make_uniform(std::vector<int32_t>& sptr, std::vector<int32_t>& col,
                     std::vector<int32_t>* aux, int32_t fill_col, int32_t fill_aux) {
  const int32_t nslices = int32_t(sptr.size()) - 1;
  if (nslices <= 0) return -1;
  int32_t wmax = 0;
  for (int32_t s = 0; s < nslices; ++s) wmax = std::max(wmax, sptr[s + 1] - sptr[s]);
  const int64_t have = sptr[nslices], want = int64_t(wmax) * nslices;
  if (want - have > have / 16) return -1;
  std::vector<int32_t> c2(size_t(want) * kSlice, fill_col), a2;
  if (aux) a2.assign(size_t(want) * kSlice, fill_aux);
  for (int32_t s = 0; s < nslices; ++s)
    for (int32_t k = 0; k < sptr[s + 1] - sptr[s]; ++k)
      for (int l = 0; l < kSlice; ++l) {
        const size_t from = size_t(sptr[s] + k) * kSlice + l, to = size_t(s * wmax + k) * kSlice + l;
        c2[to] = col[from];
        if (aux) a2[to] = (*aux)[from];
      }
  for (int32_t s = 0; s <= nslices; ++s) sptr[s] = s * wmax;
  col.swap(c2);
  if (aux) aux->swap(a2);
  return wmax;
}

// SELL-64 structure of the operator: per internal row, the couplings with nonzero star1,
// sorted by column; neighbours that are not unknowns point at the zero slot n.
void build_operator_structure(Level& L, std::vector<int32_t>& col) {
  const Mesh& m = L.mesh;
  std::vector<int64_t> off;
  std::vector<int32_t> inc;
  vertex_edges(m, off, inc);
  const int32_t n = L.n;
  const int32_t nslices = (n + kSlice - 1) / kSlice;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> rows(kSlice);
  L.sptr_h.assign(nslices + 1, 0);
  col.clear();
  L.entry_edge.clear();
  for (int32_t s = 0; s < nslices; ++s) {
    int32_t width = 0;
    for (int l = 0; l < kSlice; ++l) {
      rows[l].clear();
      const int32_t r = s * kSlice + l;
      if (r >= n) continue;
      const int32_t v = L.perm_h[r];
      for (int64_t q = off[v]; q < off[v + 1]; ++q) {
        const int32_t e = inc[q];
        if (m.star1[e] == 0.0) continue;
        const int32_t u = m.edge[2 * e] == v ? m.edge[2 * e + 1] : m.edge[2 * e];
        const int32_t c = L.inv_h[u] >= 0 ? L.inv_h[u] : n;
        rows[l].emplace_back(c, e);
      }
      std::sort(rows[l].begin(), rows[l].end());
      width = std::max<int32_t>(width, int32_t(rows[l].size()));
    }
    L.sptr_h[s + 1] = L.sptr_h[s] + width;
    const size_t base = col.size();
    col.resize(base + size_t(width) * kSlice, n);
    L.entry_edge.resize(base + size_t(width) * kSlice, -1);
    for (int l = 0; l < kSlice; ++l)
      for (size_t k = 0; k < rows[l].size(); ++k) {
        col[base + k * kSlice + l] = rows[l][k].first;
        L.entry_edge[base + k * kSlice + l] = rows[l][k].second;
      }
  }
  L.op.uw = make_uniform(L.sptr_h, col, &L.entry_edge, n, -1);
  L.op.nslices = nslices;
  L.op.ncols = L.sptr_h[nslices];
  L.nnz = 0;
  for (int32_t e : L.entry_edge) L.nnz += (e >= 0);
  // one padding column (zero slot, weight 0) so clamped loads past the last slice stay in bounds
  col.resize(col.size() + kSlice, n);
  L.entry_edge.resize(L.entry_edge.size() + kSlice, -1);
}

// 16-bit offsets col - row, with kZeroSlot16 for the zero slot; false if any offset does not
// fit in [-32767, 32767].
bool delta16(const Level& L, const std::vector<int32_t>& col, std::vector<int16_t>& out) {
  out.assign(col.size(), int16_t(kZeroSlot16));
  for (int32_t s = 0; s < L.op.nslices; ++s)
    for (int32_t k = L.sptr_h[s]; k < L.sptr_h[s + 1]; ++k)
      for (int l = 0; l < kSlice; ++l) {
        const size_t i = size_t(k) * kSlice + l;
        const int32_t row = s * kSlice + l;
        if (col[i] == L.n) continue;
        const int32_t d = col[i] - row;
        if (d < -32767 || d > 32767) return false;
        out[i] = int16_t(d);
      }
  return true;
}

// Edge weights w_e = star1_e * (k_lo + k_hi) / 2 for the SELL entries (k = 1 when empty),
// Colour classes of the level's operator for multicolour Gauss-Seidel: unknowns in increasing
// natural vertex id, each taking the smallest colour not used by an already coloured coupled
// unknown (couplings with nonzero star1, as stored in the operator); then each class packed in
// SELL-64 in internal order.
void build_gs_colors(Level& L) {
  const Mesh& m = L.mesh;
  const int32_t n = L.n;
  const int64_t nslices = L.op.nslices;
  // row entries of the operator: (column, edge) per internal row, padding excluded
  std::vector<std::vector<std::pair<int32_t, int32_t>>> rows(n);
  for (int64_t s = 0; s < nslices; ++s)
    for (int32_t k = L.sptr_h[s]; k < L.sptr_h[s + 1]; ++k)
      for (int l = 0; l < kSlice; ++l) {
        const int64_t r = s * kSlice + l;
        if (r >= n) continue;
        const size_t idx = size_t(k) * kSlice + l;
        const int32_t e = L.entry_edge[idx];
        if (e >= 0) rows[r].emplace_back(L.col_h[idx], e);
      }
  std::vector<int32_t> color(n, -1);
  int32_t ncolors = 0;
  std::vector<char> used;
  for (int32_t v = 0; v < int32_t(m.nv); ++v) {
    const int32_t r = L.inv_h[v];
    if (r < 0) continue;
    used.assign(rows[r].size() + 1, 0);
    for (const auto& ce : rows[r]) {
      const int32_t c = ce.first < n ? color[ce.first] : -1;
      if (c >= 0 && c < int32_t(used.size())) used[c] = 1;
    }
    int32_t c = 0;
    while (used[c]) ++c;
    color[r] = c;
    ncolors = std::max(ncolors, c + 1);
  }
  {
    std::vector<int32_t> rc(color.begin(), color.end());
    rc.push_back(0);   // zero slot
    L.row_color = upload(rc);
  }
  L.gs.assign(ncolors, GsColor());
  for (int32_t c = 0; c < ncolors; ++c) {
    GsColor& G = L.gs[c];
    std::vector<int32_t> ids;
    for (int32_t r = 0; r < n; ++r)
      if (color[r] == c) ids.push_back(r);
    G.nrows = int32_t(ids.size());
    G.nslices = (G.nrows + kSlice - 1) / kSlice;
    std::vector<int32_t> sptr(G.nslices + 1, 0), col;
    for (int32_t s = 0; s < G.nslices; ++s) {
      int32_t width = 0;
      for (int l = 0; l < kSlice && s * kSlice + l < G.nrows; ++l)
        width = std::max<int32_t>(width, int32_t(rows[ids[s * kSlice + l]].size()));
      sptr[s + 1] = sptr[s] + width;
      const size_t base = col.size();
      col.resize(base + size_t(width) * kSlice, n);
      G.edge_h.resize(base + size_t(width) * kSlice, -1);
      for (int l = 0; l < kSlice && s * kSlice + l < G.nrows; ++l) {
        const auto& rr = rows[ids[s * kSlice + l]];
        for (size_t k = 0; k < rr.size(); ++k) {
          col[base + k * kSlice + l] = rr[k].first;
          G.edge_h[base + k * kSlice + l] = rr[k].second;
        }
      }
    }
    G.uw = make_uniform(sptr, col, &G.edge_h, n, -1);
    col.resize(col.size() + kSlice, n);   // padding column
    G.edge_h.resize(G.edge_h.size() + kSlice, -1);
    ids.push_back(n);
    G.rowid = upload(ids);
    G.sptr = upload(sptr);
    G.col = upload(col);
  }
}

// row sums in SELL order.
// w = star1 k_e per SELL entry (ke empty: k = 1), and the row sums D
void compute_weights(const Level& L, const std::vector<double>& ke, std::vector<double>& w64,
                     std::vector<float>& w32, std::vector<double>& d64, std::vector<float>& d32) {
  const Mesh& m = L.mesh;
  const size_t ne = L.entry_edge.size();
  w64.assign(ne, 0.0);
  w32.assign(ne, 0.0f);
  for (size_t i = 0; i < ne; ++i) {
    const int32_t e = L.entry_edge[i];
    if (e < 0) continue;
    double w = m.star1[e];
    if (!ke.empty()) w = m.star1[e] * ke[e];
    w64[i] = w;
    w32[i] = static_cast<float>(w);
  }
  d64.assign(L.n + 1, 0.0);
  d32.assign(L.n + 1, 0.0f);
  for (int32_t r = 0; r < L.n; ++r) {
    const int32_t s = r / kSlice, l = r % kSlice;
    double a = 0.0;
    float b = 0.0f;
    for (int32_t k = L.sptr_h[s]; k < L.sptr_h[s + 1]; ++k) {
      a += w64[size_t(k) * kSlice + l];
      b += w32[size_t(k) * kSlice + l];
    }
    d64[r] = a;
    d32[r] = b;
  }
  // zero slot: D = 1 there, so omega * b / D is 0 for the zero slot of b
  d64[L.n] = 1.0;
  d32[L.n] = 1.0f;
}

// Dense inverse of the coarsest operator over its unknowns (Cholesky).  Natural boundaries
// (L singular, kernel = constants): the pseudo-inverse L^+ = (L + 1 1^T / n)^{-1} - 1 1^T / n,
// i.e. the minimum-norm solution, which is zero-mean for any right-hand side.
std::vector<double> coarse_inverse(const Level& L, const std::vector<double>& w64, int bc) {
  const int32_t n = L.n;
  std::vector<double> A(size_t(n) * n, 0.0);
  for (int32_t r = 0; r < n; ++r) {
    const int32_t s = r / kSlice, l = r % kSlice;
    for (int32_t k = L.sptr_h[s]; k < L.sptr_h[s + 1]; ++k) {
      const size_t i = size_t(k) * kSlice + l;
      const int32_t e = L.entry_edge[i];
      if (e < 0) continue;
      const int32_t v = L.perm_h[r];
      const int32_t u = L.mesh.edge[2 * e] == v ? L.mesh.edge[2 * e + 1] : L.mesh.edge[2 * e];
      const int32_t cc = L.inv_h[u];
      A[size_t(r) * n + r] += w64[i];
      if (cc >= 0) A[size_t(r) * n + cc] -= w64[i];
    }
  }
  if (bc == MG_BC_NATURAL)
    for (auto& a : A) a += 1.0 / n;
  // Cholesky A = G G^T (lower G)
  std::vector<double> G(A);
  for (int32_t j = 0; j < n; ++j) {
    double d = G[size_t(j) * n + j];
    for (int32_t k = 0; k < j; ++k) d -= G[size_t(j) * n + k] * G[size_t(j) * n + k];
    if (!(d > 0)) throw std::runtime_error("coarsest operator is not positive definite");
    d = std::sqrt(d);
    G[size_t(j) * n + j] = d;
    for (int32_t i = j + 1; i < n; ++i) {
      double v = G[size_t(i) * n + j];
      for (int32_t k = 0; k < j; ++k) v -= G[size_t(i) * n + k] * G[size_t(j) * n + k];
      G[size_t(i) * n + j] = v / d;
    }
  }
  // inverse column by column: solve G y = e_c, G^T x = y
  std::vector<double> inv(size_t(n) * n, 0.0), y(n);
  for (int32_t c = 0; c < n; ++c) {
    for (int32_t i = 0; i < n; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int32_t k = 0; k < i; ++k) v -= G[size_t(i) * n + k] * y[k];
      y[i] = v / G[size_t(i) * n + i];
    }
    for (int32_t i = n - 1; i >= 0; --i) {
      double v = y[i];
      for (int32_t k = i + 1; k < n; ++k) v -= G[size_t(k) * n + i] * inv[size_t(k) * n + c];
      inv[size_t(i) * n + c] = v / G[size_t(i) * n + i];
    }
  }
  if (bc == MG_BC_NATURAL)
    for (auto& a : inv) a -= 1.0 / n;
  return inv;
}

// Weighted transfers for a level made by any subdivision (used for cubic levels): three
// (parent, weight) pairs per fine unknown, and per coarse unknown the list of fine unknowns
// whose interpolation row names it, with that weight.
void build_transfer_weighted(Level& F, const Level& C) {
  F.tr.weighted = true;
  std::vector<int32_t> p3(3 * size_t(F.n + 1), C.n);
  std::vector<double> w64(3 * size_t(F.n + 1), 0.0);
  std::vector<std::vector<std::pair<int32_t, double>>> rows(C.n);
  for (int32_t k = 0; k < F.n; ++k) {
    const int32_t v = F.perm_h[k];
    for (int q = 0; q < 3; ++q) {
      const int32_t a = F.mesh.parent3[3 * v + q];
      const double w = F.mesh.pweight[3 * v + q];
      const int32_t ca = C.inv_h[a];
      p3[3 * k + q] = ca >= 0 ? ca : C.n;
      w64[3 * k + q] = ca >= 0 ? w : 0.0;
      if (ca >= 0 && w != 0.0) rows[ca].emplace_back(k, w);
    }
  }
  std::vector<float> w32(w64.begin(), w64.end());
  const int32_t nslices = (C.n + kSlice - 1) / kSlice;
  std::vector<int32_t> sptr(nslices + 1, 0), col;
  std::vector<double> rw;
  for (int32_t s = 0; s < nslices; ++s) {
    int32_t width = 0;
    for (int l = 0; l < kSlice && s * kSlice + l < C.n; ++l) {
      std::sort(rows[s * kSlice + l].begin(), rows[s * kSlice + l].end());
      width = std::max<int32_t>(width, int32_t(rows[s * kSlice + l].size()));
    }
    sptr[s + 1] = sptr[s] + width;
    const size_t base = col.size();
    col.resize(base + size_t(width) * kSlice, F.n);
    rw.resize(base + size_t(width) * kSlice, 0.0);
    for (int l = 0; l < kSlice && s * kSlice + l < C.n; ++l) {
      const auto& rr = rows[s * kSlice + l];
      for (size_t k = 0; k < rr.size(); ++k) {
        col[base + k * kSlice + l] = rr[k].first;
        rw[base + k * kSlice + l] = rr[k].second;
      }
    }
  }
  col.resize(col.size() + kSlice, F.n);   // padding column
  rw.resize(rw.size() + kSlice, 0.0);
  std::vector<float> rw32(rw.begin(), rw.end());
  F.tr.p3 = upload(p3);
  F.tr.pw64 = upload(w64);
  F.tr.pw32 = upload(w32);
  F.tr.nslices = nslices;
  F.tr.ncols = sptr[nslices];
  F.tr.rw_sptr = upload(sptr);
  F.tr.rw_col = upload(col);
  F.tr.rw64 = upload(rw);
  F.tr.rw32 = upload(rw32);
}

void build_transfer(Level& F, const Level& C) {
  if (F.mesh.scheme != 1) {
    build_transfer_weighted(F, C);
    return;
  }
  // interpolation: two coarse parents per fine unknown (zero slot for non-unknowns)
  std::vector<int32_t> pa(F.n + 1, C.n), pb(F.n + 1, C.n);
  for (int32_t k = 0; k < F.n; ++k) {
    const int32_t v = F.perm_h[k];
    const int32_t a = F.mesh.parent[2 * v], b = F.mesh.parent[2 * v + 1];
    pa[k] = C.inv_h[a] >= 0 ? C.inv_h[a] : C.n;
    pb[k] = C.inv_h[b] >= 0 ? C.inv_h[b] : C.n;
  }
  // restriction rows: kept vertex + midpoints of all incident coarse edges
  std::vector<int64_t> off;
  std::vector<int32_t> inc;
  vertex_edges(C.mesh, off, inc);
  std::vector<int32_t> self(C.n + 1, F.n);
  const int32_t nslices = (C.n + kSlice - 1) / kSlice;
  std::vector<int32_t> sptr(nslices + 1, 0), col;
  std::vector<std::vector<int32_t>> rows(kSlice);
  for (int32_t s = 0; s < nslices; ++s) {
    int32_t width = 0;
    for (int l = 0; l < kSlice; ++l) {
      rows[l].clear();
      const int32_t r = s * kSlice + l;
      if (r >= C.n) continue;
      const int32_t v = C.perm_h[r];
      self[r] = F.inv_h[v];
      for (int64_t q = off[v]; q < off[v + 1]; ++q) {
        const int32_t mid = int32_t(C.mesh.nv + inc[q]);
        if (F.inv_h[mid] >= 0) rows[l].push_back(F.inv_h[mid]);
      }
      std::sort(rows[l].begin(), rows[l].end());
      width = std::max<int32_t>(width, int32_t(rows[l].size()));
    }
    sptr[s + 1] = sptr[s] + width;
    const size_t base = col.size();
    col.resize(base + size_t(width) * kSlice, F.n);
    for (int l = 0; l < kSlice; ++l)
      for (size_t k = 0; k < rows[l].size(); ++k) col[base + k * kSlice + l] = rows[l][k];
  }
  F.tr.r_uw = make_uniform(sptr, col, nullptr, F.n, 0);
  col.resize(col.size() + kSlice, F.n);   // padding column
  F.tr.pa = upload(pa);
  F.tr.pb = upload(pb);
  // The packed forms below can be switched off (DECMG_NO_PACKED_TRANSFERS set) so that the
  // int32 kernels, used where offsets do not fit, can be checked against them.
  const bool no_pack = std::getenv("DECMG_NO_PACKED_TRANSFERS") != nullptr;
  if (!no_pack) {
    // packed parents: int16 offsets from the smallest parent id in each 64-row slice
    const int32_t ns = (F.n + kSlice - 1) / kSlice;
    std::vector<int32_t> base(size_t(std::max(ns, 1)), 0);
    std::vector<uint32_t> ab(size_t(F.n) + 1, 0u);
    bool fits = true;
    for (int32_t s = 0; s < ns && fits; ++s) {
      const int32_t r0 = s * kSlice, r1 = std::min(F.n, r0 + kSlice);
      int32_t lo = C.n;
      for (int32_t r = r0; r < r1; ++r) {
        if (pa[r] != C.n) lo = std::min(lo, pa[r]);
        if (pb[r] != C.n) lo = std::min(lo, pb[r]);
      }
      base[s] = lo;
      auto enc = [&](int32_t p, uint32_t& out) {
        if (p == C.n) {
          out = uint16_t(int16_t(kZeroSlot16));
          return true;
        }
        const int32_t off = p - lo;
        if (off < 0 || off > 32767) return false;
        out = uint16_t(off);
        return true;
      };
      for (int32_t r = r0; r < r1 && fits; ++r) {
        uint32_t ea = 0, eb = 0;
        fits = enc(pa[r], ea) && enc(pb[r], eb);
        ab[r] = ea | (eb << 16);
      }
    }
    if (fits && F.n > 0) {
      F.tr.p_base = upload(base);
      F.tr.p_ab16 = upload(ab);
    }
  }
  F.tr.r_self = upload(self);
  F.tr.nslices = nslices;
  F.tr.ncols = sptr[nslices];
  F.tr.r_sptr = upload(sptr);
  F.tr.r_col = upload(col);
  // 16-bit offsets from the kept vertex for the per-step restriction (uniform widths 1..8)
  if (!no_pack && F.tr.r_uw >= 1 && F.tr.r_uw <= 8) {
    const int32_t uw = F.tr.r_uw;
    std::vector<int16_t> c16(size_t(nslices) * uw * kSlice, int16_t(kZeroSlot16));
    bool fits = true;
    for (int32_t r = 0; r < C.n && fits; ++r)
      for (int32_t k = 0; k < uw; ++k) {
        const size_t at = size_t(r >> 6) * uw * kSlice + size_t(k) * kSlice + (r & 63);
        const int32_t c = col[at];
        if (c == F.n) continue;
        const int64_t off = int64_t(c) - self[r];
        if (off <= kZeroSlot16 || off > 32767) {
          fits = false;
          break;
        }
        c16[at] = int16_t(off);
      }
    if (fits) F.tr.r_col16 = upload(c16);
  }
}

template <typename T>
void alloc_vecs(LevelVecs<T>& V, int32_t n) {
  V.x = zeros<T>(n + 1);
  V.b = zeros<T>(n + 1);
  V.r = zeros<T>(n + 1);
  V.t = zeros<T>(n + 1);
  V.u = zeros<T>(n + 1);
}

void free_dev(void* p) {
  if (p) (void)hipFree(p);
}

template <typename T>
const T* level_weights(const Level& L);
template <>
const double* level_weights<double>(const Level& L) { return L.op.w64; }
template <>
const float* level_weights<float>(const Level& L) { return L.op.w32; }
template <typename T>
const T* level_idiag(const Level& L);
template <>
const double* level_idiag<double>(const Level& L) { return L.op.idiag64; }
template <>
const float* level_idiag<float>(const Level& L) { return L.op.idiag32; }

// Descriptors of the levels that fit the fused coarse cycle's LDS budget.  The LDS holds,
// for levels 0..ctop, x, partner and b (3 (n+1) values each), then the dense coarsest inverse
// (n0^2 doubles), then the operator and restriction slice bounds of every level; ctop is the
// highest level for which all of it fits, or -1 when even level 1 does not.
template <typename T>
void build_coarse_levels(Hierarchy& H, CoarseLevel<T>*& dev, int& ctop, std::vector<int32_t>& lds,
                         size_t& int_off, size_t& total) {
  const int nl = int(H.lv.size());
  std::vector<CoarseLevel<T>> hv(nl);
  lds.assign(nl, 0);
  ctop = -1;
  size_t vec = 0, ints = 0;
  const size_t inv_bytes = size_t(H.lv[0]->n) * H.lv[0]->n * sizeof(double);
  for (int l = 0; l < nl; ++l) {
    const Level& L = *H.lv[l];
    const size_t vec2 = vec + 3 * size_t(L.n + 1) * sizeof(T);
    const size_t ints2 = ints + size_t(L.op.nslices + 1) + (l >= 1 ? size_t(L.tr.nslices + 1) : 0);
    const size_t off2 = (vec2 + 7) / 8 * 8 + inv_bytes;
    if (off2 + ints2 * sizeof(int32_t) > size_t(H.lds_limit)) break;
    if (L.n > kCoarseFuseRows) break;
    if (l >= 1 && L.tr.weighted) break;   // the fused cycle implements the binary transfers
    CoarseLevel<T>& c = hv[l];
    c.n = L.n;
    c.lds = int32_t(vec / sizeof(T));
    c.nslices = L.op.nslices;
    c.lds_sptr = int32_t(ints);
    c.sptr = L.op.sptr;
    c.col = L.op.col;
    c.w = level_weights<T>(L);
    c.idiag = level_idiag<T>(L);
    c.color = L.row_color;
    c.ncolors = int32_t(L.gs.size());
    if (l >= 1) {
      c.pa = L.tr.pa;
      c.pb = L.tr.pb;
      c.r_self = L.tr.r_self;
      c.r_sptr = L.tr.r_sptr;
      c.r_col = L.tr.r_col;
      c.r_nslices = L.tr.nslices;
      c.lds_rsptr = int32_t(ints + L.op.nslices + 1);
    }
    lds[l] = c.lds;
    vec = vec2;
    ints = ints2;
    int_off = (vec + 7) / 8 * 8 + inv_bytes;
    total = int_off + ints * sizeof(int32_t);
    ctop = l;
    for (int32_t s = 0; s < L.op.nslices; ++s)
      H.coarse_width = std::max(H.coarse_width, L.sptr_h[s + 1] - L.sptr_h[s]);
    H.coarse_rows = std::max(H.coarse_rows, L.n);
    c.uw = L.op.uw;
    if (l >= 1) {
      c.r_uw = L.tr.r_uw;
      std::vector<int32_t> rs(L.tr.nslices + 1);
      check_hip(hipMemcpy(rs.data(), L.tr.r_sptr, rs.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost), "hipMemcpy");
      for (int32_t s = 0; s < L.tr.nslices; ++s)
        H.coarse_rwidth = std::max(H.coarse_rwidth, rs[s + 1] - rs[s]);
    }
  }
  if (ctop < 1) ctop = -1;
  dev = upload(hv);
}

template <typename T>
std::vector<T> download(const T* d, size_t n) {
  std::vector<T> h(n);
  if (n) check_hip(hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost), "hipMemcpy");
  return h;
}

// Workgroup tiles of the fused smoothing kernels of level F over its coarse level C (see
// DevTiles), on levels of at most kLaunchBoundRows rows, with binary or weighted transfers.  Leaves F.tiles empty when a row
// or restriction list is wider than 8 or a tile's rings exceed 2 kTileThreads rows; the level
// then runs one kernel per step.  (Tiles of 4096 rows on the larger C3 levels, with 1.15x
// rings, were measured slower than the streaming per-step kernels there.)
void build_tiles(Level& F, const Level& C) {
  const int32_t n = F.n, nc = C.n;
  if (n == 0 || nc == 0 || n > kLaunchBoundRows) return;
  const bool wtr = F.tr.weighted;
  const int32_t fb = kBlock;                 // owned rows per tile at most
  const int32_t capmax = 2 * kTileThreads, ccapmax = kTileThreads;
  const int32_t nsl = int32_t(F.sptr_h.size()) - 1;
  int32_t wmax = 0;
  for (int32_t s = 0; s < nsl; ++s) wmax = std::max(wmax, F.sptr_h[s + 1] - F.sptr_h[s]);
  if (wmax > 8) return;
  const int kt = wmax <= 4 ? 4 : 8;
  // restriction lists (device layout).  Binary levels: the kept vertex plus up to 8 midpoints
  // (weight 1/2); weighted levels: (fine row, weight) entries in SELL order.  Every coarse row
  // has an anchor fine row, and the tile holding the anchor restricts it: the kept vertex, or
  // the entry of largest weight (a row without entries goes to the first tile, which writes
  // its zero).
  std::vector<int32_t> self, rsptr, rcol;
  std::vector<double> rwt;
  if (wtr) {
    rsptr = download(F.tr.rw_sptr, size_t(F.tr.nslices) + 1);
    rcol = download(F.tr.rw_col, size_t(rsptr.back() + 1) * kSlice);
    rwt = download(F.tr.rw64, rcol.size());
  } else {
    self = download(F.tr.r_self, size_t(nc) + 1);
    rsptr = download(F.tr.r_sptr, size_t(F.tr.nslices) + 1);
    rcol = download(F.tr.r_col, size_t(rsptr.back() + 1) * kSlice);
  }
  auto rwidth = [&](int32_t c) { return rsptr[c / kSlice + 1] - rsptr[c / kSlice]; };
  auto ridx = [&](int32_t c, int k) {
    return size_t(rsptr[c / kSlice] + k) * kSlice + size_t(c % kSlice);
  };
  auto rentry = [&](int32_t c, int k) { return rcol[ridx(c, k)]; };
  int32_t rws = 9;   // local id slots per owned coarse row
  std::vector<int32_t> anchor(nc, -1);
  for (int32_t c = 0; c < nc; ++c) {
    if (rwidth(c) > (wtr ? 63 : 8)) return;
    if (!wtr) {
      if (self[c] < 0 || self[c] >= n)
        throw std::logic_error("restriction: kept vertex out of range");
      anchor[c] = self[c];
      continue;
    }
    rws = std::max(rws, rwidth(c));
    double best = 0.0;
    for (int k = 0; k < rwidth(c); ++k)
      if (rentry(c, k) < n && (anchor[c] < 0 || rwt[ridx(c, k)] > best)) {
        anchor[c] = rentry(c, k);
        best = rwt[ridx(c, k)];
      }
  }
  // Morton order of the rows on a lattice of the median edge length h: on a grid the rows get
  // their lattice coordinates, so runs of fb consecutive rows are aligned square patches
  double lo[3] = {1e300, 1e300, 1e300};
  for (int32_t r = 0; r < n; ++r)
    for (int c = 0; c < 3; ++c) lo[c] = std::min(lo[c], F.mesh.xyz[3 * size_t(F.perm_h[r]) + c]);
  double h = 1.0;
  {
    const Mesh& m = F.mesh;
    std::vector<double> len(m.ne);
    for (int64_t e = 0; e < m.ne; ++e) {
      const double* a = &m.xyz[3 * m.edge[2 * e]];
      const double* b = &m.xyz[3 * m.edge[2 * e + 1]];
      len[e] = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                         (b[2] - a[2]) * (b[2] - a[2]));
    }
    if (!len.empty()) {
      std::nth_element(len.begin(), len.begin() + len.size() / 2, len.end());
      if (len[len.size() / 2] > 0) h = len[len.size() / 2];
    }
  }
  std::vector<std::pair<uint64_t, int32_t>> key(n);
  for (int32_t r = 0; r < n; ++r) {
    uint32_t q[3];
    for (int c = 0; c < 3; ++c) {
      const double u = (F.mesh.xyz[3 * size_t(F.perm_h[r]) + c] - lo[c]) / h + 0.5;
      q[c] = uint32_t(std::min(2097151.0, std::max(0.0, std::floor(u))));
    }
    key[r] = {morton3(q[0], q[1], q[2]), r};
  }
  std::sort(key.begin(), key.end());
  auto width = [&](int32_t r) { return F.sptr_h[r / kSlice + 1] - F.sptr_h[r / kSlice]; };
  auto entry = [&](int32_t r, int k) {   // SELL index of entry k of row r
    return size_t(F.sptr_h[r / kSlice] + k) * kSlice + size_t(r % kSlice);
  };
  // tiles: runs of the Morton order inside one aligned lattice block of 16 x 16 (x 16) cells,
  // cut further every fb rows
  const int shift = 12;
  std::vector<int32_t> tstart;
  for (int32_t i = 0; i < n; ++i)
    if (i == 0 || (key[i].first >> shift) != (key[i - 1].first >> shift) ||
        i - tstart.back() == fb)
      tstart.push_back(i);
  tstart.push_back(n);
  const int32_t ntiles = int32_t(tstart.size()) - 1;
  // the coarse rows of every tile, by anchor
  std::vector<std::vector<int32_t>> trows(ntiles), tcown(ntiles);
  {
    std::vector<int32_t> tile_of(n, 0);
    for (int32_t b = 0; b < ntiles; ++b)
      for (int32_t i = tstart[b]; i < tstart[b + 1]; ++i) tile_of[key[i].second] = b;
    for (int32_t c = 0; c < nc; ++c) tcown[anchor[c] >= 0 ? tile_of[anchor[c]] : 0].push_back(c);
  }
  // pass 1: the rings of every tile
  std::vector<std::array<int32_t, 5>> cnt(ntiles);   // nF, n0, n1, n2, ncb
  std::vector<int32_t> lid(n, -1), fresh;
  int32_t cap = 0, ccap = 0;
  for (int32_t b = 0; b < ntiles; ++b) {
    std::vector<int32_t>& rows = trows[b];
    auto add_group = [&]() {
      std::sort(fresh.begin(), fresh.end());
      fresh.erase(std::unique(fresh.begin(), fresh.end()), fresh.end());
      for (int32_t r : fresh)
        if (lid[r] < 0) {
          lid[r] = int32_t(rows.size());
          rows.push_back(r);
        }
      fresh.clear();
    };
    const int32_t r0 = tstart[b], r1 = tstart[b + 1];
    for (int32_t i = r0; i < r1; ++i) fresh.push_back(key[i].second);
    add_group();
    const int32_t nF = int32_t(rows.size());
    const std::vector<int32_t>& cown = tcown[b];
    for (int32_t c : cown)
      for (int k = 0; k < rwidth(c); ++k)
        if (rentry(c, k) < n) fresh.push_back(rentry(c, k));
    add_group();
    const int32_t n0 = int32_t(rows.size());
    auto ring = [&](int32_t upto) {
      for (int32_t i = 0; i < upto; ++i)
        for (int k = 0; k < width(rows[i]); ++k) {
          const int32_t j = F.col_h[entry(rows[i], k)];
          if (j < n) fresh.push_back(j);
        }
      add_group();
    };
    ring(n0);
    const int32_t n1 = int32_t(rows.size());
    ring(n1);
    const int32_t n2 = int32_t(rows.size());
    for (int32_t r : rows) lid[r] = -1;
    cnt[b] = {nF, n0, n1, n2, int32_t(cown.size())};
    cap = std::max(cap, n2);
    ccap = std::max(ccap, int32_t(cown.size()));
  }
  cap = (cap + 63) / 64 * 64;
  ccap = std::max(64, (ccap + 63) / 64 * 64);
  if (cap > capmax || ccap > ccapmax) return;   // not compact: per-step kernels
  // pass 2: fixed-capacity arrays (padding: the tile's first row / coarse row, zero slot cap)
  const bool uniform = F.op.uw >= 0;
  std::vector<int32_t> meta(size_t(ntiles) * 8, 0), trow(size_t(ntiles) * cap),
      tent(uniform ? 0 : size_t(ntiles) * cap), tcrow(size_t(ntiles) * ccap, 0);
  std::vector<int16_t> tcol(size_t(ntiles) * kt * cap, int16_t(cap)),
      tcst(size_t(ntiles) * rws * ccap, int16_t(cap));
  std::vector<int32_t> tcent(wtr ? size_t(ntiles) * ccap : 0, 0);
  std::vector<char> fine_seen(n, 0), coarse_seen(nc, 0);
  for (int32_t b = 0; b < ntiles; ++b) {
    const std::vector<int32_t>& rows = trows[b];
    const std::vector<int32_t>& cown = tcown[b];
    const auto [nF, n0, n1, n2, ncb] = cnt[b];
    (void)n0;
    for (int q = 0; q < 5; ++q) meta[size_t(b) * 8 + q] = cnt[b][q];
    for (int32_t i = 0; i < n2; ++i) lid[rows[i]] = i;
    for (int32_t i = 0; i < cap; ++i) {
      const int32_t r = rows[i < n2 ? i : 0];
      trow[size_t(b) * cap + i] = r;
      if (!uniform) {
        const size_t e0 = entry(r, 0);
        if (e0 >= (size_t(1) << 27)) throw std::logic_error("tiles: entry index overflow");
        tent[size_t(b) * cap + i] = int32_t(e0 << 4) | width(r);
      }
    }
    for (int k = 0; k < kt; ++k)
      for (int32_t i = 0; i < n1; ++i) {
        const int32_t r = rows[i];
        if (k >= width(r)) continue;
        const int32_t j = F.col_h[entry(r, k)];
        tcol[(size_t(b) * kt + k) * cap + i] = int16_t(j < n ? lid[j] : cap);
      }
    for (int32_t j = 0; j < ccap; ++j) tcrow[size_t(b) * ccap + j] = ncb ? cown[j < ncb ? j : 0] : 0;
    for (int32_t j = 0; j < ncb; ++j) {
      const int32_t c = cown[j];
      // binary: slot 0 the kept vertex, slots 1.. the midpoints; weighted: slot k entry k
      const int off = wtr ? 0 : 1;
      if (!wtr) tcst[size_t(b) * rws * ccap + j] = int16_t(lid[self[c]]);
      for (int k = 0; k < rwidth(c); ++k)
        tcst[(size_t(b) * rws + k + off) * ccap + j] =
            int16_t(rentry(c, k) < n ? lid[rentry(c, k)] : cap);
      if (wtr) {
        const size_t e0 = ridx(c, 0);
        if (e0 >= (size_t(1) << 25)) throw std::logic_error("tiles: restriction index overflow");
        tcent[size_t(b) * ccap + j] = int32_t(e0 << 6) | rwidth(c);
      }
      coarse_seen[c]++;
    }
    for (int32_t i = 0; i < nF; ++i) fine_seen[rows[i]]++;
    for (int32_t r : rows) lid[r] = -1;
  }
  // every fine row is written by one tile, every coarse row restricted by one, and every
  // local id stays inside the tile's LDS rows or names its zero slot
  for (int32_t r = 0; r < n; ++r)
    if (fine_seen[r] != 1) throw std::logic_error("tiles: fine rows not partitioned");
  for (int32_t c = 0; c < nc; ++c)
    if (coarse_seen[c] != 1) throw std::logic_error("tiles: coarse rows not partitioned");
  for (int16_t v : tcol)
    if (v < 0 || v > cap) throw std::logic_error("tiles: local column out of range");
  for (int16_t v : tcst)
    if (v < 0 || v > cap) throw std::logic_error("tiles: local restriction id out of range");
  for (int32_t r : trow)
    if (r < 0 || r >= n) throw std::logic_error("tiles: row id out of range");
  for (int32_t c : tcrow)
    if (c < 0 || c >= nc) throw std::logic_error("tiles: coarse row id out of range");
  DevTiles& T = F.tiles;
  T.ntiles = ntiles;
  T.kt = kt;
  T.cap = cap;
  T.ccap = ccap;
  T.rows_total = 0;
  for (const auto& c : cnt) T.rows_total += c[3];
  T.meta = upload(meta);
  T.row = upload(trow);
  T.ent = uniform ? nullptr : upload(tent);
  T.col = upload(tcol);
  T.crow = upload(tcrow);
  T.cst = upload(tcst);
  T.rws = rws;
  T.cent = wtr ? upload(tcent) : nullptr;
}

// The IEEE binary16 encoding of v when v is exactly a binary16 number (zero, normal or
// subnormal); false otherwise.
bool half_exact(double v, uint16_t& h) {
  const float f = static_cast<float>(v);
  if (static_cast<double>(f) != v || !std::isfinite(f)) return false;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t s = (u >> 31) << 15, ef = (u >> 23) & 0xffu, mf = u & 0x7fffffu;
  if (ef == 0 && mf == 0) {   // signed zero
    h = uint16_t(s);
    return true;
  }
  if (ef == 0) return false;  // FP32 subnormals are below the binary16 range
  const int e = int(ef) - 127;
  if (e >= -14 && e <= 15) {  // binary16 normal: 10 fraction bits
    if (mf & 0x1fffu) return false;
    h = uint16_t(s | uint32_t(e + 15) << 10 | (mf >> 13));
    return true;
  }
  if (e >= -24 && e < -14) {  // binary16 subnormal: value = frac * 2^-24
    const uint32_t sig = (1u << 23) | mf;
    const int sh = -(e + 1);
    if (sig & ((1u << sh) - 1u)) return false;
    h = uint16_t(s | (sig >> sh));
    return true;
  }
  return false;
}

}  // namespace

// The form of the weights each row kernel reads (binary16, FP32 or FP64 copy) is chosen when
// the kernel is enqueued, so a captured graph keeps the choice of its capture.  Returns one bit
// per exactness flag of every level and colour class.
static std::vector<bool> weight_forms(const Hierarchy& H) {
  std::vector<bool> f;
  for (const auto& Lp : H.lv) {
    f.push_back(Lp->op.w_exact16);
    f.push_back(Lp->op.w_exact32);
    f.push_back(Lp->op.npat > 0);
    for (const GsColor& G : Lp->gs) f.push_back(G.w_exact32);
  }
  return f;
}

std::vector<double> level_edge_coeff(const Hierarchy& H, size_t l) {
  if (!H.kedge_h.empty()) return H.kedge_h[l];
  std::vector<double> ke;
  if (H.kvert_h.empty()) return ke;
  const Mesh& m = H.lv[l]->mesh;
  ke.resize(size_t(m.ne));
  for (int64_t e = 0; e < m.ne; ++e)
    ke[e] = 0.5 * (H.kvert_h[m.edge[2 * e]] + H.kvert_h[m.edge[2 * e + 1]]);
  return ke;
}

std::vector<std::vector<double>> coarsen_edge_coeff(const Hierarchy& H, std::vector<double> ke) {
  std::vector<std::vector<double>> out(H.lv.size());
  for (size_t l = H.lv.size(); l-- > 0;) {
    out[l] = ke;
    if (l == 0) break;
    const Mesh& f = H.lv[l]->mesh;
    const Mesh& c = H.lv[l - 1]->mesh;
    // vertex -> incident edges of the fine mesh, to find an edge from its endpoints
    std::vector<int64_t> vptr(size_t(f.nv) + 1, 0);
    for (int64_t e = 0; e < f.ne; ++e) {
      ++vptr[size_t(f.edge[2 * e]) + 1];
      ++vptr[size_t(f.edge[2 * e + 1]) + 1];
    }
    for (int64_t v = 0; v < f.nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int32_t> vinc(static_cast<size_t>(vptr[f.nv]));
    std::vector<int64_t> pos(vptr.begin(), vptr.end() - 1);
    for (int64_t e = 0; e < f.ne; ++e) {
      vinc[pos[f.edge[2 * e]]++] = int32_t(e);
      vinc[pos[f.edge[2 * e + 1]]++] = int32_t(e);
    }
    auto eid = [&](int32_t a, int32_t b) {
      for (int64_t k = vptr[a]; k < vptr[a + 1]; ++k) {
        const int32_t e = vinc[k];
        if (f.edge[2 * e] + f.edge[2 * e + 1] - a == b) return e;
      }
      throw std::logic_error("subdivision edge not found");
    };
    const int32_t nc = int32_t(c.nv);
    std::vector<double> kc(size_t(c.ne));
    for (int64_t e = 0; e < c.ne; ++e) {
      const int32_t a = c.edge[2 * e], b = c.edge[2 * e + 1];
      if (f.scheme == 2) {
        const int32_t p1 = nc + int32_t(2 * e), p2 = p1 + 1;
        kc[e] = (ke[eid(a, p1)] + ke[eid(p1, p2)] + ke[eid(p2, b)]) / 3.0;
      } else {
        const int32_t mid = nc + int32_t(e);
        kc[e] = 0.5 * (ke[eid(a, mid)] + ke[eid(mid, b)]);
      }
    }
    ke = std::move(kc);
  }
  return out;
}

// Row patterns of a level of uniform width (see DevOperator): the distinct sequences of
// (16-bit offset, FP64 weight) over a row's entries, numbered in order of first appearance.
// Used when there are at most kMaxRowPatterns of them (npat > 0); otherwise npat = 0.  The
// device arrays are allocated once at their largest size and rewritten in place, so graphs
// captured with them stay valid while the level keeps using patterns.
static void build_row_patterns(Level& L, const std::vector<double>& w64) {
  L.op.npat = 0;
  const int32_t n = L.n, uw = L.op.uw;
  if (n == 0 || uw < 1 || uw > 8 || !L.op.col16 || std::getenv("DECMG_NO_ROW_PATTERNS")) return;
  std::map<std::vector<uint64_t>, int32_t> ids;
  std::vector<uint8_t> pat(static_cast<size_t>(n));
  std::vector<int16_t> poff;
  std::vector<double> pw;
  std::vector<uint64_t> key(2 * size_t(uw));
  for (int32_t r = 0; r < n; ++r) {
    const size_t e0 = size_t(r / kSlice) * uw * kSlice + size_t(r % kSlice);
    for (int k = 0; k < uw; ++k) {
      const size_t i = e0 + size_t(k) * kSlice;
      const int32_t c = L.col_h[i];
      const int32_t off = c == n ? kZeroSlot16 : c - r;
      uint64_t bits;
      std::memcpy(&bits, &w64[i], 8);
      key[2 * k] = uint64_t(uint32_t(off));
      key[2 * k + 1] = bits;
    }
    auto it = ids.find(key);
    if (it == ids.end()) {
      if (int32_t(ids.size()) == kMaxRowPatterns) return;
      it = ids.emplace(key, int32_t(ids.size())).first;
      for (int k = 0; k < uw; ++k) {
        poff.push_back(int16_t(int32_t(key[2 * k])));
        pw.push_back(w64[e0 + size_t(k) * kSlice]);
      }
    }
    pat[r] = uint8_t(it->second);
  }
  const std::vector<float> pw32(pw.begin(), pw.end());
  if (!L.op.pat) {
    L.op.pat = zeros<uint8_t>(n);
    L.op.poff = zeros<int16_t>(int64_t(kMaxRowPatterns) * uw);
    L.op.pw32 = zeros<float>(int64_t(kMaxRowPatterns) * uw);
    L.op.pw64 = zeros<double>(int64_t(kMaxRowPatterns) * uw);
  }
  check_hip(hipMemcpy(L.op.pat, pat.data(), pat.size(), hipMemcpyHostToDevice), "hipMemcpy");
  check_hip(hipMemcpy(L.op.poff, poff.data(), poff.size() * 2, hipMemcpyHostToDevice), "hipMemcpy");
  check_hip(hipMemcpy(L.op.pw32, pw32.data(), pw32.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
  check_hip(hipMemcpy(L.op.pw64, pw.data(), pw.size() * 8, hipMemcpyHostToDevice), "hipMemcpy");
  L.op.npat = int32_t(ids.size());
}

void upload_weights(Hierarchy& H) {
  const std::vector<bool> forms_before = weight_forms(H);
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = *H.lv[l];
    std::vector<double> w64, d64;
    std::vector<float> w32, d32;
    const std::vector<double> ke = level_edge_coeff(H, l);
    compute_weights(L, ke, w64, w32, d64, d32);
    build_row_patterns(L, w64);
    if (!L.op.w64) {
      L.op.w64 = zeros<double>(std::max<size_t>(w64.size(), 1));
      L.op.w32 = zeros<float>(std::max<size_t>(w32.size(), 1));
      L.op.idiag64 = zeros<double>(L.n + 1);
      L.op.idiag32 = zeros<float>(L.n + 1);
    }
    L.op.w_exact32 = true;
    for (size_t i = 0; i < w64.size(); ++i)
      if (static_cast<double>(w32[i]) != w64[i]) {
        L.op.w_exact32 = false;
        break;
      }
    std::vector<uint16_t> w16(w64.size());
    L.op.w_exact16 = !w64.empty();
    for (size_t i = 0; i < w64.size() && L.op.w_exact16; ++i)
      L.op.w_exact16 = half_exact(w64[i], w16[i]);
    if (!L.op.w16) L.op.w16 = zeros<uint16_t>(std::max<size_t>(w64.size(), 1));
    if (!w64.empty()) {
      check_hip(hipMemcpy(L.op.w64, w64.data(), w64.size() * 8, hipMemcpyHostToDevice), "hipMemcpy");
      check_hip(hipMemcpy(L.op.w32, w32.data(), w32.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
      if (L.op.w_exact16)
        check_hip(hipMemcpy(L.op.w16, w16.data(), w16.size() * 2, hipMemcpyHostToDevice),
                  "hipMemcpy");
    }
    {
      std::vector<double> i64(d64.size());
      std::vector<float> i32(d32.size());
      for (size_t i = 0; i < d64.size(); ++i) {
        i64[i] = 1.0 / d64[i];
        i32[i] = 1.0f / d32[i];
      }
      check_hip(hipMemcpy(L.op.idiag64, i64.data(), i64.size() * 8, hipMemcpyHostToDevice),
                "hipMemcpy");
      check_hip(hipMemcpy(L.op.idiag32, i32.data(), i32.size() * 4, hipMemcpyHostToDevice),
                "hipMemcpy");
    }
    // weights of the Gauss-Seidel colour classes: w = star1 k_e per entry, as for the operator
    for (GsColor& G : L.gs) {
      std::vector<double> g64(G.edge_h.size(), 0.0);
      std::vector<float> g32(G.edge_h.size(), 0.0f);
      G.w_exact32 = true;
      for (size_t i = 0; i < G.edge_h.size(); ++i) {
        const int32_t e = G.edge_h[i];
        if (e < 0) continue;
        const Mesh& m = L.mesh;
        double w = m.star1[e];
        if (!ke.empty()) w = m.star1[e] * ke[e];
        g64[i] = w;
        g32[i] = static_cast<float>(w);
        if (static_cast<double>(g32[i]) != w) G.w_exact32 = false;
      }
      if (!G.w64) {
        G.w64 = zeros<double>(std::max<size_t>(g64.size(), 1));
        G.w32 = zeros<float>(std::max<size_t>(g32.size(), 1));
      }
      if (!g64.empty()) {
        check_hip(hipMemcpy(G.w64, g64.data(), g64.size() * 8, hipMemcpyHostToDevice), "hipMemcpy");
        check_hip(hipMemcpy(G.w32, g32.data(), g32.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
      }
    }
    if (l == 0 && L.n > 0) {
      std::vector<double> inv = coarse_inverse(L, w64, H.bc);
      if (!H.coarse_inv) H.coarse_inv = zeros<double>(int64_t(L.n) * L.n);
      check_hip(hipMemcpy(H.coarse_inv, inv.data(), inv.size() * 8, hipMemcpyHostToDevice),
                "hipMemcpy");
    }
  }
  if (weight_forms(H) != forms_before) {
    // graphs captured with the old weight forms would read stale copies: drop them (they are
    // captured again on next use) and tell batches built on this hierarchy to recapture theirs
    for (auto& kv : H.graphs) (void)hipGraphExecDestroy(kv.second);
    H.graphs.clear();
    ++H.weight_epoch;
  }
}

namespace {
Hierarchy* build_levels(std::unique_ptr<Hierarchy> H, std::vector<Mesh> meshes,
                        const mg_hier_opts& o);
}  // namespace

Hierarchy* build_hierarchy(const Mesh& base, const mg_hier_opts& o) {
  auto H = std::make_unique<Hierarchy>();
  H->project = o.project_sphere != 0;
  // host meshes
  std::vector<Mesh> meshes;
  meshes.push_back(base);
  for (int i = 0; i < o.n_subdiv; ++i) {
    const bool cubic = (uint32_t(o.cubic_mask) >> i) & 1u;
    Mesh f = cubic ? subdivide_cubic(meshes.back(), H->project)
                   : subdivide(meshes.back(), H->project);
    std::string err = f.build_topology();
    if (!err.empty()) throw std::invalid_argument(err);
    meshes.push_back(std::move(f));
  }
  return build_levels(std::move(H), std::move(meshes), o);
}

Hierarchy* build_hierarchy_maps(std::vector<Mesh> meshes, bool nested_ids, const mg_hier_opts& o) {
  auto H = std::make_unique<Hierarchy>();
  H->nested_ids = nested_ids;
  return build_levels(std::move(H), std::move(meshes), o);
}

namespace {
// Operators, transfers, vectors and workspaces of every level of a hierarchy over `meshes`
// (coarsest first; every level above the base carries its interpolation rows).
Hierarchy* build_levels(std::unique_ptr<Hierarchy> H, std::vector<Mesh> meshes,
                        const mg_hier_opts& o) {
  H->bc = o.bc;
  for (auto& m : meshes) {
    m.build_stars();
    m.build_boundary();
    auto L = std::make_unique<Level>();
    L->mesh = std::move(m);
    L->nv = int32_t(L->mesh.nv);
    order_level(*L, H->bc, o.order);
    H->lv.push_back(std::move(L));
  }
  if (H->lv[0]->n > kMaxCoarse)
    throw std::invalid_argument("base mesh has more than " + std::to_string(kMaxCoarse) +
                                " unknowns; the coarsest level is solved densely");
  if (H->lv[0]->n == 0) throw std::invalid_argument("base mesh has no unknowns");
  for (size_t l = 0; l < H->lv.size(); ++l) {
    Level& L = *H->lv[l];
    std::vector<int32_t> col;
    build_operator_structure(L, col);
    L.col_h = col;
    L.op.sptr = upload(L.sptr_h);
    L.op.col = upload(col);
    build_gs_colors(L);
    std::vector<int16_t> col16;
    if (delta16(L, col, col16) && !col16.empty()) L.op.col16 = upload(col16);
    L.perm = upload(L.perm_h);
    L.bnd_ids = L.bnd_h.empty() ? zeros<int32_t>(1) : upload(L.bnd_h);
    L.star0 = upload(L.mesh.star0);
    alloc_vecs(L.v64, L.n);
    alloc_vecs(L.v32, L.n);
    L.cgs = zeros<CgsScalars>(1);
    if (l > 0) build_transfer(L, *H->lv[l - 1]);
  }
  H->n0 = H->lv[0]->n;
  upload_weights(*H);
  {
    int dev = 0, lim = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    check_hip(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
              "hipDeviceGetAttribute");
    H->lds_limit = std::min(lim, kCoarseLdsMax);
  }
  build_coarse_levels(*H, H->clv64, H->ctop64, H->clds64, H->cint_off64, H->clds_total64);
  build_coarse_levels(*H, H->clv32, H->ctop32, H->clds32, H->cint_off32, H->clds_total32);
  k::prepare_coarse(*H);
  for (size_t l = 1; l < H->lv.size(); ++l) build_tiles(*H->lv[l], *H->lv[l - 1]);
  // Krylov workspace on the finest level
  const int32_t n = H->lv.back()->n;
  H->sx = zeros<double>(n + 1);
  H->sr = zeros<double>(n + 1);
  H->sp = zeros<double>(n + 1);
  H->sp2 = zeros<double>(n + 1);
  H->sq = zeros<double>(n + 1);
  H->sz = zeros<double>(n + 1);
  const int32_t nvmax = H->lv.back()->nv;
  H->sb = zeros<double>(std::max(n, nvmax) + 1);
  H->part_cap = std::max(k::blocks_for(nvmax), 1);
  H->part = zeros<double>(3 * int64_t(H->part_cap));
  H->scal = zeros<DevScalars>(1);
  H->hist_cap = kHistoryCap;
  H->hist = zeros<double>(kHistoryCap);
  check_hip(hipHostMalloc(reinterpret_cast<void**>(&H->scal_host), sizeof(DevScalars), 0),
            "hipHostMalloc");
  std::memset(H->scal_host, 0, sizeof(DevScalars));
  check_hip(hipHostMalloc(reinterpret_cast<void**>(&H->aux_host), sizeof(double), 0),
            "hipHostMalloc");
  *H->aux_host = 0.0;
  check_hip(hipStreamCreateWithFlags(&H->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
  return H.release();
}
}  // namespace

Hierarchy::~Hierarchy() {
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  free_porous(*this);
  for (auto& Lp : lv) {
    Level& L = *Lp;
    for (void* p : {(void*)L.perm, (void*)L.bnd_ids, (void*)L.star0, (void*)L.op.sptr,
                    (void*)L.op.col, (void*)L.op.col16, (void*)L.op.w64, (void*)L.op.w32,
                    (void*)L.op.w16, (void*)L.op.pat, (void*)L.op.poff, (void*)L.op.pw32,
                    (void*)L.op.pw64,
                    (void*)L.op.idiag64,
                    (void*)L.op.idiag32, (void*)L.tr.pa, (void*)L.tr.pb, (void*)L.tr.r_self,
                    (void*)L.tr.r_sptr, (void*)L.tr.r_col, (void*)L.tr.r_col16, (void*)L.tr.p_base,
                    (void*)L.tr.p_ab16, (void*)L.v64.x, (void*)L.v64.b,
                    (void*)L.v64.r, (void*)L.v64.t, (void*)L.v32.x, (void*)L.v32.b,
                    (void*)L.v32.r, (void*)L.v32.t, (void*)L.v64.u, (void*)L.v32.u,
                    (void*)L.cgs})
      free_dev(p);
    for (void* p : {(void*)L.tr.p3, (void*)L.tr.pw64, (void*)L.tr.pw32, (void*)L.tr.rw_sptr,
                    (void*)L.tr.rw_col, (void*)L.tr.rw64, (void*)L.tr.rw32})
      free_dev(p);
    for (GsColor& G : L.gs)
      for (void* p : {(void*)G.rowid, (void*)G.sptr, (void*)G.col, (void*)G.w64, (void*)G.w32})
        free_dev(p);
    free_dev(L.row_color);
    for (void* p : {(void*)L.tiles.meta, (void*)L.tiles.row, (void*)L.tiles.ent,
                    (void*)L.tiles.col, (void*)L.tiles.crow, (void*)L.tiles.cst,
                    (void*)L.tiles.cent})
      free_dev(p);
  }
  for (void* p : {(void*)clv64, (void*)clv32, (void*)coarse_inv, (void*)sx, (void*)sr, (void*)sp, (void*)sp2, (void*)sq, (void*)sz,
                  (void*)sb, (void*)part, (void*)scal, (void*)hist, (void*)kvert_d})
    free_dev(p);
  if (scal_host) (void)hipHostFree(scal_host);
  if (aux_host) (void)hipHostFree(aux_host);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

}  // namespace decmg

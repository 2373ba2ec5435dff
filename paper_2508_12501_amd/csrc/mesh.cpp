// Host mesh construction: base meshes, face maps, binary subdivision, Hodge stars.
// Compiled with -ffp-contract=off so coordinates follow plain IEEE evaluation order.
#include "mesh.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <stdexcept>

namespace decmg {

std::string Mesh::build_topology() {
  // Edge ids by first appearance over (triangle, side).  Candidate edges are bucketed by
  // their smaller endpoint; each bucket holds at most the number of sides starting there.
  std::vector<int64_t> off(nv + 1, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int32_t u = tri[3 * t + k], w = tri[3 * t + (k + 1) % 3];
      off[std::min(u, w) + 1]++;
    }
  for (int64_t v = 0; v < nv; ++v) off[v + 1] += off[v];
  std::vector<int32_t> bucket_hi(3 * nt), bucket_id(3 * nt);
  std::vector<int32_t> fill(nv, 0);
  std::vector<int8_t> uses;
  edge.clear();
  edge.reserve(2 * (nv + nt + 8));
  tri_edge.assign(3 * nt, 0);
  tri_sign.assign(3 * nt, 0);
  ne = 0;
  for (int64_t t = 0; t < nt; ++t) {
    for (int k = 0; k < 3; ++k) {
      int32_t u = tri[3 * t + k], w = tri[3 * t + (k + 1) % 3];
      if (u == w) return "degenerate triangle " + std::to_string(t);
      int32_t lo = std::min(u, w), hi = std::max(u, w);
      int64_t b = off[lo];
      int32_t id = -1;
      for (int32_t q = 0; q < fill[lo]; ++q)
        if (bucket_hi[b + q] == hi) { id = bucket_id[b + q]; break; }
      if (id < 0) {
        id = static_cast<int32_t>(ne++);
        bucket_hi[b + fill[lo]] = hi;
        bucket_id[b + fill[lo]] = id;
        fill[lo]++;
        edge.push_back(lo);
        edge.push_back(hi);
        uses.push_back(0);
      }
      if (++uses[id] > 2) return "edge (" + std::to_string(lo) + "," + std::to_string(hi) +
                                 ") is a face of more than two triangles";
      tri_edge[3 * t + k] = id;
      tri_sign[3 * t + k] = (u < w) ? 1 : -1;
    }
  }
  return "";
}

std::string Mesh::validate_vertices() const {
  std::vector<uint8_t> used(nv, 0);
  for (int64_t i = 0; i < 3 * nt; ++i) used[tri[i]] = 1;
  for (int64_t v = 0; v < nv; ++v) {
    if (!used[v]) return "vertex " + std::to_string(v) + " is in no triangle";
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(xyz[3 * v + c])) return "non-finite coordinate at vertex " + std::to_string(v);
  }
  // no two triangles on the same vertex set
  std::vector<std::array<int32_t, 3>> keys(nt);
  for (int64_t t = 0; t < nt; ++t) {
    std::array<int32_t, 3> k = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
    std::sort(k.begin(), k.end());
    keys[t] = k;
  }
  std::sort(keys.begin(), keys.end());
  for (int64_t t = 1; t < nt; ++t)
    if (keys[t] == keys[t - 1]) return "duplicate triangle on vertices " + std::to_string(keys[t][0]) +
                                       "," + std::to_string(keys[t][1]) + "," + std::to_string(keys[t][2]);
  return "";
}

namespace {
// cot of the angle at pk in triangle (pk, pi, pj): (u . v) / |u x v|.
inline double cot_at(const double* pk, const double* pi, const double* pj) {
  const double u0 = pi[0] - pk[0], u1 = pi[1] - pk[1], u2 = pi[2] - pk[2];
  const double v0 = pj[0] - pk[0], v1 = pj[1] - pk[1], v2 = pj[2] - pk[2];
  const double dot = u0 * v0 + u1 * v1 + u2 * v2;
  const double cx = u1 * v2 - u2 * v1, cy = u2 * v0 - u0 * v2, cz = u0 * v1 - u1 * v0;
  return dot / std::sqrt(cx * cx + cy * cy + cz * cz);
}
inline double dist2(const double* a, const double* b) {
  const double d0 = b[0] - a[0], d1 = b[1] - a[1], d2 = b[2] - a[2];
  return d0 * d0 + d1 * d1 + d2 * d2;
}
}  // namespace

void Mesh::build_stars() {
  // Circumcentric diagonal Hodge stars (signed): star1 = |dual|/|primal| = half the sum of
  // the cotangents of the angles facing the edge; star0 = dual-cell area, each triangle
  // giving vertex i the quadrilateral (i, mid ij, circumcentre, mid ik) of area
  // (|ij|^2 cot k + |ik|^2 cot j) / 8.
  star0.assign(nv, 0.0);
  star1.assign(ne, 0.0);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    const double* pa = &xyz[3 * a];
    const double* pb = &xyz[3 * b];
    const double* pc = &xyz[3 * c];
    const double ca = cot_at(pa, pb, pc), cb = cot_at(pb, pc, pa), cc = cot_at(pc, pa, pb);
    star1[tri_edge[3 * t + 0]] += 0.5 * cc;   // side ab faces c
    star1[tri_edge[3 * t + 1]] += 0.5 * ca;   // side bc faces a
    star1[tri_edge[3 * t + 2]] += 0.5 * cb;   // side ca faces b
    const double lab = dist2(pa, pb), lbc = dist2(pb, pc), lca = dist2(pc, pa);
    star0[a] += (lab * cc + lca * cb) / 8.0;
    star0[b] += (lbc * ca + lab * cc) / 8.0;
    star0[c] += (lca * cb + lbc * ca) / 8.0;
  }
}

void Mesh::build_boundary() {
  std::vector<int8_t> cnt(ne, 0);
  for (int64_t i = 0; i < 3 * nt; ++i) cnt[tri_edge[i]]++;
  bnd.assign(nv, 0);
  for (int64_t e = 0; e < ne; ++e)
    if (cnt[e] == 1) { bnd[edge[2 * e]] = 1; bnd[edge[2 * e + 1]] = 1; }
}

Mesh square_grid(int32_t n) {
  Mesh m;
  m.nv = int64_t(n + 1) * (n + 1);
  m.nt = 2 * int64_t(n) * n;
  m.xyz.assign(3 * m.nv, 0.0);
  for (int32_t j = 0; j <= n; ++j)
    for (int32_t i = 0; i <= n; ++i) {
      int64_t v = int64_t(j) * (n + 1) + i;
      m.xyz[3 * v + 0] = double(i) / n;
      m.xyz[3 * v + 1] = double(j) / n;
    }
  m.tri.reserve(3 * m.nt);
  for (int32_t cj = 0; cj < n; ++cj)
    for (int32_t ci = 0; ci < n; ++ci) {
      int32_t a = cj * (n + 1) + ci, b = a + 1, c = a + n + 2, d = a + n + 1;
      m.tri.insert(m.tri.end(), {a, b, c, a, c, d});
    }
  return m;
}

Mesh icosahedron() {
  const double f = (1.0 + std::sqrt(5.0)) / 2.0;
  const double raw[12][3] = {{-1, f, 0}, {1, f, 0}, {-1, -f, 0}, {1, -f, 0},
                             {0, -1, f}, {0, 1, f}, {0, -1, -f}, {0, 1, -f},
                             {f, 0, -1}, {f, 0, 1}, {-f, 0, -1}, {-f, 0, 1}};
  Mesh m;
  m.nv = 12;
  auto d2 = [&](int i, int j) { return dist2(raw[i], raw[j]); };
  for (int i = 0; i < 12; ++i)
    for (int j = i + 1; j < 12; ++j)
      for (int k = j + 1; k < 12; ++k) {
        if (std::fabs(d2(i, j) - 4) < 1e-9 && std::fabs(d2(j, k) - 4) < 1e-9 &&
            std::fabs(d2(i, k) - 4) < 1e-9) {
          double u[3], v[3], s[3];
          for (int c = 0; c < 3; ++c) {
            u[c] = raw[j][c] - raw[i][c];
            v[c] = raw[k][c] - raw[i][c];
            s[c] = raw[i][c] + raw[j][c] + raw[k][c];
          }
          const double nx = u[1] * v[2] - u[2] * v[1], ny = u[2] * v[0] - u[0] * v[2],
                       nz = u[0] * v[1] - u[1] * v[0];
          if (nx * s[0] + ny * s[1] + nz * s[2] > 0)
            m.tri.insert(m.tri.end(), {i, j, k});
          else
            m.tri.insert(m.tri.end(), {i, k, j});
        }
      }
  m.nt = int64_t(m.tri.size() / 3);
  m.xyz.resize(36);
  for (int v = 0; v < 12; ++v) {
    const double r = std::sqrt(raw[v][0] * raw[v][0] + raw[v][1] * raw[v][1] + raw[v][2] * raw[v][2]);
    for (int c = 0; c < 3; ++c) m.xyz[3 * v + c] = raw[v][c] / r;
  }
  return m;
}

// Subdivision reads the coarse mesh's edges and face maps (build_topology).
static void need_topology(const Mesh& c) {
  if (c.tri_edge.size() != 3 * size_t(c.nt) || c.edge.size() != 2 * size_t(c.ne))
    throw std::logic_error("subdivision of a mesh without its topology");
}

Mesh subdivide(const Mesh& c, bool project_sphere) {
  need_topology(c);
  Mesh f;
  f.nv = c.nv + c.ne;
  f.nt = 4 * c.nt;
  f.xyz.resize(3 * f.nv);
  std::copy(c.xyz.begin(), c.xyz.end(), f.xyz.begin());
  f.parent.resize(2 * f.nv);
  for (int64_t v = 0; v < c.nv; ++v) f.parent[2 * v] = f.parent[2 * v + 1] = int32_t(v);
  for (int64_t e = 0; e < c.ne; ++e) {
    const int32_t a = c.edge[2 * e], b = c.edge[2 * e + 1];
    double* m = &f.xyz[3 * (c.nv + e)];
    for (int k = 0; k < 3; ++k) m[k] = 0.5 * (c.xyz[3 * a + k] + c.xyz[3 * b + k]);
    if (project_sphere) {
      const double r = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
      for (int k = 0; k < 3; ++k) m[k] = m[k] / r;
    }
    f.parent[2 * (c.nv + e)] = a;
    f.parent[2 * (c.nv + e) + 1] = b;
  }
  f.scheme = 1;
  f.parent3.resize(3 * f.nv);
  f.pweight.assign(3 * f.nv, 0.0);
  for (int64_t v = 0; v < f.nv; ++v) {
    const int32_t a = f.parent[2 * v], b = f.parent[2 * v + 1];
    f.parent3[3 * v] = a;
    f.parent3[3 * v + 1] = b;
    f.parent3[3 * v + 2] = a;
    f.pweight[3 * v] = a == b ? 1.0 : 0.5;
    f.pweight[3 * v + 1] = a == b ? 0.0 : 0.5;
  }
  f.tri.resize(3 * f.nt);
  for (int64_t t = 0; t < c.nt; ++t) {
    const int32_t a = c.tri[3 * t], b = c.tri[3 * t + 1], cc = c.tri[3 * t + 2];
    const int32_t ab = int32_t(c.nv + c.tri_edge[3 * t]);
    const int32_t bc = int32_t(c.nv + c.tri_edge[3 * t + 1]);
    const int32_t ca = int32_t(c.nv + c.tri_edge[3 * t + 2]);
    const int32_t ch[4][3] = {{a, ab, ca}, {ab, b, bc}, {ca, bc, cc}, {ab, bc, ca}};
    for (int q = 0; q < 4; ++q)
      for (int k = 0; k < 3; ++k) f.tri[3 * (4 * t + q) + k] = ch[q][k];
  }
  return f;
}

Mesh subdivide_cubic(const Mesh& c, bool project_sphere) {
  need_topology(c);
  Mesh f;
  f.nv = c.nv + 2 * c.ne + c.nt;
  f.nt = 9 * c.nt;
  f.scheme = 2;
  f.xyz.resize(3 * f.nv);
  std::copy(c.xyz.begin(), c.xyz.end(), f.xyz.begin());
  f.parent3.resize(3 * f.nv);
  f.pweight.assign(3 * f.nv, 0.0);
  for (int64_t v = 0; v < c.nv; ++v) {
    for (int k = 0; k < 3; ++k) f.parent3[3 * v + k] = int32_t(v);
    f.pweight[3 * v] = 1.0;
  }
  auto push = [&](double* p) {
    if (project_sphere) {
      const double r = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      for (int k = 0; k < 3; ++k) p[k] = p[k] / r;
    }
  };
  for (int64_t e = 0; e < c.ne; ++e) {
    const int32_t a = c.edge[2 * e], b = c.edge[2 * e + 1];
    double* p1 = &f.xyz[3 * (c.nv + 2 * e)];
    double* p2 = &f.xyz[3 * (c.nv + 2 * e + 1)];
    for (int k = 0; k < 3; ++k) {
      p1[k] = (2.0 * c.xyz[3 * a + k] + c.xyz[3 * b + k]) / 3.0;
      p2[k] = (c.xyz[3 * a + k] + 2.0 * c.xyz[3 * b + k]) / 3.0;
    }
    push(p1);
    push(p2);
    const int64_t v1 = c.nv + 2 * e, v2 = v1 + 1;
    f.parent3[3 * v1] = a;
    f.parent3[3 * v1 + 1] = b;
    f.parent3[3 * v1 + 2] = a;
    f.pweight[3 * v1] = 2.0 / 3.0;
    f.pweight[3 * v1 + 1] = 1.0 / 3.0;
    f.parent3[3 * v2] = a;
    f.parent3[3 * v2 + 1] = b;
    f.parent3[3 * v2 + 2] = a;
    f.pweight[3 * v2] = 1.0 / 3.0;
    f.pweight[3 * v2 + 1] = 2.0 / 3.0;
  }
  f.tri.resize(3 * f.nt);
  for (int64_t t = 0; t < c.nt; ++t) {
    const int32_t a = c.tri[3 * t], b = c.tri[3 * t + 1], cc = c.tri[3 * t + 2];
    const int64_t m = c.nv + 2 * c.ne + t;
    double* pm = &f.xyz[3 * m];
    for (int k = 0; k < 3; ++k) pm[k] = (c.xyz[3 * a + k] + c.xyz[3 * b + k] + c.xyz[3 * cc + k]) / 3.0;
    push(pm);
    for (int k = 0; k < 3; ++k) {
      f.parent3[3 * m + k] = c.tri[3 * t + k];
      f.pweight[3 * m + k] = 1.0 / 3.0;
    }
    // the two points of side k, ordered from the side's first vertex
    auto side = [&](int k, int32_t first, int32_t& x1, int32_t& x2) {
      const int64_t e = c.tri_edge[3 * t + k];
      const int32_t lo = int32_t(c.nv + 2 * e), hi = lo + 1;
      const bool first_is_lo = c.edge[2 * e] == first;
      x1 = first_is_lo ? lo : hi;
      x2 = first_is_lo ? hi : lo;
    };
    int32_t ab1, ab2, bc1, bc2, ca1, ca2;
    side(0, a, ab1, ab2);
    side(1, b, bc1, bc2);
    side(2, cc, ca1, ca2);
    const int32_t mm = int32_t(m);
    const int32_t ch[9][3] = {{a, ab1, ca2},   {ab2, b, bc1},   {ca1, bc2, cc},
                              {ab1, ab2, mm},  {bc1, bc2, mm},  {ca1, ca2, mm},
                              {ab1, mm, ca2},  {ab2, bc1, mm},  {bc2, ca1, mm}};
    for (int q = 0; q < 9; ++q)
      for (int k = 0; k < 3; ++k) f.tri[3 * (9 * t + q) + k] = ch[q][k];
  }
  return f;
}

}  // namespace decmg
